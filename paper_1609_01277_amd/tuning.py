"""Autotuning of the fused stage kernel's launch configuration, with a JSON cache.

The library times its compiled variants (x/y tile, load-ahead depth) and z-chunk
lengths on the caller's buffers (sbli_autotune) and keeps the fastest.  Results
are cached per (grid, order, dtype, device) in a JSON file so later runs skip the
search.  Every variant gives bitwise identical results, so the cache only affects
speed.
"""
import json
import os

from . import _lib

DEFAULT_CACHE = os.environ.get("SBLI_TUNING_CACHE",
                               os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json"))


def device_tag(torch):
    """Architecture and compute-unit count of the current device.  The marketing name is not
    used: it depends on the host's amdgpu.ids table and on tools loaded into the process."""
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return "%s/%dcu" % (getattr(p, "gcnArchName", "") or p.name, p.multi_processor_count)


def cache_key(params, device_name):
    return "%dx%dx%d|order%d|%s|%s" % (params.nx, params.ny, params.nz, params.order,
                                       "f64" if params.dtype == _lib.SBLI_F64 else "f32", device_name)


def load_cache(path=DEFAULT_CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store_cache(entries, path=DEFAULT_CACHE):
    try:
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(entries, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
        return True
    except OSError:
        return False


def autotune(solver, reps=2, path=DEFAULT_CACHE, force=False):
    """Select the launch configuration of `solver` (a Solver); returns the cache entry."""
    torch = solver.torch
    key = cache_key(solver.params, device_tag(torch))
    cache = load_cache(path)
    ent = cache.get(key)
    nv = _lib.sbli_num_variants(solver.ctx)
    if ent and not force and 0 <= ent.get("variant", -1) < nv:
        info = _lib.sbli_variant_info(solver.ctx, ent["variant"])
        if list(info) == ent.get("tile", list(info)):
            _lib.sbli_set_tuning(solver.ctx, ent["variant"], ent["zchunk"])
            return dict(ent, cached=True)
    q, qt, dq = solver.empty_state(), solver.empty_state(), solver.empty_state()
    solver.tgv_init(q)
    h = 2 * 3.141592653589793 / max(solver.params.nx, solver.params.ny, solver.params.nz)
    dt = 0.1 * h * solver.params.Mach
    ms = _lib.sbli_autotune(solver.ctx, q, qt, dq, dt, reps)
    v, z = _lib.sbli_get_tuning(solver.ctx)
    ent = {"variant": v, "zchunk": z, "tile": list(_lib.sbli_variant_info(solver.ctx, v)),
           "ms_per_step": ms}
    cache = load_cache(path)
    cache[key] = ent
    store_cache(cache, path)
    del q, qt, dq
    return dict(ent, cached=False)
