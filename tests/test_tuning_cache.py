"""Host logic of the autotuner's JSON cache (CPU only): keys, loading and storing."""
import json

from paper_1609_01277_amd import _lib, tuning


def _params(nx, ny, nz, order, dtype):
    p = _lib.sbli_params()
    p.nx, p.ny, p.nz, p.order, p.dtype = nx, ny, nz, order, dtype
    return p


def test_cache_key_names_grid_order_dtype_and_device():
    k64 = tuning.cache_key(_params(512, 512, 512, 4, _lib.SBLI_F64), "MI355X")
    k32 = tuning.cache_key(_params(512, 512, 512, 4, _lib.SBLI_F32), "MI355X")
    assert k64 == "512x512x512|order4|f64|MI355X"
    assert k32 == "512x512x512|order4|f32|MI355X"
    assert tuning.cache_key(_params(64, 32, 16, 8, _lib.SBLI_F64), "other") == "64x32x16|order8|f64|other"


def test_missing_or_corrupt_cache_reads_as_empty(tmp_path):
    assert tuning.load_cache(str(tmp_path / "absent.json")) == {}
    bad = tmp_path / "bad.json"
    bad.write_text("{ not json")
    assert tuning.load_cache(str(bad)) == {}


def test_store_then_load_round_trip_leaves_no_temporary(tmp_path):
    path = tmp_path / "cache.json"
    entries = {"512x512x512|order4|f64|MI355X": {"variant": 5, "zchunk": 512, "tile": [16, 16, 1, 1, 1, 1, 0],
                                                  "ms_per_step": 18.0}}
    assert tuning.store_cache(entries, str(path))
    assert tuning.load_cache(str(path)) == entries
    assert json.loads(path.read_text()) == entries
    assert [p.name for p in tmp_path.iterdir()] == ["cache.json"]


def test_store_into_missing_directory_fails_quietly(tmp_path):
    assert tuning.store_cache({}, str(tmp_path / "no" / "such" / "dir" / "c.json")) is False


class _FakeProps:
    def __init__(self, arch, name, cus):
        self.gcnArchName, self.name, self.multi_processor_count = arch, name, cus


class _FakeCuda:
    def __init__(self, props):
        self._props = props

    def current_device(self):
        return 0

    def get_device_properties(self, i):
        return self._props


class _FakeTorch:
    def __init__(self, props):
        self.cuda = _FakeCuda(props)


def test_device_tag_uses_architecture_and_cu_count_not_marketing_name():
    # the marketing name differs between processes on one machine (it comes from a host table
    # that may be missing), so two processes must agree on the tag whatever the name reads
    a = tuning.device_tag(_FakeTorch(_FakeProps("gfx950:sramecc+:xnack-", "", 256)))
    b = tuning.device_tag(_FakeTorch(_FakeProps("gfx950:sramecc+:xnack-", "AMD Radeon Graphics", 256)))
    assert a == b == "gfx950:sramecc+:xnack-/256cu"
    assert tuning.device_tag(_FakeTorch(_FakeProps("", "dev", 8))) == "dev/8cu"
