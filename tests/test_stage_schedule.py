"""CPU model of the fused stage kernel's LDS plane bookkeeping (host logic, no GPU).

The kernel keeps, per z-iteration `it` (entering plane L = it - 2R, gradient plane
a = L - R, output plane o = L - 2R):
  - the u plane of a and the point-field plane of o, in one LDS buffer (DB = 0) or
    alternating between two by the parity of `it` (DB = 1);
  - the x/y nested fields of the last R + 1 gradient planes in a ring indexed it % (R + 1);
  - the z nested fields of the last 2R + 1 gradient planes (own column) in a ring indexed
    it % (2R + 1).
With DB = 0 an iteration has two barriers (after the u plane, after the point-field plane);
with DB = 1 one (the point-field plane is stored before it).  The model replays the
schedule and checks that every LDS read finds the plane it expects, written before a
barrier that precedes the read (or earlier by the same thread, for the own-column ring),
and that no slot is written and read by different threads between the same two barriers.
"""
import itertools

import pytest


def replay(R, zc, DB, nbuf=None):
    nbuf = (2 if DB else 1) if nbuf is None else nbuf
    iters = zc + 4 * R
    slots = {}           # (array, slot) -> (plane, phase written, own-thread data)
    access = {}          # (array, slot, phase) -> {'r', 'w'}
    phase = 0

    def write(arr, slot, plane, own=False):
        slots[(arr, slot)] = (plane, phase, own)
        if not own:
            access.setdefault((arr, slot, phase), set()).add("w")

    def read(arr, slot, plane, own=False):
        got, ph, _ = slots[(arr, slot)]
        assert got == plane, (arr, slot, got, plane)
        if own:
            assert ph <= phase
        else:
            assert ph < phase, (arr, slot, plane, "read in the phase it was written")
            access.setdefault((arr, slot, phase), set()).add("r")

    for it in range(iters):
        L = it - 2 * R
        a, o = L - R, L - 2 * R
        b = it % nbuf
        do_grad, do_out = it >= 2 * R, it >= 4 * R
        if do_grad:
            write("u", b, a)
        if DB and do_out:
            write("pl", b, o)
        phase += 1
        if do_grad:
            read("u", b, a)
            write("axy", it % (R + 1), a)
            write("az", it % (2 * R + 1), a, own=True)
        if not DB:
            if do_out:
                write("pl", 0, o)
            phase += 1
        if do_out:
            read("pl", b, o)
            read("axy", (it - R) % (R + 1), o)
            for m in range(1, R + 1):
                read("az", (it + m - R) % (2 * R + 1), o + m, own=True)
                read("az", (it - m - R) % (2 * R + 1), o - m, own=True)
    races = [k for k, v in access.items() if len(v) > 1]
    assert not races, races[:4]


@pytest.mark.parametrize("R,zc,DB", list(itertools.product((1, 2, 3, 4), (1, 2, 5, 11, 64, 512), (0, 1))))
def test_lds_schedule(R, zc, DB):
    replay(R, zc, DB)


def test_model_catches_a_single_buffer_with_one_barrier():
    # one barrier per iteration but one buffer: the next plane's stores overwrite the
    # point-field plane while the residual of the previous plane still reads it
    with pytest.raises(AssertionError):
        replay(2, 16, DB=1, nbuf=1)
