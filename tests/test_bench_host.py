"""Host logic of bench.py (CPU only): when the committed rocprofv3 counter summary
may stand for the kernel being timed, and how its counts become HBM bytes."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _summary(**over):
    c = {"kernel_source_sha256": bench.kernel_source_hash(), "n": 512, "order": 4, "dtype": "f64",
         "tile": [16, 16, 1, 1, 1, 1, 0], "zchunk": 512, "fetch_kib_per_dispatch": 1000.0,
         "write_kib_per_dispatch": 300.0, "copy_fetch_factor": 2.0, "copy_write_factor": 1.0}
    c.update(over)
    return c


@pytest.fixture
def counters(tmp_path, monkeypatch):
    path = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(path))

    def write(c):
        path.write_text(json.dumps(c))
    return write


TUNING = {"tile": [16, 16, 1, 1, 1, 1, 0], "zchunk": 512}


def test_matching_summary_gives_scaled_bytes(counters):
    counters(_summary())
    # 1024 B per KiB x (fetch x 2.0 + write x 1.0)
    assert bench.counted_traffic(512, 4, "f64", TUNING) == 1024.0 * (1000.0 * 2.0 + 300.0 * 1.0)


@pytest.mark.parametrize("over", [{"kernel_source_sha256": "0" * 64}, {"n": 256}, {"order": 8}, {"dtype": "f32"},
                                  {"tile": [32, 8, 1, 1, 1, 1, 0]}, {"zchunk": 64}])
def test_summary_of_other_kernel_or_launch_is_not_used(counters, over):
    counters(_summary(**over))
    assert bench.counted_traffic(512, 4, "f64", TUNING) is None


def test_missing_or_unreadable_summary(counters, tmp_path, monkeypatch):
    assert bench.counted_traffic(512, 4, "f64", TUNING) is None          # not written yet
    (tmp_path / "counters.json").write_text("{not json")
    assert bench.counted_traffic(512, 4, "f64", TUNING) is None
    counters(_summary())
    assert bench.counted_traffic(512, 4, "f64", None) is None           # no tuning known


def test_source_hash_covers_the_stage_kernel_sources():
    # the hash changes with any of the three sources the stage kernel is built from
    assert set(bench.KERNEL_SOURCES) == {"kernels_stage_fused.h", "stage_variants.h", "sbli_common.h"}
    assert len(bench.kernel_source_hash()) == 64
