"""Host-side helpers of bench.py whose outputs are reported numbers: the TT
difference of two solutions (through the R factor of the stacked first cores,
no full tensor), the
kernel-source hash and projection grid that key the stored traffic counters,
and the refusal of
more than one GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
import tt_inputs as ti

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tt_rel_diff_equals_the_dense_difference():
    # the difference is taken through a Householder R of the stacked first
    # cores, with no cancellation: it resolves relative differences far below
    # sqrt(eps), down to the rounding of the cores themselves
    rng = np.random.default_rng(0)
    x = ti.random_tt(40, 4, 6, 5, 3, seed=1)
    for y in (ti.random_tt(40, 4, 6, 7, 2, seed=2),                      # different ranks
              (x[0] * (1 + 1e-4 * rng.standard_normal(x[0].shape)), x[1], x[2]),   # a near copy
              (x[0] * (1 + 1e-11 * rng.standard_normal(x[0].shape)), x[1], x[2])):  # a very near copy
        X = np.einsum("ka,alb,bp->klp", *x)
        Y = np.einsum("ka,alb,bp->klp", *y)
        ref = np.linalg.norm(X - Y) / np.linalg.norm(Y)
        assert abs(bench.tt_rel_diff(x, y) - ref) <= 1e-6 * ref + 1e-15
    assert bench.tt_rel_diff(x, x) < 1e-15


def test_tt_rel_diff_over_row_chunks():
    # more rows than one chunk of the first-core R (2^20 rows)
    x = ti.random_tt((1 << 20) + 37, 3, 2, 3, 2, seed=3)
    y = (x[0].copy(), x[1].copy(), x[2].copy())
    y[0][-5:] += 1e-3
    X = np.einsum("ka,alb,bp->klp", *x)
    Y = np.einsum("ka,alb,bp->klp", *y)
    ref = np.linalg.norm(X - Y) / np.linalg.norm(Y)
    assert bench.tt_rel_diff(x, y) == pytest.approx(ref, rel=1e-8)


def test_kernel_source_hash_tracks_the_counted_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert all(os.path.exists(os.path.join(ROOT, p)) for p in bench.KERNEL_SOURCES)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_stored_traffic_requires_the_profiled_grid(tmp_path, monkeypatch):
    # counters taken at one projection grid do not describe another
    import json
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"source_hash": bench.kernel_source_hash(), "project_blocks": 256,
                             "fetch_bytes": 1.0, "write_bytes": 2.0}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.stored_traffic() is not None
    assert bench.stored_traffic(256) is not None
    assert bench.stored_traffic(512) is None
    f.write_text(json.dumps({"source_hash": "0" * 16, "project_blocks": 256}))
    assert bench.stored_traffic(256) is None
