"""Host-side helpers of bench.py whose outputs are reported numbers: the TT
difference of two solutions (from core inner products, no full tensor), the
kernel-source hash that keys the stored traffic counters, and the refusal of
more than one GPU."""
import os
import subprocess
import sys

import numpy as np

import bench
import tt_inputs as ti

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tt_rel_diff_equals_the_dense_difference():
    rng = np.random.default_rng(0)
    x = ti.random_tt(40, 4, 6, 5, 3, seed=1)
    for y in (ti.random_tt(40, 4, 6, 7, 2, seed=2),                      # different ranks
              (x[0] * (1 + 1e-4 * rng.standard_normal(x[0].shape)), x[1], x[2])):   # a near copy
        X = np.einsum("ka,alb,bp->klp", *x)
        Y = np.einsum("ka,alb,bp->klp", *y)
        ref = np.linalg.norm(X - Y) / np.linalg.norm(X)
        # ||X - Y||^2 = <X,X> + <Y,Y> - 2 <X,Y> cancels to a few eps of ||X||^2,
        # so d = ||X - Y|| / ||X|| carries an absolute error of about 2 eps / d
        eps = np.finfo(float).eps
        assert abs(bench.tt_rel_diff(x, y) - ref) <= 1e-12 * ref + 32 * eps / ref
    assert bench.tt_rel_diff(x, x) < 1e-7


def test_kernel_source_hash_tracks_the_counted_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert all(os.path.exists(os.path.join(ROOT, p)) for p in bench.KERNEL_SOURCES)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
