"""Host-side pieces of bench.py that need no GPU."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402
from workloads import serving_stream  # noqa: E402


def test_arrival_times_are_cumulative_gaps():
    s = serving_stream(20, seed=9, k_range=(1, 2), bonds=(4,))
    t = bench.arrival_times(s, 2.0)
    assert np.all(np.diff(t) >= 0)
    assert np.allclose(t, np.cumsum([r.arrival_gap for r in s]) / 2.0)
    assert bench.arrival_times(s, 0.0) == [0.0] * 20


def test_gate_flops_formula():
    # 128 x 128 saturated gate: contraction 32*64^3 + 128*64^2, SVD 4(4 m n^2 + 8 n^3), update 8*128*128*64
    f = bench.gate_flops(64, 64, 64, 64)
    assert f == 32 * 64 ** 3 + 128 * 64 ** 2 + 4 * (4 * 128 ** 3 + 8 * 128 ** 3) + 8 * 128 * 128 * 64


def test_forked_gate_fraction():
    """Fork-schedule work fraction: with one rotation per batch it is the
    mean over rotations of the gates left after each fork gate; with a
    single batch, the gates left after the earliest fork gate."""
    q2c = pytest.importorskip("paper_2207_03711_amd.q2c", reason="libq2c.so not built")
    from workloads import CONFIGS

    I = CONFIGS["q8_d16"].integrals()
    p = q2c.Problem(None, I.n_orb, I.n_elec, I.h1, I.eri, I.e_const)
    _, rot, _, _ = q2c.vqe_problem_gates(p.h)
    n = len(rot)
    fork = np.array([np.flatnonzero(rot == m)[0] for m in range(p.info["n_rotations"])])
    assert np.all(np.diff(fork) > 0)
    assert abs(bench.forked_gate_fraction(p, 2) - np.mean(n - fork) / n) < 1e-12
    assert abs(bench.forked_gate_fraction(p, 10**6) - (n - fork.min()) / n) < 1e-12
    p.close()


def test_gate_phase_split():
    cyc = {"contract": 6.0, "reduce": 45.0, "values": 17.0, "vectors": 12.0, "back": 13.0, "update": 7.0}
    s = bench.gate_phase_split(cyc)
    assert abs(s["contract"] - 0.06) < 1e-15 and abs(s["svd"] - 0.87) < 1e-15 and abs(s["update"] - 0.07) < 1e-15
    assert abs(sum(s["svd_parts"].values()) - s["svd"]) < 1e-15


def test_traffic_constant_matches_kernel_source():
    """The HBM traffic figure in the bench line belongs to one kernel source:
    a kernel change must come with new counter passes (else the bench
    reports null)."""
    assert bench.measured_traffic("q16_d64") is not None
    assert bench.measured_traffic("q8_d16") is None


def test_more_than_one_gpu_is_refused():
    """bench.py measures one GPU; asked for more it exits with status 2 and a
    message, before touching a device."""
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
