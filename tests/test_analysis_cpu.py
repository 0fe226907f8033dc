"""CPU checks of the analysis helpers the statistical GPU tests rely on
(bench.py): they must find a planted signal and nothing in its absence."""
import os

import numpy as np

import bench


def _planted(eps, n, seed):
    """Points in the unit cell with density 1 + eps sum_a cos(2 pi f_a)."""
    rng = np.random.default_rng(seed)
    x = rng.random((4 * n, 3))
    w = 1.0 + eps * np.cos(2 * np.pi * x).sum(axis=1)
    keep = rng.random(len(x)) * (1.0 + 3.0 * abs(eps)) < w
    return x[keep][:n]


def test_node_harmonic_recovers_a_planted_amplitude():
    for eps in (0.0, 0.02, -0.02):
        f = _planted(eps, 400000, 1)
        assert abs(bench.node_harmonic(f) - eps) < 0.004
    ratio, c, z = bench.cell_histogram_bias(_planted(0.02, 400000, 2))
    assert ratio > 0.03                      # corners denser than the centre
    assert abs(bench.cell_histogram_bias(_planted(0.0, 400000, 3))[0]) < 0.02


def test_pair_histogram_of_an_ideal_gas_is_flat():
    rng = np.random.default_rng(4)
    L, n = 20.0, 2000
    counts = np.zeros(20)
    for _ in range(5):
        counts += bench.pair_histogram(rng.random((n, 3)) * L, L, 5.0, 20)
    g = bench.gr_from_counts(counts, 5, n, L, 5.0)
    assert np.max(np.abs(g[4:] - 1.0)) < 0.05


def test_pair_histogram_uses_minimum_image():
    L = 10.0
    q = np.array([[0.25, 5.0, 5.0], [9.9, 5.0, 5.0], [5.0, 5.0, 5.0]])
    c = bench.pair_histogram(q, L, 5.0, 50)
    assert c[3] == 1.0                       # the pair 0.35 apart across the boundary
    assert c.sum() == 3.0                    # 4.75 and 4.9 apart: also within 5


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with status 2
    and says so, before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in (r.stdout + r.stderr)


def test_profile_summary_lists_every_step_kernel():
    """The committed counter summary that the benchmark's roofline traffic
    and step traffic are read from names its source hash and carries a
    traffic line for every kernel of the step (both y passes)."""
    with open(bench.PROFILE) as fh:
        lines = fh.read().splitlines()
    assert any(l.startswith("source hash") and len(l.split()[-1]) == 16 for l in lines)
    names = [l[len("traffic "):].rsplit(" ", 1)[0] for l in lines if l.startswith("traffic ")]
    for prefix in bench.STEP_KERNELS:
        hits = [n for n in names if n.startswith(prefix)]
        assert len(hits) == (2 if prefix == "k_y_fast<" else 1), prefix
    assert bench.PHASE_KERNEL["rhs"] in names
