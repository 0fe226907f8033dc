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


def test_compact_record_is_small_and_carries_the_headline():
    """The benchmark's last stdout line must survive a tail of a few KB: the
    compact record keeps the headline keys, the roofline and the CPU
    baseline, and summarises the other legs in a line each."""
    import json
    ph = {k: dict(avg_launch_us=10.0 + i, total_ms_per_step=0.01) for i, k in enumerate(
        ("rhs", "fft_x_fwd", "fft_y_fwd", "fft_z_solve", "fft_y_inv", "fft_x_inv", "gather", "forces"))}
    big = list(np.linspace(0, 1, 5000))
    out = dict(metric=bench.METRIC, value=2.9e10, unit="cell-steps/s", n_gpus=1, steps=200, warmup=20,
               ms_per_step=0.58, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic", config={"workload": "many_blobs_256", "grid": [256] * 3},
               blob_steps_per_s=7e6, step_hbm_fraction=0.17, step_traffic=None,
               roofline=dict(bound="alu", kernel="k_rhs_march", achieved=17.0, peak=39.3, unit="TOP/s",
                             frac=0.43, traffic=None, avg_launch_us=170.0, alg_ops_per_launch=1e9),
               phases=ph,
               cpu_baseline=dict(value=3e6, unit="cell-steps/s", cores=16, kind="oracle", sample="two steps",
                                 cpu_model="x", one_core=dict(value=2e6), all_cores=dict(value=3e6)),
               cpu_samples=dict(plain_fp64_32=dict(value=1.5e7, seconds=0.1, sample="all 10 steps"),
                                scale_512=dict(value=None, sample="not sampled")),
               fp64=dict(value=1e10, ms_per_step=1.4, steps=50, step_hbm_fraction=0.14),
               ensemble=dict(replicas=96, cells=12976128, batched=dict(ms_per_step=1.0, value=1.3e10),
                             single=dict(ms_per_step=12.0), speedup_batched_vs_single=12.0),
               scale_512=dict(fp32=dict(ms_per_step=5.7, momentum_drift_rel=1e-9),
                              fp64=dict(ms_per_step=13.8, momentum_drift_rel=1e-18),
                              max_rel_err_v=3e-5, max_rel_err_u=8e-6),
               single_blob_128=dict(vacf=big), convergence=dict(errors=big))
    line = json.dumps(bench.compact_record(out))
    assert len(line) < 4096
    c = json.loads(line)
    for k in ("metric", "value", "unit", "steps", "warmup", "ms_per_step", "dtype", "config", "roofline",
              "cpu_baseline"):
        assert k in c, k
    assert c["config"]["workload"] == "many_blobs_256"
    assert c["cpu_baseline"]["cores"] == 16 and c["cpu_baseline"]["kind"] == "oracle"
    assert c["ensemble"]["batched_ms_per_step"] == 1.0 and c["scale_512"]["max_rel_err_v"] == 3e-5
    assert c["cpu_samples"] == {"plain_fp64_32": 1.5e7, "scale_512": None}
