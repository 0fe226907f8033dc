"""Oracle parity of the register-resident FFT plans of length 128 and 512.

The fast path needs a plan on all three axes. Each grid below puts 128 on
one axis and 512 on another, and the three grids rotate them, so every
pass (x forward and inverse, y forward and inverse, and the z pass with the
Helmholtz solve and projection) runs both lengths. FP32 runs both z plans
(eight and sixteen values per thread). The last case is the 128^3
fluctuating single-blob workload: one 4-point blob with m_e = m_f, FP32
grid, from the discrete equilibrium.
"""
import numpy as np
import pytest

from oracle import icm as O
from tests.parity_cases import banner, compare, gpu_params, initial_state, load_into_gpu, oracle_params

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 2e-5
SHAPES = [(512, 16, 128), (128, 512, 16), (16, 128, 512)]


@pytest.fixture(scope="module")
def I():
    import paper_1212_6427_amd.icm as lib
    return lib


def _case(n, seed):
    p = oracle_params(n, kernel=4, kT=1e-3, dt=0.25, seed=seed, wca_eps=1e-2, wca_sigma=2.0 / 2 ** (1 / 6))
    st = initial_state(p, 6, (0.0, 1.0, -0.5), seed=seed + 1, min_sep=2.2)
    return p, st


def _run(I, p, st, steps, prec, shapes=None):
    dtype = np.float64 if prec == I.FP64 else np.float32
    sim = I.Sim([gpu_params(I, p)], [max(st.q.shape[0], 1)], prec)
    try:
        load_into_gpu(I, sim, 0, st, dtype)
        if shapes is not None:
            sim.set_fft_shapes([shapes])
        sim.step(steps)
        return sim.get_state(0)
    finally:
        sim.close()


@pytest.mark.parametrize("n", SHAPES)
def test_fast_plans_128_and_512_fp64(I, n):
    p, st = _case(n, seed=200 + n[0] // 16)
    banner("fast plans fp64 n=%s" % (n,))
    got = _run(I, p, st, 3, I.FP64)
    ref = O.run(p, st, 3)
    errs, bad = compare(got, ref, st.q, TOL64)
    print("errors:", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    assert not bad, bad


@pytest.mark.parametrize("z_small_plan", [1, 0])
@pytest.mark.parametrize("n", SHAPES)
def test_fast_plans_128_and_512_fp32(I, n, z_small_plan):
    p, st = _case(n, seed=230 + n[0] // 16)
    st.v = st.v.astype(np.float32).astype(np.float64)
    banner("fast plans fp32 n=%s z_small_plan=%d" % (n, z_small_plan))
    shapes = dict(n=n, y_columns=16, z_columns=16, z_small_plan=z_small_plan, x_threads=256)
    got = _run(I, p, st, 1, I.FP32_GRID, shapes)
    ref = O.step(p, st)
    errs, bad = compare(got, ref, st.q, TOL32)
    print("errors:", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    assert not bad, bad


def test_single_blob_128_fp32(I):
    """The 128^3 fluctuating single-blob workload, one step, m_e = m_f."""
    p = oracle_params((128, 128, 128), kernel=4, kT=1e-3, dt=0.25, seed=251)
    st = initial_state(p, 1, (1.0,), seed=252)
    st.v = st.v.astype(np.float32).astype(np.float64)
    banner("single blob 128^3 fp32")
    got = _run(I, p, st, 1, I.FP32_GRID)
    ref = O.step(p, st)
    errs, bad = compare(got, ref, st.q, TOL32)
    print("errors:", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    assert not bad, bad


# ------------------------------------------- the benchmark's 256 x 256 planes
# The x and y passes of the 256^3 benchmark (FP32), with a short z axis so
# that the oracle stays cheap.
@pytest.mark.parametrize("n", [(256, 256, 16), (256, 256, 48)])
def test_256_planes_fp32(I, n):
    p, st = _case(n, seed=260 + n[2])
    st.v = st.v.astype(np.float32).astype(np.float64)
    banner("256 planes fp32 n=%s" % (n,))
    got = _run(I, p, st, 1, I.FP32_GRID)
    ref = O.step(p, st)
    errs, bad = compare(got, ref, st.q, TOL32)
    print("errors:", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    assert not bad, bad


def test_256_planes_kick_and_projection_fp32(I):
    """The inverse x pass adding to the field (the t = 0 impulse of
    ICM_BLOBS_KICK) and the projection initialiser on 256 x 256 planes. The
    projected base field is small (max ~0.05) and the impulse of order one,
    so both a lost base and a wrong impulse exceed the tolerance."""
    from tests.parity_cases import rel_err
    import icm_inputs
    n = (256, 256, 16)
    p = oracle_params(n, kernel=3, kT=0.0, dt=0.2, seed=271)
    q = icm_inputs.separated_positions(3, n, min_sep=4.0, seed=272)
    u0 = icm_inputs.random_forces(3, seed=273, scale=0.5)
    w = icm_inputs.random_field(n, seed=274, scale=0.01).astype(np.float32).astype(np.float64)
    banner("256 planes kick and projection fp32")
    sim = I.Sim([gpu_params(I, p)], [3], I.FP32_GRID)
    try:
        sim.set_state(0, v=w.astype(np.float32), flags=I.STATE_PROJECT)
        pw = O.project(p, w)
        got = sim.get_state(0)["v"]
        assert rel_err(got, pw) < TOL32
        sim.set_blobs(0, q, u0, flags=I.BLOBS_KICK)
        got = sim.get_state(0)["v"]
        kick = O.kick_field(p, q, u0, np.zeros(3))
        assert np.max(np.abs(kick)) > 10 * np.max(np.abs(pw))
        assert rel_err(got, pw + kick) < TOL32
    finally:
        sim.close()
