"""Split (shifted) three-point kernel of Sec. III.A.2 on the GPU, against the
oracle, through the C ABI.

FP64 steps with the split kernel (thermal drift on, mixed excess masses,
non-unit constants) within 1e-11; one FP32 step within 2e-5; a context
mixing shifts, the plain three-point and the four-point kernel on one grid
shape (the split and four-point replicas share launches, each with its own
shift); the steady mobility against the oracle's spectral Stokes solve; and
the hydrodynamic radius growing with the shift.
"""
import numpy as np
import pytest

from oracle import icm as O
from tests.parity_cases import banner, compare, gpu_params, initial_state, load_into_gpu, oracle_params

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 2e-5


@pytest.fixture(scope="module")
def I():
    import paper_1212_6427_amd.icm as lib
    return lib


def _run(I, cases, states, steps, prec, tol, name):
    dtype = np.float64 if prec == I.FP64 else np.float32
    banner("%s: %d replicas, shifts %s, prec %d" % (name, len(cases), [p.kernel_shift for p in cases], prec))
    sim = I.Sim([gpu_params(I, p) for p in cases], [max(st.q.shape[0], 1) for st in states], prec)
    try:
        for r, st in enumerate(states):
            load_into_gpu(I, sim, r, st, dtype)
        sim.step(steps)
        for r, (p, st) in enumerate(zip(cases, states)):
            ref = O.run(p, st, steps)
            got = sim.get_state(r)
            errs, bad = compare(got, ref, st.q, tol)
            print("replica %d shift %g:" % (r, p.kernel_shift), {k: "%.2e" % v for k, v in errs.items()},
                  flush=True)
            assert not bad, (r, bad)
    finally:
        sim.close()


@pytest.mark.parametrize("shift", [0.5, 1.0])
def test_split_kernel_fp64(I, shift):
    p = oracle_params((24, 18, 12), kernel=3, kT=1e-3, dt=0.25, seed=201, h=0.9, rho=1.1, eta=0.8,
                      kernel_shift=shift)
    st = initial_state(p, 4, (0.0, 1.0, -0.5), seed=203, min_sep=3.0)
    _run(I, [p], [st], 3, I.FP64, TOL64, "split fp64")


def test_split_kernel_fp32_one_step(I):
    p = oracle_params((32, 48, 24), kernel=3, kT=1e-3, dt=0.25, seed=211, kernel_shift=0.7)
    st = initial_state(p, 5, (0.0, 2.0), seed=213, min_sep=3.0)
    st.v = st.v.astype(np.float32).astype(np.float64)
    _run(I, [p], [st], 1, I.FP32_GRID, TOL32, "split fp32")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mixed_shifts_and_kernels_in_one_context(I, precision):
    """Shifts 0.3 and 1.0, the plain three-point and the four-point kernel on
    one grid shape (16^3: the spectral form of the inertial correction):
    each replica matches its own oracle run."""
    specs = [(3, 0.3), (3, 1.0), (3, 0.0), (4, 0.0)]
    cases, states = [], []
    for r, (k, s) in enumerate(specs):
        p = oracle_params((16, 16, 16), kernel=k, kT=2e-3, dt=0.2, seed=221, replica=r, kernel_shift=s)
        cases.append(p)
        st = initial_state(p, 3, (0.0, 1.0), seed=230 + r, min_sep=3.0)
        if precision == "fp32":
            st.v = st.v.astype(np.float32).astype(np.float64)
        states.append(st)
    if precision == "fp64":
        _run(I, cases, states, 2, I.FP64, TOL64, "mixed shifts")
    else:
        _run(I, cases, states, 1, I.FP32_GRID, TOL32, "mixed shifts fp32")


def test_split_steady_mobility_matches_oracle(I):
    import bench
    rng = np.random.default_rng(240)
    qs = [rng.uniform(0.0, 16.0, 3) for _ in range(3)]
    banner("split steady mobility")
    mu = bench.mobility_columns(I, None, (16, 16, 16), 3, qs, kernel_shift=0.6)
    p = O.Params(n=(16, 16, 16), kernel=3, kernel_shift=0.6)
    for c, q in enumerate(qs):
        ref = O.mobility_matrix(p, q[None])
        err = np.max(np.abs(mu[c] - ref)) / np.max(np.abs(ref))
        print("q=%s err %.2e" % (q, err), flush=True)
        assert err < 1e-4


def test_hydrodynamic_radius_grows_with_the_shift(I):
    """Sec. III.A.2: widening the kernel by the shift raises the blob's
    hydrodynamic radius smoothly; s = 0 is the three-point kernel's 0.91."""
    import bench
    rng = np.random.default_rng(250)
    qs = [rng.uniform(0.0, 32.0, 3) for _ in range(6)]
    banner("R_H against the shift")
    rh = []
    for s in (0.0, 0.5, 1.0):
        mu = bench.mobility_columns(I, None, (32, 32, 32), 3, qs, kernel_shift=s)
        r = np.array([bench.hydrodynamic_radius(np.trace(m) / 3.0, 32.0) for m in mu])
        print("s=%g: R_H %.4f (%.4f .. %.4f)" % (s, r.mean(), r.min(), r.max()), flush=True)
        rh.append(r.mean())
    assert rh[0] == pytest.approx(0.906, rel=0.02)
    assert rh[0] < rh[1] < rh[2]
