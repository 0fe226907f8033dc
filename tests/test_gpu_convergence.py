"""GPU runs of the deterministic temporal-convergence test of Sec. III.D
(a blob released from rest in a harmonic potential, Eq. (E_dt_definition)),
through the C ABI in FP64.

Parity: the GPU trajectories at two time steps match the oracle's step by
step. Properties: the observed orders follow the paper's account (second
order for neutrally buoyant blobs; for a heavy blob, second order at the
larger time steps turning towards first order at small ones, the
uncontrolled J P S invariance approximation of the no-slip step).
"""
import numpy as np
import pytest

import icm_inputs
from oracle import icm as O
from tests.parity_cases import banner

pytestmark = pytest.mark.gpu

WL = icm_inputs.WORKLOADS["convergence_16"]


@pytest.fixture(scope="module")
def I():
    import paper_1212_6427_amd.icm as lib
    return lib


def _gpu_runs(I, ratios, dt, k=WL["spring_k"]):
    """Blob position after every step, one replica per excess mass."""
    import bench
    combos = [(r, I.SLIP_VISCOUS) for r in ratios]
    return bench.spring_trajectories(I, None, WL, combos, dt, k)


def _oracle_run(ratio, dt, k=WL["spring_k"]):
    p = O.Params(n=WL["n"], kernel=WL["kernel"], dt=dt, spring_k=k, slip=O.SLIP_VISCOUS)
    st = O.new_state(p, [WL["x0"]], m_e=[ratio * p.m_f])
    out = []
    for _ in range(int(round(WL["T"] / dt))):
        st = O.step(p, st)
        out.append(st.q[0].copy())
    return np.array(out)


@pytest.mark.parametrize("ratio,dt", [(0.0, 2.0), (1.0, 2.0), (10.0, 2.0), (0.0, 1.0), (10.0, 1.0),
                                      (-0.5, 0.5), (-0.5, 0.25)])
def test_spring_trajectories_match_oracle(I, ratio, dt):
    banner("spring trajectory m_e/m_f=%g dt=%g" % (ratio, dt))
    got = _gpu_runs(I, (ratio,), dt)[0]
    ref = _oracle_run(ratio, dt)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref - np.asarray(WL["x0"])))
    print("relative error %.2e" % err, flush=True)
    assert err < 1e-11


def test_light_blob_at_a_large_step_raises_the_numeric_flag(I):
    """With m_e = -m_f/2 and dt = 2 the step is unstable (the oracle's blob
    moves more than h in one step); the GPU run must stop with
    ICM_E_NUMERIC rather than return garbage."""
    import bench
    banner("numeric flag on the unstable light blob")
    got = bench.spring_trajectories(I, None, WL, [(-0.5, I.SLIP_VISCOUS)], 2.0, WL["spring_k"])
    assert np.all(np.isnan(got))
    ref = _oracle_run(-0.5, 2.0)
    assert np.max(np.abs(np.diff(ref, axis=0))) > 1.0


def _orders(E):
    return np.log2(E[:-1] / E[1:])


def test_observed_orders_follow_the_paper(I):
    import bench
    dts = (2.0, 1.0, 0.5, 0.25, 0.125, 0.0625, 0.03125)
    banner("convergence orders")
    E = bench.convergence_errors(I, None, WL,
                                 [(0.0, I.SLIP_VISCOUS), (10.0, I.SLIP_VISCOUS)], dts, WL["spring_k"])
    o0, o10 = _orders(E[0]), _orders(E[1])
    print("E(m_e=0):", E[0], "orders", o0, flush=True)
    print("E(m_e=10 m_f):", E[1], "orders", o10, flush=True)
    assert np.all(o0 > 1.8)
    assert np.all(o10[:2] > 1.9)
    assert o10[-1] < 1.6
