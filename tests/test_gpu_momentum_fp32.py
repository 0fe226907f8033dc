"""Total momentum in the FP32-grid mode over a long run.

Sec. II (after Eq. (no_slip)) and App. C: every step changes the total
momentum rho dV_f sum v + sum m_e u by exactly dt (sum_i F_i + V f_body).
In the FP32-grid mode the fluid's share, the k = 0 mode, is carried in FP64:
the diagnostics must follow the exact change at FP64 round-off for 1000
steps, and the FP32 field as stored must stay within its storage rounding of
the carried value, with no growth over the run.
"""
import numpy as np
import pytest

from tests.parity_cases import banner, gpu_params, initial_state, load_into_gpu, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def I():
    import paper_1212_6427_amd.icm as lib
    return lib


def test_fp32_momentum_follows_the_exact_change_for_1000_steps(I):
    n = (64, 64, 64)
    p = oracle_params(n, kernel=4, kT=1e-3, dt=0.25, seed=301, body=(2e-5, -1e-5, 3e-5))
    st = initial_state(p, 8, (0.0, 1.0, -0.5, 2.0), seed=302, min_sep=4.0, force_scale=0.02)
    st.v = st.v.astype(np.float32).astype(np.float64)
    vol = float(np.prod(n)) * p.h ** 3
    dP = p.dt * (st.f_const.sum(axis=0) + vol * np.asarray(p.body_force))
    banner("fp32 momentum over 1000 steps")
    sim = I.Sim([gpu_params(I, p)], [8], I.FP32_GRID)
    try:
        load_into_gpu(I, sim, 0, st, np.float32)
        got = sim.get_state(0)
        P0 = np.asarray(got["diag"]["momentum"])
        done, drift, stored = 0, [], []
        for k in (1, 10, 100, 300, 600, 1000):
            sim.step(k - done, I.STEP_GRAPH)
            done = k
            got = sim.get_state(0)
            P = np.asarray(got["diag"]["momentum"])
            expect = P0 + k * dP
            scale = np.max(np.abs(P0)) + k * np.max(np.abs(dP))
            drift.append(np.max(np.abs(P - expect)) / scale)
            # the stored FP32 field summed in FP64, plus the blobs' share
            v = got["v"].astype(np.float64)
            Pf = p.rho * p.h ** 3 * v.sum(axis=(1, 2, 3)) + (st.m_e[:, None] * got["u"]).sum(axis=0)
            vscale = p.rho * p.h ** 3 * np.abs(v).sum()
            stored.append(np.max(np.abs(Pf - P)) / vscale)
        print("carried momentum vs exact change:", ["%.1e" % x for x in drift])
        print("stored field vs carried:", ["%.1e" % x for x in stored])
        assert max(drift) < 1e-12
        # storage rounding of the field (its mean rounded to FP32 each step,
        # ~1e-9 here), not a drift growing with the steps (measured without
        # the FP64 carry: 3.5e-7 after 200 steps at 512^3)
        assert max(stored) < 2e-8
    finally:
        sim.close()
