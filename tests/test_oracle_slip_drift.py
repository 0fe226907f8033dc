"""Pins of the oracle's slip correction and thermal drift (CPU).

These terms enter the step only where the excess mass is non-zero or the
temperature is positive, and their coefficients (nu dt/2, m~_f/m~) are
invisible at rho = 1, m_e = 0 or kT = 0. The pins here run at rho != 1,
eta != 1, m_e != 0 and check what the paper fixes:

* App. C: the approximate solve of the inertial correction leaves a slip
  u^{n+1} - J v^{n+1} - Delta-u^{n+1/2} equal to
  -(nu dt/2)(J L dv^{n+1/2} - J L dv^{n-1/2}) up to the error of the
  effective-mass approximation, Eq. (rho_eff_inv_discrete). For one blob
  that error has the closed form (m_e/(rho m~)) K ((m~_f/rho) K - I) dp with
  K = J P S, and dp follows from u^{n+1} - u^n. So the residual is an exact
  identity that fixes the slip coefficient, the lagged J L dv and the FULL
  term's sign at round-off.
* Eq. (delta_u_nph): J interpolates locally linear fields exactly (moment
  conditions of Eq. (JS_invariance)), so on a shear flow the FULL centring
  term is the shear rate times the blob's midpoint displacement.
* App. C: with the viscous slip correction the scheme is second order for
  m_e != 0; without it, first order at small dt (Sec. III.D convergence test).
* App. B.2, Eq. (thermal_drift): the drift force is kT (m~_f/m~) times the
  random finite difference eps^-1 [S(q + eps W) - S(q)] W averaged over
  W ~ N(0, I), estimated here by Monte Carlo from the (separately pinned)
  spreading operator alone.
"""
import numpy as np
import pytest

from oracle import icm


def _smooth_field(p, amp, seed):
    """A divergence-free field with a few low modes (projected noise)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((3,) + tuple(reversed(p.n)))
    wh = icm.fft_field(w)
    _, _, L = icm.symbols(p)
    wh *= np.exp(0.5 * L)                  # damp the high modes
    return amp * icm.ifft_field(p, icm.project_hat(p, wh))


def _slip_expected(p, lag_c, Jn_vn, Jh_vn):
    """delta-u^{n+1/2} written from Eqs. (delta_u_nph) and (delta_u_nph_visc)."""
    nu = p.eta / p.rho
    du = np.zeros(3)
    if p.slip == icm.SLIP_FULL:
        du = du + (Jh_vn - Jn_vn)
    if p.slip in (icm.SLIP_VISCOUS, icm.SLIP_FULL):
        du = du + 0.5 * nu * p.dt * lag_c
    return du


@pytest.mark.parametrize("kernel", [3, 4])
@pytest.mark.parametrize("slip", [icm.SLIP_NONE, icm.SLIP_VISCOUS, icm.SLIP_FULL])
@pytest.mark.parametrize("ratio", [1.0, -0.4, 3.0])
def test_no_slip_residual_of_the_inertial_correction(kernel, slip, ratio):
    """App. C: u^{n+1} - J v^{n+1} - delta-u + (nu dt/2) J L dv^{n+1/2} equals
    (m_e/(rho m~)) K ((m~_f/rho) K - I) dp for one blob, exactly; checked over
    two steps, the second using the lagged term the first stored."""
    p = icm.Params(n=(16, 16, 16), kernel=kernel, rho=1.7, eta=0.6, dt=0.4, slip=slip)
    me = ratio * p.m_f
    mt = me + p.mt_f
    q0 = np.array([[7.3, 8.9, 6.2]])
    st = icm.new_state(p, q0, m_e=[me], f_const=[[0.01, -0.004, 0.006]])
    st.v = _smooth_field(p, 0.02, seed=3)
    st.u = icm.interp(p, st.v, st.q) + np.array([[0.003, -0.002, 0.001]])
    st.lag_c = np.array([[0.05, -0.03, 0.04]])
    nu = p.eta / p.rho
    for _ in range(2):
        Jn = icm.interp(p, st.v, st.q)[0]
        qh = st.q + 0.5 * p.dt * Jn
        Jh = icm.interp(p, st.v, qh)[0]
        out = icm.step(p, st)
        du = _slip_expected(p, st.lag_c[0], Jn, Jh)
        K = icm.jps_matrix(p, qh)
        c5 = p.mt_f / (p.rho * mt)
        # u^{n+1} - u^n = -(I/m_e - c5 K) dp  (steps 4, 5 and 8)
        dp = -np.linalg.solve(np.eye(3) / me - c5 * K, out.u[0] - st.u[0])
        lhs = out.u[0] - icm.interp(p, out.v, qh)[0] - du + 0.5 * nu * p.dt * out.lag_c[0]
        rem = (me / (p.rho * mt)) * (K @ ((p.mt_f / p.rho) * K - np.eye(3))) @ dp
        scale = np.max(np.abs(out.u[0]))
        assert np.max(np.abs(lhs - rem)) < 1e-12 * scale
        # the slip itself is small: the effective-mass remainder is a few
        # percent of dp / m~ (translational invariance of J P S)
        assert np.max(np.abs(rem)) < 0.1 * np.max(np.abs(dp)) / abs(mt)
        st = out


@pytest.mark.parametrize("kernel", [3, 4])
def test_full_slip_term_on_a_shear_flow(kernel):
    """Eq. (delta_u_nph): with v_x = gamma (y - y0) around the blob and a
    uniform v_y = U, J is exact on the linear profile, so
    (J^{n+1/2} - J^n) v^n = (gamma dt U / 2, 0, 0)."""
    p = icm.Params(n=(16, 20, 12), kernel=kernel, rho=1.3, eta=0.7, dt=0.5, slip=icm.SLIP_FULL)
    gamma, U, y0 = 0.004, 0.03, 10.0
    y = (np.arange(p.n[1]) + 0.5) * p.h
    st = icm.new_state(p, [[5.2, 9.7, 6.4]], m_e=[2.0 * p.m_f])
    st.v[0] = gamma * (y - y0)[None, :, None]
    st.v[1] = U
    tr = {}
    icm.step(p, st, trace=tr)
    assert tr["du"][0] == pytest.approx([gamma * p.dt * U / 2.0, 0.0, 0.0], abs=1e-16)


def _trajectory(dt, slip, ratio, slip_fn=None):
    p = icm.Params(n=(16, 16, 16), kernel=3, rho=2.0, dt=dt, spring_k=0.01, slip=slip)
    st = icm.new_state(p, [[10.0, 0.3, 0.2]], m_e=[ratio * p.m_f])
    out = []
    for _ in range(int(round(80.0 / dt))):
        st = icm.step(p, st)
        out.append(st.q[0].copy())
    return np.array(out)


def _orders(slip, ratio=1.0):
    ts = {dt: _trajectory(dt, slip, ratio) for dt in (2.0, 1.0, 0.5, 0.25)}
    E = [np.mean(np.linalg.norm(ts[a] - ts[a / 2][1::2], axis=1)) for a in (2.0, 1.0, 0.5)]
    return [np.log2(E[i] / E[i + 1]) for i in range(2)]


def test_viscous_slip_restores_second_order():
    """Sec. III.D spring test (x0 = 10, k = 0.01, T = 80) at rho = 2 and
    m_e = m_f: the viscous slip correction keeps the scheme second order
    (App. C: slip O(m_e dt^2)); without it the order drops towards one."""
    visc = _orders(icm.SLIP_VISCOUS)
    none = _orders(icm.SLIP_NONE)
    assert min(visc) > 1.9, visc
    assert none[-1] < 1.75, none


def _random_finite_difference(p, q, n_samples, seed):
    """Monte Carlo estimate of E_W[ eps^-1 (S(q + eps W) - S(q)) W ] for one
    blob, with antithetic pairs (S(q + eps W) - S(q - eps W)) / (2 eps),
    computed from the spreading operator alone."""
    rng = np.random.default_rng(seed)
    eps = 1e-4 * p.h
    acc = icm.zero_field(p)
    done = 0
    while done < n_samples:
        m = min(10000, n_samples - done)
        W = rng.standard_normal((m, 3))
        acc += icm.spread(p, W, q + eps * W) - icm.spread(p, W, q - eps * W)
        done += m
    return acc / (2.0 * eps * n_samples)


@pytest.mark.parametrize("kernel", [3, 4])
@pytest.mark.parametrize("ratio", [0.0, 1.0, -0.5])
def test_thermal_drift_is_the_random_finite_difference(kernel, ratio):
    """App. B.2, Eq. (thermal_drift): the right-hand side of step 2 with the
    drift on minus the same with it off (same noise) is
    kT (m~_f/m~) <eps^-1 [S(q + eps W) - S(q)] W>, at m_e != 0 and rho != 1."""
    p = icm.Params(n=(12, 12, 12), kernel=kernel, rho=1.3, eta=0.8, kT=2e-3, dt=0.3, seed=5)
    q = np.array([[5.37, 6.81, 4.22]])
    st = icm.new_state(p, q, m_e=[ratio * p.m_f])
    st.v = _smooth_field(p, 0.01, seed=4)
    st.u = icm.interp(p, st.v, q)
    on, off = {}, {}
    icm.step(p, st, trace=on)
    icm.step(icm.Params(**{**p.__dict__, "thermal_drift": False}), st, trace=off)
    got = on["rhs"] - off["rhs"]
    mt = ratio * p.m_f + p.mt_f
    est = p.kT * (p.mt_f / mt) * _random_finite_difference(p, on["q_half"], 40000, seed=11)
    rel = np.linalg.norm(got - est) / np.linalg.norm(est)
    assert rel < 0.05, rel
