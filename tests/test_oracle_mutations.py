"""Planted mistakes in the oracle must be caught by its pins.

Each case monkeypatches one plausible error into the oracle (on the CPU) and
checks that the named pin test then fails. This guards against pins that
would pass whatever the oracle computed.
"""
import numpy as np
import pytest

from oracle import icm
import tests.test_oracle_pins as pins


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_wrong_divergence_symbol_sign(monkeypatch):
    orig = icm.symbols

    def bad(p):
        D, G, L = orig(p)
        return [-d for d in D], G, -L
    monkeypatch.setattr(icm, "symbols", bad)
    assert _fails(pins.test_helmholtz_solve_real_space_residual)


def test_transposed_gradient_symbol(monkeypatch):
    orig = icm.symbols

    def bad(p):
        D, G, L = orig(p)
        return D, [np.conj(g) for g in G], L
    monkeypatch.setattr(icm, "symbols", bad)
    assert _fails(pins.test_projection_divergence_idempotence_mean)


def test_noise_diagonal_without_factor_two(monkeypatch):
    orig = icm.philox.stress_normals

    def bad(n, step, seed, replica):
        W = orig(n, step, seed, replica)
        for k in ("xx", "yy", "zz"):
            W[k] = W[k] / 2.0 * np.sqrt(2.0)   # variance 2 instead of 4
        return W
    monkeypatch.setattr(icm.philox, "stress_normals", bad)
    assert _fails(pins.test_noise_one_step_variance_closed_form)


def test_noise_amplitude_missing_dt(monkeypatch):
    monkeypatch.setattr(icm.Params, "noise_amplitude",
                        property(lambda self: np.sqrt(self.kT * self.eta / self.cell_volume)))
    assert _fails(pins.test_equilibrium_is_preserved_by_the_fluctuating_step)


def test_step5_coefficient_uses_m_f_not_mt_f(monkeypatch):
    monkeypatch.setattr(icm.Params, "mt_f", property(lambda self: self.m_f))
    assert _fails(pins.test_inviscid_impulse_gives_effective_mass, 1.0)


def test_dropped_g_term_breaks_momentum(monkeypatch):
    orig = icm.helmholtz_project
    calls = {"n": 0}

    def bad(p, rhs, a, b):
        calls["n"] += 1
        out = orig(p, rhs, a, b)
        return out * (1.0 if a != p.rho else 1.1)   # perturb the dv solve
    monkeypatch.setattr(icm, "helmholtz_project", bad)
    assert _fails(pins.test_momentum_conserved_exactly, icm.SLIP_VISCOUS)


def test_laplacian_missing_one_axis(monkeypatch):
    def bad(p, v):
        out = np.zeros_like(v)
        for a in range(3):
            for b in range(2):
                out[a] += icm.shift(v[a], b, 1) - 2.0 * v[a] + icm.shift(v[a], b, -1)
        return out / p.h ** 2
    monkeypatch.setattr(icm, "laplacian", bad)
    assert _fails(pins.test_single_shear_mode_decay_closed_form) or \
        _fails(pins.test_helmholtz_solve_real_space_residual)


def test_wrong_face_offset_in_interp(monkeypatch):
    orig = icm._component_weights

    def bad(p, q, alpha, deriv_axis=None):
        return orig(p, q + 0.5 * (alpha == 0) * np.array([[1.0, 0, 0]]), alpha, deriv_axis)
    monkeypatch.setattr(icm, "_component_weights", bad)
    assert _fails(pins.test_interp_brute_force_single_node)


def test_wca_force_sign(monkeypatch):
    orig = icm.wca_forces
    monkeypatch.setattr(icm, "wca_forces", lambda p, q: -orig(p, q))
    assert _fails(pins.test_wca_force_is_minus_gradient_of_potential)


def test_thermal_drift_sign(monkeypatch):
    orig = icm.dphi3
    monkeypatch.setattr(icm, "dphi3", lambda r: -orig(r))
    assert _fails(pins.test_kernel_derivative_matches_finite_difference, 3)


def test_advection_edge_average_on_the_wrong_side(monkeypatch):
    def bad(p, v):
        A = np.zeros_like(v)
        for a in range(3):
            for b in range(3):
                if a == b:
                    c = 0.5 * (v[a] + icm.shift(v[a], a, 1))
                    F = p.rho * c * c
                    A[a] += (F - icm.shift(F, a, -1)) / p.h
                else:
                    vb = 0.5 * (v[b] + icm.shift(v[b], a, 1))   # should average towards -e_a
                    va = 0.5 * (v[a] + icm.shift(v[a], b, -1))
                    F = p.rho * vb * va
                    A[a] += (icm.shift(F, b, 1) - F) / p.h
        return A
    monkeypatch.setattr(icm, "advection", bad)
    assert _fails(pins.test_advection_conserves_momentum_and_energy)
    assert _fails(pins.test_advection_converges_to_v_grad_v_for_the_abc_flow)


def test_advection_missing_density(monkeypatch):
    orig = icm.advection
    monkeypatch.setattr(icm, "advection", lambda p, v: orig(p, v) / p.rho)
    assert _fails(pins.test_advection_of_a_shear_mode_by_a_uniform_flow, 0, 1)


def test_advection_without_the_lagged_term(monkeypatch):
    orig = icm.step

    def euler(p, st):
        st = st.copy()
        st.adv_prev = None
        return orig(p, st)
    monkeypatch.setattr(icm, "step", euler)
    assert _fails(pins.test_advection_adams_bashforth_is_second_order)


# ------------------------------------------------------------ split kernel
import tests.test_oracle_split as split_pins


def test_split_kernel_both_copies_shifted_one_way(monkeypatch):
    monkeypatch.setattr(icm, "split_phi3",
                        lambda r, s: 0.5 * (icm.phi3(np.asarray(r) - 0.5 * s) + icm.phi3(np.asarray(r) - 0.5 * s)))
    assert _fails(split_pins.test_unity_and_first_moment_at_every_position, 0.5)


def test_split_kernel_without_the_half(monkeypatch):
    monkeypatch.setattr(icm, "split_phi3",
                        lambda r, s: icm.phi3(np.asarray(r) - 0.5 * s) + icm.phi3(np.asarray(r) + 0.5 * s))
    assert _fails(split_pins.test_unity_and_first_moment_at_every_position, 0.5)


def test_split_blob_volume_without_the_cross_term(monkeypatch):
    monkeypatch.setattr(icm, "phi3_autocorrelation", lambda s: 0.5)
    assert _fails(split_pins.test_blob_volume_is_the_position_average, 0.5)


def test_split_kernel_on_the_three_node_layout(monkeypatch):
    orig = icm.kernel_of

    def bad(p):
        phi, dphi, layout = orig(p)
        return phi, dphi, 3
    monkeypatch.setattr(icm, "kernel_of", bad)
    assert _fails(split_pins.test_interp_of_a_locally_linear_field_is_exact)


# --------------------------------------------- slip correction, thermal drift
import tests.test_oracle_slip_drift as slip_pins


def _slip_with(viscous_coef=None, full_sign=1.0):
    """A slip_correction with a planted mistake in one of its two terms."""
    def bad(p, lag_c, Jn_vn, Jh_vn):
        du = np.zeros_like(np.asarray(lag_c, dtype=np.float64))
        if p.slip == icm.SLIP_FULL:
            du += full_sign * (Jh_vn - Jn_vn)
        if p.slip in (icm.SLIP_VISCOUS, icm.SLIP_FULL):
            c = 0.5 * (p.eta / p.rho) * p.dt if viscous_coef is None else viscous_coef(p)
            du += c * lag_c
        return du
    return bad


def test_viscous_slip_with_eta_dt_instead_of_half_nu_dt(monkeypatch):
    monkeypatch.setattr(icm, "slip_correction", _slip_with(viscous_coef=lambda p: p.eta * p.dt))
    assert _fails(slip_pins.test_no_slip_residual_of_the_inertial_correction, 3, icm.SLIP_VISCOUS, 1.0)
    assert _fails(slip_pins.test_viscous_slip_restores_second_order)


def test_lagged_term_without_the_laplacian(monkeypatch):
    monkeypatch.setattr(icm, "lagged_viscous_term", lambda p, dv, q_h: icm.interp(p, dv, q_h))
    assert _fails(slip_pins.test_no_slip_residual_of_the_inertial_correction, 4, icm.SLIP_VISCOUS, 1.0)
    assert _fails(slip_pins.test_viscous_slip_restores_second_order)


def test_full_slip_term_with_the_wrong_sign(monkeypatch):
    monkeypatch.setattr(icm, "slip_correction", _slip_with(full_sign=-1.0))
    assert _fails(slip_pins.test_no_slip_residual_of_the_inertial_correction, 3, icm.SLIP_FULL, 1.0)
    assert _fails(slip_pins.test_full_slip_term_on_a_shear_flow, 4)


def test_thermal_drift_coefficient_with_the_wrong_sign(monkeypatch):
    orig = icm.thermal_drift_coef

    def bad(p, m_e):
        c = orig(p, m_e)
        return None if c is None else -c
    monkeypatch.setattr(icm, "thermal_drift_coef", bad)
    assert _fails(slip_pins.test_thermal_drift_is_the_random_finite_difference, 3, 0.0)


def test_thermal_drift_coefficient_without_the_mass_ratio(monkeypatch):
    def bad(p, m_e):
        if p.kT == 0.0 or not p.thermal_drift:
            return None
        return p.kT * np.ones_like(np.asarray(m_e, dtype=np.float64))
    monkeypatch.setattr(icm, "thermal_drift_coef", bad)
    assert _fails(slip_pins.test_thermal_drift_is_the_random_finite_difference, 4, 1.0)
    assert _fails(slip_pins.test_thermal_drift_is_the_random_finite_difference, 3, -0.5)
