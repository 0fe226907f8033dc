"""Shared set-up of parity cases: the same seeded inputs are handed to the
oracle and, through the C ABI, to the HIP library. Nothing here computes the
method: inputs come from icm_inputs, expected values from oracle/."""
import sys

import numpy as np

import icm_inputs
from oracle import icm as O


def banner(msg):
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def oracle_params(n, kernel=4, kT=0.0, dt=0.2, slip=O.SLIP_VISCOUS, drift=True, seed=7, replica=0, h=1.0, rho=1.0,
                  eta=1.0, body=(0.0, 0.0, 0.0), wca_eps=0.0, wca_sigma=0.0, spring_k=0.0, spring_c=(0.0, 0.0, 0.0),
                  advection=False, kernel_shift=0.0):
    return O.Params(n=tuple(n), h=h, rho=rho, eta=eta, kT=kT, dt=dt, kernel=kernel, slip=slip, thermal_drift=drift,
                    seed=seed, replica=replica, body_force=tuple(body), wca_eps=wca_eps, wca_sigma=wca_sigma,
                    spring_k=spring_k, spring_center=tuple(spring_c), advection=advection,
                    kernel_shift=kernel_shift)


def gpu_params(I, p):
    return I.make_params(p.n, h=p.h, rho=p.rho, eta=p.eta, kT=p.kT, dt=p.dt, kernel=p.kernel, slip=p.slip,
                         thermal_drift=p.thermal_drift, seed=p.seed, replica_id=p.replica,
                         body_force=p.body_force, wca_eps=p.wca_eps, wca_sigma=p.wca_sigma,
                         spring_k=p.spring_k, spring_center=p.spring_center, advection=p.advection,
                         kernel_shift=p.kernel_shift)


def initial_state(p, nb, me_ratios=(0.0,), seed=0, min_sep=3.0, force_scale=0.01, velocity_field_scale=None):
    """Seeded blobs plus an initial fluid field.

    The field is an oracle-generated equilibrium sample (kT > 0) or a
    projected random field scaled by velocity_field_scale; either way the GPU
    receives it as input data.
    """
    if nb:
        q = icm_inputs.separated_positions(nb, p.n, p.h, min_sep=min_sep, seed=seed)
    else:
        q = np.zeros((0, 3))
    me = np.resize(np.asarray(me_ratios, dtype=np.float64), nb) * p.m_f
    F = icm_inputs.random_forces(nb, seed=seed + 1, scale=force_scale)
    st = O.new_state(p, q, m_e=me, f_const=F)
    if p.kT > 0:
        st.v = O.equilibrium_field(p)
    elif velocity_field_scale:
        st.v = O.project(p, icm_inputs.random_field(p.n, seed=seed + 2, scale=velocity_field_scale))
    if nb:
        st.u = O.interp(p, st.v, st.q) + icm_inputs.random_forces(nb, seed=seed + 3, scale=1e-3) * (me != 0)[:, None]
    return st


def load_into_gpu(I, sim, replica, st, dtype):
    sim.set_blobs(replica, st.q, st.u, st.m_e, st.f_const)
    sim.set_state(replica, v=st.v.astype(dtype), lag_c=st.lag_c, step=st.step)


def rel_err(a, b):
    """Max element error relative to the largest magnitude of the reference."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.max(np.abs(b))
    if scale == 0.0:
        return float(np.max(np.abs(a)))
    return float(np.max(np.abs(a - b)) / scale)


def norm_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def compare(gpu, ref, prev_q, tol):
    """Per-component field errors and blob displacement/velocity errors."""
    errs = {}
    for a in range(3):
        errs["v%d" % a] = rel_err(gpu["v"][a], ref.v[a])
    if ref.q.shape[0]:
        errs["dq"] = rel_err(gpu["q"] - prev_q, ref.q - prev_q)
        errs["u"] = rel_err(gpu["u"], ref.u)
        if np.any(ref.lag_c != 0):
            errs["lag"] = rel_err(gpu["lag_c"], ref.lag_c)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    return errs, bad
