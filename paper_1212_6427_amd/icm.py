"""Thin ctypes binding of the gfx950 ICM library (include/icm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libicm.so. Importing this module fails loudly if the library has not been
built (python -m paper_1212_6427_amd.build); there is no fallback.

Host arrays are numpy arrays; device arrays may be passed as torch tensors
together with PTRS_DEVICE. PyTorch is used only for device memory (the
optional workspace) and streams.

In a process that also uses PyTorch-ROCm, import torch before this module:
torch carries its own copy of the HIP runtime, and libicm.so must bind to
that copy (loaded first, it satisfies libicm's dependency); loaded the other
way round the process ends up with two HIP runtimes, and the second one to
start finds no device.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libicm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libicm.so is not built; run `python -m paper_1212_6427_amd.build` "
                      "(the ICM step has no non-HIP implementation)")

_lib = ctypes.CDLL(LIB_PATH)

# status codes and flags (mirrors include/icm.h)
OK, E_INVALID, E_UNSUPPORTED, E_NOMEM, E_DEVICE, E_STATE, E_NUMERIC = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_GRID = 0, 1
SLIP_NONE, SLIP_VISCOUS, SLIP_FULL = 0, 1, 2
PTRS_DEVICE, BLOBS_KICK, STATE_PROJECT, STATE_EQUILIBRIUM = 1, 2, 4, 8
STEP_GRAPH = 1

_STATUS_NAMES = {OK: "ICM_OK", E_INVALID: "ICM_E_INVALID", E_UNSUPPORTED: "ICM_E_UNSUPPORTED",
                 E_NOMEM: "ICM_E_NOMEM", E_DEVICE: "ICM_E_DEVICE", E_STATE: "ICM_E_STATE",
                 E_NUMERIC: "ICM_E_NUMERIC"}


class icm_replica_params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("kernel", ctypes.c_int32),
        ("h", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("slip", ctypes.c_int32),
        ("thermal_drift", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("replica_id", ctypes.c_uint32),
        ("advection", ctypes.c_uint32),
        ("body_force", ctypes.c_double * 3),
        ("wca_eps", ctypes.c_double),
        ("wca_sigma", ctypes.c_double),
        ("spring_k", ctypes.c_double),
        ("spring_center", ctypes.c_double * 3),
        ("kernel_shift", ctypes.c_double),
    ]


class icm_diag(ctypes.Structure):
    _fields_ = [
        ("momentum", ctypes.c_double * 3),
        ("ke_fluid", ctypes.c_double),
        ("ke_blob", ctypes.c_double),
        ("max_div", ctypes.c_double),
        ("max_alpha", ctypes.c_double),
        ("step", ctypes.c_int64),
    ]


class icm_timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 16), ("launches", ctypes.c_int64 * 16)]


class icm_tune_result(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("y_columns", ctypes.c_int32),
        ("z_columns", ctypes.c_int32),
        ("z_small_plan", ctypes.c_int32),
        ("x_threads", ctypes.c_int32),
        ("tuned", ctypes.c_int32),
        ("rhs_z_chunk", ctypes.c_int32),
        ("us_default", ctypes.c_double),
        ("us_tuned", ctypes.c_double),
        ("us_rhs_default", ctypes.c_double),
        ("us_rhs_tuned", ctypes.c_double),
    ]


PHASES = ["gather", "blob", "forces", "rhs", "spread", "fft_x_fwd", "fft_y_fwd", "fft_z_solve", "fft_y_inv",
          "fft_x_inv", "field_ops", "advection"]

_p = ctypes.c_void_p
_lib.icm_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.POINTER(icm_replica_params),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_size_t)]
_lib.icm_workspace_bytes.restype = ctypes.c_int
_lib.icm_create.argtypes = [ctypes.c_int32, ctypes.POINTER(icm_replica_params), ctypes.POINTER(ctypes.c_int32),
                            ctypes.c_int32, _p, ctypes.c_size_t, _p, ctypes.POINTER(_p)]
_lib.icm_create.restype = ctypes.c_int
_lib.icm_set_blobs.argtypes = [_p, ctypes.c_int32, ctypes.c_int32, _p, _p, _p, _p, ctypes.c_uint32]
_lib.icm_set_blobs.restype = ctypes.c_int
_lib.icm_set_state.argtypes = [_p, ctypes.c_int32, _p, _p, _p, _p, ctypes.c_int64, ctypes.c_uint32]
_lib.icm_set_state.restype = ctypes.c_int
_lib.icm_autotune.argtypes = [_p, ctypes.POINTER(icm_tune_result), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
_lib.icm_autotune.restype = ctypes.c_int
_lib.icm_set_fft_shapes.argtypes = [_p, ctypes.POINTER(icm_tune_result), ctypes.c_int32]
_lib.icm_set_fft_shapes.restype = ctypes.c_int
_lib.icm_step.argtypes = [_p, ctypes.c_int64, ctypes.c_uint32]
_lib.icm_step.restype = ctypes.c_int
_lib.icm_get_state.argtypes = [_p, ctypes.c_int32, _p, _p, _p, _p, ctypes.POINTER(icm_diag), ctypes.c_uint32]
_lib.icm_get_state.restype = ctypes.c_int
_lib.icm_get_advection_lag.argtypes = [_p, ctypes.c_int32, _p, ctypes.POINTER(ctypes.c_int32), ctypes.c_uint32]
_lib.icm_get_advection_lag.restype = ctypes.c_int
_lib.icm_set_advection_lag.argtypes = [_p, ctypes.c_int32, _p, ctypes.c_uint32]
_lib.icm_set_advection_lag.restype = ctypes.c_int
_lib.icm_num_blobs.argtypes = [_p, ctypes.c_int32]
_lib.icm_num_blobs.restype = ctypes.c_int32
_lib.icm_set_timing.argtypes = [_p, ctypes.c_int32]
_lib.icm_set_timing.restype = ctypes.c_int
_lib.icm_get_timing.argtypes = [_p, ctypes.POINTER(icm_timing), ctypes.c_int32]
_lib.icm_get_timing.restype = ctypes.c_int
_lib.icm_solve_noalloc.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int32, _p, _p, _p]
_lib.icm_solve_noalloc.restype = ctypes.c_int
_lib.icm_destroy.argtypes = [_p]
_lib.icm_destroy.restype = None
_lib.icm_last_error.argtypes = [_p]
_lib.icm_last_error.restype = ctypes.c_char_p


class ICMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, status), msg))
        self.status = status


def _check(status, ctx=None):
    if status != OK:
        raise ICMError(status, _lib.icm_last_error(ctx).decode())


def make_params(n, h=1.0, rho=1.0, eta=1.0, kT=0.0, dt=0.1, kernel=3, slip=SLIP_VISCOUS, thermal_drift=True,
                seed=0, replica_id=0, body_force=(0.0, 0.0, 0.0), wca_eps=0.0, wca_sigma=0.0, spring_k=0.0,
                spring_center=(0.0, 0.0, 0.0), advection=False, kernel_shift=0.0):
    p = icm_replica_params()
    p.n[:] = [int(x) for x in n]
    p.kernel = int(kernel)
    p.h, p.rho, p.eta, p.kT, p.dt = float(h), float(rho), float(eta), float(kT), float(dt)
    p.slip = int(slip)
    p.thermal_drift = 1 if thermal_drift else 0
    p.seed = int(seed)
    p.replica_id = int(replica_id)
    p.advection = 1 if advection else 0
    p.body_force[:] = [float(x) for x in body_force]
    p.wca_eps, p.wca_sigma = float(wca_eps), float(wca_sigma)
    p.spring_k = float(spring_k)
    p.spring_center[:] = [float(x) for x in spring_center]
    p.kernel_shift = float(kernel_shift)
    return p


def _params_array(params):
    arr = (icm_replica_params * len(params))()
    for i, p in enumerate(params):
        arr[i] = p
    return arr


def _ptr(x, dtype):
    """ctypes pointer of a host array (made contiguous with the right dtype)
    or of a device tensor; returns (pointer, keepalive)."""
    if x is None:
        return None, None
    if hasattr(x, "data_ptr"):          # torch tensor (device or host)
        return ctypes.c_void_p(x.data_ptr()), x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(ctypes.c_void_p), a


def icm_workspace_bytes(params, max_blobs, precision):
    arr = _params_array(params)
    mb = (ctypes.c_int32 * len(params))(*[int(m) for m in max_blobs])
    out = ctypes.c_size_t(0)
    _check(_lib.icm_workspace_bytes(len(params), arr, mb, int(precision), ctypes.byref(out)))
    return out.value


def icm_create(params, max_blobs, precision, workspace=None, workspace_bytes=0, stream=None):
    """Returns an opaque context handle (ctypes.c_void_p)."""
    arr = _params_array(params)
    mb = (ctypes.c_int32 * len(params))(*[int(m) for m in max_blobs])
    ctx = ctypes.c_void_p()
    ws = ctypes.c_void_p(workspace) if workspace else None
    st = ctypes.c_void_p(stream) if stream else None
    _check(_lib.icm_create(len(params), arr, mb, int(precision), ws, int(workspace_bytes), st, ctypes.byref(ctx)))
    return ctx


def icm_set_blobs(ctx, replica, q, u=None, m_e=None, f_const=None, flags=0):
    n = int(q.shape[0]) if q is not None else 0
    pq, kq = _ptr(q, np.float64)
    pu, ku = _ptr(u, np.float64)
    pm, km = _ptr(m_e, np.float64)
    pf, kf = _ptr(f_const, np.float64)
    _check(_lib.icm_set_blobs(ctx, int(replica), n, pq, pu, pm, pf, int(flags)), ctx)


def icm_set_state(ctx, replica, v=None, q=None, u=None, lag_c=None, step=-1, flags=0, field_dtype=np.float64):
    pv, kv = _ptr(v, field_dtype)
    pq, kq = _ptr(q, np.float64)
    pu, ku = _ptr(u, np.float64)
    pl, kl = _ptr(lag_c, np.float64)
    _check(_lib.icm_set_state(ctx, int(replica), pv, pq, pu, pl, int(step), int(flags)), ctx)


def icm_autotune(ctx, capacity=64):
    """Returns one dict per grid shape with the chosen FFT launch shapes."""
    res = (icm_tune_result * capacity)()
    n = ctypes.c_int32(0)
    _check(_lib.icm_autotune(ctx, res, capacity, ctypes.byref(n)), ctx)
    out = []
    for r in res[:min(n.value, capacity)]:
        out.append(dict(n=tuple(r.n), y_columns=r.y_columns, z_columns=r.z_columns, z_small_plan=r.z_small_plan,
                        x_threads=r.x_threads, rhs_z_chunk=r.rhs_z_chunk, tuned=bool(r.tuned),
                        us_default=r.us_default, us_tuned=r.us_tuned, us_rhs_default=r.us_rhs_default,
                        us_rhs_tuned=r.us_rhs_tuned))
    return out


def icm_step(ctx, n_steps, flags=0):
    _check(_lib.icm_step(ctx, int(n_steps), int(flags)), ctx)


def icm_solve_noalloc(n, h, a, b, precision, rhs_ptr, out_ptr, stream=None):
    """out = P (a + b lambda)^-1 rhs on device fields given by address
    (e.g. torch data_ptr()), enqueued on `stream` (a hipStream_t handle);
    no context and no allocation (see include/icm.h)."""
    nn = (ctypes.c_int32 * 3)(*[int(x) for x in n])
    _check(_lib.icm_solve_noalloc(nn, float(h), float(a), float(b), int(precision), ctypes.c_void_p(rhs_ptr),
                                  ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream or 0)))


def icm_num_blobs(ctx, replica):
    return int(_lib.icm_num_blobs(ctx, int(replica)))


def icm_get_state(ctx, replica, n, field_dtype=np.float64, want_v=True, want_diag=True):
    """Returns dict(v, q, u, lag_c, diag) of host numpy arrays."""
    nx, ny, nz = n
    nb = icm_num_blobs(ctx, replica)
    v = np.empty((3, nz, ny, nx), dtype=field_dtype) if want_v else None
    q = np.empty((nb, 3))
    u = np.empty((nb, 3))
    lag = np.empty((nb, 3))
    d = icm_diag()
    _check(_lib.icm_get_state(ctx, int(replica),
                              v.ctypes.data_as(ctypes.c_void_p) if v is not None else None,
                              q.ctypes.data_as(ctypes.c_void_p), u.ctypes.data_as(ctypes.c_void_p),
                              lag.ctypes.data_as(ctypes.c_void_p),
                              ctypes.byref(d) if want_diag else None, 0), ctx)
    diag = None
    if want_diag:
        diag = dict(momentum=np.array(d.momentum[:]), ke_fluid=d.ke_fluid, ke_blob=d.ke_blob,
                    max_div=d.max_div, max_alpha=d.max_alpha, step=d.step)
    return dict(v=v, q=q, u=u, lag_c=lag, diag=diag)


def icm_get_advection_lag(ctx, replica, n, field_dtype=np.float64):
    """Returns (lag, valid): the lagged advective term (host array shaped
    like v) and whether the next step uses it."""
    nx, ny, nz = n
    lag = np.empty((3, nz, ny, nx), dtype=field_dtype)
    valid = ctypes.c_int32(0)
    _check(_lib.icm_get_advection_lag(ctx, int(replica), lag.ctypes.data_as(ctypes.c_void_p), ctypes.byref(valid), 0),
           ctx)
    return lag, bool(valid.value)


def icm_set_advection_lag(ctx, replica, lag, field_dtype=np.float64):
    """Install the lagged advective term (None: clear the history)."""
    if lag is None:
        _check(_lib.icm_set_advection_lag(ctx, int(replica), None, 0), ctx)
        return
    a = np.ascontiguousarray(lag, dtype=field_dtype)
    _check(_lib.icm_set_advection_lag(ctx, int(replica), a.ctypes.data_as(ctypes.c_void_p), 0), ctx)


def icm_set_fft_shapes(ctx, shapes):
    """Install launch shapes: a list of dicts with n, y_columns, z_columns,
    z_small_plan, x_threads and optionally rhs_z_chunk (as icm_autotune
    returns them)."""
    arr = (icm_tune_result * max(len(shapes), 1))()
    for i, sh in enumerate(shapes):
        arr[i].n[:] = [int(x) for x in sh["n"]]
        arr[i].y_columns = int(sh["y_columns"])
        arr[i].z_columns = int(sh["z_columns"])
        arr[i].z_small_plan = int(sh["z_small_plan"])
        arr[i].x_threads = int(sh["x_threads"])
        arr[i].rhs_z_chunk = int(sh.get("rhs_z_chunk", 0))
    _check(_lib.icm_set_fft_shapes(ctx, arr, len(shapes)), ctx)


def icm_set_timing(ctx, enable):
    _check(_lib.icm_set_timing(ctx, 1 if enable else 0), ctx)


def icm_get_timing(ctx, reset=False):
    """Returns {phase: (total_ms, launches)}."""
    t = icm_timing()
    _check(_lib.icm_get_timing(ctx, ctypes.byref(t), 1 if reset else 0), ctx)
    return {name: (t.ms[i], int(t.launches[i])) for i, name in enumerate(PHASES)}


def icm_destroy(ctx):
    if ctx:
        _lib.icm_destroy(ctx)


def icm_last_error(ctx=None):
    return _lib.icm_last_error(ctx).decode()


class Sim:
    """Convenience owner of one context (several replicas allowed)."""

    def __init__(self, params, max_blobs, precision=FP64, stream=None, workspace=None):
        self.params = list(params)
        self.precision = precision
        self.dtype = np.float64 if precision == FP64 else np.float32
        self._ws = workspace
        ws_ptr, ws_bytes = (None, 0)
        if workspace is not None:
            ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
        self.ctx = icm_create(self.params, max_blobs, precision, ws_ptr, ws_bytes, stream)

    def set_blobs(self, replica, q, u=None, m_e=None, f_const=None, flags=0):
        icm_set_blobs(self.ctx, replica, q, u, m_e, f_const, flags)

    def set_state(self, replica, v=None, q=None, u=None, lag_c=None, step=-1, flags=0):
        icm_set_state(self.ctx, replica, v, q, u, lag_c, step, flags, self.dtype)

    def step(self, n=1, flags=0):
        icm_step(self.ctx, n, flags)

    def autotune(self):
        return icm_autotune(self.ctx)

    def set_fft_shapes(self, shapes):
        icm_set_fft_shapes(self.ctx, shapes)

    def get_state(self, replica=0, want_v=True, want_diag=True):
        return icm_get_state(self.ctx, replica, tuple(self.params[replica].n), self.dtype, want_v, want_diag)

    def get_advection_lag(self, replica=0):
        return icm_get_advection_lag(self.ctx, replica, tuple(self.params[replica].n), self.dtype)

    def set_advection_lag(self, replica, lag):
        icm_set_advection_lag(self.ctx, replica, lag, self.dtype)

    def set_timing(self, enable):
        icm_set_timing(self.ctx, enable)

    def timing(self, reset=False):
        return icm_get_timing(self.ctx, reset)

    def close(self):
        icm_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            if self.ctx:
                self.close()
        except Exception:
            pass
