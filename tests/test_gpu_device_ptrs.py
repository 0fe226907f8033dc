"""ICM_PTRS_DEVICE: the state handed to icm_set_blobs / icm_set_state and
read back by icm_get_state as device memory on the context's GPU.

Two contexts with the same parameters get the same state, one from host
arrays and one from device buffers; after the same steps both must hold the
same state (within rounding: the spread accumulates overlapping taps in an
order the hardware picks), read back through host and device pointers, and
both must match the oracle.
"""
import ctypes

import numpy as np
import pytest

from oracle import icm as O
import icm_inputs
from tests.parity_cases import banner, compare, gpu_params, initial_state, load_into_gpu, oracle_params, rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 2e-5}


@pytest.fixture(scope="module")
def I():
    import paper_1212_6427_amd.icm as lib
    return lib


class _DeviceArray:
    """A device copy of a host array, from the HIP runtime that libicm.so is
    bound to (found by its soname); passed to the binding like a tensor."""
    _hip = None

    def __init__(self, host):
        if _DeviceArray._hip is None:
            h = ctypes.CDLL("libamdhip64.so.7")
            h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
            h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
            h.hipFree.argtypes = [ctypes.c_void_p]
            _DeviceArray._hip = h
        self.host = np.ascontiguousarray(host)
        self.shape = self.host.shape
        self.ptr = ctypes.c_void_p()
        assert self._hip.hipMalloc(ctypes.byref(self.ptr), max(self.host.nbytes, 1)) == 0
        if self.host.nbytes:
            assert self._hip.hipMemcpy(self.ptr, self.host.ctypes.data, self.host.nbytes, 1) == 0  # to device

    def data_ptr(self):
        return self.ptr.value

    def read(self):
        out = np.empty_like(self.host)
        assert self._hip.hipDeviceSynchronize() == 0
        if out.nbytes:
            assert self._hip.hipMemcpy(out.ctypes.data, self.ptr, out.nbytes, 2) == 0            # to host
        return out

    def free(self):
        self._hip.hipFree(self.ptr)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_device_pointer_state_in_and_out(I, precision):
    prec = I.FP64 if precision == "fp64" else I.FP32_GRID
    dtype = np.float64 if prec == I.FP64 else np.float32
    tol = TOL[precision]
    steps = 2 if precision == "fp64" else 1
    p = oracle_params((24, 18, 12), kernel=4, kT=1e-3, dt=0.2, seed=191, wca_eps=1e-2,
                      wca_sigma=2.0 / 2 ** (1 / 6))
    st = initial_state(p, 5, (0.0, 1.0, -0.5), seed=193, min_sep=2.5)
    st.lag_c = icm_inputs.random_forces(5, seed=194, scale=1e-3) * (st.m_e != 0)[:, None]
    st.step = 7
    st.v = st.v.astype(dtype).astype(np.float64)
    banner("device pointers %s" % precision)
    host = I.Sim([gpu_params(I, p)], [5], prec)
    dev = I.Sim([gpu_params(I, p)], [5], prec)
    bufs = []
    try:
        load_into_gpu(I, host, 0, st, dtype)
        d_q, d_u, d_me, d_f = (_DeviceArray(x) for x in (st.q, st.u, st.m_e, st.f_const))
        d_v, d_lag = _DeviceArray(st.v.astype(dtype)), _DeviceArray(st.lag_c)
        bufs += [d_q, d_u, d_me, d_f, d_v, d_lag]
        dev.set_blobs(0, d_q, d_u, d_me, d_f, flags=I.PTRS_DEVICE)
        dev.set_state(0, v=d_v, lag_c=d_lag, step=st.step, flags=I.PTRS_DEVICE)
        host.step(steps)
        dev.step(steps)
        a = host.get_state(0)
        # read the device context's state into device buffers
        o_v = _DeviceArray(np.full(st.v.shape, np.nan, dtype=dtype))
        o_q, o_u, o_lag = (_DeviceArray(np.full((5, 3), np.nan)) for _ in range(3))
        bufs += [o_v, o_q, o_u, o_lag]
        rc = I._lib.icm_get_state(dev.ctx, 0, o_v.ptr, o_q.ptr, o_u.ptr, o_lag.ptr, None, I.PTRS_DEVICE)
        assert rc == I.OK, I._lib.icm_last_error(dev.ctx).decode()
        b = dict(v=o_v.read(), q=o_q.read(), u=o_u.read(), lag_c=o_lag.read())
    finally:
        host.close()
        dev.close()
        for x in bufs:
            x.free()
    for k in ("v", "u", "lag_c"):
        e = rel_err(b[k], a[k])
        print(k, "device vs host pointers %.2e" % e, flush=True)
        assert e <= 1e-13 if precision == "fp64" else e <= 1e-6
    assert rel_err(b["q"] - st.q, a["q"] - st.q) <= (1e-13 if precision == "fp64" else 1e-6)
    ref = O.run(p, st, steps)
    errs, bad = compare(b, ref, st.q, tol)
    print("device pointers vs oracle", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    assert not bad, bad
