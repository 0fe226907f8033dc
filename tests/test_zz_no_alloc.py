"""icm_solve_noalloc: the spectral solve with no context and no device
allocation, its buffers in the library's fixed device array.

Checked through the C ABI against the existing entry point that runs the
same passes (icm_set_state with ICM_STATE_PROJECT, read back with
icm_get_state) and against the oracle's Helmholtz solve, on two calls in a
row with the second input smaller, on the register-resident and the
generic FFT paths, in FP64 and FP32; a grid beyond the array's size is
refused with a message.
"""
import ctypes

import numpy as np
import pytest

from oracle import icm as O
import icm_inputs
from tests.parity_cases import banner, rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 2e-5}


@pytest.fixture(scope="module")
def I():
    import paper_1212_6427_amd.icm as lib
    return lib


class _DeviceBuffer:
    """Device memory for the test's inputs and outputs, from the HIP runtime
    that libicm.so is bound to (found by its soname, so the process keeps one
    runtime whether or not PyTorch loaded it first)."""
    _hip = None

    def __init__(self, host):
        if _DeviceBuffer._hip is None:
            h = ctypes.CDLL("libamdhip64.so.7")
            h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
            h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
            h.hipFree.argtypes = [ctypes.c_void_p]
            _DeviceBuffer._hip = h
        self.host = np.ascontiguousarray(host)
        self.ptr = ctypes.c_void_p()
        assert self._hip.hipMalloc(ctypes.byref(self.ptr), self.host.nbytes) == 0
        assert self._hip.hipMemcpy(self.ptr, self.host.ctypes.data, self.host.nbytes, 1) == 0   # host to device

    def read(self):
        out = np.empty_like(self.host)
        assert self._hip.hipDeviceSynchronize() == 0
        assert self._hip.hipMemcpy(out.ctypes.data, self.ptr, out.nbytes, 2) == 0               # device to host
        return out

    def free(self):
        self._hip.hipFree(self.ptr)


def _noalloc(I, n, h, a, b, prec, field):
    dtype = np.float64 if prec == I.FP64 else np.float32
    src = _DeviceBuffer(field.astype(dtype))
    out = _DeviceBuffer(np.full(field.shape, np.nan, dtype=dtype))
    try:
        I.icm_solve_noalloc(n, h, a, b, prec, src.ptr.value, out.ptr.value, None)
        return out.read().astype(np.float64)
    finally:
        src.free()
        out.free()


def _project_with_context(I, n, h, prec, field):
    dtype = np.float64 if prec == I.FP64 else np.float32
    sim = I.Sim([I.make_params(n, h=h)], [1], prec)
    try:
        sim.set_state(0, v=field.astype(dtype), flags=I.STATE_PROJECT)
        return sim.get_state(0, want_diag=False)["v"].astype(np.float64)
    finally:
        sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_projection_matches_set_state_project(I, precision):
    """Two calls in a row, the second on a smaller grid: each equals the
    projection the context computes for icm_set_state(ICM_STATE_PROJECT)."""
    prec = I.FP64 if precision == "fp64" else I.FP32_GRID
    for i, (n, h) in enumerate((((64, 48, 32), 0.7), ((24, 18, 12), 1.3))):
        banner("noalloc projection %s n=%s" % (precision, n))
        w = icm_inputs.random_field(n, seed=300 + i)
        if prec == I.FP32_GRID:
            w = w.astype(np.float32).astype(np.float64)
        got = _noalloc(I, n, h, 1.0, 0.0, prec, w)
        ref = _project_with_context(I, n, h, prec, w)
        err = rel_err(got, ref)
        print("call %d n=%s rel err vs set_state(PROJECT) %.2e" % (i, n, err), flush=True)
        assert err < TOL[precision]
        # and against the oracle's projection
        assert rel_err(got, O.project(O.Params(n=n, h=h), w)) < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_helmholtz_matches_the_oracle(I, precision):
    """Step 2's operator (a = rho/dt, b = eta/2) on a fast-path grid, then a
    smaller generic-path grid: out = P (a + b lambda)^-1 rhs as the oracle's
    helmholtz_project computes it."""
    prec = I.FP64 if precision == "fp64" else I.FP32_GRID
    cases = [((32, 64, 48), 0.9, 1.1 / 0.25, 0.35), ((12, 16, 18), 1.2, 2.0, 0.8)]
    if prec == I.FP32_GRID:
        # the 256-point x and y plans of the benchmark's planes
        cases.insert(0, ((256, 256, 16), 1.0, 5.0, 0.5))
    for i, (n, h, a, b) in enumerate(cases):
        banner("noalloc helmholtz %s n=%s" % (precision, n))
        r = icm_inputs.random_field(n, seed=310 + i)
        if prec == I.FP32_GRID:
            r = r.astype(np.float32).astype(np.float64)
        got = _noalloc(I, n, h, a, b, prec, r)
        ref = O.helmholtz_project(O.Params(n=n, h=h), r, a, b)
        err = rel_err(got, ref)
        print("call %d n=%s rel err vs oracle %.2e" % (i, n, err), flush=True)
        assert err < TOL[precision]


def test_noalloc_refuses_a_grid_beyond_its_array(I):
    """256^3 in FP64 needs about 400 MB of spectrum: ICM_E_INVALID with a
    message, nothing launched; a later call still works."""
    with pytest.raises(I.ICMError) as e:
        I.icm_solve_noalloc((256, 256, 256), 1.0, 1.0, 0.0, I.FP64, 1 << 20, 1 << 20, 0)
    assert e.value.status == I.E_INVALID
    assert "scratch" in str(e.value)
    with pytest.raises(I.ICMError) as e:
        I.icm_solve_noalloc((16, 16, 15), 1.0, 1.0, 0.0, I.FP64, 1 << 20, 1 << 20, 0)
    assert e.value.status == I.E_INVALID
    n = (16, 16, 16)
    w = icm_inputs.random_field(n, seed=320)
    got = _noalloc(I, n, 1.0, 1.0, 0.0, I.FP64, w)
    assert rel_err(got, O.project(O.Params(n=n), w)) < TOL["fp64"]
