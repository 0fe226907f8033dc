"""Context set-up through the C ABI: a caller-provided workspace (no
allocation by the library), the refusal of one too small, a caller's HIP
stream, and the per-phase timers.
"""
import ctypes

import numpy as np
import pytest

from oracle import icm as O
from tests.parity_cases import banner, compare, gpu_params, initial_state, load_into_gpu, oracle_params, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def I():
    import paper_1212_6427_amd.icm as lib
    return lib


class _Workspace:
    """Device bytes from the HIP runtime that libicm.so is bound to, shaped
    like the tensor the binding accepts as a workspace."""

    def __init__(self, nbytes):
        self._hip = ctypes.CDLL("libamdhip64.so.7")
        self._hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self._hip.hipFree.argtypes = [ctypes.c_void_p]
        self.nbytes = int(nbytes)
        self.ptr = ctypes.c_void_p()
        assert self._hip.hipMalloc(ctypes.byref(self.ptr), self.nbytes) == 0

    def data_ptr(self):
        return self.ptr.value

    def numel(self):
        return self.nbytes

    def element_size(self):
        return 1

    def free(self):
        self._hip.hipFree(self.ptr)


def _cases():
    return [
        (oracle_params((32, 32, 32), kernel=4, kT=1e-3, dt=0.25, seed=211, replica=0), (0.0, 1.0), 2),
        (oracle_params((24, 18, 12), kernel=3, kT=2e-3, dt=0.2, seed=212, replica=1, wca_eps=1e-2,
                       wca_sigma=2.0 / 2 ** (1 / 6)), (0.0,), 4),
    ]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_caller_workspace(I, precision):
    """Two replicas in a context whose device memory is one caller buffer of
    icm_workspace_bytes: the same results as a library-allocated context,
    and the oracle's."""
    prec = I.FP64 if precision == "fp64" else I.FP32_GRID
    dtype = np.float64 if prec == I.FP64 else np.float32
    tol = 1e-11 if precision == "fp64" else 2e-5
    steps = 2 if precision == "fp64" else 1
    cases = _cases()
    states = [initial_state(p, nb, me, seed=220 + i, min_sep=3.0) for i, (p, me, nb) in enumerate(cases)]
    if prec == I.FP32_GRID:
        for st in states:
            st.v = st.v.astype(np.float32).astype(np.float64)
    params = [gpu_params(I, p) for p, _, _ in cases]
    caps = [nb for _, _, nb in cases]
    nbytes = I.icm_workspace_bytes(params, caps, prec)
    banner("caller workspace %s, %d bytes" % (precision, nbytes))
    ws = _Workspace(nbytes)
    own = I.Sim(params, caps, prec)
    try:
        sim = I.Sim(params, caps, prec, workspace=ws)
        try:
            for r, st in enumerate(states):
                load_into_gpu(I, sim, r, st, dtype)
                load_into_gpu(I, own, r, st, dtype)
            sim.step(steps, I.STEP_GRAPH)
            own.step(steps, I.STEP_GRAPH)
            for r, ((p, _, _), st) in enumerate(zip(cases, states)):
                a, b = sim.get_state(r), own.get_state(r)
                assert rel_err(a["v"], b["v"]) <= (1e-13 if precision == "fp64" else 1e-6)
                errs, bad = compare(a, O.run(p, st, steps), st.q, tol)
                print("replica", r, {k: "%.2e" % v for k, v in errs.items()}, flush=True)
                assert not bad, (r, bad)
        finally:
            sim.close()
    finally:
        own.close()
        ws.free()


def test_workspace_too_small_is_refused(I):
    """A caller buffer below icm_workspace_bytes: ICM_E_NOMEM with the two
    sizes in the message, and no context."""
    params = [gpu_params(I, p) for p, _, _ in _cases()]
    nbytes = I.icm_workspace_bytes(params, [2, 4], I.FP64)
    ws = _Workspace(nbytes)
    try:
        with pytest.raises(I.ICMError) as e:
            I.icm_create(params, [2, 4], I.FP64, ws.data_ptr(), nbytes - 1)
        assert e.value.status == I.E_NOMEM
        assert str(nbytes - 1) in str(e.value) and str(nbytes) in str(e.value)
    finally:
        ws.free()


def test_caller_stream(I):
    """A context created on a caller's HIP stream (default priority) enqueues
    its work there, recorded graph included; the results match the oracle."""
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    hip.hipStreamDestroy.argtypes = [ctypes.c_void_p]
    stream = ctypes.c_void_p()
    assert hip.hipStreamCreate(ctypes.byref(stream)) == 0
    p, me, nb = _cases()[0]
    st = initial_state(p, nb, me, seed=241, min_sep=3.0)
    banner("caller stream")
    try:
        sim = I.Sim([gpu_params(I, p)], [nb], I.FP64, stream=stream.value)
        try:
            load_into_gpu(I, sim, 0, st, np.float64)
            sim.step(1)
            sim.step(2, I.STEP_GRAPH)
            errs, bad = compare(sim.get_state(0), O.run(p, st, 3), st.q, 1e-11)
            print({k: "%.2e" % v for k, v in errs.items()}, flush=True)
            assert not bad, bad
        finally:
            sim.close()
    finally:
        hip.hipStreamDestroy(stream)


def test_phase_timers(I):
    """icm_set_timing brackets each phase's launches with events: after three
    eager steps every phase the plain step runs has three or more launches
    and a positive time, the advection phase none with advection off; a
    reset clears the counts, and with the timers off nothing is counted."""
    p = oracle_params((32, 32, 32), kernel=4, kT=1e-3, dt=0.25, seed=231, wca_eps=1e-2,
                      wca_sigma=2.0 / 2 ** (1 / 6))
    st = initial_state(p, 6, (0.0,), seed=232, min_sep=2.5)
    sim = I.Sim([gpu_params(I, p)], [6], I.FP32_GRID)
    try:
        load_into_gpu(I, sim, 0, st, np.float32)
        sim.set_timing(True)
        sim.step(3)
        t = sim.timing(reset=True)
        print({k: v for k, v in t.items() if v[1]}, flush=True)
        for ph in ("gather", "forces", "rhs", "fft_x_fwd", "fft_y_fwd", "fft_z_solve", "fft_y_inv", "fft_x_inv"):
            ms, n = t[ph]
            assert n >= 3 and ms > 0.0, ph
        assert t["advection"][1] == 0
        t2 = sim.timing()
        assert all(n == 0 for _, n in t2.values())
        sim.set_timing(False)
        sim.step(1)
        assert all(n == 0 for _, n in sim.timing().values())
    finally:
        sim.close()
