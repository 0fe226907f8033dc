"""Error behaviour of the C ABI on the GPU (include/icm.h): invalid calls
leave the context usable; the numeric flag puts it in an error state that
only icm_set_state clears. Every condition is forced from the host; no
kernel faults or spins."""
import numpy as np
import pytest

from oracle import icm as O
from tests.parity_cases import banner, gpu_params, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def I():
    import paper_1212_6427_amd.icm as lib
    return lib


def _sim(I, nb=2, prec=None):
    p = oracle_params((16, 16, 16), kernel=3, kT=0.0, dt=0.2)
    return p, I.Sim([gpu_params(I, p)], [nb], I.FP64 if prec is None else prec)


def test_invalid_calls_leave_the_context_usable(I):
    banner("invalid calls")
    p, sim = _sim(I)
    try:
        q = np.array([[3.0, 4.0, 5.0], [9.0, 9.0, 9.0]])
        with pytest.raises(I.ICMError) as e:
            sim.set_blobs(1, q)                      # replica out of range
        assert e.value.status == I.E_INVALID
        with pytest.raises(I.ICMError) as e:
            sim.set_blobs(0, np.zeros((3, 3)))       # more blobs than max_blobs
        assert e.value.status == I.E_INVALID
        with pytest.raises(I.ICMError) as e:
            sim.set_blobs(0, q, m_e=np.array([0.0, -p.m_f]))   # m_e must exceed -m_f
        assert e.value.status == I.E_INVALID
        with pytest.raises(I.ICMError) as e:
            sim.step(1, 0x10)                        # unknown step flag
        assert e.value.status == I.E_INVALID
        with pytest.raises(I.ICMError) as e:
            sim.step(-1)
        assert e.value.status == I.E_INVALID
        # still usable: a valid step matches the oracle
        sim.set_blobs(0, q, f_const=np.array([[0.01, 0.0, 0.0], [0.0, 0.02, 0.0]]))
        sim.step(0)
        sim.step(2, I.STEP_GRAPH)
        got = sim.get_state(0)
        st = O.new_state(p, q, f_const=np.array([[0.01, 0.0, 0.0], [0.0, 0.02, 0.0]]))
        ref = O.run(p, st, 2)
        assert np.max(np.abs(got["q"] - ref.q)) < 1e-12
        assert got["diag"]["step"] == 2
    finally:
        sim.close()


@pytest.mark.parametrize("graph", [False, True])
def test_numeric_flag_sets_the_error_state_until_set_state(I, graph):
    """A fluid field of 100 h per unit time around a blob moves it by more
    than h in one step (the advective CFL condition of Sec. III.D): the step
    returns ICM_E_NUMERIC, further steps ICM_E_STATE, and icm_set_state with
    a new state restores normal operation. (Positions stay finite, so every
    grid index stays an ordinary wrapped integer.)"""
    banner("numeric flag graph=%s" % graph)
    p, sim = _sim(I)
    try:
        q = np.array([[3.0, 4.0, 5.0], [9.0, 9.0, 9.0]])
        sim.set_blobs(0, q)
        v = np.zeros((3, 16, 16, 16))
        v[0] = 100.0                                 # uniform flow: dq = dt * 100 = 20 h
        sim.set_state(0, v=v)
        flags = I.STEP_GRAPH if graph else 0
        with pytest.raises(I.ICMError) as e:
            sim.step(1, flags)
        assert e.value.status == I.E_NUMERIC
        with pytest.raises(I.ICMError) as e:
            sim.step(1, flags)
        assert e.value.status == I.E_STATE
        st = O.new_state(p, q)
        sim.set_state(0, v=st.v, q=q, u=np.zeros((2, 3)), step=0)
        sim.step(2, flags)
        got = sim.get_state(0)
        ref = O.run(p, st, 2)
        assert np.all(np.isfinite(got["v"]))
        assert np.max(np.abs(got["q"] - ref.q)) < 1e-12
    finally:
        sim.close()
