"""Monte Carlo reference of the equilibrium pair structure (Sec. IV.A).

TEST INFRASTRUCTURE ONLY. A plain Metropolis sampler (oracle/mc_wca.c) of the
Gibbs-Boltzmann distribution P(Q) ~ exp(-U(Q)/kT), Eq. (P_Q), for particles
interacting with the WCA potential of Eq. (WCA), and the radial distribution
function g(r) of its samples: the reference the GPU time stepper's
equilibrium structure is compared with. It shares nothing with the HIP path;
only tests, the smoke check and the CPU-baseline leg of the benchmark may
import it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mc_wca.c")
_LIB = os.path.join(_HERE, "libmc_wca.so")


def build():
    """Compile the sampler with the host C compiler (in-tree)."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)


def _load():
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    d, i, ll, u64 = ctypes.c_double, ctypes.c_int, ctypes.c_longlong, ctypes.c_uint64
    pd = ctypes.POINTER(ctypes.c_double)
    lib.mc_wca_gr.argtypes = [i, d, d, d, d, pd, d, ll, ll, i, u64, d, i, pd, pd]
    lib.mc_wca_gr.restype = i
    return lib


_lib = None


def wca_gr(x0, L, eps, sigma, kT, delta, n_equil, n_sweeps, every, seed, rmax, nbins):
    """g(r) of the WCA fluid sampled by Metropolis Monte Carlo.

    x0: (N, 3) initial positions; L: periodic box side; the trial moves are
    uniform in a cube of half side delta; n_equil and n_sweeps sweeps of N
    trial moves before and during sampling, g(r) sampled every `every`
    sweeps on nbins bins of [0, rmax). Returns (bin centres, g, acceptance
    rate, final positions)."""
    global _lib
    if _lib is None:
        _lib = _load()
    x = np.ascontiguousarray(np.array(x0, dtype=np.float64).reshape(-1, 3))
    g = np.zeros(nbins)
    acc = ctypes.c_double(0.0)
    pd = ctypes.POINTER(ctypes.c_double)
    rc = _lib.mc_wca_gr(x.shape[0], float(L), float(eps), float(sigma), float(kT), x.ctypes.data_as(pd),
                        float(delta), int(n_equil), int(n_sweeps), int(every), int(seed) & (2 ** 64 - 1),
                        float(rmax), int(nbins), g.ctypes.data_as(pd), ctypes.byref(acc))
    if rc != 0:
        raise ValueError("mc_wca_gr rejected its arguments")
    r = (np.arange(nbins) + 0.5) * rmax / nbins
    return r, g, acc.value, x
