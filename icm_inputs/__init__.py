"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module holds none of the method's arithmetic: it only draws blob
positions and excess-mass choices with numpy's PCG64 generator and names the
workload configurations (grid, physical constants, kernel, step counts). Each
side (oracle or HIP library) derives its own method constants (dV, m_f, ...)
from these parameters.
"""
import numpy as np

# Workload configurations, shaped like the paper's runs (Sec. III.D, Sec. IV).
# Excess masses are given as multiples of the entrained fluid mass m_f, which
# each side computes for itself.
WORKLOADS = {
    "plain_fp64_32": dict(
        n=(32, 32, 32), h=1.0, rho=1.0, eta=1.0, kT=0.0, dt=0.1, kernel=3,
        n_blobs=1, me_over_mf=(0.0,), kick=(0.1, 0.0, 0.0),
        f_const=(0.01, 0.0, 0.0), steps=10, seed=11),
    "single_blob_128": dict(
        n=(128, 128, 128), h=1.0, rho=1.0, eta=1.0, kT=1e-3, dt=0.25, kernel=4,
        n_blobs=1, me_over_mf=(0.0, 1.0, -0.5), steps=10000, seed=12),
    "many_blobs_256": dict(
        n=(256, 256, 256), h=1.0, rho=1.0, eta=1.0, kT=1e-3, dt=0.2, kernel=4,
        n_blobs=4096, me_over_mf=(0.0,), min_sep=2.0, wca_eps=1e-2,
        wca_cutoff=2.0, steps=1000, seed=13),
    "batched_ensemble": dict(
        grids=((32, 32, 32),) * 32 + ((48, 48, 48),) * 32 + ((64, 64, 64),) * 32,
        h=1.0, rho=1.0, eta=1.0, kT=1e-3, dt=0.25, kernel=4, n_blobs=1,
        me_over_mf=(0.0, 1.0, -0.5), steps=5000, seed=14),
    "scale_512": dict(
        n=(512, 512, 512), h=1.0, rho=1.0, eta=1.0, kT=1e-3, dt=0.2, kernel=3,
        n_blobs=100000, me_over_mf=(0.0,), min_sep=2.0, wca_eps=1e-2,
        wca_cutoff=2.0, re_p=1.0, steps=200, seed=15),
    # WCA suspension at equilibrium, Sec. IV.A Table RDF (left): 1000 blobs in
    # 32^3, dt = 1, kT = eps = 1e-3, sigma = 2; excess masses 0 and m_f
    "rdf_32": dict(
        n=(32, 32, 32), h=1.0, rho=1.0, eta=1.0, kT=1e-3, dt=1.0, kernel=3, n_blobs=1000,
        wca_eps=1e-3, wca_sigma=2.0, me_over_mf=(0.0, 1.0), replicas=8, steps=20000, every=100,
        relax=20000, rmax=5.0, nbins=50, min_sep=2.0, seed=17),
    # ideal gas of neutrally buoyant blobs at equilibrium, thermal drift on
    # and off (App. B.2): 100 blobs per 16^3 box, viscous CFL 0.05
    "drift_bias_16": dict(
        n=(16, 16, 16), h=1.0, rho=1.0, eta=1.0, kT=1.0, dt=0.05, kernels=(3, 4),
        n_blobs=100, replicas=64, steps=30000, every=20, seed=16),
    # deterministic temporal-convergence test: a blob released from rest in a
    # harmonic potential centred at the origin (Sec. III.D); dt halved down
    # the list, error E(dt) between runs at dt and dt/2 up to time T
    "convergence_16": dict(
        n=(16, 16, 16), h=1.0, rho=1.0, eta=1.0, kT=0.0, kernel=3, x0=(10.0, 0.3, 0.2),
        T=80.0, spring_k=0.01, me_over_mf=(0.0, 1.0, 10.0, -0.5),
        dts=(4.0, 2.0, 1.0, 0.5, 0.25, 0.125, 0.0625, 0.03125),
        slip_test=dict(me_over_mf=10.0, spring_k=(1.0, 500.0),
                       dts=((0.4, 0.2, 0.1, 0.05, 0.025), (0.04, 0.02, 0.01, 0.005)))),
}


def uniform_positions(n_blobs, n, h=1.0, seed=0):
    """Blob positions uniform in the periodic box [0, N h)^3."""
    rng = np.random.default_rng(seed)
    box = np.asarray(n, dtype=np.float64) * h
    return rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * box


def separated_positions(n_blobs, n, h=1.0, min_sep=2.0, seed=0, max_tries=200):
    """Uniform positions with pairwise minimum-image distance >= min_sep.

    Sequential rejection sampling accelerated by a bin grid of cell size
    >= min_sep (each candidate is tested against the 27 neighbouring bins).
    """
    rng = np.random.default_rng(seed)
    box = np.asarray(n, dtype=np.float64) * h
    nbins = np.maximum((box // min_sep).astype(int), 1)
    bsize = box / nbins
    bins = {}
    pts = np.zeros((n_blobs, 3))
    count = 0
    tries = 0
    while count < n_blobs:
        tries += 1
        if tries > max_tries * n_blobs:
            raise RuntimeError("could not place blobs with the requested separation")
        c = rng.uniform(0.0, 1.0, size=3) * box
        b = tuple((c // bsize).astype(int) % nbins)
        ok = True
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    key = ((b[0] + dx) % nbins[0], (b[1] + dy) % nbins[1], (b[2] + dz) % nbins[2])
                    for idx in bins.get(key, ()):
                        d = c - pts[idx]
                        d -= box * np.round(d / box)
                        if d @ d < min_sep * min_sep:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pts[count] = c
            bins.setdefault(b, []).append(count)
            count += 1
    return pts


def excess_mass_ratios(n, choices, seed=0):
    """Per-replica (or per-blob) m_e/m_f drawn uniformly from `choices`."""
    rng = np.random.default_rng(seed)
    return np.asarray(choices, dtype=np.float64)[rng.integers(0, len(choices), size=n)]


def random_field(n, seed=0, scale=1.0):
    """A seeded random face field of shape (3, Nz, Ny, Nx) (test input only)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    return scale * rng.standard_normal((3, nz, ny, nx))


def random_forces(n_blobs, seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((n_blobs, 3))
