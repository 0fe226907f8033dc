"""Statistics of long GPU runs (FP32 grid, batched replicas, recorded step
graph), checked against what the paper fixes independently of the oracle:
discrete equipartition of the fluid (Sec. II.E, III.B.2: each face has
variance (kT/(rho dV_f)) (2/3) (N-1)/N at equilibrium, for any dt) and of the
blobs (Sec. II.F: <u_a^2> = kT/m~ with m~ = m_e + (3/2) m_f, up to the J P S
invariance error of a few percent and, for m_e != 0, a dt-dependent bias)."""
import numpy as np
import pytest

import json
import os

import icm_inputs

from .parity_cases import banner

with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.json")) as _fh:
    GOLDEN = json.load(_fh)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def I():
    import paper_1212_6427_amd.icm as lib
    return lib


def test_equipartition_fluid_and_blobs(I):
    n = (32, 32, 32)
    kT, dt, h, rho = 1e-3, 0.25, 1.0, 1.0
    m_f = rho * h ** 3 / 0.375 ** 3          # 4-point kernel blob mass
    mt_f = 1.5 * m_f
    n_fluid, n_blob = 8, 32
    params = [I.make_params(n, h=h, rho=rho, eta=1.0, kT=kT, dt=dt, kernel=4, seed=500, replica_id=r)
              for r in range(n_fluid + n_blob)]
    banner("equipartition: %d fluid-only and %d two-blob replicas of %s" % (n_fluid, n_blob, n))
    sim = I.Sim(params, [2] * len(params), I.FP32_GRID)
    try:
        for r in range(len(params)):
            if r >= n_fluid:
                # one neutrally buoyant and one heavy (m_e = m_f) blob, far apart
                q = icm_inputs.separated_positions(2, n, h, min_sep=14.0, seed=600 + r)
                sim.set_blobs(r, q, m_e=np.array([0.0, m_f]))
            sim.set_state(r, flags=I.STATE_EQUILIBRIUM)
        sim.step(200, I.STEP_GRAPH)  # relax the blobs' initial velocities
        v2 = np.zeros(3)
        nv = 0
        u2 = {0: [], 1: []}
        for s in range(60):
            sim.step(8, I.STEP_GRAPH)
            for r in range(len(params)):
                if r < n_fluid:
                    if s % 3 == 0:
                        v = sim.get_state(r, want_diag=False)["v"].astype(np.float64)
                        v2 += (v ** 2).reshape(3, -1).mean(axis=1)
                        nv += 1
                else:
                    u = sim.get_state(r, want_v=False, want_diag=False)["u"]
                    u2[0].append(u[0] ** 2)
                    u2[1].append(u[1] ** 2)
    finally:
        sim.close()
    N = np.prod(n)
    expect_v = kT / (rho * h ** 3) * (2.0 / 3.0) * (N - 1) / N
    v2 /= nv
    print("fluid <v_a^2> / expected:", v2 / expect_v, flush=True)
    # each sample mean of N faces has relative sd ~ (2 / (2 N))^(1/2); samples
    # 24 steps apart are close to independent at these wavelengths only for
    # the short modes, so the bound allows for correlated samples
    assert np.all(np.abs(v2 / expect_v - 1.0) < 0.01)
    jps_dev = GOLDEN["jps_diag_max_dev"]["value"]
    for cls, me in ((0, 0.0), (1, m_f)):
        a = np.concatenate(u2[cls])
        expect_u = kT / (me + mt_f)
        rel_sd = np.sqrt(2.0 / a.size)
        ratio = a.mean() / expect_u
        print("blob m_e = %g m_f: <u_a^2> / (kT/m~) = %.4f (sd of the mean %.3f, %d samples)"
              % (me / m_f, ratio, rel_sd, a.size), flush=True)
        if me == 0.0:
            # u = J v: its variance follows the diagonal of J P S, which the
            # paper bounds within a few percent of its translation-invariant
            # value (Sec. III.A.2)
            assert abs(ratio - 1.0) < 4 * rel_sd + jps_dev
    # the m_e = m_f class (samples 8 steps apart, well inside the blob's
    # velocity correlation time, so the sd above understates the error) is
    # checked against the paper's intercept by the heavy-blob test below


def test_thermal_drift_removes_the_grid_bias(I):
    """App. B.2: an ideal gas of neutrally buoyant blobs must sample positions
    uniformly within a grid cell. With the 3-point kernel and no thermal drift
    the blobs linger near the grid nodes (the paper sees a few percent more
    time near the cell corners); with the drift the density is flat within
    the statistical error. 32 replicas per case of 100 blobs in 16^3 boxes,
    viscous CFL 0.05; the node harmonic eps of the density
    1 + eps sum_a cos(2 pi f_a) with its standard error from the spread over
    the independent replicas."""
    import bench
    wl = icm_inputs.WORKLOADS["drift_bias_16"]
    banner("thermal drift bias: %d replicas of %d blobs, %d steps" % (wl["replicas"], wl["n_blobs"], 20000))
    per = bench.drift_bias_run(I, None, wl, 3, 20000, wl["every"], wl["replicas"])
    on, off = bench.drift_bias_summary(per[0::2]), bench.drift_bias_summary(per[1::2])
    print("with drift:", on, flush=True)
    print("without drift:", off, flush=True)
    assert off["node_harmonic"] - 5 * off["node_harmonic_se"] > 0.003
    assert off["corner_over_centre_minus_1"] > 0.015
    assert abs(on["node_harmonic"]) < 4 * on["node_harmonic_se"] + 0.001
    assert abs(on["corner_over_centre_minus_1"]) < 0.015


def test_four_point_kernel_bias_has_the_sign_of_its_jps_variation(I):
    """The same ideal gas with the four-point kernel, whose J P S is larger at
    the grid nodes than at the cell centres (opposite to the three-point
    kernel; pinned on the CPU from the oracle): without the thermal drift
    the node harmonic is negative (blobs avoid the nodes), smaller than the
    three-point kernel's since the four-point kernel's J P S varies three
    times less; with the drift it vanishes within the statistical error."""
    import bench
    wl = icm_inputs.WORKLOADS["drift_bias_16"]
    banner("thermal drift bias, four-point kernel: %d replicas of %d blobs" % (wl["replicas"], wl["n_blobs"]))
    per = bench.drift_bias_run(I, None, wl, 4, 20000, wl["every"], wl["replicas"])
    on, off = bench.drift_bias_summary(per[0::2]), bench.drift_bias_summary(per[1::2])
    print("with drift:", on, flush=True)
    print("without drift:", off, flush=True)
    assert off["node_harmonic"] + 2 * off["node_harmonic_se"] < 0.0
    assert off["node_harmonic"] > -0.006
    assert abs(on["node_harmonic"]) < 4 * on["node_harmonic_se"] + 0.001


def test_wca_suspension_reproduces_the_gibbs_boltzmann_structure(I):
    """Sec. IV.A, Table RDF: the radial distribution function of 1000 WCA
    blobs (kT = eps = 1e-3, sigma = 2, 32^3, dt = 1, i.e. viscous CFL 1)
    from the GPU dynamics must match the Monte Carlo sample of
    exp(-U/kT) (tests/golden/rdf_wca_mc.json, written by the oracle's
    sampler), for neutrally buoyant and for heavy (m_e = m_f) blobs, within
    the statistical error of the replicas (plus that of the reference) and
    |g - g_MC| < 0.03 for 1.8 < r < 4.5. The blobs start at least sigma apart
    and need ~20000 steps (dt = 1) to build the contact peak: shorter
    relaxations leave it ~2% low."""
    import json
    import os

    import bench
    wl = icm_inputs.WORKLOADS["rdf_32"]
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rdf_wca_mc.json")))
    r = np.asarray(ref["r"])
    g_mc, se_mc = np.asarray(ref["g"]), np.asarray(ref["se"])
    sel = (r > 1.8) & (r < 4.5)
    for ratio in wl["me_over_mf"]:
        banner("RDF: %d replicas of %d WCA blobs, m_e/m_f = %g" % (wl["replicas"], wl["n_blobs"], ratio))
        g = bench.rdf_run(I, None, wl, ratio, wl["replicas"], 20000, wl["every"])
        gm = g.mean(0)
        se = np.sqrt(g.var(0, ddof=1) / g.shape[0] + se_mc ** 2)
        z = np.abs(gm - g_mc)[sel] / np.maximum(se[sel], 1e-3)
        print("m_e/m_f=%g: max |g - g_MC| = %.4f, max z = %.2f" % (ratio, np.max(np.abs(gm - g_mc)[sel]), z.max()),
              flush=True)
        print(np.c_[r[sel], gm[sel], g_mc[sel], se[sel]].round(4), flush=True)
        assert np.max(np.abs(gm - g_mc)[sel]) < 0.03
        assert z.max() < 5.0


def test_heavy_blob_velocity_variance_reaches_the_paper_intercept(I):
    """Sec. IV.B: the velocity autocorrelation of a blob with m_e = m_f starts
    at C(0+) = kT / m~ = 0.8 kT / m (m = m_e + m_f). <u_a^2> m / kT must
    match the paper's 0.8 within 3% (plus three standard errors of the
    replica mean) at beta = 1/4, 1/8 and 1/16, and within 3% at beta = 1/16
    (64^3, 16 replicas, one blob each). A heavy blob's time-step bias is
    small (measured below 1% at beta = 1/4, against +11% for the light blob
    of the next test)."""
    n, kT = (64, 64, 64), 1e-3
    m_f = 1.0 / 0.375 ** 3
    m = 2.0 * m_f
    target = GOLDEN["vacf_intercept_me_eq_mf"]["value"]
    R = 16
    c0 = {}
    for dt in (0.25, 0.125, 0.0625):
        banner("heavy-blob velocity variance dt=%g" % dt)
        params = [I.make_params(n, kT=kT, dt=dt, kernel=4, seed=78, replica_id=r) for r in range(R)]
        sim = I.Sim(params, [1] * R, I.FP32_GRID)
        try:
            for r in range(R):
                sim.set_blobs(r, icm_inputs.uniform_positions(1, n, 1.0, seed=700 + r), m_e=np.array([m_f]))
                sim.set_state(r, flags=I.STATE_EQUILIBRIUM)
            sim.step(int(50 / dt), I.STEP_GRAPH)
            acc = []
            for _ in range(int(500 / dt) // 5):
                sim.step(5, I.STEP_GRAPH)
                acc.append([sim.get_state(r, want_v=False, want_diag=False)["u"][0] ** 2 for r in range(R)])
        finally:
            sim.close()
        per = np.asarray(acc).mean(axis=(0, 2)) * m / kT
        c0[dt] = (per.mean(), per.std(ddof=1) / np.sqrt(R))
        print("dt=%g: C(0+) m / kT = %.4f +- %.4f (paper %.2f)" % (dt, *c0[dt], target), flush=True)
    for dt, (mean, se) in c0.items():
        assert abs(mean - target) < 0.03 * target + 3 * se, dt
    assert abs(c0[0.0625][0] - target) < 0.03 * target


def test_light_blob_equipartition_bias_vanishes_with_the_time_step(I):
    """Sec. IV.A: for m_e != 0 the blob velocity variance carries a time-step
    bias that needs a small viscous CFL number to go away. For a light blob
    (m_e = -m_f/2, 64^3, 16 replicas) <u_a^2> m~ / kT is ~1.11 at
    beta = 0.25 and must fall towards 1 as dt is halved, reaching it within
    3% at beta = 1/16."""
    n, kT = (64, 64, 64), 1e-3
    m_f = 1.0 / 0.375 ** 3
    mt = -0.5 * m_f + 1.5 * m_f
    R = 16
    ratios = {}
    for dt in (0.25, 0.125, 0.0625):
        banner("light-blob equipartition dt=%g" % dt)
        params = [I.make_params(n, kT=kT, dt=dt, kernel=4, seed=77, replica_id=r) for r in range(R)]
        sim = I.Sim(params, [1] * R, I.FP32_GRID)
        try:
            for r in range(R):
                sim.set_blobs(r, icm_inputs.uniform_positions(1, n, 1.0, seed=500 + r), m_e=np.array([-0.5 * m_f]))
                sim.set_state(r, flags=I.STATE_EQUILIBRIUM)
            sim.step(int(50 / dt), I.STEP_GRAPH)
            acc = []
            for _ in range(int(500 / dt) // 5):
                sim.step(5, I.STEP_GRAPH)
                acc.append([sim.get_state(r, want_v=False, want_diag=False)["u"][0] ** 2 for r in range(R)])
        finally:
            sim.close()
        per = np.asarray(acc).mean(axis=(0, 2)) * mt / kT
        ratios[dt] = (per.mean(), per.std(ddof=1) / np.sqrt(R))
        print("dt=%g: <u^2> m~/kT = %.4f +- %.4f" % (dt, *ratios[dt]), flush=True)
    assert ratios[0.25][0] > ratios[0.125][0] > ratios[0.0625][0] - 3 * ratios[0.0625][1]
    assert ratios[0.25][0] - 1.0 > 0.05
    assert abs(ratios[0.0625][0] - 1.0) < 0.03
