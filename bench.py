"""Throughput of the MI355X ICM step (cell-steps/s and blob-steps/s).

Default workload (many_blobs_256): 256^3 periodic grid, FP32 grid with FP64
blob state, 4096 neutrally buoyant blobs at seeded uniform positions with
minimum separation 2h, Peskin 4-point kernel, WCA soft-sphere repulsion
(strength 1e-2, cutoff 2h), kT = 1e-3, rho = eta = 1, dt = 0.2, fluid started
from the discrete equilibrium. Inputs are synthetic and resident in HBM when
the timed region starts.

The last stdout line is one compact JSON record: the throughput of the whole
hot path, the roofline of its dominant kernel (average launch duration from
HIP events on the launch stream), the FP64 CPU oracle timed on a bounded
sample (two full steps) of the same workload, and one-line summaries of the
FP64, batched-ensemble and 512^3 legs. The full record of every leg
(advection, statistics, J P S, convergence study, per-kernel phases) is
written to --full-record; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-steps/s and blob-steps/s at 256^3; FP32 vs FP64 and batched vs single"
HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 64 lanes x 2.4 GHz (one full-rate 32-bit op per
# lane per clock), in tera lane-operations per second.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic VALU work of the right-hand-side kernel per cell (issue slots,
# transcendentals at quarter rate): Philox4x32-10 for the six normals
# (1.5 calls x 10 rounds x (2 multiplies 32x32->64 + 2 three-input xor) = 60),
# Box-Muller (3 pairs x 23 = 69), stress divergence (21), viscous and
# inertial terms (24), spread accumulation (3).
RHS_ALG_OPS_PER_CELL = 60 + 69 + 21 + 24 + 3


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(phase, n, nb, kernel, w):
    """Algorithmic HBM bytes of one launch of a phase: each field or
    spectrum element read once and written once."""
    nx, ny, nz = n
    ncell = nx * ny * nz
    nspec = nz * ny * (nx // 2 + 1)
    taps = 3 * kernel ** 3
    if phase == "rhs":
        return 6 * ncell * w                       # read v, write rhs
    if phase == "fft_x_fwd":
        return 3 * ncell * w + 3 * nspec * 2 * w   # read rhs, write spectrum
    if phase in ("fft_y_fwd", "fft_y_inv", "fft_z_solve"):
        return 2 * 3 * nspec * 2 * w               # read + write spectrum
    if phase == "fft_x_inv":
        return 3 * nspec * 2 * w + 3 * ncell * w   # read spectrum, write v
    if phase == "spread":
        return nb * taps * 2 * w                   # read-modify-write of each tap
    if phase == "gather":
        return nb * taps * w
    if phase in ("blob", "forces"):
        return nb * 3 * 8 * 4
    if phase == "field_ops":
        return 2 * 3 * ncell * w
    if phase == "advection":
        return 15 * ncell * w                      # read v, rhs and lag; write rhs and lag
    return 0


PROFILE = os.path.join(ROOT, "profiles", "many_blobs_256_fp32.md")
# every leg's full results (arrays, statistics) go to this file by default;
# stdout ends with a compact line
FULL_RECORD = os.path.join(ROOT, "bench_results", "bench_full.json")
PHASE_KERNEL = {"rhs": "k_rhs_march<float, true>", "fft_z_solve": "k_z_fast<float, 256, 8, 8, 8, 4, 0>",
                "fft_x_fwd": "k_xfwd_fast<float, 256, 16, 16, 16, 1>",
                "fft_x_inv": "k_xinv_fast<float, 256, 16, 16, 16, 1>"}


def source_hash():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1212_6427_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(phase):
    """HBM bytes per launch of a phase's kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when
    the kernel sources changed after the counters were taken."""
    kernel = PHASE_KERNEL.get(phase)
    if kernel is None or not os.path.exists(PROFILE):
        return None
    at_hash, traffic = None, {}
    with open(PROFILE) as fh:
        for line in fh:
            if line.startswith("source hash"):
                at_hash = line.split()[-1]
            elif line.startswith("traffic "):
                name, val = line[len("traffic "):].rsplit(" ", 1)
                traffic[name] = float(val)
    if at_hash != source_hash():
        return None
    return traffic.get(kernel)


# Kernels of one step of the 256^3 FP32 workload (all blobs neutrally
# buoyant, so no inertial-correction launches), each launched once per step.
STEP_KERNELS = ("k_gather_step1<", "k_pairs_cells<", "k_rhs_march<", "k_spread_overflow<",
                "k_xfwd_fast<", "k_y_fast<", "k_z_fast<", "k_xinv_fast<", "k_gather_final<")


def measured_step_traffic():
    """HBM bytes of one whole step from the committed counter summary: the
    scaled FETCH_SIZE + WRITE_SIZE of every kernel the step launches (both y
    passes), or None when the sources changed after the counters were
    taken."""
    if not os.path.exists(PROFILE):
        return None
    at_hash, total, seen = None, 0.0, 0
    with open(PROFILE) as fh:
        for line in fh:
            if line.startswith("source hash"):
                at_hash = line.split()[-1]
            elif line.startswith("traffic "):
                name, val = line[len("traffic "):].rsplit(" ", 1)
                if name.startswith(STEP_KERNELS):
                    total += float(val)
                    seen += 1
    if at_hash != source_hash() or seen < len(STEP_KERNELS) + 1:
        return None
    return total


def setup(I, torch, wl, precision, stream, advection=False):
    n = tuple(wl["n"])
    import icm_inputs
    sigma = wl["wca_cutoff"] / 2 ** (1.0 / 6.0)
    p = I.make_params(n, h=wl["h"], rho=wl["rho"], eta=wl["eta"], kT=wl["kT"], dt=wl["dt"], kernel=wl["kernel"],
                      seed=wl["seed"], wca_eps=wl["wca_eps"], wca_sigma=sigma, advection=advection)
    nb = wl["n_blobs"]
    nbytes = I.icm_workspace_bytes([p], [nb], precision)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    sim = I.Sim([p], [nb], precision, stream=stream.cuda_stream, workspace=ws)
    q = icm_inputs.separated_positions(nb, n, wl["h"], min_sep=wl["min_sep"], seed=wl["seed"])
    sim.set_blobs(0, q)
    sim.set_state(0, flags=I.STATE_EQUILIBRIUM)
    return sim, p, q


def time_steps(torch, sim, stream, steps, flags=0):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    sim.step(steps, flags)
    b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return a.elapsed_time(b) / 1000.0, wall


def profile_phases(sim, steps, n, nb, kernel, w):
    sim.set_timing(True)
    sim.timing(reset=True)
    sim.step(steps)
    t = sim.timing(reset=True)
    sim.set_timing(False)
    phases = {}
    for name, (ms, cnt) in t.items():
        if cnt == 0:
            continue
        avg_s = ms / cnt / 1000.0
        by = algorithmic_bytes(name, n, nb, kernel, w)
        phases[name] = dict(total_ms_per_step=ms / steps, launches_per_step=cnt / steps, avg_launch_us=avg_s * 1e6,
                            alg_bytes_per_launch=by, achieved_GBs=(by / avg_s / 1e9) if avg_s > 0 else None)
    return phases


def ensemble_sims(I, torch, stream, batched, tune=True):
    """The batched ensemble: 96 replicas (32 each of 32^3, 48^3, 64^3), one
    blob each with m_e / m_f drawn from {0, 1, -1/2}, FP32 grid, fluid started
    from the discrete equilibrium. batched: one context holding every replica;
    else one context per replica."""
    import icm_inputs
    wl = icm_inputs.WORKLOADS["batched_ensemble"]
    grids = wl["grids"]
    nrep = len(grids)
    ratios = icm_inputs.excess_mass_ratios(nrep, wl["me_over_mf"], seed=wl["seed"])
    m_f = wl["rho"] * wl["h"] ** 3 / (0.375 ** 3 if wl["kernel"] == 4 else 0.5 ** 3)
    params = [I.make_params(n, h=wl["h"], rho=wl["rho"], eta=wl["eta"], kT=wl["kT"], dt=wl["dt"],
                            kernel=wl["kernel"], seed=wl["seed"], replica_id=r) for r, n in enumerate(grids)]
    blobs = [(icm_inputs.uniform_positions(1, n, wl["h"], seed=wl["seed"] + 1 + r), np.array([ratios[r] * m_f]))
             for r, n in enumerate(grids)]

    def make(ps):
        nbytes = I.icm_workspace_bytes(ps, [1] * len(ps), I.FP32_GRID)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        return I.Sim(ps, [1] * len(ps), I.FP32_GRID, stream=stream.cuda_stream, workspace=ws)

    sims = [make(params)] if batched else [make([pp]) for pp in params]
    for r in range(nrep):
        sim, loc = (sims[0], r) if batched else (sims[r], 0)
        q, me = blobs[r]
        sim.set_blobs(loc, q, m_e=me)
        sim.set_state(loc, flags=I.STATE_EQUILIBRIUM)
    if tune:
        for sim in sims:
            sim.autotune()
    cells = sum(int(np.prod(n)) for n in grids)
    return sims, cells, nrep


def ensemble_leg(I, torch, stream, steps, warmup, tune=True):
    """cell-steps/s of the batched ensemble as one context (one recorded graph
    per step) against the same replicas stepped one context at a time."""
    out = {}
    for mode in ("batched", "single"):
        sims, cells, nrep = ensemble_sims(I, torch, stream, mode == "batched", tune)
        for sim in sims:
            sim.step(warmup, I.STEP_GRAPH)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for sim in sims:
            sim.step(steps, I.STEP_GRAPH)
        b.record(stream)
        torch.cuda.synchronize()
        sec = a.elapsed_time(b) / 1000.0
        wall = time.perf_counter() - t0
        for sim in sims:
            sim.close()
        out[mode] = {"value": cells * steps / sec, "unit": "cell-steps/s", "blob_steps_per_s": nrep * steps / sec,
                     "ms_per_step": sec * 1000.0 / steps, "steps": steps, "wall_s": wall, "contexts": len(sims)}
        log("ensemble %s: %.3f ms/step, %.3e cell-steps/s" % (mode, out[mode]["ms_per_step"], out[mode]["value"]))
    out["replicas"] = nrep
    out["cells"] = cells
    out["speedup_batched_vs_single"] = out["batched"]["value"] / out["single"]["value"]
    return out


def scale_leg(I, torch, stream, steps, tune=True):
    """512^3 with 10^5 three-point blobs, WCA, kT = 1e-3, dt = 0.2, a per-blob
    force F0 x (F0 = 3 pi eta nu Re_P, Re_P = 1) and the opposite uniform force
    density on the fluid: FP32 grid and FP64 runs from the same state; their
    throughput, the largest relative differences of v and u after `steps`
    steps, and the drift of the total momentum (zero net external force)."""
    import icm_inputs
    wl = icm_inputs.WORKLOADS["scale_512"]
    n = tuple(wl["n"])
    nb = wl["n_blobs"]
    h, eta, rho = wl["h"], wl["eta"], wl["rho"]
    sigma = wl["wca_cutoff"] / 2 ** (1.0 / 6.0)
    F0 = 3.0 * np.pi * eta * (eta / rho) * wl["re_p"]
    body = (-nb * F0 / (float(np.prod(n)) * h ** 3), 0.0, 0.0)
    p = I.make_params(n, h=h, rho=rho, eta=eta, kT=wl["kT"], dt=wl["dt"], kernel=wl["kernel"], seed=wl["seed"],
                      wca_eps=wl["wca_eps"], wca_sigma=sigma, body_force=body)
    q = icm_inputs.separated_positions(nb, n, h, min_sep=wl["min_sep"], seed=wl["seed"])
    F = np.zeros((nb, 3))
    F[:, 0] = F0
    out = {"grid": list(n), "n_blobs": nb, "steps": steps}
    sims = {}
    for name, prec in (("fp64", I.FP64), ("fp32", I.FP32_GRID)):
        nbytes = I.icm_workspace_bytes([p], [nb], prec)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        sims[name] = (I.Sim([p], [nb], prec, stream=stream.cuda_stream, workspace=ws), ws)
    s64, s32 = sims["fp64"][0], sims["fp32"][0]
    s64.set_blobs(0, q, f_const=F)
    s64.set_state(0, flags=I.STATE_EQUILIBRIUM)
    v0 = s64.get_state(0, want_diag=False)["v"].astype(np.float32)
    s64.set_state(0, v=v0.astype(np.float64), step=0)
    s32.set_blobs(0, q, f_const=F)
    s32.set_state(0, v=v0, step=0)
    del v0
    if tune:
        s64.autotune()
        s32.autotune()
    p0 = np.asarray(s64.get_state(0, want_v=False)["diag"]["momentum"])
    for name, sim in (("fp64", s64), ("fp32", s32)):
        sec, _ = time_steps(torch, sim, stream, steps, I.STEP_GRAPH)
        out[name] = {"value": float(np.prod(n)) * steps / sec, "unit": "cell-steps/s",
                     "blob_steps_per_s": nb * steps / sec, "ms_per_step": sec * 1000.0 / steps}
        log("scale_512 %s: %.3f ms/step" % (name, out[name]["ms_per_step"]))
    a = s64.get_state(0)
    b = s32.get_state(0)
    scale_v = max(float(np.max(np.abs(a["v"][c]))) for c in range(3))
    out["max_rel_err_v"] = max(float(np.max(np.abs(b["v"][c].astype(np.float64) - a["v"][c]))) for c in range(3)) / scale_v
    out["max_rel_err_u"] = float(np.max(np.abs(b["u"] - a["u"])) / np.max(np.abs(a["u"])))
    mscale = rho * h ** 3 * float(np.sum(np.abs(a["v"])))
    for name, st in (("fp64", a), ("fp32", b)):
        out[name]["momentum_drift_rel"] = float(np.max(np.abs(np.asarray(st["diag"]["momentum"]) - p0)) / mscale)
        out[name]["max_div"] = st["diag"]["max_div"]
    for name in sims:
        sims[name][0].close()
    log("scale_512 fp32 vs fp64 after %d steps: v %.2e, u %.2e" % (steps, out["max_rel_err_v"], out["max_rel_err_u"]))
    return out


def advection_leg(I, torch, stream, wl, steps, warmup, tune=True, flags=None):
    """The benchmark workload with the advective term on (Adams-Bashforth
    lag): step time and the advection kernel against the HBM roofline."""
    n = tuple(wl["n"])
    ncell = int(np.prod(n))
    flags = I.STEP_GRAPH if flags is None else flags
    sim, _, _ = setup(I, torch, wl, I.FP32_GRID, stream, advection=True)
    if tune:
        sim.autotune()
    sim.step(warmup, flags)
    sec, _ = time_steps(torch, sim, stream, steps, flags)
    ph = profile_phases(sim, 10, n, wl["n_blobs"], wl["kernel"], 4)
    diag = sim.get_state(0, want_v=False)["diag"]
    sim.close()
    adv = ph.get("advection", {})
    out = {"value": ncell * steps / sec, "unit": "cell-steps/s", "ms_per_step": sec * 1000.0 / steps,
           "steps": steps, "advect_kernel": adv, "max_div_after": diag["max_div"]}
    if adv.get("achieved_GBs"):
        out["advect_kernel"] = dict(adv, bound="hbm", peak=HBM_PEAK_GBS, frac=adv["achieved_GBs"] / HBM_PEAK_GBS)
    return out


def spring_trajectories(I, stream_handle, wl, combos, dt, k):
    """FP64 GPU trajectories of the spring test, the blob released from rest
    at x0, for each (m_e/m_f, slip) combination: the position after every
    step, shape (len(combos), T/dt, 3). The combinations run as replicas of
    one context; if the numeric flag stops it (a blob moving more than h in
    one step: the step is too large for that blob), each runs in a context
    of its own and a stopped run is all NaN."""
    n = tuple(wl["n"])
    m_f = wl["rho"] * wl["h"] ** 3 / 0.5 ** 3      # 3-point kernel: dV = 8 h^3
    steps = int(round(wl["T"] / dt))

    def run(sub):
        params = [I.make_params(n, h=wl["h"], rho=wl["rho"], eta=wl["eta"], kT=0.0, dt=dt, kernel=wl["kernel"],
                                slip=slip, spring_k=k, replica_id=i) for i, (_, slip) in enumerate(sub)]
        sim = I.Sim(params, [1] * len(sub), I.FP64, stream=stream_handle)
        try:
            for i, (ratio, _) in enumerate(sub):
                sim.set_blobs(i, np.array([wl["x0"]]), m_e=np.array([ratio * m_f]))
            out = np.empty((len(sub), steps, 3))
            for t in range(steps):
                sim.step(1, I.STEP_GRAPH)
                for i in range(len(sub)):
                    out[i, t] = sim.get_state(i, want_v=False, want_diag=False)["q"][0]
            return out
        finally:
            sim.close()

    try:
        return run(combos)
    except I.ICMError as e:
        if e.status != I.E_NUMERIC:
            raise
    out = np.full((len(combos), steps, 3), np.nan)
    for i, c in enumerate(combos):
        try:
            out[i] = run([c])[0]
        except I.ICMError as e:
            if e.status != I.E_NUMERIC:
                raise
    return out


def convergence_errors(I, stream_handle, wl, combos, dts, k):
    """E(dt) of Eq. (E_dt_definition) for each combination: mean distance
    between the run at dt and the run at dt/2 at the same times."""
    runs = {dt: spring_trajectories(I, stream_handle, wl, combos, dt, k) for dt in list(dts) + [dts[-1] / 2]}
    E = np.empty((len(combos), len(dts)))
    for j, dt in enumerate(dts):
        a, b = runs[dt], runs[dt / 2][:, 1::2]
        E[:, j] = np.mean(np.linalg.norm(a - b, axis=2), axis=1)
    return E


def convergence_leg(I, stream):
    """Deterministic temporal convergence of Sec. III.D on the GPU (FP64):
    E(dt) and the observed orders log2(E(dt)/E(dt/2)) for several excess
    masses (slip correction of Eq. (delta_u_nph_visc), k = 0.01), and for
    m_e = 10 m_f the three slip options at larger spring constants."""
    import icm_inputs
    wl = icm_inputs.WORKLOADS["convergence_16"]
    t0 = time.perf_counter()
    ratios = wl["me_over_mf"]
    dts = wl["dts"]
    E = convergence_errors(I, stream.cuda_stream, wl, [(r, I.SLIP_VISCOUS) for r in ratios], dts, wl["spring_k"])
    def num(x):
        return None if not np.isfinite(x) else float(x)

    out = {"dts": list(dts), "spring_k": wl["spring_k"], "slip": "viscous", "by_me_over_mf": {},
           "note": "null: the run at dt or dt/2 stopped on the numeric flag (unstable at that dt)"}
    for i, r in enumerate(ratios):
        out["by_me_over_mf"]["%g" % r] = {"E": [num(x) for x in E[i]],
                                          "order": [num(np.log2(E[i, j] / E[i, j + 1])) for j in range(len(dts) - 1)]}
    st = wl["slip_test"]
    names = {I.SLIP_NONE: "none", I.SLIP_VISCOUS: "viscous", I.SLIP_FULL: "full"}
    slips = [I.SLIP_NONE, I.SLIP_VISCOUS, I.SLIP_FULL]
    out["slip_options"] = {}
    for k, dts_k in zip(st["spring_k"], st["dts"]):
        Ek = convergence_errors(I, stream.cuda_stream, wl, [(st["me_over_mf"], s) for s in slips], dts_k, k)
        out["slip_options"]["k=%g" % k] = {"dts": list(dts_k), "me_over_mf": st["me_over_mf"],
                                           "E": {names[s]: [num(x) for x in Ek[i]] for i, s in enumerate(slips)}}
    out["wall_s"] = time.perf_counter() - t0
    return out


def cell_histogram_bias(frac):
    """Density near the cell corners (grid nodes) over density near the cell
    centre, minus one: positions within a cell, frac in [0, 1)^3; each region
    is the cube of half the cell's side around its point (1/8 of the cell)."""
    d_corner = np.minimum(frac, 1.0 - frac)
    corner = np.all(d_corner < 0.25, axis=-1)
    centre = np.all(np.abs(frac - 0.5) < 0.25, axis=-1)
    return float(corner.sum() / max(centre.sum(), 1) - 1.0), int(corner.sum()), int(centre.sum())


def node_harmonic(frac):
    """Amplitude eps of the density 1 + eps sum_a cos(2 pi f_a) over the cell
    (f: position within the cell): (2/3) times the sample mean of
    sum_a cos(2 pi f_a). Positive: blobs linger near the grid nodes."""
    return float(np.mean(np.sum(np.cos(2 * np.pi * frac), axis=-1)) * 2.0 / 3.0)


def drift_bias_run(I, stream_handle, wl, kernel, steps, every, replicas):
    """Ideal gas of neutrally buoyant blobs (no forces) at equilibrium, with
    and without the thermal drift (even / odd replicas), batched in one
    context: per replica, the positions within a cell sampled every `every`
    steps after a relaxation of `steps` // 10 steps."""
    import icm_inputs
    n = tuple(wl["n"])
    nb = wl["n_blobs"]
    params = [I.make_params(n, h=wl["h"], rho=wl["rho"], eta=wl["eta"], kT=wl["kT"], dt=wl["dt"], kernel=kernel,
                            thermal_drift=(r % 2 == 0), seed=wl["seed"], replica_id=r) for r in range(replicas)]
    sim = I.Sim(params, [nb] * replicas, I.FP32_GRID, stream=stream_handle)
    try:
        for r in range(replicas):
            sim.set_blobs(r, icm_inputs.uniform_positions(nb, n, wl["h"], seed=wl["seed"] + 1 + r))
            sim.set_state(r, flags=I.STATE_EQUILIBRIUM)
        sim.step(steps // 10, I.STEP_GRAPH)
        samples = [[] for _ in range(replicas)]
        for _ in range(steps // every):
            sim.step(every, I.STEP_GRAPH)
            for r in range(replicas):
                q = sim.get_state(r, want_v=False, want_diag=False)["q"] / wl["h"]
                samples[r].append(q - np.floor(q))
        return [np.concatenate(x) for x in samples]
    finally:
        sim.close()


def drift_bias_summary(per_replica):
    """Pooled corner/centre ratio and the node harmonic with its standard
    error from the spread over (independent) replicas."""
    eps = np.array([node_harmonic(f) for f in per_replica])
    ratio, c, z = cell_histogram_bias(np.concatenate(per_replica))
    return {"corner_over_centre_minus_1": ratio, "corner_centre_counts": [c, z],
            "node_harmonic": float(eps.mean()), "node_harmonic_se": float(eps.std(ddof=1) / np.sqrt(len(eps)))}


def drift_bias_leg(I, stream_handle, steps=None):
    """The thermal-drift check of App. B.2: positions of freely diffusing
    blobs projected on one grid cell must be uniform; without the drift they
    pile up near the grid nodes."""
    import icm_inputs
    wl = icm_inputs.WORKLOADS["drift_bias_16"]
    steps = steps or wl["steps"]
    t0 = time.perf_counter()
    out = {"grid": list(wl["n"]), "n_blobs": wl["n_blobs"], "replicas_per_case": wl["replicas"] // 2,
           "steps": steps, "sample_every": wl["every"], "kT": wl["kT"], "dt": wl["dt"], "kernels": {}}
    for kernel in wl["kernels"]:
        per = drift_bias_run(I, stream_handle, wl, kernel, steps, wl["every"], wl["replicas"])
        out["kernels"]["%d-point" % kernel] = {"with_drift": drift_bias_summary(per[0::2]),
                                               "without_drift": drift_bias_summary(per[1::2])}
    out["wall_s"] = time.perf_counter() - t0
    return out


def pair_histogram(q, L, rmax, nbins):
    """Pair counts of one configuration on nbins bins of [0, rmax)
    (minimum-image distances in a periodic cube of side L)."""
    from scipy.spatial import cKDTree
    x = np.mod(q, L)
    x[x >= L] = 0.0
    d = cKDTree(x, boxsize=L).sparse_distance_matrix(cKDTree(x, boxsize=L), rmax, output_type="ndarray")
    r = d["v"][d["i"] < d["j"]]
    return np.histogram(r, bins=nbins, range=(0.0, rmax))[0].astype(np.float64)


def gr_from_counts(counts, samples, n, L, rmax):
    """g(r): pair counts over the ideal-gas count of each spherical shell."""
    nbins = counts.shape[-1]
    edges = np.linspace(0.0, rmax, nbins + 1)
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    return counts / (samples * 0.5 * n * (n - 1) * shell / L ** 3)


def rdf_run(I, stream_handle, wl, ratio, replicas, steps, every):
    """GPU dynamics of the WCA suspension of Table RDF: `replicas`
    independent boxes batched in one context (FP32 grid), equilibrium fluid,
    blobs from seeded positions at least min_sep apart; after `relax` steps,
    g(r) of each replica from configurations every `every` steps."""
    import icm_inputs
    n = tuple(wl["n"])
    nb = wl["n_blobs"]
    L = n[0] * wl["h"]
    m_f = wl["rho"] * wl["h"] ** 3 / 0.5 ** 3 if wl["kernel"] == 3 else wl["rho"] * wl["h"] ** 3 / 0.375 ** 3
    params = [I.make_params(n, h=wl["h"], rho=wl["rho"], eta=wl["eta"], kT=wl["kT"], dt=wl["dt"], kernel=wl["kernel"],
                            wca_eps=wl["wca_eps"], wca_sigma=wl["wca_sigma"], seed=wl["seed"], replica_id=r)
              for r in range(replicas)]
    sim = I.Sim(params, [nb] * replicas, I.FP32_GRID, stream=stream_handle)
    try:
        for r in range(replicas):
            q = icm_inputs.separated_positions(nb, n, wl["h"], min_sep=wl["min_sep"], seed=wl["seed"] + 1 + r)
            sim.set_blobs(r, q, m_e=np.full(nb, ratio * m_f))
            sim.set_state(r, flags=I.STATE_EQUILIBRIUM)
        sim.step(wl["relax"], I.STEP_GRAPH)
        counts = np.zeros((replicas, wl["nbins"]))
        samples = steps // every
        for _ in range(samples):
            sim.step(every, I.STEP_GRAPH)
            for r in range(replicas):
                q = sim.get_state(r, want_v=False, want_diag=False)["q"]
                counts[r] += pair_histogram(q, L, wl["rmax"], wl["nbins"])
        return gr_from_counts(counts, samples, nb, L, wl["rmax"])
    finally:
        sim.close()


def rdf_leg(I, stream_handle, steps=None):
    """Equilibrium pair structure of the WCA suspension (Sec. IV.A, Table
    RDF) from the GPU dynamics, for each excess mass, with the replica
    spread as the statistical error."""
    import icm_inputs
    wl = icm_inputs.WORKLOADS["rdf_32"]
    steps = steps or wl["steps"]
    t0 = time.perf_counter()
    r = (np.arange(wl["nbins"]) + 0.5) * wl["rmax"] / wl["nbins"]
    out = {"grid": list(wl["n"]), "n_blobs": wl["n_blobs"], "dt": wl["dt"], "kT": wl["kT"], "wca_eps": wl["wca_eps"],
           "wca_sigma": wl["wca_sigma"], "replicas": wl["replicas"], "steps": steps, "sample_every": wl["every"],
           "r": [float(x) for x in r], "g": {}}
    for ratio in wl["me_over_mf"]:
        g = rdf_run(I, stream_handle, wl, ratio, wl["replicas"], steps, wl["every"])
        out["g"]["m_e/m_f=%g" % ratio] = {"mean": [float(x) for x in g.mean(0)],
                                          "se": [float(x) for x in g.std(0, ddof=1) / np.sqrt(g.shape[0])]}
    out["wall_s"] = time.perf_counter() - t0
    return out


def rdf_vs_reference(res):
    """Largest |g - g_MC| over 1.8 < r < 4.5 and the mean difference over
    the contact peak (2.1 < r < 2.7) against the stored Monte Carlo g(r)."""
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "rdf_wca_mc.json")))
    r = np.asarray(ref["r"])
    g_mc = np.asarray(ref["g"])
    band, peak = (r > 1.8) & (r < 4.5), (r > 2.1) & (r < 2.7)
    out = {}
    for name, v in res["g"].items():
        d = np.asarray(v["mean"]) - g_mc
        out[name] = {"max_abs_diff": float(np.max(np.abs(d[band]))), "mean_diff_contact_peak": float(np.mean(d[peak]))}
    return out


def jps_columns(I, stream_handle, n, kernel, q_list, kicked=0):
    """(3 dV / 2) J_i P S_k e_b on the GPU for each configuration in q_list
    (an (n_blobs, 3) array per entry) and b = x, y, z: one replica per
    (configuration, b) in one FP64 context. Blob `kicked` gets the impulse
    m~_f e_b (ICM_BLOBS_KICK: v = P S (m~_f e_b) / rho); one inviscid,
    deterministic step of dt = 1e-12 then leaves v unchanged and reports
    u_i = J_i v for every blob. Returns an array (len(q_list), n_blobs, 3, 3)
    with [c, i, :, b] the velocity of blob i for the kick along b."""
    nq = len(q_list)
    nb = q_list[0].shape[0]
    params = [I.make_params(n, eta=0.0, kT=0.0, dt=1e-12, kernel=kernel, replica_id=r) for r in range(3 * nq)]
    sim = I.Sim(params, [nb] * (3 * nq), I.FP64, stream=stream_handle)
    try:
        for c, q in enumerate(q_list):
            for b in range(3):
                u0 = np.zeros((nb, 3))
                u0[kicked, b] = 1.0
                sim.set_blobs(3 * c + b, q, u=u0, flags=I.BLOBS_KICK)
        sim.step(1, I.STEP_GRAPH)
        out = np.empty((nq, nb, 3, 3))
        for c in range(nq):
            for b in range(3):
                out[c, :, :, b] = sim.get_state(3 * c + b, want_v=False, want_diag=False)["u"]
        return out
    finally:
        sim.close()


def jps_leg(I, stream_handle):
    """Translational invariance of J P S (Sec. III.A.2) on the GPU: for
    random positions in a 32^3 box, the deviation of (3 dV / 2) J P S from
    the identity (diagonal and off-diagonal), and the pair term
    (3 dV / 2) J_i P S_j against the separation, for both kernels."""
    t0 = time.perf_counter()
    rng = np.random.default_rng(18)
    n = (32, 32, 32)
    out = {"grid": list(n), "kernels": {}}
    qs = [rng.uniform(0.0, 32.0, (1, 3)) for _ in range(64)]
    seps = [2.0, 3.0, 4.0, 5.0, 6.0, 8.0, 10.0, 12.0]
    base = np.array([10.3, 11.7, 12.2])
    for kernel in (3, 4):
        M = jps_columns(I, stream_handle, n, kernel, qs)[:, 0] - np.eye(3)[None]
        diag = np.abs(np.diagonal(M, axis1=1, axis2=2))
        off = np.abs(M - np.einsum("cii->ci", M)[:, :, None] * np.eye(3)[None])
        pairs = {}
        for name, d in (("x", np.array([1.0, 0.0, 0.0])), ("diagonal", np.ones(3) / np.sqrt(3.0))):
            cfg = [np.stack([base, base + l * d]) for l in seps]
            P = jps_columns(I, stream_handle, n, kernel, cfg, kicked=1)[:, 0]
            pairs[name] = [float(np.max(np.abs(x))) for x in P]
        out["kernels"]["%d-point" % kernel] = {
            "positions": len(qs), "diag_dev_mean": float(np.mean(np.diagonal(M, axis1=1, axis2=2))),
            "diag_dev_max": float(diag.max()), "offdiag_max": float(off.max()),
            "pair_separations": seps, "pair_max_entry": pairs}
    out["wall_s"] = time.perf_counter() - t0
    return out


def mobility_columns(I, stream_handle, n, kernel, qs, F=1e-8, dt=1e6, kernel_shift=0.0):
    """Periodic steady Stokes mobility of one blob per configuration on the
    GPU (FP64): the blob at q pushed by F e_b, the fluid by -F e_b / V (zero
    net force, so no mean flow), one deterministic step from rest. With
    rho / dt ~ 0 the Crank-Nicolson solve returns twice the Stokes velocity,
    and the reported blob velocity J v gives 2 mu F e_b. Returns mu as an
    array (len(qs), 3, 3), [c, :, b] for the force along b."""
    nq = len(qs)
    vol = float(np.prod(n))
    params = []
    for c in range(nq):
        for b in range(3):
            body = [0.0, 0.0, 0.0]
            body[b] = -F / vol
            params.append(I.make_params(n, eta=1.0, rho=1.0, kT=0.0, dt=dt, kernel=kernel, body_force=body,
                                        replica_id=3 * c + b, kernel_shift=kernel_shift))
    sim = I.Sim(params, [1] * (3 * nq), I.FP64, stream=stream_handle)
    try:
        for c, q in enumerate(qs):
            for b in range(3):
                f = np.zeros((1, 3))
                f[0, b] = F
                sim.set_blobs(3 * c + b, np.asarray(q).reshape(1, 3), f_const=f)
        sim.step(1, I.STEP_GRAPH)
        mu = np.empty((nq, 3, 3))
        for c in range(nq):
            for b in range(3):
                mu[c, :, b] = sim.get_state(3 * c + b, want_v=False, want_diag=False)["u"][0] / (2.0 * F)
        return mu
    finally:
        sim.close()


def hydrodynamic_radius(mu, L, eta=1.0):
    """R_H from a periodic mobility with Hasimoto's finite-size correction,
    mu = (1 - 2.837297 R/L + (4 pi / 3)(R/L)^3) / (6 pi eta R)."""
    from scipy.optimize import brentq
    f = lambda R: (1 - 2.837297 * R / L + 4.18879 * (R / L) ** 3) / (6 * np.pi * eta * R) - mu
    return brentq(f, 0.05, 0.45 * L)


def hydrodynamic_radius_leg(I, stream_handle):
    """R_H against the box size and the position within a cell
    (Sec. III.A.2): 16 random positions per box, both kernels."""
    t0 = time.perf_counter()
    rng = np.random.default_rng(19)
    out = {"positions_per_box": 16, "kernels": {}}
    for kernel in (3, 4):
        rows = {}
        for N in (16, 32, 64, 128):
            qs = [rng.uniform(0.0, N, 3) for _ in range(16)]
            mu = mobility_columns(I, stream_handle, (N, N, N), kernel, qs)
            r = np.array([hydrodynamic_radius(np.trace(m) / 3.0, float(N)) for m in mu])
            rows[str(N)] = {"R_H_mean": float(r.mean()), "R_H_min": float(r.min()), "R_H_max": float(r.max())}
        out["kernels"]["%d-point" % kernel] = rows
    # split three-point kernel (Sec. III.A.2): R_H against the shift s / h
    rows = {}
    N = 32
    for s in (0.0, 0.25, 0.5, 0.75, 1.0):
        qs = [rng.uniform(0.0, N, 3) for _ in range(16)]
        mu = mobility_columns(I, stream_handle, (N, N, N), 3, qs, kernel_shift=s)
        r = np.array([hydrodynamic_radius(np.trace(m) / 3.0, float(N)) for m in mu])
        rows["%g" % s] = {"R_H_mean": float(r.mean()), "R_H_min": float(r.min()), "R_H_max": float(r.max())}
    out["split_3pt_vs_shift_32"] = rows
    out["wall_s"] = time.perf_counter() - t0
    return out


def vacf(series, lags):
    """Velocity autocorrelation <u(t) . u(t + lag)> / 3 of a (steps, 3)
    series, averaged over the time origins."""
    u = np.asarray(series)
    return np.array([np.mean(np.sum(u[: len(u) - L] * u[L:], axis=1)) / 3.0 for L in lags])


def single_blob_leg(I, torch, stream, steps, tune=True):
    """The fluctuating single-blob workload: 128^3, FP32 grid, 4-point kernel,
    kT = 1e-3, dt = 0.25, one blob with m_e / m_f in {0, 1, -1/2} (one replica
    each, in one context), fluid from the discrete equilibrium. After 200
    relaxation steps, `steps` steps with the blob velocity recorded every step:
    equipartition <u_a^2> m~ / kT (Sec. II.F; a dt-dependent bias is expected
    for m_e != 0) and the normalised velocity autocorrelation."""
    import icm_inputs
    wl = icm_inputs.WORKLOADS["single_blob_128"]
    n = tuple(wl["n"])
    ratios = wl["me_over_mf"]
    m_f = wl["rho"] * wl["h"] ** 3 / 0.375 ** 3
    params = [I.make_params(n, h=wl["h"], rho=wl["rho"], eta=wl["eta"], kT=wl["kT"], dt=wl["dt"],
                            kernel=wl["kernel"], seed=wl["seed"], replica_id=r) for r in range(len(ratios))]
    nbytes = I.icm_workspace_bytes(params, [1] * len(params), I.FP32_GRID)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    sim = I.Sim(params, [1] * len(params), I.FP32_GRID, stream=stream.cuda_stream, workspace=ws)
    q = icm_inputs.uniform_positions(1, n, wl["h"], seed=wl["seed"] + 1)
    for r, ratio in enumerate(ratios):
        sim.set_blobs(r, q, m_e=np.array([ratio * m_f]))
        sim.set_state(r, flags=I.STATE_EQUILIBRIUM)
    if tune:
        sim.autotune()
    sim.step(200, I.STEP_GRAPH)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    series = {r: np.empty((steps, 3)) for r in range(len(ratios))}
    for t in range(steps):
        sim.step(1, I.STEP_GRAPH)
        for r in range(len(ratios)):
            series[r][t] = sim.get_state(r, want_v=False, want_diag=False)["u"][0]
    wall = time.perf_counter() - t0
    sim.close()
    lags = [0, 1, 2, 5, 10, 20, 50, 100]
    out = {"grid": list(n), "steps": steps, "wall_s_with_recording": wall, "lags_steps": lags, "classes": {}}
    kT = wl["kT"]
    for r, ratio in enumerate(ratios):
        mt = ratio * m_f + 1.5 * m_f
        c = vacf(series[r], lags)
        out["classes"]["m_e/m_f=%g" % ratio] = {"equipartition_u2_mt_over_kT": float(c[0] * mt / kT),
                                                 "vacf_normalised": [float(x / c[0]) for x in c]}
    log("single_blob_128: equipartition %s" % {k: round(v["equipartition_u2_mt_over_kT"], 3)
                                                for k, v in out["classes"].items()})
    return out


def ensemble_vacf_leg(I, torch, stream, steps, per_shape=4, tune=True):
    """Velocity autocorrelation of the batched ensemble (FP32 grid, one
    context) against the same replicas on the single-replica FP64 path (same
    Philox keys and equilibrium initial fields, so nearly the same
    trajectories): per_shape replicas of each grid shape on both paths."""
    import icm_inputs
    wl = icm_inputs.WORKLOADS["batched_ensemble"]
    grids = wl["grids"]
    nrep = len(grids)
    ratios = icm_inputs.excess_mass_ratios(nrep, wl["me_over_mf"], seed=wl["seed"])
    m_f = wl["rho"] * wl["h"] ** 3 / 0.375 ** 3
    params = [I.make_params(n, h=wl["h"], rho=wl["rho"], eta=wl["eta"], kT=wl["kT"], dt=wl["dt"],
                            kernel=wl["kernel"], seed=wl["seed"], replica_id=r) for r, n in enumerate(grids)]
    qs = [icm_inputs.uniform_positions(1, n, wl["h"], seed=wl["seed"] + 1 + r) for r, n in enumerate(grids)]
    picked = []
    for shape in sorted(set(grids)):
        picked += [r for r, n in enumerate(grids) if n == shape][:per_shape]

    def make(ps, prec):
        nbytes = I.icm_workspace_bytes(ps, [1] * len(ps), prec)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        return I.Sim(ps, [1] * len(ps), prec, stream=stream.cuda_stream, workspace=ws)

    batched = make(params, I.FP32_GRID)
    for r in range(nrep):
        batched.set_blobs(r, qs[r], m_e=np.array([ratios[r] * m_f]))
        batched.set_state(r, flags=I.STATE_EQUILIBRIUM)
    singles = {}
    for r in picked:
        sm = make([params[r]], I.FP64)
        sm.set_blobs(0, qs[r], m_e=np.array([ratios[r] * m_f]))
        sm.set_state(0, flags=I.STATE_EQUILIBRIUM)
        singles[r] = sm
    if tune:
        batched.autotune()
        for sm in singles.values():
            sm.autotune()
    ub = {r: np.empty((steps, 3)) for r in range(nrep)}
    us = {r: np.empty((steps, 3)) for r in picked}
    for t in range(steps):
        batched.step(1, I.STEP_GRAPH)
        for r in range(nrep):
            ub[r][t] = batched.get_state(r, want_v=False, want_diag=False)["u"][0]
        for r, sm in singles.items():
            sm.step(1, I.STEP_GRAPH)
            us[r][t] = sm.get_state(0, want_v=False, want_diag=False)["u"][0]
    batched.close()
    for sm in singles.values():
        sm.close()
    lags = [0, 1, 2, 5, 10, 20, 50]
    kT = wl["kT"]
    out = {"steps": steps, "replicas_batched": nrep, "replicas_fp64_single": len(picked), "lags_steps": lags,
           "classes": {}}
    worst = 0.0
    for shape in sorted(set(grids)):
        for ratio in wl["me_over_mf"]:
            members = [r for r in range(nrep) if grids[r] == shape and ratios[r] == ratio]
            if not members:
                continue
            mt = ratio * m_f + 1.5 * m_f
            cb = np.mean([vacf(ub[r], lags) for r in members], axis=0)
            entry = {"replicas": len(members), "vacf_fp32_batched": [float(x * mt / kT) for x in cb]}
            both = [r for r in members if r in us]
            if both:
                c32 = np.mean([vacf(ub[r], lags) for r in both], axis=0)
                c64 = np.mean([vacf(us[r], lags) for r in both], axis=0)
                # both lists over the replicas run on both paths (the FP32
                # list above averages every replica of the class)
                entry["vacf_fp32_batched_same_replicas"] = [float(x * mt / kT) for x in c32]
                entry["vacf_fp64_single_same_replicas"] = [float(x * mt / kT) for x in c64]
                d = float(np.max(np.abs(c32 - c64)) / abs(c64[0]))
                entry["max_diff_rel_c0"] = d
                worst = max(worst, d)
            out["classes"]["%d^3, m_e/m_f=%g" % (shape[0], ratio)] = entry
    out["max_diff_rel_c0"] = worst
    log("ensemble VACF: FP32 batched vs FP64 single, largest difference %.2e of C(0)" % worst)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, seed_positions, steps=2):
    """The FP64 oracle, untuned, on `steps` full steps of the same workload,
    timed twice: with scipy.fft's transforms spread over every host core the
    process may use (numpy's element-wise work stays on one thread), and on
    one core. About 10 s of CPU work each."""
    import scipy.fft as sfft
    from oracle import icm as O
    n = tuple(wl["n"])
    sigma = wl["wca_cutoff"] / 2 ** (1.0 / 6.0)
    p = O.Params(n=n, h=wl["h"], rho=wl["rho"], eta=wl["eta"], kT=wl["kT"], dt=wl["dt"], kernel=wl["kernel"],
                 seed=wl["seed"], wca_eps=wl["wca_eps"], wca_sigma=sigma)
    st0 = O.new_state(p, seed_positions)
    st0.v = O.equilibrium_field(p)
    cores = len(os.sched_getaffinity(0))
    ncell = int(np.prod(n))
    runs = {}
    for name, workers in (("all_cores", cores), ("one_core", 1)):
        st = st0
        with sfft.set_workers(workers):
            t0 = time.perf_counter()
            for _ in range(steps):
                st = O.step(p, st)
            dt = time.perf_counter() - t0
        runs[name] = dict(value=ncell * steps / dt, seconds=dt, fft_workers=workers,
                          blob_steps_per_s=wl["n_blobs"] * steps / dt)
    a = runs["all_cores"]
    return dict(value=a["value"], unit="cell-steps/s", cores=cores, kind="oracle",
                sample="%d full steps of %s (%dx%dx%d, %d blobs) in the FP64 numpy/scipy oracle, %.1f s with "
                       "scipy.fft on %d worker threads (element-wise numpy on one), %.1f s on one core"
                       % (steps, "many_blobs_256", n[0], n[1], n[2], wl["n_blobs"], a["seconds"], cores,
                          runs["one_core"]["seconds"]),
                cpu_model=cpu_model(), one_core=runs["one_core"], all_cores=a)


def cpu_samples():
    """The FP64 oracle, untuned, on bounded samples of the other workloads,
    with scipy.fft on every host core the process may use, in cell-steps/s
    (the initial fields are built outside the timed region):
    plain_fp64_32 all 10 steps; single_blob_128 two steps for each of its
    three excess masses; batched_ensemble one step of each of its 96
    replicas. scale_512 is not sampled: the oracle's WCA forces are all
    pairs (10^10 at 10^5 blobs, minutes per step) and its FP64 512^3 step
    holds about 25 GB of fields."""
    import scipy.fft as sfft
    import icm_inputs
    from oracle import icm as O
    cores = len(os.sched_getaffinity(0))
    W = icm_inputs.WORKLOADS

    def params(wl, n, replica=0):
        return O.Params(n=tuple(n), h=wl["h"], rho=wl["rho"], eta=wl["eta"], kT=wl["kT"], dt=wl["dt"],
                        kernel=wl["kernel"], seed=wl["seed"], replica=replica)

    def run(p, st, steps):
        t0 = time.perf_counter()
        for _ in range(steps):
            st = O.step(p, st)
        return time.perf_counter() - t0

    res = {}
    with sfft.set_workers(cores):
        wl = W["plain_fp64_32"]
        p = params(wl, wl["n"])
        q = icm_inputs.uniform_positions(1, wl["n"], wl["h"], seed=wl["seed"] + 1)
        u0 = np.array([wl["kick"]], dtype=np.float64)
        st = O.new_state(p, q, u=u0, f_const=np.array([wl["f_const"]], dtype=np.float64))
        st.v = O.kick_field(p, q, u0, st.m_e)
        sec = run(p, st, wl["steps"])
        res["plain_fp64_32"] = dict(value=int(np.prod(wl["n"])) * wl["steps"] / sec, seconds=sec,
                                    sample="all %d steps" % wl["steps"])

        wl = W["single_blob_128"]
        q = icm_inputs.uniform_positions(1, wl["n"], wl["h"], seed=wl["seed"] + 1)
        sec = 0.0
        for r, ratio in enumerate(wl["me_over_mf"]):
            p = params(wl, wl["n"], r)
            st = O.new_state(p, q, m_e=np.array([ratio * p.m_f]))
            st.v = O.equilibrium_field(p)
            st.u = O.interp(p, st.v, q)
            sec += run(p, st, 2)
        steps = 2 * len(wl["me_over_mf"])
        res["single_blob_128"] = dict(value=int(np.prod(wl["n"])) * steps / sec, seconds=sec,
                                      sample="2 steps for each of m_e/m_f = %s" % (wl["me_over_mf"],))

        wl = W["batched_ensemble"]
        ratios = icm_inputs.excess_mass_ratios(len(wl["grids"]), wl["me_over_mf"], seed=wl["seed"])
        sec, cells = 0.0, 0
        for r, n in enumerate(wl["grids"]):
            p = params(wl, n, r)
            q = icm_inputs.uniform_positions(1, n, wl["h"], seed=wl["seed"] + 1 + r)
            st = O.new_state(p, q, m_e=np.array([ratios[r] * p.m_f]))
            st.v = O.equilibrium_field(p)
            sec += run(p, st, 1)
            cells += int(np.prod(n))
        res["batched_ensemble"] = dict(value=cells / sec, seconds=sec,
                                       sample="one step of each of the %d replicas" % len(wl["grids"]))
    for k, v in res.items():
        v.update(unit="cell-steps/s", cores=cores, kind="oracle")
    res["scale_512"] = dict(value=None, sample="not sampled: all-pairs WCA over 10^5 blobs and ~25 GB of "
                                               "FP64 fields per step in the oracle")
    return res


def compact_record(out):
    """The headline keys plus one-line summaries of the other legs: the last
    stdout line, a few KB."""
    keep = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
            "vs_baseline", "dtype", "data", "config", "blob_steps_per_s", "ms_per_step_median_of_5",
            "step_hbm_fraction", "step_traffic")
    c = {k: out[k] for k in keep if k in out}
    r = out["roofline"]
    c["roofline"] = {k: r[k] for k in ("bound", "kernel", "achieved", "peak", "unit", "frac", "traffic",
                                       "avg_launch_us", "hbm_achieved_GBs") if k in r}
    if "cpu_baseline" in out:
        cb = out["cpu_baseline"]
        c["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "cpu_model")}
        c["cpu_baseline"]["one_core_value"] = cb["one_core"]["value"]
    if "cpu_samples" in out:
        c["cpu_samples"] = {k: v["value"] for k, v in out["cpu_samples"].items()}
    c["phases_us"] = {k: round(v["avg_launch_us"], 1) for k, v in out.get("phases", {}).items()}
    if "fp64" in out:
        f = out["fp64"]
        c["fp64"] = {"value": f["value"], "ms_per_step": f["ms_per_step"], "steps": f["steps"],
                     "step_hbm_fraction": f.get("step_hbm_fraction")}
    if "ensemble" in out:
        e = out["ensemble"]
        c["ensemble"] = {"replicas": e["replicas"], "cells": e["cells"],
                         "batched_ms_per_step": e["batched"]["ms_per_step"], "batched_value": e["batched"]["value"],
                         "single_ms_per_step": e["single"]["ms_per_step"],
                         "speedup_batched_vs_single": e["speedup_batched_vs_single"]}
    if "scale_512" in out:
        s = out["scale_512"]
        c["scale_512"] = {"fp32_ms_per_step": s["fp32"]["ms_per_step"], "fp64_ms_per_step": s["fp64"]["ms_per_step"],
                          "max_rel_err_v": s["max_rel_err_v"], "max_rel_err_u": s["max_rel_err_u"],
                          "momentum_drift_rel_fp32": s["fp32"]["momentum_drift_rel"],
                          "momentum_drift_rel_fp64": s["fp64"]["momentum_drift_rel"]}
    if "advection" in out:
        c["advection_ms_per_step"] = out["advection"]["ms_per_step"]
    return c


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="many_blobs_256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--ensemble-steps", type=int, default=200)
    ap.add_argument("--no-scale", action="store_true")
    ap.add_argument("--no-statistics", action="store_true",
                    help="skip the single-blob, thermal-drift and ensemble velocity-autocorrelation legs")
    ap.add_argument("--single-blob-steps", type=int, default=10000)
    ap.add_argument("--vacf-steps", type=int, default=1000)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default FFT launch shapes")
    ap.add_argument("--eager", action="store_true", help="launch the step's kernels one by one instead of replaying "
                                                         "the recorded step graph")
    ap.add_argument("--scale-steps", type=int, default=200)
    ap.add_argument("--no-advection", action="store_true", help="skip the leg with the advective term on")
    ap.add_argument("--no-convergence", action="store_true", help="skip the temporal-convergence study")
    ap.add_argument("--no-jps", action="store_true", help="skip the J P S invariance diagnostics")
    ap.add_argument("--advection-steps", type=int, default=100)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--full-record", default=FULL_RECORD, help="file for the full record of every leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device-to-device tensor copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import icm_inputs
    import paper_1212_6427_amd.icm as I

    wl = icm_inputs.WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 256 MiB read + 256 MiB written")
        del src, dst
    stream = torch.cuda.current_stream()
    n = tuple(wl["n"])
    ncell = int(np.prod(n))
    nb = wl["n_blobs"]

    log("setup FP32-grid context %s with %d blobs" % (n, nb))
    sim, p, q = setup(I, torch, wl, I.FP32_GRID, stream)
    tune = None
    if not args.no_autotune:
        tune = sim.autotune()
        log("autotuned FFT launch shapes: %s" % tune)
    step_flags = 0 if args.eager else I.STEP_GRAPH
    log("warmup %d steps" % args.warmup)
    sim.step(args.warmup, step_flags)
    log("timing %d steps (%s)" % (args.steps, "eager launches" if args.eager else "recorded step graph"))
    sec, wall = time_steps(torch, sim, stream, args.steps, step_flags)
    ms_per_step = sec * 1000.0 / args.steps
    value = ncell * args.steps / sec
    log("FP32 grid: %.3f ms/step, %.3e cell-steps/s" % (ms_per_step, value))
    # the same K steps timed four more times: run-to-run spread of the figure above
    repeats = [ms_per_step] + [time_steps(torch, sim, stream, args.steps, step_flags)[0] * 1000.0 / args.steps
                               for _ in range(4)]
    log("FP32 grid, five timings: %s ms/step" % ", ".join("%.4f" % x for x in repeats))
    phases = profile_phases(sim, args.profile_steps, n, nb, wl["kernel"], 4)
    diag = sim.get_state(0, want_v=False)["diag"]
    sim.close()
    dom = max(phases.items(), key=lambda kv: kv[1]["total_ms_per_step"])
    dom_name, dom_v = dom
    if dom_name == "rhs":
        # bound by integer and transcendental VALU work (Philox, Box-Muller)
        ops = RHS_ALG_OPS_PER_CELL * ncell
        achieved = ops / (dom_v["avg_launch_us"] * 1e-6) / 1e12
        roofline = dict(bound="alu", kernel="k_rhs_march", achieved=achieved, peak=VALU_PEAK_TOPS, unit="TOP/s",
                        frac=achieved / VALU_PEAK_TOPS, traffic=measured_traffic(dom_name),
                        alg_ops_per_launch=ops, avg_launch_us=dom_v["avg_launch_us"],
                        hbm_achieved_GBs=dom_v["achieved_GBs"], alg_bytes_per_launch=dom_v["alg_bytes_per_launch"])
    else:
        roofline = dict(bound="hbm", kernel=dom_name, achieved=dom_v["achieved_GBs"], peak=HBM_PEAK_GBS,
                        unit="GB/s", frac=dom_v["achieved_GBs"] / HBM_PEAK_GBS, traffic=measured_traffic(dom_name),
                        alg_bytes_per_launch=dom_v["alg_bytes_per_launch"], avg_launch_us=dom_v["avg_launch_us"])
    step_alg_bytes = 12 * ncell * 4
    step_traffic = measured_step_traffic()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": list(n), "n_blobs": nb, "kernel": wl["kernel"],
                   "launch": "eager" if args.eager else "recorded step graph",
                   "fft_shapes": ({k: v for k, v in tune[0].items() if k not in ("n",)} if tune else "defaults"),
                   "precision": "fp32 grid, fp64 blobs", "kT": wl["kT"], "dt": wl["dt"],
                   "forces": "WCA eps=%g cutoff=%gh" % (wl["wca_eps"], wl["wca_cutoff"])},
        "blob_steps_per_s": nb * args.steps / sec,
        "ms_per_step_repeats": repeats,
        "ms_per_step_median_of_5": float(np.median(repeats)),
        "step_hbm_fraction": step_alg_bytes / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
        # counted HBM traffic of all the step's kernels over the step time
        "step_traffic": (None if step_traffic is None else {
            "bytes_per_step": step_traffic, "achieved_GBs": step_traffic / (ms_per_step * 1e-3) / 1e9,
            "frac_of_peak": step_traffic / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9)}),
        "roofline": roofline,
        "phases": phases,
        "momentum_after": list(diag["momentum"]),
        "max_div_after": diag["max_div"],
    }
    if not args.no_fp64:
        log("setup FP64 context")
        sim64, _, _ = setup(I, torch, wl, I.FP64, stream)
        if not args.no_autotune:
            sim64.autotune()
        sim64.step(max(2, args.warmup // 4), step_flags)
        k64 = max(10, args.steps // 4)
        sec64, _ = time_steps(torch, sim64, stream, k64, step_flags)
        sim64.close()
        out["fp64"] = {"value": ncell * k64 / sec64, "ms_per_step": sec64 * 1000.0 / k64, "steps": k64,
                       "blob_steps_per_s": nb * k64 / sec64,
                       "step_hbm_fraction": 12 * ncell * 8 / sec64 * k64 / (HBM_PEAK_GBS * 1e9)}
        log("FP64: %.3f ms/step" % out["fp64"]["ms_per_step"])
    if not args.no_advection:
        log("advection on: %d steps" % args.advection_steps)
        out["advection"] = advection_leg(I, torch, stream, wl, args.advection_steps, max(2, args.warmup // 4),
                                         not args.no_autotune, step_flags)
        log("advection: %.3f ms/step, advection kernel %s us" % (
            out["advection"]["ms_per_step"], out["advection"]["advect_kernel"].get("avg_launch_us")))
    if not args.no_ensemble:
        log("batched ensemble: 96 replicas of 32^3 / 48^3 / 64^3")
        out["ensemble"] = ensemble_leg(I, torch, stream, args.ensemble_steps, max(2, args.warmup // 2),
                                       not args.no_autotune)
    if not args.no_scale:
        log("scale run: 512^3, 10^5 blobs, FP32 grid against FP64")
        out["scale_512"] = scale_leg(I, torch, stream, args.scale_steps, not args.no_autotune)
    if not args.no_statistics:
        log("single blob at 128^3: %d recorded steps per excess mass" % args.single_blob_steps)
        out["single_blob_128"] = single_blob_leg(I, torch, stream, args.single_blob_steps, not args.no_autotune)
        log("thermal-drift bias: ideal gas in 16^3 boxes, drift on and off")
        out["drift_bias_16"] = drift_bias_leg(I, stream.cuda_stream)
        log("drift bias (node harmonic, with / without drift): %s" % {
            k: ("%.4f" % v["with_drift"]["node_harmonic"], "%.4f" % v["without_drift"]["node_harmonic"])
            for k, v in out["drift_bias_16"]["kernels"].items()})
        log("WCA suspension g(r) at 32^3 (Table RDF), against the Monte Carlo reference")
        out["rdf_32"] = rdf_leg(I, stream.cuda_stream)
        out["rdf_32"]["vs_monte_carlo"] = rdf_vs_reference(out["rdf_32"])
        log("rdf: %s" % out["rdf_32"]["vs_monte_carlo"])
        log("ensemble velocity autocorrelation: %d steps" % args.vacf_steps)
        out["ensemble_vacf"] = ensemble_vacf_leg(I, torch, stream, args.vacf_steps, tune=not args.no_autotune)
    if not args.no_jps:
        log("J P S translational invariance (32^3, both kernels)")
        out["jps_32"] = jps_leg(I, stream.cuda_stream)
        log("jps: %s" % {k: (round(v["diag_dev_max"], 4), round(v["offdiag_max"], 5))
                         for k, v in out["jps_32"]["kernels"].items()})
    if not args.no_jps:
        log("hydrodynamic radius against box size and position (both kernels, split kernel shifts)")
        out["hydrodynamic_radius"] = hydrodynamic_radius_leg(I, stream.cuda_stream)
        log("R_H: %s" % {k: {n: round(v["R_H_mean"], 4) for n, v in rows.items()}
                         for k, rows in out["hydrodynamic_radius"]["kernels"].items()})
        log("R_H of the split three-point kernel against s/h (32^3): %s" % {
            s: round(v["R_H_mean"], 4) for s, v in out["hydrodynamic_radius"]["split_3pt_vs_shift_32"].items()})
    if not args.no_convergence:
        log("temporal convergence study (spring test, FP64)")
        out["convergence"] = convergence_leg(I, stream)
        log("convergence: orders %s (%.1f s)" % (
            {r: ["%.2f" % o if o is not None else "-" for o in v["order"]]
             for r, v in out["convergence"]["by_me_over_mf"].items()},
            out["convergence"]["wall_s"]))
    if not args.no_cpu_baseline:
        log("CPU oracle: two steps of the same workload, all host cores and one core")
        out["cpu_baseline"] = cpu_baseline(wl, q)
        log("CPU oracle: %s" % out["cpu_baseline"]["sample"])
        log("CPU oracle: samples of the other workloads")
        out["cpu_samples"] = cpu_samples()
        log("CPU oracle samples: %s" % {k: (None if v["value"] is None else "%.3g" % v["value"])
                                        for k, v in out["cpu_samples"].items()})
    path = os.path.abspath(args.full_record)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    log("full record written to %s" % path)
    print(json.dumps(compact_record(out)), flush=True)


if __name__ == "__main__":
    main()
