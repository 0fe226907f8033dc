"""Throughput of the MI355X ICM step (cell-steps/s and blob-steps/s).

Default workload (many_blobs_256): 256^3 periodic grid, FP32 grid with FP64
blob state, 4096 neutrally buoyant blobs at seeded uniform positions with
minimum separation 2h, Peskin 4-point kernel, WCA soft-sphere repulsion
(strength 1e-2, cutoff 2h), kT = 1e-3, rho = eta = 1, dt = 0.2, fluid started
from the discrete equilibrium. Inputs are synthetic and resident in HBM when
the timed region starts.

Prints one JSON line: the throughput of the whole hot path, the roofline of
its dominant kernel (average launch duration from HIP events on the launch
stream), an FP64 run of the same workload, and the FP64 CPU oracle timed on a
bounded sample (one full step) of the same workload.
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


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(phase, n, nb, kernel, w):
    """Algorithmic HBM bytes of one launch of a phase:
    each field or spectrum element read once and written once."""
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
    return 0


PROFILE = os.path.join(ROOT, "profiles", "many_blobs_256_fp32.md")
PHASE_KERNEL = {"rhs": "k_rhs_march<float>", "fft_z_solve": "k_z_fast<float, 256, 16, 16, 16, 1>",
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


def setup(I, torch, wl, precision, stream):
    n = tuple(wl["n"])
    import icm_inputs
    sigma = wl["wca_cutoff"] / 2 ** (1.0 / 6.0)
    p = I.make_params(n, h=wl["h"], rho=wl["rho"], eta=wl["eta"], kT=wl["kT"], dt=wl["dt"], kernel=wl["kernel"],
                      seed=wl["seed"], wca_eps=wl["wca_eps"], wca_sigma=sigma)
    nb = wl["n_blobs"]
    nbytes = I.icm_workspace_bytes([p], [nb], precision)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    sim = I.Sim([p], [nb], precision, stream=stream.cuda_stream, workspace=ws)
    q = icm_inputs.separated_positions(nb, n, wl["h"], min_sep=wl["min_sep"], seed=wl["seed"])
    sim.set_blobs(0, q)
    sim.set_state(0, flags=I.STATE_EQUILIBRIUM)
    return sim, p, q


def time_steps(torch, sim, stream, steps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    sim.step(steps)
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


def ensemble_sims(I, torch, stream, batched):
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
    cells = sum(int(np.prod(n)) for n in grids)
    return sims, cells, nrep


def ensemble_leg(I, torch, stream, steps, warmup):
    """cell-steps/s of the batched ensemble as one context (one recorded graph
    per step) against the same replicas stepped one context at a time."""
    out = {}
    for mode in ("batched", "single"):
        sims, cells, nrep = ensemble_sims(I, torch, stream, mode == "batched")
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


def cpu_baseline(wl, seed_positions):
    """The FP64 oracle, untuned, on one full step of the same workload."""
    from oracle import icm as O
    n = tuple(wl["n"])
    sigma = wl["wca_cutoff"] / 2 ** (1.0 / 6.0)
    p = O.Params(n=n, h=wl["h"], rho=wl["rho"], eta=wl["eta"], kT=wl["kT"], dt=wl["dt"], kernel=wl["kernel"],
                 seed=wl["seed"], wca_eps=wl["wca_eps"], wca_sigma=sigma)
    st = O.new_state(p, seed_positions)
    st.v = O.equilibrium_field(p)
    t0 = time.perf_counter()
    O.step(p, st)
    dt = time.perf_counter() - t0
    ncell = int(np.prod(n))
    return dict(value=ncell / dt, unit="cell-steps/s", cores=1, kind="oracle",
                sample="one full step of %s (%dx%dx%d, %d blobs) in the FP64 numpy/scipy oracle, %.1f s; "
                       "blob-steps/s %.3g; numpy and scipy.fft run single-threaded here"
                       % ("many_blobs_256", n[0], n[1], n[2], wl["n_blobs"], dt, wl["n_blobs"] / dt),
                seconds=dt)


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
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 256 MiB device-to-device tensor copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
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
    log("warmup %d steps" % args.warmup)
    sim.step(args.warmup)
    log("timing %d steps" % args.steps)
    sec, wall = time_steps(torch, sim, stream, args.steps)
    ms_per_step = sec * 1000.0 / args.steps
    value = ncell * args.steps / sec
    log("FP32 grid: %.3f ms/step, %.3e cell-steps/s" % (ms_per_step, value))
    phases = profile_phases(sim, args.profile_steps, n, nb, wl["kernel"], 4)
    diag = sim.get_state(0, want_v=False)["diag"]
    sim.close()
    dom = max(phases.items(), key=lambda kv: kv[1]["total_ms_per_step"])
    dom_name, dom_v = dom
    roofline = dict(bound="hbm", kernel=dom_name, achieved=dom_v["achieved_GBs"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=dom_v["achieved_GBs"] / HBM_PEAK_GBS, traffic=measured_traffic(dom_name),
                    alg_bytes_per_launch=dom_v["alg_bytes_per_launch"], avg_launch_us=dom_v["avg_launch_us"])
    step_alg_bytes = 12 * ncell * 4
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
                   "precision": "fp32 grid, fp64 blobs", "kT": wl["kT"], "dt": wl["dt"],
                   "forces": "WCA eps=%g cutoff=%gh" % (wl["wca_eps"], wl["wca_cutoff"])},
        "blob_steps_per_s": nb * args.steps / sec,
        "step_hbm_fraction": step_alg_bytes / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "roofline": roofline,
        "phases": phases,
        "momentum_after": list(diag["momentum"]),
        "max_div_after": diag["max_div"],
    }
    if not args.no_fp64:
        log("setup FP64 context")
        sim64, _, _ = setup(I, torch, wl, I.FP64, stream)
        sim64.step(max(2, args.warmup // 4))
        k64 = max(10, args.steps // 4)
        sec64, _ = time_steps(torch, sim64, stream, k64)
        sim64.close()
        out["fp64"] = {"value": ncell * k64 / sec64, "ms_per_step": sec64 * 1000.0 / k64, "steps": k64,
                       "blob_steps_per_s": nb * k64 / sec64}
        log("FP64: %.3f ms/step" % out["fp64"]["ms_per_step"])
    if not args.no_ensemble:
        log("batched ensemble: 96 replicas of 32^3 / 48^3 / 64^3")
        out["ensemble"] = ensemble_leg(I, torch, stream, args.ensemble_steps, max(2, args.warmup // 2))
    if not args.no_cpu_baseline:
        log("CPU oracle: one step of the same workload")
        out["cpu_baseline"] = cpu_baseline(wl, q)
        log("CPU oracle: %.1f s" % out["cpu_baseline"]["seconds"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
