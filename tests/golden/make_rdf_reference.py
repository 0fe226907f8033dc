"""Write tests/golden/rdf_wca_mc.json: g(r) of the WCA suspension of
Sec. IV.A, Table RDF (left), sampled from the Gibbs-Boltzmann distribution by
the Monte Carlo reference in oracle/ (independent chains; the spread over
chains is the statistical error). Calls only oracle/ and icm_inputs.

    python tests/golden/make_rdf_reference.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import icm_inputs  # noqa: E402
from oracle import gibbs  # noqa: E402

CHAINS, EQUIL, SWEEPS, EVERY, DELTA = 6, 2000, 20000, 20, 0.6


def main():
    wl = icm_inputs.WORKLOADS["rdf_32"]
    n = tuple(wl["n"])
    L = n[0] * wl["h"]
    gs, accs = [], []
    for c in range(CHAINS):
        x0 = icm_inputs.separated_positions(wl["n_blobs"], n, wl["h"], min_sep=wl["min_sep"], seed=wl["seed"] + 1 + c)
        r, g, acc, _ = gibbs.wca_gr(x0, L, wl["wca_eps"], wl["wca_sigma"], wl["kT"], DELTA, EQUIL, SWEEPS, EVERY,
                                    1000 + c, wl["rmax"], wl["nbins"])
        gs.append(g)
        accs.append(acc)
        print("chain %d: acceptance %.3f" % (c, acc), flush=True)
    gs = np.array(gs)
    out = {
        "cite": "Sec. IV.A, Eq. (P_Q), Eq. (WCA), Table RDF (left): 32^3 box of side 32, N = 1000, "
                "kT = eps = 1e-3, sigma = 2; Metropolis Monte Carlo reference (oracle/mc_wca.c)",
        "chains": CHAINS, "equilibration_sweeps": EQUIL, "sweeps": SWEEPS, "sample_every": EVERY,
        "trial_move_half_side": DELTA, "acceptance": accs,
        "r": [float(x) for x in r], "g": [float(x) for x in gs.mean(0)],
        "se": [float(x) for x in gs.std(0, ddof=1) / np.sqrt(CHAINS)],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "rdf_wca_mc.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
