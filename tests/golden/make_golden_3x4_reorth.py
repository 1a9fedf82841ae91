"""Writes tests/golden/cluster_3x4_reorth.json with the CPU oracle only: the
200-floor continued-fraction G(z) of all 78 orbital pairs of the 3x4
workload, every chain run with full reorthogonalisation (a test device on
both sides; the paper's recurrence tolerates the loss of orthogonality).

Why: without reorthogonalisation a 200-floor chain of this sector has lost
orthogonality long before its last floor, and its G then depends on rounding
(the oracle's own G moves by up to 5e-2 when its start vector is perturbed at
relative 1e-14).  With full reorthogonalisation the chain is the recurrence of
exact arithmetic up to rounding, and the same perturbation moves G by at most
about 1e-6, recorded here for two pairs, so G can be compared at 1e-4.

Workload as in make_golden_3x4.py (3x4, t = -1, t' = 0.3, U = 8, mu = 4,
sector (6,6); ground state from 200 fixed Lanczos steps, seed 1; the
frequency grid of 64 points in [-10, 10], eta = 0.1).

Run from the repository root:  python tests/golden/make_golden_3x4_reorth.py
(about 1.5 hours on 8 threads: 156 chains of 200 floors with 731,808 states).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import cf  # noqa: E402

M_G = 200
SENS_PAIRS = [(0, 0), (0, 5)]


def main():
    m = synth.cluster_3x4()
    t0 = time.time()
    gs = oracle.lanczos_gs(m.t, m.U, 6, 6, fixed_steps=200, want_vector=True, seed=1)
    e0 = gs["e0"]
    print(f"E0 = {e0:.15f} ({time.time() - t0:.0f} s)", flush=True)
    z = synth.omega_grid()
    pairs = [(i, j) for i in range(12) for j in range(i, 12)]
    chains = {}
    for n, (i, j) in enumerate(pairs):
        for part in (0, 1):
            phi = oracle.apply_op(12, 6, 6, gs["psi"], part, i, -1 if i == j else j)
            chains[(i, j, part)] = oracle.cf_chain(m.t, m.U, 7 if part == 0 else 5, 6, phi, M_G,
                                                   full_reorth=True)
        print(f"pair {n + 1}/{len(pairs)} ({time.time() - t0:.0f} s)", flush=True)
    G = cf.green_matrix(chains, 12, z, e0)
    # sensitivity of G to a relative 1e-14 perturbation of the start vectors
    rng = np.random.default_rng(314)
    sens = {}
    for (i, j) in SENS_PAIRS:
        worst = 0.0
        for part in (0, 1):
            phi = oracle.apply_op(12, 6, 6, gs["psi"], part, i, -1 if i == j else j)
            phi2 = phi * (1 + 1e-14 * rng.standard_normal(phi.shape))
            c2 = oracle.cf_chain(m.t, m.U, 7 if part == 0 else 5, 6, phi2, M_G, full_reorth=True)
            one = {(0, 0, part): chains[(i, j, part)]}
            two = {(0, 0, part): c2}
            g1 = cf.green_matrix(one, 1, z, e0)
            g2 = cf.green_matrix(two, 1, z, e0)
            worst = max(worst, float(np.abs(g1 - g2).max()))
        sens[f"{i},{j}"] = worst
        print(f"sensitivity {i},{j}: {worst:.2e}", flush=True)
    out = {
        "workload": "3x4 cluster t=-1 t'=0.3 U=8 mu=4, sector (6,6); GS 200 fixed steps seed 1; "
                    "continued fractions with full reorthogonalisation, 200 floors, all 78 pairs",
        "e0": e0, "max_steps": M_G,
        "z_re": list(z.real), "z_im": list(z.imag),
        "pairs": pairs,
        "G_re": [[float(G[iz, i, j].real) for (i, j) in pairs] for iz in range(z.shape[0])],
        "G_im": [[float(G[iz, i, j].imag) for (i, j) in pairs] for iz in range(z.shape[0])],
        "b0sq": {f"{i},{j},{p}": chains[(i, j, p)][0] for (i, j) in pairs for p in (0, 1)},
        "len": {f"{i},{j},{p}": int(len(chains[(i, j, p)][1])) for (i, j) in pairs for p in (0, 1)},
        "a_first": {f"{i},{j},{p}": list(chains[(i, j, p)][1][:12]) for (i, j) in pairs
                    for p in (0, 1)},
        "sensitivity_1e-14": sens,
    }
    path = os.path.join(ROOT, "tests", "golden", "cluster_3x4_reorth.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
