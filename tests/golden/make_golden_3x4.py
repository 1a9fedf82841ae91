"""Writes tests/golden/cluster_3x4.json with the CPU oracle only.

Workload: 3 rows x 4 columns, sites x + 4y, t = -1 on the 17 nearest-neighbour
bonds, t' = +0.3 on both diagonals of the 6 plaquettes, U = 8, mu = 4,
sector N_up = N_dn = 6 (dimension 853,776).  Ground state: 200 fixed
Lanczos steps from the SplitMix64 start vector of seed 1 (the plain
recurrence, no reorthogonalisation), ground state rebuilt by the second pass.
Green function: for all 78 pairs of the 12 sites, electron and hole chains of
200 steps; G(z) on z = omega + 0.1i, omega = -10 + 20k/63, k = 0..63.

Run from the repository root:  python tests/golden/make_golden_3x4.py
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


def main():
    m = synth.cluster_3x4()
    t0 = time.time()
    gs = oracle.lanczos_gs(m.t, m.U, 6, 6, fixed_steps=200, want_vector=True, seed=1)
    print(f"E0 = {gs['e0']:.15f}  residual {gs['true_residual']:.2e}  ({time.time() - t0:.0f} s)",
          flush=True)
    orbs = list(range(12))
    z = synth.omega_grid()
    ch = oracle.green_cf(m.t, m.U, 6, 6, gs["psi"], orbs, max_steps=200)
    G = cf.green_matrix(ch, 12, z, gs["e0"])
    print(f"G done ({time.time() - t0:.0f} s)", flush=True)
    pairs = [(i, j) for i in range(12) for j in range(i, 12)]
    out = {
        "workload": "3x4 t=-1 t'=0.3 U=8 mu=4 sector (6,6); 200 GS steps seed 1; 200-step chains",
        "e0": gs["e0"], "true_residual": gs["true_residual"], "gs_steps": gs["n_iter"],
        "alpha_first": list(gs["alpha"][:20]), "beta_first": list(gs["beta"][:20]),
        "z_re": list(z.real), "z_im": list(z.imag),
        "pairs": pairs,
        "b0sq": [[ch[(i, j, p)][0] for p in (0, 1)] for (i, j) in pairs],
        "G_re": [[G[iz, i, j].real for (i, j) in pairs] for iz in range(z.shape[0])],
        "G_im": [[G[iz, i, j].imag for (i, j) in pairs] for iz in range(z.shape[0])],
    }
    path = os.path.join(ROOT, "tests", "golden", "cluster_3x4.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
