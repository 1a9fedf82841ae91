"""Writes tests/golden/cluster_3x4_cf.json with the CPU oracle only: the first
40 continued-fraction floors of every chain of the 3x4 workload, and the
oracle's own sensitivity of the 200-floor G to a 1e-14 perturbation.

Workload as in make_golden_3x4.py (3x4, t = -1, t' = 0.3, U = 8, mu = 4,
sector (6,6); ground state from 200 fixed Lanczos steps, seed 1).

Why: a 200-floor chain without reorthogonalisation loses orthogonality long
before its last floor, after which its coefficients depend on rounding.  The
first floors do not, so they are compared one by one; the 200-floor G is
compared against the spread the oracle itself shows when its start vectors
are perturbed at the level of rounding (relative 1e-14, seeded).

Run from the repository root:  python tests/golden/make_golden_3x4_cf.py
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

K = 40
SENS_PAIRS = [(0, 0), (0, 5), (3, 3), (5, 6)]


def main():
    m = synth.cluster_3x4()
    t0 = time.time()
    gs = oracle.lanczos_gs(m.t, m.U, 6, 6, fixed_steps=200, want_vector=True, seed=1)
    print(f"E0 = {gs['e0']:.15f} ({time.time() - t0:.0f} s)", flush=True)
    pairs = [(i, j) for i in range(12) for j in range(i, 12)]
    first = {}
    for (i, j) in pairs:
        for part in (0, 1):
            phi = oracle.apply_op(12, 6, 6, gs["psi"], part, i, -1 if i == j else j)
            b0, a, b2 = oracle.cf_chain(m.t, m.U, 7 if part == 0 else 5, 6, phi, K)
            first[f"{i},{j},{part}"] = [b0, list(a), list(b2)]
    print(f"first {K} floors of {len(first)} chains ({time.time() - t0:.0f} s)", flush=True)
    # sensitivity of the 200-floor G of a few pairs to a 1e-14 perturbation
    z = synth.omega_grid()
    rng = np.random.default_rng(314)
    sens = {}
    for (i, j) in SENS_PAIRS:
        G = []
        for pert in (False, True):
            ch = {}
            for part in (0, 1):
                phi = oracle.apply_op(12, 6, 6, gs["psi"], part, i, -1 if i == j else j)
                if pert:
                    phi = phi * (1.0 + 1e-14 * rng.standard_normal(phi.shape[0]))
                ch[(0, 0, part)] = oracle.cf_chain(m.t, m.U, 7 if part == 0 else 5, 6, phi, 200)
            G.append(cf.green_matrix(ch, 1, z, gs["e0"])[:, 0, 0])
        sens[f"{i},{j}"] = float(np.abs(G[0] - G[1]).max())
        print(f"pair ({i},{j}): 200-floor G moves by {sens[f'{i},{j}']:.2e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    out = {"workload": "3x4 t=-1 t'=0.3 U=8 mu=4 sector (6,6); 200 GS steps seed 1",
           "floors": K, "chains": first, "sensitivity_pairs": SENS_PAIRS,
           "g200_sensitivity": sens, "perturbation": "relative 1e-14, normal, seed 314"}
    path = os.path.join(ROOT, "tests", "golden", "cluster_3x4_cf.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
