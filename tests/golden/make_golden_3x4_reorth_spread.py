"""Writes tests/golden/cluster_3x4_reorth_spread.json with the CPU oracle only:
for every one of the 156 continued-fraction chains of the 3x4 workload (200
floors, full reorthogonalisation), how far its G(z) on the 64-point grid moves
when the chain's start vector is perturbed at relative 1e-14 (seeded), i.e. the
oracle's own rounding-level spread of each pair's 200-floor G.

Why: even with full reorthogonalisation, a truncated continued fraction can be
ill-conditioned in its start vector (measured: 4e-7 for the electron chain of
orbital 6, 1e-2 for its hole chain).  The GPU test compares each pair at 1e-4
where the pair's spread allows it and within three times the spread elsewhere.

The cluster's hopping is unchanged by the reflections x -> 3 - x and
y -> 2 - y (sites x + 4y); a reflection S maps c_i to c_P(i) and the
non-degenerate ground state to +-itself, so the chain of (i, j) has the same
coefficients, and the same conditioning, as that of (P(i), P(j)).  The spread
is therefore measured on one pair of each of the 26 classes and stored for
every member; the check that each reflection leaves t unchanged is part of the
script.

Workload as in make_golden_3x4_reorth.py.  About 1.2 hours on 8 threads.
Run from the repository root:  python tests/golden/make_golden_3x4_reorth_spread.py
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


def main():
    m = synth.cluster_3x4()
    t0 = time.time()
    gs = oracle.lanczos_gs(m.t, m.U, 6, 6, fixed_steps=200, want_vector=True, seed=1)
    z = synth.omega_grid()
    rng = np.random.default_rng(2718)
    perms = []
    for fx in (0, 1):
        for fy in (0, 1):
            P = np.array([(3 - s % 4 if fx else s % 4) + 4 * (2 - s // 4 if fy else s // 4)
                          for s in range(12)])
            assert np.array_equal(m.t[np.ix_(P, P)], m.t)
            perms.append(P)
    classes = {}
    for i in range(12):
        for j in range(i, 12):
            members = {tuple(sorted((int(P[i]), int(P[j])))) for P in perms}
            rep = min(members)
            classes.setdefault(rep, set()).update(members)
    spread = {}
    for n, ((i, j), members) in enumerate(sorted(classes.items())):
        for part in (0, 1):
            nup2 = 7 if part == 0 else 5
            phi = oracle.apply_op(12, 6, 6, gs["psi"], part, i, -1 if i == j else j)
            c1 = oracle.cf_chain(m.t, m.U, nup2, 6, phi, M_G, full_reorth=True)
            phi2 = phi * (1 + 1e-14 * rng.standard_normal(phi.shape))
            c2 = oracle.cf_chain(m.t, m.U, nup2, 6, phi2, M_G, full_reorth=True)
            g1 = cf.cf_eval(*c1, z, gs["e0"], part)
            g2 = cf.cf_eval(*c2, z, gs["e0"], part)
            val = float(np.abs(g1 - g2).max())
            for a, b in members:
                spread[f"{a},{b},{part}"] = val
        print(f"class {n + 1}/{len(classes)} ({time.time() - t0:.0f} s)", flush=True)
    out = {"workload": "3x4 cluster t=-1 t'=0.3 U=8 mu=4, sector (6,6); GS 200 fixed steps seed 1; "
                       "continued fractions with full reorthogonalisation, 200 floors",
           "perturbation": "start vector times (1 + 1e-14 N(0,1)), default_rng(2718); "
                           "measured on one pair per reflection class, stored for every member",
           "spread": spread}
    path = os.path.join(ROOT, "tests", "golden", "cluster_3x4_reorth_spread.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
