"""Writes tests/golden/cdmft_chain4_4b.json with the CPU oracle only: the
CDMFT loop of the 1D Hubbard model (U = 4, mu = 2) on 4-site clusters with
4 bath orbitals (synth.cdmft_chain_4_4b), from p0 = (1, -1, 1, 1), 64
wave-vectors of the reduced zone, the Matsubara grid of beta = 50 up to
omega = 2 with uniform weights, 200-floor continued fractions, the loop
stopped when no parameter moves by more than 1e-6.  Stored: the parameters
of every iteration, the iteration count, the last distance and E0.

Run from the repository root:  python tests/golden/make_golden_cdmft.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import cdmft as C  # noqa: E402


def main():
    s = synth.cdmft_chain_4_4b()
    t0 = time.time()
    r = C.cdmft(s, s.p0, synth.k_grid_1d(64), max_iter=40, tol=1e-6)
    print(f"{r['iterations']} iterations, converged {r['converged']}, p {r['p']}, "
          f"d {r['distance']:.6e} ({time.time() - t0:.0f} s)", flush=True)
    out = {"workload": "1D Hubbard U=4 mu=2, 4-site cluster + 4 bath orbitals, sector (4,4); "
                       "64 k, beta=50, wc=2, uniform weights, 200 floors, tol 1e-6",
           "p": list(r["p"]), "history": [list(p) for p in r["history"]],
           "iterations": r["iterations"], "converged": r["converged"],
           "distance": r["distance"], "e0": r["e0"], "cpu_seconds": time.time() - t0}
    path = os.path.join(ROOT, "tests", "golden", "cdmft_chain4_4b.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
