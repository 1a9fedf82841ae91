"""Writes tests/golden/cluster_4x4.json with the CPU oracle only: the Lanczos
ground state of the 4x4 cluster (sites x + 4y, t = -1 on the 24 open-boundary
bonds, U = 8, mu = 4), sector N_up = N_dn = 8 (dimension 165,636,900), run to
the residual test (tol 1e-12, at most 600 steps) from the SplitMix64 start
vector of seed 1, plain recurrence.  Stored: E0, the step count, the residual
estimate and the first 20 alpha_n and beta_n.

Needs about 6 GB of memory; tens of minutes on 8 cores.
Run from the repository root:  python tests/golden/make_golden_4x4.py [U]
(U = 8 writes cluster_4x4.json, any other U cluster_4x4_u<U>.json).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    U = float(sys.argv[1]) if len(sys.argv) > 1 else 8.0
    m = synth.cluster_4x4(U)
    t0 = time.time()
    gs = oracle.lanczos_gs(m.t, m.U, 8, 8, max_iter=600, tol=1e-12, want_vector=False, seed=1)
    print(f"E0 = {gs['e0']:.15f} after {gs['n_iter']} steps, estimate {gs['residual_est']:.2e} "
          f"({time.time() - t0:.0f} s)", flush=True)
    out = {"workload": f"4x4 t=-1 U={U:g} mu={U / 2:g} sector (8,8); Lanczos to tol 1e-12, seed 1",
           "e0": gs["e0"], "n_iter": gs["n_iter"], "converged": gs["converged"],
           "residual_est": gs["residual_est"], "theta1": gs["theta1"],
           "alpha_first": list(gs["alpha"][:20]), "beta_first": list(gs["beta"][:20])}
    name = "cluster_4x4.json" if U == 8.0 else f"cluster_4x4_u{U:g}.json"
    path = os.path.join(ROOT, "tests", "golden", name)
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
