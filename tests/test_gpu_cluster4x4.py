"""Configuration 3 on the GPU: the 4x4 cluster (t = -1 on the 24 open-boundary
bonds, U = 8 and U = 4, mu = U/2), sector (8,8), dimension 165,636,900.  The
Lanczos ground state run to the residual test (tol 1e-12) from the SplitMix64
start vector of seed 1 must give the oracle's E0 (written by
tests/golden/make_golden_4x4.py) to relative 1e-10, with the same first
alpha_n; the FP32-vector run's E0 error is printed and bounded (1e-6).  The
ground-state vector of the second pass is checked at full size row by row:
(H psi - E0 psi)_i, with (H psi)_i from the oracle's row routine on the GPU's
psi, is bounded by the GPU's true residual |H psi - E0 psi| plus the rounding
bound of the row, and |psi| = 1."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cluster_4x4.json")


GOLD_U4 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cluster_4x4_u4.json")


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(GOLD):
        pytest.skip("golden file not generated")
    import paper_2305_18643_amd as q
    return q, json.load(open(GOLD)), synth.cluster_4x4(8.0), q.sector_basis(16, 8, 8)


def test_ground_state_converged_fp64(setup):
    q, g, m, b = setup
    print("4x4 GS fp64 to convergence", flush=True)
    r = q.lanczos_gs(m, b, want_vector=False)
    print(f"  E0 {r['e0']:.14f} after {r['n_iter']} steps (oracle {g['e0']:.14f} after "
          f"{g['n_iter']})")
    assert r["converged"]
    assert abs(r["e0"] - g["e0"]) <= 1e-10 * abs(g["e0"])
    assert np.allclose(r["alpha"][:12], g["alpha_first"][:12], rtol=1e-11, atol=1e-11)


def test_ground_state_fp32v(setup):
    q, g, m, b = setup
    print("4x4 GS fp32v, 300 steps", flush=True)
    r = q.lanczos_gs(m, b, fixed_steps=300, want_vector=False, prec="fp32v", reorth=1)
    rel = abs(r["e0"] - g["e0"]) / abs(g["e0"])
    print(f"  FP32V E0 relative error {rel:.2e}")
    assert rel <= 1e-6


def test_ground_state_converged_fp64_u4(setup):
    q, _, _, b = setup
    if not os.path.exists(GOLD_U4):
        pytest.skip("golden file not generated")
    g = json.load(open(GOLD_U4))
    m = synth.cluster_4x4(4.0)
    print("4x4 U=4 GS fp64 to convergence", flush=True)
    r = q.lanczos_gs(m, b, want_vector=False)
    print(f"  E0 {r['e0']:.14f} after {r['n_iter']} steps (oracle {g['e0']:.14f} after "
          f"{g['n_iter']})")
    assert r["converged"]
    assert abs(r["e0"] - g["e0"]) <= 1e-10 * abs(g["e0"])
    assert np.allclose(r["alpha"][:12], g["alpha_first"][:12], rtol=1e-11, atol=1e-11)


def test_ground_state_vector_full_size(setup):
    import torch
    import oracle
    q, g, m, b = setup
    print("4x4 GS fp64 with the vector", flush=True)
    r = q.lanczos_gs(m, b, want_vector=True)
    assert r["converged"] and abs(r["e0"] - g["e0"]) <= 1e-10 * abs(g["e0"])
    psi = r["psi"]
    nrm = float(torch.linalg.vector_norm(psi).item())
    print(f"  |psi| - 1 = {nrm - 1:.2e}, true residual {r['true_residual']:.3e}")
    assert abs(nrm - 1.0) < 1e-12
    assert r["true_residual"] < 1e-5
    ph = psi.cpu().numpy()
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([rng.integers(0, b.dim, 20000), np.arange(64),
                                     np.arange(b.dim - 64, b.dim)])).astype(np.int64)
    hp = oracle.hv_rows(m.t, m.U, 8, 8, ph, rows)
    bound = oracle.hv_abs_bound(m.t, m.U, 8, 8, ph, rows)
    res = np.abs(hp - r["e0"] * ph[rows])
    print(f"  max |(H psi - E0 psi)_i| on {rows.size} rows: {res.max():.3e}")
    assert np.all(res <= r["true_residual"] + 64 * 2.0 ** -53 * (bound + abs(r["e0"] * ph[rows])))
    del psi, ph
