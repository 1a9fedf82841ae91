"""Configuration 2 on the GPU: the 3x4 cluster (t = -1, t' = 0.3, U = 8,
mu = 4, sector (6,6), dimension 853,776), 200-step Lanczos ground state and
200-step continued fractions for all 78 pairs, against values written by
tests/golden/make_golden_3x4.py from the CPU oracle.  FP64 mode must match
E0 to relative 1e-10 and G to absolute 1e-4; the FP32-vector mode's errors
are printed and bounded loosely."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cluster_3x4.json")


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(GOLD):
        pytest.skip("golden file not generated")
    import paper_2305_18643_amd as q
    g = json.load(open(GOLD))
    m = synth.cluster_3x4()
    b = q.sector_basis(12, 6, 6)
    return q, g, m, b


def _gold_G(g):
    z = np.array(g["z_re"]) + 1j * np.array(g["z_im"])
    G = np.zeros((z.shape[0], 12, 12), dtype=complex)
    for p, (i, j) in enumerate(g["pairs"]):
        for iz in range(z.shape[0]):
            G[iz, i, j] = G[iz, j, i] = g["G_re"][iz][p] + 1j * g["G_im"][iz][p]
    return z, G


def test_ground_state_fp64(setup):
    q, g, m, b = setup
    print("3x4 GS fp64", flush=True)
    r = q.lanczos_gs(m, b, fixed_steps=200, seed=1)
    assert r["n_iter"] == 200
    assert abs(r["e0"] - g["e0"]) <= 1e-10 * abs(g["e0"])
    assert np.allclose(r["alpha"][:12], g["alpha_first"][:12], rtol=1e-11, atol=1e-11)
    assert r["true_residual"] < 1e-8


def test_green_fp64(setup):
    q, g, m, b = setup
    print("3x4 G fp64", flush=True)
    r = q.lanczos_gs(m, b, fixed_steps=200, seed=1)
    z, Go = _gold_G(g)
    res = q.green_cf(m, b, r["psi"], r["e0"], list(range(12)), z, max_steps=200)
    G = res["G"].cpu().numpy()
    err = np.abs(G - Go).max()
    print(f"  3x4 FP64 max |G - G_oracle| = {err:.3e}")
    for p in range(len(g["pairs"])):
        for part in (0, 1):
            assert abs(res["coef"][p, part, 0] - g["b0sq"][p][part]) < 1e-10
    assert err <= 1e-4


def test_fp32v_errors_reported(setup):
    q, g, m, b = setup
    print("3x4 fp32v", flush=True)
    r = q.lanczos_gs(m, b, fixed_steps=200, seed=1, prec="fp32v", reorth=1)
    e_rel = abs(r["e0"] - g["e0"]) / abs(g["e0"])
    z, Go = _gold_G(g)
    res = q.green_cf(m, b, r["psi"], r["e0"], list(range(12)), z, max_steps=200, prec="fp32v",
                     reorth=1)
    gerr = np.abs(res["G"].cpu().numpy() - Go).max()
    print(f"  3x4 FP32V: E0 relative error {e_rel:.3e}, max |G - G_oracle| {gerr:.3e}")
    assert e_rel < 1e-6
    assert gerr < 5e-2
