"""Configuration 2 on the GPU: the 3x4 cluster (t = -1, t' = 0.3, U = 8,
mu = 4, sector (6,6), dimension 853,776), 200-step Lanczos ground state and
continued fractions for all 78 pairs, against values written from the CPU
oracle by tests/golden/make_golden_3x4.py and make_golden_3x4_cf.py.

What is compared, and why:
  * E0 after 200 steps: relative 1e-10 (FP64);
  * the first 12 floors of all 156 chains (b0^2, a_n, b_n^2) one by one, and
    G(z) built from those 12 floors (absolute 1e-8).  Later floors depend on
    rounding: the start vectors of the two sides differ at relative 1e-14
    (their ground states do), and that difference grows about tenfold per
    floor from floor ~12 on (measured: every chain agrees to 1e-9 through
    floor 11, none beyond floor 16), saturating near 1e-5 of max |a|;
  * G(z) from the full 200 floors: without reorthogonalisation, a 200-floor
    chain of this sector is sensitive to rounding; the oracle's own 200-floor
    G moves by up to 4.9e-2 when its start vectors are perturbed at relative
    1e-14 (recorded in the golden file).  The GPU result must stay within 3
    times that spread, and the ratio is printed;
  * FP32 vectors: E0 relative 1e-6; G from 200 floors within 3 times the
    oracle's spread, errors printed.  (The chains amplify any start-vector
    difference about tenfold per floor, so FP32 storage, relative 6e-8,
    reaches the saturated level within ~10 floors: floor-by-floor
    comparisons mean nothing there, the 200-floor G is what is compared.)
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import cf

pytestmark = pytest.mark.gpu
HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLD = os.path.join(HERE, "cluster_3x4.json")
GOLD_CF = os.path.join(HERE, "cluster_3x4_cf.json")


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not (os.path.exists(GOLD) and os.path.exists(GOLD_CF)):
        pytest.skip("golden files not generated")
    import paper_2305_18643_amd as q
    g = json.load(open(GOLD))
    gc = json.load(open(GOLD_CF))
    m = synth.cluster_3x4()
    b = q.sector_basis(12, 6, 6)
    return q, g, gc, m, b


def _gold_G(g):
    z = np.array(g["z_re"]) + 1j * np.array(g["z_im"])
    G = np.zeros((z.shape[0], 12, 12), dtype=complex)
    for p, (i, j) in enumerate(g["pairs"]):
        for iz in range(z.shape[0]):
            G[iz, i, j] = G[iz, j, i] = g["G_re"][iz][p] + 1j * g["G_im"][iz][p]
    return z, G


K = 12


def _gold_GK(gc, z, e0):
    ch = {}
    for key, (b0, a, b2) in gc["chains"].items():
        i, j, part = (int(x) for x in key.split(","))
        ch[(i, j, part)] = (b0, np.array(a[:K]), np.array(b2[:K - 1]))
    return cf.green_matrix(ch, 12, z, e0)


def _floors_check(res, gc, tol_a, tol_b):
    worst_a = worst_b = 0.0
    pairs = [(i, j) for i in range(12) for j in range(i, 12)]
    for p, (i, j) in enumerate(pairs):
        for part in (0, 1):
            b0, a, b2 = gc["chains"][f"{i},{j},{part}"]
            a, b2 = a[:K], b2[:K - 1]
            co = res["coef"][p, part]
            M = res["coef"].shape[2] // 2
            assert abs(co[0] - b0) <= 1e-10
            ga = co[1:1 + K]
            gb = co[1 + M:1 + M + K - 1]
            sc = max(1.0, np.abs(a).max())
            worst_a = max(worst_a, np.abs(ga[:len(a)] - np.array(a)).max() / sc)
            worst_b = max(worst_b, np.abs(gb[:len(b2)] - np.array(b2)).max() / max(1.0, np.abs(b2).max()))
    print(f"  first {K} floors: max |da|/max|a| {worst_a:.2e}, max |db2|/max|b2| {worst_b:.2e}")
    assert worst_a <= tol_a and worst_b <= tol_b


def test_ground_state_fp64(setup):
    q, g, gc, m, b = setup
    print("3x4 GS fp64", flush=True)
    r = q.lanczos_gs(m, b, fixed_steps=200, seed=1)
    assert r["n_iter"] == 200
    assert abs(r["e0"] - g["e0"]) <= 1e-10 * abs(g["e0"])
    assert np.allclose(r["alpha"][:12], g["alpha_first"][:12], rtol=1e-11, atol=1e-11)
    assert r["true_residual"] < 1e-8


def test_green_first_floors_fp64(setup):
    q, g, gc, m, b = setup
    print(f"3x4 G fp64, {K} floors", flush=True)
    r = q.lanczos_gs(m, b, fixed_steps=200, seed=1)
    z = np.array(g["z_re"]) + 1j * np.array(g["z_im"])
    res = q.green_cf(m, b, r["psi"], r["e0"], list(range(12)), z, max_steps=K)
    _floors_check(res, gc, 1e-9, 1e-9)
    GK = _gold_GK(gc, z, g["e0"])
    err = np.abs(res["G"].cpu().numpy() - GK).max()
    print(f"  max |G_{K} - G_{K} oracle| = {err:.3e}")
    assert err <= 1e-8


def test_green_200_floors_fp64(setup):
    q, g, gc, m, b = setup
    print("3x4 G fp64, 200 floors", flush=True)
    r = q.lanczos_gs(m, b, fixed_steps=200, seed=1)
    z, Go = _gold_G(g)
    res = q.green_cf(m, b, r["psi"], r["e0"], list(range(12)), z, max_steps=200)
    err = np.abs(res["G"].cpu().numpy() - Go).max()
    spread = max(gc["g200_sensitivity"].values())
    print(f"  max |G_200 - G_200 oracle| = {err:.3e}; oracle's own spread {spread:.3e} "
          f"(ratio {err / spread:.2f})")
    assert err <= 3 * spread


def test_fp32v_errors_reported(setup):
    q, g, gc, m, b = setup
    print("3x4 fp32v", flush=True)
    r = q.lanczos_gs(m, b, fixed_steps=200, seed=1, prec="fp32v", reorth=1)
    e_rel = abs(r["e0"] - g["e0"]) / abs(g["e0"])
    z, Go = _gold_G(g)
    res = q.green_cf(m, b, r["psi"], r["e0"], list(range(12)), z, max_steps=200, prec="fp32v",
                     reorth=1)
    e200 = np.abs(res["G"].cpu().numpy() - Go).max()
    spread = max(gc["g200_sensitivity"].values())
    print(f"  3x4 FP32V: E0 relative error {e_rel:.3e}, ground-state residual "
          f"{r['true_residual']:.2e}, max |dG_200| {e200:.3e} (oracle spread {spread:.3e})")
    assert e_rel < 1e-6
    assert e200 <= 3 * spread
