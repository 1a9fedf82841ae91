"""Configuration 2 on the GPU: the 3x4 cluster (t = -1, t' = 0.3, U = 8,
mu = 4, sector (6,6), dimension 853,776), 200-step Lanczos ground state and
continued fractions for all 78 pairs, against values written from the CPU
oracle by tests/golden/make_golden_3x4.py, make_golden_3x4_cf.py and
make_golden_3x4_reorth.py.

What is compared, and why:
  * E0 after 200 steps: relative 1e-10 (FP64);
  * the first 12 floors of all 156 chains (b0^2, a_n, b_n^2) one by one, and
    G(z) built from those 12 floors (absolute 1e-8): the paper's recurrence
    agrees floor by floor until its start-vector differences (relative 1e-14,
    from the two sides' ground states) have grown, about tenfold per floor
    from floor ~12 on;
  * G(z) from 200 floors with full reorthogonalisation on both sides (a test
    device), from the same ground state: the chain is then the recurrence of
    exact arithmetic up to rounding, which makes most pairs' G independent of
    rounding but not all: a truncated continued fraction can still be
    ill-conditioned in its start vector (the oracle's own spread under a
    relative 1e-14 perturbation is 4e-7 for the electron chain of orbital 6
    and 1e-2 for its hole chain; every chain's spread is in
    cluster_3x4_reorth_spread.json).  Two measures of a pair's rounding
    sensitivity come from the oracle alone: the spread of its chains, and how
    far the oracle's G differs between pairs the cluster's reflections map
    onto each other (equal in exact arithmetic, up to 8.6e-3 apart in the
    oracle).  Pairs where both are below 1e-5 (20 of 78) are held to 1e-4
    (observed 1e-8); the others to 1e-4 plus three times the largest
    sensitivity on the workload, since the per-pair measures are single
    samples and undershoot on some pairs (observed: pair (2,9) moves by
    2.3e-3 against estimates of 6e-5, while its mirror image (1,10) agrees to
    2e-6); such pairs are printed.  Because of that
    amplification the chains start from the oracle's ground state
    (recomputed here, bitwise the golden file's) uploaded to the device: the
    GPU's own 200-step ground state differs from it at ~1e-10;
  * G(z) from 200 floors of the paper's recurrence (no reorthogonalisation),
    from the oracle's ground state: it depends on rounding once orthogonality
    is lost, so no tolerance against the oracle holds for it (the oracle
    moves by up to 5e-2 under a 1e-14 perturbation, and the GPU, from the
    same start vectors, differs from it by that order: 1.6e-2 on pair (0,0),
    four times the one spread sampled there); the differences are printed,
    and what holds whatever the rounding is asserted: -Im G_ii > 0,
    G_ij = G_ji, and |G_ij(z)| <= 2 / Im z;
  * FP32 vectors: E0 relative 1e-6; the 200-floor G with full
    reorthogonalisation against the FP64 golden, from the oracle's ground
    state and from the GPU's own FP32V one, errors printed and stated;
  * the band Lanczos Lehmann form (Q, Lambda) of all 12 orbitals, stopped
    by the paper's rule (lowest Ritz value converged to 1e-10), from the
    oracle's ground state: for each part the spectral moments
    Q Lambda^k Q^T = B^T H^k B (k = 0..3, exact for any basis of at least two
    blocks) against B^T H^k B formed from the oracle's start states and its
    own products, relative 1e-9, and Q Q^T = 1 (1e-12): a quantity that
    rounding does not move, at the paper's bar and beyond; FP32 vectors:
    the same moments to 1e-5.
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
GOLD_FR = os.path.join(HERE, "cluster_3x4_reorth.json")
GOLD_SP = os.path.join(HERE, "cluster_3x4_reorth_spread.json")


@pytest.fixture(scope="module")
def oracle_psi():
    """The oracle's 200-step ground state of the golden files (deterministic:
    every row and every dot of the oracle is summed in a fixed order)."""
    import oracle
    m = synth.cluster_3x4()
    gs = oracle.lanczos_gs(m.t, m.U, 6, 6, fixed_steps=200, want_vector=True, seed=1)
    return gs["e0"], gs["psi"]


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not (os.path.exists(GOLD) and os.path.exists(GOLD_CF) and os.path.exists(GOLD_FR)):
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


def test_green_200_floors_full_reorth_fp64(setup, oracle_psi):
    import torch
    q, g, gc, m, b = setup
    gf = json.load(open(GOLD_FR))
    print("3x4 G fp64, 200 floors, full reorthogonalisation", flush=True)
    e0, psi_o = oracle_psi
    assert e0 == gf["e0"]
    z, Go = _gold_G(gf)
    psi = torch.from_numpy(psi_o).to("cuda")
    if not os.path.exists(GOLD_SP):
        pytest.skip("per-chain spreads not generated")
    sp = json.load(open(GOLD_SP))["spread"]
    res = q.green_cf(m, b, psi, e0, list(range(12)), z, max_steps=200, reorth=2)
    G = res["G"].cpu().numpy()

    def chains(i, j):
        return sp[f"{i},{j},0"] + sp[f"{i},{j},1"]

    # two measures of how far rounding moves the oracle's own G of a pair:
    # the spread of its chains under a 1e-14 perturbation of their start
    # vectors, and how far the oracle's G differs between the pairs the
    # cluster's reflections map onto each other (equal in exact arithmetic)
    perms = [np.array([(3 - t % 4 if fx else t % 4) + 4 * (2 - t // 4 if fy else t // 4)
                       for t in range(12)]) for fx in (0, 1) for fy in (0, 1)]
    sens = {}
    for i in range(12):
        for j in range(i, 12):
            s_ij = chains(i, j) if i == j else 0.5 * (chains(i, j) + chains(i, i) + chains(j, j))
            a_ij = max(np.abs(Go[:, P[i], P[j]] - Go[:, i, j]).max() for P in perms)
            sens[(i, j)] = max(s_ij, a_ij)
    wide = 1e-4 + 3 * max(sens.values())
    strict = worst_strict = worst = 0.0
    n_strict = 0
    for (i, j), s_ij in sens.items():
        err = np.abs(G[:, i, j] - Go[:, i, j]).max()
        worst = max(worst, err)
        if s_ij <= 1e-5:
            # a well-conditioned pair: the paper's bar
            n_strict += 1
            worst_strict = max(worst_strict, err)
            assert err <= 1e-4, (i, j, err, s_ij)
        else:
            # an ill-conditioned one: within the rounding sensitivity the
            # oracle shows on this workload (the per-pair estimates are single
            # samples and undershoot on some pairs by 10-40x)
            assert err <= wide, (i, j, err, wide)
            if err > 1e-4 + 3 * s_ij:
                print(f"  pair ({i},{j}): |dG| {err:.2e} above 3x its own estimate {s_ij:.2e}")
    print(f"  {n_strict} of 78 pairs well-conditioned (oracle sensitivity <= 1e-5), held to 1e-4: "
          f"max |dG| {worst_strict:.3e}; all 78 within {wide:.3e}: max |dG| {worst:.3e}")
    # chain lengths, b0^2 and the first floors
    pairs = [(i, j) for i in range(12) for j in range(i, 12)]
    for p, (i, j) in enumerate(pairs):
        for part in (0, 1):
            key = f"{i},{j},{part}"
            assert res["len"][p, part] == gf["len"][key]
            assert abs(res["coef"][p, part, 0] - gf["b0sq"][key]) <= 1e-10
            a = np.array(gf["a_first"][key])
            assert np.abs(res["coef"][p, part, 1:1 + len(a)] - a).max() <= 1e-9 * max(1.0, np.abs(a).max())


def test_green_200_floors_paper_recurrence_fp64(setup, oracle_psi):
    import torch
    q, g, gc, m, b = setup
    print("3x4 G fp64, 200 floors, paper's recurrence", flush=True)
    e0, psi_o = oracle_psi
    z, Go = _gold_G(g)
    res = q.green_cf(m, b, torch.from_numpy(psi_o).to("cuda"), e0, list(range(12)), z,
                     max_steps=200)
    G = res["G"].cpu().numpy()
    print(f"  max |G_200 - G_200 oracle| over all pairs = {np.abs(G - Go).max():.3e} "
          "(rounding-dependent once orthogonality is lost)")
    for key, spread in gc["g200_sensitivity"].items():
        i, j = (int(x) for x in key.split(","))
        err = np.abs(G[:, i, j] - Go[:, i, j]).max()
        print(f"  pair ({i},{j}): |dG| {err:.3e}, one sample of the oracle's own "
              f"spread {spread:.3e}")
    for i in range(12):
        assert np.all(-G[:, i, i].imag > 0)
    assert np.abs(G - np.transpose(G, (0, 2, 1))).max() <= 1e-12
    # G_ij is half the sum of three chains whose weights total 2, 1 and 1.
    assert np.abs(G).max() <= 2.0 / z.imag.min()


def test_fp32v_errors_reported(setup, oracle_psi):
    import torch
    q, g, gc, m, b = setup
    gf = json.load(open(GOLD_FR))
    print("3x4 fp32v", flush=True)
    r = q.lanczos_gs(m, b, fixed_steps=200, seed=1, prec="fp32v", reorth=1)
    e_rel = abs(r["e0"] - g["e0"]) / abs(g["e0"])
    z, Go = _gold_G(gf)
    e0, psi_o = oracle_psi
    errs = {}
    for name, psi, e in (("oracle ground state", torch.from_numpy(psi_o).to("cuda"), e0),
                         ("own FP32V ground state", r["psi"], r["e0"])):
        res = q.green_cf(m, b, psi, e, list(range(12)), z, max_steps=200, prec="fp32v", reorth=2)
        G = res["G"].cpu().numpy()
        errs[name] = (np.abs(G - Go).max(), max(np.abs(G[:, i, i] - Go[:, i, i]).max()
                                                 for i in range(12)))
    print(f"  3x4 FP32V: E0 relative error {e_rel:.3e}, ground-state residual "
          f"{r['true_residual']:.2e}; 200-floor G (full reorthogonalisation) against the FP64 "
          "oracle: " + "; ".join(f"from the {k}: max |dG| {a:.3e} (diagonal {d:.3e})"
                                 for k, (a, d) in errs.items()))
    assert e_rel < 1e-6
    assert all(np.isfinite(a) for a, _ in errs.values())


def test_band_lanczos_moments(setup, oracle_psi):
    import torch
    import oracle
    q, g, gc, m, b = setup
    print("3x4 band Lanczos moments", flush=True)
    e0, psi_o = oracle_psi
    z, _ = _gold_G(g)
    psi = torch.from_numpy(psi_o).to("cuda")
    orbs = list(range(12))
    res = {prec: q.green_band(m, b, psi, e0, orbs, z, max_basis=600, etol=1e-10, prec=prec)
           for prec in ("fp64", "fp32v")}
    print(f"  R fp64 {list(res['fp64']['R'])}, fp32v {list(res['fp32v']['R'])}")
    worst = {"fp64": 0.0, "fp32v": 0.0}
    for part in range(2):
        nup2 = 7 if part == 0 else 5
        B = np.stack([oracle.apply_op(12, 6, 6, psi_o, part, mu) for mu in orbs], axis=1)
        X = B.copy()
        for k in range(4):
            Mo = B.T @ X
            for prec, gb in res.items():
                Mg = (gb["Q"][part] * gb["lam"][part] ** k) @ gb["Q"][part].T
                worst[prec] = max(worst[prec], np.abs(Mg - Mo).max() / max(1.0, np.abs(Mo).max()))
            if k < 3:
                X = np.stack([oracle.hv(m.t, m.U, nup2, 6, X[:, i]) for i in orbs], axis=1)
    print(f"  moments 0..3 against the oracle: max relative difference fp64 {worst['fp64']:.2e}, "
          f"fp32v {worst['fp32v']:.2e}")
    assert worst["fp64"] <= 1e-9
    assert worst["fp32v"] <= 1e-5
    Q = np.concatenate(res["fp64"]["Q"], axis=1)
    assert np.abs(Q @ Q.T - np.eye(12)).max() <= 1e-12
