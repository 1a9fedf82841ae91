"""CDMFT on the GPU against the oracle (oracle/cdmft.py), for the 1D
Hubbard model on 4-site clusters with 4 bath orbitals (synth.cdmft_chain_4_4b):

  * the impurity's cluster Green function on the Matsubara grid (GPU Lanczos
    and continued fractions) against the oracle's, 1e-8;
  * from the same cluster Green function: Sigma_c, Gbar and calG0^{-1},
    1e-12 of the largest entry;
  * from the same calG0^{-1}: the distance at the start (1e-12 relative) and
    the fitted bath (distance 1e-9 relative, hybridization on the grid 1e-7;
    the minimiser differs, the minimum does not);
  * the whole loop against tests/golden/cdmft_chain4_4b.json (written by the
    oracle): the same number of iterations within one, the converged bath
    energies and |hoppings| within 1e-5 and the hybridization on the grid
    within 1e-5 (a sign flip of the hoppings is the same bath: Gamma depends
    on theta theta^T), particle-hole symmetry kept at every iteration;
  * at U = 0 the loop stops after one fit with a vanishing self-energy.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import cdmft as C

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cdmft_chain4_4b.json")


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_18643_amd as q
    return q


def _grid(s):
    z = synth.matsubara_grid(s.beta, s.wc)
    return z, np.full(z.shape[0], 1.0 / z.shape[0])


def _oracle_steps(s, p, z, ks):
    Gc, e0 = C.cluster_green(s, p, z)
    sig = C.sigma(s, p, z, Gc)
    gb = C.gbar(s, z, sig, ks)
    return Gc, sig, gb, C.g0inv(gb, sig), e0


def test_cluster_green_matches_oracle(q):
    from paper_2305_18643_amd.cdmft import impurity_arrays
    s = synth.cdmft_chain_4_4b()
    z, _ = _grid(s)
    t, U = impurity_arrays(s, s.p0)
    b = q.sector_basis(8, s.nup, s.ndn)
    r = q.lanczos_gs((t, U), b)
    g = q.green_cf((t, U), b, r["psi"], r["e0"], list(range(4)), z, max_steps=200)
    Go, e0 = C.cluster_green(s, s.p0, z)
    err = np.abs(g["G"].cpu().numpy() - Go).max()
    print(f"  cdmft Gc at p0: max |dG| {err:.2e}, E0 {r['e0']:.12f} (oracle {e0:.12f})")
    assert abs(r["e0"] - e0) <= 1e-10 * abs(e0)
    assert err <= 1e-8


def test_g0inv_matches_oracle(q):
    import torch
    s = synth.cdmft_chain_4_4b()
    z, _ = _grid(s)
    ks = synth.k_grid_1d(64)
    Gc, sig, gb, G0i, _ = _oracle_steps(s, s.p0, z, ks)
    theta, eps = C.bath_of(s, s.p0)
    o = q.cdmft_g0inv(torch.from_numpy(Gc).to("cuda"), C.tc_prime(s), theta, eps, s.bonds, ks, z)
    for name, ref in (("sigma", sig), ("gbar", gb), ("g0inv", G0i)):
        err = np.abs(o[name].cpu().numpy() - ref).max()
        print(f"  {name}: max diff {err:.2e}")
        assert err <= 1e-12 * max(1.0, np.abs(ref).max())


def test_fit_matches_oracle(q):
    import torch
    s = synth.cdmft_chain_4_4b()
    z, w = _grid(s)
    _, _, _, G0i, _ = _oracle_steps(s, s.p0, z, synth.k_grid_1d(64))
    g0 = torch.from_numpy(G0i).to("cuda")
    # no step: the distance at the start
    p, d, it = q.cdmft_fit(g0, C.tc_prime(s), s.A_eps, s.A_theta, s.p0, z, w, max_iter=0)
    d0 = C.distance(s, s.p0, z, w, G0i)
    assert it == 0 and np.allclose(p, s.p0)
    assert abs(d - d0) <= 1e-12 * d0
    # the minimum
    p, d, it = q.cdmft_fit(g0, C.tc_prime(s), s.A_eps, s.A_theta, s.p0, z, w, gtol=1e-10)
    po, do, _ = C.fit(s, s.p0, z, w, G0i)
    gam = C.hybridization(*C.bath_of(s, p), z)
    gamo = C.hybridization(*C.bath_of(s, po), z)
    print(f"  fit: {it} BFGS steps, d {d:.10e} (oracle {do:.10e}), p {p} (oracle {po}), "
          f"max |dGamma| {np.abs(gam - gamo).max():.2e}")
    assert it > 0
    assert abs(d - do) <= 1e-9 * do
    assert np.abs(gam - gamo).max() <= 1e-7
    assert np.abs(C.distance_grad(s, p, z, w, G0i)).max() <= 1e-8


def test_cdmft_loop_matches_oracle(q):
    s = synth.cdmft_chain_4_4b()
    z, w = _grid(s)
    g = json.load(open(GOLD))
    r = q.cdmft(s, s.p0, synth.k_grid_1d(64), z, w, max_iter=40, tol=1e-6)
    print(f"  loop: {r['iterations']} iterations (oracle {g['iterations']}), p {r['p']} "
          f"(oracle {np.array(g['p'])}), {np.mean(r['times']) * 1e3:.1f} ms per iteration")
    assert r["converged"]
    assert abs(r["iterations"] - g["iterations"]) <= 1
    # the bath enters through theta theta^T only: a sign flip of the
    # hoppings is the same solution, so compare the energies, |tb| and Gamma
    pg = np.array(g["p"])
    assert np.abs(r["p"][:2] - pg[:2]).max() <= 1e-5
    assert np.abs(np.abs(r["p"][2:]) - np.abs(pg[2:])).max() <= 1e-5
    gam = C.hybridization(*C.bath_of(s, r["p"]), z)
    gamo = C.hybridization(*C.bath_of(s, pg), z)
    assert np.abs(gam - gamo).max() <= 1e-5
    for p in r["history"]:
        assert abs(p[0] + p[1]) <= 1e-6 * max(1.0, abs(p[0]))
        assert abs(p[2] - p[3]) <= 1e-6 * max(1.0, abs(p[2]))


def test_cdmft_noninteracting_fixed_point(q):
    s = synth.cdmft_chain_4_4b(U=0.0, mu=0.0)
    z, w = _grid(s)
    r = q.cdmft(s, s.p0, synth.k_grid_1d(64), z, w, max_iter=4, tol=1e-7)
    assert r["converged"] and r["iterations"] <= 2
    assert np.abs(r["sigma"].cpu().numpy()).max() <= 1e-9
