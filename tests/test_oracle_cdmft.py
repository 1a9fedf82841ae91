"""Pins of the oracle's CDMFT loop (oracle/cdmft.py) against what the paper
and the mathematics fix, on the CPU:

  * at U = 0 the impurity's many-body cluster Green function equals the
    cluster block of the one-body resolvent (z - t_imp)^{-1} (dense), which
    in turn equals (z - t_c' - Gamma(z))^{-1} (Schur complement of the bath):
    this fixes the hybridization function and its sign conventions, and the
    self-energy then vanishes;
  * with Sigma = 0, the super-lattice average Gbar equals the cluster block
    of the resolvent of a ring of N clusters (brute force), which fixes V(k)
    and the k sum;
  * the analytic gradient of the distance function equals central finite
    differences, and the fit ends where it vanishes;
  * at U = 0 the loop reaches its fixed point after one fit (the self-energy
    does not depend on the bath);
  * at mu = U/2 on the bipartite chain, particle-hole symmetry keeps the
    symmetric bath (eb1 = -eb2, tb1 = tb2) through the whole loop.
"""
import numpy as np
import pytest

import synth
from oracle import cdmft as C


def _setup(U=4.0):
    return synth.cdmft_chain_4_4b(U=U, mu=U / 2)


def test_hybridization_is_the_bath_schur_complement():
    s = _setup(U=0.0)
    p = np.array([0.7, -1.3, 0.9, 0.4])
    z = synth.matsubara_grid(s.beta, s.wc)
    t, U = C.impurity(s, p)
    L = s.L
    theta, eps = C.bath_of(s, p)
    gam = C.hybridization(theta, eps, z)
    Gc, _ = C.cluster_green(s, p, z)
    for iz, zz in enumerate(z):
        R = np.linalg.inv(zz * np.eye(t.shape[0]) - t)[:L, :L]
        S = np.linalg.inv(zz * np.eye(L) - C.tc_prime(s) - gam[iz])
        assert np.abs(R - S).max() <= 1e-12
        assert np.abs(Gc[iz] - R).max() <= 1e-10
    sig = C.sigma(s, p, z, Gc)
    assert np.abs(sig).max() <= 1e-9


def test_super_lattice_average_equals_a_ring():
    s = _setup(U=0.0)
    z = np.array([0.3j, 0.1 + 0.5j, -0.7 + 0.05j])
    nk, L = 16, s.L
    G = C.gbar(s, z, np.zeros((3, L, L), dtype=complex), synth.k_grid_1d(nk))
    # a ring of nk clusters, site c*L + i; bond (i, j, shift 1) joins cluster c to c+1
    H = np.zeros((nk * L, nk * L))
    for c in range(nk):
        H[c * L:(c + 1) * L, c * L:(c + 1) * L] = C.tc_prime(s)
        for (i, j, sh, t) in s.bonds:
            a, b = c * L + i, ((c + sh[0]) % nk) * L + j
            H[a, b] += t
            H[b, a] += t
    for iz, zz in enumerate(z):
        R = np.linalg.inv(zz * np.eye(nk * L) - H)[:L, :L]
        assert np.abs(G[iz] - R).max() <= 1e-12


def test_distance_gradient_matches_finite_differences():
    s = _setup()
    z = synth.matsubara_grid(s.beta, s.wc)
    w = np.full(z.shape[0], 1.0 / z.shape[0])
    rng = np.random.default_rng(7)
    G0i = rng.standard_normal((z.shape[0], 4, 4)) + 1j * rng.standard_normal((z.shape[0], 4, 4))
    p = np.array([0.8, -1.1, 0.6, 0.9])
    g = C.distance_grad(s, p, z, w, G0i)
    h = 1e-6
    for k in range(4):
        e = np.zeros(4)
        e[k] = h
        fd = (C.distance(s, p + e, z, w, G0i) - C.distance(s, p - e, z, w, G0i)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k]))
    # a fit against a reachable target: the U = 0 lattice calG0^{-1}
    L = s.L
    T = C.g0inv(C.gbar(s, z, np.zeros((z.shape[0], L, L), dtype=complex), synth.k_grid_1d(64)),
                np.zeros((z.shape[0], L, L), dtype=complex))
    pf, d, _ = C.fit(s, p, z, w, T)
    assert d <= C.distance(s, p, z, w, T)
    assert np.abs(C.distance_grad(s, pf, z, w, T)).max() <= 1e-8


def test_noninteracting_loop_is_a_fixed_point_after_one_fit():
    s = _setup(U=0.0)
    r = C.cdmft(s, s.p0, synth.k_grid_1d(64), max_iter=4, tol=1e-7)
    assert r["converged"] and r["iterations"] <= 2
    assert np.abs(r["sigma"]).max() <= 1e-9


def test_particle_hole_symmetric_bath_stays_symmetric():
    s = _setup(U=4.0)
    r = C.cdmft(s, s.p0, synth.k_grid_1d(64), max_iter=30, tol=1e-6)
    assert r["converged"]
    for p in r["history"]:
        assert abs(p[0] + p[1]) <= 1e-5 * max(1.0, abs(p[0]))
        assert abs(p[2] - p[3]) <= 1e-5 * max(1.0, abs(p[2]))
