"""Pins of the oracle's band Lanczos Green function (oracle/band.py) against
what the paper and the mathematics fix, on the CPU.

The paper's recurrence orthogonalises each new vector against the previous
band only; like the plain Lanczos method it loses orthogonality after a
while, which is why the paper stops it when the lowest eigenvalue of T has
converged.  The pins therefore use two modes of the oracle:

  * with full reorthogonalisation (a test device), the Krylov space of a
    small sector is exhausted and deflates exactly: the band Lanczos
    Lehmann representation then equals the exact Lehmann sum of dense
    diagonalisation (oracle/dense.py, sharing no code with it) to 1e-10,
    also with start states that vanish or repeat (deflation), and equals the
    continued fractions of exhausted chains;
  * the paper's recurrence itself gives the same T, Q, Lambda and G as the
    reorthogonalised one while the basis is short (before orthogonality is
    lost), and its stopping rule ends the run once the lowest eigenvalue has
    converged;
  * in both modes, Q Q^T = 1 for the concatenated electron and hole parts
    (the paper's statement, from the anticommutator), also for a truncated
    Krylov space;
  * Ritz values that carry weight in an exhausted space are eigenvalues of H.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import band, cf, dense

Z = synth.omega_grid()


def _gs(m):
    r = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True, nthreads=1)
    return r["e0"], r["psi"]


def _qqt(parts, orbs):
    """max |Q Q^T - {c_a, c+_b}| with {c_a, c+_b} = 1 when orbs[a] == orbs[b]."""
    Q = np.concatenate([parts[0][1], parts[1][1]], axis=1)
    o = np.asarray(orbs)
    return np.abs(Q @ Q.T - (o[:, None] == o[None, :])).max()


@pytest.mark.parametrize("m,orbs", [(synth.plaquette_2x2(), [0, 1, 2, 3]),
                                    (synth.random_model(501, 6, 3, 2), [0, 2, 5]),
                                    (synth.impurity_model(np.random.default_rng(3), 2), [0, 1, 2, 3]),
                                    (synth.random_model(42, 5, 2, 3), [0, 1, 2, 3, 4])],
                         ids=["2x2", "rand6", "imp6", "rand5"])
def test_band_exhausted_equals_dense_lehmann(m, orbs):
    e0, psi = _gs(m)
    G, parts = band.green_band(m.t, m.U, m.nup, m.ndn, psi, orbs, e0, Z, max_basis=2000,
                               full_reorth=True)
    Gd = dense.lehmann_green(m.t, m.U, m.nup, m.ndn, orbs, Z, psi=psi, e0=e0)
    assert np.abs(G - Gd).max() <= 1e-10
    assert _qqt(parts, orbs) <= 1e-12
    # the space deflated: the basis is not longer than the sector
    dims = [oracle.binom(m.L, m.nup + 1) * oracle.binom(m.L, m.ndn),
            oracle.binom(m.L, m.nup - 1) * oracle.binom(m.L, m.ndn)]
    for (lam, _), d in zip(parts, dims):
        assert lam.shape[0] <= d + 2
    lam, Qe = parts[0]
    ev = np.linalg.eigvalsh(dense.dense_h(m.t, m.U, m.nup + 1, m.ndn))
    wgt = (Qe ** 2).sum(axis=0)
    for x, wx in zip(lam, wgt):
        if wx > 1e-8:
            assert np.abs(ev - x).min() <= 1e-8


def test_band_deflation_of_vanishing_and_repeated_starts():
    # orbital 0 deep below the others: always occupied, c+_0 |Omega> = 0;
    # the repeated orbital 2 gives a linearly dependent start state
    m = synth.random_model(502, 6, 3, 3)
    t = m.t.copy()
    t[0, 0] = -40.0
    e0, psi = _gs(synth.Model("deep", t, m.U, 3, 3))
    orbs = [0, 2, 2, 4]
    G, parts = band.green_band(t, m.U, 3, 3, psi, orbs, e0, Z, max_basis=2000, full_reorth=True)
    Gd = dense.lehmann_green(t, m.U, 3, 3, orbs, Z, psi=psi, e0=e0)
    assert np.abs(G - Gd).max() <= 1e-10
    assert np.abs(G[:, 1, 1] - G[:, 2, 2]).max() <= 1e-12
    assert np.abs(G[:, 1, 2] - G[:, 1, 1]).max() <= 1e-12
    assert _qqt(parts, orbs) <= 1e-12


def test_band_equals_exhausted_continued_fractions():
    m = synth.random_model(503, 5, 2, 2)
    e0, psi = _gs(m)
    orbs = [1, 3, 4]
    G, _ = band.green_band(m.t, m.U, 2, 2, psi, orbs, e0, Z, max_basis=2000, full_reorth=True)
    ch = oracle.green_cf(m.t, m.U, 2, 2, psi, orbs, max_steps=300, nthreads=1)
    Gc = cf.green_matrix(ch, 3, Z, e0)
    assert np.abs(G - Gc).max() <= 1e-10


def test_band_paper_recurrence_matches_reorthogonalised_on_short_bases():
    m = synth.chain(8, U=4.0, mu=2.0, nup=4, ndn=4)
    e0, psi = _gs(m)
    orbs = [0, 1, 2, 3]
    for R in (4, 9, 24):
        G, parts = band.green_band(m.t, m.U, 4, 4, psi, orbs, e0, Z, max_basis=R)
        Gr, pr = band.green_band(m.t, m.U, 4, 4, psi, orbs, e0, Z, max_basis=R, full_reorth=True)
        assert parts[0][1].shape[1] == R
        assert _qqt(parts, orbs) <= 1e-12
        assert np.abs(G - Gr).max() <= 1e-9
        assert np.abs(parts[0][0] - pr[0][0]).max() <= 1e-9


def test_band_paper_stopping_rule():
    # the run ends once the lowest eigenvalue of T is stable over a block
    m = synth.random_model(501, 6, 3, 2)
    e0, psi = _gs(m)
    G, parts = band.green_band(m.t, m.U, 3, 2, psi, [0, 2, 5], e0, Z, max_basis=2000,
                               etol=1e-10)
    ev = np.linalg.eigvalsh(dense.dense_h(m.t, m.U, 4, 2))
    R = parts[0][0].shape[0]
    assert 3 < R < 225
    assert abs(parts[0][0][0] - ev[0]) <= 1e-9 * max(1.0, abs(ev[0]))
    assert _qqt(parts, [0, 2, 5]) <= 1e-12


@pytest.mark.parametrize("full_reorth", [False, True], ids=["paper", "reorth"])
def test_band_truncated_moments_equal_dense(full_reorth):
    # A truncated run of m complete blocks reproduces B^T H^k B for k < 2m:
    # checked against H built densely (oracle/dense.py), with R = 4 blocks.
    m = synth.chain(8, U=4.0, mu=2.0, nup=4, ndn=4)
    e0, psi = _gs(m)
    orbs = [0, 1, 2, 3]
    _, parts = band.green_band(m.t, m.U, 4, 4, psi, orbs, e0, Z, max_basis=16,
                               full_reorth=full_reorth)
    for part, (nup2, sgn) in enumerate(((5, 0), (3, 1))):
        B = np.stack([oracle.apply_op(m.L, 4, 4, psi, sgn, mu) for mu in orbs], axis=1)
        H = dense.dense_h(m.t, m.U, nup2, 4)
        lam, Q = parts[part]
        HkB = B.copy()
        for k in range(8):
            ref = B.T @ HkB
            got = (Q * lam ** k) @ Q.T
            assert np.abs(got - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
            HkB = H @ HkB
