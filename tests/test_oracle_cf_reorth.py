"""Pins of the oracle's continued-fraction chain with full
reorthogonalisation (a test device for long chains), on the CPU:

  * run to exhaustion on small sectors it gives the exact Lehmann sum of
    dense diagonalisation (oracle/dense.py, sharing no code with it);
  * truncated at M floors it is the M-step Lanczos recurrence of exact
    arithmetic: its continued fraction equals b0^2 [(z + E0 - T_M)^-1]_00
    with T_M = Q^T H Q, Q the orthonormal basis of the Krylov space
    {phi, H phi, ..., H^(M-1) phi} from a QR factorisation of the dense Krylov
    matrix;
  * on short chains (before orthogonality is lost) it equals the paper's
    recurrence without reorthogonalisation.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import cf, dense

Z = synth.omega_grid()[::4]


@pytest.mark.parametrize("seed,L,nup,ndn", [(42, 4, 2, 2), (42, 5, 2, 3), (43, 6, 3, 3)])
def test_exhausted_full_reorth_chains_equal_lehmann(seed, L, nup, ndn):
    m = synth.random_model(seed, L, nup, ndn)
    e0, psi, w = dense.ground_state(m.t, m.U, nup, ndn)
    assert w[1] - w[0] > 1e-3
    orbs = list(range(L))
    steps = max(oracle.binom(L, nup + 1), oracle.binom(L, nup - 1)) * oracle.binom(L, ndn) + 5
    ch = oracle.green_cf(m.t, m.U, nup, ndn, psi, orbs, max_steps=steps, full_reorth=True,
                         nthreads=1)
    # exact arithmetic breaks down at the dimension of the Krylov space
    for (i, j, part), (b0, a, b2) in ch.items():
        assert len(a) <= steps - 5
    G = cf.green_matrix(ch, L, Z, e0)
    Gd = dense.lehmann_green(m.t, m.U, nup, ndn, orbs, Z, psi=psi, e0=e0)
    assert np.abs(G - Gd).max() < 1e-10


@pytest.mark.parametrize("part", [0, 1])
def test_truncated_full_reorth_chain_is_krylov_projection(part):
    m = synth.random_model(43, 6, 3, 3)
    e0, psi, _ = dense.ground_state(m.t, m.U, 3, 3)
    nup2 = 4 if part == 0 else 2
    phi = oracle.apply_op(6, 3, 3, psi, part, 2)
    H = dense.dense_h(m.t, m.U, nup2, 3)
    for M in (1, 3, 6):
        b0, a, b2 = oracle.cf_chain(m.t, m.U, nup2, 3, phi, M, full_reorth=True, nthreads=1)
        assert len(a) == M
        K = np.empty((phi.shape[0], M))
        x = phi / np.linalg.norm(phi)
        for k in range(M):
            K[:, k] = x
            x = H @ x
            x = x / np.linalg.norm(x)
        Q, R = np.linalg.qr(K)
        T = Q.T @ H @ Q
        e1 = np.zeros(M)
        e1[0] = 1.0
        sgn = 1.0 if part == 0 else -1.0
        want = np.array([b0 * np.linalg.solve(zz * np.eye(M) - sgn * (T - e0 * np.eye(M)), e1)[0]
                         for zz in Z])
        got = cf.cf_eval(b0, a, b2, Z, e0, part)
        assert abs(b0 - phi @ phi) < 1e-14
        assert np.abs(got - want).max() < 1e-10, M


def test_short_chain_equals_plain_recurrence():
    m = synth.random_model(44, 6, 3, 2)
    e0, psi, _ = dense.ground_state(m.t, m.U, 3, 2)
    phi = oracle.apply_op(6, 3, 2, psi, 0, 1)
    b0, a, b2 = oracle.cf_chain(m.t, m.U, 4, 2, phi, 8, full_reorth=True, nthreads=1)
    c0, c, c2 = oracle.cf_chain(m.t, m.U, 4, 2, phi, 8, nthreads=1)
    assert b0 == c0
    assert np.allclose(a, c, rtol=0, atol=1e-12) and np.allclose(b2, c2, rtol=0, atol=1e-12)
