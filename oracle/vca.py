"""Potthoff self-energy functional for the oracle (TEST INFRASTRUCTURE ONLY;
see the package docstring).  NumPy / SciPy, FP64.

Follows the paper's subsection "Practical calculation of the Potthoff
functional": for a cluster reference system H' (variational parameters x)
with ground-state energy Omega' (= E0 of H', the chemical potential in its
hopping) and Green function G' in its Lehmann form (poles w'_r, residues
Q, eq. (spectral1)), the functional of eq. (sef4),
    Omega = Omega' - int dw/(2 pi i) (L/N) sum_k ln det[1 - V(k) G'(k, w)],
is, with the frequency integral done analytically (eq. (omega4)),
    Omega = Omega' - sum_{w'_r < 0} w'_r + (L/N) sum_k sum_{w_r(k) < 0} w_r(k),
where w_r(k) are the eigenvalues of L(k) = Lambda + Q^T V(k) Q.  Both spins
are summed (the factor 2 below: the spin blocks of G' are equal for the
spin-symmetric sectors used here).  V(k) is the difference between the
lattice's one-body matrix in the cluster basis and the reference's: the
inter-cluster bonds (same convention as the CDMFT oracle: phase
exp(2 pi i k . s) for a shift s in super-lattice units) plus any
k-independent change of the intra-cluster hopping.

The numerical form integrates along the imaginary axis: for each k,
    sum_{w_r(k) < 0} w_r(k) - sum_{w'_r < 0} w'_r
      = -(1/pi) int_0^inf dw Re ln det[1 - V(k) G'(i w)] + tr V(k) / 2,
which follows from det(1 - V G'(z)) = det(z - L(k)) / det(z - Lambda) and, for
one pole a, int_0^W Re ln(i w - a) dw = (const in a) + |a| pi / 2 + o(1).
"""
from __future__ import annotations

import numpy as np


def cluster_lehmann(t, U, nup, ndn, max_basis=4000):
    """E0, poles w' (electron part lam - E0, hole part E0 - lam) and Q
    [L, R] of the up-spin G' on every cluster orbital, from the oracle's band
    Lanczos run to exhaustion (full reorthogonalisation: exact Lehmann sum)."""
    import oracle
    from oracle import band
    L = np.asarray(t).shape[0]
    gs = oracle.lanczos_gs(t, U, nup, ndn, want_vector=True, nthreads=1)
    z = np.array([1j])
    _, parts = band.green_band(t, U, nup, ndn, gs["psi"], list(range(L)), gs["e0"], z,
                               max_basis=max_basis, full_reorth=True)
    (le, Qe), (lh, Qh) = parts
    poles = np.concatenate([le - gs["e0"], gs["e0"] - lh])
    Q = np.concatenate([Qe, Qh], axis=1)
    return gs["e0"], poles, Q


def v_of_k(L, dt, bonds, k):
    """V(k) = dt + inter-cluster hopping at k (Hermitian partner added)."""
    V = np.array(dt, dtype=np.complex128).reshape(L, L)
    for (i, j, s, t) in bonds:
        ph = np.exp(2j * np.pi * np.dot(np.asarray(k, dtype=np.float64), np.asarray(s, dtype=np.float64)))
        V[i, j] += t * ph
        V[j, i] += t * np.conj(ph)
    return V


def omega_poles(e0, poles, Q, dt, bonds, ks):
    """Eq. (omega4), both spins: the negative eigenvalues of L(k) averaged
    over the k grid, minus the negative poles of G'."""
    s = 0.0
    L = Q.shape[0]
    for k in ks:
        Lk = np.diag(poles) + Q.T @ v_of_k(L, dt, bonds, k) @ Q
        w = np.linalg.eigvalsh(0.5 * (Lk + Lk.conj().T))
        s += np.sum(w[w < 0.0])
    return e0 + 2.0 * (s / len(ks) - np.sum(poles[poles < 0.0]))


def omega_numeric(e0, poles, Q, dt, bonds, ks):
    """Eq. (sef4) with the frequency integral done numerically on the
    imaginary axis (scipy.integrate.quad on w in [0, inf))."""
    from scipy.integrate import quad
    L = Q.shape[0]
    s = 0.0
    for k in ks:
        V = v_of_k(L, dt, bonds, k)

        def f(w):
            G = (Q / (1j * w - poles)) @ Q.T
            return np.log(np.linalg.det(np.eye(L) - V @ G)).real

        val, _ = quad(f, 0.0, np.inf, epsabs=1e-12, epsrel=1e-11, limit=400)
        s += -val / np.pi + 0.5 * np.trace(V).real
    return e0 + 2.0 * s / len(ks)


def omega_free(h0, bonds, ks):
    """U = 0: the lattice grand potential per cluster, both spins: the
    negative one-body energies of h0 + V_inter(k) averaged over k."""
    L = np.asarray(h0).shape[0]
    s = 0.0
    for k in ks:
        w = np.linalg.eigvalsh(v_of_k(L, h0, bonds, k))
        s += np.sum(w[w < 0.0])
    return 2.0 * s / len(ks)
