"""Continued-fraction evaluation and CPT for the oracle (TEST INFRASTRUCTURE
ONLY; see the package docstring).  NumPy, complex128, plain loops.

Continued fractions (subsection "The Lanczos algorithm for the Green
function", eq. (jacobi)), with the ground-state energy E0 restored from the
resolvents of eq. (green):
  electron: G_e(z) = b0^2 / (z + E0 - a0 - b1^2 / (z + E0 - a1 - ...))
  hole:     G_h(z) = b0^2 / (z - E0 + a0 - b1^2 / (z - E0 + a1 - ...))
evaluated from the bottom floor up.  The off-diagonal element follows the
paper's trick for a real Hamiltonian: G_ij = (G+_ij - G_ii - G_jj)/2.

CPT (section "Cluster perturbation theory", eqs. (CPT1) and (CPT3)):
  V(k)_ij = sum over inter-cluster bonds of t exp(i k.(shift.E)) (+ h.c.),
  G(k,z) = (G_c(z)^-1 - V(k))^-1,
  G_per(k,z) = (1/L) sum_ij exp(-i k.(R_i - R_j)) G_ij(k,z),
with the partial Fourier convention t_RR'(k) = sum_r exp(i k.r) t_{R, r+R'}
of subsection "Partial Fourier transforms".
"""
from __future__ import annotations

import numpy as np


def cf_eval(b0sq: float, a, b2, z, e0: float, part: int) -> np.ndarray:
    """One continued fraction at complex frequencies z (array)."""
    z = np.asarray(z, dtype=np.complex128)
    a = np.asarray(a, dtype=np.float64)
    b2 = np.asarray(b2, dtype=np.float64)
    M = a.shape[0]
    if M == 0 or b0sq == 0.0:
        return np.zeros_like(z)
    if part == 0:
        zz = z + e0
        sgn = 1.0
    else:
        zz = z - e0
        sgn = -1.0
    g = zz - sgn * a[M - 1]
    for n in range(M - 2, -1, -1):
        g = zz - sgn * a[n] - b2[n] / g
    return b0sq / g


def green_matrix(chains: dict, n_orb: int, z, e0: float) -> np.ndarray:
    """G[z, i, j] (complex128) from the chains returned by oracle.green_cf."""
    z = np.asarray(z, dtype=np.complex128)
    G = np.zeros((z.shape[0], n_orb, n_orb), dtype=np.complex128)
    full = {}
    for (i, j, part), (b0, a, b2) in chains.items():
        full.setdefault((i, j), np.zeros(z.shape[0], dtype=np.complex128))
        full[(i, j)] += cf_eval(b0, a, b2, z, e0, part)
    for i in range(n_orb):
        G[:, i, i] = full[(i, i)]
    for i in range(n_orb):
        for j in range(i + 1, n_orb):
            gij = 0.5 * (full[(i, j)] - full[(i, i)] - full[(j, j)])
            G[:, i, j] = gij
            G[:, j, i] = gij
    return G


def v_of_k(L: int, bonds, E, k) -> np.ndarray:
    """Inter-cluster hopping V(k) (L x L complex), k in units of 2 pi.
    bonds: iterable of (i, j, (s1, s2, s3), t) meaning amplitude t between
    site i of the cluster at the origin and site j of the cluster at
    r = s1 E1 + s2 E2 + s3 E3; the Hermitian partner is added here."""
    E = np.asarray(E, dtype=np.float64).reshape(3, 3)
    kk = 2.0 * np.pi * np.asarray(k, dtype=np.float64)
    V = np.zeros((L, L), dtype=np.complex128)
    for (i, j, s, t) in bonds:
        r = np.asarray(s, dtype=np.float64) @ E
        ph = np.exp(1j * np.dot(kk, r))
        V[i, j] += t * ph
        V[j, i] += t * np.conj(ph)
    return V


def cpt_periodized(Gc: np.ndarray, R, E, bonds, ks) -> np.ndarray:
    """G_per[k, z] from the cluster Green function Gc[z, L, L]."""
    Gc = np.asarray(Gc, dtype=np.complex128)
    nz, L, _ = Gc.shape
    R = np.asarray(R, dtype=np.float64).reshape(L, 3)
    ks = np.asarray(ks, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((ks.shape[0], nz), dtype=np.complex128)
    Gcinv = np.array([np.linalg.inv(Gc[iz]) for iz in range(nz)])
    for ik, k in enumerate(ks):
        V = v_of_k(L, bonds, E, k)
        kk = 2.0 * np.pi * k
        ph = np.exp(-1j * (R @ kk))          # e^{-i k.R_i}
        P = np.outer(ph, np.conj(ph))         # e^{-i k.(R_i - R_j)}
        for iz in range(nz):
            G = np.linalg.inv(Gcinv[iz] - V)
            out[ik, iz] = np.sum(P * G) / L
    return out
