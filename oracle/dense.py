"""Dense exact diagonalisation and the exact Lehmann sum, for small sectors
(TEST INFRASTRUCTURE ONLY; see the package docstring).

This module is deliberately independent of ``ora.c``: it applies fermion
operators generically to Fock states and builds H as a dense matrix.

Fock states are 2L-bit integers b = b_up + 2^L b_dn (subsection "Coding of
the basis states", eq. (basis)): mode m < L is up orbital m, mode L + m is
down orbital m, and the creation operators of eq. (basis) are ordered by
mode index, lowest mode leftmost.  An annihilation or creation operator on
mode m therefore carries the sign (-1)^(number of occupied modes below m).

The Green function is the Lehmann sum of eq. (spectral1) with the residues
Q of the subsection "Spectral representation", for up-spin operators.
"""
from __future__ import annotations

import numpy as np


def _bits(x: int) -> int:
    return bin(x).count("1")


def apply_c(state: int, mode: int, create: bool):
    """c+_mode or c_mode on a Fock state: (sign, new_state) or None."""
    occ = (state >> mode) & 1
    if create == bool(occ):
        return None
    sign = -1.0 if _bits(state & ((1 << mode) - 1)) & 1 else 1.0
    return sign, state ^ (1 << mode)


def sector_basis(L: int, nup: int, ndn: int):
    """Fock states of sector (nup, ndn) ordered by i = I_up + d_up I_dn, where
    I_sigma is the position in the ascending list of spin strings (brute
    force over all 2^L strings)."""
    ups = [x for x in range(1 << L) if _bits(x) == nup]
    dns = [x for x in range(1 << L) if _bits(x) == ndn]
    states = [u | (d << L) for d in dns for u in ups]
    index = {s: i for i, s in enumerate(states)}
    return states, index


def dense_h(t, U, nup: int, ndn: int) -> np.ndarray:
    """H = sum_{ab,sigma} t_ab c+_a,sigma c_b,sigma + sum_k U_k n_k,up n_k,dn
    (eq. (Hubbard) with the chemical potential on the diagonal of t)."""
    t = np.asarray(t, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    L = t.shape[0]
    states, index = sector_basis(L, nup, ndn)
    d = len(states)
    H = np.zeros((d, d))
    for j, s in enumerate(states):
        for spin in (0, 1):
            off = spin * L
            for a in range(L):
                for b in range(L):
                    if t[a, b] == 0.0:
                        continue
                    r1 = apply_c(s, off + b, False)
                    if r1 is None:
                        continue
                    r2 = apply_c(r1[1], off + a, True)
                    if r2 is None:
                        continue
                    H[index[r2[1]], j] += t[a, b] * r1[0] * r2[0]
        for k in range(L):
            if (s >> k) & 1 and (s >> (L + k)) & 1:
                H[j, j] += U[k]
    return H


def op_matrix(L: int, nup: int, ndn: int, mode: int, create: bool) -> np.ndarray:
    """Matrix of c+_mode (create) or c_mode from sector (nup, ndn) to the
    sector with one more or one fewer electron of that spin."""
    spin = 0 if mode < L else 1
    dn = 1 if create else -1
    nup2, ndn2 = (nup + dn, ndn) if spin == 0 else (nup, ndn + dn)
    src, _ = sector_basis(L, nup, ndn)
    dst, dindex = sector_basis(L, nup2, ndn2)
    M = np.zeros((len(dst), len(src)))
    for j, s in enumerate(src):
        r = apply_c(s, mode, create)
        if r is not None:
            M[dindex[r[1]], j] += r[0]
    return M


def ground_state(t, U, nup: int, ndn: int):
    """(E0, psi, all eigenvalues) of the sector by numpy.linalg.eigh."""
    H = dense_h(t, U, nup, ndn)
    w, v = np.linalg.eigh(H)
    return float(w[0]), v[:, 0].copy(), w


def lehmann_green(t, U, nup: int, ndn: int, orbs, z, psi=None, e0=None) -> np.ndarray:
    """Exact up-spin G_ij(z) for i, j in ``orbs`` (eq. (spectral1)):
    electron residues <r|c+_nu|Omega> in sector (nup+1, ndn), hole residues
    <r|c_mu|Omega> in (nup-1, ndn)."""
    t = np.asarray(t, dtype=np.float64)
    L = t.shape[0]
    z = np.asarray(z, dtype=np.complex128)
    if psi is None:
        e0, psi, _ = ground_state(t, U, nup, ndn)
    n = len(orbs)
    G = np.zeros((z.shape[0], n, n), dtype=np.complex128)
    if nup + 1 <= L:
        He = dense_h(t, U, nup + 1, ndn)
        we, ve = np.linalg.eigh(He)
        q = np.array([ve.T @ (op_matrix(L, nup, ndn, m, True) @ psi) for m in orbs])
        for iz, zz in enumerate(z):
            G[iz] += (q / (zz - (we - e0))) @ q.T
    if nup - 1 >= 0:
        Hh = dense_h(t, U, nup - 1, ndn)
        wh, vh = np.linalg.eigh(Hh)
        p = np.array([vh.T @ (op_matrix(L, nup, ndn, m, False) @ psi) for m in orbs])
        for iz, zz in enumerate(z):
            G[iz] += (p / (zz + (wh - e0))) @ p.T
    return G
