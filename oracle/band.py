"""Band Lanczos Green function for the oracle (TEST INFRASTRUCTURE ONLY; see
the package docstring).  NumPy, FP64, plain loops over the basis vectors.

Follows the paper's subsection "The band Lanczos algorithm for the Green
function": the Krylov space of the p states |phi_mu> = c+_mu |Omega> (and,
for the hole part, c_mu |Omega>) is built one basis vector at a time; each new
vector H|v_j> is orthogonalised against the previous band of basis vectors,
redundant candidates are deflated, and the projected Hamiltonian T (a band of
2p diagonals around the main one, plus the entries that deflation adds) is
diagonalised, T = U diag(Lambda) U^T.  The projections of the start states on
its eigenvectors give Q (Q_mu,r = sum_k rho_k,mu U_k,r, with |phi_mu> =
sum_k rho_k,mu |v_k>), so that
    G_e(z)_mu,nu = sum_r Q_mu,r Q_nu,r / (z + E0 - Lambda_r)
    G_h(z)_mu,nu = sum_r Q_mu,r Q_nu,r / (z - E0 + Lambda_r)
(the Lehmann form of eq. (spectral1)), and the concatenated Q of both parts
satisfies Q Q^T = 1.

The recurrence is the Hermitian band Lanczos method of Freund (the paper's
reference for it), written here from its steps: normalise the next candidate
(or deflate it), orthogonalise the remaining candidates against it, form the
new candidate H|v_j>, remove its components along the band of previous basis
vectors (known from symmetry) and along v_j and the deflated look-back set
(computed), and record the coefficients in T.
"""
from __future__ import annotations

import numpy as np


def band_lanczos(matvec, B: np.ndarray, max_basis: int, dtol_rel: float = 1e-10,
                 etol: float = 0.0, full_reorth: bool = False):
    """Band Lanczos from the starting block B (n x p, columns may be zero or
    linearly dependent).  Returns (T [R x R], rho [R x p], R).

    Deflation: a candidate whose norm is <= dtol_rel * max(1, max |T_kk| so
    far) is removed.  The run stops when no candidate is left (the Krylov
    space is exhausted), when R reaches max_basis, or (etol > 0) when the
    lowest eigenvalue of T has moved by at most etol * max(1, |theta|) over
    one block of p basis vectors (tested when R is a multiple of p), the
    paper's rule against orthogonality leaks.
    full_reorth (a test device, not the paper's recurrence) also removes
    from each new candidate, and again from each candidate before its
    deflation test, its components along every earlier basis vector (two
    passes) without recording them in T, so that an exhausted space deflates
    exactly."""
    n, p = B.shape
    vhat = {k + 1: np.array(B[:, k], dtype=np.float64) for k in range(p)}  # candidates
    V = {}                       # basis vectors v_1, v_2, ...
    t = {}                       # T entries t[(i, k)]
    rho = np.zeros((max_basis + p, p))
    pc = p                       # current block size
    I = []                       # deflated look-back set
    scale = 1.0
    theta_hist = []
    j = 0
    while j < max_basis:
        j += 1
        # (1) deflation test of the next candidate
        while True:
            if full_reorth:
                # the candidate is also cleared of every earlier basis vector
                # (twice, so that what is left of a dependent candidate is at
                # rounding level and deflates)
                for _ in range(2):
                    for k in sorted(V):
                        vhat[j] = vhat[j] - float(np.dot(V[k], vhat[j])) * V[k]
            nrm = float(np.sqrt(np.dot(vhat[j], vhat[j])))
            if nrm > dtol_rel * scale:
                break
            if j - pc > 0:
                I.append(j - pc)
            pc -= 1
            if pc == 0:
                return _finish(t, rho, j - 1, p)
            for k in range(j, j + pc):
                vhat[k] = vhat[k + 1]
            del vhat[j + pc]
        # (2) normalise
        if j - pc > 0:
            t[(j, j - pc)] = nrm
        else:
            rho[j - 1, j - pc + p - 1] = nrm
        V[j] = vhat.pop(j) / nrm
        # (3) orthogonalise the other candidates against v_j
        for k in range(j + 1, j + pc):
            c = float(np.dot(V[j], vhat[k]))
            if k - pc > 0:
                t[(j, k - pc)] = c
            else:
                rho[j - 1, k - pc + p - 1] = c
            vhat[k] = vhat[k] - c * V[j]
        # (4) the new candidate
        w = matvec(V[j])
        # (5) the band of previous basis vectors, coefficients by symmetry
        for k in range(max(1, j - pc), j):
            c = t.get((j, k), 0.0)
            t[(k, j)] = c
            w = w - c * V[k]
        # (6) v_j and the look-back set, coefficients computed
        for k in sorted(set(I) | {j}):
            c = float(np.dot(V[k], w))
            t[(k, j)] = c
            w = w - c * V[k]
            if k == j:
                scale = max(scale, abs(c))
        # (7) symmetric entries of the look-back set
        for k in I:
            t[(j, k)] = t[(k, j)]
        if full_reorth:
            for _ in range(2):
                for k in sorted(V):
                    w = w - float(np.dot(V[k], w)) * V[k]
        vhat[j + pc] = w
        if not full_reorth:
            # basis vectors older than the band and outside I are not needed again
            for k in list(V):
                if k < j - p and k not in I:
                    del V[k]
        # the paper's stopping rule: convergence of the lowest eigenvalue of T,
        # tested once per block of p basis vectors against the previous block
        if etol > 0.0 and j % p == 0:
            T, _, _ = _finish(t, rho, j, p)
            th = float(np.linalg.eigvalsh(0.5 * (T + T.T))[0])
            if theta_hist and abs(th - theta_hist[-1]) <= etol * max(1.0, abs(th)):
                return _finish(t, rho, j, p)
            theta_hist.append(th)
    return _finish(t, rho, j, p)


def _finish(t, rho, R, p):
    T = np.zeros((R, R))
    for (i, k), c in t.items():
        if i <= R and k <= R:
            T[i - 1, k - 1] = c
    return T, rho[:R].copy(), R


def lehmann(T: np.ndarray, rho: np.ndarray):
    """Lambda (R) and Q (p x R) from the projected Hamiltonian."""
    if T.shape[0] == 0:
        return np.zeros(0), np.zeros((rho.shape[1], 0))
    lam, U = np.linalg.eigh(0.5 * (T + T.T))
    Q = rho.T @ U
    return lam, Q


def green_band(t, U, nup: int, ndn: int, psi: np.ndarray, orbs, e0: float, z,
               max_basis: int, dtol_rel: float = 1e-10, etol: float = 0.0,
               full_reorth: bool = False, nthreads: int = 1):
    """Up-spin G[z, i, j] for i, j in orbs by band Lanczos, electron part in
    (nup + 1, ndn) and hole part in (nup - 1, ndn).  Returns (G, parts) with
    parts = [(Lambda_e, Q_e), (Lambda_h, Q_h)] (empty when a sector does not
    exist)."""
    import oracle
    t = np.ascontiguousarray(t, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    L = t.shape[0]
    z = np.asarray(z, dtype=np.complex128)
    p = len(orbs)
    G = np.zeros((z.shape[0], p, p), dtype=np.complex128)
    parts = []
    for part in (0, 1):
        nup2 = nup + 1 if part == 0 else nup - 1
        if nup2 < 0 or nup2 > L:
            parts.append((np.zeros(0), np.zeros((p, 0))))
            continue
        B = np.stack([oracle.apply_op(L, nup, ndn, psi, part, mu) for mu in orbs], axis=1)
        T, rho, R = band_lanczos(lambda x: oracle.hv(t, U, nup2, ndn, x, nthreads=nthreads), B,
                                 max_basis, dtol_rel, etol, full_reorth)
        lam, Q = lehmann(T, rho)
        parts.append((lam, Q))
        if part == 0:
            den = z[:, None] + e0 - lam[None, :]
        else:
            den = z[:, None] - e0 + lam[None, :]
        G += np.einsum("ir,jr,zr->zij", Q, Q, 1.0 / den)
    return G, parts
