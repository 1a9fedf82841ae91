"""Symmetry-adapted basis and stored Hamiltonian of an abelian point group
with real characters (TEST INFRASTRUCTURE ONLY; see the package docstring).
NumPy / SciPy, FP64.

Follows the paper's subsection "Cluster symmetries".

* A group element g permutes the orbitals (site a -> perm[g][a]), the same
  way for both spins.  Acting on a Fock state (creation operators ordered by
  mode, up orbitals before down ones, eq. (basis)) it gives g|b> =
  phi_g(b) |gb>, where gb is the permuted occupation and phi_g(b) the sign of
  reordering the permuted creation operators; the up and down blocks are
  reordered separately, so phi_g(b) = phi_g(b_up) phi_g(b_dn).
* In the one-dimensional irreducible representation with characters chi
  (here +1 or -1), each orbit contributes at most one state, the projection of
  its representative b (the orbit member with the smallest label
  i_up + d_up i_dn, i.e. the smallest b_up + 2^L b_dn):
      |psi_b> = P|b> / |P|b>|,   P = (1/|G|) sum_g chi_g g.
  |P|b>|^2 = (1/|G|) sum_{g: gb = b} chi_g phi_g(b), which is either 0 (the
  state drops out) or m_b / |G| with m_b the size of b's stabiliser.
* Matrix element (eq. (matrixElement)): for a term H_r with
  H_r|b1> = c_r |b'>,
      <psi_b2| H_r |psi_b1> = c_r S / sqrt(m_b1 m_b2),
      S = sum_{g: g b' = b2} chi_g phi_g(b'),
  b2 being the representative of b'.  The terms of one column b1 are summed
  before they are stored (the paper's cancellation step); entries whose sum
  is at most 1e-13 max|t| in magnitude are dropped.  The diagonal
  sum_a t_aa n_a + sum_a U_a n_a,up n_a,dn is the same on the whole orbit.
* The index of a representative is found by binary search in the sorted
  list of representatives, as the paper describes.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy import sparse

DROP = 1e-13


def strings(L: int, n: int) -> np.ndarray:
    """Ascending bit strings of L orbitals with n set bits."""
    if n < 0 or n > L:
        return np.zeros(0, dtype=np.int64)
    return np.array(sorted(sum(1 << a for a in c) for c in itertools.combinations(range(L), n)),
                    dtype=np.int64)


def string_action(s: int, perm) -> tuple[int, int]:
    """(gb, phi_g(b)) for one spin string: the permuted string and the sign
    of the permutation that sorts the images of its occupied orbitals (taken
    in ascending order of the original orbitals)."""
    occ = [a for a in range(len(perm)) if (s >> a) & 1]
    img = [perm[a] for a in occ]
    inversions = sum(1 for x in range(len(img)) for y in range(x + 1, len(img)) if img[x] > img[y])
    return sum(1 << a for a in img), (-1 if inversions % 2 else 1)


def check_group(perms, chi):
    """The elements form a group (closed under composition, identity first)
    and chi is a real one-dimensional representation of it."""
    perms = [tuple(int(x) for x in p) for p in perms]
    L = len(perms[0])
    assert perms[0] == tuple(range(L)), "element 0 must be the identity"
    index = {p: k for k, p in enumerate(perms)}
    assert len(index) == len(perms), "repeated element"
    for g, p in enumerate(perms):
        assert sorted(p) == list(range(L)), "not a permutation"
        for h, q in enumerate(perms):
            pq = tuple(p[q[a]] for a in range(L))
            assert pq in index, "not closed"
            assert chi[index[pq]] == chi[g] * chi[h], "chi is not a representation"
    assert all(c in (1, -1) for c in chi)


def check_invariant(t, U, perms):
    t = np.asarray(t, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    for p in perms:
        p = np.asarray(p)
        assert np.array_equal(t[np.ix_(p, p)], t), "t is not invariant"
        assert np.array_equal(U[p], U), "U is not invariant"


def _spin_action(L, n, perms):
    """For every string of popcount n and every element: the label of its
    image and the phase."""
    S = strings(L, n)
    lab = {int(s): k for k, s in enumerate(S)}
    img = np.zeros((len(perms), len(S)), dtype=np.int64)
    ph = np.zeros((len(perms), len(S)))
    for g, p in enumerate(perms):
        for k, s in enumerate(S):
            gs, f = string_action(int(s), p)
            img[g, k] = lab[gs]
            ph[g, k] = f
    return S, img, ph


def sector_orbits(L, nup, ndn, perms, chi):
    """Orbit data of every state of the sector (labels i = i_up + d_up i_dn):
    rep[i] (smallest label of the orbit), m[i] (number of elements taking i
    to rep[i], the stabiliser size), proj[i] (sum over those elements of
    chi_g phi_g(i)), and the ascending list of representatives whose
    projected state does not vanish."""
    Su, iu, pu = _spin_action(L, nup, perms)
    Sd, idn, pd = _spin_action(L, ndn, perms)
    du, dd = len(Su), len(Sd)
    ku = np.tile(np.arange(du), dd)
    kd = np.repeat(np.arange(dd), du)
    full = ku + du * kd
    gi = np.stack([iu[g][ku] + du * idn[g][kd] for g in range(len(perms))])
    gp = np.stack([pu[g][ku] * pd[g][kd] for g in range(len(perms))])
    c = np.asarray(chi, dtype=np.float64)[:, None]
    rep = gi.min(axis=0)
    to_rep = gi == rep[None, :]
    m = to_rep.sum(axis=0)
    proj = (to_rep * c * gp).sum(axis=0)
    keep = (rep == full) & (proj > 0.5)
    return dict(Su=Su, Sd=Sd, du=du, dd=dd, rep=rep, m=m, proj=proj, basis=full[keep])


def sym_hamiltonian(t, U, nup, ndn, perms, chi):
    """(ascending representative labels, CSR matrix of H in the irrep's
    orthonormal symmetry-adapted basis).  Row/column k is representative
    basis[k]."""
    t = np.asarray(t, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    L = t.shape[0]
    check_group(perms, chi)
    check_invariant(t, U, perms)
    o = sector_orbits(L, nup, ndn, perms, chi)
    basis, du = o["basis"], o["du"]
    n = len(basis)
    if n == 0:
        return basis, sparse.csr_matrix((0, 0))
    col = np.arange(n)
    bu = basis % du
    bd = basis // du
    su, sd = o["Su"][bu], o["Sd"][bd]
    rows, cols, vals = [], [], []
    # diagonal: t_aa n_a + U_a n_a,up n_a,dn
    diag = np.zeros(n)
    for a in range(L):
        nu = (su >> a) & 1
        nd = (sd >> a) & 1
        diag += t[a, a] * (nu + nd) + U[a] * nu * nd
    rows.append(col)
    cols.append(col)
    vals.append(diag)
    lab_u = {int(s): k for k, s in enumerate(o["Su"])}
    lab_d = {int(s): k for k, s in enumerate(o["Sd"])}
    for a in range(L):
        for b in range(L):
            if a == b or t[a, b] == 0.0:
                continue
            for spin in (0, 1):
                s = su if spin == 0 else sd
                ok = (((s >> b) & 1) == 1) & (((s >> a) & 1) == 0)
                if not ok.any():
                    continue
                s0 = s[ok]
                # c+_a c_b: sign (-1)^(occupied below b) (-1)^(occupied below a after removal)
                s1 = s0 & ~(1 << b)
                nb = np.array([bin(int(x) & ((1 << b) - 1)).count("1") for x in s0])
                na = np.array([bin(int(x) & ((1 << a) - 1)).count("1") for x in s1])
                sign = np.where((nb + na) % 2 == 1, -1.0, 1.0)
                s2 = s1 | (1 << a)
                if spin == 0:
                    tu = np.array([lab_u[int(x)] for x in s2])
                    j = tu + du * bd[ok]
                else:
                    td = np.array([lab_d[int(x)] for x in s2])
                    j = bu[ok] + du * td
                r2 = o["rep"][j]
                pos = np.searchsorted(basis, r2)
                pos_c = np.minimum(pos, n - 1)
                found = basis[pos_c] == r2
                v = t[a, b] * sign * o["proj"][j] / np.sqrt(o["m"][basis[col[ok]]] * o["m"][j])
                rows.append(pos_c[found])
                cols.append(col[ok][found])
                vals.append(v[found])
    H = sparse.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(n, n)).tocsr()
    H.sum_duplicates()
    tmax = max(np.abs(t).max(), np.abs(U).max(), 1e-300)
    H.data[np.abs(H.data) <= DROP * tmax] = 0.0
    H.eliminate_zeros()
    H.sort_indices()
    return basis, H


def value_counts(H, digits=9):
    """{value: number of stored entries with that value}, values rounded."""
    v, c = np.unique(np.round(H.data, digits), return_counts=True)
    return dict(zip(v.tolist(), c.tolist()))


# ---------------------------------------------------------------- one column at a time
# The same elements computed for one representative with plain loops and the
# combinatorial labels of the strings (subsection "Coding of the basis
# states": the position of a string in the ascending list is
# sum_j C(p_j, j + 1) over its set bits p_0 < p_1 < ...), for sectors too
# large to enumerate whole.

def string_label(s: int) -> int:
    from math import comb
    lab, j = 0, 0
    a = 0
    while s >> a:
        if (s >> a) & 1:
            lab += comb(a, j + 1)
            j += 1
        a += 1
    return lab


def _state_action(bu: int, bd: int, perm):
    gu, fu = string_action(bu, perm)
    gd, fd = string_action(bd, perm)
    return gu, gd, fu * fd


def _full_label(bu, bd, d_up):
    return string_label(bu) + d_up * string_label(bd)


def orbit_info(bu: int, bd: int, perms, chi, d_up: int):
    """(representative label, m, S) of the state (bu, bd): the smallest
    label of its orbit, the number of elements taking the state there, and
    the sum of chi_g phi_g over them."""
    best, m, S = None, 0, 0
    for g, p in enumerate(perms):
        gu, gd, f = _state_action(bu, bd, p)
        lab = _full_label(gu, gd, d_up)
        if best is None or lab < best:
            best, m, S = lab, 1, chi[g] * f
        elif lab == best:
            m += 1
            S += chi[g] * f
    return best, m, S


def is_kept(bu: int, bd: int, perms, chi, d_up: int) -> bool:
    """The state is its orbit's representative and its projection survives."""
    rep, m, S = orbit_info(bu, bd, perms, chi, d_up)
    return rep == _full_label(bu, bd, d_up) and S > 0


def sym_column(t, U, bu: int, bd: int, perms, chi):
    """{representative label b2: <b2|H|b1>} for the representative
    b1 = (bu, bd): the diagonal plus every hop, summed per target and with
    the same drop rule as sym_hamiltonian."""
    from math import comb
    t = np.asarray(t, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    L = t.shape[0]
    d_up = comb(L, bin(bu).count("1"))
    rep1, m1, S1 = orbit_info(bu, bd, perms, chi, d_up)
    assert rep1 == _full_label(bu, bd, d_up) and S1 > 0, "not a kept representative"
    out = {}
    diag = 0.0
    for a in range(L):
        nu, nd = (bu >> a) & 1, (bd >> a) & 1
        diag += t[a, a] * (nu + nd) + U[a] * nu * nd
    out[rep1] = diag
    for a in range(L):
        for b in range(L):
            if a == b or t[a, b] == 0.0:
                continue
            for spin in (0, 1):
                s = bu if spin == 0 else bd
                if not ((s >> b) & 1) or ((s >> a) & 1):
                    continue
                s1 = s & ~(1 << b)
                sign = (-1) ** (bin(s & ((1 << b) - 1)).count("1") + bin(s1 & ((1 << a) - 1)).count("1"))
                s2 = s1 | (1 << a)
                tu, td = (s2, bd) if spin == 0 else (bu, s2)
                rep2, m2, S2 = orbit_info(tu, td, perms, chi, d_up)
                if S2 == 0:
                    continue
                out[rep2] = out.get(rep2, 0.0) + t[a, b] * sign * S2 / np.sqrt(m1 * m2)
    tmax = max(np.abs(t).max(), np.abs(U).max(), 1e-300)
    return {k: v for k, v in out.items() if abs(v) > DROP * tmax}
