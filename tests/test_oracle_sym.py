"""Pins of the oracle's symmetry-adapted basis (oracle/sym.py) on the CPU:

  * Table 3x4stats of the paper: the four C2v irrep dimensions of the
    half-filled 12-site cluster and the number of stored matrix elements of
    each value of the nearest-neighbour hopping operator, exactly
    (tests/golden/table_3x4stats.txt; the cluster is 4 sites along x by 3
    along y, sites numbered x + 4y, representatives the smallest label);
  * on small clusters, an independent route: the projector
    P = (1/|G|) sum_g chi_g U_g built as a dense matrix from the generic
    fermion operators of oracle/dense.py (U_g applies the permuted creation
    operators to the vacuum one by one), the normalised columns P|b> of the
    representatives as the basis B: B is orthonormal, B^T H B equals the
    oracle's stored matrix, and the spectra of all irreps together are the
    spectrum of the full sector (dense H);
  * the dimensions of all irreps add up to the sector's dimension; a model
    that is not invariant and characters that are not a representation are
    rejected.
"""
import os

import numpy as np
import pytest

import synth
from oracle import dense, sym as S

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table_3x4stats.txt")
VALUES = (-2.0, -np.sqrt(2.0), -1.0, 1.0, np.sqrt(2.0), 2.0)


def _table():
    rows = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows[f[0]] = (int(f[1]), [int(x) for x in f[2:]])
    return rows


@pytest.mark.parametrize("irrep", ["A1", "A2", "B1", "B2"])
def test_table_3x4stats(irrep):
    dim, counts = _table()[irrep]
    G = synth.c2v_rectangle(4, 3)
    basis, H = S.sym_hamiltonian(synth.nn_hopping(4, 3), np.zeros(12), 6, 6, G, synth.C2V_IRREPS[irrep])
    assert len(basis) == dim
    got = S.value_counts(H)
    want = {round(v, 9): c for v, c in zip(VALUES, counts) if c}
    assert got == want


def _dense_action(L, nup, ndn, perm):
    """U_g on the sector as a dense matrix, from the generic operators."""
    states, index = dense.sector_basis(L, nup, ndn)
    M = np.zeros((len(states), len(states)))
    for k, s in enumerate(states):
        modes = [m for m in range(2 * L) if (s >> m) & 1]
        image = [perm[m] if m < L else L + perm[m - L] for m in modes]
        # |b> = c+_{m1} ... c+_{mk} |0> with m1 < ... < mk: apply the
        # (permuted) rightmost operator first
        sign, st = 1.0, 0
        for m in reversed(image):
            r = dense.apply_c(st, m, True)
            sign *= r[0]
            st = r[1]
        M[index[st], k] += sign
    return states, M


def _projector_route(t, U, nup, ndn, perms, chi):
    L = t.shape[0]
    acts = [_dense_action(L, nup, ndn, p)[1] for p in perms]
    P = sum(c * A for c, A in zip(chi, acts)) / len(perms)
    basis, H = S.sym_hamiltonian(t, U, nup, ndn, perms, chi)
    B = P[:, basis]
    if len(basis):
        B = B / np.linalg.norm(B, axis=0)
    Hd = dense.dense_h(t, U, nup, ndn)
    return basis, H, B, Hd, P


def _plaquette(tp=0.3, U=4.0, mu=2.0):
    t = synth.nn_hopping(2, 2)
    t[0, 3] = t[3, 0] = t[1, 2] = t[2, 1] = tp
    return t - mu * np.eye(4), np.full(4, U)


def _ladder():
    t = synth.nn_hopping(3, 2)
    t[0, 4] = t[4, 0] = t[1, 3] = t[3, 1] = t[1, 5] = t[5, 1] = t[2, 4] = t[4, 2] = 0.2
    U = np.array([5.0, 3.0, 5.0, 5.0, 3.0, 5.0])
    return t - np.diag([2.5, 1.5, 2.5, 2.5, 1.5, 2.5]), U


def _chain(L=6):
    t = np.zeros((L, L))
    for a in range(L - 1):
        t[a, a + 1] = t[a + 1, a] = -1.0 + 0.1 * min(a, L - 2 - a)
    return t - 2.0 * np.eye(L), np.full(L, 4.0)


def _chain7():
    t = np.zeros((7, 7))
    for a in range(6):
        t[a, a + 1] = t[a + 1, a] = -1.0 - 0.05 * min(a, 5 - a)
    t[0, 6] = t[6, 0] = 0.3                  # a long bond the mirror maps to itself
    return t - np.diag([1.0, 2.0, 3.0, 4.0, 3.0, 2.0, 1.0]), np.array([3.0, 4.0, 5.0, 6.0, 5.0, 4.0, 3.0])


CASES = [
    ("plaquette", _plaquette, synth.c2v_rectangle(2, 2), synth.C2V_IRREPS, [(2, 2), (2, 1), (1, 0), (4, 4)]),
    ("chain7_odd", _chain7, synth.c2_chain(7), synth.C2_IRREPS, [(3, 4), (4, 2), (7, 0)]),
    ("trivial_group", _chain7, [list(range(7))], {"A": (1,)}, [(3, 3)]),
    ("ladder3x2", _ladder, synth.c2v_rectangle(3, 2), synth.C2V_IRREPS, [(3, 3), (2, 3), (0, 0)]),
    ("chain6", _chain, synth.c2_chain(6), synth.C2_IRREPS, [(3, 3), (3, 2)]),
]


@pytest.mark.parametrize("name,make,perms,irreps,sectors", CASES, ids=[c[0] for c in CASES])
def test_projector_route(name, make, perms, irreps, sectors):
    t, U = make()
    for nup, ndn in sectors:
        spectra, total = [], 0
        for irrep, chi in irreps.items():
            basis, H, B, Hd, P = _projector_route(t, U, nup, ndn, perms, chi)
            n = len(basis)
            total += n
            # the projector's rank is the irrep's dimension
            assert n == int(round(np.trace(P)))
            if n == 0:
                continue
            assert np.abs(B.T @ B - np.eye(n)).max() <= 1e-12
            assert np.abs(B.T @ Hd @ B - H.toarray()).max() <= 1e-12
            spectra.append(np.linalg.eigvalsh(H.toarray()))
        assert total == Hd.shape[0]
        full = np.linalg.eigvalsh(Hd)
        assert np.abs(np.sort(np.concatenate(spectra)) - full).max() <= 1e-10


def test_rejects_broken_symmetry():
    t, U = _plaquette()
    t2 = t.copy()
    t2[0, 1] = t2[1, 0] = -1.1
    with pytest.raises(AssertionError):
        S.sym_hamiltonian(t2, U, 2, 2, synth.c2v_rectangle(2, 2), synth.C2V_IRREPS["A1"])
    with pytest.raises(AssertionError):
        S.sym_hamiltonian(t, U, 2, 2, synth.c2v_rectangle(2, 2), (1, -1, -1, -1))


def test_column_routine_matches_whole_matrix():
    """The one-column routine (plain loops, combinatorial labels) against the
    vectorised matrix, every column of the ladder's irreps and of a 3x4 irrep's
    first and last 40 columns."""
    from math import comb
    t, U = _ladder()
    cases = [(t, U, 3, 3, synth.c2v_rectangle(3, 2), chi, None) for chi in synth.C2V_IRREPS.values()]
    m3 = synth.nn_hopping(4, 3)
    m3[0, 5] = m3[5, 0] = m3[1, 4] = m3[4, 1] = 0.3     # a t' pair and its mirror images
    m3[2, 7] = m3[7, 2] = m3[3, 6] = m3[6, 3] = 0.3
    m3[4, 9] = m3[9, 4] = m3[5, 8] = m3[8, 5] = 0.3
    m3[6, 11] = m3[11, 6] = m3[7, 10] = m3[10, 7] = 0.3
    cases.append((m3 - 4 * np.eye(12), np.full(12, 8.0), 6, 6, synth.c2v_rectangle(4, 3),
                  synth.C2V_IRREPS["B1"], 40))
    for t_, U_, nup, ndn, perms, chi, edge in cases:
        L = t_.shape[0]
        basis, H = S.sym_hamiltonian(t_, U_, nup, ndn, perms, chi)
        d_up = comb(L, nup)
        Su, Sd = S.strings(L, nup), S.strings(L, ndn)
        Hc = H.tocsc()
        cols = range(len(basis)) if edge is None else list(range(edge)) + list(range(len(basis) - edge, len(basis)))
        for c in cols:
            lab = int(basis[c])
            bu, bd = int(Su[lab % d_up]), int(Sd[lab // d_up])
            assert S.is_kept(bu, bd, perms, chi, d_up)
            col = S.sym_column(t_, U_, bu, bd, perms, chi)
            lo, hi = Hc.indptr[c], Hc.indptr[c + 1]
            want = {int(basis[r]): v for r, v in zip(Hc.indices[lo:hi], Hc.data[lo:hi])}
            assert set(col) == set(want)
            assert max(abs(col[k] - want[k]) for k in want) <= 1e-13


def test_ground_state_3x4_equals_full_sector():
    """The 3x4 cluster with t' = 0.3 (U = 8, mu = 4, (6,6)): the lowest
    eigenvalue of the A1 matrix is the full sector's ground-state energy
    (tests/golden/cluster_3x4.json, converged oracle Lanczos)."""
    import json
    from scipy.sparse.linalg import eigsh
    import synth
    m = synth.cluster_3x4()
    g = json.load(open(os.path.join(os.path.dirname(GOLD), "cluster_3x4.json")))
    _, H = S.sym_hamiltonian(m.t, m.U, 6, 6, synth.c2v_rectangle(4, 3), synth.C2V_IRREPS["A1"])
    e0 = eigsh(H, k=1, which="SA", tol=1e-14)[0][0]
    assert abs(e0 - g["e0"]) <= 1e-10 * abs(g["e0"])
