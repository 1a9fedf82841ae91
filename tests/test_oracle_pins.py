"""Pins of the CPU oracle against facts that do not come from the oracle
itself: values and examples printed in the paper, closed forms, limits,
symmetries, sum rules and brute force on tiny inputs.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import cf, dense
from tests.conftest import read_golden

Z64 = synth.omega_grid()


# ---------------------------------------------------------------- basis

def test_dimensions_from_paper():
    rows = {r[0]: [int(x) for x in r[1:]] for r in read_golden("dimensions.txt")}
    assert sum(rows["c2v_3x4"]) == oracle.binom(12, 6) ** 2 == 853776
    assert 2 * rows["chain14_symmetric_half"][0] == oracle.binom(14, 7) ** 2
    assert oracle.binom(16, 8) ** 2 == 165636900
    for L in range(1, 17):
        for N in range(0, L + 1):
            assert oracle.binom(L, N) == math.comb(L, N)


@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 11, 13])
def test_enumeration_and_rank_brute_force(L):
    for N in range(0, L + 1):
        brute = [x for x in range(1 << L) if bin(x).count("1") == N]
        st = oracle.sector_states(L, N)
        assert st.tolist() == brute
        for i, b in enumerate(brute):
            assert oracle.rank(b) == i


def test_rank_16_sites_half_filling():
    st = oracle.sector_states(16, 8)
    assert st.shape[0] == 12870
    assert np.all(np.diff(st.astype(np.int64)) > 0)
    for i in range(0, 12870, 97):
        assert oracle.rank(int(st[i])) == i
    assert oracle.rank(int(st[-1])) == 12869


def test_splitmix64_published_outputs():
    # first outputs of the SplitMix64 reference generator seeded with 1234567
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    assert [oracle.splitmix(1234567, i) for i in range(5)] == ref
    x = oracle.start_vector(1, 1000)
    assert np.all(x >= -1.0) and np.all(x < 1.0)
    u = oracle.splitmix(1, 7)
    assert x[7] == 2.0 * (u >> 11) * 2.0 ** -53 - 1.0


# ---------------------------------------------------------------- H.v

def _str_to_int(s):
    # orbital 0 is written leftmost
    return sum(1 << k for k, ch in enumerate(s) if ch == "1")


def test_worked_sign_example():
    g = {r[0]: r[1:] for r in read_golden("sign_example.txt")}
    L = int(g["L"][0])
    a, c = (int(x) for x in g["orbitals"])
    ba, bb = _str_to_int(g["string_a"][0]), _str_to_int(g["string_b"][0])
    N = bin(ba).count("1")
    t = np.zeros((L, L))
    t[a, c] = t[c, a] = 1.0
    U = np.zeros(L)
    d = oracle.binom(L, N)
    ia, ib = oracle.rank(ba), oracle.rank(bb)
    v = np.zeros(d)
    v[ib] = 1.0
    w = oracle.hv(t, U, N, 0, v)
    assert w[ia] == float(g["element_sign"][0])
    # and the dense generic-operator construction agrees
    H = dense.dense_h(t, U, N, 0)
    assert H[ia, ib] == float(g["element_sign"][0])


@pytest.mark.parametrize("seed,L,nup,ndn", [(1, 4, 2, 2), (2, 5, 2, 3), (3, 6, 3, 1),
                                            (4, 6, 0, 3), (5, 7, 3, 4), (6, 3, 3, 2)])
def test_hv_matches_dense_generic_operators(seed, L, nup, ndn):
    m = synth.random_model(seed, L, nup, ndn)
    H = dense.dense_h(m.t, m.U, nup, ndn)
    assert np.allclose(H, H.T, atol=0, rtol=0)
    v = np.random.default_rng(seed).normal(size=H.shape[0])
    w = oracle.hv(m.t, m.U, nup, ndn, v)
    assert np.max(np.abs(w - H @ v)) < 1e-12 * (1 + np.max(np.abs(H @ v)))
    rows = np.arange(0, H.shape[0], 3)
    assert np.max(np.abs(oracle.hv_rows(m.t, m.U, nup, ndn, v, rows) - w[rows])) == 0.0


@pytest.mark.parametrize("seed,L,nup,ndn", [(1, 4, 2, 2), (2, 5, 2, 3), (3, 6, 3, 1),
                                            (5, 7, 3, 4)])
def test_hv_rows_float_input_equals_double_product(seed, L, nup, ndn):
    # the FP32-input row routine reads each float, widens it exactly to
    # double and sums the same terms: bitwise the FP64 product of the widened
    # vector, which is itself pinned against the dense generic-operator H
    m = synth.random_model(seed, L, nup, ndn)
    d = oracle.binom(L, nup) * oracle.binom(L, ndn)
    v32 = np.random.default_rng(seed).normal(size=d).astype(np.float32)
    w = oracle.hv(m.t, m.U, nup, ndn, v32.astype(np.float64))
    rows = np.arange(d, dtype=np.int64)
    w32 = oracle.hv_rows(m.t, m.U, nup, ndn, v32, rows)
    assert np.array_equal(w32, w)
    H = dense.dense_h(m.t, m.U, nup, ndn)
    assert np.max(np.abs(w32 - H @ v32.astype(np.float64))) < 1e-12 * (1 + np.max(np.abs(w)))


@pytest.mark.parametrize("seed,L,nup,ndn", [(1, 4, 2, 2), (2, 5, 2, 3), (3, 6, 3, 1),
                                            (5, 7, 3, 4), (7, 6, 3, 3)])
def test_hv_abs_bound_is_sum_of_term_magnitudes(seed, L, nup, ndn):
    # the bound is sum over the terms of H of |term| |v_j|: off the diagonal
    # one hop links two states, so it is |H_ij| |v_j| from the dense
    # generic-operator H; on the diagonal it is the one-body and interaction
    # terms taken with their absolute values, which is the dense H of the model
    # with |t_kk| on the diagonal, no hopping and |U_k|
    m = synth.random_model(seed, L, nup, ndn)
    H = dense.dense_h(m.t, m.U, nup, ndn)
    tdiag = np.diag(np.abs(np.diag(m.t)))
    Dabs = np.diag(dense.dense_h(tdiag, np.abs(m.U), nup, ndn))
    Hoff = np.abs(H - np.diag(np.diag(H)))
    v = np.random.default_rng(seed + 100).normal(size=H.shape[0])
    want = Hoff @ np.abs(v) + Dabs * np.abs(v)
    got = oracle.hv_abs_bound(m.t, m.U, nup, ndn, v)
    assert np.max(np.abs(got - want) / want) < 1e-13
    # it bounds |H| |v| row by row, with equality when the diagonal terms of a
    # row share one sign (no t_kk: only U_k >= 0 terms)
    assert np.all(got >= (np.abs(H) @ np.abs(v)) * (1 - 1e-13))
    t0 = m.t - np.diag(np.diag(m.t))
    H0 = dense.dense_h(t0, np.abs(m.U), nup, ndn)
    got0 = oracle.hv_abs_bound(t0, np.abs(m.U), nup, ndn, v)
    want0 = np.abs(H0) @ np.abs(v)
    assert np.max(np.abs(got0 - want0) / want0) < 1e-13
    # row selection gives the same values
    rows = np.arange(0, H.shape[0], 2, dtype=np.int64)
    assert np.array_equal(oracle.hv_abs_bound(m.t, m.U, nup, ndn, v, rows=rows), got[rows])


def test_hv_no_double_occupancy_interaction_only():
    # t = 0: H is diagonal with sum_k t_kk n_k + U * (number of doubly occupied)
    L = 6
    t = np.diag(np.linspace(-1, 1, L))
    U = np.full(L, 3.0)
    v = np.ones(oracle.binom(L, 3) * oracle.binom(L, 2))
    w = oracle.hv(t, U, 3, 2, v)
    su, sd = oracle.sector_states(L, 3), oracle.sector_states(L, 2)
    for i in range(v.shape[0]):
        bu, bd = int(su[i % su.shape[0]]), int(sd[i // su.shape[0]])
        e = sum(t[k, k] * (((bu >> k) & 1) + ((bd >> k) & 1)) for k in range(L))
        e += 3.0 * bin(bu & bd).count("1")
        assert abs(w[i] - e) < 1e-14


# ---------------------------------------------------------------- tridiagonal

def test_tridiag_against_numpy():
    rng = np.random.default_rng(7)
    for n in (1, 2, 5, 40, 200):
        a = rng.normal(size=n)
        b = np.abs(rng.normal(size=n - 1)) + 0.01
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        ev = np.linalg.eigvalsh(T)
        assert abs(oracle.tridiag_eig(a, b, 0) - ev[0]) < 1e-12 * max(1, abs(ev[0]))
        if n > 1:
            assert abs(oracle.tridiag_eig(a, b, 1) - ev[1]) < 1e-12 * max(1, abs(ev[1]))
        x = oracle.tridiag_vec(a, b, ev[0])
        assert np.linalg.norm(T @ x - ev[0] * x) < 1e-10


# ---------------------------------------------------------------- ground state

def test_two_site_closed_form():
    for U in (0.0, 2.0, 8.0):
        for mu in (0.0, 1.5):
            m = synth.rect_cluster(2, 1, t=-1.0, U=U, mu=mu, nup=1, ndn=1)
            r = oracle.lanczos_gs(m.t, m.U, 1, 1)
            exact = (U - math.sqrt(U * U + 16.0)) / 2 - 2 * mu
            assert abs(r["e0"] - exact) < 1e-12 * max(1, abs(exact))


@pytest.mark.parametrize("name", ["2x2", "rand"])
def test_ground_state_matches_dense(name):
    if name == "2x2":
        m = synth.plaquette_2x2()
    else:
        m = synth.random_model(11, 6, 3, 2)
    e0d, psid, w = dense.ground_state(m.t, m.U, m.nup, m.ndn)
    r = oracle.lanczos_gs(m.t, m.U, m.nup, m.ndn, want_vector=True)
    assert r["converged"]
    assert abs(r["e0"] - e0d) < 1e-12 * abs(e0d)
    assert abs(np.linalg.norm(r["psi"]) - 1.0) < 1e-13
    assert abs(abs(np.dot(r["psi"], psid)) - 1.0) < 1e-10
    assert r["true_residual"] < 1e-8


def test_lanczos_ritz_values_decrease_and_bound():
    m = synth.rect_cluster(3, 2, U=4.0, mu=2.0)
    e0d = dense.ground_state(m.t, m.U, 3, 3)[0]
    r = oracle.lanczos_gs(m.t, m.U, 3, 3, fixed_steps=60)
    th = [oracle.tridiag_eig(r["alpha"][:k], r["beta"][:k - 1], 0) for k in range(1, r["n_iter"] + 1)]
    assert all(th[i + 1] <= th[i] + 1e-12 for i in range(len(th) - 1))
    assert all(x >= e0d - 1e-10 for x in th)
    assert abs(th[-1] - e0d) < 1e-11 * abs(e0d)


def test_u0_single_particle_limit():
    m = synth.random_model(21, 7, 3, 2)
    U0 = np.zeros(7)
    eps = np.linalg.eigvalsh(m.t)
    r = oracle.lanczos_gs(m.t, U0, 3, 2, want_vector=True)
    assert abs(r["e0"] - (eps[:3].sum() + eps[:2].sum())) < 1e-11
    ch = oracle.green_cf(m.t, U0, 3, 2, r["psi"], list(range(7)))
    G = cf.green_matrix(ch, 7, Z64, r["e0"])
    for iz, z in enumerate(Z64):
        G0 = np.linalg.inv(z * np.eye(7) - m.t)
        assert np.max(np.abs(G[iz] - G0)) < 1e-8


def test_atomic_limit():
    # t = 0, mu = U/2, half filling: E0 = -mu N, and tr G is state independent
    U = 6.0
    L = 4
    t = np.diag(np.full(L, -U / 2))
    Uv = np.full(L, U)
    r = oracle.lanczos_gs(t, Uv, 2, 2, want_vector=True)
    assert abs(r["e0"] + U / 2 * 4) < 1e-12
    assert r["breakdown"]
    ch = oracle.green_cf(t, Uv, 2, 2, r["psi"], list(range(L)))
    G = cf.green_matrix(ch, L, Z64, r["e0"])
    tr = np.trace(G, axis1=1, axis2=2)
    expect = 2 / (Z64 + U / 2) + (L - 2) / (Z64 - U / 2)
    assert np.max(np.abs(tr - expect)) < 1e-12


def test_particle_hole_symmetry_2x2():
    m = synth.plaquette_2x2()
    r = oracle.lanczos_gs(m.t, m.U, 2, 2, want_vector=True)
    ch = oracle.green_cf(m.t, m.U, 2, 2, r["psi"], [0, 1, 2, 3])
    for i in range(4):
        assert abs(ch[(i, i, 0)][0] - 0.5) < 1e-12
        assert abs(ch[(i, i, 1)][0] - 0.5) < 1e-12
    G = cf.green_matrix(ch, 4, Z64, r["e0"])
    Gm = G[::-1]          # the grid is symmetric under omega -> -omega
    for i in range(4):
        assert np.max(np.abs(G[:, i, i] + np.conj(Gm[:, i, i]))) < 1e-10
    # E0(Nup, Ndn) = E0(L - Nup, L - Ndn) at mu = U/2 on a bipartite cluster
    a = oracle.lanczos_gs(m.t, m.U, 1, 2)["e0"]
    b = oracle.lanczos_gs(m.t, m.U, 3, 2)["e0"]
    assert abs(a - b) < 1e-11


def test_sum_rules_and_positivity():
    m = synth.random_model(31, 6, 3, 2)
    r = oracle.lanczos_gs(m.t, m.U, 3, 2, want_vector=True)
    psi = r["psi"]
    e0 = r["e0"]
    L = 6
    ch = oracle.green_cf(m.t, m.U, 3, 2, psi, list(range(L)))
    su, sd = oracle.sector_states(L, 3), oracle.sector_states(L, 2)
    du = su.shape[0]
    p2 = psi ** 2
    idx = np.arange(psi.shape[0])
    bu, bd = su[idx % du].astype(np.int64), sd[idx // du].astype(np.int64)
    for mu in range(L):
        b0e, ae, _ = ch[(mu, mu, 0)]
        b0h, ah, _ = ch[(mu, mu, 1)]
        assert abs(b0e + b0h - 1.0) < 1e-12
        n_up = np.sum(p2 * ((bu >> mu) & 1))
        n_dn = np.sum(p2 * ((bd >> mu) & 1))
        assert abs(b0h - n_up) < 1e-12
        first = b0e * (ae[0] - e0) + b0h * (e0 - ah[0])
        assert abs(first - (m.t[mu, mu] + m.U[mu] * n_dn)) < 1e-9
    G = cf.green_matrix(ch, L, Z64, e0)
    for mu in range(L):
        assert np.all(-G[:, mu, mu].imag > 0)
    # z G(z) -> 1 at large |z|
    zb = np.array([1e6 + 0.1j])
    Gb = cf.green_matrix(ch, L, zb, e0)
    assert np.max(np.abs(zb[0] * Gb[0] - np.eye(L))) < 1e-5
    # symmetry of the real-H Green function and conjugation
    assert np.max(np.abs(G - np.transpose(G, (0, 2, 1)))) == 0.0
    Gc = cf.green_matrix(ch, L, np.conj(Z64), e0)
    assert np.max(np.abs(Gc - np.conj(G))) < 1e-13


@pytest.mark.parametrize("seed,L,nup,ndn", [(42, 4, 2, 2), (42, 5, 2, 3), (43, 6, 3, 3),
                                            (44, 5, 1, 1), (45, 6, 6, 2)])
def test_cf_green_equals_lehmann(seed, L, nup, ndn):
    m = synth.random_model(seed, L, nup, ndn)
    e0d, psid, w = dense.ground_state(m.t, m.U, nup, ndn)
    # every case here has a non-degenerate ground state (G would otherwise
    # depend on which state of the manifold Lanczos returns)
    assert w.shape[0] == 1 or w[1] - w[0] > 1e-3, "degenerate ground state"
    r = oracle.lanczos_gs(m.t, m.U, nup, ndn, want_vector=True)
    orbs = list(range(L))
    # a chain well beyond the sector dimension exhausts its Krylov space, and
    # once the copies that loss of orthogonality creates have settled the
    # continued fraction is the Lehmann sum up to rounding
    steps = 3 * max(oracle.binom(L, nup + 1), oracle.binom(L, nup - 1)) * oracle.binom(L, ndn) + 20
    ch = oracle.green_cf(m.t, m.U, nup, ndn, r["psi"], orbs, max_steps=steps)
    G = cf.green_matrix(ch, L, Z64, r["e0"])
    Gd = dense.lehmann_green(m.t, m.U, nup, ndn, orbs, Z64)
    assert np.max(np.abs(G - Gd)) < 1e-8


def test_spin_symmetry_up_equals_down():
    # with N_up = N_dn and spin-independent t, the up and down Green functions
    # coincide; the down one is the up one of the spin-swapped problem, which
    # for N_up = N_dn is the same problem: check via dense operators
    m = synth.plaquette_2x2()
    e0, psi, _ = dense.ground_state(m.t, m.U, 2, 2)
    L = 4
    z = Z64[:5]
    Gu = dense.lehmann_green(m.t, m.U, 2, 2, [0, 1, 2, 3], z, psi=psi, e0=e0)
    He = dense.dense_h(m.t, m.U, 2, 3)
    we, ve = np.linalg.eigh(He)
    q = np.array([ve.T @ (dense.op_matrix(L, 2, 2, L + k, True) @ psi) for k in range(4)])
    Hh = dense.dense_h(m.t, m.U, 2, 1)
    wh, vh = np.linalg.eigh(Hh)
    p = np.array([vh.T @ (dense.op_matrix(L, 2, 2, L + k, False) @ psi) for k in range(4)])
    Gd = np.array([(q / (zz - (we - e0))) @ q.T + (p / (zz + (wh - e0))) @ p.T for zz in z])
    assert np.max(np.abs(Gu - Gd)) < 1e-12


# ---------------------------------------------------------------- CPT

def test_fourier_convention_L2_example():
    rows = read_golden("fourier_L2.txt")
    R, E, bonds = synth.chain_lattice_2(t=-1.0)      # paper's t = 1
    tc = np.array([[0.0, -1.0], [-1.0, 0.0]])
    for k in (0.0, 0.1, 0.25, 0.37):
        full = tc + cf.v_of_k(2, bonds, E, (k, 0, 0))
        kk = 2 * np.pi * k
        for r in rows:
            i, j = int(r[0]), int(r[1])
            c0, cm, cp = (float(x) for x in r[2:])
            expect = -1.0 * (c0 + cm * np.exp(-2j * kk) + cp * np.exp(2j * kk))
            assert abs(full[i, j] - expect) < 1e-14


def test_cpt_exact_at_u0():
    m = synth.rect_cluster(2, 2, U=0.0, mu=0.7, nup=2, ndn=2)
    r = oracle.lanczos_gs(m.t, m.U, 2, 2, want_vector=True)
    ch = oracle.green_cf(m.t, m.U, 2, 2, r["psi"], [0, 1, 2, 3])
    Gc = cf.green_matrix(ch, 4, Z64, r["e0"])
    R, E, bonds = synth.cpt_square_lattice_2x2()
    ks = synth.k_grid_2d(8)
    Gp = cf.cpt_periodized(Gc, R, E, bonds, ks)
    for ik, k in enumerate(ks):
        eps = -2 * (np.cos(2 * np.pi * k[0]) + np.cos(2 * np.pi * k[1])) - 0.7
        assert np.max(np.abs(Gp[ik] - 1.0 / (Z64 - eps))) < 1e-8


def test_cpt_t0_inter_cluster_vanishes():
    # with no inter-cluster hopping CPT returns the periodised cluster G
    m = synth.plaquette_2x2()
    r = oracle.lanczos_gs(m.t, m.U, 2, 2, want_vector=True)
    ch = oracle.green_cf(m.t, m.U, 2, 2, r["psi"], [0, 1, 2, 3])
    Gc = cf.green_matrix(ch, 4, Z64, r["e0"])
    R, E, _ = synth.cpt_square_lattice_2x2()
    ks = synth.k_grid_2d(4)
    Gp = cf.cpt_periodized(Gc, R, E, [], ks)
    for ik, k in enumerate(ks):
        ph = np.exp(-1j * (R @ (2 * np.pi * k)))
        P = np.outer(ph, np.conj(ph))
        ref = np.einsum("ij,zij->z", P, Gc) / 4
        assert np.max(np.abs(Gp[ik] - ref)) < 1e-12
