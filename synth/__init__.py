"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only builds inputs: hopping matrices t_ij (with the chemical
potential and bath energies on the diagonal), on-site interactions U_i,
sectors (N_up, N_dn), frequency grids, momentum grids, CPT lattice
descriptions and point-group tables.  It holds none of the method's
arithmetic.

Conventions:
  * a model is (t, U): t is L x L real symmetric, t_ii = eps_i - mu; U has
    one entry per orbital and is 0 on bath orbitals (eq. (Hubbard) and
    eq. (cdmft1) of the paper);
  * "t = -1" means the matrix element t_ij = -1 on every nearest-neighbour
    bond, "t' = 0.3" means t_ij = +0.3 on both diagonals of every plaquette;
  * rectangular clusters number their sites x + nx*y;
  * a point group is a list of orbital permutations (identity first) and an
    irrep a tuple of characters, one per element;
  * cluster orbitals come first and bath orbitals after them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Model:
    name: str
    t: np.ndarray
    U: np.ndarray
    nup: int
    ndn: int
    meta: dict = field(default_factory=dict)

    @property
    def L(self) -> int:
        return int(self.t.shape[0])


def rect_cluster(nx: int, ny: int, t: float = -1.0, tp: float = 0.0, U: float = 8.0,
                 mu: float = 4.0, nup: int | None = None, ndn: int | None = None,
                 name: str | None = None) -> Model:
    """Open-boundary nx x ny cluster, sites x + nx*y."""
    L = nx * ny
    T = np.zeros((L, L))
    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            if x + 1 < nx:
                T[i, i + 1] = T[i + 1, i] = t
            if y + 1 < ny:
                T[i, i + nx] = T[i + nx, i] = t
            if tp != 0.0 and x + 1 < nx and y + 1 < ny:
                a, b = i, i + 1 + nx
                c, d = i + 1, i + nx
                T[a, b] = T[b, a] = tp
                T[c, d] = T[d, c] = tp
    for i in range(L):
        T[i, i] = -mu
    nup = L // 2 if nup is None else nup
    ndn = L // 2 if ndn is None else ndn
    return Model(name or f"{nx}x{ny}", T, np.full(L, float(U)), nup, ndn,
                 dict(nx=nx, ny=ny, t=t, tp=tp, U=U, mu=mu))


def chain(L: int, t: float = -1.0, U: float = 4.0, mu: float = 2.0,
          nup: int | None = None, ndn: int | None = None) -> Model:
    """Open chain of L sites."""
    m = rect_cluster(L, 1, t=t, U=U, mu=mu, nup=nup, ndn=ndn, name=f"chain{L}")
    return m


def two_site(t: float = -1.0, U: float = 4.0, mu: float = 0.0) -> Model:
    return rect_cluster(2, 1, t=t, U=U, mu=mu, nup=1, ndn=1, name="dimer")


def plaquette_2x2(U: float = 8.0, mu: float = 4.0) -> Model:
    """2x2 plaquette, t = -1, U = 8, mu = 4, sector (2, 2), dim 36."""
    return rect_cluster(2, 2, t=-1.0, U=U, mu=mu, nup=2, ndn=2, name="2x2")


def cluster_3x4(U: float = 8.0, mu: float = 4.0, tp: float = 0.3) -> Model:
    """3 rows x 4 columns, t = -1, t' = 0.3, U = 8, mu = 4, sector (6, 6)."""
    return rect_cluster(4, 3, t=-1.0, tp=tp, U=U, mu=mu, nup=6, ndn=6, name="3x4")


def cluster_4x4(U: float = 8.0) -> Model:
    """4x4, t = -1, mu = U/2, sector (8, 8), dim 165,636,900."""
    return rect_cluster(4, 4, t=-1.0, U=U, mu=U / 2, nup=8, ndn=8, name=f"4x4_U{U:g}")


def random_model(seed: int, L: int, nup: int, ndn: int, density: float = 0.6,
                 uniform_U: bool = False) -> Model:
    """A random real symmetric t with random on-site U (test input)."""
    rng = np.random.default_rng(seed)
    T = rng.normal(0.0, 1.0, (L, L))
    mask = rng.random((L, L)) < density
    T = np.where(mask, T, 0.0)
    T = np.triu(T, 1)
    T = T + T.T
    T[np.diag_indices(L)] = rng.uniform(-2.0, 2.0, L)
    U = np.full(L, rng.uniform(1, 8)) if uniform_U else rng.uniform(0.0, 8.0, L)
    return Model(f"rand{seed}_L{L}", T, U, nup, ndn, dict(seed=seed))


def omega_grid(n: int = 64, lo: float = -10.0, hi: float = 10.0, eta: float = 0.1) -> np.ndarray:
    """z_k = omega_k + i eta, omega_k = lo + (hi - lo) k / (n - 1)."""
    w = lo + (hi - lo) * np.arange(n) / (n - 1)
    return w + 1j * eta


def k_grid_2d(n: int = 16) -> np.ndarray:
    """k = (m/n, l/n, 0) in units of 2 pi, m, l = 0..n-1; row-major in (m, l)."""
    m, l = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.stack([m.ravel() / n, l.ravel() / n, np.zeros(n * n)], axis=1)


def cpt_square_lattice_2x2(t: float = -1.0):
    """Tiling of the square lattice by 2x2 plaquettes: site positions R_i
    (sites x + 2y), super-lattice vectors E = (2,0,0), (0,2,0), (0,0,1) and
    the inter-cluster nearest-neighbour bonds (i, j, shift, t): site i of the
    cluster at the origin to site j of the cluster at shift . E."""
    R = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], dtype=np.int32)
    E = np.array([[2, 0, 0], [0, 2, 0], [0, 0, 1]], dtype=np.int32)
    bonds = [(1, 0, (1, 0, 0), t), (3, 2, (1, 0, 0), t),
             (2, 0, (0, 1, 0), t), (3, 1, (0, 1, 0), t)]
    return R, E, bonds


def chain_lattice_2(t: float = -1.0):
    """1D lattice tiled by 2-site clusters (E = 2): positions and the single
    inter-cluster bond."""
    R = np.array([[0, 0, 0], [1, 0, 0]], dtype=np.int32)
    E = np.array([[2, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.int32)
    bonds = [(1, 0, (1, 0, 0), t)]
    return R, E, bonds


def impurity_model(rng: np.random.Generator, n_bath: int) -> Model:
    """2x2 plaquette (t = -1) plus n_bath bath orbitals.  Bath orbital 4 + a
    couples to cluster site a mod 4 with theta ~ U(0.2, 1) and has energy
    eps ~ U(-3, 3); U ~ U(2, 10) on the four cluster sites, mu = U/2 there;
    N_up, N_dn each drawn from {floor(n/2), ceil(n/2)}."""
    n = 4 + n_bath
    T = np.zeros((n, n))
    for (i, j) in [(0, 1), (2, 3), (0, 2), (1, 3)]:
        T[i, j] = T[j, i] = -1.0
    Uval = rng.uniform(2.0, 10.0)
    for i in range(4):
        T[i, i] = -Uval / 2
    for a in range(n_bath):
        th = rng.uniform(0.2, 1.0)
        eps = rng.uniform(-3.0, 3.0)
        T[4 + a, a % 4] = T[a % 4, 4 + a] = th
        T[4 + a, 4 + a] = eps
    U = np.zeros(n)
    U[:4] = Uval
    lo, hi = n // 2, (n + 1) // 2
    nup = int(rng.choice([lo, hi]))
    ndn = int(rng.choice([lo, hi]))
    return Model(f"imp{n}", T, U, nup, ndn, dict(n_bath=n_bath, U=Uval))


def batched_solves(seed: int = 18643, count: int = 256) -> list[Model]:
    """The batched workload: ``count`` impurity models with 2..10 bath orbitals."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nb = int(rng.integers(2, 11))
        out.append(impurity_model(rng, nb))
    return out


def serving_model(rng: np.random.Generator) -> Model:
    """A serving request: n ~ U{4..14} orbitals, open chain or (n even, coin
    flip) a 2 x n/2 ladder, t_ij ~ N(-1, 0.2) per bond, U ~ U(2, 10) on all
    orbitals, mu = U/2, sector (ceil(n/2), floor(n/2))."""
    n = int(rng.integers(4, 15))
    ladder = (n % 2 == 0) and bool(rng.integers(0, 2))
    T = np.zeros((n, n))
    if ladder:
        w = n // 2
        bonds = [(x + w * y, x + 1 + w * y) for y in range(2) for x in range(w - 1)]
        bonds += [(x, x + w) for x in range(w)]
    else:
        bonds = [(i, i + 1) for i in range(n - 1)]
    for (i, j) in bonds:
        T[i, j] = T[j, i] = rng.normal(-1.0, 0.2)
    Uval = rng.uniform(2.0, 10.0)
    T[np.diag_indices(n)] = -Uval / 2
    return Model(f"srv{n}{'L' if ladder else 'C'}", T, np.full(n, Uval), (n + 1) // 2, n // 2,
                 dict(ladder=ladder, U=Uval))


def serving_requests(seed: int = 2305, count: int = 100) -> list[Model]:
    rng = np.random.default_rng(seed)
    return [serving_model(rng) for _ in range(count)]


@dataclass
class CdmftSetup:
    """A CDMFT problem: a cluster of L sites with n_bath bath orbitals, the
    lattice it tiles, the bath parameters and the distance-function grid.

    The bath is described by linear maps from the variational parameters p:
    eps = A_eps @ p (n_bath) and theta = (A_theta @ p).reshape(L, n_bath),
    theta[mu, alpha] being the cluster-bath hopping (eq. (cdmft1) of the
    paper)."""
    name: str
    tc: np.ndarray          # L x L cluster hopping (without mu)
    mu: float
    U: float                # on every cluster site
    nup: int                # sector of the impurity (cluster + bath)
    ndn: int
    A_eps: np.ndarray       # n_bath x n_par
    A_theta: np.ndarray     # (L * n_bath) x n_par
    p0: np.ndarray          # initial variational parameters
    E: np.ndarray           # super-lattice vectors (rows)
    bonds: list             # inter-cluster bonds (i, j, shift, t)
    beta: float             # fictitious inverse temperature of the grid
    wc: float               # frequency cutoff of the distance function

    @property
    def L(self) -> int:
        return int(self.tc.shape[0])

    @property
    def n_bath(self) -> int:
        return int(self.A_eps.shape[0])


def cdmft_chain_4_4b(U: float = 4.0, mu: float = 2.0, t: float = -1.0) -> CdmftSetup:
    """The one-dimensional Hubbard model on 4-site clusters with 4 bath
    orbitals (the paper's CDMFT example, its bath figure (a)): cluster sites
    0..3 (open chain, t on each bond, period 4 along the chain); bath orbitals
    0 and 1 have energy eb1 and couple to sites 0 and 3 with -tb1, bath
    orbitals 2 and 3 have energy eb2 and couple to sites 0 and 3 with -tb2.
    Parameters p = (eb1, eb2, tb1, tb2), starting at (1, -1, 1, 1); sector
    N = 8, S_z = 0; beta = 50, cutoff 2."""
    L, nb = 4, 4
    tc = np.zeros((L, L))
    for i in range(L - 1):
        tc[i, i + 1] = tc[i + 1, i] = t
    A_eps = np.zeros((nb, 4))
    A_eps[0, 0] = A_eps[1, 0] = 1.0
    A_eps[2, 1] = A_eps[3, 1] = 1.0
    A_theta = np.zeros((L * nb, 4))
    A_theta[0 * nb + 0, 2] = -1.0
    A_theta[3 * nb + 1, 2] = -1.0
    A_theta[0 * nb + 2, 3] = -1.0
    A_theta[3 * nb + 3, 3] = -1.0
    E = np.array([[4, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.int32)
    bonds = [(3, 0, (1, 0, 0), t)]
    return CdmftSetup("chain4_4b", tc, mu, U, 4, 4, A_eps, A_theta,
                      np.array([1.0, -1.0, 1.0, 1.0]), E, bonds, 50.0, 2.0)


def matsubara_grid(beta: float, wc: float) -> np.ndarray:
    """i omega_n, omega_n = (2n + 1) pi / beta, n = 0, 1, ... up to omega_n <= wc."""
    n = np.arange(int(np.floor((wc * beta / np.pi - 1.0) / 2.0)) + 1)
    return 1j * (2 * n + 1) * np.pi / beta


def k_grid_1d(nk: int) -> np.ndarray:
    """nk points of the reduced zone of a 1D super-lattice along x, in units
    of 2 pi divided by the period: k = (m / nk, 0, 0), m = 0..nk-1, to be
    used with super-lattice shifts s as the phase exp(2 pi i k . s)."""
    return np.stack([np.arange(nk) / nk, np.zeros(nk), np.zeros(nk)], axis=1)


@dataclass
class VcaSetup:
    """A VCA problem: the cluster reference system (t_ref with -mu on its
    diagonal, U per site, sector), the k-independent part of V (the lattice's
    intra-cluster hopping minus the reference's) and the inter-cluster bonds
    (shift in super-lattice units, phase exp(2 pi i k . s))."""
    name: str
    t_ref: np.ndarray
    U: np.ndarray
    nup: int
    ndn: int
    dt: np.ndarray
    bonds: list
    h0: np.ndarray          # the lattice's intra-cluster one-body matrix (with -mu)


def vca_plaquette(U: float = 8.0, mu: float = 4.0, tp: float = -1.0, t: float = -1.0) -> VcaSetup:
    """The square lattice tiled by 2x2 plaquettes (sites x + 2y, super-lattice
    2 x 2), nearest-neighbour t; the reference plaquette has hopping tp on its
    four bonds (the variational parameter); half filling (2, 2)."""
    def plaq(tt):
        m = np.zeros((4, 4))
        for a, b in ((0, 1), (2, 3), (0, 2), (1, 3)):
            m[a, b] = m[b, a] = tt
        return m
    h0 = plaq(t) - mu * np.eye(4)
    t_ref = plaq(tp) - mu * np.eye(4)
    bonds = [(1, 0, (1, 0, 0), t), (3, 2, (1, 0, 0), t), (2, 0, (0, 1, 0), t), (3, 1, (0, 1, 0), t)]
    return VcaSetup(f"plaq_tp{tp}", t_ref, np.full(4, float(U)), 2, 2, h0 - t_ref, bonds, h0)


def vca_chain4(U: float = 4.0, mu: float = 2.0, tp: float = -1.0, t: float = -1.0) -> VcaSetup:
    """The 1D chain tiled by open 4-site clusters (period 4), nearest-neighbour
    t; the reference cluster has hopping tp on its three bonds; half filling."""
    def ch(tt):
        m = np.zeros((4, 4))
        for i in range(3):
            m[i, i + 1] = m[i + 1, i] = tt
        return m
    h0 = ch(t) - mu * np.eye(4)
    t_ref = ch(tp) - mu * np.eye(4)
    return VcaSetup(f"chain4_tp{tp}", t_ref, np.full(4, float(U)), 2, 2, h0 - t_ref,
                    [(3, 0, (1, 0, 0), t)], h0)


# ---------------------------------------------------------------- point groups
# Input data of symmetry-adapted sectors: orbital permutations (the same for
# both spins) and the characters of one-dimensional irreps.

def c2v_rectangle(nx: int, ny: int):
    """The C2v group of an nx x ny rectangle of sites a = x + nx y: the
    identity, the rotation by pi, the mirror y -> ny-1-y and the mirror
    x -> nx-1-x, in that order."""
    def site(x, y):
        return x + nx * y
    e, c2, my, mx = [], [], [], []
    for a in range(nx * ny):
        x, y = a % nx, a // nx
        e.append(a)
        c2.append(site(nx - 1 - x, ny - 1 - y))
        my.append(site(x, ny - 1 - y))
        mx.append(site(nx - 1 - x, y))
    return [e, c2, my, mx]


# characters over (identity, C2, mirror y -> -y, mirror x -> -x)
C2V_IRREPS = {"A1": (1, 1, 1, 1), "A2": (1, 1, -1, -1), "B1": (1, -1, 1, -1), "B2": (1, -1, -1, 1)}


def c2_chain(L: int):
    """The left-right mirror of an L-site chain: identity and a -> L-1-a."""
    return [list(range(L)), [L - 1 - a for a in range(L)]]


C2_IRREPS = {"A": (1, 1), "B": (1, -1)}


def nn_hopping(nx: int, ny: int, t: float = -1.0) -> np.ndarray:
    """Nearest-neighbour hopping matrix of the nx x ny rectangle (a = x + nx y)."""
    L = nx * ny
    h = np.zeros((L, L))
    for a in range(L):
        x, y = a % nx, a // nx
        if x + 1 < nx:
            h[a, a + 1] = h[a + 1, a] = t
        if y + 1 < ny:
            h[a, a + nx] = h[a + nx, a] = t
    return h
