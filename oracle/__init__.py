"""CPU FP64 oracle for the exact-diagonalisation hot path of the Pyqcm paper
(arXiv 2305.18643, section "Exact diagonalizations" and section "Cluster
perturbation theory").

TEST INFRASTRUCTURE ONLY: only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  It shares no code with the HIP library (``paper_2305_18643_amd``)
and never imports it.

Pieces:
  * ``ora.c`` (built here with gcc into ``liboracle.so``): basis, labels,
    H.v, the Lanczos ground state, the Green-function start vectors and the
    continued-fraction chains, all written as the plain definitions;
  * ``dense.py``: dense Hamiltonians from generic second quantisation and the
    exact Lehmann sum (independent of ``ora.c``);
  * ``cf.py``: continued-fraction evaluation, the off-diagonal combination and
    CPT with the G-scheme periodisation (NumPy, complex128).

Parity status of each function is stated in its docstring; anything without
an independent pin says "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ora.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_f = ctypes.POINTER(ctypes.c_float)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u32 = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = False) -> str:
    """Compile ``ora.c`` with gcc (plain -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        lib.ora_binom.restype = ctypes.c_int64
        lib.ora_binom.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.ora_enumerate.restype = ctypes.c_int64
        lib.ora_enumerate.argtypes = [ctypes.c_int, ctypes.c_int, _u32]
        lib.ora_rank.restype = ctypes.c_int64
        lib.ora_rank.argtypes = [ctypes.c_uint32]
        lib.ora_start_vector.restype = None
        lib.ora_start_vector.argtypes = [ctypes.c_uint64, ctypes.c_int64, _d]
        lib.ora_splitmix.restype = ctypes.c_uint64
        lib.ora_splitmix.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.ora_hv.restype = ctypes.c_int
        lib.ora_hv.argtypes = [ctypes.c_int, _d, _d, ctypes.c_int, ctypes.c_int, _d, _d,
                               ctypes.c_int]
        lib.ora_hv_rows.restype = ctypes.c_int
        lib.ora_hv_rows.argtypes = [ctypes.c_int, _d, _d, ctypes.c_int, ctypes.c_int, _d,
                                    _i64, ctypes.c_int64, _d, ctypes.c_int]
        lib.ora_hv_rows_f32.restype = ctypes.c_int
        lib.ora_hv_rows_f32.argtypes = [ctypes.c_int, _d, _d, ctypes.c_int, ctypes.c_int, _f,
                                        _i64, ctypes.c_int64, _d, ctypes.c_int]
        lib.ora_hv_absbound.restype = ctypes.c_int
        lib.ora_hv_absbound.argtypes = [ctypes.c_int, _d, _d, ctypes.c_int, ctypes.c_int, _d,
                                        _i64, ctypes.c_int64, _d, ctypes.c_int]
        lib.ora_tridiag_eig.restype = ctypes.c_double
        lib.ora_tridiag_eig.argtypes = [ctypes.c_int, _d, _d, ctypes.c_int]
        lib.ora_tridiag_vec.restype = None
        lib.ora_tridiag_vec.argtypes = [ctypes.c_int, _d, _d, ctypes.c_double, _d]
        lib.ora_lanczos_gs.restype = ctypes.c_int
        lib.ora_lanczos_gs.argtypes = [ctypes.c_int, _d, _d, ctypes.c_int, ctypes.c_int, _d,
                                       ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, _d, _d, _d, _d,
                                       _i32, ctypes.c_int]
        lib.ora_apply_cdag_c.restype = ctypes.c_int
        lib.ora_apply_cdag_c.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _d,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, _d]
        lib.ora_cf_chain.restype = ctypes.c_int
        lib.ora_cf_chain.argtypes = [ctypes.c_int, _d, _d, ctypes.c_int, ctypes.c_int, _d,
                                     ctypes.c_int, ctypes.c_double, _d, _d, _d, ctypes.c_int]
        lib.ora_cf_chain_full.restype = ctypes.c_int
        lib.ora_cf_chain_full.argtypes = lib.ora_cf_chain.argtypes
        _lib = lib
    return _lib


def _p(a, typ):
    return a.ctypes.data_as(typ)


def _model_arrays(t, U):
    t = np.ascontiguousarray(t, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    L = t.shape[0]
    assert t.shape == (L, L) and U.shape == (L,)
    return L, t, U


def default_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


# --------------------------------------------------------------------------
# basis (subsection "Coding of the basis states")

def binom(n: int, k: int) -> int:
    """C(n,k), the dimension of one spin factor of a sector."""
    return int(_load().ora_binom(n, k))


def sector_states(L: int, N: int) -> np.ndarray:
    """All L-bit strings with N set bits in ascending order (uint32).
    Pinned by brute force over all 2^L strings."""
    d = binom(L, N)
    out = np.zeros(max(d, 1), dtype=np.uint32)
    n = _load().ora_enumerate(L, N, _p(out, _u32))
    assert n == d
    return out[:d]


def rank(b: int) -> int:
    """Label of string b inside its sector (combinatorial number system).
    Pinned: equals the position in ``sector_states`` for every string."""
    return int(_load().ora_rank(int(b)))


def start_vector(seed: int, n: int) -> np.ndarray:
    """SplitMix64 start vector: entry i = 2*(u_i >> 11)*2^-53 - 1, with u_i the
    output number i of SplitMix64 seeded with ``seed`` (counter form).
    Pinned against the published generator's first outputs."""
    out = np.empty(n, dtype=np.float64)
    _load().ora_start_vector(seed, n, _p(out, _d))
    return out


def splitmix(seed: int, i: int) -> int:
    return int(_load().ora_splitmix(seed, i))


# --------------------------------------------------------------------------
# H.v (eq. (factorized), matrix elements of the same subsection)

def hv(t, U, nup: int, ndn: int, v: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """w = H v on sector (nup, ndn), element by element.
    Pinned against dense matrices built by ``dense.py`` from generic
    second quantisation, and against closed forms."""
    L, t, U = _model_arrays(t, U)
    v = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty_like(v)
    rc = _load().ora_hv(L, _p(t, _d), _p(U, _d), nup, ndn, _p(v, _d), _p(w, _d),
                        nthreads or default_threads())
    assert rc == 0
    return w


def hv_rows(t, U, nup: int, ndn: int, v: np.ndarray, rows, nthreads: int | None = None):
    """(H v)_i for the listed rows only; v may be float64 or float32."""
    L, t, U = _model_arrays(t, U)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.shape[0], dtype=np.float64)
    lib = _load()
    if v.dtype == np.float32:
        v = np.ascontiguousarray(v)
        rc = lib.ora_hv_rows_f32(L, _p(t, _d), _p(U, _d), nup, ndn, _p(v, _f),
                                 _p(rows, _i64), rows.shape[0], _p(out, _d),
                                 nthreads or default_threads())
    else:
        v = np.ascontiguousarray(v, dtype=np.float64)
        rc = lib.ora_hv_rows(L, _p(t, _d), _p(U, _d), nup, ndn, _p(v, _d),
                             _p(rows, _i64), rows.shape[0], _p(out, _d),
                             nthreads or default_threads())
    assert rc == 0
    return out


def hv_abs_bound(t, U, nup: int, ndn: int, v: np.ndarray, rows=None,
                 nthreads: int | None = None) -> np.ndarray:
    """sum_j |H_ij| |v_j| for every row (or the listed rows): the scale of the
    rounding error of (H v)_i."""
    L, t, U = _model_arrays(t, U)
    v = np.ascontiguousarray(v, dtype=np.float64)
    if rows is None:
        out = np.empty(v.shape[0])
        rp, n = None, 0
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.empty(rows.shape[0])
        rp, n = _p(rows, _i64), rows.shape[0]
    rc = _load().ora_hv_absbound(L, _p(t, _d), _p(U, _d), nup, ndn, _p(v, _d), rp, n,
                                 _p(out, _d), nthreads or default_threads())
    assert rc == 0
    return out


# --------------------------------------------------------------------------
# tridiagonal eigenproblem (eq. (tridiag))

def tridiag_eig(alpha, beta, k: int = 0) -> float:
    """k-th smallest eigenvalue of the tridiagonal with ``alpha`` on the
    diagonal and ``beta[n]`` between n and n+1 (Sturm bisection).
    Pinned against numpy.linalg.eigvalsh."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(np.append(np.asarray(beta, dtype=np.float64), 0.0))
    return float(_load().ora_tridiag_eig(a.shape[0], _p(a, _d), _p(b, _d), k))


def tridiag_vec(alpha, beta, theta: float) -> np.ndarray:
    """Normalised eigenvector for ``theta`` by inverse iteration."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(np.append(np.asarray(beta, dtype=np.float64), 0.0))
    x = np.empty_like(a)
    _load().ora_tridiag_vec(a.shape[0], _p(a, _d), _p(b, _d), theta, _p(x, _d))
    return x


# --------------------------------------------------------------------------
# Lanczos ground state (subsection "The Lanczos algorithm for the ground state")

def lanczos_gs(t, U, nup: int, ndn: int, *, x0=None, seed: int = 1, max_iter: int = 600,
               fixed_steps: int = 0, tol: float = 1e-12, btol: float = 1e-13,
               want_vector: bool = False, nthreads: int | None = None) -> dict:
    """Lowest state of sector (nup, ndn) by the normalised Lanczos recurrence,
    with the ground-state vector from a second identical pass.
    Pinned: dense diagonalisation, the two-site closed form, U=0 and t=0
    limits, particle-hole symmetry."""
    L, t, U = _model_arrays(t, U)
    dim = binom(L, nup) * binom(L, ndn)
    n = max(max_iter, fixed_steps)
    alpha = np.zeros(n)
    beta = np.zeros(n)
    psi = np.empty(dim) if want_vector else None
    od = np.zeros(4)
    oi = np.zeros(3, dtype=np.int32)
    if x0 is not None:
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        assert x0.shape == (dim,)
    rc = _load().ora_lanczos_gs(L, _p(t, _d), _p(U, _d), nup, ndn,
                                _p(x0, _d) if x0 is not None else None, seed, max_iter,
                                fixed_steps, tol, btol, _p(alpha, _d), _p(beta, _d),
                                _p(psi, _d) if psi is not None else None,
                                _p(od, _d), _p(oi, _i32), nthreads or default_threads())
    assert rc == 0
    M = int(oi[0])
    return dict(e0=float(od[0]), residual_est=float(od[1]), true_residual=float(od[2]),
                theta1=float(od[3]), n_iter=M, converged=bool(oi[1]), breakdown=bool(oi[2]),
                alpha=alpha[:M].copy(), beta=beta[:M].copy(), psi=psi)


# --------------------------------------------------------------------------
# Green-function chains (subsection "The Lanczos algorithm for the Green function")

def apply_op(L: int, nup: int, ndn: int, psi: np.ndarray, kind: int, mu: int,
             nu: int = -1) -> np.ndarray:
    """kind 0: (c+_mu [+ c+_nu]) psi in sector (nup+1, ndn);
    kind 1: (c_mu [+ c_nu]) psi in sector (nup-1, ndn).  Up spin."""
    nup2 = nup + 1 if kind == 0 else nup - 1
    out = np.zeros(binom(L, nup2) * binom(L, ndn))
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    rc = _load().ora_apply_cdag_c(L, nup, ndn, _p(psi, _d), kind, mu, nu, _p(out, _d))
    assert rc == 0
    return out


def cf_chain(t, U, nup: int, ndn: int, phi: np.ndarray, max_steps: int, btol: float = 1e-13,
             nthreads: int | None = None, full_reorth: bool = False):
    """Lanczos chain from phi (not normalised) in sector (nup, ndn).
    Returns (b0sq, a[len], b2[len-1]).  full_reorth: the test device that
    removes from every new vector its components along all earlier chain
    vectors (twice), not entered in T."""
    L, t, U = _model_arrays(t, U)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    a = np.zeros(max_steps)
    b2 = np.zeros(max_steps)
    b0 = np.zeros(1)
    lib = _load()
    fn = lib.ora_cf_chain_full if full_reorth else lib.ora_cf_chain
    n = fn(L, _p(t, _d), _p(U, _d), nup, ndn, _p(phi, _d), max_steps, btol,
           _p(b0, _d), _p(a, _d), _p(b2, _d), nthreads or default_threads())
    assert n >= 0
    return float(b0[0]), a[:n].copy(), b2[:max(n - 1, 0)].copy()


def green_cf(t, U, nup: int, ndn: int, psi: np.ndarray, orbs, max_steps: int = 200,
             btol: float = 1e-13, nthreads: int | None = None,
             full_reorth: bool = False) -> dict:
    """All continued fractions for the up-spin Green function restricted to
    the orbitals ``orbs``: for each pair (i <= j) of positions in ``orbs`` an
    electron chain from (c_mu + c_nu)+ psi and a hole chain from
    (c_mu + c_nu) psi (a single operator when i == j).  Returns a dict
    {(i, j, part): (b0sq, a, b2)} with part 0 = electron, 1 = hole."""
    L, t, U = _model_arrays(t, U)
    out = {}
    for i, mu in enumerate(orbs):
        for j in range(i, len(orbs)):
            nu = -1 if j == i else orbs[j]
            for part in (0, 1):
                nup2 = nup + 1 if part == 0 else nup - 1
                if nup2 < 0 or nup2 > L:
                    out[(i, j, part)] = (0.0, np.zeros(0), np.zeros(0))
                    continue
                phi = apply_op(L, nup, ndn, psi, part, mu, nu)
                out[(i, j, part)] = cf_chain(t, U, nup2, ndn, phi, max_steps, btol, nthreads,
                                             full_reorth)
    return out
