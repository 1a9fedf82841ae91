"""ctypes binding of libqcm.so (the C ABI in include/qcm.h).

Argument marshalling only: torch provides device memory (vectors and
workspaces as CUDA/HIP tensors) and the current stream; every step of the
computation runs in the library's HIP kernels.  If the library is missing or a
GPU is not available the calls raise; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqcm.so")

QCM_OK, QCM_EARG, QCM_ERANGE, QCM_EWORKSPACE, QCM_EHIP = 0, -1, -2, -3, -4
QCM_FP64, QCM_FP32V = 0, 1
PREC = {"fp64": QCM_FP64, "fp32v": QCM_FP32V, QCM_FP64: QCM_FP64, QCM_FP32V: QCM_FP32V}

_c_d = ctypes.POINTER(ctypes.c_double)
_c_i32 = ctypes.POINTER(ctypes.c_int32)
_c_sz = ctypes.POINTER(ctypes.c_size_t)


class QcmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qcm error {code}: {msg}")
        self.code = code


class Model(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("t", _c_d), ("U", _c_d)]


class Basis(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32),
                ("l_lo", ctypes.c_int32), ("l_hi", ctypes.c_int32),
                ("d_up", ctypes.c_int64), ("d_dn", ctypes.c_int64), ("dim", ctypes.c_int64),
                ("states_up", ctypes.c_void_p), ("states_dn", ctypes.c_void_p),
                ("rank_lo_up", ctypes.c_void_p), ("rank_hi_up", ctypes.c_void_p),
                ("rank_lo_dn", ctypes.c_void_p), ("rank_hi_dn", ctypes.c_void_p)]


class LanczosOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("fixed_steps", ctypes.c_int32),
                ("want_vector", ctypes.c_int32), ("reorth", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("tol", ctypes.c_double), ("btol", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("d_v0", ctypes.c_void_p)]


class GsResult(ctypes.Structure):
    _fields_ = [("e0", ctypes.c_double), ("residual_est", ctypes.c_double),
                ("true_residual", ctypes.c_double), ("theta1", ctypes.c_double),
                ("n_iter", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("breakdown", ctypes.c_int32), ("degenerate_suspect", ctypes.c_int32)]


class GreenOpts(ctypes.Structure):
    _fields_ = [("n_orb", ctypes.c_int32), ("orbs", _c_i32), ("max_steps", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("reorth", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("btol", ctypes.c_double)]


class BandOpts(ctypes.Structure):
    _fields_ = [("n_orb", ctypes.c_int32), ("pad0", ctypes.c_int32), ("orbs", _c_i32),
                ("max_basis", ctypes.c_int32), ("prec", ctypes.c_int32), ("dtol", ctypes.c_double),
                ("max_sweeps", ctypes.c_int32), ("pad1", ctypes.c_int32), ("etol", ctypes.c_double)]


class Bond(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int32), ("j", ctypes.c_int32), ("shift", ctypes.c_int32 * 3),
                ("pad", ctypes.c_int32), ("t", ctypes.c_double)]


class Group(ctypes.Structure):
    _fields_ = [("n_g", ctypes.c_int32), ("pad", ctypes.c_int32), ("perm", _c_i32), ("chi", _c_i32)]


class SymSectorC(ctypes.Structure):
    _fields_ = [("b", Basis), ("n_g", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("chi", ctypes.c_int32 * 8), ("perm", ctypes.c_int8 * 256),
                ("dim", ctypes.c_int64), ("n_words", ctypes.c_int64),
                ("bits", ctypes.c_void_p), ("base", ctypes.c_void_p),
                ("img_up", ctypes.c_void_p), ("img_dn", ctypes.c_void_p)]


class SymCsrC(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rep", ctypes.c_void_p),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("packed", ctypes.c_void_p), ("table", ctypes.c_void_p)]


class EngineOpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("reorth", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("gs_fixed_steps", ctypes.c_int32),
                ("gf_steps", ctypes.c_int32), ("max_jobs", ctypes.c_int32),
                ("tol", ctypes.c_double), ("btol", ctypes.c_double),
                ("n_z", ctypes.c_int32), ("pad", ctypes.c_int32), ("h_z", _c_d)]


class Job(ctypes.Structure):
    _fields_ = [("model", Model), ("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32),
                ("n_orb", ctypes.c_int32), ("pad", ctypes.c_int32), ("orbs", _c_i32),
                ("seed", ctypes.c_uint64), ("tag", ctypes.c_int64), ("h_G", _c_d),
                ("h_coef", _c_d), ("h_len", _c_i32), ("d_psi", ctypes.c_void_p)]


class JobResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("e0", ctypes.c_double), ("theta1", ctypes.c_double),
                ("residual_est", ctypes.c_double), ("true_residual", ctypes.c_double),
                ("n_iter", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("breakdown", ctypes.c_int32), ("status", ctypes.c_int32),
                ("bytes", ctypes.c_int64), ("rounds", ctypes.c_int32),
                ("degenerate_suspect", ctypes.c_int32)]


class EngineStats(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_int64), ("header_bytes", ctypes.c_int64),
                ("in_use", ctypes.c_int64), ("peak_in_use", ctypes.c_int64),
                ("largest_free", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("active", ctypes.c_int32), ("finished", ctypes.c_int32)]


# every symbol declared in include/qcm.h
EXPORTS = ["qcm_last_error", "qcm_version", "qcm_sector_basis", "qcm_hv",
           "qcm_lanczos_default_opts", "qcm_lanczos_gs", "qcm_green_cf", "qcm_cpt_gk",
           "qcm_engine_default_opts", "qcm_engine_create", "qcm_engine_destroy",
           "qcm_engine_job_bytes", "qcm_engine_submit", "qcm_engine_step", "qcm_engine_poll",
           "qcm_engine_info", "qcm_batch_solve", "qcm_hv_plan_create", "qcm_hv_plan_apply",
           "qcm_hv_plan_destroy", "qcm_band_default_opts", "qcm_green_band", "qcm_cdmft_g0inv",
           "qcm_cdmft_fit", "qcm_vca_omega", "qcm_vca_omega_quad", "qcm_sym_sector_build", "qcm_sym_csr_count",
           "qcm_sym_csr_fill", "qcm_sym_csr_pack", "qcm_sym_hv", "qcm_sym_lanczos_gs",
           "qcm_lehmann_form", "qcm_hv_noalloc"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libqcm.so and declare the signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() or "
                           "python paper_2305_18643_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.qcm_last_error.restype = ctypes.c_char_p
    lib.qcm_last_error.argtypes = []
    lib.qcm_version.restype = ctypes.c_int
    lib.qcm_sector_basis.restype = ctypes.c_int
    lib.qcm_sector_basis.argtypes = [ctypes.c_int32] * 3 + [vp, sz, _c_sz, ctypes.POINTER(Basis), vp]
    lib.qcm_hv.restype = ctypes.c_int
    lib.qcm_hv.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(Basis), ctypes.c_int32, vp, vp,
                           vp, sz, _c_sz, vp]
    lib.qcm_lanczos_default_opts.restype = None
    lib.qcm_lanczos_default_opts.argtypes = [ctypes.POINTER(LanczosOpts)]
    lib.qcm_lanczos_gs.restype = ctypes.c_int
    lib.qcm_lanczos_gs.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(Basis),
                                   ctypes.POINTER(LanczosOpts), _c_d, _c_d, vp,
                                   ctypes.POINTER(GsResult), vp, sz, _c_sz, vp]
    lib.qcm_green_cf.restype = ctypes.c_int
    lib.qcm_green_cf.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(Basis), vp,
                                 ctypes.c_double, ctypes.POINTER(GreenOpts), _c_d, _c_i32,
                                 ctypes.c_int32, _c_d, vp, vp, sz, _c_sz, vp]
    lib.qcm_cpt_gk.restype = ctypes.c_int
    lib.qcm_cpt_gk.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, _c_i32, _c_i32,
                               ctypes.c_int32, ctypes.POINTER(Bond), ctypes.c_int32, _c_d, vp,
                               vp, sz, _c_sz, vp]
    P = ctypes.POINTER
    lib.qcm_band_default_opts.restype = None
    lib.qcm_band_default_opts.argtypes = [P(BandOpts)]
    lib.qcm_green_band.restype = ctypes.c_int
    lib.qcm_green_band.argtypes = [P(Model), P(Basis), vp, ctypes.c_double, P(BandOpts), _c_i32,
                                   _c_d, _c_d, ctypes.c_int32, _c_d, vp, vp, sz, _c_sz, vp]
    lib.qcm_hv_noalloc.restype = ctypes.c_int
    lib.qcm_hv_noalloc.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(Basis), ctypes.c_int32, vp,
                                   vp, vp]
    lib.qcm_lehmann_form.restype = ctypes.c_int
    lib.qcm_lehmann_form.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _c_i32,
                                     _c_d, _c_d, _c_d, _c_d]
    lib.qcm_hv_plan_create.restype = ctypes.c_int
    lib.qcm_hv_plan_create.argtypes = [P(Model), P(Basis), ctypes.c_int32, vp, sz, _c_sz, vp, P(vp)]
    lib.qcm_hv_plan_apply.restype = ctypes.c_int
    lib.qcm_hv_plan_apply.argtypes = [vp, vp, vp, ctypes.c_int32, vp]
    lib.qcm_hv_plan_destroy.restype = ctypes.c_int
    lib.qcm_hv_plan_destroy.argtypes = [vp]
    lib.qcm_engine_default_opts.restype = ctypes.c_int
    lib.qcm_engine_default_opts.argtypes = [P(EngineOpts)]
    lib.qcm_engine_create.restype = ctypes.c_int
    lib.qcm_engine_create.argtypes = [P(EngineOpts), vp, sz, vp, P(vp)]
    lib.qcm_engine_destroy.restype = ctypes.c_int
    lib.qcm_engine_destroy.argtypes = [vp]
    lib.qcm_engine_job_bytes.restype = ctypes.c_int
    lib.qcm_engine_job_bytes.argtypes = [P(EngineOpts), P(Job), _c_sz]
    lib.qcm_engine_submit.restype = ctypes.c_int
    lib.qcm_engine_submit.argtypes = [vp, P(Job)]
    lib.qcm_engine_step.restype = ctypes.c_int
    lib.qcm_engine_step.argtypes = [vp, ctypes.c_int32, _c_i32]
    lib.qcm_engine_poll.restype = ctypes.c_int
    lib.qcm_engine_poll.argtypes = [vp, ctypes.c_int32, P(JobResult), _c_i32]
    lib.qcm_engine_info.restype = ctypes.c_int
    lib.qcm_engine_info.argtypes = [vp, P(EngineStats)]
    lib.qcm_batch_solve.restype = ctypes.c_int
    lib.qcm_batch_solve.argtypes = [P(EngineOpts), ctypes.c_int32, P(Job), P(JobResult), vp, sz,
                                    _c_sz, vp]
    I32, D = ctypes.c_int32, ctypes.c_double
    lib.qcm_cdmft_g0inv.restype = ctypes.c_int
    lib.qcm_cdmft_g0inv.argtypes = [I32, I32, _c_d, _c_d, _c_d, I32, P(Bond), I32, _c_d, I32, _c_d,
                                    vp, vp, vp, vp, vp, sz, _c_sz, vp]
    lib.qcm_cdmft_fit.restype = ctypes.c_int
    lib.qcm_cdmft_fit.argtypes = [I32, I32, I32, _c_d, _c_d, _c_d, I32, _c_d, _c_d, vp, _c_d, D,
                                  I32, _c_d, _c_i32, vp, sz, _c_sz, vp]
    lib.qcm_sym_sector_build.restype = ctypes.c_int
    lib.qcm_sym_sector_build.argtypes = [P(Basis), P(Group), vp, sz, _c_sz, P(SymSectorC), vp]
    lib.qcm_sym_csr_count.restype = ctypes.c_int
    lib.qcm_sym_csr_count.argtypes = [P(Model), P(SymSectorC), vp, vp, P(ctypes.c_int64), vp, sz,
                                      _c_sz, vp]
    lib.qcm_sym_csr_fill.restype = ctypes.c_int
    lib.qcm_sym_csr_fill.argtypes = [P(Model), P(SymSectorC), vp, vp, vp, vp, vp]
    lib.qcm_sym_csr_pack.restype = ctypes.c_int
    lib.qcm_sym_csr_pack.argtypes = [P(SymCsrC), vp, vp, _c_i32, vp, sz, _c_sz, vp]
    lib.qcm_sym_hv.restype = ctypes.c_int
    lib.qcm_sym_hv.argtypes = [P(SymCsrC), vp, vp, I32, vp]
    lib.qcm_sym_lanczos_gs.restype = ctypes.c_int
    lib.qcm_sym_lanczos_gs.argtypes = [P(SymCsrC), P(LanczosOpts), _c_d, _c_d, vp, P(GsResult), vp,
                                       sz, _c_sz, vp]
    lib.qcm_vca_omega_quad.restype = ctypes.c_int
    lib.qcm_vca_omega_quad.argtypes = [I32, I32, _c_d, _c_d, _c_d, I32, P(Bond), I32, _c_d, D, D, I32,
                                       _c_d, _c_d, _c_i32, vp, sz, _c_sz, vp]
    lib.qcm_vca_omega.restype = ctypes.c_int
    lib.qcm_vca_omega.argtypes = [I32, I32, _c_d, _c_d, _c_d, I32, P(Bond), I32, _c_d, D, _c_d, _c_d,
                                  vp, sz, _c_sz, vp]
    _lib = lib
    return lib


def _check(code: int):
    if code != QCM_OK:
        raise QcmError(code, _lib.qcm_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the qcm library runs only on the device")
    return torch


def _stream(torch, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _workspace(torch, nbytes: int, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class HostModel:
    """(t, U) kept alive as contiguous float64 arrays plus the C struct."""

    def __init__(self, t, U):
        self.t = np.ascontiguousarray(t, dtype=np.float64)
        self.U = np.ascontiguousarray(U, dtype=np.float64)
        L = self.t.shape[0]
        if self.t.shape != (L, L) or self.U.shape != (L,):
            raise ValueError("t must be L x L and U of length L")
        self.c = Model(L, self.t.ctypes.data_as(_c_d), self.U.ctypes.data_as(_c_d))

    @property
    def L(self):
        return self.t.shape[0]


def as_model(m) -> HostModel:
    if isinstance(m, HostModel):
        return m
    if isinstance(m, tuple):
        return HostModel(*m)
    return HostModel(m.t, m.U)


class SectorBasis:
    """A device sector basis; owns the workspace its tables live in."""

    def __init__(self, L: int, n_up: int, n_dn: int, device="cuda", stream=None):
        torch = _torch()
        lib = load_library()
        self.c = Basis()
        need = ctypes.c_size_t(0)
        _check(lib.qcm_sector_basis(L, n_up, n_dn, None, 0, ctypes.byref(need),
                                    ctypes.byref(self.c), None))
        self.ws = _workspace(torch, need.value, device)
        _check(lib.qcm_sector_basis(L, n_up, n_dn, _ptr(self.ws), self.ws.numel(),
                                    ctypes.byref(need), ctypes.byref(self.c),
                                    _stream(torch, stream)))
        self.device = self.ws.device

    L = property(lambda self: self.c.L)
    n_up = property(lambda self: self.c.n_up)
    n_dn = property(lambda self: self.c.n_dn)
    d_up = property(lambda self: self.c.d_up)
    d_dn = property(lambda self: self.c.d_dn)
    dim = property(lambda self: self.c.dim)

    def states(self, spin: int):
        """Device uint32 string list of one spin (as an int64 copy)."""
        torch = _torch()
        d = self.d_up if spin == 0 else self.d_dn
        ptr = self.c.states_up if spin == 0 else self.c.states_dn
        base = self.ws.data_ptr()
        off = ptr - base
        raw = self.ws[off: off + 4 * d].view(torch.int32)
        return raw.to(torch.int64) & 0xFFFFFFFF

    def rank_tables(self, spin: int):
        torch = _torch()
        lo = self.c.rank_lo_up if spin == 0 else self.c.rank_lo_dn
        hi = self.c.rank_hi_up if spin == 0 else self.c.rank_hi_dn
        base = self.ws.data_ptr()
        n_lo = 1 << self.c.l_lo
        n_hi = (self.c.l_lo + 1) << self.c.l_hi
        tlo = self.ws[lo - base: lo - base + 4 * n_lo].view(torch.int32)
        thi = self.ws[hi - base: hi - base + 4 * n_hi].view(torch.int32)
        return tlo, thi


def sector_basis(L: int, n_up: int, n_dn: int, device="cuda", stream=None) -> SectorBasis:
    return SectorBasis(L, n_up, n_dn, device, stream)


def hv(model, basis: SectorBasis, v, w=None, stream=None, ws=None):
    """w = H v.  v: device float64 (FP64) or float32 (FP32-vector) tensor."""
    torch = _torch()
    lib = load_library()
    m = as_model(model)
    prec = QCM_FP64 if v.dtype == torch.float64 else QCM_FP32V
    if v.dtype not in (torch.float64, torch.float32) or v.numel() != basis.dim or not v.is_contiguous():
        raise ValueError("v must be a contiguous float64/float32 tensor of length dim")
    if w is None:
        w = torch.empty_like(v)
    need = ctypes.c_size_t(0)
    _check(lib.qcm_hv(ctypes.byref(m.c), ctypes.byref(basis.c), prec, None, None, None, 0,
                      ctypes.byref(need), None))
    if ws is None or ws.numel() < need.value:
        ws = _workspace(torch, need.value, v.device)
    _check(lib.qcm_hv(ctypes.byref(m.c), ctypes.byref(basis.c), prec, _ptr(v), _ptr(w), _ptr(ws),
                      ws.numel(), ctypes.byref(need), _stream(torch, stream)))
    return w


def hv_noalloc(model, basis: SectorBasis, v, w, stream=None):
    """w = H v through qcm_hv_noalloc (tables in the library's static device
    array; nothing allocated).  v, w: device float64 or float32 tensors."""
    torch = _torch()
    lib = load_library()
    m = as_model(model)
    prec = QCM_FP64 if v.dtype == torch.float64 else QCM_FP32V
    for x in (v, w):
        if x.dtype != v.dtype or x.numel() != basis.dim or not x.is_contiguous():
            raise ValueError("v, w must be contiguous tensors of one dtype and length dim")
    _check(lib.qcm_hv_noalloc(ctypes.byref(m.c), ctypes.byref(basis.c), prec, _ptr(v), _ptr(w),
                              _stream(torch, stream)))
    return w


class HvPlan:
    """Tables of H.v built once (qcm_hv_plan_*); call it as plan(v, w)."""

    def __init__(self, model, basis: SectorBasis, prec="fp64", stream=None):
        torch = _torch()
        self.lib = load_library()
        self.m = as_model(model)
        self.basis = basis
        self.prec = PREC[prec]
        need = ctypes.c_size_t(0)
        _check(self.lib.qcm_hv_plan_create(ctypes.byref(self.m.c), ctypes.byref(basis.c),
                                           self.prec, None, 0, ctypes.byref(need), None, None))
        self.ws = _workspace(torch, need.value, basis.device)
        self.h = ctypes.c_void_p()
        _check(self.lib.qcm_hv_plan_create(ctypes.byref(self.m.c), ctypes.byref(basis.c),
                                           self.prec, _ptr(self.ws), self.ws.numel(),
                                           ctypes.byref(need), _stream(torch, stream),
                                           ctypes.byref(self.h)))

    def __call__(self, v, w, nvec=1, stream=None):
        torch = _torch()
        want = torch.float64 if self.prec == QCM_FP64 else torch.float32
        if v.dtype != want or w.dtype != want or v.numel() != nvec * self.basis.dim or \
                w.numel() != v.numel():
            raise ValueError("v, w must be nvec * dim elements of the plan's precision")
        _check(self.lib.qcm_hv_plan_apply(self.h, _ptr(v), _ptr(w), nvec, _stream(torch, stream)))
        return w

    def close(self):
        if self.h:
            _check(self.lib.qcm_hv_plan_destroy(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lanczos_gs(model, basis: SectorBasis, *, max_iter=600, fixed_steps=0, want_vector=True,
               reorth=0, prec="fp64", check_every=1, tol=1e-12, btol=1e-13, seed=1, v0=None,
               stream=None, ws=None) -> dict:
    """Lanczos ground state; returns e0, residuals, n_iter, flags, alpha, beta, psi."""
    torch = _torch()
    lib = load_library()
    m = as_model(model)
    o = LanczosOpts()
    lib.qcm_lanczos_default_opts(ctypes.byref(o))
    o.max_iter, o.fixed_steps, o.want_vector, o.reorth = max_iter, fixed_steps, int(want_vector), reorth
    o.prec, o.check_every, o.tol, o.btol, o.seed = PREC[prec], check_every, tol, btol, seed
    if v0 is not None:
        want = torch.float64 if o.prec == QCM_FP64 else torch.float32
        if v0.dtype != want or v0.numel() != basis.dim:
            raise ValueError("v0 has the wrong dtype or size")
        o.d_v0 = v0.data_ptr()
    need = ctypes.c_size_t(0)
    _check(lib.qcm_lanczos_gs(ctypes.byref(m.c), ctypes.byref(basis.c), ctypes.byref(o), None,
                              None, None, None, None, 0, ctypes.byref(need), None))
    if ws is None or ws.numel() < need.value:
        ws = _workspace(torch, need.value, basis.device)
    n = max(max_iter, fixed_steps)
    alpha = np.zeros(n)
    beta = np.zeros(n)
    psi = torch.empty(basis.dim, dtype=torch.float64, device=basis.device) if want_vector else None
    res = GsResult()
    _check(lib.qcm_lanczos_gs(ctypes.byref(m.c), ctypes.byref(basis.c), ctypes.byref(o),
                              alpha.ctypes.data_as(_c_d), beta.ctypes.data_as(_c_d), _ptr(psi),
                              ctypes.byref(res), _ptr(ws), ws.numel(), ctypes.byref(need),
                              _stream(torch, stream)))
    M = res.n_iter
    return dict(e0=res.e0, residual_est=res.residual_est, true_residual=res.true_residual,
                theta1=res.theta1, n_iter=M, converged=bool(res.converged),
                breakdown=bool(res.breakdown), degenerate_suspect=bool(res.degenerate_suspect),
                alpha=alpha[:M], beta=beta[:M], psi=psi)


def green_cf(model, basis: SectorBasis, psi, e0: float, orbs, z, *, max_steps=200, prec="fp64",
             reorth=0, btol=1e-13, stream=None, ws=None) -> dict:
    """Continued-fraction up-spin G_ij(z) for i, j in orbs; returns G (device
    complex128 [n_z, n, n]), coef (numpy [n_pairs, 2, 1 + 2 max_steps]) and
    len (numpy [n_pairs, 2])."""
    torch = _torch()
    lib = load_library()
    m = as_model(model)
    orbs_a = np.ascontiguousarray(orbs, dtype=np.int32)
    n = orbs_a.shape[0]
    npairs = n * (n + 1) // 2
    o = GreenOpts(n, orbs_a.ctypes.data_as(_c_i32), max_steps, PREC[prec], reorth, 0, btol)
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    zz = np.ascontiguousarray(np.stack([z.real, z.imag], axis=-1).ravel())
    nz = z.shape[0]
    need = ctypes.c_size_t(0)
    _check(lib.qcm_green_cf(ctypes.byref(m.c), ctypes.byref(basis.c), None, e0, ctypes.byref(o),
                            None, None, nz, zz.ctypes.data_as(_c_d), None, None, 0,
                            ctypes.byref(need), None))
    if ws is None or ws.numel() < need.value:
        ws = _workspace(torch, need.value, basis.device)
    G = torch.zeros((max(nz, 1), n, n), dtype=torch.complex128, device=basis.device)
    coef = np.zeros((npairs, 2, 1 + 2 * max_steps))
    lens = np.zeros((npairs, 2), dtype=np.int32)
    if psi.dtype != torch.float64 or psi.numel() != basis.dim:
        raise ValueError("psi must be a float64 device vector of the basis dimension")
    _check(lib.qcm_green_cf(ctypes.byref(m.c), ctypes.byref(basis.c), _ptr(psi), float(e0),
                            ctypes.byref(o), coef.ctypes.data_as(_c_d),
                            lens.ctypes.data_as(_c_i32), nz, zz.ctypes.data_as(_c_d),
                            ctypes.c_void_p(G.data_ptr()), _ptr(ws), ws.numel(),
                            ctypes.byref(need), _stream(torch, stream)))
    return dict(G=G[:nz], coef=coef, len=lens)


def green_band(model, basis: SectorBasis, psi, e0: float, orbs, z, *, max_basis=400,
               prec="fp64", dtol=1e-10, max_sweeps=40, etol=0.0, stream=None, ws=None) -> dict:
    """Band Lanczos up-spin G_ij(z) for i, j in orbs; returns G (device
    complex128 [n_z, n, n]), R (numpy [2]), lam (list of two numpy arrays) and
    Q (list of two numpy [n, R] arrays), electron part first.  etol > 0 stops
    each part once its lowest Ritz value has converged (the paper's rule);
    max_sweeps caps the eigen-solver of T at max_sweeps * R QR steps."""
    torch = _torch()
    lib = load_library()
    m = as_model(model)
    orbs_a = np.ascontiguousarray(orbs, dtype=np.int32)
    n = orbs_a.shape[0]
    o = BandOpts()
    lib.qcm_band_default_opts(ctypes.byref(o))
    o.n_orb, o.orbs, o.max_basis, o.prec = n, orbs_a.ctypes.data_as(_c_i32), max_basis, PREC[prec]
    o.dtol, o.max_sweeps, o.etol = dtol, max_sweeps, etol
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    zz = np.ascontiguousarray(np.stack([z.real, z.imag], axis=-1).ravel())
    nz = z.shape[0]
    need = ctypes.c_size_t(0)
    _check(lib.qcm_green_band(ctypes.byref(m.c), ctypes.byref(basis.c), None, e0, ctypes.byref(o),
                              None, None, None, nz, zz.ctypes.data_as(_c_d), None, None, 0,
                              ctypes.byref(need), None))
    if ws is None or ws.numel() < need.value:
        ws = _workspace(torch, need.value, basis.device)
    G = torch.zeros((max(nz, 1), n, n), dtype=torch.complex128, device=basis.device)
    R = np.zeros(2, dtype=np.int32)
    lam = np.zeros((2, max_basis))
    Q = np.zeros((2, n, max_basis))
    if psi.dtype != torch.float64 or psi.numel() != basis.dim:
        raise ValueError("psi must be a float64 device vector of the basis dimension")
    _check(lib.qcm_green_band(ctypes.byref(m.c), ctypes.byref(basis.c), _ptr(psi), float(e0),
                              ctypes.byref(o), R.ctypes.data_as(_c_i32), lam.ctypes.data_as(_c_d),
                              Q.ctypes.data_as(_c_d), nz, zz.ctypes.data_as(_c_d),
                              ctypes.c_void_p(G.data_ptr()), _ptr(ws), ws.numel(),
                              ctypes.byref(need), _stream(torch, stream)))
    Rt = int(R[0]) + int(R[1])
    poles = np.zeros(max(Rt, 1))
    Qcat = np.zeros((n, max(Rt, 1)))
    _check(lib.qcm_lehmann_form(n, max_basis, float(e0), R.ctypes.data_as(_c_i32),
                                lam.ctypes.data_as(_c_d), Q.ctypes.data_as(_c_d),
                                poles.ctypes.data_as(_c_d), Qcat.ctypes.data_as(_c_d)))
    return dict(G=G[:nz], R=R, lam=[lam[k, :R[k]].copy() for k in range(2)],
                Q=[Q[k, :, :R[k]].copy() for k in range(2)],
                poles=poles[:Rt].copy(), Q_lehmann=np.ascontiguousarray(Qcat[:, :Rt]))


def cpt_gk(Gc, R, E, bonds, ks, z=None, stream=None):
    """CPT G-scheme periodised G(k, z).  Gc: device complex128 [n_z, L, L];
    bonds: iterable of (i, j, (s1, s2, s3), t); ks [n_k, 3] in units of 2 pi.
    Returns device complex128 [n_k, n_z]."""
    torch = _torch()
    lib = load_library()
    if Gc.dtype != torch.complex128 or Gc.dim() != 3 or not Gc.is_contiguous():
        raise ValueError("Gc must be a contiguous complex128 [n_z, L, L] tensor")
    nz, L, _ = Gc.shape
    R = np.ascontiguousarray(R, dtype=np.int32).reshape(L, 3)
    E = np.ascontiguousarray(E, dtype=np.int32).reshape(3, 3)
    ks = np.ascontiguousarray(ks, dtype=np.float64).reshape(-1, 3)
    bl = list(bonds)
    barr = (Bond * max(len(bl), 1))()
    for q, (i, j, s, t) in enumerate(bl):
        barr[q].i, barr[q].j, barr[q].t = int(i), int(j), float(t)
        for a in range(3):
            barr[q].shift[a] = int(s[a])
    out = torch.zeros((ks.shape[0], nz), dtype=torch.complex128, device=Gc.device)
    need = ctypes.c_size_t(0)
    args = (L, nz)
    _check(lib.qcm_cpt_gk(*args, None, R.ctypes.data_as(_c_i32), E.ctypes.data_as(_c_i32),
                          len(bl), barr, ks.shape[0], ks.ctypes.data_as(_c_d), None, None, 0,
                          ctypes.byref(need), None))
    ws = _workspace(torch, need.value, Gc.device)
    _check(lib.qcm_cpt_gk(*args, ctypes.c_void_p(Gc.data_ptr()), R.ctypes.data_as(_c_i32),
                          E.ctypes.data_as(_c_i32), len(bl), barr, ks.shape[0],
                          ks.ctypes.data_as(_c_d), ctypes.c_void_p(out.data_ptr()), _ptr(ws),
                          ws.numel(), ctypes.byref(need), _stream(torch, stream)))
    return out


# ---------------------------------------------------------------- CDMFT

def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a if shape is None else a.reshape(shape)


def _zz(z):
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=-1).ravel()), z.shape[0]


def cdmft_g0inv(Gc, tcp, theta, eps, bonds, ks, z, *, stream=None):
    """Sigma_c, Gbar and calG0^{-1} (device complex128 [n_z, L, L] each) from
    the cluster Green function Gc (device complex128 [n_z, L, L])."""
    torch = _torch()
    lib = load_library()
    if Gc.dtype != torch.complex128 or Gc.dim() != 3 or not Gc.is_contiguous():
        raise ValueError("Gc must be a contiguous complex128 [n_z, L, L] tensor")
    nz, L, _ = Gc.shape
    tcp = _f64(tcp, (L, L))
    theta = _f64(theta).reshape(L, -1)
    nb = theta.shape[1]
    theta = np.ascontiguousarray(theta)
    eps = _f64(eps, (nb,))
    ks = _f64(ks).reshape(-1, 3)
    zz, nz2 = _zz(z)
    if nz2 != nz:
        raise ValueError("z and Gc disagree on the number of frequencies")
    bl = list(bonds)
    barr = (Bond * max(len(bl), 1))()
    for q, (i, j, sh, t) in enumerate(bl):
        barr[q].i, barr[q].j, barr[q].t = int(i), int(j), float(t)
        for a in range(3):
            barr[q].shift[a] = int(sh[a])
    out = [torch.zeros((nz, L, L), dtype=torch.complex128, device=Gc.device) for _ in range(3)]
    need = ctypes.c_size_t(0)
    args = (L, nb, tcp.ctypes.data_as(_c_d), theta.ctypes.data_as(_c_d), eps.ctypes.data_as(_c_d),
            len(bl), barr, ks.shape[0], ks.ctypes.data_as(_c_d), nz, zz.ctypes.data_as(_c_d))
    _check(lib.qcm_cdmft_g0inv(*args, None, None, None, None, None, 0, ctypes.byref(need), None))
    ws = _workspace(torch, need.value, Gc.device)
    _check(lib.qcm_cdmft_g0inv(*args, ctypes.c_void_p(Gc.data_ptr()),
                               *[ctypes.c_void_p(o.data_ptr()) for o in out], _ptr(ws), ws.numel(),
                               ctypes.byref(need), _stream(torch, stream)))
    return dict(sigma=out[0], gbar=out[1], g0inv=out[2])


def cdmft_fit(g0inv, tcp, A_eps, A_theta, p0, z, w, *, gtol=1e-10, max_iter=500, stream=None):
    """Bath parameters minimising the distance function from p0 (BFGS on the
    device).  Returns (p, distance, BFGS steps; negative if the line search
    failed)."""
    torch = _torch()
    lib = load_library()
    nz, L, _ = g0inv.shape
    A_eps = _f64(A_eps)
    npar = A_eps.shape[1]
    nb = A_eps.shape[0]
    A_theta = _f64(A_theta, (L * nb, npar))
    tcp = _f64(tcp, (L, L))
    zz, nz2 = _zz(z)
    w = _f64(w, (nz,))
    if nz2 != nz:
        raise ValueError("z and g0inv disagree on the number of frequencies")
    p = _f64(p0, (npar,)).copy()
    dist = ctypes.c_double(0.0)
    iters = ctypes.c_int32(0)
    need = ctypes.c_size_t(0)
    args = (L, nb, npar, A_eps.ctypes.data_as(_c_d), A_theta.ctypes.data_as(_c_d),
            tcp.ctypes.data_as(_c_d), nz, zz.ctypes.data_as(_c_d), w.ctypes.data_as(_c_d))
    _check(lib.qcm_cdmft_fit(*args, None, p.ctypes.data_as(_c_d), gtol, max_iter, None, None, None,
                             0, ctypes.byref(need), None))
    ws = _workspace(torch, need.value, g0inv.device)
    _check(lib.qcm_cdmft_fit(*args, ctypes.c_void_p(g0inv.data_ptr()), p.ctypes.data_as(_c_d), gtol,
                             max_iter, ctypes.byref(dist), ctypes.byref(iters), _ptr(ws), ws.numel(),
                             ctypes.byref(need), _stream(torch, stream)))
    return p, dist.value, iters.value


def _bond_array(bonds):
    bl = list(bonds)
    barr = (Bond * max(len(bl), 1))()
    for q, (i, j, sh, t) in enumerate(bl):
        barr[q].i, barr[q].j, barr[q].t = int(i), int(j), float(t)
        for a in range(3):
            barr[q].shift[a] = int(sh[a])
    return barr, len(bl)


def vca_omega(e0, poles, Q, dt, bonds, ks, *, device="cuda", stream=None):
    """Potthoff functional by the pole formula (both spins) from the
    reference's Lehmann form: e0, poles [R], Q [L, R] (up spin), dt [L, L]
    (lattice minus reference intra-cluster matrix), inter-cluster bonds and
    the wave-vectors ks [n_k, 3].  Returns (Omega, per-k sums of the negative
    eigenvalues of L(k))."""
    torch = _torch()
    lib = load_library()
    Q = _f64(Q)
    L, R = Q.shape
    poles = _f64(poles, (R,))
    dt = _f64(dt, (L, L))
    ks = _f64(ks).reshape(-1, 3)
    barr, nbond = _bond_array(bonds)
    om = ctypes.c_double(0.0)
    per = np.zeros(ks.shape[0])
    need = ctypes.c_size_t(0)
    args = (L, R, poles.ctypes.data_as(_c_d), Q.ctypes.data_as(_c_d), dt.ctypes.data_as(_c_d), nbond,
            barr, ks.shape[0], ks.ctypes.data_as(_c_d), float(e0))
    _check(lib.qcm_vca_omega(*args, None, None, None, 0, ctypes.byref(need), None))
    ws = _workspace(torch, need.value, device)
    _check(lib.qcm_vca_omega(*args, ctypes.byref(om), per.ctypes.data_as(_c_d), _ptr(ws), ws.numel(),
                             ctypes.byref(need), _stream(torch, stream)))
    return om.value, per


def vca_omega_quad(e0, poles, Q, dt, bonds, ks, *, rtol=1e-12, max_intervals=4096,
                   device="cuda", stream=None):
    """The same functional by the adaptive frequency integral of eq. (sef4)
    (qcm_vca_omega_quad).  Returns (Omega, error estimate, intervals)."""
    torch = _torch()
    lib = load_library()
    Q = _f64(Q)
    L, R = Q.shape
    poles = _f64(poles, (R,))
    dt = _f64(dt, (L, L))
    ks = _f64(ks).reshape(-1, 3)
    barr, nbond = _bond_array(bonds)
    om = ctypes.c_double(0.0)
    err = ctypes.c_double(0.0)
    niv = ctypes.c_int32(0)
    need = ctypes.c_size_t(0)
    args = (L, R, poles.ctypes.data_as(_c_d), Q.ctypes.data_as(_c_d), dt.ctypes.data_as(_c_d), nbond,
            barr, ks.shape[0], ks.ctypes.data_as(_c_d), float(e0), float(rtol), int(max_intervals))
    _check(lib.qcm_vca_omega_quad(*args, None, None, None, None, 0, ctypes.byref(need), None))
    ws = _workspace(torch, need.value, device)
    _check(lib.qcm_vca_omega_quad(*args, ctypes.byref(om), ctypes.byref(err), ctypes.byref(niv),
                                  _ptr(ws), ws.numel(), ctypes.byref(need), _stream(torch, stream)))
    return om.value, err.value, niv.value


# ---------------------------------------------------------------- batched / served solves

def engine_opts(*, prec="fp32v", reorth=None, max_iter=600, gs_fixed_steps=0, gf_steps=100,
                tol=0.0, btol=1e-13, max_jobs=256, z=()):
    """EngineOpts plus the frequency array it points to (keep both alive)."""
    o = EngineOpts()
    lib = load_library()
    _check(lib.qcm_engine_default_opts(ctypes.byref(o)))
    o.prec = PREC[prec]
    o.reorth = (1 if o.prec == QCM_FP32V else 0) if reorth is None else int(reorth)
    o.max_iter, o.gs_fixed_steps, o.gf_steps = max_iter, gs_fixed_steps, gf_steps
    o.tol, o.btol, o.max_jobs = tol, btol, max_jobs
    zc = np.asarray(z, dtype=np.complex128).ravel()
    zz = np.ascontiguousarray(np.stack([zc.real, zc.imag], axis=-1).ravel())
    o.n_z = zc.shape[0]
    o.h_z = zz.ctypes.data_as(_c_d) if zc.shape[0] else None
    return o, zz


class JobSpec:
    """One solve: model (t, U), sector, G orbitals, seed.  Holds the host
    buffers the library writes the job's outputs into."""

    def __init__(self, model, n_up, n_dn, orbs=(), seed=1, tag=0, psi=None):
        self.model = as_model(model)
        self.n_up, self.n_dn = int(n_up), int(n_dn)
        self.orbs = np.ascontiguousarray(orbs, dtype=np.int32).ravel()
        self.seed, self.tag, self.psi = int(seed), int(tag), psi
        self.G = self.coef = self.len = None

    def c_job(self, n_z: int, gf_steps: int, ctag: int) -> Job:
        n = self.orbs.shape[0]
        npairs = n * (n + 1) // 2
        self.G = np.zeros((max(n_z, 1), n, n), dtype=np.complex128)
        self.coef = np.zeros((npairs, 2, 1 + 2 * gf_steps))
        self.len = np.zeros((npairs, 2), dtype=np.int32)
        j = Job()
        j.model = self.model.c
        j.n_up, j.n_dn, j.n_orb = self.n_up, self.n_dn, n
        j.orbs = self.orbs.ctypes.data_as(_c_i32) if n else None
        j.seed, j.tag = self.seed, ctag
        if n:
            j.h_G = self.G.ctypes.data_as(_c_d) if n_z else None
            j.h_coef = self.coef.ctypes.data_as(_c_d)
            j.h_len = self.len.ctypes.data_as(_c_i32)
        j.d_psi = self.psi.data_ptr() if self.psi is not None else None
        return j

    def result(self, r: JobResult, n_z: int) -> dict:
        return dict(tag=self.tag, e0=r.e0, theta1=r.theta1, residual_est=r.residual_est,
                    true_residual=r.true_residual, n_iter=r.n_iter, converged=bool(r.converged),
                    breakdown=bool(r.breakdown), degenerate_suspect=bool(r.degenerate_suspect),
                    bytes=r.bytes, rounds=r.rounds,
                    G=self.G[:n_z] if self.orbs.shape[0] else None, coef=self.coef, len=self.len,
                    psi=self.psi)


class Engine:
    """A continuously batched solver over one device pool (qcm_engine_*)."""

    def __init__(self, pool_bytes: int, *, device="cuda", stream=None, **opts):
        torch = _torch()
        self.lib = load_library()
        self.o, self._z = engine_opts(**opts)
        self.pool = _workspace(torch, pool_bytes, device)
        self.stream = stream
        self.h = ctypes.c_void_p()
        _check(self.lib.qcm_engine_create(ctypes.byref(self.o), _ptr(self.pool), self.pool.numel(),
                                          _stream(torch, stream), ctypes.byref(self.h)))
        self._jobs = {}
        self._next = 0

    def job_bytes(self, spec: JobSpec) -> int:
        need = ctypes.c_size_t(0)
        j = spec.c_job(self.o.n_z, self.o.gf_steps, 0)
        _check(self.lib.qcm_engine_job_bytes(ctypes.byref(self.o), ctypes.byref(j),
                                             ctypes.byref(need)))
        return need.value

    def submit(self, spec: JobSpec) -> bool:
        """Admit the job if a slot and pool memory are free; False otherwise."""
        ctag = self._next
        j = spec.c_job(self.o.n_z, self.o.gf_steps, ctag)
        rc = self.lib.qcm_engine_submit(self.h, ctypes.byref(j))
        if rc == QCM_EWORKSPACE:
            return False
        _check(rc)
        self._jobs[ctag] = (spec, j)
        self._next += 1
        return True

    def step(self, rounds: int = 1) -> int:
        n = ctypes.c_int32(0)
        _check(self.lib.qcm_engine_step(self.h, rounds, ctypes.byref(n)))
        return n.value

    def poll(self) -> list:
        out = []
        buf = (JobResult * 64)()
        while True:
            k = ctypes.c_int32(0)
            _check(self.lib.qcm_engine_poll(self.h, 64, buf, ctypes.byref(k)))
            for i in range(k.value):
                spec, _ = self._jobs.pop(buf[i].tag)
                out.append(spec.result(buf[i], self.o.n_z))
            if k.value < 64:
                return out

    def info(self) -> dict:
        st = EngineStats()
        _check(self.lib.qcm_engine_info(self.h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in EngineStats._fields_}

    def close(self):
        if self.h:
            _check(self.lib.qcm_engine_destroy(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_solve(specs, *, ws_bytes=None, device="cuda", stream=None, **opts) -> list:
    """Solve every JobSpec through qcm_batch_solve; results in input order."""
    torch = _torch()
    lib = load_library()
    o, zz = engine_opts(**opts)
    n = len(specs)
    jobs = (Job * max(n, 1))()
    for i, sp in enumerate(specs):
        jobs[i] = sp.c_job(o.n_z, o.gf_steps, i)
    res = (JobResult * max(n, 1))()
    need = ctypes.c_size_t(0)
    _check(lib.qcm_batch_solve(ctypes.byref(o), n, jobs, res, None, 0, ctypes.byref(need), None))
    nb = need.value if ws_bytes is None else int(ws_bytes)
    ws = _workspace(torch, nb, device)
    _check(lib.qcm_batch_solve(ctypes.byref(o), n, jobs, res, _ptr(ws), ws.numel(),
                               ctypes.byref(need), _stream(torch, stream)))
    return [specs[i].result(res[i], o.n_z) for i in range(n)]


def batch_bytes(specs, **opts) -> int:
    """Workspace bytes qcm_batch_solve needs to hold every job at once."""
    lib = load_library()
    o, zz = engine_opts(**opts)
    n = len(specs)
    jobs = (Job * max(n, 1))()
    for i, sp in enumerate(specs):
        jobs[i] = sp.c_job(o.n_z, o.gf_steps, i)
    need = ctypes.c_size_t(0)
    _check(lib.qcm_batch_solve(ctypes.byref(o), n, jobs, None, None, 0, ctypes.byref(need), None))
    return need.value


# ---------------------------------------------------------------- symmetry-adapted sectors

class SymSector:
    """The representatives of one irrep of an abelian point group in a sector
    (qcm_sym_sector_build).  perms: [n_g][L] orbital permutations (element 0
    the identity); chi: the irrep's characters (+1/-1).  Keeps the basis and
    the workspace alive."""

    def __init__(self, basis: SectorBasis, perms, chi, stream=None):
        torch = _torch()
        lib = load_library()
        self.basis = basis
        self.perm = np.ascontiguousarray(np.asarray(perms, dtype=np.int32).ravel())
        self.chi_a = np.ascontiguousarray(np.asarray(chi, dtype=np.int32))
        self.g = Group(int(self.chi_a.shape[0]), 0, self.perm.ctypes.data_as(_c_i32),
                       self.chi_a.ctypes.data_as(_c_i32))
        self.c = SymSectorC()
        need = ctypes.c_size_t(0)
        _check(lib.qcm_sym_sector_build(ctypes.byref(basis.c), ctypes.byref(self.g), None, 0,
                                        ctypes.byref(need), ctypes.byref(self.c), None))
        self.ws = _workspace(torch, need.value, basis.device)
        _check(lib.qcm_sym_sector_build(ctypes.byref(basis.c), ctypes.byref(self.g), _ptr(self.ws),
                                        self.ws.numel(), ctypes.byref(need), ctypes.byref(self.c),
                                        _stream(torch, stream)))
        self.device = basis.device

    dim = property(lambda self: self.c.dim)


class SymHamiltonian:
    """The stored matrix of H in a symmetry-adapted sector (qcm_sym_csr_count
    and qcm_sym_csr_fill); call it as H(v) or H(v, w) for w = H v."""

    def __init__(self, model, sector: SymSector, stream=None):
        torch = _torch()
        self.lib = load_library()
        self.m = as_model(model)
        self.sector = sector
        dim = sector.dim
        dev = sector.device
        self.rep = torch.empty(max(dim, 1), dtype=torch.int32, device=dev)
        self.rowptr = torch.empty(dim + 1, dtype=torch.int64, device=dev)
        need = ctypes.c_size_t(0)
        nnz = ctypes.c_int64(0)
        _check(self.lib.qcm_sym_csr_count(ctypes.byref(self.m.c), ctypes.byref(sector.c), None,
                                          None, None, None, 0, ctypes.byref(need), None))
        ws = _workspace(torch, need.value, dev)
        st = _stream(torch, stream)
        _check(self.lib.qcm_sym_csr_count(ctypes.byref(self.m.c), ctypes.byref(sector.c),
                                          _ptr(self.rep), _ptr(self.rowptr), ctypes.byref(nnz),
                                          _ptr(ws), ws.numel(), ctypes.byref(need), st))
        self.nnz = nnz.value
        self.col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        self.val = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev)
        _check(self.lib.qcm_sym_csr_fill(ctypes.byref(self.m.c), ctypes.byref(sector.c),
                                         _ptr(self.rep), _ptr(self.rowptr), _ptr(self.col),
                                         _ptr(self.val), st))
        self.c = SymCsrC(dim, self.nnz, self.rep.data_ptr(), self.rowptr.data_ptr(),
                         self.col.data_ptr(), self.val.data_ptr(), None, None)
        self.dim = dim
        self.device = dev
        self.packed = None
        self.table = None
        self.n_values = 0

    def pack(self, stream=None) -> int:
        """Store one index per value (qcm_sym_csr_pack); afterwards the product
        and the solver read the packed elements.  Returns the number of
        distinct values, or 0 when the matrix does not fit the format (then the
        explicit elements stay in use)."""
        torch = _torch()
        need = ctypes.c_size_t(0)
        _check(self.lib.qcm_sym_csr_pack(ctypes.byref(self.c), None, None, None, None, 0,
                                         ctypes.byref(need), None))
        ws = _workspace(torch, need.value, self.device)
        pk = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.device)
        tab = torch.zeros(64, dtype=torch.float64, device=self.device)
        n = ctypes.c_int32(0)
        _check(self.lib.qcm_sym_csr_pack(ctypes.byref(self.c), _ptr(pk), _ptr(tab), ctypes.byref(n),
                                         _ptr(ws), ws.numel(), ctypes.byref(need),
                                         _stream(torch, stream)))
        self.n_values = n.value
        if n.value:
            self.packed, self.table = pk, tab
            self.c.packed, self.c.table = pk.data_ptr(), tab.data_ptr()
        return n.value

    def unpack(self):
        """Go back to the explicit elements."""
        self.packed = self.table = None
        self.c.packed = self.c.table = None
        self.n_values = 0

    def __call__(self, v, w=None, stream=None):
        torch = _torch()
        if v.dtype != torch.float64 or not v.is_contiguous() or v.numel() % max(self.dim, 1):
            raise ValueError("v must be contiguous float64 with a multiple of dim elements")
        nvec = v.numel() // max(self.dim, 1)
        if w is None:
            w = torch.empty_like(v)
        _check(self.lib.qcm_sym_hv(ctypes.byref(self.c), _ptr(v), _ptr(w), nvec,
                                   _stream(torch, stream)))
        return w


def sym_sector(basis: SectorBasis, perms, chi, stream=None) -> SymSector:
    return SymSector(basis, perms, chi, stream)


def sym_hamiltonian(model, sector: SymSector, stream=None) -> SymHamiltonian:
    return SymHamiltonian(model, sector, stream)


def sym_lanczos_gs(H: SymHamiltonian, *, max_iter=600, fixed_steps=0, want_vector=True,
                   check_every=1, tol=1e-12, btol=1e-13, seed=1, v0=None, stream=None,
                   ws=None) -> dict:
    """Lanczos ground state of a symmetry-adapted sector (FP64); the same
    results as lanczos_gs, psi in the symmetry-adapted basis."""
    torch = _torch()
    lib = load_library()
    o = LanczosOpts()
    lib.qcm_lanczos_default_opts(ctypes.byref(o))
    o.max_iter, o.fixed_steps, o.want_vector = max_iter, fixed_steps, int(want_vector)
    o.check_every, o.tol, o.btol, o.seed = check_every, tol, btol, seed
    if v0 is not None:
        if v0.dtype != torch.float64 or v0.numel() != H.dim:
            raise ValueError("v0 has the wrong dtype or size")
        o.d_v0 = v0.data_ptr()
    need = ctypes.c_size_t(0)
    _check(lib.qcm_sym_lanczos_gs(ctypes.byref(H.c), ctypes.byref(o), None, None, None, None,
                                  None, 0, ctypes.byref(need), None))
    if ws is None or ws.numel() < need.value:
        ws = _workspace(torch, need.value, H.device)
    n = max(max_iter, fixed_steps)
    alpha = np.zeros(n)
    beta = np.zeros(n)
    psi = torch.empty(H.dim, dtype=torch.float64, device=H.device) if want_vector else None
    res = GsResult()
    _check(lib.qcm_sym_lanczos_gs(ctypes.byref(H.c), ctypes.byref(o), alpha.ctypes.data_as(_c_d),
                                  beta.ctypes.data_as(_c_d), _ptr(psi), ctypes.byref(res),
                                  _ptr(ws), ws.numel(), ctypes.byref(need),
                                  _stream(torch, stream)))
    M = res.n_iter
    return dict(e0=res.e0, residual_est=res.residual_est, true_residual=res.true_residual,
                theta1=res.theta1, n_iter=M, converged=bool(res.converged),
                breakdown=bool(res.breakdown), degenerate_suspect=bool(res.degenerate_suspect),
                alpha=alpha[:M], beta=beta[:M], psi=psi)
