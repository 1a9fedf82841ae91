"""MI355X-native exact-diagonalisation hot path of the Pyqcm paper
(arXiv 2305.18643): sector basis, H.v, Lanczos ground state, continued-
fraction Green function, band Lanczos Green function, CPT, the CDMFT
self-consistency, the Potthoff functional of VCA and symmetry-adapted sectors
with a stored Hamiltonian, as hand-written HIP kernels for gfx950 behind a C ABI
(include/qcm.h).  This package is the thin Python binding."""
from ._binding import (EXPORTS, PREC, QCM_FP32V, QCM_FP64, Engine, HostModel, HvPlan, JobSpec,
                       QcmError, SectorBasis, as_model, batch_bytes, batch_solve, cdmft_fit,
                       cdmft_g0inv, cpt_gk, green_band, green_cf, hv, hv_noalloc, lanczos_gs,
                       load_library,
                       sector_basis, sym_hamiltonian, sym_lanczos_gs, sym_sector, vca_omega,
                       vca_omega_quad)
from .cdmft import cdmft
from . import vca

__all__ = ["EXPORTS", "PREC", "QCM_FP32V", "QCM_FP64", "Engine", "HostModel", "HvPlan", "JobSpec",
           "QcmError", "SectorBasis", "as_model", "batch_bytes", "batch_solve", "cdmft", "cdmft_fit",
           "cdmft_g0inv", "cpt_gk",
           "green_band", "green_cf", "hv", "hv_noalloc", "lanczos_gs", "load_library", "sector_basis",
           "sym_hamiltonian", "sym_lanczos_gs", "sym_sector", "vca", "vca_omega",
           "vca_omega_quad"]
