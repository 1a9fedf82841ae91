"""Potthoff functional of a cluster reference system on the GPU (paper:
subsection "Practical calculation of the Potthoff functional", eq. (omega4)).

The reference's ground state comes from qcm_lanczos_gs, its Lehmann form
(poles and Q on every cluster orbital) from qcm_green_band, and the k sum of
the pole formula from qcm_vca_omega (or, by the frequency integral of eq.
(sef4), from qcm_vca_omega_quad).  This module is control flow and argument
marshalling.

A problem is any object with t_ref [L, L] (reference hopping, -mu on the
diagonal), U [L], nup, ndn, dt [L, L] (lattice minus reference
intra-cluster matrix) and bonds (inter-cluster, shift in super-lattice
units)."""
from __future__ import annotations

import numpy as np

from . import _binding as B


def reference_lehmann(prob, *, max_basis=1000):
    """(E0, poles [R], Q [L, R]) of the reference's up-spin Green function."""
    L = np.asarray(prob.t_ref).shape[0]
    model = (prob.t_ref, prob.U)
    basis = B.sector_basis(L, prob.nup, prob.ndn)
    gs = B.lanczos_gs(model, basis)
    g = B.green_band(model, basis, gs["psi"], gs["e0"], list(range(L)), np.array([1j]),
                     max_basis=max_basis)
    return gs["e0"], g["poles"], g["Q_lehmann"]


def omega(prob, ks, *, max_basis=1000, method="poles", rtol=1e-12):
    """The functional (both spins) on the wave-vectors ks, by the pole formula
    (method "poles") or the adaptive frequency integral ("quad")."""
    e0, poles, Q = reference_lehmann(prob, max_basis=max_basis)
    if method == "quad":
        om, _, _ = B.vca_omega_quad(e0, poles, Q, prob.dt, prob.bonds, ks, rtol=rtol)
        return om
    if method != "poles":
        raise ValueError(f"unknown method {method!r}")
    om, _ = B.vca_omega(e0, poles, Q, prob.dt, prob.bonds, ks)
    return om
