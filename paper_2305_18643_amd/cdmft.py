"""CDMFT self-consistency on the GPU (paper: section "Cellular dynamical
mean-field theory", subsection "The CDMFT self-consistent procedure").

Each iteration: the impurity (cluster plus bath, eq. (cdmft1)) is solved
with qcm_lanczos_gs and qcm_green_cf on the cluster orbitals at the
distance function's frequencies; qcm_cdmft_g0inv gives Sigma_c, the
super-lattice average Gbar and calG0^{-1}; qcm_cdmft_fit moves the bath
parameters to the minimum of the distance function (eq. (dist_func)).  The
loop stops when no parameter moves by more than `tol`.

This module is control flow and argument marshalling (it places the bath
parameters into the impurity's hopping matrix); the arithmetic runs in the
library's kernels.

A problem is any object with the attributes
  tc [L, L] (cluster hopping without mu), mu, U (on every cluster site),
  nup, ndn (sector of the impurity), A_eps [n_bath, n_par],
  A_theta [L * n_bath, n_par] (eps = A_eps p, theta = (A_theta p).reshape(L, n_bath)),
  bonds (inter-cluster bonds (i, j, shift, t), shift in super-lattice units).
"""
from __future__ import annotations

import time

import numpy as np

from . import _binding as B


def bath_arrays(prob, p):
    """(theta [L, n_bath], eps [n_bath]) from the parameters."""
    p = np.asarray(p, dtype=np.float64)
    L = prob.tc.shape[0]
    eps = np.asarray(prob.A_eps, dtype=np.float64) @ p
    theta = (np.asarray(prob.A_theta, dtype=np.float64) @ p).reshape(L, -1)
    return theta, eps


def impurity_arrays(prob, p):
    """(t, U) of the impurity: cluster orbitals first, bath after them."""
    theta, eps = bath_arrays(prob, p)
    L, nb = theta.shape
    t = np.zeros((L + nb, L + nb))
    t[:L, :L] = np.asarray(prob.tc, dtype=np.float64) - prob.mu * np.eye(L)
    t[L:, L:] = np.diag(eps)
    t[:L, L:] = theta
    t[L:, :L] = theta.T
    U = np.concatenate([np.full(L, float(prob.U)), np.zeros(nb)])
    return t, U


def cdmft(prob, p0, ks, z, w, *, max_iter=40, tol=1e-6, max_steps=200, gtol=1e-10,
          fit_iter=500, callback=None):
    """Run the self-consistent loop from the parameters p0 on the frequency
    grid z (weights w) with the super-lattice wave-vectors ks.  Returns a dict
    with the parameters p, their history, iterations, converged, the last
    distance, E0, the device tensors Gc, sigma, gbar, g0inv of the last
    iteration, and the time spent per iteration."""
    L = prob.tc.shape[0]
    nb = np.asarray(prob.A_eps).shape[0]
    tcp = np.asarray(prob.tc, dtype=np.float64) - prob.mu * np.eye(L)
    basis = B.sector_basis(L + nb, prob.nup, prob.ndn)
    p = np.asarray(p0, dtype=np.float64).copy()
    hist, times = [p.copy()], []
    out = {}
    for it in range(1, max_iter + 1):
        t0 = time.perf_counter()
        t, U = impurity_arrays(prob, p)
        gs = B.lanczos_gs((t, U), basis)
        g = B.green_cf((t, U), basis, gs["psi"], gs["e0"], list(range(L)), z, max_steps=max_steps)
        theta, eps = bath_arrays(prob, p)
        o = B.cdmft_g0inv(g["G"], tcp, theta, eps, prob.bonds, ks, z)
        pn, d, nit = B.cdmft_fit(o["g0inv"], tcp, prob.A_eps, prob.A_theta, p, z, w, gtol=gtol,
                                 max_iter=fit_iter)
        times.append(time.perf_counter() - t0)
        hist.append(pn.copy())
        out = dict(Gc=g["G"], e0=gs["e0"], distance=d, fit_steps=nit, **o)
        moved = float(np.max(np.abs(pn - p)))
        p = pn
        if callback is not None:
            callback(it, p, d, moved)
        if moved <= tol:
            return dict(p=p, history=hist, iterations=it, converged=True, times=times, **out)
    return dict(p=p, history=hist, iterations=max_iter, converged=False, times=times, **out)
