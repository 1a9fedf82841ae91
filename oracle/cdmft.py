"""CDMFT self-consistency for the oracle (TEST INFRASTRUCTURE ONLY; see the
package docstring).  NumPy, FP64, complex128; the impurity is solved by the
oracle's own Lanczos ground state and continued fractions (oracle/ora.c and
oracle/cf.py), or by dense diagonalisation for the pins.

Follows the paper's section "Cellular dynamical mean-field theory":
  * the bath enters through the hybridization function
    Gamma(z) = sum_alpha theta[:, alpha] theta[:, alpha]^T / (z - eps_alpha)
    (eq. (hybridization), real theta), so that
    G_c^{-1}(z) = z - t_c' - Gamma(z) - Sigma_c(z), with t_c' the cluster
    hopping with -mu on its diagonal (the self-energy is what the
    interaction adds);
  * subsection "The CDMFT self-consistent procedure": from the cluster Green
    function of the impurity, the super-lattice average
    Gbar(z) = (1/N) sum_k [z - t_c' - V(k) - Sigma_c(z)]^{-1}
    (G_0^{-1}(k) = z + mu - t(k) with t(k) = t_c + V(k)), and
    calG0^{-1}(z) = Gbar^{-1}(z) + Sigma_c(z);
  * the distance function eq. (dist_func)
    d = sum_n W_n sum_{nu,nu'} |(i w_n - t_c' - Gamma(i w_n) - calG0^{-1})_{nu nu'}|^2
    minimised over the bath parameters (the minimiser is a library
    routine: scipy's BFGS on the analytic gradient);
  * then back to the impurity solution with the new bath, until the bath
    parameters stop moving.

The super-lattice Fourier transform follows the same bond convention as the
CPT oracle (oracle/cf.py, v_of_k): a bond (i, j, s, t) is the amplitude t
between site i of the cluster at the origin and site j of the cluster at
shift s, its Hermitian partner added; here k is given in units of 2 pi in
the basis reciprocal to the super-lattice vectors, so the phase is
exp(2 pi i k . s).
"""
from __future__ import annotations

import numpy as np


def bath_of(setup, p):
    """(theta [L, n_bath], eps [n_bath]) from the variational parameters."""
    p = np.asarray(p, dtype=np.float64)
    eps = setup.A_eps @ p
    theta = (setup.A_theta @ p).reshape(setup.L, setup.n_bath)
    return theta, eps


def hybridization(theta, eps, z):
    """Gamma[z, L, L] = sum_alpha theta_mu,alpha theta_nu,alpha / (z - eps_alpha)."""
    z = np.asarray(z, dtype=np.complex128)
    G = np.zeros((z.shape[0], theta.shape[0], theta.shape[0]), dtype=np.complex128)
    for a in range(theta.shape[1]):
        G += np.outer(theta[:, a], theta[:, a])[None] / (z - eps[a])[:, None, None]
    return G


def tc_prime(setup):
    """Cluster hopping with -mu on the diagonal."""
    return setup.tc - setup.mu * np.eye(setup.L)


def impurity(setup, p):
    """(t, U) of the impurity: cluster orbitals first, then the bath."""
    theta, eps = bath_of(setup, p)
    L, nb = setup.L, setup.n_bath
    t = np.zeros((L + nb, L + nb))
    t[:L, :L] = tc_prime(setup)
    t[L:, L:] = np.diag(eps)
    t[:L, L:] = theta
    t[L:, :L] = theta.T
    U = np.concatenate([np.full(L, float(setup.U)), np.zeros(nb)])
    return t, U


def cluster_green(setup, p, z, max_steps=200, nthreads=1):
    """The impurity's up-spin Green function on the cluster orbitals at z:
    Lanczos ground state of the (nup, ndn) sector, then continued fractions
    for every pair of cluster orbitals.  Returns (Gc [z, L, L], E0)."""
    import oracle
    from oracle import cf
    t, U = impurity(setup, p)
    gs = oracle.lanczos_gs(t, U, setup.nup, setup.ndn, want_vector=True, nthreads=nthreads)
    ch = oracle.green_cf(t, U, setup.nup, setup.ndn, gs["psi"], list(range(setup.L)),
                         max_steps=max_steps, nthreads=nthreads)
    return cf.green_matrix(ch, setup.L, np.asarray(z), gs["e0"]), gs["e0"]


def sigma(setup, p, z, Gc):
    """Sigma_c(z) = z - t_c' - Gamma(z) - G_c^{-1}(z)."""
    theta, eps = bath_of(setup, p)
    gam = hybridization(theta, eps, z)
    zI = np.asarray(z)[:, None, None] * np.eye(setup.L)[None]
    return zI - tc_prime(setup)[None] - gam - np.linalg.inv(Gc)


def v_of_k(L, bonds, k):
    """V(k) [L, L], phase exp(2 pi i k . s) for a bond at super-lattice shift s."""
    V = np.zeros((L, L), dtype=np.complex128)
    for (i, j, s, t) in bonds:
        ph = np.exp(2j * np.pi * np.dot(np.asarray(k, dtype=np.float64), np.asarray(s, dtype=np.float64)))
        V[i, j] += t * ph
        V[j, i] += t * np.conj(ph)
    return V


def gbar(setup, z, sig, ks):
    """Gbar(z) = (1/N) sum_k [z - t_c' - V(k) - Sigma_c(z)]^{-1}."""
    z = np.asarray(z, dtype=np.complex128)
    L = setup.L
    out = np.zeros((z.shape[0], L, L), dtype=np.complex128)
    tcp = tc_prime(setup)
    for k in ks:
        V = v_of_k(L, setup.bonds, k)
        for iz in range(z.shape[0]):
            out[iz] += np.linalg.inv(z[iz] * np.eye(L) - tcp - V - sig[iz])
    return out / len(ks)


def g0inv(gb, sig):
    """calG0^{-1}(z) = Gbar^{-1}(z) + Sigma_c(z)."""
    return np.linalg.inv(gb) + sig


def distance(setup, p, z, w, G0i):
    """d = sum_n w_n || z_n - t_c' - Gamma(z_n) - calG0^{-1}(z_n) ||_F^2."""
    theta, eps = bath_of(setup, p)
    A = (np.asarray(z)[:, None, None] * np.eye(setup.L)[None] - tc_prime(setup)[None]
         - hybridization(theta, eps, z) - G0i)
    return float(np.sum(np.asarray(w)[:, None, None] * np.abs(A) ** 2))


def distance_grad(setup, p, z, w, G0i):
    """Analytic gradient of `distance` in p (chain rule through theta, eps):
    dGamma/deps_a = theta_a theta_a^T / (z - eps_a)^2,
    dGamma_{nu nu'}/dtheta_{mu a} = (delta_{nu mu} theta_{nu' a} + theta_{nu a} delta_{nu' mu}) / (z - eps_a)."""
    theta, eps = bath_of(setup, p)
    L, nb = setup.L, setup.n_bath
    z = np.asarray(z)
    A = (z[:, None, None] * np.eye(L)[None] - tc_prime(setup)[None]
         - hybridization(theta, eps, z) - G0i)
    wA = np.asarray(w)[:, None, None] * np.conj(A)          # d = sum w conj(A) A
    g_eps = np.zeros(nb)
    g_theta = np.zeros((L, nb))
    for a in range(nb):
        inv = 1.0 / (z - eps[a])
        dG = np.outer(theta[:, a], theta[:, a])[None] * (inv ** 2)[:, None, None]
        g_eps[a] = -2.0 * np.real(np.sum(wA * dG))
        # dd/dtheta_{mu a} = -2 Re sum_n w_n sum_{nu'} [conj(A)_{mu nu'} + conj(A)_{nu' mu}] theta_{nu' a} / (z - eps_a)
        S = np.sum((wA + np.transpose(wA, (0, 2, 1))) * inv[:, None, None], axis=0)   # [L, L]
        g_theta[:, a] = -2.0 * np.real(S @ theta[:, a])
    return setup.A_eps.T @ g_eps + setup.A_theta.T @ g_theta.ravel()


def fit(setup, p0, z, w, G0i, gtol=1e-10, maxiter=500):
    """Bath parameters minimising the distance function (scipy BFGS)."""
    from scipy.optimize import minimize
    r = minimize(lambda q: distance(setup, q, z, w, G0i), np.asarray(p0, dtype=np.float64),
                 jac=lambda q: distance_grad(setup, q, z, w, G0i), method="BFGS",
                 options={"gtol": gtol, "maxiter": maxiter})
    return r.x, float(r.fun), int(r.nit)


def cdmft(setup, p0, ks, max_iter=40, tol=1e-6, max_steps=200, nthreads=1):
    """The self-consistent loop: solve, Sigma_c, Gbar, calG0^{-1}, fit, until
    max |p_new - p| <= tol.  Returns dict(p, history, iterations, converged,
    distance, Gc, sigma, gbar, g0inv, e0)."""
    z = synth_grid(setup)
    w = np.full(z.shape[0], 1.0 / z.shape[0])
    p = np.asarray(p0, dtype=np.float64).copy()
    hist = [p.copy()]
    out = {}
    for it in range(1, max_iter + 1):
        Gc, e0 = cluster_green(setup, p, z, max_steps=max_steps, nthreads=nthreads)
        sig = sigma(setup, p, z, Gc)
        gb = gbar(setup, z, sig, ks)
        G0i = g0inv(gb, sig)
        pn, d, _ = fit(setup, p, z, w, G0i)
        hist.append(pn.copy())
        out = dict(Gc=Gc, sigma=sig, gbar=gb, g0inv=G0i, e0=e0, distance=d)
        done = np.max(np.abs(pn - p)) <= tol
        p = pn
        if done:
            return dict(p=p, history=hist, iterations=it, converged=True, **out)
    return dict(p=p, history=hist, iterations=max_iter, converged=False, **out)


def synth_grid(setup):
    """The distance function's Matsubara frequencies (beta, cutoff of the setup)."""
    n = np.arange(int(np.floor((setup.wc * setup.beta / np.pi - 1.0) / 2.0)) + 1)
    return 1j * (2 * n + 1) * np.pi / setup.beta
