// CDMFT self-consistency on the device (paper: section "Cellular dynamical
// mean-field theory", eq. (hybridization) and subsection "The CDMFT
// self-consistent procedure", eq. (dist_func)).
//
//  * k_cdmft_g0inv, one workgroup per frequency: Gamma(z) from the bath,
//    Sigma_c = z - tcp - Gamma - G_c^-1, then the super-lattice average
//    Gbar = (1/n_k) sum_k [z - tcp - V(k) - Sigma_c]^-1 (one thread per k
//    point inverts its own L x L matrix; the sum is a fixed-order reduction)
//    and calG0^-1 = Gbar^-1 + Sigma_c.
//  * k_cdmft_fit, one workgroup: BFGS on the distance function
//    d(p) = sum_n w_n || z_n - tcp - Gamma(z_n; p) - calG0^-1(z_n) ||_F^2,
//    the threads sharing the entries (frequency, row, column) for d and its
//    analytic gradient (partial sums in a per-thread row of an LDS table,
//    summed by column in a fixed order), thread 0 doing the small dense
//    algebra (direction, line search bookkeeping, inverse-Hessian update)
//    between barriers.
#include <math.h>
#include <string.h>

#include <vector>

#include "lanczos_device.h"
#include "qcm_internal.h"

namespace qcm {

constexpr int kCL = QCM_CDMFT_MAX_L;
constexpr int kCB = QCM_CDMFT_MAX_BATH;
constexpr int kCP = QCM_CDMFT_MAX_PAR;

struct CBond {
    int32_t i, j;
    double s0, s1, s2, t;
};

// Inverse of the n x n complex matrix (ar, ai) (row-major, destroyed) into
// (xr, xi) by Gauss-Jordan elimination with partial pivoting.  One thread.
// Returns false when a pivot is exactly zero.
__device__ bool cinv(int n, double *ar, double *ai, double *xr, double *xi) {
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            xr[r * n + c] = r == c ? 1.0 : 0.0;
            xi[r * n + c] = 0.0;
        }
    for (int p = 0; p < n; ++p) {
        int best = p;
        double bm = -1.0;
        for (int r = p; r < n; ++r) {
            const double m = hypot(ar[r * n + p], ai[r * n + p]);
            if (m > bm) {
                bm = m;
                best = r;
            }
        }
        if (!(bm > 0.0)) return false;
        if (best != p)
            for (int c = 0; c < n; ++c) {
                double t0 = ar[p * n + c], t1 = ai[p * n + c];
                ar[p * n + c] = ar[best * n + c];
                ai[p * n + c] = ai[best * n + c];
                ar[best * n + c] = t0;
                ai[best * n + c] = t1;
                t0 = xr[p * n + c];
                t1 = xi[p * n + c];
                xr[p * n + c] = xr[best * n + c];
                xi[p * n + c] = xi[best * n + c];
                xr[best * n + c] = t0;
                xi[best * n + c] = t1;
            }
        const double pr = ar[p * n + p], pi = ai[p * n + p];
        const double den = pr * pr + pi * pi;
        const double ir = pr / den, ii = -pi / den;  // 1 / pivot
        for (int c = 0; c < n; ++c) {
            double a = ar[p * n + c], b = ai[p * n + c];
            ar[p * n + c] = a * ir - b * ii;
            ai[p * n + c] = a * ii + b * ir;
            a = xr[p * n + c];
            b = xi[p * n + c];
            xr[p * n + c] = a * ir - b * ii;
            xi[p * n + c] = a * ii + b * ir;
        }
        for (int r = 0; r < n; ++r) {
            if (r == p) continue;
            const double fr = ar[r * n + p], fi = ai[r * n + p];
            if (fr == 0.0 && fi == 0.0) continue;
            for (int c = 0; c < n; ++c) {
                ar[r * n + c] -= fr * ar[p * n + c] - fi * ai[p * n + c];
                ai[r * n + c] -= fr * ai[p * n + c] + fi * ar[p * n + c];
                xr[r * n + c] -= fr * xr[p * n + c] - fi * xi[p * n + c];
                xi[r * n + c] -= fr * xi[p * n + c] + fi * xr[p * n + c];
            }
        }
    }
    return true;
}

// Gamma_{mu nu}(z) = sum_a theta[mu][a] theta[nu][a] / (z - eps_a)
__device__ inline void gamma_entry(int nb, const double *th_mu, const double *th_nu,
                                   const double *eps, double zr, double zi, double *gr,
                                   double *gi) {
    double r = 0.0, i = 0.0;
    for (int a = 0; a < nb; ++a) {
        const double dr = zr - eps[a], den = dr * dr + zi * zi;
        const double w = th_mu[a] * th_nu[a] / den;
        r += w * dr;
        i -= w * zi;
    }
    *gr = r;
    *gi = i;
}

__global__ void __launch_bounds__(256) k_cdmft_g0inv(
    int L, int nb, const double *__restrict__ tcp, const double *__restrict__ theta,
    const double *__restrict__ eps, const CBond *__restrict__ bonds, int nbonds,
    const double *__restrict__ ks, int nk, const double *__restrict__ zs,
    const double *__restrict__ Gc, double *__restrict__ sig_o, double *__restrict__ gbar_o,
    double *__restrict__ g0i_o, int32_t *__restrict__ bad) {
    __shared__ double sr[kCL * kCL], si[kCL * kCL], gbr[kCL * kCL], gbi[kCL * kCL];
    __shared__ double red[256];
    const int t = threadIdx.x, iz = blockIdx.x, n2 = L * L;
    const double zr = zs[2 * iz], zi = zs[2 * iz + 1];
    if (t == 0) {
        double ar[kCL * kCL], ai[kCL * kCL], xr[kCL * kCL], xi[kCL * kCL];
        const double *g = Gc + 2 * (size_t)n2 * iz;
        for (int e = 0; e < n2; ++e) {
            ar[e] = g[2 * e];
            ai[e] = g[2 * e + 1];
        }
        if (!cinv(L, ar, ai, xr, xi)) bad[iz] |= 1;
        for (int m = 0; m < L; ++m)
            for (int n = 0; n < L; ++n) {
                double gr, gi;
                gamma_entry(nb, theta + m * nb, theta + n * nb, eps, zr, zi, &gr, &gi);
                const int e = m * L + n;
                sr[e] = (m == n ? zr : 0.0) - tcp[e] - gr - xr[e];
                si[e] = (m == n ? zi : 0.0) - gi - xi[e];
            }
    }
    __syncthreads();
    double pr[kCL * kCL], pi[kCL * kCL];
    for (int e = 0; e < n2; ++e) pr[e] = pi[e] = 0.0;
    for (int k = t; k < nk; k += 256) {
        double ar[kCL * kCL], ai[kCL * kCL], xr[kCL * kCL], xi[kCL * kCL];
        for (int m = 0; m < L; ++m)
            for (int n = 0; n < L; ++n) {
                const int e = m * L + n;
                ar[e] = (m == n ? zr : 0.0) - tcp[e] - sr[e];
                ai[e] = (m == n ? zi : 0.0) - si[e];
            }
        const double k0 = ks[3 * k], k1 = ks[3 * k + 1], k2 = ks[3 * k + 2];
        for (int q = 0; q < nbonds; ++q) {
            const CBond b = bonds[q];
            const double ph = 2.0 * M_PI * (k0 * b.s0 + k1 * b.s1 + k2 * b.s2);
            const double c = cos(ph), s = sin(ph);
            // subtract V: V_ij += t e^{i ph}, V_ji += t e^{-i ph}
            ar[b.i * L + b.j] -= b.t * c;
            ai[b.i * L + b.j] -= b.t * s;
            ar[b.j * L + b.i] -= b.t * c;
            ai[b.j * L + b.i] += b.t * s;
        }
        if (!cinv(L, ar, ai, xr, xi)) atomicOr(bad + iz, 2);
        for (int e = 0; e < n2; ++e) {
            pr[e] += xr[e];
            pi[e] += xi[e];
        }
    }
    for (int e = 0; e < n2; ++e) {
        const double s0 = block_sum(pr[e], red);
        const double s1 = block_sum(pi[e], red);
        if (t == 0) {
            gbr[e] = s0 / nk;
            gbi[e] = s1 / nk;
        }
    }
    __syncthreads();
    if (t == 0) {
        double ar[kCL * kCL], ai[kCL * kCL], xr[kCL * kCL], xi[kCL * kCL];
        for (int e = 0; e < n2; ++e) {
            ar[e] = gbr[e];
            ai[e] = gbi[e];
        }
        if (!cinv(L, ar, ai, xr, xi)) bad[iz] |= 4;
        const size_t o = 2 * (size_t)n2 * iz;
        for (int e = 0; e < n2; ++e) {
            if (sig_o) {
                sig_o[o + 2 * e] = sr[e];
                sig_o[o + 2 * e + 1] = si[e];
            }
            if (gbar_o) {
                gbar_o[o + 2 * e] = gbr[e];
                gbar_o[o + 2 * e + 1] = gbi[e];
            }
            g0i_o[o + 2 * e] = xr[e] + sr[e];
            g0i_o[o + 2 * e + 1] = xi[e] + si[e];
        }
    }
}

// ---------------------------------------------------------------- the fit

struct FitArgs {
    int L, nb, np, nz, max_iter;
    double gtol;
    const double *A_eps, *A_theta, *tcp, *zs, *w, *g0i;
    double *p, *out;  // p in/out [np]; out = {d, iterations}
};

// d(pp) and its gradient (into grad, LDS) by all threads; theta/eps in LDS.
// A thread takes the entries (n, m, q) of A(z_n) = z_n - tcp - Gamma - calG0^-1
// with index = thread + k * 256 and keeps its partial sums in its own row of
// `part` (np gradient components, then d); the columns are then summed in a
// fixed order, so the result depends only on the inputs.
constexpr int kPartW = kCP + 1;

__device__ double fit_eval(const FitArgs &a, const double *pp, double *grad, double *th,
                           double *ep, double *part) {
    const int t = threadIdx.x, L = a.L, nb = a.nb, np = a.np, n2 = L * L;
    for (int e = t; e < nb; e += blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < np; ++j) s += a.A_eps[e * np + j] * pp[j];
        ep[e] = s;
    }
    for (int e = t; e < L * nb; e += blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < np; ++j) s += a.A_theta[e * np + j] * pp[j];
        th[e] = s;
    }
    double *row = part + (size_t)t * kPartW;
    for (int j = 0; j <= np; ++j) row[j] = 0.0;
    __syncthreads();
    for (int item = t; item < a.nz * n2; item += blockDim.x) {
        const int n = item / n2, e = item - n * n2, m = e / L, q = e - m * L;
        const double zr = a.zs[2 * n], zi = a.zs[2 * n + 1], wn = a.w[n];
        const double *G = a.g0i + 2 * (size_t)n2 * n;
        double gr, gi;
        gamma_entry(nb, th + m * nb, th + q * nb, ep, zr, zi, &gr, &gi);
        const double Ar = (m == q ? zr : 0.0) - a.tcp[e] - gr - G[2 * e];
        const double Ai = (m == q ? zi : 0.0) - gi - G[2 * e + 1];
        row[np] += wn * (Ar * Ar + Ai * Ai);
        // w conj(A)
        const double cr = wn * Ar, ci = -wn * Ai;
        for (int b = 0; b < nb; ++b) {
            // 1/(z - eps_b) = (dr - i zi) / den
            const double dr = zr - ep[b], den = dr * dr + zi * zi;
            const double ir = dr / den, ii = -zi / den;
            // d/deps_b: -2 Re(wcA theta_mb theta_qb / (z - eps_b)^2)
            const double i2r = ir * ir - ii * ii, i2i = 2.0 * ir * ii;
            const double ge = -2.0 * th[m * nb + b] * th[q * nb + b] * (cr * i2r - ci * i2i);
            // d/dtheta_{m b}: -2 Re(wcA theta_qb / (z - eps_b)); d/dtheta_{q b}: with theta_mb
            const double re1 = cr * ir - ci * ii;
            const double gtm = -2.0 * th[q * nb + b] * re1;
            const double gtq = -2.0 * th[m * nb + b] * re1;
            for (int j = 0; j < np; ++j)
                row[j] += a.A_eps[b * np + j] * ge + a.A_theta[(m * nb + b) * np + j] * gtm +
                          a.A_theta[(q * nb + b) * np + j] * gtq;
        }
    }
    __syncthreads();
    __shared__ double dsum;
    for (int j = t; j <= np; j += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < (int)blockDim.x; ++k) s += part[(size_t)k * kPartW + j];
        if (j < np)
            grad[j] = s;
        else
            dsum = s;
    }
    __syncthreads();
    return dsum;
}

__global__ void __launch_bounds__(256) k_cdmft_fit(FitArgs a) {
    __shared__ double p[kCP], g[kCP], pt[kCP], gt[kCP], dir[kCP], sv[kCP], yv[kCP], hy[kCP];
    __shared__ double H[kCP * kCP];
    __shared__ double th[kCL * kCB], ep[kCB];
    __shared__ double part[256 * kPartW];
    __shared__ double d_sh, dt_sh, alpha_sh, slope_sh;
    __shared__ int state;  // 0 continue, 1 converged, 2 line search failed (3, 4 in the search)
    __shared__ bool stall;  // the last step did not lower d
    const int t = threadIdx.x, np = a.np;
    if (t == 0) stall = false;
    for (int j = t; j < np; j += blockDim.x) p[j] = a.p[j];
    for (int e = t; e < np * np; e += blockDim.x) H[e] = (e / np == e % np) ? 1.0 : 0.0;
    __syncthreads();
    double d = fit_eval(a, p, g, th, ep, part);
    int it = 0;
    bool first = true;
    for (; it < a.max_iter; ++it) {
        if (t == 0) {
            double gmax = 0.0;
            for (int j = 0; j < np; ++j) gmax = fmax(gmax, fabs(g[j]));
            state = (gmax <= a.gtol || stall) ? 1 : 0;
            // direction -H g; a non-descent direction restarts from -g
            double slope = 0.0;
            for (int i = 0; i < np; ++i) {
                double s = 0.0;
                for (int j = 0; j < np; ++j) s -= H[i * np + j] * g[j];
                dir[i] = s;
                slope += g[i] * s;
            }
            if (!(slope < 0.0)) {
                slope = 0.0;
                for (int i = 0; i < np; ++i) {
                    for (int j = 0; j < np; ++j) H[i * np + j] = i == j ? 1.0 : 0.0;
                    dir[i] = -g[i];
                    slope -= g[i] * g[i];
                }
            }
            slope_sh = slope;
            alpha_sh = 1.0;
            d_sh = d;
        }
        __syncthreads();
        if (state != 0) break;
        // backtracking line search (Armijo)
        bool ok = false;
        for (int ls = 0; ls < 60; ++ls) {
            for (int j = t; j < np; j += blockDim.x) pt[j] = p[j] + alpha_sh * dir[j];
            __syncthreads();
            const double dt = fit_eval(a, pt, gt, th, ep, part);
            if (t == 0) {
                dt_sh = dt;
                state = dt <= d_sh + 1e-4 * alpha_sh * slope_sh ? 3 : 0;
                if (state == 0) {
                    // a trial step below the resolution of p ends the fit there
                    double dm = 0.0, pm = 1.0;
                    for (int j = 0; j < np; ++j) {
                        dm = fmax(dm, fabs(alpha_sh * dir[j]));
                        pm = fmax(pm, fabs(p[j]));
                    }
                    if (dm <= 1e-15 * pm) state = 4;
                    alpha_sh *= 0.5;
                }
            }
            __syncthreads();
            if (state == 3) {
                ok = true;
                break;
            }
            if (state == 4) break;
        }
        if (state == 4) {
            if (t == 0) state = 1;
            __syncthreads();
            break;
        }
        if (!ok) {
            if (t == 0) state = 2;
            __syncthreads();
            break;
        }
        if (t == 0) {
            // s = pt - p, y = gt - g; inverse-Hessian BFGS update
            double sy = 0.0, yy = 0.0;
            for (int j = 0; j < np; ++j) {
                sv[j] = pt[j] - p[j];
                yv[j] = gt[j] - g[j];
                sy += sv[j] * yv[j];
                yy += yv[j] * yv[j];
            }
            if (sy > 1e-300) {
                if (first) {  // scale the initial inverse Hessian by s.y / y.y
                    const double sc = sy / yy;
                    for (int e = 0; e < np * np; ++e) H[e] *= sc;
                }
                const double rho = 1.0 / sy;
                double yHy = 0.0;
                for (int i = 0; i < np; ++i) {
                    double s = 0.0;
                    for (int j = 0; j < np; ++j) s += H[i * np + j] * yv[j];
                    hy[i] = s;
                    yHy += yv[i] * s;
                }
                // H += rho (1 + rho yHy) s s^T - rho (Hy s^T + s (Hy)^T)
                for (int i = 0; i < np; ++i)
                    for (int j = 0; j < np; ++j)
                        H[i * np + j] += rho * (1.0 + rho * yHy) * sv[i] * sv[j] -
                                         rho * (hy[i] * sv[j] + sv[i] * hy[j]);
            }
            for (int j = 0; j < np; ++j) {
                p[j] = pt[j];
                g[j] = gt[j];
            }
            stall = !(d_sh - dt_sh > 1e-15 * fabs(d_sh));
            d_sh = dt_sh;
        }
        __syncthreads();
        d = d_sh;
        first = false;
    }
    if (t == 0) {
        for (int j = 0; j < np; ++j) a.p[j] = p[j];
        a.out[0] = d;
        a.out[1] = state == 2 ? -(double)(it + 1) : (double)it;
    }
}

}  // namespace qcm

using namespace qcm;

static int check_common(const char *who, int32_t L, int32_t nb, const double *tcp, int32_t n_z,
                        const double *h_z) {
    if (L < 1 || L > kCL) return fail(QCM_ERANGE, "%s: L=%d outside 1..%d", who, L, kCL);
    if (nb < 0 || nb > kCB) return fail(QCM_ERANGE, "%s: n_bath=%d outside 0..%d", who, nb, kCB);
    if (!tcp) return fail(QCM_EARG, "%s: tcp is NULL", who);
    if (n_z < 1 || !h_z) return fail(QCM_EARG, "%s: need n_z >= 1 frequencies", who);
    return QCM_OK;
}

extern "C" int qcm_cdmft_g0inv(int32_t L, int32_t n_bath, const double *h_tcp,
                               const double *h_theta, const double *h_eps, int32_t n_bonds,
                               const qcm_bond *h_bonds, int32_t n_k, const double *h_k,
                               int32_t n_z, const double *h_z, const double *d_Gc,
                               double *d_sigma, double *d_gbar, double *d_g0inv, void *d_ws,
                               size_t ws_bytes, size_t *ws_needed, void *stream) {
    const char *who = "qcm_cdmft_g0inv";
    if (!ws_needed) return fail(QCM_EARG, "%s: ws_needed is NULL", who);
    QCM_TRY(check_common(who, L, n_bath, h_tcp, n_z, h_z));
    if (n_bath > 0 && (!h_theta || !h_eps)) return fail(QCM_EARG, "%s: NULL bath arrays", who);
    if (n_bonds < 0 || (n_bonds > 0 && !h_bonds)) return fail(QCM_EARG, "%s: bad bonds", who);
    if (n_k < 1 || !h_k) return fail(QCM_EARG, "%s: need n_k >= 1 wave-vectors", who);
    for (int q = 0; q < n_bonds; ++q)
        if (h_bonds[q].i < 0 || h_bonds[q].i >= L || h_bonds[q].j < 0 || h_bonds[q].j >= L)
            return fail(QCM_EARG, "%s: bond %d has a site out of range", who, q);
    auto layout = [&](Carver &cv, double **tcp, double **th, double **ep, CBond **bd,
                      double **kd, double **zd, int32_t **bad) {
        *tcp = cv.take<double>((size_t)L * L);
        *th = cv.take<double>((size_t)L * (n_bath > 0 ? n_bath : 1));
        *ep = cv.take<double>(n_bath > 0 ? n_bath : 1);
        *bd = cv.take<CBond>(n_bonds > 0 ? n_bonds : 1);
        *kd = cv.take<double>(3 * (size_t)n_k);
        *zd = cv.take<double>(2 * (size_t)n_z);
        *bad = cv.take<int32_t>(n_z);
    };
    double *tcp, *th, *ep, *kd, *zd;
    CBond *bd;
    int32_t *bad;
    Carver dry(nullptr);
    layout(dry, &tcp, &th, &ep, &bd, &kd, &zd, &bad);
    const size_t need = dry.off + 256;
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (ws_bytes < need) return fail(QCM_EWORKSPACE, "%s: workspace %zu < %zu", who, ws_bytes, need);
    if (!d_Gc || !d_g0inv) return fail(QCM_EARG, "%s: NULL device array", who);
    hipStream_t s = as_stream(stream);
    Carver cv(d_ws);
    layout(cv, &tcp, &th, &ep, &bd, &kd, &zd, &bad);
    std::vector<CBond> hb(n_bonds > 0 ? n_bonds : 1);
    for (int q = 0; q < n_bonds; ++q) {
        const qcm_bond &b = h_bonds[q];
        hb[q] = CBond{b.i, b.j, (double)b.shift[0], (double)b.shift[1], (double)b.shift[2], b.t};
    }
    QCM_HIP(hipMemcpyAsync(tcp, h_tcp, sizeof(double) * L * L, hipMemcpyHostToDevice, s));
    if (n_bath > 0) {
        QCM_HIP(hipMemcpyAsync(th, h_theta, sizeof(double) * L * n_bath, hipMemcpyHostToDevice, s));
        QCM_HIP(hipMemcpyAsync(ep, h_eps, sizeof(double) * n_bath, hipMemcpyHostToDevice, s));
    }
    if (n_bonds > 0)
        QCM_HIP(hipMemcpyAsync(bd, hb.data(), sizeof(CBond) * n_bonds, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(kd, h_k, sizeof(double) * 3 * n_k, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(zd, h_z, sizeof(double) * 2 * n_z, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t) * n_z, s));
    k_cdmft_g0inv<<<n_z, 256, 0, s>>>(L, n_bath, tcp, th, ep, bd, n_bonds, kd, n_k, zd, d_Gc,
                                      d_sigma, d_gbar, d_g0inv, bad);
    QCM_LAUNCH_CHECK();
    std::vector<int32_t> hbad(n_z);
    QCM_HIP(hipMemcpyAsync(hbad.data(), bad, sizeof(int32_t) * n_z, hipMemcpyDeviceToHost, s));
    QCM_HIP(hipStreamSynchronize(s));
    for (int iz = 0; iz < n_z; ++iz)
        if (hbad[iz])
            return fail(QCM_EARG, "%s: singular %s at frequency %d", who,
                        (hbad[iz] & 1) ? "G_c" : (hbad[iz] & 2) ? "lattice resolvent" : "Gbar", iz);
    return QCM_OK;
}

extern "C" int qcm_cdmft_fit(int32_t L, int32_t n_bath, int32_t n_par, const double *h_A_eps,
                             const double *h_A_theta, const double *h_tcp, int32_t n_z,
                             const double *h_z, const double *h_w, const double *d_g0inv,
                             double *h_p, double gtol, int32_t max_iter, double *h_dist,
                             int32_t *h_iters, void *d_ws, size_t ws_bytes, size_t *ws_needed,
                             void *stream) {
    const char *who = "qcm_cdmft_fit";
    if (!ws_needed) return fail(QCM_EARG, "%s: ws_needed is NULL", who);
    QCM_TRY(check_common(who, L, n_bath, h_tcp, n_z, h_z));
    if (n_par < 1 || n_par > kCP) return fail(QCM_ERANGE, "%s: n_par=%d outside 1..%d", who, n_par, kCP);
    if (!(gtol >= 0.0) || max_iter < 0) return fail(QCM_EARG, "%s: bad gtol or max_iter", who);
    auto layout = [&](Carver &cv, double **ae, double **at, double **tcp, double **zd, double **wd,
                      double **pd, double **od) {
        *ae = cv.take<double>((size_t)(n_bath > 0 ? n_bath : 1) * n_par);
        *at = cv.take<double>((size_t)L * (n_bath > 0 ? n_bath : 1) * n_par);
        *tcp = cv.take<double>((size_t)L * L);
        *zd = cv.take<double>(2 * (size_t)n_z);
        *wd = cv.take<double>(n_z);
        *pd = cv.take<double>(n_par);
        *od = cv.take<double>(2);
    };
    double *ae, *at, *tcp, *zd, *wd, *pd, *od;
    Carver dry(nullptr);
    layout(dry, &ae, &at, &tcp, &zd, &wd, &pd, &od);
    const size_t need = dry.off + 256;
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (ws_bytes < need) return fail(QCM_EWORKSPACE, "%s: workspace %zu < %zu", who, ws_bytes, need);
    if (!d_g0inv || !h_p || !h_w || (n_bath > 0 && (!h_A_eps || !h_A_theta)))
        return fail(QCM_EARG, "%s: NULL array", who);
    hipStream_t s = as_stream(stream);
    Carver cv(d_ws);
    layout(cv, &ae, &at, &tcp, &zd, &wd, &pd, &od);
    if (n_bath > 0) {
        QCM_HIP(hipMemcpyAsync(ae, h_A_eps, sizeof(double) * n_bath * n_par, hipMemcpyHostToDevice, s));
        QCM_HIP(hipMemcpyAsync(at, h_A_theta, sizeof(double) * L * n_bath * n_par,
                               hipMemcpyHostToDevice, s));
    }
    QCM_HIP(hipMemcpyAsync(tcp, h_tcp, sizeof(double) * L * L, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(zd, h_z, sizeof(double) * 2 * n_z, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(wd, h_w, sizeof(double) * n_z, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(pd, h_p, sizeof(double) * n_par, hipMemcpyHostToDevice, s));
    FitArgs a;
    a.L = L;
    a.nb = n_bath;
    a.np = n_par;
    a.nz = n_z;
    a.max_iter = max_iter;
    a.gtol = gtol;
    a.A_eps = ae;
    a.A_theta = at;
    a.tcp = tcp;
    a.zs = zd;
    a.w = wd;
    a.g0i = d_g0inv;
    a.p = pd;
    a.out = od;
    k_cdmft_fit<<<1, 256, 0, s>>>(a);
    QCM_LAUNCH_CHECK();
    double out[2];
    QCM_HIP(hipMemcpyAsync(h_p, pd, sizeof(double) * n_par, hipMemcpyDeviceToHost, s));
    QCM_HIP(hipMemcpyAsync(out, od, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
    QCM_HIP(hipStreamSynchronize(s));
    if (h_dist) *h_dist = out[0];
    if (h_iters) *h_iters = (int32_t)out[1];
    return QCM_OK;
}
