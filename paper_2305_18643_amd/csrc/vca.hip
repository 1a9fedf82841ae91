// Potthoff functional of a cluster reference system by the analytic pole
// formula (paper: subsection "Practical calculation of the Potthoff
// functional", eq. (omega4)).
//
//  * k_vca_k, one workgroup per wave-vector: V(k) (L x L), W = V(k) Q, then
//    L(k) = diag(w') + Q^T W (R x R, complex Hermitian) written in LDS as the
//    real symmetric 2R x 2R matrix [[Re, -Im], [Im, Re]], whose spectrum is
//    that of L(k) with every eigenvalue twice; a cyclic parallel Jacobi
//    method (round-robin pairing, R disjoint rotations per round) diagonalises
//    it, and half the sum of its negative eigenvalues is the k term.
//  * k_vca_sum, one workgroup: the fixed-order average over k and the
//    functional E0 + 2 (average - sum of the negative poles of G').
//
// The same functional by the frequency integral of eq. (sef4) along the
// imaginary axis (its numerical form):
//    Omega = E0 + 2 mean_k [ -(1/pi) int_0^inf Re ln det(1 - V(k) G'(iw)) dw
//                            + tr V(k) / 2 ],
// integrated by a global adaptive Gauss-Kronrod (7, 15) rule on w = c x/(1-x),
// x in [0, 1):
//  * k_vca_quad_nodes, one workgroup per node: G'(iw) = Q diag(1/(iw - w'))
//    Q^T in LDS, then one thread per wave-vector forms X = V(k) G'(iw) and
//    takes Re ln det(1 - X) from the LU factors of 1 - X (partial pivoting),
//    or, where |X|_F <= 1/4 (large w, where det(1 - X) = 1 - O(|X|^2) would
//    lose the result to rounding and the Jacobian would magnify the loss),
//    from the series -sum_n Re tr(X^n)/n; the k sum is a fixed-order block
//    reduction, times the Jacobian dw/dx.
//  * k_vca_quad_rule, one thread per interval: the 15-point Kronrod and the
//    7-point Gauss sums; their difference is the interval's error estimate.
//  * the host bisects the intervals with the largest errors until the sum of
//    the errors meets the tolerance; k_vca_quad_final adds the intervals'
//    integrals in the order of their positions and forms Omega.
#include <math.h>

#include <algorithm>
#include <vector>

#include "lanczos_device.h"
#include "qcm_internal.h"

namespace qcm {

constexpr int kVL = 8;                       // cluster sites
constexpr int kVR = QCM_VCA_MAX_R;           // poles
constexpr int kVN = 2 * kVR;                 // order of the real form
constexpr int kVQR = QCM_VCA_QUAD_MAX_R;      // poles, frequency-integral route

// Gauss-Kronrod (7, 15) on [-1, 1] (Kronrod's extension of the 7-point
// Gauss-Legendre rule, as tabulated in QUADPACK's qk15): abscissae
// x_0 > ... > x_7 = 0, the Kronrod weights, and the Gauss weights of the odd
// abscissae x_1, x_3, x_5, x_7.
__constant__ double kGkX[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
__constant__ double kGkW[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
__constant__ double kGW[4] = {0.129484966168869693270611432679082,
                              0.279705391489276667901467771423780,
                              0.381830050505118944950369775488975,
                              0.417959183673469387755102040816327};
constexpr int kGkN = 15;   // nodes per interval

struct VBond {
    int32_t i, j;
    double s0, s1, s2, t;
};

// Eigenvalues of the symmetric n x n matrix M (LDS, row stride n) by the
// cyclic parallel Jacobi method; on return the diagonal holds them.  All
// threads of the workgroup (256) take part.
__device__ void jacobi_values_lds(double *M, int n, int max_sweeps, double *cs, double *sn, int *pa,
                                  int *pb, double *red) {
    const int t = threadIdx.x, T = blockDim.x;
    const int m = (n % 2 == 0) ? n : n + 1;  // a dummy index n when n is odd
    const int np = m / 2;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double a0 = 0.0, a1 = 0.0;
        for (int e = t; e < n * n; e += T) {
            const double v = M[e];
            if (e / n != e % n) a0 += v * v;
            a1 += v * v;
        }
        const double off = block_sum(a0, red), tot = block_sum(a1, red);
        if (!(off > 1e-30 * tot)) break;
        for (int rd = 0; rd < m - 1; ++rd) {
            for (int k = t; k < np; k += T) {
                int a, b;
                if (k == 0) {
                    a = m - 1;
                    b = rd;
                } else {
                    a = (rd + k) % (m - 1);
                    b = (rd - k + (m - 1)) % (m - 1);
                }
                const int p = a < b ? a : b, q = a < b ? b : a;
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double app = M[p * n + p], aqq = M[q * n + q], apq = M[p * n + q];
                    if (fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * (fabs(app) + fabs(aqq))) {
                        const double th = (aqq - app) / (2.0 * apq);
                        const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(tt * tt + 1.0);
                        s = tt * c;
                    }
                }
                pa[k] = p;
                pb[k] = q;
                cs[k] = c;
                sn[k] = s;
            }
            __syncthreads();
            for (int e = t; e < np * n; e += T) {  // rows p, q
                const int k = e / n, col = e % n, p = pa[k], q = pb[k];
                if (q >= n || sn[k] == 0.0) continue;
                const double c = cs[k], s = sn[k];
                const double xp = M[p * n + col], xq = M[q * n + col];
                M[p * n + col] = c * xp - s * xq;
                M[q * n + col] = s * xp + c * xq;
            }
            __syncthreads();
            for (int e = t; e < n * np; e += T) {  // columns p, q
                const int row = e / np, k = e % np, p = pa[k], q = pb[k];
                if (q >= n || sn[k] == 0.0) continue;
                const double c = cs[k], s = sn[k];
                const double xp = M[row * n + p], xq = M[row * n + q];
                M[row * n + p] = c * xp - s * xq;
                M[row * n + q] = s * xp + c * xq;
            }
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(256) k_vca_k(int L, int R, const double *__restrict__ poles,
                                               const double *__restrict__ Q,
                                               const double *__restrict__ dt,
                                               const VBond *__restrict__ bonds, int nbonds,
                                               const double *__restrict__ ks,
                                               double *__restrict__ per_k) {
    extern __shared__ __align__(16) double Ms[];  // [2R][2R]
    __shared__ double Vr[kVL * kVL], Vi[kVL * kVL];
    __shared__ double Wr[kVL * kVR], Wi[kVL * kVR];
    __shared__ double cs[kVN / 2 + 1], sn[kVN / 2 + 1], red[256];
    __shared__ int pa[kVN / 2 + 1], pb[kVN / 2 + 1];
    const int t = threadIdx.x, T = blockDim.x, k = blockIdx.x, n = 2 * R;
    if (t == 0) {
        for (int e = 0; e < L * L; ++e) {
            Vr[e] = dt[e];
            Vi[e] = 0.0;
        }
        const double k0 = ks[3 * k], k1 = ks[3 * k + 1], k2 = ks[3 * k + 2];
        for (int q = 0; q < nbonds; ++q) {
            const VBond b = bonds[q];
            const double ph = 2.0 * M_PI * (k0 * b.s0 + k1 * b.s1 + k2 * b.s2);
            const double c = cos(ph), s = sin(ph);
            Vr[b.i * L + b.j] += b.t * c;
            Vi[b.i * L + b.j] += b.t * s;
            Vr[b.j * L + b.i] += b.t * c;
            Vi[b.j * L + b.i] -= b.t * s;
        }
    }
    __syncthreads();
    for (int e = t; e < L * R; e += T) {  // W = V Q
        const int i = e / R, s = e % R;
        double wr = 0.0, wi = 0.0;
        for (int j = 0; j < L; ++j) {
            const double q = Q[j * R + s];
            wr += Vr[i * L + j] * q;
            wi += Vi[i * L + j] * q;
        }
        Wr[e] = wr;
        Wi[e] = wi;
    }
    __syncthreads();
    for (int e = t; e < R * R; e += T) {  // L(k) = diag(w') + Q^T W, real form
        const int r = e / R, s = e % R;
        double lr = r == s ? poles[r] : 0.0, li = 0.0;
        for (int i = 0; i < L; ++i) {
            const double q = Q[i * R + r];
            lr += q * Wr[i * R + s];
            li += q * Wi[i * R + s];
        }
        Ms[r * n + s] = lr;
        Ms[(r + R) * n + (s + R)] = lr;
        Ms[r * n + (s + R)] = -li;
        Ms[(r + R) * n + s] = li;
    }
    __syncthreads();
    jacobi_values_lds(Ms, n, 60, cs, sn, pa, pb, red);
    if (t == 0) {
        double neg = 0.0;
        for (int r = 0; r < n; ++r) {
            const double w = Ms[r * n + r];
            if (w < 0.0) neg += w;
        }
        per_k[k] = 0.5 * neg;
    }
}

__global__ void __launch_bounds__(256) k_vca_sum(const double *__restrict__ per_k, int nk,
                                                 const double *__restrict__ poles, int R, double e0,
                                                 double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < nk; k += blockDim.x) s += per_k[k];
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) {
        double neg = 0.0;
        for (int r = 0; r < R; ++r)
            if (poles[r] < 0.0) neg += poles[r];
        out[0] = e0 + 2.0 * (tot / nk - neg);
    }
}

// V(k) = dt + inter-cluster bonds (Hermitian partner added), complex L x L
__device__ void vca_v_of_k(int L, const double *__restrict__ dt, const VBond *__restrict__ bonds,
                           int nbonds, const double *__restrict__ kv, double *Vr, double *Vi) {
    for (int e = 0; e < L * L; ++e) {
        Vr[e] = dt[e];
        Vi[e] = 0.0;
    }
    for (int q = 0; q < nbonds; ++q) {
        const VBond b = bonds[q];
        const double ph = 2.0 * M_PI * (kv[0] * b.s0 + kv[1] * b.s1 + kv[2] * b.s2);
        const double c = cos(ph), s = sin(ph);
        Vr[b.i * L + b.j] += b.t * c;
        Vi[b.i * L + b.j] += b.t * s;
        Vr[b.j * L + b.i] += b.t * c;
        Vi[b.j * L + b.i] -= b.t * s;
    }
}

// Node j: f_j = (sum_k ln|det(1 - V(k) G'(i w_j))|) dw/dx at x_j.
__global__ void __launch_bounds__(256)
    k_vca_quad_nodes(int L, int R, const double *__restrict__ poles, const double *__restrict__ Q,
                     const double *__restrict__ dt, const VBond *__restrict__ bonds, int nbonds,
                     const double *__restrict__ ks, int nk, double c, const double *__restrict__ xs,
                     double *__restrict__ f, int32_t *__restrict__ bad) {
    __shared__ double Gr[kVL * kVL], Gi[kVL * kVL], red[256];
    const int t = threadIdx.x, j = blockIdx.x;
    const double x = xs[j];
    const double w = c * x / (1.0 - x);
    const double jac = c / ((1.0 - x) * (1.0 - x));
    if (t < L * L) {   // G'_ab(iw) = sum_r Q_ar Q_br / (iw - w'_r)
        const int a = t / L, b = t % L;
        double gr = 0.0, gi = 0.0;
        for (int r = 0; r < R; ++r) {
            const double qq = Q[a * R + r] * Q[b * R + r];
            const double den = w * w + poles[r] * poles[r];
            gr += qq * (-poles[r]) / den;
            gi += qq * (-w) / den;
        }
        Gr[t] = gr;
        Gi[t] = gi;
    }
    __syncthreads();
    double acc = 0.0;
    for (int k = t; k < nk; k += blockDim.x) {
        double Vr[kVL * kVL], Vi[kVL * kVL], Mr[kVL * kVL], Mi[kVL * kVL];
        vca_v_of_k(L, dt, bonds, nbonds, ks + 3 * k, Vr, Vi);
        double nx = 0.0;
        for (int a = 0; a < L; ++a)   // X = V G'
            for (int b = 0; b < L; ++b) {
                double xr = 0.0, xi = 0.0;
                for (int e = 0; e < L; ++e) {
                    const double vr = Vr[a * L + e], vi = Vi[a * L + e];
                    const double gr = Gr[e * L + b], gi = Gi[e * L + b];
                    xr += vr * gr - vi * gi;
                    xi += vr * gi + vi * gr;
                }
                Mr[a * L + b] = xr;
                Mi[a * L + b] = xi;
                nx += xr * xr + xi * xi;
            }
        double lg = 0.0;
        if (nx <= 0.0625) {
            // |X| <= 1/4 (large w): Re ln det(1 - X) = -sum_n Re tr(X^n) / n.  The
            // determinant itself would be 1 - O(|X|^2) and lose the result to
            // rounding; the series keeps every term to its own relative accuracy.
            double Pr[kVL * kVL], Pi[kVL * kVL];
            for (int e = 0; e < L * L; ++e) {
                Pr[e] = Mr[e];
                Pi[e] = Mi[e];
            }
            for (int n = 1; n <= 64; ++n) {
                double tr = 0.0, np2 = 0.0;
                for (int a = 0; a < L; ++a) tr += Pr[a * L + a];
                lg -= tr / n;
                for (int e = 0; e < L * L; ++e) np2 += Pr[e] * Pr[e] + Pi[e] * Pi[e];
                if (np2 < 1e-36) break;
                // P <- P X, one row at a time
                for (int a = 0; a < L; ++a) {
                    double rr[kVL], ri[kVL];
                    for (int b = 0; b < L; ++b) {
                        double yr = 0.0, yi = 0.0;
                        for (int e = 0; e < L; ++e) {
                            const double pr = Pr[a * L + e], pi = Pi[a * L + e];
                            const double xr = Mr[e * L + b], xi = Mi[e * L + b];
                            yr += pr * xr - pi * xi;
                            yi += pr * xi + pi * xr;
                        }
                        rr[b] = yr;
                        ri[b] = yi;
                    }
                    for (int b = 0; b < L; ++b) {
                        Pr[a * L + b] = rr[b];
                        Pi[a * L + b] = ri[b];
                    }
                }
            }
            acc += lg;
            continue;
        }
        for (int e = 0; e < L * L; ++e) {   // M = 1 - X
            Mr[e] = (e / L == e % L ? 1.0 : 0.0) - Mr[e];
            Mi[e] = -Mi[e];
        }
        for (int col = 0; col < L; ++col) {   // LU with partial pivoting
            int piv = col;
            double best = Mr[col * L + col] * Mr[col * L + col] + Mi[col * L + col] * Mi[col * L + col];
            for (int r = col + 1; r < L; ++r) {
                const double m2 = Mr[r * L + col] * Mr[r * L + col] + Mi[r * L + col] * Mi[r * L + col];
                if (m2 > best) {
                    best = m2;
                    piv = r;
                }
            }
            if (!(best > 0.0)) {
                atomicOr(bad, 1);
                break;
            }
            if (piv != col)
                for (int e = 0; e < L; ++e) {
                    double tr = Mr[col * L + e], ti = Mi[col * L + e];
                    Mr[col * L + e] = Mr[piv * L + e];
                    Mi[col * L + e] = Mi[piv * L + e];
                    Mr[piv * L + e] = tr;
                    Mi[piv * L + e] = ti;
                }
            lg += 0.5 * log(best);
            const double pr = Mr[col * L + col], pi = Mi[col * L + col];
            for (int r = col + 1; r < L; ++r) {   // row r -= (M_r,col / pivot) row col
                const double ar = Mr[r * L + col], ai = Mi[r * L + col];
                const double fr = (ar * pr + ai * pi) / best, fi = (ai * pr - ar * pi) / best;
                for (int e = col; e < L; ++e) {
                    const double br = Mr[col * L + e], bi = Mi[col * L + e];
                    Mr[r * L + e] -= fr * br - fi * bi;
                    Mi[r * L + e] -= fr * bi + fi * br;
                }
            }
        }
        acc += lg;
    }
    const double tot = block_sum(acc, red);
    if (t == 0) f[j] = tot * jac;
}

// Nodes of the fresh intervals: interval i = [ab[2i], ab[2i+1]] in slot
// slots[i] gets the 15 abscissae m - h x_0 .. m + h x_0 and its half-width h.
__global__ void k_vca_quad_place(const double *__restrict__ ab, const int32_t *__restrict__ slots,
                                 int n, double *__restrict__ xs, double *__restrict__ half) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double m = 0.5 * (ab[2 * i] + ab[2 * i + 1]), h = 0.5 * (ab[2 * i + 1] - ab[2 * i]);
    double *x = xs + (size_t)slots[i] * kGkN;
    for (int q = 0; q < 7; ++q) {
        x[q] = m - h * kGkX[q];
        x[14 - q] = m + h * kGkX[q];
    }
    x[7] = m;
    half[slots[i]] = h;
}

// Interval i with centre m and half-width h: Kronrod and Gauss sums over its
// 15 node values (stored from x = m - h x_0 up to m + h x_0).
__global__ void k_vca_quad_rule(const int32_t *__restrict__ slots, int n, const double *__restrict__ half,
                                const double *__restrict__ f, double *__restrict__ est,
                                double *__restrict__ err) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int sl = slots[e];
    const double *fv = f + (size_t)sl * kGkN;
    double kr = kGkW[7] * fv[7], ga = kGW[3] * fv[7];
    for (int i = 0; i < 7; ++i) {
        const double pair = fv[i] + fv[14 - i];
        kr += kGkW[i] * pair;
        if (i % 2 == 1) ga += kGW[i / 2] * pair;
    }
    est[sl] = kr * half[sl];
    err[sl] = fabs((kr - ga) * half[sl]);
}

// Omega from the intervals' integrals in the order given (by position) and
// the k average of tr V(k).
__global__ void __launch_bounds__(256)
    k_vca_quad_final(const int32_t *__restrict__ order, int n, const double *__restrict__ est,
                     const double *__restrict__ err, int L, const double *__restrict__ dt,
                     const VBond *__restrict__ bonds, int nbonds, const double *__restrict__ ks,
                     int nk, double e0, double *__restrict__ out) {
    __shared__ double red[256];
    double tr = 0.0;
    for (int k = threadIdx.x; k < nk; k += blockDim.x) {
        double v = 0.0;
        for (int a = 0; a < L; ++a) v += dt[a * L + a];
        for (int q = 0; q < nbonds; ++q) {
            const VBond b = bonds[q];
            if (b.i == b.j) {
                const double ph = 2.0 * M_PI * (ks[3 * k] * b.s0 + ks[3 * k + 1] * b.s1 +
                                                ks[3 * k + 2] * b.s2);
                v += 2.0 * b.t * cos(ph);
            }
        }
        tr += v;
    }
    const double trs = block_sum(tr, red);
    if (threadIdx.x == 0) {
        double I = 0.0, E = 0.0;
        for (int i = 0; i < n; ++i) {
            I += est[order[i]];
            E += err[order[i]];
        }
        out[0] = e0 + 2.0 * (-I / (M_PI * nk) + 0.5 * trs / nk);
        out[1] = 2.0 * E / (M_PI * nk);
    }
}

}  // namespace qcm

using namespace qcm;

extern "C" int qcm_vca_omega(int32_t L, int32_t R, const double *h_poles, const double *h_Q,
                             const double *h_dt, int32_t n_bonds, const qcm_bond *h_bonds,
                             int32_t n_k, const double *h_k, double e0, double *h_omega,
                             double *h_per_k, void *d_ws, size_t ws_bytes, size_t *ws_needed,
                             void *stream) {
    const char *who = "qcm_vca_omega";
    if (!ws_needed) return fail(QCM_EARG, "%s: ws_needed is NULL", who);
    if (L < 1 || L > kVL) return fail(QCM_ERANGE, "%s: L=%d outside 1..%d", who, L, kVL);
    if (R < 1 || R > kVR) return fail(QCM_ERANGE, "%s: R=%d outside 1..%d", who, R, kVR);
    if (!h_poles || !h_Q || !h_dt) return fail(QCM_EARG, "%s: NULL host array", who);
    if (n_bonds < 0 || (n_bonds > 0 && !h_bonds)) return fail(QCM_EARG, "%s: bad bonds", who);
    if (n_k < 1 || !h_k) return fail(QCM_EARG, "%s: need n_k >= 1 wave-vectors", who);
    for (int q = 0; q < n_bonds; ++q)
        if (h_bonds[q].i < 0 || h_bonds[q].i >= L || h_bonds[q].j < 0 || h_bonds[q].j >= L)
            return fail(QCM_EARG, "%s: bond %d has a site out of range", who, q);
    auto layout = [&](Carver &cv, double **po, double **Qd, double **dtd, VBond **bd, double **kd,
                      double **pk, double **od) {
        *po = cv.take<double>(R);
        *Qd = cv.take<double>((size_t)L * R);
        *dtd = cv.take<double>((size_t)L * L);
        *bd = cv.take<VBond>(n_bonds > 0 ? n_bonds : 1);
        *kd = cv.take<double>(3 * (size_t)n_k);
        *pk = cv.take<double>(n_k);
        *od = cv.take<double>(1);
    };
    double *po, *Qd, *dtd, *kd, *pk, *od;
    VBond *bd;
    Carver dry(nullptr);
    layout(dry, &po, &Qd, &dtd, &bd, &kd, &pk, &od);
    const size_t need = dry.off + 256;
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (ws_bytes < need) return fail(QCM_EWORKSPACE, "%s: workspace %zu < %zu", who, ws_bytes, need);
    if (!h_omega) return fail(QCM_EARG, "%s: h_omega is NULL", who);
    hipStream_t s = as_stream(stream);
    Carver cv(d_ws);
    layout(cv, &po, &Qd, &dtd, &bd, &kd, &pk, &od);
    std::vector<VBond> hb(n_bonds > 0 ? n_bonds : 1);
    for (int q = 0; q < n_bonds; ++q) {
        const qcm_bond &b = h_bonds[q];
        hb[q] = VBond{b.i, b.j, (double)b.shift[0], (double)b.shift[1], (double)b.shift[2], b.t};
    }
    QCM_HIP(hipMemcpyAsync(po, h_poles, sizeof(double) * R, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(Qd, h_Q, sizeof(double) * L * R, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(dtd, h_dt, sizeof(double) * L * L, hipMemcpyHostToDevice, s));
    if (n_bonds > 0)
        QCM_HIP(hipMemcpyAsync(bd, hb.data(), sizeof(VBond) * n_bonds, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(kd, h_k, sizeof(double) * 3 * n_k, hipMemcpyHostToDevice, s));
    const size_t lds = sizeof(double) * 4 * (size_t)R * R;
    k_vca_k<<<n_k, 256, lds, s>>>(L, R, po, Qd, dtd, bd, n_bonds, kd, pk);
    QCM_LAUNCH_CHECK();
    k_vca_sum<<<1, 256, 0, s>>>(pk, n_k, po, R, e0, od);
    QCM_LAUNCH_CHECK();
    QCM_HIP(hipMemcpyAsync(h_omega, od, sizeof(double), hipMemcpyDeviceToHost, s));
    if (h_per_k)
        QCM_HIP(hipMemcpyAsync(h_per_k, pk, sizeof(double) * n_k, hipMemcpyDeviceToHost, s));
    QCM_HIP(hipStreamSynchronize(s));
    return QCM_OK;
}

extern "C" int qcm_vca_omega_quad(int32_t L, int32_t R, const double *h_poles, const double *h_Q,
                                  const double *h_dt, int32_t n_bonds, const qcm_bond *h_bonds,
                                  int32_t n_k, const double *h_k, double e0, double rtol,
                                  int32_t max_intervals, double *h_omega, double *h_err,
                                  int32_t *h_intervals, void *d_ws, size_t ws_bytes,
                                  size_t *ws_needed, void *stream) {
    const char *who = "qcm_vca_omega_quad";
    if (!ws_needed) return fail(QCM_EARG, "%s: ws_needed is NULL", who);
    if (L < 1 || L > kVL) return fail(QCM_ERANGE, "%s: L=%d outside 1..%d", who, L, kVL);
    if (R < 1 || R > kVQR) return fail(QCM_ERANGE, "%s: R=%d outside 1..%d", who, R, kVQR);
    if (!h_poles || !h_Q || !h_dt) return fail(QCM_EARG, "%s: NULL host array", who);
    if (n_bonds < 0 || (n_bonds > 0 && !h_bonds)) return fail(QCM_EARG, "%s: bad bonds", who);
    if (n_k < 1 || !h_k) return fail(QCM_EARG, "%s: need n_k >= 1 wave-vectors", who);
    if (!(rtol > 0.0)) return fail(QCM_EARG, "%s: rtol must be > 0", who);
    if (max_intervals < 8 || max_intervals > 65536)
        return fail(QCM_EARG, "%s: max_intervals %d outside 8..65536", who, max_intervals);
    for (int q = 0; q < n_bonds; ++q)
        if (h_bonds[q].i < 0 || h_bonds[q].i >= L || h_bonds[q].j < 0 || h_bonds[q].j >= L)
            return fail(QCM_EARG, "%s: bond %d has a site out of range", who, q);
    const int n0 = 8;                              // first partition of [0, 1)
    const int max_slots = n0 + 2 * max_intervals;  // every bisection adds two
    struct Ptrs {
        double *po, *Qd, *dtd, *kd, *xs, *f, *half, *est, *err, *od, *ab;
        VBond *bd;
        int32_t *slots, *bad;
    } P;
    auto layout = [&](Carver &cv) {
        P.po = cv.take<double>(R);
        P.Qd = cv.take<double>((size_t)L * R);
        P.dtd = cv.take<double>((size_t)L * L);
        P.bd = cv.take<VBond>(n_bonds > 0 ? n_bonds : 1);
        P.kd = cv.take<double>(3 * (size_t)n_k);
        P.xs = cv.take<double>((size_t)max_slots * kGkN);
        P.f = cv.take<double>((size_t)max_slots * kGkN);
        P.half = cv.take<double>(max_slots);
        P.est = cv.take<double>(max_slots);
        P.err = cv.take<double>(max_slots);
        P.od = cv.take<double>(2);
        P.ab = cv.take<double>(2 * (size_t)max_slots);
        P.slots = cv.take<int32_t>(max_slots);
        P.bad = cv.take<int32_t>(1);
    };
    Carver dry(nullptr);
    layout(dry);
    const size_t need = dry.off + 256;
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (ws_bytes < need) return fail(QCM_EWORKSPACE, "%s: workspace %zu < %zu", who, ws_bytes, need);
    if (!h_omega) return fail(QCM_EARG, "%s: h_omega is NULL", who);
    hipStream_t s = as_stream(stream);
    Carver cv(d_ws);
    layout(cv);
    std::vector<VBond> hb(n_bonds > 0 ? n_bonds : 1);
    for (int q = 0; q < n_bonds; ++q) {
        const qcm_bond &b = h_bonds[q];
        hb[q] = VBond{b.i, b.j, (double)b.shift[0], (double)b.shift[1], (double)b.shift[2], b.t};
    }
    double c = 1.0;   // scale of the map w = c x / (1 - x)
    for (int r = 0; r < R; ++r) c = fmax(c, fabs(h_poles[r]));
    QCM_HIP(hipMemcpyAsync(P.po, h_poles, sizeof(double) * R, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(P.Qd, h_Q, sizeof(double) * L * R, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(P.dtd, h_dt, sizeof(double) * L * L, hipMemcpyHostToDevice, s));
    if (n_bonds > 0)
        QCM_HIP(hipMemcpyAsync(P.bd, hb.data(), sizeof(VBond) * n_bonds, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(P.kd, h_k, sizeof(double) * 3 * n_k, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemsetAsync(P.bad, 0, sizeof(int32_t), s));

    // host bookkeeping of the partition (positions only; every sum runs on the device)
    struct Iv {
        double a, b;
        int slot;
    };
    std::vector<Iv> act;
    std::vector<double> est(max_slots, 0.0), err(max_slots, 0.0);
    int next = 0;
    std::vector<double> hab;
    std::vector<int32_t> hslot;
    auto evaluate = [&](const std::vector<Iv> &fresh) -> int {
        const int n = (int)fresh.size();
        hab.assign(2 * (size_t)n, 0.0);
        hslot.assign(n, 0);
        for (int i = 0; i < n; ++i) {
            hab[2 * i] = fresh[i].a;
            hab[2 * i + 1] = fresh[i].b;
            hslot[i] = fresh[i].slot;
        }
        // the fresh slots are consecutive, so their nodes and values are too
        const int s0 = fresh[0].slot;
        QCM_HIP(hipMemcpyAsync(P.ab, hab.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice, s));
        QCM_HIP(hipMemcpyAsync(P.slots, hslot.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        k_vca_quad_place<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(P.ab, P.slots, n, P.xs, P.half);
        k_vca_quad_nodes<<<n * kGkN, 256, 0, s>>>(L, R, P.po, P.Qd, P.dtd, P.bd, n_bonds, P.kd, n_k, c,
                                                 P.xs + (size_t)s0 * kGkN, P.f + (size_t)s0 * kGkN,
                                                 P.bad);
        k_vca_quad_rule<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(P.slots, n, P.half, P.f, P.est,
                                                                  P.err);
        QCM_LAUNCH_CHECK();
        QCM_HIP(hipMemcpyAsync(est.data() + s0, P.est + s0, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        QCM_HIP(hipMemcpyAsync(err.data() + s0, P.err + s0, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        QCM_HIP(hipStreamSynchronize(s));
        return QCM_OK;
    };
    std::vector<Iv> fresh;
    for (int i = 0; i < n0; ++i) fresh.push_back(Iv{(double)i / n0, (double)(i + 1) / n0, next++});
    QCM_TRY(evaluate(fresh));
    act = fresh;
    int32_t bad = 0;
    for (;;) {
        double tot = 0.0, tot_err = 0.0, emax = 0.0;
        for (const Iv &v : act) {
            tot += est[v.slot];
            tot_err += err[v.slot];
            emax = fmax(emax, err[v.slot]);
        }
        const double goal = fmax(rtol * fabs(tot), 1e-15 * n_k);
        if (tot_err <= goal || (int)act.size() >= max_intervals) break;
        // bisect every interval whose error is at least a quarter of the largest
        std::vector<Iv> keep;
        fresh.clear();
        for (const Iv &v : act) {
            if (err[v.slot] >= 0.25 * emax && (int)(act.size() + fresh.size() / 2) < max_intervals &&
                next + 2 <= max_slots) {
                const double m = 0.5 * (v.a + v.b);
                fresh.push_back(Iv{v.a, m, next++});
                fresh.push_back(Iv{m, v.b, next++});
            } else {
                keep.push_back(v);
            }
        }
        if (fresh.empty()) break;
        QCM_TRY(evaluate(fresh));
        keep.insert(keep.end(), fresh.begin(), fresh.end());
        act.swap(keep);
    }
    QCM_HIP(hipMemcpy(&bad, P.bad, sizeof bad, hipMemcpyDeviceToHost));
    if (bad) return fail(QCM_EARG, "%s: 1 - V G'(iw) is singular at a node", who);
    std::sort(act.begin(), act.end(), [](const Iv &x, const Iv &y) { return x.a < y.a; });
    std::vector<int32_t> order(act.size());
    for (size_t i = 0; i < act.size(); ++i) order[i] = act[i].slot;
    QCM_HIP(hipMemcpyAsync(P.slots, order.data(), sizeof(int32_t) * order.size(),
                           hipMemcpyHostToDevice, s));
    k_vca_quad_final<<<1, 256, 0, s>>>(P.slots, (int)order.size(), P.est, P.err, L, P.dtd, P.bd,
                                      n_bonds, P.kd, n_k, e0, P.od);
    QCM_LAUNCH_CHECK();
    double od[2];
    QCM_HIP(hipMemcpyAsync(od, P.od, sizeof od, hipMemcpyDeviceToHost, s));
    QCM_HIP(hipStreamSynchronize(s));
    *h_omega = od[0];
    if (h_err) *h_err = od[1];
    if (h_intervals) *h_intervals = (int32_t)act.size();
    return QCM_OK;
}
