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
#include <math.h>

#include <vector>

#include "lanczos_device.h"
#include "qcm_internal.h"

namespace qcm {

constexpr int kVL = 8;                       // cluster sites
constexpr int kVR = QCM_VCA_MAX_R;           // poles
constexpr int kVN = 2 * kVR;                 // order of the real form

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
