// Cluster perturbation theory with G-scheme periodisation (paper: section
// "Cluster perturbation theory", eqs. (CPT1) and (CPT3)):
//   V(k)_ij = sum over inter-cluster bonds of t exp(i k.r), r = shift.E,
//             plus the Hermitian partner;
//   G(k, z) = (G_c(z)^-1 - V(k))^-1;
//   G_per(k, z) = (1/L) sum_ij exp(-i k.(R_i - R_j)) G_ij(k, z),
// with exp(i k.r) the phase of the partial Fourier transform t_RR'(k) =
// sum_r exp(i k.r) t_{R, r+R'} (subsection "Partial Fourier transforms").
// One workgroup per (k, z); matrices of order L <= 32 are inverted in LDS by
// Gauss-Jordan elimination with partial pivoting.
#include <math.h>

#include "qcm_internal.h"

namespace qcm {

struct BondDev {
    int32_t i, j;
    double rx, ry, rz, t;
};

// In-place inverse of the n x n complex matrix A (row stride n) in LDS, using
// the augmented block X (identity on entry).  blockDim threads cooperate.
__device__ void lds_inverse(double *Ar, double *Ai, double *Xr, double *Xi, int n, int *piv_sh,
                            double *fac_r, double *fac_i) {
    const int t = threadIdx.x, T = blockDim.x;
    for (int p = 0; p < n; ++p) {
        if (t == 0) {
            int best = p;
            double bm = -1.0;
            for (int r = p; r < n; ++r) {
                double m = hypot(Ar[r * n + p], Ai[r * n + p]);
                if (m > bm) {
                    bm = m;
                    best = r;
                }
            }
            *piv_sh = best;
        }
        __syncthreads();
        const int q = *piv_sh;
        if (q != p) {
            for (int c = t; c < n; c += T) {
                double a = Ar[p * n + c], b = Ai[p * n + c];
                Ar[p * n + c] = Ar[q * n + c];
                Ai[p * n + c] = Ai[q * n + c];
                Ar[q * n + c] = a;
                Ai[q * n + c] = b;
                a = Xr[p * n + c];
                b = Xi[p * n + c];
                Xr[p * n + c] = Xr[q * n + c];
                Xi[p * n + c] = Xi[q * n + c];
                Xr[q * n + c] = a;
                Xi[q * n + c] = b;
            }
        }
        __syncthreads();
        // scale the pivot row by 1/pivot
        const double pr = Ar[p * n + p], pi = Ai[p * n + p];
        const double den = pr * pr + pi * pi;
        const double ir = pr / den, ii = -pi / den;
        __syncthreads();
        for (int c = t; c < n; c += T) {
            double a = Ar[p * n + c], b = Ai[p * n + c];
            Ar[p * n + c] = a * ir - b * ii;
            Ai[p * n + c] = a * ii + b * ir;
            a = Xr[p * n + c];
            b = Xi[p * n + c];
            Xr[p * n + c] = a * ir - b * ii;
            Xi[p * n + c] = a * ii + b * ir;
        }
        __syncthreads();
        for (int r = t; r < n; r += T) {
            fac_r[r] = Ar[r * n + p];
            fac_i[r] = Ai[r * n + p];
        }
        __syncthreads();
        for (int e = t; e < n * n; e += T) {
            int r = e / n, c = e % n;
            if (r == p) continue;
            double fr = fac_r[r], fi = fac_i[r];
            double a = Ar[p * n + c], b = Ai[p * n + c];
            Ar[e] -= fr * a - fi * b;
            Ai[e] -= fr * b + fi * a;
            a = Xr[p * n + c];
            b = Xi[p * n + c];
            Xr[e] -= fr * a - fi * b;
            Xi[e] -= fr * b + fi * a;
        }
        __syncthreads();
    }
}

constexpr int kMaxL = 32;

__global__ void __launch_bounds__(64) k_invert_gc(const double *__restrict__ Gc, int n, int nz,
                                                  double *__restrict__ Ginv) {
    __shared__ double Ar[kMaxL * kMaxL], Ai[kMaxL * kMaxL], Xr[kMaxL * kMaxL], Xi[kMaxL * kMaxL];
    __shared__ double fr[kMaxL], fi[kMaxL];
    __shared__ int piv;
    const int iz = blockIdx.x;
    const double *g = Gc + (int64_t)iz * n * n * 2;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        Ar[e] = g[2 * e];
        Ai[e] = g[2 * e + 1];
        Xr[e] = (e / n == e % n) ? 1.0 : 0.0;
        Xi[e] = 0.0;
    }
    __syncthreads();
    lds_inverse(Ar, Ai, Xr, Xi, n, &piv, fr, fi);
    double *o = Ginv + (int64_t)iz * n * n * 2;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        o[2 * e] = Xr[e];
        o[2 * e + 1] = Xi[e];
    }
}

__global__ void __launch_bounds__(64) k_cpt(const double *__restrict__ Ginv, int n, int nz,
                                            const BondDev *__restrict__ bonds, int nbonds,
                                            const double *__restrict__ R, const double *__restrict__ kv,
                                            double *__restrict__ Gper) {
    __shared__ double Ar[kMaxL * kMaxL], Ai[kMaxL * kMaxL], Xr[kMaxL * kMaxL], Xi[kMaxL * kMaxL];
    __shared__ double fr[kMaxL], fi[kMaxL];
    __shared__ double red_r[64], red_i[64];
    __shared__ int piv;
    const int iz = blockIdx.x % nz;
    const int ik = blockIdx.x / nz;
    const double kx = 2.0 * M_PI * kv[3 * ik], ky = 2.0 * M_PI * kv[3 * ik + 1],
                 kz = 2.0 * M_PI * kv[3 * ik + 2];
    const double *g = Ginv + (int64_t)iz * n * n * 2;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        Ar[e] = g[2 * e];
        Ai[e] = g[2 * e + 1];
        Xr[e] = (e / n == e % n) ? 1.0 : 0.0;
        Xi[e] = 0.0;
    }
    __syncthreads();
    // subtract V(k): thread 0 walks the bond list (bonds may repeat an element)
    if (threadIdx.x == 0) {
        for (int q = 0; q < nbonds; ++q) {
            const BondDev b = bonds[q];
            double ph = kx * b.rx + ky * b.ry + kz * b.rz;
            double c = cos(ph), s = sin(ph);
            Ar[b.i * n + b.j] -= b.t * c;
            Ai[b.i * n + b.j] -= b.t * s;
            Ar[b.j * n + b.i] -= b.t * c;
            Ai[b.j * n + b.i] += b.t * s;
        }
    }
    __syncthreads();
    lds_inverse(Ar, Ai, Xr, Xi, n, &piv, fr, fi);
    double sr = 0.0, si = 0.0;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        int i = e / n, j = e % n;
        double ph = -(kx * (R[3 * i] - R[3 * j]) + ky * (R[3 * i + 1] - R[3 * j + 1]) +
                      kz * (R[3 * i + 2] - R[3 * j + 2]));
        double c = cos(ph), s = sin(ph);
        sr += c * Xr[e] - s * Xi[e];
        si += c * Xi[e] + s * Xr[e];
    }
    red_r[threadIdx.x] = sr;
    red_i[threadIdx.x] = si;
    __syncthreads();
    for (int st = 32; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            red_r[threadIdx.x] += red_r[threadIdx.x + st];
            red_i[threadIdx.x] += red_i[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int64_t o = ((int64_t)ik * nz + iz) * 2;
        Gper[o] = red_r[0] / n;
        Gper[o + 1] = red_i[0] / n;
    }
}

}  // namespace qcm

using namespace qcm;

extern "C" int qcm_cpt_gk(int32_t L, int32_t n_z, const double *d_Gc, const int32_t *h_R,
                          const int32_t *h_E, int32_t n_bonds, const qcm_bond *h_bonds,
                          int32_t n_k, const double *h_k, double *d_Gper, void *d_ws,
                          size_t ws_bytes, size_t *ws_needed, void *stream) {
    if (!ws_needed) return fail(QCM_EARG, "qcm_cpt_gk: ws_needed is NULL");
    if (L < 1 || L > kMaxL) return fail(QCM_ERANGE, "qcm_cpt_gk: L=%d outside 1..%d", L, kMaxL);
    if (n_z < 0 || n_k < 0 || n_bonds < 0) return fail(QCM_EARG, "qcm_cpt_gk: negative count");
    if (!h_R || !h_E || (n_bonds > 0 && !h_bonds) || (n_k > 0 && !h_k))
        return fail(QCM_EARG, "qcm_cpt_gk: NULL host array");
    for (int q = 0; q < n_bonds; ++q)
        if (h_bonds[q].i < 0 || h_bonds[q].i >= L || h_bonds[q].j < 0 || h_bonds[q].j >= L)
            return fail(QCM_EARG, "qcm_cpt_gk: bond %d has a site out of range", q);
    Carver cv0(nullptr);
    cv0.take<double>(2 * (size_t)L * L * (n_z > 0 ? n_z : 1));
    cv0.take<BondDev>(n_bonds > 0 ? n_bonds : 1);
    cv0.take<double>(3 * (size_t)L);
    cv0.take<double>(3 * (size_t)(n_k > 0 ? n_k : 1));
    size_t need = cv0.off + 256;
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (ws_bytes < need) return fail(QCM_EWORKSPACE, "qcm_cpt_gk: workspace %zu < %zu", ws_bytes, need);
    if (n_z == 0 || n_k == 0) return QCM_OK;
    if (!d_Gc || !d_Gper) return fail(QCM_EARG, "qcm_cpt_gk: NULL device array");
    hipStream_t s = as_stream(stream);
    Carver cv(d_ws);
    double *Ginv = cv.take<double>(2 * (size_t)L * L * n_z);
    BondDev *bd = cv.take<BondDev>(n_bonds > 0 ? n_bonds : 1);
    double *Rd = cv.take<double>(3 * (size_t)L);
    double *kd = cv.take<double>(3 * (size_t)n_k);
    std::vector<BondDev> hb(n_bonds > 0 ? n_bonds : 1);
    for (int q = 0; q < n_bonds; ++q) {
        const qcm_bond &b = h_bonds[q];
        double r[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) r[c] += (double)b.shift[a] * h_E[3 * a + c];
        hb[q] = BondDev{b.i, b.j, r[0], r[1], r[2], b.t};
    }
    std::vector<double> hR(3 * L);
    for (int q = 0; q < 3 * L; ++q) hR[q] = h_R[q];
    if (n_bonds > 0)
        QCM_HIP(hipMemcpyAsync(bd, hb.data(), sizeof(BondDev) * n_bonds, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(Rd, hR.data(), sizeof(double) * 3 * L, hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(kd, h_k, sizeof(double) * 3 * n_k, hipMemcpyHostToDevice, s));
    k_invert_gc<<<n_z, 64, 0, s>>>(d_Gc, L, n_z, Ginv);
    QCM_LAUNCH_CHECK();
    k_cpt<<<(unsigned)((int64_t)n_k * n_z), 64, 0, s>>>(Ginv, L, n_z, bd, n_bonds, Rd, kd, d_Gper);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}
