// Device helpers shared by the single-solve and the batched Lanczos kernels
// (internal).  Both paths call exactly these functions, so a chain gives the
// same bits whichever path runs it.
#pragma once

#include <math.h>

#include "lanczos_engine.h"

namespace qcm {

template <typename T>
__device__ __forceinline__ double ldd(const T *p) {
    return (double)*p;
}

// Vectors and tables live in global memory, but a pointer read from a group
// table in memory (the batched engine) is generic to the compiler, which then
// emits flat accesses: those also count against the LDS counter, so every LDS
// wait waits for them too.  Cast to the global address space, the same
// accesses become global loads and stores.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> gp(T *p) {
    return (gptr<T>)p;
}
template <typename T>
__device__ __forceinline__ double ldd(gptr<const T> p) {
    return (double)*p;
}
template <typename T>
__device__ __forceinline__ double ldd(gptr<T> p) {
    return (double)*p;
}

__device__ __forceinline__ double block_sum(double x, double *sh) {
    // 256 threads, fixed tree
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

template <typename T>
__device__ __forceinline__ void st(T *p, double x) {
    *p = (T)x;
}

// number of eigenvalues of T_M below x: the sign changes of the Sturm
// sequence p_i = (a_i - x) p_{i-1} - b_{i-1}^2 p_{i-2} (p_{-1} = 1, p_{-2} = 0),
// i.e. the negative pivots q_i = p_i / p_{i-1} of the LDL^T of T_M - x, counted
// without a division.  The pair (p_i, p_{i-1}) is rescaled by a power of two
// whenever p_i leaves [2^-256, 2^256] (exact), and a vanishing p_i becomes
// -2^-700 p_{i-1} (a pivot of -2^-700, so an eigenvalue at x counts as below
// it).  |p_{i-1}| lies in [2^-256, 2^256] there, so the replacement is a
// normal number and the rescale that follows brings the pair back into range
// (a replacement that underflowed to -0 would lose this and every later sign
// change).  b2[i] = b[i]^2.  Callable on the host too (for tests).
__host__ __device__ inline int sturm_below(int M, const double *__restrict__ a,
                                           const double *__restrict__ b2, double x) {
    // branch-free body, so that the loads of later steps can go out early
    int cnt = 0;
    double pm = 1.0, pmm = 0.0;
#pragma unroll 4
    for (int i = 0; i < M; ++i) {
        const double bi = i > 0 ? b2[i - 1] : 0.0;
        double p = fma(-bi, pmm, (a[i] - x) * pm);
        p = p == 0.0 ? -0x1p-700 * pm : p;
        cnt += (p < 0.0) != (pm < 0.0);
        const int e = ilogb(p);
        const int k = (e > 256 || e < -256) ? -e : 0;
        pmm = ldexp(pm, k);
        pm = ldexp(p, k);
    }
    return cnt;
}

// k-th smallest eigenvalue by 256-way multisection: every thread tests one
// point of the current bracket; 10 rounds narrow it by 257^10.  b2 = b^2.
// hint (k = 0 only): the lowest eigenvalue of a leading block of T, which
// can only lie above that of T; once a Sturm count confirms an eigenvalue
// below it (plus 1e-12 relative) it becomes the upper end, and the first
// round then spaces its points geometrically toward that end, where the
// eigenvalue of a converging recurrence lies.  Any hint is safe: one that
// the count does not confirm is ignored.
__device__ inline double tridiag_kth(int M, const double *a, const double *b, const double *b2,
                                     int k, double *sh_lo, double *sh_hi, double hint = NAN) {
    const int t = threadIdx.x;
    __shared__ int cnts[256];
    __shared__ int first, geo;
    if (t == 0) {
        double lo = a[0], hi = a[0];
        for (int i = 0; i < M; ++i) {
            double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i < M - 1 ? fabs(b[i]) : 0.0);
            lo = fmin(lo, a[i] - r);
            hi = fmax(hi, a[i] + r);
        }
        double pad = 1e-12 * fmax(1.0, fmax(fabs(lo), fabs(hi)));
        *sh_lo = lo - pad;
        *sh_hi = hi + pad;
        geo = 0;
        if (k == 0 && isfinite(hint)) {
            const double up = hint + 1e-12 * fmax(1.0, fabs(hint));
            if (up > *sh_lo && up < *sh_hi && sturm_below(M, a, b2, up) > 0) {
                *sh_hi = up;
                geo = 1;
            }
        }
    }
    __syncthreads();
    for (int round = 0; round < 10; ++round) {
        const double lo = *sh_lo, hi = *sh_hi;
        // stop once the bracket is at the resolution of its end points
        if (!(hi - lo > 4e-16 * fmax(fabs(lo), fabs(hi)))) break;
        const bool g = round == 0 && geo;
        // point j of the round: uniform, or hi - (hi - lo) 2^(-53 (j + 1) / 256)
        auto point = [&](int j) -> double {
            return g ? hi - (hi - lo) * exp2(-53.0 * (double)(j + 1) / 256.0)
                     : lo + (hi - lo) * (double)(j + 1) / 257.0;
        };
        const double x = point(t);
        cnts[t] = sturm_below(M, a, b2, x);
        if (t == 0) first = 256;
        __syncthreads();
        // the first point with more than k eigenvalues below it (a minimum,
        // so the result does not rest on the counts being monotone)
        if (cnts[t] > k) atomicMin(&first, t);
        __syncthreads();
        if (t == 0) {
            const int j = first;
            const double nlo = j == 0 ? lo : point(j - 1);
            const double nhi = j == 256 ? hi : point(j);
            *sh_lo = nlo;
            *sh_hi = nhi;
        }
        __syncthreads();
    }
    double r = 0.5 * (*sh_lo + *sh_hi);
    __syncthreads();
    return r;
}

// Eigenvector for theta by inverse iteration: T - theta factored once by
// Gaussian elimination with row pivoting on the tridiagonal (multipliers in
// dl, swaps flagged in piv, reciprocal pivots in d, superdiagonals du, du2),
// then three solves in place on x, each normalised.  One thread.
__device__ inline void tridiag_vector(int M, const double *__restrict__ a, const double *__restrict__ b,
                                      double theta, double *__restrict__ x, double *__restrict__ d,
                                      double *__restrict__ du, double *__restrict__ du2,
                                      double *__restrict__ dl, double *__restrict__ piv) {
    double scale = 1.0;
    for (int i = 0; i < M; ++i) scale = fmax(scale, fabs(a[i]));
    const double tiny = 1e-15 * scale;
    // factorisation, the current row (di, dui) and the next one carried in
    // registers: row i is [di, dui, 0], row i+1 is [b_i, dn, dun]
    double di = a[0] - theta, dui = M > 1 ? b[0] : 0.0;
    for (int i = 0; i < M - 1; ++i) {
        double dli = b[i];
        double dn = a[i + 1] - theta;
        double dun = i < M - 2 ? b[i + 1] : 0.0;
        double du2i = 0.0;
        const bool sw = fabs(dli) > fabs(di);
        if (sw) {
            const double t0 = di;
            di = dli;
            dli = t0;
            const double t1 = dui;
            dui = dn;
            dn = t1;
            du2i = dun;
            dun = 0.0;
        }
        if (di == 0.0) di = tiny;
        const double inv = 1.0 / di;
        const double m = dli * inv;
        d[i] = inv;
        du[i] = dui;
        du2[i] = du2i;
        dl[i] = m;
        piv[i] = sw ? 1.0 : 0.0;
        dn -= m * dui;
        dun -= m * du2i;
        di = dn;
        dui = dun;
    }
    if (di == 0.0) di = tiny;
    d[M - 1] = 1.0 / di;
    for (int i = 0; i < M; ++i) x[i] = 1.0;
    for (int it = 0; it < 3; ++it) {
        // forward: the row swaps and multipliers, x_i carried
        double cur = x[0];
        for (int i = 0; i < M - 1; ++i) {
            const double nxt = x[i + 1];
            const bool sw = piv[i] != 0.0;
            const double lo = sw ? nxt : cur, hi = sw ? cur : nxt;
            x[i] = lo;
            cur = hi - dl[i] * lo;
        }
        x[M - 1] = cur;
        // back substitution, x_{i+1} and x_{i+2} carried
        double x1 = 0.0, x2 = 0.0;
        for (int i = M - 1; i >= 0; --i) {
            double s = x[i];
            if (i + 1 < M) s -= du[i] * x1;
            if (i + 2 < M) s -= du2[i] * x2;
            const double xi = s * d[i];
            x[i] = xi;
            x2 = x1;
            x1 = xi;
        }
        double nr = 0.0;
        for (int i = 0; i < M; ++i) nr += x[i] * x[i];
        nr = 1.0 / sqrt(nr);
        for (int i = 0; i < M; ++i) x[i] *= nr;
    }
    if (x[0] < 0.0)
        for (int i = 0; i < M; ++i) x[i] = -x[i];
}

// Largest T_M whose coefficients and inverse-iteration arrays are staged in
// LDS by the ground-state test (every Sturm step and every elimination step
// then reads LDS instead of waiting on a cache round trip).
constexpr int kTriLds = 640;

// The ground-state test of one workgroup (256 threads) on T_M: theta_0,
// theta_1 (only when want1; the convergence test does not need it, so the
// tests between steps skip it and the final one takes it), the eigenvector
// of theta_0 in svec, residual estimate beta[M-1] |s[M-1]| and the
// convergence flag, written to *status.  Up to kTriLds steps the work happens
// in LDS; longer T_M use `work` (5 M doubles) and beta^2 in work + 5 M (M
// doubles).
__device__ inline void tridiag_status_block(const double *__restrict__ alpha,
                                            const double *__restrict__ beta, int M, double tol,
                                            double *__restrict__ work, double *__restrict__ svec,
                                            GsStatus *__restrict__ status, bool want1 = true) {
    __shared__ double lo, hi;
    __shared__ double la[kTriLds], lb[kTriLds], lb2[kTriLds], lx[kTriLds], lw[5 * kTriLds];
    const bool in_lds = M <= kTriLds;
    const double *a = alpha, *b = beta;
    double *b2 = work + 5 * (size_t)M, *x = svec, *w = work;
    if (in_lds) {
        for (int i = threadIdx.x; i < M; i += blockDim.x) {
            la[i] = alpha[i];
            lb[i] = beta[i];
            lb2[i] = beta[i] * beta[i];
        }
        a = la;
        b = lb;
        b2 = lb2;
        x = lx;
        w = lw;
    } else {
        for (int i = threadIdx.x; i < M; i += blockDim.x) b2[i] = beta[i] * beta[i];
    }
    __syncthreads();
    // the previous test's theta_0 (of T_{M'}, M' <= M) as the hint
    const double hint = (status->M >= 1 && status->M <= M) ? status->theta0 : NAN;
    __syncthreads();
    double th0 = tridiag_kth(M, a, b, b2, 0, &lo, &hi, hint);
    double th1 = (want1 && M > 1) ? tridiag_kth(M, a, b, b2, 1, &lo, &hi) : NAN;
    if (threadIdx.x == 0) {
        const int S = in_lds ? kTriLds : M;
        tridiag_vector(M, a, b, th0, x, w, w + S, w + 2 * S, w + 3 * S, w + 4 * S);
        double est = beta[M - 1] * fabs(x[M - 1]);
        status->theta0 = th0;
        status->theta1 = th1;
        status->est = est;
        status->converged = est <= tol * fmax(1.0, fabs(th0)) ? 1 : 0;
        status->M = M;
    }
    if (in_lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < M; i += blockDim.x) svec[i] = lx[i];
    }
}

struct cplx {
    double re, im;
};

// One continued fraction at z, bottom floor first.  part 0 (electron):
// b0sq / (z + E0 - a0 - b1^2/(z + E0 - a1 - ...)); part 1 (hole):
// b0sq / (z - E0 + a0 - b1^2/(z - E0 + a1 - ...)).
__device__ inline cplx cf_value(const double *__restrict__ co, int len, int maxs, cplx z, double e0,
                         int part) {
    cplx r{0.0, 0.0};
    if (len <= 0 || co[0] == 0.0) return r;
    const double sg = part == 0 ? 1.0 : -1.0;
    const double zr = part == 0 ? z.re + e0 : z.re - e0;
    const double zi = z.im;
    const double *a = co + 1, *b2 = co + 1 + maxs;
    double gr = zr - sg * a[len - 1], gi = zi;
    for (int n = len - 2; n >= 0; --n) {
        double den = gr * gr + gi * gi;
        double qr = b2[n] * gr / den, qi = -b2[n] * gi / den;  // b2 / g
        gr = zr - sg * a[n] - qr;
        gi = zi - qi;
    }
    double den = gr * gr + gi * gi;
    r.re = co[0] * gr / den;
    r.im = -co[0] * gi / den;
    return r;
}

}  // namespace qcm
