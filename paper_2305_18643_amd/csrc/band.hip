// Band Lanczos Green function (paper: section "Exact diagonalizations",
// subsection "The band Lanczos algorithm for the Green function"; Lehmann
// form of eq. (spectral1)).
//
// For the p start states |phi_mu> = c+_mu |Omega> (electron part, sector
// N_up + 1) and c_mu |Omega> (hole part, N_up - 1), the Krylov space is built
// one basis vector v_j at a time: the next candidate is normalised (or
// deflated when its norm is negligible), the other candidates are
// orthogonalised against v_j, the new candidate H v_j is orthogonalised
// against the band of previous basis vectors (coefficients known by symmetry)
// and against v_j and the deflated look-back set (coefficients computed).
// The coefficients form the projected Hamiltonian T (a band of 2p diagonals
// plus the entries deflation adds) and the projections rho of the start
// states.  T = U diag(Lambda) U^T in one workgroup (Householder reduction,
// then implicit QR steps on the tridiagonal, both applied to rho^T, which
// ends as Q = rho^T U); G(z) = sum_r Q_mu,r Q_nu,r / (z -+ ...).
//
// The host runs the recurrence's bookkeeping (which vectors are candidates,
// basis vectors or deflated) and reads back one norm per step for the
// deflation test; vectors, coefficients and every sum stay on the device.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <vector>

#include "lanczos_device.h"

namespace qcm {

constexpr int kBandMaxP = 32;     // start states per part
constexpr int kBandMaxR = 1024;   // basis vectors per part

// element offsets of up to kBandMaxP + 1 vectors of the slot pool
struct VecList {
    int64_t off[kBandMaxP + 1];
    int32_t n;
};

// where the sums of one launch go: T (symmetric), rho, or nowhere
struct Put {
    int32_t n;
    int32_t mode[kBandMaxP + 1];   // 0: T[i][k] = T[k][i]; 1: rho[i][k]; 2: none; 3: T[i][i], scale
    int32_t i[kBandMaxP + 1], k[kBandMaxP + 1];
};

// partial[q][chunk] = <x, y_q> over one chunk of kChunk elements
template <typename T>
__global__ void __launch_bounds__(256) kbl_dots(const T *__restrict__ base, int64_t xo,
                                                VecList ys, int64_t dim, int nchunks,
                                                double *__restrict__ partial) {
    __shared__ double sh[256];
    const int q = blockIdx.y;
    const T *x = base + xo;
    const T *y = base + ys.off[q];
    const int64_t b0 = (int64_t)blockIdx.x * kChunk;
    double acc = 0.0;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        const int64_t e = b0 + k;
        if (e < dim) acc = fma(ldd(x + e), ldd(y + e), acc);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)q * nchunks + blockIdx.x] = s;
}

// res[q] = sum of the partials of sum q (fixed order), stored as `put` says
__global__ void __launch_bounds__(256) kbl_finish(const double *__restrict__ partial, int nchunks,
                                                  Put put, double *__restrict__ res,
                                                  double *__restrict__ Tm, int ldt,
                                                  double *__restrict__ rho, int p,
                                                  double *__restrict__ scal) {
    __shared__ double sh[256];
    const int q = blockIdx.x;
    double acc = 0.0;
    for (int k = threadIdx.x; k < nchunks; k += 256) acc += partial[(int64_t)q * nchunks + k];
    const double s = block_sum(acc, sh);
    if (threadIdx.x != 0) return;
    res[q] = s;
    const int i = put.i[q], k = put.k[q];
    switch (put.mode[q]) {
        case 0:
            Tm[(int64_t)i * ldt + k] = s;
            Tm[(int64_t)k * ldt + i] = s;
            break;
        case 1:
            rho[(int64_t)i * p + k] = s;
            break;
        case 3:
            Tm[(int64_t)i * ldt + i] = s;
            if (fabs(s) > scal[1]) scal[1] = fabs(s);
            break;
        default:
            break;
    }
}

// y_q -= res[q] * x for every y of the list
template <typename T>
__global__ void __launch_bounds__(256) kbl_axpys(T *__restrict__ base, int64_t xo, VecList ys,
                                                 int64_t dim, const double *__restrict__ res) {
    const int q = blockIdx.y;
    const double c = res[q];
    const T *x = base + xo;
    T *y = base + ys.off[q];
    const int64_t b0 = (int64_t)blockIdx.x * kChunk;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        const int64_t e = b0 + k;
        if (e < dim) y[e] = (T)fma(-c, ldd(x + e), ldd(y + e));
    }
}

// w -= sum_q T[iq][jq] v_q, the terms in list order (coefficients from T)
template <typename T>
__global__ void __launch_bounds__(256) kbl_sub_band(T *__restrict__ base, int64_t wo, VecList vs,
                                                    Put idx, int64_t dim,
                                                    const double *__restrict__ Tm, int ldt) {
    T *w = base + wo;
    const int64_t b0 = (int64_t)blockIdx.x * kChunk;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        const int64_t e = b0 + k;
        if (e >= dim) continue;
        double x = ldd(w + e);
        for (int q = 0; q < vs.n; ++q) {
            const double c = Tm[(int64_t)idx.i[q] * ldt + idx.k[q]];
            x = fma(-c, ldd(base + vs.off[q] + e), x);
        }
        w[e] = (T)x;
    }
}

// The coefficients of a new basis vector from the dots of its candidate x
// (res[0] = <x, x>, res[q] = <x, y_q>): c_q = res[q] / nrm for the n other
// candidates (into c, and into T or rho as `put` says), and nrm itself (mode
// 0: T[i][k] = T[k][i]; mode 1: rho[i][k]).
__global__ void kbl_coef(const double *__restrict__ res, int n, double nrm, Put put, int mode,
                         int i, int k, double *__restrict__ Tm, int ldt, double *__restrict__ rho,
                         int p, double *__restrict__ c) {
    const int t = threadIdx.x;
    if (t < n) {
        const double v = res[t + 1] / nrm;
        c[t] = v;
        if (put.mode[t] == 0) {
            Tm[(int64_t)put.i[t] * ldt + put.k[t]] = v;
            Tm[(int64_t)put.k[t] * ldt + put.i[t]] = v;
        } else {
            rho[(int64_t)put.i[t] * p + put.k[t]] = v;
        }
    }
    if (t == 0) {
        if (mode == 0) {
            Tm[(int64_t)i * ldt + k] = nrm;
            Tm[(int64_t)k * ldt + i] = nrm;
        } else {
            rho[(int64_t)i * p + k] = nrm;
        }
    }
}

// The new basis vector and the other candidates in one pass: v = x / nrm in
// place (inv = 1 / nrm), then y_q -= c_q v for each other candidate, every
// value rounded once to the storage type.  It also leaves the partial sums
// of the next step's dots, from the stored values, in kbl_dots's layout and
// order: <y_0, y_0> in row 0 and <y_0, y_q> in row q (ys lists the other
// candidates in order, y_0 the next one to become a basis vector).
template <typename T>
__global__ void __launch_bounds__(256) kbl_orth(T *__restrict__ base, int64_t xo, VecList ys,
                                                int64_t dim, int nchunks, double inv,
                                                const double *__restrict__ c,
                                                double *__restrict__ partial) {
    __shared__ double sh[256];
    const int n = ys.n;
    T *x = base + xo;
    const int64_t b0 = (int64_t)blockIdx.x * kChunk;
    double acc[kBandMaxP];
#pragma unroll
    for (int q = 0; q < kBandMaxP; ++q) acc[q] = 0.0;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        const int64_t e = b0 + k;
        if (e >= dim) break;
        const T vt = (T)(ldd(x + e) * inv);
        x[e] = vt;
        if (n == 0) continue;
        const double v = (double)vt;
        T *y0 = base + ys.off[0];
        const T a0 = (T)fma(-c[0], v, ldd(y0 + e));
        y0[e] = a0;
        const double a = (double)a0;
        acc[0] = fma(a, a, acc[0]);
#pragma unroll
        for (int q = 1; q < kBandMaxP; ++q) {
            if (q < n) {
                T *yq = base + ys.off[q];
                const T bt = (T)fma(-c[q], v, ldd(yq + e));
                yq[e] = bt;
                acc[q] = fma(a, (double)bt, acc[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kBandMaxP; ++q) {
        if (q < n) {
            const double t = block_sum(acc[q], sh);
            if (threadIdx.x == 0) partial[(int64_t)q * nchunks + blockIdx.x] = t;
        }
    }
}

constexpr int kJacT = 1024;   // threads of the eigen-solver workgroup

// sum over the kJacT threads of one workgroup, fixed tree
__device__ __forceinline__ double jac_sum(double x, double *sh) {
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int s = kJacT / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// sum over the 64 lanes of a wave (xor butterfly: every lane gets the same bits)
__device__ __forceinline__ double wave_sum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Householder reduction of the symmetric R x R matrix A (leading block, row
// stride lda; overwritten) to tridiagonal form, diagonal into dg[0..R-1] and
// couplings into of[0..R-2] (LDS).  Step k reflects the column below the
// diagonal onto its first entry: A22 <- (I - tau v v^T) A22 (I - tau v v^T),
// applied as A22 -= v q^T + q v^T with p = tau A22 v, q = p - (tau v.p / 2) v.
// The p rows of W (row stride ldw) are reflected too, W <- W (I - tau v v^T),
// one wave per row, so that W = B^T on entry ends as B^T P with T = P Tri P^T.
// Called by all kJacT threads; ends synchronised.
__device__ void house_tridiag(double *__restrict__ A, int lda, int R, double *v, double *q,
                              double *dg, double *of, double *sh, double *W, int p, int ldw) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int k = 0; k + 2 < R; ++k) {
        const int m = R - k - 1;                     // entries below the diagonal
        const int64_t b = (int64_t)(k + 1) * lda + (k + 1);   // A22 origin
        double tail = 0.0;
        for (int i = t; i < m; i += kJacT) {
            const double x = A[(int64_t)(k + 1 + i) * lda + k];
            v[i] = x;
            if (i > 0) tail = fma(x, x, tail);
        }
        const double s_tail = jac_sum(tail, sh);     // synchronises: v is complete
        const double x0 = v[0];
        if (t == 0) dg[k] = A[(int64_t)k * lda + k];
        if (!(s_tail > 0.0)) {                       // the column is reduced already
            if (t == 0) of[k] = x0;
            __syncthreads();
            continue;
        }
        const double nrm = sqrt(fma(x0, x0, s_tail));
        const double alpha = x0 > 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;                // no cancellation: opposite signs
        const double tau = 2.0 / fma(v0, v0, s_tail);
        if (t == 0) of[k] = alpha;
        __syncthreads();
        if (t == 0) v[0] = v0;
        __syncthreads();
        for (int mu = wv; mu < p; mu += kJacT / 64) {
            double *w = W + (int64_t)mu * ldw + (k + 1);
            double d = 0.0;
            for (int i = lane; i < m; i += 64) d = fma(w[i], v[i], d);
            d = tau * wave_sum(d);
            for (int i = lane; i < m; i += 64) w[i] = fma(-d, v[i], w[i]);
        }
        // p = tau A22 v, one thread per entry, reading a column of the
        // symmetric A22 (lanes of a wave stay within one row)
        double part = 0.0;
        for (int i = t; i < m; i += kJacT) {
            double acc = 0.0;
            for (int j = 0; j < m; ++j) acc = fma(A[b + (int64_t)j * lda + i], v[j], acc);
            q[i] = tau * acc;
            part = fma(v[i], q[i], part);
        }
        const double K = 0.5 * tau * jac_sum(part, sh);
        for (int i = t; i < m; i += kJacT) q[i] = fma(-K, v[i], q[i]);
        __syncthreads();
        for (int64_t e = t; e < (int64_t)m * m; e += kJacT) {
            const int i = (int)(e / m), j = (int)(e % m);
            A[b + (int64_t)i * lda + j] -= v[i] * q[j] + q[i] * v[j];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (R >= 2) {
            dg[R - 2] = A[(int64_t)(R - 2) * lda + (R - 2)];
            of[R - 2] = A[(int64_t)(R - 1) * lda + (R - 2)];
        }
        dg[R - 1] = A[(int64_t)(R - 1) * lda + (R - 1)];
    }
    __syncthreads();
}

// Lowest eigenvalue of the symmetric R x R matrix A (leading block, row
// stride lda; overwritten) for the stopping rule: Householder reduction to
// tridiagonal form, then a 1025-point Sturm multisection on the tridiagonal,
// stopped at floating-point resolution.  One workgroup of kJacT threads;
// info[2] receives the eigenvalue.
__global__ void __launch_bounds__(kJacT) kbl_lowest(double *__restrict__ A, int lda, int R,
                                                    double *__restrict__ info) {
    __shared__ double sh[kJacT];
    __shared__ double v[kBandMaxR], q[kBandMaxR], dg[kBandMaxR], of[kBandMaxR];
    __shared__ double blo, bhi;
    __shared__ int first;
    const int t = threadIdx.x;
    house_tridiag(A, lda, R, v, q, dg, of, sh, nullptr, 0, 0);
    if (t == 0) {
        double lo = dg[0], hi = dg[0];               // Gershgorin
        for (int i = 0; i < R; ++i) {
            const double r = (i > 0 ? fabs(of[i - 1]) : 0.0) + (i < R - 1 ? fabs(of[i]) : 0.0);
            lo = fmin(lo, dg[i] - r);
            hi = fmax(hi, dg[i] + r);
        }
        const double pad = 1e-12 * fmax(1.0, fmax(fabs(lo), fabs(hi)));
        blo = lo - pad;
        bhi = hi + pad;
    }
    __syncthreads();
    for (int i = t; i < R - 1; i += kJacT) of[i] = of[i] * of[i];   // squares from here on
    __syncthreads();
    for (int round = 0; round < 12; ++round) {
        const double lo = blo, hi = bhi;
        if (!(hi - lo > 4e-16 * fmax(fabs(lo), fabs(hi)))) break;
        const double x = lo + (hi - lo) * (double)(t + 1) / (double)(kJacT + 1);
        // no eigenvalue below x  <=>  every pivot of the LDL^T of T - x is positive
        double piv = 1.0;
        bool below = false;
        for (int i = 0; i < R && !below; ++i) {
            piv = (dg[i] - x) - (i > 0 ? of[i - 1] / piv : 0.0);
            if (piv == 0.0) piv = -1e-300;
            below = piv < 0.0;
        }
        if (t == 0) first = kJacT;
        __syncthreads();
        if (below) atomicMin(&first, t);
        __syncthreads();
        if (t == 0) {
            const int j = first;
            blo = j == 0 ? lo : lo + (hi - lo) * (double)j / (double)(kJacT + 1);
            bhi = j == kJacT ? hi : lo + (hi - lo) * (double)(j + 1) / (double)(kJacT + 1);
        }
        __syncthreads();
    }
    if (t == 0) info[2] = 0.5 * (blo + bhi);
}

// Lambda and Q = B^T U for the symmetric R x R matrix T = U diag(Lambda) U^T
// (leading block of A, row stride lda; overwritten) and the R x p matrix B
// (row stride p).  Householder reduction to tridiagonal form, its reflections
// applied to W = B^T from the right, then implicit symmetric QR steps with
// Wilkinson shifts on the tridiagonal (each step a rotation chase from the
// top of an unreduced block to its bottom; a coupling at most eps times a
// Gershgorin bound of |T| is set to zero), each rotation applied to the
// columns of W too.  The QR phase runs in wave 0: every lane follows the same
// recurrence and lane mu (< p <= 32) carries row mu of W.  W stays in LDS
// when W_LDS (p R doubles of dynamic LDS), else it is worked on in Q itself.
// Q is p x R (row stride R).  info[0] = QR steps; info[1] = 1 if max_steps
// ran out before every coupling vanished (Lambda, Q then unusable).
constexpr size_t kEighLdsBytes = 96 * 1024;

template <bool W_LDS>
__global__ void __launch_bounds__(kJacT) kbl_eigh(double *__restrict__ A, int lda, int R,
                                                  const double *__restrict__ Bm, int p,
                                                  int max_steps, double *__restrict__ lam,
                                                  double *__restrict__ Q, double *__restrict__ info) {
    __shared__ double sh[kJacT];
    __shared__ double v[kBandMaxR], q[kBandMaxR], dg[kBandMaxR], of[kBandMaxR];
    extern __shared__ double sW[];
    double *W = W_LDS ? sW : Q;
    const int t = threadIdx.x;
    for (int64_t e = t; e < (int64_t)p * R; e += kJacT) {
        const int mu = (int)(e / R), c = (int)(e % R);
        W[e] = Bm[(int64_t)c * p + mu];
    }
    __syncthreads();
    house_tridiag(A, lda, R, v, q, dg, of, sh, W, p, R);
    if (t >= 64) return;
    const int lane = t;
    const bool own = lane < p;
    double *wr = W + (int64_t)(own ? lane : 0) * R;
    // couplings at most eps times a Gershgorin bound of |T| count as zero
    double tn = 0.0;
    for (int r = lane; r < R; r += 64)
        tn = fmax(tn, fabs(dg[r]) + (r > 0 ? fabs(of[r - 1]) : 0.0) + (r + 1 < R ? fabs(of[r]) : 0.0));
    for (int o = 32; o > 0; o >>= 1) tn = fmax(tn, __shfl_xor(tn, o));
    const double thr = 2.220446049250313e-16 * tn;
    int hi = R - 1, steps = 0, ok = 1;
    while (hi > 0) {
        // lo: first index of the unreduced block that ends at hi
        int lo = 0;
        for (int top = hi - 1; top >= 0; top -= 64) {
            const int i = top - lane;
            bool neg = false;
            if (i >= 0) neg = !(fabs(of[i]) > thr);
            const uint64_t mk = __ballot(neg);
            if (mk) {
                const int l = __ffsll((unsigned long long)mk) - 1;   // highest such index
                lo = top - l + 1;
                if (lane == l) of[i] = 0.0;
                break;
            }
        }
        if (lo == hi) {
            --hi;
            continue;
        }
        if (steps >= max_steps) {
            ok = 0;
            break;
        }
        ++steps;
        // Wilkinson shift: the eigenvalue of the trailing 2 x 2 nearer its last entry
        const double a = dg[hi - 1], bb = of[hi - 1], cN = dg[hi];
        const double dl = 0.5 * (a - cN);
        const double h = hypot(dl, bb);
        const double shift = cN - bb * (bb / (dl + (dl >= 0.0 ? h : -h)));
        // chase: the rotation in plane (k, k+1) maps rows (k, k+1) to
        // (c r_k + s r_k+1, -s r_k + c r_k+1) and the columns alike; the first
        // one follows the shifted first column, the others remove the bulge
        // at (k+1, k-1) that the previous one left
        double x = dg[lo] - shift, z = of[lo];
        double dk = dg[lo], ek = of[lo];
        double wk = own ? wr[lo] : 0.0;
        // the entries of row k + 1 are loaded one rotation ahead
        double nd = dg[lo + 1], nek = lo + 1 < hi ? of[lo + 1] : 0.0;
        double nw = own ? wr[lo + 1] : 0.0;
        for (int k = lo; k < hi; ++k) {
            const double dk1 = nd, ek1 = nek, wk1 = nw;
            if (k + 2 <= hi) {
                nd = dg[k + 2];
                nek = k + 2 < hi ? of[k + 2] : 0.0;
                nw = own ? wr[k + 2] : 0.0;
            }
            // r = |(x, z)| and its reciprocal from one square root; the
            // scaled form only where the squares could under- or overflow
            const double r2 = fma(x, x, z * z);
            double r, c = 1.0, s = 0.0;
            if (r2 > 1e-280 && r2 < 1e280) {
                const double ir = rsqrt(r2);
                r = r2 * ir;
                c = x * ir;
                s = z * ir;
            } else {
                r = hypot(x, z);
                if (r > 0.0) {
                    const double ir = 1.0 / r;
                    c = x * ir;
                    s = z * ir;
                }
            }
            if (k > lo) of[k - 1] = r;
            const double cs = c * s, c2 = c * c, s2 = s * s, tb = 2.0 * cs * ek;
            dg[k] = c2 * dk + s2 * dk1 + tb;
            const double ne = cs * (dk1 - dk) + (c2 - s2) * ek;
            dk = s2 * dk + c2 * dk1 - tb;
            if (own) wr[k] = c * wk + s * wk1;
            wk = c * wk1 - s * wk;
            if (k + 1 < hi) {
                x = ne;
                z = s * ek1;
                ek = c * ek1;
            } else {
                of[k] = ne;
            }
        }
        dg[hi] = dk;
        if (own) wr[hi] = wk;
    }
    for (int r = lane; r < R; r += 64) lam[r] = dg[r];
    if (W_LDS)
        for (int64_t e = lane; e < (int64_t)p * R; e += 64) Q[e] = sW[e];
    if (lane == 0) {
        info[0] = steps;
        info[1] = ok ? 0.0 : 1.0;
    }
}

// Lambda and Q of one part (T in A, the start-state projections in Bm)
static int eigh_launch(double *A, int lda, int R, const double *Bm, int p, int max_steps,
                       double *lam, double *Q, double *info, hipStream_t s) {
    const size_t wl = sizeof(double) * (size_t)p * R;
    if (wl <= kEighLdsBytes)
        kbl_eigh<true><<<1, kJacT, wl, s>>>(A, lda, R, Bm, p, max_steps, lam, Q, info);
    else
        kbl_eigh<false><<<1, kJacT, 0, s>>>(A, lda, R, Bm, p, max_steps, lam, Q, info);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

// G[z][mu][nu] = sum_r Qe_mu,r Qe_nu,r / (z + E0 - le_r) + Qh_mu,r Qh_nu,r / (z - E0 + lh_r)
__global__ void kbl_green(const double *__restrict__ Qe, const double *__restrict__ le, int Re,
                          const double *__restrict__ Qh, const double *__restrict__ lh, int Rh,
                          int p, int nz, const double *__restrict__ zs, double e0,
                          double *__restrict__ G) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nz * p * p) return;
    const int iz = (int)(e / (p * p)), mn = (int)(e % (p * p));
    const int mu = mn / p, nu = mn % p;
    const double zr = zs[2 * iz], zi = zs[2 * iz + 1];
    double gr = 0.0, gi = 0.0;
    for (int r = 0; r < Re; ++r) {
        const double w = Qe[(int64_t)mu * Re + r] * Qe[(int64_t)nu * Re + r];
        const double dr = zr + e0 - le[r], den = dr * dr + zi * zi;
        gr += w * dr / den;
        gi -= w * zi / den;
    }
    for (int r = 0; r < Rh; ++r) {
        const double w = Qh[(int64_t)mu * Rh + r] * Qh[(int64_t)nu * Rh + r];
        const double dr = zr - e0 + lh[r], den = dr * dr + zi * zi;
        gr += w * dr / den;
        gi -= w * zi / den;
    }
    G[2 * e] = gr;
    G[2 * e + 1] = gi;
}

// ---------------------------------------------------------------- host side

struct BandPart {
    int valid = 0;
    SpinTables up{};
    HvOp op;
    int64_t dim = 0;
    int nchunks = 1;
    char *pool = nullptr;        // slots of dim elements
    int nslot = 0;
    double *Tm = nullptr, *rho = nullptr, *lam = nullptr, *Q = nullptr;
    double *Tc = nullptr;        // copy of T for the convergence test (etol > 0)
    double *partial = nullptr, *res = nullptr, *scal = nullptr, *info = nullptr;
    double *ahead = nullptr;     // partial dots of the next candidate, [kBandMaxP + 1][nchunks]
    double *cq = nullptr;        // coefficients c_q of the candidates against a new basis vector
    int R = 0;
};

struct BandLayout {
    ModelDev md;
    HopTables hd;
    int32_t *ops = nullptr;
    double *zd = nullptr, *G = nullptr;
    BandPart part[2];
};

static int band_layout(const qcm_model *m, const qcm_basis *gs, const qcm_band_opts *o, int n_z,
                       Carver &cv, hipStream_t s, BandLayout *B) {
    const int L = m->L, p = o->n_orb, Rm = o->max_basis;
    const size_t vs = o->prec == QCM_FP64 ? 8 : 4;
    QCM_TRY(upload_model(m, cv, &B->md, s));
    SpinTables dn = spin_from_basis(gs, 1);
    QCM_TRY(build_hop_tables(B->md, dn, cv, &B->hd, s, count_bonds(m)));
    B->ops = cv.take<int32_t>(2 * (size_t)p);
    B->zd = cv.take<double>(2 * (size_t)(n_z > 0 ? n_z : 1));
    for (int part = 0; part < 2; ++part) {
        BandPart &P = B->part[part];
        const int nup2 = part == 0 ? gs->n_up + 1 : gs->n_up - 1;
        P.valid = nup2 >= 0 && nup2 <= L;
        if (!P.valid) continue;
        QCM_TRY(build_spin_tables(L, nup2, cv, &P.up, s));
        P.op.md = B->md;
        P.op.up = P.up;
        P.op.dn = dn;
        P.op.hd = B->hd;
        P.op.dim = P.up.d * dn.d;
        QCM_TRY(build_hop_tables(B->md, P.up, cv, &P.op.hu, s, count_bonds(m)));
        P.op.split = 0;
        if (split_applies(m, nup2, P.up.d, dn.d)) QCM_TRY(split_prepare(m, P.op, cv, s));
        P.dim = P.op.dim;
        P.nchunks = (int)std::max<int64_t>(1, (int64_t)ceil_div(P.dim, kChunk));
        P.nslot = 3 * p + 3;
        P.pool = cv.take<char>(vs * (size_t)P.dim * P.nslot);
        P.Tm = cv.take<double>((size_t)Rm * Rm);
        P.rho = cv.take<double>((size_t)Rm * p);
        if (o->etol > 0.0) P.Tc = cv.take<double>((size_t)Rm * Rm);
        P.lam = cv.take<double>(Rm);
        P.Q = cv.take<double>((size_t)p * Rm);
        P.partial = cv.take<double>((size_t)(kBandMaxP + 1) * P.nchunks);
        P.ahead = cv.take<double>((size_t)(kBandMaxP + 1) * P.nchunks);
        P.cq = cv.take<double>(kBandMaxP + 1);
        P.res = cv.take<double>(kBandMaxP + 1);
        P.scal = cv.take<double>(8);
        P.info = cv.take<double>(8);
    }
    B->G = cv.take<double>(2 * (size_t)(n_z > 0 ? n_z : 1) * p * p);
    return QCM_OK;
}

// The stream (default priority), events and pinned result of the stopping
// tests, which run beside the recurrence.  They are created once and kept in
// a process-wide pool for the life of the process: a call leases a free set
// of its device (creating one only when none is free, so concurrent calls from
// other host threads get sets of their own) and returns it, after its side
// stream has drained, on every way out of band_run.  Later calls therefore
// create and destroy nothing (stream and pinned-memory teardown can wait for
// the whole device).
struct SideRes {
    int dev = -1;
    hipStream_t s = nullptr;
    hipEvent_t copied = nullptr, done = nullptr;
    double *h_theta = nullptr;
};
static std::mutex g_side_mu;
static std::vector<SideRes *> g_side_free;

struct SideTest {
    hipStream_t s = nullptr;
    hipEvent_t copied = nullptr, done = nullptr;
    double *h_theta = nullptr;
    SideRes *r = nullptr;
    int lease() {
        int dev = -1;
        QCM_HIP(hipGetDevice(&dev));
        {
            std::lock_guard<std::mutex> lock(g_side_mu);
            for (size_t k = 0; k < g_side_free.size(); ++k)
                if (g_side_free[k]->dev == dev) {
                    r = g_side_free[k];
                    g_side_free.erase(g_side_free.begin() + k);
                    break;
                }
        }
        if (!r) {
            SideRes *n = new SideRes();
            n->dev = dev;
            hipError_t e = hipStreamCreateWithFlags(&n->s, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&n->copied, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&n->done, hipEventDisableTiming);
            if (e == hipSuccess)
                e = hipHostMalloc((void **)&n->h_theta, sizeof(double), hipHostMallocDefault);
            if (e != hipSuccess) {
                if (n->h_theta) (void)hipHostFree(n->h_theta);
                if (n->done) (void)hipEventDestroy(n->done);
                if (n->copied) (void)hipEventDestroy(n->copied);
                if (n->s) (void)hipStreamDestroy(n->s);
                delete n;
                return fail(QCM_EHIP, "band Lanczos side stream: %s", hipGetErrorString(e));
            }
            r = n;
        }
        s = r->s;
        copied = r->copied;
        done = r->done;
        h_theta = r->h_theta;
        return QCM_OK;
    }
    ~SideTest() {
        if (!r) return;
        (void)hipStreamSynchronize(r->s);
        std::lock_guard<std::mutex> lock(g_side_mu);
        g_side_free.push_back(r);
    }
};

template <typename T>
static int band_run(const qcm_band_opts *o, BandPart &P, const double *d_gs, int64_t d_src_up,
                    const SpinTables &src_up, int kind, const int32_t *ops, hipStream_t s) {
    const int p = o->n_orb, Rm = o->max_basis, ldt = Rm;
    const int64_t dim = P.dim;
    const int nch = P.nchunks;
    T *base = (T *)P.pool;
    auto off = [&](int slot) { return (int64_t)slot * dim; };
    const dim3 g1((unsigned)nch, 1);
    QCM_HIP(hipMemsetAsync(P.Tm, 0, sizeof(double) * (size_t)Rm * Rm, s));
    QCM_HIP(hipMemsetAsync(P.rho, 0, sizeof(double) * (size_t)Rm * p, s));
    QCM_HIP(hipMemsetAsync(P.scal, 0, sizeof(double) * 8, s));
    // start vectors into slots 0..p-1
    QCM_TRY(apply_ops_raw(sizeof(T) == 8 ? QCM_FP64 : QCM_FP32V, d_gs, d_src_up, src_up, P.up, dim,
                          kind, ops, p, base, nch, P.partial, s));
    std::vector<int> freeslots;
    for (int q = P.nslot - 1; q >= p; --q) freeslots.push_back(q);
    std::map<int, int> cand;   // candidate index -> slot
    std::map<int, int> vslot;  // basis index -> slot
    for (int q = 0; q < p; ++q) cand[q + 1] = q;
    std::set<int> I;
    int pc = p;
    double scale = 1.0;
    int j = 0;
    double host[2];
    bool ahead = false;
    bool have_prev = false;
    double theta_prev = 0.0;
    // The paper's stopping rule, once per block: the lowest eigenvalue of T_j
    // (on a copy) against the one a block earlier.  Each test runs on a side
    // stream while the recurrence goes on; when a test at j_t finds
    // convergence the part ends at R = j_t, exactly as if it had stopped
    // there: later steps only add rows and columns to T and rho, so their
    // leading j_t block is final once step j_t is done.
    SideTest side;
    int pend_j = 0;   // basis size of the test in flight (0: none)
    int stop_at = 0;  // basis size a finished test stopped the part at
    bool near = false;
    double prev_d = 0.0;  // the change of the lowest eigenvalue at the last test
    if (o->etol > 0.0) QCM_TRY(side.lease());
    // take the result of the test in flight, waiting for it or only if done
    auto settle = [&](bool wait) -> int {
        if (!pend_j) return QCM_OK;
        if (wait) {
            QCM_HIP(hipEventSynchronize(side.done));
        } else {
            const hipError_t q = hipEventQuery(side.done);
            if (q == hipErrorNotReady) return QCM_OK;
            QCM_HIP(q);
        }
        const double th = *side.h_theta;
        if (have_prev && fabs(th - theta_prev) <= o->etol * std::max(1.0, fabs(th)))
            stop_at = pend_j;
        // when the change, shrinking at its last rate, would meet the
        // tolerance at the next test, the steps wait for that test rather
        // than run on speculatively
        const double d = fabs(th - theta_prev);
        near = have_prev && prev_d > 0.0 &&
               d * (d / prev_d) <= o->etol * std::max(1.0, fabs(th));
        if (have_prev) prev_d = d;
        have_prev = true;
        theta_prev = th;
        pend_j = 0;
        return QCM_OK;
    };
    while (j < Rm) {
        QCM_TRY(settle(near));
        if (stop_at) {
            P.R = stop_at;
            return QCM_OK;
        }
        ++j;
        double nrm = 0.0;
        for (;;) {
            // (1) the next candidate x = cand[j]: <x, x> (read back for the
            // deflation test) and <x, y_q> for the other candidates y_q =
            // cand[j + q], in rows 0..pc-1 of P.ahead.  The previous step's
            // passes left them there unless a deflation changed the list.
            if (!ahead) {
                VecList ys{};
                ys.n = pc;
                for (int q = 0; q < pc; ++q) ys.off[q] = off(cand[j + q]);
                kbl_dots<T><<<dim3(nch, pc), 256, 0, s>>>(base, off(cand[j]), ys, dim, nch,
                                                          P.ahead);
            }
            Put raw{};
            raw.n = pc;
            for (int q = 0; q < pc; ++q) raw.mode[q] = 2;
            kbl_finish<<<pc, 256, 0, s>>>(P.ahead, nch, raw, P.res, P.Tm, ldt, P.rho, p, P.scal);
            QCM_LAUNCH_CHECK();
            QCM_HIP(hipMemcpyAsync(host, P.res, sizeof(double), hipMemcpyDeviceToHost, s));
            QCM_HIP(hipMemcpyAsync(host + 1, P.scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
            QCM_HIP(hipStreamSynchronize(s));
            scale = std::max(1.0, host[1]);
            nrm = sqrt(host[0] > 0.0 ? host[0] : 0.0);
            if (nrm > o->dtol * scale) break;
            ahead = false;
            if (j - pc > 0) I.insert(j - pc);
            freeslots.push_back(cand[j]);
            --pc;
            if (pc == 0) {
                QCM_TRY(settle(true));
                P.R = stop_at ? stop_at : j - 1;
                return QCM_OK;
            }
            for (int k = j; k < j + pc; ++k) cand[k] = cand[k + 1];
            cand.erase(j + pc);
        }
        // (2, 3) v_j = x / nrm and the other candidates against it,
        // y_q -= (<x, y_q> / nrm) v_j, in one pass that also sums the dots of
        // the next candidate with the others
        const int sj = cand[j];
        cand.erase(j);
        vslot[j] = sj;
        {
            VecList ys{};
            Put put{};
            ys.n = put.n = pc - 1;
            for (int q = 0; q < pc - 1; ++q) {
                const int k = j + 1 + q;
                ys.off[q] = off(cand[k]);
                if (k - pc > 0) {
                    put.mode[q] = 0;
                    put.i[q] = j - 1;
                    put.k[q] = k - pc - 1;
                } else {
                    put.mode[q] = 1;
                    put.i[q] = j - 1;
                    put.k[q] = k - pc + p - 1;
                }
            }
            if (j - pc > 0)
                kbl_coef<<<1, 64, 0, s>>>(P.res, pc - 1, nrm, put, 0, j - 1, j - pc - 1, P.Tm, ldt,
                                          P.rho, p, P.cq);
            else
                kbl_coef<<<1, 64, 0, s>>>(P.res, pc - 1, nrm, put, 1, j - 1, j - pc + p - 1, P.Tm,
                                          ldt, P.rho, p, P.cq);
            kbl_orth<T><<<g1, 256, 0, s>>>(base, off(sj), ys, dim, nch, 1.0 / nrm, P.cq, P.ahead);
            QCM_LAUNCH_CHECK();
        }
        // (4) the new candidate w = H v_j
        if (freeslots.empty()) return fail(QCM_EHIP, "band Lanczos: out of vector slots");
        const int sw = freeslots.back();
        freeslots.pop_back();
        QCM_TRY(hv_launch(P.op, sizeof(T) == 8 ? QCM_FP64 : QCM_FP32V, base + off(sj),
                          base + off(sw), 1, s));
        // (5) the band of previous basis vectors, coefficients T[k][j] = T[j][k]
        {
            VecList vs{};
            Put idx{};
            for (int k = std::max(1, j - pc); k < j; ++k) {
                vs.off[vs.n] = off(vslot[k]);
                idx.i[vs.n] = k - 1;
                idx.k[vs.n] = j - 1;
                ++vs.n;
            }
            idx.n = vs.n;
            if (vs.n > 0) {
                kbl_sub_band<T><<<g1, 256, 0, s>>>(base, off(sw), vs, idx, dim, P.Tm, ldt);
                QCM_LAUNCH_CHECK();
            }
        }
        // (6) v_j and the look-back set, coefficients computed (in index order)
        std::set<int> K = I;
        K.insert(j);
        for (int k : K) {
            VecList one{};
            one.n = 1;
            one.off[0] = off(sw);
            Put put{};
            put.n = 1;
            put.mode[0] = k == j ? 3 : 0;
            put.i[0] = k - 1;
            put.k[0] = j - 1;
            kbl_dots<T><<<dim3(nch, 1), 256, 0, s>>>(base, off(vslot[k]), one, dim, nch, P.partial);
            kbl_finish<<<1, 256, 0, s>>>(P.partial, nch, put, P.res, P.Tm, ldt, P.rho, p, P.scal);
            kbl_axpys<T><<<dim3(nch, 1), 256, 0, s>>>(base, off(vslot[k]), one, dim, P.res);
            QCM_LAUNCH_CHECK();
        }
        cand[j + pc] = sw;
        // the next candidate's dot with w (row pc - 1), or its norm when w is
        // the next candidate itself
        {
            VecList one{};
            one.n = 1;
            one.off[0] = off(sw);
            const int x_next = pc > 1 ? cand[j + 1] : sw;
            kbl_dots<T><<<dim3(nch, 1), 256, 0, s>>>(base, off(x_next), one, dim, nch,
                                                     P.ahead + (size_t)(pc - 1) * nch);
            QCM_LAUNCH_CHECK();
            ahead = true;
        }
        // basis vectors older than the band and outside the look-back set are done
        for (auto it = vslot.begin(); it != vslot.end();) {
            if (it->first < j - p && !I.count(it->first)) {
                freeslots.push_back(it->second);
                it = vslot.erase(it);
            } else {
                ++it;
            }
        }
        // the stopping test at this block boundary, after the one in flight
        // (which holds the copy of T) has finished
        if (o->etol > 0.0 && j % p == 0) {
            QCM_TRY(settle(true));
            if (stop_at) break;
            QCM_HIP(hipMemcpy2DAsync(P.Tc, sizeof(double) * ldt, P.Tm, sizeof(double) * ldt,
                                     sizeof(double) * j, j, hipMemcpyDeviceToDevice, s));
            QCM_HIP(hipEventRecord(side.copied, s));
            QCM_HIP(hipStreamWaitEvent(side.s, side.copied, 0));
            kbl_lowest<<<1, kJacT, 0, side.s>>>(P.Tc, ldt, j, P.info);
            QCM_LAUNCH_CHECK();
            QCM_HIP(hipMemcpyAsync(side.h_theta, P.info + 2, sizeof(double),
                                   hipMemcpyDeviceToHost, side.s));
            QCM_HIP(hipEventRecord(side.done, side.s));
            pend_j = j;
        }
    }
    QCM_TRY(settle(true));
    P.R = stop_at ? stop_at : j;
    return QCM_OK;
}

}  // namespace qcm

using namespace qcm;

extern "C" int qcm_lehmann_form(int32_t n_orb, int32_t max_basis, double e0, const int32_t *h_R,
                                const double *h_lambda, const double *h_Q, double *h_poles,
                                double *h_Qout) {
    if (!h_R || !h_lambda || !h_Q || !h_poles || !h_Qout)
        return fail(QCM_EARG, "qcm_lehmann_form: NULL pointer");
    if (n_orb < 1 || max_basis < 1) return fail(QCM_EARG, "qcm_lehmann_form: n_orb, max_basis < 1");
    for (int k = 0; k < 2; ++k)
        if (h_R[k] < 0 || h_R[k] > max_basis)
            return fail(QCM_EARG, "qcm_lehmann_form: R[%d] = %d outside [0, %d]", k, h_R[k],
                        max_basis);
    const int Re = h_R[0], Rh = h_R[1], R = Re + Rh;
    // electron poles Lambda_e - E0 first, then hole poles E0 - Lambda_h
    for (int r = 0; r < Re; ++r) h_poles[r] = h_lambda[r] - e0;
    for (int r = 0; r < Rh; ++r) h_poles[Re + r] = e0 - h_lambda[max_basis + r];
    for (int i = 0; i < n_orb; ++i) {
        for (int r = 0; r < Re; ++r) h_Qout[(size_t)i * R + r] = h_Q[(size_t)i * max_basis + r];
        for (int r = 0; r < Rh; ++r)
            h_Qout[(size_t)i * R + Re + r] =
                h_Q[((size_t)n_orb + i) * max_basis + r];
    }
    return QCM_OK;
}

extern "C" void qcm_band_default_opts(qcm_band_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->max_basis = 400;
    o->prec = QCM_FP64;
    o->dtol = 1e-10;
    o->max_sweeps = 40;
    o->etol = 0.0;
}

extern "C" int qcm_green_band(const qcm_model *m, const qcm_basis *gs, const double *d_gs,
                              double e0, const qcm_band_opts *o, int32_t *h_R,
                              double *h_lambda, double *h_Q, int32_t n_z, const double *h_z,
                              double *d_G, void *d_ws, size_t ws_bytes, size_t *ws_needed,
                              void *stream) {
    if (!ws_needed || !o) return fail(QCM_EARG, "qcm_green_band: NULL ws_needed or opts");
    QCM_TRY(validate_model(m));
    QCM_TRY(check_basis(gs, m->L));
    const int L = m->L, p = o->n_orb;
    if (p < 1 || p > L || p > kBandMaxP || !o->orbs)
        return fail(QCM_EARG, "qcm_green_band: bad orbital list (1..%d orbitals)", kBandMaxP);
    for (int i = 0; i < p; ++i) {
        if (o->orbs[i] < 0 || o->orbs[i] >= L)
            return fail(QCM_EARG, "qcm_green_band: orbital %d out of range", o->orbs[i]);
        for (int k = 0; k < i; ++k)
            if (o->orbs[k] == o->orbs[i]) return fail(QCM_EARG, "qcm_green_band: repeated orbital");
    }
    if (o->max_basis < 1 || o->max_basis > kBandMaxR)
        return fail(QCM_EARG, "qcm_green_band: max_basis outside 1..%d", kBandMaxR);
    if (o->prec != QCM_FP64 && o->prec != QCM_FP32V)
        return fail(QCM_EARG, "qcm_green_band: bad prec");
    if (!(o->dtol > 0.0) || o->max_sweeps < 1 || !(o->etol >= 0.0))
        return fail(QCM_EARG, "qcm_green_band: need dtol > 0, max_sweeps >= 1, etol >= 0");
    if (n_z < 0 || (n_z > 0 && (!h_z || (!d_G && d_ws))))
        return fail(QCM_EARG, "qcm_green_band: bad frequency arguments");
    Carver dry(nullptr);
    BandLayout DB;
    QCM_TRY(band_layout(m, gs, o, n_z, dry, nullptr, &DB));
    const size_t need = dry.off + 256;
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (!d_gs) return fail(QCM_EARG, "qcm_green_band: d_gs is NULL");
    if (ws_bytes < need)
        return fail(QCM_EWORKSPACE, "qcm_green_band: workspace %zu < %zu", ws_bytes, need);
    hipStream_t s = as_stream(stream);
    Carver cv(d_ws);
    BandLayout B;
    QCM_TRY(band_layout(m, gs, o, n_z, cv, s, &B));
    std::vector<int32_t> ops(2 * (size_t)p);
    for (int i = 0; i < p; ++i) {
        ops[2 * i] = o->orbs[i];
        ops[2 * i + 1] = -1;
    }
    QCM_HIP(hipMemcpyAsync(B.ops, ops.data(), sizeof(int32_t) * ops.size(), hipMemcpyHostToDevice, s));
    if (n_z > 0)
        QCM_HIP(hipMemcpyAsync(B.zd, h_z, sizeof(double) * 2 * n_z, hipMemcpyHostToDevice, s));
    const SpinTables upg = spin_from_basis(gs, 0);
    int Rs[2] = {0, 0};
    for (int part = 0; part < 2; ++part) {
        BandPart &P = B.part[part];
        if (!P.valid) continue;
        if (o->prec == QCM_FP64)
            QCM_TRY(band_run<double>(o, P, d_gs, gs->d_up, upg, part, B.ops, s));
        else
            QCM_TRY(band_run<float>(o, P, d_gs, gs->d_up, upg, part, B.ops, s));
        Rs[part] = P.R;
        if (P.R > 0) {
            const int max_steps = (int)std::min<int64_t>((int64_t)o->max_sweeps * P.R, 1 << 30);
            QCM_TRY(eigh_launch(P.Tm, o->max_basis, P.R, P.rho, p, max_steps, P.lam, P.Q, P.info, s));
        }
    }
    if (n_z > 0) {
        const BandPart &Pe = B.part[0], &Ph = B.part[1];
        const int64_t tot = (int64_t)n_z * p * p;
        kbl_green<<<ceil_div(tot, 256), 256, 0, s>>>(Pe.Q, Pe.lam, Rs[0], Ph.Q, Ph.lam, Rs[1], p,
                                                    n_z, B.zd, e0, d_G);
        QCM_LAUNCH_CHECK();
    }
    if (h_R) {
        h_R[0] = Rs[0];
        h_R[1] = Rs[1];
    }
    for (int part = 0; part < 2; ++part) {
        const BandPart &P = B.part[part];
        const int R = Rs[part];
        if (R <= 0) continue;
        if (h_lambda)
            QCM_HIP(hipMemcpyAsync(h_lambda + (size_t)part * o->max_basis, P.lam,
                                   sizeof(double) * R, hipMemcpyDeviceToHost, s));
        if (h_Q)
            for (int mu = 0; mu < p; ++mu)
                QCM_HIP(hipMemcpyAsync(h_Q + ((size_t)part * p + mu) * o->max_basis,
                                       P.Q + (size_t)mu * R, sizeof(double) * R,
                                       hipMemcpyDeviceToHost, s));
    }
    double einfo[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int part = 0; part < 2; ++part)
        if (Rs[part] > 0)
            QCM_HIP(hipMemcpyAsync(einfo[part], B.part[part].info, sizeof einfo[part],
                                   hipMemcpyDeviceToHost, s));
    QCM_HIP(hipStreamSynchronize(s));
    for (int part = 0; part < 2; ++part)
        if (einfo[part][1] != 0.0)
            return fail(QCM_EARG, "qcm_green_band: the eigenproblem of T (part %d) did not converge "
                        "in %d QR steps (non-finite input?)", part, (int)einfo[part][0]);
    return QCM_OK;
}
