// One Lanczos step of a group of chains, as three passes over the vectors
// (internal; used by the single-solve engine and by the batched engine).
//
// A group is nvec chains in one sector (vectors [nvec][dim], consecutive).
// With v = v_n, vp = v_{n-1}, beta' = beta_{n-1}:
//   pass 1  w = H v - beta' vp, stored; partial sums of <v, w>
//           (fused into the product when rows of V fit in LDS, with the dots
//           <w, w>, <v, v> (<vp, w>, <vp, v>) that then replace pass 2;
//           otherwise the product runs first and a chunked pass subtracts and
//           sums);
//   finish  alpha_n = <v, w>;
//   pass 2  x = w - alpha_n v (not stored): partial sums of |x|^2 and, with
//           local reorthogonalisation, of <v, x> and <vp, x> (after the
//           two-pass product these come from dots its last pass already
//           summed, and this pass is skipped);
//   finish  c1 = <v, x>, c2 = <vp, x>; alpha_n += c1;
//           beta_n^2 = |x|^2 - c1^2 - c2^2 (the norm of x - c1 v - c2 vp for
//           unit v, vp orthogonal to each other, up to terms of order c^2 eps);
//   pass 3  v_{n+1} = (x - c1 v - c2 vp) / beta_n, rounded once to the storage
//           type (optionally also psi += s_n v_n for the ground-state replay).
// After the two-pass product the two finishes are ks_dots_stage and
// ks_finish_dots, and pass 3 may be deferred into the next step's in-row
// pass, which forms v_{n+1} element by element with the same operations when
// it stages a row.
// Every sum is a fixed-order two-level reduction (per block or per chunk of
// kChunk elements, then per chain), so results depend only on the inputs and
// the sector shape, not on the launch or on other groups sharing it.
#pragma once

#include "lanczos_device.h"

namespace qcm {

// Elements of V a product block stages in LDS (at least one whole row).
constexpr int64_t kTileElems = 2048;
// LDS a fused product block may use (row tile + lookup tables).
constexpr size_t kFusedLds = 144 * 1024;

// Everything a step kernel needs about one group.
struct BGroup {
    // sector and Hamiltonian (fused product)
    int64_t d_up, d_dn, dim;
    const uint32_t *su, *sd;
    const double *eu, *ed;
    const int32_t *nhu, *nhd, *colu, *cold;
    const double *cfu, *cfd;
    const double *ulut;
    const uint32_t *pku;   // packed up hops: column | (ctab index << 16), slot-major
    const double *ctab;    // hop coefficients by index (+-t_ab)
    double u_uniform;
    int32_t nbytes;
    int32_t nctab;
    int32_t rows;      // rows of V per product block
    int32_t nblk;      // product blocks per vector
    int32_t nvec, nchunks;
    int32_t na;        // alpha partials per vector (nblk when fused, else nchunks)
    int64_t pstride;   // two-pass product: stride between its five partial arrays
    int32_t n;         // step index
    int32_t reorth;
    const void *vp, *v;
    void *w;
    double *pa;        // [nvec][na]
    double *pn;        // [nvec][3][nchunks]
    double *psi;       // ground-state replay: psi += svec[n] v_n in pass 3 (or NULL)
    const double *svec;
    ChainState cs;
};

__device__ __forceinline__ int find_group(const int64_t *__restrict__ begin, int ng, int64_t x) {
    int lo = 0, hi = ng - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Work sources: many groups through a table and prefix sums of their work
// items, or one group passed by value.
struct TabSrc {
    const BGroup *G;
    const int64_t *begin;
    int ng;
    __device__ __forceinline__ const BGroup &at(int64_t x, int64_t *local) const {
        const int g = find_group(begin, ng, x);
        *local = x - begin[g];
        return G[g];
    }
};
struct OneSrc {
    BGroup g;
    __device__ __forceinline__ const BGroup &at(int64_t x, int64_t *local) const {
        *local = x;
        return g;
    }
};

inline void row_shape(int64_t d_up, int64_t d_dn, int prec, int32_t *rows, int32_t *nblk) {
    (void)prec;
    int64_t r = kTileElems / (d_up > 0 ? d_up : 1);
    if (r < 1) r = 1;
    if (r > d_dn) r = d_dn;
    if (r < 1) r = 1;
    *rows = (int32_t)r;
    *nblk = (int32_t)((d_dn + r - 1) / r);
}

inline size_t fused_lds(int64_t d_up, int32_t rows, int prec, int nbytes, double u_uniform,
                        int nctab) {
    const size_t lut = u_uniform >= 0.0 ? 0 : sizeof(double) * 256 * (size_t)nbytes;
    return lut + sizeof(double) * (size_t)nctab +
           (prec == QCM_FP64 ? 8 : 4) * (size_t)rows * (size_t)d_up;
}

// The group of chains of an engine at step n (vectors from its rotation).
BGroup engine_group(const Engine &e, int n);

// pass 1, fused: w = H v - beta' vp for `rows` rows of V held in LDS; one
// thread per element.  The in-row term gathers inside the LDS rows through
// the packed up-hop entries (coefficients from a small LDS table); the
// row-mixing term streams neighbour rows from global memory; the diagonal
// comes from the two strings.  Hop loads are issued four at a time so that
// several are in flight per thread.  Sum order per element: diagonal, up hops
// in list order, down hops in list order, then -beta' vp; all FP64, rounded
// once.  pa != NULL: partial <v, w> per block.
template <typename T, class Src>
__global__ void __launch_bounds__(256) ks_hv(Src src) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double sh[256];
    int64_t local;
    const BGroup &q = src.at(blockIdx.x, &local);
    const int64_t vec = local / q.nblk;
    const int64_t rb = local - vec * q.nblk;
    const int64_t d_up = q.d_up, d_dn = q.d_dn;
    const int64_t row0 = rb * q.rows;
    const int64_t nr = min((int64_t)q.rows, d_dn - row0);
    const int nlut = q.u_uniform >= 0.0 ? 0 : q.nbytes * 256;
    double *lut = reinterpret_cast<double *>(smem_raw);
    double *ct = lut + nlut;
    T *row = reinterpret_cast<T *>(ct + q.nctab);
    const auto v = gp((const T *)q.v) + vec * q.dim;
    const auto vp = gp((const T *)q.vp) + vec * q.dim;
    const auto w = gp((T *)q.w) + vec * q.dim;
    const auto su = gp(q.su), pku = gp(q.pku), sd = gp(q.sd);
    const auto nhu = gp(q.nhu), nhd = gp(q.nhd), cold = gp(q.cold);
    const auto eu = gp(q.eu), ed = gp(q.ed), cfd = gp(q.cfd);
    const bool sub = q.n > 0 && q.pa;
    const double b = sub ? q.cs.beta[vec * q.cs.maxs + q.n - 1] : 0.0;
    for (int k = threadIdx.x; k < nlut; k += 256) lut[k] = gp(q.ulut)[k];
    for (int k = threadIdx.x; k < q.nctab; k += 256) ct[k] = gp(q.ctab)[k];
    const int64_t nel = nr * d_up;
    const auto vblk = v + row0 * d_up;
    for (int64_t k = threadIdx.x; k < nel; k += 256) row[k] = vblk[k];
    __syncthreads();
    const uint32_t du = (uint32_t)d_up;
    double pa = 0.0, pww = 0.0, pvv = 0.0, ppw = 0.0, ppv = 0.0;
    // one element: diagonal, in-row hops through the packed entries, row-mixing
    // hops from global memory, -beta vp, rounded once
    // diagonal and in-row part of one element: returns the partial sum and v_i
    auto in_row = [&](uint32_t r, uint32_t iu, uint32_t sdn, double edn, double *vi_out) -> double {
        const uint32_t dbl = su[iu] & sdn;
        double diag = eu[iu] + edn;
        if (q.u_uniform >= 0.0) {
            diag += q.u_uniform * (double)__popc(dbl);
        } else {
            for (int byte = 0; byte < q.nbytes; ++byte)
                diag += lut[byte * 256 + ((dbl >> (8 * byte)) & 255u)];
        }
        const T *rr = row + (int64_t)r * d_up;
        const double vi = (double)rr[iu];
        *vi_out = vi;
        double acc = diag * vi;
        const int nh_u = nhu[iu];
        const auto pp = pku + iu;
        int s = 0;
        for (; s + 4 <= nh_u; s += 4) {
            const uint32_t p0 = pp[(int64_t)s * d_up], p1 = pp[(int64_t)(s + 1) * d_up];
            const uint32_t p2 = pp[(int64_t)(s + 2) * d_up], p3 = pp[(int64_t)(s + 3) * d_up];
            const double x0 = (double)rr[p0 & 0xffffu], x1 = (double)rr[p1 & 0xffffu];
            const double x2 = (double)rr[p2 & 0xffffu], x3 = (double)rr[p3 & 0xffffu];
            acc = fma(ct[p0 >> 16], x0, acc);
            acc = fma(ct[p1 >> 16], x1, acc);
            acc = fma(ct[p2 >> 16], x2, acc);
            acc = fma(ct[p3 >> 16], x3, acc);
        }
        for (; s < nh_u; ++s) {
            const uint32_t p0 = pp[(int64_t)s * d_up];
            acc = fma(ct[p0 >> 16], (double)rr[p0 & 0xffffu], acc);
        }
        return acc;
    };
    // -beta vp, round once, store, and the partials <v, w>, <w, w>, <v, v>
    // (with reorthogonalisation also <vp, w>, <vp, v>)
    auto finish = [&](int64_t i, double acc, double vi) {
        const double pv = sub ? ldd(vp + i) : 0.0;
        if (sub) acc = fma(-b, pv, acc);
        const T wt = (T)acc;
        w[i] = wt;
        const double wd = (double)wt;
        pa = fma(vi, wd, pa);
        pww = fma(wd, wd, pww);
        pvv = fma(vi, vi, pvv);
        if (q.reorth) {
            ppw = fma(pv, wd, ppw);
            ppv = fma(pv, vi, ppv);
        }
    };
    // one element: diagonal, in-row hops through the packed entries, row-mixing
    // hops from global memory, -beta vp, rounded once
    auto element = [&](uint32_t r, uint32_t iu, int64_t idn, uint32_t sdn, double edn, int nh_d,
                       gptr<const int32_t> cold_r, gptr<const double> cfd_r) {
        double vi;
        double acc = in_row(r, iu, sdn, edn, &vi);
        // row-mixing term (hop s of row idn at cold_r[s * d_dn])
        const auto vc = v + iu;
        int s = 0;
        for (; s + 4 <= nh_d; s += 4) {
            const int64_t e0 = (int64_t)s * d_dn, e1 = e0 + d_dn;
            const int64_t e2 = e1 + d_dn, e3 = e2 + d_dn;
            const double x0 = (double)vc[(int64_t)cold_r[e0] * d_up];
            const double x1 = (double)vc[(int64_t)cold_r[e1] * d_up];
            const double x2 = (double)vc[(int64_t)cold_r[e2] * d_up];
            const double x3 = (double)vc[(int64_t)cold_r[e3] * d_up];
            acc = fma(cfd_r[e0], x0, acc);
            acc = fma(cfd_r[e1], x1, acc);
            acc = fma(cfd_r[e2], x2, acc);
            acc = fma(cfd_r[e3], x3, acc);
        }
        for (; s < nh_d; ++s) {
            const int64_t e0 = (int64_t)s * d_dn;
            acc = fma(cfd_r[e0], (double)vc[(int64_t)cold_r[e0] * d_up], acc);
        }
        finish(idn * d_up + iu, acc, vi);
    };
    if (d_up >= 1024) {
        // long rows: the rows one after another, so the row index and its
        // down-hop list are wave-uniform (scalar loads) and no division is
        // needed.  Each thread takes two elements of the row at a time (iu and
        // iu + 256): they share the down-hop list, so their row-mixing gathers
        // are issued together; each element's sum keeps its own order.
        for (uint32_t r = 0; r < (uint32_t)nr; ++r) {
            const int64_t idn = row0 + r;
            const uint32_t sdn = sd[idn];
            const double edn = ed[idn];
            const int nh_d = nhd[idn];
            const auto cold_r = cold + idn;
            const auto cfd_r = cfd + idn;
            for (uint32_t iu = threadIdx.x; iu < du; iu += 512) {
                const uint32_t iu2 = iu + 256;
                if (iu2 >= du) {
                    element(r, iu, idn, sdn, edn, nh_d, cold_r, cfd_r);
                    continue;
                }
                double vi1, vi2;
                double a1 = in_row(r, iu, sdn, edn, &vi1);
                double a2 = in_row(r, iu2, sdn, edn, &vi2);
                const auto vc1 = v + iu, vc2 = v + iu2;
                int s = 0;
                for (; s + 4 <= nh_d; s += 4) {
                    const int64_t e0 = (int64_t)s * d_dn, e1 = e0 + d_dn;
                    const int64_t e2 = e1 + d_dn, e3 = e2 + d_dn;
                    const int64_t o0 = (int64_t)cold_r[e0] * d_up, o1 = (int64_t)cold_r[e1] * d_up;
                    const int64_t o2 = (int64_t)cold_r[e2] * d_up, o3 = (int64_t)cold_r[e3] * d_up;
                    const double x0 = (double)vc1[o0], y0 = (double)vc2[o0];
                    const double x1 = (double)vc1[o1], y1 = (double)vc2[o1];
                    const double x2 = (double)vc1[o2], y2 = (double)vc2[o2];
                    const double x3 = (double)vc1[o3], y3 = (double)vc2[o3];
                    const double c0 = cfd_r[e0], c1 = cfd_r[e1], c2 = cfd_r[e2], c3 = cfd_r[e3];
                    a1 = fma(c0, x0, a1);
                    a2 = fma(c0, y0, a2);
                    a1 = fma(c1, x1, a1);
                    a2 = fma(c1, y1, a2);
                    a1 = fma(c2, x2, a1);
                    a2 = fma(c2, y2, a2);
                    a1 = fma(c3, x3, a1);
                    a2 = fma(c3, y3, a2);
                }
                for (; s < nh_d; ++s) {
                    const int64_t e0 = (int64_t)s * d_dn;
                    const int64_t o0 = (int64_t)cold_r[e0] * d_up;
                    a1 = fma(cfd_r[e0], (double)vc1[o0], a1);
                    a2 = fma(cfd_r[e0], (double)vc2[o0], a2);
                }
                finish(idn * d_up + iu, a1, vi1);
                finish(idn * d_up + iu2, a2, vi2);
            }
        }
    } else {
        for (int64_t e = threadIdx.x; e < nel; e += 256) {
            const uint32_t r = (uint32_t)e / du;
            const uint32_t iu = (uint32_t)e - r * du;
            const int64_t idn = row0 + r;
            element(r, iu, idn, sd[idn], ed[idn], nhd[idn], cold + idn, cfd + idn);
        }
    }
    if (q.pa) {
        double *o = q.pa + vec * q.na + rb;
        const double t0 = block_sum(pa, sh);
        const double t1 = block_sum(pww, sh);
        const double t2 = block_sum(pvv, sh);
        if (threadIdx.x == 0) {
            o[0] = t0;
            o[q.pstride] = t1;
            o[2 * q.pstride] = t2;
        }
        if (q.reorth) {
            const double t3 = block_sum(ppw, sh);
            const double t4 = block_sum(ppv, sh);
            if (threadIdx.x == 0) {
                o[3 * q.pstride] = t3;
                o[4 * q.pstride] = t4;
            }
        }
    }
}

// chunk of a chunked pass
struct ChunkAt {
    int64_t vec, c, base;
};
__device__ __forceinline__ ChunkAt chunk_of(const BGroup &q, int64_t local) {
    ChunkAt r;
    r.vec = local / q.nchunks;
    r.c = local - r.vec * q.nchunks;
    r.base = r.c * kChunk;
    return r;
}

// pass 1, after a separate product: w -= beta' vp (n > 0); partial <v, w>
template <typename T, class Src>
__global__ void __launch_bounds__(256) ks_sub_prev(Src src) {
    __shared__ double sh[256];
    int64_t local;
    const BGroup &q = src.at(blockIdx.x, &local);
    const ChunkAt at = chunk_of(q, local);
    const int n = q.n;
    const double b = n > 0 ? q.cs.beta[at.vec * q.cs.maxs + n - 1] : 0.0;
    const int64_t off = at.vec * q.dim;
    const auto w = gp((T *)q.w) + off;
    const auto vp = gp((const T *)q.vp) + off;
    const auto v = gp((const T *)q.v) + off;
    double acc = 0.0;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        const int64_t i = at.base + k;
        if (i < q.dim) {
            double x = ldd(w + i);
            if (n > 0) {
                const T xt = (T)fma(-b, ldd(vp + i), x);
                w[i] = xt;
                x = (double)xt;
            }
            acc = fma(ldd(v + i), x, acc);
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) q.pa[at.vec * q.na + at.c] = s;
}

// pass 2: partial |x|^2 (and <v, x>, <vp, x>) with x = w - alpha_n v; with
// cond, only for chains whose dot-based finish asked for it (cs.renorm)
template <typename T, class Src>
__global__ void __launch_bounds__(256) ks_norm(Src src, int cond) {
    __shared__ double sh[256];
    int64_t local;
    const BGroup &q = src.at(blockIdx.x, &local);
    const ChunkAt at = chunk_of(q, local);
    if (cond && !q.cs.renorm[at.vec]) return;
    const double a = q.cs.alpha[at.vec * q.cs.maxs + q.n];
    const int64_t off = at.vec * q.dim;
    const auto w = gp((const T *)q.w) + off;
    const auto v = gp((const T *)q.v) + off;
    const auto vp = gp((const T *)q.vp) + off;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (q.reorth) {
        for (int k = threadIdx.x; k < kChunk; k += 256) {
            const int64_t i = at.base + k;
            if (i < q.dim) {
                const double vi = ldd(v + i);
                const double x = fma(-a, vi, ldd(w + i));
                s0 = fma(x, x, s0);
                s1 = fma(vi, x, s1);
                s2 = fma(ldd(vp + i), x, s2);
            }
        }
    } else {
        for (int k = threadIdx.x; k < kChunk; k += 256) {
            const int64_t i = at.base + k;
            if (i < q.dim) {
                const double x = fma(-a, ldd(v + i), ldd(w + i));
                s0 = fma(x, x, s0);
            }
        }
    }
    double *pn = q.pn + at.vec * 3 * q.nchunks + at.c;
    const double t0 = block_sum(s0, sh);
    if (threadIdx.x == 0) pn[0] = t0;
    if (q.reorth) {
        const double t1 = block_sum(s1, sh);
        const double t2 = block_sum(s2, sh);
        if (threadIdx.x == 0) {
            pn[q.nchunks] = t1;
            pn[2 * q.nchunks] = t2;
        }
    }
}

// sum over k = threadIdx.x, + 256, ... < n of p[k], added in that order; the
// loads go out eight at a time ahead of the additions
__device__ __forceinline__ double strided_sum(const double *__restrict__ p, int64_t n) {
    double acc = 0.0;
    int64_t k = threadIdx.x;
    for (; k + 7 * 256 < n; k += 8 * 256) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = p[k + u * 256];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += x[u];
    }
    for (; k < n; k += 256) acc += p[k];
    return acc;
}

// The dots give |x|^2 = <w,w> - 2 a <v,w> + a^2 <v,v> with an absolute
// error of a few eps <w,w>; below kDotRel <w,w> (beta < 0.03 |w|) that is no
// longer beta to about 1e-12, and the chain takes the direct norm pass
// (cs.renorm) instead, as near a breakdown or an exhausted Krylov space.
constexpr double kDotRel = 1e-3;

// beta_n from |x|^2 and the reorthogonalisation terms c1 = <v, x>,
// c2 = <vp, x> of x = w - alpha_n v, and the chain's bookkeeping
__device__ __forceinline__ void finish_beta(const ChainState &cs, int c, int n, int reorth,
                                            double s0, double s1, double s2) {
    if (reorth) cs.alpha[(int64_t)c * cs.maxs + n] += s1;
    cs.corr[c] = s1;
    cs.corr2[c] = s2;
    const double bb = s0 - s1 * s1 - s2 * s2;
    const double b = sqrt(bb > 0.0 ? bb : 0.0);
    cs.beta[(int64_t)c * cs.maxs + n] = b;
    if (!cs.done[c]) {
        const double am = cs.amax[c] > 0.0 ? cs.amax[c] : 1.0;
        if (!(b >= cs.btol * am)) cs.done[c] = 1;
        cs.len[c] = n + 1;
    }
    cs.inv[c] = cs.done[c] ? 0.0 : 1.0 / b;
}

// per-chain sums of the partials and the recurrence bookkeeping
// mode 0: alpha_n; mode 1: reorthogonalisation terms, beta_n, breakdown, from
// the norm pass; mode 2: the same from the dots of the two-pass product
// (pa: <v,w>, <w,w>, <v,v>, and with reorthogonalisation <vp,w>, <vp,v>);
// mode 3: modes 0 and 2 together, from the fused product's dots (same
// layout, q.na partials per chain), unless the dots cannot resolve beta
// (cs.renorm); mode 4: mode 1 for the chains so marked.
template <class Src>
__global__ void __launch_bounds__(256) ks_finish(Src src, int mode) {
    __shared__ double sh[256];
    int64_t local;
    const BGroup &q = src.at(blockIdx.x, &local);
    const int c = (int)local;
    const ChainState &cs = q.cs;
    const int n = q.n;
    if (mode == 0) {
        const double *p = q.pa + (int64_t)c * q.na;
        double acc = strided_sum(p, q.na);
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) {
            cs.alpha[(int64_t)c * cs.maxs + n] = s;
            cs.apre[c] = s;
            const double a = fabs(s);
            if (a > cs.amax[c]) cs.amax[c] = a;
        }
        return;
    }
    if (mode == 3) {
        const double *p = q.pa + (int64_t)c * q.na;
        const double vw = block_sum(strided_sum(p, q.na), sh);
        const double ww = block_sum(strided_sum(p + q.pstride, q.na), sh);
        const double vv = block_sum(strided_sum(p + 2 * q.pstride, q.na), sh);
        double pw = 0.0, pv = 0.0;
        if (q.reorth) {
            pw = block_sum(strided_sum(p + 3 * q.pstride, q.na), sh);
            pv = block_sum(strided_sum(p + 4 * q.pstride, q.na), sh);
        }
        if (threadIdx.x != 0) return;
        cs.alpha[(int64_t)c * cs.maxs + n] = vw;
        cs.apre[c] = vw;
        if (fabs(vw) > cs.amax[c]) cs.amax[c] = fabs(vw);
        const double a = vw;
        const double s0 = fma(a * a, vv, fma(-2.0 * a, a, ww));
        const double s1 = q.reorth ? fma(-a, vv, a) : 0.0;
        const double s2 = q.reorth ? fma(-a, pv, pw) : 0.0;
        cs.renorm[c] = !(s0 > kDotRel * ww);
        if (!cs.renorm[c]) finish_beta(cs, c, n, q.reorth, s0, s1, s2);
        return;
    }
    if (mode == 2) {
        const double *p = q.pa + (int64_t)c * q.na;
        const double ww = block_sum(strided_sum(p + q.pstride, q.na), sh);
        const double vv = block_sum(strided_sum(p + 2 * q.pstride, q.na), sh);
        double pw = 0.0, pv = 0.0;
        if (q.reorth) {
            pw = block_sum(strided_sum(p + 3 * q.pstride, q.na), sh);
            pv = block_sum(strided_sum(p + 4 * q.pstride, q.na), sh);
        }
        if (threadIdx.x != 0) return;
        const double a = cs.apre[c];   // <v, w>
        // x = w - a v: |x|^2, <v, x>, <vp, x> from the dots
        const double s0 = fma(a * a, vv, fma(-2.0 * a, a, ww));
        const double s1 = q.reorth ? fma(-a, vv, a) : 0.0;
        const double s2 = q.reorth ? fma(-a, pv, pw) : 0.0;
        finish_beta(cs, c, n, q.reorth, s0, s1, s2);
        return;
    }
    if (mode == 4 && !cs.renorm[c]) return;
    const double *p = q.pn + (int64_t)c * 3 * q.nchunks;
    const double s0 = block_sum(strided_sum(p, q.nchunks), sh);
    double s1 = 0.0, s2 = 0.0;
    if (q.reorth) {
        s1 = block_sum(strided_sum(p + q.nchunks, q.nchunks), sh);
        s2 = block_sum(strided_sum(p + 2 * q.nchunks, q.nchunks), sh);
    }
    if (threadIdx.x != 0) return;
    finish_beta(cs, c, n, q.reorth, s0, s1, s2);
}

// The two-pass product's partial arrays (three, five with
// reorthogonalisation, of q.na values per chain) are summed in two launches:
// ks_dots_stage sums contiguous ranges, one per workgroup of kDotBlocks, into
// q.pn ([chain][array][kDotBlocks]); ks_finish_dots sums those in order and
// records alpha_n and beta_n as ks_finish modes 0 and 2 do.  Each thread's
// share is summed in index order and each block's by a fixed tree.
constexpr int kDotBlocks = 64;

template <class Src>
__global__ void __launch_bounds__(256) ks_dots_stage(Src src) {
    constexpr int U = 8;
    __shared__ double sh[256];
    int64_t local;
    const BGroup &q = src.at(blockIdx.y, &local);
    const int c = (int)local;
    const int na = q.reorth ? 5 : 3;
    const int64_t len = (q.na + kDotBlocks - 1) / kDotBlocks;
    const int64_t k0 = (int64_t)blockIdx.x * len;
    const int64_t k1 = min((int64_t)q.na, k0 + len);
    const double *p = q.pa + (int64_t)c * q.na;
    double *o = q.pn + ((int64_t)c * 5) * kDotBlocks + blockIdx.x;
    for (int a = 0; a < na; ++a) {
        const double *pa = p + a * q.pstride;
        double acc = 0.0;
        int64_t k = k0 + threadIdx.x;
        for (; k + (U - 1) * 256 < k1; k += U * 256) {
            double x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = pa[k + u * 256];
#pragma unroll
            for (int u = 0; u < U; ++u) acc += x[u];
        }
        for (; k < k1; k += 256) acc += pa[k];
        const double t = block_sum(acc, sh);
        if (threadIdx.x == 0) o[a * kDotBlocks] = t;
    }
}

template <class Src>
__global__ void __launch_bounds__(kDotBlocks) ks_finish_dots(Src src) {
    __shared__ double sh[5][kDotBlocks];
    int64_t local;
    const BGroup &q = src.at(blockIdx.x, &local);
    const int c = (int)local;
    const ChainState &cs = q.cs;
    const int n = q.n;
    const int na = q.reorth ? 5 : 3;
    const int t = threadIdx.x;
    const double *p = q.pn + ((int64_t)c * 5) * kDotBlocks;
#pragma unroll
    for (int a = 0; a < 5; ++a) sh[a][t] = a < na ? p[a * kDotBlocks + t] : 0.0;
    __syncthreads();
    for (int s = kDotBlocks / 2; s > 0; s >>= 1) {
        if (t < s)
#pragma unroll
            for (int a = 0; a < 5; ++a) sh[a][t] += sh[a][t + s];
        __syncthreads();
    }
    if (t != 0) return;
    const double vw = sh[0][0], ww = sh[1][0], vv = sh[2][0];
    const double pw = q.reorth ? sh[3][0] : 0.0, pv = q.reorth ? sh[4][0] : 0.0;
    // mode 0: alpha_n = <v, w>
    cs.alpha[(int64_t)c * cs.maxs + n] = vw;
    cs.apre[c] = vw;
    if (fabs(vw) > cs.amax[c]) cs.amax[c] = fabs(vw);
    // mode 2: x = w - a v: |x|^2, <v, x>, <vp, x> from the dots (or the
    // direct norm pass when they cannot resolve beta)
    const double a = vw;
    const double s0 = fma(a * a, vv, fma(-2.0 * a, a, ww));
    const double s1 = q.reorth ? fma(-a, vv, a) : 0.0;
    const double s2 = q.reorth ? fma(-a, pv, pw) : 0.0;
    cs.renorm[c] = !(s0 > kDotRel * ww);
    if (!cs.renorm[c]) finish_beta(cs, c, n, q.reorth, s0, s1, s2);
}

// pass 3: w = (w - alpha v - c1 v - c2 vp) / beta_n; psi += svec[n] v (replay)
template <typename T, class Src>
__global__ void __launch_bounds__(256) ks_update(Src src) {
    int64_t local;
    const BGroup &q = src.at(blockIdx.x, &local);
    const ChunkAt at = chunk_of(q, local);
    const ChainState &cs = q.cs;
    const double a = cs.apre[at.vec], c1 = cs.corr[at.vec], c2 = cs.corr2[at.vec];
    const double s = cs.inv[at.vec];
    const int64_t off = at.vec * q.dim;
    const auto w = gp((T *)q.w) + off;
    const auto v = gp((const T *)q.v) + off;
    const auto vp = gp((const T *)q.vp) + off;
    const auto psi = gp(q.psi);
    const double sv = psi ? q.svec[q.n] : 0.0;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        const int64_t i = at.base + k;
        if (i < q.dim) {
            const double vi = ldd(v + i);
            double x = fma(-a, vi, ldd(w + i));
            if (q.reorth) {
                x = fma(-c1, vi, x);
                x = fma(-c2, ldd(vp + i), x);
            }
            w[i] = (T)(x * s);
            if (psi) psi[i] = fma(sv, vi, psi[i]);
        }
    }
}

// psi += svec[n] v_n alone (the last replay step)
template <typename T, class Src>
__global__ void __launch_bounds__(256) ks_accum(Src src) {
    int64_t local;
    const BGroup &q = src.at(blockIdx.x, &local);
    const ChunkAt at = chunk_of(q, local);
    const auto v = gp((const T *)q.v);
    const auto psi = gp(q.psi);
    const double sv = q.svec[q.n];
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        const int64_t i = at.base + k;
        if (i < q.dim) psi[i] = fma(sv, ldd(v + i), psi[i]);
    }
}

}  // namespace qcm
