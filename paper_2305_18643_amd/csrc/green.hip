// Continued-fraction Green function (paper: section "Exact diagonalizations",
// subsection "The Lanczos algorithm for the Green function", eqs. (green),
// (GreenCF1), (jacobi) and the off-diagonal trick for a real H).
//
// For every pair (i <= j) of the requested orbitals two chains are run:
// electron, from (c_i + c_j)+ |Omega> in sector (N_up + 1, N_dn), and hole,
// from (c_i + c_j) |Omega> in (N_up - 1, N_dn).  All chains of one part live
// in the same sector, so they run together through the multi-chain engine.
// Start vectors are built by a gather over the target sector: only the up
// string changes, the sign is (-1)^(up electrons on orbitals below the
// operator's orbital), and the down label is untouched.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "lanczos_device.h"
#include "lanczos_step.h"

namespace qcm {

struct PairOps {
    int32_t mu[2];
};

// phi_c = sum over the chain's operators of sign * psi[source], gathered per
// target element; partial sums of |phi|^2 (FP64, before rounding).
template <typename T>
__global__ void __launch_bounds__(256) k_apply_ops(
    const double *__restrict__ psi, int64_t d_src_up, const int32_t *__restrict__ rlo_src,
    const int32_t *__restrict__ rhi_src, int l_lo, int l_hi,
    const uint32_t *__restrict__ states_tgt, int64_t d_tgt_up, int64_t dim_tgt, int kind,
    const int32_t *__restrict__ ops, T *__restrict__ out, int nchunks,
    double *__restrict__ partial) {
    __shared__ double sh[256];
    const int c = blockIdx.y;
    const int o0 = ops[2 * c], o1 = ops[2 * c + 1];
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    double acc = 0.0;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        int64_t i = base + k;
        if (i >= dim_tgt) break;
        int64_t iu = i % d_tgt_up, idn = i / d_tgt_up;
        uint32_t bt = states_tgt[iu];
        double val = 0.0;
        for (int q = 0; q < 2; ++q) {
            int m = q == 0 ? o0 : o1;
            if (m < 0) continue;
            uint32_t bit = 1u << m;
            bool has = bt & bit;
            // kind 0 (creation): target has m, source lacks it; kind 1: reverse
            if ((kind == 0) != has) continue;
            uint32_t bs = bt ^ bit;
            int below = __popc(bt & (bit - 1u));
            int64_t j = (int64_t)spin_rank(rlo_src, rhi_src, l_lo, l_hi, bs) + d_src_up * idn;
            double x = psi[j];
            val += (below & 1) ? -x : x;
        }
        out[(int64_t)c * dim_tgt + i] = (T)val;
        acc = fma(val, val, acc);
    }
    // fixed tree
    const int t = threadIdx.x;
    sh[t] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    if (t == 0) partial[(int64_t)c * nchunks + blockIdx.x] = sh[0];
}

// coef[(c*2 + part) * stride]: b0sq, a[maxs], b2[maxs]; len[c*2 + part]
__global__ void k_store_coef(ChainState cs, int nvec, int part, double *__restrict__ coef,
                             int32_t *__restrict__ len, int stride) {
    int c = blockIdx.x;
    if (c >= nvec) return;
    double *o = coef + (int64_t)(c * 2 + part) * stride;
    int L = cs.len[c];
    for (int n = threadIdx.x; n < cs.maxs; n += blockDim.x) {
        o[1 + n] = n < L ? cs.alpha[(int64_t)c * cs.maxs + n] : 0.0;
        double b = cs.beta[(int64_t)c * cs.maxs + n];
        o[1 + cs.maxs + n] = n + 1 < L ? b * b : 0.0;
    }
    if (threadIdx.x == 0) {
        o[0] = cs.b0sq[c];
        len[c * 2 + part] = L;
    }
}

__global__ void k_zero_coef(int npairs, int part, double *__restrict__ coef,
                            int32_t *__restrict__ len, int stride) {
    int c = blockIdx.x;
    double *o = coef + (int64_t)(c * 2 + part) * stride;
    for (int n = threadIdx.x; n < stride; n += blockDim.x) o[n] = 0.0;
    if (threadIdx.x == 0) len[c * 2 + part] = 0;
}

// F[z][p] = G_e + G_h of pair p
__global__ void k_cf_pairs(const double *__restrict__ coef, const int32_t *__restrict__ len,
                           int npairs, int maxs, int nz, const double *__restrict__ zs, double e0,
                           double *__restrict__ F) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nz * npairs) return;
    int iz = (int)(e / npairs), p = (int)(e % npairs);
    cplx z{zs[2 * iz], zs[2 * iz + 1]};
    const int stride = 1 + 2 * maxs;
    cplx g0 = cf_value(coef + (int64_t)(p * 2 + 0) * stride, len[p * 2 + 0], maxs, z, e0, 0);
    cplx g1 = cf_value(coef + (int64_t)(p * 2 + 1) * stride, len[p * 2 + 1], maxs, z, e0, 1);
    F[2 * e] = g0.re + g1.re;
    F[2 * e + 1] = g0.im + g1.im;
}

// G[z][i][j]: diagonal pairs directly, off-diagonal (F_ij - F_ii - F_jj)/2
__global__ void k_cf_combine(const double *__restrict__ F, const int32_t *__restrict__ pidx,
                             int n, int npairs, int nz, double *__restrict__ G) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nz * n * n) return;
    int iz = (int)(e / (n * n));
    int ij = (int)(e % (n * n));
    int i = ij / n, j = ij % n;
    int a = i < j ? i : j, b = i < j ? j : i;
    const double *f = F + (int64_t)iz * npairs * 2;
    int pab = pidx[a * n + b];
    double re = f[2 * pab], im = f[2 * pab + 1];
    if (a != b) {
        int paa = pidx[a * n + a], pbb = pidx[b * n + b];
        re = 0.5 * (re - f[2 * paa] - f[2 * pbb]);
        im = 0.5 * (im - f[2 * paa + 1] - f[2 * pbb + 1]);
    }
    G[2 * e] = re;
    G[2 * e + 1] = im;
}

// Start vectors of the chains of one part into the current vectors of e,
// with their norm partials in e.partial (kind 0: creation, 1: annihilation).
// nvec start vectors (consecutive, length dim each) into out, with their
// norm partials [nvec][nchunks] in partial.
int apply_ops_raw(int prec, const double *psi, int64_t d_src_up, const SpinTables &src_up,
                  const SpinTables &tgt_up, int64_t dim, int kind, const int32_t *ops, int nvec,
                  void *out, int nchunks, double *partial, hipStream_t s) {
    const dim3 g((unsigned)nchunks, (unsigned)nvec);
    if (prec == QCM_FP64)
        k_apply_ops<double><<<g, 256, 0, s>>>(psi, d_src_up, src_up.rank_lo, src_up.rank_hi,
                                              src_up.l_lo, src_up.l_hi, tgt_up.states, tgt_up.d,
                                              dim, kind, ops, (double *)out, nchunks, partial);
    else
        k_apply_ops<float><<<g, 256, 0, s>>>(psi, d_src_up, src_up.rank_lo, src_up.rank_hi,
                                             src_up.l_lo, src_up.l_hi, tgt_up.states, tgt_up.d,
                                             dim, kind, ops, (float *)out, nchunks, partial);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

int apply_ops_launch(Engine &e, const double *psi, int64_t d_src_up, const SpinTables &src_up,
                     const SpinTables &tgt_up, int kind, const int32_t *ops, hipStream_t s) {
    return apply_ops_raw(e.prec, psi, d_src_up, src_up, tgt_up, e.dim, kind, ops, e.nvec,
                         e.vbuf[e.iv], e.nchunks, e.partial, s);
}

// Coefficients of part `part` of every pair into coef/len; e == NULL (the
// part's sector does not exist) stores empty chains.
int green_store(const Engine *e, int npairs, int part, double *coef, int32_t *len, int stride,
                hipStream_t s) {
    if (e)
        k_store_coef<<<npairs, 256, 0, s>>>(e->cs, npairs, part, coef, len, stride);
    else
        k_zero_coef<<<npairs, 256, 0, s>>>(npairs, part, coef, len, stride);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

// G[z][i][j] from the stored chains (F: scratch [nz][npairs] complex).
int green_eval(const double *coef, const int32_t *len, int n, int maxs, int nz, const double *zd,
               double e0, const int32_t *pidx, double *F, double *G, hipStream_t s) {
    const int npairs = n * (n + 1) / 2;
    if (nz <= 0) return QCM_OK;
    int64_t tot = (int64_t)nz * npairs;
    k_cf_pairs<<<ceil_div(tot, 256), 256, 0, s>>>(coef, len, npairs, maxs, nz, zd, e0, F);
    int64_t tot2 = (int64_t)nz * n * n;
    k_cf_combine<<<ceil_div(tot2, 256), 256, 0, s>>>(F, pidx, n, npairs, nz, G);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

// ---------------------------------------------------------------- full reorthogonalisation
// A test device (the paper's recurrence tolerates the loss of orthogonality):
// every chain keeps all its vectors, hist[k][c][dim] (k = floor, c = chain),
// and after w = H v_n - beta' v_{n-1} - alpha_n v_n the components of w along
// v_0..v_n are removed twice by classical Gram-Schmidt (all coefficients
// <v_k, w> from fixed-order two-level sums, then one subtraction per element
// summed in floor order, rounded once); they are not entered in T.  Then
// beta_n = |w| and v_{n+1} = w / beta_n.

constexpr int kFrPer = kChunk / 256;   // elements of a chunk per thread
constexpr size_t kFrHistBytes = (size_t)16 << 30;   // history of one group of chains

// w = w - alpha_n v, rounded once (grid: chunks x chains)
template <typename T>
__global__ void __launch_bounds__(256) k_fr_alpha(T *__restrict__ w, const T *__restrict__ v,
                                                  int64_t dim, ChainState cs, int n) {
    const int64_t c = blockIdx.y, base = (int64_t)blockIdx.x * kChunk;
    const double a = cs.alpha[c * cs.maxs + n];
    T *wc = w + c * dim;
    const T *vc = v + c * dim;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        const int64_t i = base + k;
        if (i < dim) wc[i] = (T)fma(-a, (double)vc[i], (double)wc[i]);
    }
}

// partial <v_k, w> of one chunk for k = 0..nk-1: part[(c * kmax + k) * nchunks + chunk]
template <typename T>
__global__ void __launch_bounds__(256) k_fr_dots(const T *__restrict__ hist, const T *__restrict__ w,
                                                 int64_t dim, int nvec, int nk, int kmax,
                                                 int nchunks, double *__restrict__ part) {
    __shared__ double sh[256];
    const int64_t c = blockIdx.y, ch = blockIdx.x, base = ch * kChunk;
    double x[kFrPer];
#pragma unroll
    for (int j = 0; j < kFrPer; ++j) {
        const int64_t i = base + threadIdx.x + 256 * j;
        x[j] = i < dim ? (double)w[c * dim + i] : 0.0;
    }
    for (int k = 0; k < nk; ++k) {
        const T *h = hist + ((int64_t)k * nvec + c) * dim;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < kFrPer; ++j) {
            const int64_t i = base + threadIdx.x + 256 * j;
            if (i < dim) acc = fma((double)h[i], x[j], acc);
        }
        const double t = block_sum(acc, sh);
        if (threadIdx.x == 0) part[((int64_t)c * kmax + k) * nchunks + ch] = t;
    }
}

// coef[c * kmax + k] = sum over the chunks of the partials (fixed order)
__global__ void __launch_bounds__(256) k_fr_coef(const double *__restrict__ part, int kmax,
                                                 int nchunks, double *__restrict__ coef) {
    __shared__ double sh[256];
    const int64_t k = blockIdx.x, c = blockIdx.y;
    const double s = block_sum(strided_sum(part + (c * kmax + k) * nchunks, nchunks), sh);
    if (threadIdx.x == 0) coef[c * kmax + k] = s;
}

// w = w - sum_k coef_k v_k (floors in order, FP64, rounded once)
template <typename T>
__global__ void __launch_bounds__(256) k_fr_sub(const T *__restrict__ hist, T *__restrict__ w,
                                                int64_t dim, int nvec, int nk, int kmax,
                                                const double *__restrict__ coef) {
    const int64_t c = blockIdx.y, base = (int64_t)blockIdx.x * kChunk;
    double x[kFrPer];
#pragma unroll
    for (int j = 0; j < kFrPer; ++j) {
        const int64_t i = base + threadIdx.x + 256 * j;
        x[j] = i < dim ? (double)w[c * dim + i] : 0.0;
    }
    for (int k = 0; k < nk; ++k) {
        const double ck = coef[c * kmax + k];
        const T *h = hist + ((int64_t)k * nvec + c) * dim;
#pragma unroll
        for (int j = 0; j < kFrPer; ++j) {
            const int64_t i = base + threadIdx.x + 256 * j;
            if (i < dim) x[j] = fma(-ck, (double)h[i], x[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < kFrPer; ++j) {
        const int64_t i = base + threadIdx.x + 256 * j;
        if (i < dim) w[c * dim + i] = (T)x[j];
    }
}

// partial |w|^2 of one chunk into pn[c * 3 * nchunks + chunk]
template <typename T>
__global__ void __launch_bounds__(256) k_fr_norm(const T *__restrict__ w, int64_t dim, int nchunks,
                                                 double *__restrict__ pn) {
    __shared__ double sh[256];
    const int64_t c = blockIdx.y, ch = blockIdx.x, base = ch * kChunk;
    double acc = 0.0;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        const int64_t i = base + k;
        if (i < dim) {
            const double x = (double)w[c * dim + i];
            acc = fma(x, x, acc);
        }
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) pn[c * 3 * nchunks + ch] = t;
}

// v_{n+1} = w / beta_n (zero once the chain has stopped)
template <typename T>
__global__ void __launch_bounds__(256) k_fr_store(const T *__restrict__ w, T *__restrict__ out,
                                                  int64_t dim, ChainState cs) {
    const int64_t c = blockIdx.y, base = (int64_t)blockIdx.x * kChunk;
    const double s = cs.inv[c];
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        const int64_t i = base + k;
        if (i < dim) out[c * dim + i] = (T)((double)w[c * dim + i] * s);
    }
}

// Chains of a group that fit the history cap at once.
int fr_group_size(int npairs, int maxs, int64_t dim, int prec) {
    const size_t per = (size_t)(maxs + 1) * (size_t)dim * (prec == QCM_FP64 ? 8 : 4);
    int64_t g = per > 0 ? (int64_t)(kFrHistBytes / per) : npairs;
    if (g < 1) g = 1;
    if (g > npairs) g = npairs;
    return (int)g;
}

struct FrBufs {
    void *hist;
    double *part, *coef;
};

int fr_carve(Carver &cv, int prec, int ng, int maxs, int64_t dim, FrBufs *b) {
    const size_t s = prec == QCM_FP64 ? 8 : 4;
    const int64_t nch = (int64_t)ceil_div(dim, kChunk);
    b->hist = cv.take<char>((size_t)(maxs + 1) * ng * dim * s);
    b->part = cv.take<double>((size_t)ng * (maxs + 1) * (nch > 0 ? nch : 1));
    b->coef = cv.take<double>((size_t)ng * (maxs + 1));
    return QCM_OK;
}

// One step n of the group: w = H v_n - beta' v_{n-1}, alpha_n, the two
// Gram-Schmidt passes, beta_n, v_{n+1} into hist[n + 1].
template <typename T>
int fr_step_t(Engine &e, const FrBufs &b, int n, hipStream_t s) {
    const int64_t dim = e.dim;
    const int nvec = e.nvec, kmax = e.maxs + 1, nch = e.nchunks;
    T *hist = (T *)b.hist;
    T *w = (T *)e.vbuf[2];
    T *v = hist + (int64_t)n * nvec * dim;
    T *vp = n > 0 ? hist + (int64_t)(n - 1) * nvec * dim : v;
    BGroup g = engine_group(e, n);
    g.v = v;
    g.vp = vp;
    g.w = w;
    g.na = e.nchunks;
    g.reorth = 0;
    const OneSrc src{g};
    const dim3 gc((unsigned)nch, (unsigned)nvec);
    QCM_TRY(hv_launch(e.op, e.prec, v, w, nvec, s));
    ks_sub_prev<T, OneSrc><<<(unsigned)(nvec * nch), 256, 0, s>>>(src);
    ks_finish<OneSrc><<<nvec, 256, 0, s>>>(src, 0);
    k_fr_alpha<T><<<gc, 256, 0, s>>>(w, v, dim, e.cs, n);
    for (int pass = 0; pass < 2; ++pass) {
        k_fr_dots<T><<<gc, 256, 0, s>>>(hist, w, dim, nvec, n + 1, kmax, nch, b.part);
        k_fr_coef<<<dim3((unsigned)(n + 1), (unsigned)nvec), 256, 0, s>>>(b.part, kmax, nch, b.coef);
        k_fr_sub<T><<<gc, 256, 0, s>>>(hist, w, dim, nvec, n + 1, kmax, b.coef);
    }
    k_fr_norm<T><<<gc, 256, 0, s>>>(w, dim, nch, e.pn);
    ks_finish<OneSrc><<<nvec, 256, 0, s>>>(src, 1);
    if (n + 1 < e.maxs)
        k_fr_store<T><<<gc, 256, 0, s>>>(w, hist + (int64_t)(n + 1) * nvec * dim, dim, e.cs);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

int fr_step(Engine &e, const FrBufs &b, int n, hipStream_t s) {
    if (e.prec == QCM_FP64) return fr_step_t<double>(e, b, n, s);
    return fr_step_t<float>(e, b, n, s);
}

}  // namespace qcm

using namespace qcm;

// Workspace layout of qcm_green_cf: a common block, then one part at a time
// (electron, hole) from the same offset.  Run without a base to size it.
struct GreenCommon {
    ModelDev md;
    HopTables hd;
    double *coef, *z_d, *F;
    int32_t *lenv, *ops_d, *pidx_d;
};

static int green_common(const qcm_model *m, const qcm_basis *gs, int n, int stride, int n_z,
                        Carver &cv, hipStream_t s, GreenCommon *c) {
    const int npairs = n * (n + 1) / 2;
    QCM_TRY(upload_model(m, cv, &c->md, s));
    SpinTables dn = spin_from_basis(gs, 1);
    QCM_TRY(build_hop_tables(c->md, dn, cv, &c->hd, s, count_bonds(m)));
    c->coef = cv.take<double>((size_t)npairs * 2 * stride);
    c->lenv = cv.take<int32_t>((size_t)npairs * 2);
    c->ops_d = cv.take<int32_t>((size_t)npairs * 2);
    c->pidx_d = cv.take<int32_t>((size_t)n * n);
    c->z_d = cv.take<double>(2 * (size_t)(n_z > 0 ? n_z : 1));
    c->F = cv.take<double>(2 * (size_t)(n_z > 0 ? n_z : 1) * npairs);
    return QCM_OK;
}

static int green_part(const qcm_model *m, const qcm_basis *gs, const qcm_green_opts *o, int nup2,
                      const GreenCommon &c, Carver &cv, hipStream_t s, SpinTables *up2,
                      HvOp *op, Engine *e, FrBufs *fr) {
    int npairs = o->n_orb * (o->n_orb + 1) / 2;
    QCM_TRY(build_spin_tables(m->L, nup2, cv, up2, s));
    op->md = c.md;
    op->up = *up2;
    op->dn = spin_from_basis(gs, 1);
    op->hd = c.hd;
    op->dim = up2->d * op->dn.d;
    QCM_TRY(build_hop_tables(c.md, *up2, cv, &op->hu, s, count_bonds(m)));
    op->split = 0;
    if (split_applies(m, nup2, up2->d, op->dn.d)) QCM_TRY(split_prepare(m, *op, cv, s));
    if (o->reorth == 2) {
        // chains in groups whose history fits the cap
        npairs = fr_group_size(npairs, o->max_steps, op->dim, o->prec);
        QCM_TRY(fr_carve(cv, o->prec, npairs, o->max_steps, op->dim, fr));
    }
    QCM_TRY(engine_init(*e, *op, o->prec, npairs, o->max_steps, o->btol, o->reorth, cv));
    return QCM_OK;
}

static int green_bytes(const qcm_model *m, const qcm_basis *gs, const qcm_green_opts *o, int n_z,
                       size_t *need) {
    Carver dry(nullptr);
    GreenCommon c;
    QCM_TRY(green_common(m, gs, o->n_orb, 1 + 2 * o->max_steps, n_z, dry, nullptr, &c));
    size_t end = dry.off;
    for (int part = 0; part < 2; ++part) {
        const int nup2 = part == 0 ? gs->n_up + 1 : gs->n_up - 1;
        if (nup2 < 0 || nup2 > m->L) continue;
        Carver p(nullptr);
        p.off = dry.off;
        SpinTables up2;
        HvOp op;
        Engine e;
        FrBufs fr;
        QCM_TRY(green_part(m, gs, o, nup2, c, p, nullptr, &up2, &op, &e, &fr));
        if (p.off > end) end = p.off;
    }
    *need = end + 256;
    return QCM_OK;
}

extern "C" int qcm_green_cf(const qcm_model *m, const qcm_basis *gs, const double *d_gs,
                            double e0, const qcm_green_opts *o, double *h_coef, int32_t *h_len,
                            int32_t n_z, const double *h_z, double *d_G, void *d_ws,
                            size_t ws_bytes, size_t *ws_needed, void *stream) {
    if (!ws_needed || !o) return fail(QCM_EARG, "qcm_green_cf: NULL ws_needed or opts");
    QCM_TRY(validate_model(m));
    QCM_TRY(check_basis(gs, m->L));
    const int L = m->L;
    if (o->n_orb < 1 || o->n_orb > L || !o->orbs)
        return fail(QCM_EARG, "qcm_green_cf: bad orbital list");
    for (int i = 0; i < o->n_orb; ++i) {
        if (o->orbs[i] < 0 || o->orbs[i] >= L)
            return fail(QCM_EARG, "qcm_green_cf: orbital %d out of range", o->orbs[i]);
        for (int j = 0; j < i; ++j)
            if (o->orbs[j] == o->orbs[i]) return fail(QCM_EARG, "qcm_green_cf: repeated orbital");
    }
    if (o->max_steps < 1) return fail(QCM_EARG, "qcm_green_cf: max_steps < 1");
    if (o->prec != QCM_FP64 && o->prec != QCM_FP32V)
        return fail(QCM_EARG, "qcm_green_cf: bad prec");
    if (o->reorth < 0 || o->reorth > 2) return fail(QCM_EARG, "qcm_green_cf: reorth must be 0, 1 or 2");
    if (n_z < 0 || (n_z > 0 && (!h_z || (!d_G && d_ws))))
        return fail(QCM_EARG, "qcm_green_cf: bad frequency arguments");
    size_t need = 0;
    QCM_TRY(green_bytes(m, gs, o, n_z, &need));
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (!d_gs) return fail(QCM_EARG, "qcm_green_cf: d_gs is NULL");
    if (ws_bytes < need)
        return fail(QCM_EWORKSPACE, "qcm_green_cf: workspace %zu < %zu", ws_bytes, need);

    hipStream_t s = as_stream(stream);
    const int n = o->n_orb;
    const int npairs = n * (n + 1) / 2;
    const int maxs = o->max_steps;
    const int stride = 1 + 2 * maxs;

    // pair list and index
    std::vector<int32_t> ops(2 * npairs), pidx(n * n, 0);
    {
        int p = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i; j < n; ++j) {
                ops[2 * p] = o->orbs[i];
                ops[2 * p + 1] = i == j ? -1 : o->orbs[j];
                pidx[i * n + j] = p;
                pidx[j * n + i] = p;
                ++p;
            }
    }
    Carver cv(d_ws);
    GreenCommon c;
    QCM_TRY(green_common(m, gs, n, stride, n_z, cv, s, &c));
    SpinTables upg = spin_from_basis(gs, 0);
    double *coef = c.coef, *z_d = c.z_d, *F = c.F;
    int32_t *lenv = c.lenv, *ops_d = c.ops_d, *pidx_d = c.pidx_d;
    QCM_HIP(hipMemcpyAsync(ops_d, ops.data(), sizeof(int32_t) * ops.size(), hipMemcpyHostToDevice, s));
    QCM_HIP(hipMemcpyAsync(pidx_d, pidx.data(), sizeof(int32_t) * pidx.size(),
                           hipMemcpyHostToDevice, s));
    if (n_z > 0)
        QCM_HIP(hipMemcpyAsync(z_d, h_z, sizeof(double) * 2 * n_z, hipMemcpyHostToDevice, s));
    const size_t part_base = cv.off;

    for (int part = 0; part < 2; ++part) {
        const int nup2 = part == 0 ? gs->n_up + 1 : gs->n_up - 1;
        if (nup2 < 0 || nup2 > L) {
            QCM_TRY(green_store(nullptr, npairs, part, coef, lenv, stride, s));
            continue;
        }
        cv.off = part_base;
        SpinTables up2;
        HvOp op;
        Engine e;
        FrBufs fr{};
        QCM_TRY(green_part(m, gs, o, nup2, c, cv, s, &up2, &op, &e, &fr));
        if (o->reorth == 2) {
            // groups of e.nvec chains, each with its full history
            for (int g0 = 0; g0 < npairs; g0 += e.nvec) {
                const int ng = std::min(e.nvec, npairs - g0);
                Engine eg = e;
                eg.nvec = ng;
                eg.cs.maxs = maxs;
                QCM_TRY(engine_reset(eg, s));
                QCM_TRY(apply_ops_raw(eg.prec, d_gs, gs->d_up, upg, up2, eg.dim, part,
                                      ops_d + 2 * g0, ng, fr.hist, eg.nchunks, eg.partial, s));
                eg.vbuf[eg.iv] = fr.hist;
                QCM_TRY(engine_normalize_from_partials(eg, s));
                std::vector<int32_t> done(ng);
                for (int step = 0; step < maxs; ++step) {
                    QCM_TRY(fr_step(eg, fr, step, s));
                    if ((step + 1) % 32 == 0 && step + 1 < maxs) {
                        QCM_HIP(hipMemcpyAsync(done.data(), eg.cs.done, sizeof(int32_t) * ng,
                                               hipMemcpyDeviceToHost, s));
                        QCM_HIP(hipStreamSynchronize(s));
                        bool all = true;
                        for (int k = 0; k < ng; ++k) all = all && done[k];
                        if (all) break;
                    }
                }
                QCM_TRY(green_store(&eg, ng, part, coef + (size_t)g0 * 2 * stride, lenv + 2 * g0,
                                    stride, s));
            }
            continue;
        }
        QCM_TRY(engine_reset(e, s));
        QCM_TRY(apply_ops_launch(e, d_gs, gs->d_up, upg, up2, part, ops_d, s));
        QCM_TRY(engine_normalize_from_partials(e, s));
        e.lazy = 1;   // only the coefficients are kept
        std::vector<int32_t> done(npairs);
        for (int step = 0; step < maxs; ++step) {
            QCM_TRY(engine_step(e, step, s));
            if ((step + 1) % 32 == 0 && step + 1 < maxs) {
                QCM_HIP(hipMemcpyAsync(done.data(), e.cs.done, sizeof(int32_t) * npairs,
                                       hipMemcpyDeviceToHost, s));
                QCM_HIP(hipStreamSynchronize(s));
                bool all = true;
                for (int c = 0; c < npairs; ++c) all = all && done[c];
                if (all) break;
            }
        }
        QCM_TRY(green_store(&e, npairs, part, coef, lenv, stride, s));
    }
    QCM_TRY(green_eval(coef, lenv, n, maxs, n_z, z_d, e0, pidx_d, F, d_G, s));
    if (h_coef)
        QCM_HIP(hipMemcpyAsync(h_coef, coef, sizeof(double) * npairs * 2 * stride,
                               hipMemcpyDeviceToHost, s));
    if (h_len)
        QCM_HIP(hipMemcpyAsync(h_len, lenv, sizeof(int32_t) * npairs * 2, hipMemcpyDeviceToHost, s));
    QCM_HIP(hipStreamSynchronize(s));
    return QCM_OK;
}
