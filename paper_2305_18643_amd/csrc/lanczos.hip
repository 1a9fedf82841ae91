// Lanczos recurrence on the device (paper: section "Exact diagonalizations",
// subsection "The Lanczos algorithm for the ground state", eqs. (Krylov),
// (LanczosRecursion), (tridiag)), in normalised form:
//   w = H v_n - beta_{n-1} v_{n-1};  alpha_n = <v_n, w>;  w -= alpha_n v_n;
//   beta_n = |w|;  v_{n+1} = w / beta_n          (beta_n^2 = paper's b_{n+1}^2)
//
// The engine runs nvec independent chains in one sector at once (vectors laid
// out consecutively), which is how the Green-function chains are batched.  A
// step is the three passes of lanczos_step.h.  Every dot product is a
// deterministic two-level sum (fixed blocks or chunks, then a fixed-order sum
// per chain), so results depend only on the inputs and the sector shape,
// never on launch timing or on other work sharing the GPU.
#include <math.h>

#include <string.h>

#include <algorithm>

#include "lanczos_step.h"

namespace qcm {

// ---------------------------------------------------------------- reductions

// partial[c][chunk] = sum over the chunk of x*y (vector c)
template <typename TX, typename TY>
__global__ void __launch_bounds__(256) k_dot_partial(const TX *__restrict__ x,
                                                     const TY *__restrict__ y, int64_t n,
                                                     int nchunks, double *__restrict__ partial) {
    __shared__ double sh[256];
    const int c = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    const TX *xc = x + (int64_t)c * n;
    const TY *yc = y + (int64_t)c * n;
    double acc = 0.0;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        int64_t i = base + k;
        if (i < n) acc = fma(ldd(xc + i), ldd(yc + i), acc);
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)c * nchunks + blockIdx.x] = s;
}

// Sum of the chunk partials of each chain.
// mode 2: out[c] = s (plain).
// mode 5: b0sq[c] = s, inv[c] = s > 0 ? 1/sqrt(s) : 0 (start-vector norm)
__global__ void __launch_bounds__(256) k_finish(const double *__restrict__ partial, int nchunks,
                                                int mode, ChainState cs, int n,
                                                double *__restrict__ out) {
    __shared__ double sh[256];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int k = threadIdx.x; k < nchunks; k += 256) acc += partial[(int64_t)c * nchunks + k];
    double s = block_sum(acc, sh);
    if (threadIdx.x != 0) return;
    (void)n;
    if (mode == 2) {
        out[c] = s;
    } else {
        cs.b0sq[c] = s;
        cs.inv[c] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
        if (!(s > 0.0)) {
            cs.done[c] = 1;
            cs.len[c] = 0;
        }
    }
}

// ---------------------------------------------------------------- vector updates

// x *= inv[c]
template <typename T>
__global__ void __launch_bounds__(256) k_scale(T *__restrict__ x, int64_t n_el, ChainState cs) {
    const int c = blockIdx.y;
    const double s = cs.inv[c];
    const int64_t off = (int64_t)c * n_el;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        int64_t i = base + k;
        if (i < n_el) st(x + off + i, ldd(x + off + i) * s);
    }
}

// psi += coef[n] * v  (psi FP64, one chain)
template <typename T>
__global__ void __launch_bounds__(256) k_accum(double *__restrict__ psi, const T *__restrict__ v,
                                               int64_t n_el, const double *__restrict__ coef,
                                               int n) {
    const double s = coef[n];
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        int64_t i = base + k;
        if (i < n_el) psi[i] = fma(s, ldd(v + i), psi[i]);
    }
}

// SplitMix64 start vector, entry i = 2 (u_i >> 11) 2^-53 - 1 with
// u_i = mix(seed + (i+1) * golden gamma) (Steele, Lea & Flood 2014).
template <typename T>
__global__ void __launch_bounds__(256) k_splitmix(T *__restrict__ x, int64_t n, uint64_t seed) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    double u = (double)(z >> 11) * 0x1.0p-53;
    x[i] = (T)(2.0 * u - 1.0);
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_convert(TO *__restrict__ o, const TI *__restrict__ in,
                                                 int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = (TO)in[i];
}

// partial sum of (w - theta psi)^2, FP64
__global__ void __launch_bounds__(256) k_resid_partial(const double *__restrict__ w,
                                                       const double *__restrict__ psi, double th,
                                                       int64_t n, int nchunks,
                                                       double *__restrict__ partial) {
    __shared__ double sh[256];
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    double acc = 0.0;
    for (int k = threadIdx.x; k < kChunk; k += 256) {
        int64_t i = base + k;
        if (i < n) {
            double r = fma(-th, psi[i], w[i]);
            acc = fma(r, r, acc);
        }
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// ---------------------------------------------------------------- tridiagonal

// Ground-state test on T_M: theta_0, theta_1, the eigenvector s of theta_0
// (written to svec), and the residual estimate beta[M-1] |s[M-1]|.
__global__ void __launch_bounds__(256) k_tridiag_status(const double *__restrict__ alpha,
                                                        const double *__restrict__ beta, int M,
                                                        double tol, double *__restrict__ work,
                                                        double *__restrict__ svec,
                                                        GsStatus *__restrict__ status, int want1) {
    tridiag_status_block(alpha, beta, M, tol, work, svec, status, want1 != 0);
}

// ---------------------------------------------------------------- engine

int engine_init(Engine &e, const HvOp &op, int prec, int nvec, int maxs, double btol, int reorth,
                Carver &cv) {
    e.op = op;
    e.prec = prec;
    e.nvec = nvec;
    e.dim = op.dim;
    e.maxs = maxs;
    e.reorth = reorth;
    size_t s = prec == QCM_FP64 ? 8 : 4;
    char *vecs = cv.take<char>(3 * s * (size_t)nvec * e.dim + 64);
    size_t vb = s * (size_t)nvec * e.dim;
    e.vbuf[0] = vecs;
    e.vbuf[1] = vecs + vb;
    e.vbuf[2] = vecs + 2 * vb;
    e.nchunks = (int)ceil_div(e.dim, kChunk);
    if (e.nchunks < 1) e.nchunks = 1;
    row_shape(op.up.d, op.dn.d, prec, &e.rows, &e.nblk);
    e.fused = !op.split && !op.csr.rowptr && op.up.d < 65536 &&
              fused_lds(op.up.d, e.rows, prec, op.md.nbytes, op.md.u_uniform,
                        2 * op.md.nbond) <= kFusedLds;
    // alpha partials: per fused-product block, per row-mixing workgroup when
    // the step's first pass rides on the two-pass product, else per chunk
    e.na = e.fused ? e.nblk : (op.split ? (int32_t)split_pa_count(op) : e.nchunks);
    e.partial = cv.take<double>((size_t)nvec * e.nchunks);
    int64_t npa = e.nblk > e.nchunks ? e.nblk : e.nchunks;
    if (e.na > npa) npa = e.na;
    // five partial arrays (alpha and the norm dots of the fused or two-pass
    // product)
    e.pa = cv.take<double>((size_t)nvec * npa * 5);
    // norm partials, or the two-pass step's per-range dot sums
    e.pn = cv.take<double>((size_t)nvec * std::max<size_t>(3 * (size_t)e.nchunks, 5 * kDotBlocks));
    e.cs.maxs = maxs;
    e.cs.btol = btol;
    e.cs.alpha = cv.take<double>((size_t)nvec * maxs);
    e.cs.beta = cv.take<double>((size_t)nvec * maxs);
    double *sc = cv.take<double>((size_t)nvec * 7);
    e.cs.amax = sc;
    e.cs.inv = sc + nvec;
    e.cs.corr = sc + 2 * nvec;
    e.cs.corr2 = sc + 3 * nvec;
    e.cs.b0sq = sc + 4 * nvec;
    e.scratch = sc + 5 * nvec;
    e.cs.apre = sc + 6 * nvec;
    int32_t *ic = cv.take<int32_t>((size_t)nvec * 3);
    e.cs.len = ic;
    e.cs.done = ic + nvec;
    e.cs.renorm = ic + 2 * nvec;
    e.ivp = 0;
    e.iv = 1;
    e.iw = 2;
    e.lazy = 0;
    e.pending = 0;
    return QCM_OK;
}

int engine_reset(Engine &e, hipStream_t s) {
    QCM_HIP(hipMemsetAsync(e.cs.alpha, 0, sizeof(double) * e.nvec * e.maxs, s));
    QCM_HIP(hipMemsetAsync(e.cs.beta, 0, sizeof(double) * e.nvec * e.maxs, s));
    QCM_HIP(hipMemsetAsync(e.cs.amax, 0, sizeof(double) * e.nvec * 7, s));
    QCM_HIP(hipMemsetAsync(e.cs.len, 0, sizeof(int32_t) * e.nvec * 3, s));
    size_t sz = (e.prec == QCM_FP64 ? 8 : 4) * (size_t)e.nvec * e.dim;
    e.ivp = 0;
    e.iv = 1;
    e.iw = 2;
    e.pending = 0;
    QCM_HIP(hipMemsetAsync(e.vbuf[e.ivp], 0, sz, s));
    return QCM_OK;
}

BGroup engine_group(const Engine &e, int n) {
    BGroup g;
    memset(&g, 0, sizeof g);
    const HvOp &op = e.op;
    g.d_up = op.up.d;
    g.d_dn = op.dn.d;
    g.dim = e.dim;
    g.su = op.up.states;
    g.sd = op.dn.states;
    g.eu = op.hu.ediag;
    g.ed = op.hd.ediag;
    g.nhu = op.hu.nh;
    g.nhd = op.hd.nh;
    g.colu = op.hu.col;
    g.cold = op.hd.col;
    g.cfu = op.hu.coef;
    g.cfd = op.hd.coef;
    g.ulut = op.md.ulut;
    g.pku = op.hu.pk;
    g.ctab = op.md.ctab;
    g.nctab = 2 * op.md.nbond;
    g.u_uniform = op.md.u_uniform;
    g.nbytes = op.md.nbytes;
    g.rows = e.rows;
    g.nblk = e.nblk;
    g.nvec = e.nvec;
    g.nchunks = e.nchunks;
    g.na = e.na;
    g.n = n;
    g.reorth = e.reorth;
    g.vp = e.vbuf[e.ivp];
    g.v = e.vbuf[e.iv];
    g.w = e.vbuf[e.iw];
    g.pa = e.pa;
    g.pstride = (int64_t)e.nvec * e.na;
    g.pn = e.pn;
    g.psi = nullptr;
    g.svec = nullptr;
    g.cs = e.cs;
    return g;
}

template <typename T>
static int step_t(Engine &e, int n, hipStream_t s) {
    const OneSrc src{engine_group(e, n)};
    const unsigned nk = (unsigned)e.nvec * e.nchunks;
    if (e.fused) {
        const size_t lds = fused_lds(e.op.up.d, e.rows, e.prec, e.op.md.nbytes,
                                     e.op.md.u_uniform, 2 * e.op.md.nbond);
        ks_hv<T, OneSrc><<<(unsigned)e.nvec * e.nblk, 256, lds, s>>>(src);
    } else if (e.op.split) {
        // the first pass (w -= beta' vp, partial <v, w>) inside the row-mixing
        // pass; a deferred update of the previous step inside the in-row pass
        SubPrev sp;
        sp.vp = e.vbuf[e.ivp];
        sp.beta = e.cs.beta;
        sp.maxs = e.cs.maxs;
        sp.n = n;
        sp.pa = e.pa;
        sp.pstride = (int64_t)e.nvec * e.na;
        sp.reorth = e.reorth;
        LazyUpd lz;
        if (e.pending) {
            // after the rotation: v_n is in ivp, v_{n-1} in iw (where W goes)
            lz.vold = e.vbuf[e.ivp];
            lz.vpold = e.vbuf[e.iw];
            lz.apre = e.cs.apre;
            lz.corr = e.cs.corr;
            lz.corr2 = e.cs.corr2;
            lz.inv = e.cs.inv;
            lz.reorth = e.reorth;
        }
        QCM_TRY(hv_split_launch_sub(e.op, e.prec, e.vbuf[e.iv], e.vbuf[e.iw], e.nvec, sp,
                                    e.pending ? &lz : nullptr, s));
        e.pending = 0;
        // alpha, then beta from the product's dots: no norm pass
        ks_dots_stage<OneSrc><<<dim3(kDotBlocks, (unsigned)e.nvec), 256, 0, s>>>(src);
        ks_finish_dots<OneSrc><<<e.nvec, kDotBlocks, 0, s>>>(src);
        // chains whose beta the dots cannot resolve take the direct norm
        ks_norm<T, OneSrc><<<nk, 256, 0, s>>>(src, 1);
        ks_finish<OneSrc><<<e.nvec, 256, 0, s>>>(src, 4);
    } else {
        QCM_TRY(hv_launch(e.op, e.prec, e.vbuf[e.iv], e.vbuf[e.iw], e.nvec, s));
        ks_sub_prev<T, OneSrc><<<nk, 256, 0, s>>>(src);
    }
    if (e.fused) {
        // alpha and beta from the fused product's dots; the direct norm pass
        // only for chains whose beta the dots cannot resolve
        ks_finish<OneSrc><<<e.nvec, 256, 0, s>>>(src, 3);
        ks_norm<T, OneSrc><<<nk, 256, 0, s>>>(src, 1);
        ks_finish<OneSrc><<<e.nvec, 256, 0, s>>>(src, 4);
    } else if (!e.op.split) {
        ks_finish<OneSrc><<<e.nvec, 256, 0, s>>>(src, 0);
        ks_norm<T, OneSrc><<<nk, 256, 0, s>>>(src, 0);
        ks_finish<OneSrc><<<e.nvec, 256, 0, s>>>(src, 1);
    }
    if (e.op.split && e.lazy)
        e.pending = 1;   // the next step's in-row pass forms v_{n+1}
    else
        ks_update<T, OneSrc><<<nk, 256, 0, s>>>(src);
    QCM_LAUNCH_CHECK();
    // rotate: v_{n-1} <- v_n, v_n <- the new vector, next w <- old v_{n-1}
    int t = e.ivp;
    e.ivp = e.iv;
    e.iv = e.iw;
    e.iw = t;
    return QCM_OK;
}

int engine_step(Engine &e, int n, hipStream_t s) {
    if (e.prec == QCM_FP64) return step_t<double>(e, n, s);
    return step_t<float>(e, n, s);
}

// The deferred update as its own pass (the update pass of the step before the
// rotation: w was its w, v its v, vp its vp).
template <typename T>
static int settle_t(Engine &e, hipStream_t s) {
    BGroup g = engine_group(e, 0);
    g.vp = e.vbuf[e.iw];
    g.v = e.vbuf[e.ivp];
    g.w = e.vbuf[e.iv];
    const OneSrc src{g};
    ks_update<T, OneSrc><<<(unsigned)e.nvec * e.nchunks, 256, 0, s>>>(src);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

int engine_settle(Engine &e, hipStream_t s) {
    if (!e.pending) return QCM_OK;
    e.pending = 0;
    if (e.prec == QCM_FP64) return settle_t<double>(e, s);
    return settle_t<float>(e, s);
}

// Normalise the current vectors v (chain start vectors), storing b0sq.
template <typename T>
static int normalize_t(Engine &e, hipStream_t s) {
    e.pending = 0;
    T *v = (T *)e.vbuf[e.iv];
    const dim3 g((unsigned)e.nchunks, (unsigned)e.nvec);
    k_dot_partial<T, T><<<g, 256, 0, s>>>(v, v, e.dim, e.nchunks, e.partial);
    k_finish<<<e.nvec, 256, 0, s>>>(e.partial, e.nchunks, 5, e.cs, 0, nullptr);
    k_scale<T><<<g, 256, 0, s>>>(v, e.dim, e.cs);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

int engine_normalize(Engine &e, hipStream_t s) {
    if (e.prec == QCM_FP64) return normalize_t<double>(e, s);
    return normalize_t<float>(e, s);
}

int engine_seed(Engine &e, uint64_t seed, const void *v0, hipStream_t s) {
    e.pending = 0;
    void *v = e.vbuf[e.iv];
    size_t sz = (e.prec == QCM_FP64 ? 8 : 4) * (size_t)e.dim;
    if (v0) {
        QCM_HIP(hipMemcpyAsync(v, v0, sz, hipMemcpyDeviceToDevice, s));
    } else if (e.prec == QCM_FP64) {
        k_splitmix<double><<<ceil_div(e.dim, 256), 256, 0, s>>>((double *)v, e.dim, seed);
    } else {
        k_splitmix<float><<<ceil_div(e.dim, 256), 256, 0, s>>>((float *)v, e.dim, seed);
    }
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

int engine_accum(Engine &e, double *psi, const double *coef, int n, hipStream_t s) {
    QCM_TRY(engine_settle(e, s));
    const unsigned g = (unsigned)e.nchunks;
    if (e.prec == QCM_FP64)
        k_accum<double><<<g, 256, 0, s>>>(psi, (const double *)e.vbuf[e.iv], e.dim, coef, n);
    else
        k_accum<float><<<g, 256, 0, s>>>(psi, (const float *)e.vbuf[e.iv], e.dim, coef, n);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

int tridiag_status(const double *alpha, const double *beta, int M, double tol, double *work,
                   double *svec, GsStatus *status, hipStream_t s, int want1) {
    k_tridiag_status<<<1, 256, 0, s>>>(alpha, beta, M, tol, work, svec, status, want1);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

// psi /= |psi| (FP64), through the chain state of chain 0 of e.
int psi_finalize(Engine &e, double *psi, hipStream_t s) {
    const int64_t dim = e.dim;
    int nch = (int)ceil_div(dim, kChunk);
    k_dot_partial<double, double><<<dim3(nch, 1), 256, 0, s>>>(psi, psi, dim, nch, e.partial);
    ChainState cs1 = e.cs;
    k_finish<<<1, 256, 0, s>>>(e.partial, nch, 5, cs1, 0, nullptr);
    k_scale<double><<<dim3(nch, 1), 256, 0, s>>>(psi, dim, cs1);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

int residual_norm(const HvOp &op, const double *psi, double theta, double *w64, double *partial,
                  double *out, hipStream_t s) {
    QCM_TRY(hv_launch(op, QCM_FP64, psi, w64, 1, s));
    int nch = (int)ceil_div(op.dim, kChunk);
    k_resid_partial<<<nch, 256, 0, s>>>(w64, psi, theta, op.dim, nch, partial);
    ChainState dummy{};
    k_finish<<<1, 256, 0, s>>>(partial, nch, 2, dummy, 0, out);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

}  // namespace qcm

using namespace qcm;

extern "C" void qcm_lanczos_default_opts(qcm_lanczos_opts *o) {
    if (!o) return;
    o->max_iter = 600;
    o->fixed_steps = 0;
    o->want_vector = 1;
    o->reorth = 0;
    o->prec = QCM_FP64;
    o->check_every = 1;
    o->tol = 1e-12;
    o->btol = 1e-13;
    o->seed = 1;
    o->d_v0 = nullptr;
}

namespace qcm {

int gs_run(const char *fn, const GsSetup &setup, int64_t dim, const qcm_lanczos_opts *o,
           double *h_alpha, double *h_beta, void *d_gs, qcm_gs_result *h_out, void *d_ws,
           size_t ws_bytes, size_t *ws_needed, void *stream) {
    if (!ws_needed || !o) return fail(QCM_EARG, "%s: NULL ws_needed or opts", fn);
    if (o->prec != QCM_FP64 && o->prec != QCM_FP32V)
        return fail(QCM_EARG, "%s: bad prec %d", fn, o->prec);
    if (o->max_iter < 1 && o->fixed_steps < 1)
        return fail(QCM_EARG, "%s: max_iter and fixed_steps both < 1", fn);
    if (o->want_vector && !d_gs && d_ws) return fail(QCM_EARG, "%s: want_vector needs d_gs", fn);
    if (dim < 1) return fail(QCM_EARG, "%s: empty sector", fn);
    const int limit = o->fixed_steps > 0 ? o->fixed_steps : o->max_iter;
    const int every = o->check_every > 0 ? o->check_every : 1;
    // the workspace is laid out by one function, run first without a base to
    // size it (no launch) and then on the workspace
    HvOp op;
    Engine e;
    double *svec = nullptr, *work = nullptr, *dscal = nullptr;
    GsStatus *status = nullptr;
    auto layout = [&](Carver &cv, hipStream_t st) -> int {
        QCM_TRY(setup(cv, st, &op));
        QCM_TRY(engine_init(e, op, o->prec, 1, limit, o->btol, o->reorth, cv));
        svec = cv.take<double>(limit);
        work = cv.take<double>((size_t)limit * 6);
        status = cv.take<GsStatus>(1);
        dscal = cv.take<double>(64);
        return QCM_OK;
    };
    Carver dry(nullptr);
    QCM_TRY(layout(dry, nullptr));
    const size_t need = dry.off + 256;
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (!h_out) return fail(QCM_EARG, "%s: h_out is NULL", fn);
    if (ws_bytes < need) return fail(QCM_EWORKSPACE, "%s: workspace %zu < %zu", fn, ws_bytes, need);
    hipStream_t s = as_stream(stream);
    Carver cv(d_ws);
    QCM_TRY(layout(cv, s));

    // first pass: coefficients; the status starts empty (M = 0: no hint for
    // the first test, as in the batched engine)
    QCM_HIP(hipMemsetAsync(status, 0, sizeof(GsStatus), s));
    QCM_TRY(engine_reset(e, s));
    QCM_TRY(engine_seed(e, o->seed, o->d_v0, s));
    QCM_TRY(engine_normalize(e, s));
    // the first pass needs the coefficients only: updates may be deferred
    e.lazy = 1;
    GsStatus hs{};
    int M = 0, conv = 0, brk = 0;
    int32_t done = 0;
    for (int n = 0; n < limit; ++n) {
        QCM_TRY(engine_step(e, n, s));
        M = n + 1;
        bool last = (n + 1 == limit);
        bool check = o->fixed_steps > 0 ? false : ((n + 1) % every == 0 || last);
        // breakdown is checked together with the residual test; with fixed steps
        // every `every` steps as well
        if (o->fixed_steps > 0 && ((n + 1) % every == 0 || last)) check = true;
        if (check) {
            QCM_HIP(hipMemcpyAsync(&done, e.cs.done, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            if (o->fixed_steps <= 0) {
                QCM_TRY(tridiag_status(e.cs.alpha, e.cs.beta, M, o->tol, work, svec, status, s, 0));
                QCM_HIP(hipMemcpyAsync(&hs, status, sizeof hs, hipMemcpyDeviceToHost, s));
            }
            QCM_HIP(hipStreamSynchronize(s));
            if (done) {
                brk = 1;
                conv = 1;
                // the chain stopped at len; steps after it carry zero vectors
                int32_t len = 0;
                QCM_HIP(hipMemcpy(&len, e.cs.len, sizeof len, hipMemcpyDeviceToHost));
                M = len;
                break;
            }
            if (o->fixed_steps <= 0 && hs.converged) {
                conv = 1;
                break;
            }
        }
    }
    QCM_TRY(tridiag_status(e.cs.alpha, e.cs.beta, M, o->tol, work, svec, status, s));
    QCM_HIP(hipMemcpyAsync(&hs, status, sizeof hs, hipMemcpyDeviceToHost, s));
    QCM_HIP(hipStreamSynchronize(s));
    if (o->fixed_steps <= 0 && !brk) conv = hs.converged;

    qcm_gs_result r{};
    r.e0 = hs.theta0;
    r.residual_est = hs.est;
    r.theta1 = hs.theta1;
    r.n_iter = M;
    r.converged = conv;
    r.breakdown = brk;
    r.degenerate_suspect = degenerate_suspect(hs.theta0, hs.theta1);
    r.true_residual = -1.0;

    // the coefficients of the first pass go out before the second pass reruns
    // (and rewrites, with identical values) the recurrence
    if (h_alpha) QCM_HIP(hipMemcpy(h_alpha, e.cs.alpha, sizeof(double) * M, hipMemcpyDeviceToHost));
    if (h_beta) QCM_HIP(hipMemcpy(h_beta, e.cs.beta, sizeof(double) * M, hipMemcpyDeviceToHost));

    if (o->want_vector && d_gs) {
        // second pass: identical recurrence, psi = sum_n s_n v_n
        double *psi = (double *)d_gs;
        QCM_HIP(hipMemsetAsync(psi, 0, sizeof(double) * dim, s));
        e.lazy = 0;
        QCM_TRY(engine_reset(e, s));
        QCM_TRY(engine_seed(e, o->seed, o->d_v0, s));
        QCM_TRY(engine_normalize(e, s));
        for (int n = 0; n < M; ++n) {
            QCM_TRY(engine_accum(e, psi, svec, n, s));
            if (n + 1 < M) QCM_TRY(engine_step(e, n, s));
        }
        // normalise psi and take the true residual, all FP64
        QCM_TRY(psi_finalize(e, psi, s));
        double *w64 = (double *)e.vbuf[0];  // 8*dim bytes: the first two FP32 or one FP64 vector
        QCM_TRY(residual_norm(op, psi, hs.theta0, w64, e.partial, dscal, s));
        double r2 = 0.0;
        QCM_HIP(hipMemcpyAsync(&r2, dscal, sizeof r2, hipMemcpyDeviceToHost, s));
        QCM_HIP(hipStreamSynchronize(s));
        r.true_residual = sqrt(r2);
    }
    *h_out = r;
    return QCM_OK;
}

}  // namespace qcm

extern "C" int qcm_lanczos_gs(const qcm_model *m, const qcm_basis *b, const qcm_lanczos_opts *o,
                              double *h_alpha, double *h_beta, void *d_gs, qcm_gs_result *h_out,
                              void *d_ws, size_t ws_bytes, size_t *ws_needed, void *stream) {
    if (!ws_needed || !o) return fail(QCM_EARG, "qcm_lanczos_gs: NULL ws_needed or opts");
    QCM_TRY(validate_model(m));
    QCM_TRY(check_basis(b, m->L));
    auto setup = [&](Carver &cv, hipStream_t st, HvOp *op) -> int {
        return hv_setup(m, b, cv, op, st);
    };
    return gs_run("qcm_lanczos_gs", setup, b->dim, o, h_alpha, h_beta, d_gs, h_out, d_ws,
                  ws_bytes, ws_needed, stream);
}

namespace qcm {

// Normalise the start vectors from norm partials already in e.partial.
int engine_normalize_from_partials(Engine &e, hipStream_t s) {
    e.pending = 0;
    const dim3 g((unsigned)e.nchunks, (unsigned)e.nvec);
    k_finish<<<e.nvec, 256, 0, s>>>(e.partial, e.nchunks, 5, e.cs, 0, nullptr);
    if (e.prec == QCM_FP64)
        k_scale<double><<<g, 256, 0, s>>>((double *)e.vbuf[e.iv], e.dim, e.cs);
    else
        k_scale<float><<<g, 256, 0, s>>>((float *)e.vbuf[e.iv], e.dim, e.cs);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

}  // namespace qcm
