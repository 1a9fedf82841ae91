// H.v on one (N_up, N_dn) sector (paper: section "Exact diagonalizations",
// eq. (factorized) H = K_up (x) 1 + 1 (x) K_dn + V_int, with the hopping
// element (-1)^M t_ab of subsection "Coding of the basis states" and the
// interaction counted from b_up & b_dn).
//
// A vector is the row-major d_dn x d_up matrix V[i_dn][i_up].  Then
//   W = V K_up^T  (mixing inside a row)  +  K_dn V  (mixing whole rows)  +  D o V.
// Where the row tile fits LDS and the packed up hops exist, the product runs
// in the Lanczos step's kernel (lanczos_step.h) with no subtraction and no
// partial sums; otherwise (or for long rows, in the two-pass form) here.
// The kernel below gives each workgroup one row i_dn: the row is staged in LDS,
// the inside-row term gathers from LDS, the row-mixing term streams the
// neighbour rows from global memory (coalesced along i_up), and the diagonal
// is computed from the two strings.  All sums are FP64 in registers; the
// output is rounded once to the storage type.
#include <string.h>

#include <mutex>

#include "qcm_internal.h"
#include "lanczos_step.h"

namespace qcm {

int count_bonds(const qcm_model *m) {
    int nb = 0;
    for (int a = 0; a < m->L; ++a)
        for (int b = a + 1; b < m->L; ++b)
            if (m->t[a * m->L + b] != 0.0) ++nb;
    return nb;
}

int validate_model(const qcm_model *m) {
    if (!m || !m->t || !m->U) return fail(QCM_EARG, "model, t or U is NULL");
    if (m->L < 1 || m->L > 32) return fail(QCM_ERANGE, "model L=%d outside 1..32", m->L);
    for (int a = 0; a < m->L; ++a)
        for (int b = 0; b < m->L; ++b)
            if (m->t[a * m->L + b] != m->t[b * m->L + a])
                return fail(QCM_EARG, "t is not symmetric at (%d,%d)", a, b);
    return QCM_OK;
}

size_t model_dev_bytes(int L) {
    Carver cv(nullptr);
    int nbytes = (L + 7) / 8;
    cv.take<double>((size_t)L * L);
    cv.take<int32_t>(L * L);
    cv.take<int32_t>(L * L);
    cv.take<double>(L * L);
    cv.take<double>(nbytes * 256);
    cv.take<double>(nbytes * 256);
    cv.take<double>(2 * L * L);
    return cv.off + 256;
}

// Copies the model to the device: t, the bond list, and per-byte lookup
// tables for the diagonal (sum of U_k and of t_kk over the set bits of one
// byte of a string).
int upload_model(const qcm_model *m, Carver &cv, ModelDev *md, hipStream_t s) {
    const int L = m->L;
    md->L = L;
    md->nbytes = (L + 7) / 8;
    md->nbond = count_bonds(m);
    md->t = cv.take<double>((size_t)L * L);
    md->bond_a = cv.take<int32_t>(L * L);
    md->bond_b = cv.take<int32_t>(L * L);
    md->bond_t = cv.take<double>(L * L);
    md->ulut = cv.take<double>(md->nbytes * 256);
    md->tlut = cv.take<double>(md->nbytes * 256);
    md->ctab = cv.take<double>(2 * L * L);
    double u0 = m->U[0];
    md->u_uniform = u0;
    for (int k = 0; k < L; ++k)
        if (m->U[k] != u0 || u0 < 0) md->u_uniform = -1.0;
    md->t_is_uniform = 1;
    md->t_uniform = 0.0;
    bool seen = false;
    for (int a = 0; a < L; ++a)
        for (int b = a + 1; b < L; ++b) {
            const double tab = m->t[a * L + b];
            if (tab == 0.0) continue;
            if (!seen) md->t_uniform = tab;
            else if (tab != md->t_uniform) md->t_is_uniform = 0;
            seen = true;
        }
    if (!cv.base) return QCM_OK;
    // pack everything into one host staging block laid out like the device block
    size_t total = (char *)(md->ctab + 2 * L * L) - (char *)md->t;
    std::vector<char> host(total, 0);
    auto at = [&](void *dev) { return host.data() + ((char *)dev - (char *)md->t); };
    memcpy(at(md->t), m->t, sizeof(double) * L * L);
    int nb = 0;
    int32_t *ba = (int32_t *)at(md->bond_a), *bb = (int32_t *)at(md->bond_b);
    double *bt = (double *)at(md->bond_t);
    for (int a = 0; a < L; ++a)
        for (int b = a + 1; b < L; ++b)
            if (m->t[a * L + b] != 0.0) {
                ba[nb] = a;
                bb[nb] = b;
                bt[nb] = m->t[a * L + b];
                ++nb;
            }
    double *ct = (double *)at(md->ctab);
    for (int k = 0; k < nb; ++k) {
        ct[2 * k] = bt[k];
        ct[2 * k + 1] = -bt[k];
    }
    double *ul = (double *)at(md->ulut), *tl = (double *)at(md->tlut);
    for (int byte = 0; byte < md->nbytes; ++byte)
        for (int x = 0; x < 256; ++x) {
            double su = 0, st = 0;
            for (int q = 0; q < 8; ++q) {
                int k = byte * 8 + q;
                if (k < L && ((x >> q) & 1)) {
                    su += m->U[k];
                    st += m->t[k * L + k];
                }
            }
            ul[byte * 256 + x] = su;
            tl[byte * 256 + x] = st;
        }
    QCM_HIP(hipMemcpyAsync(md->t, host.data(), total, hipMemcpyHostToDevice, s));
    return QCM_OK;
}

size_t hop_tables_bytes(const qcm_model *m, int64_t d) {
    int W = count_bonds(m);
    if (W < 1) W = 1;
    Carver cv(nullptr);
    cv.take<int32_t>(d);
    cv.take<int32_t>((size_t)W * d);
    cv.take<double>((size_t)W * d);
    cv.take<double>(d);
    if (d < 65536) cv.take<uint32_t>((size_t)W * d);
    return cv.off + 256;
}

// Hopping list of every string of one spin.  For a bond (a, b) at most one
// direction is allowed: the occupied end moves to the empty end.  The entry
// for row string x is the column label of the string with the electron moved
// and the element t_ab times (-1)^(occupied orbitals strictly between a, b).
__global__ void k_build_hops(int64_t d, int rowmajor, int W, int L, int l_lo, int l_hi,
                             const uint32_t *__restrict__ states,
                             const int32_t *__restrict__ rlo, const int32_t *__restrict__ rhi,
                             int nbond, const int32_t *__restrict__ ba,
                             const int32_t *__restrict__ bb, const double *__restrict__ bt,
                             const double *__restrict__ tlut, int nbytes,
                             int32_t *__restrict__ nh, int32_t *__restrict__ col,
                             double *__restrict__ coef, double *__restrict__ ediag,
                             uint32_t *__restrict__ pk) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d) return;
    uint32_t x = states[i];
    int n = 0;
    for (int k = 0; k < nbond; ++k) {
        int a = ba[k], b = bb[k];
        uint32_t ma = 1u << a, mb = 1u << b;
        bool oa = x & ma, ob = x & mb;
        if (oa == ob) continue;
        uint32_t y = x ^ ma ^ mb;
        uint32_t between = ((mb - 1u) & ~(ma | (ma - 1u)));  // a < b: bits a+1..b-1
        int m = __popc(x & between);
        const int64_t at = rowmajor ? i * W + n : (int64_t)n * d + i;
        const int32_t c = spin_rank(rlo, rhi, l_lo, l_hi, y);
        col[at] = c;
        coef[at] = (m & 1) ? -bt[k] : bt[k];
        if (pk) pk[at] = (uint32_t)c | ((uint32_t)(2 * k + (m & 1)) << 16);
        ++n;
    }
    nh[i] = n;
    double e = 0.0;
    for (int byte = 0; byte < nbytes; ++byte) e += tlut[byte * 256 + ((x >> (8 * byte)) & 255u)];
    ediag[i] = e;
}

int build_hop_tables(const ModelDev &md, const SpinTables &st, Carver &cv, HopTables *ht,
                     hipStream_t s, int nbond_host, int rowmajor) {
    int W = nbond_host < 1 ? 1 : nbond_host;
    ht->d = st.d;
    ht->width = W;
    ht->rowmajor = rowmajor;
    ht->nh = cv.take<int32_t>(st.d);
    ht->col = cv.take<int32_t>((size_t)W * st.d);
    ht->coef = cv.take<double>((size_t)W * st.d);
    ht->ediag = cv.take<double>(st.d);
    // packed entries (column | index of +-t_ab in the model's ctab << 16) when
    // labels fit 16 bits; slot-major layout only
    ht->pk = (!rowmajor && st.d < 65536) ? cv.take<uint32_t>((size_t)W * st.d) : nullptr;
    if (!cv.base) return QCM_OK;
    const int B = 256;
    k_build_hops<<<ceil_div(st.d, B), B, 0, s>>>(st.d, ht->rowmajor, W, st.L, st.l_lo, st.l_hi, st.states,
                                                  st.rank_lo, st.rank_hi, nbond_host, md.bond_a,
                                                  md.bond_b, md.bond_t, md.tlut, md.nbytes,
                                                  ht->nh, ht->col, ht->coef, ht->ediag,
                                                  rowmajor ? nullptr : ht->pk);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

// ---------------------------------------------------------------- the product

template <typename T>
struct Loader;
template <>
struct Loader<double> {
    __device__ static double ld(const double *p) { return __builtin_nontemporal_load(p); }
};
template <>
struct Loader<float> {
    __device__ static double ld(const float *p) { return (double)__builtin_nontemporal_load(p); }
};

struct HvArgs {
    int64_t d_up, d_dn, dim;
    const uint32_t *su, *sd;
    const double *eu, *ed;
    int32_t wu, wd;
    const int32_t *nhu, *nhd;
    const int32_t *colu, *cold;
    const double *cfu, *cfd;
    const double *ulut;
    int32_t nbytes;
    double u_uniform;
};

template <typename T, bool kRowLds>
__global__ void __launch_bounds__(1024) k_hv_rows(HvArgs a, const T *__restrict__ vin,
                                                  T *__restrict__ wout) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *ulut_s = reinterpret_cast<double *>(smem_raw);
    const int nlut = a.u_uniform >= 0.0 ? 0 : a.nbytes * 256;
    T *row = reinterpret_cast<T *>(smem_raw + sizeof(double) * nlut);

    const int64_t vec = blockIdx.y;
    const T *v = vin + vec * a.dim;
    T *w = wout + vec * a.dim;
    for (int k = threadIdx.x; k < nlut; k += blockDim.x) ulut_s[k] = a.ulut[k];

    for (int64_t idn = blockIdx.x; idn < a.d_dn; idn += gridDim.x) {
        const T *vrow = v + idn * a.d_up;
        if (kRowLds) {
            __syncthreads();
            for (int64_t k = threadIdx.x; k < a.d_up; k += blockDim.x) row[k] = vrow[k];
        }
        __syncthreads();
        const uint32_t bd = a.sd[idn];
        const double edn = a.ed[idn];
        const int nhd = a.nhd[idn];
        for (int64_t iu = threadIdx.x; iu < a.d_up; iu += blockDim.x) {
            const uint32_t bu = a.su[iu];
            const uint32_t dbl = bu & bd;
            double diag = a.eu[iu] + edn;
            if (a.u_uniform >= 0.0) {
                diag += a.u_uniform * (double)__popc(dbl);
            } else {
                for (int byte = 0; byte < a.nbytes; ++byte)
                    diag += ulut_s[byte * 256 + ((dbl >> (8 * byte)) & 255u)];
            }
            const double vi = kRowLds ? (double)row[iu] : (double)vrow[iu];
            double acc = diag * vi;
            // inside-row term: K_up
            const int nhu = a.nhu[iu];
            for (int s = 0; s < nhu; ++s) {
                const int64_t e = (int64_t)s * a.d_up + iu;
                const int32_t j = a.colu[e];
                const double x = kRowLds ? (double)row[j] : (double)vrow[j];
                acc = fma(a.cfu[e], x, acc);
            }
            // row-mixing term: K_dn
            for (int s = 0; s < nhd; ++s) {
                const int64_t e = (int64_t)s * a.d_dn + idn;
                const int32_t jd = a.cold[e];
                acc = fma(a.cfd[e], (double)v[(int64_t)jd * a.d_up + iu], acc);
            }
            w[idn * a.d_up + iu] = (T)acc;
        }
    }
}

size_t hv_scratch_bytes(const HvOp &, int, int) { return 0; }

template <typename T>
static int hv_launch_t(const HvOp &op, const void *v, void *w, int nvec, hipStream_t s) {
    {
        // rows that fit LDS with the packed up hops: the Lanczos step's product
        // kernel, with no subtraction and no partial sums
        const int prec = sizeof(T) == 8 ? QCM_FP64 : QCM_FP32V;
        int32_t rows = 0, nblk = 0;
        row_shape(op.up.d, op.dn.d, prec, &rows, &nblk);
        const size_t lds = fused_lds(op.up.d, rows, prec, op.md.nbytes, op.md.u_uniform,
                                     2 * op.md.nbond);
        if (op.hu.pk && lds <= kFusedLds) {
            BGroup g;
            memset(&g, 0, sizeof g);
            g.d_up = op.up.d;
            g.d_dn = op.dn.d;
            g.dim = op.dim;
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
            g.rows = rows;
            g.nblk = nblk;
            g.nvec = nvec;
            g.vp = v;   // not read: no subtraction
            g.v = v;
            g.w = w;
            const OneSrc src{g};
            ks_hv<T, OneSrc><<<(unsigned)((int64_t)nvec * nblk), 256, lds, s>>>(src);
            QCM_LAUNCH_CHECK();
            return QCM_OK;
        }
    }
    HvArgs a;
    a.d_up = op.up.d;
    a.d_dn = op.dn.d;
    a.dim = op.dim;
    a.su = op.up.states;
    a.sd = op.dn.states;
    a.eu = op.hu.ediag;
    a.ed = op.hd.ediag;
    a.wu = op.hu.width;
    a.wd = op.hd.width;
    a.nhu = op.hu.nh;
    a.nhd = op.hd.nh;
    a.colu = op.hu.col;
    a.cold = op.hd.col;
    a.cfu = op.hu.coef;
    a.cfd = op.hd.coef;
    a.ulut = op.md.ulut;
    a.nbytes = op.md.nbytes;
    a.u_uniform = op.md.u_uniform;
    const size_t lut = a.u_uniform >= 0.0 ? 0 : sizeof(double) * a.nbytes * 256;
    const size_t rowb = sizeof(T) * (size_t)a.d_up;
    const size_t lds_cap = 160 * 1024;
    int threads = a.d_up >= 8192 ? 1024 : a.d_up >= 2048 ? 512 : a.d_up >= 512 ? 256 : 64;
    int64_t gx = a.d_dn;
    if (gx > (int64_t(1) << 30)) gx = int64_t(1) << 30;
    dim3 grid((unsigned)gx, (unsigned)nvec);
    if (lut + rowb <= lds_cap) {
        k_hv_rows<T, true><<<grid, threads, lut + rowb, s>>>(a, (const T *)v, (T *)w);
    } else {
        k_hv_rows<T, false><<<grid, threads, lut, s>>>(a, (const T *)v, (T *)w);
    }
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

int hv_split_launch(const HvOp &op, int prec, const void *v, void *w, int nvec, hipStream_t s);

int hv_launch(const HvOp &op, int prec, const void *v, void *w, int nvec, hipStream_t s) {
    if (op.dim == 0 || nvec == 0) return QCM_OK;
    if (op.csr.rowptr) {
        if (prec != QCM_FP64) return fail(QCM_EARG, "the stored matrix runs in FP64 only");
        return sym_hv_launch(op.csr, (const double *)v, (double *)w, nvec, s);
    }
    if (op.split) return hv_split_launch(op, prec, v, w, nvec, s);
    if (prec == QCM_FP64) return hv_launch_t<double>(op, v, w, nvec, s);
    return hv_launch_t<float>(op, v, w, nvec, s);
}

// Sizes and set-up shared by every entry point that applies H.
// The bytes hv_setup carves: the same carving run without a base (no launch).
int hv_setup_bytes(const qcm_model *m, const qcm_basis *b, size_t *need) {
    Carver dry(nullptr);
    HvOp op;
    QCM_TRY(hv_setup(m, b, dry, &op, nullptr));
    *need = dry.off + 256;
    return QCM_OK;
}

int hv_setup(const qcm_model *m, const qcm_basis *b, Carver &cv, HvOp *op, hipStream_t s) {
    QCM_TRY(upload_model(m, cv, &op->md, s));
    op->up = spin_from_basis(b, 0);
    op->dn = spin_from_basis(b, 1);
    op->dim = b->dim;
    int nb = count_bonds(m);
    QCM_TRY(build_hop_tables(op->md, op->up, cv, &op->hu, s, nb));
    QCM_TRY(build_hop_tables(op->md, op->dn, cv, &op->hd, s, nb));
    op->split = 0;
    if (split_applies(m, b->n_up, b->d_up, b->d_dn)) QCM_TRY(split_prepare(m, *op, cv, s));
    return QCM_OK;
}

int check_basis(const qcm_basis *b, int L) {
    if (!b) return fail(QCM_EARG, "basis is NULL");
    if (b->L != L) return fail(QCM_EARG, "basis L=%d differs from model L=%d", b->L, L);
    if (b->d_up != binom(L, b->n_up) || b->d_dn != binom(L, b->n_dn) ||
        b->dim != b->d_up * b->d_dn)
        return fail(QCM_EARG, "basis sizes are inconsistent");
    if (b->dim > 0 && (!b->states_up || !b->states_dn || !b->rank_lo_up || !b->rank_hi_up ||
                       !b->rank_lo_dn || !b->rank_hi_dn))
        return fail(QCM_EARG, "basis has NULL device tables (was it built with a workspace?)");
    return QCM_OK;
}

}  // namespace qcm

using namespace qcm;

extern "C" int qcm_hv(const qcm_model *m, const qcm_basis *b, int32_t prec, const void *d_v,
                      void *d_w, void *d_ws, size_t ws_bytes, size_t *ws_needed, void *stream) {
    if (!ws_needed) return fail(QCM_EARG, "qcm_hv: ws_needed is NULL");
    QCM_TRY(validate_model(m));
    QCM_TRY(check_basis(b, m->L));
    if (prec != QCM_FP64 && prec != QCM_FP32V) return fail(QCM_EARG, "qcm_hv: bad prec %d", prec);
    size_t need = 0;
    QCM_TRY(hv_setup_bytes(m, b, &need));
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (ws_bytes < need) return fail(QCM_EWORKSPACE, "qcm_hv: workspace %zu < %zu", ws_bytes, need);
    if (!d_v || !d_w) return fail(QCM_EARG, "qcm_hv: NULL vector");
    size_t vb = (prec == QCM_FP64 ? 8 : 4) * (size_t)b->dim;
    const char *pv = (const char *)d_v, *pw = (const char *)d_w;
    if (pv < pw + vb && pw < pv + vb) return fail(QCM_EARG, "qcm_hv: v and w overlap");
    hipStream_t s = as_stream(stream);
    Carver cv(d_ws);
    HvOp op;
    QCM_TRY(hv_setup(m, b, cv, &op, s));
    return hv_launch(op, prec, d_v, d_w, 1, s);
}

// ---------------------------------------------------------------- allocation-free product

namespace qcm {

// The tables of the allocation-free product live in this device array, one
// copy per GPU the library runs on, held until the process ends.  Host code
// never passes the array's name to a kernel or a copy: it uses the address
// hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
}  // namespace

// The device address of `scratch` on the current device, looked up on the
// first call there.
static int static_scratch(void **out) {
    int dev = -1;
    QCM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(QCM_EARG, "qcm_hv_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        QCM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(QCM_EHIP, "qcm_hv_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QCM_OK;
}

}  // namespace qcm

extern "C" int qcm_hv_noalloc(const qcm_model *m, const qcm_basis *b, int32_t prec,
                              const void *d_v, void *d_w, void *stream) {
    QCM_TRY(validate_model(m));
    QCM_TRY(check_basis(b, m->L));
    if (prec != QCM_FP64 && prec != QCM_FP32V)
        return fail(QCM_EARG, "qcm_hv_noalloc: bad prec %d", prec);
    size_t need = 0;
    QCM_TRY(hv_setup_bytes(m, b, &need));
    if (need > kStaticScratchBytes)
        return fail(QCM_EWORKSPACE,
                    "qcm_hv_noalloc: the sector's tables need %zu bytes, more than the %zu-byte "
                    "static scratch (use qcm_hv with a workspace)",
                    need, kStaticScratchBytes);
    if (!d_v || !d_w) return fail(QCM_EARG, "qcm_hv_noalloc: NULL vector");
    size_t vb = (prec == QCM_FP64 ? 8 : 4) * (size_t)b->dim;
    const char *pv = (const char *)d_v, *pw = (const char *)d_w;
    if (pv < pw + vb && pw < pv + vb) return fail(QCM_EARG, "qcm_hv_noalloc: v and w overlap");
    void *ws = nullptr;
    QCM_TRY(static_scratch(&ws));
    hipStream_t s = as_stream(stream);
    // every table the product reads is rewritten here, so nothing carried
    // over from an earlier call needs clearing
    Carver cv(ws);
    HvOp op;
    QCM_TRY(hv_setup(m, b, cv, &op, s));
    return hv_launch(op, prec, d_v, d_w, 1, s);
}

// ---------------------------------------------------------------- plans

struct qcm_hv_plan {
    qcm::HvOp op;
    int32_t prec;
    int64_t dim;
};

extern "C" int qcm_hv_plan_create(const qcm_model *m, const qcm_basis *b, int32_t prec,
                                  void *d_ws, size_t ws_bytes, size_t *ws_needed, void *stream,
                                  qcm_hv_plan **out) {
    if (!ws_needed) return fail(QCM_EARG, "qcm_hv_plan_create: ws_needed is NULL");
    QCM_TRY(validate_model(m));
    QCM_TRY(check_basis(b, m->L));
    if (prec != QCM_FP64 && prec != QCM_FP32V)
        return fail(QCM_EARG, "qcm_hv_plan_create: bad prec %d", prec);
    size_t need = 0;
    QCM_TRY(hv_setup_bytes(m, b, &need));
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (!out) return fail(QCM_EARG, "qcm_hv_plan_create: out is NULL");
    *out = nullptr;
    if (ws_bytes < need)
        return fail(QCM_EWORKSPACE, "qcm_hv_plan_create: workspace %zu < %zu", ws_bytes, need);
    qcm_hv_plan *p = new qcm_hv_plan();
    Carver cv(d_ws);
    const int rc = hv_setup(m, b, cv, &p->op, as_stream(stream));
    if (rc != QCM_OK) {
        delete p;
        return rc;
    }
    p->prec = prec;
    p->dim = b->dim;
    *out = p;
    return QCM_OK;
}

extern "C" int qcm_hv_plan_apply(const qcm_hv_plan *p, const void *d_v, void *d_w, int32_t nvec,
                                 void *stream) {
    if (!p) return fail(QCM_EARG, "qcm_hv_plan_apply: plan is NULL");
    if (nvec < 1 || !d_v || !d_w) return fail(QCM_EARG, "qcm_hv_plan_apply: bad vectors");
    const size_t vb = (p->prec == QCM_FP64 ? 8 : 4) * (size_t)p->dim * (size_t)nvec;
    const char *pv = (const char *)d_v, *pw = (const char *)d_w;
    if (pv < pw + vb && pw < pv + vb) return fail(QCM_EARG, "qcm_hv_plan_apply: v and w overlap");
    return hv_launch(p->op, p->prec, d_v, d_w, nvec, as_stream(stream));
}

extern "C" int qcm_hv_plan_destroy(qcm_hv_plan *p) {
    delete p;
    return QCM_OK;
}
