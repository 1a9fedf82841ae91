// Internal declarations of the MI355X ED library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/qcm.h"

namespace qcm {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

#define QCM_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::qcm::fail(QCM_EHIP, "%s failed: %s (%s:%d)", #call,                \
                               hipGetErrorString(e_), __FILE__, __LINE__);               \
    } while (0)

#define QCM_LAUNCH_CHECK()                                                               \
    do {                                                                                 \
        hipError_t e_ = hipGetLastError();                                               \
        if (e_ != hipSuccess)                                                            \
            return ::qcm::fail(QCM_EHIP, "kernel launch failed: %s (%s:%d)",            \
                               hipGetErrorString(e_), __FILE__, __LINE__);               \
    } while (0)

#define QCM_TRY(expr)                                                                    \
    do {                                                                                 \
        int r_ = (expr);                                                                 \
        if (r_ != QCM_OK) return r_;                                                     \
    } while (0)

// ---------------------------------------------------------------- binomials
// C(n, k) by the multiplicative formula; exact in int64 for n <= 32.  Only used
// while building tables, never in the H.v loops.
__device__ __host__ inline int64_t binom(int n, int k) {
    if (n < 0 || k < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// ---------------------------------------------------------------- workspace
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <typename T>
    T *take(size_t n, size_t align = 256) {
        off = (off + align - 1) / align * align;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

inline size_t ceil_div(size_t a, size_t b) { return (a + b - 1) / b; }

// The ground state may be degenerate: the second Ritz value lies within
// 1e-8 max(1, |theta_0|) of the first (theta_1 is NaN for a 1x1 T).
inline int degenerate_suspect(double theta0, double theta1) {
    return (theta1 == theta1 && theta1 - theta0 < 1e-8 * (fabs(theta0) > 1.0 ? fabs(theta0) : 1.0))
               ? 1
               : 0;
}

// ---------------------------------------------------------------- sector
struct SpinTables {
    int32_t L, N, l_lo, l_hi;
    int64_t d;
    uint32_t *states;
    int32_t *rank_lo;  // [2^l_lo]
    int32_t *rank_hi;  // [(l_lo+1) * 2^l_hi]
};

__device__ __forceinline__ int32_t spin_rank(const int32_t *__restrict__ rlo,
                                             const int32_t *__restrict__ rhi, int l_lo, int l_hi,
                                             uint32_t b) {
    const uint32_t lo_mask = (l_lo >= 32) ? 0xffffffffu : ((1u << l_lo) - 1u);
    uint32_t lo = b & lo_mask;
    uint32_t hi = (l_lo >= 32) ? 0u : (b >> l_lo);
    return rlo[lo] + rhi[(size_t)__popc(lo) << l_hi | hi];
}

size_t spin_tables_bytes(int L, int N);
int build_spin_tables(int L, int N, Carver &cv, SpinTables *out, hipStream_t s);
int check_sector_args(int L, int nup, int ndn);
void basis_from_tables(const SpinTables &up, const SpinTables &dn, qcm_basis *out);
SpinTables spin_from_basis(const qcm_basis *b, int spin);

// ---------------------------------------------------------------- Hamiltonian tables
// Model data on the device and the per-spin hopping lists (ELL layout: slot-major,
// entry s of state i at [s * d + i]).
struct ModelDev {
    int32_t L;
    int32_t nbond;        // undirected bonds with t_ab != 0, a < b
    double *t;            // [L*L]
    int32_t *bond_a;      // [nbond]
    int32_t *bond_b;      // [nbond]
    double *bond_t;       // [nbond]
    double *ulut;         // [nbytes][256]: sum of U_k over set bits of one byte
    double *tlut;         // [nbytes][256]: sum of t_kk over set bits of one byte
    double *ctab;         // [2*nbond]: t_b, -t_b of bond b (hop coefficients by index)
    int32_t nbytes;       // ceil(L/8)
    double u_uniform;     // >= 0 if all U_k equal (then U * popcount), else -1
    int32_t t_is_uniform; // every bond has the same t_ab (then a hop coefficient is +-t)
    double t_uniform;     // that t_ab
};

struct HopTables {
    int64_t d;
    int32_t width;        // ELL width (max hops per state)
    int32_t rowmajor;     // 0: entry s of state i at [s * d + i]; 1: at [i * width + s]
    int32_t *nh;          // [d] number of hops of each state
    int32_t *col;         // [width * d]
    double *coef;         // [width * d]  sign * t_ab
    double *ediag;        // [d]  sum_k t_kk n_k
    uint32_t *pk = nullptr;  // [width * d] col | (ctab index << 16), slot-major; d < 65536
    int64_t *off = nullptr;  // row-major layout only: col * (length of the other spin)
};

size_t model_dev_bytes(int L);
int upload_model(const qcm_model *m, Carver &cv, ModelDev *md, hipStream_t s);
int validate_model(const qcm_model *m);
size_t hop_tables_bytes(const qcm_model *m, int64_t d);
int build_hop_tables(const ModelDev &md, const SpinTables &st, Carver &cv, HopTables *ht,
                     hipStream_t s, int nbond_host, int rowmajor = 0);

// ---------------------------------------------------------------- H.v
// The stored matrix of a symmetry-adapted sector (sym.hip): rows of H in CSR.
struct SymCsrDev {
    int64_t dim = 0;
    const int64_t *rowptr = nullptr;
    const uint32_t *col = nullptr;
    const double *val = nullptr;
    const uint32_t *pk = nullptr;    // col | value index << 26, or null
    const double *tab = nullptr;     // the distinct values when pk is set
};
int sym_hv_launch(const SymCsrDev &h, const double *v, double *w, int nvec, hipStream_t s);

struct HvOp {
    ModelDev md;
    SpinTables up, dn;
    HopTables hu, hd;
    int64_t dim;
    // two-pass path for long rows (see hv_split.hip); used when split != 0
    int split = 0;
    // in-row pass by 64-column tiles: the packed up hops (LDS offset | coefficient
    // index | sign) of tile t at tile_ent[tile_off[t] + (s / 4) * 256 + lane * 4
    // + s % 4], s < tile_nt[t] (the tile's largest hop count rounded up to 4,
    // padded with entries that read a zero slot)
    uint32_t *tile_ent = nullptr;
    // with one t for every bond, the FP32 form of the same entries: the
    // neighbour's LDS byte address in the row or in its negated copy
    uint32_t *tile_ent32 = nullptr;
    int32_t *tile_nt = nullptr, *tile_off = nullptr;
    int32_t tile_bytes = 0;       // bytes of tile_ent in use
    int32_t ntile = 0;
    HopTables hd_rm;              // down hops, row-major, with neighbour offsets
    int32_t *row_order = nullptr; // rows of V in the order the row-mixing pass takes them
    // a symmetry-adapted sector's stored matrix; used (FP64 only) when csr.rowptr != nullptr
    SymCsrDev csr;
};
// nvec vectors of length dim, consecutive (stride dim).  prec: QCM_FP64/QCM_FP32V.
int hv_launch(const HvOp &op, int prec, const void *v, void *w, int nvec, hipStream_t s);
size_t hv_scratch_bytes(const HvOp &op, int prec, int nvec);
int hv_setup_bytes(const qcm_model *m, const qcm_basis *b, size_t *need);
int hv_setup(const qcm_model *m, const qcm_basis *b, Carver &cv, HvOp *op, hipStream_t s);
// the two-pass path: whether it applies, its workspace, and its set-up
bool split_applies(const qcm_model *m, int n_up, int64_t d_up, int64_t d_dn);
int split_prepare(const qcm_model *m, HvOp &op, Carver &cv, hipStream_t s);
// The first pass of a Lanczos step fused into the two-pass product's row-mixing
// pass: w = H v - beta' vp (beta' = beta[c * maxs + n - 1] of chain c; none
// when n = 0) and, per row-mixing workgroup g (G = split_pa_count(op) of them
// per chain), the partial sums
//   pa[k * pstride + c * G + g] = <v, w>, <w, w>, <v, v> for k = 0, 1, 2,
// and with reorth also <vp, w>, <vp, v> at k = 3, 4; pstride = nvec * G.
// With them the step needs no separate norm pass: for x = w - alpha v,
// |x|^2 = <w,w> - 2 alpha <v,w> + alpha^2 <v,v>, <v, x> = <v,w> - alpha <v,v>,
// <vp, x> = <vp,w> - alpha <vp,v>.  <v, v> is measured, not taken as 1: the
// rounding of the normalisation would otherwise enter beta uncorrected and
// grow from step to step.
struct SubPrev {
    const void *vp = nullptr;
    const double *beta = nullptr;
    int maxs = 0, n = 0;
    double *pa = nullptr;
    int64_t pstride = 0;
    int reorth = 0;
};
// A Lanczos step whose previous update was deferred: the vector buffer v
// holds the unnormalised w_n of the previous step; the in-row pass forms
// v_{n+1} = (w_n - (a + c1) v_n - c2 v_{n-1}) * inv element by element, in
// the order and roundings of the separate update pass (x = w - a v, then
// - c1 v, - c2 v_{n-1} with reorthogonalisation, times inv, rounded once),
// stores it over w_n and uses it as the row.  Per chain: a = apre, c1 = corr,
// c2 = corr2, inv (0 for a stopped chain).  vpold is the buffer the product
// writes W into (read before the row's W is written).
struct LazyUpd {
    const void *vold = nullptr;    // v_n
    const void *vpold = nullptr;   // v_{n-1} (read with reorthogonalisation only)
    const double *apre = nullptr, *corr = nullptr, *corr2 = nullptr, *inv = nullptr;
    int reorth = 0;
};
int64_t split_pa_count(const HvOp &op);
int hv_split_launch_sub(const HvOp &op, int prec, void *v, void *w, int nvec, const SubPrev &sp,
                        const LazyUpd *lz, hipStream_t s);
int check_basis(const qcm_basis *b, int L);

// ---------------------------------------------------------------- misc
int count_bonds(const qcm_model *m);
inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace qcm

namespace qcm {

int build_row_offsets(HopTables &ht, int64_t d_up, Carver &cv, hipStream_t s);

}  // namespace qcm
