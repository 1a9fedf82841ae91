// Symmetry-adapted sectors of an abelian point group with real characters
// and the stored Hamiltonian in them (paper: subsection "Cluster
// symmetries", eq. (matrixElement)).
//
//  * k_sym_images: for every string of a spin and every group element, the
//    label of the permuted string and the reordering sign phi_g.
//  * k_sym_mark: one wave per 64 consecutive full-sector labels; a label is
//    kept when it is the smallest of its orbit and its projection survives
//    (sum of chi_g phi_g over its stabiliser > 0).  The wave's ballot is one
//    word of a bitmap; an exclusive prefix sum over the words' popcounts gives
//    the index of every kept representative in O(1): base[w] + popc of the
//    lower bits (this replaces the paper's binary search of the sorted list).
//  * k_sym_csr: one wave per representative (column).  Lane q takes hop
//    candidate q (bond, spin); a hop's target is mapped to its orbit's
//    representative, and the element c S / sqrt(m1 m2) is written into a
//    per-wave LDS list together with the diagonal.  Entries with the same
//    target are then summed in list order (the paper's cancellation step), sums
//    at or below the drop threshold are discarded, and the survivors are ranked
//    by column.  A first launch counts them per row, a second writes them.
//  * k_sym_spmv: w = H v over the stored rows, eight lanes per row, each
//    lane striding the row and the eight partial sums added by a fixed
//    butterfly.
#include <math.h>
#include <string.h>

#include <vector>

#include "lanczos_engine.h"
#include "qcm_internal.h"

namespace qcm {

constexpr int kSymG = QCM_SYM_MAX_G;
constexpr int kSymBonds = QCM_SYM_MAX_BONDS;
constexpr int kSymE = 2 * kSymBonds + 1;   // entries of one column before merging
constexpr int kCsrWaves = 4;               // columns per 256-thread workgroup
constexpr int kScanB = 1024;               // elements per prefix-sum block
constexpr int kSpmvLanes = 8;              // lanes per stored row (explicit elements)
constexpr int kPkLanes = 4;                // lanes per stored row (packed elements)
constexpr int kMaxVals = QCM_SYM_MAX_VALUES;
constexpr int kColBits = 26;               // packed element: column in the low 26 bits
constexpr uint32_t kColMask = (1u << kColBits) - 1u;
constexpr int kPackChunk = 16384;          // values per deduplicating workgroup
constexpr int kBlockSet = 256;             // its LDS hash set
constexpr int kMergeSet = 1024;            // the merging workgroup's set
constexpr unsigned long long kEmptyKey = ~0ull;   // a NaN pattern: never a stored value

struct SymPerm {
    int32_t n_g, L;
    int8_t p[kSymG][32];
};

struct SymSecDev {
    int64_t d_up, d_dn, dim;
    int32_t n_g, pad;
    int32_t chi[kSymG];
    int32_t l_lo_u, l_hi_u, l_lo_d, l_hi_d;
    const uint32_t *su, *sd;
    const int32_t *rlo_u, *rhi_u, *rlo_d, *rhi_d;
    const uint32_t *img_up, *img_dn;
    const uint64_t *bits;
    const int64_t *base;
};

struct SymModelDev {
    int32_t L, nbond;
    double drop;
    double tdiag[32], U[32];
    double bt[kSymBonds];
    int8_t ba[kSymBonds], bb[kSymBonds];
};

// ---------------------------------------------------------------- kernels

__global__ void __launch_bounds__(256)
    k_sym_images(const uint32_t *__restrict__ states, int64_t d, int l_lo, int l_hi,
                 const int32_t *__restrict__ rlo, const int32_t *__restrict__ rhi, SymPerm P,
                 uint32_t *__restrict__ img) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d * P.n_g) return;
    const int g = (int)(e / d);
    const int64_t k = e - (int64_t)g * d;
    const uint32_t s = states[k];
    uint64_t placed = 0;
    uint32_t out = 0;
    int inv = 0;
    // occupied orbitals in ascending order; each image is compared with the
    // images placed before it: the inversions of the permuted sequence
    for (int a = 0; a < P.L; ++a) {
        if (!((s >> a) & 1u)) continue;
        const int ga = P.p[g][a];
        inv += __popcll(placed >> ga);
        placed |= 1ull << ga;
        out |= 1u << ga;
    }
    const uint32_t lab = (uint32_t)spin_rank(rlo, rhi, l_lo, l_hi, out);
    img[e] = lab | ((uint32_t)(inv & 1) << 31);
}

__global__ void __launch_bounds__(256) k_sym_mark(SymSecDev S, int64_t full_dim, int64_t n_words,
                                                  uint64_t *__restrict__ bits,
                                                  int64_t *__restrict__ cnt) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n_words) return;   // whole waves only
    const int64_t i = w * 64 + lane;
    bool keep = false;
    if (i < full_dim) {
        const int64_t ku = i % S.d_up, kd = i / S.d_up;
        bool rep = true;
        int sum = 0;
        for (int g = 0; g < S.n_g; ++g) {
            const uint32_t a = S.img_up[(int64_t)g * S.d_up + ku];
            const uint32_t b = S.img_dn[(int64_t)g * S.d_dn + kd];
            const int64_t lab = (int64_t)(a & 0x7fffffffu) + S.d_up * (int64_t)(b & 0x7fffffffu);
            if (lab < i) rep = false;
            else if (lab == i) sum += ((a ^ b) >> 31) ? -S.chi[g] : S.chi[g];
        }
        keep = rep && sum > 0;
    }
    const uint64_t word = __ballot(keep);
    if (lane == 0) {
        bits[w] = word;
        cnt[w] = __popcll(word);
    }
}

// exclusive prefix sum within blocks of kScanB (in place allowed)
__global__ void __launch_bounds__(kScanB) k_scan_local(int64_t *__restrict__ x, int64_t n,
                                                      int64_t *__restrict__ bsum) {
    __shared__ int64_t sh[2][kScanB];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kScanB + t;
    const int64_t v = i < n ? x[i] : 0;
    sh[0][t] = v;
    __syncthreads();
    int src = 0;
    for (int off = 1; off < kScanB; off <<= 1) {
        const int64_t y = sh[src][t] + (t >= off ? sh[src][t - off] : 0);
        sh[src ^ 1][t] = y;
        src ^= 1;
        __syncthreads();
    }
    if (i < n) x[i] = sh[src][t] - v;
    if (t == kScanB - 1) bsum[blockIdx.x] = sh[src][t];
}

// exclusive prefix sum of the block sums in one workgroup, carried across chunks
__global__ void __launch_bounds__(kScanB) k_scan_tops(int64_t *__restrict__ bsum, int64_t nb) {
    __shared__ int64_t sh[2][kScanB];
    __shared__ int64_t carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += kScanB) {
        const int64_t i = c0 + t;
        const int64_t v = i < nb ? bsum[i] : 0;
        sh[0][t] = v;
        __syncthreads();
        int src = 0;
        for (int off = 1; off < kScanB; off <<= 1) {
            const int64_t y = sh[src][t] + (t >= off ? sh[src][t - off] : 0);
            sh[src ^ 1][t] = y;
            src ^= 1;
            __syncthreads();
        }
        const int64_t base = carry;
        if (i < nb) bsum[i] = base + sh[src][t] - v;
        __syncthreads();
        if (t == kScanB - 1) carry = base + sh[src][t];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanB) k_scan_add(int64_t *__restrict__ x, int64_t n,
                                                    const int64_t *__restrict__ bsum) {
    const int64_t i = (int64_t)blockIdx.x * kScanB + threadIdx.x;
    if (i < n) x[i] += bsum[blockIdx.x];
}

__global__ void k_set_i64(int64_t *p, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void __launch_bounds__(256) k_sym_reps(const uint64_t *__restrict__ bits,
                                                  const int64_t *__restrict__ base, int64_t n_words,
                                                  uint32_t *__restrict__ rep) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n_words) return;
    const uint64_t word = bits[w];
    const uint64_t bit = 1ull << lane;
    if (word & bit) rep[base[w] + __popcll(word & (bit - 1))] = (uint32_t)(w * 64 + lane);
}

__device__ __forceinline__ bool sym_index(uint64_t lab, const uint64_t *__restrict__ bits,
                                          const int64_t *__restrict__ base, int64_t *idx) {
    const uint64_t word = bits[lab >> 6];
    const uint64_t bit = 1ull << (lab & 63);
    if (!(word & bit)) return false;
    *idx = base[lab >> 6] + __popcll(word & (bit - 1));
    return true;
}

// FILL = false: rowptr[c] = number of stored elements of row c.
// FILL = true : col/val of row c at rowptr[c]...
template <bool FILL>
__global__ void __launch_bounds__(256)
    k_sym_csr(SymModelDev M, SymSecDev S, const uint32_t *__restrict__ rep,
              int64_t *__restrict__ rowptr, uint32_t *__restrict__ col_out,
              double *__restrict__ val_out) {
    __shared__ uint32_t key[kCsrWaves][kSymE];
    __shared__ double val[kCsrWaves][kSymE];
    __shared__ double sum[kCsrWaves][kSymE];
    __shared__ int8_t kept[kCsrWaves][kSymE];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * kCsrWaves + wv;
    const bool active = c < S.dim;   // inactive waves still pass the barriers
    uint32_t su = 0, sd = 0;
    int64_t ku = 0, kd = 0;
    int m1 = 1;
    if (active) {
        const uint32_t r1 = rep[c];
        ku = r1 % S.d_up;
        kd = r1 / S.d_up;
        su = S.su[ku];
        sd = S.sd[kd];
        bool fix = false;
        if (lane < S.n_g) {
            const uint32_t a = S.img_up[(int64_t)lane * S.d_up + ku];
            const uint32_t b = S.img_dn[(int64_t)lane * S.d_dn + kd];
            fix = (int64_t)(a & 0x7fffffffu) + S.d_up * (int64_t)(b & 0x7fffffffu) == (int64_t)r1;
        }
        m1 = __popcll(__ballot(fix));
        if (lane == 0) {
            double dg = 0.0;
            for (int a = 0; a < M.L; ++a) {
                const int nu = (su >> a) & 1u, nd = (sd >> a) & 1u;
                dg += M.tdiag[a] * (double)(nu + nd) + M.U[a] * (double)(nu * nd);
            }
            key[wv][0] = (uint32_t)c;
            val[wv][0] = dg;
        }
    }
    int ne = 1;
    const int ncand = 2 * M.nbond;
    for (int q0 = 0; q0 < ncand; q0 += 64) {
        const int q = q0 + lane;
        bool ok = false;
        uint32_t k2 = 0;
        double v2 = 0.0;
        if (active && q < ncand) {
            const int spin = q >= M.nbond;
            const int bd = q - spin * M.nbond;
            const int a = M.ba[bd], b = M.bb[bd];   // a < b
            const uint32_t s = spin ? sd : su;
            if (((s >> a) ^ (s >> b)) & 1u) {
                const uint32_t between = ((1u << b) - 1u) & ~((2u << a) - 1u);
                const double sign = (__popc(s & between) & 1) ? -1.0 : 1.0;
                const uint32_t s2 = s ^ ((1u << a) | (1u << b));
                int64_t ju = ku, jd = kd;
                if (spin)
                    jd = spin_rank(S.rlo_d, S.rhi_d, S.l_lo_d, S.l_hi_d, s2);
                else
                    ju = spin_rank(S.rlo_u, S.rhi_u, S.l_lo_u, S.l_hi_u, s2);
                int64_t best = INT64_MAX;
                int m2 = 0, sc = 0;
                for (int g = 0; g < S.n_g; ++g) {
                    const uint32_t ia = S.img_up[(int64_t)g * S.d_up + ju];
                    const uint32_t ib = S.img_dn[(int64_t)g * S.d_dn + jd];
                    const int64_t lab =
                        (int64_t)(ia & 0x7fffffffu) + S.d_up * (int64_t)(ib & 0x7fffffffu);
                    const int ch = ((ia ^ ib) >> 31) ? -S.chi[g] : S.chi[g];
                    if (lab < best) {
                        best = lab;
                        m2 = 1;
                        sc = ch;
                    } else if (lab == best) {
                        ++m2;
                        sc += ch;
                    }
                }
                int64_t idx = 0;
                if (sc != 0 && sym_index((uint64_t)best, S.bits, S.base, &idx)) {
                    ok = true;
                    k2 = (uint32_t)idx;
                    v2 = M.bt[bd] * sign * (double)sc / sqrt((double)(m1 * m2));
                }
            }
        }
        const uint64_t bal = __ballot(ok);
        if (ok) {
            const int pos = ne + __popcll(bal & ((1ull << lane) - 1ull));
            key[wv][pos] = k2;
            val[wv][pos] = v2;
        }
        ne += __popcll(bal);
    }
    __syncthreads();
    // merge entries with the same column, in list order
    if (active) {
        for (int e = lane; e < ne; e += 64) {
            const uint32_t k = key[wv][e];
            bool first = true;
            for (int f = 0; f < e; ++f)
                if (key[wv][f] == k) {
                    first = false;
                    break;
                }
            double x = 0.0;
            if (first)
                for (int f = e; f < ne; ++f)
                    if (key[wv][f] == k) x += val[wv][f];
            sum[wv][e] = x;
            kept[wv][e] = first && fabs(x) > M.drop;
        }
    }
    __syncthreads();
    if (active) {
        int count = 0;
        for (int e = lane; e < ne; e += 64) {
            if (!kept[wv][e]) continue;
            ++count;
            if (FILL) {
                const uint32_t k = key[wv][e];
                int pos = 0;
                for (int f = 0; f < ne; ++f) pos += kept[wv][f] && key[wv][f] < k;
                const int64_t o = rowptr[c] + pos;
                col_out[o] = k;
                val_out[o] = sum[wv][e];
            }
        }
        if (!FILL) {
            for (int off = 32; off > 0; off >>= 1) count += __shfl_xor(count, off);
            if (lane == 0) rowptr[c] = count;
        }
    }
}

__global__ void __launch_bounds__(256)
    k_sym_spmv(const int64_t *__restrict__ rowptr, const uint32_t *__restrict__ col,
               const double *__restrict__ val, int64_t dim, const double *__restrict__ v,
               double *__restrict__ w) {
    const int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kSpmvLanes;
    const int sub = threadIdx.x & (kSpmvLanes - 1);
    const int64_t off = (int64_t)blockIdx.y * dim;
    double acc = 0.0;
    if (r < dim) {
        const int64_t e = rowptr[r + 1];
        for (int64_t k = rowptr[r] + sub; k < e; k += kSpmvLanes)
            acc = fma(val[k], v[off + col[k]], acc);
    }
    for (int m = kSpmvLanes / 2; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
    if (sub == 0 && r < dim) w[off + r] = acc;
}

// w = H v from the packed elements (kPkLanes lanes per row: with 4-byte
// elements, more rows per wave in flight pay more than longer row segments)
__global__ void __launch_bounds__(256)
    k_sym_spmv_pk(const int64_t *__restrict__ rowptr, const uint32_t *__restrict__ pk,
                  const double *__restrict__ table, int64_t dim, const double *__restrict__ v,
                  double *__restrict__ w) {
    __shared__ double tab[kMaxVals];
    if (threadIdx.x < kMaxVals) tab[threadIdx.x] = table[threadIdx.x];
    __syncthreads();
    const int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kPkLanes;
    const int sub = threadIdx.x & (kPkLanes - 1);
    const int64_t off = (int64_t)blockIdx.y * dim;
    double acc = 0.0;
    if (r < dim) {
        const int64_t e = rowptr[r + 1];
        for (int64_t k = rowptr[r] + sub; k < e; k += kPkLanes) {
            const uint32_t x = pk[k];
            acc = fma(tab[x >> kColBits], v[off + (x & kColMask)], acc);
        }
    }
    for (int m = kPkLanes / 2; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
    if (sub == 0 && r < dim) w[off + r] = acc;
}

__device__ __forceinline__ uint32_t mix64(unsigned long long x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    return (uint32_t)x;
}

// Insert a 64-bit key into an LDS open-addressing set of cap (a power of two)
// slots; false when the set is full.
__device__ bool lds_set_insert(unsigned long long *set, int cap, unsigned long long key) {
    uint32_t h = mix64(key) & (uint32_t)(cap - 1);
    for (int probe = 0; probe < cap; ++probe) {
        const unsigned long long cur = set[h];
        if (cur == key) return true;
        if (cur == kEmptyKey) {
            const unsigned long long old = atomicCAS(&set[h], kEmptyKey, key);
            if (old == kEmptyKey || old == key) return true;
        }
        h = (h + 1) & (uint32_t)(cap - 1);
    }
    return false;
}

// The distinct values of one chunk of kPackChunk stored values, into the
// chunk's own segment of kMaxVals slots; flag when there are more.
__global__ void __launch_bounds__(256)
    k_sym_vals_block(const double *__restrict__ val, int64_t nnz, unsigned long long *__restrict__ seg,
                     int32_t *__restrict__ segn, int32_t *__restrict__ overflow) {
    __shared__ unsigned long long set[kBlockSet];
    __shared__ int full;
    const int t = threadIdx.x;
    for (int e = t; e < kBlockSet; e += blockDim.x) set[e] = kEmptyKey;
    if (t == 0) full = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kPackChunk;
    const int64_t end = base + kPackChunk < nnz ? base + kPackChunk : nnz;
    for (int64_t i = base + t; i < end; i += blockDim.x)
        if (!lds_set_insert(set, kBlockSet, (unsigned long long)__double_as_longlong(val[i]))) full = 1;
    __syncthreads();
    if (t == 0) {
        int n = 0;
        for (int e = 0; e < kBlockSet; ++e)
            if (set[e] != kEmptyKey) {
                if (n < kMaxVals) seg[(int64_t)blockIdx.x * kMaxVals + n] = set[e];
                ++n;
            }
        segn[blockIdx.x] = n < kMaxVals ? n : kMaxVals;
        if (n > kMaxVals || full) overflow[0] = 1;
    }
}

// Merge the segments in one workgroup; the table is the distinct values in
// ascending order (each value's index is its rank).
__global__ void __launch_bounds__(1024)
    k_sym_vals_merge(const unsigned long long *__restrict__ seg, const int32_t *__restrict__ segn,
                     int64_t nb, double *__restrict__ table, int32_t *__restrict__ nvals,
                     int32_t *__restrict__ overflow) {
    __shared__ unsigned long long set[kMergeSet];
    __shared__ unsigned long long vals[kMaxVals];
    __shared__ int full, m;
    const int t = threadIdx.x;
    for (int e = t; e < kMergeSet; e += blockDim.x) set[e] = kEmptyKey;
    if (t == 0) {
        full = 0;
        m = 0;
    }
    __syncthreads();
    for (int64_t e = t; e < nb * kMaxVals; e += blockDim.x) {
        const int64_t b = e / kMaxVals;
        const int j = (int)(e % kMaxVals);
        if (j < segn[b] && !lds_set_insert(set, kMergeSet, seg[e])) full = 1;
    }
    __syncthreads();
    if (t == 0) {
        int n = 0;
        for (int e = 0; e < kMergeSet; ++e)
            if (set[e] != kEmptyKey) {
                if (n < kMaxVals) vals[n] = set[e];
                ++n;
            }
        m = n;
        if (n > kMaxVals || full) overflow[0] = 1;
    }
    __syncthreads();
    const int n = m < kMaxVals ? m : kMaxVals;
    if (t < n) {
        const double x = __longlong_as_double((long long)vals[t]);
        int rank = 0;
        for (int j = 0; j < n; ++j) rank += __longlong_as_double((long long)vals[j]) < x;
        table[rank] = x;
    }
    if (t == 0) nvals[0] = m;
}

__global__ void __launch_bounds__(256)
    k_sym_pack(const uint32_t *__restrict__ col, const double *__restrict__ val, int64_t nnz,
               const double *__restrict__ table, int n, uint32_t *__restrict__ pk) {
    __shared__ double tab[kMaxVals];
    if (threadIdx.x < n) tab[threadIdx.x] = table[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnz) return;
    const double x = val[i];
    int lo = 0, hi = n - 1;   // x is in the table
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tab[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    pk[i] = col[i] | ((uint32_t)lo << kColBits);
}

// ---------------------------------------------------------------- host

static int scan_exclusive(int64_t *x, int64_t n, int64_t *bsum, hipStream_t s) {
    if (n <= 0) return QCM_OK;
    const int64_t nb = (int64_t)ceil_div((size_t)n, kScanB);
    k_scan_local<<<(unsigned)nb, kScanB, 0, s>>>(x, n, bsum);
    k_scan_tops<<<1, kScanB, 0, s>>>(bsum, nb);
    k_scan_add<<<(unsigned)nb, kScanB, 0, s>>>(x, n, bsum);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

static SymSecDev sec_dev(const qcm_sym_sector *s) {
    SymSecDev d;
    memset(&d, 0, sizeof d);
    d.d_up = s->b.d_up;
    d.d_dn = s->b.d_dn;
    d.dim = s->dim;
    d.n_g = s->n_g;
    for (int g = 0; g < kSymG; ++g) d.chi[g] = g < s->n_g ? s->chi[g] : 0;
    d.l_lo_u = d.l_lo_d = s->b.l_lo;
    d.l_hi_u = d.l_hi_d = s->b.l_hi;
    d.su = s->b.states_up;
    d.sd = s->b.states_dn;
    d.rlo_u = s->b.rank_lo_up;
    d.rhi_u = s->b.rank_hi_up;
    d.rlo_d = s->b.rank_lo_dn;
    d.rhi_d = s->b.rank_hi_dn;
    d.img_up = s->img_up;
    d.img_dn = s->img_dn;
    d.bits = s->bits;
    d.base = s->base;
    return d;
}

static int check_group(const qcm_group *g, int L) {
    if (!g || !g->perm || !g->chi) return fail(QCM_EARG, "group, perm or chi is NULL");
    const int n = g->n_g;
    if (n < 1 || n > kSymG) return fail(QCM_EARG, "group order %d outside 1..%d", n, kSymG);
    for (int e = 0; e < n; ++e) {
        if (g->chi[e] != 1 && g->chi[e] != -1)
            return fail(QCM_EARG, "character %d of element %d is not +-1", g->chi[e], e);
        std::vector<int> seen(L, 0);
        for (int a = 0; a < L; ++a) {
            const int p = g->perm[e * L + a];
            if (p < 0 || p >= L || seen[p]++)
                return fail(QCM_EARG, "element %d is not a permutation of %d orbitals", e, L);
            if (e == 0 && p != a) return fail(QCM_EARG, "element 0 is not the identity");
        }
    }
    for (int e = 1; e < n; ++e)
        for (int f = 0; f < e; ++f) {
            bool same = true;
            for (int a = 0; a < L && same; ++a) same = g->perm[e * L + a] == g->perm[f * L + a];
            if (same) return fail(QCM_EARG, "elements %d and %d are equal", f, e);
        }
    // closure and chi(gh) = chi(g) chi(h), with (gh)(a) = g(h(a))
    std::vector<int> comp(L);
    for (int e = 0; e < n; ++e)
        for (int f = 0; f < n; ++f) {
            for (int a = 0; a < L; ++a) comp[a] = g->perm[e * L + g->perm[f * L + a]];
            int found = -1;
            for (int h = 0; h < n && found < 0; ++h) {
                bool same = true;
                for (int a = 0; a < L && same; ++a) same = g->perm[h * L + a] == comp[a];
                if (same) found = h;
            }
            if (found < 0) return fail(QCM_EARG, "the elements are not closed under composition");
            if (g->chi[found] != g->chi[e] * g->chi[f])
                return fail(QCM_EARG, "chi is not a representation (elements %d, %d)", e, f);
        }
    return QCM_OK;
}

static int model_args(const qcm_model *m, const qcm_sym_sector *s, SymModelDev *out) {
    QCM_TRY(validate_model(m));
    if (!s) return fail(QCM_EARG, "sector is NULL");
    const int L = m->L;
    if (s->b.L != L) return fail(QCM_EARG, "model L=%d but sector L=%d", L, s->b.L);
    if (!s->bits || !s->base || !s->img_up || !s->img_dn)
        return fail(QCM_EARG, "sector has no device tables");
    for (int g = 0; g < s->n_g; ++g)
        for (int a = 0; a < L; ++a) {
            const int ga = s->perm[g * 32 + a];
            if (m->U[ga] != m->U[a])
                return fail(QCM_EARG, "U is not invariant under element %d (orbital %d)", g, a);
            for (int b = 0; b < L; ++b)
                if (m->t[ga * L + s->perm[g * 32 + b]] != m->t[a * L + b])
                    return fail(QCM_EARG, "t is not invariant under element %d at (%d,%d)", g, a, b);
        }
    SymModelDev &d = *out;
    memset(&d, 0, sizeof d);
    d.L = L;
    double tmax = 0.0;
    for (int a = 0; a < L; ++a) {
        d.tdiag[a] = m->t[a * L + a];
        d.U[a] = m->U[a];
        tmax = fmax(tmax, fabs(m->U[a]));
        for (int b = 0; b < L; ++b) tmax = fmax(tmax, fabs(m->t[a * L + b]));
    }
    int nb = 0;
    for (int a = 0; a < L; ++a)
        for (int b = a + 1; b < L; ++b)
            if (m->t[a * L + b] != 0.0) {
                if (nb == kSymBonds)
                    return fail(QCM_EARG, "more than %d bonds (pairs a < b with t_ab != 0)",
                                kSymBonds);
                d.ba[nb] = (int8_t)a;
                d.bb[nb] = (int8_t)b;
                d.bt[nb] = m->t[a * L + b];
                ++nb;
            }
    d.nbond = nb;
    d.drop = 1e-13 * (tmax > 0.0 ? tmax : 1e-300);
    return QCM_OK;
}

int sym_hv_launch(const SymCsrDev &h, const double *v, double *w, int nvec, hipStream_t s) {
    if (h.dim == 0 || nvec == 0) return QCM_OK;
    if (h.pk) {
        const dim3 grid((unsigned)ceil_div((size_t)h.dim * kPkLanes, 256), (unsigned)nvec);
        k_sym_spmv_pk<<<grid, 256, 0, s>>>(h.rowptr, h.pk, h.tab, h.dim, v, w);
    } else {
        const dim3 grid((unsigned)ceil_div((size_t)h.dim * kSpmvLanes, 256), (unsigned)nvec);
        k_sym_spmv<<<grid, 256, 0, s>>>(h.rowptr, h.col, h.val, h.dim, v, w);
    }
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

}  // namespace qcm

using namespace qcm;

extern "C" int qcm_sym_sector_build(const qcm_basis *b, const qcm_group *g, void *d_ws,
                                    size_t ws_bytes, size_t *ws_needed, qcm_sym_sector *out,
                                    void *stream) {
    if (!ws_needed || !b || !out) return fail(QCM_EARG, "qcm_sym_sector_build: NULL argument");
    if (b->L < 1 || b->L > 32) return fail(QCM_ERANGE, "qcm_sym_sector_build: L=%d", b->L);
    QCM_TRY(check_basis(b, b->L));
    if (b->dim < 1 || b->dim >= ((int64_t)1 << 32))
        return fail(QCM_EARG, "qcm_sym_sector_build: sector dimension %lld outside 1..2^32-1",
                    (long long)b->dim);
    QCM_TRY(check_group(g, b->L));
    const int n = g->n_g;
    const int64_t n_words = (int64_t)ceil_div((size_t)b->dim, 64);
    auto layout = [&](Carver &cv, qcm_sym_sector *o, int64_t **bsum) {
        o->img_up = cv.take<uint32_t>((size_t)n * b->d_up);
        o->img_dn = cv.take<uint32_t>((size_t)n * b->d_dn);
        o->bits = cv.take<uint64_t>((size_t)n_words);
        o->base = cv.take<int64_t>((size_t)n_words + 1);
        *bsum = cv.take<int64_t>(ceil_div((size_t)n_words + 1, kScanB) + 1);
    };
    qcm_sym_sector o;
    memset(&o, 0, sizeof o);
    int64_t *bsum = nullptr;
    Carver dry(nullptr);
    layout(dry, &o, &bsum);
    const size_t need = dry.off + 256;
    *ws_needed = need;
    o.b = *b;
    o.n_g = n;
    for (int e = 0; e < n; ++e) {
        o.chi[e] = g->chi[e];
        for (int a = 0; a < b->L; ++a) o.perm[e * 32 + a] = (int8_t)g->perm[e * b->L + a];
    }
    o.n_words = n_words;
    if (!d_ws) {
        *out = o;
        return QCM_OK;
    }
    if (ws_bytes < need)
        return fail(QCM_EWORKSPACE, "qcm_sym_sector_build: workspace %zu < %zu", ws_bytes, need);
    hipStream_t s = as_stream(stream);
    Carver cv(d_ws);
    layout(cv, &o, &bsum);
    SymPerm P;
    memset(&P, 0, sizeof P);
    P.n_g = n;
    P.L = b->L;
    for (int e = 0; e < n; ++e)
        for (int a = 0; a < b->L; ++a) P.p[e][a] = (int8_t)g->perm[e * b->L + a];
    k_sym_images<<<(unsigned)ceil_div((size_t)n * b->d_up, 256), 256, 0, s>>>(
        b->states_up, b->d_up, b->l_lo, b->l_hi, b->rank_lo_up, b->rank_hi_up, P,
        (uint32_t *)o.img_up);
    k_sym_images<<<(unsigned)ceil_div((size_t)n * b->d_dn, 256), 256, 0, s>>>(
        b->states_dn, b->d_dn, b->l_lo, b->l_hi, b->rank_lo_dn, b->rank_hi_dn, P,
        (uint32_t *)o.img_dn);
    QCM_LAUNCH_CHECK();
    o.dim = 0;
    SymSecDev sd = sec_dev(&o);
    int64_t *base = (int64_t *)o.base;
    k_sym_mark<<<(unsigned)ceil_div((size_t)n_words, 4), 256, 0, s>>>(sd, b->dim, n_words,
                                                                      (uint64_t *)o.bits, base);
    k_set_i64<<<1, 64, 0, s>>>(base + n_words, 0);
    QCM_LAUNCH_CHECK();
    QCM_TRY(scan_exclusive(base, n_words + 1, bsum, s));
    int64_t dim = 0;
    QCM_HIP(hipMemcpyAsync(&dim, base + n_words, sizeof dim, hipMemcpyDeviceToHost, s));
    QCM_HIP(hipStreamSynchronize(s));
    o.dim = dim;
    *out = o;
    return QCM_OK;
}

extern "C" int qcm_sym_csr_count(const qcm_model *m, const qcm_sym_sector *s, uint32_t *d_rep,
                                 int64_t *d_rowptr, int64_t *h_nnz, void *d_ws, size_t ws_bytes,
                                 size_t *ws_needed, void *stream) {
    if (!ws_needed) return fail(QCM_EARG, "qcm_sym_csr_count: ws_needed is NULL");
    SymModelDev md;
    QCM_TRY(model_args(m, s, &md));
    const size_t need = sizeof(int64_t) * (ceil_div((size_t)s->dim + 1, kScanB) + 1) + 256;
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (ws_bytes < need)
        return fail(QCM_EWORKSPACE, "qcm_sym_csr_count: workspace %zu < %zu", ws_bytes, need);
    if (!d_rep || !d_rowptr || !h_nnz) return fail(QCM_EARG, "qcm_sym_csr_count: NULL output");
    hipStream_t st = as_stream(stream);
    if (s->dim > 0) {
        k_sym_reps<<<(unsigned)ceil_div((size_t)s->n_words, 4), 256, 0, st>>>(s->bits, s->base,
                                                                            s->n_words, d_rep);
        const SymSecDev sd = sec_dev(s);
        k_sym_csr<false><<<(unsigned)ceil_div((size_t)s->dim, kCsrWaves), 256, 0, st>>>(
            md, sd, d_rep, d_rowptr, nullptr, nullptr);
    }
    k_set_i64<<<1, 64, 0, st>>>(d_rowptr + s->dim, 0);
    QCM_LAUNCH_CHECK();
    QCM_TRY(scan_exclusive(d_rowptr, s->dim + 1, (int64_t *)d_ws, st));
    QCM_HIP(hipMemcpyAsync(h_nnz, d_rowptr + s->dim, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    QCM_HIP(hipStreamSynchronize(st));
    return QCM_OK;
}

extern "C" int qcm_sym_csr_fill(const qcm_model *m, const qcm_sym_sector *s, const uint32_t *d_rep,
                                const int64_t *d_rowptr, uint32_t *d_col, double *d_val,
                                void *stream) {
    SymModelDev md;
    QCM_TRY(model_args(m, s, &md));
    if (!d_rep || !d_rowptr || !d_col || !d_val) return fail(QCM_EARG, "qcm_sym_csr_fill: NULL pointer");
    if (s->dim == 0) return QCM_OK;
    const SymSecDev sd = sec_dev(s);
    k_sym_csr<true><<<(unsigned)ceil_div((size_t)s->dim, kCsrWaves), 256, 0, as_stream(stream)>>>(
        md, sd, d_rep, (int64_t *)d_rowptr, d_col, d_val);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

static int check_csr(const qcm_sym_csr *h, const char *fn) {
    if (!h) return fail(QCM_EARG, "%s: matrix is NULL", fn);
    if (h->dim < 0 || h->dim >= ((int64_t)1 << 32) || h->nnz < 0)
        return fail(QCM_EARG, "%s: bad sizes", fn);
    if (h->packed) {
        if (!h->table) return fail(QCM_EARG, "%s: packed elements without their table", fn);
        if (h->dim > ((int64_t)1 << kColBits))
            return fail(QCM_EARG, "%s: packed elements need dim <= 2^%d", fn, kColBits);
        if (h->dim > 0 && !h->rowptr) return fail(QCM_EARG, "%s: NULL row pointers", fn);
        return QCM_OK;
    }
    if (h->dim > 0 && (!h->rowptr || (h->nnz > 0 && (!h->col || !h->val))))
        return fail(QCM_EARG, "%s: NULL matrix array", fn);
    return QCM_OK;
}

static SymCsrDev csr_dev(const qcm_sym_csr *h) {
    SymCsrDev d;
    d.dim = h->dim;
    d.rowptr = h->rowptr;
    d.col = h->col;
    d.val = h->val;
    d.pk = h->packed;
    d.tab = h->table;
    return d;
}

extern "C" int qcm_sym_csr_pack(const qcm_sym_csr *h, uint32_t *d_packed, double *d_table,
                                int32_t *h_n_values, void *d_ws, size_t ws_bytes, size_t *ws_needed,
                                void *stream) {
    const char *who = "qcm_sym_csr_pack";
    if (!ws_needed) return fail(QCM_EARG, "%s: ws_needed is NULL", who);
    QCM_TRY(check_csr(h, who));
    if (h->nnz > 0 && (!h->col || !h->val))
        return fail(QCM_EARG, "%s: packing needs the explicit columns and values", who);
    const int64_t nb = h->nnz > 0 ? (int64_t)ceil_div((size_t)h->nnz, kPackChunk) : 0;
    struct {
        unsigned long long *seg;
        int32_t *segn, *flags;
        double *tab;
    } P;
    auto layout = [&](Carver &cv) {
        P.seg = cv.take<unsigned long long>((size_t)(nb > 0 ? nb : 1) * kMaxVals);
        P.segn = cv.take<int32_t>(nb > 0 ? nb : 1);
        P.flags = cv.take<int32_t>(2);
        P.tab = cv.take<double>(kMaxVals);
    };
    Carver dry(nullptr);
    layout(dry);
    const size_t need = dry.off + 256;
    *ws_needed = need;
    if (!d_ws) return QCM_OK;
    if (ws_bytes < need) return fail(QCM_EWORKSPACE, "%s: workspace %zu < %zu", who, ws_bytes, need);
    if (!h_n_values || !d_packed || !d_table) return fail(QCM_EARG, "%s: NULL output", who);
    *h_n_values = 0;
    if (h->nnz == 0 || h->dim > ((int64_t)1 << kColBits)) return QCM_OK;
    hipStream_t s = as_stream(stream);
    Carver cv(d_ws);
    layout(cv);
    QCM_HIP(hipMemsetAsync(P.flags, 0, 2 * sizeof(int32_t), s));
    k_sym_vals_block<<<(unsigned)nb, 256, 0, s>>>(h->val, h->nnz, P.seg, P.segn, P.flags);
    k_sym_vals_merge<<<1, 1024, 0, s>>>(P.seg, P.segn, nb, P.tab, P.flags + 1, P.flags);
    QCM_LAUNCH_CHECK();
    int32_t fl[2] = {0, 0};
    QCM_HIP(hipMemcpyAsync(fl, P.flags, sizeof fl, hipMemcpyDeviceToHost, s));
    QCM_HIP(hipStreamSynchronize(s));
    if (fl[0] || fl[1] < 1 || fl[1] > kMaxVals) return QCM_OK;   // does not fit the format
    QCM_HIP(hipMemcpyAsync(d_table, P.tab, sizeof(double) * fl[1], hipMemcpyDeviceToDevice, s));
    k_sym_pack<<<(unsigned)ceil_div((size_t)h->nnz, 256), 256, 0, s>>>(h->col, h->val, h->nnz, P.tab,
                                                                     fl[1], d_packed);
    QCM_LAUNCH_CHECK();
    QCM_HIP(hipStreamSynchronize(s));
    *h_n_values = fl[1];
    return QCM_OK;
}

extern "C" int qcm_sym_hv(const qcm_sym_csr *h, const double *d_v, double *d_w, int32_t nvec,
                          void *stream) {
    QCM_TRY(check_csr(h, "qcm_sym_hv"));
    if (nvec < 1) return fail(QCM_EARG, "qcm_sym_hv: nvec %d < 1", nvec);
    if (!d_v || !d_w) return fail(QCM_EARG, "qcm_sym_hv: NULL vector");
    const size_t bytes = sizeof(double) * (size_t)h->dim * (size_t)nvec;
    const char *v = (const char *)d_v, *w = (const char *)d_w;
    if (h->dim > 0 && v < w + bytes && w < v + bytes)
        return fail(QCM_EARG, "qcm_sym_hv: v and w overlap");
    return sym_hv_launch(csr_dev(h), d_v, d_w, nvec, as_stream(stream));
}

extern "C" int qcm_sym_lanczos_gs(const qcm_sym_csr *h, const qcm_lanczos_opts *o,
                                  double *h_alpha, double *h_beta, void *d_gs,
                                  qcm_gs_result *h_out, void *d_ws, size_t ws_bytes,
                                  size_t *ws_needed, void *stream) {
    QCM_TRY(check_csr(h, "qcm_sym_lanczos_gs"));
    if (o && o->prec != QCM_FP64)
        return fail(QCM_EARG, "qcm_sym_lanczos_gs: the stored matrix runs in FP64 only");
    auto setup = [&](Carver &, hipStream_t, HvOp *op) -> int {
        op->dim = h->dim;
        op->up.d = h->dim;
        op->dn.d = 1;
        op->csr = csr_dev(h);
        return QCM_OK;
    };
    return gs_run("qcm_sym_lanczos_gs", setup, h->dim, o, h_alpha, h_beta, d_gs, h_out, d_ws,
                  ws_bytes, ws_needed, stream);
}
