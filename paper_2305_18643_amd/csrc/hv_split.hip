// H.v in two streaming passes for sectors whose rows are long (4096 to 16384
// up strings: the 4x4 half-filled sector has 12,870), paper: section "Exact
// diagonalizations", eq. (factorized) H = K_up (x) 1 + 1 (x) K_dn + V_int.
//
// With the vector as the row-major matrix V[i_dn][i_up]:
//   pass A (inside rows, K_up, and the diagonal):  W = V K_up^T + D o V
//     Persistent workgroups stage one whole row in LDS and gather the
//     neighbour values from it.  The hops of an up string are the same for
//     every row: they come from a table of 64-string tiles read through the
//     caches (1.6 MB for the 4x4 sector, resident in each XCD's L2), with the
//     LDS byte offset of the neighbour, its coefficient index and its sign in
//     one 32-bit word; a wave takes one tile at a time with a wave-uniform
//     hop count.
//   pass B (row mixing, K_dn):  W += K_dn V
//     The columns are cut into slabs; all rows of one slab are produced by the
//     workgroups of one XCD, so most neighbour segments a slab needs (about
//     13 per row) come from that XCD's L2.
// Every sum is FP64 in registers; W is rounded once per pass to the storage
// type (FP64: the same value as one rounding of the FP64 sum of pass A plus
// the row-mixing terms; FP32 vectors: two roundings).
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "lanczos_device.h"
#include "qcm_internal.h"

namespace qcm {

// Largest row length of the two-pass path: an LDS byte offset col * 8 (and
// the zero slot's 8 d_up) must fit the 17 bits the in-row entry gives it.
constexpr int64_t kSplitMaxUp = 16384;
constexpr int64_t kSplitMinUp = 4096;

// ---------------------------------------------------------------- kernels

// In-row entry of a hop, from the hopping list's packed form (column |
// coefficient index << 16):
//   bits 0..16  LDS byte offset of the neighbour in an FP64 row (col * 8)
//   bits 17..30 index of +-t_ab in the model's coefficient table
//   bit  31     sign of the coefficient (the index's parity)
// A padding entry holds the offset 8 d_up (the zero slot after the row) and
// index 0.  Slot s of lane l is entry (s / 4) 256 + 4 l + s % 4 from the
// tile's start: a lane's four consecutive slots are adjacent, one 16-byte
// load.  Block = tile of 64 up strings, thread = lane.
// out32 (or null): the FP32 entries of a model whose bonds all have the same
// t, in the same places: the neighbour's LDS byte address itself, in the row
// (col * 4) for a + sign and in the negated copy of the row (neg + col * 4)
// for a - sign; padding: the zero slot (4 d).
__global__ void k_pack_tiles(int64_t d, const int32_t *__restrict__ nh,
                             const uint32_t *__restrict__ pk, const int32_t *__restrict__ tnt,
                             const int32_t *__restrict__ toff, uint32_t *__restrict__ out,
                             uint32_t *__restrict__ out32, const uint32_t neg) {
    const int tt = blockIdx.x, lane = threadIdx.x;
    const int64_t i = (int64_t)tt * 64 + lane;
    const int n = i < d ? nh[i] : 0;
    const uint32_t pad = (uint32_t)(8 * d);
    for (int s = 0; s < tnt[tt]; ++s) {
        uint32_t e = pad, e32 = (uint32_t)(4 * d);
        if (s < n) {
            const uint32_t p = pk[(int64_t)s * d + i], col = p & 0xffffu, idx = p >> 16;
            e = (col << 3) | (idx << 17) | ((idx & 1u) << 31);
            e32 = (col << 2) + ((idx & 1u) ? neg : 0u);
        }
        const int64_t at = toff[tt] + (s >> 2) * 256 + lane * 4 + (s & 3);
        out[at] = e;
        if (out32) out32[at] = e32;
    }
}

// Byte address of the negated copy of an FP32 row in the in-row pass's LDS:
// after the row and its 64-byte zero slot.
__host__ __device__ inline uint32_t neg_row_at(int64_t d_up) {
    return (uint32_t)((4 * d_up + 64 + 15) & ~(int64_t)15);
}

// Pass A: one row of V in LDS at a time (persistent grid, one 1024-thread
// workgroup per CU, the next row prefetched in registers).  A wave takes one
// tile of 64 up strings at a time: the tile's hop count is wave-uniform and
// its entries are tile-major, so every lane runs the same hop loop with no
// masking and the entry loads are one contiguous 1 KB load per four slots
// from a wave-uniform base (2.57 -> 2.55 ms for the 4x4 H.v against one
// 256-byte load per slot); slots past a lane's own hops read the zero slot.
// The wave index is a scalar, so the tile loop, the tile's slot count and
// table offset are scalar work (2.55 -> 2.44 ms against two vector loads
// waited for in turn per tile), and the up-string bits, the up diagonal, the
// table and W go through buffer descriptors (lane offset register, scalar
// tile offset).  Eight entries are loaded, then eight neighbours gathered
// from LDS, then summed; a tile's slot count is its largest hop count
// rounded up to four, the last four taken as a group of their own (4x4
// sector: 19.0 slots per string instead of 21.4 with counts rounded up to
// eight; H.v 2.63 -> 2.60 ms in FP64, 2.60 -> 2.54 ms in FP32).  Ordering
// each tile span's strings by hop count (15-17 slots) was measured slower:
// their products are then stored scattered over the span, which costs more
// than the slots it saves.  The row sits at LDS address 0, so the masked
// entry is the gather address (halved for FP32 rows).  When every bond has
// the same t (UT), a coefficient is +-t: the entry's sign bit flips the sign
// of the neighbour value and the coefficient table is not read (FP32 rows:
// the negated copy below instead).  W = V K_up^T + D o V, written once; the
// per-element sum is the diagonal term, then the hops in list order.
// LZ > 0 (a Lanczos step after a deferred update, LazyUpd): v holds w_n; the
// prefetch of the next row also loads v_n (and v_{n-1} for LZ = 2, with
// reorthogonalisation); when the row is staged, v_{n+1} is formed and put in
// LDS, and after the row's hop loop it is stored back over w_n.
constexpr int kTileChunk = 8;
constexpr int kInrowThreads = 1024;

// Rows are loaded and stored through a buffer descriptor over the row: one
// lane offset register and a scalar offset per slot (the slot's offsets need
// no registers of their own), and the hardware's range check returns 0 for
// loads past the row and drops stores past it.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const T *row, int64_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(row), (short)0,
                                             (int)(n * (int64_t)sizeof(T)), 0x00020000);
}
template <typename T>
__device__ __forceinline__ T row_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 2));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 2));
}
template <typename T>
__device__ __forceinline__ void row_store(T x, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, x), r, voff, soff, 2);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, voff, soff, 2);
}

template <typename T, int KS, bool UT, int LZ>
__global__ void __launch_bounds__(kInrowThreads) k_hv_inrow_tile(
    const int64_t d_up, const int64_t d_dn, const uint32_t *__restrict__ su,
    const double *__restrict__ eu, const int ntile, const int32_t *__restrict__ tnt,
    const int32_t *__restrict__ toff, const uint32_t *__restrict__ ent,
    const uint32_t *__restrict__ ent32, const int ent_bytes,
    const double *__restrict__ ctab_g, const int nctab, const uint32_t *__restrict__ sd,
    const double *__restrict__ ed, const double *__restrict__ ulut_g, const int nbytes,
    const double u_uniform, const double tu, T *__restrict__ v, T *w, const LazyUpd lz) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NT = kInrowThreads;   // the launch's block size
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), nwave = NT >> 6;
    const int dup = (int)d_up;
    T *row = reinterpret_cast<T *>(smem);
    // zero slot: 64 bytes right after the row (a padding entry's offset 8 d_up,
    // halved for FP32 rows, points there).  NEG (FP32 rows, one t for every
    // bond): a negated copy of the row follows, and the entries are the
    // neighbours' LDS addresses in the row or in the copy, so that a gather
    // needs neither a mask nor a sign flip
    constexpr bool NEG = UT && sizeof(T) == 4;
    const size_t zero_at = sizeof(T) * (size_t)dup;
    const size_t neg_at = NEG ? neg_row_at(dup) : 0;
    T *rowneg = reinterpret_cast<T *>(smem + neg_at);
    const size_t tab_at =
        NEG ? neg_at + ((4 * (size_t)dup + 15) & ~(size_t)15) : (zero_at + 64 + 15) & ~(size_t)15;
    double *ct = reinterpret_cast<double *>(smem + tab_at);
    double *ulut = ct + ((nctab + 1) & ~1);
    if (tid < 16) reinterpret_cast<uint32_t *>(smem + zero_at)[tid] = 0u;
    const int nlut = u_uniform >= 0.0 ? 0 : nbytes * 256;
    for (int k = tid; k < nlut; k += NT) ulut[k] = ulut_g[k];
    if (!UT)
        for (int k = tid; k < nctab; k += NT) ct[k] = ctab_g[k];
    typedef __attribute__((address_space(3))) const T lds_t;
    const int64_t vb = (int64_t)blockIdx.y * d_up * d_dn;
    T *vv = v + vb;
    T *ww = w + vb;
    // the deferred update's operands (LZ > 0)
    const T *vo = LZ ? (const T *)lz.vold + vb : nullptr;
    const T *vpo = LZ == 2 ? (const T *)lz.vpold + vb : nullptr;
    double la = 0.0, lc1 = 0.0, lc2 = 0.0, linv = 0.0;
    if (LZ) {
        la = lz.apre[blockIdx.y];
        linv = lz.inv[blockIdx.y];
        if (LZ == 2) {
            lc1 = lz.corr[blockIdx.y];
            lc2 = lz.corr2[blockIdx.y];
        }
    }
    // slot k of a row is element tid + k NT, at byte offset voff + k sstep
    const int voff = tid * (int)sizeof(T);
    constexpr int sstep = NT * (int)sizeof(T);
    T xr[KS];
    T yr[LZ ? KS : 1];
    T zr[LZ == 2 ? KS : 1];
    auto fetch = [&](int64_t rr) {
        const int64_t o = rr * d_up;
        const __amdgpu_buffer_rsrc_t rv = row_rsrc(vv + o, d_up);
#pragma unroll
        for (int k = 0; k < KS; ++k) xr[k] = row_load<T>(rv, voff, k * sstep);
        if (LZ) {
            const __amdgpu_buffer_rsrc_t ro = row_rsrc(vo + o, d_up);
#pragma unroll
            for (int k = 0; k < KS; ++k) yr[k] = row_load<T>(ro, voff, k * sstep);
        }
        if (LZ == 2) {
            const __amdgpu_buffer_rsrc_t rp = row_rsrc(vpo + o, d_up);
#pragma unroll
            for (int k = 0; k < KS; ++k) zr[k] = row_load<T>(rp, voff, k * sstep);
        }
    };
    // the up strings' bits and diagonal, and the hop table, through buffer
    // descriptors: a lane offset register and a scalar tile offset, with no
    // 64-bit address arithmetic per tile or per group
    const __amdgpu_buffer_rsrc_t rsu = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t *>(su), (short)0, (int)(4 * d_up), 0x00020000);
    const __amdgpu_buffer_rsrc_t reu = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double *>(eu), (short)0, (int)(8 * d_up), 0x00020000);
    const __amdgpu_buffer_rsrc_t rent =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(NEG ? ent32 : ent), (short)0, ent_bytes,
                                          0x00020000);
    int64_t r = blockIdx.x;
    if (r < d_dn) fetch(r);
    for (; r < d_dn; r += gridDim.x) {
        __syncthreads();
        if (LZ) {
            // v_{n+1} as the update pass forms it (stored over w_n after the
            // hop loop)
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                const double vi = (double)yr[k];
                double x = fma(-la, vi, (double)xr[k]);
                if (LZ == 2) {
                    x = fma(-lc1, vi, x);
                    x = fma(-lc2, (double)zr[k], x);
                }
                xr[k] = (T)(x * linv);
            }
        }
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int idx = tid + k * NT;
            if (idx < dup) {
                row[idx] = xr[k];
                if (NEG) rowneg[idx] = -xr[k];
            }
        }
        __syncthreads();
        const int64_t rn = r + gridDim.x;
        if (rn < d_dn) fetch(rn);
        const uint32_t bd = sd[r];
        const double edn = ed[r];
        const __amdgpu_buffer_rsrc_t rw = row_rsrc(ww + r * d_up, d_up);
        for (int tt = wave; tt < ntile; tt += nwave) {
            const int iu = tt * 64 + lane;
            const int nt = tnt[tt];
            const int eoff = toff[tt] * 4;   // the tile's entries, in bytes
            const bool in = iu < dup;
            double acc = 0.0;
            if (in) {
                const uint32_t dbl =
                    __builtin_amdgcn_raw_buffer_load_b32(rsu, lane * 4, tt * 256, 0) & bd;
                double diag = __builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(reu, lane * 8, tt * 512, 0)) + edn;
                if (u_uniform >= 0.0) {
                    diag += u_uniform * (double)__popc(dbl);
                } else {
                    for (int byte = 0; byte < nbytes; ++byte)
                        diag += ulut[byte * 256 + ((dbl >> (8 * byte)) & 255u)];
                }
                acc = diag * (double)row[iu];
            }
            // n entries from slot s: loaded, gathered, then summed in slot order
            auto group = [&](const int s, auto n_) {
                constexpr int n = decltype(n_)::value;
                uint32_t p[n];
#pragma unroll
                for (int u = 0; u < n; u += 4) {
                    const u32x4_t q = __builtin_bit_cast(
                        u32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rent, lane * 16,
                                                                        eoff + ((s + u) >> 2) * 1024, 0));
                    p[u] = q.x;
                    p[u + 1] = q.y;
                    p[u + 2] = q.z;
                    p[u + 3] = q.w;
                }
                double x[n];
#pragma unroll
                for (int u = 0; u < n; ++u) {
                    const uint32_t off = NEG ? p[u]
                                       : sizeof(T) == 8 ? (p[u] & 0x1ffffu) : ((p[u] & 0x1ffffu) >> 1);
                    x[u] = (double)*(lds_t *)(size_t)off;
                }
#pragma unroll
                for (int u = 0; u < n; ++u) {
                    if constexpr (NEG) {
                        acc = fma(tu, x[u], acc);
                    } else if constexpr (UT) {
                        const double xs = __hiloint2double(
                            __double2hiint(x[u]) ^ (int)(p[u] & 0x80000000u), __double2loint(x[u]));
                        acc = fma(tu, xs, acc);
                    } else {
                        acc = fma(ct[(p[u] >> 17) & 0x3fffu], x[u], acc);
                    }
                }
            };
            int s = 0;
            for (; s + kTileChunk <= nt; s += kTileChunk)
                group(s, std::integral_constant<int, kTileChunk>{});
            if (s < nt) group(s, std::integral_constant<int, kTileChunk / 2>{});
            // lanes past the row are dropped by the descriptor's range check
            row_store<T>((T)acc, rw, lane * (int)sizeof(T), tt * 64 * (int)sizeof(T));
        }
        if (LZ) {
            // v_{n+1} of this row, from its LDS copy: stored after the hop
            // loop rather than when the row is staged, since the memory
            // counter completes in order and the first hop-table wait of the
            // row would otherwise wait for these stores too (4x4 Lanczos step
            // 3.49 -> 3.45 ms)
            const __amdgpu_buffer_rsrc_t rs = row_rsrc(vv + r * d_up, d_up);
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                const int idx = tid + k * NT;
                if (idx < dup) row_store<T>(row[idx], rs, voff, k * sstep);
            }
        }
    }
}

// Pass B: W += K_dn V on column slabs, hopping lists row-contiguous and
// wave-uniform (scalar loads), RI rows of a wave with 8 neighbour segments
// each in flight (RI: chosen at the launch below; for the FP64 product four
// rows were 2.5 % faster than two on the 4x4 sector, while 1, 6 or 8 rows, or
// 32-row slabs, were slower).  When d_up is even a lane takes two adjacent
// columns (one 2-element load per neighbour), which halves the load
// instructions.  Within a slab the rows are taken in row_order: grouped by
// the popcount of the high half of the down string.  Hops inside either half
// keep that popcount, so the rows an XCD has in flight find most of their
// neighbour segments among rows of the same group (4,900 rows x 1 KB for the
// 4x4 FP64 slab of the largest group: a little more than the XCD's 4 MB L2,
// so part of them come back from the Infinity Cache).
// Row-major list of the down hops of every row, as element offsets of the
// neighbour row (j_dn * d_up) and coefficients, padded to the width W.
__global__ void k_row_offsets(int64_t d_dn, int W, int64_t d_up, const int32_t *__restrict__ col,
                              int64_t *__restrict__ off) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < d_dn * W) off[e] = (int64_t)col[e] * d_up;
}

// a native two-element vector, for the non-temporal accesses to W
template <typename T>
struct NV2 {
    typedef T type __attribute__((ext_vector_type(2)));
};

template <typename T>
struct Pair;
template <>
struct Pair<double> {
    typedef double2 type;
};
template <>
struct Pair<float> {
    typedef float2 type;
};

// With SP (a Lanczos step): each stored element becomes w - beta' vp (after
// the product's own rounding, as a separate pass would do it), and every
// workgroup writes its partial <v, w> to sp.pa[vec * gridDim.x + block] (0
// for workgroups without rows), a fixed-order block sum.

typedef long long i64x8_t __attribute__((ext_vector_type(8), aligned(8)));

template <typename T, int RI, int CW, bool SP, bool BUF>
__global__ void __launch_bounds__(256) k_hv_down_acc(
    const int64_t d_up, const int64_t d_dn, const int W, const int32_t *__restrict__ nhd,
    const int64_t *__restrict__ offs, const double *__restrict__ cfd, const T *__restrict__ v,
    T *__restrict__ w, const int R, const int64_t nrb, const int64_t total, const int64_t per,
    const int32_t *__restrict__ order, const SubPrev sp) {
    typedef typename Pair<T>::type T2;
    __shared__ double sh[256];
    const int64_t p = blockIdx.x;
    const int64_t lg = (p & 7) * per + (p >> 3);  // XCD p % 8 takes a contiguous range
    if (lg >= total) {
        if (SP && threadIdx.x == 0)
            for (int k = 0; k < (sp.reorth ? 5 : 3); ++k)
                sp.pa[k * sp.pstride + (int64_t)blockIdx.y * gridDim.x + p] = 0.0;
        return;
    }
    const int64_t slab = lg / nrb, rb = lg - slab * nrb;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t c0 = slab * (64 * CW) + lane * CW;
    const bool cok = c0 < d_up;
    const int64_t vb = (int64_t)blockIdx.y * d_up * d_dn;
    const T *vv = v + vb;
    T *ww = w + vb;
    const T *vpp = SP ? (const T *)sp.vp + vb : nullptr;
    // BUF: the vector is under 2 GB, so a neighbour row's byte offset fits the
    // 32-bit scalar offset of a buffer load
    const __amdgpu_buffer_rsrc_t rvv = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T *>(vv), (short)0, BUF ? (int)(d_up * d_dn * (int64_t)sizeof(T)) : 0, 0x00020000);
    const int lvo = (int)(c0 * (int64_t)sizeof(T));
    const double bprev = (SP && sp.n > 0) ? sp.beta[(int64_t)blockIdx.y * sp.maxs + sp.n - 1] : 0.0;
    double p_vw = 0.0, p_ww = 0.0, p_vv = 0.0, p_pw = 0.0, p_pv = 0.0;
    // the element as a separate pass would leave it: product rounded once,
    // then w - beta' vp rounded once; and its shares of the step's dots
    auto fin = [&](double a, int64_t i) -> T {
        T t = (T)a;
        if (SP) {
            const double pv = sp.n > 0 ? (double)vpp[i] : 0.0;
            if (sp.n > 0) t = (T)fma(-bprev, pv, (double)t);
            const double vi = (double)vv[i], wi = (double)t;
            p_vw = fma(vi, wi, p_vw);
            p_ww = fma(wi, wi, p_ww);
            p_vv = fma(vi, vi, p_vv);
            if (sp.reorth) {
                p_pw = fma(pv, wi, p_pw);
                p_pv = fma(pv, vi, p_pv);
            }
        }
        return t;
    };
    for (int k = wave * RI; k < R; k += 4 * RI) {
        int64_t rr[RI];
        int nh[RI];
        double acc[RI][CW];
        int nmax = 0;
#pragma unroll
        for (int q = 0; q < RI; ++q) {
            const int64_t r = rb * R + k + q;
            const bool ok = r < d_dn;
            rr[q] = ok ? order[r] : 0;
            nh[q] = ok ? nhd[rr[q]] : 0;
            nmax = nh[q] > nmax ? nh[q] : nmax;
            if (CW == 2) {
                // FP64: W streams past the L2 (non-temporal), leaving it to the
                // neighbour segments (4x4 product 2.69 -> 2.64 ms; FP32 vectors
                // were 2 % slower that way)
                typedef typename NV2<T>::type V2;
                V2 a2 = {T(0), T(0)};
                if (ok && cok) {
                    const V2 *pw = reinterpret_cast<const V2 *>(ww + rr[q] * d_up + c0);
                    a2 = sizeof(T) == 8 ? __builtin_nontemporal_load(pw) : *pw;
                }
                acc[q][0] = (double)a2.x;
                acc[q][CW - 1] = (double)a2.y;
            } else {
                acc[q][0] = (ok && cok) ? (double)ww[rr[q] * d_up + c0] : 0.0;
            }
        }
        if (rb * R + k >= d_dn) break;
        for (int s0 = 0; s0 < nmax; s0 += 8) {
            T x[RI][8][CW];
            double cf[RI][8];
#pragma unroll
            for (int q = 0; q < RI; ++q) {
                // the plain product takes the group's eight neighbour offsets
                // as one 64-byte scalar load (entries past the row's hops, or
                // past the table's last row into its slack, are loaded but not
                // used), so that the neighbour loads are not each held up by a
                // scalar load (4x4 FP32 product 2.32 -> 2.20 ms, FP64
                // unchanged); the Lanczos form loads them one by one (its FP32
                // step was 2 % slower with the batch)
                const int64_t *olp = offs + rr[q] * W + s0;
                i64x8_t ol;
                if constexpr (!SP) ol = *reinterpret_cast<const i64x8_t *>(olp);
                const double *cl = cfd + rr[q] * W;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool ok = s0 + u < nh[q];
                    const int64_t jo = ok ? (SP ? olp[u] : ol[u]) : 0;
                    cf[q][u] = ok ? cl[s0 + u] : 0.0;
                    if (CW == 2 && BUF) {
                        // through the vector's descriptor: the neighbour row
                        // as a scalar offset, the lane's columns as a
                        // constant register (lanes past the row read the
                        // next row's columns, which they do not store; the
                        // range check covers the last row)
                        T2 t2 = T2{};
                        if (ok) {
                            if constexpr (sizeof(T) == 8)
                                t2 = __builtin_bit_cast(T2, __builtin_amdgcn_raw_buffer_load_b128(
                                                                rvv, lvo, (int)(jo * 8), 0));
                            else
                                t2 = __builtin_bit_cast(T2, __builtin_amdgcn_raw_buffer_load_b64(
                                                                rvv, lvo, (int)(jo * 4), 0));
                        }
                        x[q][u][0] = t2.x;
                        x[q][u][CW - 1] = t2.y;
                    } else if (CW == 2) {
                        T2 t2 = (ok && cok) ? *reinterpret_cast<const T2 *>(vv + jo + c0) : T2{};
                        x[q][u][0] = t2.x;
                        x[q][u][CW - 1] = t2.y;
                    } else {
                        x[q][u][0] = (ok && cok) ? vv[jo + c0] : T(0);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < RI; ++q)
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int c = 0; c < CW; ++c)
                        acc[q][c] = fma(cf[q][u], (double)x[q][u][c], acc[q][c]);
        }
        if (cok) {
#pragma unroll
            for (int q = 0; q < RI; ++q)
                if (rb * R + k + q < d_dn) {
                    const int64_t i = rr[q] * d_up + c0;
                    if (CW == 2) {
                        typedef typename NV2<T>::type V2;
                        V2 o2;
                        o2.x = fin(acc[q][0], i);
                        o2.y = fin(acc[q][CW - 1], i + 1);
                        if (sizeof(T) == 8)
                            __builtin_nontemporal_store(o2, reinterpret_cast<V2 *>(ww + i));
                        else
                            *reinterpret_cast<V2 *>(ww + i) = o2;
                    } else {
                        ww[i] = fin(acc[q][0], i);
                    }
                }
        }
    }
    if (SP) {
        double *o = sp.pa + (int64_t)blockIdx.y * gridDim.x + p;
        const double t0 = block_sum(p_vw, sh);
        const double t1 = block_sum(p_ww, sh);
        const double t2 = block_sum(p_vv, sh);
        if (threadIdx.x == 0) {
            o[0] = t0;
            o[sp.pstride] = t1;
            o[2 * sp.pstride] = t2;
        }
        if (sp.reorth) {
            const double t3 = block_sum(p_pw, sh);
            const double t4 = block_sum(p_pv, sh);
            if (threadIdx.x == 0) {
                o[3 * sp.pstride] = t3;
                o[4 * sp.pstride] = t4;
            }
        }
    }
}

// ---------------------------------------------------------------- set-up and launch

int build_row_offsets(HopTables &ht, int64_t d_up, Carver &cv, hipStream_t s) {
    // eight entries of slack: the row-mixing pass reads a row's hops eight at
    // a time
    ht.off = cv.take<int64_t>((size_t)ht.width * ht.d + 8);
    if (!cv.base) return QCM_OK;
    const int64_t n = (int64_t)ht.width * ht.d;
    k_row_offsets<<<ceil_div(n, 256), 256, 0, s>>>(ht.d, ht.width, d_up, ht.col, ht.off);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}


static size_t inrow_lds_bytes(const HvOp &op, int prec) {
    const size_t es = prec == QCM_FP64 ? 8 : 4;
    // the row, the 64-byte zero slot (FP32 rows with one t for every bond:
    // then the negated row), then the coefficient and U tables
    size_t row = (es * (size_t)op.up.d + 64 + 15) & ~(size_t)15;
    if (prec != QCM_FP64 && op.md.t_is_uniform)
        row = neg_row_at(op.up.d) + ((4 * (size_t)op.up.d + 15) & ~(size_t)15);
    const size_t nct = (size_t)((2 * op.md.nbond + 1) & ~1);
    const size_t lut = op.md.u_uniform >= 0.0 ? 0 : 256 * (size_t)op.md.nbytes;
    return row + 8 * (nct + lut);
}

template <typename T>
static int split_launch_t(const HvOp &op, void *v, void *w, int nvec, hipStream_t s,
                          const SubPrev *sp, const LazyUpd *lzp) {
    const int64_t d_up = op.up.d, d_dn = op.dn.d;
    const HopTables &hd_rm = op.hd_rm;
    const size_t lds = inrow_lds_bytes(op, sizeof(T) == 8 ? QCM_FP64 : QCM_FP32V);
    if (lds > 160 * 1024) return fail(QCM_EARG, "in-row pass: the row does not fit LDS");
    const int ks = (int)((d_up + 1023) / 1024);
    const int nctab = 2 * op.md.nbond;
    // pass A: in-row term and diagonal, writes W (and first forms v from a
    // deferred update)
    dim3 gp((unsigned)std::min<int64_t>(d_dn, 256), (unsigned)nvec);
    const LazyUpd lz = lzp ? *lzp : LazyUpd{};
    const int lzm = lzp ? (lz.reorth ? 2 : 1) : 0;
#define QCM_PK_L(KS_, UT_, LZ_)                                                                \
    k_hv_inrow_tile<T, KS_, UT_, LZ_><<<gp, 1024, lds, s>>>(                                   \
        d_up, d_dn, op.up.states, op.hu.ediag, op.ntile, op.tile_nt, op.tile_off, op.tile_ent, \
        op.tile_ent32, op.tile_bytes,                                                          \
        op.md.ctab, nctab, op.dn.states, op.hd.ediag, op.md.ulut, op.md.nbytes,                \
        op.md.u_uniform, op.md.t_uniform, (T *)v, (T *)w, lz)
#define QCM_PK_U(KS_, UT_)                                                                     \
    do {                                                                                       \
        if (lzm == 0)                                                                          \
            QCM_PK_L(KS_, UT_, 0);                                                             \
        else if (lzm == 1)                                                                     \
            QCM_PK_L(KS_, UT_, 1);                                                             \
        else                                                                                   \
            QCM_PK_L(KS_, UT_, 2);                                                             \
    } while (0)
#define QCM_PK(KS_)                                                                            \
    if (ks <= KS_) {                                                                           \
        if (op.md.t_is_uniform)                                                                \
            QCM_PK_U(KS_, true);                                                               \
        else                                                                                   \
            QCM_PK_U(KS_, false);                                                              \
    } else
    // one instantiation per slot count, so that no slot past the row is
    // carried through the hop loop (4x4 H.v 2.70 -> 2.67 ms with 13 slots
    // instead of 16)
    QCM_PK(4) QCM_PK(5) QCM_PK(6) QCM_PK(7) QCM_PK(8) QCM_PK(9) QCM_PK(10) QCM_PK(11) QCM_PK(12)
    QCM_PK(13) QCM_PK(14) QCM_PK(15) QCM_PK(16) { return fail(QCM_EARG, "in-row pass: row too long"); }
#undef QCM_PK
#undef QCM_PK_U
#undef QCM_PK_L
    QCM_LAUNCH_CHECK();
    // pass B: row mixing, accumulates into W
    const int R = 16;
    const int cw = (d_up % 2 == 0) ? 2 : 1;
    const int64_t nslab = (d_up + 64 * cw - 1) / (64 * cw);
    const int64_t nrb = (d_dn + R - 1) / R;
    const int64_t total = nslab * nrb;
    const int64_t per = (total + 7) / 8;
    dim3 g1((unsigned)(8 * per), (unsigned)nvec);
    const SubPrev none{};
    // neighbour loads through the vector's descriptor when its byte offsets
    // fit the 32-bit scalar offset (4x4 FP32 product 2.20 -> 1.74 ms, FP64
    // unchanged)
    const bool buf = d_up * d_dn * (int64_t)sizeof(T) < ((int64_t)1 << 31);
#define QCM_DACC_K(RI, CW, SP_, BUF_, SPV)                                                     \
    k_hv_down_acc<T, RI, CW, SP_, BUF_><<<g1, 256, 0, s>>>(                                    \
        d_up, d_dn, hd_rm.width, hd_rm.nh, hd_rm.off, hd_rm.coef, (const T *)v, (T *)w, R, nrb, \
        total, per, op.row_order, SPV)
#define QCM_DACC(RI, CW)                                                                       \
    do {                                                                                       \
        if constexpr (CW == 2) {                                                               \
            if (sp && buf)                                                                     \
                QCM_DACC_K(RI, CW, true, true, *sp);                                           \
            else if (sp)                                                                       \
                QCM_DACC_K(RI, CW, true, false, *sp);                                          \
            else if (buf)                                                                      \
                QCM_DACC_K(RI, CW, false, true, none);                                         \
            else                                                                               \
                QCM_DACC_K(RI, CW, false, false, none);                                        \
        } else {                                                                               \
            if (sp)                                                                            \
                QCM_DACC_K(RI, CW, true, false, *sp);                                          \
            else                                                                               \
                QCM_DACC_K(RI, CW, false, false, none);                                        \
        }                                                                                      \
    } while (0)
    // Rows in flight per wave, measured on the 4x4 sector: FP64 keeps four
    // for the product alone; its Lanczos form (the epilogue needs more
    // registers) is faster with two, which leave room for five waves per SIMD
    // instead of three; FP32 vectors are fastest with one (product 2.80 ->
    // 2.55 ms, step 3.97 -> 3.28 ms against two).
    if (cw == 2 && sizeof(T) == 8 && !sp)
        QCM_DACC(4, 2);
    else if (cw == 2 && sizeof(T) == 8)
        QCM_DACC(2, 2);
    else if (cw == 2)
        QCM_DACC(1, 2);
    else
        QCM_DACC(2, 1);
#undef QCM_DACC
#undef QCM_DACC_K
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

// Workgroups of the row-mixing pass per vector: the length of the partial
// <v, w> array a fused Lanczos step writes per chain.
int64_t split_pa_count(const HvOp &op) {
    const int64_t d_up = op.up.d, d_dn = op.dn.d;
    const int R = 16;
    const int cw = (d_up % 2 == 0) ? 2 : 1;
    const int64_t nslab = (d_up + 64 * cw - 1) / (64 * cw);
    const int64_t total = nslab * ((d_dn + R - 1) / R);
    return 8 * ((total + 7) / 8);
}

// ---------------------------------------------------------------- dispatch

bool split_applies(const qcm_model *m, int n_up, int64_t d_up, int64_t d_dn) {
    (void)n_up;
    if (d_up < kSplitMinUp || d_up > kSplitMaxUp || d_dn < 1) return false;
    // the FP64 row, its zero slot, the coefficient table and the U lookup
    // table in LDS
    const size_t nct = (size_t)((2 * count_bonds(m) + 1) & ~1);
    const size_t lut = 256 * (size_t)((m->L + 7) / 8);
    return 8 * (size_t)d_up + 64 + 16 + 8 * (nct + lut) <= 160 * 1024;
}

int split_prepare(const qcm_model *m, HvOp &op, Carver &cv, hipStream_t s) {
    // decided from the sector, not from op.hu.pk: a dry run (no base) carves
    // null pointers and must take the same path as the real one
    if (op.hu.rowmajor || op.up.d > kSplitMaxUp)
        return fail(QCM_EARG, "two-pass product: no packed up hops for this sector");
    // the padding entry's offset 8 d_up must fit the entry's 17 offset bits
    if (8 * op.up.d >= ((int64_t)1 << 17))
        return fail(QCM_EARG, "two-pass product: row of %lld strings too long", (long long)op.up.d);
    const int64_t du = op.up.d;
    op.ntile = (int32_t)((du + 63) / 64);
    const int wr = (op.hu.width + kTileChunk - 1) / kTileChunk * kTileChunk;
    op.tile_ent = cv.take<uint32_t>((size_t)op.ntile * wr * 64);
    op.tile_ent32 = op.md.t_is_uniform ? cv.take<uint32_t>((size_t)op.ntile * wr * 64) : nullptr;
    op.tile_nt = cv.take<int32_t>(op.ntile);
    op.tile_off = cv.take<int32_t>(op.ntile);
    QCM_TRY(build_hop_tables(op.md, op.dn, cv, &op.hd_rm, s, count_bonds(m), 1));
    QCM_TRY(build_row_offsets(op.hd_rm, op.up.d, cv, s));
    // rows grouped by the popcount of the high half of the down string, so
    // that the rows in flight and their in-class neighbours share L2
    op.row_order = cv.take<int32_t>(op.dn.d);
    if (cv.base) {
        const int L = op.dn.L, N = op.dn.N, llo = (L + 1) / 2;
        std::vector<int32_t> ord;
        ord.reserve(op.dn.d);
        for (int k = 0; k <= L - llo; ++k) {
            int32_t idx = 0;
            for (uint64_t x = 0; x < (uint64_t(1) << L); ++x) {
                if (__builtin_popcountll(x) != N) continue;
                if (__builtin_popcountll(x >> llo) == k) ord.push_back(idx);
                ++idx;
            }
        }
        if ((int64_t)ord.size() != op.dn.d) return fail(QCM_EARG, "row order size");
        QCM_HIP(hipMemcpyAsync(op.row_order, ord.data(), sizeof(int32_t) * ord.size(),
                               hipMemcpyHostToDevice, s));
        QCM_HIP(hipStreamSynchronize(s));   // ord is pageable and about to go
    }
    if (cv.base) {
        // each tile's slot count from the hop counts (read back once)
        std::vector<int32_t> nh(du), tnt(op.ntile), toff(op.ntile);
        QCM_HIP(hipMemcpyAsync(nh.data(), op.hu.nh, sizeof(int32_t) * du, hipMemcpyDeviceToHost, s));
        QCM_HIP(hipStreamSynchronize(s));
        int32_t o = 0;
        for (int tt = 0; tt < op.ntile; ++tt) {
            int mx = 0;
            for (int l = 0; l < 64 && tt * 64 + l < du; ++l) mx = std::max(mx, nh[tt * 64 + l]);
            tnt[tt] = (mx + 3) / 4 * 4;
            toff[tt] = o;
            o += tnt[tt] * 64;
        }
        op.tile_bytes = 4 * o;
        QCM_HIP(hipMemcpyAsync(op.tile_nt, tnt.data(), sizeof(int32_t) * op.ntile,
                               hipMemcpyHostToDevice, s));
        QCM_HIP(hipMemcpyAsync(op.tile_off, toff.data(), sizeof(int32_t) * op.ntile,
                               hipMemcpyHostToDevice, s));
        k_pack_tiles<<<op.ntile, 64, 0, s>>>(du, op.hu.nh, op.hu.pk, op.tile_nt, op.tile_off,
                                              op.tile_ent, op.tile_ent32, neg_row_at(du));
        QCM_LAUNCH_CHECK();
        QCM_HIP(hipStreamSynchronize(s));   // tnt and toff are pageable and about to go
    }
    op.split = 1;
    return QCM_OK;
}

// v is only read here (the plain product writes W alone)
int hv_split_launch(const HvOp &op, int prec, const void *v, void *w, int nvec, hipStream_t s) {
    void *vm = const_cast<void *>(v);
    if (prec == QCM_FP64) return split_launch_t<double>(op, vm, w, nvec, s, nullptr, nullptr);
    return split_launch_t<float>(op, vm, w, nvec, s, nullptr, nullptr);
}

int hv_split_launch_sub(const HvOp &op, int prec, void *v, void *w, int nvec, const SubPrev &sp,
                        const LazyUpd *lz, hipStream_t s) {
    if (prec == QCM_FP64) return split_launch_t<double>(op, v, w, nvec, s, &sp, lz);
    return split_launch_t<float>(op, v, w, nvec, s, &sp, lz);
}

}  // namespace qcm
