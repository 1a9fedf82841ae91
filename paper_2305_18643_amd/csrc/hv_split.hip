// H.v in two streaming passes for sectors whose rows are too long to keep the
// neighbour rows on chip (paper: section "Exact diagonalizations", eq.
// (factorized) H = K_up (x) 1 + 1 (x) K_dn + V_int).
//
// With the vector as the row-major matrix V[i_dn][i_up]:
//   pass 1 (row mixing, K_dn):  W = K_dn V
//     The columns are cut into slabs of 64 (FP64) or 128 (FP32) values; all
//     rows of one slab are produced by the workgroups of one XCD, so the
//     neighbour rows a slab needs (about 13 per row) are read from that XCD's
//     L2 instead of HBM.  The hopping list of a row is wave-uniform (scalar
//     loads), the neighbour values are 512-byte coalesced segments.
//   pass 2 (inside rows, K_up, and the diagonal):  W += V K_up^T + D o V
//     Persistent workgroups stage one whole row in LDS and gather the
//     neighbour values from it.  The hopping of the up string b = (h, l) is
//     described by small tables indexed by its low half l and its high half h
//     (all staged in LDS): a hop inside l shifts the label by an amount that
//     depends on l only, a hop inside h by an amount that depends on h only,
//     and a hop across the halves lands at base(h') + rlo[l'].
// Every sum is FP64 in registers; W is rounded once per pass to the storage
// type (FP64: exact same sums as one pass; FP32 vectors: two roundings).
#include <string.h>

#include <algorithm>

#include "qcm_internal.h"

namespace qcm {

// ---------------------------------------------------------------- host tables

static int64_t hbinom(int n, int k) { return binom(n, k); }

struct HostSplit {
    int l_lo, l_hi, nb;
    std::vector<double> coef, e_lo, e_hi;
    std::vector<uint64_t> hi_ent;
    std::vector<int32_t> rlo, lo_off, hi_off;
    std::vector<uint32_t> lo_ent;
    // team layout
    std::vector<int32_t> cls, llist, hlist, hbase, xbond;
    std::vector<uint64_t> xtab;
    int max_lo = 0, max_hi = 0;
};

static bool make_host_split(const qcm_model *m, int N, HostSplit &H) {
    const int L = m->L;
    const int l_lo = (L + 1) / 2, l_hi = L - l_lo;
    H.l_lo = l_lo;
    H.l_hi = l_hi;
    std::vector<int> ba, bb;
    std::vector<double> bt;
    for (int a = 0; a < L; ++a)
        for (int b = a + 1; b < L; ++b)
            if (m->t[a * L + b] != 0.0) {
                ba.push_back(a);
                bb.push_back(b);
                bt.push_back(m->t[a * L + b]);
            }
    const int nb = (int)ba.size();
    H.nb = nb;
    if (nb >= (1 << 9)) return false;
    H.coef.assign(2 * nb + 2, 0.0);  // last entries: zero, used by padding
    for (int k = 0; k < nb; ++k) {
        H.coef[2 * k] = bt[k];
        H.coef[2 * k + 1] = -bt[k];
    }
    const int nlo = 1 << l_lo, nhi = 1 << l_hi;
    // rank tables of the split (combinatorial sums)
    H.rlo.resize(nlo);
    for (int x = 0; x < nlo; ++x) {
        int64_t r = 0;
        int j = 0;
        for (int p = 0; p < l_lo; ++p)
            if ((x >> p) & 1) r += hbinom(p, ++j);
        H.rlo[x] = (int32_t)r;
    }
    auto rhi = [&](int n, int y) -> int64_t {
        int64_t r = 0;
        int j = 0;
        for (int q = 0; q < l_hi; ++q)
            if ((y >> q) & 1) r += hbinom(l_lo + q, n + (++j));
        return r;
    };
    H.e_lo.assign(nlo, 0.0);
    H.e_hi.assign(nhi, 0.0);
    for (int x = 0; x < nlo; ++x)
        for (int p = 0; p < l_lo; ++p)
            if ((x >> p) & 1) H.e_lo[x] += m->t[p * L + p];
    for (int y = 0; y < nhi; ++y)
        for (int q = 0; q < l_hi; ++q)
            if ((y >> q) & 1) H.e_hi[y] += m->t[(l_lo + q) * L + (l_lo + q)];
    // lo hops: both ends below l_lo
    H.lo_off.assign(nlo + 1, 0);
    for (int x = 0; x < nlo; ++x) {
        for (int k = 0; k < nb; ++k) {
            int a = ba[k], b = bb[k];
            if (b >= l_lo) continue;
            bool oa = (x >> a) & 1, ob = (x >> b) & 1;
            if (oa == ob) continue;
            int y = x ^ (1 << a) ^ (1 << b);
            int between = __builtin_popcount(x & ((1u << b) - 1u) & ~((2u << a) - 1u));
            int64_t d = (int64_t)H.rlo[y] - H.rlo[x];
            if (d < -32768 || d > 32767) return false;
            uint32_t ci = 2 * k + (between & 1);
            H.lo_ent.push_back((uint32_t)(uint16_t)(int16_t)d | (ci << 16));
        }
        H.lo_off[x + 1] = (int32_t)H.lo_ent.size();
    }
    // hi and cross hops, per high half h (group of columns with that high half)
    H.hi_off.assign(nhi + 1, 0);
    for (int y = 0; y < nhi; ++y) {
        int n_l = N - __builtin_popcount(y);
        if (n_l >= 0 && n_l <= l_lo) {
            int64_t base = rhi(n_l, y);
            for (int k = 0; k < nb; ++k) {
                int a = ba[k], b = bb[k];
                if (a < l_lo) continue;
                int qa = a - l_lo, qb = b - l_lo;
                bool oa = (y >> qa) & 1, ob = (y >> qb) & 1;
                if (oa == ob) continue;
                int y2 = y ^ (1 << qa) ^ (1 << qb);
                int between = __builtin_popcount(y & ((1u << qb) - 1u) & ~((2u << qa) - 1u));
                int64_t d = rhi(n_l, y2) - base;
                uint64_t ci = 2 * k + (between & 1);
                H.hi_ent.push_back((uint64_t)(uint32_t)(int32_t)d | (ci << 32));
            }
        }
        H.hi_off[y + 1] = (int32_t)H.hi_ent.size();
        H.max_hi = std::max(H.max_hi, H.hi_off[y + 1] - H.hi_off[y]);
    }
    for (int x = 0; x < nlo; ++x) H.max_lo = std::max(H.max_lo, H.lo_off[x + 1] - H.lo_off[x]);
    // classes: low halves of popcount n (ascending = by rlo) times high halves
    // of popcount N - n (ascending), each high half a contiguous label range
    for (int n = 0; n <= l_lo; ++n) {
        int nh = N - n;
        if (nh < 0 || nh > l_hi) continue;
        int cl = (int)hbinom(l_lo, n), ch = (int)hbinom(l_hi, nh);
        H.cls.push_back(cl);
        H.cls.push_back(ch);
        H.cls.push_back((int)H.llist.size());
        H.cls.push_back((int)H.hlist.size());
        std::vector<int> ls;
        for (int x = 0; x < nlo; ++x)
            if (__builtin_popcount(x) == n) ls.push_back(x);
        std::sort(ls.begin(), ls.end(), [&](int a, int b) { return H.rlo[a] < H.rlo[b]; });
        for (int x : ls) H.llist.push_back(x);
        for (int y = 0; y < nhi; ++y)
            if (__builtin_popcount(y) == nh) {
                H.hlist.push_back(y);
                H.hbase.push_back((int32_t)rhi(n, y));
            }
    }
    // cross bonds (one low end a, one high end b) and, per high half, the
    // high-half part of each: valid, direction, base of the target group, parity
    std::vector<int> xk;
    for (int k = 0; k < nb; ++k)
        if (ba[k] < l_lo && bb[k] >= l_lo) xk.push_back(k);
    for (int k : xk) H.xbond.push_back(ba[k] | (k << 8));
    const int nxb = (int)xk.size();
    H.xtab.assign((size_t)nhi * std::max(nxb, 1), 0);
    for (int y = 0; y < nhi; ++y) {
        int n_l = N - __builtin_popcount(y);
        if (n_l < 0 || n_l > l_lo) continue;
        for (int q = 0; q < nxb; ++q) {
            int k = xk[q];
            int qb = bb[k] - l_lo;
            int dir = ((y >> qb) & 1) ? 1 : 0;
            int n2 = dir == 0 ? n_l - 1 : n_l + 1;
            if (n2 < 0 || n2 > l_lo) continue;
            int64_t base2 = rhi(n2, y ^ (1 << qb));
            int par = __builtin_popcount(y & ((1u << qb) - 1u)) & 1;
            uint64_t meta = 1u | (dir << 1) | (par << 2);
            H.xtab[(size_t)y * nxb + q] = (uint64_t)(uint32_t)(int32_t)base2 | (meta << 32);
        }
    }
    return true;
}

static SplitLayout layout_of(const HostSplit &H) {
    SplitLayout o;
    size_t p = 0;
    auto put = [&](size_t n, size_t sz) {
        p = (p + 15) / 16 * 16;
        int32_t r = (int32_t)p;
        p += n * sz;
        return r;
    };
    o.off_coef = put(H.coef.size(), 8);
    o.off_elo = put(H.e_lo.size(), 8);
    o.off_ehi = put(H.e_hi.size(), 8);
    o.off_hient = put(H.hi_ent.size(), 8);
    o.off_rlo = put(H.rlo.size(), 4);
    o.off_looff = put(H.lo_off.size(), 4);
    o.off_hioff = put(H.hi_off.size(), 4);
    o.off_loent = put(H.lo_ent.size(), 4);
    o.off_xtab = put(H.xtab.size(), 8);
    o.off_cls = put(H.cls.size(), 4);
    o.off_llist = put(H.llist.size(), 4);
    o.off_hlist = put(H.hlist.size(), 4);
    o.off_hbase = put(H.hbase.size(), 4);
    o.off_xbond = put(H.xbond.size(), 4);
    o.bytes = (int32_t)((p + 15) / 16 * 16);
    o.ncls = (int32_t)(H.cls.size() / 4);
    o.nxb = (int32_t)H.xbond.size();
    o.max_lo = H.max_lo;
    o.zero_coef = 2 * H.nb;
    o.max_hi = H.max_hi;
    return o;
}

bool split_tables_size(const qcm_model *m, int N, size_t *bytes) {
    HostSplit H;
    if (!make_host_split(m, N, H)) return false;
    *bytes = layout_of(H).bytes;
    return true;
}

// ---------------------------------------------------------------- kernels

struct SplitArgs {
    int32_t l_lo;
    uint32_t lo_mask;
    SplitLayout lay;
};

template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
    using type = double2;
};
template <>
struct Vec2<float> {
    using type = float2;
};

// pass A of the team layout: W = V K_up^T + D o V, one row at a time in LDS.
// Threads are grouped in teams that share one low half l: the hops inside l
// are read once into registers and reused for every high half the team
// walks; the high-half hops are the same for the whole team.  The next row is
// prefetched into registers while the current one is computed.
template <typename T, int KS, int MAXLO, int MAXXB>
__global__ void __launch_bounds__(1024) k_hv_inrow_team(
    const int64_t d_up, const int64_t d_dn, const uint32_t *__restrict__ sd,
    const double *__restrict__ ed, const double *__restrict__ ulut_g, const int nbytes,
    const double u_uniform, const SplitArgs sp, const unsigned char *__restrict__ blob,
    const T *__restrict__ v, T *__restrict__ w) {
    extern __shared__ __align__(16) unsigned char smem[];
    const SplitLayout &lay = sp.lay;
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(blob);
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        for (int k = threadIdx.x; k < lay.bytes / 16; k += blockDim.x) dst[k] = src[k];
    }
    const int nlut = u_uniform >= 0.0 ? 0 : nbytes * 256;
    double *ulut = reinterpret_cast<double *>(smem + lay.bytes);
    for (int k = threadIdx.x; k < nlut; k += blockDim.x) ulut[k] = ulut_g[k];
    T *row = reinterpret_cast<T *>(smem + lay.bytes + 8 * nlut);
    const double *coef = reinterpret_cast<const double *>(smem + lay.off_coef);
    const double *elo = reinterpret_cast<const double *>(smem + lay.off_elo);
    const double *ehi = reinterpret_cast<const double *>(smem + lay.off_ehi);
    const uint64_t *hient = reinterpret_cast<const uint64_t *>(smem + lay.off_hient);
    const uint64_t *xtab = reinterpret_cast<const uint64_t *>(smem + lay.off_xtab);
    const int32_t *rlo = reinterpret_cast<const int32_t *>(smem + lay.off_rlo);
    const int32_t *looff = reinterpret_cast<const int32_t *>(smem + lay.off_looff);
    const int32_t *hioff = reinterpret_cast<const int32_t *>(smem + lay.off_hioff);
    const uint32_t *loent = reinterpret_cast<const uint32_t *>(smem + lay.off_loent);
    const int32_t *cls = reinterpret_cast<const int32_t *>(smem + lay.off_cls);
    const int32_t *llist = reinterpret_cast<const int32_t *>(smem + lay.off_llist);
    const int32_t *hlist = reinterpret_cast<const int32_t *>(smem + lay.off_hlist);
    const int32_t *hbase = reinterpret_cast<const int32_t *>(smem + lay.off_hbase);
    const int32_t *xbond = reinterpret_cast<const int32_t *>(smem + lay.off_xbond);
    const int NT = blockDim.x, tid = threadIdx.x;
    const int64_t vb = (int64_t)blockIdx.y * d_up * d_dn;
    const T *vv = v + vb;
    T *ww = w + vb;

    const int dup = (int)d_up;
    T xr[KS];
    int64_t r = blockIdx.x;
    {
        const T *src = vv + r * d_up;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int idx = tid + k * NT;
            xr[k] = (r < d_dn && idx < dup) ? __builtin_nontemporal_load(src + idx) : T(0);
        }
    }
    for (; r < d_dn; r += gridDim.x) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int idx = tid + k * NT;
            if (idx < dup) row[idx] = xr[k];
        }
        __syncthreads();
        const int64_t rn = r + gridDim.x;
        if (rn < d_dn) {
            const T *src = vv + rn * d_up;
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                const int idx = tid + k * NT;
                if (idx < dup) xr[k] = __builtin_nontemporal_load(src + idx);
            }
        }
        const uint32_t bd = sd[r];
        const double edn = ed[r];
        T *wrow = ww + r * d_up;
        for (int c = 0; c < lay.ncls; ++c) {
            const int cl = cls[4 * c], ch = cls[4 * c + 1];
            const int lofs = cls[4 * c + 2], hofs = cls[4 * c + 3];
            const bool fits = cl <= NT;
            const int nteam = fits ? NT / cl : 1;
            const int nq = fits ? 1 : (cl + NT - 1) / NT;
            for (int q = 0; q < nq; ++q) {
                const int lidx = fits ? tid % cl : tid + q * NT;
                const int team = fits ? tid / cl : 0;
                if (team >= nteam || lidx >= cl) continue;
                const uint32_t l = (uint32_t)llist[lofs + lidx];
                const int e0 = looff[l], nlo = looff[l + 1] - e0;
                // packed (int16 label shift | coefficient index << 16); padding
                // entries point at the zero coefficient kept after the table
                uint32_t le[MAXLO];
#pragma unroll
                for (int k = 0; k < MAXLO; ++k)
                    le[k] = k < nlo ? loent[e0 + k] : ((uint32_t)lay.zero_coef << 16);
                int xo[MAXXB];
                int xf[MAXXB];
#pragma unroll
                for (int q2 = 0; q2 < MAXXB; ++q2) {
                    xo[q2] = 0;
                    xf[q2] = 0;
                    if (q2 < lay.nxb) {
                        const int a = xbond[q2] & 255;
                        xo[q2] = rlo[l ^ (1u << a)];
                        xf[q2] = ((l >> a) & 1) | ((__popc(l >> (a + 1)) & 1) << 1);
                    }
                }
                const double el = elo[l];
                for (int g = team; g < ch; g += nteam) {
                    const uint32_t h = (uint32_t)hlist[hofs + g];
                    const int i = hbase[hofs + g] + lidx;
                    const uint32_t dbl = ((h << sp.l_lo) | l) & bd;
                    double diag = el + ehi[h] + edn;
                    if (u_uniform >= 0.0) {
                        diag += u_uniform * (double)__popc(dbl);
                    } else {
                        for (int byte = 0; byte < nbytes; ++byte)
                            diag += ulut[byte * 256 + ((dbl >> (8 * byte)) & 255u)];
                    }
                    double acc = diag * (double)row[i];
#pragma unroll
                    for (int k = 0; k < MAXLO; ++k)
                        if (k < lay.max_lo)
                            acc = fma(coef[le[k] >> 16], (double)row[i + (int)(int16_t)(le[k] & 0xffffu)],
                                      acc);
                    for (int e = hioff[h], e1 = hioff[h + 1]; e < e1; ++e) {
                        const uint64_t ent = hient[e];
                        acc = fma(coef[(uint32_t)(ent >> 32)], (double)row[i + (int)(uint32_t)ent], acc);
                    }
#pragma unroll
                    for (int q2 = 0; q2 < MAXXB; ++q2) {
                        if (q2 < lay.nxb) {
                            const uint64_t ent = xtab[(size_t)h * lay.nxb + q2];
                            const uint32_t meta = (uint32_t)(ent >> 32);
                            // valid, and the low end in the state the direction needs
                            if ((meta & 1u) && ((xf[q2] & 1) != (int)((meta >> 1) & 1u))) {
                                const int tgt = (int)(uint32_t)ent + xo[q2];
                                const int sg = (int)((meta >> 2) & 1u) ^ (xf[q2] >> 1);
                                const double c = coef[2 * (xbond[q2] >> 8) + sg];
                                acc = fma(c, (double)row[tgt], acc);
                            }
                        }
                    }
                    __builtin_nontemporal_store((T)acc, wrow + i);
                }
            }
        }
    }
}

// pass B of the team layout: W += K_dn V on column slabs, hopping lists
// row-contiguous and wave-uniform (scalar loads), 8 neighbour segments in
// flight per wave.  When d_up is even a lane takes two adjacent columns
// (one 2-element load per neighbour), which halves the load instructions.  Within a slab the rows are taken in row_order: grouped by
// the popcount of the high half of the down string.  Hops inside either half
// keep that popcount, so the rows an XCD has in flight find most of their
// neighbour segments among rows of the same group, a working set that fits
// its L2 (4,900 rows x 512 B for the 4x4 FP64 slab of the largest group).
// Row-major list of the down hops of every row, as element offsets of the
// neighbour row (j_dn * d_up) and coefficients, padded to the width W.
__global__ void k_row_offsets(int64_t d_dn, int W, int64_t d_up, const int32_t *__restrict__ col,
                              int64_t *__restrict__ off) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < d_dn * W) off[e] = (int64_t)col[e] * d_up;
}

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

template <typename T, int RI, int CW>
__global__ void __launch_bounds__(256) k_hv_down_acc(
    const int64_t d_up, const int64_t d_dn, const int W, const int32_t *__restrict__ nhd,
    const int64_t *__restrict__ offs, const double *__restrict__ cfd, const T *__restrict__ v,
    T *__restrict__ w, const int R, const int64_t nrb, const int64_t total, const int64_t per,
    const int32_t *__restrict__ order) {
    typedef typename Pair<T>::type T2;
    const int64_t p = blockIdx.x;
    const int64_t lg = (p & 7) * per + (p >> 3);  // XCD p % 8 takes a contiguous range
    if (lg >= total) return;
    const int64_t slab = lg / nrb, rb = lg - slab * nrb;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t c0 = slab * (64 * CW) + lane * CW;
    const bool cok = c0 < d_up;
    const int64_t vb = (int64_t)blockIdx.y * d_up * d_dn;
    const T *vv = v + vb;
    T *ww = w + vb;
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
                T2 a2 = (ok && cok) ? *reinterpret_cast<const T2 *>(ww + rr[q] * d_up + c0) : T2{};
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
                const int64_t *ol = offs + rr[q] * W;
                const double *cl = cfd + rr[q] * W;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool ok = s0 + u < nh[q];
                    const int64_t jo = ok ? ol[s0 + u] : 0;
                    cf[q][u] = ok ? cl[s0 + u] : 0.0;
                    if (CW == 2) {
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
                    if (CW == 2) {
                        T2 o2;
                        o2.x = (T)acc[q][0];
                        o2.y = (T)acc[q][CW - 1];
                        *reinterpret_cast<T2 *>(ww + rr[q] * d_up + c0) = o2;
                    } else {
                        ww[rr[q] * d_up + c0] = (T)acc[q][0];
                    }
                }
        }
    }
}

// ---------------------------------------------------------------- set-up and launch

int build_split_tables(const qcm_model *m, int N, Carver &cv, SplitTables *st, hipStream_t s) {
    HostSplit H;
    if (!make_host_split(m, N, H)) return fail(QCM_EARG, "split tables do not apply");
    SplitLayout lay = layout_of(H);
    st->l_lo = H.l_lo;
    st->l_hi = H.l_hi;
    st->nbond = H.nb;
    st->lay = lay;
    st->blob = cv.take<unsigned char>(lay.bytes, 256);
    if (!cv.base) return QCM_OK;
    std::vector<unsigned char> hb(lay.bytes, 0);
    auto cp = [&](int32_t off, const void *src, size_t n) {
        if (n) memcpy(hb.data() + off, src, n);
    };
    cp(lay.off_coef, H.coef.data(), 8 * H.coef.size());
    cp(lay.off_elo, H.e_lo.data(), 8 * H.e_lo.size());
    cp(lay.off_ehi, H.e_hi.data(), 8 * H.e_hi.size());
    cp(lay.off_hient, H.hi_ent.data(), 8 * H.hi_ent.size());
    cp(lay.off_rlo, H.rlo.data(), 4 * H.rlo.size());
    cp(lay.off_looff, H.lo_off.data(), 4 * H.lo_off.size());
    cp(lay.off_hioff, H.hi_off.data(), 4 * H.hi_off.size());
    cp(lay.off_loent, H.lo_ent.data(), 4 * H.lo_ent.size());
    cp(lay.off_xtab, H.xtab.data(), 8 * H.xtab.size());
    cp(lay.off_cls, H.cls.data(), 4 * H.cls.size());
    cp(lay.off_llist, H.llist.data(), 4 * H.llist.size());
    cp(lay.off_hlist, H.hlist.data(), 4 * H.hlist.size());
    cp(lay.off_hbase, H.hbase.data(), 4 * H.hbase.size());
    cp(lay.off_xbond, H.xbond.data(), 4 * H.xbond.size());
    QCM_HIP(hipMemcpyAsync(st->blob, hb.data(), lay.bytes, hipMemcpyHostToDevice, s));
    return QCM_OK;
}

size_t hv2_lds_bytes(const SplitTables &st, int prec, int64_t d_up, int nbytes, double u_uniform) {
    size_t s = prec == QCM_FP64 ? 8 : 4;
    size_t lut = u_uniform >= 0.0 ? 0 : 8 * 256 * (size_t)nbytes;
    return (size_t)st.lay.bytes + lut + s * d_up;
}



template <typename T, int KS, int MAXLO, int MAXXB>
static void launch_team(dim3 g, size_t lds, hipStream_t s, const HvOp &op, const SplitArgs &sa,
                        const SplitTables &st, const void *v, void *w) {
    k_hv_inrow_team<T, KS, MAXLO, MAXXB><<<g, 1024, lds, s>>>(
        op.up.d, op.dn.d, op.dn.states, op.hd.ediag, op.md.ulut, op.md.nbytes, op.md.u_uniform, sa,
        (const unsigned char *)st.blob, (const T *)v, (T *)w);
}

template <typename T>
static int hv3_launch_t(const HvOp &op, const SplitTables &st, const HopTables &hd_rm,
                        const void *v, void *w, int nvec, hipStream_t s) {
    const int64_t d_up = op.up.d, d_dn = op.dn.d;
    SplitArgs sa;
    sa.l_lo = st.l_lo;
    sa.lo_mask = (1u << st.l_lo) - 1u;
    sa.lay = st.lay;
    const size_t lds = hv2_lds_bytes(st, sizeof(T) == 8 ? QCM_FP64 : QCM_FP32V, d_up,
                                     op.md.nbytes, op.md.u_uniform);
    const int per_cu = lds <= 80 * 1024 ? 2 : 1;
    const int64_t g2x = std::min<int64_t>(d_dn, 256 * per_cu);
    dim3 g2((unsigned)g2x, (unsigned)nvec);
    const int ks = (int)((d_up + 1023) / 1024);
    const int lo = st.lay.max_lo, xb = st.lay.nxb;
    if (ks > 16 || lo > 16 || xb > 16) return fail(QCM_EARG, "team layout does not apply");
    // pass A: in-row term and diagonal, writes W
#define QCM_TEAM(KS_, LO_, XB_)                                                       \
    if (ks <= KS_ && lo <= LO_ && xb <= XB_) {                                         \
        launch_team<T, KS_, LO_, XB_>(g2, lds, s, op, sa, st, v, w);                   \
    } else
    QCM_TEAM(4, 8, 4) QCM_TEAM(4, 8, 8) QCM_TEAM(4, 12, 16) QCM_TEAM(8, 8, 8) QCM_TEAM(8, 12, 16)
    QCM_TEAM(13, 12, 4) QCM_TEAM(16, 12, 4) QCM_TEAM(16, 12, 8) QCM_TEAM(16, 16, 16) {}
#undef QCM_TEAM
    QCM_LAUNCH_CHECK();
    // pass B: row mixing, accumulates into W
    const int R = 16;
    const int cw = (d_up % 2 == 0) ? 2 : 1;
    const int64_t nslab = (d_up + 64 * cw - 1) / (64 * cw);
    const int64_t nrb = (d_dn + R - 1) / R;
    const int64_t total = nslab * nrb;
    const int64_t per = (total + 7) / 8;
    dim3 g1((unsigned)(8 * per), (unsigned)nvec);
    if (cw == 2)
        k_hv_down_acc<T, 2, 2><<<g1, 256, 0, s>>>(d_up, d_dn, hd_rm.width, hd_rm.nh, hd_rm.off,
                                                  hd_rm.coef, (const T *)v, (T *)w, R, nrb, total,
                                                  per, op.row_order);
    else
        k_hv_down_acc<T, 2, 1><<<g1, 256, 0, s>>>(d_up, d_dn, hd_rm.width, hd_rm.nh, hd_rm.off,
                                                  hd_rm.coef, (const T *)v, (T *)w, R, nrb, total,
                                                  per, op.row_order);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

int hv3_launch(const HvOp &op, const SplitTables &st, const HopTables &hd_rm, int prec,
               const void *v, void *w, int nvec, hipStream_t s) {
    if (prec == QCM_FP64) return hv3_launch_t<double>(op, st, hd_rm, v, w, nvec, s);
    return hv3_launch_t<float>(op, st, hd_rm, v, w, nvec, s);
}


int build_row_offsets(HopTables &ht, int64_t d_up, Carver &cv, hipStream_t s) {
    ht.off = cv.take<int64_t>((size_t)ht.width * ht.d);
    if (!cv.base) return QCM_OK;
    const int64_t n = (int64_t)ht.width * ht.d;
    k_row_offsets<<<ceil_div(n, 256), 256, 0, s>>>(ht.d, ht.width, d_up, ht.col, ht.off);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}


// ---------------------------------------------------------------- dispatch

static_assert(sizeof(SplitLayout) <= sizeof(((HvOp *)nullptr)->split_lay), "layout size");

bool split_applies(const qcm_model *m, int n_up, int64_t d_up, int64_t d_dn) {
    if (d_up < 4096 || d_up > 16 * 1024 || d_dn < 1) return false;
    HostSplit H;
    if (!make_host_split(m, n_up, H)) return false;
    SplitLayout lay = layout_of(H);
    if (lay.max_lo > 16 || lay.nxb > 16) return false;
    // FP64 rows must fit in LDS beside the tables and the U lookup table
    const size_t lut = 8 * 256 * (size_t)((m->L + 7) / 8);
    return (size_t)lay.bytes + lut + 8 * (size_t)d_up <= 160 * 1024;
}

size_t split_bytes(const qcm_model *m, int n_up, int64_t d_up, int64_t d_dn) {
    HostSplit H;
    if (!make_host_split(m, n_up, H)) return 0;
    size_t W = count_bonds(m) < 1 ? 1 : count_bonds(m);
    Carver cv(nullptr);
    cv.take<unsigned char>(layout_of(H).bytes);
    cv.take<int32_t>(d_dn);
    cv.take<int32_t>(W * d_dn);
    cv.take<double>(W * d_dn);
    cv.take<double>(d_dn);
    cv.take<int64_t>(W * d_dn);
    cv.take<int32_t>(d_dn);
    return cv.off + 1024;
}

int split_prepare(const qcm_model *m, HvOp &op, Carver &cv, hipStream_t s) {
    SplitTables st;
    QCM_TRY(build_split_tables(m, op.up.N, cv, &st, s));
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
    }
    op.split = 1;
    op.split_blob = st.blob;
    op.split_lo = st.l_lo;
    memcpy(op.split_lay, &st.lay, sizeof(SplitLayout));
    return QCM_OK;
}

int hv_split_launch(const HvOp &op, int prec, const void *v, void *w, int nvec, hipStream_t s) {
    SplitTables st;
    st.l_lo = op.split_lo;
    st.l_hi = op.up.L - op.split_lo;
    st.nbond = 0;
    memcpy(&st.lay, op.split_lay, sizeof(SplitLayout));
    st.blob = op.split_blob;
    return hv3_launch(op, st, op.hd_rm, prec, v, w, nvec, s);
}



}  // namespace qcm
