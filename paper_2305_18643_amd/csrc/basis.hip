// Sector basis and label tables (paper: section "Exact diagonalizations",
// subsection "Coding of the basis states").
//
// The states of one spin are the L-bit strings of popcount N in ascending
// order; the label of a string is its position, which equals the
// combinatorial-number-system sum  sum_j C(p_j, j+1)  over its set bits
// p_0 < p_1 < ...  The device keeps two small tables that split this sum at
// bit l_lo = ceil(L/2):
//   rank(b) = rank_lo[b_lo] + rank_hi[popc(b_lo)][b_hi]
// so any label costs two table reads, for every L <= 32.
#include <stdarg.h>
#include <stdio.h>

#include "qcm_internal.h"

namespace qcm {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

int fail(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

const char *last_error() { return g_err.c_str(); }

// i-th string (ascending) of popcount N: greedy decomposition of i in the
// combinatorial number system, highest set bit first.
__global__ void k_unrank(int L, int N, int64_t d, uint32_t *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d) return;
    int64_t r = i;
    uint32_t b = 0;
    int p = L - 1;
    for (int k = N; k >= 1; --k) {
        while (binom(p, k) > r) --p;
        b |= 1u << p;
        r -= binom(p, k);
        --p;
    }
    out[i] = b;
}

__global__ void k_rank_lo(int l_lo, int32_t *__restrict__ out) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (int64_t(1) << l_lo)) return;
    int64_t r = 0;
    int j = 0;
    for (int p = 0; p < l_lo; ++p)
        if ((x >> p) & 1) r += binom(p, ++j);
    out[x] = (int32_t)r;
}

__global__ void k_rank_hi(int l_lo, int l_hi, int32_t *__restrict__ out) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t per = int64_t(1) << l_hi;
    if (e >= per * (l_lo + 1)) return;
    int n = (int)(e / per);
    int64_t y = e % per;
    int64_t r = 0;
    int j = 0;
    for (int q = 0; q < l_hi; ++q)
        if ((y >> q) & 1) r += binom(l_lo + q, n + (++j));
    out[e] = (int32_t)r;
}

int check_sector_args(int L, int nup, int ndn) {
    if (L < 1 || L > 32) return fail(QCM_ERANGE, "L=%d outside 1..32", L);
    if (nup < 0 || nup > L || ndn < 0 || ndn > L)
        return fail(QCM_ERANGE, "sector (%d,%d) invalid for L=%d", nup, ndn, L);
    if (binom(L, nup) >= (int64_t(1) << 31) || binom(L, ndn) >= (int64_t(1) << 31))
        return fail(QCM_ERANGE, "spin sector dimension exceeds 2^31-1");
    return QCM_OK;
}

static void split_bits(int L, int *l_lo, int *l_hi) {
    *l_lo = (L + 1) / 2;
    *l_hi = L - *l_lo;
}

size_t spin_tables_bytes(int L, int N) {
    int l_lo, l_hi;
    split_bits(L, &l_lo, &l_hi);
    Carver cv(nullptr);
    cv.take<uint32_t>(binom(L, N));
    cv.take<int32_t>(size_t(1) << l_lo);
    cv.take<int32_t>((size_t)(l_lo + 1) << l_hi);
    return cv.off + 256;
}

int build_spin_tables(int L, int N, Carver &cv, SpinTables *out, hipStream_t s) {
    SpinTables t;
    t.L = L;
    t.N = N;
    split_bits(L, &t.l_lo, &t.l_hi);
    t.d = binom(L, N);
    t.states = cv.take<uint32_t>(t.d);
    t.rank_lo = cv.take<int32_t>(size_t(1) << t.l_lo);
    t.rank_hi = cv.take<int32_t>((size_t)(t.l_lo + 1) << t.l_hi);
    if (cv.base) {
        const int B = 256;
        k_unrank<<<ceil_div(t.d, B), B, 0, s>>>(L, N, t.d, t.states);
        QCM_LAUNCH_CHECK();
        k_rank_lo<<<ceil_div(size_t(1) << t.l_lo, B), B, 0, s>>>(t.l_lo, t.rank_lo);
        QCM_LAUNCH_CHECK();
        k_rank_hi<<<ceil_div((size_t)(t.l_lo + 1) << t.l_hi, B), B, 0, s>>>(t.l_lo, t.l_hi,
                                                                             t.rank_hi);
        QCM_LAUNCH_CHECK();
    }
    *out = t;
    return QCM_OK;
}

void basis_from_tables(const SpinTables &up, const SpinTables &dn, qcm_basis *out) {
    out->L = up.L;
    out->n_up = up.N;
    out->n_dn = dn.N;
    out->l_lo = up.l_lo;
    out->l_hi = up.l_hi;
    out->d_up = up.d;
    out->d_dn = dn.d;
    out->dim = up.d * dn.d;
    out->states_up = up.states;
    out->states_dn = dn.states;
    out->rank_lo_up = up.rank_lo;
    out->rank_hi_up = up.rank_hi;
    out->rank_lo_dn = dn.rank_lo;
    out->rank_hi_dn = dn.rank_hi;
}

SpinTables spin_from_basis(const qcm_basis *b, int spin) {
    SpinTables t;
    t.L = b->L;
    t.N = spin == 0 ? b->n_up : b->n_dn;
    t.l_lo = b->l_lo;
    t.l_hi = b->l_hi;
    t.d = spin == 0 ? b->d_up : b->d_dn;
    t.states = const_cast<uint32_t *>(spin == 0 ? b->states_up : b->states_dn);
    t.rank_lo = const_cast<int32_t *>(spin == 0 ? b->rank_lo_up : b->rank_lo_dn);
    t.rank_hi = const_cast<int32_t *>(spin == 0 ? b->rank_hi_up : b->rank_hi_dn);
    return t;
}

}  // namespace qcm

using namespace qcm;

extern "C" const char *qcm_last_error(void) { return last_error(); }

extern "C" int qcm_version(void) { return 100; }

extern "C" int qcm_sector_basis(int32_t L, int32_t n_up, int32_t n_dn, void *d_ws,
                                size_t ws_bytes, size_t *ws_needed, qcm_basis *out,
                                void *stream) {
    if (!ws_needed || !out) return fail(QCM_EARG, "qcm_sector_basis: NULL ws_needed or out");
    QCM_TRY(check_sector_args(L, n_up, n_dn));
    size_t need = spin_tables_bytes(L, n_up) + spin_tables_bytes(L, n_dn) + 512;
    *ws_needed = need;
    SpinTables up, dn;
    if (!d_ws) {
        Carver cv(nullptr);
        build_spin_tables(L, n_up, cv, &up, nullptr);
        build_spin_tables(L, n_dn, cv, &dn, nullptr);
        basis_from_tables(up, dn, out);
        return QCM_OK;
    }
    if (ws_bytes < need)
        return fail(QCM_EWORKSPACE, "qcm_sector_basis: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = as_stream(stream);
    Carver cv(d_ws);
    QCM_TRY(build_spin_tables(L, n_up, cv, &up, s));
    QCM_TRY(build_spin_tables(L, n_dn, cv, &dn, s));
    basis_from_tables(up, dn, out);
    return QCM_OK;
}
