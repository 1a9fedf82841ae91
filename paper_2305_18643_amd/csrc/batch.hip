// Batched and continuously served ED solves: many independent jobs (a model
// and a sector each) in flight on one GPU at once.
//
// A job is one ground-state solve followed by its Green-function chains
// (paper: section "Exact diagonalizations", subsections "The Lanczos
// algorithm for the ground state" and "The Lanczos algorithm for the Green
// function"), run through four phases:
//   GS1  the Lanczos recurrence until the residual test on T_M is met;
//   GS2  the identical recurrence replayed, psi = sum_n s_n v_n, then psi is
//        normalised and its true residual taken;
//   GF   the electron and hole chains of every orbital pair, both parts at
//        once (each part is one multi-chain group in its own sector);
//   end  continued fractions evaluated on the frequency grid, results copied
//        to the caller's host buffers, device memory returned to the pool.
//
// The engine advances every admitted job by one Lanczos step per round.  A
// round is a fixed sequence of launches whatever the number of jobs: each
// launch covers the work of all jobs through a table of groups (one group =
// the chains of one job in one sector) and per-launch prefix sums over the
// groups' blocks, chunks or chains; a workgroup finds its group by binary
// search.  Jobs join and leave between rounds, so a request that arrives
// while others run is admitted as soon as a slot and pool memory are free
// (continuous batching).
//
// Every kernel reproduces, element by element and chunk by chunk, the
// arithmetic of the single-solve path (same FP64 accumulation order in the
// product, same fixed-chunk two-level sums, same tridiagonal solver), so the
// result of a job is bitwise independent of which other jobs share its
// rounds and equals what the single-solve calls return.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <vector>

#include "lanczos_step.h"

namespace qcm {

// Longest row of V a product block stages in LDS (up-spin strings of one
// sector).  Jobs with a longer up-spin sector use the single-solve calls.
constexpr int64_t kMaxRow = 8192;

// ---------------------------------------------------------------- round tables

// per-job end-of-round test and status gathering
struct BCtl {
    int32_t test;   // run the ground-state test on T_m
    int32_t m;
    double tol;
    const double *alpha, *beta;
    double *work, *svec;
    GsStatus *status;
    const int32_t *done0, *done1;
    int32_t n0, n1;
    const int32_t *len0;
};

struct BStat {
    GsStatus gs;
    int32_t all_done;
    int32_t len0;
    int32_t pad[2];
};

// ---------------------------------------------------------------- kernels

__global__ void __launch_bounds__(256) kb_control(const BCtl *__restrict__ C,
                                                  BStat *__restrict__ out) {
    const BCtl &c = C[blockIdx.x];
    if (c.test) tridiag_status_block(c.alpha, c.beta, c.m, c.tol, c.work, c.svec, c.status, false);
    if (threadIdx.x == 0) {
        BStat r;
        r.gs = *c.status;
        int all = 1;
        for (int k = 0; k < c.n0; ++k) all &= c.done0[k] != 0;
        for (int k = 0; k < c.n1; ++k) all &= c.done1[k] != 0;
        r.all_done = all;
        r.len0 = c.len0 ? *c.len0 : 0;
        r.pad[0] = r.pad[1] = 0;
        out[blockIdx.x] = r;
    }
}

// ---------------------------------------------------------------- host side

enum { PH_GS1 = 0, PH_GS2 = 1, PH_GF = 2 };

struct Part {
    int valid = 0;
    SpinTables up{};
    HopTables hu{};
    Engine e{};
};

struct Job {
    qcm_job d{};
    std::vector<double> t, U;
    std::vector<int32_t> orbs, ops, pidx;
    int npairs = 0;
    size_t off = 0, bytes = 0;
    int phase = PH_GS1, n = 0, M = 0, conv = 0, brk = 0;
    int64_t round0 = 0;
    ModelDev md{};
    SpinTables dn{};
    HopTables hd{};
    Part gs, gf[2];
    double *psi = nullptr, *svec = nullptr, *work = nullptr, *dscal = nullptr;
    GsStatus *status = nullptr;
    double *coef = nullptr, *F = nullptr, *G = nullptr;
    int32_t *len = nullptr, *ops_d = nullptr, *pidx_d = nullptr;
    BStat last{};
    // host copies taken at the end
    GsStatus fin_gs{};
    double fin_r2 = 0.0;
};

}  // namespace qcm

using namespace qcm;

struct qcm_engine {
    qcm_engine_opts o{};
    std::vector<double> z;
    char *pool = nullptr;
    size_t pool_bytes = 0, hdr = 0;
    hipStream_t s = nullptr;
    std::map<size_t, size_t> free_;  // offset -> bytes
    size_t in_use = 0, peak = 0;
    int64_t rounds = 0;
    std::vector<Job *> active;
    std::deque<qcm_job_result> finished;
    // round tables: pinned host copy and its device image at the pool start
    char *h_tab = nullptr, *d_tab = nullptr;
    size_t tab_bytes = 0;
    BStat *h_stat = nullptr, *d_stat = nullptr;
    double *d_z = nullptr;
    int max_groups = 0;
    int failed = 0;   // a round failed (HIP error): the engine only accepts destroy
};

namespace qcm {

static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static int check_engine_opts(const qcm_engine_opts *o) {
    if (!o) return fail(QCM_EARG, "engine options are NULL");
    if (o->prec != QCM_FP64 && o->prec != QCM_FP32V)
        return fail(QCM_EARG, "engine: bad prec %d", o->prec);
    if (o->max_iter < 1 && o->gs_fixed_steps < 1)
        return fail(QCM_EARG, "engine: max_iter and gs_fixed_steps both < 1");
    if (o->gf_steps < 1) return fail(QCM_EARG, "engine: gf_steps < 1");
    if (o->max_jobs < 1 || o->max_jobs > 65536)
        return fail(QCM_EARG, "engine: max_jobs %d outside 1..65536", o->max_jobs);
    if (o->n_z < 0 || (o->n_z > 0 && !o->h_z)) return fail(QCM_EARG, "engine: bad frequency grid");
    return QCM_OK;
}

static int gs_limit(const qcm_engine_opts &o) {
    return o.gs_fixed_steps > 0 ? o.gs_fixed_steps : o.max_iter;
}

// table layout inside h_tab / d_tab
struct TabLayout {
    size_t groups, accs, hvb, chb, cnb, acb, ctl, bytes;
};
static TabLayout tab_layout(int max_jobs) {
    TabLayout t;
    const int mg = 2 * max_jobs;
    Carver cv(nullptr);
    t.groups = (cv.take<BGroup>(mg), cv.off - sizeof(BGroup) * mg);
    t.accs = (cv.take<BGroup>(max_jobs), cv.off - sizeof(BGroup) * max_jobs);
    t.hvb = (cv.take<int64_t>(mg + 1), cv.off - sizeof(int64_t) * (mg + 1));
    t.chb = (cv.take<int64_t>(mg + 1), cv.off - sizeof(int64_t) * (mg + 1));
    t.cnb = (cv.take<int64_t>(mg + 1), cv.off - sizeof(int64_t) * (mg + 1));
    t.acb = (cv.take<int64_t>(max_jobs + 1), cv.off - sizeof(int64_t) * (max_jobs + 1));
    t.ctl = (cv.take<BCtl>(max_jobs), cv.off - sizeof(BCtl) * max_jobs);
    t.bytes = round_up(cv.off, 256);
    return t;
}

static size_t header_bytes(const qcm_engine_opts &o) {
    TabLayout t = tab_layout(o.max_jobs);
    return t.bytes + round_up(sizeof(BStat) * o.max_jobs, 256) +
           round_up(sizeof(double) * 2 * (o.n_z > 0 ? o.n_z : 1), 256);
}

static int check_job(const qcm_engine_opts &o, const qcm_job *j) {
    if (!j) return fail(QCM_EARG, "job is NULL");
    QCM_TRY(validate_model(&j->model));
    const int L = j->model.L;
    QCM_TRY(check_sector_args(L, j->n_up, j->n_dn));
    if (j->n_orb < 0 || j->n_orb > L || (j->n_orb > 0 && !j->orbs))
        return fail(QCM_EARG, "job: bad orbital list");
    for (int i = 0; i < j->n_orb; ++i) {
        if (j->orbs[i] < 0 || j->orbs[i] >= L)
            return fail(QCM_EARG, "job: orbital %d out of range", j->orbs[i]);
        for (int k = 0; k < i; ++k)
            if (j->orbs[k] == j->orbs[i]) return fail(QCM_EARG, "job: repeated orbital");
    }
    int nups[3] = {j->n_up, j->n_orb > 0 ? j->n_up + 1 : -1, j->n_orb > 0 ? j->n_up - 1 : -1};
    for (int k = 0; k < 3; ++k) {
        if (nups[k] < 0 || nups[k] > L) continue;
        if (binom(L, nups[k]) > kMaxRow)
            return fail(QCM_ERANGE,
                        "job: up-spin sector of %lld strings exceeds the engine's row limit %lld "
                        "(use the single-solve calls)",
                        (long long)binom(L, nups[k]), (long long)kMaxRow);
    }
    (void)o;
    return QCM_OK;
}

static HvOp part_op(const Job &j, const Part &p) {
    HvOp op;
    op.md = j.md;
    op.up = p.up;
    op.dn = j.dn;
    op.hu = p.hu;
    op.hd = j.hd;
    op.dim = p.up.d * j.dn.d;
    op.split = 0;
    return op;
}

// Lays the job out from cv (sizes only when cv.base is NULL) and, when
// building, enqueues the table construction.
static int job_layout(const qcm_engine_opts &o, Job &j, Carver &cv, hipStream_t s) {
    const qcm_model *m = &j.d.model;
    const int L = m->L;
    const int nb = count_bonds(m);
    const int prec = o.prec;
    QCM_TRY(upload_model(m, cv, &j.md, s));
    QCM_TRY(build_spin_tables(L, j.d.n_dn, cv, &j.dn, s));
    QCM_TRY(build_hop_tables(j.md, j.dn, cv, &j.hd, s, nb));
    QCM_TRY(build_spin_tables(L, j.d.n_up, cv, &j.gs.up, s));
    QCM_TRY(build_hop_tables(j.md, j.gs.up, cv, &j.gs.hu, s, nb));
    j.gs.valid = 1;
    for (int p = 0; p < 2; ++p) {
        Part &q = j.gf[p];
        const int nup2 = p == 0 ? j.d.n_up + 1 : j.d.n_up - 1;
        q.valid = j.npairs > 0 && nup2 >= 0 && nup2 <= L;
        if (!q.valid) continue;
        QCM_TRY(build_spin_tables(L, nup2, cv, &q.up, s));
        QCM_TRY(build_hop_tables(j.md, q.up, cv, &q.hu, s, nb));
    }
    const int64_t dim = j.gs.up.d * j.dn.d;
    const int lim = gs_limit(o);
    j.psi = cv.take<double>(dim);
    j.svec = cv.take<double>(lim);
    j.work = cv.take<double>((size_t)lim * 6);
    j.status = cv.take<GsStatus>(1);
    j.dscal = cv.take<double>(64);
    const int n = j.d.n_orb;
    const int stride = 1 + 2 * o.gf_steps;
    const int nz = o.n_z > 0 ? o.n_z : 1;
    if (j.npairs > 0) {
        j.coef = cv.take<double>((size_t)j.npairs * 2 * stride);
        j.len = cv.take<int32_t>((size_t)j.npairs * 2);
        j.ops_d = cv.take<int32_t>((size_t)j.npairs * 2);
        j.pidx_d = cv.take<int32_t>((size_t)n * n);
        j.F = cv.take<double>(2 * (size_t)nz * j.npairs);
        j.G = cv.take<double>(2 * (size_t)nz * n * n);
    }
    // vectors and chain state: the ground-state chain and the Green-function
    // chains never live at the same time and share one area
    const size_t area = cv.off;
    Carver c1(cv.base);
    c1.off = area;
    QCM_TRY(engine_init(j.gs.e, part_op(j, j.gs), prec, 1, lim, o.btol, o.reorth, c1));
    size_t end = c1.off;
    Carver c2(cv.base);
    c2.off = area;
    for (int p = 0; p < 2; ++p)
        if (j.gf[p].valid)
            QCM_TRY(engine_init(j.gf[p].e, part_op(j, j.gf[p]), prec, j.npairs, o.gf_steps,
                                o.btol, o.reorth, c2));
    cv.off = std::max(end, c2.off);
    if (cv.base && j.npairs > 0) {
        QCM_HIP(hipMemcpyAsync(j.ops_d, j.ops.data(), sizeof(int32_t) * j.ops.size(),
                               hipMemcpyHostToDevice, s));
        QCM_HIP(hipMemcpyAsync(j.pidx_d, j.pidx.data(), sizeof(int32_t) * j.pidx.size(),
                               hipMemcpyHostToDevice, s));
    }
    return QCM_OK;
}

static Job *make_job(const qcm_job *src) {
    Job *j = new Job();
    j->d = *src;
    const int L = src->model.L;
    j->t.assign(src->model.t, src->model.t + (size_t)L * L);
    j->U.assign(src->model.U, src->model.U + L);
    j->d.model.t = j->t.data();
    j->d.model.U = j->U.data();
    const int n = src->n_orb;
    j->orbs.assign(src->orbs, src->orbs + n);
    j->d.orbs = j->orbs.data();
    j->npairs = n * (n + 1) / 2;
    j->ops.assign(2 * (size_t)j->npairs, -1);
    j->pidx.assign((size_t)n * n, 0);
    int p = 0;
    for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b) {
            j->ops[2 * p] = j->orbs[a];
            j->ops[2 * p + 1] = a == b ? -1 : j->orbs[b];
            j->pidx[a * n + b] = p;
            j->pidx[b * n + a] = p;
            ++p;
        }
    return j;
}

static int job_bytes_of(const qcm_engine_opts &o, Job &j, size_t *bytes) {
    Carver cv(nullptr);
    QCM_TRY(job_layout(o, j, cv, nullptr));
    *bytes = round_up(cv.off, 256) + 256;
    return QCM_OK;
}

// ---------------------------------------------------------------- pool

static bool pool_alloc(qcm_engine *E, size_t bytes, size_t *off) {
    for (auto it = E->free_.begin(); it != E->free_.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            size_t rest = it->second - bytes;
            size_t at = it->first + bytes;
            E->free_.erase(it);
            if (rest > 0) E->free_[at] = rest;
            E->in_use += bytes;
            E->peak = std::max(E->peak, E->in_use);
            return true;
        }
    }
    return false;
}

static void pool_free(qcm_engine *E, size_t off, size_t bytes) {
    E->in_use -= bytes;
    auto it = E->free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != E->free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        E->free_.erase(nx);
    }
    if (it != E->free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            E->free_.erase(it);
        }
    }
}

static size_t pool_largest(const qcm_engine *E) {
    size_t m = 0;
    for (auto &kv : E->free_) m = std::max(m, kv.second);
    return m;
}

// ---------------------------------------------------------------- phases

static int start_gs(qcm_engine *E, Job &j, int pass) {
    hipStream_t s = E->s;
    if (pass == 1) QCM_HIP(hipMemsetAsync(j.psi, 0, sizeof(double) * j.gs.e.dim, s));
    QCM_TRY(engine_reset(j.gs.e, s));
    QCM_TRY(engine_seed(j.gs.e, j.d.seed, nullptr, s));
    QCM_TRY(engine_normalize(j.gs.e, s));
    j.phase = pass == 0 ? PH_GS1 : PH_GS2;
    j.n = 0;
    return QCM_OK;
}

static int start_gf(qcm_engine *E, Job &j) {
    hipStream_t s = E->s;
    for (int p = 0; p < 2; ++p) {
        Part &q = j.gf[p];
        if (!q.valid) continue;
        QCM_TRY(engine_reset(q.e, s));
        QCM_TRY(apply_ops_launch(q.e, j.psi, j.gs.up.d, j.gs.up, q.up, p, j.ops_d, s));
        QCM_TRY(engine_normalize_from_partials(q.e, s));
    }
    j.phase = PH_GF;
    j.n = 0;
    return QCM_OK;
}

// end of the ground-state replay: psi normalised, its true residual
static int finish_gs(qcm_engine *E, Job &j) {
    QCM_TRY(psi_finalize(j.gs.e, j.psi, E->s));
    double *w64 = (double *)j.gs.e.vbuf[0];
    QCM_TRY(residual_norm(part_op(j, j.gs), j.psi, j.last.gs.theta0, w64, j.gs.e.partial,
                          j.dscal, E->s));
    return QCM_OK;
}

// enqueue the end of a job: coefficients, G on the grid, copies to the host
static int finish_job(qcm_engine *E, Job &j) {
    hipStream_t s = E->s;
    const int stride = 1 + 2 * E->o.gf_steps;
    if (j.npairs > 0) {
        for (int p = 0; p < 2; ++p)
            QCM_TRY(green_store(j.gf[p].valid ? &j.gf[p].e : nullptr, j.npairs, p, j.coef, j.len,
                                stride, s));
        QCM_TRY(green_eval(j.coef, j.len, j.d.n_orb, E->o.gf_steps, E->o.n_z, E->d_z,
                           j.last.gs.theta0, j.pidx_d, j.F, j.G, s));
        const int n = j.d.n_orb;
        if (j.d.h_G && E->o.n_z > 0)
            QCM_HIP(hipMemcpyAsync(j.d.h_G, j.G, sizeof(double) * 2 * E->o.n_z * n * n,
                                   hipMemcpyDeviceToHost, s));
        if (j.d.h_coef)
            QCM_HIP(hipMemcpyAsync(j.d.h_coef, j.coef, sizeof(double) * j.npairs * 2 * stride,
                                   hipMemcpyDeviceToHost, s));
        if (j.d.h_len)
            QCM_HIP(hipMemcpyAsync(j.d.h_len, j.len, sizeof(int32_t) * j.npairs * 2,
                                   hipMemcpyDeviceToHost, s));
    }
    if (j.d.d_psi)
        QCM_HIP(hipMemcpyAsync(j.d.d_psi, j.psi, sizeof(double) * j.gs.e.dim,
                               hipMemcpyDeviceToDevice, s));
    QCM_HIP(hipMemcpyAsync(&j.fin_gs, j.status, sizeof(GsStatus), hipMemcpyDeviceToHost, s));
    QCM_HIP(hipMemcpyAsync(&j.fin_r2, j.dscal, sizeof(double), hipMemcpyDeviceToHost, s));
    return QCM_OK;
}

static void rotate(Engine &e) {
    int t = e.ivp;
    e.ivp = e.iv;
    e.iv = e.iw;
    e.iw = t;
}

template <typename T>
static int launch_round(qcm_engine *E, int ng, int na, int nc, size_t lds, const TabLayout &tl,
                        const int64_t *hvb, const int64_t *chb, const int64_t *cnb,
                        const int64_t *acb) {
    hipStream_t s = E->s;
    const BGroup *G = (const BGroup *)(E->d_tab + tl.groups);
    const BGroup *A = (const BGroup *)(E->d_tab + tl.accs);
    const TabSrc hv{G, (const int64_t *)(E->d_tab + tl.hvb), ng};
    const TabSrc ch{G, (const int64_t *)(E->d_tab + tl.chb), ng};
    const TabSrc cn{G, (const int64_t *)(E->d_tab + tl.cnb), ng};
    const TabSrc ac{A, (const int64_t *)(E->d_tab + tl.acb), na};
    const BCtl *C = (const BCtl *)(E->d_tab + tl.ctl);
    if (na > 0 && acb[na] > 0) ks_accum<T, TabSrc><<<(unsigned)acb[na], 256, 0, s>>>(ac);
    if (ng > 0) {
        const unsigned nh = (unsigned)hvb[ng], nk = (unsigned)chb[ng], nn = (unsigned)cnb[ng];
        ks_hv<T, TabSrc><<<nh, 256, lds, s>>>(hv);
        // alpha and beta from the product's dots; the direct norm pass only
        // for chains whose beta the dots cannot resolve
        ks_finish<TabSrc><<<nn, 256, 0, s>>>(cn, 3);
        ks_norm<T, TabSrc><<<nk, 256, 0, s>>>(ch, 1);
        ks_finish<TabSrc><<<nn, 256, 0, s>>>(cn, 4);
        ks_update<T, TabSrc><<<nk, 256, 0, s>>>(ch);
    }
    if (nc > 0) kb_control<<<nc, 256, 0, s>>>(C, E->d_stat);
    QCM_LAUNCH_CHECK();
    return QCM_OK;
}

static int complete(qcm_engine *E, Job &j) {
    qcm_job_result r{};
    r.tag = j.d.tag;
    r.e0 = j.fin_gs.theta0;
    r.theta1 = j.fin_gs.theta1;
    r.residual_est = j.fin_gs.est;
    r.true_residual = sqrt(j.fin_r2);
    r.n_iter = j.M;
    r.converged = j.conv;
    r.breakdown = j.brk;
    r.status = QCM_OK;
    r.bytes = (int64_t)j.bytes;
    r.rounds = (int32_t)(E->rounds - j.round0);
    r.degenerate_suspect = degenerate_suspect(j.fin_gs.theta0, j.fin_gs.theta1);
    E->finished.push_back(r);
    pool_free(E, j.off, j.bytes);
    return QCM_OK;
}

// One round: every active job advances one step of its phase.
static int run_round(qcm_engine *E) {
    const qcm_engine_opts &o = E->o;
    const TabLayout tl = tab_layout(o.max_jobs);
    BGroup *G = (BGroup *)(E->h_tab + tl.groups);
    BGroup *A = (BGroup *)(E->h_tab + tl.accs);
    int64_t *hvb = (int64_t *)(E->h_tab + tl.hvb);
    int64_t *chb = (int64_t *)(E->h_tab + tl.chb);
    int64_t *cnb = (int64_t *)(E->h_tab + tl.cnb);
    int64_t *acb = (int64_t *)(E->h_tab + tl.acb);
    BCtl *C = (BCtl *)(E->h_tab + tl.ctl);
    const int lim = gs_limit(o);
    int ng = 0, na = 0, nc = 0;
    size_t lds = 0;
    hvb[0] = chb[0] = cnb[0] = acb[0] = 0;
    auto add_group = [&](const Job &j, const Part &p, bool replay) {
        G[ng] = engine_group(p.e, j.n);
        if (replay) {
            G[ng].psi = j.psi;
            G[ng].svec = j.svec;
        }
        lds = std::max(lds, fused_lds(p.up.d, p.e.rows, o.prec, j.md.nbytes, j.md.u_uniform,
                                      2 * j.md.nbond));
        hvb[ng + 1] = hvb[ng] + (int64_t)p.e.nvec * p.e.nblk;
        chb[ng + 1] = chb[ng] + (int64_t)p.e.nvec * p.e.nchunks;
        cnb[ng + 1] = cnb[ng] + p.e.nvec;
        ++ng;
    };
    for (Job *jp : E->active) {
        Job &j = *jp;
        BCtl &c = C[nc++];
        memset(&c, 0, sizeof c);
        c.status = j.status;
        c.tol = o.tol;
        if (j.phase == PH_GS1) {
            add_group(j, j.gs, false);
            c.test = (o.gs_fixed_steps <= 0) ? 1 : 0;
            c.m = j.n + 1;
            c.alpha = j.gs.e.cs.alpha;
            c.beta = j.gs.e.cs.beta;
            c.work = j.work;
            c.svec = j.svec;
            c.done0 = j.gs.e.cs.done;
            c.n0 = 1;
            c.len0 = j.gs.e.cs.len;
        } else if (j.phase == PH_GS2) {
            // replay: psi += s_n v_n, fused into the step while one follows
            if (j.n + 1 < j.M) {
                add_group(j, j.gs, true);
            } else {
                A[na] = engine_group(j.gs.e, j.n);
                A[na].psi = j.psi;
                A[na].svec = j.svec;
                acb[na + 1] = acb[na] + j.gs.e.nchunks;
                ++na;
            }
        } else {
            for (int p = 0; p < 2; ++p)
                if (j.gf[p].valid) add_group(j, j.gf[p], false);
            if (j.gf[0].valid) {
                c.done0 = j.gf[0].e.cs.done;
                c.n0 = j.npairs;
            }
            if (j.gf[1].valid) {
                c.done1 = j.gf[1].e.cs.done;
                c.n1 = j.npairs;
            }
        }
    }
    QCM_HIP(hipMemcpyAsync(E->d_tab, E->h_tab, tl.bytes, hipMemcpyHostToDevice, E->s));
    if (o.prec == QCM_FP64)
        QCM_TRY(launch_round<double>(E, ng, na, nc, lds, tl, hvb, chb, cnb, acb));
    else
        QCM_TRY(launch_round<float>(E, ng, na, nc, lds, tl, hvb, chb, cnb, acb));
    QCM_HIP(hipMemcpyAsync(E->h_stat, E->d_stat, sizeof(BStat) * nc, hipMemcpyDeviceToHost, E->s));
    QCM_HIP(hipStreamSynchronize(E->s));
    ++E->rounds;

    // transitions, in the order of the single-solve calls
    std::vector<Job *> ending;
    std::vector<Job *> still;
    int k = 0;
    for (Job *jp : E->active) {
        Job &j = *jp;
        j.last = E->h_stat[k++];
        bool ends = false;
        if (j.phase == PH_GS1) {
            rotate(j.gs.e);
            const bool last = j.n + 1 == lim;
            bool stop = false;
            if (j.last.all_done) {
                j.brk = 1;
                j.conv = 1;
                j.M = j.last.len0;
                stop = true;
            } else if (o.gs_fixed_steps <= 0 && j.last.gs.converged) {
                j.conv = 1;
                j.M = j.n + 1;
                stop = true;
            } else if (last) {
                j.M = lim;
                j.conv = o.gs_fixed_steps <= 0 ? j.last.gs.converged : 0;
                stop = true;
            }
            if (stop) {
                QCM_TRY(tridiag_status(j.gs.e.cs.alpha, j.gs.e.cs.beta, j.M, o.tol, j.work,
                                       j.svec, j.status, E->s));
                QCM_TRY(start_gs(E, j, 1));
            } else {
                ++j.n;
            }
        } else if (j.phase == PH_GS2) {
            if (j.n + 1 < j.M) rotate(j.gs.e);
            ++j.n;
            if (j.n == j.M) {
                QCM_TRY(finish_gs(E, j));
                if (j.npairs > 0)
                    QCM_TRY(start_gf(E, j));
                else
                    ends = true;
            }
        } else {
            for (int p = 0; p < 2; ++p)
                if (j.gf[p].valid) rotate(j.gf[p].e);
            ++j.n;
            if (j.n == o.gf_steps || j.last.all_done) ends = true;
        }
        if (ends) {
            QCM_TRY(finish_job(E, j));
            ending.push_back(jp);
        } else {
            still.push_back(jp);
        }
    }
    if (!ending.empty()) {
        QCM_HIP(hipStreamSynchronize(E->s));
        for (Job *jp : ending) {
            QCM_TRY(complete(E, *jp));
            delete jp;
        }
    }
    E->active.swap(still);
    return QCM_OK;
}

}  // namespace qcm

// ---------------------------------------------------------------- C ABI

extern "C" int qcm_engine_default_opts(qcm_engine_opts *o) {
    if (!o) return fail(QCM_EARG, "qcm_engine_default_opts: NULL");
    memset(o, 0, sizeof *o);
    o->prec = QCM_FP32V;
    o->reorth = 1;
    o->max_iter = 600;
    o->gs_fixed_steps = 0;
    o->gf_steps = 100;
    o->tol = 0.0;
    o->btol = 1e-13;
    o->max_jobs = 256;
    o->n_z = 0;
    o->h_z = nullptr;
    return QCM_OK;
}

extern "C" int qcm_engine_create(const qcm_engine_opts *o, void *d_pool, size_t pool_bytes,
                                 void *stream, qcm_engine **out) {
    if (!out) return fail(QCM_EARG, "qcm_engine_create: out is NULL");
    *out = nullptr;
    QCM_TRY(check_engine_opts(o));
    if (!d_pool) return fail(QCM_EARG, "qcm_engine_create: pool is NULL");
    if (((uintptr_t)d_pool) % 256 != 0)
        return fail(QCM_EARG, "qcm_engine_create: pool is not 256-byte aligned");
    const size_t hdr = header_bytes(*o);
    if (pool_bytes < hdr + 256)
        return fail(QCM_EWORKSPACE, "qcm_engine_create: pool %zu < %zu bytes", pool_bytes,
                    hdr + 256);
    qcm_engine *E = new qcm_engine();
    E->o = *o;
    if (!(E->o.tol > 0.0)) E->o.tol = o->prec == QCM_FP64 ? 1e-12 : 1e-7;
    if (o->n_z > 0) E->z.assign(o->h_z, o->h_z + 2 * (size_t)o->n_z);
    E->o.h_z = E->z.data();
    E->pool = (char *)d_pool;
    E->pool_bytes = pool_bytes;
    E->s = as_stream(stream);
    const TabLayout tl = tab_layout(o->max_jobs);
    E->tab_bytes = tl.bytes;
    E->d_tab = E->pool;
    E->d_stat = (BStat *)(E->pool + tl.bytes);
    E->d_z = (double *)(E->pool + tl.bytes + round_up(sizeof(BStat) * o->max_jobs, 256));
    E->hdr = hdr;
    const size_t usable = (pool_bytes - hdr) / 256 * 256;
    E->free_[hdr] = usable;
    hipError_t e1 = hipHostMalloc((void **)&E->h_tab, tl.bytes, hipHostMallocDefault);
    hipError_t e2 = e1 == hipSuccess ? hipHostMalloc((void **)&E->h_stat,
                                                     sizeof(BStat) * o->max_jobs,
                                                     hipHostMallocDefault)
                                     : e1;
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (E->h_tab) (void)hipHostFree(E->h_tab);
        delete E;
        return fail(QCM_EHIP, "qcm_engine_create: pinned host allocation failed: %s",
                    hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    }
    memset(E->h_tab, 0, tl.bytes);
    if (o->n_z > 0) {
        hipError_t e3 = hipMemcpyAsync(E->d_z, E->z.data(), sizeof(double) * 2 * o->n_z,
                                       hipMemcpyHostToDevice, E->s);
        if (e3 != hipSuccess) {
            (void)hipHostFree(E->h_tab);
            (void)hipHostFree(E->h_stat);
            delete E;
            return fail(QCM_EHIP, "qcm_engine_create: %s", hipGetErrorString(e3));
        }
    }
    *out = E;
    return QCM_OK;
}

extern "C" int qcm_engine_destroy(qcm_engine *E) {
    if (!E) return QCM_OK;
    hipError_t e = hipStreamSynchronize(E->s);
    for (Job *j : E->active) delete j;
    if (E->h_tab) (void)hipHostFree(E->h_tab);
    if (E->h_stat) (void)hipHostFree(E->h_stat);
    delete E;
    if (e != hipSuccess) return fail(QCM_EHIP, "qcm_engine_destroy: %s", hipGetErrorString(e));
    return QCM_OK;
}

extern "C" int qcm_engine_job_bytes(const qcm_engine_opts *o, const qcm_job *j, size_t *bytes) {
    if (!bytes) return fail(QCM_EARG, "qcm_engine_job_bytes: bytes is NULL");
    QCM_TRY(check_engine_opts(o));
    QCM_TRY(check_job(*o, j));
    Job *x = make_job(j);
    const int rc = job_bytes_of(*o, *x, bytes);
    delete x;
    return rc;
}

extern "C" int qcm_engine_submit(qcm_engine *E, const qcm_job *j) {
    if (!E) return fail(QCM_EARG, "qcm_engine_submit: engine is NULL");
    if (E->failed) return fail(QCM_EHIP, "qcm_engine_submit: engine failed earlier; destroy it");
    QCM_TRY(check_job(E->o, j));
    if ((int)E->active.size() >= E->o.max_jobs)
        return fail(QCM_EWORKSPACE, "qcm_engine_submit: all %d slots busy", E->o.max_jobs);
    Job *x = make_job(j);
    size_t bytes = 0;
    {
        const int rc = job_bytes_of(E->o, *x, &bytes);
        if (rc != QCM_OK) {
            delete x;
            return rc;
        }
    }
    size_t off = 0;
    if (!pool_alloc(E, bytes, &off)) {
        delete x;
        return fail(QCM_EWORKSPACE, "qcm_engine_submit: job needs %zu bytes, largest free block %zu",
                    bytes, pool_largest(E));
    }
    x->off = off;
    x->bytes = bytes;
    x->round0 = E->rounds;
    Carver cv(E->pool + off);
    int rc = job_layout(E->o, *x, cv, E->s);
    if (rc == QCM_OK) {
        hipError_t e = hipMemsetAsync(x->status, 0, sizeof(GsStatus), E->s);
        if (e != hipSuccess) rc = fail(QCM_EHIP, "qcm_engine_submit: %s", hipGetErrorString(e));
    }
    if (rc == QCM_OK) rc = start_gs(E, *x, 0);
    if (rc != QCM_OK) {
        pool_free(E, off, bytes);
        delete x;
        return rc;
    }
    E->active.push_back(x);
    return QCM_OK;
}

extern "C" int qcm_engine_step(qcm_engine *E, int32_t rounds, int32_t *n_active) {
    if (!E) return fail(QCM_EARG, "qcm_engine_step: engine is NULL");
    if (rounds < 0) return fail(QCM_EARG, "qcm_engine_step: rounds < 0");
    if (E->failed) return fail(QCM_EHIP, "qcm_engine_step: engine failed earlier; destroy it");
    for (int r = 0; r < rounds && !E->active.empty(); ++r) {
        const int rc = run_round(E);
        if (rc != QCM_OK) {
            // jobs stay in `active` (destroy frees them); their device state is
            // undefined after a failed launch or copy
            E->failed = 1;
            return rc;
        }
    }
    if (n_active) *n_active = (int32_t)E->active.size();
    return QCM_OK;
}

extern "C" int qcm_engine_poll(qcm_engine *E, int32_t max_out, qcm_job_result *h_res,
                               int32_t *n_out) {
    if (!E || !n_out || max_out < 0 || (max_out > 0 && !h_res))
        return fail(QCM_EARG, "qcm_engine_poll: bad arguments");
    int k = 0;
    while (k < max_out && !E->finished.empty()) {
        h_res[k++] = E->finished.front();
        E->finished.pop_front();
    }
    *n_out = k;
    return QCM_OK;
}

extern "C" int qcm_engine_info(const qcm_engine *E, qcm_engine_stats *out) {
    if (!E || !out) return fail(QCM_EARG, "qcm_engine_info: bad arguments");
    out->pool_bytes = (int64_t)E->pool_bytes;
    out->header_bytes = (int64_t)E->hdr;
    out->in_use = (int64_t)E->in_use;
    out->peak_in_use = (int64_t)E->peak;
    out->largest_free = (int64_t)pool_largest(E);
    out->rounds = E->rounds;
    out->active = (int32_t)E->active.size();
    out->finished = (int32_t)E->finished.size();
    return QCM_OK;
}

extern "C" int qcm_batch_solve(const qcm_engine_opts *o, int32_t n_jobs, const qcm_job *jobs,
                               qcm_job_result *h_res, void *d_ws, size_t ws_bytes,
                               size_t *ws_needed, void *stream) {
    if (!ws_needed) return fail(QCM_EARG, "qcm_batch_solve: ws_needed is NULL");
    QCM_TRY(check_engine_opts(o));
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(QCM_EARG, "qcm_batch_solve: bad jobs");
    size_t sum = 0, big = 0;
    std::vector<size_t> bytes(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        QCM_TRY(check_job(*o, &jobs[i]));
        Job *x = make_job(&jobs[i]);
        const int rc = job_bytes_of(*o, *x, &bytes[i]);
        delete x;
        if (rc != QCM_OK) return rc;
        sum += bytes[i];
        big = std::max(big, bytes[i]);
    }
    const size_t hdr = header_bytes(*o) + 256;
    *ws_needed = hdr + sum;
    if (!d_ws) return QCM_OK;
    if (!h_res) return fail(QCM_EARG, "qcm_batch_solve: h_res is NULL");
    if (ws_bytes < hdr + big)
        return fail(QCM_EWORKSPACE, "qcm_batch_solve: workspace %zu < %zu (largest job)", ws_bytes,
                    hdr + big);
    qcm_engine *E = nullptr;
    QCM_TRY(qcm_engine_create(o, d_ws, ws_bytes, stream, &E));
    int rc = QCM_OK;
    int next = 0, got = 0;
    std::vector<qcm_job_result> res(64);
    while (got < n_jobs && rc == QCM_OK) {
        // admit in order while the next job fits
        while (next < n_jobs && (int)E->active.size() < E->o.max_jobs &&
               pool_largest(E) >= bytes[next]) {
            qcm_job jj = jobs[next];
            jj.tag = next;
            rc = qcm_engine_submit(E, &jj);
            if (rc != QCM_OK) break;
            ++next;
        }
        if (rc != QCM_OK) break;
        if (E->active.empty()) {
            rc = fail(QCM_EWORKSPACE, "qcm_batch_solve: job %d does not fit the workspace", next);
            break;
        }
        rc = run_round(E);
        while (rc == QCM_OK && !E->finished.empty()) {
            qcm_job_result r = E->finished.front();
            E->finished.pop_front();
            const int idx = (int)r.tag;
            r.tag = jobs[idx].tag;
            h_res[idx] = r;
            ++got;
        }
    }
    int rc2 = qcm_engine_destroy(E);
    return rc != QCM_OK ? rc : rc2;
}
