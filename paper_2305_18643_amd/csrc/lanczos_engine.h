// Multi-chain Lanczos engine shared by the ground-state and Green-function
// entry points (internal).
#pragma once

#include <functional>

#include "qcm_internal.h"

namespace qcm {

// Elements per reduction chunk: the fixed first level of every dot product.
constexpr int kChunk = 8192;

// Per-chain recurrence state, all on the device.  alpha/beta are [nvec][maxs].
struct ChainState {
    int maxs;
    double btol;
    double *alpha, *beta;
    double *amax;   // running max |alpha| per chain
    double *inv;    // 1/beta (or 0 once the chain has stopped), then 1/|phi|
    double *corr, *corr2;   // reorthogonalisation coefficients of the last step
    double *apre;   // alpha of the last step before its reorthogonalisation term
    double *b0sq;   // <phi|phi> of the start vector
    int32_t *len;   // number of steps recorded
    int32_t *done;  // chain stopped (breakdown or empty start)
    int32_t *renorm;  // this step's beta needs the direct norm pass (see ks_finish)
};

struct GsStatus {
    double theta0, theta1, est;
    int32_t converged, M;
};

struct Engine {
    HvOp op;
    int prec, nvec, maxs, reorth, nchunks;
    int64_t dim;
    void *vbuf[3];
    int ivp, iv, iw;
    double *partial;   // [nvec][nchunks]: start-vector and psi norms
    double *pa;        // [nvec][na]: alpha partials of a step
    double *pn;        // [nvec][3][nchunks]: norm partials of a step
    int32_t na, rows, nblk;
    int32_t fused;     // product fused with the first pass (rows fit LDS)
    // Deferred update (two-pass product only): with lazy set, a step leaves
    // the unnormalised w_n in the buffer of v_{n+1} (pending) and the next
    // step's in-row pass forms v_{n+1} while it stages the rows; whatever
    // reads the vectors in between calls engine_settle first.
    int32_t lazy, pending;
    double *scratch;
    ChainState cs;
};

int engine_init(Engine &e, const HvOp &op, int prec, int nvec, int maxs, double btol, int reorth,
                Carver &cv);
int engine_reset(Engine &e, hipStream_t s);
int engine_seed(Engine &e, uint64_t seed, const void *v0, hipStream_t s);
int engine_normalize(Engine &e, hipStream_t s);
int engine_step(Engine &e, int n, hipStream_t s);
int engine_settle(Engine &e, hipStream_t s);
int engine_accum(Engine &e, double *psi, const double *coef, int n, hipStream_t s);
int engine_normalize_from_partials(Engine &e, hipStream_t s);
int psi_finalize(Engine &e, double *psi, hipStream_t s);
// |H psi - theta psi| into *out (device), FP64; w64 holds dim doubles
int residual_norm(const HvOp &op, const double *psi, double theta, double *w64, double *partial,
                  double *out, hipStream_t s);
// Green-function pieces (green.hip)
int apply_ops_raw(int prec, const double *psi, int64_t d_src_up, const SpinTables &src_up,
                  const SpinTables &tgt_up, int64_t dim, int kind, const int32_t *ops, int nvec,
                  void *out, int nchunks, double *partial, hipStream_t s);
int apply_ops_launch(Engine &e, const double *psi, int64_t d_src_up, const SpinTables &src_up,
                     const SpinTables &tgt_up, int kind, const int32_t *ops, hipStream_t s);
int green_store(const Engine *e, int npairs, int part, double *coef, int32_t *len, int stride,
                hipStream_t s);
int green_eval(const double *coef, const int32_t *len, int n, int maxs, int nz, const double *zd,
               double e0, const int32_t *pidx, double *F, double *G, hipStream_t s);
// want1 = 0: skip theta_1 (status->theta1 = NaN); the tests between steps
int tridiag_status(const double *alpha, const double *beta, int M, double tol, double *work,
                   double *svec, GsStatus *status, hipStream_t s, int want1 = 1);
// The ground-state solver of qcm_lanczos_gs over any product: setup carves
// the product's tables (or, without a base, only sizes them) and fills op.
using GsSetup = std::function<int(Carver &, hipStream_t, HvOp *)>;
int gs_run(const char *fn, const GsSetup &setup, int64_t dim, const qcm_lanczos_opts *o,
           double *h_alpha, double *h_beta, void *d_gs, qcm_gs_result *h_out, void *d_ws,
           size_t ws_bytes, size_t *ws_needed, void *stream);

}  // namespace qcm
