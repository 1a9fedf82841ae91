/*
 * qcm.h — C ABI of the MI355X exact-diagonalisation hot path.
 *
 * The library computes, for the cluster Hubbard model in one fixed
 * (N_up, N_dn) sector, the sparse product H.v, the Lanczos ground state, the
 * continued-fraction Green function and the CPT Green function G(k, z), as
 * described in arXiv 2305.18643 (Pyqcm), section "Exact diagonalizations"
 * and section "Cluster perturbation theory".
 *
 * General rules (apply to every call):
 *  - Every call returns an int: QCM_OK (0) on success, a negative QCM_E* code
 *    on failure.  Nothing throws.  qcm_last_error() returns a thread-local
 *    message describing the last failure of the calling thread.
 *  - Arguments are validated before anything is enqueued; on a validation
 *    error no output is touched.  On QCM_EHIP the outputs are undefined.
 *  - "device" pointers are HIP device memory (e.g. torch tensors on the GPU);
 *    "host" pointers are ordinary process memory.  The caller owns every
 *    buffer.  The library never allocates device memory: each call that needs
 *    scratch space takes a device workspace (d_ws, ws_bytes).  Passing
 *    d_ws == NULL asks for the size only: the call writes the number of bytes
 *    it needs to *ws_needed and returns QCM_OK without enqueueing anything.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued on it.  Calls documented as "synchronises" wait
 *    for that stream before returning because they return host results.
 *  - Vector layout: element i of a sector vector is the basis state with
 *    up string B_up(i mod d_up) and down string B_dn(i div d_up), i.e. the
 *    vector is a row-major d_dn x d_up matrix whose rows are indexed by the
 *    down string (subsection "Coding of the basis states").
 *  - Spin strings: bit k of a string is the occupation of orbital k.  The
 *    states of one spin are the strings of popcount N in ascending numeric
 *    order and their label is their position in that list.
 *  - Fermion sign convention: every up creation operator stands to the left of
 *    every down creation operator and, within one spin, orbital order is
 *    ascending (eq. (basis)).
 */
#ifndef QCM_H
#define QCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    QCM_OK = 0,
    QCM_EARG = -1,        /* invalid argument (NULL, bad size, asymmetric t, ...) */
    QCM_ERANGE = -2,      /* L > 32, N > L, sector too large for 32-bit spin labels */
    QCM_EWORKSPACE = -3,  /* workspace smaller than required */
    QCM_EHIP = -4         /* a HIP runtime call failed; message has the HIP error */
};

/* Vector storage precision. */
enum {
    QCM_FP64 = 0,   /* vectors stored and computed in FP64 */
    QCM_FP32V = 1   /* vectors stored in FP32; every product accumulates in FP64,
                       dot products, alpha/beta, reorthogonalisation and the
                       tridiagonal eigenproblem stay FP64 */
};

/* Message for the last failing call on this thread ("" if none). */
const char *qcm_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int qcm_version(void);

/*
 * The cluster (or cluster + bath) Hamiltonian
 *   H = sum_{a,b,sigma} t_ab c+_{a sigma} c_{b sigma} + sum_k U_k n_{k up} n_{k dn}
 * (eq. (Hubbard); eq. (cdmft1) for bath orbitals, which carry U_k = 0).
 * The chemical potential and any bath energy sit on the diagonal of t
 * (t_kk = eps_k - mu).  t must be real symmetric.  Host memory, read during
 * the call only.
 */
typedef struct qcm_model {
    int32_t L;          /* number of orbitals, 1..32 */
    const double *t;    /* host [L*L], row-major, t[a*L+b] = t_ab */
    const double *U;    /* host [L], on-site interaction per orbital */
} qcm_model;

/*
 * A sector (N_up, N_dn) and its look-up tables (subsection "Coding of the
 * basis states": the two-way tables B_sigma and I_sigma).  Filled by
 * qcm_sector_basis; the device pointers point into the workspace given to
 * that call, which the caller must keep alive and unmodified while the basis
 * is in use.  rank tables: label of a string b of popcount N is
 *   rank_lo[b & (2^Llo - 1)] + rank_hi[popc(b & (2^Llo-1)) * 2^Lhi + (b >> Llo)]
 * with Llo = ceil(L/2), Lhi = L - Llo.
 */
typedef struct qcm_basis {
    int32_t L, n_up, n_dn;
    int32_t l_lo, l_hi;
    int64_t d_up, d_dn, dim;            /* dim = d_up * d_dn */
    const uint32_t *states_up;          /* device [d_up], ascending */
    const uint32_t *states_dn;          /* device [d_dn], ascending */
    const int32_t *rank_lo_up, *rank_hi_up;   /* device rank tables, up spin */
    const int32_t *rank_lo_dn, *rank_hi_dn;   /* device rank tables, down spin */
} qcm_basis;

/*
 * qcm_sector_basis — enumerate the sector (n_up, n_dn) of L orbitals on the
 * device: the ascending string lists of each spin and their rank tables
 * (subsection "Coding of the basis states", sector dimension d = d(N_up)
 * d(N_dn) with d(N) = C(L, N)).
 *   L, n_up, n_dn : 1 <= L <= 32, 0 <= n <= L; each C(L, n) < 2^31.
 *   d_ws, ws_bytes: device workspace; holds the tables afterwards.
 *   ws_needed     : host, receives the bytes needed (always written).
 *   out           : host, filled with sizes and device pointers (also when
 *                   d_ws == NULL, with NULL pointers).
 * Errors: QCM_ERANGE for bad L/N, QCM_EWORKSPACE, QCM_EHIP.  Asynchronous.
 */
int qcm_sector_basis(int32_t L, int32_t n_up, int32_t n_dn, void *d_ws, size_t ws_bytes,
                     size_t *ws_needed, qcm_basis *out, void *stream);

/*
 * qcm_hv — w = H v on one sector (eq. (factorized): H = K_up (x) 1 +
 * 1 (x) K_dn + V_int, with the hopping sign (-1)^M t_ab of the subsection
 * "Coding of the basis states" and the interaction counted from
 * b_up & b_dn).
 *   m     : the model; b: a basis from qcm_sector_basis with b->L == m->L.
 *   prec  : QCM_FP64 (d_v, d_w are double[dim]) or QCM_FP32V (float[dim];
 *           accumulation in FP64, one rounding on store).
 *   d_v   : device input vector, not modified.  d_w: device output, must
 *           not overlap d_v.
 *   d_ws  : device workspace for the model-dependent hopping tables.
 * Errors: QCM_EARG (t not symmetric, L mismatch, overlap), QCM_EWORKSPACE,
 * QCM_EHIP.  Asynchronous.
 */
int qcm_hv(const qcm_model *m, const qcm_basis *b, int32_t prec, const void *d_v, void *d_w,
           void *d_ws, size_t ws_bytes, size_t *ws_needed, void *stream);

/*
 * qcm_hv_noalloc — the product of qcm_hv (same kernels, same result bit for
 * bit) for callers that cannot allocate device memory or pass a workspace
 * (tight serving loops, hosts that forbid hipMalloc).  It is not meant for
 * stream capture: the model is copied from host memory on every call, and on
 * sectors with long rows the set-up waits for the stream once.  The hopping
 * tables go to a fixed device-resident array of
 * 32 MiB per GPU that the library holds until the process ends (the first
 * call on a device looks up its address there); the call allocates nothing.
 * Sectors whose tables need more (qcm_hv's size query above 32 MiB; the
 * 16-orbital (8, 8) sector needs about 18 MB) are rejected with
 * QCM_EWORKSPACE before anything is enqueued.
 *   m, b, prec, d_v, d_w, stream: as in qcm_hv.
 * Every call on one GPU rewrites that GPU's array: calls that overlap on one
 * GPU (other streams, other host threads) race and give undefined results;
 * serialise them.  Nothing in the array needs clearing between calls.
 * Errors: QCM_EARG, QCM_EWORKSPACE, QCM_EHIP.  Asynchronous apart from that
 * wait.
 */
int qcm_hv_noalloc(const qcm_model *m, const qcm_basis *b, int32_t prec, const void *d_v,
                   void *d_w, void *stream);

/*
 * Plans: the tables of qcm_hv built once and applied many times.
 * qcm_hv_plan_create builds the model- and sector-dependent tables into d_ws
 * (size query with d_ws == NULL, as everywhere) and returns a host handle;
 * the caller keeps d_ws and the basis alive and unmodified while the plan is
 * used.  qcm_hv_plan_apply computes w = H v for nvec consecutive vectors of
 * length dim (d_v, d_w device, in the plan's precision, not overlapping), the
 * same product and arithmetic as qcm_hv, with no table work.  Asynchronous.
 * qcm_hv_plan_destroy frees the handle (not d_ws).
 */
typedef struct qcm_hv_plan qcm_hv_plan;   /* opaque */
int qcm_hv_plan_create(const qcm_model *m, const qcm_basis *b, int32_t prec, void *d_ws,
                       size_t ws_bytes, size_t *ws_needed, void *stream, qcm_hv_plan **out);
int qcm_hv_plan_apply(const qcm_hv_plan *p, const void *d_v, void *d_w, int32_t nvec,
                      void *stream);
int qcm_hv_plan_destroy(qcm_hv_plan *p);

/* Options of the Lanczos ground-state solver. */
typedef struct qcm_lanczos_opts {
    int32_t max_iter;     /* cap on Lanczos steps (the paper's default is 600) */
    int32_t fixed_steps;  /* >0: run exactly this many steps (fewer only on
                             breakdown) and skip the residual test */
    int32_t want_vector;  /* 1: second pass rebuilding the ground state into d_gs */
    int32_t reorth;       /* 0: none (the paper's recurrence); 1: local
                             reorthogonalisation of each new vector against the
                             two previous ones, FP64 dot products */
    int32_t prec;         /* QCM_FP64 or QCM_FP32V */
    int32_t check_every;  /* residual test every this many steps (>= 1) */
    double tol;           /* stop when beta_M |s_M| <= tol * max(1, |theta_0|) */
    double btol;          /* breakdown when beta < btol * max |alpha| */
    uint64_t seed;        /* SplitMix64 seed of the start vector (when d_v0 == NULL) */
    const void *d_v0;     /* device start vector in the vector precision, or NULL */
} qcm_lanczos_opts;

/* Fill `o` with defaults: max_iter 600, fixed_steps 0, want_vector 1,
 * reorth 0, prec QCM_FP64, check_every 1, tol 1e-12, btol 1e-13, seed 1. */
void qcm_lanczos_default_opts(qcm_lanczos_opts *o);

typedef struct qcm_gs_result {
    double e0;            /* lowest eigenvalue of the Lanczos tridiagonal T_M */
    double residual_est;  /* beta_M * |last component of its eigenvector| */
    double true_residual; /* |H psi - e0 psi| (FP64), when want_vector; else -1 */
    double theta1;        /* second-lowest eigenvalue of T_M (may be a copy of e0
                             created by loss of orthogonality) */
    int32_t n_iter;       /* M, number of Lanczos steps */
    int32_t converged;    /* residual test met (or breakdown) */
    int32_t breakdown;    /* Krylov space exhausted */
    int32_t degenerate_suspect;  /* 1 when theta1 - e0 < 1e-8 max(1, |e0|): the
                             ground state may be degenerate, so the returned
                             vector is one state of a manifold and G built on it
                             is not unique (the paper hands such cases to other
                             methods, subsection "The Lanczos algorithm for the
                             ground state").  Single-vector Lanczos cannot tell
                             a true second eigenvalue from a copy of e0 made by
                             loss of orthogonality (which appears only after e0
                             has converged, e.g. with long fixed_steps runs), nor
                             see a degenerate partner before rounding feeds it
                             in: the flag asks for a closer look (a dense check
                             or a second start vector), it does not decide. */
} qcm_gs_result;

/*
 * qcm_lanczos_gs — lowest eigenpair of H in the sector by the Lanczos
 * recurrence (subsection "The Lanczos algorithm for the ground state",
 * eqs. (Krylov), (LanczosRecursion), (tridiag)), in normalised form:
 * v_0 = x/|x|; w = H v_n - beta_{n-1} v_{n-1}; alpha_n = <v_n, w>;
 * w -= alpha_n v_n; beta_n = |w|; v_{n+1} = w / beta_n.  beta_n^2 is the
 * paper's b_{n+1}^2.  The ground-state vector is rebuilt by a second
 * identical pass, psi = sum_n s_n v_n, and normalised.
 *   Start vector when d_v0 == NULL: x_i = 2 (u_i >> 11) 2^-53 - 1, u_i the
 *   output number i of SplitMix64 seeded with `seed`.
 *   h_alpha, h_beta: host [max(max_iter, fixed_steps)] or NULL; receive
 *   alpha_n and beta_n (beta[n] couples n and n+1).
 *   d_gs  : device double[dim] or NULL; the normalised ground state
 *           (FP64 in both precisions).  Needs want_vector = 1.
 *   h_out : host result.
 * Errors: QCM_EARG, QCM_EWORKSPACE, QCM_EHIP.  Synchronises the stream.
 * Non-convergence is not an error (converged = 0).
 */
int qcm_lanczos_gs(const qcm_model *m, const qcm_basis *b, const qcm_lanczos_opts *o,
                   double *h_alpha, double *h_beta, void *d_gs, qcm_gs_result *h_out,
                   void *d_ws, size_t ws_bytes, size_t *ws_needed, void *stream);

/* Options of the continued-fraction Green function. */
typedef struct qcm_green_opts {
    int32_t n_orb;        /* number of orbitals in `orbs` */
    const int32_t *orbs;  /* host [n_orb], distinct orbitals in [0, L) */
    int32_t max_steps;    /* Lanczos steps per chain (continued-fraction floors) */
    int32_t prec;         /* QCM_FP64 or QCM_FP32V vector storage */
    int32_t reorth;       /* as in qcm_lanczos_opts */
    int32_t pad;
    double btol;          /* chain stops when beta < btol * max |alpha| */
} qcm_green_opts;

/*
 * qcm_green_cf — up-spin zero-temperature Green function G_ij(z), i, j in
 * `orbs`, from Lanczos continued fractions (subsection "The Lanczos
 * algorithm for the Green function", eqs. (green), (GreenCF1), (jacobi)):
 *  - for each pair p = (i <= j): an electron chain from
 *    (c_i + c_j)+ |Omega> in sector (n_up + 1, n_dn) and a hole chain from
 *    (c_i + c_j) |Omega> in (n_up - 1, n_dn) (a single operator if i == j);
 *  - b0^2 = <phi|phi>, then Lanczos from phi/b0 gives a_n, b_n;
 *  - G_e(z) = b0^2/(z + E0 - a_0 - b_1^2/(z + E0 - a_1 - ...)),
 *    G_h(z) = b0^2/(z - E0 + a_0 - b_1^2/(z - E0 + a_1 - ...));
 *  - G_ii = G_e + G_h; G_ij = (G+_ij - G_ii - G_jj)/2 for a real H.
 *   gs    : basis of the ground-state sector; d_gs: device double[gs->dim],
 *           the normalised ground state; e0: its energy.
 *   h_coef: host [n_pairs][2][1 + 2*max_steps] or NULL, pairs ordered
 *           (0,0),(0,1),...,(0,n-1),(1,1),...; part 0 = electron, 1 = hole;
 *           each entry holds b0sq, then a[max_steps], then b2[max_steps]
 *           (b2[n] = b_{n+1}^2 couples floors n and n+1).
 *   h_len : host [n_pairs][2] or NULL, number of floors of each chain.
 *   n_z, h_z: host complex frequencies [n_z] as (re, im) pairs.
 *   d_G   : device complex128 [n_z][n_orb][n_orb] (re, im interleaved).
 * Errors: QCM_EARG, QCM_EWORKSPACE, QCM_EHIP.  Synchronises the stream.
 */
int qcm_green_cf(const qcm_model *m, const qcm_basis *gs, const double *d_gs, double e0,
                 const qcm_green_opts *o, double *h_coef, int32_t *h_len, int32_t n_z,
                 const double *h_z, double *d_G, void *d_ws, size_t ws_bytes, size_t *ws_needed,
                 void *stream);

/* Options of the band Lanczos Green function. */
typedef struct qcm_band_opts {
    int32_t n_orb;        /* p: number of orbitals (start states), 1..32 */
    int32_t pad0;
    const int32_t *orbs;  /* host [n_orb], distinct orbitals in [0, L) */
    int32_t max_basis;    /* basis vectors per part, 1..1024 */
    int32_t prec;         /* QCM_FP64 or QCM_FP32V vector storage */
    double dtol;          /* deflation: candidate norm <= dtol * max(1, max |T_kk|) */
    int32_t max_sweeps;   /* eigenproblem of T: at most max_sweeps * R implicit QR
                             steps in all (40; about 2 R are needed) */
    int32_t pad1;
    double etol;          /* > 0: stop once the lowest eigenvalue of T has moved by at
                             most etol * max(1, |theta|) over one block of n_orb basis
                             vectors (checked when the basis size is a multiple of
                             n_orb); 0: run to max_basis or exhaustion */
} qcm_band_opts;

/* Fill `o` with defaults: max_basis 400, FP64, dtol 1e-10, max_sweeps 40, etol 0
 * (no orbitals). */
void qcm_band_default_opts(qcm_band_opts *o);

/*
 * qcm_green_band — up-spin G_ij(z) for i, j in `orbs` by the band Lanczos
 * method (subsection "The band Lanczos algorithm for the Green function"):
 * for the electron part the start states c+_i |Omega> in (n_up + 1, n_dn),
 * for the hole part c_i |Omega> in (n_up - 1, n_dn); the Krylov space of
 * all start states is built one basis vector at a time, each new vector
 * orthogonalised against the band of previous vectors, redundant candidates
 * deflated, and stopped at max_basis vectors, when no candidate is left, or
 * (etol > 0) when the lowest eigenvalue of T has converged, the paper's rule
 * against orthogonality leaks.
 * The projected Hamiltonian T of each part is diagonalised on the device
 * (Householder reduction to tridiagonal form, then implicit QR steps with
 * Wilkinson shifts, both applied to the start-state projections), giving the
 * Lehmann representation
 *   G_ij(z) = sum_r Qe_ir Qe_jr / (z + E0 - Le_r) + sum_r Qh_ir Qh_jr / (z - E0 + Lh_r),
 * with [Qe Qh][Qe Qh]^T = 1 (the anticommutator).
 *   gs, d_gs, e0: as in qcm_green_cf.
 *   h_R     : host int32 [2] or NULL, basis size of each part (0 if the sector
 *             does not exist or every start state vanishes).
 *   h_lambda: host [2][max_basis] or NULL, Lambda of each part (first R used).
 *   h_Q     : host [2][n_orb][max_basis] or NULL, Q of each part.
 *   n_z, h_z, d_G: as in qcm_green_cf (device complex128 [n_z][n_orb][n_orb]).
 * Workspace: 3 n_orb + 3 vectors per part plus one max_basis^2 FP64 matrix
 * (two with etol > 0).
 * With etol > 0 the stopping tests run on a side stream (default priority,
 * waiting on `stream` through events) with 8 bytes of pinned host memory; the
 * library creates one such set per device the first time it is needed (one
 * more per concurrent caller) and reuses it for the life of the process.  The
 * result is the same as with the tests in order on `stream`.
 * Errors: QCM_EARG (also when the QR steps run out, which takes a non-finite
 * T), QCM_EWORKSPACE, QCM_EHIP.  Synchronises the stream.
 */
int qcm_green_band(const qcm_model *m, const qcm_basis *gs, const double *d_gs, double e0,
                   const qcm_band_opts *o, int32_t *h_R, double *h_lambda, double *h_Q,
                   int32_t n_z, const double *h_z, double *d_G, void *d_ws, size_t ws_bytes,
                   size_t *ws_needed, void *stream);

/*
 * qcm_lehmann_form — the Lehmann representation of eq. (spectral1) from the
 * output of qcm_green_band: the poles measured from the ground-state energy,
 *   electron r < R_e:  w_r = Lambda_e[r] - e0,   Q[:, r]       = Q_e[:, r],
 *   hole     r < R_h:  w_{R_e + r} = e0 - Lambda_h[r], Q[:, R_e + r] = Q_h[:, r],
 * so that G_ij(z) = sum_r Q_ir Q_jr / (z - w_r).
 *   n_orb, max_basis: as passed to qcm_green_band; h_R, h_lambda, h_Q: its
 *   host outputs ([2], [2][max_basis], [2][n_orb][max_basis]).
 *   h_poles: host [h_R[0] + h_R[1]]; h_Qout: host [n_orb][h_R[0] + h_R[1]].
 * Host arithmetic only (no device work).  Errors: QCM_EARG (NULL pointer,
 * R outside [0, max_basis]).
 */
int qcm_lehmann_form(int32_t n_orb, int32_t max_basis, double e0, const int32_t *h_R,
                     const double *h_lambda, const double *h_Q, double *h_poles, double *h_Qout);

/* An inter-cluster hopping term for CPT: amplitude t between site i of the
 * cluster at the origin and site j of the cluster at shift[0] E1 +
 * shift[1] E2 + shift[2] E3.  Its Hermitian partner is implied. */
typedef struct qcm_bond {
    int32_t i, j;
    int32_t shift[3];
    int32_t pad;
    double t;
} qcm_bond;

/*
 * qcm_cpt_gk — CPT Green function with G-scheme periodisation (section
 * "Cluster perturbation theory", eqs. (CPT1), (CPT3)):
 *   V(k)_ij = sum_bonds t exp(i k.r) (+ Hermitian partner), r = shift.E,
 *   G(k, z) = (G_c(z)^-1 - V(k))^-1,
 *   G_per(k, z) = (1/L) sum_ij exp(-i k.(R_i - R_j)) G_ij(k, z),
 * with the partial Fourier convention of subsection "Partial Fourier
 * transforms".
 *   L     : cluster sites (<= 32); n_z: frequencies; d_Gc: device complex128
 *           [n_z][L][L], the cluster Green function (e.g. from qcm_green_cf).
 *   h_R   : host int32 [L][3] site positions; h_E: host int32 [3][3]
 *           super-lattice vectors (rows).
 *   n_bonds, h_bonds: host inter-cluster bonds.
 *   n_k, h_k: host double [n_k][3], wave-vectors in units of 2 pi.
 *   d_Gper: device complex128 [n_k][n_z].
 *   d_ws  : device workspace.
 * Errors: QCM_EARG, QCM_EWORKSPACE, QCM_EHIP.  Asynchronous.
 */
int qcm_cpt_gk(int32_t L, int32_t n_z, const double *d_Gc, const int32_t *h_R,
               const int32_t *h_E, int32_t n_bonds, const qcm_bond *h_bonds, int32_t n_k,
               const double *h_k, double *d_Gper, void *d_ws, size_t ws_bytes,
               size_t *ws_needed, void *stream);

/* ------------------------------------------------------------------------
 * CDMFT self-consistency (section "Cellular dynamical mean-field theory",
 * subsection "The CDMFT self-consistent procedure").  The impurity (cluster
 * of L sites plus n_bath bath orbitals, eq. (cdmft1)) is solved with
 * qcm_lanczos_gs and qcm_green_cf on the cluster orbitals; these two calls
 * take the cluster Green function from there to the new bath.
 *
 * The bath: theta[mu][alpha] (cluster site mu, bath orbital alpha) and
 * eps[alpha]; the hybridization function (eq. (hybridization)) is
 *   Gamma(z) = sum_alpha theta[:, alpha] theta[:, alpha]^T / (z - eps_alpha).
 * tcp is the cluster hopping with -mu on its diagonal.  Inter-cluster bonds
 * use qcm_bond with the shift in units of the super-lattice vectors and the
 * phase exp(2 pi i k.shift) (k in units of 2 pi in the reciprocal basis of
 * the super-lattice), the Hermitian partner added.
 * ------------------------------------------------------------------------ */

/* Largest cluster and bath handled by the CDMFT calls. */
#define QCM_CDMFT_MAX_L 8
#define QCM_CDMFT_MAX_BATH 16
#define QCM_CDMFT_MAX_PAR 32

/*
 * qcm_cdmft_g0inv — from the cluster Green function G_c(z_n) of the impurity:
 *   Sigma_c(z) = z - tcp - Gamma(z) - G_c(z)^-1,
 *   Gbar(z)    = (1/n_k) sum_k [z - tcp - V(k) - Sigma_c(z)]^-1 (super-lattice
 *                average; V(k) from the bonds),
 *   calG0(z)^-1 = Gbar(z)^-1 + Sigma_c(z).
 *   L (1..8), n_bath (0..16); h_tcp: host [L][L]; h_theta: host [L][n_bath];
 *   h_eps: host [n_bath]; n_bonds, h_bonds: host inter-cluster bonds;
 *   n_k >= 1, h_k: host double [n_k][3]; n_z, h_z: host complex [n_z] (re, im).
 *   d_Gc: device complex128 [n_z][L][L] (as qcm_green_cf writes it).
 *   d_sigma, d_gbar, d_g0inv: device complex128 [n_z][L][L] (d_sigma and
 *   d_gbar may be NULL).  Each output is a fixed-order sum: it depends only
 *   on the inputs.
 * Errors: QCM_EARG (also for a singular matrix: the message names it),
 * QCM_EWORKSPACE, QCM_EHIP.  Synchronises the stream.
 */
int qcm_cdmft_g0inv(int32_t L, int32_t n_bath, const double *h_tcp, const double *h_theta,
                    const double *h_eps, int32_t n_bonds, const qcm_bond *h_bonds, int32_t n_k,
                    const double *h_k, int32_t n_z, const double *h_z, const double *d_Gc,
                    double *d_sigma, double *d_gbar, double *d_g0inv, void *d_ws,
                    size_t ws_bytes, size_t *ws_needed, void *stream);

/*
 * qcm_cdmft_fit — the bath parameters p (n_par, 1..32) that minimise the
 * distance function (eq. (dist_func))
 *   d(p) = sum_n w_n || z_n - tcp - Gamma(z_n; p) - calG0^-1(z_n) ||_F^2,
 * with eps = A_eps p and theta = A_theta p (linear maps from the parameters,
 * so that symmetry-related bath entries share a parameter).  BFGS from the
 * given p, with the analytic gradient and a backtracking (Armijo) line
 * search, on the device in one workgroup, until max_j |dd/dp_j| <= gtol, a
 * step no longer lowers d by more than 1e-15 d, the trial step falls below
 * 1e-15 max(1, |p|) (the resolution of FP64), or max_iter steps.
 *   h_A_eps: host [n_bath][n_par]; h_A_theta: host [L * n_bath][n_par]
 *   (row mu * n_bath + alpha); h_tcp, n_z, h_z: as above; h_w: host [n_z]
 *   weights; d_g0inv: device complex128 [n_z][L][L] (from qcm_cdmft_g0inv).
 *   h_p: host [n_par], start in, minimiser out; h_dist: host, d at the
 *   result; h_iters: host, BFGS steps taken (negative if the line search
 *   failed: h_p then holds the best point found).
 * Errors: QCM_EARG, QCM_EWORKSPACE, QCM_EHIP.  Synchronises the stream.
 */
int qcm_cdmft_fit(int32_t L, int32_t n_bath, int32_t n_par, const double *h_A_eps,
                  const double *h_A_theta, const double *h_tcp, int32_t n_z, const double *h_z,
                  const double *h_w, const double *d_g0inv, double *h_p, double gtol,
                  int32_t max_iter, double *h_dist, int32_t *h_iters, void *d_ws, size_t ws_bytes,
                  size_t *ws_needed, void *stream);

/*
 * qcm_vca_omega — the Potthoff functional of a cluster reference system by
 * the analytic pole formula (subsection "Practical calculation of the
 * Potthoff functional", eq. (omega4)), both spins:
 *   Omega = E0 + 2 [ (1/n_k) sum_k sum_{w_r(k) < 0} w_r(k) - sum_{w'_r < 0} w'_r ],
 * where w'_r are the poles of the reference's up-spin G' in its Lehmann form
 * (eq. (spectral1): electron poles Lambda_e - E0, hole poles E0 - Lambda_h,
 * e.g. from qcm_green_band) with residues Q, and w_r(k) the eigenvalues of
 *   L(k) = diag(w') + Q^T V(k) Q,
 * V(k) = dt + the inter-cluster hopping at k (bonds as for qcm_cdmft_g0inv,
 * phase exp(2 pi i k.shift)); dt is the lattice's intra-cluster one-body
 * matrix minus the reference's.  Each L(k) (complex Hermitian) is
 * diagonalised on the device (one workgroup per k, parallel Jacobi in LDS on
 * its real 2R x 2R form); the k average is a fixed-order sum.
 *   L: cluster sites (1..8); R: poles (1..64); h_poles: host [R];
 *   h_Q: host [L][R]; h_dt: host [L][L]; n_bonds, h_bonds; n_k >= 1,
 *   h_k: host [n_k][3]; e0: the reference's ground-state energy.
 *   h_omega: host, the functional; h_per_k: host [n_k] or NULL, the sum of
 *   the negative w_r(k) of each k (one spin).
 * Errors: QCM_EARG, QCM_ERANGE, QCM_EWORKSPACE, QCM_EHIP.  Synchronises the
 * stream.
 */
#define QCM_VCA_MAX_R 64
int qcm_vca_omega(int32_t L, int32_t R, const double *h_poles, const double *h_Q,
                  const double *h_dt, int32_t n_bonds, const qcm_bond *h_bonds, int32_t n_k,
                  const double *h_k, double e0, double *h_omega, double *h_per_k, void *d_ws,
                  size_t ws_bytes, size_t *ws_needed, void *stream);

/*
 * qcm_vca_omega_quad — the same functional by the frequency integral of
 * eq. (sef4) along the imaginary axis (its numerical form):
 *   Omega = e0 + 2 mean_k [ -(1/pi) int_0^inf Re ln det(1 - V(k) G'(iw)) dw
 *                           + tr V(k) / 2 ],
 * with G'(iw) = Q diag(1/(iw - poles)) Q^T; Re ln det(1 - X), X = V G', comes
 * from the LU factors of 1 - X, or from -sum_n Re tr(X^n)/n where
 * |X|_F <= 1/4 (there the determinant is 1 - O(|X|^2) and would lose the
 * result to rounding).  Global adaptive Gauss-Kronrod
 * (7, 15) quadrature on w = c x / (1 - x), x in [0, 1), c = max(1, max |pole|),
 * starting from 8 equal intervals: each round bisects every interval whose
 * error estimate |K15 - G7| is at least a quarter of the largest, until the sum
 * of the estimates is at most max(rtol |integral|, 1e-15 n_k) or max_intervals
 * is reached.  Its cost grows as R (pole sum) and n_k L^3 per node, not R^3,
 * so it suits reference systems with many poles.
 *   arguments as in qcm_vca_omega, with 1 <= R <= QCM_VCA_QUAD_MAX_R, and
 *   rtol         : relative tolerance of the integral (> 0);
 *   max_intervals: 8..65536;
 *   h_omega      : host, receives Omega;
 *   h_err        : host or NULL, the error estimate carried into Omega;
 *   h_intervals  : host or NULL, the number of intervals at the end.
 * Errors: QCM_ERANGE, QCM_EARG (also when 1 - V G' is singular at a node),
 * QCM_EWORKSPACE, QCM_EHIP.  Synchronises the stream.
 */
#define QCM_VCA_QUAD_MAX_R 4096
int qcm_vca_omega_quad(int32_t L, int32_t R, const double *h_poles, const double *h_Q,
                       const double *h_dt, int32_t n_bonds, const qcm_bond *h_bonds, int32_t n_k,
                       const double *h_k, double e0, double rtol, int32_t max_intervals,
                       double *h_omega, double *h_err, int32_t *h_intervals, void *d_ws,
                       size_t ws_bytes, size_t *ws_needed, void *stream);

/* ------------------------------------------------------------------------
 * Symmetry-adapted sectors of an abelian point group with real characters
 * (subsection "Cluster symmetries"; Table 3x4stats).
 *
 * A group element permutes the orbitals, the same way for both spins.  On a
 * basis state it gives g|b> = phi_g(b)|gb>, phi_g(b) the sign of reordering
 * the permuted creation operators of each spin.  In the irrep with characters
 * chi (each +1 or -1) an orbit holds at most one state, the normalised
 * projection of its representative: the orbit member with the smallest
 * label i_up + d_up i_dn.  The representative is kept when the projection
 * does not vanish.  Its stabiliser size m gives |P|b>|^2 = m/|G|.
 *
 * The Hamiltonian is stored.  For a term with H_r|b1> = c |b'>, b2 the
 * representative of b', the element is (eq. (matrixElement))
 *   <b2|H_r|b1> = c S / sqrt(m_b1 m_b2),  S = sum_{g: g b' = b2} chi_g phi_g(b').
 * The terms of one state are summed before being stored (the paper's
 * cancellation step).  Sums of magnitude at most 1e-13 max(|t|, |U|) are
 * dropped.
 *
 * Building a sector's matrix takes three calls, each sized by the previous one:
 *   qcm_sym_sector_build -> dim;
 *   qcm_sym_csr_count    -> representatives, row pointers, nnz;
 *   qcm_sym_csr_fill     -> columns and values.
 * qcm_sym_hv and qcm_sym_lanczos_gs then use the stored matrix.  FP64 only.
 * ------------------------------------------------------------------------ */

#define QCM_SYM_MAX_G 8        /* group order */
#define QCM_SYM_MAX_BONDS 128  /* pairs a < b with t_ab != 0 */

typedef struct qcm_group {
    int32_t n_g;            /* order |G|, 1..QCM_SYM_MAX_G; element 0 is the identity */
    int32_t pad;
    const int32_t *perm;    /* host [n_g * L]: perm[g*L + a] = image of orbital a under g */
    const int32_t *chi;     /* host [n_g]: the irrep's characters, +1 or -1 */
} qcm_group;

typedef struct qcm_sym_sector {
    qcm_basis b;                          /* the full sector (copied; its tables must stay alive) */
    int32_t n_g;
    int32_t pad;
    int32_t chi[QCM_SYM_MAX_G];
    int8_t perm[QCM_SYM_MAX_G * 32];      /* perm[g*32 + a] */
    int64_t dim;                          /* states of the irrep */
    int64_t n_words;                      /* ceil(b.dim / 64) */
    const uint64_t *bits;                 /* device [n_words]: bit i of the full-sector labels
                                             set iff label i is a kept representative */
    const int64_t *base;                  /* device [n_words]: kept representatives below word w */
    const uint32_t *img_up;               /* device [n_g * d_up]: label of g b_up, with bit 31
                                             set when phi_g(b_up) = -1 */
    const uint32_t *img_dn;               /* device [n_g * d_dn]: likewise for down strings */
} qcm_sym_sector;

/* The stored matrix: row k holds the elements <b2|H|b_k> of representative
 * k, columns ascending (H is real symmetric, so row k is also column k). */
typedef struct qcm_sym_csr {
    int64_t dim, nnz;
    const uint32_t *rep;      /* device [dim]: full-sector label of each representative, ascending */
    const int64_t *rowptr;    /* device [dim + 1] */
    const uint32_t *col;      /* device [nnz] */
    const double *val;        /* device [nnz] */
    const uint32_t *packed;   /* device [nnz] or NULL: col | (index into table) << 26, from
                                 qcm_sym_csr_pack; when set, the product reads it instead of
                                 col and val */
    const double *table;      /* device [QCM_SYM_MAX_VALUES] or NULL: the distinct values */
} qcm_sym_csr;

#define QCM_SYM_MAX_VALUES 64

/*
 * qcm_sym_sector_build — the irrep's representatives of a sector.
 *   b     : a basis from qcm_sector_basis, b->dim < 2^32.
 *   g     : the group and irrep (host).  Checked: element 0 is the identity,
 *           every element is a permutation of the b->L orbitals, the set is
 *           closed under composition, and chi is a representation (chi_gh =
 *           chi_g chi_h, values +-1).
 *   d_ws  : device workspace; holds bits, base and the image tables afterwards.
 *   out   : host; filled (dim too) on success.
 * Errors: QCM_EARG, QCM_EWORKSPACE, QCM_EHIP.  Synchronises the stream (dim is
 * read back).
 */
int qcm_sym_sector_build(const qcm_basis *b, const qcm_group *g, void *d_ws, size_t ws_bytes,
                         size_t *ws_needed, qcm_sym_sector *out, void *stream);

/*
 * qcm_sym_csr_count — the representatives and the number of stored
 * elements of each row.
 *   m       : the model, invariant under the group (t_{g(a)g(b)} = t_ab and
 *             U_{g(a)} = U_a, bitwise); at most QCM_SYM_MAX_BONDS bonds.
 *   s       : a sector from qcm_sym_sector_build with s->b.L == m->L.
 *   d_rep   : device uint32 [s->dim], receives the representatives' labels.
 *   d_rowptr: device int64 [s->dim + 1], receives the row pointers.
 *   h_nnz   : host, receives the number of stored elements.
 *   d_ws    : device workspace (prefix-sum partials).
 * Errors: QCM_EARG, QCM_EWORKSPACE, QCM_EHIP.  Synchronises the stream.
 */
int qcm_sym_csr_count(const qcm_model *m, const qcm_sym_sector *s, uint32_t *d_rep,
                      int64_t *d_rowptr, int64_t *h_nnz, void *d_ws, size_t ws_bytes,
                      size_t *ws_needed, void *stream);

/*
 * qcm_sym_csr_fill — the columns and values, into d_col (uint32 [nnz]) and
 * d_val (double [nnz]), device, from the d_rep and d_rowptr of
 * qcm_sym_csr_count with the same model and sector.  Errors: QCM_EARG,
 * QCM_EHIP.  Asynchronous.
 */
int qcm_sym_csr_fill(const qcm_model *m, const qcm_sym_sector *s, const uint32_t *d_rep,
                     const int64_t *d_rowptr, uint32_t *d_col, double *d_val, void *stream);

/*
 * qcm_sym_csr_pack — the stored matrix with one index per value (the paper
 * suggests storing, for each distinct value, only the positions of its
 * elements).  When the matrix holds at most QCM_SYM_MAX_VALUES distinct
 * values and h->dim <= 2^26, writes every element as
 * col | (index of its value) << 26 into d_packed (device uint32 [nnz]) and the
 * distinct values, ascending, into d_table (device double
 * [QCM_SYM_MAX_VALUES]); *h_n_values receives their number.  Otherwise
 * *h_n_values = 0 and nothing is written.  h itself is not modified: set its
 * packed and table fields to use the result.  The packed product reads four
 * bytes per element instead of twelve; it sums the same products in another
 * order than the explicit one (equal up to rounding).
 * Errors: QCM_EARG, QCM_EWORKSPACE, QCM_EHIP.  Synchronises the stream.
 */
int qcm_sym_csr_pack(const qcm_sym_csr *h, uint32_t *d_packed, double *d_table,
                     int32_t *h_n_values, void *d_ws, size_t ws_bytes, size_t *ws_needed,
                     void *stream);

/*
 * qcm_sym_hv — w = H v with the stored matrix, for nvec consecutive FP64
 * vectors of length h->dim (device, not overlapping).  Errors: QCM_EARG,
 * QCM_EHIP.  Asynchronous.
 */
int qcm_sym_hv(const qcm_sym_csr *h, const double *d_v, double *d_w, int32_t nvec, void *stream);

/*
 * qcm_sym_lanczos_gs — the Lanczos ground state of the irrep (the same
 * recurrence, tests, two passes and results as qcm_lanczos_gs, on the stored
 * matrix).  o->prec must be QCM_FP64; d_gs is a device double [h->dim] in the
 * symmetry-adapted basis.  Errors: QCM_EARG, QCM_EWORKSPACE, QCM_EHIP.
 * Synchronises the stream.
 */
int qcm_sym_lanczos_gs(const qcm_sym_csr *h, const qcm_lanczos_opts *o, double *h_alpha,
                       double *h_beta, void *d_gs, qcm_gs_result *h_out, void *d_ws,
                       size_t ws_bytes, size_t *ws_needed, void *stream);

/* ------------------------------------------------------------------------
 * Batched and continuously served solves.
 *
 * A job is a model, a sector and (optionally) a block of orbitals: the
 * engine computes its ground state exactly as qcm_lanczos_gs does (two
 * passes, true residual) and then the Green-function chains of that block as
 * qcm_green_cf does, and evaluates G on the engine's frequency grid.  Many
 * jobs of different sizes are in flight at once: every round advances each
 * admitted job by one Lanczos step, with one set of launches covering all of
 * them.  A job's results depend only on the job (not on the other jobs in
 * flight), and equal those of the single-solve calls with the same options.
 *
 * Memory: the caller hands the engine one device pool at creation; the
 * engine keeps its tables at the start of the pool and gives each admitted
 * job one block of it (first fit), returned when the job completes.  A job is
 * admitted only if a slot and a large enough block are free: this is the
 * admission by memory budget.  The engine also allocates a small pinned host
 * buffer (hipHostMalloc) for its per-round tables, freed by
 * qcm_engine_destroy.  An engine is used by one host thread at a time.
 * Limits: every up-spin sector of a job (N_up and, with orbitals, N_up +- 1)
 * has at most 8192 strings (every sector of up to 15 orbitals qualifies);
 * larger sectors are for the single-solve calls.
 * ------------------------------------------------------------------------ */

typedef struct qcm_engine qcm_engine;   /* opaque */

typedef struct qcm_engine_opts {
    int32_t prec;            /* QCM_FP64 or QCM_FP32V storage of every vector */
    int32_t reorth;          /* local reorthogonalisation in every chain (0/1) */
    int32_t max_iter;        /* ground-state step cap (residual test every step) */
    int32_t gs_fixed_steps;  /* > 0: exactly this many ground-state steps
                                (fewer only on breakdown), no residual test */
    int32_t gf_steps;        /* continued-fraction floors per chain (M_G) */
    int32_t max_jobs;        /* jobs in flight at once (slots), 1..65536 */
    double tol;              /* residual test, as in qcm_lanczos_opts; <= 0: automatic,
                                1e-12 with QCM_FP64 and 1e-7 with QCM_FP32V (FP32
                                storage floors the residual estimate near 1e-7) */
    double btol;             /* breakdown threshold, as in qcm_lanczos_opts */
    int32_t n_z;             /* frequencies of the grid (0: no G evaluation) */
    int32_t pad;
    const double *h_z;       /* host complex [n_z] as (re, im); copied at creation */
} qcm_engine_opts;

/* Defaults: FP32V with reorthogonalisation, max_iter 600, gf_steps 100,
 * automatic tol (0), btol 1e-13, max_jobs 256, no grid. */
int qcm_engine_default_opts(qcm_engine_opts *o);

typedef struct qcm_job {
    qcm_model model;         /* host; copied at submission */
    int32_t n_up, n_dn;      /* ground-state sector */
    int32_t n_orb;           /* orbitals of the G block (0: ground state only) */
    int32_t pad;
    const int32_t *orbs;     /* host [n_orb], distinct; copied */
    uint64_t seed;           /* SplitMix64 seed of the start vector */
    int64_t tag;             /* caller's identifier, returned in the result */
    double *h_G;             /* host complex128 [n_z][n_orb][n_orb] or NULL */
    double *h_coef;          /* host [n_pairs][2][1 + 2*gf_steps] or NULL (layout of
                                qcm_green_cf) */
    int32_t *h_len;          /* host [n_pairs][2] or NULL */
    double *d_psi;           /* device double[dim] or NULL: receives the ground state */
} qcm_job;

typedef struct qcm_job_result {
    int64_t tag;
    double e0, theta1, residual_est, true_residual;   /* as in qcm_gs_result */
    int32_t n_iter, converged, breakdown;
    int32_t status;          /* QCM_OK */
    int64_t bytes;           /* pool bytes the job held */
    int32_t rounds;          /* rounds from admission to completion */
    int32_t degenerate_suspect;  /* as in qcm_gs_result */
} qcm_job_result;

typedef struct qcm_engine_stats {
    int64_t pool_bytes, header_bytes, in_use, peak_in_use, largest_free, rounds;
    int32_t active, finished;   /* jobs in flight; results waiting for poll */
} qcm_engine_stats;

/*
 * qcm_engine_create — an engine over the device pool d_pool (256-byte
 * aligned, pool_bytes long), enqueueing on `stream`.  *out receives the
 * handle.  Errors: QCM_EARG, QCM_EWORKSPACE (pool smaller than the tables),
 * QCM_EHIP.
 */
int qcm_engine_create(const qcm_engine_opts *o, void *d_pool, size_t pool_bytes, void *stream,
                      qcm_engine **out);

/* Waits for the stream, drops unfinished jobs, frees the host side. */
int qcm_engine_destroy(qcm_engine *e);

/* Pool bytes a job would hold under options o (validates the job). */
int qcm_engine_job_bytes(const qcm_engine_opts *o, const qcm_job *j, size_t *bytes);

/*
 * qcm_engine_submit — admit a job: copies it, builds its tables and start
 * vector (enqueued).  QCM_EWORKSPACE if no slot or no pool block is free now
 * (nothing is done; submit again after some jobs complete); QCM_EARG /
 * QCM_ERANGE for an invalid job.  The host buffers h_G, h_coef, h_len and
 * the device buffer d_psi must stay valid until the job's result is polled.
 */
int qcm_engine_submit(qcm_engine *e, const qcm_job *j);

/*
 * qcm_engine_step — run up to `rounds` rounds (stops early when no job is in
 * flight).  Completed jobs have their outputs written and their results
 * queued for qcm_engine_poll.  *n_active (may be NULL) receives the number of
 * jobs still in flight.  Synchronises the stream after every round.  After a
 * QCM_EHIP from a round the engine is unusable (submit and step return
 * QCM_EHIP); destroy it.
 */
int qcm_engine_step(qcm_engine *e, int32_t rounds, int32_t *n_active);

/* Up to max_out completed results, oldest first; *n_out receives the count. */
int qcm_engine_poll(qcm_engine *e, int32_t max_out, qcm_job_result *h_res, int32_t *n_out);

/* Pool occupancy and counters. */
int qcm_engine_info(const qcm_engine *e, qcm_engine_stats *out);

/*
 * qcm_batch_solve — solve n_jobs jobs through an engine built in d_ws,
 * admitting them in order as memory allows, and write result i of job i to
 * h_res[i].  With d_ws == NULL, *ws_needed receives the bytes that hold every
 * job at once (any workspace that holds the engine tables and the largest
 * job works, with fewer jobs in flight).  Synchronises the stream.
 */
int qcm_batch_solve(const qcm_engine_opts *o, int32_t n_jobs, const qcm_job *jobs,
                    qcm_job_result *h_res, void *d_ws, size_t ws_bytes, size_t *ws_needed,
                    void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QCM_H */
