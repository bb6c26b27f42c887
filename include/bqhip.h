/*
 * bqhip.h -- C ABI of the MI355X (gfx950) library for the hot path of BQCD's
 * Hybrid Monte Carlo (arXiv:1711.03836): the even-odd preconditioned
 * Wilson-clover fermion matrix with chemical potential and the conjugate
 * gradient solve of M^dag M x = b built on it.
 *
 * Operator (Eq. 1 and Eq. 2 of the section on fermion actions):
 *   (M psi)(x) = T(x) psi(x) - kappa (D psi)(x)
 *   (D psi)(x) = sum_mu [ f+_mu(x) U_mu(x)(1 - gamma_mu) psi(x+mu)
 *                       + f-_mu(x) U_mu(x-mu)^dag (1 + gamma_mu) psi(x-mu) ]
 *   with f+-_{x,y,z} = 1, f+_t = e^{+mu}, f-_t = e^{-mu}, times t_bc on hops
 *   that cross the time boundary;
 *   T(x) = 1 + kappa c_SW sum_{mu<nu} sigma_{mu nu} (-i F_{mu nu}(x)),
 *   sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu], F = (Q - Q^dag)/8 from the
 *   four-leaf clover, made traceless; Euclidean chiral basis
 *   (gamma_5 = diag(1,1,-1,-1)), so T is two Hermitian 6x6 blocks per site.
 * Checkerboard storage (the volume/2 arrays of the section on SIMD
 * vectorization): even sites have x1+x2+x3+x4 even.  The Schur system lives
 * on odd sites:  Mhat = T_oo - kappa^2 D_oe T_ee^-1 D_eo.
 * Solver: cg from the solver list of the section on algorithms (Tables 1-2
 * time this solver), with FP32/FP16 inner iterations and FP64 reliable
 * updates as options.
 *
 * Conventions of this ABI
 *   - Every function returns an int: BQ_OK (0) or a negative BQ_ERR_* code;
 *     bq_last_error() returns a thread-local message for the last failure.
 *     No C++ exception crosses the ABI.
 *   - Canonical host layout (C order, complex128 = two doubles re, im):
 *       site index  i = x1 + L1*(x2 + L2*(x3 + L3*x4)), directions 0..3 = x,y,z,t
 *       links       U[mu][i][a][b]             4*V*9 complex
 *       spinors     psi[rhs][i][spin][colour]  nrhs*V*12 complex
 *     A pointer flagged `on_device` is a device pointer (e.g. a torch tensor's
 *     data_ptr) in the same canonical layout; otherwise it is host memory.
 *   - Handles (context, gauge, op, field) are owned by the library until their
 *     *_free / *_destroy call; freeing NULL is a no-op.  Fields hold data in the
 *     library's own device layout (site-tiled checkerboards); bq_field_put /
 *     bq_field_get convert from / to the canonical layout.
 *   - `stream` is a hipStream_t or NULL.  Work is ordered after earlier work on
 *     that stream; NULL selects the context's own stream (a non-blocking stream:
 *     work on the device's null stream is not waited for, so a caller whose
 *     data comes from the null stream synchronizes it first).  bq_apply is
 *     asynchronous on that stream; every other call returns when its results
 *     are complete.
 *   - All lattice extents must be even and >= 2, with fewer than 2^24 sites
 *     per parity (V/2 < 16777216; 48^3x96 has 5.3 M, 64^3x120 has 15.7 M);
 *     BQ_ERR_INVALID otherwise.
 *   - A context is not thread-safe: one host thread per context at a time.
 */
#ifndef BQHIP_H
#define BQHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BQ_OK 0
#define BQ_PENDING 1                /* bq_server_result: the request is still queued or running */
#define BQ_ERR_INVALID (-1)         /* bad argument: NULL, odd or < 2 extent, nrhs < 1, tol <= 0, mismatch */
#define BQ_ERR_OOM (-2)             /* HBM budget exceeded or device allocation failed */
#define BQ_ERR_NOT_CONVERGED (-3)   /* maxiter reached; x holds the last iterate, info is filled */
#define BQ_ERR_NONFINITE (-4)       /* NaN/Inf met in the source or during the solve */
#define BQ_ERR_CLOVER_NOT_HPD (-5)  /* a clover block is not positive definite (kappa c_SW too large) */
#define BQ_ERR_BUSY (-6)            /* freeing a gauge field that live operators still use */
#define BQ_ERR_DEVICE (-7)          /* a HIP runtime call failed */
#define BQ_ERR_UNSUPPORTED (-8)     /* valid request this library version does not provide */

enum { BQ_F64 = 0, BQ_F32 = 1, BQ_F16 = 2 };            /* storage precision of a field / inner solve */
enum { BQ_EVEN = 0, BQ_ODD = 1, BQ_FULL = 2 };          /* sites a field holds */

/* Operator kinds for bq_apply (in -> out subsets in brackets). */
enum {
    BQ_OP_M = 0,              /* M = T - kappa D                         [FULL -> FULL]  */
    BQ_OP_MDAG = 1,           /* M^dag                                   [FULL -> FULL]  */
    BQ_OP_MHAT = 2,           /* T_oo - kappa^2 D_oe T_ee^-1 D_eo        [ODD  -> ODD]   */
    BQ_OP_MHATDAG = 3,        /* Mhat^dag                                [ODD  -> ODD]   */
    BQ_OP_MHATDAG_MHAT = 4,   /* Mhat^dag Mhat                           [ODD  -> ODD]   */
    BQ_OP_DEO = 5,            /* D restricted to even rows, odd columns  [ODD  -> EVEN]  */
    BQ_OP_DOE = 6,            /* D, odd rows, even columns               [EVEN -> ODD]   */
    BQ_OP_DEO_DAG = 7,        /* (D^dag)_eo                              [ODD  -> EVEN]  */
    BQ_OP_DOE_DAG = 8,        /* (D^dag)_oe                              [EVEN -> ODD]   */
    BQ_OP_K1 = 9,             /* T_ee^-1 D_eo (the fused EO-clover Dslash) [ODD -> EVEN] */
    BQ_OP_K1_DAG = 10,        /* T_ee^-1 (D^dag)_eo                      [ODD  -> EVEN]  */
    BQ_OP_CLOVER = 11,        /* T                                       [FULL -> FULL]  */
    BQ_OP_CLOVER_INV = 12,    /* T_ee^-1                                 [EVEN -> EVEN]  */
    BQ_OP_MDAGM = 13          /* M^dag M                                 [FULL -> FULL]  */
};

/* Linear systems for bq_solve. */
enum {
    BQ_SYS_NORMAL = 0,        /* Mhat^dag Mhat x = b on odd sites (b, x: ODD fields)                 */
    BQ_SYS_M = 1,             /* M x = b on the full lattice through the odd-site Schur system:
                                 bhat = b_o + kappa D_oe T_ee^-1 b_e, CG on Mhat^dag Mhat x_o = Mhat^dag bhat,
                                 x_e = T_ee^-1 (b_e + kappa D_eo x_o)           (b, x: FULL fields) */
    BQ_SYS_FULL_NORMAL = 2,   /* M^dag M x = b on the full lattice, no preconditioning (FULL fields) */
    BQ_SYS_MHAT = 3           /* Mhat x = b on odd sites (b, x: ODD fields); CG solves it as
                                 Mhat^dag Mhat x = Mhat^dag b, BiCGstab directly */
};

/* Solvers of bq_solve (the solver list of section "Algorithms": cg, BiCGstab, block cg). */
enum {
    BQ_SOLVER_CG = 0,         /* CG on the normal equations, per column, mixed precision by reliable updates */
    BQ_SOLVER_BICGSTAB = 1,   /* BiCGstab on Mhat itself (BQ_SYS_M, BQ_SYS_MHAT): one Krylov space per
                                 column, FP64 or FP32 inner iterations restarted from FP64 residuals */
    BQ_SOLVER_BLOCK_CG = 2    /* block CG on Mhat^dag Mhat (BQ_SYS_NORMAL, BQ_SYS_M, BQ_SYS_MHAT): all
                                 columns in one Krylov space, FP64 */
};

typedef struct bq_context_s* bq_context;
typedef struct bq_gauge_s* bq_gauge;
typedef struct bq_op_s* bq_op;
typedef struct bq_field_s* bq_field;
typedef struct bq_server_s* bq_server;

typedef struct {
    double tol;        /* stop when the FP64 true residual |b' - A x| <= tol |b'| (A, b' of the CG system) */
    int maxiter;       /* bound on inner CG iterations per right-hand side */
    int inner_prec;    /* BQ_F64, BQ_F32 or BQ_F16 arithmetic/storage of the inner iterations */
    double delta;      /* reliable update when |r_inner| < delta * max|r| since the last update
                          (0: 0.01 for FP32 inner iterations, 0.1 for FP16) */
    int system;        /* BQ_SYS_* */
    int chunk;         /* iterations between reliable-update passes and host convergence checks
                          (0: default 4).  A column that requests a reliable update idles until
                          the end of its chunk; short chunks waste less, long ones launch less. */
    int use_graph;     /* 1: capture a chunk of iterations in a hipGraph and replay it (CG only) */
    int solver;        /* BQ_SOLVER_* (0: CG) */
} bq_solve_params;

typedef struct {
    int iters;              /* inner iterations (BiCGstab: two operator applications each) */
    int reliable_updates;   /* FP64 true-residual recomputations (BiCGstab: restarts) */
    double true_rel_resid;  /* |b' - A x| / |b'| of the system the solver iterates on, recomputed in FP64
                               (CG: the normal system; BiCGstab: Mhat x = bhat) */
    double full_rel_resid;  /* BQ_SYS_M: |b - M x| / |b|; BQ_SYS_MHAT: |b - Mhat x| / |b|;
                               otherwise equal to true_rel_resid */
    int converged;          /* 1 if true_rel_resid <= tol */
    int status;             /* BQ_OK or the per-column error code */
} bq_solve_info;

/* Accounting of the last bq_solve / bq_trace on an operator. */
typedef struct {
    double bytes;        /* algorithmic HBM bytes: every kernel's inputs read once and outputs written once
                            (links and clover once per launch, spinors once per active right-hand side) */
    double seconds;      /* device time of the call, HIP events on the solve stream */
    long long launches;  /* kernel launches (kernels inside graph replays included) */
    int chunks;          /* host convergence checks */
    int iterations;      /* lockstep inner iterations executed for the batch */
} bq_solve_stats;

/* Library version (major*10000 + minor*100 + patch). */
int bq_version(void);

/* Thread-local description of the last error, or "" (never NULL). */
const char* bq_last_error(void);

/* Device allocator of the caller (e.g. torch's caching allocator): alloc returns `bytes` of
 * device memory on the context's device, aligned to 256 bytes, or NULL; dealloc gives a block
 * back.  alloc_ctx is passed through unchanged. */
typedef void* (*bq_alloc_fn)(size_t bytes, void* alloc_ctx);
typedef void (*bq_dealloc_fn)(void* ptr, void* alloc_ctx);

/* Create a context on HIP device `device` (the library object that holds a device, a stream,
 * an HBM budget and the stencil tuning table; the paper's interface to QUDA, section "QUDA",
 * has BQCD hand a gauge field and a source to a GPU library and receive the solution).
 *   hbm_budget_bytes  bound on the device memory the context may hold (0 = 90% of the
 *                     device's free memory); an allocation above it fails with BQ_ERR_OOM.
 *   alloc, dealloc    route every device allocation of the context (fields, links, clover,
 *                     workspaces) through the caller's allocator; both NULL = hipMalloc/hipFree.
 *                     Before a block goes back to dealloc the library waits for the device
 *                     to finish the work queued on it.  Giving only one is BQ_ERR_INVALID; a
 *                     block not aligned to 256 bytes is handed back and reported as
 *                     BQ_ERR_INVALID, NULL as BQ_ERR_OOM.
 *   out               receives the handle, owned by the caller until bq_context_destroy.
 * The context owns a HIP stream (default priority).  Errors: BQ_ERR_INVALID (bad device,
 * NULL out), BQ_ERR_DEVICE. */
int bq_context_create(int device, uint64_t hbm_budget_bytes, bq_alloc_fn alloc, bq_dealloc_fn dealloc,
                      void* alloc_ctx, bq_context* out);
/* Destroy a context.  If gauge fields, fields or servers created on it are still alive, the
 * context is freed together with the last of them (so handles may be freed in any order).
 * NULL is a no-op. */
int bq_context_destroy(bq_context ctx);
/* Bytes of device memory the context currently holds (its own accounting, padding included). */
int bq_context_hbm_used(bq_context ctx, uint64_t* used);

/* Upload the gauge links U_mu(x) of Eq. 1 (section "Fermion actions").
 *   dims[4]          lattice extents (x, y, z, t), each even and >= 2.
 *   links            U[mu][i][3][3] in the canonical layout above, FP64 complex; host memory, or
 *                    device memory when links_on_device != 0.  Read during the call only.
 *   t_bc             sign a fermion picks up on a hop across the time boundary: -1 antiperiodic,
 *                    +1 periodic (space is periodic).
 * The library keeps FP64, FP32 and FP16 copies in its checkerboard layout (the volume/2 arrays
 * of section "SIMD vectorization and MPI").  Links are used as given.  The two-row form
 * (row 2 rebuilt as conj(row0 x row1), valid for SU(3) only) is kept for a precision only if
 * every link is SU(3) to within that precision (max |U U^dag - 1|, |det U - 1| <= 1e-13 for
 * FP64, 1e-6 for FP32, 1e-3 for FP16); otherwise FP64/FP32 stencils read all 18 reals, and FP16
 * storage and the server, which need the two-row form, return BQ_ERR_UNSUPPORTED.
 * Errors: BQ_ERR_INVALID (NULL, bad extents or t_bc), BQ_ERR_NONFINITE (a non-finite link),
 * BQ_ERR_OOM, BQ_ERR_DEVICE. */
int bq_gauge_upload(bq_context ctx, const int dims[4], const double* links, int links_on_device, int t_bc,
                    bq_gauge* out);
/* The largest distance of an uploaded link from SU(3): max(|(U U^dag - 1)_ab|, |det U - 1|). */
int bq_gauge_su3_deviation(bq_gauge g, double* dev);
/* Average plaquette (section "Measurements"): mean over sites and the 6 planes of
 * Re tr U_{mu nu}(x) / 3, FP64. */
int bq_gauge_plaquette(bq_gauge g, double* plaq);
/* BQ_ERR_BUSY while operators built on g are alive or server sessions hold it
 * (bq_server_release); NULL is a no-op. */
int bq_gauge_free(bq_gauge g);

/* Build the fermion matrix M(U; kappa, c_SW, mu) of Eq. 1 (hopping term with chemical
 * potential mu: e^{+mu} on forward, e^{-mu} on backward time hops) and Eq. 2 (clover term
 * -(i/2) kappa c_SW sigma_{mu nu} F_{mu nu}; the CPT-breaking lambda term is not provided,
 * lambda = 0): the clover field T on both parities and T_ee^-1, built and inverted in FP64
 * (Cholesky per 6x6 block), with FP32/FP16 copies.  The handle keeps g alive (bq_gauge_free
 * returns BQ_ERR_BUSY until bq_op_free).  Errors: BQ_ERR_INVALID (NULL, non-finite
 * parameters), BQ_ERR_CLOVER_NOT_HPD (a clover block is not positive definite), BQ_ERR_OOM. */
int bq_op_create(bq_gauge g, double kappa, double csw, double mu, bq_op* out);
int bq_op_free(bq_op op);

/* A device field of nrhs right-hand sides on `subset` sites (BQ_EVEN, BQ_ODD: one checkerboard
 * of section "SIMD vectorization and MPI"; BQ_FULL: both) in storage precision prec, zeroed.
 * Errors: BQ_ERR_INVALID (bad extents, subset, precision, nrhs < 1), BQ_ERR_OOM. */
int bq_field_create(bq_context ctx, const int dims[4], int subset, int prec, int nrhs, bq_field* out);
int bq_field_free(bq_field f);
/* Copy nrhs canonical spinors (nrhs*V*12 complex, full lattice) into the field, converting to
 * its precision (round to nearest even; FP16 with a per-site FP32 scale); only sites of the
 * field's subset are read.  src may be host or device memory (src_on_device); the call
 * returns when the copy is complete.  Errors: BQ_ERR_INVALID, BQ_ERR_OOM, BQ_ERR_DEVICE. */
int bq_field_put(bq_field f, const double* src, int src_on_device, void* stream);
/* Copy the field out to nrhs canonical spinors (FP64); only sites of the field's subset are
 * written, other sites of dst are left untouched. */
int bq_field_get(bq_field f, double* dst, int dst_on_device, void* stream);

/* out = Op in for Op = BQ_OP_* (Eq. 1 and Eq. 2; the EO kinds restrict M to the checkerboards
 * of section "SIMD vectorization and MPI"); in and out must have the subsets listed with
 * the kinds, the same precision and the same nrhs, and be different fields.  Asynchronous on
 * `stream` (NULL: the context's stream); kinds that need an intermediate field (M^dag M and the
 * Mhat kinds) allocate it and wait for the stream before returning.  Errors: BQ_ERR_INVALID
 * (kind, subsets, precisions, lattices), BQ_ERR_UNSUPPORTED (no link copy, see
 * bq_gauge_upload), BQ_ERR_OOM, BQ_ERR_DEVICE. */
int bq_apply(bq_op op, int kind, bq_field in, bq_field out, void* stream);

/* Bytes of the static per-device array that holds the work fields of bq_apply_noalloc. */
#define BQ_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* bq_apply for callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same kinds, fields and results as bq_apply,
 * but the intermediate fields of M^dag M and of the Mhat kinds live in one static array of
 * BQ_NOALLOC_SCRATCH_BYTES per device (loaded with the library on that device and held until the
 * process ends), so the call allocates and frees nothing and never waits: it only enqueues its
 * kernels on `stream` (NULL: the context's stream).  Every call on a device shares that device's
 * array and leaves its intermediate there; each call writes its intermediate in full before
 * reading it, so nothing has to start at zero.  Calls that overlap on one device (other streams,
 * threads or contexts) race on the array: the caller orders them.  Room: per column, Mhat and
 * Mhat^dag need one half-lattice spinor of the field's precision, Mhat^dag Mhat two, M^dag M one
 * full-lattice spinor (plus tile padding); the other kinds need none.  Errors as bq_apply, and
 * BQ_ERR_INVALID, with nothing enqueued, when the work fields do not fit. */
int bq_apply_noalloc(bq_op op, int kind, bq_field in, bq_field out, void* stream);

/* Solve the system params->system for all nrhs columns of b at once with a solver of the solver
 * list of section "Algorithms" (params->solver):
 *   BQ_SOLVER_CG        cg, the solver Tables 1-2 time: one fused multi-right-hand-side launch per
 *                       operator step, per-column CG scalars on the device, FP32/FP16 inner
 *                       iterations with FP64 reliable updates when params->inner_prec asks for them;
 *   BQ_SOLVER_BICGSTAB  BiCGstab on Mhat (BQ_SYS_M, BQ_SYS_MHAT), FP64 or FP32 inner iterations;
 *   BQ_SOLVER_BLOCK_CG  block CG on Mhat^dag Mhat (the block part of the list's "block multishift
 *                       cg"), FP64, nrhs <= 16: all columns in one block Krylov space, with the
 *                       N x N step matrices formed on the device.  A run ends when every column's
 *                       recursive residual reaches tol; the FP64 residual is then recomputed and
 *                       the columns that miss tol start a new run from it (at most 8 runs; counted
 *                       in reliable_updates).  Columns that are numerically dependent at the start
 *                       of a run (pivot below 1e-12 of their norm in a Cholesky pass) wait for the
 *                       next run; a zero column gets x = 0.
 * b and x are FP64 fields with the subset of the system (BQ_SYS_NORMAL, BQ_SYS_MHAT: ODD,
 * otherwise FULL) and the same nrhs; x receives the solutions.  info points to nrhs entries
 * (may be NULL).  Returns BQ_ERR_NOT_CONVERGED if some column did not reach tol within maxiter
 * (x then holds the last iterate, info is filled), BQ_ERR_NONFINITE for a non-finite source or
 * breakdown, BQ_ERR_INVALID / BQ_ERR_UNSUPPORTED for bad parameters or combinations.  Blocks
 * until the solve is complete. */
int bq_solve(bq_op op, bq_field b, bq_field x, const bq_solve_params* params, bq_solve_info* info, void* stream);

/* Stochastic traces Tr(M^-1) and Tr(M^-2) (section "Measurements"; the abstract's Tr(D^-n))
 * with nnoise complex Z2 noise vectors eta_n (components (+-1 +- i)/sqrt(2) from SplitMix64
 * used as a counter-based generator with seed `seed`: component (n, i, spin s, colour c) uses
 * output k = (n*V + i)*12 + 3s + c; bit 63 gives the real sign, bit 62 the imaginary), solved
 * `block` at a time with params (system forced to BQ_SYS_M).  The noise is generated on the
 * device.  t1[2n], t1[2n+1] = Re, Im of eta_n^dag M^-1 eta_n; t2 likewise for M^-2 (host
 * arrays of 2*nnoise doubles).  info: nnoise entries for the first solve and nnoise for the
 * second (may be NULL).  Errors as bq_solve. */
int bq_trace(bq_op op, uint64_t seed, int nnoise, int block, const bq_solve_params* params, double* t1, double* t2,
             bq_solve_info* info);

/* Multishift CG (section "Algorithms": the "multishift cg" of the solver list; RHMC's rational
 * approximations need (W^dag W + b_k)^-1 for every pole b_k): solve
 *     (Mhat^dag Mhat + shifts[k]) x[k] = b        on odd sites, for k = 0..nshift-1,
 * for every column of b at once.  The shifts share the Krylov space of the smallest shift
 * (collinear residuals), so one Mhat^dag Mhat application per iteration serves all shifts and
 * columns; FP64 throughout (params->inner_prec must be BQ_F64, params->system BQ_SYS_NORMAL,
 * params->chunk iterations between host checks, default 8).
 *   b          ODD FP64 field, nrhs columns.
 *   shifts     nshift (1..16) finite values >= 0.
 *   x          nshift distinct ODD FP64 fields with b's nrhs; x[k] receives the solutions of shift k.
 *   info       nshift*nrhs entries (may be NULL), info[k*nrhs + col]: a shift stops when its
 *              recursive residual |zeta_k r| <= tol |b|; true_rel_resid (= full_rel_resid) is
 *              |b - (A + shifts[k]) x[k]| / |b| recomputed in FP64 afterwards.
 * params->solver = BQ_SOLVER_BLOCK_CG gives block multishift CG (the list's "block multishift cg";
 * nrhs <= 16): the columns share one block Krylov space as well, and the block residual of each
 * shift is R xi_k for the base residual block R and an nrhs x nrhs matrix xi_k per shift, whose
 * recurrences follow from the three-term block relations of the base and shifted systems; a shift
 * stops when |R xi_k e_col| <= tol |b_col| for all its columns.  There are no restarts: columns
 * numerically dependent on others are not solved (their info reports BQ_ERR_NOT_CONVERGED).
 * Errors: BQ_ERR_INVALID, BQ_ERR_UNSUPPORTED (inner precision), BQ_ERR_NOT_CONVERGED (x holds the
 * last iterates), BQ_ERR_NONFINITE, BQ_ERR_OOM. */
int bq_solve_multishift(bq_op op, bq_field b, int nshift, const double* shifts, bq_field* x,
                        const bq_solve_params* params, bq_solve_info* info, void* stream);

/* Terms of bq_trace_estimators, per noise eta, with x1 = M^-1 eta and E[eta eta^dag] = 1:
 * the traces of section "Measurements" and the abstract's traces for kappa, c_SW and chemical
 * potential reweighting (Tr(M^-1 dM/dp) = d ln det M / dp). */
enum {
    BQ_TR_MINV = 0,       /* eta^dag x1                    -> Tr M^-1                        */
    BQ_TR_MINV2 = 1,      /* eta^dag M^-1 x1               -> Tr M^-2                        */
    BQ_TR_G5_MINV = 2,    /* eta^dag gamma_5 x1            -> Tr gamma_5 M^-1                */
    BQ_TR_MDAGM_INV = 3,  /* |x1|^2                        -> Tr (M M^dag)^-1 = Tr (M^dag M)^-1 */
    BQ_TR_DM_DKAPPA = 4,  /* eta^dag (dM/dkappa) x1        -> Tr M^-1 dM/dkappa, dM/dkappa = c_SW S - D */
    BQ_TR_DM_DCSW = 5,    /* eta^dag (dM/dc_SW) x1         -> Tr M^-1 dM/dc_SW,  dM/dc_SW = kappa S    */
    BQ_TR_DM_DMU = 6,     /* eta^dag (dM/dmu) x1           -> Tr M^-1 dM/dmu,    dM/dmu = -kappa dD/dmu */
    BQ_TR_COUNT = 7
};

/* All BQ_TR_* terms per noise (S = sum_{mu<nu} sigma_{mu nu} F_{mu nu}, the clover term of Eq. 2
 * without kappa c_SW; dD/dmu = Eq. 1's time hops with +e^{+mu} forward and -e^{-mu} backward).
 * Noise, blocking and params as bq_trace (system forced to BQ_SYS_M).  est receives
 * nnoise*BQ_TR_COUNT*2 doubles: est[(n*BQ_TR_COUNT + term)*2 + {0, 1}] = Re, Im.  info as bq_trace.
 * Holds three FP64 full-lattice fields of `block` columns besides the solver workspace. */
int bq_trace_estimators(bq_op op, uint64_t seed, int nnoise, int block, const bq_solve_params* params, double* est,
                        bq_solve_info* info);

/* Statistics of the last bq_solve or bq_trace call on op. */
int bq_solve_stats_get(bq_op op, bq_solve_stats* out);

/* Time `reps` back-to-back launches of one operator kind on fields in/out with HIP events
 * recorded on the stream the kernels run on; *ms = mean per launch, *bytes = algorithmic
 * bytes one launch must move (each input read once, each output written once). */
int bq_time_apply(bq_op op, int kind, bq_field in, bq_field out, int reps, void* stream, double* ms, double* bytes);

/* Reference rate of the device's memory (measurement aid, no counterpart in the paper): time
 * `reps` launches of a plain copy of `bytes` (a multiple of 16) between two buffers the context
 * allocates for the call, with HIP events on `stream` (NULL: the context's stream); *ms = mean
 * per copy, which moves 2 * bytes.  Errors: BQ_ERR_INVALID, BQ_ERR_OOM, BQ_ERR_DEVICE. */
int bq_time_copy(bq_context ctx, uint64_t bytes, int reps, void* stream, double* ms);

/* Stencil configuration (the project's autotuner; no counterpart in the paper) used for a given
 * precision and column count (set by
 * bq_autotune or explicitly; otherwise a default).  recon: 12 or 18 reals per
 * link; R: columns per thread; bs: sites per workgroup (64, 128, 256 or 512;
 * the column groups of those sites run in the same workgroup, up to 512 threads).
 * march: 0, or the length of the time segments of the t-marching stencil, in
 * which a wavefront walks `march` consecutive time planes of one tile position
 * and keeps the backward time hop of each plane from the forward time hop two
 * planes earlier (up to bs/64 column groups per workgroup).  It applies to
 * lattices whose (x,y) planes hold whole 64-site tiles and whose L_t it divides;
 * elsewhere the plain stencil runs.  lds: 1 selects the tile-shared stencil when a tile has
 * several column groups (nrhs > R): one 64-site tile per workgroup with up to bs/64 (at most 16;
 * FP64 at most 12) column-group waves, whose links (rebuilt to 3x3) and clover are staged in LDS once and read
 * from there by every wave (march is then ignored; bs may be any multiple of 64 up to 1024);
 * lds: 2 is the same with R = 1 only, where each wave also takes the x and y neighbours that
 * lie in its own tile from the other lanes' registers instead of from memory.
 * order: the traversal of the 64-site tiles by the plain and tile-shared stencils on lattices
 * whose (x,y) planes hold whole tiles: 0 visits them in blocks of 4x4 (z,t) planes; 1 gives each
 * of the 8 XCDs one slab of L_z/gcd(L_z,8) z planes and walks it t plane by t plane (ignored by
 * the t-marching stencil and on other lattices); 2 is order 1 where it applies and, on any lattice
 * with a multiple of 8 tile blocks, has each XCD walk its tile blocks once per column-group chunk
 * (fewer columns in flight per XCD; links and clover are read once per chunk).  Errors: BQ_ERR_INVALID for a configuration
 * that is not compiled or out of range.  Results do not depend on the configuration. */
int bq_tune_get(bq_context ctx, int prec, int nrhs, int* recon, int* R, int* bs, int* march, int* lds, int* order);
int bq_tune_set(bq_context ctx, int prec, int nrhs, int recon, int R, int bs, int march, int lds, int order);
/* Time the candidate configurations for (op's lattice, prec, nrhs) on op and keep the fastest. */
int bq_autotune(bq_op op, int prec, int nrhs);

/* ---------------------------------------------------------------------------
 * Continuous-batching solve server (many requests, mixed lattices and kappa).
 * The paper has no serving layer; the server batches solves of the cg solver (section
 * "Algorithms") from many callers.
 * Requests M x = b (the BQ_SYS_M system) on resident gauge fields are queued by
 * bq_server_submit and advanced by bq_server_step.  Requests run in sessions (by
 * default one per gauge field, mu and inner precision, see bq_server_set_sessions;
 * `slots` columns each) that advance
 * independently, one chunk of CG iterations at a time, on streams of their own:
 * a step retires the requests whose columns have converged in the sessions whose
 * chunk has finished, admits queued requests into free column slots of those
 * sessions when their operator fits in the context's HBM budget, and starts
 * their next chunk.  Columns of one session have their own
 * kappa and clover and share the link reads; a request gives the same result
 * alone and batched with others.  Single host thread per server.  Sessions overlap
 * only on separate hardware queues: HIP maps a process's streams onto
 * GPU_MAX_HW_QUEUES queues (4 unless set before the runtime starts), and streams
 * that share a queue run in submission order, so a process serving k sessions
 * should set it to k + 2 or more (its own stream and the context's).
 * ------------------------------------------------------------------------- */
int bq_server_create(bq_context ctx, int slots, int chunk, bq_server* out);
/* Admission order within a session: a request that does not fit (too few free slots, or its
 * operator over the HBM budget) waits at the head of its session's queue; later requests that
 * do fit may pass it (backfill) in up to `steps` scheduling steps that admit into its session;
 * steps in which the session has a chunk in flight do not count.  After that the session
 * admits nothing else until the waiting request fits.  0 = strict arrival order.  Default 8. */
int bq_server_set_backfill(bq_server s, int steps);
/* Sessions per (gauge field, mu, inner precision), 1..8 (default 1).  With more than one, a
 * request goes to the fullest idle session of its key that has room for its columns, and a new
 * session (its own workspace and stream) is opened when none has, up to this number: a wide
 * request then starts beside a full session instead of waiting for its slots.  The admission
 * order and backfill above hold per key.  Errors: BQ_ERR_INVALID. */
int bq_server_set_sessions(bq_server s, int per_key);
/* b: nrhs canonical spinors; x: an array of the same size that receives the solutions.
 * Each may be host or device memory (the runtime tells them apart by address; device
 * sources skip the PCIe transfers).  Both are owned by the caller and must stay valid
 * until the request retires.  The result's full_rel_resid is |b - M x| / |b| on the full
 * lattice, recomputed in FP64 at retirement.  Errors: BQ_ERR_INVALID (NULL, nrhs outside
 * 1..slots, tol <= 0, non-finite kappa, c_SW or mu), BQ_ERR_UNSUPPORTED (g is not SU(3), see
 * bq_gauge_upload).  A request whose operator cannot be built (BQ_ERR_CLOVER_NOT_HPD) is
 * finished by the step that tries to admit it, with that status. */
int bq_server_submit(bq_server s, bq_gauge g, double kappa, double csw, double mu, const double* b, double* x,
                     int nrhs, double tol, int inner_prec, int maxiter, uint64_t* ticket);
/* One scheduling step.  It returns once at least one session's chunk has finished since
 * the step began (waiting for one if none had), or at once when no chunk is in flight;
 * chunks started by the step are still running when it returns.  Up to max_done tickets
 * completed in this step are written to done_tickets, *ndone = their number. */
int bq_server_step(bq_server s, uint64_t* done_tickets, int max_done, int* ndone);
/* BQ_PENDING while queued or running; afterwards the request's status (info[nrhs]
 * filled) and the ticket is forgotten. */
int bq_server_result(bq_server s, uint64_t ticket, bq_solve_info* info);
int bq_server_pending(bq_server s, int* queued, int* running);
/* Free the sessions (workspaces, streams, and the operators of retired requests that a session
 * keeps for its next requests) the server holds for gauge field g, so that g can be freed;
 * BQ_ERR_BUSY while a request on g is queued or running.  Kept operators are also freed when
 * the context's HBM budget refuses a session or an operator. */
int bq_server_release(bq_server s, bq_gauge g);
/* Free the server, its sessions and its requests' operators (results not yet collected are lost). */
int bq_server_free(bq_server s);

#ifdef __cplusplus
}
#endif

#endif /* BQHIP_H */
