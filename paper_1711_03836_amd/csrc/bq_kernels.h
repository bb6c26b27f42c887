// Host-side launch interface of the HIP kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "bq_device.h"

namespace bq {

// Epilogues fused into the hopping kernel.  `hop` is D (or D^dag) applied to
// the input field at the output site, `v` a field on the output parity.
enum {
    EPI_HOP = 0,   // out = a*v + f*hop                     (D_eo, D_oe, source preparation)
    EPI_TINV = 1,  // out = C (a*v + f*hop), C = clover blocks given (T_ee^-1 for K1 / reconstruction)
    EPI_TV = 2,    // out = C v + f*hop (+ |out|^2 partials)  (K2 of Mhat, full M)
    EPI_TVR = 3,   // w = C v + f*hop; r_out = r_in - alpha*w (+ |r_out|^2 partials)  (CG residual update)
};

// most columns one launch can give their own operator (kappa, clover)
constexpr int kMaxCols = 32;

struct FieldArg {
    void* d = nullptr;       // storage units
    float* s = nullptr;      // FP16 per-site scales
    size_t cstride = 0;      // units between columns
    size_t sstride = 0;      // floats between scale columns
};

struct HopLaunch {
    int prec = PREC_F64;     // storage precision of in/out/v/links/clover
    int rprec = PREC_F64;    // precision of r_in/r_out (EPI_TVR)
    int recon = 18;          // 18 or 12 reals per link
    int dagger = 0;
    int epi = EPI_HOP;
    int R = 1;               // columns per thread
    int bs = 256;            // sites per workgroup (a multiple of 64)
    int march = 0;           // > 0: t-marching kernel with segments of `march` time planes
                             //      (needs whole tiles per (x,y) plane and march | L_t)
    int lds = 0;             // 1: tile-shared kernel (links and clover staged in LDS) when a tile has
                             //    several column groups; 2: the same with one column per wave and the
                             //    x and y neighbour spinors exchanged between lanes
    Geom g{};
    int parity = 0;          // output parity
    int ncol = 1;
    const void* U[8] = {};   // links [parity*4 + mu], each on its own parity
    FieldArg in, out, v, r_in, r_out;
    const void* clov = nullptr;   // clover blocks on the output parity
    const double* alpha = nullptr;
    double* partial = nullptr;    // |.|^2 per wavefront of 64 sites: partial[c * pstride + wave]
    int nwaves = 0;               // waves of this launch (bound on `wave`)
    int pstride = 0;              // partial entries per column
    const int* status = nullptr;
    int statmask = 1;
    double ef = 1, eb = 1;   // time-hop coefficients of the forward / backward term
    int tbc = -1;
    double f = 1, a = 0;
    int percol = 0;                    // 1: column c uses cclov[c] and cf[c] instead of clov and f
    const void* cclov[kMaxCols] = {};
    double cf[kMaxCols] = {};
};

hipError_t launch_hop(const HopLaunch& L, hipStream_t st);
bool hop_variant_exists(int prec, int rprec, int recon, int R, int epi);

// clover
struct CloverBuild {
    Geom g{};
    const double2* U64[8] = {};   // FP64 links, 18 reals
    double ckappa = 0;            // kappa * c_SW
    double2* T[2] = {};           // out: T on parity 0/1 (packed blocks, FP64); may be null
    double2* Tinv[2] = {};        // out: T^-1 on parity 0/1; may be null
    double2* B[2] = {};           // out: sum_{mu<nu} sigma (x) F (kappa-independent), may be null
    int* bad = nullptr;           // set to 1 if some block is not positive definite
};
hipError_t launch_clover_build(const CloverBuild& c, hipStream_t st);
// T = 1 + ck*B and T^-1 from a stored B (per-kappa rebuild)
hipError_t launch_clover_from_B(const Geom& g, int parity, const double2* B, double ck, double2* T, double2* Tinv,
                                int* bad, hipStream_t st);
hipError_t launch_clover_apply(int prec, const Geom& g, const void* clov, FieldArg in, FieldArg out, int ncol,
                               hipStream_t st, const void* const* cclov = nullptr, const int* status = nullptr,
                               int statmask = 0);
hipError_t launch_clover_convert(int prec, const double2* src, void* dst, int Vh, hipStream_t st);

// layout conversion
hipError_t launch_links_import(const double2* canon, const Geom& g, int parity, int prec, int recon, void* const dst[4],
                               hipStream_t st);
hipError_t launch_spinor_import(const double2* canon, int ncol, const Geom& g, int parity, int prec, FieldArg dst,
                                hipStream_t st);
hipError_t launch_spinor_export(FieldArg src, int ncol, const Geom& g, int parity, int prec, double2* canon,
                                hipStream_t st);
// distance of the canonical FP64 links from SU(3): one partial maximum per part (see link_su3_parts)
int link_su3_parts(size_t nlinks);
hipError_t launch_link_su3_dev(const double2* canon, size_t nlinks, double* partial, hipStream_t st);
hipError_t launch_plaquette(const Geom& g, const double2* const U64[8], double* partial, int nparts, hipStream_t st);

// BLAS-1 and reductions
hipError_t launch_convert(int src_prec, FieldArg src, int dst_prec, FieldArg dst, int Vh, int ncol,
                          const int* status, int statmask, hipStream_t st);
hipError_t launch_norm2(int prec, FieldArg x, int Vh, int ncol, double* partial, int nwaves, hipStream_t st);
hipError_t launch_zero(int prec, FieldArg x, int Vh, int ncol, const int* status, int statmask, hipStream_t st);
hipError_t launch_copy16(const void* src, void* dst, size_t n16, hipStream_t st);  // n16 16-byte words
// x += alpha p ; p = r + beta p   (CG; per column, by status)
hipError_t launch_cg_update(int xprec, FieldArg x, int pprec, FieldArg p, int rprec, FieldArg r, int Vh, int ncol,
                            const double* alpha, const double* beta, const int* status, hipStream_t st);
// reliable update pieces: y += x (x low precision), x = 0
hipError_t launch_accum(int xprec, FieldArg x, FieldArg y64, int Vh, int ncol, const int* status, int statmask,
                        hipStream_t st);
// p = lowp(r64) + beta p (restart after a reliable update), rs = lowp(r64)
hipError_t launch_restart(FieldArg r64, int rsprec, FieldArg rs, int pprec, FieldArg p, int Vh, int ncol,
                          const double* beta, const int* flag, hipStream_t st);
// <x, y> (gamma5: <x, gamma_5 y>) per column, FP64; partials [col][re/im][wave]
hipError_t launch_dot(int prec, FieldArg x, FieldArg y, int Vh, int ncol, double* partial, int nwaves,
                      hipStream_t st, int gamma5 = 0);
hipError_t launch_z2_noise(uint64_t seed, long n0, const Geom& g, int parity, FieldArg dst, int ncol,
                           hipStream_t st);

// y += a x per column (a real, the same for every column) with |y|^2 partials per wave (FP64)
hipError_t launch_axpy_norm(FieldArg x, FieldArg y, double a, int n, int ncol, double* partial, int nwaves,
                            hipStream_t st);

// ---------------------------------------------------------------------------
// multishift CG: (A + sigma_k) x_k = b for all shifts in the Krylov space of the base system
// A + sigma_b (sigma_b the smallest shift), with collinear shifted residuals r_k = zeta_k r
// ---------------------------------------------------------------------------
constexpr int kMaxShifts = 16;
struct MsState {
    // per column
    double* rho;      // |r|^2
    double* alpha;    // base alpha_j
    double* alpha_prev;
    double* beta;     // base beta_j
    double* beta_prev;
    double* stop2;    // (tol |b|)^2
    int* status;      // COL_ACTIVE / COL_DONE / COL_FAILED
    int* iters;
    // per column and shift, index c * nshift + k
    double* zeta;      // zeta_j
    double* zeta_prev; // zeta_{j-1}
    double* zeta_new;  // zeta_{j+1}
    double* ak;        // shift alpha
    double* bk;        // shift beta
    int* act;          // shift still iterating
    int* kiters;       // iterations of the shift
    int nshift, base;
    double shift[kMaxShifts];  // sigma_k - sigma_b
};
struct MsFields {
    FieldArg r, w, p;              // base residual, A p (without the base shift), base direction
    FieldArg x[kMaxShifts];        // solutions
    FieldArg pk[kMaxShifts];       // shift directions (pk[base] = p)
};
hipError_t launch_ms_init(const MsState& s, int ncol, double tol2, hipStream_t st);
hipError_t launch_fin_ms_alpha(const MsState& s, const double* pq, const double* pp, int nwaves, int ncol,
                               double sigma_b, hipStream_t st);
hipError_t launch_fin_ms_beta(const MsState& s, const double* pr, int nwaves, int ncol, hipStream_t st);
// r -= alpha (w + sigma_b p); x_k += ak p_k (active shifts); |r|^2 partials
hipError_t launch_ms_update1(const MsState& s, const MsFields& f, double sigma_b, int n, int ncol, double* partial,
                             int nwaves, hipStream_t st);
// p_k = zeta_{j+1} r + bk p_k (active shifts other than the base); p = r + beta p; |p|^2 partials
hipError_t launch_ms_update2(const MsState& s, const MsFields& f, int n, int ncol, double* partial, int nwaves,
                             hipStream_t st);

// ---------------------------------------------------------------------------
// block (multishift) CG: one block Krylov space for N <= kBlockMax columns; the N x N step
// matrices live on the device and are computed there by one wavefront, so a run needs no host
// round trip per iteration
// ---------------------------------------------------------------------------
constexpr int kBlockMax = 16;   // columns of a block solve
constexpr int kGramTiles = 8;   // 64-site tiles one wavefront sums before it writes its partial
// control words
enum { BC_K = 0, BC_STOP = 1, BC_BREAK = 2, BC_NA = 3, BC_MASK = 4, BC_IDX = 5,
       BC_FROZEN = BC_IDX + kBlockMax, BC_COUNT = BC_FROZEN + kMaxShifts };
// matrix slots (kBlockMax x kBlockMax complex each, row-major).  "Full" matrices are indexed by
// column number and vanish outside the active columns; "packed" ones hold the na x na block of the
// active columns in the order of the active list.
enum { BM_PQ = 0,       // full: P^dag (A P + sigma_b P)
       BM_RR = 1,       // full: R^dag R of the current residual block
       BM_RRN = 2,      // full: R^dag R of the new residual block
       BM_ALPHA = 3,    // full: base step matrix alpha_k
       BM_BETA = 4,     // full: base direction matrix beta_k
       BM_AINV = 5,     // packed: alpha_k^-1
       BM_C = 6,        // packed: alpha_k^-1 beta_k
       BM_SHIFT = 7 };  // per shift s at BM_SHIFT + 6 s: packed xi_k, packed xi_k-1, packed alpha^s_k-1,
                        // full xi_k (for the direction update), full alpha^s_k, full beta^s_k-1
constexpr int kBlockMats = BM_SHIFT + 6 * kMaxShifts;
struct BlockState {
    double2* mats;   // kBlockMats matrices
    double* thr;     // per column: (tol |b_c|)^2
    int* ctrl;       // BC_* words
    int* colstat;    // per column: COL_ACTIVE while in the block, COL_DONE otherwise (stencil filter)
    int* sstat;      // per shift and column [s * ncol + c]: 0 iterating, 1 converged
    int* siters;     // per shift and column: iteration at which it converged
    int ncol, nshift, base;
    double sigma_b;                // shift of the base system (added to A P)
    double shift[kMaxShifts];      // sigma_s - sigma_b
};
struct BlockFields {
    FieldArg x[kMaxShifts];        // solutions (x[base] is the base iterate)
    FieldArg p[kMaxShifts];        // directions (p[base] is the base direction)
};
// partial Gram sums of <X_i, Y_j + s Z_j> over the active columns (Z may be null); one set of
// kBlockMax^2 complex numbers per group of kGramTiles tiles
hipError_t launch_block_gram(FieldArg X, FieldArg Y, FieldArg Z, double s, const BlockState& S, int vh, int tiles,
                             double2* partial, hipStream_t st);
// fixed-order sum of the partials into matrix slot `slot` (full)
hipError_t launch_block_gram_fin(const BlockState& S, const double2* partial, int tiles, int slot, hipStream_t st);
// 0: start of a run (active list from colstat and the Gram matrix in BM_RR, dependent columns
// dropped); 1: alpha and the shift recurrences (after BM_PQ); 2: convergence, beta (after BM_RRN)
hipError_t launch_block_step(const BlockState& S, int phase, hipStream_t st);
// x_base += P alpha, R -= (W + sigma_b P) alpha
hipError_t launch_block_xr(const BlockState& S, FieldArg x, FieldArg p, FieldArg w, FieldArg r, size_t units,
                           hipStream_t st);
// P = R + P beta
hipError_t launch_block_p(const BlockState& S, FieldArg p, FieldArg r, size_t units, hipStream_t st);
// every shift s other than the base: p_s = R xi + p_s beta_s, x_s += p_s alpha_s
hipError_t launch_block_shift(const BlockState& S, const BlockFields& f, FieldArg r, size_t units, hipStream_t st);

// ---------------------------------------------------------------------------
// BiCGstab on Mhat (inner precision FP64 or FP32, FP64 reductions, FP64 restarts)
// ---------------------------------------------------------------------------
struct BicgScalars {
    double2* rho;     // <rhat, r>
    double2* alpha;
    double2* omega;
    double2* beta;
    double* r2;       // |r|^2 of the inner iteration
    double* stop2;    // inner goal |r|^2
    double* tol2b2;   // (tol |b|)^2 of the FP64 system
    double delta2;    // inner goal relative to the last FP64 residual
    int* status;      // COL_ACTIVE, COL_STOPPED (inner goal reached), COL_DONE, COL_FAILED
    int* iters;
    int* nrel;        // FP64 residual recomputations
    int* restart;     // set by the reliable pass for columns that restart
};
hipError_t launch_bicg_p(int prec, FieldArg r, FieldArg p, FieldArg v, const BicgScalars& s, int n, int ncol,
                         hipStream_t st);
// partials of <a1, b1> and (a2.d != null) <a2, b2>, [col][re1, im1, re2, im2][wave]
hipError_t launch_dots2(int prec, FieldArg a1, FieldArg b1, FieldArg a2, FieldArg b2, const int* status, int n,
                        int ncol, double* partial, int nwaves, hipStream_t st);
hipError_t launch_bicg_s(int prec, FieldArg r, FieldArg v, FieldArg s_, const BicgScalars& s, int n, int ncol,
                         hipStream_t st);
hipError_t launch_bicg_xr(int prec, FieldArg x, FieldArg p, FieldArg s_, FieldArg t, FieldArg r, FieldArg rhat,
                          const BicgScalars& s, int n, int ncol, double* partial, int nwaves, hipStream_t st);
// step 0: alpha, 1: omega, 2: rho / beta / stop test, 3: reliable pass decision (partials of |r64|^2)
hipError_t launch_fin_bicg(int step, const BicgScalars& s, const double* partial, int nwaves, int ncol,
                           hipStream_t st);

// CG finalisation kernels (one block per column)
struct CgScalars {
    double* rho;      // |r|^2 of the current iterate
    double* pAp;
    double* alpha;
    double* beta;
    double* stop2;    // (tol * |b|)^2
    double* rmax2;    // reliable-update reference |r|^2 (delta test)
    double delta2;    // delta^2 (0 = no reliable trigger)
    int* status;
    int* iters;
    int* restart;
    int* nrel;        // reliable updates per column
};
hipError_t launch_fin_alpha(const CgScalars& s, const double* partial, int nwaves, int ncol, hipStream_t st);
hipError_t launch_fin_beta(const CgScalars& s, const double* partial, int nwaves, int ncol, hipStream_t st);
hipError_t launch_fin_reliable(const CgScalars& s, const double* partial, int nwaves, int ncol, hipStream_t st);
hipError_t launch_fin_sum(const double* partial, int nwaves, int ncol, double* out, hipStream_t st);
// stop2 = tol2 * rho, rmax2 = rho, counters cleared, status from rho (rho holds |b|^2 on entry);
// with `sel` only columns with sel[c] != 0 are initialised, and tol2 is per column (tol2c) if given
hipError_t launch_cg_init(const CgScalars& s, int ncol, double tol2, hipStream_t st, const int* sel = nullptr,
                          const double* tol2c = nullptr, const double* rho_src = nullptr);
// status[c] = value for every column with sel[c] != 0
hipError_t launch_set_status(int* status, const int* sel, int ncol, int value, hipStream_t st);

}  // namespace bq
