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
hipError_t launch_plaquette(const Geom& g, const double2* const U64[8], double* partial, int nparts, hipStream_t st);

// BLAS-1 and reductions
hipError_t launch_convert(int src_prec, FieldArg src, int dst_prec, FieldArg dst, int Vh, int ncol,
                          const int* status, int statmask, hipStream_t st);
hipError_t launch_norm2(int prec, FieldArg x, int Vh, int ncol, double* partial, int nwaves, hipStream_t st);
hipError_t launch_zero(int prec, FieldArg x, int Vh, int ncol, const int* status, int statmask, hipStream_t st);
// x += alpha p ; p = r + beta p   (CG; per column, by status)
hipError_t launch_cg_update(int xprec, FieldArg x, int pprec, FieldArg p, int rprec, FieldArg r, int Vh, int ncol,
                            const double* alpha, const double* beta, const int* status, hipStream_t st);
// reliable update pieces: y += x (x low precision), x = 0
hipError_t launch_accum(int xprec, FieldArg x, FieldArg y64, int Vh, int ncol, const int* status, int statmask,
                        hipStream_t st);
// p = lowp(r64) + beta p (restart after a reliable update), rs = lowp(r64)
hipError_t launch_restart(FieldArg r64, int rsprec, FieldArg rs, int pprec, FieldArg p, int Vh, int ncol,
                          const double* beta, const int* flag, hipStream_t st);
hipError_t launch_dot(int prec, FieldArg x, FieldArg y, int Vh, int ncol, double* partial, int nwaves,
                      hipStream_t st);
hipError_t launch_z2_noise(uint64_t seed, long n0, const Geom& g, int parity, FieldArg dst, int ncol,
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
