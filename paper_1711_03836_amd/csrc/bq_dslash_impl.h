// The hopping-term stencil (Eq. 1) with fused clover epilogues (Eq. 2).
// Internal header: bq_dslash_inst.hip instantiates it for one storage precision
// and one number of columns per thread per compilation.
//
// One thread owns one output site of one checkerboard and R right-hand sides.
// For each of the 8 hops it loads the link once, and for each of its columns
// loads the neighbour spinor, projects it to a half spinor with (1 -+ gamma_mu),
// multiplies by U or U^dag, and accumulates the reconstructed spinor.  The
// epilogue then applies the clover blocks and the linear combination required
// by the caller, so that an operator application never writes the raw hop.
#pragma once

#include <algorithm>
#include <type_traits>

#include "bq_kernels.h"

namespace bq {
namespace dslash {

// ---------------------------------------------------------------------------
// spin projection in the chiral basis; S = -1 for (1 - gamma_mu), +1 for (1 + gamma_mu)
// spinor index s*3 + c; half spinor index k*3 + c (k = 0, 1)
// ---------------------------------------------------------------------------

template <typename T, int S> __device__ __forceinline__ cx<T> pmi(cx<T> a) { return S > 0 ? cmuli(a) : cmulmi(a); }  // S*i*a

template <typename T, int MU, int S>
__device__ __forceinline__ void project(const cx<T> (&p)[12], cx<T> (&h)[6])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cx<T> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        if constexpr (MU == 0) {          // h0 = p0 + S i p3, h1 = p1 + S i p2
            h[c] = cadd(p0, pmi<T, S>(p3));
            h[3 + c] = cadd(p1, pmi<T, S>(p2));
        } else if constexpr (MU == 1) {   // h0 = p0 - S p3, h1 = p1 + S p2
            h[c] = S > 0 ? csub(p0, p3) : cadd(p0, p3);
            h[3 + c] = S > 0 ? cadd(p1, p2) : csub(p1, p2);
        } else if constexpr (MU == 2) {   // h0 = p0 + S i p2, h1 = p1 - S i p3
            h[c] = cadd(p0, pmi<T, S>(p2));
            h[3 + c] = csub(p1, pmi<T, S>(p3));
        } else {                          // h0 = p0 + S p2, h1 = p1 + S p3
            h[c] = S > 0 ? cadd(p0, p2) : csub(p0, p2);
            h[3 + c] = S > 0 ? cadd(p1, p3) : csub(p1, p3);
        }
    }
}

// acc += (1 + S gamma_mu) psi, given h = the projected (and colour-rotated) half spinor
template <typename T, int MU, int S>
__device__ __forceinline__ void reconstruct_add(cx<T> (&acc)[12], const cx<T> (&h)[6])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cx<T> h0 = h[c], h1 = h[3 + c];
        acc[c] = cadd(acc[c], h0);
        acc[3 + c] = cadd(acc[3 + c], h1);
        if constexpr (MU == 0) {          // rows 2,3 = -S i h1, -S i h0
            acc[6 + c] = csub(acc[6 + c], pmi<T, S>(h1));
            acc[9 + c] = csub(acc[9 + c], pmi<T, S>(h0));
        } else if constexpr (MU == 1) {   // rows 2,3 = S h1, -S h0
            acc[6 + c] = S > 0 ? cadd(acc[6 + c], h1) : csub(acc[6 + c], h1);
            acc[9 + c] = S > 0 ? csub(acc[9 + c], h0) : cadd(acc[9 + c], h0);
        } else if constexpr (MU == 2) {   // rows 2,3 = -S i h0, S i h1
            acc[6 + c] = csub(acc[6 + c], pmi<T, S>(h0));
            acc[9 + c] = cadd(acc[9 + c], pmi<T, S>(h1));
        } else {                          // rows 2,3 = S h0, S h1
            acc[6 + c] = S > 0 ? cadd(acc[6 + c], h0) : csub(acc[6 + c], h0);
            acc[9 + c] = S > 0 ? cadd(acc[9 + c], h1) : csub(acc[9 + c], h1);
        }
    }
}

// acc += k (1 + S gamma_mu) psi, given the unscaled half spinor h (the scale folded into FMAs)
template <typename T, int MU, int S>
__device__ __forceinline__ void reconstruct_add_k(cx<T> (&acc)[12], const cx<T> (&h)[6], T k)
{
    auto fma_c = [](T kk, cx<T> v, cx<T> a) { return cx<T>{fmadd(kk, v.re, a.re), fmadd(kk, v.im, a.im)}; };
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const cx<T> h0 = h[c], h1 = h[3 + c];
        acc[c] = fma_c(k, h0, acc[c]);
        acc[3 + c] = fma_c(k, h1, acc[3 + c]);
        if constexpr (MU == 0) {          // rows 2,3 = -S i h1, -S i h0
            acc[6 + c] = fma_c(-k, pmi<T, S>(h1), acc[6 + c]);
            acc[9 + c] = fma_c(-k, pmi<T, S>(h0), acc[9 + c]);
        } else if constexpr (MU == 1) {   // rows 2,3 = S h1, -S h0
            acc[6 + c] = fma_c(S > 0 ? k : -k, h1, acc[6 + c]);
            acc[9 + c] = fma_c(S > 0 ? -k : k, h0, acc[9 + c]);
        } else if constexpr (MU == 2) {   // rows 2,3 = -S i h0, S i h1
            acc[6 + c] = fma_c(-k, pmi<T, S>(h0), acc[6 + c]);
            acc[9 + c] = fma_c(k, pmi<T, S>(h1), acc[9 + c]);
        } else {                          // rows 2,3 = S h0, S h1
            acc[6 + c] = fma_c(S > 0 ? k : -k, h0, acc[6 + c]);
            acc[9 + c] = fma_c(S > 0 ? k : -k, h1, acc[9 + c]);
        }
    }
}

// ---------------------------------------------------------------------------
// links
// ---------------------------------------------------------------------------

// Raw storage units of N complex values of one site, as loaded (FP16: unpacked later).
template <class P, int N>
struct Raw {
    static_assert(N % P::cpu == 0, "FP16 objects hold an even number of complex values");
    typename P::unit u[N / P::cpu];
};

template <class P, int N>
__device__ __forceinline__ void unpack_raw(const Raw<P, N>& r, cx<typename P::real> (&v)[N])
{
    if constexpr (P::id == PREC_F16) {
#pragma unroll
        for (int c = 0; c < N / 2; c++) CxIO<P16, 2>::unpack(r.u[c], v[2 * c], v[2 * c + 1]);
    } else {
#pragma unroll
        for (int c = 0; c < N; c++) v[c] = {r.u[c].x, r.u[c].y};
    }
}

template <int RECON> constexpr int link_cx() { return RECON == 18 ? 9 : 6; }

// The N storage units of site j (object of N units) through a buffer resource: one 16-byte
// load per unit pair (8-byte units) or per unit (16-byte units), a last odd unit alone.
template <class P, int N, int AUX>
__device__ __forceinline__ void load_units(__amdgpu_buffer_rsrc_t rs, int j, Raw<P, N>& out)
{
    using U = typename P::unit;
    constexpr int NU = N / P::cpu;
    if constexpr (sizeof(U) == 16) {
#pragma unroll
        for (int c = 0; c < NU; c++) {
            const bq_u4v v = buf_load16<AUX>(rs, (uint32_t)toff<U>(j, c, NU) * 16u);
            out.u[c] = __builtin_bit_cast(U, v);
        }
    } else {
#pragma unroll
        for (int c = 0; c + 1 < NU; c += 2) {
            const bq_u4v v = buf_load16<AUX>(rs, (uint32_t)toff<U>(j, c, NU) * 8u);
            out.u[c] = __builtin_bit_cast(U, bq_u2v_b{v.x, v.y});
            out.u[c + 1] = __builtin_bit_cast(U, bq_u2v_b{v.z, v.w});
        }
        if constexpr (NU & 1) out.u[NU - 1] = __builtin_bit_cast(U, buf_load8<AUX>(rs, (uint32_t)toff<U>(j, NU - 1, NU) * 8u));
    }
}

// link from its stored rows; with 12-real storage the third row of the SU(3) matrix is
// conj(row0 x row1)
template <class P, int RECON>
__device__ __forceinline__ void link_from_raw(const Raw<P, link_cx<RECON>()>& r, cx<typename P::real> (&u)[9])
{
    using T = typename P::real;
    if constexpr (RECON == 18) {
        unpack_raw<P, 9>(r, u);
    } else {
        cx<T> w[6];
        unpack_raw<P, 6>(r, w);
#pragma unroll
        for (int k = 0; k < 6; k++) u[k] = w[k];
        const cx<T> w0 = csub(cmul(w[1], w[5]), cmul(w[2], w[4]));
        const cx<T> w1 = csub(cmul(w[2], w[3]), cmul(w[0], w[5]));
        const cx<T> w2 = csub(cmul(w[0], w[4]), cmul(w[1], w[3]));
        u[6] = {w0.re, -w0.im};
        u[7] = {w1.re, -w1.im};
        u[8] = {w2.re, -w2.im};
    }
}

template <typename T>
__device__ __forceinline__ void mul_U(const cx<T> (&u)[9], const cx<T> (&h)[6], cx<T> (&y)[6])
{
#pragma unroll
    for (int k = 0; k < 2; k++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cx<T> s = cmul(u[a * 3 + 0], h[k * 3 + 0]);
            s = cmac(s, u[a * 3 + 1], h[k * 3 + 1]);
            s = cmac(s, u[a * 3 + 2], h[k * 3 + 2]);
            y[k * 3 + a] = s;
        }
}

template <typename T>
__device__ __forceinline__ void mul_Ud(const cx<T> (&u)[9], const cx<T> (&h)[6], cx<T> (&y)[6])
{
#pragma unroll
    for (int k = 0; k < 2; k++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cx<T> s = {T(0), T(0)};
            s = cmacc(s, u[0 * 3 + a], h[k * 3 + 0]);
            s = cmacc(s, u[1 * 3 + a], h[k * 3 + 1]);
            s = cmacc(s, u[2 * 3 + a], h[k * 3 + 2]);
            y[k * 3 + a] = s;
        }
}

// ---------------------------------------------------------------------------
// one hop product y = k U (1 + S gamma_mu) psi (BW: U^dag), from raw storage: unpack,
// project, scale the half spinor, multiply.  FP16 storage is unpacked to FP32 and all
// arithmetic is FP32; its factor k (site scale, times e^{+-mu} in time) is folded into the
// FMAs of the reconstruction by the caller instead (SCALE = false).
// ---------------------------------------------------------------------------

template <class P, int RECON, bool BW>
struct PLink {
    cx<typename P::real> u[9];
};

template <class P, int RECON, bool BW>
__device__ __forceinline__ void prep_link(const Raw<P, link_cx<RECON>()>& raw, PLink<P, RECON, BW>& L)
{
    link_from_raw<P, RECON>(raw, L.u);
}

template <class P, int RECON, int MU, int S, bool BW, bool SCALE>
__device__ __forceinline__ void hop_product(const PLink<P, RECON, BW>& L, const Raw<P, 12>& sp,
                                            typename P::real k, cx<typename P::real> (&y)[6])
{
    using T = typename P::real;
    cx<T> p[12], h[6];
    unpack_raw<P, 12>(sp, p);
    project<T, MU, S>(p, h);
    if constexpr (SCALE) {
#pragma unroll
        for (int q = 0; q < 6; q++) h[q] = cscale(k, h[q]);
    }
    if constexpr (BW) mul_Ud(L.u, h, y);
    else mul_U(L.u, h, y);
}

// ---------------------------------------------------------------------------
// clover: two packed Hermitian 6x6 blocks per site, 18 complex each:
//   [0..2]  diagonal (d0 + i d1, d2 + i d3, d4 + i d5)
//   [3..17] strictly lower triangle A[i][j], i > j, at 3 + i(i-1)/2 + j
// block 0 acts on spins 0,1 (components 0..5), block 1 on spins 2,3.
// ---------------------------------------------------------------------------

template <class P, int LA>
__device__ __forceinline__ void load_clover_block(const typename P::unit* __restrict__ C, int j, int blk,
                                                  cx<typename P::real> (&c)[18])
{
    using U = typename P::unit;
    constexpr int NU = 36 / P::cpu;  // units of both blocks
    // The resource starts at the wave's own tile (j's tile is uniform over the wave), so offsets
    // stay within one tile: an FP64 clover array of a large lattice exceeds 4 GiB.
    const int tile = __builtin_amdgcn_readfirstlane(j >> kTileLog);
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(C + (size_t)tile * NU * kTile);
    j &= kTile - 1;
    auto single = [&](int g) {
        if constexpr (sizeof(U) == 16) return __builtin_bit_cast(U, buf_load16<LA>(rs, (uint32_t)toff<U>(j, g, NU) * 16u));
        else return __builtin_bit_cast(U, buf_load8<LA>(rs, (uint32_t)toff<U>(j, g, NU) * 8u));
    };
    auto pair = [&](int g, U& a, U& b) {  // g even: units g, g+1 with one 16-byte load
        if constexpr (sizeof(U) == 8) {
            const bq_u4v v = buf_load16<LA>(rs, (uint32_t)toff<U>(j, g, NU) * 8u);
            a = __builtin_bit_cast(U, bq_u2v_b{v.x, v.y});
            b = __builtin_bit_cast(U, bq_u2v_b{v.z, v.w});
        }
    };
    if constexpr (P::id == PREC_F64) {
#pragma unroll
        for (int k = 0; k < 18; k++) {
            const U t = single(blk * 18 + k);
            c[k] = {t.x, t.y};
        }
    } else if constexpr (P::id == PREC_F32) {
#pragma unroll
        for (int m = 0; m < 9; m++) {
            U a, b;
            pair(blk * 18 + 2 * m, a, b);
            c[2 * m] = {a.x, a.y};
            c[2 * m + 1] = {b.x, b.y};
        }
    } else {  // 9 units per block: block 0 is units 0..8, block 1 units 9..17
        U u[9];
        if (blk == 0) {
#pragma unroll
            for (int m = 0; m < 4; m++) pair(2 * m, u[2 * m], u[2 * m + 1]);
            u[8] = single(8);
        } else {
            u[0] = single(9);
#pragma unroll
            for (int m = 0; m < 4; m++) pair(10 + 2 * m, u[1 + 2 * m], u[2 + 2 * m]);
        }
#pragma unroll
        for (int k = 0; k < 9; k++) CxIO<P16, 2>::unpack(u[k], c[2 * k], c[2 * k + 1]);
    }
}

// the same block from a tile's clover copy in LDS, laid out [unit][lane]
template <class P>
__device__ __forceinline__ void load_clover_block_lds(const typename P::unit* S, int lane, int blk,
                                                      cx<typename P::real> (&c)[18])
{
    if constexpr (P::id == PREC_F16) {
#pragma unroll
        for (int k = 0; k < 9; k++) CxIO<P16, 2>::unpack(S[(blk * 9 + k) * kTile + lane], c[2 * k], c[2 * k + 1]);
    } else {
#pragma unroll
        for (int k = 0; k < 18; k++) {
            const auto t = S[(blk * 18 + k) * kTile + lane];
            c[k] = {t.x, t.y};
        }
    }
}

template <typename T>
__device__ __forceinline__ void clover_mul(const cx<T> (&c)[18], const cx<T>* x, cx<T>* y)
{
    const T d[6] = {c[0].re, c[0].im, c[1].re, c[1].im, c[2].re, c[2].im};
#pragma unroll
    for (int i = 0; i < 6; i++) y[i] = cscale(d[i], x[i]);
#pragma unroll
    for (int i = 1; i < 6; i++)
#pragma unroll
        for (int jj = 0; jj < i; jj++) {
            const cx<T> A = c[3 + i * (i - 1) / 2 + jj];
            y[i] = cmac(y[i], A, x[jj]);
            y[jj] = cmacc(y[jj], A, x[i]);
        }
}

// clover_mul with the block read from the tile's LDS copy entry by entry as it is used (FP32 and
// FP64 storage), instead of all 18 entries into registers first: the same products in the same
// order, with 36 fewer values live
template <class P>
__device__ __forceinline__ void clover_mul_lds(const typename P::unit* S, int lane, int blk,
                                               const cx<typename P::real>* x, cx<typename P::real>* y)
{
    static_assert(P::id != PREC_F16, "FP16 clover units hold two entries");
    using T = typename P::real;
    auto entry = [&](int k) {
        const auto t = S[(blk * 18 + k) * kTile + lane];
        return cx<T>{t.x, t.y};
    };
    const cx<T> d01 = entry(0), d23 = entry(1), d45 = entry(2);
    const T d[6] = {d01.re, d01.im, d23.re, d23.im, d45.re, d45.im};
#pragma unroll
    for (int i = 0; i < 6; i++) y[i] = cscale(d[i], x[i]);
#pragma unroll
    for (int i = 1; i < 6; i++)
#pragma unroll
        for (int jj = 0; jj < i; jj++) {
            const cx<T> A = entry(3 + i * (i - 1) / 2 + jj);
            y[i] = cmac(y[i], A, x[jj]);
            y[jj] = cmacc(y[jj], A, x[i]);
        }
}

// half of a spinor (block `blk`: complex 6*blk .. 6*blk+5) for FP32/FP64 storage
template <class P>
__device__ __forceinline__ void load_spinor_part(const SpinorPtr<P>& f, int col, int j, int blk,
                                                 cx<typename P::real> (&v)[6])
{
    if constexpr (P::id == PREC_F16) {
        const uint2* b = f.d + col * f.cstride;
        float s = f.s[col * f.sstride + j];
#pragma unroll
        for (int u = 0; u < 3; u++) {
            CxIO<P16, 2>::unpack(at(b, j, blk * 3 + u, 6), v[2 * u], v[2 * u + 1]);
            v[2 * u] = cscale(s, v[2 * u]);
            v[2 * u + 1] = cscale(s, v[2 * u + 1]);
        }
    } else {
        const typename P::unit* b = f.d + col * f.cstride;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            auto t = at(b, j, blk * 6 + k, 12);
            v[k] = {t.x, t.y};
        }
    }
}

// ---------------------------------------------------------------------------
// kernel
// ---------------------------------------------------------------------------

template <class P, class PR>
struct Args {
    Geom g;
    int parity, ncol;
    const typename P::unit* U[8];
    SpinorPtr<P> in, out, v;
    SpinorPtr<PR> rin, rout;
    const typename P::unit* clov;
    const double* alpha;
    double* partial;
    int nwaves, pstride;
    int tpb, gw, nch;  // tiles per workgroup, column groups per workgroup, group chunks
    int nblk;          // tile blocks
    const int* status;
    int statmask;
    typename P::real ef, eb, ef_bc, eb_bc;  // time coefficients, without / with the boundary sign
    typename P::real f, a;
    // per-column operators (columns of different kappa on one gauge field): clover blocks and f
    int percol;
    const typename P::unit* cclov[kMaxCols];
    typename P::real cf[kMaxCols];
};

template <bool PC, class P, class PR>
__device__ __forceinline__ typename P::real colf(const Args<P, PR>& A, int c)
{
    if constexpr (PC) return A.cf[c];
    else return A.f;
}

// End of one hop's phase.  Without it the compiler issues the loads of all
// eight hops first and sinks their arithmetic to the end of the kernel, which
// keeps every loaded value live and spills.  Pinning the accumulators in
// registers forces each hop's arithmetic to finish before the next hop's
// loads are issued.
template <typename T, int R>
__device__ __forceinline__ void phase_end(const bool (&act)[R], cx<T> (&acc)[R][12])
{
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int k = 0; k < 12; k++) asm volatile("" : "+v"(acc[r][k].re), "+v"(acc[r][k].im));
    asm volatile("" ::: "memory");
}

// The 8 half hops of the stencil, H = 2*mu + (0 forward, 1 backward).  A half hop's raw data
// is its link and the R neighbour spinors.  With prefetching, the raw data of the next half hop
// is loaded before the arithmetic of the current one, so that every wave keeps loads in flight
// while it computes; without, each column's spinor is loaded just before its arithmetic.
template <class P, int R, int RECON>
struct HalfHop {
    int jn;                                // neighbour site
    Raw<P, link_cx<RECON>()> link;
    Raw<P, 12> sp[R];
    float sc[P::id == PREC_F16 ? R : 1];  // FP16 spinor scales
};

template <class P, class PR, int R, int RECON>
__device__ __forceinline__ void hh_load_spinor(const Args<P, PR>& A, int c, int r, HalfHop<P, R, RECON>& d)
{
    load_units<P, 12, 0>(buf_rsrc(A.in.d + c * A.in.cstride), d.jn, d.sp[r]);
    if constexpr (P::id == PREC_F16) d.sc[r] = buf_load4f(buf_rsrc(A.in.s + c * A.in.sstride), (uint32_t)d.jn * 4u);
}

// neighbour index and link of half hop H: forward U_mu(x) stored at x, backward U_mu(x - mu)
// stored at the neighbour (other parity)
template <class P, class PR, int R, int RECON, int H, int LA>
__device__ __forceinline__ void hh_load_link(const Args<P, PR>& A, const Site& s, HalfHop<P, R, RECON>& d)
{
    constexpr int MU = H >> 1;
    constexpr bool BW = H & 1;
    d.jn = nbr(A.g, s, MU, BW ? -1 : +1);
    const typename P::unit* __restrict__ U = A.U[(BW ? 1 - A.parity : A.parity) * 4 + MU];
    const int jl = BW ? d.jn : s.j;
    load_units<P, link_cx<RECON>(), LA>(buf_rsrc(U), jl, d.link);
}

template <class P, class PR, int R, int RECON, int H, int LA>
__device__ __forceinline__ void hh_load(const Args<P, PR>& A, const Site& s, const bool (&act)[R], int c0,
                                        HalfHop<P, R, RECON>& d)
{
    hh_load_link<P, PR, R, RECON, H, LA>(A, s, d);
#pragma unroll
    for (int r = 0; r < R; r++)
        if (act[r]) hh_load_spinor(A, c0 + r, r, d);
}

// forward:  acc += f U_mu(x) (1 + SF gamma_mu) psi(x + mu)
// backward: acc += f U_mu(x - mu)^dag (1 - SF gamma_mu) psi(x - mu)
// SF = -1 for M, +1 for the adjoint; f = e^{+-mu} (times the boundary sign) in time, else 1.
// LOAD: load each column's spinor here, just before its arithmetic.
template <class P, class PR, int R, int DAG, int RECON, int H, bool LOAD>
__device__ __forceinline__ void hh_compute(const Args<P, PR>& A, const Site& s, const bool (&act)[R], int c0,
                                           HalfHop<P, R, RECON>& d, cx<typename P::real> (&acc)[R][12])
{
    using T = typename P::real;
    constexpr int MU = H >> 1;
    constexpr bool BW = H & 1;
    constexpr int S = (DAG ? +1 : -1) * (BW ? -1 : +1);
    PLink<P, RECON, BW> L;
    prep_link<P, RECON, BW>(d.link, L);
    T coef = T(1);
    if constexpr (MU == 3) {
        if constexpr (BW) coef = (s.t == 0) ? A.eb_bc : A.eb;
        else coef = (s.t == A.g.L[3] - 1) ? A.ef_bc : A.ef;
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        if (!act[r]) continue;
        if constexpr (LOAD) hh_load_spinor(A, c0 + r, r, d);
        cx<T> y[6];
        if constexpr (P::id == PREC_F16) {
            hop_product<P, RECON, MU, S, BW, false>(L, d.sp[r], T(1), y);
            reconstruct_add_k<T, MU, S>(acc[r], y, (MU == 3) ? coef * d.sc[r] : d.sc[r]);
        } else {
            hop_product<P, RECON, MU, S, BW, MU == 3>(L, d.sp[r], coef, y);
            reconstruct_add<T, MU, S>(acc[r], y);
        }
    }
}

// Loading one half hop ahead doubles the raw data held in registers; it is used where the
// two buffers fit without spilling (one FP64 column, up to two FP32, up to three FP16).
template <class P, int R>
constexpr bool prefetch_hops()
{
    return P::id == PREC_F64 ? R <= 1 : (P::id == PREC_F32 ? R <= 2 : R <= 3);
}

template <class P, class PR, int R, int DAG, int RECON, int H, bool PF, int LA>
__device__ __forceinline__ void hh_step(const Args<P, PR>& A, const Site& s, const bool (&act)[R], int c0,
                                        HalfHop<P, R, RECON> (&d)[2], cx<typename P::real> (&acc)[R][12])
{
    if constexpr (PF) {
        if constexpr (H < 7) hh_load<P, PR, R, RECON, H + 1, LA>(A, s, act, c0, d[(H + 1) & 1]);
        hh_compute<P, PR, R, DAG, RECON, H, false>(A, s, act, c0, d[H & 1], acc);
    } else {
        hh_load_link<P, PR, R, RECON, H, LA>(A, s, d[0]);
        hh_compute<P, PR, R, DAG, RECON, H, true>(A, s, act, c0, d[0], acc);
    }
    phase_end(act, acc);
}

template <class P, class PR, int R, int DAG, int RECON, int LA>
__device__ __forceinline__ void hop_all(const Args<P, PR>& A, const Site& s, const bool (&act)[R], int c0,
                                        cx<typename P::real> (&acc)[R][12])
{
    constexpr bool PF = prefetch_hops<P, R>();
    HalfHop<P, R, RECON> d[2];
    if constexpr (PF) hh_load<P, PR, R, RECON, 0, LA>(A, s, act, c0, d[0]);
    hh_step<P, PR, R, DAG, RECON, 0, PF, LA>(A, s, act, c0, d, acc);
    hh_step<P, PR, R, DAG, RECON, 1, PF, LA>(A, s, act, c0, d, acc);
    hh_step<P, PR, R, DAG, RECON, 2, PF, LA>(A, s, act, c0, d, acc);
    hh_step<P, PR, R, DAG, RECON, 3, PF, LA>(A, s, act, c0, d, acc);
    hh_step<P, PR, R, DAG, RECON, 4, PF, LA>(A, s, act, c0, d, acc);
    hh_step<P, PR, R, DAG, RECON, 5, PF, LA>(A, s, act, c0, d, acc);
    hh_step<P, PR, R, DAG, RECON, 6, PF, LA>(A, s, act, c0, d, acc);
    hh_step<P, PR, R, DAG, RECON, 7, PF, LA>(A, s, act, c0, d, acc);
}

// Epilogue of one tile for R columns: the linear combination and clover factor the caller
// asked for (EPI), the store, and for EPI_TV / EPI_TVR the per-wave |.|^2 partials.  Lanes with
// no active column pass nrm = 0 to the wave reduction.
// SL: the workgroup staged the tile's (shared) clover in LDS at sclov
template <class P, class PR, int R, int EPI, bool PC, int LA, bool SL = false>
__device__ __forceinline__ void epilogue(const Args<P, PR>& A, int j, const bool (&act)[R], bool any, int c0,
                                         cx<typename P::real> (&acc)[R][12],
                                         const typename P::unit* sclov = nullptr)
{
    static_assert(!(SL && PC), "per-column clover is not staged");
    // FP32 and FP64 read the staged clover entry by entry inside the multiply (cmul_blk); FP16
    // units hold two entries and are unpacked whole
    constexpr bool STREAM = SL && P::id != PREC_F16;
    auto clover_block = [&](const typename P::unit* C, int blk, cx<typename P::real>(&cb)[18]) {
        if constexpr (STREAM) {
            (void)C, (void)blk, (void)cb;
        } else if constexpr (SL) {
            load_clover_block_lds<P>(sclov, j & (kTile - 1), blk, cb);
        } else {
            load_clover_block<P, PC ? kBufNT : LA>(C, j, blk, cb);
        }
    };
    auto cmul_blk = [&](const cx<typename P::real>(&cb)[18], int blk, const cx<typename P::real>* x,
                        cx<typename P::real>* y) {
        if constexpr (STREAM) clover_mul_lds<P>(sclov, j & (kTile - 1), blk, x, y);
        else clover_mul(cb, x, y);
    };
    using T = typename P::real;
    using TR = typename PR::real;
    constexpr int CA = PC ? kBufNT : LA;  // per-column clover is read by one wave only
    double nrm[R];
#pragma unroll
    for (int r = 0; r < R; r++) nrm[r] = 0.0;
    if (any) {
    if constexpr (EPI == EPI_HOP || EPI == EPI_TINV) {
        // w = a*v + f*hop
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (!act[r]) continue;
            const T f = colf<PC>(A, c0 + r);
            if (A.v.d != nullptr) {
                cx<T> v[12];
                load_spinor(A.v, c0 + r, j, v);
#pragma unroll
                for (int k = 0; k < 12; k++) acc[r][k] = caxpy(f, acc[r][k], cscale(A.a, v[k]));
            } else {
#pragma unroll
                for (int k = 0; k < 12; k++) acc[r][k] = cscale(f, acc[r][k]);
            }
        }
        if constexpr (EPI == EPI_TINV) {
#pragma unroll
            for (int blk = 0; blk < 2; blk++) {
                cx<T> cb[18];
                if constexpr (!PC) clover_block(A.clov, blk, cb);
#pragma unroll
                for (int r = 0; r < R; r++) {
                    if (!act[r]) continue;
                    if constexpr (PC) load_clover_block<P, CA>(A.cclov[c0 + r], j, blk, cb);
                    cx<T> x[6];
#pragma unroll
                    for (int k = 0; k < 6; k++) x[k] = acc[r][blk * 6 + k];
                    cmul_blk(cb, blk, x, &acc[r][blk * 6]);
                }
                phase_end(act, acc);
            }
        }
#pragma unroll
        for (int r = 0; r < R; r++)
            if (act[r]) store_spinor<P, true>(A.out, c0 + r, j, acc[r]);
    } else if constexpr (EPI == EPI_TV) {
        // out = C v + f*hop, assembled in place (FP16 storage needs the whole site for its scale)
#pragma unroll
        for (int blk = 0; blk < 2; blk++) {
            cx<T> cb[18];
            if constexpr (!PC) clover_block(A.clov, blk, cb);
#pragma unroll
            for (int r = 0; r < R; r++) {
                if (!act[r]) continue;
                if constexpr (PC) load_clover_block<P, CA>(A.cclov[c0 + r], j, blk, cb);
                const T f = colf<PC>(A, c0 + r);
                cx<T> x[6], y[6];
                load_spinor_part(A.v, c0 + r, j, blk, x);
                cmul_blk(cb, blk, x, y);
                // |out|^2 in FP64 as the block is assembled (the terms in site order, as summed
                // over the whole site)
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    acc[r][blk * 6 + k] = caxpy(f, acc[r][blk * 6 + k], y[k]);
                    const cx<T> o = acc[r][blk * 6 + k];
                    nrm[r] += (double)o.re * o.re + (double)o.im * o.im;
                }
            }
            phase_end(act, acc);
        }
#pragma unroll
        for (int r = 0; r < R; r++)
            if (act[r]) store_spinor(A.out, c0 + r, j, acc[r]);
    } else {
        // w = C v + f*hop ; r_out = r_in - alpha*w, one clover block (half spinor) at a time
        static_assert(PR::id != PREC_F16, "the residual is kept in FP32 or FP64");
#pragma unroll
        for (int blk = 0; blk < 2; blk++) {
            cx<T> cb[18];
            if constexpr (!PC) clover_block(A.clov, blk, cb);
#pragma unroll
            for (int r = 0; r < R; r++) {
                if (!act[r]) continue;
                const int c = c0 + r;
                if constexpr (PC) load_clover_block<P, CA>(A.cclov[c], j, blk, cb);
                const T f = colf<PC>(A, c);
                const TR al = A.alpha ? (TR)A.alpha[c] : TR(1);
                cx<T> x[6], y[6];
                load_spinor_part(A.v, c, j, blk, x);
                cmul_blk(cb, blk, x, y);
                cx<TR> rv[6];
                load_spinor_part(A.rin, c, j, blk, rv);
                typename PR::unit* rb = A.rout.d + c * A.rout.cstride;
                double n = 0.0;
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    const cx<T> w = caxpy(f, acc[r][blk * 6 + k], y[k]);
                    rv[k].re = fmadd(-al, (TR)w.re, rv[k].re);
                    rv[k].im = fmadd(-al, (TR)w.im, rv[k].im);
                    st_stream(&at(rb, j, blk * 6 + k, 12), {rv[k].re, rv[k].im});
                    n += (double)rv[k].re * rv[k].re + (double)rv[k].im * rv[k].im;
                }
                nrm[r] += n;
            }
            phase_end(act, acc);
        }
    }
    }
    if constexpr (EPI == EPI_TV || EPI == EPI_TVR) {
        if (A.partial != nullptr) {
            const int wave = j >> kTileLog;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const double t = wave_sum(nrm[r]);
                const int c = c0 + r;
                if ((threadIdx.x & 63) == 0 && c < A.ncol && wave < A.nwaves && col_selected(A.status, A.statmask, c))
                    A.partial[(size_t)c * A.pstride + wave] = t;
            }
        }
    }
}

// One work item: tile block `tblk` (tpb tiles) x column-group chunk `chunk` (gw groups of R
// columns).  Wave w of the workgroup handles tile w / gw and group w % gw, so all groups of a
// tile run side by side and share the links and clover through L1/L2.
template <class P, class PR, int R, int DAG, int EPI, int RECON, bool PC, int LA>
__device__ __forceinline__ void hop_item(const Args<P, PR>& A, int tblk, int chunk)
{
    using T = typename P::real;
    const int w = threadIdx.x >> kTileLog;
    const int lane = threadIdx.x & (kTile - 1);
    const int gl = w % A.gw;
    const int lt = tblk * A.tpb + w / A.gw;
    const int grp = chunk * A.gw + gl;
    const int j = lt < A.g.ntiles ? tile_at(A.g, lt) * kTile + lane : A.g.ntiles * kTile;
    const int c0 = __builtin_amdgcn_readfirstlane(grp * R);  // uniform over the wave
    bool act[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int c = c0 + r;
        act[r] = j < A.g.Vh && c < A.ncol && col_selected(A.status, A.statmask, c);
        any |= act[r];
    }
    cx<T> acc[R][12];
    if (any) {
        const Site s = site_of(A.g, A.parity, j);
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
            for (int k = 0; k < 12; k++) acc[r][k] = {T(0), T(0)};
        hop_all<P, PR, R, DAG, RECON, LA>(A, s, act, c0, acc);
    }
    epilogue<P, PR, R, EPI, PC, LA>(A, j, act, any, c0, acc);
}

// ---------------------------------------------------------------------------
// t-marching variant (lattices whose (x,y) planes hold whole tiles)
//
// A wave owns one tile position (x,y block and z) and R columns and walks `seg` consecutive
// time planes.  Lane i keeps its (x,y,z) block position, and the cb index of its site moves
// by whole tiles from plane to plane, so the time neighbours of lane i are lane i of the same
// tile position one plane up or down.  The site of lane i on plane t+2 is the site on plane t
// shifted by 2 in time, so the backward time hop of plane t+2 reads the spinor that the
// forward time hop of plane t reads: that term is computed then, from the same load, and kept
// in registers for two planes.  Waves of neighbouring z positions march side by side, so the
// z hops of one wave read the data its neighbours have just loaded.
// ---------------------------------------------------------------------------

// y = f U_t(x - t)^dag (1 - SF gamma_t) psi(x - t) for the output site whose backward time
// neighbour is the half hop's neighbour site, for each active column
// (FP16: y unscaled, its factor in ky)
template <class P, class PR, int R, int DAG, int RECON>
__device__ __forceinline__ void t_backward(const HalfHop<P, R, RECON>& d, const PLink<P, RECON, true>& L,
                                           typename P::real coef, const bool (&act)[R],
                                           cx<typename P::real> (&y)[R][6], typename P::real (&ky)[R])
{
    constexpr int S = DAG ? -1 : +1;
#pragma unroll
    for (int r = 0; r < R; r++) {
        if (!act[r]) continue;
        if constexpr (P::id == PREC_F16) {
            hop_product<P, RECON, 3, S, true, false>(L, d.sp[r], 1.0f, y[r]);
            ky[r] = coef * d.sc[r];
        } else {
            hop_product<P, RECON, 3, S, true, true>(L, d.sp[r], coef, y[r]);
        }
    }
}

template <class P, class PR, int R, int DAG, int RECON>
__device__ __forceinline__ void t_link(const Args<P, PR>& A, int par, int jl, PLink<P, RECON, true>& L)
{
    constexpr int LU = link_cx<RECON>() / P::cpu;
    Raw<P, link_cx<RECON>()> raw;
    const typename P::unit* __restrict__ U = A.U[par * 4 + 3];
#pragma unroll
    for (int k = 0; k < LU; k++) raw.u[k] = ld_stream(&at(U, jl, k, LU));
    prep_link<P, RECON, true>(raw, L);
}

template <class P, class PR, int R, int DAG, int EPI, int RECON, bool PC, int LA>
__global__ __launch_bounds__(512) void k_hop_march(const Args<P, PR> A, int npos, int seg, int nseg)
{
    using T = typename P::real;
    constexpr int SB = DAG ? -1 : +1;  // backward projector (1 + SB gamma_t)
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int ch = lb % A.nch;
    const int rest = lb / A.nch;
    const int pos = rest % npos;
    const int sg = rest / npos;
    const int w = threadIdx.x >> kTileLog;
    const int lane = threadIdx.x & (kTile - 1);
    const int c0 = __builtin_amdgcn_readfirstlane((ch * A.gw + w) * R);  // uniform over the wave
    const int Lt = A.g.L[3];
    bool act[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int c = c0 + r;
        act[r] = c < A.ncol && col_selected(A.status, A.statmask, c);
        any |= act[r];
    }
    if (!any) return;  // uniform over the wave: no column of this group is selected
    const int t0 = sg * seg;
    auto site_at = [&](int t) { return site_of(A.g, A.parity, (pos + npos * t) * kTile + lane); };

    // backward time terms of the current plane (B0) and the next (B1); the arrays are swapped
    // after each plane so that they are indexed by constants only and stay in registers
    cx<T> B0[R][6], B1[R][6];
    T K0[R], K1[R];  // FP16: factors of B0, B1
#pragma unroll
    for (int q = 0; q < 2; q++) {
        const int t = (t0 + q) % Lt;
        const Site s = site_at(t);
        HalfHop<P, R, RECON> d;
        hh_load<P, PR, R, RECON, 7, LA>(A, s, act, c0, d);
        PLink<P, RECON, true> L;
        prep_link<P, RECON, true>(d.link, L);
        t_backward<P, PR, R, DAG, RECON>(d, L, t == 0 ? A.eb_bc : A.eb, act, q == 0 ? B0 : B1, q == 0 ? K0 : K1);
    }

    for (int i = 0; i < seg; i++) {
        const int t = t0 + i;
        const Site s = site_at(t);
        cx<T> acc[R][12];
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
            for (int k = 0; k < 12; k++) acc[r][k] = {T(0), T(0)};
        // the carried terms take the registers of a second prefetch buffer: no prefetching here
        HalfHop<P, R, RECON> d[2];
        hh_step<P, PR, R, DAG, RECON, 0, false, LA>(A, s, act, c0, d, acc);
        hh_step<P, PR, R, DAG, RECON, 1, false, LA>(A, s, act, c0, d, acc);
        hh_step<P, PR, R, DAG, RECON, 2, false, LA>(A, s, act, c0, d, acc);
        hh_step<P, PR, R, DAG, RECON, 3, false, LA>(A, s, act, c0, d, acc);
        hh_step<P, PR, R, DAG, RECON, 4, false, LA>(A, s, act, c0, d, acc);
        hh_step<P, PR, R, DAG, RECON, 5, false, LA>(A, s, act, c0, d, acc);
        // forward time hop; its spinors also give the backward time term of plane t + 2
        hh_load<P, PR, R, RECON, 6, LA>(A, s, act, c0, d[0]);
        hh_compute<P, PR, R, DAG, RECON, 6, false>(A, s, act, c0, d[0], acc);
        // backward time hop of plane t, kept from plane t - 2
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (!act[r]) continue;
            if constexpr (P::id == PREC_F16) reconstruct_add_k<T, 3, SB>(acc[r], B0[r], K0[r]);
            else reconstruct_add<T, 3, SB>(acc[r], B0[r]);
        }
        phase_end(act, acc);
        if (i + 2 < seg) {
            PLink<P, RECON, true> L;
            t_link<P, PR, R, DAG, RECON>(A, 1 - A.parity, d[0].jn, L);
            t_backward<P, PR, R, DAG, RECON>(d[0], L, (t + 2) % Lt == 0 ? A.eb_bc : A.eb, act, B0, K0);
        }
#pragma unroll
        for (int r = 0; r < R; r++) {
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const cx<T> b = B0[r][k];
                B0[r][k] = B1[r][k];
                B1[r][k] = b;
            }
            const T kk = K0[r];
            K0[r] = K1[r];
            K1[r] = kk;
        }
        epilogue<P, PR, R, EPI, PC, LA>(A, s.j, act, true, c0, acc);
    }
}

// One work item per workgroup; blocks are mapped XCD-contiguously (see xcd_remap).
template <class P, class PR, int R, int DAG, int EPI, int RECON, bool PC, int LA>
__global__ __launch_bounds__(512) void k_hop(const Args<P, PR> A)
{
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    int tblk, chunk;
    item_of(A.g, lb, A.nblk, A.nch, tblk, chunk);
    hop_item<P, PR, R, DAG, EPI, RECON, PC, LA>(A, tblk, chunk);
}

// ---------------------------------------------------------------------------
// Tile-shared variant for several column groups per tile (tune field `lds`).
//
// A workgroup owns one 64-site tile and up to 16 column-group waves.  It first loads the tile's
// 8 links per site (rebuilt to full 3x3 matrices) and, for a shared clover, the tile's clover
// blocks into LDS, once; every wave then reads them from LDS.  The waves of the plain kernel
// each read the same links and clover through the vector memory pipeline, whose address unit is
// what limits a multi-column launch; here each wave issues only its neighbour-spinor loads and
// its stores.  Per site and column the arithmetic is the plain kernel's, in the same order, so
// the results are bitwise equal.
// ---------------------------------------------------------------------------

template <class P>
struct LinkLds {
    using C = typename std::conditional<sizeof(typename P::real) == 8, double2, float2>::type;
};

// LDS bytes of a tile: links (8 x 9 complex in the real type of P) + clover units (shared clover)
template <class P, bool CLOV>
constexpr int tile_lds_bytes()
{
    return 8 * 9 * kTile * (int)sizeof(typename LinkLds<P>::C) +
           (CLOV ? clover_units<P>() * kTile * (int)sizeof(typename P::unit) : 0);
}

// Whether a launch stages the tile's clover: only epilogues that apply a clover read it (EPI_HOP
// launches have no clover array), per-column clover is read by one wave each, and FP64 keeps its
// clover in global memory since its links alone fill 72 KB of LDS per tile.
template <class P, bool PC, int EPI> constexpr bool clover_in_lds() { return !PC && P::id != PREC_F64 && EPI != EPI_HOP; }

// prefetch depth of the tile-shared kernel: neighbour spinors of the next NB - 1 half hops are in
// flight while a half hop computes (its links come from LDS and need no prefetch)
template <class P, int R> constexpr int lds_ring() { return 2; }

// value of lane `src` (0..63) of the wave, for every lane (ds_bpermute through the LDS crossbar)
__device__ __forceinline__ float lane_get(int src, float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_get(int src, double v)
{
    const int2 w = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_ds_bpermute(src << 2, w.x),
                                                __builtin_amdgcn_ds_bpermute(src << 2, w.y)));
}

// Half hop H (x or y direction) from the wave's own input tile: lane i holds the input-parity
// spinor with its own checkerboard index, base + i, which for most lanes is where an x or y
// neighbour lives.  Every lane projects its spinor with the half hop's projector and the
// destination lane takes it from the source lane; lanes whose neighbour lies outside the tile
// load it and project it themselves.  The arithmetic is the plain kernel's: the projection of
// the neighbour spinor, the SU(3) product and the reconstruction, in the same order.
template <class P, class PR, int DAG, int RECON, int H>
__device__ __forceinline__ void hh_xchg(const Args<P, PR>& A, const Site& s, bool act, int c0, int base,
                                        const Raw<P, 12>& own, float own_sc,
                                        const typename LinkLds<P>::C* __restrict__ lk, int lane,
                                        cx<typename P::real> (&acc)[12])
{
    using T = typename P::real;
    constexpr int MU = H >> 1;
    constexpr bool BW = H & 1;
    constexpr int S = (DAG ? +1 : -1) * (BW ? -1 : +1);
    static_assert(MU < 3, "time hops are loaded");
    const int jn = nbr(A.g, s, MU, BW ? -1 : +1);
    const int src = jn - base;
    const bool in = act && (unsigned)src < (unsigned)kTile;
    cx<T> h[6];
    {
        cx<T> p[12], hs[6];
        unpack_raw<P, 12>(own, p);
        project<T, MU, S>(p, hs);
        const int sl = src & (kTile - 1);
#pragma unroll
        for (int q = 0; q < 6; q++) h[q] = {lane_get(sl, hs[q].re), lane_get(sl, hs[q].im)};
    }
    float hsc = 1.0f;
    if constexpr (P::id == PREC_F16) hsc = lane_get(src & (kTile - 1), own_sc);
    if (act && !in) {  // neighbour outside the tile: load it
        HalfHop<P, 1, RECON> d;
        d.jn = jn;
        hh_load_spinor(A, c0, 0, d);
        cx<T> p[12];
        unpack_raw<P, 12>(d.sp[0], p);
        project<T, MU, S>(p, h);
        if constexpr (P::id == PREC_F16) hsc = d.sc[0];
    }
    PLink<P, RECON, BW> L;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const auto t = lk[(H * 9 + k) * kTile + lane];
        L.u[k] = {(T)t.x, (T)t.y};
    }
    if (act) {
        cx<T> y[6];
        if constexpr (BW) mul_Ud(L.u, h, y);
        else mul_U(L.u, h, y);
        if constexpr (P::id == PREC_F16) reconstruct_add_k<T, MU, S>(acc, y, hsc);
        else reconstruct_add<T, MU, S>(acc, y);
    }
    const bool a1[1] = {act};
    cx<T>(&acc1)[1][12] = *reinterpret_cast<cx<T>(*)[1][12]>(&acc);
    phase_end(a1, acc1);
}

template <class P, class PR, int R, int RECON, int NB, int H>
__device__ __forceinline__ void lds_issue(const Args<P, PR>& A, const Site& s, const bool (&act)[R], int c0,
                                          HalfHop<P, R, RECON> (&d)[NB])
{
    if constexpr (H < 8) {
        HalfHop<P, R, RECON>& nx = d[H % NB];
        nx.jn = nbr(A.g, s, H >> 1, (H & 1) ? -1 : +1);
#pragma unroll
        for (int r = 0; r < R; r++)
            if (act[r]) hh_load_spinor(A, c0 + r, r, nx);
    }
}

template <class P, class PR, int R, int DAG, int RECON, int NB, int H>
__device__ __forceinline__ void hh_step_lds(const Args<P, PR>& A, const Site& s, const bool (&act)[R], int c0,
                                            const typename LinkLds<P>::C* __restrict__ lk, int lane,
                                            HalfHop<P, R, RECON> (&d)[NB], cx<typename P::real> (&acc)[R][12])
{
    using T = typename P::real;
    constexpr int MU = H >> 1;
    constexpr bool BW = H & 1;
    constexpr int S = (DAG ? +1 : -1) * (BW ? -1 : +1);
    lds_issue<P, PR, R, RECON, NB, H + NB - 1>(A, s, act, c0, d);
    HalfHop<P, R, RECON>& cur = d[H % NB];
    PLink<P, RECON, BW> L;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const auto t = lk[(H * 9 + k) * kTile + lane];
        L.u[k] = {(T)t.x, (T)t.y};
    }
    T coef = T(1);
    if constexpr (MU == 3) {
        if constexpr (BW) coef = (s.t == 0) ? A.eb_bc : A.eb;
        else coef = (s.t == A.g.L[3] - 1) ? A.ef_bc : A.ef;
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        if (!act[r]) continue;
        cx<T> y[6];
        if constexpr (P::id == PREC_F16) {
            hop_product<P, RECON, MU, S, BW, false>(L, cur.sp[r], T(1), y);
            reconstruct_add_k<T, MU, S>(acc[r], y, (MU == 3) ? coef * cur.sc[r] : cur.sc[r]);
        } else {
            hop_product<P, RECON, MU, S, BW, MU == 3>(L, cur.sp[r], coef, y);
            reconstruct_add<T, MU, S>(acc[r], y);
        }
    }
    phase_end(act, acc);
}

// FP64 holds twice the registers per column: its workgroups stop at 12 column waves (768 threads)
template <class P> constexpr int lds_max_threads() { return P::id == PREC_F64 ? 768 : 1024; }
// Waves per SIMD the compiler must leave room for.  A 12-wave workgroup puts 3 waves on each
// SIMD, so two of them per CU need 6 (at most 80 VGPRs); left to itself the compiler gives the
// FP32 K2 and K2-dagger stencils 90-96 VGPRs (FP16 storage 82), and then only one workgroup
// fits a CU.  FP64 workgroups stop at 12 waves of 3 per SIMD with up to 168 VGPRs.
template <class P, int R, bool XCHG> constexpr int lds_min_waves()
{
    return P::id != PREC_F64 && R == 1 && !XCHG ? 6 : 1;
}

template <class P, class PR, int R, int DAG, int EPI, int RECON, bool PC, int LA, bool XCHG>
__global__ __launch_bounds__(lds_max_threads<P>()) __attribute__((amdgpu_waves_per_eu(lds_min_waves<P, R, XCHG>(), 8))) void k_hop_lds(const Args<P, PR> A)
{
    using T = typename P::real;
    using LC = typename LinkLds<P>::C;
    using U = typename P::unit;
    constexpr bool CL = clover_in_lds<P, PC, EPI>();
    extern __shared__ __align__(16) unsigned char smem[];
    LC* lk = (LC*)smem;                               // [8 half hops][9][64]
    U* sc = (U*)(smem + 8 * 9 * kTile * sizeof(LC));  // [clover units][64]
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    int lt, chunk;
    item_of(A.g, lb, A.nblk, A.nch, lt, chunk);
    {
        // A workgroup none of whose columns is selected (a reliable-update pass over a few columns)
        // stages nothing; the test is the same for every thread of the workgroup.
        bool sel = false;
        for (int c = chunk * A.gw * R; c < (chunk + 1) * A.gw * R && c < A.ncol; c++)
            sel |= col_selected(A.status, A.statmask, c);
        if (!sel) return;
    }
    const int tile = tile_at(A.g, lt);                // lt < ntiles: one tile per workgroup
    const int base = tile * kTile;
    // 1. stage the tile's links (8 half hops x 64 sites) and clover
    for (int t = threadIdx.x; t < 8 * kTile; t += blockDim.x) {
        const int site = t & (kTile - 1), H = t >> kTileLog;
        const int mu = H >> 1;
        const bool bw = H & 1;
        const int j = base + site;
        cx<T> u[9];
        if (j < A.g.Vh) {
            const Site st = site_of(A.g, A.parity, j);
            const int jn = nbr(A.g, st, mu, bw ? -1 : +1);
            Raw<P, link_cx<RECON>()> raw;
            load_units<P, link_cx<RECON>(), LA>(buf_rsrc(A.U[(bw ? 1 - A.parity : A.parity) * 4 + mu]), bw ? jn : j, raw);
            link_from_raw<P, RECON>(raw, u);
        } else {
#pragma unroll
            for (int k = 0; k < 9; k++) u[k] = {T(0), T(0)};
        }
#pragma unroll
        for (int k = 0; k < 9; k++) lk[(H * 9 + k) * kTile + site] = LC{u[k].re, u[k].im};
    }
    if constexpr (CL) {
        constexpr int NU = clover_units<P>();  // 36 (FP32) or 18 (FP16) 8-byte units, stored in pairs
        const U* C = (const U*)A.clov + (size_t)tile * NU * kTile;
        const __amdgpu_buffer_rsrc_t rs = buf_rsrc(C);
        for (int t = threadIdx.x; t < (NU / 2) * kTile; t += blockDim.x) {
            const int site = t & (kTile - 1), q = t >> kTileLog;
            const bq_u4v v = buf_load16<LA>(rs, (uint32_t)toff<U>(site, 2 * q, NU) * 8u);
            sc[(2 * q) * kTile + site] = __builtin_bit_cast(U, bq_u2v_b{v.x, v.y});
            sc[(2 * q + 1) * kTile + site] = __builtin_bit_cast(U, bq_u2v_b{v.z, v.w});
        }
    }
    __syncthreads();
    // 2. one column group per wave
    const int w = threadIdx.x >> kTileLog;
    const int lane = threadIdx.x & (kTile - 1);
    const int j = base + lane;
    const int c0 = __builtin_amdgcn_readfirstlane((chunk * A.gw + w) * R);
    bool act[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int c = c0 + r;
        act[r] = j < A.g.Vh && c < A.ncol && col_selected(A.status, A.statmask, c);
        any |= act[r];
    }
    cx<T> acc[R][12];
    if constexpr (XCHG) {
        // x and y half hops by lane exchange from the own input tile (all lanes take part in the
        // exchange; the wave's column is uniform), then the z and t half hops as loads
        static_assert(R == 1, "lane exchange holds one column per wave");
        if (c0 >= A.ncol || !col_selected(A.status, A.statmask, c0)) return;  // uniform over the wave
        const bool act0 = act[0];
        const Site s = site_of(A.g, A.parity, act0 ? j : base);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[0][k] = {T(0), T(0)};
        Raw<P, 12> own;
        float own_sc = 0.0f;
        if (act0) {
            HalfHop<P, 1, RECON> o;
            o.jn = j;
            hh_load_spinor(A, c0, 0, o);
            own = o.sp[0];
            if constexpr (P::id == PREC_F16) own_sc = o.sc[0];
        } else {
#pragma unroll
            for (int k = 0; k < 12 / P::cpu; k++) __builtin_memset(&own.u[k], 0, sizeof(own.u[k]));
        }
        constexpr int NB = 2;
        HalfHop<P, R, RECON> d[NB];
        hh_xchg<P, PR, DAG, RECON, 0>(A, s, act0, c0, base, own, own_sc, lk, lane, acc[0]);
        hh_xchg<P, PR, DAG, RECON, 1>(A, s, act0, c0, base, own, own_sc, lk, lane, acc[0]);
        hh_xchg<P, PR, DAG, RECON, 2>(A, s, act0, c0, base, own, own_sc, lk, lane, acc[0]);
        lds_issue<P, PR, R, RECON, NB, 4>(A, s, act, c0, d);
        hh_xchg<P, PR, DAG, RECON, 3>(A, s, act0, c0, base, own, own_sc, lk, lane, acc[0]);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 4>(A, s, act, c0, lk, lane, d, acc);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 5>(A, s, act, c0, lk, lane, d, acc);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 6>(A, s, act, c0, lk, lane, d, acc);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 7>(A, s, act, c0, lk, lane, d, acc);
    } else if (any) {
        const Site s = site_of(A.g, A.parity, j);
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
            for (int k = 0; k < 12; k++) acc[r][k] = {T(0), T(0)};
        constexpr int NB = lds_ring<P, R>();
        HalfHop<P, R, RECON> d[NB];
        lds_issue<P, PR, R, RECON, NB, 0>(A, s, act, c0, d);
        if constexpr (NB > 2) lds_issue<P, PR, R, RECON, NB, 1>(A, s, act, c0, d);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 0>(A, s, act, c0, lk, lane, d, acc);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 1>(A, s, act, c0, lk, lane, d, acc);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 2>(A, s, act, c0, lk, lane, d, acc);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 3>(A, s, act, c0, lk, lane, d, acc);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 4>(A, s, act, c0, lk, lane, d, acc);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 5>(A, s, act, c0, lk, lane, d, acc);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 6>(A, s, act, c0, lk, lane, d, acc);
        hh_step_lds<P, PR, R, DAG, RECON, NB, 7>(A, s, act, c0, lk, lane, d, acc);
    }
    epilogue<P, PR, R, EPI, PC, LA, CL>(A, j, act, any, c0, acc, CL ? sc : nullptr);
}

template <class P>
SpinorPtr<P> sp(const FieldArg& f)
{
    return SpinorPtr<P>{(typename P::unit*)f.d, f.s, f.cstride, f.sstride};
}

template <class P, class PR, int R, int DAG, int EPI, int RECON, bool PC>
hipError_t launch_t(const HopLaunch& L, hipStream_t st)
{
    using T = typename P::real;
    Args<P, PR> A;
    A.g = L.g;
    A.parity = L.parity;
    A.ncol = L.ncol;
    for (int k = 0; k < 8; k++) A.U[k] = (const typename P::unit*)L.U[k];
    A.in = sp<P>(L.in);
    A.out = sp<P>(L.out);
    A.v = sp<P>(L.v);
    A.rin = sp<PR>(L.r_in);
    A.rout = sp<PR>(L.r_out);
    A.clov = (const typename P::unit*)L.clov;
    A.alpha = L.alpha;
    A.partial = L.partial;
    A.nwaves = L.nwaves;
    A.pstride = L.pstride ? L.pstride : L.nwaves;
    A.status = L.status;
    A.statmask = L.statmask;
    A.ef = (T)L.ef;
    A.eb = (T)L.eb;
    A.ef_bc = (T)(L.ef * L.tbc);
    A.eb_bc = (T)(L.eb * L.tbc);
    A.f = (T)L.f;
    A.a = (T)L.a;
    A.percol = L.percol;
    for (int c = 0; c < kMaxCols; c++) {
        A.cclov[c] = (const typename P::unit*)L.cclov[c];
        A.cf[c] = (T)L.cf[c];
    }
    if (L.percol && L.ncol > kMaxCols) return hipErrorInvalidValue;
    const int G = (L.ncol + R - 1) / R;
    // With more than one column group per tile, the other groups' waves read the same links
    // (and, without per-column clover, the same clover) soon after: load those through the
    // caches.  With one group they are read once and streamed (non-temporal).
    const bool shared = G > 1;
    if (L.march > 0) {
        // t-marching: one tile position x column-group chunk x time segment per workgroup,
        // at most bs / 64 column groups per workgroup
        if (!L.g.blocked || L.g.L[3] % L.march != 0) return hipErrorInvalidValue;
        const int gmax = std::max(1, std::min(8, L.bs / kTile));
        A.nch = (G + gmax - 1) / gmax;
        A.gw = (G + A.nch - 1) / A.nch;
        A.tpb = 1;
        const int npos = L.g.ntiles / L.g.L[3];
        const int nseg = L.g.L[3] / L.march;
        A.nblk = npos * nseg;
        if (shared)
            hipLaunchKernelGGL((k_hop_march<P, PR, R, DAG, EPI, RECON, PC, 0>), dim3(A.nblk * A.nch), dim3(kTile * A.gw),
                               0, st, A, npos, L.march, nseg);
        else
            hipLaunchKernelGGL((k_hop_march<P, PR, R, DAG, EPI, RECON, PC, kBufNT>), dim3(A.nblk * A.nch),
                               dim3(kTile * A.gw), 0, st, A, npos, L.march, nseg);
        return hipGetLastError();
    }
    if (L.lds && G > 1) {
        // tile-shared: one tile per workgroup, up to 16 column-group waves, links (and clover) in LDS
        constexpr bool CL = clover_in_lds<P, PC, EPI>();
        constexpr int lds_bytes = tile_lds_bytes<P, CL>();
        if (CL && L.clov == nullptr) return hipErrorInvalidValue;  // the epilogue needs a clover array
        A.tpb = 1;
        A.gw = std::min(G, std::max(1, std::min(lds_max_threads<P>() / kTile, L.bs / kTile)));  // bs / 64 waves at most
        A.nch = (G + A.gw - 1) / A.gw;
        A.gw = (G + A.nch - 1) / A.nch;  // balance the chunks
        A.nblk = L.g.ntiles;
        // G > 1 here: the other column groups' waves of a tile read the same clover (FP64 keeps it
        // in global memory), so loads go through the caches
        auto launch = [&](auto kern, bool& attr) -> hipError_t {
            if (!attr) {  // once per instantiation: allow more than 64 KB of dynamic LDS
                const hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                         lds_bytes);
                if (e != hipSuccess) return e;
                attr = true;
            }
            hipLaunchKernelGGL(kern, dim3(A.nblk * A.nch), dim3(kTile * A.gw), lds_bytes, st, A);
            return hipGetLastError();
        };
        if constexpr (R == 1) {
            if (L.lds == 2) {
                static bool attr_x = false;
                return launch(k_hop_lds<P, PR, R, DAG, EPI, RECON, PC, 0, true>, attr_x);
            }
        }
        static bool attr = false;
        return launch(k_hop_lds<P, PR, R, DAG, EPI, RECON, PC, 0, false>, attr);
    }
    // L.bs = sites per workgroup (a multiple of 64); at most 512 threads per workgroup
    const int tpb = std::max(1, L.bs / kTile);
    A.tpb = tpb;
    A.gw = std::max(1, std::min(G, 512 / (tpb * kTile)));
    A.nch = (G + A.gw - 1) / A.gw;
    A.nblk = (L.g.ntiles + tpb - 1) / tpb;
    if (shared)
        hipLaunchKernelGGL((k_hop<P, PR, R, DAG, EPI, RECON, PC, 0>), dim3(A.nblk * A.nch), dim3(tpb * kTile * A.gw), 0, st, A);
    else
        hipLaunchKernelGGL((k_hop<P, PR, R, DAG, EPI, RECON, PC, kBufNT>), dim3(A.nblk * A.nch), dim3(tpb * kTile * A.gw), 0,
                           st, A);
    return hipGetLastError();
}

// per-column operators (kappa-batched serving) are instantiated for 12-real links only
template <class P, class PR, int R, int DAG, int EPI>
hipError_t by_recon(const HopLaunch& L, hipStream_t st)
{
    if (L.percol) {
        if (L.recon != 12) return hipErrorInvalidValue;
        return launch_t<P, PR, R, DAG, EPI, 12, true>(L, st);
    }
    if constexpr (P::id == PREC_F16) {
        if (L.recon != 12) return hipErrorInvalidValue;
        return launch_t<P, PR, R, DAG, EPI, 12, false>(L, st);
    } else {
        if (L.recon == 12) return launch_t<P, PR, R, DAG, EPI, 12, false>(L, st);
        if (L.recon == 18) return launch_t<P, PR, R, DAG, EPI, 18, false>(L, st);
        return hipErrorInvalidValue;
    }
}

template <class P, class PR, int R, int DAG>
hipError_t by_epi(const HopLaunch& L, hipStream_t st)
{
    switch (L.epi) {
    case EPI_HOP: return by_recon<P, PR, R, DAG, EPI_HOP>(L, st);
    case EPI_TINV: return by_recon<P, PR, R, DAG, EPI_TINV>(L, st);
    case EPI_TV: return by_recon<P, PR, R, DAG, EPI_TV>(L, st);
    case EPI_TVR: return by_recon<P, PR, R, DAG, EPI_TVR>(L, st);
    }
    return hipErrorInvalidValue;
}

template <class P, class PR, int R>
hipError_t by_dag(const HopLaunch& L, hipStream_t st)
{
    return L.dagger ? by_epi<P, PR, R, 1>(L, st) : by_epi<P, PR, R, 0>(L, st);
}

// columns per thread: FP64 keeps R <= 2 (R >= 3 exceeds 256 VGPRs and spills)
template <class P> constexpr int max_R() { return P::id == PREC_F64 ? 2 : 4; }

}  // namespace dslash
}  // namespace bq
