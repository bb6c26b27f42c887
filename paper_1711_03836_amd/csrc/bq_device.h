// Device-side building blocks of the HIP library: data layout, precision
// storage, complex arithmetic, lattice geometry.  Internal header, shared only
// by the library's own .hip sources.
//
// Layout (all fields live on one checkerboard = one parity, Vh = V/2 sites):
//   a site-tiled structure of arrays.  Sites are grouped in tiles of 64 (one
//   wavefront).  Inside a tile, 16-byte storage units (FP64) occupy 64
//   consecutive slots per unit: lane l reads slot l of a contiguous run,
//     offset(j, c) = ((j/64)*nunits + c)*64 + j%64.
//   Units of 8 bytes (FP32, FP16) are stored in pairs, two units of one site
//   side by side, so that a lane reads both with one 16-byte load:
//     offset(j, c) = ((j/64)*nunits + c - c%2)*64 + 2*(j%64) + c%2,
//   except that the last unit of an object with an odd unit count is stored
//   alone, as for 16-byte units.  With either rule a tile of an object covers
//   nunits*64 consecutive units.  The innermost index runs over the sites of a
//   wavefront, as the paper's SIMD layout puts a vector of sites innermost (5.1).
//
// Storage units per precision:
//   FP64: one complex per unit (double2, 16 B)
//   FP32: one complex per unit (float2,   8 B)
//   FP16: two complex per unit (4 x half, 8 B); spinors carry a per-site FP32
//         scale (max |re|,|im| over the site), links and clover are stored unscaled.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace bq {

constexpr int kTileLog = 6;
constexpr int kTile = 1 << kTileLog;

// offset, in units of U, of unit c (of nunits) of site j
template <class U>
__host__ __device__ __forceinline__ size_t toff(int j, int c, int nunits)
{
    const size_t tile = (size_t)(j >> kTileLog) * nunits * kTile;
    const int lane = j & (kTile - 1);
    if constexpr (sizeof(U) > 8) {
        return tile + (size_t)c * kTile + lane;
    } else {
        if ((nunits & 1) && c == nunits - 1) return tile + (size_t)c * kTile + lane;
        return tile + (size_t)(c & ~1) * kTile + 2 * lane + (c & 1);
    }
}
// Buffer-resource loads: the base address lives in scalar registers and each lane supplies a
// 32-bit byte offset, so a load needs one vector register for its address instead of two and
// no 64-bit address arithmetic.  Offsets from the resource base must stay below 4 GiB: with
// V/2 < 2^24 sites per parity a spinor column (at most 192 B per site) and a link array (144 B)
// do; clover arrays (576 B per site in FP64) are addressed from the base of the wave's tile.
typedef unsigned bq_u4v __attribute__((ext_vector_type(4)));
typedef unsigned bq_u2v_b __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)0xffffffff, 0x00020000);
}
constexpr int kBufNT = 2;  // non-temporal cache policy
template <int AUX>
__device__ __forceinline__ bq_u4v buf_load16(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX);
}
template <int AUX>
__device__ __forceinline__ bq_u2v_b buf_load8(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX);
}
__device__ __forceinline__ float buf_load4f(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

template <class U>
__host__ __device__ __forceinline__ U& at(U* p, int j, int c, int nunits)
{
    return p[toff<U>(j, c, nunits)];
}
template <class U>
__host__ __device__ __forceinline__ const U& at(const U* p, int j, int c, int nunits)
{
    return p[toff<U>(j, c, nunits)];
}

__host__ __device__ __forceinline__ int pad_sites(int n) { return (n + kTile - 1) & ~(kTile - 1); }

// ---------------------------------------------------------------------------
// complex arithmetic with explicit fused multiply-adds
// ---------------------------------------------------------------------------

template <typename T>
struct cx {
    T re, im;
};

template <typename T> __device__ __forceinline__ T fmadd(T a, T b, T c);
template <> __device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <> __device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T> __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cx<T> cscale(T s, cx<T> a) { return {s * a.re, s * a.im}; }
// i*a and -i*a
template <typename T> __device__ __forceinline__ cx<T> cmuli(cx<T> a) { return {-a.im, a.re}; }
template <typename T> __device__ __forceinline__ cx<T> cmulmi(cx<T> a) { return {a.im, -a.re}; }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {fmadd(a.re, b.re, -a.im * b.im), fmadd(a.re, b.im, a.im * b.re)};
}
// acc + a*b
template <typename T> __device__ __forceinline__ cx<T> cmac(cx<T> acc, cx<T> a, cx<T> b)
{
    acc.re = fmadd(a.re, b.re, acc.re);
    acc.re = fmadd(-a.im, b.im, acc.re);
    acc.im = fmadd(a.re, b.im, acc.im);
    acc.im = fmadd(a.im, b.re, acc.im);
    return acc;
}
// acc + conj(a)*b
template <typename T> __device__ __forceinline__ cx<T> cmacc(cx<T> acc, cx<T> a, cx<T> b)
{
    acc.re = fmadd(a.re, b.re, acc.re);
    acc.re = fmadd(a.im, b.im, acc.re);
    acc.im = fmadd(a.re, b.im, acc.im);
    acc.im = fmadd(-a.im, b.re, acc.im);
    return acc;
}
// acc + s*a (real s)
template <typename T> __device__ __forceinline__ cx<T> caxpy(T s, cx<T> a, cx<T> acc)
{
    return {fmadd(s, a.re, acc.re), fmadd(s, a.im, acc.im)};
}
template <typename T> __device__ __forceinline__ T cnorm2(cx<T> a) { return fmadd(a.re, a.re, a.im * a.im); }

// ---------------------------------------------------------------------------
// precisions
// ---------------------------------------------------------------------------

enum { PREC_F64 = 0, PREC_F32 = 1, PREC_F16 = 2 };

struct P64 {
    using real = double;
    using unit = double2;
    static constexpr int id = PREC_F64;
    static constexpr int cpu = 1;  // complex numbers per storage unit
};
struct P32 {
    using real = float;
    using unit = float2;
    static constexpr int id = PREC_F32;
    static constexpr int cpu = 1;
};
struct P16 {
    using real = float;
    using unit = uint2;  // four binary16 values
    static constexpr int id = PREC_F16;
    static constexpr int cpu = 2;
};

__device__ __forceinline__ float h2f(uint32_t bits16) { return __half2float(__ushort_as_half((unsigned short)bits16)); }
__device__ __forceinline__ uint32_t f2h(float f) { return (uint32_t)__half_as_ushort(__float2half_rn(f)); }

// Streaming accesses: links and clover are read once per launch and outputs written once;
// non-temporal loads/stores keep them from evicting the neighbour spinors that the stencil
// re-reads from L2.
typedef double bq_d2v __attribute__((ext_vector_type(2)));
typedef float bq_f2v __attribute__((ext_vector_type(2)));
typedef unsigned bq_u2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 ld_stream(const double2* p)
{
    const bq_d2v t = __builtin_nontemporal_load((const bq_d2v*)p);
    return make_double2(t.x, t.y);
}
__device__ __forceinline__ float2 ld_stream(const float2* p)
{
    const bq_f2v t = __builtin_nontemporal_load((const bq_f2v*)p);
    return make_float2(t.x, t.y);
}
__device__ __forceinline__ uint2 ld_stream(const uint2* p)
{
    const bq_u2v t = __builtin_nontemporal_load((const bq_u2v*)p);
    return make_uint2(t.x, t.y);
}
__device__ __forceinline__ void st_stream(double2* p, double2 v)
{
    bq_d2v t = {v.x, v.y};
    __builtin_nontemporal_store(t, (bq_d2v*)p);
}
__device__ __forceinline__ void st_stream(float2* p, float2 v)
{
    bq_f2v t = {v.x, v.y};
    __builtin_nontemporal_store(t, (bq_f2v*)p);
}
__device__ __forceinline__ void st_stream(uint2* p, uint2 v)
{
    bq_u2v t = {v.x, v.y};
    __builtin_nontemporal_store(t, (bq_u2v*)p);
}

template <class P, int N> struct CxIO;

template <int N> struct CxIO<P64, N> {
    static constexpr int nu = N;
    __device__ __forceinline__ static void load(const double2* __restrict__ b, int j, cx<double> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N; c++) { double2 t = at(b, j, c, N); v[c] = {t.x, t.y}; }
    }
    __device__ __forceinline__ static void load_cached(const double2* __restrict__ b, int j, cx<double> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N; c++) { double2 t = at(b, j, c, N); v[c] = {t.x, t.y}; }
    }
    __device__ __forceinline__ static void store(double2* __restrict__ b, int j, const cx<double> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N; c++) at(b, j, c, N) = make_double2(v[c].re, v[c].im);
    }
    __device__ __forceinline__ static void load_stream(const double2* __restrict__ b, int j, cx<double> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N; c++) { double2 t = ld_stream(&at(b, j, c, N)); v[c] = {t.x, t.y}; }
    }
    __device__ __forceinline__ static void store_stream(double2* __restrict__ b, int j, const cx<double> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N; c++) st_stream(&at(b, j, c, N), make_double2(v[c].re, v[c].im));
    }
};

template <int N> struct CxIO<P32, N> {
    static constexpr int nu = N;
    __device__ __forceinline__ static void load(const float2* __restrict__ b, int j, cx<float> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N; c++) { float2 t = at(b, j, c, N); v[c] = {t.x, t.y}; }
    }
    __device__ __forceinline__ static void load_cached(const float2* __restrict__ b, int j, cx<float> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N; c++) { float2 t = at(b, j, c, N); v[c] = {t.x, t.y}; }
    }
    __device__ __forceinline__ static void store(float2* __restrict__ b, int j, const cx<float> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N; c++) at(b, j, c, N) = make_float2(v[c].re, v[c].im);
    }
    __device__ __forceinline__ static void load_stream(const float2* __restrict__ b, int j, cx<float> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N; c++) { float2 t = ld_stream(&at(b, j, c, N)); v[c] = {t.x, t.y}; }
    }
    __device__ __forceinline__ static void store_stream(float2* __restrict__ b, int j, const cx<float> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N; c++) st_stream(&at(b, j, c, N), make_float2(v[c].re, v[c].im));
    }
};

template <int N> struct CxIO<P16, N> {
    static_assert(N % 2 == 0, "FP16 objects hold an even number of complex values");
    static constexpr int nu = N / 2;
    __device__ __forceinline__ static void unpack(uint2 t, cx<float>& a, cx<float>& b)
    {
        a = {h2f(t.x & 0xffffu), h2f(t.x >> 16)};
        b = {h2f(t.y & 0xffffu), h2f(t.y >> 16)};
    }
    __device__ __forceinline__ static uint2 pack(cx<float> a, cx<float> b)
    {
        return make_uint2(f2h(a.re) | (f2h(a.im) << 16), f2h(b.re) | (f2h(b.im) << 16));
    }
    __device__ __forceinline__ static void load(const uint2* __restrict__ b, int j, cx<float> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N / 2; c++) unpack(at(b, j, c, N / 2), v[2 * c], v[2 * c + 1]);
    }
    __device__ __forceinline__ static void load_cached(const uint2* __restrict__ b, int j, cx<float> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N / 2; c++) unpack(at(b, j, c, N / 2), v[2 * c], v[2 * c + 1]);
    }
    __device__ __forceinline__ static void store(uint2* __restrict__ b, int j, const cx<float> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N / 2; c++) at(b, j, c, N / 2) = pack(v[2 * c], v[2 * c + 1]);
    }
    __device__ __forceinline__ static void load_stream(const uint2* __restrict__ b, int j, cx<float> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N / 2; c++) unpack(ld_stream(&at(b, j, c, N / 2)), v[2 * c], v[2 * c + 1]);
    }
    __device__ __forceinline__ static void store_stream(uint2* __restrict__ b, int j, const cx<float> (&v)[N])
    {
#pragma unroll
        for (int c = 0; c < N / 2; c++) st_stream(&at(b, j, c, N / 2), pack(v[2 * c], v[2 * c + 1]));
    }
};

// Units of storage for one site of each object.
template <class P> __host__ __device__ constexpr int spinor_units() { return 12 / P::cpu; }
template <class P> __host__ __device__ constexpr int clover_units() { return 36 / P::cpu; }  // two packed 6x6 blocks
template <class P, int RECON> __host__ __device__ constexpr int link_units() { return (RECON == 18 ? 9 : 6) / P::cpu; }

// A spinor field on one parity: data (+ per-site scale for FP16), column stride in units.
template <class P>
struct SpinorPtr {
    typename P::unit* d;
    float* s;        // FP16 only: per-site scale, column stride = sstride
    size_t cstride;  // units between columns
    size_t sstride;  // floats between columns of the scale array
};

template <class P>
__device__ __forceinline__ void load_spinor(const SpinorPtr<P>& f, int col, int j, cx<typename P::real> (&v)[12])
{
    CxIO<P, 12>::load_cached(f.d + col * f.cstride, j, v);
    if constexpr (P::id == PREC_F16) {
        float s = f.s[col * f.sstride + j];
#pragma unroll
        for (int k = 0; k < 12; k++) v[k] = cscale(s, v[k]);
    }
}

template <class P, bool STREAM = false>
__device__ __forceinline__ void store_spinor(const SpinorPtr<P>& f, int col, int j, cx<typename P::real> (&v)[12])
{
    if constexpr (P::id == PREC_F16) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; k++) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        float inv = m > 0.f ? 1.0f / m : 0.f;
        cx<float> w[12];
#pragma unroll
        for (int k = 0; k < 12; k++) w[k] = cscale(inv, v[k]);
        if constexpr (STREAM) {
            CxIO<P, 12>::store_stream(f.d + col * f.cstride, j, w);
        } else {
            CxIO<P, 12>::store(f.d + col * f.cstride, j, w);
        }
        f.s[col * f.sstride + j] = m;
    } else if constexpr (STREAM) {
        CxIO<P, 12>::store_stream(f.d + col * f.cstride, j, v);
    } else {
        CxIO<P, 12>::store(f.d + col * f.cstride, j, v);
    }
}

// ---------------------------------------------------------------------------
// geometry on one checkerboard
// ---------------------------------------------------------------------------

struct Geom {
    int L[4];     // extents x, y, z, t (all even)
    int Lxh;      // L[0] / 2
    int Vh;       // sites per parity
    int sy, sz, st;        // checkerboard-index strides of a y, z, t step
    float inv_Lxh, inv_Ly, inv_Lz;
    // Traversal order of the 64-site tiles by stencil kernels: when an (x,y) plane of a
    // checkerboard holds a whole number `nu` of tiles, tiles are visited plane by plane in
    // blocks of zb x tb (z,t) planes, so that the +-t and +-z neighbours of the planes in
    // flight are a few planes away instead of a whole time slice.  ntiles = tiles per parity.
    int ntiles, blocked, nu, zb, tb, nzb;
    float inv_nu, inv_zb, inv_tb, inv_nzb;
    // Order of a launch's (tile block, column-group chunk) work items: 0 the chunks of a tile block
    // one after another; 1 each XCD's share of tile blocks walked once per chunk (item_of)
    int cmajor;
};

// exact quotient/remainder of n < 2^24 by d using a float reciprocal and one correction
__device__ __forceinline__ int fdiv(int n, int d, float inv)
{
    int q = (int)((float)n * inv);
    int r = n - q * d;
    q += (r >= d) - (r < 0);
    return q;
}

// physical tile visited at logical position `lt` (see Geom)
__device__ __forceinline__ int tile_at(const Geom& g, int lt)
{
    if (!g.blocked) return lt;
    const int r1 = fdiv(lt, g.nu, g.inv_nu);
    const int u = lt - r1 * g.nu;
    const int r2 = fdiv(r1, g.zb, g.inv_zb);
    const int zl = r1 - r2 * g.zb;
    const int r3 = fdiv(r2, g.tb, g.inv_tb);
    const int tl = r2 - r3 * g.tb;
    const int ti = fdiv(r3, g.nzb, g.inv_nzb);
    const int zi = r3 - ti * g.nzb;
    return u + g.nu * ((zi * g.zb + zl) + g.L[2] * (ti * g.tb + tl));
}

struct Site {
    int j;        // checkerboard index
    int xh, y, z, t;
    int x;        // full x coordinate
};

__device__ __forceinline__ Site site_of(const Geom& g, int parity, int j)
{
    Site s;
    s.j = j;
    int r1 = fdiv(j, g.Lxh, g.inv_Lxh);
    s.xh = j - r1 * g.Lxh;
    int r2 = fdiv(r1, g.L[1], g.inv_Ly);
    s.y = r1 - r2 * g.L[1];
    s.t = fdiv(r2, g.L[2], g.inv_Lz);
    s.z = r2 - s.t * g.L[2];
    s.x = 2 * s.xh + ((parity + s.y + s.z + s.t) & 1);
    return s;
}

// checkerboard index of the neighbour x + dir*mu_hat (dir = +1/-1), periodic
__device__ __forceinline__ int nbr(const Geom& g, const Site& s, int mu, int dir)
{
    switch (mu) {
    case 0: {
        int x = s.x + dir;
        x = x < 0 ? g.L[0] - 1 : (x == g.L[0] ? 0 : x);
        return s.j - s.xh + (x >> 1);
    }
    case 1:
        if (dir > 0) return s.y == g.L[1] - 1 ? s.j - (g.L[1] - 1) * g.sy : s.j + g.sy;
        return s.y == 0 ? s.j + (g.L[1] - 1) * g.sy : s.j - g.sy;
    case 2:
        if (dir > 0) return s.z == g.L[2] - 1 ? s.j - (g.L[2] - 1) * g.sz : s.j + g.sz;
        return s.z == 0 ? s.j + (g.L[2] - 1) * g.sz : s.j - g.sz;
    default:
        if (dir > 0) return s.t == g.L[3] - 1 ? s.j - (g.L[3] - 1) * g.st : s.j + g.st;
        return s.t == 0 ? s.j + (g.L[3] - 1) * g.st : s.j - g.st;
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Give each XCD one contiguous range of logical blocks so that neighbouring
// sites, and the column groups of one site block, share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Work item (tile block, column-group chunk) of logical block lb of a launch of nblk tile blocks x
// nch chunks, lb from xcd_remap so that each XCD holds a contiguous range of nblk * nch / 8
// blocks.  Chunk-major (g.cmajor, nblk a multiple of 8): an XCD walks its nblk / 8 tile blocks for
// chunk 0, then for chunk 1, ..., so fewer columns are in flight on one XCD at a time; otherwise
// the chunks of a tile block are adjacent and share its links and clover through the caches.
__device__ __forceinline__ void item_of(const Geom& g, int lb, int nblk, int nch, int& tblk, int& chunk)
{
    if (g.cmajor && nch > 1 && (nblk & 7) == 0) {
        const int per = nblk >> 3;
        const int x = lb / (per * nch);
        const int local = lb - x * per * nch;
        chunk = local / per;
        tblk = x * per + (local - chunk * per);
    } else {
        tblk = lb / nch;
        chunk = lb - tblk * nch;
    }
}

// CG column states (the solver's per-column state machine)
enum { COL_ACTIVE = 0, COL_JUST_STOPPED = 1, COL_STOPPED = 2, COL_DONE = 3, COL_FAILED = 4 };

__device__ __forceinline__ bool col_selected(const int* status, int statmask, int c)
{
    return status == nullptr || ((statmask >> status[c]) & 1);
}

// wavefront sum (deterministic butterfly) of a double, result valid in every lane
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace bq
