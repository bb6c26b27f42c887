// Layout conversion, BLAS-1 updates, deterministic FP64 reductions and the
// per-column CG finalisation kernels.
//
// Reductions: every kernel that reduces writes one FP64 partial per wavefront
// of 64 consecutive sites (a butterfly inside the wave), and a finalisation
// kernel sums a column's partials in a fixed order in one workgroup.  The
// partials depend only on which 64 sites a wave covers, so a column's result
// is the same bit for bit whatever the block size, column tile or batch it
// was computed in.
#include "bq_kernels.h"

namespace bq {
namespace {

template <class P>
__host__ __device__ SpinorPtr<P> sp(const FieldArg& f)
{
    return SpinorPtr<P>{(typename P::unit*)f.d, f.s, f.cstride, f.sstride};
}

__device__ __forceinline__ int lex_of(const Geom& g, int parity, int j)
{
    const Site s = site_of(g, parity, j);
    return s.x + g.L[0] * (s.y + g.L[1] * (s.z + g.L[2] * s.t));
}

// --------------------------------------------------------------------------
// layout conversion between the canonical lexicographic complex128 arrays and
// the site-tiled checkerboard storage
// --------------------------------------------------------------------------

template <class P, int NC>
__global__ void k_links_import(const double2* __restrict__ canon, const Geom g, int parity, typename P::unit* d0,
                               typename P::unit* d1, typename P::unit* d2, typename P::unit* d3)
{
    using T = typename P::real;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.Vh) return;
    const size_t V = 2 * (size_t)g.Vh;
    const int lex = lex_of(g, parity, j);
    typename P::unit* dst[4] = {d0, d1, d2, d3};
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        cx<T> u[NC];
#pragma unroll
        for (int k = 0; k < NC; k++) {
            const double2 t = canon[((size_t)mu * V + lex) * 9 + k];
            u[k] = {(T)t.x, (T)t.y};
        }
        CxIO<P, NC>::store(dst[mu], j, u);
    }
}

template <class P>
__global__ void k_spinor_import(const double2* __restrict__ canon, const Geom g, int parity, SpinorPtr<P> f)
{
    using T = typename P::real;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= g.Vh) return;
    const size_t V = 2 * (size_t)g.Vh;
    const int lex = lex_of(g, parity, j);
    cx<T> v[12];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const double2 t = canon[((size_t)c * V + lex) * 12 + k];
        v[k] = {(T)t.x, (T)t.y};
    }
    store_spinor(f, c, j, v);
}

template <class P>
__global__ void k_spinor_export(SpinorPtr<P> f, const Geom g, int parity, double2* __restrict__ canon)
{
    using T = typename P::real;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= g.Vh) return;
    const size_t V = 2 * (size_t)g.Vh;
    const int lex = lex_of(g, parity, j);
    cx<T> v[12];
    load_spinor(f, c, j, v);
#pragma unroll
    for (int k = 0; k < 12; k++) canon[((size_t)c * V + lex) * 12 + k] = make_double2((double)v[k].re, (double)v[k].im);
}

// --------------------------------------------------------------------------
// BLAS-1 over n sites (a parity half, or both halves of a full field)
// --------------------------------------------------------------------------

template <class PS, class PD>
__global__ void k_convert(SpinorPtr<PS> src, SpinorPtr<PD> dst, int n, const int* status, int statmask)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= n || !col_selected(status, statmask, c)) return;
    cx<typename PS::real> a[12];
    cx<typename PD::real> b[12];
    load_spinor(src, c, j, a);
#pragma unroll
    for (int k = 0; k < 12; k++) b[k] = {(typename PD::real)a[k].re, (typename PD::real)a[k].im};
    store_spinor(dst, c, j, b);
}

template <class P>
__global__ void k_zero(SpinorPtr<P> x, int n, const int* status, int statmask)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= n || !col_selected(status, statmask, c)) return;
    cx<typename P::real> z[12];
#pragma unroll
    for (int k = 0; k < 12; k++) z[k] = {0, 0};
    store_spinor(x, c, j, z);
}

template <class P>
__global__ void k_norm2(SpinorPtr<P> x, int n, double* partial, int nwaves)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    double s = 0.0;
    if (j < n) {
        cx<typename P::real> v[12];
        load_spinor(x, c, j, v);
#pragma unroll
        for (int k = 0; k < 12; k++) s += (double)v[k].re * v[k].re + (double)v[k].im * v[k].im;
    }
    s = wave_sum(s);
    const int w = j >> kTileLog;
    if ((threadIdx.x & 63) == 0 && w < nwaves) partial[(size_t)c * nwaves + w] = s;
}

// <x, y> = sum conj(x) y (G5: <x, gamma_5 y>, gamma_5 = diag(1,1,-1,-1) in spin), FP64 fields;
// partials [col][re/im][wave]
template <bool G5>
__global__ void k_dot(SpinorPtr<P64> x, SpinorPtr<P64> y, int n, double* partial, int nwaves)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    double re = 0.0, im = 0.0;
    if (j < n) {
        cx<double> a[12], b[12];
        load_spinor(x, c, j, a);
        load_spinor(y, c, j, b);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const double sg = (G5 && k >= 6) ? -1.0 : 1.0;  // components 6..11 are spins 2 and 3
            re += sg * (a[k].re * b[k].re + a[k].im * b[k].im);
            im += sg * (a[k].re * b[k].im - a[k].im * b[k].re);
        }
    }
    re = wave_sum(re);
    im = wave_sum(im);
    const int w = j >> kTileLog;
    if ((threadIdx.x & 63) == 0 && w < nwaves) {
        partial[((size_t)c * 2 + 0) * nwaves + w] = re;
        partial[((size_t)c * 2 + 1) * nwaves + w] = im;
    }
}

// x += alpha p (active and just-stopped columns); p = r + beta p (active columns)
template <class PX, class PP, class PR>
__global__ void k_cg_update(SpinorPtr<PX> x, SpinorPtr<PP> p, SpinorPtr<PR> r, int n, const double* alpha,
                            const double* beta, const int* status)
{
    using TX = typename PX::real;
    using TP = typename PP::real;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    const int st = status ? status[c] : COL_ACTIVE;
    if (j >= n || (st != COL_ACTIVE && st != COL_JUST_STOPPED)) return;
    cx<TP> pv[12];
    load_spinor(p, c, j, pv);
    {
        const TX a = (TX)alpha[c];
        cx<TX> xv[12];
        load_spinor(x, c, j, xv);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            xv[k].re = fmadd(a, (TX)pv[k].re, xv[k].re);
            xv[k].im = fmadd(a, (TX)pv[k].im, xv[k].im);
        }
        store_spinor(x, c, j, xv);
    }
    if (st == COL_ACTIVE) {
        const TP b = (TP)beta[c];
        cx<typename PR::real> rv[12];
        load_spinor(r, c, j, rv);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            pv[k].re = fmadd(b, pv[k].re, (TP)rv[k].re);
            pv[k].im = fmadd(b, pv[k].im, (TP)rv[k].im);
        }
        store_spinor(p, c, j, pv);
    }
}

// y64 += x ; x = 0
template <class PX>
__global__ void k_accum(SpinorPtr<PX> x, SpinorPtr<P64> y, int n, const int* status, int statmask)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= n || !col_selected(status, statmask, c)) return;
    cx<typename PX::real> xv[12];
    cx<double> yv[12];
    load_spinor(x, c, j, xv);
    load_spinor(y, c, j, yv);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        yv[k].re += (double)xv[k].re;
        yv[k].im += (double)xv[k].im;
        xv[k] = {0, 0};
    }
    store_spinor(y, c, j, yv);
    store_spinor(x, c, j, xv);
}

// rs = lowp(r64) ; p = rs + beta p   (columns with flag set)
template <class PRS, class PP>
__global__ void k_restart(SpinorPtr<P64> r64, SpinorPtr<PRS> rs, SpinorPtr<PP> p, int n, const double* beta,
                          const int* flag, int write_rs)
{
    using TP = typename PP::real;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= n || !flag[c]) return;
    cx<double> rv[12];
    load_spinor(r64, c, j, rv);
    if (write_rs) {
        cx<typename PRS::real> t[12];
#pragma unroll
        for (int k = 0; k < 12; k++) t[k] = {(typename PRS::real)rv[k].re, (typename PRS::real)rv[k].im};
        store_spinor(rs, c, j, t);
#pragma unroll
        for (int k = 0; k < 12; k++) rv[k] = {(double)t[k].re, (double)t[k].im};
    }
    const TP b = (TP)beta[c];
    cx<TP> pv[12];
    load_spinor(p, c, j, pv);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        pv[k].re = fmadd(b, pv[k].re, (TP)rv[k].re);
        pv[k].im = fmadd(b, pv[k].im, (TP)rv[k].im);
    }
    store_spinor(p, c, j, pv);
}

// Distance of every link from SU(3): max over links of max(max_ab |(U U^dag - 1)_ab|, |det U - 1|),
// one partial maximum per workgroup (the host takes the maximum of the partials).
__global__ void k_link_su3_dev(const double2* __restrict__ canon, size_t nlinks, double* partial)
{
    __shared__ double w[4];
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double dev = 0.0;
    if (k < nlinks) {
        cx<double> u[9];
#pragma unroll
        for (int e = 0; e < 9; e++) {
            const double2 t = canon[k * 9 + e];
            u[e] = {t.x, t.y};
        }
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                cx<double> s = {0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 3; c++) s = cmacc(s, u[b * 3 + c], u[a * 3 + c]);  // sum_c U_ac conj(U_bc)
                if (a == b) s.re -= 1.0;
                dev = fmax(dev, fmax(fabs(s.re), fabs(s.im)));
            }
        const cx<double> m0 = csub(cmul(u[4], u[8]), cmul(u[5], u[7]));
        const cx<double> m1 = csub(cmul(u[5], u[6]), cmul(u[3], u[8]));
        const cx<double> m2 = csub(cmul(u[3], u[7]), cmul(u[4], u[6]));
        cx<double> det = cmul(u[0], m0);
        det = cmac(det, u[1], m1);
        det = cmac(det, u[2], m2);
        det.re -= 1.0;
        dev = fmax(dev, sqrt(cnorm2(det)));
        if (!isfinite(dev)) dev = INFINITY;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off, 64));
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = dev;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(w[0], w[1]), fmax(w[2], w[3]));
}

// complex Z2 noise from SplitMix64 used as a counter-based generator:
// output k of stream `seed` is mix(seed + (k+1) * 0x9E3779B97F4A7C15);
// component (noise n, lexicographic site i, spin s, colour c) uses k = (n*V + i)*12 + 3s + c,
// bit 63 -> sign of the real part, bit 62 -> sign of the imaginary part, |eta| = 1.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_z2_noise(uint64_t seed, long n0, const Geom g, int parity, SpinorPtr<P64> f)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= g.Vh) return;
    const uint64_t V = 2 * (uint64_t)g.Vh;
    const uint64_t lex = (uint64_t)lex_of(g, parity, j);
    const double h = 0.70710678118654752440;
    cx<double> v[12];
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const uint64_t ctr = ((uint64_t)(n0 + c) * V + lex) * 12 + k;
        const uint64_t z = mix64(seed + (ctr + 1) * 0x9E3779B97F4A7C15ull);
        v[k] = {(z >> 63) & 1 ? -h : h, (z >> 62) & 1 ? -h : h};
    }
    store_spinor(f, c, j, v);
}

// --------------------------------------------------------------------------
// per-column finalisation (one workgroup of 256 threads per column)
// --------------------------------------------------------------------------

__device__ double block_sum(const double* __restrict__ part, int n)
{
    // eight independent partial sums per thread keep eight loads in flight; which element goes
    // to which sum depends on n only, so the result is deterministic for a given lattice
    __shared__ double w[4];
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 7 * 256 < n; i += 8 * 256) {
#pragma unroll
        for (int k = 0; k < 8; k++) a[k] += part[i + k * 256];
    }
    for (; i < n; i += 256) a[0] += part[i];
    double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    s = wave_sum(s);
    __syncthreads();  // a previous call's readers of w are done before it is overwritten
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
    __syncthreads();
    return (w[0] + w[1]) + (w[2] + w[3]);
}

__global__ void k_fin_sum(const double* partial, int nwaves, double* out)
{
    const int c = blockIdx.x;
    const double s = block_sum(partial + (size_t)c * nwaves, nwaves);
    if (threadIdx.x == 0) out[c] = s;
}

__global__ void k_fin_alpha(const CgScalars s, const double* partial, int nwaves)
{
    const int c = blockIdx.x;
    const int st = s.status[c];
    if (st != COL_ACTIVE && st != COL_JUST_STOPPED) return;  // uniform per block
    const double pAp = st == COL_ACTIVE ? block_sum(partial + (size_t)c * nwaves, nwaves) : 0.0;
    if (threadIdx.x != 0) return;
    if (st == COL_JUST_STOPPED) {
        s.status[c] = COL_STOPPED;
        return;
    }
    s.pAp[c] = pAp;
    if (!(pAp > 0.0) || !isfinite(pAp)) {
        s.alpha[c] = 0.0;
        s.status[c] = COL_FAILED;
    } else {
        s.alpha[c] = s.rho[c] / pAp;
    }
}

__global__ void k_fin_beta(const CgScalars s, const double* partial, int nwaves)
{
    const int c = blockIdx.x;
    if (s.status[c] != COL_ACTIVE) return;
    const double rho = block_sum(partial + (size_t)c * nwaves, nwaves);
    if (threadIdx.x != 0) return;
    s.iters[c] += 1;
    if (!isfinite(rho)) {
        s.status[c] = COL_FAILED;
    } else if (rho <= s.stop2[c] || (s.delta2 > 0.0 && rho <= s.delta2 * s.rmax2[c])) {
        s.status[c] = COL_JUST_STOPPED;  // x still takes this iteration's alpha*p
    } else {
        s.beta[c] = rho / s.rho[c];
        s.rho[c] = rho;
        if (rho > s.rmax2[c]) s.rmax2[c] = rho;
    }
}

__global__ void k_fin_reliable(const CgScalars s, const double* partial, int nwaves)
{
    const int c = blockIdx.x;
    const int st = s.status[c];
    const bool sel = st == COL_JUST_STOPPED || st == COL_STOPPED;
    const double r2 = sel ? block_sum(partial + (size_t)c * nwaves, nwaves) : 0.0;
    if (threadIdx.x != 0) return;
    s.restart[c] = 0;
    if (!sel) return;
    s.nrel[c] += 1;
    if (!isfinite(r2)) {
        s.status[c] = COL_FAILED;
    } else if (r2 <= s.stop2[c]) {
        s.rho[c] = r2;
        s.status[c] = COL_DONE;
    } else {
        s.beta[c] = r2 / s.rho[c];
        s.rho[c] = r2;
        s.rmax2[c] = r2;
        s.status[c] = COL_ACTIVE;
        s.restart[c] = 1;
    }
}

// ---------------------------------------------------------------------------
// dispatch helpers
// ---------------------------------------------------------------------------

constexpr int kBS = 256;

inline dim3 grid2(int n, int ncol) { return dim3((n + kBS - 1) / kBS, ncol); }

inline bool prec_ok(int prec) { return prec == PREC_F64 || prec == PREC_F32 || prec == PREC_F16; }

}  // namespace

hipError_t launch_links_import(const double2* canon, const Geom& g, int parity, int prec, int recon, void* const dst[4],
                               hipStream_t st)
{
    const dim3 grid((g.Vh + kBS - 1) / kBS);
#define LI(P, NC)                                                                                                 \
    hipLaunchKernelGGL((k_links_import<P, NC>), grid, dim3(kBS), 0, st, canon, g, parity, (P::unit*)dst[0],       \
                       (P::unit*)dst[1], (P::unit*)dst[2], (P::unit*)dst[3])
    if (prec == PREC_F64 && recon == 18) LI(P64, 9);
    else if (prec == PREC_F64 && recon == 12) LI(P64, 6);
    else if (prec == PREC_F32 && recon == 18) LI(P32, 9);
    else if (prec == PREC_F32 && recon == 12) LI(P32, 6);
    else if (prec == PREC_F16 && recon == 12) LI(P16, 6);
    else return hipErrorInvalidValue;
#undef LI
    return hipGetLastError();
}

hipError_t launch_spinor_import(const double2* canon, int ncol, const Geom& g, int parity, int prec, FieldArg dst,
                                hipStream_t st)
{
    const dim3 grid = grid2(g.Vh, ncol);
    switch (prec) {
    case PREC_F64: hipLaunchKernelGGL(k_spinor_import<P64>, grid, dim3(kBS), 0, st, canon, g, parity, sp<P64>(dst)); break;
    case PREC_F32: hipLaunchKernelGGL(k_spinor_import<P32>, grid, dim3(kBS), 0, st, canon, g, parity, sp<P32>(dst)); break;
    case PREC_F16: hipLaunchKernelGGL(k_spinor_import<P16>, grid, dim3(kBS), 0, st, canon, g, parity, sp<P16>(dst)); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_spinor_export(FieldArg src, int ncol, const Geom& g, int parity, int prec, double2* canon,
                                hipStream_t st)
{
    const dim3 grid = grid2(g.Vh, ncol);
    switch (prec) {
    case PREC_F64: hipLaunchKernelGGL(k_spinor_export<P64>, grid, dim3(kBS), 0, st, sp<P64>(src), g, parity, canon); break;
    case PREC_F32: hipLaunchKernelGGL(k_spinor_export<P32>, grid, dim3(kBS), 0, st, sp<P32>(src), g, parity, canon); break;
    case PREC_F16: hipLaunchKernelGGL(k_spinor_export<P16>, grid, dim3(kBS), 0, st, sp<P16>(src), g, parity, canon); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_convert(int sprec, FieldArg src, int dprec, FieldArg dst, int n, int ncol, const int* status,
                          int statmask, hipStream_t st)
{
    const dim3 grid = grid2(n, ncol);
#define CV(PS, PD) hipLaunchKernelGGL((k_convert<PS, PD>), grid, dim3(kBS), 0, st, sp<PS>(src), sp<PD>(dst), n, status, statmask)
    if (!prec_ok(sprec) || !prec_ok(dprec)) return hipErrorInvalidValue;
    const int key = sprec * 3 + dprec;
    switch (key) {
    case PREC_F64 * 3 + PREC_F64: CV(P64, P64); break;
    case PREC_F64 * 3 + PREC_F32: CV(P64, P32); break;
    case PREC_F64 * 3 + PREC_F16: CV(P64, P16); break;
    case PREC_F32 * 3 + PREC_F64: CV(P32, P64); break;
    case PREC_F32 * 3 + PREC_F32: CV(P32, P32); break;
    case PREC_F32 * 3 + PREC_F16: CV(P32, P16); break;
    case PREC_F16 * 3 + PREC_F64: CV(P16, P64); break;
    case PREC_F16 * 3 + PREC_F32: CV(P16, P32); break;
    case PREC_F16 * 3 + PREC_F16: CV(P16, P16); break;
    default: return hipErrorInvalidValue;
    }
#undef CV
    return hipGetLastError();
}

hipError_t launch_norm2(int prec, FieldArg x, int n, int ncol, double* partial, int nwaves, hipStream_t st)
{
    const dim3 grid = grid2(n, ncol);
    switch (prec) {
    case PREC_F64: hipLaunchKernelGGL(k_norm2<P64>, grid, dim3(kBS), 0, st, sp<P64>(x), n, partial, nwaves); break;
    case PREC_F32: hipLaunchKernelGGL(k_norm2<P32>, grid, dim3(kBS), 0, st, sp<P32>(x), n, partial, nwaves); break;
    case PREC_F16: hipLaunchKernelGGL(k_norm2<P16>, grid, dim3(kBS), 0, st, sp<P16>(x), n, partial, nwaves); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Plain copy of n 16-byte words, one word per thread, non-temporal on both sides: the reference
// rate against which the stencils' HBM bandwidth is read.
__global__ __launch_bounds__(256) void k_copy16(const bq_u4v* __restrict__ src, bq_u4v* __restrict__ dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_copy16(const void* src, void* dst, size_t n, hipStream_t st)
{
    const size_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, st, (const bq_u4v*)src, (bq_u4v*)dst, n);
    return hipGetLastError();
}

hipError_t launch_zero(int prec, FieldArg x, int n, int ncol, const int* status, int statmask, hipStream_t st)
{
    const dim3 grid = grid2(n, ncol);
    switch (prec) {
    case PREC_F64: hipLaunchKernelGGL(k_zero<P64>, grid, dim3(kBS), 0, st, sp<P64>(x), n, status, statmask); break;
    case PREC_F32: hipLaunchKernelGGL(k_zero<P32>, grid, dim3(kBS), 0, st, sp<P32>(x), n, status, statmask); break;
    case PREC_F16: hipLaunchKernelGGL(k_zero<P16>, grid, dim3(kBS), 0, st, sp<P16>(x), n, status, statmask); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dot(int prec, FieldArg x, FieldArg y, int n, int ncol, double* partial, int nwaves, hipStream_t st,
                      int gamma5)
{
    if (prec != PREC_F64) return hipErrorInvalidValue;
    if (gamma5)
        hipLaunchKernelGGL(k_dot<true>, grid2(n, ncol), dim3(kBS), 0, st, sp<P64>(x), sp<P64>(y), n, partial, nwaves);
    else
        hipLaunchKernelGGL(k_dot<false>, grid2(n, ncol), dim3(kBS), 0, st, sp<P64>(x), sp<P64>(y), n, partial, nwaves);
    return hipGetLastError();
}

hipError_t launch_cg_update(int xprec, FieldArg x, int pprec, FieldArg p, int rprec, FieldArg r, int n, int ncol,
                            const double* alpha, const double* beta, const int* status, hipStream_t st)
{
    const dim3 grid = grid2(n, ncol);
#define UP(PX, PP, PR) \
    hipLaunchKernelGGL((k_cg_update<PX, PP, PR>), grid, dim3(kBS), 0, st, sp<PX>(x), sp<PP>(p), sp<PR>(r), n, alpha, beta, status)
    if (xprec == PREC_F64 && pprec == PREC_F64 && rprec == PREC_F64) UP(P64, P64, P64);
    else if (xprec == PREC_F32 && pprec == PREC_F32 && rprec == PREC_F32) UP(P32, P32, P32);
    else if (xprec == PREC_F32 && pprec == PREC_F16 && rprec == PREC_F32) UP(P32, P16, P32);
    else return hipErrorInvalidValue;
#undef UP
    return hipGetLastError();
}

hipError_t launch_accum(int xprec, FieldArg x, FieldArg y64, int n, int ncol, const int* status, int statmask,
                        hipStream_t st)
{
    const dim3 grid = grid2(n, ncol);
    if (xprec == PREC_F32)
        hipLaunchKernelGGL(k_accum<P32>, grid, dim3(kBS), 0, st, sp<P32>(x), sp<P64>(y64), n, status, statmask);
    else if (xprec == PREC_F64)
        hipLaunchKernelGGL(k_accum<P64>, grid, dim3(kBS), 0, st, sp<P64>(x), sp<P64>(y64), n, status, statmask);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_restart(FieldArg r64, int rsprec, FieldArg rs, int pprec, FieldArg p, int n, int ncol,
                          const double* beta, const int* flag, hipStream_t st)
{
    const dim3 grid = grid2(n, ncol);
    const int write_rs = rs.d != r64.d;
#define RS(PRS, PP) \
    hipLaunchKernelGGL((k_restart<PRS, PP>), grid, dim3(kBS), 0, st, sp<P64>(r64), sp<PRS>(rs), sp<PP>(p), n, beta, flag, write_rs)
    if (rsprec == PREC_F64 && pprec == PREC_F64) RS(P64, P64);
    else if (rsprec == PREC_F32 && pprec == PREC_F32) RS(P32, P32);
    else if (rsprec == PREC_F32 && pprec == PREC_F16) RS(P32, P16);
    else return hipErrorInvalidValue;
#undef RS
    return hipGetLastError();
}

int link_su3_parts(size_t nlinks) { return (int)((nlinks + kBS - 1) / kBS); }

hipError_t launch_link_su3_dev(const double2* canon, size_t nlinks, double* partial, hipStream_t st)
{
    if (nlinks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_link_su3_dev, dim3(link_su3_parts(nlinks)), dim3(kBS), 0, st, canon, nlinks, partial);
    return hipGetLastError();
}

hipError_t launch_z2_noise(uint64_t seed, long n0, const Geom& g, int parity, FieldArg dst, int ncol, hipStream_t st)
{
    hipLaunchKernelGGL(k_z2_noise, grid2(g.Vh, ncol), dim3(kBS), 0, st, seed, n0, g, parity, sp<P64>(dst));
    return hipGetLastError();
}

hipError_t launch_fin_alpha(const CgScalars& s, const double* partial, int nwaves, int ncol, hipStream_t st)
{
    hipLaunchKernelGGL(k_fin_alpha, dim3(ncol), dim3(256), 0, st, s, partial, nwaves);
    return hipGetLastError();
}

hipError_t launch_fin_beta(const CgScalars& s, const double* partial, int nwaves, int ncol, hipStream_t st)
{
    hipLaunchKernelGGL(k_fin_beta, dim3(ncol), dim3(256), 0, st, s, partial, nwaves);
    return hipGetLastError();
}

hipError_t launch_fin_reliable(const CgScalars& s, const double* partial, int nwaves, int ncol, hipStream_t st)
{
    hipLaunchKernelGGL(k_fin_reliable, dim3(ncol), dim3(256), 0, st, s, partial, nwaves);
    return hipGetLastError();
}

hipError_t launch_fin_sum(const double* partial, int nwaves, int ncol, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_fin_sum, dim3(ncol), dim3(256), 0, st, partial, nwaves, out);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// multishift CG
// --------------------------------------------------------------------------

namespace {

__global__ void k_axpy_norm(SpinorPtr<P64> x, SpinorPtr<P64> y, double a, int n, double* partial, int nwaves)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    double s = 0.0;
    if (j < n) {
        cx<double> xv[12], yv[12];
        load_spinor(x, c, j, xv);
        load_spinor(y, c, j, yv);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            yv[k].re = fmadd(a, xv[k].re, yv[k].re);
            yv[k].im = fmadd(a, xv[k].im, yv[k].im);
            s += yv[k].re * yv[k].re + yv[k].im * yv[k].im;
        }
        store_spinor(y, c, j, yv);
    }
    s = wave_sum(s);
    const int w = j >> kTileLog;
    if ((threadIdx.x & 63) == 0 && w < nwaves) partial[(size_t)c * nwaves + w] = s;
}

__global__ void k_ms_init(const MsState s, int ncol, double tol2)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    const double r2 = s.rho[c];
    s.stop2[c] = tol2 * r2;
    s.alpha_prev[c] = 1.0;
    s.beta_prev[c] = 0.0;
    s.iters[c] = 0;
    const int st = !isfinite(r2) ? COL_FAILED : (r2 > 0.0 ? COL_ACTIVE : COL_DONE);
    s.status[c] = st;
    for (int k = 0; k < s.nshift; k++) {
        const int i = c * s.nshift + k;
        s.zeta[i] = s.zeta_prev[i] = s.zeta_new[i] = 1.0;
        s.ak[i] = s.bk[i] = 0.0;
        s.act[i] = st == COL_ACTIVE;
        s.kiters[i] = 0;
    }
}

// alpha of the base system and, per active shift, zeta_{j+1} and the shift's alpha
__global__ void k_fin_ms_alpha(const MsState s, const double* pq, const double* pp, int nwaves, double sigma_b)
{
    const int c = blockIdx.x;
    if (s.status[c] != COL_ACTIVE) return;  // uniform per block
    const double qq = block_sum(pq + (size_t)c * nwaves, nwaves);
    const double ppn = sigma_b != 0.0 ? block_sum(pp + (size_t)c * nwaves, nwaves) : 0.0;
    if (threadIdx.x != 0) return;
    const double pAp = qq + sigma_b * ppn;
    if (!(pAp > 0.0) || !isfinite(pAp)) {
        s.status[c] = COL_FAILED;
        return;
    }
    const double al = s.rho[c] / pAp, ap = s.alpha_prev[c], bp = s.beta_prev[c];
    s.alpha[c] = al;
    for (int k = 0; k < s.nshift; k++) {
        const int i = c * s.nshift + k;
        if (!s.act[i]) continue;
        const double z = s.zeta[i], zp = s.zeta_prev[i];
        const double zn = z * zp * ap / (al * bp * (zp - z) + zp * ap * (1.0 + s.shift[k] * al));
        s.zeta_new[i] = zn;
        s.ak[i] = al * zn / z;
    }
}

// beta of the base system; per shift: beta, convergence (|zeta_{j+1}| |r_{j+1}| <= tol |b|), rotation
__global__ void k_fin_ms_beta(const MsState s, const double* pr, int nwaves)
{
    const int c = blockIdx.x;
    if (s.status[c] != COL_ACTIVE) return;
    const double rho = block_sum(pr + (size_t)c * nwaves, nwaves);
    if (threadIdx.x != 0) return;
    s.iters[c] += 1;
    if (!isfinite(rho)) {
        s.status[c] = COL_FAILED;
        return;
    }
    const double be = rho / s.rho[c];
    int any = 0;
    for (int k = 0; k < s.nshift; k++) {
        const int i = c * s.nshift + k;
        if (!s.act[i]) continue;
        const double z = s.zeta[i], zn = s.zeta_new[i];
        const double q = zn / z;
        s.bk[i] = be * q * q;
        s.kiters[i] += 1;
        if (zn * zn * rho <= s.stop2[c] || !isfinite(zn)) {
            s.act[i] = 0;
        } else {
            s.zeta_prev[i] = z;
            s.zeta[i] = zn;
            any = 1;
        }
    }
    s.alpha_prev[c] = s.alpha[c];
    s.beta_prev[c] = be;
    s.beta[c] = be;
    s.rho[c] = rho;
    if (!any) s.status[c] = COL_DONE;
}

__global__ void k_ms_update1(const MsState s, const MsFields f, double sigma_b, int n, double* partial, int nwaves)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    const bool on = s.status[c] == COL_ACTIVE;  // uniform per block
    double nr = 0.0;
    if (on && j < n) {
        const SpinorPtr<P64> r = sp<P64>(f.r), w = sp<P64>(f.w), p = sp<P64>(f.p);
        const double al = s.alpha[c];
        cx<double> rv[12], wv[12], pv[12];
        load_spinor(r, c, j, rv);
        load_spinor(w, c, j, wv);
        load_spinor(p, c, j, pv);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            rv[k].re = fmadd(-al, fmadd(sigma_b, pv[k].re, wv[k].re), rv[k].re);
            rv[k].im = fmadd(-al, fmadd(sigma_b, pv[k].im, wv[k].im), rv[k].im);
            nr += rv[k].re * rv[k].re + rv[k].im * rv[k].im;
        }
        store_spinor(r, c, j, rv);
        for (int q = 0; q < s.nshift; q++) {
            const int i = c * s.nshift + q;
            if (!s.act[i]) continue;
            const double a = s.ak[i];
            cx<double> xv[12], pk[12];
            const SpinorPtr<P64> X = sp<P64>(f.x[q]);
            load_spinor(X, c, j, xv);
            if (q == s.base) {
#pragma unroll
                for (int k = 0; k < 12; k++) pk[k] = pv[k];
            } else {
                load_spinor(sp<P64>(f.pk[q]), c, j, pk);
            }
#pragma unroll
            for (int k = 0; k < 12; k++) {
                xv[k].re = fmadd(a, pk[k].re, xv[k].re);
                xv[k].im = fmadd(a, pk[k].im, xv[k].im);
            }
            store_spinor(X, c, j, xv);
        }
    }
    nr = wave_sum(nr);
    const int w = j >> kTileLog;
    if (on && (threadIdx.x & 63) == 0 && w < nwaves) partial[(size_t)c * nwaves + w] = nr;
}

__global__ void k_ms_update2(const MsState s, const MsFields f, int n, double* partial, int nwaves)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    const bool on = s.status[c] == COL_ACTIVE;
    double np = 0.0;
    if (on && j < n) {
        const SpinorPtr<P64> r = sp<P64>(f.r), p = sp<P64>(f.p);
        cx<double> rv[12], pv[12];
        load_spinor(r, c, j, rv);
        for (int q = 0; q < s.nshift; q++) {
            const int i = c * s.nshift + q;
            if (q == s.base || !s.act[i]) continue;
            const double z = s.zeta[i], b = s.bk[i];
            const SpinorPtr<P64> P = sp<P64>(f.pk[q]);
            cx<double> pk[12];
            load_spinor(P, c, j, pk);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                pk[k].re = fmadd(b, pk[k].re, z * rv[k].re);
                pk[k].im = fmadd(b, pk[k].im, z * rv[k].im);
            }
            store_spinor(P, c, j, pk);
        }
        load_spinor(p, c, j, pv);
        const double be = s.beta[c];
#pragma unroll
        for (int k = 0; k < 12; k++) {
            pv[k].re = fmadd(be, pv[k].re, rv[k].re);
            pv[k].im = fmadd(be, pv[k].im, rv[k].im);
            np += pv[k].re * pv[k].re + pv[k].im * pv[k].im;
        }
        store_spinor(p, c, j, pv);
    }
    np = wave_sum(np);
    const int w = j >> kTileLog;
    if (on && (threadIdx.x & 63) == 0 && w < nwaves) partial[(size_t)c * nwaves + w] = np;
}

}  // namespace

hipError_t launch_axpy_norm(FieldArg x, FieldArg y, double a, int n, int ncol, double* partial, int nwaves,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_axpy_norm, grid2(n, ncol), dim3(kBS), 0, st, sp<P64>(x), sp<P64>(y), a, n, partial, nwaves);
    return hipGetLastError();
}

hipError_t launch_ms_init(const MsState& s, int ncol, double tol2, hipStream_t st)
{
    hipLaunchKernelGGL(k_ms_init, dim3((ncol + 63) / 64), dim3(64), 0, st, s, ncol, tol2);
    return hipGetLastError();
}

hipError_t launch_fin_ms_alpha(const MsState& s, const double* pq, const double* pp, int nwaves, int ncol,
                               double sigma_b, hipStream_t st)
{
    hipLaunchKernelGGL(k_fin_ms_alpha, dim3(ncol), dim3(256), 0, st, s, pq, pp, nwaves, sigma_b);
    return hipGetLastError();
}

hipError_t launch_fin_ms_beta(const MsState& s, const double* pr, int nwaves, int ncol, hipStream_t st)
{
    hipLaunchKernelGGL(k_fin_ms_beta, dim3(ncol), dim3(256), 0, st, s, pr, nwaves);
    return hipGetLastError();
}

hipError_t launch_ms_update1(const MsState& s, const MsFields& f, double sigma_b, int n, int ncol, double* partial,
                             int nwaves, hipStream_t st)
{
    if (s.nshift < 1 || s.nshift > kMaxShifts) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ms_update1, grid2(n, ncol), dim3(kBS), 0, st, s, f, sigma_b, n, partial, nwaves);
    return hipGetLastError();
}

hipError_t launch_ms_update2(const MsState& s, const MsFields& f, int n, int ncol, double* partial, int nwaves,
                             hipStream_t st)
{
    if (s.nshift < 1 || s.nshift > kMaxShifts) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ms_update2, grid2(n, ncol), dim3(kBS), 0, st, s, f, n, partial, nwaves);
    return hipGetLastError();
}

}  // namespace bq

namespace bq {
namespace {
__global__ void k_cg_init(const CgScalars s, int ncol, double tol2, const int* sel, const double* tol2c,
                          const double* rho_src)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol || (sel && !sel[c])) return;
    if (rho_src) s.rho[c] = rho_src[c];
    const double r2 = s.rho[c];
    s.stop2[c] = (tol2c ? tol2c[c] : tol2) * r2;
    s.rmax2[c] = r2;
    s.iters[c] = 0;
    s.nrel[c] = 0;
    s.restart[c] = 0;
    s.alpha[c] = 0.0;
    s.beta[c] = 0.0;
    s.status[c] = !isfinite(r2) ? COL_FAILED : (r2 > 0.0 ? COL_ACTIVE : COL_DONE);
}
}  // namespace

hipError_t launch_cg_init(const CgScalars& s, int ncol, double tol2, hipStream_t st, const int* sel,
                          const double* tol2c, const double* rho_src)
{
    hipLaunchKernelGGL(k_cg_init, dim3((ncol + 63) / 64), dim3(64), 0, st, s, ncol, tol2, sel, tol2c, rho_src);
    return hipGetLastError();
}

__global__ void k_set_status(int* status, const int* sel, int ncol, int value)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncol && sel[c]) status[c] = value;
}

hipError_t launch_set_status(int* status, const int* sel, int ncol, int value, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_status, dim3((ncol + 63) / 64), dim3(64), 0, st, status, sel, ncol, value);
    return hipGetLastError();
}
}  // namespace bq
