// Vector kernels of the solver list's non-Hermitian and block solvers (section "Algorithms":
// BiCGstab, block cg): fused updates and per-column FP64 reductions, one partial per wavefront
// of 64 sites and a fixed-order finalisation per column, as in the CG kernels, so a column's
// result does not depend on the other columns of a batch.
#include "bq_kernels.h"

namespace bq {
namespace {

template <class P>
SpinorPtr<P> sp(const FieldArg& f)
{
    return SpinorPtr<P>{(typename P::unit*)f.d, f.s, f.cstride, f.sstride};
}

constexpr int kBS = 256;
inline dim3 grid2(int n, int ncol) { return dim3((n + kBS - 1) / kBS, ncol); }

__device__ __forceinline__ double bsum(const double* __restrict__ part, int n)
{
    // fixed assignment of elements to threads and a fixed combination order
    __shared__ double w[4];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * 256 < n; i += 4 * 256) {
        a0 += part[i];
        a1 += part[i + 256];
        a2 += part[i + 512];
        a3 += part[i + 768];
    }
    for (; i < n; i += 256) a0 += part[i];
    double s = (a0 + a1) + (a2 + a3);
    s = wave_sum(s);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
    __syncthreads();
    return (w[0] + w[1]) + (w[2] + w[3]);
}

__device__ __forceinline__ bool on(const int* status, int c) { return status[c] == COL_ACTIVE; }

// complex scalar helpers on (re, im) pairs stored as double2
__device__ __forceinline__ double2 zmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ double2 zdiv(double2 a, double2 b)
{
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ bool zfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// --------------------------------------------------------------------------
// BiCGstab (van der Vorst) on Mhat, per column, inner precision P, FP64 reductions
// --------------------------------------------------------------------------

// p = r + beta (p - omega v)
template <class P>
__global__ void k_bicg_p(SpinorPtr<P> r, SpinorPtr<P> p, SpinorPtr<P> v, const BicgScalars s, int n)
{
    using T = typename P::real;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= n || !on(s.status, c)) return;
    const double2 be = s.beta[c], om = s.omega[c];
    const T br = (T)be.x, bi = (T)be.y, orr = (T)om.x, oi = (T)om.y;
    cx<T> rv[12], pv[12], vv[12];
    load_spinor(r, c, j, rv);
    load_spinor(p, c, j, pv);
    load_spinor(v, c, j, vv);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        // d = p - omega v ; p = r + beta d
        const cx<T> d = {pv[k].re - (orr * vv[k].re - oi * vv[k].im), pv[k].im - (orr * vv[k].im + oi * vv[k].re)};
        pv[k] = {rv[k].re + (br * d.re - bi * d.im), rv[k].im + (br * d.im + bi * d.re)};
    }
    store_spinor(p, c, j, pv);
}

// partials of <a1, b1> and <a2, b2> (complex, FP64 accumulation): [col][4][wave]
template <class P>
__global__ void k_dots2(SpinorPtr<P> a1, SpinorPtr<P> b1, SpinorPtr<P> a2, SpinorPtr<P> b2, const int* status,
                        int n, double* partial, int nwaves)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (!on(status, c)) return;  // uniform per block
    double d[4] = {0.0, 0.0, 0.0, 0.0};
    if (j < n) {
        cx<typename P::real> x[12], y[12];
        load_spinor(a1, c, j, x);
        load_spinor(b1, c, j, y);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            d[0] += (double)x[k].re * y[k].re + (double)x[k].im * y[k].im;
            d[1] += (double)x[k].re * y[k].im - (double)x[k].im * y[k].re;
        }
        if (a2.d) {
            load_spinor(a2, c, j, x);
            load_spinor(b2, c, j, y);
#pragma unroll
            for (int k = 0; k < 12; k++) {
                d[2] += (double)x[k].re * y[k].re + (double)x[k].im * y[k].im;
                d[3] += (double)x[k].re * y[k].im - (double)x[k].im * y[k].re;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; q++) d[q] = wave_sum(d[q]);
    const int w = j >> kTileLog;
    if ((threadIdx.x & 63) == 0 && w < nwaves)
#pragma unroll
        for (int q = 0; q < 4; q++) partial[((size_t)c * 4 + q) * nwaves + w] = d[q];
}

// s = r - alpha v
template <class P>
__global__ void k_bicg_s(SpinorPtr<P> r, SpinorPtr<P> v, SpinorPtr<P> s_, const BicgScalars s, int n)
{
    using T = typename P::real;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= n || !on(s.status, c)) return;
    const double2 al = s.alpha[c];
    const T ar = (T)al.x, ai = (T)al.y;
    cx<T> rv[12], vv[12];
    load_spinor(r, c, j, rv);
    load_spinor(v, c, j, vv);
#pragma unroll
    for (int k = 0; k < 12; k++) rv[k] = {rv[k].re - (ar * vv[k].re - ai * vv[k].im), rv[k].im - (ar * vv[k].im + ai * vv[k].re)};
    store_spinor(s_, c, j, rv);
}

// x += alpha p + omega s ; r = s - omega t ; partials of <rhat, r> and <r, r>
template <class P>
__global__ void k_bicg_xr(SpinorPtr<P> x, SpinorPtr<P> p, SpinorPtr<P> s_, SpinorPtr<P> t, SpinorPtr<P> r,
                          SpinorPtr<P> rhat, const BicgScalars s, int n, double* partial, int nwaves)
{
    using T = typename P::real;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (!on(s.status, c)) return;
    double d[4] = {0.0, 0.0, 0.0, 0.0};
    if (j < n) {
        const double2 al = s.alpha[c], om = s.omega[c];
        const T ar = (T)al.x, ai = (T)al.y, orr = (T)om.x, oi = (T)om.y;
        cx<T> xv[12], pv[12], sv[12], tv[12], hv[12];
        load_spinor(x, c, j, xv);
        load_spinor(p, c, j, pv);
        load_spinor(s_, c, j, sv);
        load_spinor(t, c, j, tv);
        load_spinor(rhat, c, j, hv);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            xv[k].re += (ar * pv[k].re - ai * pv[k].im) + (orr * sv[k].re - oi * sv[k].im);
            xv[k].im += (ar * pv[k].im + ai * pv[k].re) + (orr * sv[k].im + oi * sv[k].re);
            sv[k] = {sv[k].re - (orr * tv[k].re - oi * tv[k].im), sv[k].im - (orr * tv[k].im + oi * tv[k].re)};
            d[0] += (double)hv[k].re * sv[k].re + (double)hv[k].im * sv[k].im;
            d[1] += (double)hv[k].re * sv[k].im - (double)hv[k].im * sv[k].re;
            d[2] += (double)sv[k].re * sv[k].re + (double)sv[k].im * sv[k].im;
        }
        store_spinor(x, c, j, xv);
        store_spinor(r, c, j, sv);
    }
#pragma unroll
    for (int q = 0; q < 3; q++) d[q] = wave_sum(d[q]);
    const int w = j >> kTileLog;
    if ((threadIdx.x & 63) == 0 && w < nwaves)
#pragma unroll
        for (int q = 0; q < 4; q++) partial[((size_t)c * 4 + q) * nwaves + w] = d[q];
}

// alpha = rho / <rhat, v>
__global__ void k_fin_bicg_alpha(const BicgScalars s, const double* partial, int nwaves)
{
    const int c = blockIdx.x;
    if (!on(s.status, c)) return;
    const double* pc = partial + (size_t)c * 4 * nwaves;
    const double re = bsum(pc, nwaves), im = bsum(pc + nwaves, nwaves);
    if (threadIdx.x != 0) return;
    const double2 hv = make_double2(re, im);
    if (!(hv.x * hv.x + hv.y * hv.y > 0.0) || !zfinite(hv)) {
        s.status[c] = COL_FAILED;
        return;
    }
    s.alpha[c] = zdiv(s.rho[c], hv);
}

// omega = <t, s> / <t, t>
__global__ void k_fin_bicg_omega(const BicgScalars s, const double* partial, int nwaves)
{
    const int c = blockIdx.x;
    if (!on(s.status, c)) return;
    const double* pc = partial + (size_t)c * 4 * nwaves;
    const double tsr = bsum(pc, nwaves), tsi = bsum(pc + nwaves, nwaves), tt = bsum(pc + 2 * nwaves, nwaves);
    if (threadIdx.x != 0) return;
    if (!(tt > 0.0) || !isfinite(tt)) {
        s.status[c] = COL_FAILED;
        return;
    }
    s.omega[c] = make_double2(tsr / tt, tsi / tt);
}

// rho' = <rhat, r>, |r|^2: stop test, beta = (rho'/rho)(alpha/omega)
__global__ void k_fin_bicg_rho(const BicgScalars s, const double* partial, int nwaves)
{
    const int c = blockIdx.x;
    if (!on(s.status, c)) return;
    const double* pc = partial + (size_t)c * 4 * nwaves;
    const double hr = bsum(pc, nwaves), hi = bsum(pc + nwaves, nwaves), rr = bsum(pc + 2 * nwaves, nwaves);
    if (threadIdx.x != 0) return;
    s.iters[c] += 1;
    const double2 rn = make_double2(hr, hi);
    if (!isfinite(rr) || !zfinite(rn)) {
        s.status[c] = COL_FAILED;
        return;
    }
    s.r2[c] = rr;
    if (rr <= s.stop2[c]) {  // inner goal reached: the next reliable pass folds x and decides
        s.status[c] = COL_STOPPED;
        return;
    }
    const double2 om = s.omega[c];
    if (!(rn.x * rn.x + rn.y * rn.y > 0.0) || !(om.x * om.x + om.y * om.y > 0.0)) {
        s.status[c] = COL_STOPPED;  // breakdown: restart from the true residual
        return;
    }
    s.beta[c] = zmul(zdiv(rn, s.rho[c]), zdiv(s.alpha[c], om));
    s.rho[c] = rn;
}

// after the FP64 residual r64 of the columns in COL_STOPPED: done, or restart the inner iteration
// (status COL_JUST_STOPPED and restart = 1 until the inner vectors are reset) with inner goal
// |r| <= delta |r64| (never below tol |b|)
__global__ void k_fin_bicg_reliable(const BicgScalars s, const double* partial, int nwaves, int ncol)
{
    const int c = blockIdx.x;
    if (c >= ncol || s.status[c] != COL_STOPPED) {
        if (threadIdx.x == 0 && c < ncol) s.restart[c] = 0;
        return;
    }
    const double r2 = bsum(partial + (size_t)c * nwaves, nwaves);
    if (threadIdx.x != 0) return;
    s.nrel[c] += 1;
    s.restart[c] = 0;
    if (!isfinite(r2)) {
        s.status[c] = COL_FAILED;
    } else if (r2 <= s.tol2b2[c]) {
        s.status[c] = COL_DONE;
    } else {
        s.status[c] = COL_JUST_STOPPED;  // restarting: the host resets the inner vectors, then activates
        s.restart[c] = 1;
        s.stop2[c] = fmax(s.delta2 * r2, s.tol2b2[c]);
        s.rho[c] = make_double2(r2, 0.0);  // rhat = r after the restart
        s.alpha[c] = s.omega[c] = make_double2(1.0, 0.0);
        s.beta[c] = make_double2(0.0, 0.0);
    }
}

}  // namespace

#define BQ_PREC_SWITCH(prec, CALL)                                         \
    switch (prec) {                                                        \
    case PREC_F64: { using P = P64; CALL; } break;                         \
    case PREC_F32: { using P = P32; CALL; } break;                         \
    default: return hipErrorInvalidValue;                                  \
    }

hipError_t launch_bicg_p(int prec, FieldArg r, FieldArg p, FieldArg v, const BicgScalars& s, int n, int ncol,
                         hipStream_t st)
{
    BQ_PREC_SWITCH(prec, hipLaunchKernelGGL(k_bicg_p<P>, grid2(n, ncol), dim3(kBS), 0, st, sp<P>(r), sp<P>(p), sp<P>(v), s, n))
    return hipGetLastError();
}

hipError_t launch_dots2(int prec, FieldArg a1, FieldArg b1, FieldArg a2, FieldArg b2, const int* status, int n,
                        int ncol, double* partial, int nwaves, hipStream_t st)
{
    BQ_PREC_SWITCH(prec, hipLaunchKernelGGL(k_dots2<P>, grid2(n, ncol), dim3(kBS), 0, st, sp<P>(a1), sp<P>(b1),
                                            sp<P>(a2), sp<P>(b2), status, n, partial, nwaves))
    return hipGetLastError();
}

hipError_t launch_bicg_s(int prec, FieldArg r, FieldArg v, FieldArg s_, const BicgScalars& s, int n, int ncol,
                         hipStream_t st)
{
    BQ_PREC_SWITCH(prec, hipLaunchKernelGGL(k_bicg_s<P>, grid2(n, ncol), dim3(kBS), 0, st, sp<P>(r), sp<P>(v), sp<P>(s_), s, n))
    return hipGetLastError();
}

hipError_t launch_bicg_xr(int prec, FieldArg x, FieldArg p, FieldArg s_, FieldArg t, FieldArg r, FieldArg rhat,
                          const BicgScalars& s, int n, int ncol, double* partial, int nwaves, hipStream_t st)
{
    BQ_PREC_SWITCH(prec, hipLaunchKernelGGL(k_bicg_xr<P>, grid2(n, ncol), dim3(kBS), 0, st, sp<P>(x), sp<P>(p),
                                            sp<P>(s_), sp<P>(t), sp<P>(r), sp<P>(rhat), s, n, partial, nwaves))
    return hipGetLastError();
}
#undef BQ_PREC_SWITCH

hipError_t launch_fin_bicg(int step, const BicgScalars& s, const double* partial, int nwaves, int ncol, hipStream_t st)
{
    switch (step) {
    case 0: hipLaunchKernelGGL(k_fin_bicg_alpha, dim3(ncol), dim3(256), 0, st, s, partial, nwaves); break;
    case 1: hipLaunchKernelGGL(k_fin_bicg_omega, dim3(ncol), dim3(256), 0, st, s, partial, nwaves); break;
    case 2: hipLaunchKernelGGL(k_fin_bicg_rho, dim3(ncol), dim3(256), 0, st, s, partial, nwaves); break;
    case 3: hipLaunchKernelGGL(k_fin_bicg_reliable, dim3(ncol), dim3(256), 0, st, s, partial, nwaves, ncol); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bq
