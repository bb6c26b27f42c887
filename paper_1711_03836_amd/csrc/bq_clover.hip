// Clover term of Eq. 2 on the device: field strength from the four-leaf
// clover, the two Hermitian 6x6 blocks per site and their inverses.
//
// In the chiral basis sigma_{mu nu} is block diagonal; with the Hermitian
// field strengths G_{mu nu} = -i F_{mu nu} (mu,nu = 0..3 for x,y,z,t) the
// clover matrix T = 1 + kappa c_SW sum_{mu<nu} sigma_{mu nu} (x) G_{mu nu} is
//   block +/- = 1 + ck [ s3 (x) (G01 -/+ G23) + s2 (x) (G02 +/- G13) + s1 (x) (G12 -/+ G03) ]
// (s1,s2,s3 Pauli matrices acting on the two spins of the block), i.e.
//   [[ 1 + ck X3,  ck (X1 - i X2) ], [ ck (X1 + i X2),  1 - ck X3 ]].
// Blocks are inverted with a complex Cholesky factorisation, which also
// checks positive definiteness.
#include "bq_kernels.h"

namespace bq {
namespace {

using c64 = cx<double>;

struct M3 {
    c64 m[9];
};

__device__ __forceinline__ M3 m3_mul(const M3& a, const M3& b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
            c64 s = cmul(a.m[i * 3 + 0], b.m[0 * 3 + k]);
            s = cmac(s, a.m[i * 3 + 1], b.m[1 * 3 + k]);
            s = cmac(s, a.m[i * 3 + 2], b.m[2 * 3 + k]);
            c.m[i * 3 + k] = s;
        }
    return c;
}

// a * b^dag
__device__ __forceinline__ M3 m3_mul_nd(const M3& a, const M3& b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
            c64 s = {0, 0};
            s = cmac(s, a.m[i * 3 + 0], c64{b.m[k * 3 + 0].re, -b.m[k * 3 + 0].im});
            s = cmac(s, a.m[i * 3 + 1], c64{b.m[k * 3 + 1].re, -b.m[k * 3 + 1].im});
            s = cmac(s, a.m[i * 3 + 2], c64{b.m[k * 3 + 2].re, -b.m[k * 3 + 2].im});
            c.m[i * 3 + k] = s;
        }
    return c;
}

// a^dag * b
__device__ __forceinline__ M3 m3_mul_dn(const M3& a, const M3& b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
            c64 s = {0, 0};
            s = cmacc(s, a.m[0 * 3 + i], b.m[0 * 3 + k]);
            s = cmacc(s, a.m[1 * 3 + i], b.m[1 * 3 + k]);
            s = cmacc(s, a.m[2 * 3 + i], b.m[2 * 3 + k]);
            c.m[i * 3 + k] = s;
        }
    return c;
}

struct Coord {
    int x[4];
};

__device__ __forceinline__ Coord shift(const Geom& g, Coord c, int mu, int d)
{
    int v = c.x[mu] + d;
    c.x[mu] = v < 0 ? v + g.L[mu] : (v >= g.L[mu] ? v - g.L[mu] : v);
    return c;
}

__device__ __forceinline__ M3 link_at(const Geom& g, const double2* const* U, const Coord& c, int mu)
{
    const int par = (c.x[0] + c.x[1] + c.x[2] + c.x[3]) & 1;
    const int lex = c.x[0] + g.L[0] * (c.x[1] + g.L[1] * (c.x[2] + g.L[2] * c.x[3]));
    const int j = lex >> 1;
    const double2* b = U[par * 4 + mu];
    M3 m;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        double2 t = at(b, j, k, 9);
        m.m[k] = {t.x, t.y};
    }
    return m;
}

// Hermitian traceless G = (Q - Q^dag)/(8i) of the four leaves in plane (mu, nu) at site c
__device__ M3 field_strength(const Geom& g, const double2* const* U, const Coord& c, int mu, int nu)
{
    const Coord xpm = shift(g, c, mu, +1), xpn = shift(g, c, nu, +1);
    const Coord xmm = shift(g, c, mu, -1), xmn = shift(g, c, nu, -1);
    const Coord xpn_mm = shift(g, xpn, mu, -1);
    const Coord xmm_mn = shift(g, xmm, nu, -1);
    const Coord xmn_pm = shift(g, xmn, mu, +1);

    const M3 Umu_x = link_at(g, U, c, mu), Unu_x = link_at(g, U, c, nu);
    M3 Q;
    // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
    {
        M3 a = m3_mul(Umu_x, link_at(g, U, xpm, nu));
        a = m3_mul_nd(a, link_at(g, U, xpn, mu));
        Q = m3_mul_nd(a, Unu_x);
    }
    // leaf 2: U_nu(x) U_mu(x+nu-mu)^dag U_nu(x-mu)^dag U_mu(x-mu)
    {
        M3 a = m3_mul_nd(Unu_x, link_at(g, U, xpn_mm, mu));
        a = m3_mul_nd(a, link_at(g, U, xmm, nu));
        a = m3_mul(a, link_at(g, U, xmm, mu));
#pragma unroll
        for (int k = 0; k < 9; k++) Q.m[k] = cadd(Q.m[k], a.m[k]);
    }
    // leaf 3: U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
    {
        // U_mu(x-mu)^dag U_nu(x-mu-nu)^dag = (U_nu(x-mu-nu) U_mu(x-mu))^dag
        const M3 ba = m3_mul(link_at(g, U, xmm_mn, nu), link_at(g, U, xmm, mu));
        M3 t;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int k = 0; k < 3; k++) t.m[i * 3 + k] = {ba.m[k * 3 + i].re, -ba.m[k * 3 + i].im};
        t = m3_mul(t, link_at(g, U, xmm_mn, mu));
        t = m3_mul(t, link_at(g, U, xmn, nu));
#pragma unroll
        for (int k = 0; k < 9; k++) Q.m[k] = cadd(Q.m[k], t.m[k]);
    }
    // leaf 4: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^dag
    {
        M3 a = m3_mul_dn(link_at(g, U, xmn, nu), link_at(g, U, xmn, mu));
        a = m3_mul(a, link_at(g, U, xmn_pm, nu));
        a = m3_mul_nd(a, Umu_x);
#pragma unroll
        for (int k = 0; k < 9; k++) Q.m[k] = cadd(Q.m[k], a.m[k]);
    }
    // G = (Q - Q^dag) / (8 i): G_ik = -i (Q_ik - conj(Q_ki)) / 8
    M3 G;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const c64 d = {Q.m[i * 3 + k].re - Q.m[k * 3 + i].re, Q.m[i * 3 + k].im + Q.m[k * 3 + i].im};
            G.m[i * 3 + k] = {d.im * 0.125, -d.re * 0.125};
        }
    const double tr = (G.m[0].re + G.m[4].re + G.m[8].re) / 3.0;
    G.m[0].re -= tr;
    G.m[4].re -= tr;
    G.m[8].re -= tr;
    return G;
}

// dense Hermitian 6x6 block helpers
struct H6 {
    c64 a[36];
};

__device__ __forceinline__ void pack_store(double2* T, int j, int blk, const H6& A)
{
    if (T == nullptr) return;
    at(T, j, blk * 18 + 0, 36) = make_double2(A.a[0].re, A.a[7].re);
    at(T, j, blk * 18 + 1, 36) = make_double2(A.a[14].re, A.a[21].re);
    at(T, j, blk * 18 + 2, 36) = make_double2(A.a[28].re, A.a[35].re);
#pragma unroll
    for (int i = 1; i < 6; i++)
#pragma unroll
        for (int k = 0; k < i; k++) {
            const c64 v = A.a[i * 6 + k];
            at(T, j, blk * 18 + 3 + i * (i - 1) / 2 + k, 36) = make_double2(v.re, v.im);
        }
}

__device__ __forceinline__ H6 pack_load(const double2* T, int j, int blk)
{
    H6 A;
    double2 d0 = at(T, j, blk * 18 + 0, 36), d1 = at(T, j, blk * 18 + 1, 36), d2 = at(T, j, blk * 18 + 2, 36);
    const double d[6] = {d0.x, d0.y, d1.x, d1.y, d2.x, d2.y};
#pragma unroll
    for (int i = 0; i < 6; i++) A.a[i * 6 + i] = {d[i], 0.0};
#pragma unroll
    for (int i = 1; i < 6; i++)
#pragma unroll
        for (int k = 0; k < i; k++) {
            double2 t = at(T, j, blk * 18 + 3 + i * (i - 1) / 2 + k, 36);
            A.a[i * 6 + k] = {t.x, t.y};
            A.a[k * 6 + i] = {t.x, -t.y};
        }
    return A;
}

// inverse of a Hermitian positive-definite 6x6 block by Cholesky A = L L^dag; returns false if not HPD
__device__ bool hpd_inverse(const H6& A, H6& Ai)
{
    c64 L[36];
#pragma unroll
    for (int k = 0; k < 36; k++) L[k] = {0, 0};
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; j++) {
        double s = A.a[j * 6 + j].re;
#pragma unroll
        for (int k = 0; k < j; k++) s -= cnorm2(L[j * 6 + k]);
        ok = ok && (s > 0.0) && isfinite(s);
        const double ljj = sqrt(s > 0.0 ? s : 1.0);
        const double inv = 1.0 / ljj;
        L[j * 6 + j] = {ljj, 0.0};
#pragma unroll
        for (int i = j + 1; i < 6; i++) {
            c64 t = A.a[i * 6 + j];
#pragma unroll
            for (int k = 0; k < j; k++) {
                // t -= L[i][k] * conj(L[j][k])
                const c64 a = L[i * 6 + k], b = L[j * 6 + k];
                t.re -= a.re * b.re + a.im * b.im;
                t.im -= a.im * b.re - a.re * b.im;
            }
            L[i * 6 + j] = cscale(inv, t);
        }
    }
    // W = L^-1 (lower triangular)
    c64 W[36];
#pragma unroll
    for (int k = 0; k < 36; k++) W[k] = {0, 0};
#pragma unroll
    for (int i = 0; i < 6; i++) {
        const double inv = 1.0 / L[i * 6 + i].re;
        W[i * 6 + i] = {inv, 0.0};
#pragma unroll
        for (int j = 0; j < i; j++) {
            c64 s = {0, 0};
#pragma unroll
            for (int k = j; k < i; k++) s = cmac(s, L[i * 6 + k], W[k * 6 + j]);
            W[i * 6 + j] = cscale(-inv, s);
        }
    }
    // A^-1 = W^dag W
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int j = 0; j <= i; j++) {
            c64 s = {0, 0};
#pragma unroll
            for (int k = i; k < 6; k++) s = cmacc(s, W[k * 6 + i], W[k * 6 + j]);
            Ai.a[i * 6 + j] = s;
            Ai.a[j * 6 + i] = {s.re, -s.im};
        }
#pragma unroll
    for (int i = 0; i < 6; i++) Ai.a[i * 6 + i].im = 0.0;
    return ok;
}

// B block (without identity and kappa c_SW) from X1, X2, X3
__device__ __forceinline__ H6 block_from(const M3& X1, const M3& X2, const M3& X3)
{
    H6 B;
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) {
            const c64 x1 = X1.m[a * 3 + b], x2 = X2.m[a * 3 + b], x3 = X3.m[a * 3 + b];
            B.a[a * 6 + b] = x3;                                   // (0,0): X3
            B.a[(3 + a) * 6 + 3 + b] = {-x3.re, -x3.im};           // (1,1): -X3
            B.a[a * 6 + 3 + b] = {x1.re + x2.im, x1.im - x2.re};   // (0,1): X1 - i X2
            B.a[(3 + a) * 6 + b] = {x1.re - x2.im, x1.im + x2.re}; // (1,0): X1 + i X2
        }
    return B;
}

__global__ __launch_bounds__(64) void k_clover_build(const CloverBuild c, int parity)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= c.g.Vh) return;
    const Site s = site_of(c.g, parity, j);
    Coord x;
    x.x[0] = s.x;
    x.x[1] = s.y;
    x.x[2] = s.z;
    x.x[3] = s.t;
    const double2* U[8];
    for (int k = 0; k < 8; k++) U[k] = c.U64[k];
    const M3 G01 = field_strength(c.g, U, x, 0, 1), G02 = field_strength(c.g, U, x, 0, 2);
    const M3 G03 = field_strength(c.g, U, x, 0, 3), G12 = field_strength(c.g, U, x, 1, 2);
    const M3 G13 = field_strength(c.g, U, x, 1, 3), G23 = field_strength(c.g, U, x, 2, 3);
    bool ok = true;
#pragma unroll
    for (int blk = 0; blk < 2; blk++) {
        const double sg = blk == 0 ? -1.0 : +1.0;  // block 0: X3 = G01 - G23, X2 = G02 + G13, X1 = G12 - G03
        M3 X1, X2, X3;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            X3.m[k] = {G01.m[k].re + sg * G23.m[k].re, G01.m[k].im + sg * G23.m[k].im};
            X2.m[k] = {G02.m[k].re - sg * G13.m[k].re, G02.m[k].im - sg * G13.m[k].im};
            X1.m[k] = {G12.m[k].re + sg * G03.m[k].re, G12.m[k].im + sg * G03.m[k].im};
        }
        const H6 B = block_from(X1, X2, X3);
        if (c.B[parity]) pack_store(c.B[parity], j, blk, B);
        H6 T;
#pragma unroll
        for (int k = 0; k < 36; k++) T.a[k] = cscale(c.ckappa, B.a[k]);
#pragma unroll
        for (int i = 0; i < 6; i++) T.a[i * 6 + i].re += 1.0;
        if (c.T[parity]) pack_store(c.T[parity], j, blk, T);
        if (c.Tinv[parity]) {
            H6 Ti;
            ok = hpd_inverse(T, Ti) && ok;
            pack_store(c.Tinv[parity], j, blk, Ti);
        }
    }
    if (!ok && c.bad) *c.bad = 1;
}

__global__ __launch_bounds__(64) void k_clover_from_B(const Geom g, const double2* B, double ck, double2* T, double2* Tinv, int* bad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.Vh) return;
    bool ok = true;
#pragma unroll 1
    for (int blk = 0; blk < 2; blk++) {
        H6 A = pack_load(B, j, blk);
#pragma unroll
        for (int k = 0; k < 36; k++) A.a[k] = cscale(ck, A.a[k]);
#pragma unroll
        for (int i = 0; i < 6; i++) A.a[i * 6 + i].re += 1.0;
        if (T) pack_store(T, j, blk, A);
        if (Tinv) {
            H6 Ai;
            ok = hpd_inverse(A, Ai) && ok;
            pack_store(Tinv, j, blk, Ai);
        }
    }
    if (!ok && bad) *bad = 1;
}

struct CloverCols {
    const void* p[kMaxCols];
};

template <class P>
__global__ void k_clover_apply(const Geom g, const typename P::unit* C0, SpinorPtr<P> in, SpinorPtr<P> out, int ncol,
                               int percol, const CloverCols cc, const int* status, int statmask)
{
    using T = typename P::real;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= g.Vh || c >= ncol || (status && !col_selected(status, statmask, c))) return;
    const typename P::unit* C = percol ? (const typename P::unit*)cc.p[c] : C0;
    cx<T> v[12], y[12];
    load_spinor(in, c, j, v);
#pragma unroll
    for (int blk = 0; blk < 2; blk++) {
        cx<T> cb[18];
        if constexpr (P::id == PREC_F16) {
#pragma unroll
            for (int u = 0; u < 9; u++) CxIO<P16, 2>::unpack(at(C, j, blk * 9 + u, 18), cb[2 * u], cb[2 * u + 1]);
        } else {
#pragma unroll
            for (int k = 0; k < 18; k++) {
                auto t = at(C, j, blk * 18 + k, 36);
                cb[k] = {t.x, t.y};
            }
        }
        const T d[6] = {cb[0].re, cb[0].im, cb[1].re, cb[1].im, cb[2].re, cb[2].im};
#pragma unroll
        for (int i = 0; i < 6; i++) y[blk * 6 + i] = cscale(d[i], v[blk * 6 + i]);
#pragma unroll
        for (int i = 1; i < 6; i++)
#pragma unroll
            for (int k = 0; k < i; k++) {
                const cx<T> A = cb[3 + i * (i - 1) / 2 + k];
                y[blk * 6 + i] = cmac(y[blk * 6 + i], A, v[blk * 6 + k]);
                y[blk * 6 + k] = cmacc(y[blk * 6 + k], A, v[blk * 6 + i]);
            }
    }
    store_spinor(out, c, j, y);
}

// FP64 -> FP32 clover, one storage unit of one site per thread (the two precisions' tiles
// order their units differently)
__global__ void k_clover_convert32(const double2* src, float2* dst, int Vh)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int u = blockIdx.y;
    if (j >= Vh) return;
    const double2 t = at(src, j, u, 36);
    at(dst, j, u, 36) = make_float2((float)t.x, (float)t.y);
}

// FP64 packed clover (36 complex/site) -> FP16 (18 units of 2 complex/site)
__global__ void k_clover_convert16(const double2* src, uint2* dst, int Vh)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int u = blockIdx.y;  // 0..17
    if (j >= Vh) return;
    double2 a = at(src, j, 2 * u, 36), b = at(src, j, 2 * u + 1, 36);
    at(dst, j, u, 18) = CxIO<P16, 2>::pack(cx<float>{(float)a.x, (float)a.y}, cx<float>{(float)b.x, (float)b.y});
}

// sum over the 6 planes of Re tr U_{mu nu}(x) / 3, one FP64 partial per wavefront
struct LinkTable {
    const double2* U[8];
};

__global__ __launch_bounds__(64) void k_plaquette_v(const Geom g, const LinkTable t, int parity, double* partial, int nwaves)
{
    // kernel arguments cannot hold a pointer-to-pointer into host memory; copy the table into registers
    const double2* U[8];
    for (int k = 0; k < 8; k++) U[k] = t.U[k];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (j < g.Vh) {
        const Site s = site_of(g, parity, j);
        Coord x;
        x.x[0] = s.x;
        x.x[1] = s.y;
        x.x[2] = s.z;
        x.x[3] = s.t;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                M3 a = m3_mul(link_at(g, U, x, mu), link_at(g, U, shift(g, x, mu, +1), nu));
                a = m3_mul_nd(a, link_at(g, U, shift(g, x, nu, +1), mu));
                a = m3_mul_nd(a, link_at(g, U, x, nu));
                acc += (a.m[0].re + a.m[4].re + a.m[8].re) / 3.0;
            }
    }
    acc = wave_sum(acc);
    const int w = j >> kTileLog;
    if ((threadIdx.x & 63) == 0 && w < nwaves) partial[w] = acc;
}

}  // namespace

hipError_t launch_plaquette(const Geom& g, const double2* const U64[8], double* partial, int nparts, hipStream_t st)
{
    // partial: 2 * (padded Vh / 64) entries, parity 0 first
    LinkTable t;
    for (int k = 0; k < 8; k++) t.U[k] = U64[k];
    const int nw = pad_sites(g.Vh) / kTile;
    if (nparts < 2 * nw) return hipErrorInvalidValue;
    for (int p = 0; p < 2; p++)
        hipLaunchKernelGGL(k_plaquette_v, dim3((g.Vh + 63) / 64), dim3(64), 0, st, g, t, p, partial + p * nw, nw);
    return hipGetLastError();
}

hipError_t launch_clover_build(const CloverBuild& c, hipStream_t st)
{
    const int bs = 64;
    for (int p = 0; p < 2; p++)
        hipLaunchKernelGGL(k_clover_build, dim3((c.g.Vh + bs - 1) / bs), dim3(bs), 0, st, c, p);
    return hipGetLastError();
}

hipError_t launch_clover_from_B(const Geom& g, int parity, const double2* B, double ck, double2* T, double2* Tinv,
                                int* bad, hipStream_t st)
{
    (void)parity;
    const int bs = 64;
    hipLaunchKernelGGL(k_clover_from_B, dim3((g.Vh + bs - 1) / bs), dim3(bs), 0, st, g, B, ck, T, Tinv, bad);
    return hipGetLastError();
}

hipError_t launch_clover_apply(int prec, const Geom& g, const void* clov, FieldArg in, FieldArg out, int ncol,
                               hipStream_t st, const void* const* cclov, const int* status, int statmask)
{
    const int bs = 128;
    dim3 grid((g.Vh + bs - 1) / bs, ncol);
    CloverCols cc{};
    const int percol = cclov != nullptr;
    if (percol) {
        if (ncol > kMaxCols) return hipErrorInvalidValue;
        for (int c = 0; c < ncol; c++) cc.p[c] = cclov[c];
    }
    switch (prec) {
    case PREC_F64:
        hipLaunchKernelGGL(k_clover_apply<P64>, grid, dim3(bs), 0, st, g, (const double2*)clov,
                           SpinorPtr<P64>{(double2*)in.d, in.s, in.cstride, in.sstride},
                           SpinorPtr<P64>{(double2*)out.d, out.s, out.cstride, out.sstride}, ncol, percol, cc, status, statmask);
        break;
    case PREC_F32:
        hipLaunchKernelGGL(k_clover_apply<P32>, grid, dim3(bs), 0, st, g, (const float2*)clov,
                           SpinorPtr<P32>{(float2*)in.d, in.s, in.cstride, in.sstride},
                           SpinorPtr<P32>{(float2*)out.d, out.s, out.cstride, out.sstride}, ncol, percol, cc, status, statmask);
        break;
    case PREC_F16:
        hipLaunchKernelGGL(k_clover_apply<P16>, grid, dim3(bs), 0, st, g, (const uint2*)clov,
                           SpinorPtr<P16>{(uint2*)in.d, in.s, in.cstride, in.sstride},
                           SpinorPtr<P16>{(uint2*)out.d, out.s, out.cstride, out.sstride}, ncol, percol, cc, status, statmask);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_clover_convert(int prec, const double2* src, void* dst, int Vh, hipStream_t st)
{
    const int bs = 256;
    const int Vp = pad_sites(Vh);
    if (prec == PREC_F32) {
        hipLaunchKernelGGL(k_clover_convert32, dim3((Vp + bs - 1) / bs, 36), dim3(bs), 0, st, src, (float2*)dst, Vp);
    } else if (prec == PREC_F16) {
        hipLaunchKernelGGL(k_clover_convert16, dim3((Vh + bs - 1) / bs, 18), dim3(bs), 0, st, src, (uint2*)dst, Vh);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bq
