// Block CG and block multishift CG (the solver list's "block multishift cg"), device side.
//
// All right-hand sides share one block Krylov space of the base system A + sigma_b.  Its N x N
// step matrices, alpha = (P^dag A P)^-1 (R^dag R) and beta = (R^dag R)^-1 (R'^dag R'), and the
// shift recurrences (the residual block of shift s is R xi_s with an N x N matrix xi_s) are
// formed on the device by one wavefront from Gram matrices that the streaming kernels reduce;
// the field updates are column combinations with those matrices.  Fields are FP64 odd-site
// spinors in the site-tiled layout, so unit t of every column belongs to the same site and
// spin-colour component and a column combination is a loop over units.
#include "bq_kernels.h"

namespace bq {
namespace {

constexpr int LD = kBlockMax;

__device__ __forceinline__ double2 cz() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a += b c
__device__ __forceinline__ void cfma(double2& a, double2 b, double2 c)
{
    a.x = fma(b.x, c.x, fma(-b.y, c.y, a.x));
    a.y = fma(b.x, c.y, fma(b.y, c.x, a.y));
}
// a += conj(b) c
__device__ __forceinline__ void cfmac(double2& a, double2 b, double2 c)
{
    a.x = fma(b.x, c.x, fma(b.y, c.y, a.x));
    a.y = fma(b.x, c.y, fma(-b.y, c.x, a.y));
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b)
{
    const double d = 1.0 / cabs2(b);
    return make_double2((a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d);
}
__device__ __forceinline__ double2 cscal(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

__device__ __forceinline__ double2* mat(const BlockState& S, int slot) { return S.mats + (size_t)slot * LD * LD; }
__device__ __forceinline__ bool on(unsigned mask, int i) { return (mask >> i) & 1u; }

// --------------------------------------------------------------------------
// Gram matrices
// --------------------------------------------------------------------------

// One wavefront per group of kGramTiles tiles (lane = site of the tile), one 4 x 4 block of
// (i, j) column pairs per grid row; the 16 sums are reduced over the wave by a fixed butterfly,
// so the partials depend only on the lattice and the columns.
__global__ __launch_bounds__(256) void k_block_gram(FieldArg X, FieldArg Y, FieldArg Z, double s, BlockState S,
                                                    int vh, int tiles, double2* partial)
{
    if (S.ctrl[BC_STOP]) return;
    const int lane = threadIdx.x & 63;
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int ngroups = (tiles + kGramTiles - 1) / kGramTiles;
    if (g >= ngroups) return;  // uniform over the wave
    const int nb = (S.ncol + 3) / 4;
    const int i0 = 4 * ((int)blockIdx.y / nb), j0 = 4 * ((int)blockIdx.y % nb);
    const unsigned mask = (unsigned)S.ctrl[BC_MASK];
    const double2* x = (const double2*)X.d;
    const double2* y = (const double2*)Y.d;
    const double2* z = (const double2*)Z.d;
    bool xon[4], yon[4];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        xon[a] = i0 + a < S.ncol && on(mask, i0 + a);
        yon[a] = j0 + a < S.ncol && on(mask, j0 + a);
    }
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = cz();
    const int t1 = min(tiles, (g + 1) * kGramTiles);
    for (int tile = g * kGramTiles; tile < t1; tile++) {
        const bool site = tile * 64 + lane < vh;
        const size_t u0 = (size_t)tile * 12 * 64 + lane;
        for (int c = 0; c < 12; c++) {
            const size_t u = u0 + (size_t)c * 64;
            double2 xv[4], yv[4];
#pragma unroll
            for (int a = 0; a < 4; a++) {
                xv[a] = (xon[a] && site) ? x[(size_t)(i0 + a) * X.cstride + u] : cz();
                double2 v = cz();
                if (yon[a] && site) {
                    v = y[(size_t)(j0 + a) * Y.cstride + u];
                    if (z) {
                        const double2 w = z[(size_t)(j0 + a) * Z.cstride + u];
                        v.x = fma(s, w.x, v.x);
                        v.y = fma(s, w.y, v.y);
                    }
                }
                yv[a] = v;
            }
#pragma unroll
            for (int a = 0; a < 4; a++)
#pragma unroll
                for (int b = 0; b < 4; b++) cfmac(acc[a][b], xv[a], yv[b]);
        }
    }
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                acc[a][b].x += __shfl_xor(acc[a][b].x, o);
                acc[a][b].y += __shfl_xor(acc[a][b].y, o);
            }
    if (lane == 0) {
        double2* out = partial + ((size_t)g * nb * nb + blockIdx.y) * 16;
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) out[a * 4 + b] = acc[a][b];
    }
}

// One workgroup per matrix entry (i, j): the group partials summed in a fixed order.
__global__ __launch_bounds__(256) void k_block_gram_fin(BlockState S, const double2* partial, int tiles, int slot)
{
    if (S.ctrl[BC_STOP]) return;
    const int N = S.ncol;
    const int i = blockIdx.x / N, j = blockIdx.x % N;
    const int nb = (N + 3) / 4;
    const int blk = (i / 4) * nb + j / 4, e = (i % 4) * 4 + j % 4;
    const int ngroups = (tiles + kGramTiles - 1) / kGramTiles;
    double2 a = cz();
    for (int g = threadIdx.x; g < ngroups; g += 256) a = cadd(a, partial[((size_t)g * nb * nb + blk) * 16 + e]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a.x += __shfl_xor(a.x, o);
        a.y += __shfl_xor(a.y, o);
    }
    __shared__ double2 w[4];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) mat(S, slot)[i * LD + j] = cadd(cadd(w[0], w[1]), cadd(w[2], w[3]));
}

// --------------------------------------------------------------------------
// N x N complex algebra by one wavefront: lane j works on column j; every helper starts with
// its inputs in LDS and ends with a barrier.  A failed factorisation returns false on every
// lane alike (the test reads the same LDS word everywhere).
// --------------------------------------------------------------------------
typedef double2 Mat[LD][LD];

struct StepLds {
    Mat a, b, c, d, e, f, g;
    double2 aug[LD][2 * LD];
    double2 fac[LD];
    int idx[LD];
    int pos[LD];  // packed position of a column, -1 if not active
};

__device__ void m_gather(Mat& D, const double2* full, const StepLds& L, int n)
{
    const int j = threadIdx.x;
    if (j < n)
        for (int i = 0; i < n; i++) D[i][j] = full[L.idx[i] * LD + L.idx[j]];
    __syncthreads();
}

__device__ void m_load(Mat& D, const double2* packed, int n)
{
    const int j = threadIdx.x;
    if (j < n)
        for (int i = 0; i < n; i++) D[i][j] = packed[i * LD + j];
    __syncthreads();
}

__device__ void m_store(double2* packed, const Mat& D, int n)
{
    const int j = threadIdx.x;
    if (j < n)
        for (int i = 0; i < n; i++) packed[i * LD + j] = D[i][j];
}

// the full matrix of a packed block: zero outside the active rows and columns
__device__ void m_scatter(double2* full, const Mat& D, const StepLds& L)
{
    for (int e = threadIdx.x; e < LD * LD; e += 64) {
        const int pi = L.pos[e / LD], pj = L.pos[e % LD];
        full[e] = (pi >= 0 && pj >= 0) ? D[pi][pj] : cz();
    }
    __syncthreads();
}

__device__ void m_identity(Mat& D, int n)
{
    const int j = threadIdx.x;
    if (j < n)
        for (int i = 0; i < n; i++) D[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    __syncthreads();
}

// C = A B
__device__ void m_mul(Mat& C, const Mat& A, const Mat& B, int n)
{
    const int j = threadIdx.x;
    if (j < n)
        for (int i = 0; i < n; i++) {
            double2 s = cz();
            for (int k = 0; k < n; k++) cfma(s, A[i][k], B[k][j]);
            C[i][j] = s;
        }
    __syncthreads();
}

// C = A + B + d 1 (C may alias A or B)
__device__ void m_add_diag(Mat& C, const Mat& A, const Mat& B, double d, int n)
{
    const int j = threadIdx.x;
    if (j < n)
        for (int i = 0; i < n; i++) {
            double2 v = cadd(A[i][j], B[i][j]);
            if (i == j) v.x += d;
            C[i][j] = v;
        }
    __syncthreads();
}

// C = A + d 1 (C may alias A)
__device__ void m_shift(Mat& C, const Mat& A, double d, int n)
{
    const int j = threadIdx.x;
    if (j < n)
        for (int i = 0; i < n; i++) {
            double2 v = A[i][j];
            if (i == j) v.x += d;
            C[i][j] = v;
        }
    __syncthreads();
}

// C = A - B (C may alias A or B)
__device__ void m_sub(Mat& C, const Mat& A, const Mat& B, int n)
{
    const int j = threadIdx.x;
    if (j < n)
        for (int i = 0; i < n; i++) C[i][j] = csub(A[i][j], B[i][j]);
    __syncthreads();
}

// X = G^-1 B for Hermitian positive definite G (Cholesky G = L L^dag in W); X distinct from G, B, W
__device__ bool m_chol_solve(Mat& X, const Mat& G, const Mat& B, int n, Mat& W)
{
    const int j = threadIdx.x;
    if (j < n)
        for (int i = 0; i < n; i++) W[i][j] = G[i][j];
    __syncthreads();
    for (int k = 0; k < n; k++) {
        const double d = W[k][k].x;
        if (!(d > 0.0) || !isfinite(d)) return false;
        const double lk = sqrt(d);
        __syncthreads();
        if (j > k && j < n) W[j][k] = cscal(1.0 / lk, W[j][k]);
        if (j == k) W[k][k] = make_double2(lk, 0.0);
        __syncthreads();
        if (j > k && j < n) {
            const double2 ljk = cconj(W[j][k]);
            for (int i = j; i < n; i++) W[i][j] = csub(W[i][j], cmul(W[i][k], ljk));
        }
        __syncthreads();
    }
    if (j < n) {
        for (int i = 0; i < n; i++) {
            double2 y = B[i][j];
            for (int k = 0; k < i; k++) y = csub(y, cmul(W[i][k], X[k][j]));
            X[i][j] = cscal(1.0 / W[i][i].x, y);
        }
        for (int i = n - 1; i >= 0; i--) {
            double2 y = X[i][j];
            for (int k = i + 1; k < n; k++) y = csub(y, cmul(cconj(W[k][i]), X[k][j]));
            X[i][j] = cscal(1.0 / W[i][i].x, y);
        }
    }
    __syncthreads();
    return true;
}

// Y = A^-1 by Gauss-Jordan elimination with partial pivoting on [A | 1]
__device__ bool m_inv(Mat& Y, const Mat& A, int n, StepLds& L)
{
    const int j = threadIdx.x;
    const int m = 2 * n;
    if (j < m)
        for (int i = 0; i < n; i++) L.aug[i][j] = j < n ? A[i][j] : make_double2(j - n == i ? 1.0 : 0.0, 0.0);
    __syncthreads();
    for (int k = 0; k < n; k++) {
        int p = k;
        double best = cabs2(L.aug[k][k]);
        for (int i = k + 1; i < n; i++) {
            const double v = cabs2(L.aug[i][k]);
            if (v > best) {
                best = v;
                p = i;
            }
        }
        if (!(best > 0.0) || !isfinite(best)) return false;
        __syncthreads();
        if (p != k && j < m) {
            const double2 t = L.aug[k][j];
            L.aug[k][j] = L.aug[p][j];
            L.aug[p][j] = t;
        }
        __syncthreads();
        const double2 piv = L.aug[k][k];
        if (j < n) L.fac[j] = L.aug[j][k];
        __syncthreads();
        if (j < m) {
            const double2 pk = cdiv(L.aug[k][j], piv);
            for (int i = 0; i < n; i++)
                if (i != k) L.aug[i][j] = csub(L.aug[i][j], cmul(L.fac[i], pk));
            L.aug[k][j] = pk;
        }
        __syncthreads();
    }
    if (j < n)
        for (int i = 0; i < n; i++) Y[i][j] = L.aug[i][n + j];
    __syncthreads();
    return true;
}

__device__ void stop_run(const BlockState& S, bool breakdown)
{
    if (threadIdx.x == 0) {
        S.ctrl[BC_STOP] = 1;
        if (breakdown) S.ctrl[BC_BREAK] = 1;
    }
    // the stencils skip every column from here on
    for (int c = threadIdx.x; c < S.ncol; c += 64)
        if (S.colstat[c] == COL_ACTIVE) S.colstat[c] = COL_DONE;
}

// the active list of the run into LDS (idx: packed position -> column, pos: column -> position)
__device__ void load_active(const BlockState& S, StepLds& L, int& n)
{
    n = S.ctrl[BC_NA];
    if (threadIdx.x < LD) {
        L.idx[threadIdx.x] = threadIdx.x < n ? S.ctrl[BC_IDX + threadIdx.x] : -1;
        L.pos[threadIdx.x] = -1;
    }
    __syncthreads();
    if (threadIdx.x < n) L.pos[L.idx[threadIdx.x]] = threadIdx.x;
    __syncthreads();
}

// Start of a run: the candidates are the columns with colstat COL_ACTIVE and BM_RR holds their
// Gram matrix.  A Cholesky pass in column order keeps a column only if its pivot stays above
// 1e-12 of its diagonal entry (numerically independent of the kept ones before it); the others
// leave the run.
__device__ void step_start(const BlockState& S, StepLds& L)
{
    if (threadIdx.x == 0) {
        const double2* G = mat(S, BM_RR);
        int cand[LD], nc = 0;
        for (int c = 0; c < S.ncol; c++)
            if (S.colstat[c] == COL_ACTIVE) cand[nc++] = c;
        // lower factor of the kept columns, in L.a (rows and columns by candidate number)
        int keep[LD];
        unsigned mask = 0;
        int na = 0;
        for (int k = 0; k < nc; k++) {
            const double g = G[cand[k] * LD + cand[k]].x;
            double d = g;
            for (int q = 0; q < k; q++)
                if (keep[q]) d -= cabs2(L.a[k][q]);
            keep[k] = isfinite(g) && g > 0.0 && d > 1e-12 * g;
            if (!keep[k]) {
                S.colstat[cand[k]] = COL_DONE;
                continue;
            }
            const double lk = sqrt(d);
            L.a[k][k] = make_double2(lk, 0.0);
            for (int i = k + 1; i < nc; i++) {
                double2 v = G[cand[i] * LD + cand[k]];
                for (int q = 0; q < k; q++)
                    if (keep[q]) v = csub(v, cmul(L.a[i][q], cconj(L.a[k][q])));
                L.a[i][k] = cscal(1.0 / lk, v);
            }
            L.idx[na] = cand[k];
            S.ctrl[BC_IDX + na++] = cand[k];
            mask |= 1u << cand[k];
        }
        L.fac[0].x = na;  // handed to the other lanes through LDS
        S.ctrl[BC_NA] = na;
        S.ctrl[BC_MASK] = (int)mask;
        S.ctrl[BC_K] = 0;
        S.ctrl[BC_BREAK] = 0;
        S.ctrl[BC_STOP] = na == 0;
        for (int s = 0; s < S.nshift; s++) {
            S.ctrl[BC_FROZEN + s] = 0;
            for (int c = 0; c < S.ncol; c++)
                if (on(mask, c)) {
                    S.sstat[s * S.ncol + c] = 0;
                    S.siters[s * S.ncol + c] = 0;
                }
        }
    }
    __syncthreads();
    const int n = (int)L.fac[0].x;
    m_identity(L.b, n);
    for (int s = 0; s < S.nshift; s++)
        if (s != S.base) m_store(mat(S, BM_SHIFT + 6 * s), L.b, n);
}

// After BM_PQ: alpha_k, and for every shift still iterating alpha^s_k, beta^s_k-1, xi_k+1.
__device__ void step_alpha(const BlockState& S, StepLds& L)
{
    int n;
    load_active(S, L, n);
    const int k = S.ctrl[BC_K];
    m_gather(L.a, mat(S, BM_PQ), L, n);
    m_gather(L.b, mat(S, BM_RR), L, n);
    bool ok = m_chol_solve(L.c, L.a, L.b, n, L.d);  // alpha in L.c
    if (!ok) {
        stop_run(S, true);
        return;
    }
    m_scatter(mat(S, BM_ALPHA), L.c, L);
    if (S.nshift == 1) return;
    ok = m_inv(L.a, L.c, n, L);  // alpha^-1 in L.a
    if (!ok) {
        stop_run(S, true);
        return;
    }
    m_store(mat(S, BM_AINV), L.a, n);
    for (int s = 0; s < S.nshift; s++) {
        if (s == S.base || S.ctrl[BC_FROZEN + s]) continue;
        double2* sm = mat(S, BM_SHIFT + 6 * s);
        const double d = S.shift[s];
        m_load(L.b, sm, n);  // xi_k
        if (k == 0) {
            // alpha^s_0 = (alpha_0^-1 + d)^-1, beta^s_-1 = 0
            m_shift(L.c, L.a, d, n);  // alpha_0^-1 + d
            ok = m_inv(L.d, L.c, n, L);
            if (!ok) break;
            const int j = threadIdx.x;
            if (j < n)
                for (int i = 0; i < n; i++) L.e[i][j] = cz();
            __syncthreads();
        } else {
            // with C = alpha_k-1^-1 beta_k-1 and T = xi_k-1^-1 C xi_k:
            // (alpha^s_k)^-1 = xi_k^-1 (alpha_k^-1 + C + d) xi_k - T,  beta^s_k-1 = alpha^s_k-1 T
            m_load(L.g, mat(S, BM_C), n);
            m_load(L.c, sm + 1 * LD * LD, n);  // xi_k-1
            ok = m_inv(L.d, L.c, n, L);        // xi_k-1^-1
            if (!ok) break;
            m_mul(L.c, L.d, L.g, n);
            m_mul(L.f, L.c, L.b, n);           // T
            m_add_diag(L.c, L.a, L.g, d, n);   // alpha_k^-1 + C + d
            m_mul(L.d, L.c, L.b, n);
            ok = m_inv(L.c, L.b, n, L);        // xi_k^-1
            if (!ok) break;
            m_mul(L.e, L.c, L.d, n);
            m_sub(L.c, L.e, L.f, n);           // (alpha^s_k)^-1
            ok = m_inv(L.d, L.c, n, L);        // alpha^s_k
            if (!ok) break;
            m_load(L.c, sm + 2 * LD * LD, n);  // alpha^s_k-1
            m_mul(L.e, L.c, L.f, n);           // beta^s_k-1
        }
        // kernel-facing full matrices: xi_k, alpha^s_k, beta^s_k-1
        m_scatter(sm + 3 * LD * LD, L.b, L);
        m_scatter(sm + 4 * LD * LD, L.d, L);
        m_scatter(sm + 5 * LD * LD, L.e, L);
        // xi_k+1 = alpha_k^-1 xi_k alpha^s_k; keep xi_k and alpha^s_k for the next step
        m_mul(L.c, L.a, L.b, n);
        m_mul(L.e, L.c, L.d, n);
        m_store(sm + 1 * LD * LD, L.b, n);
        m_store(sm + 2 * LD * LD, L.d, n);
        m_store(sm, L.e, n);
        __syncthreads();
    }
    if (!ok) stop_run(S, true);
}

// After BM_RRN: per shift and column |R xi e_c|^2 against (tol |b_c|)^2, then beta_k.
__device__ void step_beta(const BlockState& S, StepLds& L)
{
    int n;
    load_active(S, L, n);
    const int k = S.ctrl[BC_K];
    m_gather(L.a, mat(S, BM_RRN), L, n);
    __shared__ int all_done, bad;
    if (threadIdx.x == 0) {
        all_done = 1;
        bad = 0;
    }
    __syncthreads();
    for (int s = 0; s < S.nshift; s++) {
        const bool base = s == S.base;
        if (!base && S.ctrl[BC_FROZEN + s]) continue;
        if (!base) m_load(L.b, mat(S, BM_SHIFT + 6 * s), n);  // xi_k+1
        __shared__ int conv;
        if (threadIdx.x == 0) conv = 1;
        __syncthreads();
        const int a = threadIdx.x;
        if (a < n) {
            double r2;
            if (base) {
                r2 = L.a[a][a].x;
            } else {
                double2 acc = cz();
                for (int p = 0; p < n; p++) {
                    double2 t = cz();
                    for (int q = 0; q < n; q++) cfma(t, L.a[p][q], L.b[q][a]);
                    cfmac(acc, L.b[p][a], t);
                }
                r2 = acc.x;
            }
            const int c = L.idx[a];
            const int e = s * S.ncol + c;
            if (!isfinite(r2)) atomicOr(&bad, 1);
            if (S.sstat[e] == 0 && r2 <= S.thr[c]) {
                S.sstat[e] = 1;
                S.siters[e] = k + 1;
            }
            if (S.sstat[e] == 0) atomicAnd(&conv, 0);
        }
        __syncthreads();
        if (!conv) atomicAnd(&all_done, 0);
        if (!base && conv && threadIdx.x == 0) S.ctrl[BC_FROZEN + s] = 1;
        __syncthreads();
    }
    if (threadIdx.x == 0) S.ctrl[BC_K] = k + 1;
    if (bad || all_done) {
        stop_run(S, bad != 0);
        return;
    }
    m_gather(L.b, mat(S, BM_RR), L, n);
    if (!m_chol_solve(L.c, L.b, L.a, n, L.d)) {  // beta in L.c
        stop_run(S, true);
        return;
    }
    m_scatter(mat(S, BM_BETA), L.c, L);
    if (S.nshift > 1) {
        m_load(L.b, mat(S, BM_AINV), n);
        m_mul(L.d, L.b, L.c, n);
        m_store(mat(S, BM_C), L.d, n);
    }
    // R^dag R of the new residual becomes the current one
    for (int e = threadIdx.x; e < LD * LD; e += 64) mat(S, BM_RR)[e] = mat(S, BM_RRN)[e];
}

__global__ __launch_bounds__(64) void k_block_step(BlockState S, int phase)
{
    __shared__ StepLds L;
    if (phase == 0) {
        step_start(S, L);
        return;
    }
    if (S.ctrl[BC_STOP]) return;
    if (phase == 1)
        step_alpha(S, L);
    else
        step_beta(S, L);
}

// --------------------------------------------------------------------------
// column combinations (one thread per unit = site and spin-colour component)
// --------------------------------------------------------------------------

template <int NM>
__global__ __launch_bounds__(256) void k_block_xr(BlockState S, FieldArg X, FieldArg P, FieldArg W, FieldArg R,
                                                  size_t units)
{
    if (S.ctrl[BC_STOP]) return;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= units) return;
    const unsigned mask = (unsigned)S.ctrl[BC_MASK];
    const double2* A = mat(S, BM_ALPHA);
    const double2* pp = (const double2*)P.d;
    const double2* wp = (const double2*)W.d;
    double2* xp = (double2*)X.d;
    double2* rp = (double2*)R.d;
    double2 p[NM], w[NM];
#pragma unroll
    for (int i = 0; i < NM; i++) {
        p[i] = cz();
        w[i] = cz();
        if (i < S.ncol && on(mask, i)) {
            p[i] = pp[(size_t)i * P.cstride + t];
            const double2 v = wp[(size_t)i * W.cstride + t];
            w[i] = make_double2(fma(S.sigma_b, p[i].x, v.x), fma(S.sigma_b, p[i].y, v.y));
        }
    }
#pragma unroll
    for (int m = 0; m < NM; m++) {
        if (m >= S.ncol || !on(mask, m)) continue;
        double2 dx = cz(), dr = cz();
#pragma unroll
        for (int i = 0; i < NM; i++) {
            if (i >= S.ncol || !on(mask, i)) continue;
            const double2 a = A[i * LD + m];
            cfma(dx, p[i], a);
            cfma(dr, w[i], a);
        }
        double2& xr = xp[(size_t)m * X.cstride + t];
        double2& rr = rp[(size_t)m * R.cstride + t];
        xr = cadd(xr, dx);
        rr = csub(rr, dr);
    }
}

template <int NM>
__global__ __launch_bounds__(256) void k_block_p(BlockState S, FieldArg P, FieldArg R, size_t units)
{
    if (S.ctrl[BC_STOP]) return;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= units) return;
    const unsigned mask = (unsigned)S.ctrl[BC_MASK];
    const double2* B = mat(S, BM_BETA);
    double2* pp = (double2*)P.d;
    const double2* rp = (const double2*)R.d;
    double2 p[NM];
#pragma unroll
    for (int i = 0; i < NM; i++) p[i] = (i < S.ncol && on(mask, i)) ? pp[(size_t)i * P.cstride + t] : cz();
#pragma unroll
    for (int m = 0; m < NM; m++) {
        if (m >= S.ncol || !on(mask, m)) continue;
        double2 v = rp[(size_t)m * R.cstride + t];
#pragma unroll
        for (int i = 0; i < NM; i++)
            if (i < S.ncol && on(mask, i)) cfma(v, p[i], B[i * LD + m]);
        pp[(size_t)m * P.cstride + t] = v;
    }
}

template <int NM>
__global__ __launch_bounds__(256) void k_block_shift(BlockState S, BlockFields f, FieldArg R, size_t units)
{
    const int s = blockIdx.y;
    if (S.ctrl[BC_STOP] || s == S.base || S.ctrl[BC_FROZEN + s]) return;
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= units) return;
    const unsigned mask = (unsigned)S.ctrl[BC_MASK];
    const double2* sm = mat(S, BM_SHIFT + 6 * s);
    const double2* Xi = sm + 3 * LD * LD;
    const double2* As = sm + 4 * LD * LD;
    const double2* Bs = sm + 5 * LD * LD;
    const double2* rp = (const double2*)R.d;
    double2* pp = (double2*)f.p[s].d;
    double2* xp = (double2*)f.x[s].d;
    const size_t pc = f.p[s].cstride, xc = f.x[s].cstride;
    double2 r[NM], p[NM], pn[NM];
#pragma unroll
    for (int i = 0; i < NM; i++) {
        const bool a = i < S.ncol && on(mask, i);
        r[i] = a ? rp[(size_t)i * R.cstride + t] : cz();
        p[i] = a ? pp[(size_t)i * pc + t] : cz();
    }
#pragma unroll
    for (int m = 0; m < NM; m++) {
        pn[m] = cz();
        if (m >= S.ncol || !on(mask, m)) continue;
        double2 v = cz();
#pragma unroll
        for (int i = 0; i < NM; i++) {
            if (i >= S.ncol || !on(mask, i)) continue;
            cfma(v, r[i], Xi[i * LD + m]);
            cfma(v, p[i], Bs[i * LD + m]);
        }
        pn[m] = v;
        pp[(size_t)m * pc + t] = v;
    }
#pragma unroll
    for (int m = 0; m < NM; m++) {
        if (m >= S.ncol || !on(mask, m)) continue;
        double2 v = xp[(size_t)m * xc + t];
#pragma unroll
        for (int i = 0; i < NM; i++)
            if (i < S.ncol && on(mask, i)) cfma(v, pn[i], As[i * LD + m]);
        xp[(size_t)m * xc + t] = v;
    }
}

inline dim3 unit_grid(size_t units, int y = 1) { return dim3((unsigned)((units + 255) / 256), y); }

}  // namespace

hipError_t launch_block_gram(FieldArg X, FieldArg Y, FieldArg Z, double s, const BlockState& S, int vh, int tiles,
                             double2* partial, hipStream_t st)
{
    if (S.ncol < 1 || S.ncol > kBlockMax) return hipErrorInvalidValue;
    const int ngroups = (tiles + kGramTiles - 1) / kGramTiles;
    const int nb = (S.ncol + 3) / 4;
    hipLaunchKernelGGL(k_block_gram, dim3((ngroups + 3) / 4, nb * nb), dim3(256), 0, st, X, Y, Z, s, S, vh, tiles,
                       partial);
    return hipGetLastError();
}

hipError_t launch_block_gram_fin(const BlockState& S, const double2* partial, int tiles, int slot, hipStream_t st)
{
    if (S.ncol < 1 || S.ncol > kBlockMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_block_gram_fin, dim3(S.ncol * S.ncol), dim3(256), 0, st, S, partial, tiles, slot);
    return hipGetLastError();
}

hipError_t launch_block_step(const BlockState& S, int phase, hipStream_t st)
{
    if (S.ncol < 1 || S.ncol > kBlockMax || S.nshift < 1 || S.nshift > kMaxShifts) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_block_step, dim3(1), dim3(64), 0, st, S, phase);
    return hipGetLastError();
}

#define BQ_BLOCK_DISPATCH(KERNEL, GRID, ...)                                                                     \
    switch ((S.ncol + 3) / 4) {                                                                                 \
    case 1: hipLaunchKernelGGL(KERNEL<4>, GRID, dim3(256), 0, st, __VA_ARGS__); break;                          \
    case 2: hipLaunchKernelGGL(KERNEL<8>, GRID, dim3(256), 0, st, __VA_ARGS__); break;                          \
    case 3: hipLaunchKernelGGL(KERNEL<12>, GRID, dim3(256), 0, st, __VA_ARGS__); break;                         \
    case 4: hipLaunchKernelGGL(KERNEL<16>, GRID, dim3(256), 0, st, __VA_ARGS__); break;                         \
    default: return hipErrorInvalidValue;                                                                       \
    }

hipError_t launch_block_xr(const BlockState& S, FieldArg x, FieldArg p, FieldArg w, FieldArg r, size_t units,
                           hipStream_t st)
{
    BQ_BLOCK_DISPATCH(k_block_xr, unit_grid(units), S, x, p, w, r, units)
    return hipGetLastError();
}

hipError_t launch_block_p(const BlockState& S, FieldArg p, FieldArg r, size_t units, hipStream_t st)
{
    BQ_BLOCK_DISPATCH(k_block_p, unit_grid(units), S, p, r, units)
    return hipGetLastError();
}

hipError_t launch_block_shift(const BlockState& S, const BlockFields& f, FieldArg r, size_t units, hipStream_t st)
{
    if (S.nshift < 1 || S.nshift > kMaxShifts) return hipErrorInvalidValue;
    BQ_BLOCK_DISPATCH(k_block_shift, unit_grid(units, S.nshift), S, f, r, units)
    return hipGetLastError();
}

}  // namespace bq
