/*
 * bq_oracle.c -- plain, slow FP64 CPU oracle for the even-odd preconditioned
 * Wilson-clover fermion matrix with chemical potential and CG on M^dag M.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or generator with the HIP library; the product never calls it.
 *
 * Everything here is the definition written out, on the full lattice:
 *   - array of structures, lexicographic sites i = x1 + L1*(x2 + L2*(x3 + L3*x4));
 *   - spinor psi[(i*4 + s)*3 + c], link U[((mu*V + i)*3 + a)*3 + b] (double complex);
 *   - clover T(x) kept as a dense 12x12 matrix per site, index s*3 + c;
 *   - gamma matrices kept as dense 4x4 matrices, projectors applied as matrices.
 * No spin projection, no packing, no blocking, no even-odd storage.
 *
 * Readings of points the paper leaves open (all stated once here):
 *   - Euclidean chiral basis, gamma_5 = diag(1,1,-1,-1);
 *   - sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu];
 *   - F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dag)/8 from the four-leaf clover,
 *     made traceless; the Hermitian field strength is -i F;
 *   - clover term of Eq. 2 summed over ordered pairs mu,nu, so that
 *     T = 1 + kappa c_SW sum_{mu<nu} sigma_{mu nu} (x) (-i F_{mu nu});
 *   - real chemical potential: forward time hops carry e^{+mu}, backward e^{-mu}
 *     (Eq. 1); periodic space, time boundary sign t_bc (-1 = antiperiodic);
 *   - even sites have (x1+x2+x3+x4) even; the Schur system lives on odd sites:
 *     Mhat = T_oo - kappa^2 D_oe T_ee^{-1} D_eo.
 * Parity unpinned relative to the paper: the paper prints no operator value or
 * worked example, so the basis, the trace subtraction, the sign of the clover
 * term, the even-odd form, the noise convention and the link generator are
 * pinned only as the definitions stated above.  Every function below is pinned
 * by the CPU tests against closed forms, invariants, brute force or dense
 * linear algebra.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define NSC 12 /* spin x colour components per site */

/* ------------------------------------------------------------------ */
/* Dirac algebra                                                       */
/* ------------------------------------------------------------------ */

static cplx GAM[4][4][4];       /* gamma_mu, mu = 0..3 for x,y,z,t */
static cplx SIG[4][4][4][4];    /* sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] */
static int algebra_ready = 0;

static void init_algebra(void)
{
    if (algebra_ready) return;
    memset(GAM, 0, sizeof(GAM));
    /* gamma_1 */
    GAM[0][0][3] = I;  GAM[0][1][2] = I;  GAM[0][2][1] = -I; GAM[0][3][0] = -I;
    /* gamma_2 */
    GAM[1][0][3] = -1; GAM[1][1][2] = 1;  GAM[1][2][1] = 1;  GAM[1][3][0] = -1;
    /* gamma_3 */
    GAM[2][0][2] = I;  GAM[2][1][3] = -I; GAM[2][2][0] = -I; GAM[2][3][1] = I;
    /* gamma_4 */
    GAM[3][0][2] = 1;  GAM[3][1][3] = 1;  GAM[3][2][0] = 1;  GAM[3][3][1] = 1;
    for (int mu = 0; mu < 4; mu++)
        for (int nu = 0; nu < 4; nu++)
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    cplx comm = 0;
                    for (int k = 0; k < 4; k++)
                        comm += GAM[mu][a][k] * GAM[nu][k][b] - GAM[nu][a][k] * GAM[mu][k][b];
                    SIG[mu][nu][a][b] = 0.5 * I * comm;
                }
    algebra_ready = 1;
}

/* Build the tables once at load time so that no parallel region initialises them. */
__attribute__((constructor)) static void oracle_load(void) { init_algebra(); }

/* ------------------------------------------------------------------ */
/* Geometry                                                            */
/* ------------------------------------------------------------------ */

static long vol(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void site_coords(const int L[4], long i, int x[4])
{
    for (int mu = 0; mu < 4; mu++) { x[mu] = (int)(i % L[mu]); i /= L[mu]; }
}

static long site_index(const int L[4], const int x[4])
{
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

/* neighbour x + step*mu_hat with periodic wrap (step = +1 or -1) */
static long neighbour(const int L[4], long i, int mu, int step)
{
    int x[4];
    site_coords(L, i, x);
    x[mu] = (x[mu] + step + L[mu]) % L[mu];
    return site_index(L, x);
}

static int parity_of(const int L[4], long i)
{
    int x[4];
    site_coords(L, i, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

/* Hop coefficients of Eq. 1 at site x:
 * fwd(x, mu): multiplies U_mu(x)(1-gamma_mu) psi(x+mu);
 * bwd(x, mu): multiplies U_mu(x-mu)^dag (1+gamma_mu) psi(x-mu).
 * Time hops carry e^{+-mu_ch}; a hop that crosses the time boundary carries t_bc. */
static cplx coef_fwd(const int L[4], long i, int mu, int t_bc, double mu_ch)
{
    if (mu != 3) return 1.0;
    int x[4];
    site_coords(L, i, x);
    return exp(mu_ch) * (x[3] == L[3] - 1 ? (double)t_bc : 1.0);
}

static cplx coef_bwd(const int L[4], long i, int mu, int t_bc, double mu_ch)
{
    if (mu != 3) return 1.0;
    int x[4];
    site_coords(L, i, x);
    return exp(-mu_ch) * (x[3] == 0 ? (double)t_bc : 1.0);
}

/* ------------------------------------------------------------------ */
/* Small dense helpers                                                 */
/* ------------------------------------------------------------------ */

static const cplx *link(const cplx *U, long V, int mu, long i) { return U + ((long)mu * V + i) * 9; }

/* out[s][a] += coef * sum_{s',b} W[a][b](^dag) (1 + sgn*gamma_mu)[s][s'] in[s'][b] */
static void add_hop_term(cplx *out, const cplx *W, int W_dag, int mu, double sgn, cplx coef, const cplx *in)
{
    cplx proj[4][3];
    for (int s = 0; s < 4; s++)
        for (int c = 0; c < 3; c++) {
            cplx acc = in[s * 3 + c];
            for (int t = 0; t < 4; t++) acc += sgn * GAM[mu][s][t] * in[t * 3 + c];
            proj[s][c] = acc;
        }
    for (int s = 0; s < 4; s++)
        for (int a = 0; a < 3; a++) {
            cplx acc = 0;
            for (int b = 0; b < 3; b++) {
                cplx w = W_dag ? conj(W[b * 3 + a]) : W[a * 3 + b];
                acc += w * proj[s][b];
            }
            out[s * 3 + a] += coef * acc;
        }
}

/* y = A x (adj = 0) or A^dag x (adj = 1) for a dense 12x12 A */
static void mat12_apply(const cplx *A, int adj, const cplx *x, cplx *y)
{
    for (int r = 0; r < NSC; r++) {
        cplx acc = 0;
        for (int k = 0; k < NSC; k++) acc += (adj ? conj(A[k * NSC + r]) : A[r * NSC + k]) * x[k];
        y[r] = acc;
    }
}

/* 3x3 complex products */
static void m3_mul(const cplx *A, const cplx *B, cplx *C)
{
    cplx t[9];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            cplx acc = 0;
            for (int k = 0; k < 3; k++) acc += A[a * 3 + k] * B[k * 3 + b];
            t[a * 3 + b] = acc;
        }
    memcpy(C, t, sizeof(t));
}

static void m3_dag(const cplx *A, cplx *B)
{
    cplx t[9];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) t[a * 3 + b] = conj(A[b * 3 + a]);
    memcpy(B, t, sizeof(t));
}

/* ------------------------------------------------------------------ */
/* Hopping term D (Eq. 1) and its adjoint                               */
/* ------------------------------------------------------------------ */

/* (D psi)(x) at one site, or (D^dag psi)(x) when dagger != 0, with the neighbour
 * values given explicitly: nb[mu][0] = psi(x+mu), nb[mu][1] = psi(x-mu).
 *   D psi(x)     = sum_mu fwd(x) U_mu(x)(1-g_mu)psi(x+mu) + bwd(x) U_mu(x-mu)^dag (1+g_mu) psi(x-mu)
 *   D^dag psi(x) = sum_mu conj(bwd(x+mu)) U_mu(x)(1+g_mu)psi(x+mu)
 *                       + conj(fwd(x-mu)) U_mu(x-mu)^dag (1-g_mu) psi(x-mu)
 * The adjoint is written out as the conjugate transpose of each matrix element
 * D^dag(x,y) = D(y,x)^dag, not as gamma_5 D gamma_5. */
static void hop_site_nb(const int L[4], const cplx *U, int t_bc, double mu_ch, int dagger, long i,
                        const cplx *const nb[4][2], cplx *out12)
{
    init_algebra();
    long V = vol(L);
    for (int k = 0; k < NSC; k++) out12[k] = 0;
    for (int mu = 0; mu < 4; mu++) {
        long f = neighbour(L, i, mu, +1);
        long b = neighbour(L, i, mu, -1);
        if (!dagger) {
            add_hop_term(out12, link(U, V, mu, i), 0, mu, -1.0, coef_fwd(L, i, mu, t_bc, mu_ch), nb[mu][0]);
            add_hop_term(out12, link(U, V, mu, b), 1, mu, +1.0, coef_bwd(L, i, mu, t_bc, mu_ch), nb[mu][1]);
        } else {
            add_hop_term(out12, link(U, V, mu, i), 0, mu, +1.0, conj(coef_bwd(L, f, mu, t_bc, mu_ch)), nb[mu][0]);
            add_hop_term(out12, link(U, V, mu, b), 1, mu, -1.0, conj(coef_fwd(L, b, mu, t_bc, mu_ch)), nb[mu][1]);
        }
    }
}

void or_hop_site(const int L[4], const cplx *U, int t_bc, double mu_ch, int dagger,
                 const cplx *in, long i, cplx *out12)
{
    const cplx *nb[4][2];
    for (int mu = 0; mu < 4; mu++) {
        nb[mu][0] = in + neighbour(L, i, mu, +1) * NSC;
        nb[mu][1] = in + neighbour(L, i, mu, -1) * NSC;
    }
    hop_site_nb(L, U, t_bc, mu_ch, dagger, i, nb, out12);
}

void or_hop(const int L[4], const cplx *U, int t_bc, double mu_ch, int dagger, const cplx *in, cplx *out)
{
    init_algebra();
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) or_hop_site(L, U, t_bc, mu_ch, dagger, in, i, out + i * NSC);
}

/* ------------------------------------------------------------------ */
/* Clover term (Eq. 2)                                                 */
/* ------------------------------------------------------------------ */

/* Four-leaf clover Q_{mu nu}(x): the four plaquettes in the mu-nu plane that
 * touch x, each traversed counter-clockwise (mu then nu) starting at x. */
static void clover_leaves(const int L[4], const cplx *U, long i, int mu, int nu, cplx *Q)
{
    long V = vol(L);
    long xpm = neighbour(L, i, mu, +1), xpn = neighbour(L, i, nu, +1);
    long xmm = neighbour(L, i, mu, -1), xmn = neighbour(L, i, nu, -1);
    long xpn_mm = neighbour(L, xpn, mu, -1);
    long xmm_mn = neighbour(L, xmm, nu, -1);
    long xmn_pm = neighbour(L, xmn, mu, +1);
    cplx A[9], B[9], P[9];
    for (int k = 0; k < 9; k++) Q[k] = 0;

    /* U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
    m3_mul(link(U, V, mu, i), link(U, V, nu, xpm), P);
    m3_dag(link(U, V, mu, xpn), A); m3_mul(P, A, P);
    m3_dag(link(U, V, nu, i), A);   m3_mul(P, A, P);
    for (int k = 0; k < 9; k++) Q[k] += P[k];

    /* U_nu(x) U_mu(x+nu-mu)^dag U_nu(x-mu)^dag U_mu(x-mu) */
    m3_dag(link(U, V, mu, xpn_mm), A); m3_mul(link(U, V, nu, i), A, P);
    m3_dag(link(U, V, nu, xmm), A);    m3_mul(P, A, P);
    m3_mul(P, link(U, V, mu, xmm), P);
    for (int k = 0; k < 9; k++) Q[k] += P[k];

    /* U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu) */
    m3_dag(link(U, V, mu, xmm), A); m3_dag(link(U, V, nu, xmm_mn), B); m3_mul(A, B, P);
    m3_mul(P, link(U, V, mu, xmm_mn), P);
    m3_mul(P, link(U, V, nu, xmn), P);
    for (int k = 0; k < 9; k++) Q[k] += P[k];

    /* U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^dag */
    m3_dag(link(U, V, nu, xmn), A); m3_mul(A, link(U, V, mu, xmn), P);
    m3_mul(P, link(U, V, nu, xmn_pm), P);
    m3_dag(link(U, V, mu, i), A);   m3_mul(P, A, P);
    for (int k = 0; k < 9; k++) Q[k] += P[k];
}

/* Hermitian traceless field strength Fh_{mu nu}(x) = -i (Q - Q^dag)/8, trace removed. */
void or_field_strength_site(const int L[4], const cplx *U, long i, int mu, int nu, cplx *Fh)
{
    cplx Q[9];
    clover_leaves(L, U, i, mu, nu, Q);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) Fh[a * 3 + b] = -I * (Q[a * 3 + b] - conj(Q[b * 3 + a])) / 8.0;
    cplx tr = (Fh[0] + Fh[4] + Fh[8]) / 3.0;
    Fh[0] -= tr; Fh[4] -= tr; Fh[8] -= tr;
}

/* T(x) = 1 + kappa c_SW sum_{mu<nu} sigma_{mu nu} (x) Fh_{mu nu}(x), dense 12x12. */
void or_clover_site(const int L[4], const cplx *U, double kappa, double csw, long i, cplx *T)
{
    init_algebra();
    for (int k = 0; k < NSC * NSC; k++) T[k] = 0;
    for (int k = 0; k < NSC; k++) T[k * NSC + k] = 1.0;
    for (int mu = 0; mu < 4; mu++)
        for (int nu = mu + 1; nu < 4; nu++) {
            cplx Fh[9];
            or_field_strength_site(L, U, i, mu, nu, Fh);
            for (int s = 0; s < 4; s++)
                for (int a = 0; a < 3; a++)
                    for (int t = 0; t < 4; t++)
                        for (int b = 0; b < 3; b++)
                            T[(s * 3 + a) * NSC + t * 3 + b] += kappa * csw * SIG[mu][nu][s][t] * Fh[a * 3 + b];
        }
}

void or_clover(const int L[4], const cplx *U, double kappa, double csw, cplx *T)
{
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) or_clover_site(L, U, kappa, csw, i, T + i * NSC * NSC);
}

/* Dense inverse by Gauss-Jordan elimination with partial pivoting.  Returns 0, or -1 if singular. */
int or_invert12(const cplx *A, cplx *Ainv)
{
    cplx M[NSC][2 * NSC];
    for (int r = 0; r < NSC; r++)
        for (int c = 0; c < NSC; c++) {
            M[r][c] = A[r * NSC + c];
            M[r][NSC + c] = (r == c) ? 1.0 : 0.0;
        }
    for (int col = 0; col < NSC; col++) {
        int piv = col;
        for (int r = col + 1; r < NSC; r++)
            if (cabs(M[r][col]) > cabs(M[piv][col])) piv = r;
        if (cabs(M[piv][col]) == 0.0) return -1;
        if (piv != col)
            for (int c = 0; c < 2 * NSC; c++) { cplx t = M[col][c]; M[col][c] = M[piv][c]; M[piv][c] = t; }
        cplx d = M[col][col];
        for (int c = 0; c < 2 * NSC; c++) M[col][c] /= d;
        for (int r = 0; r < NSC; r++) {
            if (r == col) continue;
            cplx f = M[r][col];
            if (f == 0) continue;
            for (int c = 0; c < 2 * NSC; c++) M[r][c] -= f * M[col][c];
        }
    }
    for (int r = 0; r < NSC; r++)
        for (int c = 0; c < NSC; c++) Ainv[r * NSC + c] = M[r][NSC + c];
    return 0;
}

int or_clover_invert(const int L[4], const cplx *T, cplx *Tinv)
{
    long V = vol(L);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long i = 0; i < V; i++)
        if (or_invert12(T + i * NSC * NSC, Tinv + i * NSC * NSC)) bad = 1;
    return bad ? -1 : 0;
}

/* out = T in (adj = 0) or T^dag in (adj = 1), site by site; parity_mask: bit p set = apply on parity p, others zeroed */
void or_clover_apply(const int L[4], const cplx *T, int adj, int parity_mask, const cplx *in, cplx *out)
{
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        if ((parity_mask >> parity_of(L, i)) & 1)
            mat12_apply(T + i * NSC * NSC, adj, in + i * NSC, out + i * NSC);
        else
            for (int k = 0; k < NSC; k++) out[i * NSC + k] = 0;
    }
}

/* ------------------------------------------------------------------ */
/* Full fermion matrix M = T - kappa D and its adjoint                  */
/* ------------------------------------------------------------------ */

void or_M_site(const int L[4], const cplx *U, const cplx *T, double kappa, int t_bc, double mu_ch,
               int dagger, const cplx *in, long i, cplx *out12)
{
    cplx h[NSC], t[NSC];
    or_hop_site(L, U, t_bc, mu_ch, dagger, in, i, h);
    mat12_apply(T + i * NSC * NSC, dagger, in + i * NSC, t);
    for (int k = 0; k < NSC; k++) out12[k] = t[k] - kappa * h[k];
}

void or_apply_M(const int L[4], const cplx *U, const cplx *T, double kappa, int t_bc, double mu_ch,
                int dagger, const cplx *in, cplx *out)
{
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) or_M_site(L, U, T, kappa, t_bc, mu_ch, dagger, in, i, out + i * NSC);
}

/* ------------------------------------------------------------------ */
/* Even-odd Schur complement on odd sites                               */
/* ------------------------------------------------------------------ */

/* zero every site whose parity is not p */
static void keep_parity(const int L[4], int p, cplx *v)
{
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++)
        if (parity_of(L, i) != p)
            for (int k = 0; k < NSC; k++) v[i * NSC + k] = 0;
}

/* Mhat v = T_oo v_o - kappa^2 D_oe T_ee^{-1} D_eo v_o             (dagger = 0)
 * Mhat^dag v = T_oo^dag v_o - kappa^2 (D^dag)_oe T_ee^{-dag} (D^dag)_eo v_o (dagger = 1)
 * in/out are full-lattice arrays; only odd sites of `in` are read, even sites of `out` are 0.
 * work: two full-lattice scratch arrays (2*V*12). */
void or_apply_Mhat(const int L[4], const cplx *U, const cplx *T, const cplx *Tinv, double kappa,
                   int t_bc, double mu_ch, int dagger, const cplx *in, cplx *out, cplx *work)
{
    long V = vol(L);
    cplx *a = work, *b = work + V * NSC;
    memcpy(b, in, sizeof(cplx) * V * NSC);
    keep_parity(L, 1, b);                          /* v_o */
    or_hop(L, U, t_bc, mu_ch, dagger, b, a);       /* D v_o */
    keep_parity(L, 0, a);                          /* (D)_eo v_o on even sites */
    or_clover_apply(L, Tinv, dagger, 1 << 0, a, out); /* T_ee^{-1}(^dag) on even sites */
    or_hop(L, U, t_bc, mu_ch, dagger, out, a);     /* D on the even field */
    or_clover_apply(L, T, dagger, 1 << 1, b, out); /* T_oo(^dag) v_o */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++)
        if (parity_of(L, i) == 1)
            for (int k = 0; k < NSC; k++) out[i * NSC + k] -= kappa * kappa * a[i * NSC + k];
}

/* bhat = b_o + kappa D_oe T_ee^{-1} b_e  (result on odd sites, even sites 0); work: 2*V*12 */
void or_eo_prepare(const int L[4], const cplx *U, const cplx *Tinv, double kappa, int t_bc, double mu_ch,
                   const cplx *b, cplx *bhat, cplx *work)
{
    long V = vol(L);
    cplx *a = work, *c = work + V * NSC;
    or_clover_apply(L, Tinv, 0, 1 << 0, b, a);     /* T_ee^{-1} b_e */
    or_hop(L, U, t_bc, mu_ch, 0, a, c);
    for (long i = 0; i < V; i++)
        for (int k = 0; k < NSC; k++)
            bhat[i * NSC + k] = parity_of(L, i) == 1 ? b[i * NSC + k] + kappa * c[i * NSC + k] : 0.0;
}

/* x_e = T_ee^{-1}(b_e + kappa D_eo x_o); x holds x_o on odd sites on entry, full x on exit. work: 2*V*12 */
void or_eo_reconstruct(const int L[4], const cplx *U, const cplx *Tinv, double kappa, int t_bc, double mu_ch,
                       const cplx *b, cplx *x, cplx *work)
{
    long V = vol(L);
    cplx *a = work, *c = work + V * NSC;
    keep_parity(L, 1, x);
    or_hop(L, U, t_bc, mu_ch, 0, x, a);
    for (long i = 0; i < V; i++)
        for (int k = 0; k < NSC; k++) a[i * NSC + k] = b[i * NSC + k] + kappa * a[i * NSC + k];
    or_clover_apply(L, Tinv, 0, 1 << 0, a, c);
    for (long i = 0; i < V; i++)
        if (parity_of(L, i) == 0)
            for (int k = 0; k < NSC; k++) x[i * NSC + k] = c[i * NSC + k];
}

/* ------------------------------------------------------------------ */
/* Conjugate gradient on A = Op^dag Op                                  */
/* ------------------------------------------------------------------ */

static double dotr(long n, const cplx *a, const cplx *b) /* Re <a, b> */
{
    double s = 0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (long k = 0; k < n; k++) s += creal(conj(a[k]) * b[k]);
    return s;
}

/* system 0: A = M^dag M on the full lattice; system 1: A = Mhat^dag Mhat on odd sites.
 * Plain CG from x = 0, stopping when ||r|| <= tol ||b||.  Returns iterations, or -1 if
 * maxiter was reached.  x receives the iterate. */
int or_cg(const int L[4], const cplx *U, const cplx *T, const cplx *Tinv, double kappa, int t_bc,
          double mu_ch, int system, const cplx *b, cplx *x, double tol, int maxiter)
{
    long V = vol(L), n = V * NSC;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    cplx *Ap = malloc(sizeof(cplx) * n), *work = malloc(sizeof(cplx) * 2 * n);
    for (long k = 0; k < n; k++) { x[k] = 0; r[k] = b[k]; p[k] = b[k]; }
    double rho = dotr(n, r, r), bn = sqrt(dotr(n, b, b));
    int it = 0, done = sqrt(rho) <= tol * bn;
    while (!done && it < maxiter) {
        if (system == 0) {
            or_apply_M(L, U, T, kappa, t_bc, mu_ch, 0, p, q);
            or_apply_M(L, U, T, kappa, t_bc, mu_ch, 1, q, Ap);
        } else {
            or_apply_Mhat(L, U, T, Tinv, kappa, t_bc, mu_ch, 0, p, q, work);
            or_apply_Mhat(L, U, T, Tinv, kappa, t_bc, mu_ch, 1, q, Ap, work);
        }
        double alpha = rho / dotr(n, p, Ap);
        for (long k = 0; k < n; k++) { x[k] += alpha * p[k]; r[k] -= alpha * Ap[k]; }
        double rho_new = dotr(n, r, r);
        it++;
        if (sqrt(rho_new) <= tol * bn) { done = 1; break; }
        double beta = rho_new / rho;
        for (long k = 0; k < n; k++) p[k] = r[k] + beta * p[k];
        rho = rho_new;
    }
    free(r); free(p); free(q); free(Ap); free(work);
    return done ? it : -1;
}

/* ------------------------------------------------------------------ */
/* Derivatives of M with respect to the action's parameters (the        */
/* reweighting traces Tr(M^-1 dM/dp) named in the abstract)              */
/* ------------------------------------------------------------------ */

/* S(x) = sum_{mu<nu} sigma_{mu nu} (x) Fh_{mu nu}(x), dense 12x12 per site: the clover term of
 * Eq. 2 without its factor kappa c_SW, so that T = 1 + kappa c_SW S, dT/dkappa = c_SW S and
 * dT/dc_SW = kappa S. */
void or_sigma_F(const int L[4], const cplx *U, cplx *S)
{
    init_algebra();
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        cplx *Si = S + i * NSC * NSC;
        for (int k = 0; k < NSC * NSC; k++) Si[k] = 0;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                cplx Fh[9];
                or_field_strength_site(L, U, i, mu, nu, Fh);
                for (int s = 0; s < 4; s++)
                    for (int a = 0; a < 3; a++)
                        for (int t = 0; t < 4; t++)
                            for (int b = 0; b < 3; b++)
                                Si[(s * 3 + a) * NSC + t * 3 + b] += SIG[mu][nu][s][t] * Fh[a * 3 + b];
            }
    }
}

/* (dD/dmu psi)(x): only the time hops of Eq. 1 depend on mu; the forward hop's factor e^{+mu}
 * differentiates to +e^{+mu}, the backward hop's e^{-mu} to -e^{-mu}; the boundary sign stays. */
void or_hop_dmu(const int L[4], const cplx *U, int t_bc, double mu_ch, const cplx *in, cplx *out)
{
    init_algebra();
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++) {
        cplx *o = out + i * NSC;
        for (int k = 0; k < NSC; k++) o[k] = 0;
        long f = neighbour(L, i, 3, +1), b = neighbour(L, i, 3, -1);
        add_hop_term(o, link(U, V, 3, i), 0, 3, -1.0, coef_fwd(L, i, 3, t_bc, mu_ch), in + f * NSC);
        add_hop_term(o, link(U, V, 3, b), 1, 3, +1.0, -coef_bwd(L, i, 3, t_bc, mu_ch), in + b * NSC);
    }
}

/* ------------------------------------------------------------------ */
/* Gauge observables                                                    */
/* ------------------------------------------------------------------ */

/* average over sites and the 6 planes of Re tr U_{mu nu}(x) / 3 */
double or_plaquette(const int L[4], const cplx *U)
{
    long V = vol(L);
    double s = 0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (long i = 0; i < V; i++)
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                cplx P[9], A[9];
                m3_mul(link(U, V, mu, i), link(U, V, nu, neighbour(L, i, mu, +1)), P);
                m3_dag(link(U, V, mu, neighbour(L, i, nu, +1)), A); m3_mul(P, A, P);
                m3_dag(link(U, V, nu, i), A); m3_mul(P, A, P);
                s += creal(P[0] + P[4] + P[8]) / 3.0;
            }
    return s / (6.0 * V);
}

/* ------------------------------------------------------------------ */
/* Complex Z2 noise from a counter-based generator                     */
/* ------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea, Flood 2014) used as a counter-based generator:
 * output k of the stream with seed s is mix(s + (k+1) * 0x9E3779B97F4A7C15). */
static uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Noise vector n: component (i, s, c) uses counter k = (n*V + i)*12 + s*3 + c;
 * bit 63 of the output gives the sign of the real part, bit 62 the imaginary part;
 * eta = (+-1 +- i)/sqrt(2). */
void or_z2_noise(const int L[4], uint64_t seed, long n, cplx *eta)
{
    long V = vol(L);
    const double h = 1.0 / sqrt(2.0);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; i++)
        for (int k = 0; k < NSC; k++) {
            uint64_t z = splitmix64_at(seed, (uint64_t)((n * V + i) * NSC + k));
            double re = (z >> 63) & 1 ? -h : h;
            double im = (z >> 62) & 1 ? -h : h;
            eta[i * NSC + k] = re + I * im;
        }
}

/* ------------------------------------------------------------------ */
/* Sampled outputs for large lattices                                   */
/* ------------------------------------------------------------------ */

/* Mhat (or Mhat^dag) at a list of odd sites, each computed from its definition:
 *   Mhat v(x) = T(x) v(x) - kappa^2 sum_{y ~ x} D(x,y) T^{-1}(y) sum_{z ~ y} D(y,z) v(z),
 * with T and T^{-1} built at the sites needed (no full clover field).  The neighbours
 * y of an odd x are even and their neighbours z are odd, so only odd sites of `in`
 * are read. */
void or_Mhat_sites(const int L[4], const cplx *U, double kappa, double csw, int t_bc, double mu_ch,
                   int dagger, const cplx *in, long nsite, const long *sites, cplx *out)
{
#pragma omp parallel for schedule(dynamic)
    for (long s = 0; s < nsite; s++) {
        long x = sites[s];
        cplx w[4][2][NSC];
        const cplx *nb[4][2];
        for (int mu = 0; mu < 4; mu++)
            for (int d = 0; d < 2; d++) {
                long y = neighbour(L, x, mu, d == 0 ? +1 : -1);
                cplx h[NSC], T[NSC * NSC], Ti[NSC * NSC];
                or_hop_site(L, U, t_bc, mu_ch, dagger, in, y, h);
                or_clover_site(L, U, kappa, csw, y, T);
                or_invert12(T, Ti);
                mat12_apply(Ti, dagger, h, w[mu][d]);
                nb[mu][d] = w[mu][d];
            }
        cplx h[NSC], T[NSC * NSC], t[NSC];
        hop_site_nb(L, U, t_bc, mu_ch, dagger, x, nb, h);
        or_clover_site(L, U, kappa, csw, x, T);
        mat12_apply(T, dagger, in + x * NSC, t);
        for (int k = 0; k < NSC; k++) out[s * NSC + k] = t[k] - kappa * kappa * h[k];
    }
}

/* M (or M^dag) at a list of sites, clover built at those sites only. */
void or_M_sites(const int L[4], const cplx *U, double kappa, double csw, int t_bc, double mu_ch,
                int dagger, const cplx *in, long nsite, const long *sites, cplx *out)
{
#pragma omp parallel for schedule(dynamic)
    for (long s = 0; s < nsite; s++) {
        long x = sites[s];
        cplx h[NSC], T[NSC * NSC], t[NSC];
        or_hop_site(L, U, t_bc, mu_ch, dagger, in, x, h);
        or_clover_site(L, U, kappa, csw, x, T);
        mat12_apply(T, dagger, in + x * NSC, t);
        for (int k = 0; k < NSC; k++) out[s * NSC + k] = t[k] - kappa * h[k];
    }
}

/* T(x) at a list of sites (dense 12x12 each). */
void or_clover_sites(const int L[4], const cplx *U, double kappa, double csw, long nsite, const long *sites,
                     cplx *out)
{
#pragma omp parallel for schedule(dynamic)
    for (long s = 0; s < nsite; s++) or_clover_site(L, U, kappa, csw, sites[s], out + s * NSC * NSC);
}

int or_num_threads(void)
{
    int n = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
#endif
    return n;
}
