/*
 * oracle.c -- plain CPU reference of the per-cell drag update
 *
 *     v(t+dt) = exp(dt K) v
 *
 * computed by the Taylor scaling-and-squaring method of Sewanou, Laibe and
 * Commercon (arXiv:2509.25347), Sect. 2.3 and Appendix B.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity checker for the HIP
 * library.  It is deliberately slow: single-threaded, dense (N+1)x(N+1)
 * matrices, textbook triple loops, every step in the paper's order.  It shares
 * no code, header, table or constant with the HIP library; only tests, the
 * smoke check and the benchmark's CPU-baseline leg load it.  Build with
 * -O2 -ffp-contract=off (no fused multiply-add, no fast-math) so that every
 * operation below is one IEEE-754 double rounding.
 *
 * Notation (paper Sect. 2.2, eqs. DragEqVar2-3 and jacobian):
 *   N dust species, n = N+1 fluids, index 0 = gas, 1..N = dust.
 *   a_i = dt / t_i           (dt times the inverse stopping time alpha_i)
 *   e_i = rho_i / rho_g      (dust-to-gas ratio epsilon_i)
 * The paper writes the drag ODE for momenta with the arrowhead matrix Omega
 * (eq. jacobian).  Its velocity form K = D^-1 Omega D, D = diag(rho), has the
 * same exponential up to that similarity and is what is evolved here:
 *   A = dt K:  A00 = -sum_i e_i a_i,  A0i = e_i a_i,  Ai0 = a_i,  Aii = -a_i.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   - the norm is the 1-norm of A in the velocity form;
 *   - s-hat = ceil(log2(||A|| / theta_{m_K})), taken exactly (the paper prints
 *     both floor and ceil; only ceil keeps ||A / 2^s|| <= theta);
 *   - in Alg. 1, m* = m_{k*} wherever the paper writes m_k after changing k*;
 *   - squarings carry Y = X - I (Y <- 2Y + Y Y), which is the paper's X <- X X
 *     rearranged; the literal X-form is kept behind a flag for comparison;
 *   - theta_m are the values of eq. B8 recomputed to full double precision;
 *     they agree with every digit Table B.1 prints.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* ---- Table B.1 (k, m_k, q_k, r_k, theta_{m_k}) for u = 2^-53 ------------ */
/* theta_{m_k}: largest theta with -log(1 - f_m(theta)) / theta <= u (eq. B8),
 * recomputed; Table B.1 prints them to five digits.  Row 5 is printed as
 * "2/9962 x 10^-1" in the source, read as 2.9962e-1. */
static const int TB_M[10] = {0, 2, 4, 6, 9, 12, 16, 20, 25, 30};
static const int TB_Q[10] = {0, 1, 2, 2, 3, 3, 4, 4, 5, 5};
static const int TB_R[10] = {0, 2, 2, 3, 3, 4, 4, 5, 5, 6};
static const double TB_THETA[10] = {
    0.0,
    2.580956802971767e-08,
    3.3971688399769617e-04,
    9.065656407595102e-03,
    8.957760203223343e-02,
    2.996158913811581e-01,
    7.802874256626574e-01,
    1.438252596804337e+00,
    2.4285825244428265e+00,
    3.5396663487436895e+00,
};

/* b_i = 1/i!, i = 0..30, each the double nearest to the exact rational. */
static const double TAYLOR_B[31] = {
    1.0,
    1.0,
    0.5,
    0.16666666666666666,
    0.041666666666666664,
    0.008333333333333333,
    0.001388888888888889,
    0.0001984126984126984,
    2.48015873015873e-05,
    2.7557319223985893e-06,
    2.755731922398589e-07,
    2.505210838544172e-08,
    2.08767569878681e-09,
    1.6059043836821613e-10,
    1.1470745597729725e-11,
    7.647163731819816e-13,
    4.779477332387385e-14,
    2.8114572543455206e-15,
    1.5619206968586225e-16,
    8.22063524662433e-18,
    4.110317623312165e-19,
    1.9572941063391263e-20,
    8.896791392450574e-22,
    3.868170170630684e-23,
    1.6117375710961184e-24,
    6.446950284384474e-26,
    2.4795962632247976e-27,
    9.183689863795546e-29,
    3.279889237069838e-30,
    1.1309962886447716e-31,
    3.7699876288159054e-33,
};

int orc_table_row(int k, int *m, int *q, int *r, double *theta)
{
    if (k < 1 || k > 9) return -1;
    *m = TB_M[k];
    *q = TB_Q[k];
    *r = TB_R[k];
    *theta = TB_THETA[k];
    return 0;
}

double orc_taylor_coef(int i)
{
    if (i < 0 || i > 30) return NAN;
    return TAYLOR_B[i];
}

/* ---- Alg. 1: choice of (k*, m*, s*) --------------------------------------- */
/* Appendix B, "First modification" (Alg. 1 with options 0, 1, 2 and a cap K
 * on the products of the polynomial stage), stated through its cost model:
 * row k of Table B.1 costs Pi_{m_k} = k products, each squaring one more, and
 * row k is admissible for a scaling 2^-s when ||A|| / 2^s <= theta_{m_k}
 * (eq. B8).
 *   Base choice: without scaling, the cheapest admissible row; when no row
 *   up to K is, row K with s-hat, the fewest squarings that make it
 *   admissible.
 *   Trades: the options then replace (k, s) by (k + dk, s + ds) if that pair
 *   is admissible, trying in order one product fewer at the same s
 *   (option >= 1, rows 7..9) and two or three polynomial products for one or
 *   two squarings, the same total cost at a lower degree (option 2, rows
 *   8..9 and row 9).  The first admissible trade is taken.
 * The comparisons are exact: ||A|| 2^-s is an exact scaling of a double.
 * nrm must be finite. */
typedef struct {
    int dk, ds, min_option, k_lo, k_hi;
} select_trade;

static const select_trade SELECT_TRADES[3] = {
    {-1, 0, 1, 7, 9},
    {-2, 1, 2, 8, 9},
    {-3, 2, 2, 9, 9},
};

void orc_select(double nrm, int K, int option, int *kout, int *mout, int *sout)
{
    int k, s = 0;
    if (nrm <= TB_THETA[K]) {
        k = 1;
        while (nrm > TB_THETA[k]) ++k;
    } else {
        k = K;
        while (nrm > ldexp(TB_THETA[K], s)) ++s;
    }
    for (int t = 0; t < 3; ++t) {
        const select_trade *tr = &SELECT_TRADES[t];
        if (option < tr->min_option || k < tr->k_lo || k > tr->k_hi) continue;
        if (ldexp(nrm, -(s + tr->ds)) <= TB_THETA[k + tr->dk]) {
            k += tr->dk;
            s += tr->ds;
            break;
        }
    }
    *kout = k;
    *mout = TB_M[k];
    *sout = s;
}

/* ---- dense helpers (row-major n x n) -------------------------------------- */
static void mat_mul(int n, const double *X, const double *Y, double *Z)
{
    /* Z = X Y, inner index ascending */
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += X[i * n + k] * Y[k * n + j];
            Z[i * n + j] = acc;
        }
}

static void mat_mul_tn(int n, const double *X, const double *Y, double *Z)
{
    /* Z = X^T Y */
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += X[k * n + i] * Y[k * n + j];
            Z[i * n + j] = acc;
        }
}

static void mat_mul_nt(int n, const double *X, const double *Y, double *Z)
{
    /* Z = X Y^T */
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += X[i * n + k] * Y[j * n + k];
            Z[i * n + j] = acc;
        }
}

/* ---- step 1: the drag matrix and its 1-norm ------------------------------- */
/* Per-cell inputs -> A = dt K (velocity form) and ||A||_1.  Returns the
 * bad-input bits of the cell (0 when the cell is valid). */
int orc_build(int N, double dt, double rho_g, const double *rho_d,
              const double *t_stop, double *A, double *a, double *e,
              double *nrm)
{
    const int n = N + 1;
    int bad = 0;
    if (!(isfinite(rho_g) && rho_g > 0.0)) bad |= ORC_BAD_DENSITY;
    for (int i = 0; i < N; ++i) {
        if (!(isfinite(rho_d[i]) && rho_d[i] >= 0.0)) bad |= ORC_BAD_DENSITY;
        if (!(t_stop[i] > 0.0)) bad |= ORC_BAD_STOPPING_TIME; /* NaN fails too */
    }
    memset(A, 0, sizeof(double) * n * n);
    if (bad) { *nrm = NAN; return bad; }

    double s = 0.0;
    int overflow = 0;
    for (int i = 1; i <= N; ++i) {
        a[i - 1] = dt / t_stop[i - 1];        /* t = +inf gives a = 0 */
        e[i - 1] = rho_d[i - 1] / rho_g;
        double p = e[i - 1] * a[i - 1];
        A[0 * n + i] = p;                     /* gas row: back-reaction */
        A[i * n + 0] = a[i - 1];              /* dust rows: drag toward gas */
        A[i * n + i] = -a[i - 1];
        s += p;
        if (!isfinite(a[i - 1]) || !isfinite(p)) overflow = 1;
    }
    A[0] = -s;

    /* 1-norm: the largest column sum of |A_ij|, rows summed in order */
    double best = 0.0;
    for (int j = 0; j < n; ++j) {
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += fabs(A[i * n + j]);
        if (c > best) best = c;
    }
    *nrm = best;
    /* an entry of dt K that overflowed (0 * inf included) makes the cell bad */
    if (overflow || !isfinite(best)) { *nrm = NAN; return ORC_BAD_NORM; }
    return 0;
}

/* ---- steps 2-6: the scaled Taylor polynomial and the squarings ----------- */
/* Workspace for one cell; sized for n <= ORC_NMAX. */
typedef struct {
    double P[6][ORC_NMAX * ORC_NMAX];    /* P[j] = B^j, j = 1..q (q <= 5) */
    double Bbar[ORC_NMAX * ORC_NMAX];
    double F[ORC_NMAX * ORC_NMAX];
    double T[ORC_NMAX * ORC_NMAX];
    double U[ORC_NMAX * ORC_NMAX];
} work_t;

/* 1-norm (largest column sum of absolute values) of an n x n matrix. */
static double norm1(int n, const double *X)
{
    double best = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += fabs(X[i * n + j]);
        if (s > best) best = s;
    }
    return best;
}

/* b_exp of the second modification (Appendix B, eq. Pat_Stk6 and the
 * "compute bound" algorithm): an estimate of ||e^-B|| from the blocks of
 * T_m(-B),
 *     b_exp = ||b0 I + Bhat_0|| + sum_{l=1}^{r-1} ||Bhat_l|| ||B^q||^l,
 *     Bhat_l = sum_{j=1}^{q} (-1)^(ql+j) b_{ql+j} B^j,
 * accumulated from l = r-1 down (Horner in ||B^q||).  Reading: the index of
 * Bhat inside the loop is l (the printed listings write r-1 in one version
 * and k in the other). */
static double bound_bexp(int n, int q, int r, work_t *w)
{
    const int nn = n * n;
    const double nq = norm1(n, w->P[q]);
    double b = 0.0;
    for (int l = r - 1; l >= 0; --l) {
        memset(w->Bbar, 0, sizeof(double) * nn);
        for (int j = 1; j <= q; ++j) {
            const int i = q * l + j;
            const double c = (i % 2 ? -1.0 : 1.0) * TAYLOR_B[i];
            for (int t = 0; t < nn; ++t) w->Bbar[t] += c * w->P[j][t];
        }
        if (l >= 1) {
            b = (norm1(n, w->Bbar) + b) * nq;
        } else {
            for (int i = 0; i < n; ++i) w->Bbar[i * n + i] += TAYLOR_B[0];
            b = b + norm1(n, w->Bbar);
        }
    }
    return b;
}

/* Taylor stage of the merged Paterson-Stockmeyer / Horner evaluation
 * (Appendix B, "New Taylor polynomial evaluation", eqs. Pat_Stk-Pat_Stk3):
 *   T_m(B) = b0 I + sum_{k=0}^{r-1} Bbar_k (B^q)^k,
 *   Bbar_k = sum_{j=1}^{q} b_{qk+j} B^j.
 * The identity term is left out, so F = T_m(B) - I.  The paper recomputes
 * the powers B^j inside the k loop to avoid storing them; they are the same
 * products in the same order, so they are computed once here.
 *
 * bound_test != 0 adds Sastre's second modification (eqs. Pat_Stk4-Pat_stk7
 * and the evaluation with the bound test): before the product that carries
 * the accumulated higher blocks T = Bbar_k + F to level k, the part
 * T (B^q)^k is dropped when b_exp ||T|| ||B^q||^k <= u (u = 2^-53): since
 * ||e^B||^-1 <= ||e^-B|| ~ b_exp, it is then below u relative to ||e^B||.
 * *skipped counts the products saved (NULL: not reported). */
static void taylor_minus_identity(int n, const double *B, int q, int r,
                                  work_t *w, double *F, int bound_test,
                                  int *skipped)
{
    const int nn = n * n;
    memcpy(w->P[1], B, sizeof(double) * nn);
    for (int j = 2; j <= q; ++j) mat_mul(n, B, w->P[j - 1], w->P[j]);

    double bexp = 0.0, nq = 0.0;
    if (bound_test) {
        bexp = bound_bexp(n, q, r, w);
        nq = norm1(n, w->P[q]);
    }
    int skips = 0;
    memset(F, 0, sizeof(double) * nn);
    for (int k = r - 1; k >= 0; --k) {
        memset(w->Bbar, 0, sizeof(double) * nn);
        for (int j = 1; j <= q; ++j) {
            const double b = TAYLOR_B[q * k + j];
            for (int t = 0; t < nn; ++t) w->Bbar[t] += b * w->P[j][t];
        }
        for (int t = 0; t < nn; ++t) w->T[t] = w->Bbar[t] + F[t];
        if (k >= 1) {
            int drop = 0;
            if (bound_test) {
                double pk = 1.0;
                for (int i = 0; i < k; ++i) pk *= nq;
                drop = bexp * norm1(n, w->T) * pk <= ldexp(1.0, -53);
            }
            if (drop) {
                memset(F, 0, sizeof(double) * nn);   /* T (B^q)^k neglected */
                ++skips;
            } else {
                mat_mul(n, w->T, w->P[q], F);       /* F = (Bbar_k + F) B^q */
            }
        } else {
            memcpy(F, w->T, sizeof(double) * nn);
        }
    }
    if (skipped) *skipped = skips;
}

/* The Taylor stage alone on a given (already scaled) n x n matrix B:
 * F = T_m(B) - I for row k of Table B.1, with or without the bound test;
 * *skipped = products saved, *bexp_out = b_exp (either may be NULL). */
int orc_taylor_stage(int n, const double *B, int k, int bound_test, double *F,
                     int *skipped, double *bexp_out)
{
    if (n < 1 || n > ORC_NMAX || k < 1 || k > 9) return -1;
    work_t *w = (work_t *)malloc(sizeof(work_t));
    if (!w) return -2;
    taylor_minus_identity(n, B, TB_Q[k], TB_R[k], w, F, bound_test, skipped);
    if (bexp_out) *bexp_out = bound_bexp(n, TB_Q[k], TB_R[k], w);
    free(w);
    return 0;
}

/* ---- the diagonal Pade scaling step (Sect. 2.3, eq. PadeEqu, p = q = m) ---- */
/* Degrees m and theta_m: the largest theta for which the backward error of
 * the diagonal approximant r_m = N_mm / D_mm, log(e^-x r_m(x)) =
 * sum_{k > 2m} c_k x^k, satisfies sum_k |c_k| theta^(k-1) <= u = 2^-53 (the
 * criterion eq. B8 applies to the Taylor polynomial), computed in
 * multiprecision from the power series.  The paper defines the approximant
 * but gives no degree table; this one is the test's own. */
static const int PADE_M[5] = {3, 5, 7, 9, 13};
static const double PADE_THETA[5] = {
    1.4955852179582915e-02,
    2.539398330063232e-01,
    9.504178996162932e-01,
    2.0978479612570675e+00,
    5.371920351148153e+00,
};

/* c_j = (2m - j)! m! / ((2m)! j! (m - j)!), j = 0..m: the coefficients of
 * N_mm in eq. PadeEqu (those of D_mm are (-1)^j c_j), by the ratio of
 * consecutive terms in binary128 and one rounding to double. */
static void pade_coefs(int m, double *c)
{
    __float128 x = 1;
    for (int j = 0; j <= m; ++j) {
        c[j] = (double)x;
        x = x * (__float128)(m - j) / ((__float128)(2 * m - j) * (__float128)(j + 1));
    }
}

int orc_pade_row(int i, int *m, double *theta, double *coef)
{
    if (i < 0 || i > 4) return -1;
    if (m) *m = PADE_M[i];
    if (theta) *theta = PADE_THETA[i];
    if (coef) pade_coefs(PADE_M[i], coef);
    return 0;
}

/* (m, s) for a finite ||A||_1: the lowest degree whose theta covers ||A||
 * (s = 0), else m = 13 and the smallest s with ||A|| <= theta_13 2^s
 * (exact power-of-two comparisons). */
void orc_pade_select(double nrm, int *mout, int *sout)
{
    for (int i = 0; i < 4; ++i) {
        if (nrm <= PADE_THETA[i]) { *mout = PADE_M[i]; *sout = 0; return; }
    }
    int sh = 0;
    while (nrm > ldexp(PADE_THETA[4], sh)) ++sh;
    *mout = 13;
    *sout = sh;
}

/* Z = r_m(B) - I.  With V and U the even and odd parts of N_mm(B),
 * D_mm(B) = V - U and N_mm(B) = V + U, so r_m(B) - I = D^-1 (N - D) solves
 *     (V - U) Z = 2 U
 * (no cancellation for small B).  Powers by plain products; the system by
 * Gaussian elimination with partial pivoting on all n right-hand sides.
 * Returns 0, or -1 for a zero pivot. */
static int pade_minus_identity(int n, const double *B, int m, work_t *w, double *Z)
{
    const int nn = n * n;
    double c[14];
    pade_coefs(m, c);
    double *V = w->Bbar, *U = w->F, *cur = w->P[1], *nxt = w->P[2];
    memset(V, 0, sizeof(double) * nn);
    memset(U, 0, sizeof(double) * nn);
    for (int i = 0; i < n; ++i) V[i * n + i] = c[0];
    memcpy(cur, B, sizeof(double) * nn);
    for (int j = 1; j <= m; ++j) {
        if (j > 1) {
            mat_mul(n, B, cur, nxt);
            double *t = cur; cur = nxt; nxt = t;
        }
        double *acc = (j & 1) ? U : V;
        for (int t = 0; t < nn; ++t) acc[t] += c[j] * cur[t];
    }
    double *M = w->T;
    for (int t = 0; t < nn; ++t) {
        M[t] = V[t] - U[t];
        Z[t] = 2.0 * U[t];
    }
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(M[i * n + k]) > fabs(M[p * n + k])) p = i;
        if (M[p * n + k] == 0.0) return -1;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = M[k * n + j]; M[k * n + j] = M[p * n + j]; M[p * n + j] = t;
                t = Z[k * n + j]; Z[k * n + j] = Z[p * n + j]; Z[p * n + j] = t;
            }
        }
        for (int i = k + 1; i < n; ++i) {
            const double f = M[i * n + k] / M[k * n + k];
            for (int j = k; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
            for (int j = 0; j < n; ++j) Z[i * n + j] -= f * Z[k * n + j];
        }
    }
    for (int k = n - 1; k >= 0; --k)
        for (int j = 0; j < n; ++j) {
            double acc = Z[k * n + j];
            for (int i = k + 1; i < n; ++i) acc -= M[k * n + i] * Z[i * n + j];
            Z[k * n + j] = acc / M[k * n + k];
        }
    return 0;
}

/* option: Alg. 1 option (0, 1, 2), ORed with ORC_BOUND_TEST for the second
 * modification in the Taylor stage, or with ORC_PADE for the diagonal Pade
 * scaling step instead of the Taylor one (Alg. 1 and K then unused). */
static void expm_ws(int n, const double *A, double nrm, int K, int option,
                    int xform, double *Y, int *kms, work_t *w)
{
    const int nn = n * n;
    const int bound_test = option & ORC_BOUND_TEST;
    const int pade = option & ORC_PADE;
    option &= 3;
    int k, m, s;
    if (pade) {
        k = 0;
        orc_pade_select(nrm, &m, &s);
    } else {
        orc_select(nrm, K, option, &k, &m, &s);
    }
    kms[0] = k; kms[1] = m; kms[2] = s;

    double *B = w->U;
    for (int t = 0; t < nn; ++t) B[t] = ldexp(A[t], -s);     /* 2^-s A */

    if (pade) {
        if (pade_minus_identity(n, B, m, w, Y) != 0)
            for (int t = 0; t < nn; ++t) Y[t] = NAN;
    } else {
        taylor_minus_identity(n, B, TB_Q[k], TB_R[k], w, Y, bound_test, NULL);
    }

    if (!xform) {
        /* Y-form squaring: (I+Y)^2 = I + 2Y + Y Y */
        for (int it = 0; it < s; ++it) {
            mat_mul(n, Y, Y, w->T);
            for (int t = 0; t < nn; ++t) Y[t] = 2.0 * Y[t] + w->T[t];
        }
    } else {
        /* paper-literal X <- X X on X = T_m(B) */
        for (int i = 0; i < n; ++i) Y[i * n + i] += 1.0;
        for (int it = 0; it < s; ++it) {
            mat_mul(n, Y, Y, w->T);
            memcpy(Y, w->T, sizeof(double) * nn);
        }
        for (int i = 0; i < n; ++i) Y[i * n + i] -= 1.0;
    }
}

int orc_expm(int N, const double *A, double nrm, int K, int option, int xform,
             double *Y, int *kms)
{
    const int n = N + 1;
    if (n > ORC_NMAX || K < 1 || K > 9 || (option & ~(ORC_BOUND_TEST | ORC_PADE)) < 0 ||
        (option & ~(ORC_BOUND_TEST | ORC_PADE)) > 2)
        return -1;
    if (!isfinite(nrm)) return -1;
    work_t *w = (work_t *)malloc(sizeof(work_t));
    if (!w) return -2;
    expm_ws(n, A, nrm, K, option, xform, Y, kms, w);
    free(w);
    return 0;
}

/* ---- step 7: apply to every cell of an SoA grid -------------------------- */
/* Layout (the same as the library's): rho_g[c], rho_d[i*ld + c],
 * t_stop[i*ld + c], v[(d*(N+1) + j)*ld + c], j = 0 gas, 1..N dust.
 * kms (optional) receives k*, m*, s* at kms[c], kms[ld + c], kms[2 ld + c];
 * nrm (optional) receives ||A||_1 at nrm[c].  Returns the OR of the
 * bad-input bits of all cells; a bad cell's outputs are NaN. */
int orc_apply_cells(int64_t C, int N, int D, int64_t ld, double dt, int K,
                    int option, int xform, const double *rho_g,
                    const double *rho_d, const double *t_stop,
                    const double *v_in, double *v_out, int32_t *kms,
                    double *nrm_out)
{
    const int n = N + 1, nn = n * n;
    if (n > ORC_NMAX || D < 1 || D > 3 || ld < C) return -1;
    if (K < 1 || K > 9 || (option & ~(ORC_BOUND_TEST | ORC_PADE)) < 0 ||
        (option & ~(ORC_BOUND_TEST | ORC_PADE)) > 2)
        return -1;
    double *A = (double *)malloc(sizeof(double) * nn);
    double *Y = (double *)malloc(sizeof(double) * nn);
    work_t *w = (work_t *)malloc(sizeof(work_t));
    double rd[ORC_NMAX], ts[ORC_NMAX], a[ORC_NMAX], e[ORC_NMAX];
    double vin[ORC_NMAX], vout[ORC_NMAX];
    int status = 0;
    if (!A || !Y || !w) { free(A); free(Y); free(w); return -2; }

    for (int64_t c = 0; c < C; ++c) {
        for (int i = 0; i < N; ++i) {
            rd[i] = rho_d[i * ld + c];
            ts[i] = t_stop[i * ld + c];
        }
        double nrm;
        int bad = orc_build(N, dt, rho_g[c], rd, ts, A, a, e, &nrm);
        for (int d = 0; d < D && !bad; ++d)
            for (int j = 0; j < n; ++j)
                if (!isfinite(v_in[(d * n + j) * ld + c])) bad |= ORC_BAD_VELOCITY;
        int km[3] = {0, 0, 0};
        if (!bad) {
            expm_ws(n, A, nrm, K, option, xform, Y, km, w);
            for (int d = 0; d < D; ++d) {
                for (int j = 0; j < n; ++j) vin[j] = v_in[(d * n + j) * ld + c];
                for (int j = 0; j < n; ++j) {
                    double acc = 0.0;
                    for (int t = 0; t < n; ++t) acc += Y[j * n + t] * vin[t];
                    vout[j] = vin[j] + acc;   /* v' = v + (E - I) v */
                }
                for (int j = 0; j < n; ++j) v_out[(d * n + j) * ld + c] = vout[j];
            }
        } else {
            for (int d = 0; d < D; ++d)
                for (int j = 0; j < n; ++j) v_out[(d * n + j) * ld + c] = NAN;
        }
        status |= bad;
        if (kms) { kms[c] = km[0]; kms[ld + c] = km[1]; kms[2 * ld + c] = km[2]; }
        if (nrm_out) nrm_out[c] = nrm;
    }
    free(A);
    free(Y);
    free(w);
    return status;
}

/* Full exponential of one cell, E = exp(dt K) (dense n x n, row-major). */
int orc_cell_expm(int N, double dt, double rho_g, const double *rho_d,
                  const double *t_stop, int K, int option, int xform,
                  double *E, int *kms)
{
    const int n = N + 1;
    if (n > ORC_NMAX) return -1;
    double A[ORC_NMAX * ORC_NMAX], a[ORC_NMAX], e[ORC_NMAX], nrm;
    int bad = orc_build(N, dt, rho_g, rho_d, t_stop, A, a, e, &nrm);
    if (bad) return bad;
    orc_expm(N, A, nrm, K, option, xform, E, kms);
    for (int i = 0; i < n; ++i) E[i * n + i] += 1.0;
    return 0;
}

/* ---- reverse-mode gradient ----------------------------------------------- */
/* For the loss L = sum_d w_d . v'_d, the gradient of the computed approximant
 * with (k*, m*, s*) frozen, taken backwards through the stored chain:
 * apply, the s squarings, the Horner steps, the Bbar sums, the powers, the
 * scaling, and finally the entries of A as functions of (a_i, e_i).
 *
 * orc_grad_A: given A and G = dL/dY (the adjoint of the final Y), returns
 * dL/dA (n x n).  In exact arithmetic this is the Frechet derivative of the
 * approximant at A^T in the direction G. */
int orc_grad_A(int N, const double *A, double nrm, int K, int option,
               const double *G, double *Abar, int *kms)
{
    const int n = N + 1, nn = n * n;
    /* the gradient is of the evaluation without the bound test */
    if (n > ORC_NMAX || !isfinite(nrm) || option < 0 || option > 2) return -1;
    int k, m, s;
    orc_select(nrm, K, option, &k, &m, &s);
    kms[0] = k; kms[1] = m; kms[2] = s;
    const int q = TB_Q[k], r = TB_R[k];

    /* forward pass, storing every intermediate */
    double *B = (double *)malloc(sizeof(double) * nn);
    double *P = (double *)malloc(sizeof(double) * nn * (q + 1));
    double *H = (double *)malloc(sizeof(double) * nn * r);   /* Bbar_k + F */
    double *Ys = (double *)malloc(sizeof(double) * nn * (s + 1));
    double *T = (double *)malloc(sizeof(double) * nn);
    double *Bb = (double *)malloc(sizeof(double) * nn);
    double *F = (double *)malloc(sizeof(double) * nn);
    if (!B || !P || !H || !Ys || !T || !Bb || !F) {
        free(B); free(P); free(H); free(Ys); free(T); free(Bb); free(F);
        return -2;
    }
    for (int t = 0; t < nn; ++t) B[t] = ldexp(A[t], -s);
    memcpy(P + nn * 1, B, sizeof(double) * nn);
    for (int j = 2; j <= q; ++j) mat_mul(n, B, P + nn * (j - 1), P + nn * j);
    memset(F, 0, sizeof(double) * nn);
    for (int kk = r - 1; kk >= 0; --kk) {
        memset(Bb, 0, sizeof(double) * nn);
        for (int j = 1; j <= q; ++j) {
            const double b = TAYLOR_B[q * kk + j];
            for (int t = 0; t < nn; ++t) Bb[t] += b * P[nn * j + t];
        }
        double *Hk = H + nn * kk;
        for (int t = 0; t < nn; ++t) Hk[t] = Bb[t] + F[t];
        if (kk >= 1) mat_mul(n, Hk, P + nn * q, F);
        else memcpy(F, Hk, sizeof(double) * nn);
    }
    memcpy(Ys, F, sizeof(double) * nn);
    for (int it = 0; it < s; ++it) {
        double *Yi = Ys + nn * it, *Yn = Ys + nn * (it + 1);
        mat_mul(n, Yi, Yi, T);
        for (int t = 0; t < nn; ++t) Yn[t] = 2.0 * Yi[t] + T[t];
    }

    /* backward pass */
    double *Ybar = (double *)malloc(sizeof(double) * nn);
    double *U = (double *)malloc(sizeof(double) * nn);
    double *Pbar = (double *)calloc((size_t)nn * (q + 1), sizeof(double));
    double *Bbarbar = (double *)malloc(sizeof(double) * nn);
    memcpy(Ybar, G, sizeof(double) * nn);
    for (int it = s - 1; it >= 0; --it) {
        /* Y_{it+1} = 2 Y_it + Y_it Y_it */
        const double *Yi = Ys + nn * it;
        mat_mul_nt(n, Ybar, Yi, T);          /* Ybar Y^T */
        mat_mul_tn(n, Yi, Ybar, U);          /* Y^T Ybar */
        for (int t = 0; t < nn; ++t) Ybar[t] = 2.0 * Ybar[t] + T[t] + U[t];
    }
    /* Horner, reversed.  Step kk >= 1: F_kk = H_kk P_q with H_kk = Bbar_kk + F_{kk+1};
     * step 0: F_0 = H_0.  Fbar of the running F starts at Ybar. */
    double *Fbar = Ybar;
    for (int kk = 0; kk <= r - 1; ++kk) {
        double *Hbar = U;
        if (kk == 0) {
            memcpy(Hbar, Fbar, sizeof(double) * nn);
        } else {
            const double *Hk = H + nn * kk;
            mat_mul_nt(n, Fbar, P + nn * q, Hbar);        /* Fbar P_q^T */
            mat_mul_tn(n, Hk, Fbar, T);                   /* H^T Fbar  */
            for (int t = 0; t < nn; ++t) Pbar[nn * q + t] += T[t];
        }
        /* H_kk = Bbar_kk + F_{kk+1}: both receive Hbar */
        memcpy(Bbarbar, Hbar, sizeof(double) * nn);
        for (int j = 1; j <= q; ++j) {
            const double b = TAYLOR_B[q * kk + j];
            for (int t = 0; t < nn; ++t) Pbar[nn * j + t] += b * Bbarbar[t];
        }
        memcpy(Fbar, Hbar, sizeof(double) * nn);
    }
    /* powers, reversed: P_j = B P_{j-1} */
    double *Bbar_total = Bbarbar;
    memset(Bbar_total, 0, sizeof(double) * nn);
    for (int j = q; j >= 2; --j) {
        mat_mul_nt(n, Pbar + nn * j, P + nn * (j - 1), T);  /* Pbar_j P_{j-1}^T */
        for (int t = 0; t < nn; ++t) Bbar_total[t] += T[t];
        mat_mul_tn(n, B, Pbar + nn * j, T);                   /* B^T Pbar_j */
        for (int t = 0; t < nn; ++t) Pbar[nn * (j - 1) + t] += T[t];
    }
    for (int t = 0; t < nn; ++t) Bbar_total[t] += Pbar[nn * 1 + t];
    for (int t = 0; t < nn; ++t) Abar[t] = ldexp(Bbar_total[t], -s);

    free(B); free(P); free(H); free(Ys); free(T); free(Bb); free(F);
    free(Ybar); free(U); free(Pbar); free(Bbarbar);
    return 0;
}

/* Gradients of L = sum_d w_d . v'_d over an SoA grid.
 * Outputs (any may be NULL): v_out, g_v (layout of v), g_logt and g_rho_d
 * ([N][ld]), g_rho_g ([C]).  dL/dlog t_i = -a_i dL/da_i,
 * dL/drho_i = (dL/de_i) / rho_g, dL/drho_g = -sum_i e_i (dL/de_i) / rho_g. */
int orc_grad_cells(int64_t C, int N, int D, int64_t ld, double dt, int K,
                   int option, const double *rho_g, const double *rho_d,
                   const double *t_stop, const double *v_in, const double *w_in,
                   double *v_out, double *g_v, double *g_logt,
                   double *g_rho_d, double *g_rho_g)
{
    const int n = N + 1, nn = n * n;
    if (n > ORC_NMAX || D < 1 || D > 3 || ld < C) return -1;
    double *A = (double *)malloc(sizeof(double) * nn);
    double *Y = (double *)malloc(sizeof(double) * nn);
    double *G = (double *)malloc(sizeof(double) * nn);
    double *Ab = (double *)malloc(sizeof(double) * nn);
    double rd[ORC_NMAX], ts[ORC_NMAX], a[ORC_NMAX], e[ORC_NMAX];
    double vv[3][ORC_NMAX], ww[3][ORC_NMAX];
    int status = 0;

    for (int64_t c = 0; c < C; ++c) {
        for (int i = 0; i < N; ++i) {
            rd[i] = rho_d[i * ld + c];
            ts[i] = t_stop[i * ld + c];
        }
        double nrm;
        int bad = orc_build(N, dt, rho_g[c], rd, ts, A, a, e, &nrm);
        for (int d = 0; d < D; ++d)
            for (int j = 0; j < n; ++j) {
                vv[d][j] = v_in[(d * n + j) * ld + c];
                ww[d][j] = w_in[(d * n + j) * ld + c];
                if (!bad && !(isfinite(vv[d][j]) && isfinite(ww[d][j])))
                    bad |= ORC_BAD_VELOCITY;
            }
        status |= bad;
        if (bad) {
            for (int d = 0; d < D; ++d)
                for (int j = 0; j < n; ++j) {
                    if (v_out) v_out[(d * n + j) * ld + c] = NAN;
                    if (g_v) g_v[(d * n + j) * ld + c] = NAN;
                }
            for (int i = 0; i < N; ++i) {
                if (g_logt) g_logt[i * ld + c] = NAN;
                if (g_rho_d) g_rho_d[i * ld + c] = NAN;
            }
            if (g_rho_g) g_rho_g[c] = NAN;
            continue;
        }
        int km[3];
        orc_expm(N, A, nrm, K, option, 0, Y, km);
        /* G = dL/dY = sum_d w_d v_d^T */
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int d = 0; d < D; ++d) acc += ww[d][i] * vv[d][j];
                G[i * n + j] = acc;
            }
        for (int d = 0; d < D; ++d) {
            for (int j = 0; j < n; ++j) {
                double acc = 0.0, accT = 0.0;
                for (int t = 0; t < n; ++t) {
                    acc += Y[j * n + t] * vv[d][t];
                    accT += Y[t * n + j] * ww[d][t];
                }
                if (v_out) v_out[(d * n + j) * ld + c] = vv[d][j] + acc;
                if (g_v) g_v[(d * n + j) * ld + c] = ww[d][j] + accT;
            }
        }
        orc_grad_A(N, A, nrm, K, option, G, Ab, km);
        double sum_ge = 0.0;
        for (int i = 1; i <= N; ++i) {
            const double Ab00 = Ab[0], Ab0i = Ab[0 * n + i];
            const double Abi0 = Ab[i * n + 0], Abii = Ab[i * n + i];
            const double ei = e[i - 1], ai = a[i - 1];
            /* A00 = -sum e a, A0i = e a, Ai0 = a, Aii = -a */
            const double dLda = -ei * Ab00 + ei * Ab0i + Abi0 - Abii;
            const double dLde = -ai * Ab00 + ai * Ab0i;
            if (g_logt) g_logt[(i - 1) * ld + c] = -ai * dLda;
            if (g_rho_d) g_rho_d[(i - 1) * ld + c] = dLde / rho_g[c];
            sum_ge += ei * dLde;
        }
        if (g_rho_g) g_rho_g[c] = -sum_ge / rho_g[c];
    }
    free(A); free(Y); free(G); free(Ab);
    return status;
}
