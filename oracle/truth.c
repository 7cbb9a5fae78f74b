/*
 * truth.c -- independent long-double references for the exponential of the
 * drag matrix (TEST INFRASTRUCTURE ONLY; see oracle.c).
 *
 * These do not use scaling and squaring.  They pin the oracle to results
 * that follow from the mathematics alone:
 *
 * truth_expm_eigen -- exp(dt K) from the eigen-decomposition of the
 *   symmetrised matrix.  With w = (1, sqrt(e_1), .., sqrt(e_N)),
 *   S = diag(w) A diag(w)^-1 is a symmetric arrowhead matrix
 *   (S00 = -sum e_i a_i, S0i = a_i sqrt(e_i), Sii = -a_i).  Its eigenvalues
 *   are 0 (eigenvector w) and the N roots of the secular equation
 *   1 + sum_i e_i a_i / (lambda + a_i) = 0, one between each pair of
 *   consecutive poles -a_(j+1) < lambda < -a_(j) and one below -a_max; the
 *   eigenvector of a root is (1, a_i sqrt(e_i) / (lambda + a_i)).  Each root
 *   is bracketed by bisection with the origin moved to the nearer pole, so
 *   lambda + a_i keeps its relative accuracy.  Requires e_i > 0 and distinct
 *   a_i > 0 (returns -1 otherwise).  The exact result is
 *   E_jk = (w_k / w_j) sum_l x_jl x_kl exp(lambda_l).
 *
 * truth_expm_taylor -- the plain power series sum_{i<=terms} A^i / i! in long
 *   double, meaningful for ||A||_1 <= 7 (the largest term then stays below
 *   e^7 and the long-double cancellation error below 1e-16).
 *
 * truth_expm_general -- exp(dt K) for every valid cell, by the same
 *   eigen-decomposition after splitting off the species it cannot take:
 *   a species with a_i = 0 (t_i = inf) is decoupled (its row and column of K
 *   vanish); a species with e_i = 0 and a_i > 0 has no back-reaction, so it is
 *   the gas velocity filtered by its own relaxation,
 *     v_i(1) = e^{-a_i} v_i(0) + a_i int_0^1 e^{-a_i (1 - tau)} v_g(tau) dtau,
 *   with v_g(tau) a sum of the modes e^{lambda_l tau} of the rest; species
 *   with equal a_i (and e_i > 0) relax as one species of summed e (the
 *   e-weighted mean velocity), their differences decaying as e^{-a_i}.
 *
 * truth_apply_cells -- v' = E v on an SoA grid with E from
 *   truth_expm_general; cells with invalid inputs get NaN.
 *
 * truth_grad_cells -- the exact gradient of L = sum_d w_d . (E v_d) with
 *   respect to v, log t_i, rho_i and rho_g on an SoA grid.  dL/dA for
 *   L = <G, exp(A)>, G = sum_d w_d v_d^T, is the Frechet derivative of the
 *   exponential at A^T in the direction G; with A = W^-1 S W (S the
 *   symmetrised matrix, W = diag(w)) it is W L_S[W^-1 G W] W^-1, where for
 *   symmetric S = Q diag(lam) Q^T the derivative is the Daleckii-Krein form
 *   L_S[X] = Q (Phi o (Q^T X Q)) Q^T with the divided differences
 *   Phi_lm = (e^lam_l - e^lam_m) / (lam_l - lam_m) (e^lam_l on the
 *   diagonal).  The chain rule through A00 = -sum e_i a_i, A0i = e_i a_i,
 *   Ai0 = a_i, Aii = -a_i, a_i = dt / t_i, e_i = rho_i / rho_g follows.
 *   Cells the eigen-decomposition cannot take (see truth_expm_eigen) get NaN.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

typedef long double ld_t;

/* f(mu) with lambda = -a_p + mu, written with the shifted differences
 * lambda + a_i = mu + (a_i - a_p). */
static ld_t secular(int N, const ld_t *a, const ld_t *e, int p, ld_t mu)
{
    ld_t f = 1.0L;
    for (int i = 0; i < N; ++i) {
        ld_t den = (i == p) ? mu : mu + (a[i] - a[p]);
        f += e[i] * a[i] / den;
    }
    return f;
}

/* Root of the secular equation in the open interval (lo, hi) of lambda, where
 * f(lo+) = +inf and f(hi-) = -inf (f decreases between poles).  p_lo / p_hi
 * are the pole indices bounding the interval (-1: none).  Returns the pole
 * index p used as origin and mu = lambda + a_p. */
static void secular_root(int N, const ld_t *a, const ld_t *e, ld_t lo, ld_t hi,
                         int p_lo, int p_hi, int *p_out, ld_t *mu_out)
{
    ld_t mid = 0.5L * (lo + hi);
    int p;
    if (p_hi < 0) {
        p = p_lo;
    } else if (p_lo < 0) {
        p = p_hi;
    } else {
        /* f decreasing: f(mid) > 0 means the root is right of mid (near hi) */
        ld_t fm = secular(N, a, e, p_hi, mid + a[p_hi]);
        p = (fm > 0) ? p_hi : p_lo;
    }
    ld_t mlo = lo + a[p], mhi = hi + a[p];
    if (p == p_lo) mlo = 0.0L; /* exact pole on the left */
    if (p == p_hi) mhi = 0.0L; /* exact pole on the right */
    for (int it = 0; it < 400; ++it) {
        ld_t mm = 0.5L * (mlo + mhi);
        if (mm == mlo || mm == mhi) break;
        ld_t f = secular(N, a, e, p, mm);
        if (f > 0) mlo = mm;
        else mhi = mm;
    }
    *p_out = p;
    *mu_out = 0.5L * (mlo + mhi);
}

int truth_expm_eigen(int N, double dt, double rho_g, const double *rho_d,
                     const double *t_stop, double *E)
{
    const int n = N + 1;
    if (N < 1 || n > ORC_NMAX) return -1;
    ld_t a[ORC_NMAX], e[ORC_NMAX], w[ORC_NMAX];
    int ord[ORC_NMAX];
    for (int i = 0; i < N; ++i) {
        a[i] = (ld_t)dt / (ld_t)t_stop[i];
        e[i] = (ld_t)rho_d[i] / (ld_t)rho_g;
        if (!(a[i] > 0) || !(e[i] > 0) || !isfinite((double)a[i])) return -1;
        ord[i] = i;
    }
    /* species sorted by a ascending (insertion sort) */
    for (int i = 1; i < N; ++i) {
        int t = ord[i], j = i - 1;
        while (j >= 0 && a[ord[j]] > a[t]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = t;
    }
    for (int i = 1; i < N; ++i)
        if (!(a[ord[i]] > a[ord[i - 1]])) return -1;

    w[0] = 1.0L;
    for (int i = 0; i < N; ++i) w[i + 1] = sqrtl(e[i]);

    /* eigenvectors of S as columns of X (n x n), eigenvalues lam */
    ld_t X[ORC_NMAX][ORC_NMAX], lam[ORC_NMAX];
    /* the conserved mode: lambda = 0, x = w */
    lam[0] = 0.0L;
    for (int j = 0; j < n; ++j) X[j][0] = w[j];

    ld_t sum_ea = 0.0L;
    for (int i = 0; i < N; ++i) sum_ea += e[i] * a[i];
    for (int r = 0; r < N; ++r) {
        /* interval between -a_(r+1) (left) and -a_(r) (right); the last one
         * is (-a_max - sum e a, -a_max) */
        int p_hi = ord[r];
        int p_lo = (r + 1 < N) ? ord[r + 1] : -1;
        ld_t hi = -a[p_hi];
        ld_t lo = (p_lo >= 0) ? -a[p_lo] : -a[p_hi] - sum_ea;
        int p;
        ld_t mu;
        secular_root(N, a, e, lo, hi, p_lo, p_hi, &p, &mu);
        lam[r + 1] = -a[p] + mu;
        X[0][r + 1] = 1.0L;
        for (int i = 0; i < N; ++i) {
            ld_t den = (i == p) ? mu : mu + (a[i] - a[p]);
            X[i + 1][r + 1] = a[i] * sqrtl(e[i]) / den;
        }
    }
    for (int l = 0; l < n; ++l) {
        ld_t nrm2 = 0.0L;
        for (int j = 0; j < n; ++j) nrm2 += X[j][l] * X[j][l];
        ld_t inv = 1.0L / sqrtl(nrm2);
        for (int j = 0; j < n; ++j) X[j][l] *= inv;
    }
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
            ld_t acc = 0.0L;
            for (int l = 0; l < n; ++l) acc += X[j][l] * X[k][l] * expl(lam[l]);
            E[j * n + k] = (double)(acc * w[k] / w[j]);
        }
    return 0;
}

int truth_expm_taylor(int n, const double *A, int terms, double *E)
{
    if (n < 1 || n > ORC_NMAX) return -1;
    ld_t T[ORC_NMAX * ORC_NMAX], U[ORC_NMAX * ORC_NMAX], S[ORC_NMAX * ORC_NMAX];
    for (int i = 0; i < n * n; ++i) { T[i] = 0.0L; S[i] = 0.0L; }
    for (int i = 0; i < n; ++i) { T[i * n + i] = 1.0L; S[i * n + i] = 1.0L; }
    for (int it = 1; it <= terms; ++it) {
        /* T <- T A / it */
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                ld_t acc = 0.0L;
                for (int k = 0; k < n; ++k) acc += T[i * n + k] * (ld_t)A[k * n + j];
                U[i * n + j] = acc / (ld_t)it;
            }
        memcpy(T, U, sizeof(ld_t) * n * n);
        for (int i = 0; i < n * n; ++i) S[i] += T[i];
    }
    for (int i = 0; i < n * n; ++i) E[i] = (double)S[i];
    return 0;
}

/* Modes of the arrowhead system of G species with distinct a_g > 0 and
 * e_g > 0 (the gas is index 0): eigenvalue l of dt K is lam = -a[orig[l]] +
 * mu[l] (orig[l] = -1 for the conserved mode, lam = 0), and
 * E_jk(t) = sum_l c[j][k][l] exp(lam_l t) with
 * c[j][k][l] = X[j][l] X[k][l] w[k] / w[j]. */
static void arrow_modes(int G, const ld_t *a, const ld_t *e, int *orig, ld_t *mu,
                        ld_t X[ORC_NMAX][ORC_NMAX], ld_t *w)
{
    const int n = G + 1;
    int ord[ORC_NMAX];
    for (int i = 0; i < G; ++i) ord[i] = i;
    for (int i = 1; i < G; ++i) {
        int t = ord[i], j = i - 1;
        while (j >= 0 && a[ord[j]] > a[t]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = t;
    }
    w[0] = 1.0L;
    for (int i = 0; i < G; ++i) w[i + 1] = sqrtl(e[i]);
    orig[0] = -1;
    mu[0] = 0.0L;
    for (int j = 0; j < n; ++j) X[j][0] = w[j];
    ld_t sum_ea = 0.0L;
    for (int i = 0; i < G; ++i) sum_ea += e[i] * a[i];
    for (int r = 0; r < G; ++r) {
        int p_hi = ord[r];
        int p_lo = (r + 1 < G) ? ord[r + 1] : -1;
        ld_t hi = -a[p_hi];
        ld_t lo = (p_lo >= 0) ? -a[p_lo] : -a[p_hi] - sum_ea;
        int p;
        ld_t m;
        secular_root(G, a, e, lo, hi, p_lo, p_hi, &p, &m);
        orig[r + 1] = p;
        mu[r + 1] = m;
        X[0][r + 1] = 1.0L;
        for (int i = 0; i < G; ++i) {
            ld_t den = (i == p) ? m : m + (a[i] - a[p]);
            X[i + 1][r + 1] = a[i] * sqrtl(e[i]) / den;
        }
    }
    for (int l = 0; l < n; ++l) {
        ld_t nrm2 = 0.0L;
        for (int j = 0; j < n; ++j) nrm2 += X[j][l] * X[j][l];
        ld_t inv = 1.0L / sqrtl(nrm2);
        for (int j = 0; j < n; ++j) X[j][l] *= inv;
    }
}

/* int_0^1 e^{-b (1 - tau)} e^{lam tau} dtau, with x = lam + b passed
 * separately (formed without cancellation by the caller). */
static ld_t filtered_mode(ld_t lam, ld_t b, ld_t x)
{
    if (fabsl(x) > 0.5L) return (expl(lam) - expl(-b)) / x;
    if (x == 0.0L) return expl(-b);
    return expl(-b) * (expm1l(x) / x);
}

int truth_expm_general(int N, double dt, double rho_g, const double *rho_d,
                       const double *t_stop, double *E)
{
    const int n = N + 1;
    if (N < 1 || n > ORC_NMAX) return -1;
    if (!(dt >= 0) || !isfinite(dt) || !(rho_g > 0) || !isfinite(rho_g)) return -1;
    ld_t a[ORC_NMAX], e[ORC_NMAX];
    for (int i = 0; i < N; ++i) {
        if (!(t_stop[i] > 0) || !(rho_d[i] >= 0) || !isfinite(rho_d[i])) return -1;
        a[i] = (ld_t)dt / (ld_t)t_stop[i]; /* t = inf -> a = 0 */
        e[i] = (ld_t)rho_d[i] / (ld_t)rho_g;
        if (!isfinite((double)a[i])) return -1;
    }
    /* groups of the active species (a > 0, e > 0) by equal a */
    int grp[ORC_NMAX]; /* group of species i, -1 if not active */
    ld_t ag[ORC_NMAX], eg[ORC_NMAX];
    int G = 0;
    for (int i = 0; i < N; ++i) {
        grp[i] = -1;
        if (!(a[i] > 0) || !(e[i] > 0)) continue;
        int g = 0;
        while (g < G && ag[g] != a[i]) ++g;
        if (g == G) { ag[G] = a[i]; eg[G] = 0.0L; ++G; }
        eg[g] += e[i];
        grp[i] = g;
    }
    int orig[ORC_NMAX];
    ld_t mu[ORC_NMAX], X[ORC_NMAX][ORC_NMAX], w[ORC_NMAX], lam[ORC_NMAX], el[ORC_NMAX];
    arrow_modes(G, ag, eg, orig, mu, X, w);
    for (int l = 0; l <= G; ++l) {
        lam[l] = (orig[l] < 0) ? 0.0L : -ag[orig[l]] + mu[l];
        el[l] = expl(lam[l]);
    }
    /* merged-system entry (j, k) over gas = 0 and groups 1..G at t = 1 */
#define MERGED(j, k, acc)                                                    \
    do {                                                                     \
        acc = 0.0L;                                                          \
        for (int l_ = 0; l_ <= G; ++l_) acc += X[j][l_] * X[k][l_] * el[l_]; \
        acc = acc * w[k] / w[j];                                             \
    } while (0)
    for (int i = 0; i < n * n; ++i) E[i] = 0.0;
    ld_t m00;
    MERGED(0, 0, m00);
    E[0] = (double)m00;
    for (int k = 0; k < N; ++k)
        if (grp[k] >= 0) {
            ld_t m0h;
            MERGED(0, grp[k] + 1, m0h);
            E[k + 1] = (double)(m0h * e[k] / eg[grp[k]]);
        }
    for (int i = 0; i < N; ++i) {
        double *row = E + (size_t)(i + 1) * n;
        if (!(a[i] > 0)) { /* decoupled */
            row[i + 1] = 1.0;
            continue;
        }
        if (grp[i] >= 0) { /* active */
            const int g = grp[i];
            ld_t mg0;
            MERGED(g + 1, 0, mg0);
            row[0] = (double)mg0;
            const ld_t dec = expl(-ag[g]);
            for (int k = 0; k < N; ++k) {
                if (grp[k] < 0) continue;
                ld_t mgh;
                MERGED(g + 1, grp[k] + 1, mgh);
                ld_t v = mgh * e[k] / eg[grp[k]];
                if (grp[k] == g) v += dec * ((k == i ? 1.0L : 0.0L) - e[k] / eg[g]);
                row[k + 1] = (double)v;
            }
            continue;
        }
        /* passive: driven by v_g(tau) = sum_l c[0][k][l] e^{lam_l tau} */
        ld_t fl[ORC_NMAX];
        for (int l = 0; l <= G; ++l) {
            ld_t x = (orig[l] < 0) ? a[i] : (a[i] - ag[orig[l]]) + mu[l];
            fl[l] = a[i] * filtered_mode(lam[l], a[i], x);
        }
        ld_t acc = 0.0L;
        for (int l = 0; l <= G; ++l) acc += X[0][l] * X[0][l] * fl[l];
        row[0] = (double)acc;
        for (int k = 0; k < N; ++k) {
            if (grp[k] < 0) continue;
            const int h = grp[k] + 1;
            ld_t c = 0.0L;
            for (int l = 0; l <= G; ++l) c += X[0][l] * X[h][l] * fl[l];
            row[k + 1] = (double)(c * w[h] / w[0] * e[k] / eg[grp[k]]);
        }
        row[i + 1] = (double)expl(-a[i]);
    }
#undef MERGED
    return 0;
}

int truth_apply_cells(int64_t C, int N, int D, int64_t ld, double dt,
                      const double *rho_g, const double *rho_d,
                      const double *t_stop, const double *v_in, double *v_out)
{
    const int n = N + 1;
    if (C < 0 || N < 1 || n > ORC_NMAX || D < 1 || ld < C) return -1;
    double E[ORC_NMAX * ORC_NMAX], rd[ORC_NMAX], ts[ORC_NMAX];
    int bad = 0;
    for (int64_t c = 0; c < C; ++c) {
        for (int i = 0; i < N; ++i) {
            rd[i] = rho_d[(size_t)i * ld + c];
            ts[i] = t_stop[(size_t)i * ld + c];
        }
        int rc = truth_expm_general(N, dt, rho_g[c], rd, ts, E);
        for (int d = 0; d < D; ++d) {
            const double *v = v_in + (size_t)d * n * ld + c;
            double *o = v_out + (size_t)d * n * ld + c;
            int vbad = 0;
            for (int k = 0; k < n; ++k) vbad |= !isfinite(v[(size_t)k * ld]);
            for (int j = 0; j < n; ++j) {
                if (rc != 0 || vbad) {
                    o[(size_t)j * ld] = NAN;
                    continue;
                }
                ld_t acc = 0.0L;
                for (int k = 0; k < n; ++k) acc += (ld_t)E[j * n + k] * (ld_t)v[(size_t)k * ld];
                o[(size_t)j * ld] = (double)acc;
            }
        }
        bad += (rc != 0);
    }
    return bad;
}

/* e^x - e^y over x - y, without cancellation when x and y are close */
static ld_t exp_divdiff(ld_t x, ld_t y)
{
    ld_t d = x - y;
    if (d == 0.0L) return expl(y);
    if (fabsl(d) > 0.5L) return (expl(x) - expl(y)) / d;
    return expl(y) * (expm1l(d) / d);
}

int truth_grad_cells(int64_t C, int N, int D, int64_t ld, double dt,
                     const double *rho_g, const double *rho_d,
                     const double *t_stop, const double *v_in, const double *w_in,
                     double *g_v, double *g_logt, double *g_rho_d, double *g_rho_g)
{
    const int n = N + 1;
    if (C < 0 || N < 1 || n > ORC_NMAX || D < 1 || ld < C) return -1;
    int bad_cells = 0;
    for (int64_t c = 0; c < C; ++c) {
        ld_t a[ORC_NMAX], e[ORC_NMAX];
        int ok = (dt > 0) && isfinite(dt) && (rho_g[c] > 0) && isfinite(rho_g[c]);
        for (int i = 0; i < N && ok; ++i) {
            const double ts = t_stop[(size_t)i * ld + c], rd = rho_d[(size_t)i * ld + c];
            a[i] = (ld_t)dt / (ld_t)ts;
            e[i] = (ld_t)rd / (ld_t)rho_g[c];
            ok = (ts > 0) && (rd > 0) && isfinite(rd) && (a[i] > 0) && isfinite((double)a[i]);
        }
        for (int i = 0; i < N && ok; ++i)
            for (int j = 0; j < i && ok; ++j) ok = (a[i] != a[j]);
        for (int d = 0; d < D && ok; ++d)
            for (int j = 0; j < n && ok; ++j)
                ok = isfinite(v_in[((size_t)d * n + j) * ld + c]) &&
                     isfinite(w_in[((size_t)d * n + j) * ld + c]);
        if (!ok) {
            ++bad_cells;
            for (int d = 0; d < D; ++d)
                for (int j = 0; j < n; ++j) g_v[((size_t)d * n + j) * ld + c] = NAN;
            for (int i = 0; i < N; ++i) {
                g_logt[(size_t)i * ld + c] = NAN;
                g_rho_d[(size_t)i * ld + c] = NAN;
            }
            g_rho_g[c] = NAN;
            continue;
        }
        int orig[ORC_NMAX];
        ld_t mu[ORC_NMAX], X[ORC_NMAX][ORC_NMAX], w[ORC_NMAX], lam[ORC_NMAX], el[ORC_NMAX];
        arrow_modes(N, a, e, orig, mu, X, w);
        for (int l = 0; l < n; ++l) {
            lam[l] = (orig[l] < 0) ? 0.0L : -a[orig[l]] + mu[l];
            el[l] = expl(lam[l]);
        }
        /* E (for dL/dv = E^T w) and G = sum_d w_d v_d^T */
        ld_t E[ORC_NMAX][ORC_NMAX], G[ORC_NMAX][ORC_NMAX];
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                ld_t acc = 0.0L;
                for (int l = 0; l < n; ++l) acc += X[j][l] * X[k][l] * el[l];
                E[j][k] = acc * w[k] / w[j];
                ld_t g = 0.0L;
                for (int d = 0; d < D; ++d)
                    g += (ld_t)w_in[((size_t)d * n + j) * ld + c] *
                         (ld_t)v_in[((size_t)d * n + k) * ld + c];
                G[j][k] = g;
            }
        for (int d = 0; d < D; ++d)
            for (int k = 0; k < n; ++k) {
                ld_t acc = 0.0L;
                for (int j = 0; j < n; ++j) acc += E[j][k] * (ld_t)w_in[((size_t)d * n + j) * ld + c];
                g_v[((size_t)d * n + k) * ld + c] = (double)acc;
            }
        /* H = X^T (W^-1 G W) X, then Phi o H, then back: L = X (Phi o H) X^T */
        ld_t T1[ORC_NMAX][ORC_NMAX], H[ORC_NMAX][ORC_NMAX], L[ORC_NMAX][ORC_NMAX];
        for (int j = 0; j < n; ++j)
            for (int m = 0; m < n; ++m) {
                ld_t acc = 0.0L;
                for (int k = 0; k < n; ++k) acc += (G[j][k] * w[k] / w[j]) * X[k][m];
                T1[j][m] = acc;
            }
        for (int l = 0; l < n; ++l)
            for (int m = 0; m < n; ++m) {
                ld_t acc = 0.0L;
                for (int j = 0; j < n; ++j) acc += X[j][l] * T1[j][m];
                H[l][m] = acc * exp_divdiff(lam[l], lam[m]);
            }
        for (int l = 0; l < n; ++l)
            for (int k = 0; k < n; ++k) {
                ld_t acc = 0.0L;
                for (int m = 0; m < n; ++m) acc += H[l][m] * X[k][m];
                T1[l][k] = acc;
            }
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                ld_t acc = 0.0L;
                for (int l = 0; l < n; ++l) acc += X[j][l] * T1[l][k];
                L[j][k] = acc * w[j] / w[k]; /* Abar */
            }
        ld_t grg = 0.0L;
        for (int i = 0; i < N; ++i) {
            const ld_t ga = L[0][i + 1] * e[i] + L[i + 1][0] - L[i + 1][i + 1] - L[0][0] * e[i];
            const ld_t ge = a[i] * (L[0][i + 1] - L[0][0]);
            g_logt[(size_t)i * ld + c] = (double)(-a[i] * ga);
            g_rho_d[(size_t)i * ld + c] = (double)(ge / (ld_t)rho_g[c]);
            grg -= ge * e[i] / (ld_t)rho_g[c];
        }
        g_rho_g[c] = (double)grg;
    }
    return bad_cells;
}
