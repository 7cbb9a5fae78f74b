/*
 * rk1.c -- oracle of the first-order implicit drag step (test infrastructure).
 *
 * The implicit RK1 (backward Euler) step of the drag ODE alone solves
 *     (I - dt K) v' = v
 * per cell and velocity component (the linear system of the paper's
 * appendix on implicit solvers, eq. analytic_1, written for velocities).
 * The oracle is that definition: the dense (N+1) x (N+1) matrix I - dt K,
 * solved by Gaussian elimination with partial pivoting, all in binary128
 * (__float128, u = 2^-113) and rounded once to double.  The matrix is built
 * in binary128 from the inputs themselves (a_i = dt / t_i, e_i = rho_i /
 * rho_g, p_i = e_i a_i, the gas diagonal -sum_i p_i), not from dt K rounded
 * to double: in a stiff cell a double A00 is off by u sum_i p_i, which moves
 * the conserved mode of the solution by about u ||dt K|| (1e-10 at
 * ||dt K|| = 1e6), and any elimination in double loses u cond(I - dt K) the
 * same way.  With the exact entries the oracle is the solution of the
 * backward Euler step itself, conserving rho_g v_g + sum_i rho_i v_i to the
 * last bit.  Bad cells are detected by orc_build, as for the exponential.
 * The O(N) closed form the paper derives for this arrowhead system is what
 * the GPU kernel computes; it is not used here.
 */
#include <math.h>
#include <stdlib.h>

#include "oracle.h"

typedef __float128 quad;

static quad qabs(quad x) { return x < 0 ? -x : x; }

/* Solve M x = b in place (b <- x) for the n x n row-major M (destroyed).
 * Returns 0, or -1 for a zero pivot. */
static int gauss_solve(int n, quad *M, quad *b)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (qabs(M[i * n + k]) > qabs(M[p * n + k])) p = i;
        if (M[p * n + k] == 0) return -1;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                quad t = M[k * n + j];
                M[k * n + j] = M[p * n + j];
                M[p * n + j] = t;
            }
            quad t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            quad f = M[i * n + k] / M[k * n + k];
            for (int j = k; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
            b[i] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        quad s = b[k];
        for (int j = k + 1; j < n; ++j) s -= M[k * n + j] * b[j];
        b[k] = s / M[k * n + k];
    }
    return 0;
}

/* v_out = (I - dt K)^{-1} v_in for C cells, SoA layout as orc_apply_cells.
 * Returns the OR of the bad-input bits; a bad cell's outputs are NaN. */
int orc_rk1_cells(int64_t C, int N, int D, int64_t ld, double dt,
                  const double *rho_g, const double *rho_d,
                  const double *t_stop, const double *v_in, double *v_out)
{
    const int n = N + 1;
    if (n > ORC_NMAX || D < 1 || D > 3 || ld < C) return -1;
    double A[ORC_NMAX * ORC_NMAX];
    quad M[ORC_NMAX * ORC_NMAX], x[ORC_NMAX], qa[ORC_NMAX], qp[ORC_NMAX];
    double rd[ORC_NMAX], ts[ORC_NMAX], a[ORC_NMAX], e[ORC_NMAX];
    int status = 0;
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
        for (int d = 0; d < D; ++d) {
            for (int j = 0; j < n; ++j) x[j] = v_in[(d * n + j) * ld + c];
            int ok = !bad;
            if (ok) {
                /* I - dt K with the entries taken in binary128 from the
                 * inputs (t_i = +inf gives a_i = 0) */
                quad sp = 0;
                for (int i = 0; i < N; ++i) {
                    qa[i] = (quad)dt / (quad)ts[i];
                    qp[i] = (quad)rd[i] / (quad)rho_g[c] * qa[i];
                    sp += qp[i];
                }
                for (int k = 0; k < n * n; ++k) M[k] = 0;
                M[0] = 1 + sp;
                for (int i = 1; i < n; ++i) {
                    M[i] = -qp[i - 1];
                    M[i * n] = -qa[i - 1];
                    M[i * n + i] = 1 + qa[i - 1];
                }
                ok = gauss_solve(n, M, x) == 0;
            }
            for (int j = 0; j < n; ++j) v_out[(d * n + j) * ld + c] = ok ? (double)x[j] : NAN;
        }
        status |= bad;
    }
    return status;
}
