/*
 * rk1.c -- oracle of the first-order implicit drag step (test infrastructure).
 *
 * The implicit RK1 (backward Euler) step of the drag ODE alone solves
 *     (I - dt K) v' = v
 * per cell and velocity component (the linear system of the paper's
 * appendix on implicit solvers, eq. analytic_1, written for velocities).
 * The oracle is that definition: the dense (N+1) x (N+1) matrix I - dt K
 * built from orc_build's dt K, solved by Gaussian elimination with partial
 * pivoting.  Any elimination order subtracts nearly equal numbers when the
 * identity is tiny against dt K (stiff cells: the Schur complement of the
 * gas row is 1 + sum_i p_i / (1 + a_i), formed from terms of size sum_i p_i),
 * so the forward error is about u cond(I - dt K), 1e6 and more here.  The
 * elimination therefore runs in binary128 (__float128, u = 2^-113) and the
 * result is rounded once to double: the oracle is the exact solution of the
 * system to the last bit.
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
    quad M[ORC_NMAX * ORC_NMAX], x[ORC_NMAX];
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
                /* I - dt K from the doubles of dt K (a_i, p_i as the method
                 * rounds them), then exact in binary128 */
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j)
                        M[i * n + j] = (quad)(i == j ? 1.0 : 0.0) - (quad)A[i * n + j];
                ok = gauss_solve(n, M, x) == 0;
            }
            for (int j = 0; j < n; ++j) v_out[(d * n + j) * ld + c] = ok ? (double)x[j] : NAN;
        }
        status |= bad;
    }
    return status;
}
