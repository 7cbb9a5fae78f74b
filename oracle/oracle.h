/*
 * oracle.h -- interface of the CPU reference (test infrastructure only).
 *
 * Used by the tests, the smoke check and the benchmark's CPU-baseline leg
 * through ctypes.  Never included by the HIP library.
 */
#ifndef DRAG_ORACLE_H
#define DRAG_ORACLE_H

#include <stdint.h>

/* option bit: Sastre's second modification (the bound test) in the Taylor
 * stage of orc_expm / orc_cell_expm / orc_apply_cells */
#define ORC_BOUND_TEST 4
/* option bit: the diagonal Pade scaling step (eq. PadeEqu) instead of Taylor */
#define ORC_PADE 8

#define ORC_NMAX 33 /* largest n = N+1 the oracle handles (N <= 32) */

/* bad-input bits of a cell; the cell's outputs are NaN when any is set */
#define ORC_BAD_DENSITY       1 /* rho_g not finite or <= 0, rho_d not finite or < 0 */
#define ORC_BAD_STOPPING_TIME 2 /* t_i NaN or <= 0 (t_i = +inf is valid: a_i = 0) */
#define ORC_BAD_VELOCITY      4 /* a velocity (or loss weight) not finite */
#define ORC_BAD_NORM          8 /* an entry or the 1-norm of dt K overflowed */

int orc_table_row(int k, int *m, int *q, int *r, double *theta);
double orc_taylor_coef(int i);
void orc_select(double nrm, int K, int option, int *k, int *m, int *s);
int orc_build(int N, double dt, double rho_g, const double *rho_d,
              const double *t_stop, double *A, double *a, double *e,
              double *nrm);
int orc_expm(int N, const double *A, double nrm, int K, int option, int xform,
             double *Y, int *kms);
int orc_cell_expm(int N, double dt, double rho_g, const double *rho_d,
                  const double *t_stop, int K, int option, int xform,
                  double *E, int *kms);
int orc_pade_row(int i, int *m, double *theta, double *coef);
void orc_pade_select(double nrm, int *mout, int *sout);
int orc_taylor_stage(int n, const double *B, int k, int bound_test, double *F,
                     int *skipped, double *bexp_out);
int orc_apply_cells(int64_t C, int N, int D, int64_t ld, double dt, int K,
                    int option, int xform, const double *rho_g,
                    const double *rho_d, const double *t_stop,
                    const double *v_in, double *v_out, int32_t *kms,
                    double *nrm_out);
int orc_grad_A(int N, const double *A, double nrm, int K, int option,
               const double *G, double *Abar, int *kms);
int orc_grad_cells(int64_t C, int N, int D, int64_t ld, double dt, int K,
                   int option, const double *rho_g, const double *rho_d,
                   const double *t_stop, const double *v_in, const double *w_in,
                   double *v_out, double *g_v, double *g_logt,
                   double *g_rho_d, double *g_rho_g);

/* independent truths, long double (truth.c) */
/* rk1.c: the implicit RK1 drag step v' = (I - dt K)^{-1} v (dense solve) */
int orc_rk1_cells(int64_t C, int N, int D, int64_t ld, double dt,
                  const double *rho_g, const double *rho_d,
                  const double *t_stop, const double *v_in, double *v_out);
int truth_expm_eigen(int N, double dt, double rho_g, const double *rho_d,
                     const double *t_stop, double *E);
int truth_expm_taylor(int n, const double *A, int terms, double *E);
int truth_expm_general(int N, double dt, double rho_g, const double *rho_d,
                       const double *t_stop, double *E);
int truth_apply_cells(int64_t C, int N, int D, int64_t ld, double dt,
                      const double *rho_g, const double *rho_d,
                      const double *t_stop, const double *v_in, double *v_out);
int truth_grad_cells(int64_t C, int N, int D, int64_t ld, double dt,
                     const double *rho_g, const double *rho_d,
                     const double *t_stop, const double *v_in, const double *w_in,
                     double *g_v, double *g_logt, double *g_rho_d, double *g_rho_g);

#endif
