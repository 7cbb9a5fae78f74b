/*
 * dragexp.h -- C ABI of the MI355X (gfx950) drag-update library.
 *
 * For every cell of a grid the library advances the gas and N dust velocities
 * through one drag step,
 *
 *     v(t + dt) = exp(dt K) v,
 *
 * the exact solution of the linear drag ODE of Sewanou, Laibe and Commercon
 * (arXiv:2509.25347), Sect. 2.2, eqs. DragEq-jacobian and ExacSolEqu, written
 * for velocities: dv_i/dt = -(v_i - v_g)/t_i for dust species i and
 * dv_g/dt = sum_i (rho_i/rho_g)(v_i - v_g)/t_i for the gas.  The exponential
 * is the Taylor scaling-and-squaring approximant of Sect. 2.3 and Appendix B
 * (Alg. 1 option `option`, at most `k_max` products in the polynomial stage),
 * accurate to the IEEE double unit round-off u = 2^-53 in the backward sense
 * (eqs. B1-B8).  All arithmetic is FP64.
 *
 * Memory layout (structure of arrays, the cell index fastest, leading
 * dimension ld >= n_cells, all in elements):
 *     rho_g  [C]                 gas density                  rho_g[c]
 *     rho_d  [N][ld]             dust densities               rho_d[i*ld + c]
 *     t_stop [N][ld]             stopping times T_s,i         t_stop[i*ld + c]
 *     v      [D][N+1][ld]        velocities, row 0 = gas      v[(d*(N+1) + j)*ld + c]
 * with N = n_species in [1, 16] and D = n_dim in [1, 3]; the D components
 * share one matrix K.  drag_build, drag_expm_apply and drag_expm_steps also
 * take N = 17..32 (a large-N kernel: one cell per wavefront on 2 x 2 blocks
 * of MFMA tiles, the plain Taylor step, K_AUTO = 7; built for cases such as
 * the paper's 20-species Collisions test, not tuned); the other calls
 * return DRAG_ERR_N_SPECIES above 16.
 *
 * Ownership and synchronisation: every array pointer is a device pointer
 * owned by the caller, in memory of the current device (hipSetDevice), where
 * the kernels run; `stream` must belong to that device too (neither is
 * checked: a pointer of another device is read across the fabric or faults).
 * drag_build, drag_expm_apply, drag_expm_apply_backward and
 * drag_clear_status only enqueue work on `stream` (a hipStream_t; NULL is
 * the null stream): they never allocate device memory, never synchronise, and
 * return before the work is done.  drag_get_status and drag_plan_autotune
 * synchronise `stream`; the batched plan calls allocate and free the plan's
 * own device tables and graph (drag_plan_batched, drag_plan_destroy, and a
 * re-capture inside drag_expm_apply_batched when the pointers change).
 *
 * Errors: a negative return value is an argument error found on the host
 * before anything was enqueued.  Invalid per-cell data (rho_g not finite or
 * <= 0; rho_d not finite or < 0; t_stop NaN or <= 0; a velocity not finite;
 * ||dt K||_1 overflowing) is not an argument error: that cell's outputs are
 * NaN and the matching DRAG_CELL_* bit is ORed into a per-device sticky
 * status word (drag_get_status / drag_clear_status).  t_stop = +inf is valid
 * (a decoupled species); rho_d = 0 is valid (no back-reaction).
 */
#ifndef DRAGEXP_H
#define DRAGEXP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------- */
#define DRAG_OK                 0
#define DRAG_ERR_NULL_DESC     -1  /* desc pointer is NULL */
#define DRAG_ERR_N_CELLS       -2  /* n_cells < 0 */
#define DRAG_ERR_N_SPECIES     -3  /* n_species outside [1, 16] */
#define DRAG_ERR_N_DIM         -4  /* n_dim outside [1, 3] */
#define DRAG_ERR_LD            -5  /* ld < n_cells, or ld too large for 64-bit offsets */
#define DRAG_ERR_DT            -6  /* dt NaN, infinite or < 0 */
#define DRAG_ERR_K_MAX         -7  /* k_max outside [0, 9] */
#define DRAG_ERR_OPTION        -8  /* option not 0, 1 or 2 (| DRAG_OPTION_BOUND_TEST
                                      where accepted) */
#define DRAG_ERR_NULL_POINTER  -9  /* a required array pointer is NULL (n_cells > 0) */
#define DRAG_ERR_ALIAS        -10  /* an output overlaps an input it may not alias */
#define DRAG_ERR_PLAN         -11  /* invalid batched plan or block table */
#define DRAG_ERR_STEPS        -12  /* n_steps < 0 (drag_expm_steps) */
#define DRAG_ERR_SCRATCH      -13  /* the batch's tables exceed the static buffer
                                      (drag_expm_apply_batched_static) */
#define DRAG_ERR_HIP          -20  /* the HIP runtime reported an error */

/* per-cell bits of the sticky device status word */
#define DRAG_CELL_BAD_DENSITY       1
#define DRAG_CELL_BAD_STOPPING_TIME 2
#define DRAG_CELL_BAD_VELOCITY      4
#define DRAG_CELL_BAD_NORM          8

/* k_max = DRAG_K_AUTO: the Taylor cap K is the library's per-N choice */
#define DRAG_K_AUTO 0

/* an opaque hipStream_t */
typedef void *drag_stream_t;

typedef struct drag_desc {
    int64_t n_cells;   /* C >= 0; C = 0 is a no-op */
    int32_t n_species; /* N in [1, 16]; up to 32 for the forward calls */
    int32_t n_dim;     /* D in [1, 3] */
    int64_t ld;        /* leading dimension of every [.][ld] array, >= C */
    double dt;         /* finite, >= 0; dt = 0 returns v unchanged (every value
                          equal; a -0.0 entry may come back as +0.0) */
    int32_t k_max;     /* K of Alg. 1, 1..9 (9: m up to 30, Table B.1), or
                          DRAG_K_AUTO: the library's tuned K for n_species
                          (drag_get_k_max) */
    int32_t option;    /* Alg. 1 option: 0 standard, 1, 2 (fewest products),
                          optionally ORed with DRAG_OPTION_BOUND_TEST */
} drag_desc;

/*
 * option bit: Sastre's second modification in the Taylor stage (Appendix B,
 * eqs. Pat_Stk4-Pat_Stk7, the bound b_exp of eq. Pat_Stk6 and the
 * evaluation with the bound test): a Horner product of the Paterson-
 * Stockmeyer evaluation is skipped when the accumulated higher-degree part
 * it would carry is below u relative to the estimate b_exp of ||e^-A||.
 * drag_expm_apply and drag_expm_steps then run the MFMA kernel for every N
 * (the test works on the kernel's own Paterson-Stockmeyer blocks of the
 * reduced N x N matrix); drag_build ignores the bit; the adjoint and the
 * batched plan reject it (DRAG_ERR_OPTION).  Results stay u-accurate; the
 * products saved are data-dependent (none on the stiff N = 16 workload).
 */
#define DRAG_OPTION_BOUND_TEST 4

/*
 * option bit: the diagonal (m, m) Pade approximant of Sect. 2.3 (eq.
 * PadeEqu, p = q = m) as the scaling step instead of the Taylor polynomial:
 * m in {3, 5, 7, 9, 13} is the lowest degree whose theta_m covers
 * ||dt K||_1, else m = 13 with the smallest s such that ||dt K||_1 / 2^s <=
 * theta_13 (theta_m: the largest theta for which the backward error of r_m
 * is below u, the criterion of eq. B8; drag_pade_row).  Each cell solves
 * D_mm Z = N_mm - D_mm on its 16 x 16 tile (Gauss-Jordan with partial
 * pivoting over the wavefront).  drag_expm_apply and drag_expm_steps run
 * the MFMA kernel for every N; drag_build reports (k, m, s) = (0, m, s);
 * the adjoint and the batched plan reject it, and so does combining it with
 * DRAG_OPTION_BOUND_TEST (DRAG_ERR_OPTION).  Alg. 1's option bits and k_max
 * are not used.
 */
#define DRAG_OPTION_PADE 8

/* Fill `d` with the defaults: k_max = 9, option = 2, ld = n_cells. */
void drag_desc_init(drag_desc *d, int64_t n_cells, int32_t n_species,
                    int32_t n_dim, double dt);

/*
 * drag_build -- the per-cell quantities of the method (Sect. 2.2 eqs.
 * DragEqVar2-3; Appendix B, Alg. 1):
 *   a_out[i*ld + c] = dt / t_i           (IEEE-rounded division)
 *   e_out[i*ld + c] = rho_i / rho_g
 *   norm_out[c]     = ||dt K||_1: the largest column sum of |dt K| in the
 *                     velocity form, the gas column summed gas row first and
 *                     then the species in ascending order, without fused
 *                     multiply-adds (so it is reproducible bit for bit)
 *   k_out, m_out, s_out [c]: (k*, m*, s*) of Alg. 1 for that norm.
 * Any output pointer may be NULL (not computed).  Bad cells get NaN
 * a/e/norm and k = m = s = 0.
 */
int drag_build(const drag_desc *desc, const double *rho_g, const double *rho_d,
               const double *t_stop, double *a_out, double *e_out,
               double *norm_out, int32_t *k_out, int32_t *m_out,
               int32_t *s_out, drag_stream_t stream);

/*
 * drag_expm_apply -- v_out = exp(dt K) v_in for every cell (Sect. 2.2 eq.
 * ExacSolEqu; Sect. 2.3; Appendix B Alg. 1 and the Taylor evaluation).
 * v_out may be the same pointer as v_in (in place); any other overlap of
 * v_out with an input is DRAG_ERR_ALIAS.
 */
int drag_expm_apply(const drag_desc *desc, const double *rho_g,
                    const double *rho_d, const double *t_stop,
                    const double *v_in, double *v_out, drag_stream_t stream);

/*
 * drag_expm_steps -- n_steps successive drag steps of the same dt, as a time
 * integration of the drag ODE alone (the Collisions test of Sect. 3: gas
 * and dust relaxing toward the common centre-of-mass velocity), each step
 * the drag_expm_apply update of the state the previous step left:
 *     v_out = E^n_steps v_in,  E = the approximant of exp(dt K).
 *   history [n_steps][D][N+1][ld] or NULL: the state after every step
 *           (history[i] after step i + 1); must not overlap any other array.
 * v_out may equal v_in.  n_steps = 0 copies v_in to v_out.  The steps are
 * n_steps launches on `stream` (no synchronisation); DRAG_ERR_STEPS for
 * n_steps < 0.
 */
int drag_expm_steps(const drag_desc *desc, const double *rho_g,
                    const double *rho_d, const double *t_stop,
                    const double *v_in, double *v_out, int64_t n_steps,
                    double *history, drag_stream_t stream);

/*
 * drag_rk1_apply -- the first-order implicit (backward Euler) drag step, the
 * cost and accuracy yardstick the paper compares the exponential with
 * (Sect. 4, Fig. 6; appendix on implicit solvers, eqs. analytic_1 to
 * analytic_4):
 *     v_out = (I - dt K)^-1 v_in
 * for every cell and velocity component, by the O(N) closed form of that
 * arrowhead system (one cell per lane; bound by HBM bandwidth).  Same
 * layout, aliasing rules, bad-cell flags and NaN outputs as drag_expm_apply;
 * desc->k_max and desc->option are validated but not used.  dt = 0 returns v
 * unchanged (as for drag_expm_apply); a species with t_i = +inf keeps its
 * velocity.
 * The result is first-order accurate in dt (||v_out - exp(dt K) v_in|| is
 * O(dt^2) per step) and relaxes to the barycentric velocity as dt/t_i grows.
 */
int drag_rk1_apply(const drag_desc *desc, const double *rho_g,
                   const double *rho_d, const double *t_stop,
                   const double *v_in, double *v_out, drag_stream_t stream);

/*
 * drag_expm_apply_backward -- the adjoint of drag_expm_apply for the loss
 * L = sum_{d,j,c} grad_v_out[d][j][c] * v_out[d][j][c] (the chain rule of a
 * training step: grad_v_out = dL/dv_out).  The exponential is differentiated
 * with (k*, m*, s*) held fixed, as the Frechet derivative of the same Taylor
 * scaling-and-squaring approximant (Sect. 2.3, Appendix B); nothing is
 * stored between forward and backward: the Taylor stage and the squaring
 * chain are recomputed alongside their derivatives.
 *   v_out       [D][N+1][ld] or NULL: the forward result (fused forward)
 *   grad_v_in   [D][N+1][ld] or NULL: dL/dv_in
 *   grad_log_t  [N][ld] or NULL:      dL/d(log t_i)
 *   grad_t_stop [N][ld] or NULL:      dL/d t_i  (= dL/d(log t_i) / t_i)
 *   grad_rho_d  [N][ld] or NULL:      dL/d rho_i
 *   grad_rho_g  [C] or NULL:          dL/d rho_g
 * No output may overlap an input or another output.  Bad cells get NaN in
 * every output, as in drag_expm_apply.
 */
int drag_expm_apply_backward(const drag_desc *desc, const double *rho_g,
                             const double *rho_d, const double *t_stop,
                             const double *v_in, const double *grad_v_out,
                             double *v_out, double *grad_v_in,
                             double *grad_log_t, double *grad_t_stop,
                             double *grad_rho_d, double *grad_rho_g,
                             drag_stream_t stream);

/* ---- batched blocks with uneven species counts -------------------------- */
/*
 * The paper's Dyablo implementation divides the grid into blocks of cells and
 * runs one data-parallel loop per block (Sect. 3.4, Performance); here a
 * batch is n_blocks blocks of block_cells cells (AMR-style blocks), block b
 * with its own species count N_b in [1, 16].  Block b's fields are one
 * contiguous slab of the caller's `fields` buffer starting at element
 * field_offset[b] (as returned by drag_plan_offsets):
 *     rho_g [block_cells] | rho_d [N_b][block_cells] | t_stop [N_b][block_cells]
 * and its velocities one slab of `v` starting at v_offset[b]:
 *     v [D][N_b + 1][block_cells].
 * The plan (created once, on the host and the current device) holds the
 * device block table, the launch configuration chosen per N by the
 * autotuner, and an instantiated hipGraph of the whole update: the lane
 * grids and the MFMA launches as two concurrent branches.
 */
typedef struct drag_plan drag_plan;

typedef struct drag_batch_desc {
    int32_t n_blocks;         /* >= 1 */
    int32_t block_cells;      /* cells per block, >= 1 */
    int32_t n_dim;            /* D in [1, 3] */
    int32_t k_max;            /* 1..9 for every block, or DRAG_K_AUTO: per N,
                                 drag_get_k_max at plan creation, then the
                                 autotuner's choice (drag_plan_k_max) */
    int32_t option;           /* 0, 1, 2 */
    double dt;                /* finite, >= 0 */
    const int32_t *n_species; /* host array [n_blocks], each in [1, 16] */
} drag_batch_desc;

int drag_plan_batched(const drag_batch_desc *desc, drag_plan **out);
/* Element offsets of every block's slabs and the total buffer sizes. */
int drag_plan_offsets(const drag_plan *plan, int64_t *field_offset,
                      int64_t *v_offset, int64_t *fields_total,
                      int64_t *v_total);
/* v_out may equal v_in; otherwise no overlap.  Replays the plan's graph
 * when the pointers match the captured ones, else updates it first. */
int drag_expm_apply_batched(drag_plan *plan, const double *fields,
                            const double *v_in, double *v_out,
                            drag_stream_t stream);
/* Time every launch configuration of the plan on the caller's data (lane
 * bound x MFMA form, the Taylor and the Pade per-N grids included; each
 * run computes the full, valid result into v_out, then synchronises
 * `stream`), keep the fastest, and report its lane-mapping bound: blocks
 * with N_b <= *lane_max_out run one cell per lane, the others on the FP64
 * MFMA path (a quad of cells per wavefront) in the form that timed fastest
 * (drag_plan_config).  A DRAG_K_AUTO plan then also times each species
 * count's launch for every Taylor cap K = 3..9 and keeps the fastest per N
 * (drag_plan_k_max); v_out ends with the chosen configuration's result.
 * The next drag_expm_apply_batched re-captures. */
int drag_plan_autotune(drag_plan *plan, const double *fields,
                       const double *v_in, double *v_out,
                       drag_stream_t stream, int32_t *lane_max_out);
/* The plan's current launch configuration: the lane-mapping bound and how
 * the MFMA branch runs: DRAG_MFMA_PERSISTENT (a persistent grid over a work
 * queue of a few cells per item), DRAG_MFMA_GRID (one plain grid over its
 * blocks, N at run time), DRAG_MFMA_PER_N (one plain grid per species
 * count, each compiled for it) or DRAG_MFMA_PER_N_PADE (the same grids with
 * the diagonal Pade scaling step of Sect. 2.3, eq. PadeEqu, instead of the
 * Taylor one: those blocks then give drag_expm_apply's result with option
 * DRAG_OPTION_PADE, bit for bit; the plan's k_max and option do not apply to
 * them).  Either pointer may be NULL. */
#define DRAG_MFMA_PERSISTENT 0
#define DRAG_MFMA_GRID 1
#define DRAG_MFMA_PER_N 2
#define DRAG_MFMA_PER_N_PADE 3
int drag_plan_config(const drag_plan *plan, int32_t *lane_max,
                     int32_t *mfma_mode);
/* Pin a launch configuration instead of the tuned one: lane_max in 4..12 and
 * an mfma_mode above (DRAG_ERR_OPTION otherwise, the plan unchanged).  The
 * next drag_expm_apply_batched re-captures; results do not depend on it. */
int drag_plan_set_config(drag_plan *plan, int32_t lane_max, int32_t mfma_mode);
/* The Taylor cap K each species count runs with (k_max[N - 1], N = 1..16).
 * A block of N_b species gives exactly drag_expm_apply's result with
 * k_max = k_max[N_b - 1] and the same mapping. */
int drag_plan_k_max(const drag_plan *plan, int32_t *k_max);
int drag_plan_destroy(drag_plan *plan);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the batched
 * update of `desc` without a plan, allocating nothing.  The blocks are laid
 * out as drag_plan_offsets reports for a plan of the same desc.  The result
 * is bit for bit that of drag_expm_apply_batched on such a plan pinned to
 * drag_plan_set_config(plan, 10, DRAG_MFMA_PER_N) (one lane per cell to 8
 * species, two lanes per cell for 9 and 10, one MFMA grid per species count
 * above), every block with the Taylor cap desc->k_max (DRAG_K_AUTO: the
 * cap drag_get_k_max gives its species count; no tuning).
 *
 * The block offsets and work items (16 bytes per block, plus 16 bytes per
 * 64-cell item of blocks with N_b <= 8, per 32-cell item of blocks with
 * N_b = 9, 10, and per block above) live in a static device buffer of
 * DRAG_STATIC_SCRATCH_BYTES that every GPU the library runs on holds until
 * the process ends; a batch whose tables do not fit returns DRAG_ERR_SCRATCH
 * before anything is enqueued (4096 blocks of 512 cells take about 0.5 MiB).
 * Each call copies its tables from host memory into that buffer on `stream`,
 * then enqueues the kernels on `stream`; it neither synchronises nor creates
 * streams, events or graphs.  Every call on one GPU shares that GPU's buffer:
 * calls that overlap on one GPU (different streams, or host threads racing)
 * overwrite each other's tables, so serialise them (for instance on one
 * stream).  Calls from several host threads of one process are serialised on
 * the host.  Errors as drag_expm_apply_batched, plus DRAG_ERR_SCRATCH.
 */
#define DRAG_STATIC_SCRATCH_BYTES (1u << 20)
int drag_expm_apply_batched_static(const drag_batch_desc *desc,
                                   const double *fields, const double *v_in,
                                   double *v_out, drag_stream_t stream);

/* ---- status and introspection -------------------------------------------- */
/* Synchronise `stream`, then read the current device's sticky status word. */
int drag_get_status(drag_stream_t stream, int32_t *host_status);
/* Enqueue a reset of the current device's status word on `stream`. */
int drag_clear_status(drag_stream_t stream);
const char *drag_status_string(int code);

/* Row k (1..9) of the library's copy of Table B.1 (Appendix B). */
int drag_table_row(int k, int32_t *m, int32_t *q, int32_t *r, double *theta);
/* Row 0..4 of the Pade scaling step's table: degree m, theta_m and the
 * numerator coefficients c_0..c_m (coef may be NULL; the denominator's are
 * (-1)^j c_j).  DRAG_ERR_OPTION for another row. */
int drag_pade_row(int32_t row, int32_t *m, double *theta, double *coef);
/* (k*, m*, s*) of Alg. 1 for a finite norm, computed on the host by the same
 * code the kernels run. */
int drag_select(double norm, int32_t k_max, int32_t option, int32_t *k,
                int32_t *m, int32_t *s);

/* ---- launch tuning ------------------------------------------------------------ */
/* The per-N mapping used by drag_expm_apply, drag_expm_apply_backward and
 * the batched plan (for species count n_species, host-side, per process; the
 * setters, like drag_set_k_max, are not synchronised: set them before
 * launching from several host threads):
 *   DRAG_MAP_LANE  vector ALU: one cell per lane for N <= 8, one cell per
 *                  pair of lanes for the forward at N = 9..12 (the adjoint:
 *                  one lane to N = 7, a pair at 8..10, and the MFMA kernel
 *                  above 10);
 *   DRAG_MAP_WAVE  FP64 MFMA: four cells per 64-lane wavefront, one
 *                  exponential at a time on 16 x 16 tiles (the adjoint for
 *                  N <= 8 on one tile holding the 2N x 2N block form);
 *   DRAG_MAP_AUTO  the measured default (the forward: lane to N = 12, MFMA
 *                  above; the adjoint: lane to N = 10).
 * DRAG_ERR_OPTION for an unknown mapping or LANE with N > 12.
 * drag_get_mapping reports the forward's mapping. */
#define DRAG_MAP_AUTO 0
#define DRAG_MAP_LANE 1
#define DRAG_MAP_WAVE 2
/* The Taylor cap K that DRAG_K_AUTO stands for, per species count (host-side,
 * per process).  Every K gives an approximant accurate to u (Alg. 1 keeps
 * ||dt K / 2^s||_1 <= theta_m); K trades polynomial degree against
 * squarings.  The defaults were measured on MI355X (2^18 cells per N): K = 3
 * or 4 for N <= 4, 5 for N = 5-6, 6 for N = 7-12 (0.72-0.99 of the time at
 * K = 9 on the vector-ALU kernels), 7 for N >= 13 (the MFMA kernel).  drag_set_k_max(N, 0)
 * restores the default; DRAG_ERR_N_SPECIES / DRAG_ERR_K_MAX otherwise. */
int drag_set_k_max(int32_t n_species, int32_t k_max);
int drag_get_k_max(int32_t n_species, int32_t *k_max);
int drag_set_mapping(int32_t n_species, int32_t mapping);
int drag_get_mapping(int32_t n_species, int32_t *mapping);

#ifdef __cplusplus
}
#endif

#endif /* DRAGEXP_H */
