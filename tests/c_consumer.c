/*
 * c_consumer.c -- the C ABI of include/dragexp.h driven from plain C, with no
 * Python in the loop (test infrastructure: it also links the CPU oracle to
 * check the result).
 *
 *   c_consumer --host-only          argument errors and host-side calls only
 *   c_consumer N C D SEED           one drag_expm_apply on the GPU against
 *                                   the oracle; prints "max_err <e>"
 *
 * Inputs are drawn with splitmix64 (a counter-based generator, Steele, Lea and
 * Flood 2014): rho_g ~ U[0.5, 2], eps_i ~ 10^U[-3, 0] with rho_i = eps_i rho_g,
 * t_i ~ 10^U[-3, 1], v ~ U[-1, 1], dt = 1.  The error of a cell is
 * max |v'_gpu - v'_oracle| over its components and velocities, relative to
 * the cell's max |v_in|.  Exit status 0 when every check passes.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "dragexp.h"
#include "oracle.h"

static uint64_t splitmix64(uint64_t *state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static double uniform(uint64_t *state, double lo, double hi) {
  const double u = (double)(splitmix64(state) >> 11) * 0x1.0p-53;
  return lo + (hi - lo) * u;
}

static int expect(int got, int want, const char *what) {
  if (got == want) return 0;
  fprintf(stderr, "%s: returned %d (%s), expected %d\n", what, got, drag_status_string(got),
          want);
  return 1;
}

static int host_only(void) {
  int bad = 0;
  drag_desc d;
  drag_desc_init(&d, 16, 4, 3, 1.0);
  bad |= d.ld != 16 || d.k_max != 9 || d.option != 2;
  double dummy[1] = {0.0};
  bad |= expect(drag_expm_apply(NULL, dummy, dummy, dummy, dummy, dummy, NULL),
                DRAG_ERR_NULL_DESC, "NULL descriptor");
  drag_desc e = d;
  e.n_species = 0;
  bad |= expect(drag_expm_apply(&e, dummy, dummy, dummy, dummy, dummy, NULL),
                DRAG_ERR_N_SPECIES, "n_species = 0");
  e = d;
  e.n_dim = 4;
  bad |= expect(drag_expm_apply(&e, dummy, dummy, dummy, dummy, dummy, NULL), DRAG_ERR_N_DIM,
                "n_dim = 4");
  e = d;
  e.dt = -1.0;
  bad |= expect(drag_expm_apply(&e, dummy, dummy, dummy, dummy, dummy, NULL), DRAG_ERR_DT,
                "dt < 0");
  e = d;
  e.ld = 8;
  bad |= expect(drag_expm_apply(&e, dummy, dummy, dummy, dummy, dummy, NULL), DRAG_ERR_LD,
                "ld < n_cells");
  bad |= expect(drag_expm_apply(&d, NULL, dummy, dummy, dummy, dummy, NULL),
                DRAG_ERR_NULL_POINTER, "NULL rho_g");
  int32_t k, m, s;
  bad |= expect(drag_select(1.0, 9, 2, &k, &m, &s), DRAG_OK, "drag_select");
  bad |= drag_status_string(DRAG_ERR_LD) == NULL;
  printf("host-only %s\n", bad ? "FAILED" : "ok");
  return bad;
}

#define HIP_OK(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));            \
      return 2;                                                             \
    }                                                                       \
  } while (0)

int main(int argc, char **argv) {
  if (argc == 2 && strcmp(argv[1], "--host-only") == 0) return host_only();
  if (argc != 5) {
    fprintf(stderr, "usage: %s --host-only | N C D SEED\n", argv[0]);
    return 2;
  }
  const int N = atoi(argv[1]), D = atoi(argv[3]);
  const int64_t C = atoll(argv[2]);
  uint64_t state = strtoull(argv[4], NULL, 10);
  if (N < 1 || N > 16 || D < 1 || D > 3 || C < 1 || C > (1 << 22)) {
    fprintf(stderr, "bad sizes\n");
    return 2;
  }
  const size_t nf = (size_t)N * C, nv = (size_t)D * (N + 1) * C;
  double *rg = malloc(C * sizeof(double)), *rd = malloc(nf * sizeof(double));
  double *ts = malloc(nf * sizeof(double)), *v = malloc(nv * sizeof(double));
  double *got = malloc(nv * sizeof(double)), *ref = malloc(nv * sizeof(double));
  int32_t *kms = malloc(3 * C * sizeof(int32_t));
  double *nrm = malloc(C * sizeof(double));
  if (!rg || !rd || !ts || !v || !got || !ref || !kms || !nrm) return 2;
  for (int64_t c = 0; c < C; ++c) rg[c] = uniform(&state, 0.5, 2.0);
  for (int i = 0; i < N; ++i)
    for (int64_t c = 0; c < C; ++c) {
      rd[i * C + c] = pow(10.0, uniform(&state, -3.0, 0.0)) * rg[c];
      ts[i * C + c] = pow(10.0, uniform(&state, -3.0, 1.0));
    }
  for (size_t x = 0; x < nv; ++x) v[x] = uniform(&state, -1.0, 1.0);

  double *d_rg, *d_rd, *d_ts, *d_v, *d_out;
  HIP_OK(hipMalloc((void **)&d_rg, C * sizeof(double)));
  HIP_OK(hipMalloc((void **)&d_rd, nf * sizeof(double)));
  HIP_OK(hipMalloc((void **)&d_ts, nf * sizeof(double)));
  HIP_OK(hipMalloc((void **)&d_v, nv * sizeof(double)));
  HIP_OK(hipMalloc((void **)&d_out, nv * sizeof(double)));
  HIP_OK(hipMemcpy(d_rg, rg, C * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_rd, rd, nf * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_ts, ts, nf * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_v, v, nv * sizeof(double), hipMemcpyHostToDevice));

  drag_desc d;
  drag_desc_init(&d, C, N, D, 1.0);
  int bad = expect(drag_clear_status(NULL), DRAG_OK, "drag_clear_status");
  bad |= expect(drag_expm_apply(&d, d_rg, d_rd, d_ts, d_v, d_out, NULL), DRAG_OK,
                "drag_expm_apply");
  int32_t status = -1;
  bad |= expect(drag_get_status(NULL, &status), DRAG_OK, "drag_get_status");
  bad |= status != 0;
  HIP_OK(hipMemcpy(got, d_out, nv * sizeof(double), hipMemcpyDeviceToHost));

  const int orc = orc_apply_cells(C, N, D, C, 1.0, 9, 2, 0, rg, rd, ts, v, ref, kms, nrm);
  bad |= orc != 0;
  /* per cell: 1e-13 plus the oracle's own floor from its dense squarings,
   * 4 u ||dt K||_1 (the tight per-cell bars are the parity tests' business) */
  double max_err = 0.0, worst = 0.0;
  for (int64_t c = 0; c < C; ++c) {
    double scale = 0.0, e = 0.0;
    for (int64_t r = 0; r < (int64_t)D * (N + 1); ++r) scale = fmax(scale, fabs(v[r * C + c]));
    for (int64_t r = 0; r < (int64_t)D * (N + 1); ++r)
      e = fmax(e, fabs(got[r * C + c] - ref[r * C + c]));
    if (!(e <= 1e300)) e = INFINITY;  /* a NaN output counts as a failure */
    max_err = fmax(max_err, e / scale);
    worst = fmax(worst, e / scale / (1e-13 + 4.0 * 0x1.0p-53 * nrm[c]));
  }
  bad |= !(worst <= 1.0);
  printf("max_err %.3e bar_ratio %.3f status %d oracle %d\n", max_err, worst, (int)status, orc);
  (void)hipFree(d_rg);
  (void)hipFree(d_rd);
  (void)hipFree(d_ts);
  (void)hipFree(d_v);
  (void)hipFree(d_out);
  free(rg), free(rd), free(ts), free(v), free(got), free(ref), free(kms), free(nrm);
  return bad ? 1 : 0;
}
