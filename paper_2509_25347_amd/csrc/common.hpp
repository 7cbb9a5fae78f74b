// common.hpp -- constants, Alg. 1 and per-cell set-up shared by every kernel
// of the drag library (gfx950, FP64).
//
// Method: Sewanou, Laibe and Commercon, arXiv:2509.25347, Sect. 2.3 and
// Appendix B (Taylor scaling and squaring of dt K).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dragexp {

constexpr int kMaxSpecies = 16;

// Table B.1: m_k, q_k, r_k for k = 1..9 (index 0 unused).
constexpr int kTabM[10] = {0, 2, 4, 6, 9, 12, 16, 20, 25, 30};
constexpr int kTabQ[10] = {0, 1, 2, 2, 3, 3, 4, 4, 5, 5};
constexpr int kTabR[10] = {0, 2, 2, 3, 3, 4, 4, 5, 5, 6};

// theta_{m_k}: the largest theta with -log(1 - f_m(theta))/theta <= 2^-53
// (eq. B8), to full double precision.  Table B.1 prints five digits of each
// (row 5 garbled as "2/9962", i.e. 2.9962e-1).
constexpr double kTheta[10] = {
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

// Taylor coefficients 1/i!, i = 0..30, each correctly rounded.
constexpr double kInvFact[31] = {
    1.0, 1.0, 0.5,
    1.6666666666666666e-01, 4.1666666666666664e-02, 8.3333333333333332e-03,
    1.3888888888888889e-03, 1.9841269841269841e-04, 2.4801587301587302e-05,
    2.7557319223985893e-06, 2.7557319223985888e-07, 2.5052108385441720e-08,
    2.0876756987868100e-09, 1.6059043836821613e-10, 1.1470745597729725e-11,
    7.6471637318198164e-13, 4.7794773323873853e-14, 2.8114572543455206e-15,
    1.5619206968586225e-16, 8.2206352466243295e-18, 4.1103176233121648e-19,
    1.9572941063391263e-20, 8.8967913924505741e-22, 3.8681701706306841e-23,
    1.6117375710961184e-24, 6.4469502843844736e-26, 2.4795962632247976e-27,
    9.1836898637955460e-29, 3.2798892370698378e-30, 1.1309962886447716e-31,
    3.7699876288159054e-33,
};

// per-cell bad-input bits (same values as the DRAG_CELL_* macros)
constexpr unsigned kBadDensity = 1u;
constexpr unsigned kBadStoppingTime = 2u;
constexpr unsigned kBadVelocity = 4u;
constexpr unsigned kBadNorm = 8u;

struct Kms {
  int k, m, s;
};

// Sticky per-device status word: the OR of the bad-input bits of every cell
// processed since the last reset (the library is one translation unit).
__device__ unsigned int g_status_word;

// Alg. 1 (Appendix B, "First modification"): (k*, m*, s*) for a finite
// ||A||_1 with at most K products in the polynomial stage.  The scaled
// branch's s-hat = ceil(log2(nrm / theta_K)) is the smallest s >= 0 with
// nrm <= theta_K 2^s, found with exact power-of-two comparisons after a
// frexp estimate, so host and device agree bit for bit.
__host__ __device__ inline Kms select_kms(double nrm, int K, int option) {
  Kms r{K, kTabM[K], 0};
  const double thK = kTheta[K];
  if (nrm <= thK) {
    int k = K;
    for (int j = 1; j <= K; ++j) {
      if (nrm <= kTheta[j]) {
        k = j;
        break;
      }
    }
    r.k = k;
    r.m = kTabM[k];
    r.s = 0;
    if (option == 2) {
      if (k >= 8 && nrm <= 2.0 * kTheta[k - 2]) {
        r.k = k - 2;
        r.m = kTabM[r.k];
        r.s = 1;
      } else if (k == 9 && nrm <= 4.0 * kTheta[k - 3]) {
        r.k = k - 3;
        r.m = kTabM[r.k];
        r.s = 2;
      }
    }
    return r;
  }
  int en, et;
  frexp(nrm, &en);
  frexp(thK, &et);
  int sh = en - et - 1;  // nrm / thK lies in (2^(en-et-1), 2^(en-et+1))
  if (sh < 0) sh = 0;
  while (nrm > ldexp(thK, sh)) ++sh;
  r.s = sh;
  const double x = ldexp(nrm, -sh);
  if (option > 0) {
    if (K >= 7 && x <= kTheta[K - 1]) {
      r.k = K - 1;
      r.m = kTabM[r.k];
    } else if (option == 2) {
      if (K >= 8 && x <= 2.0 * kTheta[K - 2]) {
        r.k = K - 2;
        r.m = kTabM[r.k];
        r.s = sh + 1;
      } else if (K == 9 && x <= 4.0 * kTheta[K - 3]) {
        r.k = K - 3;
        r.m = kTabM[r.k];
        r.s = sh + 2;
      }
    }
  }
  return r;
}

// Launch parameters common to the per-cell kernels.
struct CellArgs {
  const double* rho_g;
  const double* rho_d;
  const double* t_stop;
  const double* v_in;
  double* v_out;
  int64_t n_cells;
  int64_t ld;
  double dt;
  int n_dim;
  int k_max;
  int option;  // Alg. 1 option, 0..2
};

struct BackArgs {
  const double* rho_g;
  const double* rho_d;
  const double* t_stop;
  const double* v_in;
  const double* w;  // dL/dv_out
  double* v_out;
  double* g_v;
  double* g_logt;
  double* g_t;
  double* g_rho_d;
  double* g_rho_g;
  int64_t n_cells;
  int64_t ld;
  double dt;
  int n_dim;
  int k_max;
  int option;
};

// One species' drag coefficients, rounded exactly as the definition reads:
// a = dt / t (t = +inf gives 0), e = rho_i / rho_g, p = e a (the gas-row
// entry of dt K).  The library is compiled with -ffp-contract=off: a * b + c
// is two roundings unless written fma(a, b, c), so p and the sums of the norm
// are reproducible bit for bit.
struct Species {
  double a, e, p;
};

__device__ __forceinline__ Species species_coeffs(double dt, double t, double rho_i,
                                                  double rho_gas) {
  Species s;
  s.a = dt / t;
  s.e = rho_i / rho_gas;
  s.p = s.e * s.a;
  return s;
}

__device__ __forceinline__ unsigned species_bad(double t, double rho_i) {
  unsigned bad = 0;
  if (!(isfinite(rho_i) && rho_i >= 0.0)) bad |= kBadDensity;
  if (!(t > 0.0)) bad |= kBadStoppingTime;
  return bad;
}

__device__ __forceinline__ unsigned gas_bad(double rho_gas) {
  return (isfinite(rho_gas) && rho_gas > 0.0) ? 0u : kBadDensity;
}

}  // namespace dragexp
