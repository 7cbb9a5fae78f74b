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
// ||A||_1 with at most K products in the polynomial stage, from the method's
// cost model: row k of Table B.1 costs k products (Pi_{m_k}) and every
// squaring one more; row k serves a scaling 2^-s when ||A|| 2^-s <=
// theta_{m_k} (eq. B8).  The base pair is the cheapest row that needs no
// scaling, or else row K with s-hat = ceil(log2(||A|| / theta_K)), the
// fewest squarings that serve it (found with exact power-of-two comparisons
// after a frexp estimate, so host and device agree bit for bit).  The
// options then allow trades that keep the cost: one product fewer at the
// same s (option >= 1, rows 7..9), or two or three products of the
// polynomial for one or two squarings at a lower degree (option 2, rows 8..9,
// row 9); the first trade whose pair still serves is taken.
struct KmsTrade {
  int dk, ds, min_option, k_lo, k_hi;
};
constexpr KmsTrade kKmsTrades[3] = {{-1, 0, 1, 7, 9}, {-2, 1, 2, 8, 9}, {-3, 2, 2, 9, 9}};

__host__ __device__ inline Kms select_kms(double nrm, int K, int option) {
  int k = K, s = 0;
  if (nrm <= kTheta[K]) {
    k = 1;
    while (nrm > kTheta[k]) ++k;
  } else {
    int en, et;
    frexp(nrm, &en);
    frexp(kTheta[K], &et);
    s = en - et - 1;  // nrm / theta_K lies in (2^(en-et-1), 2^(en-et+1))
    if (s < 0) s = 0;
    while (nrm > ldexp(kTheta[K], s)) ++s;
  }
  for (int t = 0; t < 3; ++t) {
    const KmsTrade tr = kKmsTrades[t];
    if (option < tr.min_option || k < tr.k_lo || k > tr.k_hi) continue;
    if (ldexp(nrm, -(s + tr.ds)) <= kTheta[k + tr.dk]) {
      k += tr.dk;
      s += tr.ds;
      break;
    }
  }
  return Kms{k, kTabM[k], s};
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
