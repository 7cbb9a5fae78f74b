// rk1.hpp -- the first-order implicit (backward Euler) drag step, one cell per
// lane, by the O(N) closed form of the paper's appendix on implicit solvers
// (eqs. analytic_1 to analytic_4).
//
// The step solves (I - dt K) x = v per cell and velocity component.  In the
// velocity form (A = dt K: A00 = -sum p_i, A0i = p_i, Ai0 = a_i, Aii = -a_i,
// a_i = dt / t_i, p_i = e_i a_i) the system is an arrowhead: row i > 0 gives
// x_i in terms of x_0, and substituting into row 0 leaves one scalar equation.
// With h_i = a_i / (1 + a_i) and w_i = p_i / (1 + a_i) = e_i h_i,
//     x_0 = v_0 + (sum_i w_i (v_i - v_0)) / (1 + sum_i w_i),
//     x_i = v_i + h_i (x_0 - v_i),
// which is the paper's q_0 = (b_0 + dt B) / A and its back substitution,
// rewritten around the old velocities (the paper's form solves for momenta
// and divides by 1 + sum e_i (1 - 1/(1 + a_i)), whose terms lose all their
// digits when a_i is tiny; a_i / (1 + a_i) keeps them).  Every term is a
// product of nonnegative weights, so the forward error stays a few N u of the
// velocities for any stiffness.
//
// The kernel reads rho_g, rho_d, t_stop and v once and writes v' once: it is
// bound by HBM bandwidth (8 + 16 N + 16 D (N + 1) bytes per cell).  Bad cells
// are flagged exactly as by the exponential (density and stopping-time bits;
// else an entry of dt K or ||dt K||_1 overflowing; else a velocity that is
// not finite) and get NaN outputs.  A species with a_i = 0 (dt = 0 or
// t_i = +inf) keeps its velocity bit for bit, and so does the gas when every
// w_i is 0.
#pragma once

#include "common.hpp"

namespace dragexp {

// Cache policy of the streams, by N.  Every byte is touched once, so the
// choice is only which traffic bypasses the caches' normal allocation
// (nontemporal loads and stores).  Measured on MI355X over 2^20 stiff cells,
// D = 3, the best of the four policies: N <= 6 nontemporal stores (7.0 TB/s
// at N = 4-5 against 5.7 with none), N = 7-11 nontemporal loads (6.4-6.5
// against 5.2), N >= 12 both (5.7-5.8 against 5.2).  The split follows the
// register count: 4 or fewer wavefronts per SIMD from N = 12 on.
template <int N>
struct Rk1Policy {
  static constexpr bool kNtLoad = N >= 7;
  static constexpr bool kNtStore = N <= 6 || N >= 12;
};

template <bool NT>
__device__ __forceinline__ double rk1_load(const double* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <bool NT>
__device__ __forceinline__ void rk1_store(double* p, double x) {
  if constexpr (NT) __builtin_nontemporal_store(x, p);
  else *p = x;
}

template <int N>
__device__ __forceinline__ void rk1_cell(const CellArgs& A, int64_t c) {
  constexpr bool NL = Rk1Policy<N>::kNtLoad, NS = Rk1Policy<N>::kNtStore;
  const int64_t ld = A.ld;
  const double rg = rk1_load<NL>(A.rho_g + c);
  unsigned bad = gas_bad(rg);
  double h[N], w[N];
  double s = 0.0, nrm, sw = 0.0;
  bool finite = true;
  {
    double a[N], p[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double t = rk1_load<NL>(A.t_stop + i * ld + c);
      const double r = rk1_load<NL>(A.rho_d + i * ld + c);
      bad |= species_bad(t, r);
      const Species sp = species_coeffs(A.dt, t, r, rg);
      a[i] = sp.a;
      p[i] = sp.p;
      h[i] = sp.a / (1.0 + sp.a);
      w[i] = sp.e * h[i];
    }
    // the overflow test of the exponential path: every entry of dt K and its
    // 1-norm finite, the sums taken in the same order
#pragma unroll
    for (int i = 0; i < N; ++i) {
      s = s + p[i];
      finite = finite && isfinite(a[i]) && isfinite(p[i]);
    }
    nrm = s;
#pragma unroll
    for (int i = 0; i < N; ++i) nrm = nrm + a[i];
#pragma unroll
    for (int i = 0; i < N; ++i) nrm = fmax(nrm, p[i] + a[i]);
  }
  if (!bad && !(finite && isfinite(nrm))) bad |= kBadNorm;
#pragma unroll
  for (int i = 0; i < N; ++i) sw = sw + w[i];
  const double rs = 1.0 / (1.0 + sw);

  const int n1 = N + 1;
  const double qnan = __builtin_nan("");
  bool vfin = true;
  for (int d = 0; d < A.n_dim; ++d) {
    double v[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      v[j] = rk1_load<NL>(A.v_in + (int64_t)(d * n1 + j) * ld + c);
      vfin = vfin && isfinite(v[j]);
    }
    double num = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) num = fma(w[i], v[i + 1] - v[0], num);
    const double x0 = sw == 0.0 ? v[0] : fma(num, rs, v[0]);
    const bool nan_out = bad || !vfin;
    rk1_store<NS>(A.v_out + (int64_t)(d * n1) * ld + c, nan_out ? qnan : x0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double xi = h[i] == 0.0 ? v[i + 1] : fma(h[i], x0 - v[i + 1], v[i + 1]);
      rk1_store<NS>(A.v_out + (int64_t)(d * n1 + 1 + i) * ld + c, nan_out ? qnan : xi);
    }
  }
  if (!vfin && !bad) {
    // a later component was not finite: the components written before it
    // become NaN too (same lane, same addresses, so the stores stay ordered)
    bad = kBadVelocity;
    for (int d = 0; d < A.n_dim; ++d)
      for (int j = 0; j <= N; ++j) rk1_store<NS>(A.v_out + (int64_t)(d * n1 + j) * ld + c, qnan);
  }
  if (bad) atomicOr(&g_status_word, bad);
}

template <int N>
__global__ void __launch_bounds__(256) k_rk1_lane(CellArgs A, int xcd_blocks) {
  // XCD-aware order as in the exponential's lane kernel
  const int bid = blockIdx.x;
  const int64_t logical = (int64_t)(bid & 7) * xcd_blocks + (bid >> 3);
  const int64_t c = logical * 256 + threadIdx.x;
  if (c < A.n_cells) rk1_cell<N>(A, c);
}

}  // namespace dragexp
