// wave.hpp -- one cell per 64-lane wavefront, FP64 MFMA (v_mfma_f64_16x16x4).
//
// The cell's relative-velocity matrix (the N x N reduced form described in
// lane.hpp) is held as one 16 x 16 tile, zero-padded when N < 16: the
// species block of the drag problem is exactly the MFMA tile for N = 16.
// Every dense product of the method -- the powers of the scaled matrix, the
// Horner steps of the Paterson-Stockmeyer evaluation and the s squarings --
// is a chain of four 16x16x4 FP64 MFMAs (k = 16).
//
// Register layouts of v_mfma_f64_16x16x4 (lane l = 16 g + j, g = l / 16):
//   A operand (16 x 4, step t):  A[i = j][4t + g]
//   B operand (4 x 16, step t):  B[4t + g][j]
//   C / D (16 x 16, 4 values):   D[4v + g][j], v = 0..3 (rows interleaved
//                                 across the four lane groups)
// Products re-distribute the D layout into the A and B layouts through a
// 16 x 17 LDS tile per operand (the pad column keeps the transposed reads
// of the A operand free of bank conflicts).
#pragma once

#include "common.hpp"

namespace dragexp {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kLdsStride = 17;
constexpr int kStageDoubles = 16 * kLdsStride;

__device__ __forceinline__ double readlane_f64(double x, int l) {
  const long long bits = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)bits, l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ unsigned wave_or_u32(unsigned x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x |= (unsigned)__shfl_xor((int)x, off, 64);
  return x;
}

__device__ __forceinline__ void stage_tile(double* buf, int g, int j, const v4d& X) {
#pragma unroll
  for (int v = 0; v < 4; ++v) buf[(4 * v + g) * kLdsStride + j] = X[v];
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void load_a_ops(const double* buf, int g, int i, double (&A)[4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) A[t] = buf[i * kLdsStride + 4 * t + g];
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void load_b_ops(const double* buf, int g, int j, double (&B)[4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) B[t] = buf[(4 * t + g) * kLdsStride + j];
  __builtin_amdgcn_wave_barrier();
}

// D = A B + C over k = 16.
__device__ __forceinline__ v4d mma16(const double (&A)[4], const double (&B)[4], v4d acc) {
#pragma unroll
  for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[t], B[t], acc, 0, 0, 0);
  return acc;
}

// Per-cell set-up of the wave kernel: the lane with j = lane % 16 < N owns
// species j.  Every lane computes the norm's sums in ascending species
// order from broadcast values, so ||A||_1 is the same bits as the
// definition.  Returns the bad-input bits (uniform over the wavefront).
// N is a run-time argument throughout the MFMA path (it only bounds loops
// and masks the padded rows and columns of the 16 x 16 tile); the per-N
// kernels pass a constant and the compiler folds it.
struct WaveCell {
  double aj, ej, pj;  // species j = lane % 16 (0 for j >= N)
  double sigma, nrm;
  unsigned bad;
  Kms kms;
};

__device__ __forceinline__ void wave_setup(WaveCell& W, const int N, const double* rho_g,
                                           const double* rho_d, const double* t_stop,
                                           int64_t ld, int64_t cell, double dt, int K,
                                           int option, int j) {
  const double rg = rho_g[cell];
  unsigned bad = gas_bad(rg);
  W.aj = W.ej = W.pj = 0.0;
  if (j < N) {
    const double t = t_stop[j * ld + cell];
    const double r = rho_d[j * ld + cell];
    bad |= species_bad(t, r);
    const Species sp = species_coeffs(dt, t, r, rg);
    W.aj = sp.a;
    W.ej = sp.e;
    W.pj = sp.p;
  }
  const bool fin_j = isfinite(W.aj) && isfinite(W.pj);
  bad = wave_or_u32(bad);
  double s = 0.0, sig = 1.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    s = s + readlane_f64(W.pj, i);
    sig = sig + readlane_f64(W.ej, i);
  }
  double nrm = s;
#pragma unroll
  for (int i = 0; i < N; ++i) nrm = nrm + readlane_f64(W.aj, i);
#pragma unroll
  for (int i = 0; i < N; ++i) nrm = fmax(nrm, readlane_f64(W.pj, i) + readlane_f64(W.aj, i));
  const bool all_fin = __all(fin_j) && isfinite(nrm);
  if (!bad && !all_fin) bad |= kBadNorm;
  W.bad = bad;
  W.sigma = sig;
  W.nrm = nrm;
  W.kms = bad ? Kms{1, 2, 0} : select_kms(nrm, K, option);
}

// Z = T_m(2^-s At)^(2^s) - I in the D layout (rows 4v+g, column j).
__device__ __forceinline__ v4d wave_expm(const WaveCell& W, const int N, int g, int j,
                                         double* bufX, double* bufY) {
  const int s = W.kms.s;
  const int q = kTabQ[W.kms.k], r = kTabR[W.kms.k];
  const double bj = ldexp(W.aj, -s);
  const double pbj = ldexp(W.pj, -s);

  // M = 2^-s At, D layout: M[row][j] = -b_row [row == j] - pb_j (row, j < N)
  v4d M;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = 4 * v + g;
    M[v] = (row < N && j < N) ? ((row == j ? -bj : 0.0) - pbj) : 0.0;
  }
  // M as the A operand: M[i = j][col = 4t + g]
  double Ma[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int col = 4 * t + g;
    const double pbc = __shfl(pbj, col, 64);
    Ma[t] = (j < N && col < N) ? ((j == col ? -bj : 0.0) - pbc) : 0.0;
  }

  // powers P_1 = M, P_jj = M P_{jj-1} (Sect. 2.3: the power sequence of
  // the Paterson-Stockmeyer evaluation, q <= 5)
  v4d P[6];
  P[1] = M;
#pragma unroll
  for (int jj = 2; jj <= 5; ++jj) {
    if (jj <= q) {
      double Bt[4];
      stage_tile(bufX, g, j, P[jj - 1]);
      load_b_ops(bufX, g, j, Bt);
      P[jj] = mma16(Ma, Bt, v4d{0.0, 0.0, 0.0, 0.0});
    } else {
      P[jj] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  }
  v4d Pq = P[1];
#pragma unroll
  for (int jj = 2; jj <= 5; ++jj)
    if (jj == q) Pq = P[jj];

  // Bbar_k = sum_{jj=1}^{q} b_{qk+jj} P_jj
  auto bbar = [&](int k) {
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int jj = 1; jj <= 5; ++jj) {
      if (jj <= q) {
        const double c = kInvFact[q * k + jj];
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = fma(c, P[jj][v], acc[v]);
      }
    }
    return acc;
  };

  // Horner: F = Bbar_{r-1}; F = Bbar_k + F P_q, k = r-2..0.  F = T_m(M) - I.
  double Bq[4];
  stage_tile(bufY, g, j, Pq);
  load_b_ops(bufY, g, j, Bq);
  v4d F = bbar(r - 1);
  for (int k = r - 2; k >= 0; --k) {
    double Af[4];
    stage_tile(bufX, g, j, F);
    load_a_ops(bufX, g, j, Af);
    F = mma16(Af, Bq, bbar(k));
  }

  // squarings, Y-form: Z <- 2 Z + Z Z
  v4d Z = F;
  for (int it = 0; it < s; ++it) {
    double Az[4], Bz[4];
    stage_tile(bufX, g, j, Z);
    load_a_ops(bufX, g, j, Az);
    load_b_ops(bufX, g, j, Bz);
    Z = mma16(Az, Bz, Z + Z);
  }
  return Z;
}

// The forward update of one cell by a whole wavefront (lane = 0..63), with
// two 16 x 17 LDS tiles private to the wavefront.
__device__ __forceinline__ void wave_forward_cell(const CellArgs& A, const int N, int64_t cell,
                                                  int lane, double* bufX, double* bufY) {
  const int g = lane >> 4, j = lane & 15;
  const int64_t ld = A.ld;
  const int n1 = N + 1;
  const int D = A.n_dim;

  WaveCell W;
  wave_setup(W, N, A.rho_g, A.rho_d, A.t_stop, ld, cell, A.dt, A.k_max, A.option, j);

  // velocities: lane (g, col = j < D) loads the relative velocities of rows
  // 4t + g as the B operand of the final product
  double v0 = 0.0;
  double Bd[4] = {0.0, 0.0, 0.0, 0.0};
  bool vfin = true;
  if (j < D) {
    v0 = A.v_in[(int64_t)(j * n1) * ld + cell];
    vfin = isfinite(v0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int row = 4 * t + g;
      if (row < N) {
        const double x = A.v_in[(int64_t)(j * n1 + 1 + row) * ld + cell];
        vfin = vfin && isfinite(x);
        Bd[t] = x - v0;
      }
    }
  }
  unsigned bad = W.bad | (__all(vfin) ? 0u : kBadVelocity);
  if (bad) {
    if (lane < D * n1) A.v_out[(int64_t)lane * ld + cell] = __builtin_nan("");
    if (lane == 0) atomicOr(&g_status_word, bad);
    return;
  }

  const v4d Z = wave_expm(W, N, g, j, bufX, bufY);

  // u = Z dv for every component at once
  double Az[4];
  stage_tile(bufX, g, j, Z);
  load_a_ops(bufX, g, j, Az);
  const v4d U = mma16(Az, Bd, v4d{0.0, 0.0, 0.0, 0.0});
  double eu = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = 4 * v + g;
    const double er = __shfl(W.ej, row, 64);
    if (row < N) eu = fma(er, U[v], eu);
  }
  eu += __shfl_xor(eu, 16, 64);
  eu += __shfl_xor(eu, 32, 64);
  const double d0 = -eu / W.sigma;
  if (j < D) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * v + g;
      if (row < N) {
        const int64_t idx = (int64_t)(j * n1 + 1 + row) * ld + cell;
        const double x = A.v_in[idx];
        A.v_out[idx] = x + (d0 + U[v]);
      }
    }
    if (g == 0) A.v_out[(int64_t)(j * n1) * ld + cell] = v0 + d0;
  }
}

template <int N>
__global__ void __launch_bounds__(256) k_forward_wave(CellArgs A, int xcd_blocks) {
  __shared__ double lds[4 * 2 * kStageDoubles];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int bid = blockIdx.x;
  const int64_t logical = (int64_t)(bid & 7) * xcd_blocks + (bid >> 3);
  const int64_t cell = logical * 4 + w;
  if (cell >= A.n_cells) return;  // uniform over the wavefront
  double* bufX = lds + (2 * w) * kStageDoubles;
  wave_forward_cell(A, N, cell, lane, bufX, bufX + kStageDoubles);
}

}  // namespace dragexp
