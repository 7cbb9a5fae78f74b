// wave.hpp -- the MFMA mapping: a cell's exponential on a whole 64-lane
// wavefront, FP64 MFMA (v_mfma_f64_16x16x4).
//
// The cell's relative-velocity matrix (the N x N reduced form described in
// lane.hpp) is held as one 16 x 16 tile, zero-padded when N < 16: the
// species block of the drag problem is exactly the MFMA tile for N = 16.
// Dense products of the method (Horner steps of the Paterson-Stockmeyer
// evaluation, the s squarings, the apply) are chains of 16x16x4 FP64 MFMAs:
// four (k = 16), or ceil(N / 4) where the kernel is compiled for N.
//
// Register layouts of v_mfma_f64_16x16x4 (lane l = 16 g + j, g = l / 16):
//   A operand (16 x 4, step t):  A[i = j][4t + g]
//   B operand (4 x 16, step t):  B[4t + g][j]
//   C / D (16 x 16, 4 values):   D[4v + g][j], v = 0..3 (rows interleaved
//                                 across the four lane groups)
// The D layout is the B layout (register t of lane 16 g + j holds row 4 t + g,
// column j), so a product's B operand comes straight from registers; the A
// operand (the transpose of that pattern) is re-laid through a 16 x 17 LDS
// tile (the pad column keeps the transposed reads free of bank conflicts).
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

__device__ __forceinline__ void stage_tile(double* buf, int g, int j, const v4d& X) {
#pragma unroll
  for (int v = 0; v < 4; ++v) buf[(4 * v + g) * kLdsStride + j] = X[v];
  __builtin_amdgcn_wave_barrier();
}

// The A operand of the first KT steps (columns 0 .. 4 KT - 1 of the tile).
template <int KT = 4>
__device__ __forceinline__ void load_a_ops(const double* buf, int g, int i, double (&A)[4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) A[t] = t < KT ? buf[i * kLdsStride + 4 * t + g] : 0.0;
  __builtin_amdgcn_wave_barrier();
}

// D = A B + C over k = 16.
__device__ __forceinline__ v4d mma16(const double (&A)[4], const double (&B)[4], v4d acc) {
#pragma unroll
  for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[t], B[t], acc, 0, 0, 0);
  return acc;
}

// D = A B + C over k = 4 KT.  When the contraction runs over the species of
// an N x N block zero-padded to the tile (rows N .. 15 of B zero), the steps
// t >= ceil(N / 4) add exact zeros, so KT = ceil(N / 4) gives the same
// values as k = 16 with 4 - KT fewer MFMAs.
template <int KT>
__device__ __forceinline__ v4d mma_k(const double (&A)[4], const double (&B)[4], v4d acc) {
#pragma unroll
  for (int t = 0; t < KT; ++t)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[t], B[t], acc, 0, 0, 0);
  return acc;
}

// MFMA steps of an N-species contraction (N = 0: not known at compile time).
constexpr int mfma_steps(int N) { return N > 0 ? (N + 3) / 4 : 4; }

// ---- the forward update: four cells per wavefront ---------------------------
//
// One wavefront takes a quad of four consecutive cells.  The set-up (loads,
// coefficients, ||A||_1, Alg. 1) runs once for the quad with lane 16 g + j
// holding species j of cell g, so every 16-lane row of the wavefront is one
// cell and the row-wise sums of the norm are DPP broadcasts.  The
// exponential then runs cell by cell on the whole wavefront:
//   * products by the scaled matrix M = -diag(b) - 1 pb^T (the powers of the
//     Paterson-Stockmeyer stage) are its diagonal-plus-rank-one form, on the
//     vector ALU: a 16-row weighted column sum and one FMA per element;
//   * the Horner steps and the squarings are dense 16 x 16 products on the
//     matrix cores.  Their B operand is the D layout itself (lane 16 g + j,
//     register t holds row 4 t + g, column j), so only the A operand goes
//     through a 16 x 17 LDS tile;
//   * each squaring Z <- 2 Z + Z Z is issued as (Z + 2 I) Z: 2 I is added to
//     the staged copy by one LDS add on the diagonal, so no vector
//     instruction is spent on 2 Z.

// Broadcast lane L of every 16-lane row to the whole row (DPP row_newbcast).
template <int L>
__device__ __forceinline__ double row_bcast(double x) {
  return __builtin_amdgcn_update_dpp(0.0, x, 0x150 + L, 0xf, 0xf, true);
}

// A 64-bit value rotated by R lanes within each 16-lane row (two 32-bit DPP
// moves; 64-bit DPP only has the broadcast form).
template <int R>
__device__ __forceinline__ double row_ror64(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x120 + R, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x120 + R, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

template <int R>
__device__ __forceinline__ unsigned row_ror32(unsigned x) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x120 + R, 0xf, 0xf, true);
}

__device__ __forceinline__ double row_max(double x) {
  x = fmax(x, row_ror64<8>(x));
  x = fmax(x, row_ror64<4>(x));
  x = fmax(x, row_ror64<2>(x));
  return fmax(x, row_ror64<1>(x));
}

__device__ __forceinline__ unsigned row_or(unsigned x) {
  x |= row_ror32<8>(x);
  x |= row_ror32<4>(x);
  x |= row_ror32<2>(x);
  return x | row_ror32<1>(x);
}

// x(lane 16 g + j) summed over the four rows g, (x0 + x1) + (x2 + x3), the
// same bits in every row (v_permlane16_swap / v_permlane32_swap exchange
// rows 0 <-> 1, 2 <-> 3 and 0,1 <-> 2,3).
__device__ __forceinline__ double swap_sum16(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32),
                                                   false, false);
  const double d0 = __builtin_bit_cast(double, ((long long)hi[0] << 32) | lo[0]);
  const double d1 = __builtin_bit_cast(double, ((long long)hi[1] << 32) | lo[1]);
  return d0 + d1;
}

__device__ __forceinline__ double swap_sum32(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32),
                                                   false, false);
  const double d0 = __builtin_bit_cast(double, ((long long)hi[0] << 32) | lo[0]);
  const double d1 = __builtin_bit_cast(double, ((long long)hi[1] << 32) | lo[1]);
  return d0 + d1;
}

__device__ __forceinline__ double sum_rows(double x) { return swap_sum32(swap_sum16(x)); }

// Sequential row sum init + x(lane 0) + x(lane 1) + ... + x(lane N-1) of every
// row: one rounding per addition, ascending species order.
template <int L = 0>
__device__ __forceinline__ double row_chain(double acc, double x, const int N) {
  if constexpr (L < kMaxSpecies) {
    if (L < N) return row_chain<L + 1>(acc + row_bcast<L>(x), x, N);
  }
  return acc;
}

// Per-wavefront LDS: the A-operand staging tile and the quad's coefficients.
// Species j of quad cell c sits at 16 c + (4 (j & 3) + (j >> 2)), so the four
// species 4 v + g (v = 0..3) that lane 16 g + j needs are contiguous.
constexpr int kQuadVel = 3 * 17 * 4;  // velocities of the quad: [D (N+1)][4 cells]
constexpr int kQuadDoubles = kStageDoubles + 3 * 64 + kQuadVel;

__device__ __forceinline__ int quad_slot(int j) { return 4 * (j & 3) + (j >> 2); }

struct QuadRows {
  double nb[4];  // -b of rows 4 v + g  (b = 2^-s a)
  double pb[4];  // pb of rows 4 v + g  (pb = 2^-s p)
  double nbj, npbj;  // -b_j, -pb_j of column j
};

// X <- M X for M = -diag(b) - 1 pb^T (rows >= N of the result stay zero).
__device__ __forceinline__ v4d mul_M(const v4d& X, const QuadRows& R, const double (&rm)[4]) {
  double part = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) part = fma(R.pb[v], X[v], part);
  const double cs = -sum_rows(part);  // -(pb^T X)_j
  v4d Y;
#pragma unroll
  for (int v = 0; v < 4; ++v) Y[v] = fma(R.nb[v], X[v], cs * rm[v]);
  return Y;
}

// Split m <= q r of the Paterson-Stockmeyer evaluation used by the MFMA
// forward.  Table B.1 chooses (q, r) to minimise dense products; here the
// powers are structured products on the vector ALU (about 72 cycles per cell
// each, against 256 for a 16 x 16 MFMA product), so the cheapest split of the
// same degree shifts toward more powers: minimise 72 (q - 1) + 256 (r - 1) +
// 16 q r (the B-bar sums) over q <= 5, r = ceil(m / q).  Coefficients of
// degree above m are zero, so every split evaluates the same T_m.
constexpr int kPsQ[10] = {0, 2, 4, 3, 5, 4, 4, 5, 5, 5};
constexpr int kPsR[10] = {0, 1, 1, 2, 2, 3, 4, 4, 5, 6};

// T_m(M) - I by the Paterson-Stockmeyer scheme with Q powers (Sect. 2.3):
// P_jj = M^jj in the structured form, Bbar_k = sum_{jj=1}^{Q} b_{Qk+jj} P_jj,
// then Horner F = Bbar_{r-1}; F = Bbar_k + F P_Q, k = r-2..0 on the matrix
// cores (P_Q is the B operand straight from registers).
// ||X||_1 of a tile in the D layout (largest column sum of |X|), the same in
// every lane: the four row pieces of column j summed over the lane rows, then
// the largest over the 16 columns.  Additions are paired the same way in
// every lane and max is exact, so the value is bit-identical across lanes.
__device__ __forceinline__ double norm1_tile(const v4d& X) {
  const double part = (fabs(X[0]) + fabs(X[1])) + (fabs(X[2]) + fabs(X[3]));
  return row_max(sum_rows(part));
}

template <int Q, bool BT = false, int KT = 4>
__device__ __forceinline__ v4d quad_poly(const v4d& M, const QuadRows& R, const double (&rm)[4],
                                         int m, int r, double* stage, int g, int j) {
  v4d P[Q + 1];
  P[1] = M;
#pragma unroll
  for (int jj = 2; jj <= Q; ++jj) P[jj] = mul_M(P[jj - 1], R, rm);
  double Bq[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) Bq[t] = P[Q][t];
  auto bbar = [&](int k) {
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int jj = 1; jj <= Q; ++jj) {
      const double cf = (Q * k + jj <= m) ? kInvFact[Q * k + jj] : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = fma(cf, P[jj][v], acc[v]);
    }
    return acc;
  };
  v4d F = bbar(r - 1);
  if constexpr (!BT) {
    for (int k = r - 2; k >= 0; --k) {
      double Af[4];
      stage_tile(stage, g, j, F);
      load_a_ops<KT>(stage, g, j, Af);
      F = mma_k<KT>(Af, Bq, bbar(k));
    }
    return F;
  } else {
  // Second modification (Appendix B, eqs. Pat_Stk4-Pat_Stk6) on this split:
  // b_exp = ||I + Bhat_0|| + sum_{l>=1} ||Bhat_l|| ||M^Q||^l estimates
  // ||e^-M|| from the blocks of T_m(-M); before the product that carries the
  // accumulated F to level k, F (M^Q)^(k+1) is dropped when
  // b_exp ||F|| ||M^Q||^(k+1) <= u, i.e. when it is below u relative to
  // ||e^M||.  The decisions are wave-uniform (the norms are the same bits in
  // every lane), so a dropped product is not issued.
  auto bhat = [&](int l) {
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int jj = 1; jj <= Q; ++jj) {
      const int i = Q * l + jj;
      const double cf = (i <= m) ? ((i & 1) ? -kInvFact[i] : kInvFact[i]) : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = fma(cf, P[jj][v], acc[v]);
    }
    return acc;
  };
  const double nq = norm1_tile(P[Q]);
  double bexp = 0.0;
  for (int l = r - 1; l >= 1; --l) bexp = (norm1_tile(bhat(l)) + bexp) * nq;
  {
    v4d H = bhat(0);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (4 * v + g == j) H[v] += rm[v];  // the identity of the N x N block
    bexp = bexp + norm1_tile(H);
  }
  for (int k = r - 2; k >= 0; --k) {
    double pk = 1.0;  // ||M^Q||^(k+1)
    for (int i = 0; i <= k; ++i) pk *= nq;
    const bool neg = bexp * norm1_tile(F) * pk <= 0x1p-53;
    if (__builtin_amdgcn_readfirstlane((int)neg)) {
      F = bbar(k);
    } else {
      double Af[4];
      stage_tile(stage, g, j, F);
      load_a_ops<KT>(stage, g, j, Af);
      F = mma_k<KT>(Af, Bq, bbar(k));
    }
  }
  return F;
  }
}

#include "pade.hpp"  // the Pade scaling step, built on the helpers above

// One squaring of the Y form, Z <- 2 Z + Z Z, issued as (Z + 2 I) Z: Z is
// staged, lanes 0..15 add 2 to the diagonal of the staged copy, the copy is
// read back as the A operand, Z itself is the B operand and the accumulator
// starts at zero.  The extra rounding of the diagonal entries 2 + Z_jj is
// of the same size as that of the sum 2 Z + Z Z.
template <int KT = 4>
__device__ __forceinline__ v4d square_step(const v4d& Z, double* stage, int g, int j,
                                           int diag_slot) {
  double Az[4], Bz[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) Bz[t] = Z[t];
  stage_tile(stage, g, j, Z);
  if (g == 0) atomicAdd(stage + diag_slot, 2.0);
  __builtin_amdgcn_wave_barrier();
  load_a_ops<KT>(stage, g, j, Az);
  return mma_k<KT>(Az, Bz, v4d{0.0, 0.0, 0.0, 0.0});
}

// The forward update of cells c0 .. c0+3 (those below n_cells) by one
// wavefront (lane = 0..63) with its private LDS block `lds`.
// Set-up of a quad (cells c0 .. c0+3, row g = cell c0 + g, lane j = species
// j): loads, coefficients (Eq. 2: a = dt / t, e = rho_i / rho_g, p = e a),
// ||A||_1 and Alg. 1.  The coefficients go to the quad's LDS tables (q*),
// species j >= N as zeros; the per-cell values come back row-uniform.
constexpr int kStageTaylor = 0;
constexpr int kStageTaylorBound = 1;
constexpr int kStagePade = 2;

struct QuadCell {
  unsigned bad;  // bad-input bits of the row's cell
  int kpack;     // k* | s* << 4
  double sig;    // 1 + sum_i e_i
};

__device__ __forceinline__ QuadCell quad_setup(const double* rho_g, const double* rho_d,
                                               const double* t_stop, int64_t n_cells, int64_t ld,
                                               double dt, int K, int option, const int N,
                                               int64_t c0, int g, int j, double* qa, double* qe,
                                               double* qp, bool pade = false) {
  const int64_t cg = c0 + g;
  double aj = 0.0, ej = 0.0, pj = 0.0;
  unsigned bad = 0;
  if (cg < n_cells) {
    const double rg = rho_g[cg];
    bad = gas_bad(rg);
    if (j < N) {
      const double t = t_stop[j * ld + cg];
      const double r = rho_d[j * ld + cg];
      bad |= species_bad(t, r);
      const Species sp = species_coeffs(dt, t, r, rg);
      aj = sp.a;
      ej = sp.e;
      pj = sp.p;
    }
  }
  constexpr unsigned kNonFinite = 0x100u;
  if (!(isfinite(aj) && isfinite(pj))) bad |= kNonFinite;
  bad = row_or(bad);
  // ||A||_1 = max(gas column, species columns): gas column |A00| + a_1 + ..
  // + a_N with |A00| = p_1 + .. + p_N, both sums in ascending order as in
  // the definition; species column j is p_j + a_j.
  const double s_row = row_chain(0.0, pj, N);
  const double col0 = row_chain(s_row, aj, N);
  const double nrm = fmax(col0, row_max(pj + aj));
  QuadCell Q;
  Q.sig = row_chain(1.0, ej, N);
  if ((bad & 0xffu) == 0u && ((bad & kNonFinite) || !isfinite(nrm))) bad = kBadNorm;
  Q.bad = bad & 0xffu;
  if (pade) {  // the Pade table row instead of k*
    const PadeSel ps = pade_select(Q.bad ? 0.0 : nrm);
    Q.kpack = ps.row | (ps.s << 4);
  } else {
    const Kms km = select_kms(Q.bad ? 0.0 : nrm, K, option);
    Q.kpack = km.k | (km.s << 4);
  }
  const int slot = 16 * g + quad_slot(j);
  qa[slot] = aj;
  qe[slot] = ej;
  qp[slot] = pj;
  __builtin_amdgcn_wave_barrier();
  return Q;
}

// With store = false the outputs stay in the quad's LDS block (vs) for the
// workgroup to store (group_store).
// METHOD: the scaling step (kStageTaylor, kStageTaylorBound: with the
// second modification, kStagePade: the diagonal Pade approximant).
// KT: MFMA steps per product, mfma_steps(N) where N is a compile-time
// constant of the caller, else 4.
template <int METHOD = kStageTaylor, int KT = 4>
__device__ __forceinline__ void wave_forward_quad(const CellArgs& A, const int N, int64_t c0,
                                                  int lane, double* lds, bool store = true) {
  const int g = lane >> 4, j = lane & 15;
  const int64_t ld = A.ld;
  const int n1 = N + 1;
  const int D = A.n_dim;
  double* stage = lds;
  double* qa = lds + kStageDoubles;
  double* qe = qa + 64;
  double* qp = qe + 64;

  const QuadCell Q = quad_setup(A.rho_g, A.rho_d, A.t_stop, A.n_cells, ld, A.dt, A.k_max,
                                A.option, N, c0, g, j, qa, qe, qp, METHOD == kStagePade);
  // the four cells' bad bits, (k*, s*) and 1 / sigma as scalars
  const double rsig = 1.0 / Q.sig;
  unsigned bad_s[4];
  int kp_s[4];
  double rsig_s[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    bad_s[r] = (unsigned)__builtin_amdgcn_readlane((int)Q.bad, 16 * r);
    kp_s[r] = __builtin_amdgcn_readlane(Q.kpack, 16 * r);
    rsig_s[r] = readlane_f64(rsig, 16 * r);
  }

  // lane constants of the tile layout
  double rm[4];  // 1 for rows < N
#pragma unroll
  for (int v = 0; v < 4; ++v) rm[v] = (4 * v + g < N) ? 1.0 : 0.0;
  const int diag_slot = j * kLdsStride + j;

  // the quad's velocities through LDS: rows (component, species) x 4
  // consecutive cells, loaded and stored with 4 lanes per 32-byte row piece.
  // All loads precede all stores, so v_out may alias v_in.
  double* vs = qp + 64;
  const int rows = D * n1;
  for (int f = lane; f < 4 * rows; f += 64) {
    const int64_t cell = c0 + (f & 3);
    vs[f] = cell < A.n_cells ? A.v_in[(int64_t)(f >> 2) * ld + cell] : 0.0;
  }
  __builtin_amdgcn_wave_barrier();

#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    const int64_t cell = c0 + c;
    if (cell >= A.n_cells) break;  // uniform
    // lane (g, j < D): component j of the gas (v0) and of species rows 4 v + g
    // (x[v]); read again at the apply rather than kept through the squarings
    auto read_v = [&](double& v0, double (&x)[4]) {
      v0 = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) x[v] = 0.0;
      if (j < D) {
        v0 = vs[(j * n1) * 4 + c];
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (4 * v + g < N) x[v] = vs[(j * n1 + 1 + 4 * v + g) * 4 + c];
      }
      __builtin_amdgcn_wave_barrier();
    };
    double v0, x[4];
    read_v(v0, x);

    unsigned cbad = c == 0 ? bad_s[0] : c == 1 ? bad_s[1] : c == 2 ? bad_s[2] : bad_s[3];
    bool vfin = isfinite(v0);
#pragma unroll
    for (int v = 0; v < 4; ++v) vfin = vfin && isfinite(x[v]);
    if (!__all(vfin) && !cbad) cbad = kBadVelocity;
    if (cbad) {
      if (lane < rows) vs[lane * 4 + c] = __builtin_nan("");
      if (lane == 0) atomicOr(&g_status_word, cbad);
      __builtin_amdgcn_wave_barrier();
      continue;
    }
    const int kp = c == 0 ? kp_s[0] : c == 1 ? kp_s[1] : c == 2 ? kp_s[2] : kp_s[3];
    const int kk = kp & 15, s = kp >> 4;  // kk: k*, or the Pade table row
    const int q = kPsQ[kk], r = kPsR[kk], m = kTabM[kk];
    const double crsig = c == 0 ? rsig_s[0] : c == 1 ? rsig_s[1] : c == 2 ? rsig_s[2] : rsig_s[3];

    // scaled coefficients of this cell
    QuadRows R;
    {
      const double* ra = qa + 16 * c + 4 * g;
      const double* rp = qp + 16 * c + 4 * g;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        R.nb[v] = -ldexp(ra[v], -s);
        R.pb[v] = ldexp(rp[v], -s);
      }
      const int sj = 16 * c + quad_slot(j);
      R.nbj = -ldexp(qa[sj], -s);
      R.npbj = -ldexp(qp[sj], -s);
    }
    __builtin_amdgcn_wave_barrier();

    // M = 2^-s At in the D layout: M[row][j] = -b_row [row == j] - pb_j
    v4d M;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double dg = (4 * v + g == j) ? 1.0 : 0.0;
      M[v] = fma(dg, R.nbj, R.npbj * rm[v]);
    }
    v4d Z;
    constexpr bool BT = METHOD == kStageTaylorBound;
    if constexpr (METHOD == kStagePade) {
      Z = pade_stage(M, R, rm, kk, N, stage, g, j);
    } else {
      switch (q) {  // uniform; one code path per power count
        case 2: Z = quad_poly<2, BT, KT>(M, R, rm, m, r, stage, g, j); break;
        case 3: Z = quad_poly<3, BT, KT>(M, R, rm, m, r, stage, g, j); break;
        case 4: Z = quad_poly<4, BT, KT>(M, R, rm, m, r, stage, g, j); break;
        default: Z = quad_poly<5, BT, KT>(M, R, rm, m, r, stage, g, j); break;
      }
    }

    // squarings Z <- (Z + 2 I) Z, two per trip so that the result and
    // the operand registers alternate
    int it = 0;
    for (; it + 2 <= s; it += 2) {
      const v4d Z1 = square_step<KT>(Z, stage, g, j, diag_slot);
      Z = square_step<KT>(Z1, stage, g, j, diag_slot);
    }
    if (it < s) Z = square_step<KT>(Z, stage, g, j, diag_slot);

    // u = Z dv for every component at once (B operand: lane (g, j < D) holds
    // the relative velocities of rows 4 t + g, component j)
    read_v(v0, x);
    double Bd[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) Bd[t] = (j < D && 4 * t + g < N) ? x[t] - v0 : 0.0;
    double Az[4];
    stage_tile(stage, g, j, Z);
    load_a_ops<KT>(stage, g, j, Az);
    const v4d U = mma_k<KT>(Az, Bd, v4d{0.0, 0.0, 0.0, 0.0});
    double eu = 0.0;
    const double* re = qe + 16 * c + 4 * g;  // e of rows 4 v + g
#pragma unroll
    for (int v = 0; v < 4; ++v) eu = fma(re[v], U[v], eu);
    eu = sum_rows(eu);
    const double d0 = -eu * crsig;
    if (j < D) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (4 * v + g < N) vs[(j * n1 + 1 + 4 * v + g) * 4 + c] = x[v] + (d0 + U[v]);
      }
      if (g == 0) vs[(j * n1) * 4 + c] = v0 + d0;
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (!store) return;
  for (int f = lane; f < 4 * rows; f += 64) {
    const int64_t cell = c0 + (f & 3);
    if (cell < A.n_cells) A.v_out[(int64_t)(f >> 2) * ld + cell] = vs[f];
  }
}

// Offset of the velocity block inside a quad's LDS block.
constexpr int kQuadVelOffset = kStageDoubles + 3 * 64;

// The workgroup's 16 cells g0 .. g0+15 (quads of its four wavefronts, in
// order) stored from LDS a full 128-byte row piece at a time, so that every
// output cache line is written whole by one store instruction.  Call after a
// barrier that follows every wavefront's wave_forward_quad(store = false).
__device__ __forceinline__ void group_store(const CellArgs& A, const int N, int64_t g0,
                                            const double* lds) {
  const int rows = A.n_dim * (N + 1);
  for (int f = threadIdx.x; f < 16 * rows; f += 256) {
    const int row = f >> 4, cell = f & 15;
    if (g0 + cell < A.n_cells)
      A.v_out[(int64_t)row * A.ld + g0 + cell] =
          lds[(cell >> 2) * kQuadDoubles + kQuadVelOffset + row * 4 + (cell & 3)];
  }
}

template <int N, int METHOD = kStageTaylor>
__global__ void __launch_bounds__(256, METHOD == kStageTaylor ? 5 : 4)
    k_forward_wave(CellArgs A, int xcd_blocks) {
  __shared__ double lds[4 * kQuadDoubles];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int bid = blockIdx.x;
  const int64_t logical = (int64_t)(bid & 7) * xcd_blocks + (bid >> 3);
  const int64_t g0 = logical * 16;  // the workgroup's first cell
  if (g0 >= A.n_cells) return;     // uniform over the workgroup
  const int64_t c0 = g0 + 4 * w;
  if (c0 < A.n_cells)
    wave_forward_quad<METHOD, mfma_steps(N)>(A, N, c0, lane, lds + w * kQuadDoubles, false);
  __syncthreads();
  group_store(A, N, g0, lds);
}

}  // namespace dragexp
