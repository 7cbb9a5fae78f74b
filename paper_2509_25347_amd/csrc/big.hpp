// big.hpp -- the forward update for N = 17..32 species: one cell per
// wavefront, the reduced N x N matrix (lane.hpp) in a 32 x 32 tile held as
// 2 x 2 blocks of the 16 x 16 MFMA D layout:
//     block b = 2 I + J, register v of lane 16 g + j:
//     row 16 I + 4 v + g, column 16 J + j.
// The Taylor polynomial is evaluated by Horner in the structured matrix
// M = 2^-s At = -diag(b) - 1 pb^T on the vector ALU (F <- (F + c I) M costs
// a row sum and one FMA per element, no powers to keep), the s squarings
// and the apply are dense 32 x 32 products: eight 16 x 16 block products of
// four FP64 MFMAs, the A operands through a 32 x 33 LDS tile.  Same Alg. 1,
// norm, bad-cell rules and reduced form as the other kernels.  Beyond the
// 16 species of the paper's performance runs (its 20-species Collisions
// test is the use), so this path is built for coverage, not tuned.
#pragma once

#include "common.hpp"
#include "wave.hpp"

namespace dragexp {

constexpr int kBigMaxSpecies = 32;
constexpr int kBigStride = 33;
constexpr int kBigTile = 32 * kBigStride;
// per wavefront: tile | a[32] | e[32] | p[32] | velocities [3][33]
constexpr int kBigDoubles = kBigTile + 3 * 32 + 3 * 33;

__device__ __forceinline__ double row_sum16(double x) {
  x = x + row_ror64<8>(x);
  x = x + row_ror64<4>(x);
  x = x + row_ror64<2>(x);
  return x + row_ror64<1>(x);
}

// stage the four blocks (plus `diag` on the diagonal) into the LDS tile
__device__ __forceinline__ void big_stage(double* t, int g, int j, const v4d (&X)[4], double diag) {
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int J = 0; J < 2; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        t[(16 * I + 4 * v + g) * kBigStride + 16 * J + j] =
            X[2 * I + J][v] + ((I == J && 4 * v + g == j) ? diag : 0.0);
  __builtin_amdgcn_wave_barrier();
}

// A operand of block (I, K) of the staged tile, steps t = 0..3
__device__ __forceinline__ void big_a_ops(const double* t, int g, int j, int I, int K,
                                          double (&A)[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) A[s] = t[(16 * I + j) * kBigStride + 16 * K + 4 * s + g];
}

// C = staged * Y (32 x 32)
__device__ __forceinline__ void big_product(const double* t, int g, int j, const v4d (&Y)[4],
                                            v4d (&C)[4]) {
  double A0[4], A1[4];
#pragma unroll
  for (int I = 0; I < 2; ++I) {
    big_a_ops(t, g, j, I, 0, A0);
    big_a_ops(t, g, j, I, 1, A1);
#pragma unroll
    for (int J = 0; J < 2; ++J) {
      double B0[4], B1[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        B0[s] = Y[J][s];
        B1[s] = Y[2 + J][s];
      }
      C[2 * I + J] = mma16(A0, B0, mma16(A1, B1, v4d{0.0, 0.0, 0.0, 0.0}));
    }
  }
  __builtin_amdgcn_wave_barrier();
}

__global__ void __launch_bounds__(256) k_forward_big(CellArgs A, const int N, int xcd_blocks) {
  __shared__ double lds[4 * kBigDoubles];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, j = lane & 15;
  const int bid = blockIdx.x;
  const int64_t logical = (int64_t)(bid & 7) * xcd_blocks + (bid >> 3);
  const int64_t c = logical * 4 + w;  // this wavefront's cell
  if (c >= A.n_cells) return;         // uniform over the wavefront
  const int64_t ld = A.ld;
  const int D = A.n_dim, n1 = N + 1;
  double* tile = lds + w * kBigDoubles;
  double* qa = tile + kBigTile;
  double* qe = qa + 32;
  double* qp = qe + 32;
  double* vs = qp + 32;

  // set-up: lane l < N holds species l
  const double rg = A.rho_g[c];
  unsigned bad = gas_bad(rg);
  double al = 0.0, el = 0.0, pl = 0.0;
  if (lane < N) {
    const double t = A.t_stop[lane * ld + c];
    const double r = A.rho_d[lane * ld + c];
    bad |= species_bad(t, r);
    const Species sp = species_coeffs(A.dt, t, r, rg);
    al = sp.a;
    el = sp.e;
    pl = sp.p;
  }
  const bool all_fin = __all(isfinite(al) && isfinite(pl));
  {  // OR of the bad bits over the wavefront
    unsigned any = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (__any((bad >> b) & 1u)) any |= 1u << b;
    bad = any;
  }
  if (lane < 32) {
    qa[lane] = al;
    qe[lane] = el;
    qp[lane] = pl;
  }
  for (int f = lane; f < D * n1; f += 64) vs[f] = A.v_in[(int64_t)f * ld + c];
  __builtin_amdgcn_wave_barrier();
  // ||A||_1 and sigma in the defining order (ascending species, one rounding
  // per addition), as uniform scalars
  double s_row = 0.0, sig = 1.0;
  for (int l = 0; l < N; ++l) {
    s_row = s_row + qp[l];
    sig = sig + qe[l];
  }
  double nrm = s_row;
  for (int l = 0; l < N; ++l) nrm = nrm + qa[l];
  for (int l = 0; l < N; ++l) nrm = fmax(nrm, qp[l] + qa[l]);
  if (!bad && !(all_fin && isfinite(nrm))) bad = kBadNorm;
  bool vfin = true;
  for (int f = lane; f < D * n1; f += 64) vfin = vfin && isfinite(vs[f]);
  if (!__all(vfin) && !bad) bad = kBadVelocity;
  if (bad) {
    for (int f = lane; f < D * n1; f += 64) A.v_out[(int64_t)f * ld + c] = __builtin_nan("");
    if (lane == 0) atomicOr(&g_status_word, bad);
    return;
  }
  const Kms km = select_kms(nrm, A.k_max, A.option);
  const int m = km.m, s = km.s;

  // column coefficients of this lane (column 16 J + j) and the row mask
  double nbc[2], npbc[2];
#pragma unroll
  for (int J = 0; J < 2; ++J) {
    const int col = 16 * J + j;
    nbc[J] = col < N ? -ldexp(qa[col], -s) : 0.0;
    npbc[J] = col < N ? -ldexp(qp[col], -s) : 0.0;
  }

  // Horner in M: F <- (F + c_i I) M, i = m..1, gives T_m(M) - I
  v4d F[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) F[b] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int i = m; i >= 1; --i) {
    const double ci = kInvFact[i];
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (4 * v + g == j && 16 * I + 4 * v + g < N) F[3 * I][v] += ci;
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double rs = row_sum16(F[2 * I][v] + F[2 * I + 1][v]);
#pragma unroll
        for (int J = 0; J < 2; ++J) F[2 * I + J][v] = fma(F[2 * I + J][v], nbc[J], rs * npbc[J]);
      }
  }

  // s squarings Z <- (Z + 2 I) Z
  for (int it = 0; it < s; ++it) {
    big_stage(tile, g, j, F, 2.0);
    v4d Cn[4];
    big_product(tile, g, j, F, Cn);
#pragma unroll
    for (int b = 0; b < 4; ++b) F[b] = Cn[b];
  }

  // u = Z dv for every component (B operand: lane (g, j < D) holds the
  // relative velocities of rows 16 K + 4 t + g, component j)
  v4d Bd[4];
#pragma unroll
  for (int K = 0; K < 2; ++K)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = 16 * K + 4 * t + g;
      Bd[2 * K][t] = (j < D && r < N) ? vs[j * n1 + 1 + r] - vs[j * n1] : 0.0;
      Bd[2 * K + 1][t] = 0.0;
    }
  big_stage(tile, g, j, F, 0.0);
  v4d U[4];
  big_product(tile, g, j, Bd, U);  // column block 0 holds the components
  double eu = 0.0;
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * I + 4 * v + g;
      eu = fma(r < N ? qe[r] : 0.0, U[2 * I][v], eu);
    }
  eu = sum_rows(eu);
  const double d0 = -eu / sig;
  __builtin_amdgcn_wave_barrier();
  if (j < D) {
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * I + 4 * v + g;
        if (r < N) vs[j * n1 + 1 + r] = vs[j * n1 + 1 + r] + (d0 + U[2 * I][v]);
      }
    if (g == 0) vs[j * n1] = vs[j * n1] + d0;
  }
  __builtin_amdgcn_wave_barrier();
  for (int f = lane; f < D * n1; f += 64) A.v_out[(int64_t)f * ld + c] = vs[f];
}

}  // namespace dragexp
