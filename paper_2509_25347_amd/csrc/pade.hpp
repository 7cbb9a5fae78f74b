// pade.hpp -- the diagonal Pade scaling step on the MFMA tile (Sect. 2.3,
// eq. PadeEqu with p = q = m), as an alternative to the Taylor stage.
//
// Included by wave.hpp inside namespace dragexp, after its tile helpers
// (v4d, the D layout, mul_M, stage_tile); not a header of its own.
//
// For the scaled reduced matrix M (N x N in a 16 x 16 tile), with V and U
// the even and odd parts of the numerator N_mm(M) = sum_j c_j M^j, the
// denominator is D_mm(M) = V - U, and
//     Z = r_m(M) - I = (V - U)^-1 (2 U),
// the Y form the squarings take (no cancellation for small M).  The powers
// are structured products on the vector ALU (mul_M); the solve is a
// Gauss-Jordan elimination over the wavefront with partial pivoting done by
// row choice rather than row swaps: step k picks the unused row p with the
// largest |D[p][k]|, removes column k from every other row, and at the end
// row p holds piv_k * e_k on the left and piv_k * Z[k] on the right, so Z is
// gathered by one LDS pass that writes row p to row k.
#pragma once

// Degrees and theta_m of the diagonal approximant r_m: the largest theta for
// which the backward error series log(e^-x r_m(x)) = sum_{k>2m} c_k x^k has
// sum_k |c_k| theta^(k-1) <= 2^-53 (the criterion eq. B8 puts on the Taylor
// polynomial), evaluated in multiprecision.
constexpr int kPadeRows = 5;
constexpr int kPadeM[kPadeRows] = {3, 5, 7, 9, 13};
constexpr double kPadeTheta[kPadeRows] = {
    1.4955852179582915e-02, 2.539398330063232e-01, 9.504178996162932e-01,
    2.0978479612570675e+00, 5.371920351148153e+00,
};
// c_j = (2m - j)! m! / ((2m)! j! (m - j)!), j = 0..m, correctly rounded
// (the numerator's coefficients; the denominator's are (-1)^j c_j).
constexpr double kPadeC[kPadeRows][14] = {
    {1.0, 0.5, 0.1, 0.008333333333333333},
    {1.0, 0.5, 0.1111111111111111, 0.013888888888888888, 0.000992063492063492,
     3.306878306878307e-05},
    {1.0, 0.5, 0.11538461538461539, 0.016025641025641024, 0.001456876456876457,
     8.741258741258741e-05, 3.2375032375032376e-06, 5.781255781255781e-08},
    {1.0, 0.5, 0.11764705882352941, 0.01715686274509804, 0.001715686274509804,
     0.00012254901960784314, 6.2845651080945196e-06, 2.2444875386051856e-07,
     5.101108042284513e-09, 5.66789782476057e-11},
    {1.0, 0.5, 0.12, 0.018333333333333333, 0.0019927536231884057, 0.00016304347826086958,
     1.0351966873706003e-05, 5.175983436853002e-07, 2.0431513566525008e-08,
     6.306022705717595e-10, 1.48377004840414e-11, 2.529153491597966e-13,
     2.8101705462199623e-15, 1.5440497506703088e-17},
};

// Row of the table and s for a finite ||A||_1: the lowest degree whose theta
// covers the norm (s = 0), else m = 13 and the smallest s with
// ||A|| <= theta_13 2^s (exact power-of-two comparisons).
struct PadeSel {
  int row, s;
};

__host__ __device__ inline PadeSel pade_select(double nrm) {
  for (int i = 0; i < kPadeRows - 1; ++i)
    if (nrm <= kPadeTheta[i]) return PadeSel{i, 0};
  int sh = 0;
  while (nrm > ldexp(kPadeTheta[kPadeRows - 1], sh)) ++sh;
  return PadeSel{kPadeRows - 1, sh};
}

// Z = r_m(M) - I for the cell on this wavefront (row = Pade table row).
__device__ __forceinline__ v4d pade_stage(const v4d& M, const QuadRows& R, const double (&rm)[4],
                                          int row, int N, double* stage, int g, int j) {
  const int m = kPadeM[row];
  const double* c = kPadeC[row];
  // numerator parts: V (even powers, c_0 I on the N x N block), U (odd)
  v4d P = M, U, V;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    U[v] = c[1] * M[v];
    V[v] = (4 * v + g == j) ? c[0] * rm[v] : 0.0;
  }
  for (int jj = 2; jj <= m; ++jj) {
    P = mul_M(P, R, rm);
    const double cj = c[jj];
    if (jj & 1) {
#pragma unroll
      for (int v = 0; v < 4; ++v) U[v] = fma(cj, P[v], U[v]);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) V[v] = fma(cj, P[v], V[v]);
    }
  }
  // Gauss-Jordan on [V - U | 2 U]; the padding rows stay zero
  v4d A, B;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    A[v] = V[v] - U[v];
    B[v] = 2.0 * U[v];
  }
  int col[4] = {0, 0, 0, 0};       // the pivot column each of my rows took
  double dpiv[4] = {1.0, 1.0, 1.0, 1.0};
  unsigned used = 0;                // pivot rows so far (uniform)
  for (int k = 0; k < N; ++k) {
    // candidates of column k: my rows 4 v + g, unused and below N
    double best = -1.0;
    int best_r = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * v + g;
      const double a = (r < N && !((used >> r) & 1u)) ? fabs(A[v]) : -1.0;
      if (a > best) {
        best = a;
        best_r = r;
      }
    }
    // the largest over the four lane groups of column k (ties: lowest row)
    double pbest = -1.0;
    int p = 0;
#pragma unroll
    for (int gg = 0; gg < 4; ++gg) {
      const double b = readlane_f64(best, 16 * gg + k);
      const int br = __builtin_amdgcn_readlane(best_r, 16 * gg + k);
      if (b > pbest || (b == pbest && br < p)) {
        pbest = b;
        p = br;
      }
    }
    used |= 1u << p;
    const int vp = p >> 2, gp = p & 3;
    // the pivot row's entries of my column, and the pivot itself
    const double xa = vp == 0 ? A[0] : vp == 1 ? A[1] : vp == 2 ? A[2] : A[3];
    const double xb = vp == 0 ? B[0] : vp == 1 ? B[1] : vp == 2 ? B[2] : B[3];
    const double pa = __shfl(xa, 16 * gp + j, 64);
    const double pb = __shfl(xb, 16 * gp + j, 64);
    const double piv = readlane_f64(xa, 16 * gp + k);
    const double rpiv = 1.0 / piv;
    // eliminate column k from every other row
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * v + g;
      const double f = __shfl(A[v], 16 * g + k, 64) * rpiv;
      if (r == p) {
        col[v] = k;
        dpiv[v] = piv;
      } else if (r < N) {
        A[v] = fma(-f, pa, A[v]);
        B[v] = fma(-f, pb, B[v]);
      }
    }
  }
  // row p_k holds piv_k Z[k]: scatter to row k through the staging tile
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (4 * v + g < N) stage[col[v] * kLdsStride + j] = B[v] / dpiv[v];
  __builtin_amdgcn_wave_barrier();
  v4d Z;
#pragma unroll
  for (int v = 0; v < 4; ++v) Z[v] = (4 * v + g < N) ? stage[(4 * v + g) * kLdsStride + j] : 0.0;
  __builtin_amdgcn_wave_barrier();
  return Z;
}
