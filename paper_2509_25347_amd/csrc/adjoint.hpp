// adjoint.hpp -- fused forward + adjoint of v' = exp(dt K) v.
//
// Loss L = sum_{c,j} w[c][j] v'[c][j] (w = dL/dv', c the velocity component).
// In the relative-velocity form (lane.hpp) with W_c = sum_j w[c][j],
//     L = sum_c ( w_c . v_c + ubar_c . (Z dv_c) ),
//     ubar_c[i] = w_c[1+i] - W_c e_i / sigma,
// so Z enters through <G, Z> with G = sum_c ubar_c dv_c^T, and
//     dL/dAt = L_R(At^T, G),
// the Frechet derivative of the approximant R(X) = T_m(2^-s X)^(2^s) at At^T
// in the direction G (the adjoint of a real matrix polynomial's derivative is
// its derivative at the transpose).  It is evaluated forward-mode alongside
// R(At^T) itself, with (k*, m*, s*) held fixed and nothing stored:
//     B = 2^-s At^T,  dB = 2^-s G,
//     powers        P_j = B P_{j-1},  dP_j = dB P_{j-1} + B dP_{j-1},
//     Horner        F <- Bbar_k + F P_q,  dF <- dBbar_k + dF P_q + F dP_q,
//     squarings     Y <- 2Y + Y Y,        dY <- 2dY + dY Y + Y dY.
// At the end Y = Z^T (the forward result, transposed) and dY = dL/dAt.  The
// chain rule through At_jk = -a_j [j == k] - e_k a_k, a = dt/t, e = rho/rho_g
// and the direct dependence of the gas update on e gives the parameter
// gradients; dL/dv follows from dv = v_dust - v_gas and Z^T ubar.
#pragma once

#include "common.hpp"
#include "lane.hpp"
#include "wave.hpp"

namespace dragexp {

// ---- one cell per lane --------------------------------------------------------

// At N = 6 the kernel needs 291 registers (1 wave/SIMD); bounding it to 2
// waves spills 63 VGPRs to scratch and still runs 13-17 % faster.  At N = 7
// the same bound spills 438 and runs 2.9x slower, so it keeps 1.
template <int N>
__global__ void __launch_bounds__(256, N == 6 ? 2 : 1) k_backward_lane(BackArgs A, int xcd_blocks) {
  const int bid = blockIdx.x;
  const int64_t logical = (int64_t)(bid & 7) * xcd_blocks + (bid >> 3);
  const int64_t c = logical * 256 + threadIdx.x;
  const bool active = c < A.n_cells;
  const int64_t cc = active ? c : 0;
  const int64_t ld = A.ld;
  const int n1 = N + 1;
  const int D = A.n_dim;

  LaneCell<N> C;
  lane_setup<N>(C, A.rho_g, A.rho_d, A.t_stop, ld, cc, A.dt, A.k_max, A.option);
  bool fin = true;
  for (int d = 0; d < D; ++d) {
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      const int64_t idx = (int64_t)(d * n1 + j) * ld + cc;
      fin = fin && isfinite(A.v_in[idx]) && isfinite(A.w[idx]);
    }
  }
  if (!fin && !C.bad) {
    C.bad = kBadVelocity;
#pragma unroll
    for (int i = 0; i < N; ++i) C.a[i] = C.e[i] = C.p[i] = 0.0;
    C.sigma = 1.0;
    C.kms = select_kms(0.0, A.k_max, A.option);
  }
  const int s = C.kms.s;

  // dB = 2^-s G, G = sum_c ubar_c dv_c^T
  double dB[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < N; ++k) dB[i][k] = 0.0;
  if (!C.bad) {
    for (int d = 0; d < D; ++d) {
      double v[N + 1], w[N + 1];
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        const int64_t idx = (int64_t)(d * n1 + j) * ld + cc;
        v[j] = A.v_in[idx];
        w[j] = A.w[idx];
      }
      double W = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) W += w[j];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const double ub = w[i + 1] - W * C.e[i] / C.sigma;
#pragma unroll
        for (int k = 0; k < N; ++k) dB[i][k] = fma(ub, v[k + 1] - v[0], dB[i][k]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < N; ++k) dB[i][k] = ldexp(dB[i][k], -s);

  double b[N], pb[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    b[i] = ldexp(C.a[i], -s);
    pb[i] = ldexp(C.p[i], -s);
  }

  // Taylor stage and its derivative, Horner in B = M^T:
  // B_jk = -b_j [j == k] - pb_j, so (H B)_ik = -H_ik b_k - (H pb)_i.
  double Y[N][N], dY[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < N; ++k) Y[i][k] = dY[i][k] = 0.0;
  const int m_max = wave_max_int(C.kms.m);
  for (int it = m_max; it >= 1; --it) {
    const double cf = (it <= C.kms.m) ? kInvFact[it] : 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double h[N];
#pragma unroll
      for (int k = 0; k < N; ++k) h[k] = Y[i][k] + (k == i ? cf : 0.0);
      double hp = 0.0, fp = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        hp = fma(h[k], pb[k], hp);
        fp = fma(dY[i][k], pb[k], fp);
      }
#pragma unroll
      for (int k = 0; k < N; ++k) {
        double acc = fma(-dY[i][k], b[k], -fp);
#pragma unroll
        for (int l = 0; l < N; ++l) acc = fma(h[l], dB[l][k], acc);
        dY[i][k] = acc;
        Y[i][k] = fma(-h[k], b[k], -hp);
      }
    }
  }

  // squarings with the Frechet recurrence, the 2 Y and 2 dY terms folded
  // into the right factor Y + 2 I:
  //   dY <- dY (Y + 2I) + Y dY,   Y <- Y (Y + 2I)
  const int s_max = wave_max_int(s);
  for (int it = 0; it < s_max; ++it) {
    if (it < s) {
      double d2[N];
#pragma unroll
      for (int l = 0; l < N; ++l) d2[l] = Y[l][l] + 2.0;
      double T[N][N];
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k) {
          double acc = dY[i][0] * (k == 0 ? d2[0] : Y[0][k]);
#pragma unroll
          for (int l = 1; l < N; ++l) acc = fma(dY[i][l], l == k ? d2[l] : Y[l][k], acc);
#pragma unroll
          for (int l = 0; l < N; ++l) acc = fma(Y[i][l], dY[l][k], acc);
          T[i][k] = acc;
        }
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k) dY[i][k] = T[i][k];
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k) {
          double acc = Y[i][0] * (k == 0 ? d2[0] : Y[0][k]);
#pragma unroll
          for (int l = 1; l < N; ++l) acc = fma(Y[i][l], l == k ? d2[l] : Y[l][k], acc);
          T[i][k] = acc;
        }
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int k = 0; k < N; ++k) Y[i][k] = T[i][k];
    }
  }

  // outputs: Y = Z^T, dY = dL/dAt.  The species coefficients are recomputed
  // from the inputs (same roundings) so they need not stay live in VGPRs
  // through the squarings.
  const double qnan = __builtin_nan("");
  const double rg = A.rho_g[cc];
  double ea[N], aa[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const Species sp = species_coeffs(A.dt, A.t_stop[k * ld + cc], A.rho_d[k * ld + cc], rg);
    ea[k] = C.bad ? 0.0 : sp.e;
    aa[k] = C.bad ? 0.0 : sp.a;
  }
  const double sigma = C.sigma;
  double ge_dir[N];
#pragma unroll
  for (int k = 0; k < N; ++k) ge_dir[k] = 0.0;
  for (int d = 0; d < D; ++d) {
    double v[N + 1], w[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      const int64_t idx = (int64_t)(d * n1 + j) * ld + cc;
      v[j] = A.v_in[idx];
      w[j] = A.w[idx];
    }
    double W = 0.0;
#pragma unroll
    for (int j = 0; j <= N; ++j) W += w[j];
    double dv[N], u[N], ub[N];
#pragma unroll
    for (int k = 0; k < N; ++k) dv[k] = v[k + 1] - v[0];
    double eu = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) acc = fma(Y[k][i], dv[k], acc);  // (Z dv)_i
      u[i] = acc;
      eu = fma(ea[i], acc, eu);
      ub[i] = w[i + 1] - W * ea[i] / sigma;
    }
    const double d0 = -eu / sigma;
    double zt_sum = 0.0, zt[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) acc = fma(Y[j][k], ub[k], acc);  // (Z^T ubar)_j
      zt[j] = acc;
      zt_sum += acc;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) ge_dir[k] = fma(-d0 - u[k], W / sigma, ge_dir[k]);
    if (active) {
      if (A.v_out) {
        A.v_out[(int64_t)(d * n1) * ld + c] = C.bad ? qnan : v[0] + d0;
#pragma unroll
        for (int j = 0; j < N; ++j)
          A.v_out[(int64_t)(d * n1 + 1 + j) * ld + c] = C.bad ? qnan : v[j + 1] + (d0 + u[j]);
      }
      if (A.g_v) {
        A.g_v[(int64_t)(d * n1) * ld + c] = C.bad ? qnan : w[0] - zt_sum;
#pragma unroll
        for (int j = 0; j < N; ++j)
          A.g_v[(int64_t)(d * n1 + 1 + j) * ld + c] = C.bad ? qnan : w[j + 1] + zt[j];
      }
    }
  }
  if (active) {
    double sum_ege = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double col = 0.0;
#pragma unroll
      for (int j = 0; j < N; ++j) col += dY[j][k];
      const double ga = -dY[k][k] - ea[k] * col;
      const double ge = -aa[k] * col + ge_dir[k];
      const double glt = -aa[k] * ga;
      sum_ege = fma(ea[k], ge, sum_ege);
      if (A.g_logt) A.g_logt[k * ld + c] = C.bad ? qnan : glt;
      if (A.g_t) A.g_t[k * ld + c] = C.bad ? qnan : glt / A.t_stop[k * ld + c];
      if (A.g_rho_d) A.g_rho_d[k * ld + c] = C.bad ? qnan : ge / rg;
    }
    if (A.g_rho_g) A.g_rho_g[c] = C.bad ? qnan : -sum_ege / rg;
    if (C.bad) atomicOr(&g_status_word, C.bad);
  }
}

// ---- MFMA adjoint, N = 9..16: a quad of cells per wavefront ---------------------
//
// The recurrences run on separate 16 x 16 tiles for Y and dY.  As in the
// forward kernel the B operand of every product comes straight from the D
// layout and only A operands are staged through LDS; products by B = M^T
// (diagonal plus rank one: (B X)[r][c] = -b_r X[r][c] - pb_r sum_l X[l][c])
// run on the vector ALU; a squaring step is
//     Y' = (Y + 2I) Y,   dY' = dY Y + (Y + 2I) dY,
// with Y + 2I formed in the staged copy by one LDS add on the diagonal.

__device__ __forceinline__ double groups_sum(double x) { return sum_rows(x); }

// X <- B X for B = M^T (rows >= N stay zero: nb, npb are zero there).
__device__ __forceinline__ v4d mul_Bt(const v4d& X, const double (&nb)[4], const double (&npb)[4]) {
  const double cs = sum_rows(X[0] + X[1] + X[2] + X[3]);  // column sums of X
  v4d Y;
#pragma unroll
  for (int v = 0; v < 4; ++v) Y[v] = fma(nb[v], X[v], npb[v] * cs);
  return Y;
}

// T_m(B) - I and its derivative in the direction dB by the Paterson-Stockmeyer
// scheme with Q powers: P_p = B P_{p-1} (structured), dP_p = dB P_{p-1} +
// B dP_{p-1}; Horner F <- Bbar_k + F P_Q, dF <- dBbar_k + dF P_Q + F dP_Q.
template <int Q, int KT = 4>
__device__ __forceinline__ void bwd_poly(const v4d& Bt, const v4d& dB, const double (&dBA)[4],
                                         const double (&nb)[4], const double (&npb)[4], int r,
                                         double* stage, double* stage2, int g, int j, v4d& F,
                                         v4d& dF) {
  const v4d zero4 = {0.0, 0.0, 0.0, 0.0};
  v4d P[Q + 1], dP[Q + 1];
  P[1] = Bt;
  dP[1] = dB;
#pragma unroll
  for (int p = 2; p <= Q; ++p) {
    double Bp[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) Bp[t] = P[p - 1][t];
    P[p] = mul_Bt(P[p - 1], nb, npb);
    dP[p] = mma_k<KT>(dBA, Bp, mul_Bt(dP[p - 1], nb, npb));
  }
  double Bq[4], dBq[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    Bq[t] = P[Q][t];
    dBq[t] = dP[Q][t];
  }
  auto comb = [&](const v4d (&X)[Q + 1], int k) {
    v4d acc = zero4;
#pragma unroll
    for (int p = 1; p <= Q; ++p) {
      const double cf = kInvFact[Q * k + p];
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = fma(cf, X[p][v], acc[v]);
    }
    return acc;
  };
  F = comb(P, r - 1);
  dF = comb(dP, r - 1);
  for (int k = r - 2; k >= 0; --k) {
    double AF[4], AdF[4];
    stage_tile(stage, g, j, F);
    stage_tile(stage2, g, j, dF);
    load_a_ops<KT>(stage, g, j, AF);
    load_a_ops<KT>(stage2, g, j, AdF);
    dF = mma_k<KT>(AF, dBq, mma_k<KT>(AdF, Bq, comb(dP, k)));
    F = mma_k<KT>(AF, Bq, comb(P, k));
  }
}

// KT: MFMA steps per product (mfma_steps(N) for a compile-time N, else 4).
template <int KT = 4>
__device__ __forceinline__ void wave_backward_quad(const BackArgs& A, const int N, int64_t c0,
                                                   int lane, double* lds) {
  const int g = lane >> 4, j = lane & 15;
  const int64_t ld = A.ld;
  const int n1 = N + 1;
  const int D = A.n_dim;
  const v4d zero4 = {0.0, 0.0, 0.0, 0.0};
  double* stage = lds;                    // Y (and F) staging
  double* stage2 = lds + kQuadDoubles;    // dY (and dF, dB) staging
  double* qa = lds + kStageDoubles;
  double* qe = qa + 64;
  double* qp = qe + 64;

  const QuadCell Q = quad_setup(A.rho_g, A.rho_d, A.t_stop, A.n_cells, ld, A.dt, A.k_max,
                                A.option, N, c0, g, j, qa, qe, qp);
  const double rsig_q = 1.0 / Q.sig;  // 1 / sigma of the row's cell
  const int diag_slot = j * kLdsStride + j;

  // velocity and weight data, lane (g = component, j = species)
  const bool comp = g < D;
  const bool cj = comp && j < N;
  auto load_vw = [&](int64_t cell, double& v0, double& vj, double& w0, double& wj) {
    v0 = vj = w0 = wj = 0.0;
    if (comp && cell < A.n_cells) {
      const int64_t base = (int64_t)(g * n1) * ld + cell;
      v0 = A.v_in[base];
      w0 = A.w[base];
      if (j < N) {
        vj = A.v_in[base + (int64_t)(1 + j) * ld];
        wj = A.w[base + (int64_t)(1 + j) * ld];
      }
    }
  };
  double v0n, vjn, w0n, wjn;
  load_vw(c0, v0n, vjn, w0n, wjn);

#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    const int64_t cell = c0 + c;
    if (cell >= A.n_cells) break;  // uniform
    const double v0 = v0n, vj = vjn, w0 = w0n, wj = wjn;
    if (c < 3) load_vw(cell + 1, v0n, vjn, w0n, wjn);  // prefetch the next cell

    unsigned bad = (unsigned)__builtin_amdgcn_readlane((int)Q.bad, 16 * c);
    const bool fin = isfinite(v0) && isfinite(vj) && isfinite(w0) && isfinite(wj);
    if (!__all(fin) && !bad) bad = kBadVelocity;
    if (bad) {
      const double qnan = __builtin_nan("");
      if (lane < D * n1) {
        if (A.v_out) A.v_out[(int64_t)lane * ld + cell] = qnan;
        if (A.g_v) A.g_v[(int64_t)lane * ld + cell] = qnan;
      }
      if (lane < N) {
        if (A.g_logt) A.g_logt[lane * ld + cell] = qnan;
        if (A.g_t) A.g_t[lane * ld + cell] = qnan;
        if (A.g_rho_d) A.g_rho_d[lane * ld + cell] = qnan;
      }
      if (lane == 0) {
        if (A.g_rho_g) A.g_rho_g[cell] = qnan;
        atomicOr(&g_status_word, bad);
      }
      continue;
    }
    const int kp = __builtin_amdgcn_readlane(Q.kpack, 16 * c);
    const int kk = kp & 15, s = kp >> 4;
    const int q = kTabQ[kk], r = kTabR[kk];
    const double rsig = readlane_f64(rsig_q, 16 * c);

    const int sj = 16 * c + quad_slot(j);
    const double ej = qe[sj], aj = qa[sj], nbj = -ldexp(aj, -s);
    double nb[4], npb[4];  // -b, -pb of rows 4 v + g
    {
      const double* ra = qa + 16 * c + 4 * g;
      const double* rp = qp + 16 * c + 4 * g;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        nb[v] = -ldexp(ra[v], -s);
        npb[v] = -ldexp(rp[v], -s);
      }
    }
    __builtin_amdgcn_wave_barrier();

    const double Wsum = row_chain(w0, cj ? wj : 0.0, N);  // W_c of this lane's component
    const double dv = cj ? vj - v0 : 0.0;
    const double ub = cj ? wj - Wsum * ej * rsig : 0.0;

    // dB = 2^-s G, G = Ubar dV^T: one MFMA with k = the velocity component
    v4d dB = __builtin_amdgcn_mfma_f64_16x16x4f64(ub, dv, zero4, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) dB[v] = ldexp(dB[v], -s);
    double dBA[4];
    stage_tile(stage2, g, j, dB);
    load_a_ops<KT>(stage2, g, j, dBA);

    // B = M^T: B[row][col] = -b_row [row == col] - pb_row
    v4d Bt;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double dg = (4 * v + g == j) ? 1.0 : 0.0;
      Bt[v] = (j < N) ? fma(dg, nbj, npb[v]) : 0.0;
    }
    v4d F, dF;
    switch (q) {  // uniform; one code path per power count
      case 1: bwd_poly<1, KT>(Bt, dB, dBA, nb, npb, r, stage, stage2, g, j, F, dF); break;
      case 2: bwd_poly<2, KT>(Bt, dB, dBA, nb, npb, r, stage, stage2, g, j, F, dF); break;
      case 3: bwd_poly<3, KT>(Bt, dB, dBA, nb, npb, r, stage, stage2, g, j, F, dF); break;
      case 4: bwd_poly<4, KT>(Bt, dB, dBA, nb, npb, r, stage, stage2, g, j, F, dF); break;
      default: bwd_poly<5, KT>(Bt, dB, dBA, nb, npb, r, stage, stage2, g, j, F, dF); break;
    }

    // squarings with the Frechet recurrence
    v4d Y = F, dY = dF;
    for (int it = 0; it < s; ++it) {
      double AY[4], AdY[4], BY[4], BdY[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        BY[t] = Y[t];
        BdY[t] = dY[t];
      }
      stage_tile(stage, g, j, Y);
      stage_tile(stage2, g, j, dY);
      if (g == 0) atomicAdd(stage + diag_slot, 2.0);
      __builtin_amdgcn_wave_barrier();
      load_a_ops<KT>(stage, g, j, AY);    // Y + 2I
      load_a_ops<KT>(stage2, g, j, AdY);  // dY
      dY = mma_k<KT>(AdY, BY, mma_k<KT>(AY, BdY, zero4));
      Y = mma_k<KT>(AY, BY, zero4);
    }

    // Y = Z^T, dY = dL/dAt.  u_c = Z dv_c = (dV^T Y)[c];  Z^T ubar_c = (Ubar^T Z)[c]
    double YB[4], ZB[4], DvA[4], UbA[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) YB[t] = Y[t];
    stage_tile(stage, g, j, Y);
    load_a_ops<KT>(stage, g, j, ZB);  // Z = Y^T as the B operand
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      // A operand rows are components: lane (g, i) takes component i, species 4t+g
      const int src = (j < D) ? 16 * j + 4 * t + g : 0;
      const double a1 = __shfl(dv, src, 64), a2 = __shfl(ub, src, 64);
      DvA[t] = (j < D) ? a1 : 0.0;
      UbA[t] = (j < D) ? a2 : 0.0;
    }
    const v4d Um = mma_k<KT>(DvA, YB, zero4);  // lane (g, j) [0]: u_g[j]
    const v4d Vm = mma_k<KT>(UbA, ZB, zero4);  // lane (g, j) [0]: (Z^T ubar_g)_j
    const double u = cj ? Um[0] : 0.0;
    const double zt = cj ? Vm[0] : 0.0;
    const double eu = row_chain(0.0, ej * u, N);
    const double d0 = -eu * rsig;
    const double zt_sum = row_chain(0.0, zt, N);
    if (comp) {
      const int64_t base = (int64_t)(g * n1) * ld + cell;
      if (A.v_out) {
        if (j < N) A.v_out[base + (int64_t)(1 + j) * ld] = vj + (d0 + u);
        if (j == 0) A.v_out[base] = v0 + d0;
      }
      if (A.g_v) {
        if (j < N) A.g_v[base + (int64_t)(1 + j) * ld] = wj + zt;
        if (j == 0) A.g_v[base] = w0 - zt_sum;
      }
    }
    // direct dependence of the gas update on e, summed over components
    const double ge_dir = groups_sum(cj ? (-d0 - u) * (Wsum * rsig) : 0.0);
    // column sums and diagonal of dL/dAt (D layout: rows 4v+g of column j)
    const double col = groups_sum(dY[0] + dY[1] + dY[2] + dY[3]);
    double dg = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (4 * v + g == j) dg = dY[v];
    dg = groups_sum(dg);
    if (g == 0) {
      const double rrg = 1.0 / A.rho_g[cell];
      double ge = 0.0;
      if (j < N) {
        const double ga = -dg - ej * col;
        ge = -aj * col + ge_dir;
        const double glt = -aj * ga;
        if (A.g_logt) A.g_logt[j * ld + cell] = glt;
        if (A.g_t) A.g_t[j * ld + cell] = glt / A.t_stop[j * ld + cell];
        if (A.g_rho_d) A.g_rho_d[j * ld + cell] = ge * rrg;
      }
      const double sum_ege = row_chain(0.0, ej * ge, N);
      if (j == 0 && A.g_rho_g) A.g_rho_g[cell] = -sum_ege * rrg;
    }
  }
}

// 3 waves/SIMD: 23 VGPRs spill (194 registers otherwise, 2 waves), and the
// third wavefront still makes it 5-7 % faster (interleaved timings, N = 11-16).
template <int N>
__global__ void __launch_bounds__(256, 3) k_backward_wave(BackArgs A, int xcd_blocks) {
  // per wavefront: the quad block (staging tile + coefficient tables) and a
  // second staging tile
  __shared__ double lds[4 * (kQuadDoubles + kStageDoubles)];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int bid = blockIdx.x;
  const int64_t logical = (int64_t)(bid & 7) * xcd_blocks + (bid >> 3);
  const int64_t c0 = (logical * 4 + w) * 4;
  if (c0 >= A.n_cells) return;  // uniform over the wavefront
  wave_backward_quad<mfma_steps(N)>(A, N, c0, lane, lds + w * (kQuadDoubles + kStageDoubles));
}

// ---- N <= 8: the block form on one 16 x 16 tile -------------------------------
//
// For a polynomial f, f([[X, E], [0, X]]) = [[f(X), L_f(X, E)], [0, f(X)]],
// and the approximant R is a polynomial stage followed by squarings, so one
// evaluation of R on the 2N x 2N block matrix
//     Xh = [[B, dB], [0, B]],  B = 2^-s At^T,  dB = 2^-s G
// with the same (k*, m*, s*) yields Y = R(At^T) - I and dY = L_R(At^T, G)
// together: each squaring Yh <- 2 Yh + Yh Yh is one 16 x 16 product instead
// of the three of the separate recurrences.  The blocks sit at offsets 0 and
// 8 of the tile (species i of the first block is row / column i, of the
// second 8 + i); rows and columns of species >= N are zero.  A wavefront
// takes a quad of cells, set up once as in the forward kernel.

// T_m(X) - I for a dense tile X by the Paterson-Stockmeyer scheme with Q
// powers, all products on the matrix cores (XA: X as the A operand).
template <int Q>
__device__ __forceinline__ v4d mfma_poly(const v4d& X, const double (&XA)[4], int r,
                                         double* stage, int g, int j) {
  const v4d zero4 = {0.0, 0.0, 0.0, 0.0};
  v4d P[Q + 1];
  P[1] = X;
#pragma unroll
  for (int p = 2; p <= Q; ++p) {
    double Bp[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) Bp[t] = P[p - 1][t];
    P[p] = mma16(XA, Bp, zero4);
  }
  double Bq[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) Bq[t] = P[Q][t];
  auto bbar = [&](int k) {
    v4d acc = zero4;
#pragma unroll
    for (int p = 1; p <= Q; ++p) {
      const double cf = kInvFact[Q * k + p];
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = fma(cf, P[p][v], acc[v]);
    }
    return acc;
  };
  v4d F = bbar(r - 1);
  for (int k = r - 2; k >= 0; --k) {
    double Af[4];
    stage_tile(stage, g, j, F);
    load_a_ops(stage, g, j, Af);
    F = mma16(Af, Bq, bbar(k));
  }
  return F;
}

__device__ __forceinline__ void wave_backward_block_quad(const BackArgs& A, const int N,
                                                         int64_t c0, int lane, double* lds) {
  const int g = lane >> 4, j = lane & 15;
  const int jj = j & 7;  // species of this lane's column in either block
  const int64_t ld = A.ld;
  const int n1 = N + 1;
  const int D = A.n_dim;
  const v4d zero4 = {0.0, 0.0, 0.0, 0.0};
  double* stage = lds;
  double* qa = lds + kStageDoubles;
  double* qe = qa + 64;
  double* qp = qe + 64;

  const QuadCell Q = quad_setup(A.rho_g, A.rho_d, A.t_stop, A.n_cells, ld, A.dt, A.k_max,
                                A.option, N, c0, g, j, qa, qe, qp);
  const double rsig_q = 1.0 / Q.sig;  // 1 / sigma of the row's cell
  const int diag_slot = j * kLdsStride + j;

  // velocity and weight data, lane (g = component, j): species jj
  const bool comp = g < D;
  const bool cj = comp && jj < N;
  auto load_vw = [&](int64_t cell, double& v0, double& vj, double& w0, double& wj) {
    v0 = vj = w0 = wj = 0.0;
    if (comp && cell < A.n_cells) {
      const int64_t base = (int64_t)(g * n1) * ld + cell;
      v0 = A.v_in[base];
      w0 = A.w[base];
      if (jj < N) {
        vj = A.v_in[base + (int64_t)(1 + jj) * ld];
        wj = A.w[base + (int64_t)(1 + jj) * ld];
      }
    }
  };
  double v0n, vjn, w0n, wjn;
  load_vw(c0, v0n, vjn, w0n, wjn);

#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    const int64_t cell = c0 + c;
    if (cell >= A.n_cells) break;  // uniform
    const double v0 = v0n, vj = vjn, w0 = w0n, wj = wjn;
    if (c < 3) load_vw(cell + 1, v0n, vjn, w0n, wjn);  // prefetch the next cell

    unsigned bad = (unsigned)__builtin_amdgcn_readlane((int)Q.bad, 16 * c);
    const bool fin = isfinite(v0) && isfinite(vj) && isfinite(w0) && isfinite(wj);
    if (!__all(fin) && !bad) bad = kBadVelocity;
    if (bad) {
      const double qnan = __builtin_nan("");
      if (lane < D * n1) {
        if (A.v_out) A.v_out[(int64_t)lane * ld + cell] = qnan;
        if (A.g_v) A.g_v[(int64_t)lane * ld + cell] = qnan;
      }
      if (lane < N) {
        if (A.g_logt) A.g_logt[lane * ld + cell] = qnan;
        if (A.g_t) A.g_t[lane * ld + cell] = qnan;
        if (A.g_rho_d) A.g_rho_d[lane * ld + cell] = qnan;
      }
      if (lane == 0) {
        if (A.g_rho_g) A.g_rho_g[cell] = qnan;
        atomicOr(&g_status_word, bad);
      }
      continue;
    }
    const int kp = __builtin_amdgcn_readlane(Q.kpack, 16 * c);
    const int kk = kp & 15, s = kp >> 4;
    const int q = kTabQ[kk], r = kTabR[kk];
    const double rsig = readlane_f64(rsig_q, 16 * c);

    const int sj = 16 * c + quad_slot(jj);
    const double ej = qe[sj], aj = qa[sj];
    double nb[2], npb[2];  // -b, -pb of species 4 v + g, v = 0, 1
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int sr = 16 * c + quad_slot(4 * v + g);
      nb[v] = -ldexp(qa[sr], -s);
      npb[v] = -ldexp(qp[sr], -s);
    }
    __builtin_amdgcn_wave_barrier();

    // W_c (lane row g = component c), ubar, dv
    const double Wsum = row_chain(w0, cj && j < 8 ? wj : 0.0, 8);
    const double dv = cj ? vj - v0 : 0.0;
    const double ub = cj ? wj - Wsum * ej * rsig : 0.0;

    // dB = 2^-s G at rows 0..7, columns 8..15: one MFMA over the components
    // (A[i][c] = ubar_c[i] from lanes j < 8, B[c][8 + k] = dv_c[k] from lanes
    // j >= 8)
    v4d Xh = __builtin_amdgcn_mfma_f64_16x16x4f64(j < 8 ? ub : 0.0, j < 8 ? 0.0 : dv, zero4, 0,
                                                  0, 0);
    // B = M^T on the diagonal blocks: B[i][k] = -b_i [i == k] - pb_i
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * v + g;
      const bool diag_block = (row < 8) == (j < 8);
      const double bdiag = ((row & 7) == jj) ? nb[v & 1] : 0.0;
      const double val = (jj < N && (row & 7) < N) ? bdiag + npb[v & 1] : 0.0;
      Xh[v] = diag_block ? val : ldexp(Xh[v], -s);
    }

    // powers Xh^p on the matrix cores: Xh is the A operand for all of them
    // (one LDS transposition), each power the B operand of the next
    double XA[4];
    stage_tile(stage, g, j, Xh);
    load_a_ops(stage, g, j, XA);
    v4d F;
    switch (q) {  // uniform; one code path per power count
      case 1: F = mfma_poly<1>(Xh, XA, r, stage, g, j); break;
      case 2: F = mfma_poly<2>(Xh, XA, r, stage, g, j); break;
      case 3: F = mfma_poly<3>(Xh, XA, r, stage, g, j); break;
      case 4: F = mfma_poly<4>(Xh, XA, r, stage, g, j); break;
      default: F = mfma_poly<5>(Xh, XA, r, stage, g, j); break;
    }
    // squarings of the block matrix, (Yh + 2 I) Yh
    v4d Y = F;
    int it = 0;
    for (; it + 2 <= s; it += 2) {
      const v4d Y1 = square_step(Y, stage, g, j, diag_slot);
      Y = square_step(Y1, stage, g, j, diag_slot);
    }
    if (it < s) Y = square_step(Y, stage, g, j, diag_slot);

    // Y = Z^T in the upper-left block, dY = dL/dAt in the upper-right.
    // u_c = Z dv_c = (dV^T Y)[c] and Z^T ubar_c = (Ubar^T Y^T)[c]: A operands
    // rows = components (lane (g, i) takes component i, species 4t+g).
    double YB[4], ZB[4], DvA[4], UbA[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) YB[t] = Y[t];
    stage_tile(stage, g, j, Y);
    load_a_ops(stage, g, j, ZB);  // Yh^T as the B operand
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int src = (j < D && t < 2) ? 16 * j + 4 * t + g : 0;
      const double a1 = __shfl(dv, src, 64), a2 = __shfl(ub, src, 64);
      DvA[t] = (j < D && t < 2) ? a1 : 0.0;
      UbA[t] = (j < D && t < 2) ? a2 : 0.0;
    }
    const v4d Um = mma16(DvA, YB, zero4);  // lane (g, j) [0]: u_g[j]
    const v4d Vm = mma16(UbA, ZB, zero4);  // lane (g, j) [0]: (Z^T ubar_g)_j
    const double u = (cj && j < 8) ? Um[0] : 0.0;
    const double zt = (cj && j < 8) ? Vm[0] : 0.0;
    const double eu = row_chain(0.0, ej * u, 8);
    const double d0 = -eu * rsig;
    const double zt_sum = row_chain(0.0, zt, 8);
    if (comp && j < 8) {
      const int64_t base = (int64_t)(g * n1) * ld + cell;
      if (A.v_out) {
        if (jj < N) A.v_out[base + (int64_t)(1 + jj) * ld] = vj + (d0 + u);
        if (j == 0) A.v_out[base] = v0 + d0;
      }
      if (A.g_v) {
        if (jj < N) A.g_v[base + (int64_t)(1 + jj) * ld] = wj + zt;
        if (j == 0) A.g_v[base] = w0 - zt_sum;
      }
    }
    // direct dependence of the gas update on e, summed over components
    const double ge_dir = groups_sum(cj ? (-d0 - u) * (Wsum * rsig) : 0.0);
    // column sums and diagonal of dY (upper-right block, rows 4v+g, v < 2,
    // column 8 + k), moved to lane k of each row
    double col = (j < 8) ? 0.0 : Y[0] + Y[1];
    double dg = 0.0;
#pragma unroll
    for (int v = 0; v < 2; ++v)
      if (j >= 8 && 4 * v + g == jj) dg = Y[v];
    col = row_ror64<8>(groups_sum(col));
    dg = row_ror64<8>(groups_sum(dg));
    if (g == 0) {
      const double rrg = 1.0 / A.rho_g[cell];
      double ge = 0.0;
      if (j < N) {
        const double ga = -dg - ej * col;
        ge = -aj * col + ge_dir;
        const double glt = -aj * ga;
        if (A.g_logt) A.g_logt[j * ld + cell] = glt;
        if (A.g_t) A.g_t[j * ld + cell] = glt / A.t_stop[j * ld + cell];
        if (A.g_rho_d) A.g_rho_d[j * ld + cell] = ge * rrg;
      }
      const double sum_ege = row_chain(0.0, ej * ge, N);
      if (j == 0 && A.g_rho_g) A.g_rho_g[cell] = -sum_ege * rrg;
    }
  }
}

template <int N>
__global__ void __launch_bounds__(256) k_backward_block(BackArgs A, int xcd_blocks) {
  static_assert(N <= 8, "the block form needs 2N <= 16");
  __shared__ double lds[4 * kQuadDoubles];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int bid = blockIdx.x;
  const int64_t logical = (int64_t)(bid & 7) * xcd_blocks + (bid >> 3);
  const int64_t c0 = (logical * 4 + w) * 4;
  if (c0 >= A.n_cells) return;  // uniform over the wavefront
  wave_backward_block_quad(A, N, c0, lane, lds + w * kQuadDoubles);
}

}  // namespace dragexp
