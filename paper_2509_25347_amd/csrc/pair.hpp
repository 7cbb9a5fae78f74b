// pair.hpp -- two lanes per cell: the fused forward + adjoint (used at
// N = 8..10) and the forward (N = 9..12).
//
// The one-lane adjoint keeps Y, dY and a product buffer (3 N^2 doubles) in
// one lane: at N = 8 that exceeds the register file and spills.  Here the two
// lanes 2p, 2p+1 of a pair share cell p: lane h holds rows h H .. h H + H - 1
// (H = ceil(N / 2)) of Y and dY, so each lane keeps 2 H^2 + H 2H doubles
// instead of 3 N^2.
//
// Column order.  Every lane stores its rows with the columns in a
// lane-relative order: first the H columns of its own half, then the H of
// the other half (relative column kappa <-> global column h H + kappa for
// kappa < H, (1 - h) H + kappa - H otherwise).  Then all register indices are
// compile-time constants: the diagonal element of own row r is column r,
// the partner's row r' is global row (1 - h) H + r' = relative column H + r',
// and the partner's copy of a register, fetched with one DPP quad_perm swap
// per dword, maps its relative column kappa_p to mine by a half rotation
// (kappa = (kappa_p + H) mod 2H).
//
// The recurrences are those of the one-lane kernel (adjoint.hpp): Horner in
// B = M^T with the Frechet derivative in the direction dB = 2^-s G, then the
// squarings dY <- dY (Y + 2I) + Y dY, Y <- Y (Y + 2I).  The products of the
// Horner stage are row-local (no exchange); each squaring fetches the
// partner's rows of Y and dY once (and Y again for the second product).
// dB = 2^-s sum_c ubar_c dv_c^T is used in its rank-D form: h dB = 2^-s
// sum_c (h . ubar_c) dv_c^T, with ubar and dv kept in LDS.
#pragma once

#include "common.hpp"
#include "lane.hpp"

namespace dragexp {

// The other lane's value of x in the pair (DPP quad_perm [1, 0, 3, 2]).
__device__ __forceinline__ double pair_swap(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0xB1, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0xB1, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// x(lane 0 of the pair) + x(lane 1): the same bits in both lanes.
__device__ __forceinline__ double pair_sum(double x, int h) {
  const double y = pair_swap(x);
  return h == 0 ? x + y : y + x;
}

template <int H>
__device__ __forceinline__ void pair_copy(double (&W)[H][2 * H], const double (&Z)[H][2 * H]) {
#pragma unroll
  for (int r = 0; r < H; ++r)
#pragma unroll
    for (int k = 0; k < 2 * H; ++k) W[r][k] = Z[r][k];
}

// kMinWaves: waves per SIMD the register allocation must allow (2 forces
// N = 7, 8 into 256 registers at the price of a few spills in the squaring
// loop; 1 lets them use accumulation registers instead).  N = 9, 10 need
// more than 256 (Y, dY and the product rows: 3 H 2H doubles) and run at 1.
template <int N, int kMinWaves = 2>
__global__ void __launch_bounds__(256, kMinWaves) k_backward_pair(BackArgs A, int xcd_blocks) {
  constexpr int H = (N + 1) / 2;  // rows per lane
  constexpr int W2 = 2 * H;       // padded width
  constexpr int kCells = 128;     // cells per workgroup (two lanes each)
  // per cell, global column order, zero padded: ubar[3][W2], dv[3][W2], a[W2], e[W2],
  // then per component the gas velocity, the gas weight w_0 and W = sum_j w_j (the
  // output stage rebuilds v and w from these instead of reading them again),
  // stored entry-major (entry x of pair pl at sm[x * kStride + pl]): the pairs of a
  // wavefront read consecutive doubles, and the two lanes of a pair, whose entries
  // lie H apart, fall on the other half of the banks (kStride = 2 mod 4)
  constexpr int kStride = kCells + 2;
  constexpr int kGas = 8 * W2;  // v_0[3], w_0[3], W[3]
  constexpr bool kRebuild = N <= 8;
  __shared__ double sm[(kGas + 9) * kStride];

  const int bid = blockIdx.x;
  const int64_t logical = (int64_t)(bid & 7) * xcd_blocks + (bid >> 3);
  const int pl = threadIdx.x >> 1;  // pair within the workgroup
  const int h = threadIdx.x & 1;    // half
  const int64_t c = logical * kCells + pl;
  const bool active = c < A.n_cells;
  const int64_t cc = active ? c : 0;  // an inactive pair computes on cell 0, stores nothing
  const int64_t ld = A.ld;
  const int n1 = N + 1;
  const int D = A.n_dim;
  double* my = sm + pl;  // entry x of this pair at my[x * kStride]

  // relative column kappa of this lane <-> global column
  auto gcol = [&](int kappa) { return kappa < H ? h * H + kappa : (1 - h) * H + kappa - H; };

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
  if (!fin && !C.bad) C.bad = kBadVelocity;
  if (C.bad) {
#pragma unroll
    for (int i = 0; i < N; ++i) C.a[i] = C.e[i] = C.p[i] = 0.0;
    C.sigma = 1.0;
    C.kms = select_kms(0.0, A.k_max, A.option);
  }
  const int s = C.kms.s, m = C.kms.m;

  // scaled coefficients in this lane's relative order
  double nb[W2], npb[W2];
#pragma unroll
  for (int kap = 0; kap < W2; ++kap) {
    const int g = gcol(kap);
    double a = 0.0, p = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {  // select by value: no private-array indexing
      a = (g == k) ? C.a[k] : a;
      p = (g == k) ? C.p[k] : p;
    }
    nb[kap] = -ldexp(a, -s);
    npb[kap] = -ldexp(p, -s);
  }

  // ubar and dv of every component to LDS (lane 0 of the pair writes)
  if (h == 0) {
    for (int d = 0; d < 3; ++d) {
      double v[N + 1], w[N + 1];
      double W = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        const int64_t idx = (int64_t)(d * n1 + j) * ld + cc;
        v[j] = (d < D && !C.bad) ? A.v_in[idx] : 0.0;
        w[j] = (d < D && !C.bad) ? A.w[idx] : 0.0;
        W += w[j];
      }
#pragma unroll
      for (int k = 0; k < W2; ++k) {
        my[(d * W2 + k) * kStride] = k < N ? w[k + 1] - W * C.e[k < N ? k : 0] / C.sigma : 0.0;
        my[((3 + d) * W2 + k) * kStride] = k < N ? v[k + 1] - v[0] : 0.0;
      }
      my[(kGas + d) * kStride] = v[0];
      my[(kGas + 3 + d) * kStride] = w[0];
      my[(kGas + 6 + d) * kStride] = W;
    }
#pragma unroll
    for (int k = 0; k < W2; ++k) {
      my[(6 * W2 + k) * kStride] = k < N ? C.a[k < N ? k : 0] : 0.0;
      my[(7 * W2 + k) * kStride] = k < N ? C.e[k < N ? k : 0] : 0.0;
    }
  }
  const double sigma = C.sigma;
  const unsigned bad = C.bad;
  __syncthreads();

  // Horner in B = M^T with its derivative:
  //   Y  <- (Y + c I) B,  dY <- dY B + (Y + c I) dB,  (X B)_ik = -X_ik b_k - (X pb)_i
  // The direction term (Y + c I) dB = 2^-s sum_d t_d dv_d^T needs only the
  // vectors t_d = (Y + c I) ubar_d.  Y is a polynomial in B, so it commutes
  // with B, and z_d = Y ubar_d follows its own recurrence z_d <- B t_d,
  // (B x)_j = -b_j x_j - pb_j sum_k x_k: O(N) per degree instead of the
  // matrix-vector product (own rows here, the sum over the pair).  At
  // N = 8 that is 374 instead of 432 instructions per degree (5 % off the
  // kernel); at N = 9, 10, where the kernel already holds accumulation
  // registers, the 3 H more live values cost more than they save (3-5 %
  // slower), so there t_d is the product with the rows of Y.
  constexpr bool kVecDir = N <= 8;
  double Y[H][W2], dY[H][W2], z[3][H];
#pragma unroll
  for (int r = 0; r < H; ++r) {
#pragma unroll
    for (int k = 0; k < W2; ++k) Y[r][k] = dY[r][k] = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) z[d][r] = 0.0;
  }
  const int m_max = wave_max_int(m);
  for (int it = m_max; it >= 1; --it) {
    const double cf = (it <= m) ? kInvFact[it] : 0.0;
    double hp[H], fp[H];
#pragma unroll
    for (int r = 0; r < H; ++r) {
      Y[r][r] += cf;  // own row r is global row h H + r = relative column r
      hp[r] = 0.0;
      fp[r] = 0.0;
#pragma unroll
      for (int k = 0; k < W2; ++k) {
        hp[r] = fma(Y[r][k], -npb[k], hp[r]);
        fp[r] = fma(dY[r][k], -npb[k], fp[r]);
      }
#pragma unroll
      for (int k = 0; k < W2; ++k) dY[r][k] = fma(dY[r][k], nb[k], -fp[r]);
    }
    // + (Y + cI) dB = 2^-s sum_d t_d dv_d^T, t_d = z_d + c ubar_d
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (!kVecDir || d >= D) continue;
      double dv[W2], t[H];
#pragma unroll
      for (int k = 0; k < W2; ++k) dv[k] = my[((3 + d) * W2 + gcol(k)) * kStride];
      double S = 0.0;
#pragma unroll
      for (int r = 0; r < H; ++r) {
        t[r] = fma(cf, my[(d * W2 + h * H + r) * kStride], z[d][r]);
        S += t[r];
      }
      S = pair_sum(S, h);
#pragma unroll
      for (int r = 0; r < H; ++r) {
        const double ts = ldexp(t[r], -s);
#pragma unroll
        for (int k = 0; k < W2; ++k) dY[r][k] = fma(ts, dv[k], dY[r][k]);
        z[d][r] = fma(nb[r], t[r], npb[r] * S);
      }
    }
    // ... or with t_d from the rows of Y + c I
    for (int d = 0; d < D && !kVecDir; ++d) {
      double ub[W2], dv[W2];
#pragma unroll
      for (int k = 0; k < W2; ++k) {
        const int g = gcol(k);
        ub[k] = my[(d * W2 + g) * kStride];
        dv[k] = my[((3 + d) * W2 + g) * kStride];
      }
#pragma unroll
      for (int r = 0; r < H; ++r) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < W2; ++k) t = fma(Y[r][k], ub[k], t);
        t = ldexp(t, -s);
#pragma unroll
        for (int k = 0; k < W2; ++k) dY[r][k] = fma(t, dv[k], dY[r][k]);
      }
    }
#pragma unroll
    for (int r = 0; r < H; ++r)
#pragma unroll
      for (int k = 0; k < W2; ++k) Y[r][k] = fma(Y[r][k], nb[k], -hp[r]);
  }

  // squarings with the Frechet recurrence: dY <- dY (Y + 2I) + Y dY, then
  // Y <- Y (Y + 2I); the partner's rows come by DPP, columns half-rotated
  const int s_max = wave_max_int(s);
  for (int it = 0; it < s_max; ++it) {
    if (it < s) {
      double T[H][W2];
#pragma unroll
      for (int r = 0; r < H; ++r)
#pragma unroll
        for (int k = 0; k < W2; ++k) T[r][k] = 0.0;
      // own rows r2 (relative column r2 of a row of mine)
#pragma unroll
      for (int r2 = 0; r2 < H; ++r2) {
#pragma unroll
        for (int r = 0; r < H; ++r)
#pragma unroll
          for (int k = 0; k < W2; ++k) {
            const double wv = k == r2 ? Y[r2][k] + 2.0 : Y[r2][k];
            T[r][k] = fma(dY[r][r2], wv, fma(Y[r][r2], dY[r2][k], T[r][k]));
          }
      }
      // partner rows r2 (relative column H + r2 of a row of mine), fetched
      // one element at a time to keep the live set small
#pragma unroll
      for (int r2 = 0; r2 < H; ++r2)
#pragma unroll
        for (int k = 0; k < W2; ++k) {
          const double sy = pair_swap(Y[r2][(k + H) % W2]);
          const double py = k == H + r2 ? sy + 2.0 : sy;
          const double pdy = pair_swap(dY[r2][(k + H) % W2]);
#pragma unroll
          for (int r = 0; r < H; ++r)
            T[r][k] = fma(dY[r][H + r2], py, fma(Y[r][H + r2], pdy, T[r][k]));
        }
#pragma unroll
      for (int r = 0; r < H; ++r)
#pragma unroll
        for (int k = 0; k < W2; ++k) dY[r][k] = T[r][k];
      // An empty asm that "rewrites" Y: the partner's copies of Y fetched for
      // dY above are fetched again below instead of being kept live across
      // the copy (2 H W2 more registers, which spilled: 33 VGPRs at N = 8,
      // 28-30 at N = 9, 10; the refetch is 8-14 % faster, same bits).
#pragma unroll
      for (int r = 0; r < H; ++r)
#pragma unroll
        for (int k = 0; k < W2; ++k) asm volatile("" : "+v"(Y[r][k]));
      // Y <- Y (Y + 2I)
#pragma unroll
      for (int r = 0; r < H; ++r)
#pragma unroll
        for (int k = 0; k < W2; ++k) T[r][k] = 0.0;
#pragma unroll
      for (int r2 = 0; r2 < H; ++r2) {
#pragma unroll
        for (int r = 0; r < H; ++r)
#pragma unroll
          for (int k = 0; k < W2; ++k)
            T[r][k] = fma(Y[r][r2], k == r2 ? Y[r2][k] + 2.0 : Y[r2][k], T[r][k]);
      }
#pragma unroll
      for (int r2 = 0; r2 < H; ++r2)
#pragma unroll
        for (int k = 0; k < W2; ++k) {
          const double sy = pair_swap(Y[r2][(k + H) % W2]);
          const double py = k == H + r2 ? sy + 2.0 : sy;
#pragma unroll
          for (int r = 0; r < H; ++r) T[r][k] = fma(Y[r][H + r2], py, T[r][k]);
        }
#pragma unroll
      for (int r = 0; r < H; ++r)
#pragma unroll
        for (int k = 0; k < W2; ++k) Y[r][k] = T[r][k];
    }
  }

  // outputs: Y = Z^T, dY = dL/dAt (rows of this lane).  Own species are the
  // global indices h H + r, r < H (own rows = own-half relative columns).
  const double qnan = __builtin_nan("");
  const double rg = A.rho_g[cc];
  const double rsig = 1.0 / sigma;
  double ge_dir[H];
#pragma unroll
  for (int r = 0; r < H; ++r) ge_dir[r] = 0.0;
  for (int d = 0; d < D; ++d) {
    double ub[W2], dv[W2];
#pragma unroll
    for (int k = 0; k < W2; ++k) {
      const int g = gcol(k);
      ub[k] = my[(d * W2 + g) * kStride];
      dv[k] = my[((3 + d) * W2 + g) * kStride];
    }
    // u = Z dv: column sums of Y weighted by dv over own rows, plus the partner's
    double up[W2];
#pragma unroll
    for (int k = 0; k < W2; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < H; ++r) acc = fma(Y[r][k], dv[r], acc);  // dv of own row r
      up[k] = acc;
    }
    double u[W2];
#pragma unroll
    for (int k = 0; k < W2; ++k) u[k] = up[k] + pair_swap(up[(k + H) % W2]);
    double eu_own = 0.0, zt[H], zt_own = 0.0;
#pragma unroll
    for (int r = 0; r < H; ++r) {
      const double e_r = my[(7 * W2 + h * H + r) * kStride];
      eu_own = fma(e_r, u[r], eu_own);
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < W2; ++k) acc = fma(Y[r][k], ub[k], acc);  // (Z^T ubar)_(own row r)
      zt[r] = acc;
      zt_own += acc;
    }
    const double eu = pair_sum(eu_own, h);
    const double d0 = -eu * rsig;
    const double zt_sum = pair_sum(zt_own, h);
    // v and w of this cell: at N <= 8 rebuilt from LDS (v_k = v_0 + dv_k,
    // w_k = ubar_k + W e_k / sigma, each within a rounding of the input) rather
    // than read again from memory after the squarings; at N = 9, 10 the
    // rebuild's registers would spill, so those read them again, and so does
    // dt = 0 (Z = 0: v' and dL/dv equal v and w)
    const bool reread = !kRebuild || A.dt == 0.0;  // uniform
    const double W = my[(kGas + 6 + d) * kStride];
    const int64_t base = (int64_t)(d * n1) * ld + c;
#pragma unroll
    for (int r = 0; r < H; ++r) ge_dir[r] = fma(-d0 - u[r], W * rsig, ge_dir[r]);
    if (active) {
      const double v0 = kRebuild ? my[(kGas + d) * kStride] : A.v_in[base];
      const double w0 = kRebuild ? my[(kGas + 3 + d) * kStride] : A.w[base];
#pragma unroll
      for (int r = 0; r < H; ++r) {
        const int k = h * H + r;
        if (k < N) {
          const int64_t idx = base + (int64_t)(1 + k) * ld;
          const double e_k = my[(7 * W2 + k) * kStride];
          double vk, wk;
          if (reread) {
            vk = A.v_in[idx];
            wk = A.w[idx];
          } else {
            vk = v0 + dv[r];
            wk = ub[r] + W * e_k / sigma;
          }
          if (A.v_out) A.v_out[idx] = bad ? qnan : vk + (d0 + u[r]);
          if (A.g_v) A.g_v[idx] = bad ? qnan : wk + zt[r];
        }
      }
      if (h == 0) {
        if (A.v_out) A.v_out[base] = bad ? qnan : v0 + d0;
        if (A.g_v) A.g_v[base] = bad ? qnan : w0 - zt_sum;
      }
    }
  }
  // column sums and diagonal of dL/dAt for the own species
  double colp[W2];
#pragma unroll
  for (int k = 0; k < W2; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < H; ++r) acc += dY[r][k];
    colp[k] = acc;
  }
  double sum_ege = 0.0;
#pragma unroll
  for (int r = 0; r < H; ++r) {
    const int k = h * H + r;
    const double col = colp[r] + pair_swap(colp[(r + H) % W2]);
    const double e_k = my[(7 * W2 + h * H + r) * kStride];
    const double a_k = my[(6 * W2 + h * H + r) * kStride];
    const double ga = -dY[r][r] - e_k * col;
    const double ge = -a_k * col + ge_dir[r];
    const double glt = -a_k * ga;
    sum_ege = fma(e_k, ge, sum_ege);
    if (active && k < N) {
      if (A.g_logt) A.g_logt[k * ld + c] = bad ? qnan : glt;
      if (A.g_t) A.g_t[k * ld + c] = bad ? qnan : glt / A.t_stop[k * ld + c];
      if (A.g_rho_d) A.g_rho_d[k * ld + c] = bad ? qnan : ge / rg;
    }
  }
  const double sum_all = pair_sum(sum_ege, h);
  if (active && h == 0) {
    if (A.g_rho_g) A.g_rho_g[c] = bad ? qnan : -sum_all / rg;
    if (bad) atomicOr(&g_status_word, bad);
  }
}

// One squaring W = Z (Z + 2I) of the rows of this lane (lane-relative
// columns; the partner's rows fetched element by element by DPP, one swap per
// dword, used for all H own rows).  With go false, W = Z.
template <int H>
__device__ __forceinline__ void pair_square_step(bool go, const double (&Z)[H][2 * H],
                                                 double (&W)[H][2 * H]) {
  constexpr int W2 = 2 * H;
  if (!go) {
    pair_copy<H>(W, Z);
    return;
  }
  // own rows of the right factor: relative column l of my rows is my row l
  // (the chains start with a product rather than an FMA into zero)
#pragma unroll
  for (int l = 0; l < H; ++l) {
#pragma unroll
    for (int k = 0; k < W2; ++k) {
      const double b = k == l ? Z[l][k] + 2.0 : Z[l][k];
#pragma unroll
      for (int r = 0; r < H; ++r) W[r][k] = l == 0 ? Z[r][l] * b : fma(Z[r][l], b, W[r][k]);
    }
  }
  // the partner's rows: its row l is my relative column H + l
#pragma unroll
  for (int l = 0; l < H; ++l) {
#pragma unroll
    for (int k = 0; k < W2; ++k) {
      const double sz = pair_swap(Z[l][(k + H) % W2]);
      const double b = k == H + l ? sz + 2.0 : sz;
#pragma unroll
      for (int r = 0; r < H; ++r) W[r][k] = fma(Z[r][H + l], b, W[r][k]);
    }
  }
}

// The forward with two lanes per cell, for the species counts where one lane
// cannot hold Z and the squaring's product buffer (2 N^2 doubles) and the
// 16 x 16 MFMA tile is mostly padding (N = 9..12).
// Same layout as the adjoint above: lane h holds rows h H .. h H + H - 1 in
// the lane-relative column order.  Horner in the structured matrix,
// F <- (F + c I) M with (F M)_ik = -F_ik b_k - (sum_l F_il) pb_k, is
// row-local; each squaring W = Z (Z + 2I) fetches the partner's rows of Z
// element by element (one DPP swap per dword, used for all H own rows); the
// apply u = Z dv is row-local and e.u a pair sum.
// The forward update of cell c by the pair of lanes (h = 0, 1) that share
// it.  Both lanes of every pair of the wavefront must call it together (DPP
// swaps, wavefront-wide maxima of m and s); a spare pair passes any valid
// cell as cc, computes on it and stores nothing.  vs is the pair's LDS
// staging of its velocities (entry d (N + 1) + j at vs[x * vstride], 3 (N + 1)
// entries): lane 0 reads them once, for the finiteness check, and the apply
// stage takes them from there (read again from memory after the squarings,
// they had been evicted from L2: 1.25-1.32x the algorithmic reads at N = 9, 10).
template <int N>
__device__ __forceinline__ void pair_forward_cell(const CellArgs& A, int64_t c, int64_t cc,
                                                  bool active, int h, double* vs, int vstride) {
  constexpr int H = (N + 1) / 2;
  constexpr int W2 = 2 * H;
  const int64_t ld = A.ld;
  const int n1 = N + 1;
  const int D = A.n_dim;
  auto gcol = [&](int kappa) { return kappa < H ? h * H + kappa : (1 - h) * H + kappa - H; };

  LaneCell<N> C;
  lane_setup<N>(C, A.rho_g, A.rho_d, A.t_stop, ld, cc, A.dt, A.k_max, A.option);
  double fin = 1.0;
  if (h == 0) {
    for (int d = 0; d < D; ++d) {
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        const double x = A.v_in[(int64_t)(d * n1 + j) * ld + cc];
        vs[(d * n1 + j) * vstride] = x;
        fin = isfinite(x) ? fin : 0.0;
      }
    }
  }
  const double fin_pair = pair_swap(fin);  // lane 1 takes lane 0's verdict
  const bool vfin = (h == 0 ? fin : fin_pair) != 0.0;
  if (!vfin && !C.bad) C.bad = kBadVelocity;
  const int s = C.kms.s, m = C.kms.m;

  // scaled coefficients and e in the lane-relative column order
  double nb[W2], npb[W2], er[H];
#pragma unroll
  for (int kap = 0; kap < W2; ++kap) {
    const int g = gcol(kap);
    double a = 0.0, p = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {  // select by value: no private-array indexing
      a = (g == k) ? C.a[k] : a;
      p = (g == k) ? C.p[k] : p;
    }
    nb[kap] = -ldexp(a, -s);
    npb[kap] = -ldexp(p, -s);
  }
#pragma unroll
  for (int r = 0; r < H; ++r) {
    double e = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) e = (h * H + r == k) ? C.e[k] : e;
    er[r] = e;
  }

  // Horner: Z = T_m(M) - I, own rows only
  double Z[H][W2];
#pragma unroll
  for (int r = 0; r < H; ++r)
#pragma unroll
    for (int k = 0; k < W2; ++k) Z[r][k] = 0.0;
  const int m_max = wave_max_int(m);
  for (int it = m_max; it >= 1; --it) {
    const double cf = (it <= m) ? kInvFact[it] : 0.0;
#pragma unroll
    for (int r = 0; r < H; ++r) {
      if (h * H + r < N) Z[r][r] += cf;  // own row r = relative column r
      double rs = 0.0;
#pragma unroll
      for (int k = 0; k < W2; ++k) rs += Z[r][k];
#pragma unroll
      for (int k = 0; k < W2; ++k) Z[r][k] = fma(rs, npb[k], Z[r][k] * nb[k]);
    }
  }

  // squarings Z <- Z (Z + 2I), two per trip between Z and T.  Each lane
  // squares under its own s (the product that may or may not be taken is
  // formed in temporaries and moved: H W2 moves per squaring); for H <= 5 a
  // branch-free loop runs first, up to the wavefront's smallest s.  At H = 6
  // the branch-free loop was allocated worse than the branching one (more
  // moves and accumulation-register traffic; 5 % slower at N = 12).
  const int s_max = wave_max_int(s);
  const int s_min = H <= 5 ? wave_min_int(s) : 0;
  double T[H][W2];
  int it = 0;
  for (; it + 2 <= s_min; it += 2) {
    pair_square_step<H>(true, Z, T);
    pair_square_step<H>(true, T, Z);
  }
  for (; it + 2 <= s_max; it += 2) {
    pair_square_step<H>(it < s, Z, T);
    pair_square_step<H>(it + 1 < s, T, Z);
  }
  if (it < s) {
    pair_square_step<H>(true, Z, T);
    pair_copy<H>(Z, T);
  }

  // apply: u = Z dv for the own rows, e.u summed over the pair
  const double qnan = __builtin_nan("");
  for (int d = 0; d < D; ++d) {
    const int64_t base = (int64_t)(d * n1) * ld;
    const double v0 = vs[(d * n1) * vstride];
    double dv[W2];
#pragma unroll
    for (int k = 0; k < W2; ++k) {
      const int g = gcol(k);  // a run-time row index is fine for LDS
      dv[k] = g < N ? vs[(d * n1 + 1 + g) * vstride] - v0 : 0.0;
    }
    double u[H], eu_own = 0.0;
#pragma unroll
    for (int r = 0; r < H; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < W2; ++k) acc = fma(Z[r][k], dv[k], acc);
      u[r] = acc;
      eu_own = fma(er[r], acc, eu_own);
    }
    const double d0 = -pair_sum(eu_own, h) / C.sigma;
    if (active) {
#pragma unroll
      for (int r = 0; r < H; ++r) {
        const int k = h * H + r;
        if (k < N) {
          const int64_t idx = base + (int64_t)(1 + k) * ld + c;
          A.v_out[idx] = C.bad ? qnan : vs[(d * n1 + 1 + k) * vstride] + (d0 + u[r]);
        }
      }
      if (h == 0) A.v_out[base + c] = C.bad ? qnan : v0 + d0;
    }
  }
  if (C.bad && active && h == 0) atomicOr(&g_status_word, C.bad);
}

// Waves per SIMD the forward's register allocation must allow: 2 up to
// N = 10 (nothing spills, the squarings alternating between Z and T, and
// the second wavefront hides the latencies: 1.27-1.36x faster than 1 wave
// with accumulation registers), 1 above (Z and the product buffer alone
// fill 256 registers).
template <int N>
constexpr int pair_fwd_min_waves() { return N <= 10 ? 2 : 1; }

template <int N>
__global__ void __launch_bounds__(256, pair_fwd_min_waves<N>()) k_forward_pair(CellArgs A,
                                                                              int xcd_blocks) {
  constexpr int kCells = 128;  // cells per workgroup, two lanes each
  constexpr int kStride = kCells + 2;
  __shared__ double vsm[3 * (N + 1) * kStride];
  const int bid = blockIdx.x;
  const int64_t logical = (int64_t)(bid & 7) * xcd_blocks + (bid >> 3);
  const int pl = threadIdx.x >> 1;
  const int64_t c = logical * kCells + pl;
  const bool active = c < A.n_cells;
  pair_forward_cell<N>(A, c, active ? c : 0, active, threadIdx.x & 1, vsm + pl, kStride);
}

}  // namespace dragexp
