// lane.hpp -- one cell per lane (VALU), for small species counts N.
//
// Every lane owns one cell and keeps the N x N matrices of that cell in its
// own VGPRs; all arithmetic is scalar FP64 with explicit fma().
//
// Reduced form.  The drag matrix A = dt K (velocity form: A00 = -sum e_i a_i,
// A0i = e_i a_i, Ai0 = a_i, Aii = -a_i) has the right null vector 1 (its rows
// sum to zero) and the left null vector rho (momentum, Sect. 2.1).  In the
// coordinates (v_g, dv_i = v_i - v_g) it is block triangular, and the
// relative velocities obey dv' = At dv with the N x N matrix
//     At_jk = -a_j [j == k] - p_k,   p_k = e_k a_k,
// while the gas velocity follows from conservation of total momentum
// rho_g v_g + sum_i rho_i v_i.  For any polynomial T (the Taylor
// approximant, and its 2^s-th power) T(A) acts exactly as T(At) on dv and as
// momentum conservation on v_g, so with Z = T_m(2^-s At)^(2^s) - I,
//     u      = Z dv,
//     v_g'   = v_g - (e . u) / (1 + sum_i e_i),
//     v_i'   = v_i + (v_g' - v_g) + u_i,
// is the paper's approximant applied to v, up to rounding.  The scaling
// s and degree m come from ||A||_1 of the full matrix (Alg. 1), exactly as
// in the paper; the conserved mode no longer passes through the squarings.
#pragma once

#include "common.hpp"

namespace dragexp {

// Horner evaluation of F = sum_{i=1}^{m} c_i M^i = T_m(M) - I for the
// structured M = 2^-s At: M_jk = -b_j [j == k] - pb_k.  Right products by M
// cost O(N^2): (F M)_ik = -F_ik b_k - (sum_l F_il) pb_k.  Lanes of one
// wavefront may have different m; the loop runs to the wavefront's largest
// m and each lane adds only its own coefficients (a zero F stays zero).
template <int N>
__device__ __forceinline__ void lane_taylor(double (&F)[N][N], const double (&b)[N],
                                            const double (&pb)[N], int m, int m_max) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < N; ++k) F[i][k] = 0.0;
  for (int it = m_max; it >= 1; --it) {
    const double c = (it <= m) ? kInvFact[it] : 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      F[i][i] += c;
      double rs = 0.0;
#pragma unroll
      for (int l = 0; l < N; ++l) rs += F[i][l];
#pragma unroll
      for (int k = 0; k < N; ++k) F[i][k] = fma(-F[i][k], b[k], -rs * pb[k]);
    }
  }
}

// One Y-form squaring W <- 2 Z + Z Z (the paper's X <- X X with X = I + Z),
// written as Z (Z + 2 I): the right factor's diagonal gets 2, so no separate
// 2 Z term.  The extra rounding of 2 + Z_ll is of the size of the sum's own.
template <int N>
__device__ __forceinline__ void lane_square_to(double (&W)[N][N], const double (&Z)[N][N]) {
  double d[N];
#pragma unroll
  for (int l = 0; l < N; ++l) d[l] = Z[l][l] + 2.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double acc = Z[i][0] * (k == 0 ? d[0] : Z[0][k]);
#pragma unroll
      for (int l = 1; l < N; ++l) acc = fma(Z[i][l], l == k ? d[l] : Z[l][k], acc);
      W[i][k] = acc;
    }
}

template <int N>
__device__ __forceinline__ void lane_copy(double (&W)[N][N], const double (&Z)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = 0; k < N; ++k) W[i][k] = Z[i][k];
}

__device__ __forceinline__ int wave_max_int(int x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}

// Per-cell set-up: coefficients, ||A||_1 (bit-exact order), Alg. 1.
template <int N>
struct LaneCell {
  double a[N], e[N], p[N];
  double sigma;  // 1 + sum e_i
  double nrm;
  unsigned bad;
  Kms kms;
};

// The rest of the set-up once the coefficients are in C: ||A||_1 (the gas
// column |A00| + a_1 + .. + a_N, the species columns p_i + a_i; sums in
// ascending order, one rounding per operation), sigma and Alg. 1.
template <int N>
__device__ __forceinline__ void lane_setup_norm(LaneCell<N>& C, int K, int option) {
  double s = 0.0, sig = 1.0;
  bool finite = true;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    s = s + C.p[i];
    sig = sig + C.e[i];
    finite = finite && isfinite(C.a[i]) && isfinite(C.p[i]);
  }
  double nrm = s;
#pragma unroll
  for (int i = 0; i < N; ++i) nrm = nrm + C.a[i];
#pragma unroll
  for (int i = 0; i < N; ++i) nrm = fmax(nrm, C.p[i] + C.a[i]);
  if (!C.bad && !(finite && isfinite(nrm))) C.bad |= kBadNorm;
  C.sigma = sig;
  C.nrm = nrm;
  if (C.bad) {
    // run the rest of the lane on a harmless zero matrix; outputs are NaN
#pragma unroll
    for (int i = 0; i < N; ++i) C.a[i] = C.e[i] = C.p[i] = 0.0;
    C.sigma = 1.0;
    nrm = 0.0;
  }
  C.kms = select_kms(nrm, K, option);
}

// Set-up from memory; each species is loaded just before its coefficients.
template <int N>
__device__ __forceinline__ void lane_setup(LaneCell<N>& C, const double* rho_g,
                                           const double* rho_d, const double* t_stop,
                                           int64_t ld, int64_t c, double dt, int K,
                                           int option) {
  const double rg = rho_g[c];
  C.bad = gas_bad(rg);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double t = t_stop[i * ld + c];
    const double r = rho_d[i * ld + c];
    C.bad |= species_bad(t, r);
    const Species sp = species_coeffs(dt, t, r, rg);
    C.a[i] = sp.a;
    C.e[i] = sp.e;
    C.p[i] = sp.p;
  }
  lane_setup_norm<N>(C, K, option);
}

// Set-up from inputs already in registers.
template <int N>
__device__ __forceinline__ void lane_setup_values(LaneCell<N>& C, double rg,
                                                  const double (&rd)[N], const double (&ts)[N],
                                                  double dt, int K, int option) {
  C.bad = gas_bad(rg);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    C.bad |= species_bad(ts[i], rd[i]);
    const Species sp = species_coeffs(dt, ts[i], rd[i], rg);
    C.a[i] = sp.a;
    C.e[i] = sp.e;
    C.p[i] = sp.p;
  }
  lane_setup_norm<N>(C, K, option);
}

// Z = T_m(2^-s At)^(2^s) - I for the lane's cell.
template <int N>
__device__ __forceinline__ void lane_expm(double (&Z)[N][N], const LaneCell<N>& C) {
  double b[N], pb[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    b[i] = ldexp(C.a[i], -C.kms.s);
    pb[i] = ldexp(C.p[i], -C.kms.s);
  }
  const int m_max = wave_max_int(C.kms.m);
  lane_taylor<N>(Z, b, pb, C.kms.m, m_max);
  // squarings to the wavefront's largest s, each lane under its own s; two
  // per trip between Z and T so that no copy is needed on the common path
  const int s = C.kms.s;
  const int s_max = wave_max_int(s);
  double T[N][N];
  int it = 0;
  for (; it + 2 <= s_max; it += 2) {
    if (it < s) lane_square_to<N>(T, Z);
    else lane_copy<N>(T, Z);
    if (it + 1 < s) lane_square_to<N>(Z, T);
    else lane_copy<N>(Z, T);
  }
  if (it < s) {
    lane_square_to<N>(T, Z);
    lane_copy<N>(Z, T);
  }
}

// v' = v + E v - v for component d of the lane's cell: u = Z dv on the
// relative velocities, the gas by momentum conservation; NaN for a bad cell.
template <int N>
__device__ __forceinline__ void lane_apply_component(const CellArgs& A, const LaneCell<N>& C,
                                                     const double (&Z)[N][N],
                                                     const double (&v)[N + 1], int d, int64_t c,
                                                     bool active) {
  const int n1 = N + 1;
  double dv[N], u[N];
#pragma unroll
  for (int j = 0; j < N; ++j) dv[j] = v[j + 1] - v[0];
  double eu = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) acc = fma(Z[i][k], dv[k], acc);
    u[i] = acc;
    eu = fma(C.e[i], acc, eu);
  }
  const double d0 = -eu / C.sigma;
  if (active) {
    const double qnan = __builtin_nan("");
    A.v_out[(int64_t)(d * n1) * A.ld + c] = C.bad ? qnan : v[0] + d0;
#pragma unroll
    for (int j = 0; j < N; ++j)
      A.v_out[(int64_t)(d * n1 + 1 + j) * A.ld + c] = C.bad ? qnan : v[j + 1] + (d0 + u[j]);
  }
}

// The forward update of cell c by one lane.  Every lane of the wavefront
// must call it together (the Taylor and squaring loops run to the
// wavefront's largest m and s); an inactive lane passes the index of any
// valid cell as cc, computes on it and stores nothing.
template <int N>
__device__ __forceinline__ void lane_forward_cell(const CellArgs& A, int64_t c, int64_t cc,
                                                  bool active) {
  LaneCell<N> C;
  lane_setup<N>(C, A.rho_g, A.rho_d, A.t_stop, A.ld, cc, A.dt, A.k_max, A.option);
  double Z[N][N];
  lane_expm<N>(Z, C);

  const int n1 = N + 1;
  // every velocity of the cell must be finite, else all its outputs are NaN
  bool vfin = true;
  for (int d = 0; d < A.n_dim; ++d) {
#pragma unroll
    for (int j = 0; j <= N; ++j) vfin = vfin && isfinite(A.v_in[(int64_t)(d * n1 + j) * A.ld + cc]);
  }
  if (!vfin && !C.bad) C.bad = kBadVelocity;
  for (int d = 0; d < A.n_dim; ++d) {
    double v[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) v[j] = A.v_in[(int64_t)(d * n1 + j) * A.ld + cc];
    double dv[N], u[N];
#pragma unroll
    for (int j = 0; j < N; ++j) dv[j] = v[j + 1] - v[0];
    double eu = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) acc = fma(Z[i][k], dv[k], acc);
      u[i] = acc;
      eu = fma(C.e[i], acc, eu);
    }
    const double d0 = -eu / C.sigma;
    if (active) {
      const double qnan = __builtin_nan("");
      A.v_out[(int64_t)(d * n1) * A.ld + c] = C.bad ? qnan : v[0] + d0;
#pragma unroll
      for (int j = 0; j < N; ++j)
        A.v_out[(int64_t)(d * n1 + 1 + j) * A.ld + c] = C.bad ? qnan : v[j + 1] + (d0 + u[j]);
    }
  }
  if (C.bad && active) atomicOr(&g_status_word, C.bad);
}

// Coefficient inputs of one cell held in registers: gas and species
// densities and stopping times; with the velocities (up to three
// components) for the full prefetch.
template <int N>
struct LaneCoefs {
  double rg, rd[N], ts[N];
};
template <int N>
struct LaneInputs : LaneCoefs<N> {
  double v[3][N + 1];
};

// Element `off / 8` of a row of `bytes` bytes through a raw buffer load: the
// row's base lives in a scalar resource and every load of a cell shares one
// 32-bit lane offset, so prefetching a cell's inputs holds one address
// register, not a 64-bit address per row.  An offset past the row reads 0.
// The resource: stride 0 (raw), num_records = bytes (bit pattern; up to
// 2^32 - 8 here), and the CDNA word-3 flags for 32-bit untyped data.
__device__ __forceinline__ double row_at(const double* row, uint32_t bytes, uint32_t off) {
  constexpr int kRawBufferFlags = 0x00020000;
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(row), (short)0, (int)bytes, kRawBufferFlags);
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// Inputs of cell c, given as the byte offset off = 8 c (c < n_cells < 2^29,
// so that 8 n_cells fits in 32 bits).
template <int N>
__device__ __forceinline__ void lane_load(LaneCoefs<N>& X, const CellArgs& A, uint32_t off) {
  const uint32_t bytes = (uint32_t)(8 * A.n_cells);
  X.rg = row_at(A.rho_g, bytes, off);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    X.ts[i] = row_at(A.t_stop + i * A.ld, bytes, off);
    X.rd[i] = row_at(A.rho_d + i * A.ld, bytes, off);
  }
}

// ... and the velocities; components past n_dim repeat the last one (cache
// hits, never used), which keeps the loads unconditional.
template <int N>
__device__ __forceinline__ void lane_load(LaneInputs<N>& X, const CellArgs& A, uint32_t off) {
  lane_load<N>(static_cast<LaneCoefs<N>&>(X), A, off);
  const uint32_t bytes = (uint32_t)(8 * A.n_cells);
  const int n1 = N + 1;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int dd = d < A.n_dim ? d : A.n_dim - 1;
#pragma unroll
    for (int j = 0; j <= N; ++j) X.v[d][j] = row_at(A.v_in + (int64_t)(dd * n1 + j) * A.ld, bytes, off);
  }
}

// The forward update of cell c from inputs already in registers (all lanes
// of the wavefront together, as lane_forward_cell).
template <int N>
__device__ __forceinline__ void lane_forward_loaded(const CellArgs& A, const LaneInputs<N>& X,
                                                   int64_t c, bool active) {
  LaneCell<N> C;
  lane_setup_values<N>(C, X.rg, X.rd, X.ts, A.dt, A.k_max, A.option);
  double Z[N][N];
  lane_expm<N>(Z, C);
  bool vfin = true;
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int j = 0; j <= N; ++j) vfin = vfin && isfinite(X.v[d][j]);
  if (!vfin && !C.bad) C.bad = kBadVelocity;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (d < A.n_dim) lane_apply_component<N>(A, C, Z, X.v[d], d, c, active);
  if (C.bad && active) atomicOr(&g_status_word, C.bad);
}

// Streaming form of the one-lane forward.  The one-shot grid runs its
// wavefronts in lock-step generations (all load, then all compute while HBM
// idles, then all store), so its time is the sum of the memory and the
// arithmetic phases.  Here a grid of at most the resident wavefronts walks
// the cells with a stride, and each lane loads the inputs of its next cell
// before it computes the current one: the loads of one cell overlap the
// arithmetic of the previous.  Same arithmetic as k_forward_lane, per cell.
// Needs n_cells < 2^29 (32-bit byte offsets and row sizes).
template <int N>
__global__ void __launch_bounds__(256) k_forward_lane_stream(CellArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t n = A.n_cells;
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t w0 = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63);  // the wavefront's first cell
  if (w0 >= n) return;                                             // uniform over the wavefront
  LaneInputs<N> cur;
  lane_load<N>(cur, A, (uint32_t)(8 * (w0 + lane < n ? w0 + lane : w0)));
  for (;;) {
    const int64_t c = w0 + lane;
    const bool active = c < n;
    const int64_t w1 = w0 + stride;  // uniform: the loop and the prefetch branch
    LaneInputs<N> nxt;
    if (w1 < n) lane_load<N>(nxt, A, (uint32_t)(8 * (w1 + lane < n ? w1 + lane : w1)));
    lane_forward_loaded<N>(A, cur, c, active);
    if (w1 >= n) break;
    cur = nxt;
    w0 = w1;
  }
}

// One-shot one-lane forward.  EARLY issues every load of the cell, the
// velocities included, before the exponential, so that they arrive during
// it (n_cells < 2^29); otherwise the velocities are read after it, which
// keeps fewer registers live.
template <int N, bool EARLY = false>
__global__ void __launch_bounds__(256) k_forward_lane(CellArgs A, int xcd_blocks) {
  // XCD-aware order: consecutive workgroup ids go to different XCDs, so
  // hand each XCD a contiguous range of cells.
  const int bid = blockIdx.x;
  const int64_t logical = (int64_t)(bid & 7) * xcd_blocks + (bid >> 3);
  const int64_t c = logical * 256 + threadIdx.x;
  const bool active = c < A.n_cells;
  if constexpr (EARLY) {
    LaneInputs<N> X;
    lane_load<N>(X, A, (uint32_t)(8 * (active ? c : 0)));
    lane_forward_loaded<N>(A, X, c, active);
  } else {
    lane_forward_cell<N>(A, c, active ? c : 0, active);
  }
}

}  // namespace dragexp
