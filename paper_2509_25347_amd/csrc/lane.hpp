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
// structured M = 2^-s At: M_jk = -b_j [j == k] - pb_k.  Each degree is one
// left product F <- M (F + c_i I), which the structure makes 2 N^2 + N
// operations: (M G)_ik = -b_i G_ik - cs_k with the weighted column sums
// cs_k = sum_l pb_l G_lk (a right product needs 3 N^2: a plain row sum, then
// one multiply and one fma per entry).  Polynomials in M commute with M, so
// both orders evaluate the same T_m.  Lanes of one wavefront may have
// different m; the loop runs to the wavefront's largest m (wave-uniform, so
// the coefficient is a scalar load) and each lane adds only its own
// coefficients (a zero F stays zero).
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
    for (int i = 0; i < N; ++i) F[i][i] += c;
    double cs[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double acc = pb[0] * F[0][k];
#pragma unroll
      for (int l = 1; l < N; ++l) acc = fma(pb[l], F[l][k], acc);
      cs[k] = acc;
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int k = 0; k < N; ++k) F[i][k] = fma(-b[i], F[i][k], -cs[k]);
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

// Largest x over the wavefront, returned as a wave-uniform (scalar) value so
// that loops bounded by it run on scalar counters.
__device__ __forceinline__ int wave_max_int(int x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return __builtin_amdgcn_readfirstlane(x);
}

// Smallest x over the wavefront, wave-uniform like wave_max_int.
__device__ __forceinline__ int wave_min_int(int x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = min(x, __shfl_xor(x, off, 64));
  return __builtin_amdgcn_readfirstlane(x);
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
  // squarings to the wavefront's largest s, each lane under its own s, two
  // per trip between Z and T.  Up to the wavefront's smallest s every lane
  // squares, with no branch; past it the lanes that are done copy, and the
  // product that may or may not be taken is formed in temporaries and moved
  // (N^2 moves per squaring, 12-25 % of the squaring's instructions).
  const int s = C.kms.s;
  const int s_max = wave_max_int(s);
  const int s_min = wave_min_int(s);
  double T[N][N];
  int it = 0;
  for (; it + 2 <= s_min; it += 2) {
    lane_square_to<N>(T, Z);
    lane_square_to<N>(Z, T);
  }
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

// Raw buffer accesses for the one-lane kernels' inputs and outputs: one
// scalar resource per array (per velocity component), the row as a
// wave-uniform SGPR offset j * row shared by every array, and the cell as
// one 32-bit lane offset shared by every access of the cell.  Prefetching a
// cell's inputs then holds one address register, and the 2N + 1 + D (N + 1)
// rows cost a few resources and N + 1 row offsets instead of a resource or a
// 64-bit address per row (a resource per row needed four SGPRs each: 176 at
// N = 8, which the compiler spilled).  The resource:
// stride 0 (raw), num_records = the array's bytes (bit pattern, below 2^32:
// the host checks 8 ((rows - 1) ld + n_cells) < 2^32), and the CDNA word-3
// flags for 32-bit untyped data; an offset at or past the end reads 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const double* base, uint32_t bytes) {
  constexpr int kRawBufferFlags = 0x00020000;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, (int)bytes,
                                           kRawBufferFlags);
}

__device__ __forceinline__ double rsrc_at(__amdgpu_buffer_rsrc_t r, uint32_t lane_off,
                                          uint32_t row_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, row_off, 0));
}

// ... and the vector store of x at the same kind of address (an offset at or
// past the end is dropped).
__device__ __forceinline__ void rsrc_put(__amdgpu_buffer_rsrc_t r, uint32_t lane_off,
                                         uint32_t row_off, double x) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, lane_off, row_off, 0);
}

// Bytes of an SoA array of `rows` rows of n_cells cells, leading dimension ld.
__device__ __forceinline__ uint32_t array_bytes(int64_t rows, const CellArgs& A) {
  return (uint32_t)(8 * ((rows - 1) * A.ld + A.n_cells));
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
    // stores through a resource for the component's rows, with the same
    // scalar row offsets j * row as the loads (rather than a 64-bit address
    // per row)
    const uint32_t row = (uint32_t)(8 * A.ld);
    const __amdgpu_buffer_rsrc_t r =
        raw_rsrc(A.v_out + (int64_t)d * n1 * A.ld, array_bytes(n1, A));
    const uint32_t off = (uint32_t)(8 * c);
    const double qnan = __builtin_nan("");
    rsrc_put(r, off, 0u, C.bad ? qnan : v[0] + d0);
#pragma unroll
    for (int j = 0; j < N; ++j)
      rsrc_put(r, off, (uint32_t)(1 + j) * row, C.bad ? qnan : v[j + 1] + (d0 + u[j]));
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

// Inputs of cell c, given as the byte offset off = 8 c.
template <int N>
__device__ __forceinline__ void lane_load(LaneCoefs<N>& X, const CellArgs& A, uint32_t off) {
  const uint32_t row = (uint32_t)(8 * A.ld);
  X.rg = rsrc_at(raw_rsrc(A.rho_g, array_bytes(1, A)), off, 0u);
  const __amdgpu_buffer_rsrc_t rt = raw_rsrc(A.t_stop, array_bytes(N, A));
  const __amdgpu_buffer_rsrc_t rd = raw_rsrc(A.rho_d, array_bytes(N, A));
#pragma unroll
  for (int i = 0; i < N; ++i) {
    X.ts[i] = rsrc_at(rt, off, (uint32_t)i * row);
    X.rd[i] = rsrc_at(rd, off, (uint32_t)i * row);
  }
}

// ... and the velocities; components past n_dim repeat the last one (cache
// hits, never used), which keeps the loads unconditional.
template <int N>
__device__ __forceinline__ void lane_load(LaneInputs<N>& X, const CellArgs& A, uint32_t off) {
  lane_load<N>(static_cast<LaneCoefs<N>&>(X), A, off);
  const uint32_t row = (uint32_t)(8 * A.ld);
  const int n1 = N + 1;
  // one resource per component, so that the row offsets j * row are the
  // species rows' own (N + 1 scalar offsets in all, not D (N + 1))
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int dd = d < A.n_dim ? d : A.n_dim - 1;
    const __amdgpu_buffer_rsrc_t rv =
        raw_rsrc(A.v_in + (int64_t)dd * n1 * A.ld, array_bytes(n1, A));
#pragma unroll
    for (int j = 0; j <= N; ++j) X.v[d][j] = rsrc_at(rv, off, (uint32_t)j * row);
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
// Needs every input array within 2^32 bytes (lane_buffers_fit on the host).
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
// it (every input array within 2^32 bytes); otherwise the velocities are read after it, which
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
