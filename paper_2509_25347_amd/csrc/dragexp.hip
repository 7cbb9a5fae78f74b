// dragexp.hip -- kernels and C ABI of the MI355X drag-update library.
//
// v(t+dt) = exp(dt K) v per cell, Taylor scaling and squaring (Sewanou,
// Laibe and Commercon, arXiv:2509.25347, Sect. 2.3 and Appendix B).  The ABI
// is declared and documented in include/dragexp.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/dragexp.h"
#include "common.hpp"
#include "lane.hpp"
#include "wave.hpp"
#include "adjoint.hpp"
#include "pair.hpp"
#include "batched.hpp"
#include "rk1.hpp"
#include "big.hpp"

namespace dragexp {

constexpr int kLaneMaxN = 8;   // one lane per cell
constexpr int kPairMaxN = 12;  // two lanes per cell (forward)
constexpr int kPairBwdMaxN = 10;  // two lanes per cell (adjoint)

// ---- drag_build -------------------------------------------------------------
struct BuildArgs {
  const double* rho_g;
  const double* rho_d;
  const double* t_stop;
  double* a_out;
  double* e_out;
  double* norm_out;
  int32_t* k_out;
  int32_t* m_out;
  int32_t* s_out;
  int64_t n_cells, ld;
  double dt;
  int n_species, k_max, option;
  int pade = 0;  // report the Pade scaling step's (m, s) instead of Alg. 1's
};

__global__ void __launch_bounds__(256) k_build(BuildArgs B, int xcd_blocks) {
  const int bid = blockIdx.x;
  const int64_t logical = (int64_t)(bid & 7) * xcd_blocks + (bid >> 3);
  const int64_t c = logical * 256 + threadIdx.x;
  if (c >= B.n_cells) return;
  const int N = B.n_species;
  const int64_t ld = B.ld;
  const double rg = B.rho_g[c];
  unsigned bad = gas_bad(rg);
  double s = 0.0;
  bool finite = true;
  for (int i = 0; i < N; ++i) {
    const double t = B.t_stop[i * ld + c], r = B.rho_d[i * ld + c];
    bad |= species_bad(t, r);
    const Species sp = species_coeffs(B.dt, t, r, rg);
    s = s + sp.p;
    finite = finite && isfinite(sp.a) && isfinite(sp.p);
  }
  double nrm = s;
  for (int i = 0; i < N; ++i) {
    const Species sp = species_coeffs(B.dt, B.t_stop[i * ld + c], B.rho_d[i * ld + c], rg);
    nrm = nrm + sp.a;
  }
  for (int i = 0; i < N; ++i) {
    const Species sp = species_coeffs(B.dt, B.t_stop[i * ld + c], B.rho_d[i * ld + c], rg);
    nrm = fmax(nrm, sp.p + sp.a);
  }
  if (!bad && !(finite && isfinite(nrm))) bad |= kBadNorm;
  const double qnan = __builtin_nan("");
  for (int i = 0; i < N; ++i) {
    const Species sp = species_coeffs(B.dt, B.t_stop[i * ld + c], B.rho_d[i * ld + c], rg);
    if (B.a_out) B.a_out[i * ld + c] = bad ? qnan : sp.a;
    if (B.e_out) B.e_out[i * ld + c] = bad ? qnan : sp.e;
  }
  Kms km = bad ? Kms{0, 0, 0} : select_kms(nrm, B.k_max, B.option);
  if (B.pade && !bad) {  // the Pade scaling step's (0, m, s)
    const PadeSel ps = pade_select(nrm);
    km = Kms{0, kPadeM[ps.row], ps.s};
  }
  if (B.norm_out) B.norm_out[c] = bad ? qnan : nrm;
  if (B.k_out) B.k_out[c] = km.k;
  if (B.m_out) B.m_out[c] = km.m;
  if (B.s_out) B.s_out[c] = km.s;
  if (bad) atomicOr(&g_status_word, bad);
}

__global__ void k_clear_status() { g_status_word = 0u; }

// ---- launch helpers ------------------------------------------------------------
struct Grid {
  unsigned blocks;  // multiple of 8
  int xcd_blocks;   // blocks / 8
};

static Grid grid_for(int64_t n_units) {
  int64_t b = (n_units + 7) / 8 * 8;
  if (b < 8) b = 8;
  return Grid{(unsigned)b, (int)(b / 8)};
}

static int hip_status(hipError_t e) { return e == hipSuccess ? DRAG_OK : DRAG_ERR_HIP; }

// Compute units per device id (0 until asked).
static std::atomic<int> g_device_cus[64];

// Workgroups of 256 threads of `kernel` resident on the current device at
// once (`per_cu`, the kernel's occupancy, is cached by the caller).
static int resident_blocks(const void* kernel, std::atomic<int>& per_cu, int* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DRAG_ERR_HIP;
  int cus = g_device_cus[dev].load(std::memory_order_relaxed);
  if (cus == 0) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return DRAG_ERR_HIP;
    g_device_cus[dev].store(cus, std::memory_order_relaxed);
  }
  int pc = per_cu.load(std::memory_order_relaxed);
  if (pc == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, kernel, 256, 0) != hipSuccess)
      return DRAG_ERR_HIP;
    if (pc < 1) pc = 1;
    per_cu.store(pc, std::memory_order_relaxed);
  }
  *out = pc * cus;
  return DRAG_OK;
}

// The one-lane forward: the streaming kernel (prefetch of the next cell,
// a grid of the resident wavefronts) for N = 7, 8, where few wavefronts fit
// on a SIMD (2 and 1) to hide the loads; the one-shot kernel below, where
// enough are resident and the prefetch registers would cut them (1.03-1.17x
// slower at N = 5, 6).  The one-shot kernel issues all of a cell's loads up
// front except at N = 3, where the velocities' registers would cut the
// resident wavefronts from 8 to 5 (interleaved timings, 2^18-2^20 cells).
// The batched lane grids keep the plain form: each wavefront takes one item,
// and issuing every load up front there was 0.5 % slower per replay.
constexpr int kLaneStreamMinN = 7;
constexpr bool lane_early_loads(int n) { return n != 3 && n < kLaneStreamMinN; }

// The raw buffer accesses of the one-lane kernels address each array with
// 32-bit byte offsets: its last byte, 8 ((rows - 1) ld + n_cells), must lie
// below 2^32 (the velocities in and out, D (N + 1) rows, are the largest).
template <int N>
static bool lane_buffers_fit(const CellArgs& A) {
  const int64_t rows = (int64_t)A.n_dim * (N + 1);
  return A.ld < (int64_t(1) << 32) && 8 * ((rows - 1) * A.ld + A.n_cells) < (int64_t(1) << 32);
}

template <int N>
static int launch_forward_lane(const CellArgs& A, hipStream_t st) {
  if constexpr (N >= kLaneStreamMinN) {
    if (lane_buffers_fit<N>(A)) {
      static std::atomic<int> per_cu{0};
      int resident = 0;
      const int rc = resident_blocks(reinterpret_cast<const void*>(&k_forward_lane_stream<N>),
                                     per_cu, &resident);
      if (rc) return rc;
      const int64_t need = (A.n_cells + 255) / 256;
      const unsigned blocks = (unsigned)(need < resident ? (need < 1 ? 1 : need) : resident);
      hipLaunchKernelGGL(k_forward_lane_stream<N>, dim3(blocks), dim3(256), 0, st, A);
      return hip_status(hipGetLastError());
    }
  }
  const Grid gr = grid_for((A.n_cells + 255) / 256);
  if constexpr (lane_early_loads(N)) {
    if (lane_buffers_fit<N>(A)) {
      hipLaunchKernelGGL((k_forward_lane<N, true>), dim3(gr.blocks), dim3(256), 0, st, A,
                         gr.xcd_blocks);
      return hip_status(hipGetLastError());
    }
  }
  hipLaunchKernelGGL(k_forward_lane<N>, dim3(gr.blocks), dim3(256), 0, st, A, gr.xcd_blocks);
  return hip_status(hipGetLastError());
}

template <int N, int METHOD = kStageTaylor>
static int launch_forward_wave(const CellArgs& A, hipStream_t st) {
  const Grid gr = grid_for((A.n_cells + 15) / 16);  // a quad of cells per wavefront
  hipLaunchKernelGGL((k_forward_wave<N, METHOD>), dim3(gr.blocks), dim3(256), 0, st, A,
                     gr.xcd_blocks);
  return hip_status(hipGetLastError());
}

template <int N>
static int launch_rk1(const CellArgs& A, hipStream_t st) {
  const Grid gr = grid_for((A.n_cells + 255) / 256);
  hipLaunchKernelGGL(k_rk1_lane<N>, dim3(gr.blocks), dim3(256), 0, st, A, gr.xcd_blocks);
  return hip_status(hipGetLastError());
}

// N = 17..32: one cell per wavefront, four per workgroup
static int launch_forward_big(const CellArgs& A, int N, hipStream_t st) {
  const Grid gr = grid_for((A.n_cells + 3) / 4);
  hipLaunchKernelGGL(k_forward_big, dim3(gr.blocks), dim3(256), 0, st, A, N, gr.xcd_blocks);
  return hip_status(hipGetLastError());
}

template <int N>
static int launch_forward_pair(const CellArgs& A, hipStream_t st) {
  const Grid gr = grid_for((A.n_cells + 127) / 128);  // 128 cells per workgroup
  hipLaunchKernelGGL(k_forward_pair<N>, dim3(gr.blocks), dim3(256), 0, st, A, gr.xcd_blocks);
  return hip_status(hipGetLastError());
}

using FwdFn = int (*)(const CellArgs&, hipStream_t);
using BwdFn = int (*)(const BackArgs&, hipStream_t);

template <int N>
static int launch_backward_lane(const BackArgs& A, hipStream_t st) {
  const Grid gr = grid_for((A.n_cells + 255) / 256);
  hipLaunchKernelGGL(k_backward_lane<N>, dim3(gr.blocks), dim3(256), 0, st, A, gr.xcd_blocks);
  return hip_status(hipGetLastError());
}

// two lanes per cell (pair.hpp), 128 cells per workgroup
template <int N>
static int launch_backward_pair(const BackArgs& A, hipStream_t st) {
  const Grid gr = grid_for((A.n_cells + 127) / 128);
  hipLaunchKernelGGL((k_backward_pair<N, (N >= 9 ? 1 : 2)>), dim3(gr.blocks), dim3(256), 0, st, A,
                     gr.xcd_blocks);
  return hip_status(hipGetLastError());
}

template <int N>
static int launch_backward_wave(const BackArgs& A, hipStream_t st) {
  const Grid gr = grid_for((A.n_cells + 15) / 16);  // a quad of cells per wavefront
  hipLaunchKernelGGL(k_backward_wave<N>, dim3(gr.blocks), dim3(256), 0, st, A, gr.xcd_blocks);
  return hip_status(hipGetLastError());
}

// N <= 8: the block form (both blocks of [[B, dB], [0, B]] on one tile).
template <int N>
static int launch_backward_block(const BackArgs& A, hipStream_t st) {
  const Grid gr = grid_for((A.n_cells + 15) / 16);  // a quad of cells per wavefront
  hipLaunchKernelGGL(k_backward_block<N>, dim3(gr.blocks), dim3(256), 0, st, A, gr.xcd_blocks);
  return hip_status(hipGetLastError());
}

static BwdFn wave_bwd(int N) {
  static const BwdFn tab[16] = {
      launch_backward_block<1>, launch_backward_block<2>, launch_backward_block<3>,
      launch_backward_block<4>, launch_backward_block<5>, launch_backward_block<6>,
      launch_backward_block<7>, launch_backward_block<8>, launch_backward_wave<9>,
      launch_backward_wave<10>, launch_backward_wave<11>, launch_backward_wave<12>,
      launch_backward_wave<13>, launch_backward_wave<14>, launch_backward_wave<15>,
      launch_backward_wave<16>};
  return tab[N - 1];
}

static BwdFn lane_bwd(int N) {
  static const BwdFn tab[kPairBwdMaxN] = {
      launch_backward_lane<1>, launch_backward_lane<2>, launch_backward_lane<3>,
      launch_backward_lane<4>, launch_backward_lane<5>, launch_backward_lane<6>,
      launch_backward_lane<7>, launch_backward_pair<8>, launch_backward_pair<9>,
      launch_backward_pair<10>};
  return tab[N - 1];
}

static FwdFn wave_fwd(int N) {
  static const FwdFn tab[16] = {
      launch_forward_wave<1>,  launch_forward_wave<2>,  launch_forward_wave<3>,
      launch_forward_wave<4>,  launch_forward_wave<5>,  launch_forward_wave<6>,
      launch_forward_wave<7>,  launch_forward_wave<8>,  launch_forward_wave<9>,
      launch_forward_wave<10>, launch_forward_wave<11>, launch_forward_wave<12>,
      launch_forward_wave<13>, launch_forward_wave<14>, launch_forward_wave<15>,
      launch_forward_wave<16>};
  return tab[N - 1];
}

static FwdFn rk1_fwd(int N) {
  static const FwdFn tab[16] = {
      launch_rk1<1>,  launch_rk1<2>,  launch_rk1<3>,  launch_rk1<4>,
      launch_rk1<5>,  launch_rk1<6>,  launch_rk1<7>,  launch_rk1<8>,
      launch_rk1<9>,  launch_rk1<10>, launch_rk1<11>, launch_rk1<12>,
      launch_rk1<13>, launch_rk1<14>, launch_rk1<15>, launch_rk1<16>};
  return tab[N - 1];
}

// The MFMA forward with another scaling step, for every N: Sastre's second
// modification in the Taylor stage (the bound test), or the diagonal Pade
// approximant.
template <int METHOD>
static FwdFn wave_fwd_method(int N) {
  static const FwdFn tab[16] = {
      launch_forward_wave<1, METHOD>,  launch_forward_wave<2, METHOD>,
      launch_forward_wave<3, METHOD>,  launch_forward_wave<4, METHOD>,
      launch_forward_wave<5, METHOD>,  launch_forward_wave<6, METHOD>,
      launch_forward_wave<7, METHOD>,  launch_forward_wave<8, METHOD>,
      launch_forward_wave<9, METHOD>,  launch_forward_wave<10, METHOD>,
      launch_forward_wave<11, METHOD>, launch_forward_wave<12, METHOD>,
      launch_forward_wave<13, METHOD>, launch_forward_wave<14, METHOD>,
      launch_forward_wave<15, METHOD>, launch_forward_wave<16, METHOD>};
  return tab[N - 1];
}

// The vector-ALU forward: one lane per cell up to N = 8, a pair of lanes per
// cell for N = 9..12.
static FwdFn lane_fwd(int N) {
  static const FwdFn tab[kPairMaxN] = {
      launch_forward_lane<1>,  launch_forward_lane<2>,  launch_forward_lane<3>,
      launch_forward_lane<4>,  launch_forward_lane<5>,  launch_forward_lane<6>,
      launch_forward_lane<7>,  launch_forward_lane<8>,  launch_forward_pair<9>,
      launch_forward_pair<10>, launch_forward_pair<11>, launch_forward_pair<12>};
  return tab[N - 1];
}

// Tuned default mapping per N (index N - 1).  Overridable with
// drag_set_mapping.  The vector ALU up to N = 12 (one lane per cell to 8, two
// lanes per cell for 9..12: measured on MI355X over 2^18 cells, 2.0x faster
// than the MFMA tile at N = 9, 10 and 1.1x at 11, 12, whose 16 x 16 tile is
// mostly padding there), the MFMA kernel above.
static int g_default_map[16] = {
    DRAG_MAP_LANE, DRAG_MAP_LANE, DRAG_MAP_LANE, DRAG_MAP_LANE,
    DRAG_MAP_LANE, DRAG_MAP_LANE, DRAG_MAP_LANE, DRAG_MAP_LANE,
    DRAG_MAP_LANE, DRAG_MAP_LANE, DRAG_MAP_LANE, DRAG_MAP_LANE,
    DRAG_MAP_WAVE, DRAG_MAP_WAVE, DRAG_MAP_WAVE, DRAG_MAP_WAVE};
static int g_map_override[16] = {0};

// Default mapping of the adjoint.  The lane mapping keeps Y, dY and a
// product buffer per cell in registers: one lane per cell up to N = 7, two
// lanes per cell at N = 8..10, where one lane spills (pair.hpp).  Measured on
// MI355X (2^18 stiff cells): N = 8 one lane 1.64 ms, two lanes 0.77 ms, MFMA
// block form 1.08 ms; N = 7 one lane 0.54 ms, MFMA 1.07 ms; N = 9, 10 two
// lanes 1.51 / 1.56 ms against 2.83 / 2.84 for the MFMA kernel (1.5x on the
// jittered cells).
static int g_default_map_bwd[16] = {
    DRAG_MAP_LANE, DRAG_MAP_LANE, DRAG_MAP_LANE, DRAG_MAP_LANE,
    DRAG_MAP_LANE, DRAG_MAP_LANE, DRAG_MAP_LANE, DRAG_MAP_LANE,
    DRAG_MAP_LANE, DRAG_MAP_LANE, DRAG_MAP_WAVE, DRAG_MAP_WAVE,
    DRAG_MAP_WAVE, DRAG_MAP_WAVE, DRAG_MAP_WAVE, DRAG_MAP_WAVE};

static int mapping_for(int N) {
  const int o = g_map_override[N - 1];
  int m = o ? o : g_default_map[N - 1];
  if (m == DRAG_MAP_LANE && N > kPairMaxN) m = DRAG_MAP_WAVE;
  return m;
}

static int mapping_for_bwd(int N) {
  const int o = g_map_override[N - 1];
  int m = o ? o : g_default_map_bwd[N - 1];
  if (m == DRAG_MAP_LANE && N > kPairBwdMaxN) m = DRAG_MAP_WAVE;
  return m;
}

// Taylor cap K of Alg. 1 used when a descriptor asks for DRAG_K_AUTO (index
// N - 1), overridable with drag_set_k_max.  Every K gives an approximant
// accurate to u (the selection keeps ||A / 2^s|| <= theta_m); K only trades
// polynomial degree against squarings.  The one-lane kernel evaluates the
// polynomial by Horner in the structured matrix (m steps of 2 N^2 + N) and
// squares densely (N^3 per squaring), so small N prefers low degrees; the
// MFMA kernel is flat for K >= 7.  The table holds, per N, the K with the
// least summed time over the stiff and the jittered recipes (2^18 cells,
// `bench.py --k-sweep`: every K = 2..9, interleaved repeats): against K = 9
// it takes 0.84-0.96 of the time for N = 2..8, 0.92-0.95 on the
// two-lanes-per-cell kernel (N = 9..12), 0.99 on the MFMA kernel; at
// N = 1, 2, 8, 10 another K is faster by 0.4-1.3 %, about the spread of
// repeated runs.
static const int g_default_kmax[16] = {4, 3, 4, 5, 5, 6, 5, 6, 6, 6, 6, 6, 7, 7, 7, 7};
static int g_kmax_override[16] = {0};

static int k_for(int k_max, int N) {
  if (k_max != DRAG_K_AUTO) return k_max;
  if (N > kMaxSpecies) return 7;  // the large-N kernel: K = 6-7 within 3 % (N = 17..32)
  const int o = g_kmax_override[N - 1];
  return o ? o : g_default_kmax[N - 1];
}

// ---- argument checks -------------------------------------------------------------
// max_species: 16 (one MFMA tile), or 32 for the entry points that have the
// large-N forward kernel (drag_build, drag_expm_apply, drag_expm_steps).
static int check_desc(const drag_desc* d, int max_species = kMaxSpecies) {
  if (!d) return DRAG_ERR_NULL_DESC;
  if (d->n_cells < 0) return DRAG_ERR_N_CELLS;
  if (d->n_species < 1 || d->n_species > max_species) return DRAG_ERR_N_SPECIES;
  if (d->n_dim < 1 || d->n_dim > 3) return DRAG_ERR_N_DIM;
  if (d->ld < d->n_cells || d->ld < 1) return DRAG_ERR_LD;
  // every index (row * ld + c) must fit in int64 with room to spare
  if (d->ld > (INT64_MAX / 64)) return DRAG_ERR_LD;
  if (!(d->dt >= 0.0) || !isfinite(d->dt)) return DRAG_ERR_DT;
  if (d->k_max < DRAG_K_AUTO || d->k_max > 9) return DRAG_ERR_K_MAX;
  const int opt = d->option & ~(DRAG_OPTION_BOUND_TEST | DRAG_OPTION_PADE);
  if (opt < 0 || opt > 2) return DRAG_ERR_OPTION;
  if ((d->option & DRAG_OPTION_BOUND_TEST) && (d->option & DRAG_OPTION_PADE))
    return DRAG_ERR_OPTION;
  return DRAG_OK;
}

// [first, last) byte ranges of the arrays, for overlap checks
struct Range {
  uintptr_t lo, hi;
};

static Range span(const void* p, int64_t rows, int64_t ld, int64_t n_cells) {
  if (!p || n_cells == 0) return Range{0, 0};
  const uintptr_t lo = (uintptr_t)p;
  const uintptr_t hi = lo + (uintptr_t)(((rows - 1) * ld + n_cells) * (int64_t)sizeof(double));
  return Range{lo, hi};
}

static bool overlap(Range a, Range b) {
  if (a.lo == a.hi || b.lo == b.hi) return false;
  return a.lo < b.hi && b.lo < a.hi;
}


// ---- batched plans ----------------------------------------------------------------
constexpr int kBatchVariants = 9;
constexpr int kBatchLmax[kBatchVariants] = {4, 5, 6, 7, 8, 9, 10, 11, 12};
constexpr int kWaveItemCells = 8;
// how the MFMA branch runs: a persistent grid over the item queue, a plain
// grid over the blocks (N at run time), or one plain grid per N
constexpr int kWavePersistent = 0;
constexpr int kWaveGrid = 1;
constexpr int kWavePerN = 2;
constexpr int kWavePerNPade = 3;  // per-N grids with the Pade scaling step
constexpr int kWaveModes = 4;
// smallest Taylor cap the plan's autotuner tries (K = 1, 2 cap m at 2 and 4:
// every cell then needs many squarings)
constexpr int kTuneKMin = 3;

struct BatchVariant {
  int lmax = 6;
  BatchItem* d_wave = nullptr;  // MFMA queue (blocks with N > lmax)
  int n_wave = 0;
  BatchItem* d_wave_blocks = nullptr;  // the same blocks whole, for the plain grid
  int n_wave_blocks = 0;
  BatchItem* d_wave_n[kMaxSpecies + 1] = {};  // the same blocks whole, per N
  int n_wave_n[kMaxSpecies + 1] = {};
  BatchItem* d_lane[kPairMaxN + 1] = {};  // lane (64-cell) or pair (32-cell) items per N <= lmax
  int n_lane[kPairMaxN + 1] = {};
};

template <int N>
static void launch_batched_lane(const BatchArgs& B, hipStream_t st) {
  hipLaunchKernelGGL(k_batched_lane<N>, dim3((B.n_items + 3) / 4), dim3(256), 0, st, B);
}

template <int N, int METHOD>
static void launch_batched_wave_n(const BatchArgs& B, int gpb, hipStream_t st) {
  const Grid gr = grid_for((int64_t)B.n_items * gpb);
  hipLaunchKernelGGL((k_batched_wave_grid<N, METHOD>), dim3(gr.blocks), dim3(256), 0, st, B,
                     gpb, gr.xcd_blocks);
}

template <int METHOD>
static void batched_wave_n_method(int N, const BatchArgs& B, int gpb, hipStream_t st) {
  switch (N) {
    case 5: launch_batched_wave_n<5, METHOD>(B, gpb, st); break;
    case 6: launch_batched_wave_n<6, METHOD>(B, gpb, st); break;
    case 7: launch_batched_wave_n<7, METHOD>(B, gpb, st); break;
    case 8: launch_batched_wave_n<8, METHOD>(B, gpb, st); break;
    case 9: launch_batched_wave_n<9, METHOD>(B, gpb, st); break;
    case 10: launch_batched_wave_n<10, METHOD>(B, gpb, st); break;
    case 11: launch_batched_wave_n<11, METHOD>(B, gpb, st); break;
    case 12: launch_batched_wave_n<12, METHOD>(B, gpb, st); break;
    case 13: launch_batched_wave_n<13, METHOD>(B, gpb, st); break;
    case 14: launch_batched_wave_n<14, METHOD>(B, gpb, st); break;
    case 15: launch_batched_wave_n<15, METHOD>(B, gpb, st); break;
    default: launch_batched_wave_n<16, METHOD>(B, gpb, st); break;
  }
}

// N = 5..16: the species counts the MFMA branch can hold (LMAX >= 4)
static void batched_wave_n(int N, const BatchArgs& B, int gpb, hipStream_t st,
                           bool pade = false) {
  if (pade) batched_wave_n_method<kStagePade>(N, B, gpb, st);
  else batched_wave_n_method<kStageTaylor>(N, B, gpb, st);
}

template <int N>
static void launch_batched_pair(const BatchArgs& B, hipStream_t st) {
  hipLaunchKernelGGL(k_batched_pair<N>, dim3((B.n_items + 3) / 4), dim3(256), 0, st, B);
}

static void batched_lane(int N, const BatchArgs& B, hipStream_t st) {
  switch (N) {
    case 1: launch_batched_lane<1>(B, st); break;
    case 2: launch_batched_lane<2>(B, st); break;
    case 3: launch_batched_lane<3>(B, st); break;
    case 4: launch_batched_lane<4>(B, st); break;
    case 5: launch_batched_lane<5>(B, st); break;
    case 6: launch_batched_lane<6>(B, st); break;
    case 7: launch_batched_lane<7>(B, st); break;
    case 8: launch_batched_lane<8>(B, st); break;
    case 9: launch_batched_pair<9>(B, st); break;
    case 10: launch_batched_pair<10>(B, st); break;
    case 11: launch_batched_pair<11>(B, st); break;
    default: launch_batched_pair<12>(B, st); break;
  }
}

}  // namespace dragexp

struct drag_plan {
  int device = 0;
  int n_blocks = 0, block_cells = 0, n_dim = 0, k_max = 9, option = 2;
  int k_n[dragexp::kMaxSpecies + 1] = {};  // Taylor cap per N (index N)
  double dt = 0.0;
  std::vector<int32_t> n_species;
  std::vector<int64_t> field_off, v_off;
  int64_t fields_total = 0, v_total = 0;
  int lmax = 6;
  int wave_mode = dragexp::kWaveGrid;
  dragexp::BatchVariant var[dragexp::kBatchVariants];
  int wave_grid = 0;
  int64_t* d_field_off = nullptr;
  int64_t* d_v_off = nullptr;
  unsigned int* d_counter = nullptr;
  hipStream_t cap_stream = nullptr, side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const double* g_fields = nullptr;
  const double* g_vin = nullptr;
  double* g_vout = nullptr;
  int g_lmax = 0;
  int g_mode = -1;
};

namespace dragexp {

static void plan_drop_graph(drag_plan* P) {
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  P->exec = nullptr;
  P->graph = nullptr;
  P->g_fields = P->g_vin = nullptr;
  P->g_vout = nullptr;
  P->g_lmax = 0;
  P->g_mode = -1;
}

static void plan_free(drag_plan* P) {
  plan_drop_graph(P);
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  if (P->ev_join) (void)hipEventDestroy(P->ev_join);
  if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
  if (P->side_stream) (void)hipStreamDestroy(P->side_stream);
  for (BatchVariant& V : P->var) {
    if (V.d_wave) (void)hipFree(V.d_wave);
    if (V.d_wave_blocks) (void)hipFree(V.d_wave_blocks);
    for (BatchItem* p : V.d_wave_n)
      if (p) (void)hipFree(p);
    for (BatchItem* p : V.d_lane)
      if (p) (void)hipFree(p);
  }
  if (P->d_field_off) (void)hipFree(P->d_field_off);
  if (P->d_v_off) (void)hipFree(P->d_v_off);
  if (P->d_counter) (void)hipFree(P->d_counter);
  delete P;
}

static int upload(BatchItem** dst, const std::vector<BatchItem>& host) {
  if (host.empty()) return DRAG_OK;
  if (hipMalloc(dst, sizeof(BatchItem) * host.size()) != hipSuccess) return DRAG_ERR_HIP;
  if (hipMemcpy(*dst, host.data(), sizeof(BatchItem) * host.size(), hipMemcpyHostToDevice) !=
      hipSuccess)
    return DRAG_ERR_HIP;
  return DRAG_OK;
}

static int plan_init(drag_plan* P, const drag_batch_desc* bd) {
  if (hipGetDevice(&P->device) != hipSuccess) return DRAG_ERR_HIP;
  P->n_blocks = bd->n_blocks;
  P->block_cells = bd->block_cells;
  P->n_dim = bd->n_dim;
  P->k_max = bd->k_max;
  for (int n = 1; n <= kMaxSpecies; ++n) P->k_n[n] = k_for(bd->k_max, n);
  P->option = bd->option;
  P->dt = bd->dt;
  P->n_species.assign(bd->n_species, bd->n_species + bd->n_blocks);
  const int64_t bc = bd->block_cells, D = bd->n_dim;
  P->field_off.resize(P->n_blocks);
  P->v_off.resize(P->n_blocks);
  int64_t fo = 0, vo = 0;
  for (int b = 0; b < P->n_blocks; ++b) {
    const int64_t n = P->n_species[b];
    P->field_off[b] = fo;
    P->v_off[b] = vo;
    fo += bc * (1 + 2 * n);
    vo += bc * D * (n + 1);
  }
  P->fields_total = fo;
  P->v_total = vo;
  for (int v = 0; v < kBatchVariants; ++v) {
    BatchVariant& V = P->var[v];
    V.lmax = kBatchLmax[v];
    std::vector<BatchItem> wave, wave_blocks;
    std::vector<BatchItem> lane[kPairMaxN + 1], wave_n[kMaxSpecies + 1];
    for (int b = 0; b < P->n_blocks; ++b) {
      const int n = P->n_species[b];
      const bool is_lane = n <= V.lmax;
      if (!is_lane) {
        wave_blocks.push_back(BatchItem{b, n, 0, P->block_cells});
        wave_n[n].push_back(BatchItem{b, n, 0, P->block_cells});
      }
      const int step = is_lane ? (n <= kLaneMaxN ? 64 : 32) : kWaveItemCells;
      for (int first = 0; first < P->block_cells; first += step) {
        const BatchItem it{b, n, first, std::min(step, P->block_cells - first)};
        if (is_lane) lane[n].push_back(it);
        else wave.push_back(it);
      }
    }
    V.n_wave = (int)wave.size();
    V.n_wave_blocks = (int)wave_blocks.size();
    int rc = upload(&V.d_wave, wave);
    if (!rc) rc = upload(&V.d_wave_blocks, wave_blocks);
    for (int n = 1; n <= kPairMaxN && !rc; ++n) {
      V.n_lane[n] = (int)lane[n].size();
      rc = upload(&V.d_lane[n], lane[n]);
    }
    for (int n = 1; n <= kMaxSpecies && !rc; ++n) {
      V.n_wave_n[n] = (int)wave_n[n].size();
      rc = upload(&V.d_wave_n[n], wave_n[n]);
    }
    if (rc) return rc;
  }
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched_wave, 256, 0) != hipSuccess)
    return DRAG_ERR_HIP;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess)
    return DRAG_ERR_HIP;
  P->wave_grid = (per_cu < 1 ? 1 : per_cu) * cus;
  if (hipMalloc(&P->d_field_off, sizeof(int64_t) * P->n_blocks) != hipSuccess) return DRAG_ERR_HIP;
  if (hipMalloc(&P->d_v_off, sizeof(int64_t) * P->n_blocks) != hipSuccess) return DRAG_ERR_HIP;
  if (hipMalloc(&P->d_counter, sizeof(unsigned int)) != hipSuccess) return DRAG_ERR_HIP;
  if (hipMemcpy(P->d_field_off, P->field_off.data(), sizeof(int64_t) * P->n_blocks,
                hipMemcpyHostToDevice) != hipSuccess)
    return DRAG_ERR_HIP;
  if (hipMemcpy(P->d_v_off, P->v_off.data(), sizeof(int64_t) * P->n_blocks,
                hipMemcpyHostToDevice) != hipSuccess)
    return DRAG_ERR_HIP;
  if (hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return DRAG_ERR_HIP;
  if (hipStreamCreateWithFlags(&P->side_stream, hipStreamNonBlocking) != hipSuccess)
    return DRAG_ERR_HIP;
  if (hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess)
    return DRAG_ERR_HIP;
  if (hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming) != hipSuccess)
    return DRAG_ERR_HIP;
  return DRAG_OK;
}

// Enqueue one batched update (variant lmax): the MFMA grids on `main`, the
// lane grids on `side` between a fork and a join (the largest two-lane grid
// after the MFMA grids on `main`): captured, this is the plan's graph.
static int plan_enqueue(drag_plan* P, int lmax, int mode, const double* fields,
                        const double* v_in, double* v_out, hipStream_t main, hipStream_t side) {
  int v = 0;
  while (v + 1 < kBatchVariants && kBatchLmax[v] != lmax) ++v;
  const BatchVariant& V = P->var[v];
  BatchArgs B{nullptr, P->d_field_off, P->d_v_off, fields, v_in, v_out, P->d_counter,
              0,       P->block_cells, P->n_dim, P->option, P->dt, {}};
  for (int n = 0; n <= kMaxSpecies; ++n) B.k_max_n[n] = P->k_n[n];
  if (hipEventRecord(P->ev_fork, main) != hipSuccess) return DRAG_ERR_HIP;
  if (hipStreamWaitEvent(side, P->ev_fork, 0) != hipSuccess) return DRAG_ERR_HIP;
  // The largest two-lane grid (N = lmax) goes to the end of the MFMA branch:
  // behind the one-lane grids it ran alone after the MFMA grids had ended.
  const int tail_n = lmax > kLaneMaxN ? lmax : 0;
  for (int n = 1; n <= kPairMaxN; ++n) {
    if (V.n_lane[n] == 0 || n == tail_n) continue;
    BatchArgs L = B;
    L.items = V.d_lane[n];
    L.n_items = V.n_lane[n];
    batched_lane(n, L, side);
  }
  if (hipEventRecord(P->ev_join, side) != hipSuccess) return DRAG_ERR_HIP;
  if (V.n_wave > 0 && mode == kWavePersistent) {
    BatchArgs W = B;
    W.items = V.d_wave;
    W.n_items = V.n_wave;
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, main, P->d_counter);
    hipLaunchKernelGGL(k_batched_wave, dim3(P->wave_grid), dim3(256), 0, main, W);
  } else if (V.n_wave > 0 && mode == kWaveGrid) {
    BatchArgs W = B;
    W.items = V.d_wave_blocks;
    W.n_items = V.n_wave_blocks;
    const int gpb = (P->block_cells + 15) / 16;
    const Grid gr = grid_for((int64_t)V.n_wave_blocks * gpb);
    hipLaunchKernelGGL(k_batched_wave_grid<0>, dim3(gr.blocks), dim3(256), 0, main, W, gpb,
                       gr.xcd_blocks);
  } else if (V.n_wave > 0) {
    const int gpb = (P->block_cells + 15) / 16;
    for (int n = kMaxSpecies; n > lmax; --n) {  // largest N (longest blocks) first
      if (V.n_wave_n[n] == 0) continue;
      BatchArgs W = B;
      W.items = V.d_wave_n[n];
      W.n_items = V.n_wave_n[n];
      batched_wave_n(n, W, gpb, main, mode == kWavePerNPade);
    }
  }
  if (tail_n && V.n_lane[tail_n] > 0) {
    BatchArgs L = B;
    L.items = V.d_lane[tail_n];
    L.n_items = V.n_lane[tail_n];
    batched_lane(tail_n, L, main);
  }
  if (hipStreamWaitEvent(main, P->ev_join, 0) != hipSuccess) return DRAG_ERR_HIP;
  return hip_status(hipGetLastError());
}

// Capture the update for these pointers and this lmax into the plan's graph.
static int plan_capture(drag_plan* P, int lmax, int mode, const double* fields,
                        const double* v_in, double* v_out) {
  plan_drop_graph(P);
  if (hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return DRAG_ERR_HIP;
  const int rc =
      plan_enqueue(P, lmax, mode, fields, v_in, v_out, P->cap_stream, P->side_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(P->cap_stream, &g);
  if (rc || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return DRAG_ERR_HIP;
  }
  P->graph = g;
  if (hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0) != hipSuccess) {
    P->exec = nullptr;
    return DRAG_ERR_HIP;
  }
  P->g_fields = fields;
  P->g_vin = v_in;
  P->g_vout = v_out;
  P->g_lmax = lmax;
  P->g_mode = mode;
  return DRAG_OK;
}

// ---- the batched update without allocation ------------------------------------
// A fixed device buffer per GPU (file scope, so the code object reserves it on
// every device the library loads on, until the process ends) holds the block
// offsets and the work items that drag_plan_batched would allocate; the host
// builds them in a fixed host buffer and copies them on the caller's stream.
// In host code `scratch` names a host-side stand-in: the device address comes
// from hipGetSymbolAddress, once per device, and only that address is used.
constexpr size_t kStaticScratchBytes = DRAG_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kStaticLaneMax = 10;  // the configuration the static call runs
constexpr int kMaxDevices = 64;

static std::mutex g_static_mu;  // one static call at a time per process (host buffer)
static void* g_scratch_dev[kMaxDevices] = {};
alignas(256) static unsigned char g_scratch_host[kStaticScratchBytes];

// Device address of this device's scratch array (resolved at the first call
// on the device, with the device current).
static int scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return DRAG_ERR_HIP;
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DRAG_ERR_HIP;
    g_scratch_dev[dev] = ptr;
  }
  *out = (unsigned char*)g_scratch_dev[dev];
  return DRAG_OK;
}

// Byte layout of the tables in the scratch buffer for one batch: field and
// velocity offsets [n_blocks] each, then the items of each lane-mapped N
// (64-cell items to 8 species, 32-cell pair items above) and each MFMA N
// (whole blocks), every table 16-byte aligned.
struct StaticLayout {
  size_t off_field = 0, off_v = 0, off_lane[kPairMaxN + 1] = {}, off_wave[kMaxSpecies + 1] = {};
  int n_lane[kPairMaxN + 1] = {}, n_wave[kMaxSpecies + 1] = {};
  size_t bytes = 0;
};

static StaticLayout static_layout(const drag_batch_desc* bd) {
  StaticLayout L;
  const int bc = bd->block_cells;
  for (int b = 0; b < bd->n_blocks; ++b) {
    const int n = bd->n_species[b];
    if (n <= kStaticLaneMax) L.n_lane[n] += (bc + (n <= kLaneMaxN ? 63 : 31)) / (n <= kLaneMaxN ? 64 : 32);
    else L.n_wave[n] += 1;
  }
  size_t at = 0;
  L.off_field = at;
  at += sizeof(int64_t) * (size_t)bd->n_blocks;
  L.off_v = at;
  at += sizeof(int64_t) * (size_t)bd->n_blocks;
  for (int n = 1; n <= kStaticLaneMax; ++n) {
    L.off_lane[n] = at;
    at += sizeof(BatchItem) * (size_t)L.n_lane[n];
  }
  for (int n = kStaticLaneMax + 1; n <= kMaxSpecies; ++n) {
    L.off_wave[n] = at;
    at += sizeof(BatchItem) * (size_t)L.n_wave[n];
  }
  L.bytes = at;
  return L;
}

// Fill the host buffer with the tables of static_layout (same items, in the
// same order, as the plan's configuration (kStaticLaneMax, per-N grids)).
static void static_tables(const drag_batch_desc* bd, const StaticLayout& L, unsigned char* host,
                          int64_t* fields_total, int64_t* v_total) {
  int64_t* fo = (int64_t*)(host + L.off_field);
  int64_t* vo = (int64_t*)(host + L.off_v);
  const int64_t bc = bd->block_cells, D = bd->n_dim;
  int64_t f = 0, v = 0;
  int fill_lane[kPairMaxN + 1] = {}, fill_wave[kMaxSpecies + 1] = {};
  for (int b = 0; b < bd->n_blocks; ++b) {
    const int n = bd->n_species[b];
    fo[b] = f;
    vo[b] = v;
    f += bc * (1 + 2 * n);
    v += bc * D * (n + 1);
    if (n <= kStaticLaneMax) {
      BatchItem* it = (BatchItem*)(host + L.off_lane[n]);
      const int step = n <= kLaneMaxN ? 64 : 32;
      for (int first = 0; first < bd->block_cells; first += step)
        it[fill_lane[n]++] = BatchItem{b, n, first, std::min(step, bd->block_cells - first)};
    } else {
      BatchItem* it = (BatchItem*)(host + L.off_wave[n]);
      it[fill_wave[n]++] = BatchItem{b, n, 0, bd->block_cells};
    }
  }
  *fields_total = f;
  *v_total = v;
}

}  // namespace dragexp

using namespace dragexp;

extern "C" {

void drag_desc_init(drag_desc* d, int64_t n_cells, int32_t n_species, int32_t n_dim,
                    double dt) {
  if (!d) return;
  d->n_cells = n_cells;
  d->n_species = n_species;
  d->n_dim = n_dim;
  d->ld = n_cells;
  d->dt = dt;
  d->k_max = 9;
  d->option = 2;
}

int drag_build(const drag_desc* d, const double* rho_g, const double* rho_d,
               const double* t_stop, double* a_out, double* e_out, double* norm_out,
               int32_t* k_out, int32_t* m_out, int32_t* s_out, drag_stream_t stream) {
  int rc = check_desc(d, kBigMaxSpecies);
  if (rc) return rc;
  if (d->n_cells == 0) return DRAG_OK;
  if (!rho_g || !rho_d || !t_stop) return DRAG_ERR_NULL_POINTER;
  const int64_t C = d->n_cells, ld = d->ld, N = d->n_species;
  const Range in[3] = {span(rho_g, 1, ld, C), span(rho_d, N, ld, C), span(t_stop, N, ld, C)};
  const Range out[6] = {span(a_out, N, ld, C), span(e_out, N, ld, C), span(norm_out, 1, ld, C),
                        Range{(uintptr_t)k_out, k_out ? (uintptr_t)(k_out + C) : 0},
                        Range{(uintptr_t)m_out, m_out ? (uintptr_t)(m_out + C) : 0},
                        Range{(uintptr_t)s_out, s_out ? (uintptr_t)(s_out + C) : 0}};
  for (const Range& o : out) {
    for (const Range& i : in)
      if (overlap(o, i)) return DRAG_ERR_ALIAS;
  }
  for (int x = 0; x < 6; ++x)
    for (int y = x + 1; y < 6; ++y)
      if (overlap(out[x], out[y])) return DRAG_ERR_ALIAS;
  BuildArgs B{rho_g, rho_d, t_stop, a_out, e_out, norm_out, k_out, m_out, s_out,
              C,     ld,    d->dt,  (int)N, k_for(d->k_max, (int)N), d->option & 3};
  B.pade = (d->option & DRAG_OPTION_PADE) ? 1 : 0;
  const Grid gr = grid_for((C + 255) / 256);
  hipLaunchKernelGGL(k_build, dim3(gr.blocks), dim3(256), 0, (hipStream_t)stream, B,
                     gr.xcd_blocks);
  return hip_status(hipGetLastError());
}

int drag_expm_apply(const drag_desc* d, const double* rho_g, const double* rho_d,
                    const double* t_stop, const double* v_in, double* v_out,
                    drag_stream_t stream) {
  int rc = check_desc(d, kBigMaxSpecies);
  if (rc) return rc;
  if (d->n_cells == 0) return DRAG_OK;
  if (!rho_g || !rho_d || !t_stop || !v_in || !v_out) return DRAG_ERR_NULL_POINTER;
  const int64_t C = d->n_cells, ld = d->ld, N = d->n_species, D = d->n_dim;
  const Range ro = span(v_out, D * (N + 1), ld, C);
  if (overlap(ro, span(rho_g, 1, ld, C)) || overlap(ro, span(rho_d, N, ld, C)) ||
      overlap(ro, span(t_stop, N, ld, C)))
    return DRAG_ERR_ALIAS;
  if ((const double*)v_out != v_in && overlap(ro, span(v_in, D * (N + 1), ld, C)))
    return DRAG_ERR_ALIAS;
  CellArgs A{rho_g, rho_d, t_stop, v_in, v_out, C,
             ld,    d->dt, (int)D, k_for(d->k_max, (int)N), d->option & 3};
  if (N > kMaxSpecies) {  // the large-N kernel has the plain Taylor step only
    if (d->option & (DRAG_OPTION_PADE | DRAG_OPTION_BOUND_TEST)) return DRAG_ERR_OPTION;
    return launch_forward_big(A, (int)N, (hipStream_t)stream);
  }
  if (d->option & DRAG_OPTION_PADE)
    return wave_fwd_method<kStagePade>((int)N)(A, (hipStream_t)stream);
  if (d->option & DRAG_OPTION_BOUND_TEST)
    return wave_fwd_method<kStageTaylorBound>((int)N)(A, (hipStream_t)stream);
  const int map = mapping_for((int)N);
  return map == DRAG_MAP_LANE ? lane_fwd((int)N)(A, (hipStream_t)stream)
                              : wave_fwd((int)N)(A, (hipStream_t)stream);
}

int drag_rk1_apply(const drag_desc* d, const double* rho_g, const double* rho_d,
                   const double* t_stop, const double* v_in, double* v_out,
                   drag_stream_t stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (d->n_cells == 0) return DRAG_OK;
  if (!rho_g || !rho_d || !t_stop || !v_in || !v_out) return DRAG_ERR_NULL_POINTER;
  const int64_t C = d->n_cells, ld = d->ld, N = d->n_species, D = d->n_dim;
  const Range ro = span(v_out, D * (N + 1), ld, C);
  if (overlap(ro, span(rho_g, 1, ld, C)) || overlap(ro, span(rho_d, N, ld, C)) ||
      overlap(ro, span(t_stop, N, ld, C)))
    return DRAG_ERR_ALIAS;
  if ((const double*)v_out != v_in && overlap(ro, span(v_in, D * (N + 1), ld, C)))
    return DRAG_ERR_ALIAS;
  CellArgs A{rho_g, rho_d, t_stop, v_in, v_out, C, ld, d->dt, (int)D, d->k_max, d->option & 3};
  return rk1_fwd((int)N)(A, (hipStream_t)stream);
}

int drag_expm_steps(const drag_desc* d, const double* rho_g, const double* rho_d,
                    const double* t_stop, const double* v_in, double* v_out, int64_t n_steps,
                    double* history, drag_stream_t stream) {
  int rc = check_desc(d, kBigMaxSpecies);
  if (rc) return rc;
  if (n_steps < 0) return DRAG_ERR_STEPS;
  if (d->n_cells == 0 || n_steps == 0) {
    if (d->n_cells && n_steps == 0 && (const double*)v_out != v_in) {
      if (!v_in || !v_out) return DRAG_ERR_NULL_POINTER;
      // zero steps: v_out = v_in
      drag_desc one = *d;
      one.dt = 0.0;  // the identity (equal values)
      return drag_expm_apply(&one, rho_g, rho_d, t_stop, v_in, v_out, stream);
    }
    return DRAG_OK;
  }
  if (!rho_g || !rho_d || !t_stop || !v_in || !v_out) return DRAG_ERR_NULL_POINTER;
  const int64_t C = d->n_cells, ld = d->ld, N = d->n_species, D = d->n_dim;
  const int64_t slab = D * (N + 1) * ld;  // elements of one velocity state
  if (history) {
    if (n_steps > INT64_MAX / slab) return DRAG_ERR_STEPS;
    const Range rh{(uintptr_t)history, (uintptr_t)(history + n_steps * slab)};
    if (overlap(rh, span(rho_g, 1, ld, C)) || overlap(rh, span(rho_d, N, ld, C)) ||
        overlap(rh, span(t_stop, N, ld, C)) || overlap(rh, span(v_in, D * (N + 1), ld, C)) ||
        overlap(rh, span(v_out, D * (N + 1), ld, C)))
      return DRAG_ERR_ALIAS;
  }
  // step i reads the state after step i - 1 and writes history[i] (or v_out)
  const double* src = v_in;
  for (int64_t i = 0; i < n_steps; ++i) {
    double* dst = history ? history + i * slab : v_out;
    rc = drag_expm_apply(d, rho_g, rho_d, t_stop, src, dst, stream);
    if (rc) return rc;
    src = dst;
  }
  if (history) {
    const size_t bytes = sizeof(double) * (size_t)((D * (N + 1) - 1) * ld + C);
    if (hipMemcpyAsync(v_out, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream) !=
        hipSuccess)
      return DRAG_ERR_HIP;
  }
  return DRAG_OK;
}

int drag_expm_apply_backward(const drag_desc* d, const double* rho_g, const double* rho_d,
                             const double* t_stop, const double* v_in, const double* w,
                             double* v_out, double* g_v, double* g_logt, double* g_t,
                             double* g_rho_d, double* g_rho_g, drag_stream_t stream) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (d->n_cells == 0) return DRAG_OK;
  if (!rho_g || !rho_d || !t_stop || !v_in || !w) return DRAG_ERR_NULL_POINTER;
  const int64_t C = d->n_cells, ld = d->ld, N = d->n_species, D = d->n_dim;
  const int64_t nv = D * (N + 1);
  const Range in[5] = {span(rho_g, 1, ld, C), span(rho_d, N, ld, C), span(t_stop, N, ld, C),
                       span(v_in, nv, ld, C), span(w, nv, ld, C)};
  const Range out[6] = {span(v_out, nv, ld, C), span(g_v, nv, ld, C), span(g_logt, N, ld, C),
                        span(g_t, N, ld, C), span(g_rho_d, N, ld, C), span(g_rho_g, 1, ld, C)};
  for (int x = 0; x < 6; ++x) {
    for (const Range& i : in)
      if (overlap(out[x], i)) return DRAG_ERR_ALIAS;
    for (int y = x + 1; y < 6; ++y)
      if (overlap(out[x], out[y])) return DRAG_ERR_ALIAS;
  }
  // the adjoint differentiates the Taylor evaluation without the bound test
  if (d->option & (DRAG_OPTION_BOUND_TEST | DRAG_OPTION_PADE)) return DRAG_ERR_OPTION;
  BackArgs B{rho_g, rho_d, t_stop, v_in, w, v_out, g_v, g_logt, g_t, g_rho_d, g_rho_g,
             C,     ld,    d->dt,  (int)D, k_for(d->k_max, (int)N), d->option};
  const int map = mapping_for_bwd((int)N);
  return map == DRAG_MAP_LANE ? lane_bwd((int)N)(B, (hipStream_t)stream)
                              : wave_bwd((int)N)(B, (hipStream_t)stream);
}

int drag_plan_batched(const drag_batch_desc* bd, drag_plan** out) {
  if (!out) return DRAG_ERR_NULL_POINTER;
  *out = nullptr;
  if (!bd) return DRAG_ERR_NULL_DESC;
  if (bd->n_blocks < 1 || bd->block_cells < 1 || !bd->n_species) return DRAG_ERR_PLAN;
  if (bd->n_dim < 1 || bd->n_dim > 3) return DRAG_ERR_N_DIM;
  if (!(bd->dt >= 0.0) || !isfinite(bd->dt)) return DRAG_ERR_DT;
  if (bd->k_max < DRAG_K_AUTO || bd->k_max > 9) return DRAG_ERR_K_MAX;
  if (bd->option < 0 || bd->option > 2) return DRAG_ERR_OPTION;
  for (int b = 0; b < bd->n_blocks; ++b)
    if (bd->n_species[b] < 1 || bd->n_species[b] > kMaxSpecies) return DRAG_ERR_N_SPECIES;
  drag_plan* P = new drag_plan();
  int rc = plan_init(P, bd);
  if (rc) {
    plan_free(P);
    return rc;
  }
  *out = P;
  return DRAG_OK;
}

int drag_plan_offsets(const drag_plan* P, int64_t* field_offset, int64_t* v_offset,
                      int64_t* fields_total, int64_t* v_total) {
  if (!P) return DRAG_ERR_PLAN;
  if (field_offset)
    memcpy(field_offset, P->field_off.data(), sizeof(int64_t) * P->field_off.size());
  if (v_offset) memcpy(v_offset, P->v_off.data(), sizeof(int64_t) * P->v_off.size());
  if (fields_total) *fields_total = P->fields_total;
  if (v_total) *v_total = P->v_total;
  return DRAG_OK;
}

int drag_expm_apply_batched(drag_plan* P, const double* fields, const double* v_in,
                            double* v_out, drag_stream_t stream) {
  if (!P) return DRAG_ERR_PLAN;
  if (!fields || !v_in || !v_out) return DRAG_ERR_NULL_POINTER;
  const Range rf{(uintptr_t)fields, (uintptr_t)(fields + P->fields_total)};
  const Range ri{(uintptr_t)v_in, (uintptr_t)(v_in + P->v_total)};
  const Range ro{(uintptr_t)v_out, (uintptr_t)(v_out + P->v_total)};
  if (overlap(ro, rf)) return DRAG_ERR_ALIAS;
  if ((const double*)v_out != v_in && overlap(ro, ri)) return DRAG_ERR_ALIAS;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != P->device) return DRAG_ERR_PLAN;
  if (!P->exec || P->g_fields != fields || P->g_vin != v_in || P->g_vout != v_out ||
      P->g_lmax != P->lmax || P->g_mode != P->wave_mode) {
    const int rc = plan_capture(P, P->lmax, P->wave_mode, fields, v_in, v_out);
    if (rc) return rc;
  }
  return hip_status(hipGraphLaunch(P->exec, (hipStream_t)stream));
}

int drag_plan_autotune(drag_plan* P, const double* fields, const double* v_in, double* v_out,
                       drag_stream_t stream, int32_t* lane_max_out) {
  if (!P) return DRAG_ERR_PLAN;
  if (!fields || !v_in || !v_out) return DRAG_ERR_NULL_POINTER;
  const Range rf{(uintptr_t)fields, (uintptr_t)(fields + P->fields_total)};
  const Range ri{(uintptr_t)v_in, (uintptr_t)(v_in + P->v_total)};
  const Range ro{(uintptr_t)v_out, (uintptr_t)(v_out + P->v_total)};
  if (overlap(ro, rf) || overlap(ro, ri)) return DRAG_ERR_ALIAS;  // runs repeat: no in-place
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return DRAG_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DRAG_ERR_HIP;
  }
  float best_ms = 0.0f;
  int best = P->lmax, best_mode = P->wave_mode, rc = DRAG_OK;
  bool have = false;
  for (int mode = 0; mode < kWaveModes && rc == DRAG_OK; ++mode) {
    for (int v = 0; v < kBatchVariants && rc == DRAG_OK; ++v) {
      rc = plan_capture(P, kBatchLmax[v], mode, fields, v_in, v_out);
      float ms = 0.0f;
      for (int rep = 0; rep < 3 && rc == DRAG_OK; ++rep) {  // rep 0 warms up
        rc = hip_status(hipEventRecord(e0, st));
        if (!rc) rc = hip_status(hipGraphLaunch(P->exec, st));
        if (!rc) rc = hip_status(hipEventRecord(e1, st));
        if (!rc) rc = hip_status(hipEventSynchronize(e1));
        float t = 0.0f;
        if (!rc) rc = hip_status(hipEventElapsedTime(&t, e0, e1));
        if (rep == 1 || (rep > 1 && t < ms)) ms = t;
      }
      if (!rc && (!have || ms < best_ms)) {
        have = true;
        best_ms = ms;
        best = kBatchLmax[v];
        best_mode = mode;
      }
    }
  }
  if (!rc) {
    P->lmax = best;
    P->wave_mode = best_mode;
  }
  // Taylor cap per species count (a DRAG_K_AUTO plan only): each N's own
  // launch (its lane grid, or its MFMA grid compiled for N) timed alone for
  // every K; the per-cell code is the same in every MFMA form, so the choice
  // carries over to the persistent and run-time-N grids.
  if (!rc && P->k_max == DRAG_K_AUTO) {
    int v = 0;
    while (v + 1 < kBatchVariants && kBatchLmax[v] != P->lmax) ++v;
    const BatchVariant& V = P->var[v];
    const int gpb = (P->block_cells + 15) / 16;
    BatchArgs B{nullptr, P->d_field_off, P->d_v_off, fields, v_in, v_out, P->d_counter,
                0,       P->block_cells, P->n_dim, P->option, P->dt, {}};
    for (int n = 1; n <= kMaxSpecies; ++n) B.k_max_n[n] = P->k_n[n];
    for (int n = 1; n <= kMaxSpecies && rc == DRAG_OK; ++n) {
      const bool lane = n <= P->lmax;
      if ((lane ? V.n_lane[n] : V.n_wave_n[n]) == 0) continue;
      if (!lane && P->wave_mode == kWavePerNPade) continue;  // the Pade step takes no cap
      BatchArgs X = B;
      X.items = lane ? V.d_lane[n] : V.d_wave_n[n];
      X.n_items = lane ? V.n_lane[n] : V.n_wave_n[n];
      float kbest_ms = 0.0f;
      int kbest = P->k_n[n];
      for (int K = kTuneKMin; K <= 9 && rc == DRAG_OK; ++K) {
        X.k_max_n[n] = K;
        float ms = 0.0f;
        for (int rep = 0; rep < 3 && rc == DRAG_OK; ++rep) {  // rep 0 warms up
          rc = hip_status(hipEventRecord(e0, st));
          if (!rc) {
            if (lane) batched_lane(n, X, st);
            else batched_wave_n(n, X, gpb, st);
            rc = hip_status(hipGetLastError());
          }
          if (!rc) rc = hip_status(hipEventRecord(e1, st));
          if (!rc) rc = hip_status(hipEventSynchronize(e1));
          float t = 0.0f;
          if (!rc) rc = hip_status(hipEventElapsedTime(&t, e0, e1));
          if (rep == 1 || (rep > 1 && t < ms)) ms = t;
        }
        if (!rc && (K == kTuneKMin || ms < kbest_ms)) {
          kbest_ms = ms;
          kbest = K;
        }
      }
      if (!rc) P->k_n[n] = kbest;
    }
    // leave v_out holding the result of the chosen configuration
    if (!rc) rc = plan_enqueue(P, P->lmax, P->wave_mode, fields, v_in, v_out, st, P->side_stream);
    if (!rc) rc = hip_status(hipStreamSynchronize(st));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  plan_drop_graph(P);
  if (rc) return rc;
  if (lane_max_out) *lane_max_out = P->lmax;
  return DRAG_OK;
}

int drag_plan_k_max(const drag_plan* P, int32_t* k_max) {
  if (!P) return DRAG_ERR_PLAN;
  if (!k_max) return DRAG_ERR_NULL_POINTER;
  for (int n = 1; n <= kMaxSpecies; ++n) k_max[n - 1] = P->k_n[n];
  return DRAG_OK;
}

int drag_plan_config(const drag_plan* P, int32_t* lane_max, int32_t* mfma_mode) {
  if (!P) return DRAG_ERR_PLAN;
  if (lane_max) *lane_max = P->lmax;
  if (mfma_mode) *mfma_mode = P->wave_mode;
  return DRAG_OK;
}

int drag_plan_set_config(drag_plan* P, int32_t lane_max, int32_t mfma_mode) {
  if (!P) return DRAG_ERR_PLAN;
  bool known = false;
  for (int v = 0; v < kBatchVariants; ++v) known = known || kBatchLmax[v] == lane_max;
  if (!known || mfma_mode < 0 || mfma_mode >= kWaveModes) return DRAG_ERR_OPTION;
  P->lmax = lane_max;
  P->wave_mode = mfma_mode;
  return DRAG_OK;
}

int drag_plan_destroy(drag_plan* P) {
  if (!P) return DRAG_OK;
  plan_free(P);
  return DRAG_OK;
}

int drag_expm_apply_batched_static(const drag_batch_desc* bd, const double* fields,
                                   const double* v_in, double* v_out, drag_stream_t stream) {
  if (!bd) return DRAG_ERR_NULL_DESC;
  if (bd->n_blocks < 1 || bd->block_cells < 1 || !bd->n_species) return DRAG_ERR_PLAN;
  if (bd->n_dim < 1 || bd->n_dim > 3) return DRAG_ERR_N_DIM;
  if (!(bd->dt >= 0.0) || !isfinite(bd->dt)) return DRAG_ERR_DT;
  if (bd->k_max < DRAG_K_AUTO || bd->k_max > 9) return DRAG_ERR_K_MAX;
  if (bd->option < 0 || bd->option > 2) return DRAG_ERR_OPTION;
  for (int b = 0; b < bd->n_blocks; ++b)
    if (bd->n_species[b] < 1 || bd->n_species[b] > kMaxSpecies) return DRAG_ERR_N_SPECIES;
  if (!fields || !v_in || !v_out) return DRAG_ERR_NULL_POINTER;
  const StaticLayout L = static_layout(bd);
  if (L.bytes > kStaticScratchBytes) return DRAG_ERR_SCRATCH;
  std::lock_guard<std::mutex> lock(g_static_mu);
  int64_t fields_total = 0, v_total = 0;
  static_tables(bd, L, g_scratch_host, &fields_total, &v_total);
  const Range rf{(uintptr_t)fields, (uintptr_t)(fields + fields_total)};
  const Range ri{(uintptr_t)v_in, (uintptr_t)(v_in + v_total)};
  const Range ro{(uintptr_t)v_out, (uintptr_t)(v_out + v_total)};
  if (overlap(ro, rf)) return DRAG_ERR_ALIAS;
  if ((const double*)v_out != v_in && overlap(ro, ri)) return DRAG_ERR_ALIAS;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DRAG_ERR_HIP;
  unsigned char* base = nullptr;
  int rc = scratch_address(dev, &base);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  // a copy from pageable host memory: the runtime has read the host buffer
  // when the call returns, so the buffer may be refilled by the next call
  rc = hip_status(hipMemcpyAsync(base, g_scratch_host, L.bytes, hipMemcpyHostToDevice, st));
  if (rc) return rc;
  BatchArgs B{nullptr, (const int64_t*)(base + L.off_field), (const int64_t*)(base + L.off_v),
              fields, v_in, v_out, nullptr, 0, bd->block_cells, bd->n_dim, bd->option, bd->dt,
              {}};
  for (int n = 0; n <= kMaxSpecies; ++n) B.k_max_n[n] = n ? k_for(bd->k_max, n) : 0;
  for (int n = 1; n <= kStaticLaneMax; ++n) {
    if (L.n_lane[n] == 0) continue;
    BatchArgs X = B;
    X.items = (const BatchItem*)(base + L.off_lane[n]);
    X.n_items = L.n_lane[n];
    batched_lane(n, X, st);
  }
  const int gpb = (bd->block_cells + 15) / 16;
  for (int n = kMaxSpecies; n > kStaticLaneMax; --n) {
    if (L.n_wave[n] == 0) continue;
    BatchArgs X = B;
    X.items = (const BatchItem*)(base + L.off_wave[n]);
    X.n_items = L.n_wave[n];
    batched_wave_n(n, X, gpb, st);
  }
  return hip_status(hipGetLastError());
}

int drag_get_status(drag_stream_t stream, int32_t* host_status) {
  if (!host_status) return DRAG_ERR_NULL_POINTER;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return DRAG_ERR_HIP;
  unsigned v = 0;
  e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_status_word), sizeof(v), 0, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return DRAG_ERR_HIP;
  *host_status = (int32_t)v;
  return DRAG_OK;
}

int drag_clear_status(drag_stream_t stream) {
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, (hipStream_t)stream);
  return hip_status(hipGetLastError());
}

const char* drag_status_string(int code) {
  switch (code) {
    case DRAG_OK: return "ok";
    case DRAG_ERR_NULL_DESC: return "descriptor pointer is NULL";
    case DRAG_ERR_N_CELLS: return "n_cells < 0";
    case DRAG_ERR_N_SPECIES: return "n_species outside [1, 16] (or [1, 32] for the forward calls)";
    case DRAG_ERR_N_DIM: return "n_dim outside [1, 3]";
    case DRAG_ERR_STEPS: return "n_steps < 0, or the history would overflow 64-bit offsets";
    case DRAG_ERR_SCRATCH: return "the batch's block tables exceed the static scratch buffer";
    case DRAG_ERR_LD: return "ld < n_cells or ld too large";
    case DRAG_ERR_DT: return "dt is NaN, infinite or negative";
    case DRAG_ERR_K_MAX: return "k_max outside [0 (auto), 9]";
    case DRAG_ERR_OPTION: return "option not 0, 1 or 2, or a bound-test bit this call does not take";
    case DRAG_ERR_NULL_POINTER: return "a required pointer is NULL";
    case DRAG_ERR_ALIAS: return "an output overlaps an input";
    case DRAG_ERR_PLAN: return "invalid batched plan or block table";
    case DRAG_ERR_HIP: return "HIP runtime error";
    default: return "unknown status code";
  }
}

int drag_table_row(int k, int32_t* m, int32_t* q, int32_t* r, double* theta) {
  if (k < 1 || k > 9) return DRAG_ERR_K_MAX;
  if (m) *m = kTabM[k];
  if (q) *q = kTabQ[k];
  if (r) *r = kTabR[k];
  if (theta) *theta = kTheta[k];
  return DRAG_OK;
}

int drag_select(double norm, int32_t k_max, int32_t option, int32_t* k, int32_t* m,
                int32_t* s) {
  if (k_max < 1 || k_max > 9) return DRAG_ERR_K_MAX;
  if (option < 0 || option > 2) return DRAG_ERR_OPTION;
  if (!(norm >= 0.0) || !isfinite(norm)) return DRAG_ERR_DT;
  const Kms r = select_kms(norm, k_max, option);
  if (k) *k = r.k;
  if (m) *m = r.m;
  if (s) *s = r.s;
  return DRAG_OK;
}

int drag_pade_row(int32_t row, int32_t* m, double* theta, double* coef) {
  if (row < 0 || row >= kPadeRows) return DRAG_ERR_OPTION;
  if (m) *m = kPadeM[row];
  if (theta) *theta = kPadeTheta[row];
  if (coef)
    for (int j = 0; j <= kPadeM[row]; ++j) coef[j] = kPadeC[row][j];
  return DRAG_OK;
}

int drag_set_k_max(int32_t n_species, int32_t k_max) {
  if (n_species < 1 || n_species > kMaxSpecies) return DRAG_ERR_N_SPECIES;
  if (k_max < DRAG_K_AUTO || k_max > 9) return DRAG_ERR_K_MAX;
  g_kmax_override[n_species - 1] = k_max;
  return DRAG_OK;
}

int drag_get_k_max(int32_t n_species, int32_t* k_max) {
  if (n_species < 1 || n_species > kMaxSpecies) return DRAG_ERR_N_SPECIES;
  if (!k_max) return DRAG_ERR_NULL_POINTER;
  *k_max = k_for(DRAG_K_AUTO, n_species);
  return DRAG_OK;
}

int drag_set_mapping(int32_t n_species, int32_t mapping) {
  if (n_species < 1 || n_species > kMaxSpecies) return DRAG_ERR_N_SPECIES;
  if (mapping != DRAG_MAP_AUTO && mapping != DRAG_MAP_LANE && mapping != DRAG_MAP_WAVE)
    return DRAG_ERR_OPTION;
  if (mapping == DRAG_MAP_LANE && n_species > kPairMaxN) return DRAG_ERR_OPTION;
  g_map_override[n_species - 1] = mapping;
  return DRAG_OK;
}

int drag_get_mapping(int32_t n_species, int32_t* mapping) {
  if (n_species < 1 || n_species > kMaxSpecies) return DRAG_ERR_N_SPECIES;
  if (!mapping) return DRAG_ERR_NULL_POINTER;
  *mapping = mapping_for(n_species);
  return DRAG_OK;
}

}  // extern "C"
