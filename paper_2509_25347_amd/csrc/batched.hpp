// batched.hpp -- AMR-style blocks with uneven species counts N_b in [1, 16],
// all updated by one hipGraph launch.
//
// Blocks are split by mapping.  Blocks with N_b > LMAX run on the MFMA path
// (a quad of cells per wavefront) in one of three forms the autotuner picks
// from: a persistent grid (N taken at run time, so a single code path serves
// N = LMAX+1..16) whose wavefronts take work items of a few cells from a
// device counter with one atomic add until the queue is empty, so blocks of
// uneven cost balance themselves; one plain grid over those blocks (N at run
// time); or one plain grid per N, each compiled for its N.  Blocks with N_b <= LMAX run one cell
// per lane in one grid per N (one 64-cell item per wavefront), each compiled
// with exactly the registers its N needs.  The plan captures all of them
// into one graph whose lane and MFMA branches are independent, so they can
// overlap.  Every item runs the same per-cell device code as the plain per-N
// launches: a block's result is bit-identical to drag_expm_apply on that
// block with the same mapping.
//
// LMAX is the tuned knob (drag_plan_autotune): the lane mapping is several
// times faster per cell for small N, but its register demand grows as N^2.
#pragma once

#include "common.hpp"
#include "lane.hpp"
#include "pair.hpp"
#include "wave.hpp"

namespace dragexp {

struct BatchItem {
  int32_t block;  // block index
  int32_t n;      // species count of the block
  int32_t first;  // first cell of the item within the block
  int32_t count;  // cells in the item; lane items hold at most 64
};

struct BatchArgs {
  const BatchItem* items;
  const int64_t* field_off;  // element offset of each block's field slab
  const int64_t* v_off;      // element offset of each block's velocity slab
  const double* fields;
  const double* v_in;
  double* v_out;
  unsigned int* counter;     // MFMA queue head (persistent grid only)
  int n_items;
  int block_cells;
  int n_dim;
  int option;
  double dt;
  int k_max_n[kMaxSpecies + 1];  // Taylor cap K of Alg. 1 per species count (index N)
};

__global__ void k_batch_reset(unsigned int* counter) { *counter = 0u; }

__device__ __forceinline__ CellArgs block_args(const BatchArgs& B, const BatchItem& it) {
  const int bc = B.block_cells;
  CellArgs A;
  A.rho_g = B.fields + B.field_off[it.block];
  A.rho_d = A.rho_g + bc;
  A.t_stop = A.rho_d + (int64_t)it.n * bc;
  A.v_in = B.v_in + B.v_off[it.block];
  A.v_out = B.v_out + B.v_off[it.block];
  A.n_cells = bc;
  A.ld = bc;
  A.dt = B.dt;
  A.n_dim = B.n_dim;
  A.k_max = B.k_max_n[it.n];
  A.option = B.option;
  return A;
}

// Persistent MFMA grid over the queue of wave items.
__global__ void __launch_bounds__(256) k_batched_wave(BatchArgs B) {
  __shared__ double lds[4 * kQuadDoubles];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* mine = lds + w * kQuadDoubles;
  for (;;) {
    int idx = 0;
    if (lane == 0) idx = (int)atomicAdd(B.counter, 1u);
    // wave-uniform from here on: the item and its pointers live in SGPRs
    idx = __builtin_amdgcn_readfirstlane(__shfl(idx, 0, 64));
    if (idx >= B.n_items) break;  // every wavefront leaves once the queue is empty
    const BatchItem it = B.items[idx];
    CellArgs A = block_args(B, it);
    A.n_cells = (int64_t)it.first + it.count;  // quads stay inside the item
    for (int k = 0; k < it.count; k += 4)
      wave_forward_quad(A, it.n, (int64_t)it.first + k, lane, mine);
  }
}

// The same MFMA work as a plain grid: workgroup w takes 16 consecutive cells
// of one wave-mapped block (a quad per wavefront).  No loop, so none of the
// loop-invariant state the persistent grid keeps live across items; the
// hardware dispatcher balances the workgroups.  NC = 0 serves every N (taken
// from the item at run time); NC > 0 is a grid over the blocks of that one N,
// compiled for it like the plain per-N kernels.  METHOD is the scaling step
// of the per-N grids: the Taylor approximant, or the diagonal Pade one
// (kStagePade, as drag_expm_apply's Pade option).  The autotuner picks among
// the persistent grid, one run-time-N grid and the per-N grids of either
// method.
template <int NC, int METHOD = kStageTaylor>
__global__ void __launch_bounds__(256, METHOD == kStageTaylor ? 5 : 4)
    k_batched_wave_grid(BatchArgs B, int groups_per_block, int xcd_blocks) {
  __shared__ double lds[4 * kQuadDoubles];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // XCD-aware order (the grid is a multiple of 8): each XCD gets a
  // contiguous run of workgroups, hence whole blocks
  const int wg = (blockIdx.x & 7) * xcd_blocks + (blockIdx.x >> 3);
  const int item = __builtin_amdgcn_readfirstlane(wg / groups_per_block);
  const int g0 = __builtin_amdgcn_readfirstlane((wg % groups_per_block) * 16);
  if (item >= B.n_items || g0 >= B.block_cells) return;  // uniform over the workgroup
  const BatchItem it = B.items[item];  // one whole block
  const CellArgs A = block_args(B, it);
  const int n = NC > 0 ? NC : it.n;
  const int c0 = g0 + 4 * w;
  if (c0 < B.block_cells)
    wave_forward_quad<METHOD, mfma_steps(NC)>(A, n, c0, lane, lds + w * kQuadDoubles, false);
  __syncthreads();
  group_store(A, n, g0, lds);
}

// One 64-cell lane item per wavefront, all items of one species count N.
template <int N>
__global__ void __launch_bounds__(256) k_batched_lane(BatchArgs B) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int idx = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + w);
  if (idx >= B.n_items) return;  // uniform over the wavefront
  const BatchItem it = B.items[idx];
  const CellArgs A = block_args(B, it);
  const bool active = lane < it.count;
  const int64_t c = (int64_t)it.first + lane;
  lane_forward_cell<N>(A, c, active ? c : it.first, active);
}

// One 32-cell item per wavefront, two lanes per cell (N = 9..12).
template <int N>
__global__ void __launch_bounds__(256, pair_fwd_min_waves<N>()) k_batched_pair(BatchArgs B) {
  constexpr int kStride = 128 + 2;  // 32 pairs per wavefront, 4 wavefronts
  __shared__ double vsm[3 * (N + 1) * kStride];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int idx = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + w);
  if (idx >= B.n_items) return;  // uniform over the wavefront
  const BatchItem it = B.items[idx];
  const CellArgs A = block_args(B, it);
  const int p = lane >> 1;
  const bool active = p < it.count;
  const int64_t c = (int64_t)it.first + p;
  pair_forward_cell<N>(A, c, active ? c : it.first, active, lane & 1, vsm + (threadIdx.x >> 1),
                       kStride);
}

}  // namespace dragexp
