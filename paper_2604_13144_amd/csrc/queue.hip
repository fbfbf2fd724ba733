// Work-queue form of the evolve kernel (TEPAI_WORK_QUEUE).
//
// The samples of a batch are independent (sec. "Circuit parallelisation"),
// so where and in which order their work runs is free.  evolve_kernel runs
// one workgroup per slot and leaves placement to the hardware dispatcher,
// which deals workgroups to the eight XCDs in turn, so each XCD works through
// its own share of the launch order.  Here a grid of as many workgroups as
// the device holds at once (one per CU: registers and LDS admit no more)
// takes slot indices from a counter in the workspace, in the batch's launch
// order (decreasing bond cap): whichever CU frees up first starts the next
// sample of the one global list.
//
// The engine of kernels.hip is compiled here a second time, its kernels and
// launchers left out, so that adding this kernel leaves the code generated
// for the one-slot kernels as it is: how the compiler treats the shared
// device functions depends on the set of kernels that call them.
#define TEPAI_ENGINE_ONLY
#include "kernels.hip"

namespace tepai {
namespace {

// queue[0] must be 0 at launch (queue_reset_kernel, on the same stream);
// every workgroup leaves the loop at the first index at or beyond the slot
// count.  The work per slot is evolve_kernel's.
template <int RPL, bool MIX>
__global__ __launch_bounds__(NT) void evolve_queue_kernel(EngineArgs a, uint32_t n_layers,
                                                          uint32_t* queue) {
  __shared__ Shared sh;
  __shared__ z2 Jl[jl_size<RPL>()];
  __shared__ uint32_t next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(queue, 1u);
    sync_block();
    const uint32_t item = next;
    sync_block();   // every thread holds the index before thread 0 takes another
    if (item >= a.count) break;
    const int slot = (int)a.launch_order[item];
    const Slot S = make_slot<MIX>(a, slot, Jl);
    load_state(a, slot, sh);
    const uint32_t sample = (uint32_t)(a.first_sample + slot);
    const uint32_t L = a.l_eff;
    const uint32_t layer0 = a.states[slot].layer;
    for (uint32_t layer = layer0; layer < layer0 + n_layers; ++layer) {
      const uint64_t g0 = (uint64_t)layer * L;
      int nz = 0, nc = 0;
      for (uint32_t r = threadIdx.x; r < L; r += NT) {
        const uint8_t c = draw_setting(a.rows[r], a.seed, sample, g0 + r);
        sh.choice[r] = c;
        nz += c != 0;
        nc += c == 2;
      }
      const double tz = block_sum((double)nz, sh.red);
      const double tc = block_sum((double)nc, sh.red);
      if (threadIdx.x == 0) {
        sh.n_gates += (uint64_t)tz;
        sh.n_c += (int)tc;
      }
      sync_block();
      for (uint32_t r = 0; r < L; ++r) {
        const int c = sh.choice[r];
        if (c == 0) continue;
        process_gate<RPL, MIX>(S, a.rows[r], c, (int)layer, sh);
      }
      flush<RPL, MIX>(S, sh);     // runs end at Trotter-step boundaries
      sync_block();
    }
    store_state(a, slot, sh, layer0 + n_layers);
    sync_block();   // the slot's state is out before the LDS takes the next one
  }
}

__global__ void queue_reset_kernel(uint32_t* queue) {
  if (threadIdx.x == 0) queue[0] = 0u;
}

template <bool MIX>
void evolve_queue_rpl(const EngineArgs& a, uint32_t n_layers, uint32_t* queue, uint32_t grid,
                      hipStream_t s) {
  switch (rows_per_lane(a.chi_max)) {
    case 1: hipLaunchKernelGGL((evolve_queue_kernel<1, MIX>), dim3(grid), dim3(NT), 0, s, a, n_layers, queue); break;
    case 2: hipLaunchKernelGGL((evolve_queue_kernel<2, MIX>), dim3(grid), dim3(NT), 0, s, a, n_layers, queue); break;
    case 4: hipLaunchKernelGGL((evolve_queue_kernel<4, MIX>), dim3(grid), dim3(NT), 0, s, a, n_layers, queue); break;
    default: hipLaunchKernelGGL((evolve_queue_kernel<8, MIX>), dim3(grid), dim3(NT), 0, s, a, n_layers, queue); break;
  }
}

template <bool MIX>
hipError_t queue_blocks_per_cu(uint32_t chi_max, int* n) {
  switch (rows_per_lane(chi_max)) {
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, evolve_queue_kernel<1, MIX>, NT, 0);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, evolve_queue_kernel<2, MIX>, NT, 0);
    case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, evolve_queue_kernel<4, MIX>, NT, 0);
    default: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, evolve_queue_kernel<8, MIX>, NT, 0);
  }
}

}  // namespace

hipError_t evolve_queue_grid(const EngineArgs& a, int device, uint32_t* grid) {
  int cus = 0, per_cu = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e == hipSuccess)
    e = a.mixed ? queue_blocks_per_cu<true>(a.chi_max, &per_cu)
                : queue_blocks_per_cu<false>(a.chi_max, &per_cu);
  if (e != hipSuccess) return e;
  *grid = (uint32_t)((cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1));
  return hipSuccess;
}

hipError_t launch_evolve_queue(const EngineArgs& a, uint32_t n_layers, uint32_t* queue,
                               uint32_t grid, hipStream_t s) {
  (void)hipGetLastError();
  grid = grid < 1 ? 1 : grid > a.count ? a.count : grid;
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, s, queue);
  if (a.mixed)
    evolve_queue_rpl<true>(a, n_layers, queue, grid, s);
  else
    evolve_queue_rpl<false>(a, n_layers, queue, grid, s);
  return hipGetLastError();
}

}  // namespace tepai
