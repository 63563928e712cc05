// Persistent batched stepping: one kernel does many launches' worth of steps over a batch's
// instance table, its workgroups meeting at bounded grid barriers between launches.  Kept apart
// from the step kernel's header: it reuses that kernel's per-tile work (step_tile) and the
// open-top pass without changing them.
#pragma once
#include "lbm_step.hpp"

namespace lbm {

// ------------------------------------------------------------------------- persistent batches

// Grid barrier of a persistent launch.  count grows by one per workgroup and barrier and is
// cleared before each launch, so barrier j is complete when it reaches G (j + 1).  The wait is
// bounded: a workgroup that has spun spin_limit times (or sees another one give up) sets abort and
// returns false, and every workgroup then leaves the kernel, so a launch whose workgroups are not
// all resident at once ends with abort set instead of hanging.
struct GridBar {
  unsigned count;
  unsigned abort;
  unsigned ticket[NXCD];  // tiles handed out so far to the workgroups of each XCD's band
};

__device__ __forceinline__ bool grid_barrier(GridBar* bar, unsigned target, unsigned spin_limit) {
  __shared__ unsigned ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    // release: the workgroup's stores (ordered before this thread by the workgroup barrier) are
    // visible at device scope before its arrival is
    __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0u, good = 1u;
    // Poll with relaxed loads (device-coherent, so they see the other workgroups' arrivals) and
    // acquire once at the end: an acquiring load invalidates the XCD's L2, and doing that on every
    // poll would throw away the lines that workgroups already past the barrier have just loaded.
    while (__hip_atomic_load(&bar->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins >= spin_limit) {
        __hip_atomic_store(&bar->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0u;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the other workgroups' stores are visible
    ok = good;
  }
  __syncthreads();
  return ok != 0u;
}

// Clears the barrier before a persistent launch (a kernel, so that it can live in a graph).
__global__ void grid_bar_reset_kernel(GridBar* bar) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    bar->count = 0u;
    bar->abort = 0u;
    for (int x = 0; x < NXCD; ++x) bar->ticket[x] = 0u;
  }
}

// nlaunch launches of shape S in one kernel: the workgroups (all resident, gridDim.x a multiple of
// the 8 XCDs) loop over the tiles of every active instance for one launch's steps, meet at a grid
// barrier, run the open-top pass of the entries that have one (then meet again), and go on with the
// next launch.  Each XCD's workgroups take a contiguous band of tiles, as the remap of step_kernel
// does, one tile at a time from a counter of the band (tiles cost unequally -- boundary tiles take
// the general path -- so a fixed share per workgroup would leave the barrier waiting for the
// workgroups that hold the slow ones).  In launch L every workgroup of the band draws until it gets
// a ticket past the band, so the band hands out exactly (band length + its workgroups) tickets per
// launch and launch L starts from L times that.  Every node's arithmetic is that of step_kernel, so
// results are bit-identical to nlaunch launches of it.
template <typename real, class S, int QG>
__global__ __launch_bounds__(S::NT) void persist_kernel(const InstDesc<real>* __restrict__ table, int ninst,
                                                        const long long* __restrict__ clock, int total_tiles,
                                                        int nlaunch, int open, GridBar* bar, unsigned spin_limit) {
  __shared__ TileLds<real, S, QG> lds;
  __shared__ double part[OPEN_NT / 64];
  __shared__ int drawn;
  const long long c0 = *clock;
  const int G = gridDim.x;
  const int xcd = blockIdx.x % NXCD, gx = G / NXCD;
  const int band = (total_tiles + NXCD - 1) / NXCD;
  const int b0 = min(total_tiles, xcd * band), b1 = min(total_tiles, b0 + band);
  const unsigned per_launch = (unsigned)(b1 - b0 + gx);
  const LaunchWin w{0, 0, 0, 0, 0, 0};
  unsigned nbar = 0u;
  for (int L = 0; L < nlaunch; ++L) {
    const long long t = c0 + (long long)L * S::DEPTH;
    for (;;) {
      if (threadIdx.x == 0)
        drawn = (int)(__hip_atomic_fetch_add(&bar->ticket[xcd], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                      (unsigned)L * per_launch);
      __syncthreads();
      const int k = __builtin_amdgcn_readfirstlane(drawn);  // uniform: keeps the tile's indexing scalar
      __syncthreads();  // every thread has read the ticket before the next draw
      if (k >= b1 - b0) break;
      // the thread index enters the tile as an opaque value, so that the compiler derives the
      // per-thread addresses inside the loop instead of keeping them live across it (which spilled)
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      step_tile<real, S, QG>(table, ninst, t, w, b0 + k, lds, tid);
      __syncthreads();  // the next tile reuses the LDS
    }
    if (!grid_barrier(bar, (unsigned)G * ++nbar, spin_limit)) return;
    if (open) {
      for (int i = blockIdx.x; i < ninst; i += G) open_top_body<real>(table[i], t, w, part);
      if (!grid_barrier(bar, (unsigned)G * ++nbar, spin_limit)) return;
    }
  }
}

}  // namespace lbm
