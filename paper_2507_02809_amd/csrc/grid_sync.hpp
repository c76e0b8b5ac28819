// The device-wide barrier of the persistent dense-transform block solvers (the P^{-1} segment kernel
// synchronises through its reduction slots instead: phase_sync in pinv_kernel.hpp).
// Every workgroup of such a grid must be resident at once: the launchers take the grid's CU slots
// from the per-device pool first (residency.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include "residency.hpp"

namespace tsfde {

// the device's pool of CU slots for persistent grids, and the longest barrier wait in wall-clock
// periods (pinv_persistent.hip)
ResidencyBudget& residency_budget(int dev, int ncu);
unsigned long long barrier_ticks(int dev);

// Device-wide barrier: arrive on a counter, wait until all blocks of this epoch arrived.  The
// release increment and the acquire fence after the wait (both at agent scope) make every block's
// earlier writes visible to every block; the wait itself polls with relaxed loads, so that the
// cache invalidation of the acquire happens once per barrier rather than once per poll.
//
// The wait is bounded.  bar[0] is the arrival counter and bar[1] an abort word: a block that has
// waited longer than `ticks` periods of the constant wall clock sets the abort word, and from then
// on every barrier of the launch (and of the later segment launches of the same P^-1, which keep
// the word) returns at once.  The grid then runs its remaining, bounded loops on meaningless
// values and exits normally; the host finds the word set and reports an error.  A wait can only
// last that long when the grid's workgroups are not all resident at once.
// nb: the workgroups that meet at this barrier (the launch's grid, or one problem's share of it).
__device__ __forceinline__ void grid_barrier_n(unsigned* bar, unsigned long long ticks, unsigned& epoch, int nb) {
    __syncthreads();
    if (nb > 1) {
        epoch += (unsigned)nb;
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                const unsigned long long t0 = (unsigned long long)wall_clock64();
                while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
                    if (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
                    if ((unsigned long long)wall_clock64() - t0 > ticks) {
                        __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned long long ticks, unsigned& epoch) {
    grid_barrier_n(bar, ticks, epoch, (int)gridDim.x);
}

}  // namespace tsfde
