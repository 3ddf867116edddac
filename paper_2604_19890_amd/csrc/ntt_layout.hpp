// Thread and LDS layout shared by the transform kernels (ntt.hip) and the key-switching
// kernels built on the same passes (keyswitch.hip).
#pragma once
#include "ctx.hpp"

namespace nttl {

constexpr int NT_MAX = 256;

__device__ __forceinline__ int lds_idx(int sl, int k, int S) { return sl * (S + (S >> 4) + 1) + k + (k >> 4); }

// Ordering point for an LDS exchange among the lanes of one wavefront.  The LDS
// instructions of a wave are performed in issue order, so it suffices to keep
// the compiler from moving LDS accesses across this point; no s_barrier is
// issued and the other waves of the block run on.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS exchange point of a pass.  In a contiguous pass (tmin = 1) the T <= 16
// threads of a sub-transform are consecutive lanes of one wave (T divides 64)
// and each sub-transform has LDS rows of its own, so the exchange stays inside
// the wave; a column pass spreads a sub-transform over the block's waves.
__device__ __forceinline__ void pass_sync(bool wave_local) {
  if (wave_local)
    wave_lds_sync();
  else
    __syncthreads();
}

}  // namespace nttl
