// Deterministic two-stage reduction with a last-block epilogue.
#pragma once
#include "eth_epilogue.h"
#include "eth_internal.h"

namespace eth {

// Called by every thread of a block after it computed its per-thread
// contributions `v[0..nvals)`.  Block `bid` (0..rc.nblocks) of right-hand
// side `rhs` stores its partial sums; the last block to arrive sums all
// partials in block order, stores the totals and runs the epilogue.
template <int NT>
__device__ inline void reduce_and_finish(const RedCtx& rc, int rhs, int bid, double* v,
                                         double* sh) {
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  __shared__ int s_last;
  for (int k = 0; k < rc.nvals; ++k) {
    double t = block_sum<NT>(v[k], sh);
    if (tid == 0)
      __hip_atomic_store(&rc.partials[((long long)rhs * rc.nvals + k) * rc.nblocks + bid], t,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (tid == 0) {
    __threadfence();
    unsigned t = atomicAdd(&rc.tickets[rhs], 1u);
    s_last = (t == (unsigned)(rc.nblocks - 1));
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  double tot[kMaxRedVals];
  for (int k = 0; k < rc.nvals; ++k) {
    const double* p = rc.partials + ((long long)rhs * rc.nvals + k) * rc.nblocks;
    double a = 0.0;
    for (int i = tid; i < rc.nblocks; i += NT)
      a += __hip_atomic_load(&p[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tot[k] = block_sum<NT>(a, sh);
  }
  if (tid == 0) {
    rc.tickets[rhs] = 0u;
    if (rc.result)
      for (int k = 0; k < rc.nvals; ++k) rc.result[(long long)rhs * rc.nvals + k] = tot[k];
    if (rc.epi) run_epilogue(rc.epi, rc.epi_state, rhs, tot);
    __threadfence();
  }
}

}  // namespace eth
