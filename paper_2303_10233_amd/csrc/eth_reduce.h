// Deterministic two-stage reductions.  Every block of a reducing kernel
// stores its block sums; the totals are formed in a fixed order by a small
// second kernel (launch_reduce_finish, k_vector.hip) that also runs the
// epilogue.  A kernel boundary orders the partial sums before their use, so
// no block waits on another and no device-wide fence is taken per block
// (a last-block ticket costs a serialised release of the L2 per block).
// With a single block per right-hand side that block finishes by itself.
#pragma once
#include "eth_epilogue.h"
#include "eth_internal.h"

namespace eth {

// Called by every thread of a block after it computed its per-thread
// contributions `v[0..nvals)`; `bid` in [0, rc.nblocks).
template <int NT>
__device__ inline void reduce_and_finish(const RedCtx& rc, int rhs, int bid, double* v, double* sh) {
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  double tot[kMaxRedVals];
  for (int k = 0; k < rc.nvals; ++k) {
    tot[k] = block_sum<NT>(v[k], sh);
    if (tid == 0 && rc.nblocks > 1) rc.partials[((long long)rhs * rc.nvals + k) * rc.nblocks + bid] = tot[k];
  }
  if (rc.nblocks == 1 && tid == 0) {
    if (rc.result)
      for (int k = 0; k < rc.nvals; ++k) rc.result[(long long)rhs * rc.nvals + k] = tot[k];
    if (rc.epi) run_epilogue(rc.epi, rc.epi_state, rhs, tot);
  }
}

}  // namespace eth
