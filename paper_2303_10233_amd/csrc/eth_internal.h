// Internal declarations shared by the HIP translation units of libeth.
// gfx950 (CDNA4): 64-wide wavefronts; all reductions are deterministic
// (fixed shuffle tree within a wave, fixed order across waves and blocks).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <cstdlib>
#include <string>

namespace eth {

// ----------------------------------------------------------------------------
// Geometry of one mesh level.  Layout of a full vector:
//   [u_x (nq*nq) | u_y (nq*nq) | p_k (n+1)^2 | p_0 n^2],  nq = 2n+1.
// ----------------------------------------------------------------------------
struct Geo {
  int n;       // elements per side
  int nq;      // 2n+1 Q2 nodes per side
  int nv;      // nq*nq
  int nk;      // (n+1)^2
  int n0;      // n*n
  long long N; // 2 nv + nk + n0
  double h;    // element side
  __host__ __device__ long long off_uy() const { return nv; }
  __host__ __device__ long long off_pk() const { return 2LL * nv; }
  __host__ __device__ long long off_p0() const { return 2LL * nv + nk; }
};

inline Geo make_geo(int n, double h) {
  Geo g;
  g.n = n;
  g.nq = 2 * n + 1;
  g.nv = g.nq * g.nq;
  g.nk = (n + 1) * (n + 1);
  g.n0 = n * n;
  g.N = 2LL * g.nv + g.nk + g.n0;
  g.h = h;
  return g;
}

constexpr int kWave = 64;

// message of the last failing call made without a handle (eth_setup and the
// handle-free entry points); read by eth_last_error(NULL)
extern thread_local std::string g_setup_error;

// ----------------------------------------------------------------------------
// XCD band order.  The eight XCDs take a grid's workgroups round-robin, each
// with its own L2; a tiled stencil kernel whose vertically neighbouring tiles
// share halo rows then fetches those rows once per XCD.  Grids of at least
// `remap_min` tiles are renumbered so that XCD j (workgroups j, j+8, ...) takes
// the j-th contiguous band of tiles in row-major order; smaller grids keep the
// plain order.  The threshold comes from the host (xcd_remap_min), where
// ETH_DEBUG_XCD_REMAP_MIN can force it down for tests.
// ----------------------------------------------------------------------------
constexpr int kXcdRemapMin = 2048;
inline int xcd_remap_min() {
  const char* e = std::getenv("ETH_DEBUG_XCD_REMAP_MIN");
  return e ? std::atoi(e) : kXcdRemapMin;
}
__device__ __forceinline__ void xcd_band_tile(int remap_min, int& tile_x, int& tile_y) {
  tile_x = blockIdx.x;
  tile_y = blockIdx.y;
  const int T = gridDim.x * gridDim.y;
  if (T < remap_min) return;
  const int old_id = blockIdx.x + gridDim.x * blockIdx.y;
  const int q = T / 8, r = T % 8, j = old_id % 8, m = old_id / 8;
  const int nid = j * q + (j < r ? j : r) + m;
  tile_x = nid % gridDim.x;
  tile_y = nid / gridDim.x;
}

// ----------------------------------------------------------------------------
// Deterministic reductions
// ----------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum over a block of NT threads (NT multiple of 64).  Result valid in every
// thread.  `sh` must hold NT/64 doubles.
template <int NT>
__device__ inline double block_sum(double v, double* sh) {
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  v = wave_sum(v);
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += sh[i];
  __syncthreads();
  return t;
}

// ----------------------------------------------------------------------------
// Staging of a tile into LDS with every global load issued before the first
// LDS store: a grid-stride loop that loads and stores per iteration waits for
// each load in turn, and at a few hundred nanoseconds per L2/HBM round trip
// that serial chain dominates the small kernels.  load(k, a, b) fills the two
// values of staged entry k (0 <= k < COUNT).
// ----------------------------------------------------------------------------
template <int NT, int COUNT, typename T, typename Load>
__device__ __forceinline__ void stage2(T* __restrict__ d0, T* __restrict__ d1, int tid, Load load) {
  constexpr int IT = (COUNT + NT - 1) / NT;
  T a[IT], b[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int k = tid + i * NT;
    a[i] = T(0);
    b[i] = T(0);
    if (k < COUNT) load(k, a[i], b[i]);
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int k = tid + i * NT;
    if (k < COUNT) {
      d0[k] = a[i];
      d1[k] = b[i];
    }
  }
}

template <int NT, int COUNT, typename T, typename Load>
__device__ __forceinline__ void stage1(T* __restrict__ d0, int tid, Load load) {
  constexpr int IT = (COUNT + NT - 1) / NT;
  T a[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int k = tid + i * NT;
    a[i] = T(0);
    if (k < COUNT) load(k, a[i]);
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int k = tid + i * NT;
    if (k < COUNT) d0[k] = a[i];
  }
}

// Reduction context: every block of right-hand side `rhs` writes one partial
// (or `nvals` partials); a second kernel sums them in block order and hands
// the totals to an epilogue (eth_reduce.h).
constexpr int kMaxRedVals = 4;
struct RedCtx {
  double* partials;    // [batch][nvals][nblocks]
  double* result;      // [batch][nvals] totals (may be null)
  int nblocks;         // blocks per right-hand side
  int nvals;           // values reduced per block (<= kMaxRedVals)
  int epi;             // epilogue id (eth_epilogue.h), 0 = none
  void* epi_state;     // epilogue state array
  int defer;           // 1: no finishing launch; the consuming kernel sums the partials
};

// ----------------------------------------------------------------------------
// Error handling helpers (host)
// ----------------------------------------------------------------------------
struct HipError {
  hipError_t err;
  std::string where;
};

#define ETH_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) throw ::eth::HipError{e_, std::string(#call)};       \
  } while (0)

#define ETH_LAUNCH_CHECK() ETH_HIP(hipGetLastError())

}  // namespace eth
