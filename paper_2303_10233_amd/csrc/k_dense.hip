// Dense inverse of the coarsest-level operator of a multigrid (FP64), built
// on the GPU whenever the operator changes (the wind of an Oseen problem).
//
// In-place blocked Gauss-Jordan elimination without pivoting, which needs
// every leading principal block to be nonsingular: true for the positive-real
// coarse convection-diffusion matrices (F + F^T positive definite, so every
// principal submatrix and every Schur complement is positive real).  With
// pivot block P (rows and columns p0 .. p0 + pb - 1) and Pi = A_PP^{-1}, one
// step replaces
//     A_ij  by  A_ij - A_iP Pi A_Pj     (i, j outside P)
//     A_Pj  by  Pi A_Pj,   A_iP  by  -A_iP Pi,   A_PP  by  Pi,
// and after the last block A holds A^{-1}.  The pivot order is the natural
// one, as in unblocked Gauss-Jordan; the blocking only regroups the updates
// into rank-64 products, so one pass over the matrix per 64 pivots.
#include "eth_kernels.h"

namespace eth {
namespace {

constexpr int BK = 64;     // pivot block and tile side

// Pi = A_PP^{-1} by unblocked Gauss-Jordan on [A_PP | I] in LDS (one block;
// 1024 threads, so that the LDS latency of the 64 dependent steps hides)
constexpr int PT = 1024;
__global__ __launch_bounds__(PT) void k_bgj_pivot(const double* __restrict__ A, int ni, int p0, int pb,
                                                  double* __restrict__ Pi) {
  __shared__ double M[BK][2 * BK + 1];
  __shared__ double fac[BK];
  const int tid = threadIdx.x;
  for (int k = tid; k < BK * 2 * BK; k += PT) {
    const int r = k / (2 * BK), c = k % (2 * BK);
    double v = 0.0;
    if (r < pb && c < pb) v = A[(long long)(p0 + r) * ni + p0 + c];
    else if (r < pb && c == BK + r) v = 1.0;
    M[r][c] = v;
  }
  __syncthreads();
  for (int k = 0; k < pb; ++k) {
    const double piv = M[k][k];
    __syncthreads();
    if (tid < 2 * BK) M[k][tid] /= piv;
    else if (tid < 3 * BK) fac[tid - 2 * BK] = M[tid - 2 * BK][k];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < BK * 2 * BK / PT; ++q) {
      const int e = tid + q * PT, r = e / (2 * BK), c = e % (2 * BK);
      if (r != k && r < pb) M[r][c] -= fac[r] * M[k][c];
    }
    __syncthreads();
  }
  for (int e = tid; e < BK * BK; e += PT) {
    const int r = e / BK, c = e % BK;
    Pi[e] = (r < pb && c < pb) ? M[r][BK + c] : 0.0;
  }
}

// R = Pi A_P,: (BK x ni, rows >= pb zero) and C = A_:,P (ni x BK, columns >= pb zero)
__global__ __launch_bounds__(256) void k_bgj_panel(const double* __restrict__ A, int ni, int p0, int pb,
                                                   const double* __restrict__ Pi, double* __restrict__ R,
                                                   double* __restrict__ C, int row_blocks) {
  __shared__ double Ps[BK][BK + 1];
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < row_blocks) {
    for (int e = tid; e < BK * BK; e += 256) Ps[e / BK][e % BK] = Pi[e];
    __syncthreads();
    const int j = blockIdx.x * 256 + tid;
    if (j >= ni) return;
    double a[BK];
#pragma unroll
    for (int m = 0; m < BK; ++m) a[m] = m < pb ? A[(long long)(p0 + m) * ni + j] : 0.0;
    for (int k = 0; k < BK; ++k) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < BK; ++m) acc += Ps[k][m] * a[m];
      R[(long long)k * ni + j] = acc;
    }
    return;
  }
  const long long e = (long long)(blockIdx.x - row_blocks) * 256 + tid;
  if (e >= (long long)ni * BK) return;
  const int i = (int)(e / BK), k = (int)(e % BK);
  C[e] = k < pb ? A[(long long)i * ni + p0 + k] : 0.0;
}

// every 64 x 64 tile of A: the rank-pb update, or the row / column / pivot
// block replacement (tiles are aligned with the pivot block).  A thread owns
// a 4 x 4 block of the tile; both operands are read from LDS as 16-byte pairs.
constexpr int LDP = BK + 2;   // padded LDS row (keeps 16-byte alignment)
__global__ __launch_bounds__(256) void k_bgj_update(double* __restrict__ A, int ni, int p0,
                                                    const double* __restrict__ Pi,
                                                    const double* __restrict__ R,
                                                    const double* __restrict__ C) {
  __shared__ __align__(16) double Ct[BK][LDP];   // [k][row of the tile]
  __shared__ __align__(16) double Rs[BK][LDP];   // [k][column of the tile]
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.y * BK, j0 = blockIdx.x * BK;
  const bool prow = i0 == p0, pcol = j0 == p0;
  for (int e = tid; e < BK * BK; e += 256) {
    const int k = e / BK, c = e % BK, j = j0 + c;
    Rs[k][c] = pcol ? Pi[k * BK + c] : (j < ni ? R[(long long)k * ni + j] : 0.0);
  }
  if (!prow)
    for (int e = tid; e < BK * BK; e += 256) {
      const int r = e / BK, k = e % BK, i = i0 + r;
      Ct[k][r] = i < ni ? C[(long long)i * BK + k] : 0.0;
    }
  __syncthreads();
  const int r0 = ty * 4, c0 = tx * 4;
  if (prow) {
    for (int a = 0; a < 4; ++a) {
      const int i = i0 + r0 + a;
      if (i >= ni) break;
      for (int b = 0; b < 4; ++b) {
        const int j = j0 + c0 + b;
        if (j < ni) A[(long long)i * ni + j] = Rs[r0 + a][c0 + b];
      }
    }
    return;
  }
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 4
  for (int k = 0; k < BK; ++k) {
    const double2 ca = *reinterpret_cast<const double2*>(&Ct[k][r0]);
    const double2 cb = *reinterpret_cast<const double2*>(&Ct[k][r0 + 2]);
    const double2 ra = *reinterpret_cast<const double2*>(&Rs[k][c0]);
    const double2 rb = *reinterpret_cast<const double2*>(&Rs[k][c0 + 2]);
    const double cv[4] = {ca.x, ca.y, cb.x, cb.y}, rv[4] = {ra.x, ra.y, rb.x, rb.y};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += cv[a] * rv[b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + r0 + a;
    if (i >= ni) break;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + c0 + b;
      if (j >= ni) continue;
      const long long o = (long long)i * ni + j;
      A[o] = pcol ? -acc[a][b] : A[o] - acc[a][b];
    }
  }
}

// at = a^T through 64 x 64 LDS tiles (coalesced reads and writes)
__global__ __launch_bounds__(256) void k_transpose_tiled(const double* __restrict__ a, int ni,
                                                         double* __restrict__ at) {
  __shared__ double t[BK][BK + 1];
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  const int i0 = blockIdx.y * BK, j0 = blockIdx.x * BK;
  for (int r = ty; r < BK; r += 4) {
    const int i = i0 + r, j = j0 + tx;
    if (i < ni && j < ni) t[r][tx] = a[(long long)i * ni + j];
  }
  __syncthreads();
  for (int r = ty; r < BK; r += 4) {
    const int i = j0 + r, j = i0 + tx;   // at[i][j] = a[j][i]
    if (i < ni && j < ni) at[(long long)i * ni + j] = t[tx][r];
  }
}

__global__ void k_symmetrize(double* __restrict__ A, int ni) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)ni * ni) return;
  const int i = (int)(t / ni), j = (int)(t % ni);
  if (j <= i) return;   // each pair once, by the thread of its upper entry
  const long long o = (long long)j * ni + i;
  const double v = 0.5 * (A[t] + A[o]);
  A[t] = v;
  A[o] = v;
}

__global__ void k_to_float(const double* __restrict__ a, float* __restrict__ f, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = (float)a[i];
}

}  // namespace

void launch_to_float(const double* a, float* f, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_float, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, f, n);
  ETH_LAUNCH_CHECK();
}

void launch_symmetrize(double* A, int ni, hipStream_t st) {
  const long long n = (long long)ni * ni;
  hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, ni);
  ETH_LAUNCH_CHECK();
}

size_t dense_inverse_work(int ni) { return (size_t)BK * BK + 2 * (size_t)BK * ni; }

void launch_dense_inverse(double* A, int ni, double* work, hipStream_t st) {
  double* Pi = work;
  double* R = Pi + BK * BK;
  double* C = R + (size_t)BK * ni;
  const int tiles = (ni + BK - 1) / BK;
  const int row_blocks = (ni + 255) / 256;
  const int c_blocks = (int)(((long long)ni * BK + 255) / 256);
  for (int p0 = 0; p0 < ni; p0 += BK) {
    const int pb = ni - p0 < BK ? ni - p0 : BK;
    hipLaunchKernelGGL(k_bgj_pivot, dim3(1), dim3(PT), 0, st, A, ni, p0, pb, Pi);
    ETH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bgj_panel, dim3(row_blocks + c_blocks), dim3(256), 0, st, A, ni, p0, pb, Pi, R, C,
                       row_blocks);
    ETH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bgj_update, dim3(tiles, tiles), dim3(256), 0, st, A, ni, p0, Pi, R, C);
    ETH_LAUNCH_CHECK();
  }
}

void launch_transpose(const double* a, int ni, double* at, hipStream_t st) {
  const int tiles = (ni + BK - 1) / BK;
  hipLaunchKernelGGL(k_transpose_tiled, dim3(tiles, tiles), dim3(256), 0, st, a, ni, at);
  ETH_LAUNCH_CHECK();
}

}  // namespace eth
