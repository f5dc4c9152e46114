// Restarted flexible GMRES with right preconditioning (Sec. 3: GMRES for the
// Oseen system, monitored by the Euclidean residual of eq:residual-norm).
// Arnoldi uses classical Gram-Schmidt applied twice (CGS2); the Hessenberg
// Givens rotations, the residual estimate and the convergence test run on
// the device in the last block of the norm reduction.  FP64 throughout.
//
// Basis layout: V[i] for right-hand side r at V + (i * batch + r) * ld,
// likewise Z.  Per right-hand side a GmresScalars record (eth_kernels.h).
#include "eth_kernels.h"
#include "eth_reduce.h"

namespace eth {
namespace {

constexpr int NT = 256;
constexpr int CH = 16;         // basis vectors per pass of the multi-dot

__device__ inline const double* vec(const double* base, int i, int batch, int rhs, long long ld) {
  return base + ((long long)i * batch + rhs) * ld;
}

// h_i = <v_i, w> for i = 0..nv-1: block partials P[i * nb + block].  A pass
// takes CH basis vectors against one read of w; the CH sums of a pass are
// reduced per wavefront by shuffles, then across the block's wavefronts in
// wavefront order behind one barrier (the order block_sum uses, so the
// partials are the same bits as one block_sum per vector).  Measured at
// n = 2048 with 26 vectors: 2255 us (8 per pass, a barrier pair per vector),
// 2166 us (this form), 3014 us (32 per pass: register pressure).
__global__ __launch_bounds__(NT) void k_gm_mdot(long long N, int nv, const double* __restrict__ V,
                                                const double* __restrict__ w, long long ld, int batch,
                                                double* __restrict__ partials,
                                                const GmresScalars* __restrict__ S) {
  __shared__ double sred[NT / 64][CH];
  const int rhs = blockIdx.y;
  if (!S[rhs].active) return;
  const double* wr = w + (long long)rhs * ld;
  const int nb = gridDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* P = partials + (long long)rhs * 64 * nb;
  for (int i0 = 0; i0 < nv; i0 += CH) {
    double acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = 0.0;
    for (long long k = (long long)blockIdx.x * NT + threadIdx.x; k < N; k += (long long)nb * NT) {
      const double wk = wr[k];
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (i0 + c < nv) acc[c] += vec(V, i0 + c, batch, rhs, ld)[k] * wk;
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (i0 + c >= nv) break;
      const double t = wave_sum(acc[c]);
      if (lane == 0) sred[wave][c] = t;
    }
    __syncthreads();
    if (threadIdx.x < CH && i0 + (int)threadIdx.x < nv) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) t += sred[q][threadIdx.x];
      P[(long long)(i0 + threadIdx.x) * nb + blockIdx.x] = t;
    }
    __syncthreads();
  }
}

// the multi-dot totals in block order, one single-wave block per coefficient
// (all coefficients in parallel)
__global__ __launch_bounds__(64) void k_gm_mdot_finish(int nb, const double* __restrict__ partials,
                                                       GmresScalars* __restrict__ S, int which) {
  const int i = blockIdx.x, rhs = blockIdx.y;
  if (!S[rhs].active) return;
  const double* P = partials + (long long)rhs * 64 * nb;
  double* out = which == 0 ? S[rhs].h1 : S[rhs].h2;
  const int lane = threadIdx.x;
  double a = 0.0;
  for (int b = lane; b < nb; b += 64) a += P[(long long)i * nb + b];
  a = wave_sum(a);
  if (lane == 0) out[i] = a;
}

// block partials of ||w||^2; mode 0: RHS whose Arnoldi step runs, mode 1:
// RHS not yet converged (restart)
__global__ __launch_bounds__(NT) void k_gm_sumsq(long long N, const double* __restrict__ w, long long ld,
                                                 double* __restrict__ partials,
                                                 const GmresScalars* __restrict__ S, int mode) {
  __shared__ double sred[NT / 64];
  const int rhs = blockIdx.y;
  const GmresScalars& G = S[rhs];
  if (mode == 0 ? !G.active : (G.converged || G.status < 0)) return;
  const double* wr = w + (long long)rhs * ld;
  const int nb = gridDim.x;
  double a = 0.0;
  for (long long k = (long long)blockIdx.x * NT + threadIdx.x; k < N; k += (long long)nb * NT)
    a += wr[k] * wr[k];
  const double t = block_sum<NT>(a, sred);
  if (threadIdx.x == 0) partials[(long long)rhs * 64 * nb + blockIdx.x] = t;
}

__device__ inline double sum_partials(const double* __restrict__ P, int nb, double* sred) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += NT) s += P[b];
  return block_sum<NT>(s, sred);
}

// w -= sum_{i<nv} c_i v_i   (c = h1 or h2 of the record)
__global__ void k_gm_maxpy(long long N, int nv, const double* __restrict__ V, double* __restrict__ w,
                           long long ld, int batch, const GmresScalars* __restrict__ S, int which) {
  __shared__ double sc[64];
  const int rhs = blockIdx.y;
  if (!S[rhs].active) return;
  const double* c = which == 0 ? S[rhs].h1 : S[rhs].h2;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) sc[i] = c[i];
  __syncthreads();
  double* wr = w + (long long)rhs * ld;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < N;
       k += (long long)gridDim.x * blockDim.x) {
    double a = wr[k];
    for (int i = 0; i < nv; ++i) a -= sc[i] * vec(V, i, batch, rhs, ld)[k];
    wr[k] = a;
  }
}

// ||w||^2 from the partials, then the Givens step for column j of the
// Hessenberg matrix
__global__ __launch_bounds__(NT) void k_gm_givens(int j, int nb, const double* __restrict__ partials,
                                                  GmresScalars* __restrict__ S) {
  __shared__ double sred[NT / 64];
  __shared__ double hc[66], lcs[64], lsn[64];
  const int rhs = blockIdx.x;
  GmresScalars& G = S[rhs];
  if (!G.active) return;
  const double s = sum_partials(partials + (long long)rhs * 64 * nb, nb, sred);
  // the new Hessenberg column and the earlier rotations are read in parallel;
  // the rotation recurrence then runs on LDS values
  const int m1 = G.m + 1;
  double* Hc = G.H + (long long)j * m1;
  for (int i = threadIdx.x; i <= j; i += NT) hc[i] = G.h1[i] + G.h2[i];
  for (int i = threadIdx.x; i < j; i += NT) {
    lcs[i] = G.cs[i];
    lsn[i] = G.sn[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double hn = sqrt(s);
    hc[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double t0 = lcs[i] * hc[i] + lsn[i] * hc[i + 1];
      hc[i + 1] = -lsn[i] * hc[i] + lcs[i] * hc[i + 1];
      hc[i] = t0;
    }
    const double r = hypot(hc[j], hc[j + 1]);
    double c = 1.0, sn = 0.0;
    if (r > 0.0) {
      c = hc[j] / r;
      sn = hc[j + 1] / r;
    }
    G.cs[j] = c;
    G.sn[j] = sn;
    hc[j] = r;
    hc[j + 1] = 0.0;
    G.g[j + 1] = -sn * G.g[j];
    G.g[j] = c * G.g[j];
    G.res = fabs(G.g[j + 1]);
    G.iters += 1;
    G.kend = j + 1;
    if (G.hist && G.iters < G.hist_len) G.hist[G.iters] = G.res;
    G.inv = hn > 0.0 ? 1.0 / hn : 0.0;
    if (!(G.res == G.res) || r == 0.0) {   // NaN or singular Hessenberg column
      G.status = kStBreakdown;
      G.active = 0;
    } else if (G.res <= G.target || hn == 0.0 || j == G.m - 1 || G.iters >= G.maxit) {
      G.active = 0;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += NT) Hc[i] = hc[i];
}

// V[i] *= inv  (the pending normalisation of the new Arnoldi vector)
__global__ void k_gm_scale(long long N, double* __restrict__ v, long long ld, const GmresScalars* __restrict__ S,
                           int beta_phase) {
  const int rhs = blockIdx.y;
  const GmresScalars& G = S[rhs];
  if (!G.active) return;
  (void)beta_phase;
  const double s = G.inv;
  double* vr = v + (long long)rhs * ld;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < N;
       k += (long long)gridDim.x * blockDim.x)
    vr[k] *= s;
}

// restart: beta = ||r_0|| -> g = [beta, 0, ...], convergence test, flags
__global__ __launch_bounds__(NT) void k_gm_beta(int nb, const double* __restrict__ partials,
                                                GmresScalars* __restrict__ S) {
  __shared__ double sred[NT / 64];
  const int rhs = blockIdx.x;
  GmresScalars& G = S[rhs];
  if (G.converged || G.status < 0) return;
  const double s = sum_partials(partials + (long long)rhs * 64 * nb, nb, sred);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(s);
  G.beta = beta;
  G.res = beta;
  if (G.iters == 0 && G.hist && G.hist_len > 0) G.hist[0] = beta;
  G.kend = 0;
  if (!(beta == beta)) {
    G.status = kStBreakdown;
    G.active = 0;
    G.update = 0;
  } else if (beta <= G.target) {
    G.converged = 1;
    G.active = 0;
    G.update = 0;
  } else if (G.iters >= G.maxit) {
    G.status = kStMaxit;
    G.active = 0;
    G.update = 0;
  } else {
    G.g[0] = beta;
    G.inv = 1.0 / beta;
    G.active = 1;
    G.update = 1;
  }
}

// y = H(0:k,0:k)^{-1} g(0:k) (upper triangular after the rotations)
__global__ void k_gm_solve_y(GmresScalars* __restrict__ S) {
  const int rhs = blockIdx.x;
  GmresScalars& G = S[rhs];
  if (!G.update || threadIdx.x != 0) return;
  const int k = G.kend, m1 = G.m + 1;
  for (int i = k - 1; i >= 0; --i) {
    double a = G.g[i];
    for (int l = i + 1; l < k; ++l) a -= G.H[(long long)l * m1 + i] * G.y[l];
    G.y[i] = a / G.H[(long long)i * m1 + i];
  }
}

// x += sum_{i<k} y_i z_i
__global__ void k_gm_xupdate(long long N, const double* __restrict__ Z, double* __restrict__ x,
                             long long ld, int batch, const GmresScalars* __restrict__ S) {
  __shared__ double sy[64];
  const int rhs = blockIdx.y;
  const GmresScalars& G = S[rhs];
  if (!G.update) return;
  const int k = G.kend;
  for (int i = threadIdx.x; i < k; i += blockDim.x) sy[i] = G.y[i];
  __syncthreads();
  double* xr = x + (long long)rhs * ld;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N;
       e += (long long)gridDim.x * blockDim.x) {
    double a = xr[e];
    for (int i = 0; i < k; ++i) a += sy[i] * vec(Z, i, batch, rhs, ld)[e];
    xr[e] = a;
  }
}

// x[off, off+count) = 0 on right-hand sides whose GMRES record is active
__global__ void k_gm_zero_range(double* __restrict__ x, long long ld, long long off, long long count,
                                const GmresScalars* __restrict__ S) {
  const int rhs = blockIdx.y;
  if (S && !S[rhs].active) return;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (long long)gridDim.x * blockDim.x)
    x[(long long)rhs * ld + off + k] = 0.0;
}

constexpr int kGmBlocksMax = 1024;   // partial sums per RHS: 64 * kGmBlocksMax

unsigned blocks(long long n) {
  long long b = (n + 1023) / 1024;
  return (unsigned)(b < 1 ? 1 : (b > kGmBlocksMax ? kGmBlocksMax : b));
}

}  // namespace

int gmres_blocks(long long N) { return (int)blocks(N); }

void launch_gm_mdot(long long N, int nv, const double* V, const double* w, long long ld, int batch,
                    double* partials, GmresScalars* S, int which, hipStream_t st) {
  const unsigned nb = blocks(N);
  hipLaunchKernelGGL(k_gm_mdot, dim3(nb, batch), dim3(NT), 0, st, N, nv, V, w, ld, batch, partials, S);
  ETH_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gm_mdot_finish, dim3(nv, batch), dim3(64), 0, st, (int)nb, partials, S, which);
  ETH_LAUNCH_CHECK();
}
void launch_gm_maxpy(long long N, int nv, const double* V, double* w, long long ld, int batch,
                     const GmresScalars* S, int which, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_maxpy, dim3(blocks(N), batch), dim3(256), 0, st, N, nv, V, w, ld, batch, S, which);
  ETH_LAUNCH_CHECK();
}
void launch_gm_norm_givens(long long N, int j, const double* w, long long ld, int batch, double* partials,
                           GmresScalars* S, hipStream_t st) {
  const unsigned nb = blocks(N);
  hipLaunchKernelGGL(k_gm_sumsq, dim3(nb, batch), dim3(NT), 0, st, N, w, ld, partials, S, 0);
  ETH_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gm_givens, dim3(batch), dim3(NT), 0, st, j, (int)nb, partials, S);
  ETH_LAUNCH_CHECK();
}
void launch_gm_scale(long long N, double* v, long long ld, int batch, const GmresScalars* S, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_scale, dim3(blocks(N), batch), dim3(256), 0, st, N, v, ld, S, 0);
  ETH_LAUNCH_CHECK();
}
void launch_gm_beta(long long N, const double* v, long long ld, int batch, double* partials, GmresScalars* S,
                    hipStream_t st) {
  const unsigned nb = blocks(N);
  hipLaunchKernelGGL(k_gm_sumsq, dim3(nb, batch), dim3(NT), 0, st, N, v, ld, partials, S, 1);
  ETH_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gm_beta, dim3(batch), dim3(NT), 0, st, (int)nb, partials, S);
  ETH_LAUNCH_CHECK();
}
void launch_gm_finish(long long N, const double* Z, double* x, long long ld, int batch, GmresScalars* S,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_gm_solve_y, dim3(batch), dim3(64), 0, st, S);
  ETH_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gm_xupdate, dim3(blocks(N), batch), dim3(256), 0, st, N, Z, x, ld, batch, S);
  ETH_LAUNCH_CHECK();
}
void launch_gm_zero_range(double* x, long long ld, long long off, long long count, int batch,
                          const GmresScalars* S, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_zero_range, dim3(blocks(count), batch), dim3(256), 0, st, x, ld, off, count, S);
  ETH_LAUNCH_CHECK();
}

}  // namespace eth
