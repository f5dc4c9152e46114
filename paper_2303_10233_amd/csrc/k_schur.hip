// Pressure-mass solve by elimination of the P0 block (Sec. 2.3: Q_0 = h^2 I
// is diagonal):  M_Q = [Q_k R^T; R Q_0] gives
//     z_k = S_k^+ (r_k - R^T Q_0^{-1} r_0),   z_0 = Q_0^{-1} (r_0 - R z_k),
// S_k = Q_k - R^T Q_0^{-1} R, a Q1 operator with null space the constants.
// On a uniform mesh R^T Q_0^{-1} R has the element-local form (h^2/16) 1 1^T,
// so S_k x at Q1 node (c, d) is a 3x3 stencil with tensor weights
//     h^2 ( wx wy / 36 - ux uy / 16 ),  wx = [l, 2(l + r), r], ux = [l, l + r, r]
// (l, r: 1 if the element on that side exists), h^2 * 7/144 per adjacent
// element on the diagonal.  The multigrid for S_k uses the same stencil
// with the finest h on every level (S_k behaves like h^2 times a Laplacian,
// so this matches the Galerkin coarse operator on smooth modes).
#include "eth_kernels.h"

namespace eth {
namespace {

// (S x)(c, d) / h2 on Q1 vectors of one level (global loads of the 3x3 block)
template <typename T>
__device__ __forceinline__ double sk_row(const T* x, int c, int d, int n) {
  const int lx = (c > 0), rx = (c < n), ly = (d > 0), ry = (d < n);
  const double wx[3] = {(double)lx, 2.0 * (lx + rx), (double)rx};
  const double wy[3] = {(double)ly, 2.0 * (ly + ry), (double)ry};
  const double ux[3] = {(double)lx, (double)(lx + rx), (double)rx};
  const double uy[3] = {(double)ly, (double)(ly + ry), (double)ry};
  double v[3][3];
#pragma unroll
  for (int bb = 0; bb < 3; ++bb)
#pragma unroll
    for (int aa = 0; aa < 3; ++aa) {
      const int cc = c + aa - 1, dd = d + bb - 1;
      v[bb][aa] = (cc >= 0 && cc <= n && dd >= 0 && dd <= n) ? (double)x[(long long)dd * (n + 1) + cc] : 0.0;
    }
  double acc = 0.0;
#pragma unroll
  for (int bb = 0; bb < 3; ++bb)
#pragma unroll
    for (int aa = 0; aa < 3; ++aa)
      acc += (wx[aa] * wy[bb] * (1.0 / 36.0) - ux[aa] * uy[bb] * (1.0 / 16.0)) * v[bb][aa];
  return acc;
}

__device__ __forceinline__ double sk_diag(int c, int d, int n) {
  return (double)(((c > 0) + (c < n)) * ((d > 0) + (d < n))) * (7.0 / 144.0);
}

// MODE 0: out = S x;  1: Chebyshev-Jacobi step over out (has_prev 0: from
// the given x ignoring out, 1: out holds x_prev, 2: x_prev = 0);  2: out = b - S x
template <typename T, int MODE>
__global__ void k_sk_op(Geo g, double h2, const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ out,
                        double alpha, double beta, int has_prev, Gate gate) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  if (k >= g.nk) return;
  const int n = g.n, c = k % (n + 1), d = k / (n + 1);
  const T* xr = x + (long long)rhs * g.nk;
  const long long o = (long long)rhs * g.nk + k;
  const double sx = h2 * sk_row(xr, c, d, n);
  if constexpr (MODE == 0) {
    out[o] = (T)sx;
  } else if constexpr (MODE == 2) {
    out[o] = (T)((double)b[o] - sx);
  } else {
    const double xc = (double)xr[k];
    double xn = xc + beta * ((double)b[o] - sx) / (h2 * sk_diag(c, d, n));
    if (has_prev == 1) xn += alpha * (xc - (double)out[o]);
    else if (has_prev == 2) xn += alpha * xc;
    out[o] = (T)xn;
  }
}

__global__ void k_sk_diag_inv(Geo g, double h2, double* __restrict__ dinv) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.nk) return;
  const int n = g.n;
  dinv[k] = 1.0 / (h2 * sk_diag(k % (n + 1), k / (n + 1), n));
}

// b_k = r_k - R^T Q_0^{-1} r_0 (r: projected pressure vectors [rhs][n_k + n_0]); x = 0
template <typename T>
__global__ void k_schur_rhs(Geo g, const T* __restrict__ r, T* __restrict__ bq, T* __restrict__ xq, Gate gate) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  if (k >= g.nk) return;
  const int n = g.n, c = k % (n + 1), d = k / (n + 1);
  const long long np = (long long)g.nk + g.n0;
  const T* rr = r + (long long)rhs * np;
  double s = 0.0;
#pragma unroll
  for (int eb = -1; eb <= 0; ++eb)
#pragma unroll
    for (int ea = -1; ea <= 0; ++ea) {
      const int e = c + ea, f = d + eb;
      if (e >= 0 && e < n && f >= 0 && f < n) s += (double)rr[g.nk + (long long)f * n + e];
    }
  bq[(long long)rhs * g.nk + k] = (T)((double)rr[k] - 0.25 * s);
  xq[(long long)rhs * g.nk + k] = T(0);
}

// z = [z_k; Q_0^{-1}(r_0 - R z_k)] into pressure vectors [rhs][n_k + n_0]
template <typename T>
__global__ void k_schur_p0(Geo g, const T* __restrict__ r, const T* __restrict__ zk, T* __restrict__ z,
                           Gate gate) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  const long long np = (long long)g.nk + g.n0;
  if (i >= np) return;
  const T* zr = zk + (long long)rhs * g.nk;
  T* out = z + (long long)rhs * np;
  if (i < g.nk) {
    out[i] = zr[i];
    return;
  }
  const int n = g.n;
  const int e = (int)(i - g.nk) % n, f = (int)(i - g.nk) / n;
  const long long q = (long long)f * (n + 1) + e;
  const double s = (double)zr[q] + (double)zr[q + 1] + (double)zr[q + n + 1] + (double)zr[q + n + 2];
  out[i] = (T)((double)r[(long long)rhs * np + i] / (g.h * g.h) - 0.25 * s);
}

inline unsigned nb(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <typename T>
void launch_sk_op(const Geo& g, double h2, int mode, const T* b, const T* x, T* out, double alpha, double beta,
                  int has_prev, int batch, Gate gate, hipStream_t st) {
  const dim3 grid(nb(g.nk), batch);
  if (mode == 0)
    hipLaunchKernelGGL((k_sk_op<T, 0>), grid, dim3(256), 0, st, g, h2, b, x, out, alpha, beta, has_prev, gate);
  else if (mode == 1)
    hipLaunchKernelGGL((k_sk_op<T, 1>), grid, dim3(256), 0, st, g, h2, b, x, out, alpha, beta, has_prev, gate);
  else
    hipLaunchKernelGGL((k_sk_op<T, 2>), grid, dim3(256), 0, st, g, h2, b, x, out, alpha, beta, has_prev, gate);
  ETH_LAUNCH_CHECK();
}

void launch_sk_diag_inv(const Geo& g, double h2, double* dinv, hipStream_t st) {
  hipLaunchKernelGGL(k_sk_diag_inv, dim3(nb(g.nk)), dim3(256), 0, st, g, h2, dinv);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_schur_rhs(const Geo& g, const T* r, T* bq, T* xq, int batch, Gate gate, hipStream_t st) {
  hipLaunchKernelGGL(k_schur_rhs<T>, dim3(nb(g.nk), batch), dim3(256), 0, st, g, r, bq, xq, gate);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_schur_p0(const Geo& g, const T* r, const T* zk, T* z, int batch, Gate gate, hipStream_t st) {
  hipLaunchKernelGGL(k_schur_p0<T>, dim3(nb((long long)g.nk + g.n0), batch), dim3(256), 0, st, g, r, zk, z,
                     gate);
  ETH_LAUNCH_CHECK();
}

#define ETH_INST(T)                                                                                   \
  template void launch_sk_op<T>(const Geo&, double, int, const T*, const T*, T*, double, double, int, \
                                int, Gate, hipStream_t);                                              \
  template void launch_schur_rhs<T>(const Geo&, const T*, T*, T*, int, Gate, hipStream_t);            \
  template void launch_schur_p0<T>(const Geo&, const T*, const T*, T*, int, Gate, hipStream_t);
ETH_INST(double)
ETH_INST(float)
#undef ETH_INST

}  // namespace eth
