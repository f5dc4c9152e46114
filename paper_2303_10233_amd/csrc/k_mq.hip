// Pressure-mass solves for the frame Q1 + P0 (Sec. 2.2-2.3).
//
// M_Q = [[Q_k, R^T], [R, Q_0]] on a uniform mesh of square elements:
//   Q_k = Mp (x) Mp with the 1-D Q1 mass rows (h/6)[1, 2*(#elements), 1],
//   R_{T,a} = h^2/4 for the four vertices a of element T,  Q_0 = h^2 I.
// diag(M_Q): (h^2/36) * 2m_x * 2m_y at a Q1 node touching m_x (m_y) element
// columns (rows), h^2 at an element.  The frame null vector is k = [1; -1].
//
// Solves are the bordered systems [[M_S, k], [k^T, 0]] of Sec. 2.2:
//  * M_S = diag(M_Q): z = D^{-1}(r - lam k), lam = k^T D^{-1} r / k^T D^{-1} k;
//  * M_S from Chebyshev semi-iteration based on symmetric Gauss-Seidel
//    (Sec. 2.3): the input is projected onto k^perp, `steps` Chebyshev steps
//    each take one symmetric multicolour sweep (colours: the four parity
//    classes of Q1 nodes, then all elements; forward 0..4, backward 3..0),
//    and the output is projected onto k^perp.
#include "eth_kernels.h"
#include "eth_reduce.h"

namespace eth {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ double mq_diag(const Geo& g, long long i) {
  const double h2 = g.h * g.h;
  if (i >= g.nk) return h2;
  const int n = g.n;
  const int c = (int)(i % (n + 1)), d = (int)(i / (n + 1));
  const int mx = (c > 0) + (c < n), my = (d > 0) + (d < n);
  return h2 * (4.0 * mx * my) / 36.0;
}

__global__ __launch_bounds__(NT) void k_mq_diag_dot(Geo g, const double* __restrict__ r,
                                                    long long ld, RedCtx rc, Gate gate) {
  __shared__ double sred[NT / 64];
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  const double* rr = r + (long long)rhs * ld + g.off_pk();
  const long long np = (long long)g.nk + g.n0;
  double a = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < np; i += (long long)gridDim.x * NT) {
    const double v = rr[i] / mq_diag(g, i);
    a += (i < g.nk) ? v : -v;
  }
  double v[1] = {a};
  reduce_and_finish<NT>(rc, rhs, blockIdx.x, v, sred);
}

__global__ void k_mq_diag_apply(Geo g, const double* __restrict__ r, double* __restrict__ z,
                                long long ld, const double* __restrict__ lam, double scale,
                                Gate gate) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  const long long np = (long long)g.nk + g.n0;
  if (i >= np) return;
  const long long o = (long long)rhs * ld + g.off_pk() + i;
  const double kv = (i < g.nk) ? 1.0 : -1.0;
  z[o] = scale * (r[o] - lam[rhs] * kv) / mq_diag(g, i);
}

// sum_i k_i x_i over pressure vectors (stride ldx, pressure block at offset off)
template <typename T>
__global__ __launch_bounds__(NT) void k_mq_kdot(Geo g, const T* __restrict__ x, long long ldx,
                                                long long off, RedCtx rc, Gate gate) {
  __shared__ double sred[NT / 64];
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  const T* xr = x + (long long)rhs * ldx + off;
  const long long np = (long long)g.nk + g.n0;
  double a = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < np; i += (long long)gridDim.x * NT) {
    const double v = (double)xr[i];
    a += (i < g.nk) ? v : -v;
  }
  double v[1] = {a};
  reduce_and_finish<NT>(rc, rhs, blockIdx.x, v, sred);
}

// r_T = (T)(r_p - coef k); z = t = d = 0
template <typename T>
__global__ void k_mq_project_in(Geo g, const double* __restrict__ r, long long ld, T* __restrict__ rt,
                                T* __restrict__ z, T* __restrict__ t, T* __restrict__ d,
                                const double* __restrict__ coef, Gate gate) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  const long long np = (long long)g.nk + g.n0;
  if (i >= np) return;
  const double kv = (i < g.nk) ? 1.0 : -1.0;
  const long long o = (long long)rhs * np + i;
  rt[o] = (T)(r[(long long)rhs * ld + g.off_pk() + i] - coef[rhs] * kv);
  z[o] = T(0);
  t[o] = T(0);
  d[o] = T(0);
}

// one colour of a Gauss-Seidel sweep for M_Q t = r:
// t_i += (r_i - (M_Q t)_i) / D_ii for the nodes i of the colour
template <typename T>
__global__ void k_mq_colour(Geo g, const T* __restrict__ r, T* __restrict__ t, int colour, Gate gate) {
  const int rhs = blockIdx.z;
  if (gate.off(rhs)) return;
  const int n = g.n;
  const long long np = (long long)g.nk + g.n0;
  const T* rr = r + (long long)rhs * np;
  T* tk = t + (long long)rhs * np;
  const T* t0 = tk + g.nk;
  const double h2 = g.h * g.h;
  if (colour < 4) {
    const int c = 2 * (blockIdx.x * blockDim.x + threadIdx.x) + (colour & 1);
    const int d = 2 * (blockIdx.y * blockDim.y + threadIdx.y) + (colour >> 1);
    if (c > n || d > n) return;
    const int lx = (c > 0), rx = (c < n), ly = (d > 0), ry = (d < n);
    const double wx[3] = {(double)lx, 2.0 * (lx + rx), (double)rx};
    const double wy[3] = {(double)ly, 2.0 * (ly + ry), (double)ry};
    double acc = 0.0;
#pragma unroll
    for (int b = -1; b <= 1; ++b) {
      if (wy[b + 1] == 0.0) continue;
      double s = 0.0;
#pragma unroll
      for (int a = -1; a <= 1; ++a) {
        if (wx[a + 1] == 0.0) continue;
        s += wx[a + 1] * (double)tk[(long long)(d + b) * (n + 1) + (c + a)];
      }
      acc += wy[b + 1] * s;
    }
    acc *= h2 / 36.0;
    double e = 0.0;   // elements around the node
    for (int b = -1; b <= 0; ++b)
      for (int a = -1; a <= 0; ++a) {
        const int ex = c + a, ey = d + b;
        if (ex >= 0 && ex < n && ey >= 0 && ey < n) e += (double)t0[(long long)ey * n + ex];
      }
    acc += 0.25 * h2 * e;
    const long long i = (long long)d * (n + 1) + c;
    const double D = h2 * (4.0 * (lx + rx) * (ly + ry)) / 36.0;
    tk[i] = (T)((double)tk[i] + ((double)rr[i] - acc) / D);
  } else {
    const int ex = blockIdx.x * blockDim.x + threadIdx.x;
    const int ey = blockIdx.y * blockDim.y + threadIdx.y;
    if (ex >= n || ey >= n) return;
    const long long q = (long long)ey * (n + 1) + ex;
    const double s = (double)tk[q] + (double)tk[q + 1] + (double)tk[q + n + 1] + (double)tk[q + n + 2];
    const long long e = (long long)ey * n + ex;
    // t0 new = t0 + (r0 - h^2/4 s - h^2 t0) / h^2 = r0 / h^2 - s / 4
    tk[g.nk + e] = (T)((double)rr[g.nk + e] / h2 - 0.25 * s);
  }
}

// s = t - z;  d = first ? b*s : a*d + b*s;  z += d;  t = z
template <typename T>
__global__ void k_mq_cheb_combine(Geo g, T* __restrict__ t, T* __restrict__ z, T* __restrict__ d,
                                  double a, double b, int first, Gate gate) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  const long long np = (long long)g.nk + g.n0;
  if (i >= np) return;
  const long long o = (long long)rhs * np + i;
  const double zo = (double)z[o];
  const double s = (double)t[o] - zo;
  const double dn = first ? b * s : a * (double)d[o] + b * s;
  const double zn = zo + dn;
  d[o] = (T)dn;
  z[o] = (T)zn;
  t[o] = (T)zn;
}

// out_p = scale * (z - coef k)
template <typename T>
__global__ void k_mq_project_out(Geo g, const T* __restrict__ z, double* __restrict__ out, long long ld,
                                 const double* __restrict__ coef, double scale, Gate gate) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  const long long np = (long long)g.nk + g.n0;
  if (i >= np) return;
  const double kv = (i < g.nk) ? 1.0 : -1.0;
  out[(long long)rhs * ld + g.off_pk() + i] = scale * ((double)z[(long long)rhs * np + i] - coef[rhs] * kv);
}

inline unsigned nb(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_mq_diag_dot(const Geo& g, const double* r, long long ld, int batch, const RedCtx& rc,
                        Gate gate, hipStream_t st) {
  hipLaunchKernelGGL(k_mq_diag_dot, dim3(rc.nblocks, batch), dim3(NT), 0, st, g, r, ld, rc, gate);
  ETH_LAUNCH_CHECK();
}

void launch_mq_diag_apply(const Geo& g, const double* r, double* z, long long ld, int batch,
                          const double* lam, double scale, Gate gate, hipStream_t st) {
  const long long np = (long long)g.nk + g.n0;
  hipLaunchKernelGGL(k_mq_diag_apply, dim3(nb(np), batch), dim3(256), 0, st, g, r, z, ld, lam, scale,
                     gate);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_mq_kdot(const Geo& g, const T* x, long long ldx, long long off, int batch,
                    const RedCtx& rc, Gate gate, hipStream_t st) {
  hipLaunchKernelGGL(k_mq_kdot<T>, dim3(rc.nblocks, batch), dim3(NT), 0, st, g, x, ldx, off, rc, gate);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_mq_project_in(const Geo& g, const double* r, long long ld, T* rt, T* z, T* t, T* d,
                          int batch, const double* coef, Gate gate, hipStream_t st) {
  const long long np = (long long)g.nk + g.n0;
  hipLaunchKernelGGL(k_mq_project_in<T>, dim3(nb(np), batch), dim3(256), 0, st, g, r, ld, rt, z, t, d,
                     coef, gate);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_mq_colour(const Geo& g, const T* r, T* t, int colour, int batch, Gate gate,
                      hipStream_t st) {
  dim3 block(64, 4);
  int sx, sy;
  if (colour < 4) {
    sx = (g.n + 1 - (colour & 1) + 1) / 2;
    sy = (g.n + 1 - (colour >> 1) + 1) / 2;
  } else {
    sx = g.n;
    sy = g.n;
  }
  dim3 grid((sx + 63) / 64, (sy + 3) / 4, batch);
  hipLaunchKernelGGL(k_mq_colour<T>, grid, block, 0, st, g, r, t, colour, gate);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_mq_cheb_combine(const Geo& g, T* t, T* z, T* d, double a, double b, int first,
                            int batch, Gate gate, hipStream_t st) {
  const long long np = (long long)g.nk + g.n0;
  hipLaunchKernelGGL(k_mq_cheb_combine<T>, dim3(nb(np), batch), dim3(256), 0, st, g, t, z, d, a, b,
                     first, gate);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_mq_project_out(const Geo& g, const T* z, double* out, long long ld, int batch,
                           const double* coef, double scale, Gate gate, hipStream_t st) {
  const long long np = (long long)g.nk + g.n0;
  hipLaunchKernelGGL(k_mq_project_out<T>, dim3(nb(np), batch), dim3(256), 0, st, g, z, out, ld, coef,
                     scale, gate);
  ETH_LAUNCH_CHECK();
}

#define ETH_INST(T)                                                                               \
  template void launch_mq_kdot<T>(const Geo&, const T*, long long, long long, int, const RedCtx&,  \
                                  Gate, hipStream_t);                                              \
  template void launch_mq_project_in<T>(const Geo&, const double*, long long, T*, T*, T*, T*, int, \
                                        const double*, Gate, hipStream_t);                         \
  template void launch_mq_colour<T>(const Geo&, const T*, T*, int, int, Gate, hipStream_t);        \
  template void launch_mq_cheb_combine<T>(const Geo&, T*, T*, T*, double, double, int, int, Gate,  \
                                          hipStream_t);                                            \
  template void launch_mq_project_out<T>(const Geo&, const T*, double*, long long, int,            \
                                         const double*, double, Gate, hipStream_t);
ETH_INST(double)
ETH_INST(float)
#undef ETH_INST

}  // namespace eth
