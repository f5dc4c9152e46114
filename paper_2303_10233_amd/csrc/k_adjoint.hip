// Kernels of the discrete adjoint of J(u) = 1/2 (u - u_t)^T M_v (u - u_t)
// for the lifted saddle-point systems (Sec. 2 eq:saddle_point, Sec. 3
// eq:oseen-system): the Q2 velocity mass product over all nodes (the
// misfit, its gradient dJ/du = M_v e and dJ/df = M_v lambda), and the
// viscosity sensitivity -lambda_u^T (A u)_I.  FP64.
#include "eth_fem.h"
#include "eth_kernels.h"
#include "eth_reduce.h"

namespace eth {
namespace {

constexpr int NT = 256;

// assembled 1-D Q2 mass entry between nodes I and J of an n-element line,
// in units of h/30 (boundary rows get the one-sided element sums)
__device__ inline int mass1d(int I, int J, int n) {
  const int Me[3][3] = {{4, 2, -1}, {2, 16, 2}, {-1, 2, 4}};
  int lo = (I > J ? I : J) - 2;
  lo = lo <= 0 ? 0 : (lo + 1) / 2;
  int hi = (I < J ? I : J) / 2;
  if (hi > n - 1) hi = n - 1;
  int s = 0;
  for (int e = lo; e <= hi; ++e) s += Me[I - 2 * e][J - 2 * e];
  return s;
}

__device__ inline bool on_boundary(int I, int J, int top) {
  return I == 0 || J == 0 || I == top || J == top;
}

// e = x - xt (xt optional; boundary nodes of e zero when MASK), y = M_v e at
// every node (optional), J = 1/2 e^T M_v e per RHS (optional reduction).
// Grid: (node blocks, 2 components, batch).
template <bool MASK>
__global__ __launch_bounds__(NT) void k_velocity_mass(Geo g, const double* __restrict__ x, long long ldx,
                                                      const double* __restrict__ xt, long long ldt,
                                                      double* __restrict__ y, long long ldy, RedCtx rc,
                                                      int reduce) {
  __shared__ double sred[NT / 64];
  const int node = blockIdx.x * NT + threadIdx.x;
  const int c = blockIdx.y, rhs = blockIdx.z;
  const int nq = g.nq, top = nq - 1, n = g.n;
  const double* xr = x + (long long)rhs * ldx + (long long)c * g.nv;
  const double* tr = xt ? xt + (long long)rhs * ldt + (long long)c * g.nv : nullptr;
  auto e_at = [&](int I, int J) -> double {
    if (MASK && on_boundary(I, J, top)) return 0.0;
    const long long o = (long long)J * nq + I;
    return tr ? xr[o] - tr[o] : xr[o];
  };
  double contrib = 0.0;
  if (node < g.nv) {
    const int I = node % nq, J = node / nq;
    double acc = 0.0;
    for (int bb = -2; bb <= 2; ++bb) {
      const int J2 = J + bb;
      if (J2 < 0 || J2 > top) continue;
      const int my = mass1d(J, J2, n);
      if (my == 0) continue;
      double t = 0.0;
      for (int aa = -2; aa <= 2; ++aa) {
        const int I2 = I + aa;
        if (I2 < 0 || I2 > top) continue;
        const int mx = mass1d(I, I2, n);
        if (mx != 0) t += mx * e_at(I2, J2);
      }
      acc += my * t;
    }
    const double v = acc * (g.h * g.h / 900.0);
    if (y) y[(long long)rhs * ldy + (long long)c * g.nv + node] = v;
    if (reduce) contrib = 0.5 * e_at(I, J) * v;
  }
  if (reduce) {
    double vals[1] = {contrib};
    reduce_and_finish<NT>(rc, rhs, blockIdx.y * gridDim.x + blockIdx.x, vals, sred);
  }
}

// out[rhs] = -sum over interior velocity rows of lambda * (A u)   (A: unit
// viscosity vector Laplacian acting on the full u, boundary values included)
__global__ __launch_bounds__(NT) void k_grad_viscosity(Geo g, const double* __restrict__ lam, long long ldl,
                                                       const double* __restrict__ x, long long ldx, RedCtx rc) {
  __shared__ double sred[NT / 64];
  const int node = blockIdx.x * NT + threadIdx.x;
  const int c = blockIdx.y, rhs = blockIdx.z;
  const int nq = g.nq, top = nq - 1;
  double contrib = 0.0;
  if (node < g.nv) {
    const int I = node % nq, J = node / nq;
    if (!on_boundary(I, J, top)) {
      const double* u = x + (long long)rhs * ldx + (long long)c * g.nv;
      const int pi = I & 1, pj = J & 1;
      double acc = 0.0;
      for (int bb = -2; bb <= 2; ++bb)
        for (int aa = -2; aa <= 2; ++aa) {
          const int w = K1(pi, aa) * M1(pj, bb) + M1(pi, aa) * K1(pj, bb);
          if (w != 0) acc += w * u[(long long)(J + bb) * nq + (I + aa)];
        }
      contrib = -lam[(long long)rhs * ldl + (long long)c * g.nv + node] * acc / 90.0;
    }
  }
  double vals[1] = {contrib};
  reduce_and_finish<NT>(rc, rhs, blockIdx.y * gridDim.x + blockIdx.x, vals, sred);
}

// x_u <- diag(M_v)^{-1} x_u on the interior velocity nodes (zero on the
// boundary) and x_p <- 0: the M^{-1} between B^T and B in B M^{-1} B^T
// (two-field PCD and LSC).  The assembled diagonal of the Q2 mass matrix is
// (h/30)^2 m(I) m(J) with m = 8 at a vertex and 16 at a mid node.
__global__ __launch_bounds__(NT) void k_vel_minv(Geo g, double* __restrict__ x) {
  const long long k = (long long)blockIdx.x * NT + threadIdx.x;
  const long long np = (long long)g.nk + g.n0;
  if (k >= 2LL * g.nv + np) return;
  if (k >= 2LL * g.nv) {
    x[k] = 0.0;
    return;
  }
  const int node = (int)(k % g.nv), nq = g.nq, top = nq - 1;
  const int I = node % nq, J = node / nq;
  if (on_boundary(I, J, top)) {
    x[k] = 0.0;
    return;
  }
  const double mi = (I & 1) ? 16.0 : 8.0, mj = (J & 1) ? 16.0 : 8.0;
  const double d = (g.h / 30.0) * (g.h / 30.0) * mi * mj;
  x[k] = x[k] / d;
}

inline unsigned nblk(long long n) { return (unsigned)((n + NT - 1) / NT); }

}  // namespace

void launch_vel_minv(const Geo& g, double* x, hipStream_t st) {
  hipLaunchKernelGGL(k_vel_minv, dim3(nblk(g.N)), dim3(NT), 0, st, g, x);
  ETH_LAUNCH_CHECK();
}

int adjoint_blocks(const Geo& g) { return 2 * (int)nblk(g.nv); }

void launch_velocity_mass(const Geo& g, const double* x, long long ldx, const double* xt, long long ldt,
                          int mask_boundary, double* y, long long ldy, const RedCtx* half_energy, int batch,
                          hipStream_t st) {
  dim3 grid(nblk(g.nv), 2, batch);
  RedCtx rc{};
  int reduce = 0;
  if (half_energy) {
    rc = *half_energy;
    rc.nblocks = (int)(grid.x * grid.y);
    reduce = 1;
  }
  if (mask_boundary)
    hipLaunchKernelGGL(k_velocity_mass<true>, grid, dim3(NT), 0, st, g, x, ldx, xt, ldt, y, ldy, rc, reduce);
  else
    hipLaunchKernelGGL(k_velocity_mass<false>, grid, dim3(NT), 0, st, g, x, ldx, xt, ldt, y, ldy, rc, reduce);
  ETH_LAUNCH_CHECK();
  if (reduce) launch_reduce_finish(rc, batch, no_gate(), st);
}

void launch_grad_viscosity(const Geo& g, const double* lam, long long ldl, const double* x, long long ldx,
                           const RedCtx& rc_in, int batch, hipStream_t st) {
  dim3 grid(nblk(g.nv), 2, batch);
  RedCtx rc = rc_in;
  rc.nblocks = (int)(grid.x * grid.y);
  hipLaunchKernelGGL(k_grad_viscosity, grid, dim3(NT), 0, st, g, lam, ldl, x, ldx, rc);
  ETH_LAUNCH_CHECK();
  launch_reduce_finish(rc, batch, no_gate(), st);
}

}  // namespace eth
