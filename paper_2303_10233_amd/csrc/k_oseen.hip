// Kernels of the Oseen preconditioners (Sec. 3: block upper triangular
// preconditioners with M_1 and the stage-I PCD Schur approximation of
// eq:discrete-commutator1x).
//
//  * velocity block F = nu A + N(w): geometric multigrid with damped Jacobi
//    smoothing; the convection of every element touching a block's cells is
//    integrated in LDS (4x4 Gauss, exact for a Q2 wind) and gathered per node;
//  * Q1 pieces of PCD: Q_1 (Q1 mass) Chebyshev-Jacobi solve, F_1 (Q1
//    convection-diffusion with the Q2 wind, natural boundary conditions) and
//    A_p = B_1 diag(M_v)^{-1} B_1^T over the interior velocity nodes, applied
//    matrix-free through the velocity nodes staged in LDS.
#include "eth_fem.h"
#include "eth_kernels.h"
#include "eth_reduce.h"

namespace eth {
namespace {

constexpr int TX = 32, TY = 8, NT = TX * TY;
// fused Q_1 Chebyshev-Jacobi solve: owned tile side, halo, region side, threads
constexpr int Q1TQ = 16, Q1H = 12, Q1R = Q1TQ + 2 * Q1H, Q1NT = 512;
// A_p multigrid tail: threads, Q1 values of all its levels (n <= 32 on the first),
// velocity values of its first level
constexpr int APT_NT = 1024, APT_Q = 1600, APT_V = 65 * 65;
constexpr int VX = 2 * TX + 4, VY = 2 * TY + 4;

__host__ __device__ inline double diag90(int pi, int pj) {
  return (pi + pj == 0) ? 224.0 : (pi + pj == 1) ? 352.0 : 512.0;
}

// ---------------------------------------------------------------- wind
__global__ void k_inject_wind(Geo gf, Geo gc, const double* __restrict__ wf, double* __restrict__ wc) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2LL * gc.nv) return;
  const int comp = (int)(k / gc.nv), node = (int)(k % gc.nv);
  const int r = gf.n / gc.n;
  const int I = node % gc.nq, J = node / gc.nq;
  wc[k] = wf[(long long)comp * gf.nv + (long long)(r * J) * gf.nq + r * I];
}

// N_T[l][k] = h sum_q W phi_l (w . grad_ref phi_k) for one element with
// local wind w[c][j][i]; only the requested row l (lx, ly).
__device__ inline void conv_row(const double (*w)[3][3], double h, int lx, int ly, double* row) {
  double W[NG], GB[NG][3], GD[NG][3];
  gauss_tables(W, GB, GD);
  for (int k = 0; k < 9; ++k) row[k] = 0.0;
  for (int qy = 0; qy < NG; ++qy)
    for (int qx = 0; qx < NG; ++qx) {
      double wx = 0.0, wy = 0.0;
      for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i) {
          const double b = GB[qx][i] * GB[qy][j];
          wx += b * w[0][j][i];
          wy += b * w[1][j][i];
        }
      const double f = h * W[qx] * W[qy] * GB[qx][lx] * GB[qy][ly];
      for (int kj = 0; kj < 3; ++kj)
        for (int ki = 0; ki < 3; ++ki)
          row[3 * kj + ki] += f * (wx * GD[qx][ki] * GB[qy][kj] + wy * GB[qx][ki] * GD[qy][kj]);
    }
}

__device__ inline void load_elem_wind(const Geo& g, const double* wind, int e, int f, double (*w)[3][3]) {
  for (int c = 0; c < 2; ++c)
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i)
        w[c][j][i] = wind[(long long)c * g.nv + (long long)(2 * f + j) * g.nq + (2 * e + i)];
}

// diag(F) = nu diag(A) + diag(N(w)) at every node (0 on the boundary)
__global__ void k_cd_diag(Geo g, const double* __restrict__ wind, double nu, double* __restrict__ dF) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= g.nv) return;
  const int I = node % g.nq, J = node / g.nq, top = g.nq - 1;
  if (I == 0 || J == 0 || I == top || J == top) {
    dF[node] = 0.0;
    return;
  }
  double v = nu * diag90(I & 1, J & 1) / 90.0;
  for (int f = (J - 2 + 1) / 2; f <= J / 2; ++f) {
    if (f < 0 || f >= g.n || J - 2 * f > 2 || J - 2 * f < 0) continue;
    for (int e = (I - 2 + 1) / 2; e <= I / 2; ++e) {
      if (e < 0 || e >= g.n || I - 2 * e > 2 || I - 2 * e < 0) continue;
      double w[2][3][3], row[9];
      load_elem_wind(g, wind, e, f, w);
      const int lx = I - 2 * e, ly = J - 2 * f;
      conv_row(w, g.h, lx, ly, row);
      v += row[3 * ly + lx];
    }
  }
  dF[node] = v;
}

// Dense [F | I] on the interior nodes (coarsest level): one thread per row
// The coarse F = nu A + N(w) on the interior nodes of one level as a dense
// row-major matrix (A must be zero on entry); one thread per row, visiting
// only the (at most 2 x 2) elements that hold the row's node.
__global__ void k_dense_convdiff(Geo g, const double* __restrict__ wind, double nu,
                                 double* __restrict__ A, int ni) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= ni) return;
  const int m = g.nq - 2;
  const int I = 1 + row % m, J = 1 + row / m;
  double* a = A + (long long)row * ni;
  const double Ke[3][3] = {{7, -8, 1}, {-8, 16, -8}, {1, -8, 7}};
  const double Me[3][3] = {{4, 2, -1}, {2, 16, 2}, {-1, 2, 4}};
  const int f_lo = J >= 2 ? (J - 1) / 2 : 0, f_hi = J / 2 < g.n - 1 ? J / 2 : g.n - 1;
  const int e_lo = I >= 2 ? (I - 1) / 2 : 0, e_hi = I / 2 < g.n - 1 ? I / 2 : g.n - 1;
  for (int f = f_lo; f <= f_hi; ++f) {
    const int ly = J - 2 * f;
    if (ly < 0 || ly > 2) continue;
    for (int e = e_lo; e <= e_hi; ++e) {
      const int lx = I - 2 * e;
      if (lx < 0 || lx > 2) continue;
      double w[2][3][3], row9[9];
      load_elem_wind(g, wind, e, f, w);
      conv_row(w, g.h, lx, ly, row9);
      for (int kj = 0; kj < 3; ++kj)
        for (int ki = 0; ki < 3; ++ki) {
          const int Ic = 2 * e + ki, Jc = 2 * f + kj;
          if (Ic < 1 || Jc < 1 || Ic > m || Jc > m) continue;
          const double aT = (Ke[lx][ki] * Me[ly][kj] + Me[lx][ki] * Ke[ly][kj]) / 90.0;
          a[(Jc - 1) * m + (Ic - 1)] += nu * aT + row9[3 * kj + ki];
        }
    }
  }
}

// One damped Jacobi step (MODE 0: out = x + omega D_F^{-1}(b - F x)) or the
// residual (MODE 1: out = b - F x) on the planes [rhs][component][nv] of a
// multigrid level; with out64 (MODE 0) the result goes, times out_scale, to
// the velocity part of FP64 vectors instead.  TRANS: F^T = nu A + N^T (same
// diagonal).
// The element convection and the stencil sums run in the storage type T
// (FP32 in the mixed-precision preconditioner), and the wind comes in T too
// (the level's wind rounded once at set-up).
template <typename T, int MODE, bool TRANS>
__global__ __launch_bounds__(NT) void k_cd_step(Geo g, const T* __restrict__ wind,
                                                const double* __restrict__ dF, double nu,
                                                const T* __restrict__ b, const T* __restrict__ x,
                                                T* __restrict__ out, double omega,
                                                double* __restrict__ out64, long long ld64,
                                                double out_scale, Gate gate) {
  using C = T;
  __shared__ C sx[VY][VX];
  __shared__ C sw[2][VY][VX];
  __shared__ C sN[(TY + 1) * (TX + 1)][9];
  const int plane = blockIdx.z;
  if (gate.off(plane >> 1)) return;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const int ex0 = blockIdx.x * TX, ey0 = blockIdx.y * TY;
  const int n = g.n, nq = g.nq, top = 2 * n;
  const long long po = (long long)plane * g.nv;
  const int I0 = 2 * ex0 - 2, J0 = 2 * ey0 - 2;
  stage2<NT, VX * VY>(&sw[0][0][0], &sw[1][0][0], tid, [&](int k, C& w0, C& w1) {
    const int I = I0 + k % VX, J = J0 + k / VX;
    if (I >= 0 && I <= top && J >= 0 && J <= top) {
      const long long o = (long long)J * nq + I;
      w0 = (C)wind[o];
      w1 = (C)wind[g.nv + o];
    }
  });
  stage1<NT, VX * VY>(&sx[0][0], tid, [&](int k, C& xv) {
    const int I = I0 + k % VX, J = J0 + k / VX;
    if (I > 0 && J > 0 && I < top && J < top) xv = (C)x[po + (long long)J * nq + I];
  });
  __syncthreads();
  for (int k = tid; k < (TX + 1) * (TY + 1); k += NT) {
    const int lex = k % (TX + 1), ley = k / (TX + 1);
    const int e = ex0 - 1 + lex, f = ey0 - 1 + ley;
    if (e < 0 || e >= n || f < 0 || f >= n) continue;
    C ul[3][3], wl[2][3][3], ol[3][3];
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) {
        ul[j][i] = sx[2 * ley + j][2 * lex + i];
        wl[0][j][i] = sw[0][2 * ley + j][2 * lex + i];
        wl[1][j][i] = sw[1][2 * ley + j][2 * lex + i];
      }
    element_convection1<C, C, TRANS>(ul, wl, (C)g.h, ol);
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) sN[k][3 * j + i] = ol[j][i];
  }
  __syncthreads();
  const int ex = ex0 + tx, ey = ey0 + ty;
  if (ex > n || ey > n) return;
  // a value of boundary node (I, J): zero (the residual and the step are zero there)
  auto write_zero = [&](int I, int J) {
    if (I > top || J > top) return;
    const long long o = (long long)J * nq + I;
    if constexpr (MODE == 1) out[po + o] = T(0);
    else if (out64) out64[(long long)(plane >> 1) * ld64 + (long long)(plane & 1) * g.nv + o] = 0.0;
    else out[po + o] = T(0);
  };
  // the grid covers elements 0 .. n-1 (ceil(n / TX) x ceil(n / TY) tiles);
  // where no tile reaches ex = n (or ey = n), the last element column (row)
  // also writes boundary node column (row) 2n
  if (ex == n - 1 && n % TX == 0) {
    write_zero(top, 2 * ey);
    write_zero(top, 2 * ey + 1);
    if (ey == n - 1 && n % TY == 0) write_zero(top, top);
  }
  if (ey == n - 1 && n % TY == 0) {
    write_zero(2 * ex, top);
    write_zero(2 * ex + 1, top);
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int I = 2 * ex + i, J = 2 * ey + j;
      if (I > top || J > top) continue;
      const long long o = (long long)J * nq + I;
      const bool bnd = (I == 0 || J == 0 || I == top || J == top);
      double res = 0.0, xn = 0.0;
      if (!bnd) {
        const int lx = 2 * tx + i + 2, ly = 2 * ty + j + 2;
        C ax = 0;
#pragma unroll
        for (int bb = -2; bb <= 2; ++bb)
#pragma unroll
          for (int aa = -2; aa <= 2; ++aa) {
            const int c = K1(i, aa) * M1(j, bb) + M1(i, aa) * K1(j, bb);
            if (c != 0) ax += (C)c * sx[ly + bb][lx + aa];
          }
        C cv = 0;
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
          if (j == 1 && bb == 0) continue;
#pragma unroll
          for (int aa = 0; aa < 2; ++aa) {
            if (i == 1 && aa == 0) continue;
            const int e = ex - 1 + aa, f = ey - 1 + bb;
            if (e < 0 || e >= n || f < 0 || f >= n) continue;
            const int k = (ty + bb) * (TX + 1) + (tx + aa);
            cv += sN[k][3 * (j + 2 * (1 - bb)) + (i + 2 * (1 - aa))];
          }
        }
        res = (double)b[po + o] - ((double)(C)(nu / 90.0) * (double)ax + (double)cv);
        xn = (double)sx[ly][lx] + omega * res / dF[o];
      }
      if constexpr (MODE == 1) {
        out[po + o] = (T)res;
      } else if (out64) {
        out64[(long long)(plane >> 1) * ld64 + (long long)(plane & 1) * g.nv + o] = out_scale * xn;
      } else {
        out[po + o] = (T)xn;
      }
    }
  }
}

// ---------------------------------------------------------------- Q1 pieces
// Q1 mass (h^2/36) sum w_x w_y x over the 3x3 neighbourhood, w = [l, 2(l+r), r]
template <typename T>
__device__ inline double q1_mass_row(const T* x, int c, int d, int n, double h2) {
  const int lx = (c > 0), rx = (c < n), ly = (d > 0), ry = (d < n);
  const double wx[3] = {(double)lx, 2.0 * (lx + rx), (double)rx};
  const double wy[3] = {(double)ly, 2.0 * (ly + ry), (double)ry};
  double acc = 0.0;
  for (int bb = -1; bb <= 1; ++bb) {
    if (wy[bb + 1] == 0.0) continue;
    double s = 0.0;
    for (int aa = -1; aa <= 1; ++aa) {
      if (wx[aa + 1] == 0.0) continue;
      s += wx[aa + 1] * (double)x[(long long)(d + bb) * (n + 1) + (c + aa)];
    }
    acc += wy[bb + 1] * s;
  }
  return acc * h2 / 36.0;
}

// Chebyshev step for Q_1 x = b (Jacobi): x_new = x + alpha (x - x_prev) + beta D^{-1}(b - Q_1 x);
// has_prev 0: first step from x = 0 (x_new = beta D^{-1} b); output over xo.
template <typename T>
__global__ void k_q1mass_cheb(Geo g, const T* __restrict__ b, const T* __restrict__ x,
                              T* __restrict__ xo, double alpha, double beta, int has_prev, Gate gate) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  if (k >= g.nk) return;
  const int n = g.n, c = k % (n + 1), d = k / (n + 1);
  const long long o = (long long)rhs * g.nk + k;
  const double h2 = g.h * g.h;
  const double D = h2 * ((c > 0) + (c < n)) * ((d > 0) + (d < n)) / 9.0;
  if (has_prev == 0) {
    xo[o] = (T)(beta * (double)b[o] / D);
    return;
  }
  const T* xr = x + (long long)rhs * g.nk;
  const double xc = (double)xr[k];
  const double r = (double)b[o] - q1_mass_row(xr, c, d, n, h2);
  const double prev = (has_prev == 2) ? 0.0 : (double)xo[o];   // 2: previous iterate is zero
  xo[o] = (T)(xc + alpha * (xc - prev) + beta * r / D);
}

// All steps of the Chebyshev-Jacobi solve Q_1 x = b in one launch.  A block
// owns Q1TQ x Q1TQ nodes (the last block of a row or column also node n),
// stages b on a region widened by Q1H nodes and iterates on the region in
// LDS; the outermost ring of the region is never updated, and each stencil
// step spreads its stale values inward by one node at most, so the owned
// nodes are exact for steps <= Q1H.  Every step is the arithmetic of
// k_q1mass_cheb (the same expressions, each iterate rounded to T), so the
// result equals the one-launch-per-step solve bit for bit.
template <typename T>
__device__ inline double q1_mass_row_local(const T* x, int lx, int ly, int c, int d, int n, double h2) {
  const int lxf = (c > 0), rx = (c < n), lyf = (d > 0), ry = (d < n);
  const double wx[3] = {(double)lxf, 2.0 * (lxf + rx), (double)rx};
  const double wy[3] = {(double)lyf, 2.0 * (lyf + ry), (double)ry};
  double acc = 0.0;
  for (int bb = -1; bb <= 1; ++bb) {
    if (wy[bb + 1] == 0.0) continue;
    double s = 0.0;
    for (int aa = -1; aa <= 1; ++aa) {
      if (wx[aa + 1] == 0.0) continue;
      s += wx[aa + 1] * (double)x[(ly + bb) * Q1R + (lx + aa)];
    }
    acc += wy[bb + 1] * s;
  }
  return acc * h2 / 36.0;
}

template <typename T>
__global__ __launch_bounds__(Q1NT) void k_q1mass_cheb_fused(Geo g, const T* __restrict__ b,
                                                           T* __restrict__ out, Q1Cheb cc, Gate gate) {
  __shared__ T sb[Q1R * Q1R];
  __shared__ T sx[2][Q1R * Q1R];
  const int rhs = blockIdx.z;
  if (gate.off(rhs)) return;   // uniform per block
  const int n = g.n, tid = threadIdx.x;
  const int c0 = blockIdx.x * Q1TQ, d0 = blockIdx.y * Q1TQ;
  const int gx = c0 - Q1H, gy = d0 - Q1H;
  const bool last_x = blockIdx.x == gridDim.x - 1, last_y = blockIdx.y == gridDim.y - 1;
  const T* br = b + (long long)rhs * g.nk;
  const double h2 = g.h * g.h;
  constexpr int IT = (Q1R * Q1R + Q1NT - 1) / Q1NT;
  // staging of b and the first step x_1 = beta_0 D^{-1} b
  T bv[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int k = tid + i * Q1NT, c = gx + k % Q1R, d = gy + k / Q1R;
    bv[i] = T(0);
    if (k < Q1R * Q1R && c >= 0 && c <= n && d >= 0 && d <= n) bv[i] = br[(long long)d * (n + 1) + c];
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int k = tid + i * Q1NT, c = gx + k % Q1R, d = gy + k / Q1R;
    if (k >= Q1R * Q1R) break;
    T x1 = T(0);
    if (c >= 0 && c <= n && d >= 0 && d <= n) {
      const double D = h2 * ((c > 0) + (c < n)) * ((d > 0) + (d < n)) / 9.0;
      x1 = (T)(cc.b[0] * (double)bv[i] / D);
    }
    sb[k] = bv[i];
    sx[0][k] = x1;
    sx[1][k] = T(0);
  }
  __syncthreads();
  int cur = 0;
  for (int s = 1; s < cc.steps; ++s) {
    const double alpha = cc.a[s], beta = cc.b[s];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int k = tid + i * Q1NT, lx = k % Q1R, ly = k / Q1R, c = gx + lx, d = gy + ly;
      if (k >= Q1R * Q1R) break;
      if (lx == 0 || ly == 0 || lx == Q1R - 1 || ly == Q1R - 1 || c < 0 || c > n || d < 0 || d > n) continue;
      const double D = h2 * ((c > 0) + (c < n)) * ((d > 0) + (d < n)) / 9.0;
      const double xc = (double)sx[cur][k];
      const double r = (double)sb[k] - q1_mass_row_local(sx[cur], lx, ly, c, d, n, h2);
      const double prev = (s == 1) ? 0.0 : (double)sx[cur ^ 1][k];   // step 1: the previous iterate is zero
      sx[cur ^ 1][k] = (T)(xc + alpha * (xc - prev) + beta * r / D);
    }
    __syncthreads();
    cur ^= 1;
  }
  T* outr = out + (long long)rhs * g.nk;
  constexpr int OW = Q1TQ + 1;   // owned nodes per side, node n included for the last tiles
  for (int k = tid; k < OW * OW; k += Q1NT) {
    const int ox = k % OW, oy = k / OW, c = c0 + ox, d = d0 + oy;
    if ((ox == Q1TQ && !last_x) || (oy == Q1TQ && !last_y) || c > n || d > n) continue;
    outr[(long long)d * (n + 1) + c] = sx[cur][(oy + Q1H) * Q1R + (ox + Q1H)];
  }
}

// y = F_1 x on Q1 vectors: F_1 = nu int grad psi_j . grad psi_i + int (w . grad psi_j) psi_i
// (TRANS: y = F_1^T x, convection int (w . grad psi_i) psi_j)
template <typename T, bool TRANS>
__global__ void k_f1_apply(Geo g, const double* __restrict__ wind, double nu,
                           const T* __restrict__ x, T* __restrict__ y, Gate gate) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  if (k >= g.nk) return;
  const int n = g.n, c = k % (n + 1), d = k / (n + 1);
  const T* xr = x + (long long)rhs * g.nk;
  double W[NG], GB[NG][3], GD[NG][3];
  gauss_tables(W, GB, GD);
  const double kq[2][2] = {{1, -1}, {-1, 1}};
  const double mq[2][2] = {{2.0 / 6, 1.0 / 6}, {1.0 / 6, 2.0 / 6}};
  double acc = 0.0;
  for (int f = d - 1; f <= d; ++f) {
    if (f < 0 || f >= n) continue;
    for (int e = c - 1; e <= c; ++e) {
      if (e < 0 || e >= n) continue;
      const int ax = c - e, ay = d - f;   // local Q1 index of the node
      double w[2][3][3];
      load_elem_wind(g, wind, e, f, w);
      double xl[2][2];
      for (int by = 0; by < 2; ++by)
        for (int bx = 0; bx < 2; ++bx) xl[by][bx] = (double)xr[(long long)(f + by) * (n + 1) + (e + bx)];
      // diffusion row
      double s = 0.0;
      for (int by = 0; by < 2; ++by)
        for (int bx = 0; bx < 2; ++bx)
          s += nu * (kq[ax][bx] * mq[ay][by] + mq[ax][bx] * kq[ay][by]) * xl[by][bx];
      // convection row: h sum_q W psi_a (w_x d_xi x_h + w_y d_eta x_h); the Q1
      // basis at the Gauss points follows from the Q2 one: psi_0 = phi_0 +
      // phi_1/2, psi_1 = phi_2 + phi_1/2
      for (int qy = 0; qy < NG; ++qy) {
        const double py[2] = {GB[qy][0] + 0.5 * GB[qy][1], GB[qy][2] + 0.5 * GB[qy][1]};
        for (int qx = 0; qx < NG; ++qx) {
          const double px[2] = {GB[qx][0] + 0.5 * GB[qx][1], GB[qx][2] + 0.5 * GB[qx][1]};
          double wx = 0.0, wy = 0.0;
          for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
              const double bb = GB[qx][i] * GB[qy][j];
              wx += bb * w[0][j][i];
              wy += bb * w[1][j][i];
            }
          if constexpr (!TRANS) {
            const double ddx = (xl[0][1] - xl[0][0]) * py[0] + (xl[1][1] - xl[1][0]) * py[1];
            const double ddy = (xl[1][0] - xl[0][0]) * px[0] + (xl[1][1] - xl[0][1]) * px[1];
            s += g.h * W[qx] * W[qy] * px[ax] * py[ay] * (wx * ddx + wy * ddy);
          } else {
            // d psi_a / d xi = (2 ax - 1) py[ay], d psi_a / d eta = (2 ay - 1) px[ax]
            const double xv = xl[0][0] * px[0] * py[0] + xl[0][1] * px[1] * py[0] +
                              xl[1][0] * px[0] * py[1] + xl[1][1] * px[1] * py[1];
            const double dpx = (2 * ax - 1) * py[ay], dpy = (2 * ay - 1) * px[ax];
            s += g.h * W[qx] * W[qy] * xv * (wx * dpx + wy * dpy);
          }
        }
      }
      acc += s;
    }
  }
  y[(long long)rhs * g.nk + k] = (T)acc;
}

// A_p = B_1 diag(M_v)^{-1} B_1^T over the interior velocity nodes, on a tile
// of 32 x 8 Q1 nodes.  Velocity values t = diag(M_v)^{-1} B_1^T x are formed
// in LDS for the nodes the tile's rows touch, then y = B_1 t.
//   MODE 0: out = A_p x;  MODE 1: Chebyshev step over xo (has_prev 0/1/2 as
//   for the velocity smoother);  MODE 2: out = b - A_p x.
constexpr int QX = 32, QY = 8;
constexpr int XQX = QX + 4, XQY = QY + 4;          // Q1 patch, halo 2
constexpr int TVX = 2 * QX + 3, TVY = 2 * QY + 3;  // velocity patch

// 6*G and 6/h*Mpq for a velocity node of parity i and Q1 offset dc (as in k_saddle)
__device__ __forceinline__ double g6(int i, int dc) {
  return i == 0 ? (dc == -1 ? 1.0 : dc == 0 ? 0.0 : -1.0) : (dc == -1 ? 0.0 : dc == 0 ? 4.0 : -4.0);
}
__device__ __forceinline__ double mq6(int j, int dd) {
  return j == 0 ? (dd == 0 ? 2.0 : 0.0) : (dd == -1 ? 0.0 : 2.0);
}
__device__ __forceinline__ double mv_diag(int i, int j, double h2) {   // diag of the Q2 mass
  return h2 / 900.0 * (i ? 16.0 : 8.0) * (j ? 16.0 : 8.0);
}

template <typename T, int MODE>
__global__ __launch_bounds__(QX * QY) void k_ap_op(Geo g, const T* __restrict__ b,
                                                   const T* __restrict__ x, T* __restrict__ out,
                                                   double alpha, double beta, int has_prev,
                                                   const double* __restrict__ dAp, Gate gate) {
  __shared__ double sx[XQY][XQX];
  __shared__ double st[2][TVY][TVX];
  const int rhs = blockIdx.z;
  if (gate.off(rhs)) return;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * QX + tx;
  const int c0 = blockIdx.x * QX, d0 = blockIdx.y * QY;
  const int n = g.n, top = 2 * n;
  const T* xr = x + (long long)rhs * g.nk;
  stage1<QX * QY, XQX * XQY>(&sx[0][0], tid, [&](int k, double& v) {
    const int c = c0 - 2 + k % XQX, d = d0 - 2 + k / XQX;
    if (c >= 0 && c <= n && d >= 0 && d <= n) v = (double)xr[(long long)d * (n + 1) + c];
  });
  __syncthreads();
  const double h = g.h, h2 = h * h;
  const double sB = -h / 36.0;
  for (int k = tid; k < TVX * TVY; k += QX * QY) {
    const int lx = k % TVX, ly = k / TVX;
    const int I = 2 * c0 - 2 + lx, J = 2 * d0 - 2 + ly;
    double tvx = 0.0, tvy = 0.0;
    if (I >= 1 && I < top && J >= 1 && J < top) {
      const int ex = I >> 1, i = I & 1, ey = J >> 1, j = J & 1;
      double ax = 0.0, ay = 0.0;
      for (int dd = -1; dd <= 1; ++dd)
        for (int dc = -1; dc <= 1; ++dc) {
          const double p = sx[ey + dd - (d0 - 2)][ex + dc - (c0 - 2)];
          ax += g6(i, dc) * mq6(j, dd) * p;
          ay += mq6(i, dc) * g6(j, dd) * p;
        }
      const double inv = 1.0 / mv_diag(i, j, h2);
      tvx = sB * ax * inv;
      tvy = sB * ay * inv;
    }
    st[0][ly][lx] = tvx;
    st[1][ly][lx] = tvy;
  }
  __syncthreads();
  const int c = c0 + tx, d = d0 + ty;
  if (c > n || d > n) return;
  const int Lx = c > 0, Rx = c < n, Ly = d > 0, Ry = d < n;
  const double Gx[5] = {-1.0 * Lx, -4.0 * Lx, 5.0 * Lx - 5.0 * Rx, 4.0 * Rx, 1.0 * Rx};
  const double Mx[5] = {0.0, 2.0 * Lx, 1.0 * Lx + 1.0 * Rx, 2.0 * Rx, 0.0};
  const double Gy[5] = {-1.0 * Ly, -4.0 * Ly, 5.0 * Ly - 5.0 * Ry, 4.0 * Ry, 1.0 * Ry};
  const double My[5] = {0.0, 2.0 * Ly, 1.0 * Ly + 1.0 * Ry, 2.0 * Ry, 0.0};
  const int lx = 2 * tx + 2, ly = 2 * ty + 2;   // velocity node (2c, 2d) in the patch
  double s = 0.0;
  for (int q = -2; q <= 2; ++q) {
    double a1 = 0.0, a2 = 0.0;
    for (int o = -2; o <= 2; ++o) {
      a1 += Gx[o + 2] * st[0][ly + q][lx + o];
      a2 += Mx[o + 2] * st[1][ly + q][lx + o];
    }
    s += My[q + 2] * a1 + Gy[q + 2] * a2;
  }
  const double y = sB * s;
  const long long o = (long long)rhs * g.nk + (long long)d * (n + 1) + c;
  if constexpr (MODE == 0) {
    out[o] = (T)y;
  } else if constexpr (MODE == 2) {
    out[o] = (T)((double)b[o] - y);
  } else {
    const double xc = sx[ty + 2][tx + 2];
    double xn = xc + beta * ((double)b[o] - y) / dAp[(long long)d * (n + 1) + c];
    if (has_prev == 1) xn += alpha * (xc - (double)out[o]);
    else if (has_prev == 2) xn += alpha * xc;
    out[o] = (T)xn;
  }
}

// The A_p multigrid from its first level with n <= 32 down to the coarsest
// and back in one launch per right-hand side (one block): every level's
// vectors stay in LDS, each operation is the arithmetic of the per-level
// kernels (k_ap_op, k_q1_restrict, k_q1_prolong_add, k_q1_dense_solve: the
// same expressions in the same order, every vector rounded to T where those
// store it), so the result equals the per-level launches bit for bit.
template <typename T>
__global__ __launch_bounds__(APT_NT) void k_ap_tail(ApTail tl, const T* __restrict__ b0, T* __restrict__ x0,
                                                    Gate gate) {
  __shared__ T qb[APT_Q], qv[2][APT_Q];
  __shared__ double stv[2][APT_V];
  __shared__ double sdap[APT_Q];   // diag(A_p) of every level, at the level offsets of qb
  const int rhs = blockIdx.x;
  if (gate.off(rhs)) return;   // uniform per block
  const int tid = threadIdx.x;
  // bit t: which of qv[0], qv[1] holds the iterate of level t (uniform)
  unsigned curm = 0;
  auto cur = [&](int t) { return (int)((curm >> t) & 1u); };
  {
    const int nk = (tl.n[0] + 1) * (tl.n[0] + 1);
    for (int k = tid; k < nk; k += APT_NT) {
      qb[k] = b0[(long long)rhs * nk + k];
      qv[0][k] = T(0);
    }
    // the Jacobi diagonals are read in every smoothing step: staged once
    for (int t = 0; t < tl.nlev; ++t) {
      const int nt = (tl.n[t] + 1) * (tl.n[t] + 1);
      for (int k = tid; k < nt; k += APT_NT) sdap[tl.off[t] + k] = tl.dAp[t][k];
    }
  }
  __syncthreads();
  // y = A_p x on level t (MODE 1: Chebyshev step into the other array, MODE 2:
  // residual into the other array), as k_ap_op
  auto ap = [&](int t, int mode, double alpha, double beta, int has_prev) __attribute__((always_inline)) {
    const int n = tl.n[t], nq = 2 * n + 1, top = 2 * n, n1 = n + 1;
    const T* X = qv[cur(t)] + tl.off[t];
    T* O = qv[cur(t) ^ 1] + tl.off[t];
    const T* B = qb + tl.off[t];
    const double* DA = sdap + tl.off[t];
    const double h = tl.h[t], h2 = h * h, sB = -h / 36.0;
    // 1 / diag(M_v) takes four values per level (by the parities of I, J)
    const double inv00 = 1.0 / mv_diag(0, 0, h2), inv10 = 1.0 / mv_diag(1, 0, h2),
                 inv01 = 1.0 / mv_diag(0, 1, h2), inv11 = 1.0 / mv_diag(1, 1, h2);
    for (int k = tid; k < nq * nq; k += APT_NT) {
      const int I = k % nq, J = k / nq;
      double tvx = 0.0, tvy = 0.0;
      if (I >= 1 && I < top && J >= 1 && J < top) {
        const int ex = I >> 1, i = I & 1, ey = J >> 1, j = J & 1;
        double ax = 0.0, ay = 0.0;
#pragma unroll
        for (int dd = -1; dd <= 1; ++dd)
#pragma unroll
          for (int dc = -1; dc <= 1; ++dc) {
            const int c = ex + dc, d = ey + dd;
            const double p = (c >= 0 && c <= n && d >= 0 && d <= n) ? (double)X[d * n1 + c] : 0.0;
            ax += g6(i, dc) * mq6(j, dd) * p;
            ay += mq6(i, dc) * g6(j, dd) * p;
          }
        const double inv = j ? (i ? inv11 : inv01) : (i ? inv10 : inv00);
        tvx = sB * ax * inv;
        tvy = sB * ay * inv;
      }
      stv[0][k] = tvx;
      stv[1][k] = tvy;
    }
    __syncthreads();
    for (int k = tid; k < n1 * n1; k += APT_NT) {
      const int c = k % n1, d = k / n1;
      const int Lx = c > 0, Rx = c < n, Ly = d > 0, Ry = d < n;
      const double Gx[5] = {-1.0 * Lx, -4.0 * Lx, 5.0 * Lx - 5.0 * Rx, 4.0 * Rx, 1.0 * Rx};
      const double Mx[5] = {0.0, 2.0 * Lx, 1.0 * Lx + 1.0 * Rx, 2.0 * Rx, 0.0};
      const double Gy[5] = {-1.0 * Ly, -4.0 * Ly, 5.0 * Ly - 5.0 * Ry, 4.0 * Ry, 1.0 * Ry};
      const double My[5] = {0.0, 2.0 * Ly, 1.0 * Ly + 1.0 * Ry, 2.0 * Ry, 0.0};
      double s = 0.0;
#pragma unroll
      for (int q = -2; q <= 2; ++q) {
        const int J = 2 * d + q;
        double a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
          const int I = 2 * c + o;
          const bool in = I >= 0 && I <= top && J >= 0 && J <= top;
          a1 += Gx[o + 2] * (in ? stv[0][J * nq + I] : 0.0);
          a2 += Mx[o + 2] * (in ? stv[1][J * nq + I] : 0.0);
        }
        s += My[q + 2] * a1 + Gy[q + 2] * a2;
      }
      const double y = sB * s;
      if (mode == 2) {
        O[k] = (T)((double)B[k] - y);
      } else {
        const double xc = (double)X[k];
        double xn = xc + beta * ((double)B[k] - y) / DA[k];
        if (has_prev == 1) xn += alpha * (xc - (double)O[k]);
        else if (has_prev == 2) xn += alpha * xc;
        O[k] = (T)xn;
      }
    }
    __syncthreads();
    if (mode == 1) curm ^= 1u << t;
  };
  const int L = tl.nlev, deg = tl.deg;
  for (int t = 0; t + 1 < L; ++t) {
    for (int k = 0; k < deg; ++k) ap(t, 1, tl.ca[t][k], tl.cb[t][k], k == 0 ? 0 : 1);
    ap(t, 2, 0.0, 0.0, 0);
    // restriction of the residual (in the other array) as k_q1_restrict; x_c = 0
    const int nf = tl.n[t], nc = tl.n[t + 1];
    const T* rf = qv[cur(t) ^ 1] + tl.off[t];
    const double w[3] = {0.5, 1.0, 0.5};
    for (int k = tid; k < (nc + 1) * (nc + 1); k += APT_NT) {
      const int C = k % (nc + 1), D = k / (nc + 1);
      double s = 0.0;
#pragma unroll
      for (int q = -1; q <= 1; ++q) {
        const int j = 2 * D + q;
        if (j < 0 || j > nf) continue;
#pragma unroll
        for (int o = -1; o <= 1; ++o) {
          const int i = 2 * C + o;
          if (i < 0 || i > nf) continue;
          s += w[o + 1] * w[q + 1] * (double)rf[j * (nf + 1) + i];
        }
      }
      qb[tl.off[t + 1] + k] = (T)s;
      qv[cur(t + 1)][tl.off[t + 1] + k] = T(0);
    }
    __syncthreads();
  }
  {
    // coarsest level: x = Ainv b as k_q1_dense_solve (one wave per row)
    const int t = L - 1, ni = tl.ni;
    const int lane = tid & 63, wave = tid >> 6;
    const T* B = qb + tl.off[t];
    T* X = qv[cur(t)] + tl.off[t];
    for (int i = wave; i < ni; i += APT_NT / 64) {
      double s = 0.0;
      for (int j = lane; j < ni; j += 64) s += tl.Ainv[(long long)i * ni + j] * (double)B[j];
      s = wave_sum(s);
      if (lane == 0) X[i] = (T)s;
    }
    __syncthreads();
  }
  for (int t = L - 2; t >= 0; --t) {
    // x_f += P x_c as k_q1_prolong_add
    const int nf = tl.n[t], nc = tl.n[t + 1] + 1;
    const T* xr = qv[cur(t + 1)] + tl.off[t + 1];
    T* xf = qv[cur(t)] + tl.off[t];
    for (int k = tid; k < (nf + 1) * (nf + 1); k += APT_NT) {
      const int i = k % (nf + 1), j = k / (nf + 1);
      auto v = [&](int a, int b2) { return (double)xr[b2 * nc + a]; };
      double s;
      const int a0 = i >> 1, bb0 = j >> 1;
      if ((i & 1) == 0 && (j & 1) == 0) s = v(a0, bb0);
      else if ((j & 1) == 0) s = 0.5 * (v(a0, bb0) + v(a0 + 1, bb0));
      else if ((i & 1) == 0) s = 0.5 * (v(a0, bb0) + v(a0, bb0 + 1));
      else s = 0.25 * (v(a0, bb0) + v(a0 + 1, bb0) + v(a0, bb0 + 1) + v(a0 + 1, bb0 + 1));
      xf[k] = (T)((double)xf[k] + s);
    }
    __syncthreads();
    for (int k = 0; k < deg; ++k) ap(t, 1, tl.ca[t][k], tl.cb[t][k], k == 0 ? 0 : 1);
  }
  {
    const int nk = (tl.n[0] + 1) * (tl.n[0] + 1);
    const T* X = qv[cur(0)];
    for (int k = tid; k < nk; k += APT_NT) x0[(long long)rhs * nk + k] = X[k];
  }
}

// diag(A_p) at every Q1 node
__global__ void k_ap_diag(Geo g, double* __restrict__ dAp) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.nk) return;
  const int n = g.n, c = k % (n + 1), d = k / (n + 1), top = 2 * n;
  const int Lx = c > 0, Rx = c < n, Ly = d > 0, Ry = d < n;
  const double Gx[5] = {-1.0 * Lx, -4.0 * Lx, 5.0 * Lx - 5.0 * Rx, 4.0 * Rx, 1.0 * Rx};
  const double Mx[5] = {0.0, 2.0 * Lx, 1.0 * Lx + 1.0 * Rx, 2.0 * Rx, 0.0};
  const double Gy[5] = {-1.0 * Ly, -4.0 * Ly, 5.0 * Ly - 5.0 * Ry, 4.0 * Ry, 1.0 * Ry};
  const double My[5] = {0.0, 2.0 * Ly, 1.0 * Ly + 1.0 * Ry, 2.0 * Ry, 0.0};
  const double sB = g.h / 36.0, h2 = g.h * g.h;
  double s = 0.0;
  for (int q = -2; q <= 2; ++q)
    for (int o = -2; o <= 2; ++o) {
      const int I = 2 * c + o, J = 2 * d + q;
      if (I < 1 || J < 1 || I >= top || J >= top) continue;
      const double bx = sB * Gx[o + 2] * My[q + 2], by = sB * Mx[o + 2] * Gy[q + 2];
      s += (bx * bx + by * by) / mv_diag(I & 1, J & 1, h2);
    }
  dAp[k] = s;
}

// Q1 restriction b_c = P^T r_f (bilinear weights [1/2, 1, 1/2]); x_c = 0
template <typename T>
__global__ void k_q1_restrict(Geo gf, Geo gc, const T* __restrict__ rf, T* __restrict__ bc,
                              T* __restrict__ xc, Gate gate) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  if (k >= gc.nk) return;
  const int C = k % (gc.n + 1), D = k / (gc.n + 1), nf = gf.n;
  const double w[3] = {0.5, 1.0, 0.5};
  double s = 0.0;
  for (int q = -1; q <= 1; ++q) {
    const int j = 2 * D + q;
    if (j < 0 || j > nf) continue;
    for (int o = -1; o <= 1; ++o) {
      const int i = 2 * C + o;
      if (i < 0 || i > nf) continue;
      s += w[o + 1] * w[q + 1] * (double)rf[(long long)rhs * gf.nk + (long long)j * (nf + 1) + i];
    }
  }
  bc[(long long)rhs * gc.nk + k] = (T)s;
  xc[(long long)rhs * gc.nk + k] = T(0);
}

template <typename T>
__global__ void k_q1_prolong_add(Geo gf, Geo gc, const T* __restrict__ xc, T* __restrict__ xf, Gate gate) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  if (k >= gf.nk) return;
  const int i = k % (gf.n + 1), j = k / (gf.n + 1), nc = gc.n + 1;
  const T* xr = xc + (long long)rhs * gc.nk;
  auto v = [&](int a, int b2) { return (double)xr[(long long)b2 * nc + a]; };
  double s;
  const int a0 = i >> 1, b0 = j >> 1;
  if ((i & 1) == 0 && (j & 1) == 0) s = v(a0, b0);
  else if ((j & 1) == 0) s = 0.5 * (v(a0, b0) + v(a0 + 1, b0));
  else if ((i & 1) == 0) s = 0.5 * (v(a0, b0) + v(a0, b0 + 1));
  else s = 0.25 * (v(a0, b0) + v(a0 + 1, b0) + v(a0, b0 + 1) + v(a0 + 1, b0 + 1));
  const long long o = (long long)rhs * gf.nk + k;
  xf[o] = (T)((double)xf[o] + s);
}

// sum of a Q1 vector per RHS (for mean projections)
template <typename T>
__global__ __launch_bounds__(256) void k_q1_sum(Geo g, const T* __restrict__ x, RedCtx rc, Gate gate) {
  __shared__ double sred[4];
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  double a = 0.0;
  for (int k = blockIdx.x * 256 + threadIdx.x; k < g.nk; k += gridDim.x * 256)
    a += (double)x[(long long)rhs * g.nk + k];
  double v[1] = {a};
  reduce_and_finish<256>(rc, rhs, blockIdx.x, v, sred);
}

// out = scale * (x - mean) where mean = sums[rhs] / nk;  out may be FP64 (pk
// part of a full vector with stride ld) or T
template <typename TI, typename TO>
__global__ void k_q1_shift(Geo g, const TI* __restrict__ x, long long ldx, long long offx,
                           TO* __restrict__ out, long long ldo, long long offo,
                           const double* __restrict__ sums, double scale, Gate gate) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  if (k >= g.nk) return;
  const double m = sums ? sums[rhs] / g.nk : 0.0;
  out[(long long)rhs * ldo + offo + k] = (TO)(scale * ((double)x[(long long)rhs * ldx + offx + k] - m));
}

// dense [A_p + s 1 1^T | I] from the columns A_p e_j (stored as a batch)
// A = (C + C^T)/2 + shift 1 1^T from the columns C of a symmetric operator
__global__ void k_dense_sym_shift(const double* __restrict__ cols, int ni, double shift,
                                  double* __restrict__ A) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)ni * ni) return;
  const int i = (int)(t / ni), j = (int)(t % ni);
  A[t] = 0.5 * (cols[(long long)j * ni + i] + cols[(long long)i * ni + j]) + shift;
}

__global__ void k_unit_columns(double* __restrict__ cols, int ni) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)ni * ni) return;
  cols[t] = ((t / ni) == (t % ni)) ? 1.0 : 0.0;
}

// Q1 dense solve x = Ainv b per RHS (small coarsest level; one block per RHS)
// (one wave per row, lanes along the row: independent loads, a shuffle sum)
template <typename T>
__global__ void k_q1_dense_solve(const double* __restrict__ Ainv, int ni, const T* __restrict__ b,
                                 T* __restrict__ x, Gate gate) {
  const int rhs = blockIdx.x;
  if (gate.off(rhs)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = wave; i < ni; i += nw) {
    double s = 0.0;
    for (int j = lane; j < ni; j += 64) s += Ainv[(long long)i * ni + j] * (double)b[(long long)rhs * ni + j];
    s = wave_sum(s);
    if (lane == 0) x[(long long)rhs * ni + i] = (T)s;
  }
}

// max over the nodes of |w| (one block; the maximum is independent of the
// order in which it is taken)
__global__ __launch_bounds__(1024) void k_wind_speed_max(Geo g, const double* __restrict__ w,
                                                         double* __restrict__ out) {
  __shared__ double sm[1024 / 64];
  double m = 0.0;
  for (int i = threadIdx.x; i < g.nv; i += 1024) {
    const double a = w[i], b = w[(long long)g.nv + i];
    m = fmax(m, sqrt(a * a + b * b));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sm[0];
    for (int k = 1; k < 1024 / 64; ++k) t = fmax(t, sm[k]);
    *out = t;
  }
}

// y = F_0 (scale * x) on the elements (two-field PCD, Sec. 3.1): the
// cell-centred operator of -nu Lap + w . grad from the jumps across interior
// edges -- diffusion nu (x_T - x_U) per edge (|e| / d = 1 on squares),
// convection by the upwind value times the edge flux F_e = int_e w . n,
// integrated exactly from the edge's three nodal wind values (Simpson).
// x, y: element vectors (n^2, index ey*n + ex).
__global__ void k_p0_cd_apply(Geo g, const double* __restrict__ wind, double nu, const double* __restrict__ x,
                              double scale, double* __restrict__ y) {
  const int T = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = g.n;
  if (T >= n * n) return;
  const int ex = T % n, ey = T / n, nq = g.nq;
  const double h = g.h;
  const double* wx = wind;
  const double* wy = wind + g.nv;
  auto vflux = [&](int I) {   // int over the vertical edge x = x0 + (I/2) h of element row ey of w_x
    const int J0 = 2 * ey;
    return (wx[(long long)J0 * nq + I] + 4 * wx[(long long)(J0 + 1) * nq + I] + wx[(long long)(J0 + 2) * nq + I]) *
           h / 6.0;
  };
  auto hflux = [&](int J) {   // int over the horizontal edge y = y0 + (J/2) h of element column ex of w_y
    const int I0 = 2 * ex;
    return (wy[(long long)J * nq + I0] + 4 * wy[(long long)J * nq + I0 + 1] + wy[(long long)J * nq + I0 + 2]) *
           h / 6.0;
  };
  const double xt = scale * x[T];
  double acc = 0.0;
  auto edge = [&](int U, double out) {
    const double xu = scale * x[U];
    acc += nu * xt;
    acc += -nu * xu;
    acc += out > 0 ? out * xt : out * xu;
  };
  if (ex > 0) edge(T - 1, -vflux(2 * ex));
  if (ex < n - 1) edge(T + 1, vflux(2 * ex + 2));
  if (ey > 0) edge(T - n, -hflux(2 * ey));
  if (ey < n - 1) edge(T + n, hflux(2 * ey + 2));
  y[T] = acc;
}

inline unsigned nb(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_p0_cd_apply(const Geo& g, const double* wind, double nu, const double* x, double scale, double* y,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_p0_cd_apply, dim3(nb((long long)g.n * g.n)), dim3(256), 0, st, g, wind, nu, x, scale, y);
  ETH_LAUNCH_CHECK();
}

void launch_wind_speed_max(const Geo& g, const double* wind, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_wind_speed_max, dim3(1), dim3(1024), 0, st, g, wind, out);
  ETH_LAUNCH_CHECK();
}

void launch_inject_wind(const Geo& gf, const Geo& gc, const double* wf, double* wc, hipStream_t st) {
  hipLaunchKernelGGL(k_inject_wind, dim3(nb(2LL * gc.nv)), dim3(256), 0, st, gf, gc, wf, wc);
  ETH_LAUNCH_CHECK();
}
void launch_cd_diag(const Geo& g, const double* wind, double nu, double* dF, hipStream_t st) {
  hipLaunchKernelGGL(k_cd_diag, dim3(nb(g.nv)), dim3(256), 0, st, g, wind, nu, dF);
  ETH_LAUNCH_CHECK();
}
void launch_dense_convdiff(const Geo& g, const double* wind, double nu, double* A, int ni,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_dense_convdiff, dim3(nb(ni, 64)), dim3(64), 0, st, g, wind, nu, A, ni);
  ETH_LAUNCH_CHECK();
}
template <typename T>
void launch_cd_step(const Geo& g, const T* wind, const double* dF, double nu, const T* b,
                    const T* x, T* out, double omega, int residual, int nplanes, double* out64,
                    long long ld64, double out_scale, Gate gate, hipStream_t st, int transpose) {
  dim3 grid((g.n + TX - 1) / TX, (g.n + TY - 1) / TY, nplanes);
  auto kern = residual ? (transpose ? k_cd_step<T, 1, true> : k_cd_step<T, 1, false>)
                       : (transpose ? k_cd_step<T, 0, true> : k_cd_step<T, 0, false>);
  hipLaunchKernelGGL(kern, grid, dim3(TX, TY), 0, st, g, wind, dF, nu, b, x, out, omega, out64, ld64,
                     out_scale, gate);
  ETH_LAUNCH_CHECK();
}
template <typename T>
void launch_ap_tail(const ApTail& tl, const T* b0, T* x0, int batch, Gate gate, hipStream_t st) {
  int q = 0;
  for (int t = 0; t < tl.nlev; ++t) {
    if (tl.off[t] != q) throw std::invalid_argument("A_p multigrid tail: level offsets");
    q += (tl.n[t] + 1) * (tl.n[t] + 1);
  }
  if (tl.nlev < 1 || tl.nlev > APT_L || tl.n[0] > 32 || q > APT_Q || tl.deg < 1 || tl.deg > 4 ||
      tl.ni != (tl.n[tl.nlev - 1] + 1) * (tl.n[tl.nlev - 1] + 1))
    throw std::invalid_argument("A_p multigrid tail: unsupported levels");
  hipLaunchKernelGGL(k_ap_tail<T>, dim3(batch), dim3(APT_NT), 0, st, tl, b0, x0, gate);
  ETH_LAUNCH_CHECK();
}
template <typename T>
void launch_q1mass_cheb_fused(const Geo& g, const T* b, T* out, const Q1Cheb& cc, int batch, Gate gate,
                              hipStream_t st) {
  if (cc.steps < 1 || cc.steps > Q1H) throw std::invalid_argument("fused Q_1 solve: 1 .. 12 steps");
  const unsigned t = (unsigned)((g.n + Q1TQ - 1) / Q1TQ);
  hipLaunchKernelGGL(k_q1mass_cheb_fused<T>, dim3(t, t, batch), dim3(Q1NT), 0, st, g, b, out, cc, gate);
  ETH_LAUNCH_CHECK();
}
template <typename T>
void launch_q1mass_cheb(const Geo& g, const T* b, const T* x, T* xo, double alpha, double beta,
                        int has_prev, int batch, Gate gate, hipStream_t st) {
  hipLaunchKernelGGL(k_q1mass_cheb<T>, dim3(nb(g.nk), batch), dim3(256), 0, st, g, b, x, xo, alpha, beta,
                     has_prev, gate);
  ETH_LAUNCH_CHECK();
}
template <typename T>
void launch_f1_apply(const Geo& g, const double* wind, double nu, const T* x, T* y, int batch,
                     Gate gate, hipStream_t st, int transpose) {
  if (transpose)
    hipLaunchKernelGGL((k_f1_apply<T, true>), dim3(nb(g.nk), batch), dim3(256), 0, st, g, wind, nu, x, y,
                       gate);
  else
    hipLaunchKernelGGL((k_f1_apply<T, false>), dim3(nb(g.nk), batch), dim3(256), 0, st, g, wind, nu, x, y,
                       gate);
  ETH_LAUNCH_CHECK();
}
template <typename T>
void launch_ap_op(const Geo& g, int mode, const T* b, const T* x, T* out, double alpha, double beta,
                  int has_prev, const double* dAp, int batch, Gate gate, hipStream_t st) {
  dim3 grid((g.n + 1 + QX - 1) / QX, (g.n + 1 + QY - 1) / QY, batch);
  dim3 block(QX, QY);
  if (mode == 0)
    hipLaunchKernelGGL((k_ap_op<T, 0>), grid, block, 0, st, g, b, x, out, alpha, beta, has_prev, dAp, gate);
  else if (mode == 1)
    hipLaunchKernelGGL((k_ap_op<T, 1>), grid, block, 0, st, g, b, x, out, alpha, beta, has_prev, dAp, gate);
  else
    hipLaunchKernelGGL((k_ap_op<T, 2>), grid, block, 0, st, g, b, x, out, alpha, beta, has_prev, dAp, gate);
  ETH_LAUNCH_CHECK();
}
void launch_ap_diag(const Geo& g, double* dAp, hipStream_t st) {
  hipLaunchKernelGGL(k_ap_diag, dim3(nb(g.nk)), dim3(256), 0, st, g, dAp);
  ETH_LAUNCH_CHECK();
}
template <typename T>
void launch_q1_restrict(const Geo& gf, const Geo& gc, const T* rf, T* bc, T* xc, int batch, Gate gate,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_q1_restrict<T>, dim3(nb(gc.nk), batch), dim3(256), 0, st, gf, gc, rf, bc, xc, gate);
  ETH_LAUNCH_CHECK();
}
template <typename T>
void launch_q1_prolong_add(const Geo& gf, const Geo& gc, const T* xc, T* xf, int batch, Gate gate,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_q1_prolong_add<T>, dim3(nb(gf.nk), batch), dim3(256), 0, st, gf, gc, xc, xf, gate);
  ETH_LAUNCH_CHECK();
}
template <typename T>
void launch_q1_sum(const Geo& g, const T* x, const RedCtx& rc, int batch, Gate gate, hipStream_t st) {
  hipLaunchKernelGGL(k_q1_sum<T>, dim3(rc.nblocks, batch), dim3(256), 0, st, g, x, rc, gate);
  ETH_LAUNCH_CHECK();
  launch_reduce_finish(rc, batch, gate, st);
}
template <typename TI, typename TO>
void launch_q1_shift(const Geo& g, const TI* x, long long ldx, long long offx, TO* out, long long ldo,
                     long long offo, const double* sums, double scale, int batch, Gate gate,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_q1_shift<TI, TO>), dim3(nb(g.nk), batch), dim3(256), 0, st, g, x, ldx, offx, out,
                     ldo, offo, sums, scale, gate);
  ETH_LAUNCH_CHECK();
}
void launch_unit_columns(double* cols, int ni, hipStream_t st) {
  hipLaunchKernelGGL(k_unit_columns, dim3(nb((long long)ni * ni)), dim3(256), 0, st, cols, ni);
  ETH_LAUNCH_CHECK();
}
void launch_dense_sym_shift(const double* cols, int ni, double shift, double* A, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_sym_shift, dim3(nb((long long)ni * ni)), dim3(256), 0, st, cols, ni, shift, A);
  ETH_LAUNCH_CHECK();
}
template <typename T>
void launch_q1_dense_solve(const double* Ainv, int ni, const T* b, T* x, int batch, Gate gate,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_q1_dense_solve<T>, dim3(batch), dim3(256), 0, st, Ainv, ni, b, x, gate);
  ETH_LAUNCH_CHECK();
}

#define ETH_INST(T)                                                                                  \
  template void launch_cd_step<T>(const Geo&, const T*, const double*, double, const T*, const T*, \
                                  T*, double, int, int, double*, long long, double, Gate, hipStream_t, \
                                  int);                                                               \
  template void launch_ap_tail<T>(const ApTail&, const T*, T*, int, Gate, hipStream_t);              \
  template void launch_q1mass_cheb_fused<T>(const Geo&, const T*, T*, const Q1Cheb&, int, Gate,       \
                                           hipStream_t);                                             \
  template void launch_q1mass_cheb<T>(const Geo&, const T*, const T*, T*, double, double, int, int,    \
                                      Gate, hipStream_t);                                             \
  template void launch_f1_apply<T>(const Geo&, const double*, double, const T*, T*, int, Gate,          \
                                   hipStream_t, int);                                                \
  template void launch_ap_op<T>(const Geo&, int, const T*, const T*, T*, double, double, int,          \
                                const double*, int, Gate, hipStream_t);                              \
  template void launch_q1_restrict<T>(const Geo&, const Geo&, const T*, T*, T*, int, Gate, hipStream_t);\
  template void launch_q1_prolong_add<T>(const Geo&, const Geo&, const T*, T*, int, Gate, hipStream_t); \
  template void launch_q1_sum<T>(const Geo&, const T*, const RedCtx&, int, Gate, hipStream_t);          \
  template void launch_q1_dense_solve<T>(const double*, int, const T*, T*, int, Gate, hipStream_t);
ETH_INST(double)
ETH_INST(float)
#undef ETH_INST
#define ETH_INST2(TI, TO)                                                                            \
  template void launch_q1_shift<TI, TO>(const Geo&, const TI*, long long, long long, TO*, long long,   \
                                        long long, const double*, double, int, Gate, hipStream_t);
ETH_INST2(double, double)
ETH_INST2(double, float)
ETH_INST2(float, double)
ETH_INST2(float, float)
#undef ETH_INST2

}  // namespace eth
