// Geometric multigrid for the scalar Q2 Laplacian (velocity block of the
// Stokes preconditioner, eq:stokes_pre), templated on the storage type
// (double, or float in mixed precision).  Planes hold all (2n+1)^2 nodes of
// one velocity component with zero boundary values.
//
// Uniform-grid facts used here (derived from the 1-D Q2 element matrices):
//  * A = K (x) M + M (x) K with integer 1-D rows over 90 (h-free), so the
//    same stencil serves every level;
//  * diag(A) = 224/90 (vertex,vertex), 352/90 (vertex,mid), 512/90 (mid,mid);
//  * the 1-D Q2 prolongation injects coarse nodes and gives the new fine
//    nodes at 1/4 and 3/4 of a coarse element the weights (3/8, 3/4, -1/8)
//    and (-1/8, 3/4, 3/8) of the coarse (left, mid, right) nodes; restriction
//    is its transpose, P^T rows (1/8)[-1,0,3,8,3,0,-1] at a coarse vertex and
//    (1/8)[6,8,6] at a coarse mid node.
#include <climits>

#include "eth_kernels.h"

namespace eth {
namespace {

constexpr int NX = 64, NY = 16, NT = 256;   // smoother tile (nodes), 4 nodes per thread
constexpr int HX = NX + 4, HY = NY + 4;

template <typename A>
__device__ __forceinline__ void k1row(int p, A* k) {
  if (p == 0) { k[0] = 1; k[1] = -8; k[2] = 14; k[3] = -8; k[4] = 1; }
  else        { k[0] = 0; k[1] = -8; k[2] = 16; k[3] = -8; k[4] = 0; }
}
template <typename A>
__device__ __forceinline__ void m1row(int p, A* m) {
  if (p == 0) { m[0] = -1; m[1] = 2; m[2] = 8; m[3] = 2; m[4] = -1; }
  else        { m[0] = 0; m[1] = 2; m[2] = 16; m[3] = 2; m[4] = 0; }
}
template <typename A = double>
__device__ __forceinline__ A diag90(int pi, int pj) {
  return (pi + pj == 0) ? A(224) : (pi + pj == 1) ? A(352) : A(512);
}

// 90 * (A u)(node) from a staged patch s (row pitch P), centre at (lx, ly)
template <typename T, int P>
__device__ __forceinline__ double lap90(const T* s, int lx, int ly, int pi, int pj) {
  double kx[5], mx[5], ky[5], my[5];
  k1row(pi, kx); m1row(pi, mx); k1row(pj, ky); m1row(pj, my);
  double acc = 0.0;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    double tk = 0.0, tm = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const double u = (double)s[(ly + b - 2) * P + (lx + a - 2)];
      tk += kx[a] * u;
      tm += mx[a] * u;
    }
    acc += my[b] * tk + ky[b] * tm;
  }
  return acc;
}

// One Chebyshev update of node (lx, ly) of a staged patch s (row pitch P):
// x + beta D^{-1}(b - A x), plus alpha (x - xprev) (has_prev 1) or alpha x
// (has_prev 2).  The expressions and their order are those of k_cheb_step
// (x-direction K and M sums per staged row, then the y combination), so the
// fused kernels below give its results.
template <typename T, int P>
__device__ __forceinline__ T cheb_node(const T* s, int lx, int ly, int pi, int pj, T bval, T xprev, T ta,
                                       T tb, int has_prev) {
  using A = T;
  A kx[5], mx[5], ky[5], my[5];
  k1row(pi, kx);
  m1row(pi, mx);
  k1row(pj, ky);
  m1row(pj, my);
  A tk[5], tm[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const T* row = s + (ly - 2 + j) * P + lx - 2;
    A a = 0, c = 0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const A u = (A)row[q];
      a += kx[q] * u;
      c += mx[q] * u;
    }
    tk[j] = a;
    tm[j] = c;
  }
  A acc = 0;
#pragma unroll
  for (int q = 0; q < 5; ++q) acc += my[q] * tk[q] + ky[q] * tm[q];
  const A xc = (A)s[ly * P + lx];
  const A res = (A)bval - acc / A(90);
  A xn = xc + tb * res * (A(90) / diag90<A>(pi, pj));
  if (has_prev == 1) xn += ta * (xc - (A)xprev);
  else if (has_prev == 2) xn += ta * xc;
  return xn;
}

// One Chebyshev step  x_new = x + alpha (x - x_prev) + beta D^{-1} (b - A x)
// on every plane; x_new overwrites x_prev (xo).  With out64 the result is
// instead written (times out_scale) to the velocity part of FP64 vectors.
template <typename T>
__global__ __launch_bounds__(NT) void k_cheb_step(Geo g, const T* __restrict__ b,
                                                  const T* __restrict__ x, T* __restrict__ xo,
                                                  double alpha, double beta, int has_prev,
                                                  double* __restrict__ out64, long long ld64,
                                                  double out_scale, Gate gate, int remap_min) {
  __shared__ T s[HY * HX];
  const int plane = blockIdx.z;
  const bool off = gate.off(plane >> 1);   // tested after the staging (overlapped load)
  const int nq = g.nq, top = nq - 1;
  const long long po = (long long)plane * g.nv;
  int tile_x, tile_y;
  xcd_band_tile(remap_min, tile_x, tile_y);   // large grids in XCD band order (shared halo rows in L2)
  const int I0 = tile_x * NX, J0 = tile_y * NY;
  const int tid = threadIdx.x;
  // a thread takes four consecutive rows of one column: the x-direction sums
  // (K and M rows of its column parity) of each of the eight staged rows
  // they touch are formed once and shared by the rows above and below, five
  // LDS loads per staged row instead of twenty-five per node (the sums are
  // those of lap90, in the same order).  Its b and x_prev values are loaded
  // with the staging, before the barrier.
  constexpr int RPT = NY / 4;             // rows per thread
  const int tx = tid & 63, ty = tid >> 6;
  const int I = I0 + tx, Jt = J0 + RPT * ty;
  T bv[RPT], pv[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int J = Jt + r;
    bv[r] = pv[r] = T(0);
    if (I > 0 && J > 0 && I < top && J < top) {
      const long long o = po + (long long)J * nq + I;
      bv[r] = b[o];
      if (has_prev == 1) pv[r] = xo[o];
    }
  }
  stage1<NT, HX * HY>(s, tid, [&](int k, T& v) {
    const int I = I0 + k % HX - 2, J = J0 + k / HX - 2;
    if (I >= 0 && I <= top && J >= 0 && J <= top) v = x[po + (long long)J * nq + I];
  });
  if (off) return;   // uniform per block
  __syncthreads();
  if (I > top || Jt > top) return;
  const int pi = I & 1;
  using A = T;   // arithmetic in the storage type (FP32 in mixed precision)
  A kx[5], mx[5];
  k1row(pi, kx);
  m1row(pi, mx);
  A tk[RPT + 4], tm[RPT + 4], xcen[RPT + 4];
  const int lx = tx + 2;
  // x-direction sums of staged row RPT * ty + j, formed just before first use
  auto xsums = [&](int j) {
    const T* row = s + (RPT * ty + j) * HX + lx - 2;
    A a = 0, c = 0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const A u = (A)row[q];
      a += kx[q] * u;
      c += mx[q] * u;
      if (q == 2) xcen[j] = u;
    }
    tk[j] = a;
    tm[j] = c;
  };
#pragma unroll
  for (int j = 0; j < 4; ++j) xsums(j);
  const A ta = (A)alpha, tb = (A)beta;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int J = Jt + r;
    if (J > top) break;
    xsums(r + 4);
    A xn = 0;
    if (I > 0 && J > 0 && I < top && J < top) {
      const int pj = J & 1;
      A ky[5], my[5];
      k1row(pj, ky);
      m1row(pj, my);
      A acc = 0;
#pragma unroll
      for (int q = 0; q < 5; ++q) acc += my[q] * tk[r + q] + ky[q] * tm[r + q];
      const A xc = xcen[r + 2];
      const A res = (A)bv[r] - acc / A(90);
      xn = xc + tb * res * (A(90) / diag90<A>(pi, pj));
      if (has_prev == 1) xn += ta * (xc - (A)pv[r]);
      else if (has_prev == 2) xn += ta * xc;
    }
    if (out64) {
      out64[(long long)(plane >> 1) * ld64 + (long long)(plane & 1) * g.nv +
            (long long)J * nq + I] = out_scale * (double)xn;
    } else {
      xo[po + (long long)J * nq + I] = (T)xn;
    }
  }
}

// b = r_u (velocity part of an FP64 vector), x = beta D^{-1} b
template <typename T>
__global__ void k_vcycle_entry(Geo g, const double* __restrict__ r, const double* __restrict__ sub,
                               long long ld, T* __restrict__ b, T* __restrict__ x, double beta,
                               Gate gate) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  if (k >= 2LL * g.nv) return;
  const int node = (int)(k % g.nv);
  const int I = node % g.nq, J = node / g.nq, top = g.nq - 1;
  const long long o = (long long)rhs * 2 * g.nv + k;
  if (I == 0 || J == 0 || I == top || J == top) {
    b[o] = T(0);
    x[o] = T(0);
    return;
  }
  const double rv = sub ? r[(long long)rhs * ld + k] - sub[(long long)rhs * ld + k]
                        : r[(long long)rhs * ld + k];
  const T bv = (T)rv;
  b[o] = bv;
  x[o] = (T)(beta * (double)bv * 90.0 / diag90(I & 1, J & 1));
}

// 1-D restriction weight (times 8) of fine offset o in -3..3 for a coarse
// node of parity p (0 vertex, 1 mid)
template <typename A = double>
__device__ __forceinline__ A rw8(int p, int o) {
  if (p == 0) return o == 0 ? A(8) : (o == 1 || o == -1) ? A(3) : (o == 3 || o == -3) ? A(-1) : A(0);
  return o == 0 ? A(8) : (o == 1 || o == -1) ? A(6) : A(0);
}

constexpr int CT = 16;                  // coarse tile side
constexpr int RF = 2 * CT + 5;          // fine residual patch side
constexpr int XF = RF + 4;              // fine iterate patch side

// Coarse rhs b_c = P^T (b_f - A_f x_f); x_c = beta_c D_c^{-1} b_c.
// RES_GIVEN: bf already holds the fine residual (xf unused), b_c = P^T bf.
// PRE: xf holds the first pre-smoothing iterate x1 (x0 = 0); the block first
// takes the second Chebyshev step x2 = x1 + alpha x1 + beta D^{-1}(b - A x1)
// on its patch (from x1 staged with two more layers), writes x2 on the fine
// nodes it owns (2 per coarse node and direction) to x2out, and restricts
// the residual of x2: the smoothing launch before the restriction is saved.
constexpr int XP = XF + 4;              // first-iterate patch side (PRE)

template <typename T, bool RES_GIVEN, bool PRE = false>
__global__ __launch_bounds__(NT) void k_restrict(Geo gf, Geo gc, const T* __restrict__ bf,
                                                 const T* __restrict__ xf, T* __restrict__ bc,
                                                 T* __restrict__ xc, double beta_c, Gate gate,
                                                 int remap_min, T* __restrict__ x2out = nullptr,
                                                 double pre_alpha = 0.0, double pre_beta = 0.0) {
  using A = T;   // arithmetic in the storage type (FP32 in mixed precision)
  __shared__ T sx[XF * XF];
  __shared__ A sr[RF * RF];
  __shared__ T s1[PRE ? XP * XP : 1];
  const int plane = blockIdx.z;
  const bool off = gate.off(plane >> 1);   // tested after the staging (overlapped load)
  const int nqf = gf.nq, topf = nqf - 1, nqc = gc.nq, topc = nqc - 1;
  const long long pf = (long long)plane * gf.nv, pc = (long long)plane * gc.nv;
  int tile_x, tile_y;
  xcd_band_tile(remap_min, tile_x, tile_y);   // large grids in XCD band order (shared halo rows in L2)
  const int C0x = tile_x * CT, C0y = tile_y * CT;
  const int F0x = 2 * C0x - 3, F0y = 2 * C0y - 3;     // residual patch origin
  const int tid = threadIdx.x;
  // The residual patch is computed by RG groups of RF threads: a thread takes
  // one column and RR consecutive rows, and forms the x-direction sums of
  // each staged row of its window once (five LDS loads per staged row instead
  // of twenty-five per node; the sums are those of lap90, in the same order).
  // Its fine right-hand side values are loaded before anything waits.
  constexpr int RG = 6, RR = (RF + RG - 1) / RG;
  static_assert(RF * RG <= NT, "residual groups must fit the block");
  const int rcol = tid % RF, rgrp = tid / RF, ly0 = rgrp * RR;
  const bool rt = rgrp < RG;
  const int Ir = F0x + rcol;
  T bv[RR];
#pragma unroll
  for (int i = 0; i < RR; ++i) {
    const int J = F0y + ly0 + i;
    bv[i] = T(0);
    if (rt && ly0 + i < RF && Ir > 0 && Ir < topf && J > 0 && J < topf)
      bv[i] = bf[pf + (long long)J * nqf + Ir];
  }
  if constexpr (PRE) {
    stage1<NT, XP * XP>(s1, tid, [&](int k, T& v) {
      const int I = F0x - 4 + k % XP, J = F0y - 4 + k / XP;
      if (I >= 0 && I <= topf && J >= 0 && J <= topf) v = xf[pf + (long long)J * nqf + I];
    });
    if (off) return;   // uniform per block
    __syncthreads();
    // x2 on the iterate patch (zero outside the grid and on its boundary)
    const A ta = (A)pre_alpha, tb = (A)pre_beta;
    for (int k = tid; k < XF * XF; k += NT) {
      const int lx = k % XF, ly = k / XF;
      const int I = F0x - 2 + lx, J = F0y - 2 + ly;
      T v = T(0);
      if (I > 0 && I < topf && J > 0 && J < topf)
        v = (T)cheb_node<T, XP>(s1, lx + 2, ly + 2, I & 1, J & 1, bf[pf + (long long)J * nqf + I], T(0),
                                ta, tb, 2);
      sx[k] = v;
    }
    __syncthreads();
    // the fine nodes this block owns: [2 C0, 2 C0 + 2 CT) per direction
    for (int k = tid; k < 4 * CT * CT; k += NT) {
      const int I = 2 * C0x + k % (2 * CT), J = 2 * C0y + k / (2 * CT);
      if (I > topf || J > topf) continue;
      x2out[pf + (long long)J * nqf + I] = sx[(J - F0y + 2) * XF + (I - F0x + 2)];
    }
  } else if constexpr (!RES_GIVEN) {
    stage1<NT, XF * XF>(sx, tid, [&](int k, T& v) {
      const int I = F0x - 2 + k % XF, J = F0y - 2 + k / XF;
      if (I >= 0 && I <= topf && J >= 0 && J <= topf) v = xf[pf + (long long)J * nqf + I];
    });
  }
  if (off) return;   // uniform per block
  if constexpr (!RES_GIVEN && !PRE) __syncthreads();
  if (rt) {
    A tk[RES_GIVEN ? 1 : RR + 4], tm[RES_GIVEN ? 1 : RR + 4];
    A kx[5], mx[5];
    k1row(Ir & 1, kx);
    m1row(Ir & 1, mx);
    // x-direction sums of staged row ly0 + j (rows past the patch feed no
    // residual row); formed just before first use so that few are live
    auto xsums = [&](int j) {
      A a = 0, c = 0;
      if (ly0 + j < XF) {
        const T* row = sx + (ly0 + j) * XF + rcol;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const A u = (A)row[q];
          a += kx[q] * u;
          c += mx[q] * u;
        }
      }
      tk[j] = a;
      tm[j] = c;
    };
    if constexpr (!RES_GIVEN) {
#pragma unroll
      for (int j = 0; j < 4; ++j) xsums(j);
    }
#pragma unroll
    for (int i = 0; i < RR; ++i) {
      const int ly = ly0 + i;
      if (ly >= RF) break;
      if constexpr (!RES_GIVEN) xsums(i + 4);
      const int J = F0y + ly;
      A r = 0;
      if (Ir > 0 && Ir < topf && J > 0 && J < topf) {
        r = (A)bv[i];
        if constexpr (!RES_GIVEN) {
          A ky[5], my[5];
          k1row(J & 1, ky);
          m1row(J & 1, my);
          A acc = 0;
#pragma unroll
          for (int q = 0; q < 5; ++q) acc += my[q] * tk[i + q] + ky[q] * tm[i + q];
          r -= acc / A(90);
        }
      }
      sr[ly * RF + rcol] = r;
    }
  }
  __syncthreads();
  for (int k = tid; k < CT * CT; k += NT) {
    const int cx = k % CT, cy = k / CT;
    const int Ic = C0x + cx, Jc = C0y + cy;
    if (Ic > topc || Jc > topc) continue;
    const long long o = pc + (long long)Jc * nqc + Ic;
    if (Ic == 0 || Jc == 0 || Ic == topc || Jc == topc) {
      bc[o] = T(0);
      xc[o] = T(0);
      continue;
    }
    const int pi = Ic & 1, pj = Jc & 1;
    const int lx = 2 * cx + 3, ly = 2 * cy + 3;
    A acc = 0;
#pragma unroll
    for (int q = -3; q <= 3; ++q) {
      const A wy = rw8<A>(pj, q);
      if (wy == A(0)) continue;
      A t = 0;
#pragma unroll
      for (int o2 = -3; o2 <= 3; ++o2) t += rw8<A>(pi, o2) * sr[(ly + q) * RF + lx + o2];
      acc += wy * t;
    }
    acc *= A(1.0 / 64.0);
    bc[o] = (T)acc;
    xc[o] = (T)(A(beta_c) * acc * A(90) / diag90<A>(pi, pj));
  }
}

// 1-D Q2 prolongation weights of fine node F: the coarse nodes and weights
// (injection at even F, (3/8, 3/4, -1/8) or its mirror at odd F); returns the count
__device__ __forceinline__ int prolong_weights(int F, int* idx, double* w) {
  if ((F & 1) == 0) {
    idx[0] = F >> 1;
    w[0] = 1.0;
    return 1;
  }
  const int k = (F - 1) >> 1;
  if ((k & 1) == 0) {
    idx[0] = k; idx[1] = k + 1; idx[2] = k + 2;
    w[0] = 0.375; w[1] = 0.75; w[2] = -0.125;
  } else {
    idx[0] = k - 1; idx[1] = k; idx[2] = k + 1;
    w[0] = -0.125; w[1] = 0.75; w[2] = 0.375;
  }
  return 3;
}

// x_f += P x_c on interior fine nodes.  A thread takes one fine column I
// and the four fine rows 4e .. 4e+3 inside coarse element row e: it combines
// the three coarse rows 2e .. 2e+2 in x once (an even I injects one coarse
// column, written as three terms with weights (1, 0, 0), so no lane of a wave
// branches) and forms its four rows from them, so that a fine node costs
// about two coarse loads instead of up to nine.  The sums are the same
// expressions in the same order as the one-node-per-thread form.
template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add(Geo gf, Geo gc, const T* __restrict__ xc,
                                                     T* __restrict__ xf, Gate gate) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = blockIdx.y * blockDim.y + threadIdx.y;
  const int plane = blockIdx.z;
  if (gate.off(plane >> 1)) return;
  const int topf = gf.nq - 1, nce = (gc.nq - 1) / 2;   // coarse elements per side
  if (I <= 0 || I >= topf || e >= nce) return;
  int ix0, ix1, ix2;
  double wx0, wx1, wx2;
  if ((I & 1) == 0) {
    ix0 = ix1 = ix2 = I >> 1;
    wx0 = 1.0; wx1 = 0.0; wx2 = 0.0;
  } else {
    const int k = (I - 1) >> 1;
    if ((k & 1) == 0) {
      ix0 = k; ix1 = k + 1; ix2 = k + 2;
      wx0 = 0.375; wx1 = 0.75; wx2 = -0.125;
    } else {
      ix0 = k - 1; ix1 = k; ix2 = k + 1;
      wx0 = -0.125; wx1 = 0.75; wx2 = 0.375;
    }
  }
  const T* c0 = xc + (long long)plane * gc.nv + (long long)(2 * e) * gc.nq;
  double t[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const T* row = c0 + (long long)b * gc.nq;
    double v = 0.0;
    v += wx0 * (double)row[ix0];
    v += wx1 * (double)row[ix1];
    v += wx2 * (double)row[ix2];
    t[b] = v;
  }
  T* f = xf + (long long)plane * gf.nv + (long long)(4 * e) * gf.nq + I;
  const long long q = gf.nq;
  // fine row 4e injects coarse row 2e, 4e+2 injects 2e+1; 4e+1 and 4e+3
  // take (3/8, 3/4, -1/8) and (-1/8, 3/4, 3/8) of rows 2e .. 2e+2
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  a0 += 1.0 * t[0];
  a1 += 0.375 * t[0];
  a1 += 0.75 * t[1];
  a1 += -0.125 * t[2];
  a2 += 1.0 * t[1];
  a3 += -0.125 * t[0];
  a3 += 0.75 * t[1];
  a3 += 0.375 * t[2];
  const T f0 = e > 0 ? f[0] : T(0), f1 = f[q], f2 = f[2 * q], f3 = f[3 * q];
  if (e > 0) f[0] = (T)((double)f0 + a0);   // fine row 0 is the boundary
  f[q] = (T)((double)f1 + a1);
  f[2 * q] = (T)((double)f2 + a2);
  f[3 * q] = (T)((double)f3 + a3);
}

// Coarse-grid correction and both post-smoothing steps of a V(., 2) cycle in
// one launch: x0 = x + P x_c on the tile with four layers of halo (the
// expressions of k_prolong_add), x1 = x0 + beta0 D^{-1}(b - A x0) with two,
// x2 = x1 + alpha1 (x1 - x0) + beta1 D^{-1}(b - A x1) on the tile (the
// expressions of k_cheb_step), written to xout (or, times out_scale, to the
// velocity part of FP64 vectors).  Two launches and their gaps are saved
// per level.
constexpr int PX = NX + 8, PY = NY + 8;              // x0 patch (halo 4)
constexpr int QX = NX + 4, QY = NY + 4;              // x1 patch (halo 2)
constexpr int CWX = NX / 2 + 8, CWY = NY / 2 + 8;    // coarse staging

template <typename T>
__device__ __forceinline__ double prolong_row_sum(const T* sc, int row, int I, int cx0) {
  // t[b] of k_prolong_add for coarse row `row` (staged) and fine column I
  int ix0, ix1, ix2;
  double wx0, wx1, wx2;
  if ((I & 1) == 0) {
    ix0 = ix1 = ix2 = I >> 1;
    wx0 = 1.0; wx1 = 0.0; wx2 = 0.0;
  } else {
    const int k = (I - 1) >> 1;
    if ((k & 1) == 0) {
      ix0 = k; ix1 = k + 1; ix2 = k + 2;
      wx0 = 0.375; wx1 = 0.75; wx2 = -0.125;
    } else {
      ix0 = k - 1; ix1 = k; ix2 = k + 1;
      wx0 = -0.125; wx1 = 0.75; wx2 = 0.375;
    }
  }
  const T* r = sc + row * CWX - cx0;
  double v = 0.0;
  v += wx0 * (double)r[ix0];
  v += wx1 * (double)r[ix1];
  v += wx2 * (double)r[ix2];
  return v;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_post2(Geo gf, Geo gc, const T* __restrict__ b,
                                              const T* __restrict__ xold, const T* __restrict__ xc,
                                              T* __restrict__ xout, double alpha1, double beta0,
                                              double beta1, double* __restrict__ out64, long long ld64,
                                              double out_scale, Gate gate, int remap_min) {
  __shared__ T sc[CWY * CWX];
  __shared__ T s0[PY * PX];
  __shared__ T s1[QY * QX];
  const int plane = blockIdx.z;
  const bool off = gate.off(plane >> 1);
  const int nqf = gf.nq, topf = nqf - 1, nqc = gc.nq, topc = nqc - 1;
  const long long pf = (long long)plane * gf.nv, pc = (long long)plane * gc.nv;
  int tile_x, tile_y;
  xcd_band_tile(remap_min, tile_x, tile_y);
  const int I0 = tile_x * NX, J0 = tile_y * NY;
  const int cx0 = I0 / 2 - 4, cy0 = J0 / 2 - 4;
  const int tid = threadIdx.x;
  stage1<NT, CWX * CWY>(sc, tid, [&](int k, T& v) {
    const int Ic = cx0 + k % CWX, Jc = cy0 + k / CWX;
    if (Ic >= 0 && Ic <= topc && Jc >= 0 && Jc <= topc) v = xc[pc + (long long)Jc * nqc + Ic];
  });
  stage1<NT, PX * PY>(s0, tid, [&](int k, T& v) {
    const int I = I0 - 4 + k % PX, J = J0 - 4 + k / PX;
    if (I >= 0 && I <= topf && J >= 0 && J <= topf) v = xold[pf + (long long)J * nqf + I];
  });
  if (off) return;   // uniform per block
  __syncthreads();
  // x0 = x + P x_c on the interior nodes of the patch
  for (int k = tid; k < PX * PY; k += NT) {
    const int I = I0 - 4 + k % PX, J = J0 - 4 + k / PX;
    if (I <= 0 || I >= topf || J <= 0 || J >= topf) continue;
    const int e = J >> 2, q = J & 3;
    const int r0 = 2 * e - cy0;
    double a = 0.0;
    if (q == 0) {
      const double t0 = prolong_row_sum(sc, r0, I, cx0);
      a += 1.0 * t0;
    } else if (q == 2) {
      const double t1 = prolong_row_sum(sc, r0 + 1, I, cx0);
      a += 1.0 * t1;
    } else {
      const double t0 = prolong_row_sum(sc, r0, I, cx0);
      const double t1 = prolong_row_sum(sc, r0 + 1, I, cx0);
      const double t2 = prolong_row_sum(sc, r0 + 2, I, cx0);
      if (q == 1) {
        a += 0.375 * t0;
        a += 0.75 * t1;
        a += -0.125 * t2;
      } else {
        a += -0.125 * t0;
        a += 0.75 * t1;
        a += 0.375 * t2;
      }
    }
    s0[k] = (T)((double)s0[k] + a);
  }
  __syncthreads();
  const T tb0 = (T)beta0, ta1 = (T)alpha1, tb1 = (T)beta1;
  for (int k = tid; k < QX * QY; k += NT) {
    const int lx = k % QX, ly = k / QX;
    const int I = I0 - 2 + lx, J = J0 - 2 + ly;
    T v = T(0);
    if (I > 0 && I < topf && J > 0 && J < topf)
      v = cheb_node<T, PX>(s0, lx + 2, ly + 2, I & 1, J & 1, b[pf + (long long)J * nqf + I], T(0), T(0),
                           tb0, 0);
    s1[k] = v;
  }
  __syncthreads();
  for (int k = tid; k < NX * NY; k += NT) {
    const int lx = k % NX, ly = k / NX;
    const int I = I0 + lx, J = J0 + ly;
    if (I > topf || J > topf) continue;
    T xn = T(0);
    if (I > 0 && I < topf && J > 0 && J < topf)
      xn = cheb_node<T, QX>(s1, lx + 2, ly + 2, I & 1, J & 1, b[pf + (long long)J * nqf + I],
                            s0[(ly + 4) * PX + lx + 4], ta1, tb1, 1);
    if (out64) {
      out64[(long long)(plane >> 1) * ld64 + (long long)(plane & 1) * gf.nv + (long long)J * nqf + I] =
          out_scale * (double)xn;
    } else {
      xout[pf + (long long)J * nqf + I] = xn;
    }
  }
}

// Dense solve x = Ainv b on the ni interior nodes of the two planes of one
// RHS, in two launches: the interior values of both planes are gathered into
// a contiguous FP64 buffer (from T planes or, in64, from an FP64 vector), then
// every wave multiplies two rows of Ainv (FP64, or its FP32 copy in mixed
// precision: the matrix read is the cost) with both gathered planes, eight
// loads in flight per lane, FP64 sums.  Output to T planes or (out64, times
// out_scale) to an FP64 vector.
template <typename T>
__global__ void k_dense_gather(Geo g, int ni, const T* __restrict__ b, const double* __restrict__ in64,
                               long long ldin, double* __restrict__ gb, Gate gate) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (gate.off(rhs) || k >= 2 * ni) return;
  const int nq = g.nq, m = nq - 2;
  const int comp = k / ni, i = k % ni;
  const long long node = (long long)(1 + i / m) * nq + (1 + i % m);
  gb[(long long)rhs * 2 * ni + k] = in64 ? in64[(long long)rhs * ldin + (long long)comp * g.nv + node]
                                         : (double)b[((long long)rhs * 2 + comp) * g.nv + node];
}

constexpr int DS_WAVES = 4, DS_RW = 2;   // waves per block, rows per wave
template <typename T, typename M>
__global__ __launch_bounds__(64 * DS_WAVES) void k_dense_mv(Geo g, const M* __restrict__ A, int ni,
                                                            const double* __restrict__ gb,
                                                            T* __restrict__ x, double* __restrict__ out64,
                                                            long long ld64, double out_scale, Gate gate) {
  const int rhs = blockIdx.y;
  if (gate.off(rhs)) return;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int row0 = (blockIdx.x * DS_WAVES + wid) * DS_RW;
  if (row0 >= ni) return;
  const bool two = row0 + 1 < ni;
  const M* a0 = A + (long long)row0 * ni;
  const M* a1 = two ? a0 + ni : a0;
  const double* u = gb + (long long)rhs * 2 * ni;
  const double* v = u + ni;
  double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
  int j = lane;
  for (; j + 64 < ni; j += 128) {
    const double p0 = (double)a0[j], p1 = (double)a1[j], q0 = (double)a0[j + 64], q1 = (double)a1[j + 64];
    const double u0 = u[j], v0 = v[j], u1 = u[j + 64], v1 = v[j + 64];
    // each lane sums its columns in increasing order (j, j + 64, ...)
    s00 = fma(p0, u0, s00);
    s01 = fma(p0, v0, s01);
    s10 = fma(p1, u0, s10);
    s11 = fma(p1, v0, s11);
    s00 = fma(q0, u1, s00);
    s01 = fma(q0, v1, s01);
    s10 = fma(q1, u1, s10);
    s11 = fma(q1, v1, s11);
  }
  if (j < ni) {
    const double p0 = (double)a0[j], p1 = (double)a1[j];
    s00 = fma(p0, u[j], s00);
    s01 = fma(p0, v[j], s01);
    s10 = fma(p1, u[j], s10);
    s11 = fma(p1, v[j], s11);
  }
  s00 = wave_sum(s00);
  s01 = wave_sum(s01);
  s10 = wave_sum(s10);
  s11 = wave_sum(s11);
  if (lane == 0) {
    const int nq = g.nq, m = nq - 2;
    for (int r = 0; r < (two ? 2 : 1); ++r) {
      const int row = row0 + r;
      const long long node = (long long)(1 + row / m) * nq + (1 + row % m);
      const double su = r == 0 ? s00 : s10, sv = r == 0 ? s01 : s11;
      if (out64) {
        out64[(long long)rhs * ld64 + node] = out_scale * su;
        out64[(long long)rhs * ld64 + g.nv + node] = out_scale * sv;
      } else {
        x[((long long)rhs * 2) * g.nv + node] = (T)su;
        x[((long long)rhs * 2 + 1) * g.nv + node] = (T)sv;
      }
    }
  }
}

template <typename T>
__global__ void k_zero_plane_boundary(Geo g, T* __restrict__ x, Gate gate) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int plane = blockIdx.y;
  if (gate.off(plane >> 1)) return;
  const int nq = g.nq, m = nq - 1, nb = 4 * m;
  if (k >= nb) return;
  int node;
  if (k < m) node = k;
  else if (k < 2 * m) node = (k - m) * nq + m;
  else if (k < 3 * m) node = m * nq + (m - (k - 2 * m));
  else node = (m - (k - 3 * m)) * nq;
  x[(long long)plane * g.nv + node] = T(0);
}

// ---------------------------------------------------------------------------
// The coarse end of the V-cycle in one launch: levels l0 .. L-1 (all with at
// most 65^2 nodes) of one plane live in LDS for the whole descent and ascent,
// so the ~25 launches of the small levels (each a few microseconds of fixed
// cost) become one.  Per level: the remaining pre-smoothing Chebyshev steps,
// residual + restriction (with the first step of the next level), the dense
// coarsest solve, and on the way up prolongation + post-smoothing; the
// arithmetic of every node is that of the per-level kernels above.
// ---------------------------------------------------------------------------
constexpr int TAIL_NT = 1024;

// 90 * (A u) at interior node (I, J) of a level with row pitch nq (LDS, no
// halo).  The +-2 offsets of a mid node carry zero weights and would fall
// outside the level's array next to the boundary, so they are not read.
template <typename T>
__device__ __forceinline__ double lap90_rt(const T* s, int nq, int I, int J) {
  double kx[5], mx[5], ky[5], my[5];
  const int pi = I & 1, pj = J & 1;
  k1row(pi, kx); m1row(pi, mx); k1row(pj, ky); m1row(pj, my);
  double acc = 0.0;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    if (pj && (b == 0 || b == 4)) continue;
    double tk = 0.0, tm = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      if (pi && (a == 0 || a == 4)) continue;
      const double u = (double)s[(J + b - 2) * nq + (I + a - 2)];
      tk += kx[a] * u;
      tm += mx[a] * u;
    }
    acc += my[b] * tk + ky[b] * tm;
  }
  return acc;
}

template <typename T>
__device__ void tail_cheb(const T* b, const T* x, T* xo, int nq, double alpha, double beta, int has_prev) {
  const int top = nq - 1, nv = nq * nq;
  for (int k = threadIdx.x; k < nv; k += TAIL_NT) {
    const int I = k % nq, J = k / nq;
    double xn = 0.0;
    if (I > 0 && J > 0 && I < top && J < top) {
      const double xc = (double)x[k];
      const double res = (double)b[k] - lap90_rt(x, nq, I, J) / 90.0;
      xn = xc + beta * res * (90.0 / diag90(I & 1, J & 1));
      if (has_prev == 1) xn += alpha * (xc - (double)xo[k]);
      else if (has_prev == 2) xn += alpha * xc;
    }
    xo[k] = (T)xn;
  }
  __syncthreads();
}

// LDS layout of the tail: per level [b | x_A | x_B] (nv values each); which of
// x_A / x_B holds the current iterate is one bit per level in `flip`
__device__ __forceinline__ int tail_base(const TailLevels& tl, int l) {
  int off = 0;
  for (int k = 0; k < l; ++k) off += 3 * (2 * tl.n[k] + 1) * (2 * tl.n[k] + 1);
  return off;
}

template <typename T>
__global__ __launch_bounds__(TAIL_NT) void k_vcycle_tail(TailLevels tl, const double* __restrict__ Ainv,
                                                         int ni, const T* __restrict__ b0,
                                                         T* __restrict__ x0, Gate gate) {
  extern __shared__ __align__(16) unsigned char tail_smem[];
  T* sm = reinterpret_cast<T*>(tail_smem);
  const int plane = blockIdx.x;
  if (gate.off(plane >> 1)) return;
  const int nl = tl.nlev, deg = tl.deg;
  unsigned flip = 0u;
  auto nqof = [&](int l) { return 2 * tl.n[l] + 1; };
  auto Bp = [&](int l) { return sm + tail_base(tl, l); };
  auto Xp = [&](int l) {
    const int nv = nqof(l) * nqof(l);
    return sm + tail_base(tl, l) + nv * (((flip >> l) & 1u) ? 2 : 1);
  };
  auto XOp = [&](int l) {
    const int nv = nqof(l) * nqof(l);
    return sm + tail_base(tl, l) + nv * (((flip >> l) & 1u) ? 1 : 2);
  };
  {
    const int nq = nqof(0), nv = nq * nq;
    const long long po = (long long)plane * nv;
    T* B = Bp(0);
    T* X = Xp(0);
    constexpr int IT = 5;   // issue five pairs of loads before the stores
    for (int k0 = threadIdx.x; k0 < nv; k0 += IT * TAIL_NT) {
      T bv[IT], xv[IT];
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int k = k0 + i * TAIL_NT;
        bv[i] = k < nv ? b0[po + k] : T(0);
        xv[i] = k < nv ? x0[po + k] : T(0);
      }
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const int k = k0 + i * TAIL_NT;
        if (k < nv) {
          B[k] = bv[i];
          X[k] = xv[i];
        }
      }
    }
  }
  __syncthreads();
  // descent
  for (int l = 0; l + 1 < nl; ++l) {
    const int nq = nqof(l), top = nq - 1, nv = nq * nq;
    for (int k = 1; k < deg; ++k) {
      tail_cheb(Bp(l), Xp(l), XOp(l), nq, tl.ca[l][k], tl.cb[l][k], k == 1 ? 2 : 1);
      flip ^= (1u << l);
    }
    // residual into the spare iterate buffer, then restriction with the
    // first step of level l+1
    {
      const T* B = Bp(l);
      const T* X = Xp(l);
      T* R = XOp(l);
      for (int k = threadIdx.x; k < nv; k += TAIL_NT) {
        const int I = k % nq, J = k / nq;
        double r = 0.0;
        if (I > 0 && J > 0 && I < top && J < top) r = (double)B[k] - lap90_rt(X, nq, I, J) / 90.0;
        R[k] = (T)r;
      }
    }
    __syncthreads();
    {
      const T* R = XOp(l);
      T* Bc = Bp(l + 1);
      T* Xc = Xp(l + 1);
      const int nqc = nqof(l + 1), topc = nqc - 1, nvc = nqc * nqc;
      const double beta_c = (l + 2 < nl) ? tl.cb[l + 1][0] : 0.0;
      for (int k = threadIdx.x; k < nvc; k += TAIL_NT) {
        const int Ic = k % nqc, Jc = k / nqc;
        if (Ic == 0 || Jc == 0 || Ic == topc || Jc == topc) {
          Bc[k] = T(0);
          Xc[k] = T(0);
          continue;
        }
        const int pi = Ic & 1, pj = Jc & 1;
        double acc = 0.0;
#pragma unroll
        for (int q = -3; q <= 3; ++q) {
          const double wy = rw8(pj, q);
          if (wy == 0.0) continue;
          const int J = 2 * Jc + q;
          double t = 0.0;
#pragma unroll
          for (int o2 = -3; o2 <= 3; ++o2) {
            const int I = 2 * Ic + o2;
            if (I < 0 || I > top || J < 0 || J > top) continue;
            t += rw8(pi, o2) * (double)R[J * nq + I];
          }
          acc += wy * t;
        }
        acc *= (1.0 / 64.0);
        Bc[k] = (T)acc;
        Xc[k] = (T)(beta_c * acc * 90.0 / diag90(pi, pj));
      }
    }
    __syncthreads();
  }
  // coarsest level: x = Ainv b on the interior nodes, one wave per row and
  // the lanes along the row (independent loads, a shuffle sum per row)
  {
    const int l = nl - 1;
    const int nq = nqof(l), m = nq - 2;
    const T* B = Bp(l);
    T* X = Xp(l);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = wave; i < ni; i += TAIL_NT / 64) {
      const double* a = Ainv + (long long)i * ni;
      double s0 = 0.0;
      for (int j = lane; j < ni; j += 64) s0 += a[j] * (double)B[(1 + j / m) * nq + 1 + j % m];
      s0 = wave_sum(s0);
      if (lane == 0) X[(1 + i / m) * nq + 1 + i % m] = (T)s0;
    }
    __syncthreads();
  }
  // ascent
  for (int l = nl - 2; l >= 0; --l) {
    const int nq = nqof(l), top = nq - 1, nv = nq * nq;
    const int nqc = nqof(l + 1);
    {
      const T* Xc = Xp(l + 1);
      T* X = Xp(l);
      for (int k = threadIdx.x; k < nv; k += TAIL_NT) {
        const int I = k % nq, J = k / nq;
        if (I <= 0 || J <= 0 || I >= top || J >= top) continue;
        int ix[3], iy[3];
        double wx[3], wy[3];
        const int cx = prolong_weights(I, ix, wx), cy = prolong_weights(J, iy, wy);
        double acc = 0.0;
        for (int b = 0; b < cy; ++b) {
          double t = 0.0;
          for (int a = 0; a < cx; ++a) t += wx[a] * (double)Xc[iy[b] * nqc + ix[a]];
          acc += wy[b] * t;
        }
        X[k] = (T)((double)X[k] + acc);
      }
    }
    __syncthreads();
    for (int k = 0; k < deg; ++k) {
      tail_cheb(Bp(l), Xp(l), XOp(l), nq, tl.ca[l][k], tl.cb[l][k], k == 0 ? 0 : 1);
      flip ^= (1u << l);
    }
  }
  {
    const int nq = nqof(0), nv = nq * nq;
    const long long po = (long long)plane * nv;
    const T* X = Xp(0);
    for (int k = threadIdx.x; k < nv; k += TAIL_NT) x0[po + k] = X[k];
  }
}

// ---- setup helpers (FP64) ----
__global__ void k_dense_laplacian(Geo g, double* __restrict__ A, int ni) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)ni * ni) return;
  const int i = (int)(k / ni), j = (int)(k % ni);
  const int m = g.nq - 2;
  const int Ii = 1 + i % m, Ji = 1 + i / m, Ij = 1 + j % m, Jj = 1 + j / m;
  const int dx = Ij - Ii, dy = Jj - Ji;
  double v = 0.0;
  if (dx >= -2 && dx <= 2 && dy >= -2 && dy <= 2) {
    double kx[5], mx[5], ky[5], my[5];
    k1row(Ii & 1, kx); m1row(Ii & 1, mx); k1row(Ji & 1, ky); m1row(Ji & 1, my);
    v = (kx[dx + 2] * my[dy + 2] + mx[dx + 2] * ky[dy + 2]) / 90.0;
  }
  A[k] = v;
}

// mode 0: y = A x, mode 1: y = D^{-1} x, on one FP64 plane (interior nodes; boundary 0)
__global__ void k_plane_op(Geo g, int mode, const double* __restrict__ x, double* __restrict__ y) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  const int top = g.nq - 1;
  if (I > top || J > top) return;
  double v = 0.0;
  if (I > 0 && J > 0 && I < top && J < top) {
    if (mode == 1) {
      v = x[(long long)J * g.nq + I] * 90.0 / diag90(I & 1, J & 1);
    } else {
      double kx[5], mx[5], ky[5], my[5];
      k1row(I & 1, kx); m1row(I & 1, mx); k1row(J & 1, ky); m1row(J & 1, my);
      double acc = 0.0;
      for (int b = 0; b < 5; ++b)
        for (int a = 0; a < 5; ++a) {
          const int Ia = I + a - 2, Jb = J + b - 2;
          if (Ia < 1 || Jb < 1 || Ia >= top || Jb >= top) continue;
          acc += (kx[a] * my[b] + mx[a] * ky[b]) * x[(long long)Jb * g.nq + Ia];
        }
      v = acc / 90.0;
    }
  }
  y[(long long)J * g.nq + I] = v;
}

}  // namespace

template <typename T>
void launch_cheb_step(const Geo& g, const T* b, const T* x, T* xo, double alpha, double beta,
                      int has_prev, int nplanes, double* out64, long long ld64,
                      double out_scale, Gate gate, int batch, hipStream_t st) {
  (void)batch;
  dim3 grid((g.nq + NX - 1) / NX, (g.nq + NY - 1) / NY, nplanes);
  // XCD band order for FP32 planes only: measured at 2048^2 it took the FP32
  // step from 108 to 101 us and the FP64 step from 199 to 222 us
  const int rm = sizeof(T) == 4 ? xcd_remap_min() : INT_MAX;
  hipLaunchKernelGGL(k_cheb_step<T>, grid, dim3(NT), 0, st, g, b, x, xo, alpha, beta, has_prev,
                     out64, ld64, out_scale, gate, rm);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_vcycle_entry(const Geo& g, const double* r, long long ld, T* b, T* x, double beta,
                         int batch, Gate gate, hipStream_t st, const double* sub) {
  const long long n = 2LL * g.nv;
  hipLaunchKernelGGL(k_vcycle_entry<T>, dim3((unsigned)((n + 255) / 256), batch), dim3(256), 0, st,
                     g, r, sub, ld, b, x, beta, gate);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_restrict(const Geo& gf, const Geo& gc, const T* bf, const T* xf, T* bc, T* xc,
                     double beta_c, int nplanes, int batch, Gate gate, hipStream_t st) {
  (void)batch;
  dim3 grid((gc.nq + CT - 1) / CT, (gc.nq + CT - 1) / CT, nplanes);
  const int rm = xcd_remap_min();
  if (xf)
    hipLaunchKernelGGL((k_restrict<T, false>), grid, dim3(NT), 0, st, gf, gc, bf, xf, bc, xc, beta_c, gate, rm);
  else
    hipLaunchKernelGGL((k_restrict<T, true>), grid, dim3(NT), 0, st, gf, gc, bf, xf, bc, xc, beta_c, gate, rm);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_restrict_pre(const Geo& gf, const Geo& gc, const T* bf, const T* x1, T* x2out, double alpha,
                         double beta, T* bc, T* xc, double beta_c, int nplanes, Gate gate, hipStream_t st) {
  dim3 grid((gc.nq + CT - 1) / CT, (gc.nq + CT - 1) / CT, nplanes);
  const int rm = xcd_remap_min();
  hipLaunchKernelGGL((k_restrict<T, false, true>), grid, dim3(NT), 0, st, gf, gc, bf, x1, bc, xc, beta_c, gate,
                     rm, x2out, alpha, beta);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_post2(const Geo& gf, const Geo& gc, const T* b, const T* xold, const T* xc, T* xout, double alpha1,
                  double beta0, double beta1, int nplanes, double* out64, long long ld64, double out_scale,
                  Gate gate, hipStream_t st) {
  if (gf.nq - 1 != 2 * (gc.nq - 1) || (gc.nq - 1) % 2 != 0)
    throw std::invalid_argument("prolongation needs a fine level of twice the coarse elements");
  dim3 grid((gf.nq + NX - 1) / NX, (gf.nq + NY - 1) / NY, nplanes);
  const int rm = sizeof(T) == 4 ? xcd_remap_min() : INT_MAX;
  hipLaunchKernelGGL(k_post2<T>, grid, dim3(NT), 0, st, gf, gc, b, xold, xc, xout, alpha1, beta0, beta1, out64,
                     ld64, out_scale, gate, rm);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_prolong_add(const Geo& gf, const Geo& gc, const T* xc, T* xf, int nplanes, int batch,
                        Gate gate, hipStream_t st) {
  (void)batch;
  if (gf.nq - 1 != 2 * (gc.nq - 1) || (gc.nq - 1) % 2 != 0)
    throw std::invalid_argument("prolongation needs a fine level of twice the coarse elements");
  const int nce = (gc.nq - 1) / 2;
  dim3 block(64, 4);
  dim3 grid((gf.nq - 1 + 63) / 64, (nce + 3) / 4, nplanes);
  hipLaunchKernelGGL(k_prolong_add<T>, grid, block, 0, st, gf, gc, xc, xf, gate);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_dense_solve(const Geo& g, const double* Ainv, const float* AinvF, int ni, const T* b, T* x,
                        int nplanes, double* out64, long long ld64, double out_scale, const double* in64,
                        long long ldin, double* gbuf, int batch, Gate gate, hipStream_t st) {
  (void)nplanes;
  hipLaunchKernelGGL(k_dense_gather<T>, dim3((2 * ni + 255) / 256, batch), dim3(256), 0, st, g, ni, b, in64,
                     ldin, gbuf, gate);
  ETH_LAUNCH_CHECK();
  const dim3 grid((ni + DS_WAVES * DS_RW - 1) / (DS_WAVES * DS_RW), batch);
  if (AinvF)
    hipLaunchKernelGGL((k_dense_mv<T, float>), grid, dim3(64 * DS_WAVES), 0, st, g, AinvF, ni, gbuf, x, out64,
                       ld64, out_scale, gate);
  else
    hipLaunchKernelGGL((k_dense_mv<T, double>), grid, dim3(64 * DS_WAVES), 0, st, g, Ainv, ni, gbuf, x, out64,
                       ld64, out_scale, gate);
  ETH_LAUNCH_CHECK();
  if (!out64) {
    const int nb = 4 * (g.nq - 1);
    hipLaunchKernelGGL(k_zero_plane_boundary<T>, dim3((nb + 255) / 256, 2 * batch), dim3(256), 0, st,
                       g, x, gate);
    ETH_LAUNCH_CHECK();
  }
}

size_t vcycle_tail_lds(const TailLevels& tl, size_t elem) {
  size_t v = 0;
  for (int l = 0; l < tl.nlev; ++l) v += 3 * (size_t)(2 * tl.n[l] + 1) * (2 * tl.n[l] + 1);
  return v * elem;
}

template <typename T>
void launch_vcycle_tail(const TailLevels& tl, const double* Ainv, int ni, const T* b0, T* x0, int nplanes,
                        Gate gate, hipStream_t st) {
  const size_t lds = vcycle_tail_lds(tl, sizeof(T));
  hipLaunchKernelGGL(k_vcycle_tail<T>, dim3(nplanes), dim3(TAIL_NT), lds, st, tl, Ainv, ni, b0, x0, gate);
  ETH_LAUNCH_CHECK();
}

template <typename T>
hipError_t prepare_vcycle_tail(size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vcycle_tail<T>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

void launch_dense_laplacian(const Geo& g, double* A, int ni, hipStream_t st) {
  const long long n = (long long)ni * ni;
  hipLaunchKernelGGL(k_dense_laplacian, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, A, ni);
  ETH_LAUNCH_CHECK();
}

void launch_plane_op(const Geo& g, int mode, const double* x, double* y, hipStream_t st) {
  dim3 block(64, 4);
  dim3 grid((g.nq + 63) / 64, (g.nq + 3) / 4);
  hipLaunchKernelGGL(k_plane_op, grid, block, 0, st, g, mode, x, y);
  ETH_LAUNCH_CHECK();
}

#define ETH_INST(T)                                                                             \
  template void launch_cheb_step<T>(const Geo&, const T*, const T*, T*, double, double, int, int, \
                                    double*, long long, double, Gate, int, hipStream_t);         \
  template void launch_vcycle_entry<T>(const Geo&, const double*, long long, T*, T*, double, int, \
                                       Gate, hipStream_t, const double*);                        \
  template void launch_restrict<T>(const Geo&, const Geo&, const T*, const T*, T*, T*, double,    \
                                   int, int, Gate, hipStream_t);                                 \
  template void launch_prolong_add<T>(const Geo&, const Geo&, const T*, T*, int, int, Gate,       \
                                      hipStream_t);                                              \
  template void launch_restrict_pre<T>(const Geo&, const Geo&, const T*, const T*, T*, double,   \
                                       double, T*, T*, double, int, Gate, hipStream_t);          \
  template void launch_post2<T>(const Geo&, const Geo&, const T*, const T*, const T*, T*, double, \
                                double, double, int, double*, long long, double, Gate,          \
                                hipStream_t);                                                    \
  template void launch_dense_solve<T>(const Geo&, const double*, const float*, int, const T*, T*, int, double*, \
                                      long long, double, const double*, long long, double*, int,  \
                                      Gate, hipStream_t);                                         \
  template void launch_vcycle_tail<T>(const TailLevels&, const double*, int, const T*, T*, int,    \
                                      Gate, hipStream_t);                                         \
  template hipError_t prepare_vcycle_tail<T>(size_t);
ETH_INST(double)
ETH_INST(float)
#undef ETH_INST

}  // namespace eth
