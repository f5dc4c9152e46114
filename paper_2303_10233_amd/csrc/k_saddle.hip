// Matrix-free enriched Taylor-Hood saddle-point operator on a uniform mesh of
// square Q2 elements (eq:saddle_point), FP64, gather form (no atomics).
//
// Assembled 1-D Q2 rows on a uniform grid (node parity p: 0 vertex, 1 mid):
//   stiffness  K: vertex (1/(3h))[1,-8,14,-8,1], mid (1/(3h))[-8,16,-8]
//   mass       M: vertex (h/30)[-1,2,8,2,-1],    mid (h/30)[2,16,2]
// The scalar Laplacian is K (x) M + M (x) K, so every coefficient is an
// integer over 90, independent of h.  The divergence rows (Q1 and P0 test
// functions) and their transposes come from the 1-D factors
//   G  = int psi_a phi_j'   and  Mpq = int psi_a phi_j   (Q1 rows),
//   g0 = int phi_j'         and  m0  = int phi_j         (P0 rows),
// assembled per node parity; B = -(G (x) Mpq) for u_x and -(Mpq (x) G) for
// u_y (x factor first), with the sign of b(u,p) = -int p div u.
//
// One thread owns a "cell" (ex, ey), 0 <= ex, ey <= n: the four velocity
// nodes (2ex+i, 2ey+j), i,j in {0,1}, of both components, the Q1 node
// (ex, ey) and the element (ex, ey).  A 32 x 8 block of cells stages its
// velocity patch (halo 2 nodes), Q1 patch (halo 1) and P0 patch in LDS.
#include "eth_fem.h"
#include "eth_kernels.h"
#include "eth_reduce.h"

namespace eth {
namespace {

constexpr int TX = 32, TY = 8, NT = TX * TY;
constexpr int VX = 2 * TX + 4, VY = 2 * TY + 4;
constexpr int PX = TX + 2, PY = TY + 2;
constexpr int EX = TX + 1, EY = TY + 1;

// 6 * G(c - ex) for a velocity node of parity i (dc in -1..1)
__host__ __device__ constexpr int G6(int i, int dc) {
  return i == 0 ? (dc == -1 ? 1 : dc == 0 ? 0 : -1) : (dc == -1 ? 0 : dc == 0 ? 4 : -4);
}
// 6/h * Mpq(d - ey) for a velocity node of parity j
__host__ __device__ constexpr int Mq6(int j, int dd) {
  return j == 0 ? (dd == 0 ? 2 : 0) : (dd == -1 ? 0 : 2);
}
// g0 and 6/h * m0 for a velocity node of parity i / j, element offset de in {-1, 0}
__host__ __device__ constexpr int g1(int i, int de) {
  return i == 0 ? (de == -1 ? 1 : -1) : 0;
}
__host__ __device__ constexpr int m6(int j, int df) {
  return j == 0 ? 1 : (df == -1 ? 0 : 4);
}

// MODE 0: operator apply (boundary velocity masked, boundary rows 0).
// MODE 1: lift: y = [M_v f; 0] - K_unmasked [u_B; 0]; boundary rows = u_B.
// CONV adds the convection N(w) (TRANS: N(w)^T) of the nodal Q2 wind.
template <int MODE, bool DOT, bool CONV, bool TRANS>
__global__ __launch_bounds__(NT) void k_saddle(Geo g, double nu, const double* __restrict__ x,
                                               long long ldx,
                                               double* __restrict__ y, long long ld,
                                               const double* __restrict__ f, long long ldf,
                                               const double* __restrict__ wind,
                                               Gate gate, RedCtx rc, ClearFlag clear) {
  __shared__ double su[2][VY][VX];
  __shared__ double sf[MODE == 1 ? 2 : 1][MODE == 1 ? VY : 1][MODE == 1 ? VX : 1];
  __shared__ double sw[CONV ? 2 : 1][CONV ? VY : 1][CONV ? VX : 1];
  __shared__ double sN[CONV ? 2 : 1][CONV ? (TY + 1) * (TX + 1) : 1][9];
  __shared__ double spk[PY][PX];
  __shared__ double sp0[EY][EX];
  __shared__ double sred[NT / 64];

  const int rhs = blockIdx.z;
  clear.apply(rhs);
  if (gate.off(rhs)) return;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * TX + tx;
  const int ex0 = blockIdx.x * TX, ey0 = blockIdx.y * TY;
  const int n = g.n, nq = g.nq, top = 2 * n;
  const double* xr = x + (long long)rhs * ldx;
  double* yr = y + (long long)rhs * ld;

  // ---- stage the patches ----
  const int I0 = 2 * ex0 - 2, J0 = 2 * ey0 - 2;
  for (int k = tid; k < VX * VY; k += NT) {
    const int lx = k % VX, ly = k / VX;
    const int I = I0 + lx, J = J0 + ly;
    double vx = 0.0, vy = 0.0;
    const bool inside = (MODE == 0) ? (I >= 1 && I < top && J >= 1 && J < top)
                                    : (I >= 0 && I <= top && J >= 0 && J <= top);
    if (inside) {
      const long long o = (long long)J * nq + I;
      vx = xr[o];
      vy = xr[g.nv + o];
    }
    su[0][ly][lx] = vx;
    su[1][ly][lx] = vy;
    if constexpr (CONV) {
      double wxv = 0.0, wyv = 0.0;
      if (I >= 0 && I <= top && J >= 0 && J <= top) {
        const long long o = (long long)J * nq + I;
        wxv = wind[o];
        wyv = wind[g.nv + o];
      }
      sw[0][ly][lx] = wxv;
      sw[1][ly][lx] = wyv;
    }
    if constexpr (MODE == 1) {
      double fx = 0.0, fy = 0.0;
      if (f && I >= 0 && I <= top && J >= 0 && J <= top) {
        const double* fr = f + (long long)rhs * ldf;
        const long long o = (long long)J * nq + I;
        fx = fr[o];
        fy = fr[g.nv + o];
      }
      sf[0][ly][lx] = fx;
      sf[1][ly][lx] = fy;
    }
  }
  if constexpr (MODE == 0) {
    for (int k = tid; k < PX * PY; k += NT) {
      const int lx = k % PX, ly = k / PX;
      const int c = ex0 - 1 + lx, d = ey0 - 1 + ly;
      spk[ly][lx] = (c >= 0 && c <= n && d >= 0 && d <= n)
                        ? xr[g.off_pk() + (long long)d * (n + 1) + c]
                        : 0.0;
    }
    for (int k = tid; k < EX * EY; k += NT) {
      const int lx = k % EX, ly = k / EX;
      const int e = ex0 - 1 + lx, ff = ey0 - 1 + ly;
      sp0[ly][lx] = (e >= 0 && e < n && ff >= 0 && ff < n)
                        ? xr[g.off_p0() + (long long)ff * n + e]
                        : 0.0;
    }
  }
  __syncthreads();

  if constexpr (CONV) {
    // convection of every element touching the block's cells:
    // elements (ex0-1 .. ex0+TX-1) x (ey0-1 .. ey0+TY-1)
    for (int k = tid; k < (TX + 1) * (TY + 1); k += NT) {
      const int lex = k % (TX + 1), ley = k / (TX + 1);
      const int e = ex0 - 1 + lex, ff = ey0 - 1 + ley;
      if (e < 0 || e >= n || ff < 0 || ff >= n) continue;
      double ul[2][3][3], wl[2][3][3], ol[2][3][3];
      const int bx = 2 * lex, by = 2 * ley;   // local velocity index of node (2e, 2f)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            ul[c][j][i] = su[c][by + j][bx + i];
            wl[c][j][i] = sw[c][by + j][bx + i];
          }
      element_convection<TRANS>(ul, wl, g.h, ol);
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int i = 0; i < 3; ++i) sN[c][k][3 * j + i] = ol[c][j][i];
    }
    __syncthreads();
  }

  const int ex = ex0 + tx, ey = ey0 + ty;
  const double h = g.h;
  const double sA = nu / 90.0;
  const double sB = -h / 36.0, sB0 = -h / 6.0;
  const double sM = h * h / 900.0;
  double acc = 0.0;

  if (ex <= n && ey <= n) {
    // ---- velocity rows ----
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int I = 2 * ex + i, J = 2 * ey + j;
        if (I > top || J > top) continue;
        const int lx = 2 * tx + i + 2, ly = 2 * ty + j + 2;
        const long long o = (long long)J * nq + I;
        const bool bnd = (I == 0 || J == 0 || I == top || J == top);
        if (bnd) {
          if constexpr (MODE == 0) {
            yr[o] = 0.0;
            yr[g.nv + o] = 0.0;
          } else {
            yr[o] = su[0][ly][lx];
            yr[g.nv + o] = su[1][ly][lx];
          }
          continue;
        }
        double ax = 0.0, ay = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
        for (int b = -2; b <= 2; ++b) {
#pragma unroll
          for (int a = -2; a <= 2; ++a) {
            const int c = K1(i, a) * M1(j, b) + M1(i, a) * K1(j, b);
            if (c != 0) {
              ax += c * su[0][ly + b][lx + a];
              ay += c * su[1][ly + b][lx + a];
            }
            if constexpr (MODE == 1) {
              const int cm = M1(i, a) * M1(j, b);
              if (cm != 0) {
                mx += cm * sf[0][ly + b][lx + a];
                my += cm * sf[1][ly + b][lx + a];
              }
            }
          }
        }
        double vx = sA * ax, vy = sA * ay;
        if constexpr (CONV) {
          // elements containing node (2ex+i, 2ey+j): (ex-1+a', ey-1+b') for the
          // vertex parities, local index (i + 2(1-a'), j + 2(1-b'))
          double cx = 0.0, cy = 0.0;
#pragma unroll
          for (int bb = 0; bb < 2; ++bb) {
            if (j == 1 && bb == 0) continue;
#pragma unroll
            for (int aa = 0; aa < 2; ++aa) {
              if (i == 1 && aa == 0) continue;
              const int e = ex - 1 + aa, ff = ey - 1 + bb;
              if (e < 0 || e >= n || ff < 0 || ff >= n) continue;
              const int k = (ty + bb) * (TX + 1) + (tx + aa);
              const int li = i + 2 * (1 - aa), lj = j + 2 * (1 - bb);   // I - 2e, J - 2f
              cx += sN[0][k][3 * lj + li];
              cy += sN[1][k][3 * lj + li];
            }
          }
          vx += cx;
          vy += cy;
        }
        if constexpr (MODE == 0) {
          double bx = 0.0, by = 0.0, b0x = 0.0, b0y = 0.0;
#pragma unroll
          for (int dd = -1; dd <= 1; ++dd) {
#pragma unroll
            for (int dc = -1; dc <= 1; ++dc) {
              const double p = spk[ty + 1 + dd][tx + 1 + dc];
              const int cx = G6(i, dc) * Mq6(j, dd);
              const int cy = Mq6(i, dc) * G6(j, dd);
              if (cx != 0) bx += cx * p;
              if (cy != 0) by += cy * p;
            }
          }
#pragma unroll
          for (int df = -1; df <= 0; ++df) {
#pragma unroll
            for (int de = -1; de <= 0; ++de) {
              const double p = sp0[ty + 1 + df][tx + 1 + de];
              const int cx = g1(i, de) * m6(j, df);
              const int cy = m6(i, de) * g1(j, df);
              if (cx != 0) b0x += cx * p;
              if (cy != 0) b0y += cy * p;
            }
          }
          vx += sB * bx + sB0 * b0x;
          vy += sB * by + sB0 * b0y;
          yr[o] = vx;
          yr[g.nv + o] = vy;
          if constexpr (DOT) acc += vx * su[0][ly][lx] + vy * su[1][ly][lx];
        } else {
          yr[o] = sM * mx - vx;
          yr[g.nv + o] = sM * my - vy;
        }
      }
    }
    // ---- Q1 pressure row (c, d) = (ex, ey) ----
    // 1-D rows assembled from the elements that exist on each side of the
    // node (6 * G and 6/h * Mpq): left element [-1,-4,5] / [0,2,1] at offsets
    // -2..0, right element [-5,4,1] / [1,2,0] at offsets 0..2.
    {
      const int lx = 2 * tx + 2, ly = 2 * ty + 2;
      const int Lx = ex > 0, Rx = ex < n, Ly = ey > 0, Ry = ey < n;
      const double Gx[5] = {-1.0 * Lx, -4.0 * Lx, 5.0 * Lx - 5.0 * Rx, 4.0 * Rx, 1.0 * Rx};
      const double Mx[5] = {0.0, 2.0 * Lx, 1.0 * Lx + 1.0 * Rx, 2.0 * Rx, 0.0};
      const double Gy[5] = {-1.0 * Ly, -4.0 * Ly, 5.0 * Ly - 5.0 * Ry, 4.0 * Ry, 1.0 * Ry};
      const double My[5] = {0.0, 2.0 * Ly, 1.0 * Ly + 1.0 * Ry, 2.0 * Ry, 0.0};
      double s = 0.0;
#pragma unroll
      for (int q = -2; q <= 2; ++q) {
        double tx_ = 0.0, ty_ = 0.0;
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
          tx_ += Gx[o + 2] * su[0][ly + q][lx + o];
          ty_ += Mx[o + 2] * su[1][ly + q][lx + o];
        }
        s += My[q + 2] * tx_ + Gy[q + 2] * ty_;
      }
      const double v = sB * s;
      const long long o = g.off_pk() + (long long)ey * (n + 1) + ex;
      if constexpr (MODE == 0) {
        yr[o] = v;
        if constexpr (DOT) acc += v * spk[ty + 1][tx + 1];
      } else {
        yr[o] = -v;
      }
    }
    // ---- P0 pressure row (element ex, ey) ----
    if (ex < n && ey < n) {
      const int lx = 2 * tx + 2, ly = 2 * ty + 2;
      constexpr int g0[3] = {-1, 0, 1};
      constexpr int m0[3] = {1, 4, 1};
      double s = 0.0;
#pragma unroll
      for (int q = 0; q <= 2; ++q) {
#pragma unroll
        for (int o = 0; o <= 2; ++o) {
          const int cx = g0[o] * m0[q];
          const int cy = m0[o] * g0[q];
          if (cx != 0) s += cx * su[0][ly + q][lx + o];
          if (cy != 0) s += cy * su[1][ly + q][lx + o];
        }
      }
      const double v = sB0 * s;
      const long long o = g.off_p0() + (long long)ey * n + ex;
      if constexpr (MODE == 0) {
        yr[o] = v;
        if constexpr (DOT) acc += v * sp0[ty + 1][tx + 1];
      } else {
        yr[o] = -v;
      }
    }
  }
  if constexpr (DOT) {
    double vals[1] = {acc};
    reduce_and_finish<NT>(rc, rhs, blockIdx.x + gridDim.x * blockIdx.y, vals, sred);
  }
}

__global__ void k_dirichlet_lid(Geo g, double lid_u, int corner_mode, double* ub) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2LL * g.nv) return;
  const int comp = (int)(k / g.nv);
  const int o = (int)(k % g.nv);
  const int I = o % g.nq, J = o / g.nq;
  double v = 0.0;
  if (comp == 0 && J == g.nq - 1) {
    v = lid_u;
    if (corner_mode == 0 && (I == 0 || I == g.nq - 1)) v = 0.0;
    if (corner_mode == 2) {
      // regularised lid lid_u (1 - xi^4), xi in [-1, 1] across the top wall
      const double xi = 2.0 * I / (g.nq - 1) - 1.0, xi2 = xi * xi;
      v = lid_u * (1.0 - xi2 * xi2);
    }
  }
  ub[k] = v;
}

}  // namespace

int saddle_blocks(const Geo& g) { return apply_blocks(g); }

void launch_apply_stokes(const Geo& g, double nu, const double* x, double* y, long long ld,
                         int batch, Gate gate, const RedCtx* dot, hipStream_t st, ClearFlag clear) {
  launch_apply(g, nu, nullptr, 0, x, y, ld, batch, gate, dot, st, clear);
}

void launch_lift_rhs(const Geo& g, double nu, const double* wind, const double* ub,
                     const double* f, long long ldf, double* b, long long ld, int batch,
                     hipStream_t st) {
  dim3 grid((g.n + 1 + TX - 1) / TX, (g.n + 1 + TY - 1) / TY, batch);
  dim3 block(TX, TY);
  RedCtx none{};
  // every batch entry shares the same Dirichlet data: ld of the input is 0
  if (wind)
    hipLaunchKernelGGL((k_saddle<1, false, true, false>), grid, block, 0, st, g, nu, ub, 0LL, b, ld,
                       f, ldf, wind, no_gate(), none, no_clear());
  else
    hipLaunchKernelGGL((k_saddle<1, false, false, false>), grid, block, 0, st, g, nu, ub, 0LL, b, ld,
                       f, ldf, nullptr, no_gate(), none, no_clear());
  ETH_LAUNCH_CHECK();
}

void launch_apply_oseen(const Geo& g, double nu, const double* wind, int transpose,
                        const double* x, double* y, long long ld, int batch, Gate gate,
                        const RedCtx* dot, hipStream_t st, ClearFlag clear) {
  launch_apply(g, nu, wind, transpose, x, y, ld, batch, gate, dot, st, clear);
}

void launch_dirichlet_lid(const Geo& g, double lid_u, int corner_mode, double* ub,
                          hipStream_t st) {
  const long long total = 2LL * g.nv;
  hipLaunchKernelGGL(k_dirichlet_lid, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g,
                     lid_u, corner_mode, ub);
  ETH_LAUNCH_CHECK();
}

}  // namespace eth
