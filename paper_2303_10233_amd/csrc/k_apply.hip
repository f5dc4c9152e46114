// The saddle-point operator apply y = K x (eq:saddle_point; Oseen
// eq:oseen-system) in node-parallel form, FP64.
//
// A block of 64 x 4 threads owns a tile of 64 x 16 velocity nodes (lanes
// run along x, so every global load and store is a contiguous 512-byte
// segment), the 32 x 8 Q1 nodes and elements whose lower-left vertex lies in
// it.  The velocity patch (halo 2), the Q1 patch and the P0 patch are staged
// in LDS.
//
// Velocity rows use the tensor structure A = K (x) M + M (x) K of the Q2
// Laplacian (assembled 1-D rows, vertex (1/(3h))[1,-8,14,-8,1] and
// (h/30)[-1,2,8,2,-1], mid (1/(3h))[-8,16,-8] and (h/30)[2,16,2]): a thread
// owns one column of four consecutive rows; it forms the x-direction sums
// sum_a K(I,a) u and sum_a M(I,a) u for the eight rows its outputs touch and
// combines them along y in registers -- 20 LDS reads per node and component
// instead of the 25-point stencil.  B^T p, the Q1 rows of B u and the P0 rows
// follow the same 1-D factors as the element matrices (see k_saddle.hip).
// Oseen adds the element convection N(w) (or N(w)^T), integrated per element
// in LDS by sum factorisation and gathered per node.
#include "eth_fem.h"
#include "eth_kernels.h"
#include "eth_reduce.h"

namespace eth {
namespace {

constexpr int AX = 64, AY = 4, RPT = 4;        // threads (x, y); rows per thread
constexpr int TYN = AY * RPT;                  // 16 velocity rows per tile
constexpr int NTA = AX * AY;
static_assert(RPT % 2 == 0, "rows 2m and 2m+1 of a thread share their pressure rows");
constexpr int UX = AX + 4, UY = TYN + 4;       // velocity patch with halo 2
constexpr int QX = AX / 2 + 2, QY = TYN / 2 + 2;   // Q1 nodes c0-1 .. c0+AX/2
constexpr int EXP = AX / 2 + 1, EYP = TYN / 2 + 1;  // elements c0-1 .. c0+AX/2-1

__device__ __forceinline__ double k1c(int p, int a) { return (double)K1(p, a); }
__device__ __forceinline__ double m1c(int p, int a) { return (double)M1(p, a); }

// 6 G, 6/h Mpq, g0, 6/h m0 factors of B for a velocity node of parity i (as in k_saddle)
__device__ __forceinline__ double G6(int i, int dc) {
  return i == 0 ? (dc == -1 ? 1.0 : dc == 0 ? 0.0 : -1.0) : (dc == -1 ? 0.0 : dc == 0 ? 4.0 : -4.0);
}
__device__ __forceinline__ double Mq6(int j, int dd) {
  return j == 0 ? (dd == 0 ? 2.0 : 0.0) : (dd == -1 ? 0.0 : 2.0);
}
__device__ __forceinline__ double g1(int i, int de) { return i == 0 ? (de == -1 ? 1.0 : -1.0) : 0.0; }
__device__ __forceinline__ double m6(int j, int df) { return j == 0 ? 1.0 : (df == -1 ? 0.0 : 4.0); }

template <bool DOT, bool CONV, bool TRANS>
__global__ __launch_bounds__(NTA) void k_apply(Geo g, double nu, const double* __restrict__ x,
                                               double* __restrict__ y, long long ld,
                                               const double* __restrict__ wind, Gate gate, RedCtx rc,
                                               ClearFlag clear, int remap_min) {
  __shared__ double su[2][UY][UX];
  __shared__ double sw[CONV ? 2 : 1][CONV ? UY : 1][CONV ? UX : 1];
  __shared__ double sc[CONV ? 2 : 1][CONV ? UY : 1][CONV ? UX : 1];   // N(w) u (or N(w)^T u) per patch node
  __shared__ double spk[QY][QX];
  __shared__ double sp0[EYP][EXP];
  __shared__ double sred[NTA / 64];

  const int rhs = blockIdx.z;
  clear.apply(rhs);
  const bool off = gate.off(rhs);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * AX + tx;
  // large grids in XCD band order (vertically neighbouring tiles share two
  // halo rows; within a band those stay in the XCD's own L2)
  int tile_x, tile_y;
  xcd_band_tile(remap_min, tile_x, tile_y);
  const int I0 = tile_x * AX, J0 = tile_y * TYN;
  const int c0 = I0 / 2, d0 = J0 / 2;
  const int n = g.n, nq = g.nq, top = 2 * n;
  const double* xr = x + (long long)rhs * ld;
  double* yr = y + (long long)rhs * ld;

  // ---- stage the patches (boundary velocity masked); all loads in flight ----
  stage2<NTA, UX * UY>(&su[0][0][0], &su[1][0][0], tid, [&](int k, double& vx, double& vy) {
    const int I = I0 - 2 + k % UX, J = J0 - 2 + k / UX;
    if (I >= 1 && I < top && J >= 1 && J < top) {
      const long long o = (long long)J * nq + I;
      vx = xr[o];
      vy = xr[g.nv + o];
    }
  });
  if constexpr (CONV) {
    stage2<NTA, UX * UY>(&sw[0][0][0], &sw[1][0][0], tid, [&](int k, double& w0, double& w1) {
      const int I = I0 - 2 + k % UX, J = J0 - 2 + k / UX;
      if (I >= 0 && I <= top && J >= 0 && J <= top) {
        const long long o = (long long)J * nq + I;
        w0 = wind[o];
        w1 = wind[g.nv + o];
      }
    });
  }
  stage1<NTA, QX * QY>(&spk[0][0], tid, [&](int k, double& v) {
    const int c = c0 - 1 + k % QX, d = d0 - 1 + k / QX;
    if (c >= 0 && c <= n && d >= 0 && d <= n) v = xr[g.off_pk() + (long long)d * (n + 1) + c];
  });
  stage1<NTA, EXP * EYP>(&sp0[0][0], tid, [&](int k, double& v) {
    const int e = c0 - 1 + k % EXP, f = d0 - 1 + k / EXP;
    if (e >= 0 && e < n && f >= 0 && f < n) v = xr[g.off_p0() + (long long)f * n + e];
  });
  if constexpr (CONV) {
    for (int k = tid; k < 2 * UY * UX; k += NTA) (&sc[0][0][0])[k] = 0.0;
  }
  if (off) return;   // uniform per block; the gate load overlapped the staging loads
  __syncthreads();

  if constexpr (CONV) {
    // elements (c0-1 .. c0+AX/2-1) x (d0-1 .. d0+TYN/2-1) in four classes by
    // the parity of their local index: elements of one class share no node,
    // so each adds its nine values to the node accumulator without conflict,
    // and the classes follow one another (a fixed summation order per node).
    // One thread per element and velocity component.
#pragma unroll 1
    for (int cl = 0; cl < 4; ++cl) {
      const int qx = cl & 1, qy = cl >> 1;
      const int cxn = (EXP - qx + 1) / 2, cyn = (EYP - qy + 1) / 2, cnt = cxn * cyn;
      for (int m = tid; m < 2 * cnt; m += NTA) {
        const int c = m / cnt, idx = m % cnt;
        const int lex = qx + 2 * (idx % cxn), ley = qy + 2 * (idx / cxn);
        const int e = c0 - 1 + lex, f = d0 - 1 + ley;
        if (e < 0 || e >= n || f < 0 || f >= n) continue;
        const int bx = 2 * lex, by = 2 * ley;   // local index of node (2e, 2f)
        double wl[2][3][3], ul[3][3], ol[3][3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            wl[0][j][i] = sw[0][by + j][bx + i];
            wl[1][j][i] = sw[1][by + j][bx + i];
            ul[j][i] = su[c][by + j][bx + i];
          }
        element_convection1<double, double, TRANS>(ul, wl, g.h, ol);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
          for (int i = 0; i < 3; ++i) sc[c][by + j][bx + i] += ol[j][i];
      }
      __syncthreads();
    }
  }

  const double h = g.h;
  const double sA = nu / 90.0, sB = -h / 36.0, sB0 = -h / 6.0;
  double acc = 0.0;

  // ---- velocity rows: column I, rows J0 + RPT*ty .. +RPT-1 ----
  {
    const int I = I0 + tx;
    const int pi = I & 1;
    const int lx = tx + 2;
    const int lr0 = RPT * ty;   // local patch row of the first x-sum row (= output row - 2)
    double kc[5], mc[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      kc[a] = pi ? k1c(1, a - 2) : k1c(0, a - 2);
      mc[a] = pi ? m1c(1, a - 2) : m1c(0, a - 2);
    }
    double tK[2][RPT + 4], tM[2][RPT + 4];
    // x-direction sums of patch row lr0 + r, formed just before first use
    // so that few of them are live at once
    auto xsums = [&](int r) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double sk = 0.0, sm = 0.0;
#pragma unroll
        for (int a = 0; a < 5; ++a) {
          const double u = su[c][lr0 + r][lx + a - 2];
          sk += kc[a] * u;
          sm += mc[a] * u;
        }
        tK[c][r] = sk;
        tM[c][r] = sm;
      }
    };
#pragma unroll
    for (int r = 0; r < 4; ++r) xsums(r);
    const int ex = I >> 1, lq = ex - (c0 - 1);   // local Q1 / element column of the node
    double pq[3][3], pz[2][2];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      xsums(r + 4);
      const int J = J0 + lr0 + r;
      // rows 2m and 2m+1 share ey = J / 2 (J0 + lr0 is a multiple of 4):
      // their Q1 rows ey-1..ey+1 and P0 rows ey-1, ey are copied once (in
      // the patches whatever J is)
      const int lqy = (J >> 1) - (d0 - 1);
      if ((r & 1) == 0) {
#pragma unroll
        for (int dd = 0; dd < 3; ++dd)
#pragma unroll
          for (int dc = 0; dc < 3; ++dc) pq[dd][dc] = spk[lqy + dd - 1][lq + dc - 1];
#pragma unroll
        for (int df = 0; df < 2; ++df)
#pragma unroll
          for (int de = 0; de < 2; ++de) pz[df][de] = sp0[lqy + df - 1][lq + de - 1];
      }
      if (I > top || J > top) continue;
      const long long o = (long long)J * nq + I;
      if (I == 0 || J == 0 || I == top || J == top) {
        yr[o] = 0.0;
        yr[g.nv + o] = 0.0;
        continue;
      }
      const int pj = J & 1;
      double vx = 0.0, vy = 0.0;
#pragma unroll
      for (int b = 0; b < 5; ++b) {
        const double mb = pj ? m1c(1, b - 2) : m1c(0, b - 2);
        const double kb = pj ? k1c(1, b - 2) : k1c(0, b - 2);
        vx += mb * tK[0][r + b] + kb * tM[0][r + b];
        vy += mb * tK[1][r + b] + kb * tM[1][r + b];
      }
      vx *= sA;
      vy *= sA;
      // B^T p: Q1 part (rows ey-1..ey+1 of the Q1 patch) and P0 part
      double bx = 0.0, by = 0.0;
#pragma unroll
      for (int dd = -1; dd <= 1; ++dd)
#pragma unroll
        for (int dc = -1; dc <= 1; ++dc) {
          const double p = pq[dd + 1][dc + 1];
          bx += G6(pi, dc) * Mq6(pj, dd) * p;
          by += Mq6(pi, dc) * G6(pj, dd) * p;
        }
      double b0x = 0.0, b0y = 0.0;
#pragma unroll
      for (int df = -1; df <= 0; ++df)
#pragma unroll
        for (int de = -1; de <= 0; ++de) {
          const double p = pz[df + 1][de + 1];
          b0x += g1(pi, de) * m6(pj, df) * p;
          b0y += m6(pi, de) * g1(pj, df) * p;
        }
      vx += sB * bx + sB0 * b0x;
      vy += sB * by + sB0 * b0y;
      if constexpr (CONV) {
        vx += sc[0][lr0 + r + 2][lx];
        vy += sc[1][lr0 + r + 2][lx];
      }
      yr[o] = vx;
      yr[g.nv + o] = vy;
      if constexpr (DOT) acc += vx * su[0][lr0 + r + 2][lx] + vy * su[1][lr0 + r + 2][lx];
    }
  }

  // ---- Q1 rows and P0 rows: node / element (c0 + qc, d0 + qd) ----
  {
    const int qc = tid % (AX / 2), qd = tid / (AX / 2);   // 32 x 8
    const int c = c0 + qc, d = d0 + qd;
    const int lx = 2 * qc + 2, ly = 2 * qd + 2;   // velocity node (2c, 2d) in the patch
    if (c <= n && d <= n) {
      const int Lx = c > 0, Rx = c < n, Ly = d > 0, Ry = d < n;
      const double Gx[5] = {-1.0 * Lx, -4.0 * Lx, 5.0 * Lx - 5.0 * Rx, 4.0 * Rx, 1.0 * Rx};
      const double Mx[5] = {0.0, 2.0 * Lx, 1.0 * Lx + 1.0 * Rx, 2.0 * Rx, 0.0};
      const double Gy[5] = {-1.0 * Ly, -4.0 * Ly, 5.0 * Ly - 5.0 * Ry, 4.0 * Ry, 1.0 * Ry};
      const double My[5] = {0.0, 2.0 * Ly, 1.0 * Ly + 1.0 * Ry, 2.0 * Ry, 0.0};
      constexpr double g0[3] = {-1.0, 0.0, 1.0};
      constexpr double m0[3] = {1.0, 4.0, 1.0};
      // the P0 row of element (c, d) reads the 3 x 3 corner of the Q1 row's
      // 5 x 5 window: both come from one pass over the window's rows
      double s = 0.0, s0 = 0.0;
#pragma unroll
      for (int q = -2; q <= 2; ++q) {
        double u0[5], u1[5];
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
          u0[o + 2] = su[0][ly + q][lx + o];
          u1[o + 2] = su[1][ly + q][lx + o];
        }
        double a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
          a1 += Gx[o + 2] * u0[o + 2];
          a2 += Mx[o + 2] * u1[o + 2];
        }
        s += My[q + 2] * a1 + Gy[q + 2] * a2;
        if (q >= 0) {
#pragma unroll
          for (int o = 0; o <= 2; ++o) s0 += g0[o] * m0[q] * u0[o + 2] + m0[o] * g0[q] * u1[o + 2];
        }
      }
      const double v = sB * s;
      yr[g.off_pk() + (long long)d * (n + 1) + c] = v;
      if constexpr (DOT) acc += v * spk[qd + 1][qc + 1];
      if (c < n && d < n) {
        const double v0 = sB0 * s0;
        yr[g.off_p0() + (long long)d * n + c] = v0;
        if constexpr (DOT) acc += v0 * sp0[qd + 1][qc + 1];
      }
    }
  }
  if constexpr (DOT) {
    double vals[1] = {acc};
    reduce_and_finish<NTA>(rc, rhs, blockIdx.x + gridDim.x * blockIdx.y, vals, sred);
  }
}

inline dim3 apply_grid(const Geo& g, int batch) {
  return dim3((g.nq + AX - 1) / AX, (g.nq + TYN - 1) / TYN, batch);
}

}  // namespace

int apply_blocks(const Geo& g) {
  const dim3 gr = apply_grid(g, 1);
  return (int)(gr.x * gr.y);
}

void launch_apply(const Geo& g, double nu, const double* wind, int transpose, const double* x, double* y,
                  long long ld, int batch, Gate gate, const RedCtx* dot, hipStream_t st, ClearFlag clear) {
  RedCtx rc{};
  if (dot) {
    rc = *dot;
    rc.nblocks = apply_blocks(g);
  }
  const dim3 grid = apply_grid(g, batch), block(AX, AY);
  const int remap = xcd_remap_min();
#define ETH_APPLY(D, C, T)                                                                        \
  hipLaunchKernelGGL((k_apply<D, C, T>), grid, block, 0, st, g, nu, x, y, ld, wind, gate, rc, clear, remap)
  if (!wind) {
    if (dot) ETH_APPLY(true, false, false);
    else ETH_APPLY(false, false, false);
  } else if (!transpose) {
    if (dot) ETH_APPLY(true, true, false);
    else ETH_APPLY(false, true, false);
  } else {
    if (dot) ETH_APPLY(true, true, true);
    else ETH_APPLY(false, true, true);
  }
#undef ETH_APPLY
  ETH_LAUNCH_CHECK();
  if (dot) launch_reduce_finish(rc, batch, gate, st);
}

}  // namespace eth
