// Device-side finite-element helpers shared by the operator kernels:
// assembled 1-D Q2 stencils on a uniform grid, a 4-point Gauss rule with the
// 1-D Q2 basis values, and element-level convection by sum factorisation.
#pragma once
#include <hip/hip_runtime.h>

namespace eth {

// Assembled 1-D Q2 rows (node parity p: 0 vertex, 1 mid), offsets o in -2..2:
// stiffness (1/(3h)) K1, mass (h/30) M1.
__host__ __device__ constexpr inline int K1(int p, int o) {
  return p == 0 ? (o == 0 ? 14 : (o == -1 || o == 1) ? -8 : 1)
                : (o == 0 ? 16 : (o == -1 || o == 1) ? -8 : 0);
}
__host__ __device__ constexpr inline int M1(int p, int o) {
  return p == 0 ? (o == 0 ? 8 : (o == -1 || o == 1) ? 2 : -1)
                : (o == 0 ? 16 : (o == -1 || o == 1) ? 2 : 0);
}
// 4-point Gauss-Legendre rule on [0,1] and the 1-D Q2 basis / derivative
// values at its points: GB[q][i] = phi_i(xi_q), GD[q][i] = phi_i'(xi_q).
constexpr int NG = 4;
__device__ __forceinline__ void gauss_tables(double* W, double (*GB)[3], double (*GD)[3]) {
  const double t1 = 0.33998104358485626480, t2 = 0.86113631159405257522;
  const double w1 = 0.65214515486254614263, w2 = 0.34785484513745385737;
  const double xq[NG] = {0.5 * (1 - t2), 0.5 * (1 - t1), 0.5 * (1 + t1), 0.5 * (1 + t2)};
  W[0] = 0.5 * w2;
  W[1] = 0.5 * w1;
  W[2] = 0.5 * w1;
  W[3] = 0.5 * w2;
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const double t = xq[q];
    GB[q][0] = (1 - t) * (1 - 2 * t);
    GB[q][1] = 4 * t * (1 - t);
    GB[q][2] = t * (2 * t - 1);
    GD[q][0] = 4 * t - 3;
    GD[q][1] = 4 - 8 * t;
    GD[q][2] = 4 * t - 1;
  }
}

// Convection on one element, both velocity components, 4x4 Gauss: exact for
// any Q2 wind (the integrand w phi_i d(phi_j) has degree <= 6 per direction).
//   TRANS = false: out_i = int (w . grad u_h) phi_i       (N u)
//   TRANS = true : out_i = int (w . grad phi_i) u_h       (N^T u)
// u[c][j][i], w[c][j][i]: local nodal values (x index i); out[c][j][i].
template <bool TRANS>
__device__ inline void element_convection(const double (*u)[3][3], const double (*w)[3][3], double h,
                                          double (*out)[3][3]) {
  double W[NG], GB[NG][3], GD[NG][3];
  gauss_tables(W, GB, GD);
  double wq[2][NG][NG];   // wind at the Gauss points [comp][qy][qx]
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int qy = 0; qy < NG; ++qy)
#pragma unroll
      for (int qx = 0; qx < NG; ++qx) {
        double a = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double t = 0.0;
#pragma unroll
          for (int i = 0; i < 3; ++i) t += GB[qx][i] * w[c][j][i];
          a += GB[qy][j] * t;
        }
        wq[c][qy][qx] = a;
      }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if constexpr (!TRANS) {
      double cv[NG][NG];
#pragma unroll
      for (int qy = 0; qy < NG; ++qy)
#pragma unroll
        for (int qx = 0; qx < NG; ++qx) {
          double ux = 0.0, uy = 0.0;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            double tx = 0.0, ty = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              tx += GD[qx][i] * u[c][j][i];
              ty += GB[qx][i] * u[c][j][i];
            }
            ux += GB[qy][j] * tx;
            uy += GD[qy][j] * ty;
          }
          cv[qy][qx] = W[qx] * W[qy] * (wq[0][qy][qx] * ux + wq[1][qy][qx] * uy);
        }
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          double a = 0.0;
#pragma unroll
          for (int qy = 0; qy < NG; ++qy) {
            double t = 0.0;
#pragma unroll
            for (int qx = 0; qx < NG; ++qx) t += GB[qx][i] * cv[qy][qx];
            a += GB[qy][j] * t;
          }
          out[c][j][i] = h * a;
        }
    } else {
      double gx[NG][NG], gy[NG][NG];
#pragma unroll
      for (int qy = 0; qy < NG; ++qy)
#pragma unroll
        for (int qx = 0; qx < NG; ++qx) {
          double uv = 0.0;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) t += GB[qx][i] * u[c][j][i];
            uv += GB[qy][j] * t;
          }
          const double wu = W[qx] * W[qy] * uv;
          gx[qy][qx] = wq[0][qy][qx] * wu;
          gy[qy][qx] = wq[1][qy][qx] * wu;
        }
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          double a = 0.0;
#pragma unroll
          for (int qy = 0; qy < NG; ++qy) {
            double tx = 0.0, ty = 0.0;
#pragma unroll
            for (int qx = 0; qx < NG; ++qx) {
              tx += GD[qx][i] * gx[qy][qx];
              ty += GB[qx][i] * gy[qy][qx];
            }
            a += GB[qy][j] * tx + GD[qy][j] * ty;
          }
          out[c][j][i] = h * a;
        }
    }
  }
}


// Convection on one element for ONE velocity component:
//   TRANS = false: out_i = int (w . grad u_h) phi_i   (N u)
//   TRANS = true : out_i = int (w . grad phi_i) u_h   (N^T u)
// by sum factorisation over the 4 x 4 Gauss points (x first, then y), in the
// arithmetic type C (FP32 inside the mixed-precision smoother).
template <typename C, typename TW, bool TRANS = false>
__device__ inline void element_convection1(const C (*u)[3], const TW (*w)[3][3], C h, C (*out)[3]) {
  double Wd[NG], GBd[NG][3], GDd[NG][3];
  gauss_tables(Wd, GBd, GDd);
  C W[NG], GB[NG][3], GD[NG][3];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    W[q] = (C)Wd[q];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      GB[q][i] = (C)GBd[q][i];
      GD[q][i] = (C)GDd[q][i];
    }
  }
  // along x: row j of the element at Gauss abscissa qx
  C wx1[3][NG], wy1[3][NG], ud1[3][NG], ub1[3][NG];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int qx = 0; qx < NG; ++qx) {
      C a = 0, b = 0, c = 0, d = 0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        a += GB[qx][i] * (C)w[0][j][i];
        b += GB[qx][i] * (C)w[1][j][i];
        c += GD[qx][i] * u[j][i];
        d += GB[qx][i] * u[j][i];
      }
      wx1[j][qx] = a;
      wy1[j][qx] = b;
      ud1[j][qx] = c;
      ub1[j][qx] = d;
    }
  // along y: the Gauss point values, weighted
  C c0[NG][NG], c1[NG][NG];
#pragma unroll
  for (int qy = 0; qy < NG; ++qy)
#pragma unroll
    for (int qx = 0; qx < NG; ++qx) {
      C wx = 0, wy = 0, ux = 0, uy = 0, uv = 0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        wx += GB[qy][j] * wx1[j][qx];
        wy += GB[qy][j] * wy1[j][qx];
        if constexpr (!TRANS) {
          ux += GB[qy][j] * ud1[j][qx];
          uy += GD[qy][j] * ub1[j][qx];
        } else {
          uv += GB[qy][j] * ub1[j][qx];
        }
      }
      const C ww = W[qx] * W[qy];
      if constexpr (!TRANS) {
        c0[qy][qx] = ww * (wx * ux + wy * uy);
      } else {
        c0[qy][qx] = ww * wx * uv;   // pairs with d(phi_i)/dx
        c1[qy][qx] = ww * wy * uv;   // pairs with d(phi_i)/dy
      }
    }
  // test functions: x first, then y
  C s0[NG][3], s1[NG][3];
#pragma unroll
  for (int qy = 0; qy < NG; ++qy)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      C a = 0, b = 0;
#pragma unroll
      for (int qx = 0; qx < NG; ++qx) {
        if constexpr (!TRANS) {
          a += GB[qx][i] * c0[qy][qx];
        } else {
          a += GD[qx][i] * c0[qy][qx];
          b += GB[qx][i] * c1[qy][qx];
        }
      }
      s0[qy][i] = a;
      s1[qy][i] = b;
    }
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      C a = 0;
#pragma unroll
      for (int qy = 0; qy < NG; ++qy) {
        if constexpr (!TRANS) a += GB[qy][j] * s0[qy][i];
        else a += GB[qy][j] * s0[qy][i] + GD[qy][j] * s1[qy][i];
      }
      out[j][i] = h * a;
    }
}

}  // namespace eth
