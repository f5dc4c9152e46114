// Flow over a step: one Chebyshev step of the pressure-mass solve (Sec. 2.3,
// Chebyshev semi-iteration based on symmetric Gauss-Seidel) in a single
// launch, the symmetric multicolour sweep temporally blocked in LDS.
//
// The solve runs on the bounding box of the step, [-1, L] x [-1, 1] (or the
// channel's [-1, L] x [0, 1]), in squares of side h: Q1 node (c, d) at
// d (ex + 1) + c, then element (e, f) at (ex + 1)(ey + 1) + f ex + e.  The
// elements e < hx, f < hy (the corner below the inflow channel) are absent,
// and so are the nodes that touch no element; their entries stay zero.  A
// node's row of M_Q sums the element matrices of its present elements:
//   (M_Q t)_a = (h^2/36) sum_b w_ab t_b + (h^2/4) sum_{present T at a} t_T,
// w = 4 P at a itself (P = number of present elements around a), 2 x (their
// number on that side) at an edge neighbour, 1 at a diagonal neighbour whose
// shared element is present; an element's row is h^2 t_T + (h^2/4) x (sum of
// its four vertex values).  The colours are those of the sparse path: the
// four parity classes (c mod 2, d mod 2) of Q1 nodes, then the elements.
//
// A block owns TQ x TQ Q1 nodes and the elements with the same lower-left
// vertex (the last block of a row or column of tiles also owns the last
// node of the box on that side); it stages a region widened by 10 nodes,
// runs the nine colour passes 0, 1, 2, 3, 4, 3, 2, 1, 0 on the whole region
// (each pass spreads stale halo values inward by one node at most), and
// forms, on what it owns,
//   s = t - z_k,  d = first ? b s : a d + b s,  z_{k+1} = z_k + d,
// which is the sparse path's step (the sweep of r - M z_k from zero, added
// to z_k) in another rounding order.  Staged nodes and elements are held in
// four arrays by the parity of their local index, so that the lanes of a
// colour pass read consecutive LDS words.
#include "eth_step.h"

namespace eth {
namespace {

__device__ __forceinline__ bool gated(const int* gate) { return gate && *gate == 0; }

constexpr int SHALO = 10;   // nine passes; even, so local and global parities agree

template <int TQ>
struct StepMqTile {
  static constexpr int RQ = TQ + 2 * SHALO;      // staged nodes per side
  static constexpr int RE = RQ - 1;              // staged elements per side
  static constexpr int QW = RQ / 2;              // entries per row of a parity array
  static constexpr int QS = QW * QW + (48 - (QW * QW) % 32) % 32;   // array stride (16 mod 32)
  static constexpr int NC = QW - 1;              // nodes per side, colour and pass
  static constexpr int FT = 64 * ((QW * QW + 63) / 64);
  static constexpr int IQ = (RQ * RQ + FT - 1) / FT;
  static constexpr int IE = (RE * RE + FT - 1) / FT;
  static_assert(TQ % 2 == 0, "parity of local and global indices must agree");
  static_assert(NC * NC <= FT && QW * QW <= FT && (TQ + 1) * (TQ + 1) <= FT,
                "one node per colour, one element per parity array and one owned node per thread");
};

template <int QW, int QS>
__device__ __forceinline__ int sidx(int x, int y) {
  return ((x & 1) + 2 * (y & 1)) * QS + (x >> 1) + (y >> 1) * QW;
}
__host__ __device__ constexpr int half_floor(int v) { return v < 0 ? -1 : v / 2; }
// offset from base hx + hy QW of a node (or element) of parity (px, py) to
// the one whose local index differs by (dx, dy)
template <int QW, int QS>
__host__ __device__ constexpr int soff(int px, int py, int dx, int dy) {
  return QS * (((px + dx) & 1) + 2 * ((py + dy) & 1)) + half_floor(px + dx) + QW * half_floor(py + dy);
}

__device__ __forceinline__ bool present(const StepBox& b, int e, int f) {
  return e >= 0 && f >= 0 && e < b.ex && f < b.ey && !(e < b.hx && f < b.hy);
}

template <typename T>
__device__ __forceinline__ T fma_s(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

// Gauss-Seidel update of a Q1 node: q9[(j+1)*3 + (i+1)] = t at node (c+i,
// d+j), e4 = t at the elements SW, SE, NW, NE of the node, m = their
// presence bits (1, 2, 4, 8), scale = 9 / (h^2 P)
template <typename T>
__device__ __forceinline__ T step_q1_update(T t, T r, const T* q9, const T* e4, int m, T h2_36, T h2_4, T scale) {
#pragma clang fp contract(off)
  const T sw = T(m & 1), se = T((m >> 1) & 1), nw = T((m >> 2) & 1), ne = T((m >> 3) & 1);
  const T two = T(2);
  T q = (T(4) * (((sw + se) + (nw + ne)))) * q9[4];
  q = fma_s(two * (sw + se), q9[1], q);
  q = fma_s(two * (nw + ne), q9[7], q);
  q = fma_s(two * (sw + nw), q9[3], q);
  q = fma_s(two * (se + ne), q9[5], q);
  q = fma_s(sw, q9[0], q);
  q = fma_s(se, q9[2], q);
  q = fma_s(nw, q9[6], q);
  q = fma_s(ne, q9[8], q);
  const T e = fma_s(ne, e4[3], fma_s(nw, e4[2], fma_s(se, e4[1], sw * e4[0])));
  const T acc = fma_s(h2_4, e, q * h2_36);
  return fma_s(r - acc, scale, t);
}

// element: t_T = r_T / h^2 - (sum of the four vertex values) / 4
template <typename T>
__device__ __forceinline__ T step_p0_update(T r, T v00, T v10, T v01, T v11, T inv_h2) {
#pragma clang fp contract(off)
  return r * inv_h2 - T(0.25) * ((v00 + v10) + (v01 + v11));
}

template <typename T, int TQ>
__global__ __launch_bounds__(StepMqTile<TQ>::FT) void k_step_mq_fused(StepBox b, const T* __restrict__ r,
                                                                      const T* __restrict__ zin,
                                                                      T* __restrict__ zout, T* d, double a,
                                                                      double bc, int first,
                                                                      const int* __restrict__ gate) {
  using Tl = StepMqTile<TQ>;
  constexpr int RQ = Tl::RQ, RE = Tl::RE, QW = Tl::QW, QS = Tl::QS, NC = Tl::NC, FT = Tl::FT, IQ = Tl::IQ,
                IE = Tl::IE;
  __shared__ T tq[4 * QS];
  __shared__ T rq[4 * QS];
  __shared__ T te[4 * QS];
  __shared__ T re[4 * QS];
  if (gated(gate)) return;
  const int ex = b.ex, ey = b.ey, nqx = ex + 1;
  const long long nq = (long long)(ex + 1) * (ey + 1);
  const int c0 = blockIdx.x * TQ, d0 = blockIdx.y * TQ;
  const bool last_x = blockIdx.x == gridDim.x - 1, last_y = blockIdx.y == gridDim.y - 1;
  const int gx = c0 - SHALO, gy = d0 - SHALO;
  const int tid = threadIdx.x;
  const T h2 = T(b.h * b.h);
  const T h2_36 = T(b.h * b.h / 36.0), h2_4 = T(0.25 * b.h * b.h), inv_h2 = T(1.0 / (b.h * b.h));

  // the owned node and element of this thread, z_k and d fetched first so
  // that their latency overlaps the staging
  const int onx = tid % (TQ + 1), ony = tid / (TQ + 1);
  const int oc = c0 + onx, od = d0 + ony;
  bool own_q = tid < (TQ + 1) * (TQ + 1) && (onx < TQ || last_x) && (ony < TQ || last_y) && oc <= ex && od <= ey;
  if (own_q)
    own_q = present(b, oc - 1, od - 1) || present(b, oc, od - 1) || present(b, oc - 1, od) || present(b, oc, od);
  const int oex = tid % TQ, oey = tid / TQ;
  const int oe = c0 + oex, of = d0 + oey;
  const bool own_e = tid < TQ * TQ && present(b, oe, of);
  const long long iq = (long long)od * nqx + oc, ie = nq + (long long)of * ex + oe;
  T zq = T(0), dq = T(0), ze = T(0), de = T(0);
  if (!first) {
    if (own_q) {
      zq = zin[iq];
      dq = d[iq];
    }
    if (own_e) {
      ze = zin[ie];
      de = d[ie];
    }
  }
  // staging: every global load of the region before the first LDS store
  {
    T tv[IQ], rv[IQ], tw[IE], rw[IE];
#pragma unroll
    for (int i = 0; i < IQ; ++i) {
      const int k = tid + i * FT;
      const int c = gx + k % RQ, dd = gy + k / RQ;
      tv[i] = rv[i] = T(0);
      if (k < RQ * RQ && c >= 0 && c <= ex && dd >= 0 && dd <= ey) {
        const long long o = (long long)dd * nqx + c;
        rv[i] = r[o];
        if (!first) tv[i] = zin[o];
      }
    }
#pragma unroll
    for (int i = 0; i < IE; ++i) {
      const int k = tid + i * FT;
      const int e = gx + k % RE, f = gy + k / RE;
      tw[i] = rw[i] = T(0);
      if (k < RE * RE && e >= 0 && e < ex && f >= 0 && f < ey) {
        const long long o = nq + (long long)f * ex + e;
        rw[i] = r[o];
        if (!first) tw[i] = zin[o];
      }
    }
#pragma unroll
    for (int i = 0; i < IQ; ++i) {
      const int k = tid + i * FT;
      if (k < RQ * RQ) {
        const int li = sidx<QW, QS>(k % RQ, k / RQ);
        tq[li] = tv[i];
        rq[li] = rv[i];
      }
    }
#pragma unroll
    for (int i = 0; i < IE; ++i) {
      const int k = tid + i * FT;
      if (k < RE * RE) {
        const int li = sidx<QW, QS>(k % RE, k / RE);
        te[li] = tw[i];
        re[li] = rw[i];
      }
    }
  }
  // the node of each colour this thread updates in every pass: base index
  // hx + hy QW | presence bits << 16 (-1: none), its right-hand side and
  // scale; the element of each parity array, its presence and right-hand side
  int qb[4];
  T qsc[4];
#pragma unroll
  for (int colour = 0; colour < 4; ++colour) {
    const int px = colour & 1, py = colour >> 1;
    const int hx = tid % NC + 1 - px, hy = tid / NC + 1 - py;
    const int c = gx + 2 * hx + px, dd = gy + 2 * hy + py;
    int m = 0;
    if (tid < NC * NC) {
      m = (present(b, c - 1, dd - 1) ? 1 : 0) | (present(b, c, dd - 1) ? 2 : 0) | (present(b, c - 1, dd) ? 4 : 0) |
          (present(b, c, dd) ? 8 : 0);
    }
    const int P = (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1) + ((m >> 3) & 1);
    qb[colour] = P > 0 ? (hx + hy * QW) | (m << 16) : -1;
    qsc[colour] = P > 0 ? T(9) / (h2 * T(P)) : T(0);
  }
  unsigned emask = 0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int qx = p & 1, qy = p >> 1;
    const int hx = tid % QW, hy = tid / QW;
    const int e = gx + 2 * hx + qx, f = gy + 2 * hy + qy;
    const bool ok = tid < QW * QW && hx < QW - qx && hy < QW - qy && present(b, e, f);
    emask |= (ok ? 1u : 0u) << p;
  }
  __syncthreads();
  T qr[4], er[4];
#pragma unroll
  for (int colour = 0; colour < 4; ++colour) {
    const int v = qb[colour];
    qr[colour] = v >= 0 ? rq[colour * QS + (v & 0xffff)] : T(0);
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) er[p] = ((emask >> p) & 1u) ? re[p * QS + tid] : T(0);

  constexpr int order[9] = {0, 1, 2, 3, 4, 3, 2, 1, 0};
#pragma unroll
  for (int pass = 0; pass < 9; ++pass) {
    const int colour = order[pass];
    if (colour < 4) {
      const int px = colour & 1, py = colour >> 1;
      const int v = qb[colour];
      if (v >= 0) {
        const int base = v & 0xffff;
        T q9[9], e4[4];
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
#pragma unroll
          for (int ii = 0; ii < 3; ++ii) q9[jj * 3 + ii] = tq[base + soff<QW, QS>(px, py, ii - 1, jj - 1)];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
          for (int ii = 0; ii < 2; ++ii) e4[jj * 2 + ii] = te[base + soff<QW, QS>(px, py, ii - 1, jj - 1)];
        tq[base + soff<QW, QS>(px, py, 0, 0)] =
            step_q1_update<T>(q9[4], qr[colour], q9, e4, (v >> 16) & 15, h2_36, h2_4, qsc[colour]);
      }
    } else {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        if (!((emask >> p) & 1u)) continue;
        const int qx = p & 1, qy = p >> 1;
        te[p * QS + tid] = step_p0_update<T>(er[p], tq[tid + soff<QW, QS>(qx, qy, 0, 0)],
                                             tq[tid + soff<QW, QS>(qx, qy, 1, 0)],
                                             tq[tid + soff<QW, QS>(qx, qy, 0, 1)],
                                             tq[tid + soff<QW, QS>(qx, qy, 1, 1)], inv_h2);
      }
    }
    __syncthreads();
  }
  // Chebyshev combination on the owned node and element
  const T ta = T(a), tb = T(bc);
  auto combine = [&](T t, T z0, T d0, long long o) {
#pragma clang fp contract(off)
    const T s = t - z0;
    const T dn = first ? tb * s : ta * d0 + tb * s;
    d[o] = dn;
    zout[o] = z0 + dn;
  };
  if (own_q) combine(tq[sidx<QW, QS>(onx + SHALO, ony + SHALO)], zq, dq, iq);
  if (own_e) combine(te[sidx<QW, QS>(oex + SHALO, oey + SHALO)], ze, de, ie);
}

}  // namespace

int step_mq_tiles(const StepBox& b, int tile) {
  return ((b.ex + tile - 1) / tile) * ((b.ey + tile - 1) / tile);
}

template <typename T>
void launch_step_mq_fused(const StepBox& b, int tile, const T* r, const T* zin, T* zout, T* d, double a,
                          double bc, int first, const int* gate, hipStream_t st) {
  if (b.ex < 1 || b.ey < 1) throw std::invalid_argument("empty step box");
#define ETH_SMQ(TQ)                                                                                        \
  hipLaunchKernelGGL((k_step_mq_fused<T, TQ>), dim3((b.ex + TQ - 1) / TQ, (b.ey + TQ - 1) / TQ),            \
                     dim3(StepMqTile<TQ>::FT), 0, st, b, r, zin, zout, d, a, bc, first, gate)
  if (tile == 8) ETH_SMQ(8);
  else if (tile == 16) ETH_SMQ(16);
  else throw std::invalid_argument("step M_Q tile must be 8 or 16");
#undef ETH_SMQ
  ETH_LAUNCH_CHECK();
}

template void launch_step_mq_fused<double>(const StepBox&, int, const double*, const double*, double*, double*,
                                           double, double, int, const int*, hipStream_t);
template void launch_step_mq_fused<float>(const StepBox&, int, const float*, const float*, float*, float*, double,
                                          double, int, const int*, hipStream_t);

}  // namespace eth
