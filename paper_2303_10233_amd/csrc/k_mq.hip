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

#include <stdexcept>

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


// Gauss-Seidel update of one Q1 coefficient of M_Q t = r, in the storage
// precision T.  tq9[(b+1)*3 + (a+1)] = t at Q1 node (c+a, d+b), te4[(b+1)*2 +
// (a+1)] = t at element (c+a, d+b) (a, b in {-1, 0}); L*/R* flag whether the
// node has a left/right (lower/upper) element column (row).
//   (M_Q t)_a = (h^2/36) sum w_x w_y t + (h^2/4) sum_{elements} t_0,
//   D_aa = h^2 m_x m_y / 9  with m = number of adjacent element columns/rows.
// The inverse diagonal factor inv_h2_9 / (m_x m_y) of a node, with m_x = Lx +
// Rx and m_y = Ly + Ry: a division, formed once per node where the node is
// updated in many passes.
template <typename T>
__device__ __forceinline__ T q1_gs_scale(int Lx, int Rx, int Ly, int Ry, T inv_h2_9) {
  return inv_h2_9 / T((Lx + Rx) * (Ly + Ry));
}
template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}
template <typename T>
__device__ __forceinline__ T q1_gs_update_s(T t, T r, const T* tq9, const T* te4, int Lx, int Rx,
                                            int Ly, int Ry, T h2_36, T h2_4, T scale) {
  // every fused multiply-add is written out (and no other contraction is
  // allowed), so the fused and the per-colour kernels round alike
#pragma clang fp contract(off)
  const T wx0 = T(Lx), wx1 = T(2 * (Lx + Rx)), wx2 = T(Rx);
  const T wy0 = T(Ly), wy1 = T(2 * (Ly + Ry)), wy2 = T(Ry);
  const T s0 = fma_t(wx2, tq9[2], fma_t(wx1, tq9[1], wx0 * tq9[0]));
  const T s1 = fma_t(wx2, tq9[5], fma_t(wx1, tq9[4], wx0 * tq9[3]));
  const T s2 = fma_t(wx2, tq9[8], fma_t(wx1, tq9[7], wx0 * tq9[6]));
  const T qk = fma_t(wy2, s2, fma_t(wy1, s1, wy0 * s0)) * h2_36;
  const T e = fma_t(te4[1], T(Rx * Ly), te4[0] * T(Lx * Ly)) + fma_t(te4[3], T(Rx * Ry), te4[2] * T(Lx * Ry));
  const T acc = fma_t(h2_4, e, qk);
  return fma_t(r - acc, scale, t);
}
template <typename T>
__device__ __forceinline__ T q1_gs_update(T t, T r, const T* tq9, const T* te4, int Lx, int Rx,
                                          int Ly, int Ry, T h2_36, T h2_4, T inv_h2_9) {
  return q1_gs_update_s<T>(t, r, tq9, te4, Lx, Rx, Ly, Ry, h2_36, h2_4,
                           q1_gs_scale<T>(Lx, Rx, Ly, Ry, inv_h2_9));
}

// Gauss-Seidel update of one element coefficient: t_0 = r_0/h^2 - (sum of
// the four vertex values)/4
template <typename T>
__device__ __forceinline__ T p0_gs_update(T r, T v00, T v10, T v01, T v11, T inv_h2) {
#pragma clang fp contract(off)
  return r * inv_h2 - T(0.25) * ((v00 + v10) + (v01 + v11));
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
    const int Lx = (c > 0), Rx = (c < n), Ly = (d > 0), Ry = (d < n);
    T q9[9], e4[4];
#pragma unroll
    for (int b = -1; b <= 1; ++b)
#pragma unroll
      for (int a = -1; a <= 1; ++a) {
        const int cc = c + a, dd = d + b;
        q9[(b + 1) * 3 + (a + 1)] =
            (cc >= 0 && cc <= n && dd >= 0 && dd <= n) ? tk[(long long)dd * (n + 1) + cc] : T(0);
      }
#pragma unroll
    for (int b = -1; b <= 0; ++b)
#pragma unroll
      for (int a = -1; a <= 0; ++a) {
        const int ex = c + a, ey = d + b;
        e4[(b + 1) * 2 + (a + 1)] =
            (ex >= 0 && ex < n && ey >= 0 && ey < n) ? t0[(long long)ey * n + ex] : T(0);
      }
    const long long i = (long long)d * (n + 1) + c;
    tk[i] = q1_gs_update<T>(tk[i], rr[i], q9, e4, Lx, Rx, Ly, Ry, T(h2 / 36.0), T(0.25 * h2),
                            T(9.0 / h2));
  } else {
    const int ex = blockIdx.x * blockDim.x + threadIdx.x;
    const int ey = blockIdx.y * blockDim.y + threadIdx.y;
    if (ex >= n || ey >= n) return;
    const long long q = (long long)ey * (n + 1) + ex;
    const long long e = (long long)ey * n + ex;
    tk[g.nk + e] = p0_gs_update<T>(rr[g.nk + e], tk[q], tk[q + 1], tk[q + n + 1], tk[q + n + 2],
                                   T(1.0 / h2));
  }
}

// Chebyshev combination of one entry: s = t - z0, d = first ? b s : a d + b s;
// returns z0 + d (the new d in dn)
template <typename T>
__device__ __forceinline__ T cheb_combine(T t, T z0, T d, T a, T b, int first, T& dn) {
#pragma clang fp contract(off)
  const T sv = t - z0;
  dn = first ? b * sv : a * d + b * sv;
  return z0 + dn;
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
  const T ta = T(a), tb = T(b);
  const T z0 = first ? T(0) : z[o];
  T dn;
  const T zn = cheb_combine<T>(t[o], z0, first ? T(0) : d[o], ta, tb, first, dn);
  d[o] = dn;
  z[o] = zn;
  t[o] = zn;
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


// ---------------------------------------------------------------------------
// One Chebyshev step of the pressure-mass solve in a single launch: the
// symmetric multicolour Gauss-Seidel sweep from z_k (colours 0,1,2,3,4,3,2,1,0)
// is temporally blocked in LDS.  A block owns TQ x TQ Q1 nodes and the
// elements with the same lower-left vertex (the last block of a row or column
// of tiles also owns node n of its rows or columns: its halo on that side
// lies outside the mesh, so the grid is ceil(n / TQ) blocks per side, 16 x 16
// = one per CU for n = 256 and TQ = 16); it stages a region widened by
// HALO nodes, runs the nine colour passes on the whole region (each pass can
// spread stale halo values inward by one node at most, so the owned part is
// exact after nine passes) and then forms
//   s = t - z_k,  d = first ? b s : a d + b s,  z_{k+1} = z_k + d.
// ST = 2 runs two Chebyshev steps per launch on a region widened by 20: the
// first combination is formed on the whole region (z_k and d held in
// registers per staged node), the second sweep starts from it, and the
// owned part is exact after eighteen passes.
// The tile side TQ (8, 16, 24, 32 or 64) and ST are chosen per problem by timing the
// candidates at set-up: small meshes want many blocks, large meshes less
// halo (the redundancy is ((TQ + 2 HALO) / TQ)^2 per launch).
// Node updates share q1_gs_update / p0_gs_update with the per-colour kernel,
// so every tile size gives the bit-identical sweep.
// ---------------------------------------------------------------------------
constexpr int HALO1 = 10;   // halo of one step (nine passes), even
static_assert(HALO1 % 2 == 0, "parity of local and global indices must agree");

// LDS layout: the staged nodes (and elements) are split into four arrays by
// the parity of their local (x, y) index, each row-major with QW = RQ / 2
// entries per row.  A colour pass then reads and writes consecutive entries
// of each array from consecutive lanes (no bank conflicts, where a row-major
// layout has every lane of a pass on even or on odd banks), and the offsets
// of the nine neighbours and four elements of a node are constants of the
// colour.  The arrays start QS apart, QS = 16 (mod 32), so that lanes that
// alternate between two of them (the element pass) hit different banks.
template <int TQ, int ST = 1>
struct MqTile {
  static constexpr int HALO = HALO1 * ST;
  static constexpr int RQ = TQ + 2 * HALO;        // staged Q1 nodes per side (even)
  static constexpr int RE = RQ - 1;               // staged elements per side
  static constexpr int QW = RQ / 2;               // entries per row of a parity array
  static constexpr int QS = QW * QW + (48 - (QW * QW) % 32) % 32;   // array stride
  static constexpr int NC = QW - 1;               // colour nodes per side and pass
  // threads: one per entry of a parity array where that fits a block (so a
  // colour pass and each quarter of the element pass take one round)
  static constexpr int FT = TQ >= 32 ? 1024 : 64 * ((QW * QW + 63) / 64);
  static constexpr int OWN = (TQ * TQ + FT - 1) / FT;   // owned nodes per thread
  // right-hand sides of the thread's nodes kept in registers across passes
  // and z_k, d of its owned nodes fetched before the sweep (TQ = 64 reads
  // them when needed: two nodes per colour, eight elements and four owned
  // nodes per thread would exceed the register budget of 1024 threads)
  static constexpr bool CACHE_R = TQ <= 32;
  static_assert(TQ % 2 == 0, "parity of local and global indices must agree");
  static_assert(QS % 32 == 16, "parity arrays must start on opposite bank halves");
  static_assert(ST == 1 || TQ == 16 || TQ == 24, "two steps per launch: 16 x 16 or 24 x 24 tiles (and FP32)");
};

// index in the parity arrays of local node (or element) (x, y)
template <int QW, int QS>
__device__ __forceinline__ int par_idx(int x, int y) {
  return ((x & 1) + 2 * (y & 1)) * QS + (x >> 1) + (y >> 1) * QW;
}
// floor(v / 2) for v in {-1, 0, 1, 2}
__host__ __device__ constexpr int fl2(int v) { return v < 0 ? -1 : v / 2; }
// offset from the base hx + hy*QW of a node of parity (px, py) to the node
// (or element) whose local index differs by (dx, dy)
template <int QW, int QS>
__host__ __device__ constexpr int par_off(int px, int py, int dx, int dy) {
  return QS * (((px + dx) & 1) + 2 * ((py + dy) & 1)) + fl2(px + dx) + QW * fl2(py + dy);
}

// src (first step only, may be null): take r from the FP64 vectors, projected
// on k^perp as r - coef k (coef null: as it is), and store it to the workspace r (owned entries) for
// the later steps.  sink (last step only, may be null): write scale z_{k+1}
// straight to the pressure part of the FP64 vectors instead of the workspace.
// din / dout: the Chebyshev direction d before and after (the same array for
// ST = 1, where a block touches only its owned entries; two arrays for ST = 2,
// which reads d over its whole region).
template <typename T, int TQ, int ST>
__global__ __launch_bounds__((MqTile<TQ, ST>::FT)) void k_mq_cheb_fused(Geo g, T* __restrict__ r,
                                                                      const T* __restrict__ zin,
                                                                      T* __restrict__ zout, const T* din,
                                                                      T* dout, double a, double b, double a2,
                                                                      double b2, int first, Gate gate,
                                                                      MqSource src, MqSink sink) {
  using Tl = MqTile<TQ, ST>;
  constexpr int RQ = Tl::RQ, RE = Tl::RE, QW = Tl::QW, QS = Tl::QS, NC = Tl::NC, FT = Tl::FT,
                OWN = Tl::OWN, HALO = Tl::HALO;
  __shared__ T tq[4 * QS];
  __shared__ T rq[4 * QS];
  __shared__ T te[4 * QS];
  __shared__ T re[4 * QS];
  // the pressure solve is the longer of the two concurrent preconditioner
  // branches: its waves issue first on a SIMD shared with the V-cycle's
  __builtin_amdgcn_s_setprio(2);
  const int rhs = blockIdx.z;
  const bool off = gate.off(rhs);   // tested after the staging, so its load overlaps them
  const int n = g.n;
  const long long np = (long long)g.nk + g.n0;
  T* rr = r + (long long)rhs * np;
  const double* r64 = src.r ? src.r + (long long)rhs * src.ld + g.off_pk() : nullptr;
  const double cf = (src.r && src.coef) ? src.coef[rhs] : 0.0;
  double* o64 = sink.out ? sink.out + (long long)rhs * sink.ld + g.off_pk() : nullptr;
  const T* zi = zin + (long long)rhs * np;
  const int c0 = blockIdx.x * TQ, d0 = blockIdx.y * TQ;
  const bool last_x = blockIdx.x == gridDim.x - 1, last_y = blockIdx.y == gridDim.y - 1;
  const int gx = c0 - HALO, gy = d0 - HALO;      // global index of local 0
  const double h2 = g.h * g.h;
  const T h2_36 = T(h2 / 36.0), h2_4 = T(0.25 * h2), inv_h2_9 = T(9.0 / h2), inv_h2 = T(1.0 / h2);
  const int tid = threadIdx.x;
  T* zo = zout + (long long)rhs * np;
  const T* dr = din + (long long)rhs * np;
  T* dw = dout + (long long)rhs * np;
  // the owned node / element values of z_k and d, fetched before the staging
  // so that their latency overlaps it
  // (two steps per launch keep z_k and d of every staged node instead)
  constexpr bool PF = Tl::CACHE_R && ST == 1;   // TQ = 64 reads them at the end instead (registers)
  constexpr int OWP = PF ? OWN : 1;
  T z0q[OWP], d0q[OWP], z0e[OWP], d0e[OWP];
  if constexpr (PF) {
#pragma unroll
    for (int i = 0; i < OWN; ++i) {
      const int idx = tid + i * FT, ox = idx % TQ, oy = idx / TQ;
      const int oc = c0 + ox, od = d0 + oy;
      z0q[i] = d0q[i] = z0e[i] = d0e[i] = T(0);
      if (!first && idx < TQ * TQ) {
        if (oc <= n && od <= n) {
          const long long oq = (long long)od * (n + 1) + oc;
          z0q[i] = zi[oq];
          d0q[i] = dr[oq];
        }
        if (oc < n && od < n) {
          const long long oe = g.nk + (long long)od * n + oc;
          z0e[i] = zi[oe];
          d0e[i] = dr[oe];
        }
      }
    }
  }
  // staging: every global load of the region before the first LDS store (in
  // two rounds, nodes then elements, for FP64 tiles of 1024 threads, whose
  // registers would not hold both)
  // (the projection is the expression of k_mq_project_in, so both paths agree bit for bit)
  constexpr int IQ = (RQ * RQ + FT - 1) / FT, IE = (RE * RE + FT - 1) / FT;
  // two steps per launch: z_k and d at every staged node / element
  constexpr int KQ = ST == 2 ? IQ : 1, KE = ST == 2 ? IE : 1;
  T zk[KQ], dk[KQ], zke[KE], dke[KE];
  auto load_node = [&](int k, T& tv, T& rv, T& dv) {
    tv = rv = dv = T(0);
    const int c = gx + k % RQ, dd = gy + k / RQ;
    if (k < RQ * RQ && c >= 0 && c <= n && dd >= 0 && dd <= n) {
      const long long q = (long long)dd * (n + 1) + c;
      rv = r64 ? (T)(r64[q] - cf * 1.0) : rr[q];
      if (!first) {
        tv = zi[q];
        if constexpr (ST == 2) dv = dr[q];
      }
    }
  };
  auto load_element = [&](int k, T& tv, T& rv, T& dv) {
    tv = rv = dv = T(0);
    const int e = gx + k % RE, f = gy + k / RE;
    if (k < RE * RE && e >= 0 && e < n && f >= 0 && f < n) {
      const long long q = g.nk + (long long)f * n + e;
      rv = r64 ? (T)(r64[q] - cf * -1.0) : rr[q];
      if (!first) {
        tv = zi[q];
        if constexpr (ST == 2) dv = dr[q];
      }
    }
  };
  auto store_nodes = [&](const T* tv, const T* rv) {
#pragma unroll
    for (int i = 0; i < IQ; ++i) {
      const int k = tid + i * FT;
      if (k < RQ * RQ) {
        const int li = par_idx<QW, QS>(k % RQ, k / RQ);
        tq[li] = tv[i];
        rq[li] = rv[i];
      }
    }
  };
  auto store_elements = [&](const T* tw, const T* rw) {
#pragma unroll
    for (int i = 0; i < IE; ++i) {
      const int k = tid + i * FT;
      if (k < RE * RE) {
        const int li = par_idx<QW, QS>(k % RE, k / RE);
        te[li] = tw[i];
        re[li] = rw[i];
      }
    }
  };
  if constexpr (sizeof(T) == 8 && TQ >= 32) {
    {
      T tv[IQ], rv[IQ], dv;
#pragma unroll
      for (int i = 0; i < IQ; ++i) load_node(tid + i * FT, tv[i], rv[i], dv);
      store_nodes(tv, rv);
    }
    T tw[IE], rw[IE], dx;
#pragma unroll
    for (int i = 0; i < IE; ++i) load_element(tid + i * FT, tw[i], rw[i], dx);
    store_elements(tw, rw);
  } else {
    T tv[IQ], rv[IQ], dv[IQ], tw[IE], rw[IE], de[IE];
#pragma unroll
    for (int i = 0; i < IQ; ++i) load_node(tid + i * FT, tv[i], rv[i], dv[i]);
#pragma unroll
    for (int i = 0; i < IE; ++i) load_element(tid + i * FT, tw[i], rw[i], de[i]);
    store_nodes(tv, rv);
    store_elements(tw, rw);
    if constexpr (ST == 2) {
#pragma unroll
      for (int i = 0; i < IQ; ++i) {
        zk[i] = tv[i];
        dk[i] = dv[i];
      }
#pragma unroll
      for (int i = 0; i < IE; ++i) {
        zke[i] = tw[i];
        dke[i] = de[i];
      }
    }
  }
  if (off) return;   // uniform per block
  // A thread updates the same node of a colour (and the same elements) in
  // every pass: the base index hx + hy*QW of each, its boundary flags and its
  // right-hand side are set up once here, so that a pass is only the stencil
  // loads, the update and the barrier.
  constexpr int CPT = (NC * NC + FT - 1) / FT;   // nodes per thread and colour
  constexpr int EPQ = (QW * QW + FT - 1) / FT;   // elements per thread and parity array
  static_assert(4 * EPQ <= 32, "element validity bits");
  // qb: base | Lx << 16 | Rx << 17 | Ly << 18 | Ry << 19 (-1: none)
  int qb[4][CPT];
#pragma unroll
  for (int colour = 0; colour < 4; ++colour)
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int px = colour & 1, py = colour >> 1;
      const int idx = tid + j * FT;
      const int hx = idx % NC + 1 - px, hy = idx / NC + 1 - py;
      const int c = gx + 2 * hx + px, dd = gy + 2 * hy + py;
      const bool ok = idx < NC * NC && c >= 0 && c <= n && dd >= 0 && dd <= n;
      qb[colour][j] = ok ? (hx + hy * QW) | ((c > 0) << 16) | ((c < n) << 17) | ((dd > 0) << 18) |
                               ((dd < n) << 19)
                         : -1;
    }
  // element of parity array p (qx = p & 1, qy = p >> 1), entry j = tid + i*FT
  unsigned emask = 0;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int i = 0; i < EPQ; ++i) {
      const int qx = p & 1, qy = p >> 1;
      const int jj = tid + i * FT, hx = jj % QW, hy = jj / QW;
      const int e = gx + 2 * hx + qx, f = gy + 2 * hy + qy;
      const bool ok = jj < QW * QW && hx < QW - qx && hy < QW - qy && e >= 0 && e < n && f >= 0 && f < n;
      emask |= (ok ? 1u : 0u) << (p * EPQ + i);
    }
  __syncthreads();
  constexpr bool CR = Tl::CACHE_R;
  // with CR the right-hand sides of the thread's nodes are kept in registers
  // across the passes, with CS also their inverse diagonal factors (not for
  // FP64 32 x 32 tiles, whose 1024 threads have no registers to spare)
  constexpr bool CS = CR && !(sizeof(T) == 8 && TQ >= 32);
  T qr[4][CR ? CPT : 1], er[4][CR ? EPQ : 1], qsc[4][CS ? CPT : 1];
  if constexpr (CR) {
#pragma unroll
    for (int colour = 0; colour < 4; ++colour)
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        const int v = qb[colour][j];
        qr[colour][j] = v >= 0 ? rq[colour * QS + (v & 0xffff)] : T(0);
        if constexpr (CS)
          qsc[colour][j] = q1_gs_scale<T>((v >> 16) & 1, (v >> 17) & 1, (v >> 18) & 1, (v >> 19) & 1, inv_h2_9);
      }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int i = 0; i < EPQ; ++i)
        er[p][i] = (emask >> (p * EPQ + i)) & 1u ? re[p * QS + tid + i * FT] : T(0);
  }
  auto sweep = [&]() {
  constexpr int order[9] = {0, 1, 2, 3, 4, 3, 2, 1, 0};
#pragma unroll
  for (int pass = 0; pass < 9; ++pass) {
    const int colour = order[pass];
    if (colour < 4) {
      const int px = colour & 1, py = colour >> 1;
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        const int v = qb[colour][j];
        if (v < 0) continue;
        const int base = v & 0xffff;
        T q9[9], e4[4];
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
          for (int aa = 0; aa < 3; ++aa) q9[bb * 3 + aa] = tq[base + par_off<QW, QS>(px, py, aa - 1, bb - 1)];
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
          for (int aa = 0; aa < 2; ++aa) e4[bb * 2 + aa] = te[base + par_off<QW, QS>(px, py, aa - 1, bb - 1)];
        const int li = base + par_off<QW, QS>(px, py, 0, 0);
        const int Lx = (v >> 16) & 1, Rx = (v >> 17) & 1, Ly = (v >> 18) & 1, Ry = (v >> 19) & 1;
        const T sc = CS ? qsc[colour][CS ? j : 0] : q1_gs_scale<T>(Lx, Rx, Ly, Ry, inv_h2_9);
        tq[li] = q1_gs_update_s<T>(q9[4], CR ? qr[colour][CR ? j : 0] : rq[li], q9, e4, Lx, Rx, Ly, Ry, h2_36,
                                   h2_4, sc);
      }
    } else {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int qx = p & 1, qy = p >> 1;
#pragma unroll
        for (int i = 0; i < EPQ; ++i) {
          if (!((emask >> (p * EPQ + i)) & 1u)) continue;
          const int base = tid + i * FT, k = p * QS + base;
          te[k] = p0_gs_update<T>(CR ? er[p][CR ? i : 0] : re[k], tq[base + par_off<QW, QS>(qx, qy, 0, 0)],
                                  tq[base + par_off<QW, QS>(qx, qy, 1, 0)],
                                  tq[base + par_off<QW, QS>(qx, qy, 0, 1)],
                                  tq[base + par_off<QW, QS>(qx, qy, 1, 1)], inv_h2);
        }
      }
    }
    __syncthreads();
  }
  };
  sweep();
  const T ta = T(a), tb = T(b);
  if constexpr (ST == 2) {
    // first combination on the whole region, the second sweep from it
#pragma unroll
    for (int i = 0; i < IQ; ++i) {
      const int k = tid + i * FT;
      if (k < RQ * RQ) {
        const int li = par_idx<QW, QS>(k % RQ, k / RQ);
        T dn;
        zk[i] = cheb_combine<T>(tq[li], zk[i], dk[i], ta, tb, first, dn);
        dk[i] = dn;
        tq[li] = zk[i];
      }
    }
#pragma unroll
    for (int i = 0; i < IE; ++i) {
      const int k = tid + i * FT;
      if (k < RE * RE) {
        const int li = par_idx<QW, QS>(k % RE, k / RE);
        T dn;
        zke[i] = cheb_combine<T>(te[li], zke[i], dke[i], ta, tb, first, dn);
        dke[i] = dn;
        te[li] = zke[i];
      }
    }
    __syncthreads();
    sweep();
    // second combination on the owned nodes and elements, in staging order
    const T ta2 = T(a2), tb2 = T(b2);
#pragma unroll
    for (int i = 0; i < IQ; ++i) {
      const int k = tid + i * FT, lx = k % RQ, ly = k / RQ;
      const int c = gx + lx, dd = gy + ly;
      if (k >= RQ * RQ || lx < HALO || (lx >= HALO + TQ && !last_x) || ly < HALO ||
          (ly >= HALO + TQ && !last_y) || c > n || dd > n)
        continue;
      const int li = par_idx<QW, QS>(lx, ly);
      const long long oq = (long long)dd * (n + 1) + c;
      T dn;
      const T zn = cheb_combine<T>(tq[li], zk[i], dk[i], ta2, tb2, 0, dn);
      if (o64) {
        o64[oq] = sink.scale * (double)zn;
      } else {
        dw[oq] = dn;
        zo[oq] = zn;
      }
      if (r64) rr[oq] = rq[li];
    }
#pragma unroll
    for (int i = 0; i < IE; ++i) {
      const int k = tid + i * FT, lx = k % RE, ly = k / RE;
      const int e = gx + lx, f = gy + ly;
      if (k >= RE * RE || lx < HALO || lx >= HALO + TQ || ly < HALO || ly >= HALO + TQ || e >= n || f >= n)
        continue;
      const int li = par_idx<QW, QS>(lx, ly);
      const long long oe = g.nk + (long long)f * n + e;
      T dn;
      const T zn = cheb_combine<T>(te[li], zke[i], dke[i], ta2, tb2, 0, dn);
      if (o64) {
        o64[oe] = sink.scale * (double)zn;
      } else {
        dw[oe] = dn;
        zo[oe] = zn;
      }
      if (r64) rr[oe] = re[li];
    }
    return;
  }
  // Chebyshev combination on the owned nodes and elements
  auto finish = [&](long long q, int lo, T zq, T dq, const T* tl, const T* rl) {
    T dn;
    const T zn = cheb_combine<T>(tl[lo], zq, dq, ta, tb, first, dn);
    if (o64) {
      o64[q] = sink.scale * (double)zn;
    } else {
      dw[q] = dn;
      zo[q] = zn;
    }
    if (r64) rr[q] = rl[lo];
  };
#pragma unroll
  for (int i = 0; i < OWN; ++i) {
    const int idx = tid + i * FT, ox = idx % TQ, oy = idx / TQ;
    if (idx >= TQ * TQ) break;
    const int oc = c0 + ox, od = d0 + oy;
    const int lo = par_idx<QW, QS>(ox + HALO, oy + HALO);
    if (oc <= n && od <= n) {
      const long long oq = (long long)od * (n + 1) + oc;
      const T zq = PF ? z0q[PF ? i : 0] : (first ? T(0) : zi[oq]);
      const T dq = PF ? d0q[PF ? i : 0] : (first ? T(0) : dr[oq]);
      finish(oq, lo, zq, dq, tq, rq);
    }
    if (oc < n && od < n) {
      const long long oe = g.nk + (long long)od * n + oc;
      const T ze = PF ? z0e[PF ? i : 0] : (first ? T(0) : zi[oe]);
      const T de = PF ? d0e[PF ? i : 0] : (first ? T(0) : dr[oe]);
      finish(oe, lo, ze, de, te, re);
    }
  }
  // node n of the rows / columns of the last tiles (column ox = TQ, row
  // oy = TQ, their corner), one per thread on the threads the loop above left
  // idle where there are any (2 TQ + 1 <= FT)
  if (last_x || last_y) {
    const int x = (tid + FT - (TQ * TQ) % FT) % FT;
    const int ox = x < TQ ? TQ : (x < 2 * TQ ? x - TQ : TQ);
    const int oy = x < TQ ? x : TQ;
    const int oc = c0 + ox, od = d0 + oy;
    const bool mine = x < 2 * TQ + 1 && (ox < TQ || last_x) && (oy < TQ || last_y) && oc <= n && od <= n;
    if (mine) {
      const long long oq = (long long)od * (n + 1) + oc;
      finish(oq, par_idx<QW, QS>(ox + HALO, oy + HALO), first ? T(0) : zi[oq], first ? T(0) : dr[oq], tq, rq);
    }
  }
}

inline unsigned nb(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_mq_diag_dot(const Geo& g, const double* r, long long ld, int batch, const RedCtx& rc,
                        Gate gate, hipStream_t st) {
  hipLaunchKernelGGL(k_mq_diag_dot, dim3(rc.nblocks, batch), dim3(NT), 0, st, g, r, ld, rc, gate);
  ETH_LAUNCH_CHECK();
  launch_reduce_finish(rc, batch, gate, st);
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
  launch_reduce_finish(rc, batch, gate, st);
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


template <typename T>
void launch_mq_cheb_fused(const Geo& g, T* r, const T* zin, T* zout, const T* din, T* dout, double a,
                          double b, double a2, double b2, int steps, int first, int batch, Gate gate,
                          hipStream_t st, int tile, const MqSource* src, const MqSink* sink) {
  if (tile == 64 && sizeof(T) != 4) throw std::invalid_argument("M_Q tile 64 needs the FP32 preconditioner");
  if (steps == 2 && ((tile != 16 && tile != 24) || din == dout))
    throw std::invalid_argument("two M_Q steps per launch need 16 x 16 or 24 x 24 tiles and separate d arrays");
  const int tq = (tile == 8 || tile == 16 || tile == 24 || tile == 64) ? tile : 32;
  const MqSource s = src ? *src : MqSource{};
  const MqSink k = sink ? *sink : MqSink{};
#define ETH_MQF(TQ, ST)                                                                                \
  hipLaunchKernelGGL((k_mq_cheb_fused<T, TQ, ST>),                                                    \
                     dim3((g.n + TQ - 1) / TQ, (g.n + TQ - 1) / TQ, batch),                           \
                     dim3(MqTile<TQ, ST>::FT), 0, st, g, r, zin, zout, din, dout, a, b, a2, b2, first, \
                     gate, s, k)
  if (steps == 2) {
    // FP32 only: z_k and d of every staged entry would not fit FP64 registers
    if constexpr (sizeof(T) == 4) {
      if (tq == 24) ETH_MQF(24, 2);
      else ETH_MQF(16, 2);
    } else {
      throw std::invalid_argument("two M_Q steps per launch need the FP32 preconditioner");
    }
  } else if (tq == 8) {
    ETH_MQF(8, 1);
  } else if (tq == 16) {
    ETH_MQF(16, 1);
  } else if (tq == 24) {
    ETH_MQF(24, 1);
  } else if (tq == 64) {
    // the 84^2 + 83^2 staged values of two arrays fit the LDS in FP32 only
    if constexpr (sizeof(T) == 4) ETH_MQF(64, 1);
  } else {
    ETH_MQF(32, 1);
  }
#undef ETH_MQF
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
                                         const double*, double, Gate, hipStream_t);               \
  template void launch_mq_cheb_fused<T>(const Geo&, T*, const T*, T*, const T*, T*, double, double,  \
                                        double, double, int, int, int, Gate, hipStream_t, int,          \
                                        const MqSource*, const MqSink*);
ETH_INST(double)
ETH_INST(float)
#undef ETH_INST

}  // namespace eth
