// Sliced-ELL sparse kernels for the step domain: one thread per row, 64 rows
// (one wavefront) per slice, the entries of a slice stored column-major so
// that a wavefront reads 64 consecutive values and column indices per step.
// Sums are formed in FP64 whatever the storage type of the matrix (V) and
// of the vectors (T).
#include "eth_step.h"

#include <cstdlib>

namespace eth {

namespace {
constexpr int NT = 256;

__device__ __forceinline__ bool gated(const int* gate) { return gate && *gate == 0; }

// four entries per round: the column indices and values of a round are
// loaded together, then the four vector entries they address, so a thread
// has several independent loads in flight instead of one dependent chain
// (eight per round with predicated tails measured slower: 142 -> 201 ms per
// solve at m = 64)
template <typename T, typename V>
__device__ __forceinline__ double row_dot(const SellView<V>& A, int row, const T* __restrict__ x) {
  const int slice = row >> 6, lane = row & 63;
  const int beg = A.ptr[slice];
  const int width = (A.ptr[slice + 1] - beg) >> 6;
  const int* c = A.col + beg + lane;
  const V* v = A.val + beg + lane;
  double s = 0.0;
  int k = 0;
  for (; k + 4 <= width; k += 4) {
    const int c0 = c[64 * k], c1 = c[64 * (k + 1)], c2 = c[64 * (k + 2)], c3 = c[64 * (k + 3)];
    const double v0 = (double)v[64 * k], v1 = (double)v[64 * (k + 1)], v2 = (double)v[64 * (k + 2)],
                 v3 = (double)v[64 * (k + 3)];
    const double x0 = (double)x[c0], x1 = (double)x[c1], x2 = (double)x[c2], x3 = (double)x[c3];
    s += v0 * x0;
    s += v1 * x1;
    s += v2 * x2;
    s += v3 * x3;
  }
  for (; k < width; ++k) s += (double)v[64 * k] * (double)x[c[64 * k]];
  return s;
}

// the same row sums for two vectors x0, x1 from one read of the row's
// entries (each sum in row_dot's order, so bit for bit row_dot's)
template <typename T, typename V>
__device__ __forceinline__ void row_dot2(const SellView<V>& A, int row, const T* __restrict__ x0,
                                         const T* __restrict__ x1, double& s0, double& s1) {
  const int slice = row >> 6, lane = row & 63;
  const int beg = A.ptr[slice];
  const int width = (A.ptr[slice + 1] - beg) >> 6;
  const int* c = A.col + beg + lane;
  const V* v = A.val + beg + lane;
  double a = 0.0, e = 0.0;
  int k = 0;
  for (; k + 4 <= width; k += 4) {
    const int c0 = c[64 * k], c1 = c[64 * (k + 1)], c2 = c[64 * (k + 2)], c3 = c[64 * (k + 3)];
    const double v0 = (double)v[64 * k], v1 = (double)v[64 * (k + 1)], v2 = (double)v[64 * (k + 2)],
                 v3 = (double)v[64 * (k + 3)];
    const double p0 = (double)x0[c0], p1 = (double)x0[c1], p2 = (double)x0[c2], p3 = (double)x0[c3];
    const double q0 = (double)x1[c0], q1 = (double)x1[c1], q2 = (double)x1[c2], q3 = (double)x1[c3];
    a += v0 * p0;
    a += v1 * p1;
    a += v2 * p2;
    a += v3 * p3;
    e += v0 * q0;
    e += v1 * q1;
    e += v2 * q2;
    e += v3 * q3;
  }
  for (; k < width; ++k) {
    const double vk = (double)v[64 * k];
    const int ck = c[64 * k];
    a += vk * (double)x0[ck];
    e += vk * (double)x1[ck];
  }
  s0 = a;
  s1 = e;
}

// NV vectors per thread (1, or 2: the row's entries read once for a pair of
// vectors, the pairs on blockIdx.y)
template <typename T, typename V, int MODE, int NV>
__global__ __launch_bounds__(NT) void k_sell(SellView<V> A, const T* __restrict__ x, long long sx,
                                              const T* __restrict__ b, long long sb, T* __restrict__ y,
                                              long long sy, double w, double alpha, int has_prev,
                                              const int* __restrict__ gate) {
  if (gated(gate)) return;
  const int row = blockIdx.x * NT + threadIdx.x;
  if (row >= A.rows) return;
  const int vec0 = blockIdx.y * NV;
  double s[NV];
  if constexpr (NV == 2) {
    if (x) row_dot2(A, row, x + vec0 * sx, x + (vec0 + 1) * sx, s[0], s[1]);
    else s[0] = s[1] = 0.0;
  } else {
    s[0] = x ? row_dot(A, row, x + vec0 * sx) : 0.0;
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const int vec = vec0 + q;
    const T* xv = x ? x + vec * sx : nullptr;
    T* yv = y + vec * sy;
    if constexpr (MODE == 0 || MODE == 1) {
      if constexpr (MODE == 0) yv[row] = (T)s[q];
      else yv[row] = (T)((double)yv[row] + s[q]);
    } else {
      const T* bv = b + vec * sb;
      const double res = (double)bv[row] - s[q];
      if constexpr (MODE == 2) {
        yv[row] = (T)res;
      } else {
        const double xc = xv ? (double)xv[row] : 0.0;
        double xn = xc + w * (double)A.dinv[row] * res;
        if constexpr (MODE == 4) {
          if (has_prev == 1) xn += alpha * (xc - (double)yv[row]);
          else if (has_prev == 2) xn += alpha * xc;
        }
        yv[row] = (T)xn;
      }
    }
  }
}

// First kernel of a Chebyshev-SGS step on M_Q: res = r - M x (x == null:
// res = r) over all rows, and the first colour pass of a symmetric sweep
// from zero, s = D^{-1} res on colour 0 and s = 0 elsewhere.
template <typename T, typename V>
__global__ __launch_bounds__(NT) void k_sgs_enter(SellView<V> A, const unsigned char* __restrict__ colour,
                                                   const T* __restrict__ x, const T* __restrict__ r,
                                                   T* __restrict__ res, T* __restrict__ s,
                                                   const int* __restrict__ gate) {
  if (gated(gate)) return;
  const int row = blockIdx.x * NT + threadIdx.x;
  if (row >= A.rows) return;
  const double q = (double)r[row] - (x ? row_dot(A, row, x) : 0.0);
  res[row] = (T)q;
  s[row] = colour[row] == 0 ? (T)(q * (double)A.dinv[row]) : T(0);
}

// Last kernel of the step: the closing colour-0 pass of the sweep, then the
// Chebyshev update d = alpha d + beta s, x = x + d (x_zero: x = d).
template <typename T, typename V>
__global__ __launch_bounds__(NT) void k_sgs_leave(SellView<V> A, const unsigned char* __restrict__ colour,
                                                   const T* __restrict__ res, T* __restrict__ s,
                                                   T* __restrict__ d, T* __restrict__ x, double alpha,
                                                   double beta, int x_zero, const int* __restrict__ gate) {
  if (gated(gate)) return;
  const int row = blockIdx.x * NT + threadIdx.x;
  if (row >= A.rows) return;
  double sv = (double)s[row];
  if (colour[row] == 0) {
    // the neighbours read here are of other colours: final for this pass
    sv = (double)(T)(sv + ((double)res[row] - row_dot(A, row, s)) * (double)A.dinv[row]);
  }
  // the first step starts the direction afresh: d is not read (its memory
  // may hold anything, NaN included, before the first step writes it)
  const double dn = x_zero ? (double)(T)(beta * sv) : (double)(T)(alpha * (double)d[row] + beta * sv);
  d[row] = (T)dn;
  x[row] = x_zero ? (T)dn : (T)((double)x[row] + dn);
}

// One colour pass on a colour-ordered matrix: the rows of the class are the
// contiguous range [off, off + count) and their entries an ELL block
// (entry k of row i at k * count + i), so a thread loads its entries
// directly, without a row list or slice offsets in the dependent chain.
template <typename T, typename V>
__device__ __forceinline__ double ell_dot(const EllView<V>& E, int i, const T* __restrict__ x) {
  const int* c = E.col + i;
  const V* v = E.val + i;
  const int n = E.count;
  double s = 0.0;
  int k = 0;
  for (; k + 4 <= E.width; k += 4) {
    const int c0 = c[k * n], c1 = c[(k + 1) * n], c2 = c[(k + 2) * n], c3 = c[(k + 3) * n];
    const double v0 = (double)v[k * n], v1 = (double)v[(k + 1) * n], v2 = (double)v[(k + 2) * n],
                 v3 = (double)v[(k + 3) * n];
    const double x0 = (double)x[c0], x1 = (double)x[c1], x2 = (double)x[c2], x3 = (double)x[c3];
    s += v0 * x0;
    s += v1 * x1;
    s += v2 * x2;
    s += v3 * x3;
  }
  for (; k < E.width; ++k) s += (double)v[k * n] * (double)x[c[k * n]];
  return s;
}

template <typename T, typename V>
__global__ __launch_bounds__(NT) void k_ell_colour(EllView<V> E, const T* __restrict__ b, T* __restrict__ x,
                                                    const int* __restrict__ gate) {
  if (gated(gate)) return;
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= E.count) return;
  const int r = E.off + i;
  const double s = ell_dot(E, i, x);
  x[r] = (T)((double)x[r] + ((double)b[r] - s) * (double)E.dinv[i]);
}

// The middle of the sweep in one launch over the colour-3 rows: every
// element has exactly one corner of each Q1 colour, so the thread of a
// colour-3 node alone takes its forward update, then the colour-4 (element)
// updates of the elements around it (rows from E4.off on; their other
// corners are final from the earlier passes), then its backward update; no
// other thread reads or writes those entries in this launch.
template <typename T, typename V>
__global__ __launch_bounds__(NT) void k_ell_middle(EllView<V> E3, EllView<V> E4, const T* __restrict__ b,
                                                    T* __restrict__ x, const int* __restrict__ gate) {
  if (gated(gate)) return;
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= E3.count) return;
  const int r = E3.off + i;
  x[r] = (T)((double)x[r] + ((double)b[r] - ell_dot(E3, i, x)) * (double)E3.dinv[i]);
  int prev = -1;
  for (int k = 0; k < E3.width; ++k) {
    const int e = E3.col[k * E3.count + i];
    if (e < E4.off || e == prev) continue;   // Q1 columns, and padding repeating the last column
    prev = e;
    const int j = e - E4.off;
    x[e] = (T)((double)x[e] + ((double)b[e] - ell_dot(E4, j, x)) * (double)E4.dinv[j]);
  }
  x[r] = (T)((double)x[r] + ((double)b[r] - ell_dot(E3, i, x)) * (double)E3.dinv[i]);
}

// y[i] = (To)(a * x[idx[i]])  (gather) or y[idx[i]] = (To)(a * x[i])  (scatter)
template <typename Ti, typename To, bool SCATTER>
__global__ __launch_bounds__(NT) void k_permute(int n, const int* __restrict__ idx, double a,
                                                 const Ti* __restrict__ x, To* __restrict__ y,
                                                 const int* __restrict__ gate) {
  if (gated(gate)) return;
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  if constexpr (SCATTER) y[idx[i]] = (To)(a * (double)x[i]);
  else y[i] = (To)(a * (double)x[idx[i]]);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_dense_apply(const double* __restrict__ Ainv, int n,
                                                     const T* __restrict__ b, long long sb, T* __restrict__ x,
                                                     long long sx, const int* __restrict__ gate) {
  if (gated(gate)) return;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  const int vec = blockIdx.y;
  if (row >= n) return;
  const T* bv = b + vec * sb;
  const double* a = Ainv + (size_t)row * n;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += a[j] * (double)bv[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) x[vec * sx + row] = (T)s;
}

template <typename Ti, typename To>
__global__ __launch_bounds__(NT) void k_vcombine(long long n, double a, const Ti* __restrict__ x, double c,
                                                  const Ti* __restrict__ z, To* __restrict__ y,
                                                  const int* __restrict__ gate) {
  if (gated(gate)) return;
  const long long i = (long long)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  double v = a * (double)x[i];
  if (z) v += c * (double)z[i];
  y[i] = (To)v;
}

// frame projection: partials of sum(p_1) - sum(p_0), then the shift
constexpr int FP_PER = 4 * NT;
template <typename T>
__global__ __launch_bounds__(NT) void k_frame_partial(int nk, int np, const T* __restrict__ p,
                                                       double* __restrict__ part, const int* __restrict__ gate) {
  if (gated(gate)) return;
  __shared__ double red[NT / 64];
  double s = 0.0;
  const int base = blockIdx.x * FP_PER;
  for (int k = threadIdx.x; k < FP_PER; k += NT) {
    const int i = base + k;
    if (i < np) s += (i < nk ? 1.0 : -1.0) * (double)p[i];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_frame_shift(int nk, int np, int nparts, const double* __restrict__ part,
                                                     T* __restrict__ p, const int* __restrict__ gate) {
  if (gated(gate)) return;
  __shared__ double tot;
  if (threadIdx.x == 0) {   // every block sums the partials in the same order
    double t = 0.0;
    for (int k = 0; k < nparts; ++k) t += part[k];
    tot = t / (double)np;
  }
  __syncthreads();
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= np) return;
  p[i] = (T)((double)p[i] - (i < nk ? tot : -tot));
}

unsigned nblk(long long n) { return (unsigned)((n + NT - 1) / NT); }
// ETH_DEBUG_SELL_UNPAIRED=1: one vector per thread also for pairs
bool sell_unpaired() {
  const char* e = std::getenv("ETH_DEBUG_SELL_UNPAIRED");
  return e && e[0] == '1';
}
}  // namespace

template <typename T, typename V>
void launch_sell(const Sell& A, int mode, const T* x, long long sx, const T* b, long long sb, T* y, long long sy,
                 int nvec, double w, double alpha, int has_prev, const int* gate, hipStream_t st) {
  const SellView<V> v = view<V>(A);
  // pairs of vectors share one read of the matrix (the two velocity
  // components of the F levels and transfers) where the matrix is large:
  // measured 3-5 % faster step solves at m = 128, within 1 % at m = 64 and
  // 2 % slower at m = 32 (half the blocks)
  const bool pair = nvec % 2 == 0 && A.rows >= (1 << 17) && !sell_unpaired();
  const dim3 grid(nblk(A.rows), pair ? nvec / 2 : nvec);
#define ETH_SELL(M)                                                                                        \
  if (pair)                                                                                                \
    hipLaunchKernelGGL((k_sell<T, V, M, 2>), grid, dim3(NT), 0, st, v, x, sx, b, sb, y, sy, w, alpha,     \
                       has_prev, gate);                                                                    \
  else                                                                                                     \
    hipLaunchKernelGGL((k_sell<T, V, M, 1>), grid, dim3(NT), 0, st, v, x, sx, b, sb, y, sy, w, alpha,     \
                       has_prev, gate)
  switch (mode) {
    case 0: ETH_SELL(0); break;
    case 1: ETH_SELL(1); break;
    case 2: ETH_SELL(2); break;
    case 3: ETH_SELL(3); break;
    default: ETH_SELL(4); break;
  }
#undef ETH_SELL
  ETH_LAUNCH_CHECK();
}

template <typename T, typename V>
void launch_sgs_enter(const Sell& A, const unsigned char* colour, const T* x, const T* r, T* res, T* s,
                      const int* gate, hipStream_t st) {
  hipLaunchKernelGGL((k_sgs_enter<T, V>), dim3(nblk(A.rows)), dim3(NT), 0, st, view<V>(A), colour, x, r, res, s,
                     gate);
  ETH_LAUNCH_CHECK();
}

template <typename T, typename V>
void launch_ell_colour(const Ell& E, const T* b, T* x, const int* gate, hipStream_t st) {
  if (E.count <= 0) return;
  hipLaunchKernelGGL((k_ell_colour<T, V>), dim3(nblk(E.count)), dim3(NT), 0, st, eview<V>(E), b, x, gate);
  ETH_LAUNCH_CHECK();
}

template <typename T, typename V>
void launch_ell_middle(const Ell& E3, const Ell& E4, const T* b, T* x, const int* gate, hipStream_t st) {
  if (E3.count <= 0) return;
  hipLaunchKernelGGL((k_ell_middle<T, V>), dim3(nblk(E3.count)), dim3(NT), 0, st, eview<V>(E3), eview<V>(E4), b,
                     x, gate);
  ETH_LAUNCH_CHECK();
}

template <typename Ti, typename To>
void launch_permute(int n, const int* idx, bool scatter, double a, const Ti* x, To* y, const int* gate,
                    hipStream_t st) {
  if (scatter)
    hipLaunchKernelGGL((k_permute<Ti, To, true>), dim3(nblk(n)), dim3(NT), 0, st, n, idx, a, x, y, gate);
  else
    hipLaunchKernelGGL((k_permute<Ti, To, false>), dim3(nblk(n)), dim3(NT), 0, st, n, idx, a, x, y, gate);
  ETH_LAUNCH_CHECK();
}

template <typename T, typename V>
void launch_sgs_leave(const Sell& A, const unsigned char* colour, const T* res, T* s, T* d, T* x, double alpha,
                      double beta, int x_zero, const int* gate, hipStream_t st) {
  hipLaunchKernelGGL((k_sgs_leave<T, V>), dim3(nblk(A.rows)), dim3(NT), 0, st, view<V>(A), colour, res, s, d, x,
                     alpha, beta, x_zero, gate);
  ETH_LAUNCH_CHECK();
}

template <typename T>
void launch_dense_apply(const double* Ainv, int n, const T* b, long long sb, T* x, long long sx, int nvec,
                        const int* gate, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_apply<T>, dim3((n + NT / 64 - 1) / (NT / 64), nvec), dim3(NT), 0, st, Ainv, n, b, sb,
                     x, sx, gate);
  ETH_LAUNCH_CHECK();
}

template <typename Ti, typename To>
void launch_vcombine(long long n, double a, const Ti* x, double c, const Ti* z, To* y, const int* gate,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_vcombine<Ti, To>), dim3(nblk(n)), dim3(NT), 0, st, n, a, x, c, z, y, gate);
  ETH_LAUNCH_CHECK();
}

int frame_project_blocks(int np) { return (np + FP_PER - 1) / FP_PER; }

void launch_frame_project(double* part, int nk, int n0, void* p, bool fp32, const int* gate, hipStream_t st) {
  const int np = nk + n0, nb = frame_project_blocks(np);
  if (fp32) {
    hipLaunchKernelGGL(k_frame_partial<float>, dim3(nb), dim3(NT), 0, st, nk, np, (const float*)p, part, gate);
    ETH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_frame_shift<float>, dim3(nblk(np)), dim3(NT), 0, st, nk, np, nb, part, (float*)p, gate);
  } else {
    hipLaunchKernelGGL(k_frame_partial<double>, dim3(nb), dim3(NT), 0, st, nk, np, (const double*)p, part, gate);
    ETH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_frame_shift<double>, dim3(nblk(np)), dim3(NT), 0, st, nk, np, nb, part, (double*)p, gate);
  }
  ETH_LAUNCH_CHECK();
}

void launch_frame_partials(double* part, int nk, int n0, const double* p, hipStream_t st) {
  const int np = nk + n0, nb = frame_project_blocks(np);
  hipLaunchKernelGGL(k_frame_partial<double>, dim3(nb), dim3(NT), 0, st, nk, np, p, part, nullptr);
  ETH_LAUNCH_CHECK();
}

#define ETH_SELL_INST(T, V)                                                                                  \
  template void launch_sell<T, V>(const Sell&, int, const T*, long long, const T*, long long, T*, long long, \
                                  int, double, double, int, const int*, hipStream_t);                      \
  template void launch_sgs_enter<T, V>(const Sell&, const unsigned char*, const T*, const T*, T*, T*, const int*, \
                                       hipStream_t);                                                       \
  template void launch_sgs_leave<T, V>(const Sell&, const unsigned char*, const T*, T*, T*, T*, double, double, \
                                       int, const int*, hipStream_t);                                        \
  template void launch_ell_colour<T, V>(const Ell&, const T*, T*, const int*, hipStream_t);                 \
  template void launch_ell_middle<T, V>(const Ell&, const Ell&, const T*, T*, const int*, hipStream_t);
ETH_SELL_INST(double, double)
ETH_SELL_INST(float, float)
template void launch_dense_apply<double>(const double*, int, const double*, long long, double*, long long, int,
                                         const int*, hipStream_t);
template void launch_dense_apply<float>(const double*, int, const float*, long long, float*, long long, int,
                                        const int*, hipStream_t);
template void launch_permute<double, double>(int, const int*, bool, double, const double*, double*, const int*,
                                             hipStream_t);
template void launch_permute<double, float>(int, const int*, bool, double, const double*, float*, const int*,
                                            hipStream_t);
template void launch_permute<float, double>(int, const int*, bool, double, const float*, double*, const int*,
                                            hipStream_t);
template void launch_permute<float, float>(int, const int*, bool, double, const float*, float*, const int*,
                                           hipStream_t);
template void launch_vcombine<double, double>(long long, double, const double*, double, const double*, double*,
                                              const int*, hipStream_t);
template void launch_vcombine<double, float>(long long, double, const double*, double, const double*, float*,
                                             const int*, hipStream_t);
template void launch_vcombine<float, double>(long long, double, const float*, double, const float*, double*,
                                             const int*, hipStream_t);
template void launch_vcombine<float, float>(long long, double, const float*, double, const float*, float*,
                                            const int*, hipStream_t);

}  // namespace eth
