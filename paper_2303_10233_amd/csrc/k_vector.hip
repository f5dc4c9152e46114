// Krylov vector kernels: fused MINRES updates (alg:minres), deterministic dot
// products and the pressure canonicalisation.  FP64 throughout.
#include <hip/hip_cooperative_groups.h>

#include "eth_kernels.h"
#include "eth_reduce.h"

namespace eth {
namespace {

constexpr int NT = 256;
constexpr int kVecBlocksMax = 512;    // grid-stride cap per RHS for reductions

__global__ __launch_bounds__(NT) void k_dot(long long n, const double* __restrict__ x,
                                            const double* __restrict__ y, long long ld,
                                            RedCtx rc, Gate gate, ClearFlag clear) {
  __shared__ double sred[NT / 64];
  const int rhs = blockIdx.y;
  // (the first block of each right-hand side: here the RHS is blockIdx.y)
  if (clear.p && blockIdx.x == 0 && threadIdx.x == 0) clear.p[(long long)rhs * clear.stride] = 0;
  if (gate.off(rhs)) return;
  const double* xr = x + (long long)rhs * ld;
  const double* yr = y + (long long)rhs * ld;
  // four independent partial sums keep four loads of each vector in flight
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const long long stride = (long long)gridDim.x * NT;
  long long i = (long long)blockIdx.x * NT + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    a0 += xr[i] * yr[i];
    a1 += xr[i + stride] * yr[i + stride];
    a2 += xr[i + 2 * stride] * yr[i + 2 * stride];
    a3 += xr[i + 3 * stride] * yr[i + 3 * stride];
  }
  for (; i < n; i += stride) a0 += xr[i] * yr[i];
  double v[1] = {(a0 + a1) + (a2 + a3)};
  reduce_and_finish<NT>(rc, rhs, blockIdx.x, v, sred);
}

__global__ void k_axpby(long long n, double a, const double* __restrict__ x, double b,
                        double* __restrict__ y, long long ld) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long o = (long long)blockIdx.y * ld + i;
  y[o] = a * x[o] + b * y[o];
}

__global__ void k_copy(long long n, const double* __restrict__ x, long long ldx,
                       double* __restrict__ y, long long ldy) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[(long long)blockIdx.y * ldy + i] = x[(long long)blockIdx.y * ldx + i];
}

__global__ void k_vmul(long long n, const double* __restrict__ d, double* __restrict__ y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] *= d[i];
}

__global__ void k_fill(long long n, double v, double* __restrict__ y, long long ld) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[(long long)blockIdx.y * ld + i] = v;
}

// boundary node k (0 .. 4*(nq-1)-1) of one component -> node index
__device__ inline int boundary_node(int k, int nq) {
  const int m = nq - 1;
  if (k < m) return k;                              // bottom, I = 0..m-1
  if (k < 2 * m) return (k - m) * nq + m;           // right,  J = 0..m-1
  if (k < 3 * m) return m * nq + (m - (k - 2 * m)); // top,    I = m..1
  return (m - (k - 3 * m)) * nq;                    // left,   J = m..1
}

__global__ void k_zero_boundary(Geo g, double* __restrict__ y, long long ld) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = 4 * (g.nq - 1);
  if (k >= 2 * nb) return;
  const int comp = k / nb;
  y[(long long)blockIdx.y * ld + (long long)comp * g.nv + boundary_node(k % nb, g.nq)] = 0.0;
}

__global__ void k_copy_boundary(Geo g, const double* __restrict__ b, double* __restrict__ x,
                                long long ld) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int nb = 4 * (g.nq - 1);
  if (k >= 2 * nb) return;
  const int comp = k / nb;
  const long long o = (long long)blockIdx.y * ld + (long long)comp * g.nv + boundary_node(k % nb, g.nq);
  x[o] = b[o];
}

// v = b - y on interior rows, 0 on boundary velocity rows
__global__ void k_residual_init(Geo g, const double* __restrict__ b, const double* __restrict__ y,
                                double* __restrict__ v, long long ld) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  const long long o = (long long)blockIdx.y * ld + i;
  bool bnd = false;
  if (i < 2LL * g.nv) {
    const int node = (int)(i % g.nv);
    const int I = node % g.nq, J = node / g.nq;
    bnd = (I == 0 || J == 0 || I == g.nq - 1 || J == g.nq - 1);
  }
  v[o] = bnd ? 0.0 : b[o] - y[o];
}

constexpr int FIN_LOADS = 8;
// total of nb block partials by one wavefront (every lane gets it)
__device__ inline double finish_total(const double* __restrict__ p, int nb, int lane) {
  double a = 0.0;
  for (int base = 0; base < nb; base += kWave * FIN_LOADS) {
    double v[FIN_LOADS];
#pragma unroll
    for (int j = 0; j < FIN_LOADS; ++j) {
      const int i = base + j * kWave + lane;
      v[j] = i < nb ? p[i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < FIN_LOADS; ++j) a += v[j];
  }
  return wave_sum(a);
}

// v_{j+1} = vy*y - va*v_j - vb*v_{j-1}   (written over v_{j-1}).  With
// nb > 1 the reduction of <K zhat_j, zhat_j> left its nb block partials
// unfinished: every block sums them (the finishing kernel's order) and forms
// the coefficients itself (the delta epilogue reads only fields no block
// writes here), and block 0 stores delta, the coefficients and the history
// entry, as the finishing launch would have.
// With wx.z set, the same pass also makes the pending w/x update of the
// previous iteration (k_minres_wx's arithmetic on the previous iteration's
// buffers, while wx_todo is set, also once the solve has stopped).
__global__ void k_minres_v(long long n, const double* __restrict__ y, const double* __restrict__ v,
                           double* __restrict__ vp, long long ld, MinresScalars* __restrict__ s,
                           const double* __restrict__ partials, int nb, MinresWx wx) {
  __shared__ double cf[3];
  const int rhs = blockIdx.y;
  const MinresScalars& S = s[rhs];
  const bool do_v = S.active != 0;
  const bool do_wx = wx.z != nullptr && S.wx_todo != 0;
  if (!do_v && !do_wx) return;
  const long long o = (long long)rhs * ld;
  if (!do_v) {
    const double cz = S.wz, cp = S.wp, cw = S.wc, cx = S.xc;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
      const double wn = cz * wx.z[o + i] - cp * wx.wprev_io[o + i] - cw * wx.w[o + i];
      wx.wprev_io[o + i] = wn;
      wx.x[o + i] += cx * wn;
    }
    return;
  }
  double vy, va, vb;
  if (nb > 1) {
    if (threadIdx.x < kWave) {
      const double tot = finish_total(partials + (long long)rhs * nb, nb, threadIdx.x);
      if (threadIdx.x == 0) {
        MinresScalars loc = S;
        if (blockIdx.x != 0) loc.hist_delta = nullptr;
        minres_delta(loc, tot);
        cf[0] = loc.vy;
        cf[1] = loc.va;
        cf[2] = loc.vb;
        if (blockIdx.x == 0) {
          s[rhs].delta = loc.delta;
          s[rhs].vy = loc.vy;
          s[rhs].va = loc.va;
          s[rhs].vb = loc.vb;
        }
      }
    }
    __syncthreads();
    vy = cf[0];
    va = cf[1];
    vb = cf[2];
  } else {
    vy = S.vy;
    va = S.va;
    vb = S.vb;
  }
  if (do_wx) {
    const double cz = S.wz, cp = S.wp, cw = S.wc, cx = S.xc;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
      vp[o + i] = vy * y[o + i] - va * v[o + i] - vb * vp[o + i];
      const double wn = cz * wx.z[o + i] - cp * wx.wprev_io[o + i] - cw * wx.w[o + i];
      wx.wprev_io[o + i] = wn;
      wx.x[o + i] += cx * wn;
    }
  } else {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
      vp[o + i] = vy * y[o + i] - va * v[o + i] - vb * vp[o + i];
  }
}

// w_{j+1} = wz*zhat_j - wp*w_{j-1} - wc*w_j (written over w_{j-1}); x += xc*w_{j+1}
// Runs while the Givens step of this iteration is pending (wx_todo); the
// flag is cleared by the first kernel of the next iteration.
__global__ void k_minres_wx(long long n, const double* __restrict__ z, double* __restrict__ wp,
                            const double* __restrict__ w, double* __restrict__ x, long long ld,
                            const MinresScalars* __restrict__ s) {
  const int rhs = blockIdx.y;
  const MinresScalars& S = s[rhs];
  if (!S.wx_todo) return;
  const double cz = S.wz, cp = S.wp, cw = S.wc, cx = S.xc;
  const long long o = (long long)rhs * ld;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double wn = cz * z[o + i] - cp * wp[o + i] - cw * w[o + i];
    wp[o + i] = wn;
    x[o + i] += cx * wn;
  }
}

// flag of every right-hand side = 0
__global__ void k_clear_flag(ClearFlag f, int batch) {
  const int r = threadIdx.x;
  if (r < batch) f.p[(long long)r * f.stride] = 0;
}

__global__ __launch_bounds__(NT) void k_pressure_sums(Geo g, const double* __restrict__ x,
                                                      long long ld, RedCtx rc) {
  __shared__ double sred[NT / 64];
  const int rhs = blockIdx.y;
  const double* xr = x + (long long)rhs * ld + g.off_pk();
  double a = 0.0, b = 0.0;
  const long long np = (long long)g.nk + g.n0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < np; i += (long long)gridDim.x * NT) {
    if (i < g.nk) a += xr[i];
    else b += xr[i];
  }
  double v[2] = {a, b};
  reduce_and_finish<NT>(rc, rhs, blockIdx.x, v, sred);
}

__global__ void k_pressure_shift(Geo g, double* __restrict__ x, long long ld,
                                 const double* __restrict__ sums) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long np = (long long)g.nk + g.n0;
  if (i >= np) return;
  const int rhs = blockIdx.y;
  const double m = (i < g.nk) ? sums[2 * rhs] / g.nk : sums[2 * rhs + 1] / g.n0;
  x[(long long)rhs * ld + g.off_pk() + i] -= m;
}

// One wave per right-hand side: every lane sums its partials (eight loads in
// flight per lane and round, a fixed order), then a shuffle reduction; no LDS
// and no barrier, since this launch sits between two dependent kernels of
// the Krylov iteration.
__global__ __launch_bounds__(kWave) void k_reduce_finish(RedCtx rc, Gate gate) {
  const int rhs = blockIdx.x;
  if (gate.off(rhs)) return;
  const int lane = threadIdx.x;
  double tot[kMaxRedVals];
  for (int k = 0; k < rc.nvals; ++k)
    tot[k] = finish_total(rc.partials + ((long long)rhs * rc.nvals + k) * rc.nblocks, rc.nblocks, lane);
  if (lane == 0) {
    if (rc.result)
      for (int k = 0; k < rc.nvals; ++k) rc.result[(long long)rhs * rc.nvals + k] = tot[k];
    if (rc.epi) run_epilogue(rc.epi, rc.epi_state, rhs, tot);
  }
}

inline unsigned blocks_for(long long n, int nt) { return (unsigned)((n + nt - 1) / nt); }

}  // namespace

void launch_reduce_finish(const RedCtx& rc, int batch, Gate gate, hipStream_t st) {
  if (rc.nblocks <= 1 || rc.defer) return;
  hipLaunchKernelGGL(k_reduce_finish, dim3(batch), dim3(kWave), 0, st, rc, gate);
  ETH_LAUNCH_CHECK();
}

int dot_blocks(long long n) {
  long long b = (n + NT * 4 - 1) / (NT * 4);
  if (b < 1) b = 1;
  if (b > kVecBlocksMax) b = kVecBlocksMax;
  return (int)b;
}

void launch_dot(long long n, const double* x, const double* y, long long ld, int batch,
                const RedCtx& rc, Gate gate, hipStream_t st, ClearFlag clear) {
  hipLaunchKernelGGL(k_dot, dim3(rc.nblocks, batch), dim3(NT), 0, st, n, x, y, ld, rc, gate, clear);
  ETH_LAUNCH_CHECK();
  launch_reduce_finish(rc, batch, gate, st);
}

void launch_axpby(long long n, double a, const double* x, double b, double* y, long long ld,
                  int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n, 256), batch), dim3(256), 0, st, n, a, x, b, y, ld);
  ETH_LAUNCH_CHECK();
}

void launch_copy(long long n, const double* x, long long ldx, double* y, long long ldy,
                 int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(blocks_for(n, 256), batch), dim3(256), 0, st, n, x, ldx, y, ldy);
  ETH_LAUNCH_CHECK();
}

void launch_fill(long long n, double v, double* y, long long ld, int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256), batch), dim3(256), 0, st, n, v, y, ld);
  ETH_LAUNCH_CHECK();
}

void launch_vmul(long long n, const double* d, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_vmul, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, d, y);
  ETH_LAUNCH_CHECK();
}

void launch_zero_boundary(const Geo& g, double* y, long long ld, int batch, hipStream_t st) {
  const int nb = 2 * 4 * (g.nq - 1);
  hipLaunchKernelGGL(k_zero_boundary, dim3(blocks_for(nb, 256), batch), dim3(256), 0, st, g, y, ld);
  ETH_LAUNCH_CHECK();
}

void launch_copy_boundary(const Geo& g, const double* b, double* x, long long ld, int batch,
                          hipStream_t st) {
  const int nb = 2 * 4 * (g.nq - 1);
  hipLaunchKernelGGL(k_copy_boundary, dim3(blocks_for(nb, 256), batch), dim3(256), 0, st, g, b, x, ld);
  ETH_LAUNCH_CHECK();
}

void launch_residual_init(const Geo& g, const double* b, const double* y, double* v,
                          long long ld, int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_residual_init, dim3(blocks_for(g.N, 256), batch), dim3(256), 0, st, g, b, y,
                     v, ld);
  ETH_LAUNCH_CHECK();
}

static unsigned update_blocks(long long n) {
  long long b = (n + 256 * 4 - 1) / (256 * 4);
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return (unsigned)b;
}

void launch_minres_v(long long n, const double* y, const double* v, double* vprev_io,
                     long long ld, int batch, MinresScalars* s, hipStream_t st, const double* partials,
                     int nb, MinresWx wx) {
  hipLaunchKernelGGL(k_minres_v, dim3(update_blocks(n), batch), dim3(256), 0, st, n, y, v,
                     vprev_io, ld, s, partials, partials ? nb : 0, wx);
  ETH_LAUNCH_CHECK();
}

void launch_clear_flag(const ClearFlag& f, int batch, hipStream_t st) {
  if (!f.p || batch < 1) return;
  for (int r0 = 0; r0 < batch; r0 += 256) {
    const int nb = batch - r0 < 256 ? batch - r0 : 256;
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(256), 0, st, ClearFlag{f.p + (long long)r0 * f.stride, f.stride},
                       nb);
    ETH_LAUNCH_CHECK();
  }
}

void launch_minres_wx(long long n, const double* z, double* wprev_io, const double* w,
                      double* x, long long ld, int batch, const MinresScalars* s, hipStream_t st) {
  hipLaunchKernelGGL(k_minres_wx, dim3(update_blocks(n), batch), dim3(256), 0, st, n, z,
                     wprev_io, w, x, ld, s);
  ETH_LAUNCH_CHECK();
}

void launch_pressure_sums(const Geo& g, const double* x, long long ld, int batch,
                          double* partials, double* out, hipStream_t st) {
  RedCtx rc{};
  rc.partials = partials;
  rc.result = out;
  rc.nblocks = dot_blocks((long long)g.nk + g.n0);
  rc.nvals = 2;
  hipLaunchKernelGGL(k_pressure_sums, dim3(rc.nblocks, batch), dim3(NT), 0, st, g, x, ld, rc);
  ETH_LAUNCH_CHECK();
  launch_reduce_finish(rc, batch, no_gate(), st);
}

void launch_pressure_shift(const Geo& g, double* x, long long ld, int batch,
                           const double* sums, hipStream_t st) {
  const long long np = (long long)g.nk + g.n0;
  hipLaunchKernelGGL(k_pressure_shift, dim3(blocks_for(np, 256), batch), dim3(256), 0, st, g, x,
                     ld, sums);
  ETH_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Synchronisation probes for the choice between kernel boundaries and a
// persistent kernel: every round each thread of a one-block-per-CU grid
// writes one value that the next round of another block reads (a halo-like
// dependency), separated either by a grid-wide barrier inside one cooperative
// launch or by the boundary between dependent launches.
namespace {
// step r reads slice (b + 1) mod nb of buffer r mod 2 and writes slice b of
// the other buffer, so one barrier per step orders everything
__device__ __forceinline__ void ring_step(double* buf, int nb, int b, int t, int r) {
  const double* src = buf + (long long)(r & 1) * 256 * nb;
  double* dst = buf + (long long)((r + 1) & 1) * 256 * nb;
  dst[(long long)b * 256 + t] = src[(long long)((b + 1) % nb) * 256 + t] + (double)r;
}

__global__ __launch_bounds__(256) void k_sync_step(double* __restrict__ buf, int round) {
  ring_step(buf, gridDim.x, blockIdx.x, threadIdx.x, round);
}

__global__ __launch_bounds__(256) void k_grid_sync_rounds(double* __restrict__ buf, int rounds) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  for (int r = 0; r < rounds; ++r) {
    ring_step(buf, gridDim.x, blockIdx.x, threadIdx.x, r);
    grid.sync();
  }
}
}  // namespace

int sync_probe_blocks() {
  int dev = 0, cus = 0;
  ETH_HIP(hipGetDevice(&dev));
  ETH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  return cus;
}

void launch_sync_step(double* buf, int round, hipStream_t st) {
  hipLaunchKernelGGL(k_sync_step, dim3(sync_probe_blocks()), dim3(256), 0, st, buf, round);
  ETH_LAUNCH_CHECK();
}

void launch_grid_sync_rounds(double* buf, int rounds, hipStream_t st) {
  void* args[] = {(void*)&buf, (void*)&rounds};
  ETH_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_grid_sync_rounds),
                                     dim3(sync_probe_blocks()), dim3(256), args, 0, st));
}

}  // namespace eth
