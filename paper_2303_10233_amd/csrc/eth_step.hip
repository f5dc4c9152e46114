// Flow over a step (Sec. 3, the inflow-outflow example): problem set-up from
// the host assembly, the preconditioners of Sec. 3.1 on sliced-ELL
// operators, flexible GMRES with the two-stage PCD driver, Picard steps, and
// their C ABI (eth.h, "flow over a step").
//
// Preconditioner pieces (the same algorithms as for the enclosed cavity):
//   F^{-1}   one V(2,2) cycle, damped Jacobi (omega), levels m, m/2, ... with
//            the wind injected and the viscosity max(nu, |w|_max h / (2 Pe_max));
//            dense inverse on the coarsest level;
//   A_p^{-1} one V(2,2) Chebyshev-Jacobi cycle over re-discretised
//            A_p = B_1 diag(M_v)^{-1} B_1^T, bilinear transfers;
//   Q_1^{-1} Chebyshev-Jacobi on [1/4, 9/4];
//   M_Q^+    Chebyshev semi-iteration based on multicolour symmetric
//            Gauss-Seidel (colours: Q1 node parities, then the elements),
//            with the frame projection onto k^perp before and after.
// Stage I (reduced system):  z_p = -A_p^{-1} F_1 Q_1^{-1} r_p,
//                            z_u = F^{-1}(r_u - B_1^T z_p)     (eq:discrete-commutator1x)
// Stage II (full system, M_1 of eq:nse-precon-ref):
//                            z_p = -nu M_Q^+ r_p,  z_u = F^{-1}(r_u - B^T z_p).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/eth.h"
#include "eth_kernels.h"
#include "eth_step.h"

namespace eth {

namespace {
constexpr int NT = 256;

__global__ void k_scatter_copy(const int* __restrict__ idx, int count, const double* __restrict__ src,
                               double* __restrict__ dst) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < count) dst[idx[i]] = src[idx[i]];
}
__global__ void k_scatter_zero(const int* __restrict__ idx, int count, double* __restrict__ dst) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < count) dst[idx[i]] = 0.0;
}
// element pressures p_0 of x: partial sums, then the shift along k that
// gives them mean zero (p_1 += c, p_0 -= c)
__global__ void k_p0_partial(const double* __restrict__ p0, int n0, double* __restrict__ part) {
  __shared__ double red[NT / 64];
  double s = 0.0;
  for (int i = blockIdx.x * 1024 + threadIdx.x; i < min(n0, (int)(blockIdx.x + 1) * 1024); i += NT) s += p0[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}
__global__ void k_p0_shift(double* __restrict__ p, int nk, int n0, const double* __restrict__ part, int nparts) {
  __shared__ double c;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < nparts; ++k) t += part[k];
    c = t / (double)n0;
  }
  __syncthreads();
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < nk) p[i] += c;
  else if (i < nk + n0) p[i] -= c;
}
unsigned nblk(long long n) { return (unsigned)((n + NT - 1) / NT); }

void cheb_ab(double lo, double hi, int d, std::vector<double>& a, std::vector<double>& b) {
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  a.assign(d, 0.0);
  b.assign(d, 0.0);
  double rho = 1.0 / sigma;
  b[0] = 1.0 / theta;
  for (int k = 1; k < d; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    a[k] = rn * rho;
    b[k] = 2.0 * rn / delta;
    rho = rn;
  }
}

struct Range {
  explicit Range(const char* n) { roctxRangePushA(n); }
  ~Range() { roctxRangePop(); }
};
}  // namespace

struct StepProblem {
  eth_step_desc d{};
  hipStream_t st = nullptr;
  bool own_stream = false, mixed = false, has_wind = false;
  std::string err;
  std::vector<StepMesh> ms;
  std::vector<StepElem> el;
  std::vector<double> wind;          // host copy of the finest wind (2 nv)
  std::vector<double> lnu;           // viscosity per level
  Csr B;                             // finest B (host)
  std::vector<void*> owned;
  // device operators
  Sell K, Q1, F1, MQ;
  Sell Bt;                           // B^T on the free velocity rows (2 n_v x n_p): the preconditioners' B^T z_p
  std::vector<Sell> F, P, R, Ap, Pq, Rq;
  double* Finv = nullptr;
  double* Apinv = nullptr;
  int nFc = 0, nAc = 0;
  std::vector<double> ap_lam;
  std::vector<std::array<double, 2>> ap_a, ap_b;   // degree-2 Chebyshev per A_p level
  std::vector<double> q1a, q1b, mqa, mqb;
  unsigned char* mq_colour = nullptr;   // colour of every pressure row (colour order)
  // M_Q is held in colour order (the Q1 classes 0..3, then the elements):
  // MQ is the permuted matrix, mq_ell[c] the ELL block of class c, mq_perm
  // the pressure index of each row of the colour order
  std::array<Ell, 5> mq_ell{};
  int* mq_perm = nullptr;
  int* dir_idx = nullptr;
  int ndir = 0;
  // workspaces
  double *kb = nullptr, *kx = nullptr, *ky = nullptr, *kz = nullptr, *kv = nullptr, *kw = nullptr;
  double* kpb = nullptr;             // right-hand side of the current Picard step
  std::vector<void*> vb, vt, qb, qt;
  std::vector<std::array<void*, 2>> vx, qx;
  void *q1x[2] = {nullptr, nullptr}, *mr = nullptr, *mxx = nullptr, *md = nullptr, *msg = nullptr, *mres = nullptr;
  double* fpart = nullptr;
  double* p0part = nullptr;
  // FGMRES
  int gm_m = 50, hist_len = 4097;
  double *gV = nullptr, *gZ = nullptr, *gArr = nullptr, *gpart = nullptr, *ghist = nullptr;
  GmresScalars* d_gm = nullptr;
  GmresScalars* h_gm = nullptr;
  double* h_red = nullptr;
  double* red_part = nullptr;
  double* red_res = nullptr;
  hipStream_t gst = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::map<std::array<int, 4>, hipGraphExec_t> graphs;

  ~StepProblem();
  bool nan_fill = false;   // ETH_DEBUG_NAN_FILL=1: workspaces start as NaN
  bool sgs_split = false;  // ETH_DEBUG_UNFUSED_MQ=1: colours 3, 4, 3 as three launches
  // M_Q solved on the bounding box of the step, one launch per Chebyshev
  // step (ETH_DEBUG_STEP_MQ_ELL=1: the colour-ordered sparse sweep, seven
  // launches per step); tile side 8 or 16 (ETH_STEP_MQ_TILE), by default 16
  // from 128 blocks on (measured: 8 faster at m = 32, 16 at m = 64 and 128)
  bool mq_box = true;
  int mq_box_tile = 16;
  StepBox box;
  int* box_idx = nullptr;            // pressure index -> box entry
  void *bx_r = nullptr, *bx_d = nullptr;
  void* bx_z[2] = {nullptr, nullptr};
  template <typename X>
  X* alloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&p, n * sizeof(X)) != hipSuccess) throw std::bad_alloc();
    owned.push_back(p);
    if (nan_fill) ETH_HIP(hipMemset(p, 0xff, n * sizeof(X)));   // all-ones bytes: a NaN in FP32 and FP64
    return static_cast<X*>(p);
  }
  void* allocT(size_t n) { return mixed ? (void*)alloc<float>(n) : (void*)alloc<double>(n); }
  void upload(Sell& s, const Csr& A, bool f32, bool dinv);
  void upload_ell(Ell& e, const Csr& A, int off, int count);
  void setup(const eth_step_desc& desc);
  void assemble_wind();   // F levels, K, F1 and the coarse inverse from `wind`
  long long N() const { return ms[0].N(); }
  int nv() const { return ms[0].nv; }
  int nk() const { return ms[0].nk; }
  int n0() const { return ms[0].n0; }

  void apply(const double* x, double* y, const int* gate) {
    launch_sell<double, double>(K, 0, x, 0, nullptr, 0, y, 0, 1, 0.0, 0.0, 0, gate, st);
  }
  template <typename T>
  int cycle_F(int l, const int* gate);
  template <typename T>
  int cycle_Ap(int l, const int* gate);
  template <typename T>
  void vcycle_F(const double* r, const double* sub, double* z, const int* gate);
  template <typename T>
  void pcd(const double* r, double* z, const int* gate);
  template <typename T>
  void m1(const double* r, double* z, const int* gate);
  template <typename T>
  void mq_solve(const int* gate);   // mr (projected) -> mxx (projected)
  template <typename T>
  void mq_solve_box(const int* gate);   // the same on the bounding box
  void precond(int kind, const double* r, double* z, const int* gate) {
    if (mixed) kind == 2 ? pcd<float>(r, z, gate) : m1<float>(r, z, gate);
    else kind == 2 ? pcd<double>(r, z, gate) : m1<double>(r, z, gate);
  }
  const int* gm_gate() const { return &d_gm[0].active; }
  void arnoldi_steps(int kind, bool reduced, int j0, int j1);
  void arnoldi_steps_graph(int kind, bool reduced, int j0, int j1);
  void run_fgmres(int kind, bool reduced, const double* b, double* x, int m, int maxit, double atol,
                  bool use_graph);
  int solve(const eth_solve_opts& o, const double* b, double* x, eth_solve_info* info,
            std::vector<double>* hist_out);
  double norm(const double* v);
};

StepProblem::~StepProblem() {
  if (st) (void)hipStreamSynchronize(st);
  for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
  if (gst) (void)hipStreamDestroy(gst);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  for (void* p : owned) (void)hipFree(p);
  if (h_gm) (void)hipHostFree(h_gm);
  if (h_red) (void)hipHostFree(h_red);
  if (own_stream && st) (void)hipStreamDestroy(st);
}

// CSR -> sliced ELL (64 rows per slice, column-major within a slice); padded
// entries repeat the row's last column with value 0
void StepProblem::upload(Sell& s, const Csr& A, bool f32, bool dinv) {
  const int slices = (A.rows + 63) / 64;
  std::vector<int> ptr, col;
  std::vector<double> val;
  sell_layout(A, ptr, col, val);
  const size_t tot = (size_t)ptr[slices];
  const bool same = s.ptr && s.rows == A.rows && s.stored == (long long)tot;
  if (!same) {
    s.rows = A.rows;
    s.cols = A.cols;
    s.stored = (long long)tot;
    s.ptr = alloc<int>(slices + 1);
    s.col = alloc<int>(tot);
    s.val = alloc<double>(tot);
    s.valf = f32 ? alloc<float>(tot) : nullptr;
    if (dinv) {
      s.dinv = alloc<double>(A.rows);
      s.dinvf = f32 ? alloc<float>(A.rows) : nullptr;
    }
  }
  ETH_HIP(hipMemcpy(s.ptr, ptr.data(), sizeof(int) * ptr.size(), hipMemcpyHostToDevice));
  ETH_HIP(hipMemcpy(s.col, col.data(), sizeof(int) * tot, hipMemcpyHostToDevice));
  ETH_HIP(hipMemcpy(s.val, val.data(), sizeof(double) * tot, hipMemcpyHostToDevice));
  if (s.valf) {
    std::vector<float> vf(val.begin(), val.end());
    ETH_HIP(hipMemcpy(s.valf, vf.data(), sizeof(float) * tot, hipMemcpyHostToDevice));
  }
  if (s.dinv) {
    std::vector<double> di(A.rows);
    for (int r = 0; r < A.rows; ++r) {
      const double dd = A.diag(r);
      di[r] = dd != 0.0 ? 1.0 / dd : 0.0;
    }
    ETH_HIP(hipMemcpy(s.dinv, di.data(), sizeof(double) * A.rows, hipMemcpyHostToDevice));
    if (s.dinvf) {
      std::vector<float> df(di.begin(), di.end());
      ETH_HIP(hipMemcpy(s.dinvf, df.data(), sizeof(float) * A.rows, hipMemcpyHostToDevice));
    }
  }
}

// rows [off, off + count) of A as an ELL block (entry k of row i at
// k * count + i; padding repeats the row's last column with value 0)
void StepProblem::upload_ell(Ell& e, const Csr& A, int off, int count) {
  int w = 0;
  for (int i = 0; i < count; ++i) w = std::max(w, A.ptr[off + i + 1] - A.ptr[off + i]);
  std::vector<int> col((size_t)w * count, 0);
  std::vector<double> val((size_t)w * count, 0.0), di(count, 0.0);
  for (int i = 0; i < count; ++i) {
    const int r = off + i, b = A.ptr[r], len = A.ptr[r + 1] - b;
    int last = r;
    for (int k = 0; k < w; ++k) {
      if (k < len) {
        last = A.col[b + k];
        val[(size_t)k * count + i] = A.val[b + k];
      }
      col[(size_t)k * count + i] = last;
    }
    const double dd = A.diag(r);
    di[i] = dd != 0.0 ? 1.0 / dd : 0.0;
  }
  e.off = off;
  e.count = count;
  e.width = w;
  e.col = alloc<int>(col.size());
  e.val = alloc<double>(val.size());
  e.dinv = alloc<double>(count);
  ETH_HIP(hipMemcpy(e.col, col.data(), sizeof(int) * col.size(), hipMemcpyHostToDevice));
  ETH_HIP(hipMemcpy(e.val, val.data(), sizeof(double) * val.size(), hipMemcpyHostToDevice));
  ETH_HIP(hipMemcpy(e.dinv, di.data(), sizeof(double) * di.size(), hipMemcpyHostToDevice));
  if (mixed) {
    std::vector<float> vf(val.begin(), val.end()), df(di.begin(), di.end());
    e.valf = alloc<float>(vf.size());
    e.dinvf = alloc<float>(df.size());
    ETH_HIP(hipMemcpy(e.valf, vf.data(), sizeof(float) * vf.size(), hipMemcpyHostToDevice));
    ETH_HIP(hipMemcpy(e.dinvf, df.data(), sizeof(float) * df.size(), hipMemcpyHostToDevice));
  }
}

void StepProblem::setup(const eth_step_desc& desc) {
  Range range("eth_step_setup");
  d = desc;
  if (const char* e = std::getenv("ETH_DEBUG_NAN_FILL")) nan_fill = (e[0] == '1');
  if (const char* e = std::getenv("ETH_DEBUG_UNFUSED_MQ")) sgs_split = (e[0] == '1');
  if (const char* e = std::getenv("ETH_DEBUG_STEP_MQ_ELL")) mq_box = (e[0] != '1');
  if (d.m < 1) throw std::invalid_argument("m must be >= 1");
  if (d.length == 0) d.length = 5;
  if (d.length < 1) throw std::invalid_argument("length must be >= 1");
  if (!(d.nu > 0.0)) throw std::invalid_argument("nu must be > 0");
  if (d.precision != ETH_FP64 && d.precision != ETH_MIXED) throw std::invalid_argument("invalid precision");
  mixed = d.precision == ETH_MIXED;
  if (d.coarse_m <= 0) d.coarse_m = 4;
  if (d.gmg_omega <= 0.0) d.gmg_omega = 0.7;
  if (d.gmg_peclet_max < 0.0) throw std::invalid_argument("gmg_peclet_max must be >= 0");
  if (d.pcd_q1_steps <= 0) d.pcd_q1_steps = 10;
  if (d.pcd_inflow_bc != 0 && d.pcd_inflow_bc != 1) throw std::invalid_argument("pcd_inflow_bc must be 0 or 1");
  if (d.mq_steps <= 0) d.mq_steps = 20;
  if (d.mq_cheb_lo <= 0.0) d.mq_cheb_lo = std::min(0.01, 0.4 / ((double)d.m * (1 + d.length)));
  if (!(d.mq_cheb_lo < 1.0)) throw std::invalid_argument("mq_cheb_lo must be < 1");
  if (d.gmres_restart <= 0) d.gmres_restart = 50;
  if (d.gmres_restart > 63) throw std::invalid_argument("gmres_restart must be <= 63");
  gm_m = d.gmres_restart;
  if (d.stream) {
    st = static_cast<hipStream_t>(d.stream);
  } else {
    ETH_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    own_stream = true;
  }
  // hierarchy
  std::vector<int> mlev{d.m};
  while (mlev.back() % 2 == 0 && mlev.back() > d.coarse_m) mlev.push_back(mlev.back() / 2);
  ms.resize(mlev.size());
  el.resize(mlev.size());
  for (size_t l = 0; l < mlev.size(); ++l) {
    ms[l].build(mlev[l], d.length, d.channel != 0);
    el[l].build(ms[l].h);
  }
  if (ms.back().nv > 4000) throw std::invalid_argument("coarsest step level too large for the dense solve (m must be 2^k * c with c <= coarse_m small)");
  const int L = (int)ms.size();
  const StepMesh& g = ms[0];
  // fixed operators
  B = step_assemble_B(g, el[0]);
  {
    // the velocity rows of K restricted to its pressure columns, entries in
    // K's order (so B^T z_p here has the bits of K [0; z_p])
    const Csr T = csr_transpose(B);   // 2 n_v x n_p
    Csr Bv;
    Bv.rows = T.rows;
    Bv.cols = T.cols;
    Bv.ptr.assign(T.rows + 1, 0);
    for (int r = 0; r < T.rows; ++r) {
      if (!g.dirichlet[r % g.nv])
        for (int k = T.ptr[r]; k < T.ptr[r + 1]; ++k) {
          Bv.col.push_back(T.col[k]);
          Bv.val.push_back(T.val[k]);
        }
      Bv.ptr[r + 1] = (int)Bv.col.size();
    }
    upload(Bt, Bv, false, false);
  }
  upload(Q1, step_assemble_Q1(g, el[0]), mixed, true);
  F.resize(L);
  P.resize(L > 1 ? L - 1 : 0);
  R.resize(P.size());
  Ap.resize(L);
  Pq.resize(P.size());
  Rq.resize(P.size());
  std::vector<Csr> aph(L);
  for (int l = 0; l < L; ++l) {
    const Csr Bl = l == 0 ? B : step_assemble_B(ms[l], el[l]);
    aph[l] = step_assemble_Ap(ms[l], el[l], Bl);
    upload(Ap[l], aph[l], mixed, true);
  }
  for (int l = 0; l + 1 < L; ++l) {
    const Csr p = step_q2_prolongation(ms[l], ms[l + 1]);
    upload(P[l], p, mixed, false);
    upload(R[l], csr_transpose(p), mixed, false);
    const Csr pq = step_q1_prolongation(ms[l], ms[l + 1]);
    upload(Pq[l], pq, mixed, false);
    upload(Rq[l], csr_transpose(pq), mixed, false);
  }
  ap_lam.assign(L > 1 ? L - 1 : 0, 0.0);
  ap_a.resize(ap_lam.size());
  ap_b.resize(ap_lam.size());
  for (int l = 0; l + 1 < L; ++l) {
    ap_lam[l] = lambda_max_dinv(aph[l]);
    std::vector<double> a, b;
    cheb_ab(0.3 * ap_lam[l], 1.1 * ap_lam[l], 2, a, b);
    ap_a[l] = {a[0], a[1]};
    ap_b[l] = {b[0], b[1]};
  }
  {
    const std::vector<double> inv = dense_inverse(aph[L - 1]);
    nAc = aph[L - 1].rows;
    Apinv = alloc<double>(inv.size());
    ETH_HIP(hipMemcpy(Apinv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice));
  }
  cheb_ab(0.25, 2.25, d.pcd_q1_steps, q1a, q1b);
  cheb_ab(d.mq_cheb_lo, 1.0, d.mq_steps, mqa, mqb);
  // multicolour classes of M_Q: Q1 node parities (I mod 2) + 2 (J mod 2),
  // then the elements; M_Q is stored with its rows and columns in this order
  {
    std::array<std::vector<int>, 5> rows;
    for (int k = 0; k < g.nk; ++k) rows[(g.q1_I[k] & 1) + 2 * (g.q1_J[k] & 1)].push_back(k);
    for (int e = 0; e < g.n0; ++e) rows[4].push_back(g.nk + e);
    const int np = g.nk + g.n0;
    std::vector<int> perm, inv(np);
    std::array<int, 6> off{};
    for (int c = 0; c < 5; ++c) {
      off[c] = (int)perm.size();
      perm.insert(perm.end(), rows[c].begin(), rows[c].end());
    }
    off[5] = np;
    for (int i = 0; i < np; ++i) inv[perm[i]] = i;
    const Csr M = step_assemble_MQ(g, el[0]);
    Csr Mp;
    Mp.rows = Mp.cols = np;
    Mp.ptr.assign(np + 1, 0);
    std::vector<std::pair<int, double>> row;
    for (int i = 0; i < np; ++i) {
      const int r = perm[i];
      row.clear();
      for (int k = M.ptr[r]; k < M.ptr[r + 1]; ++k) row.emplace_back(inv[M.col[k]], M.val[k]);
      std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
      for (const auto& e : row) {
        Mp.col.push_back(e.first);
        Mp.val.push_back(e.second);
      }
      Mp.ptr[i + 1] = (int)Mp.col.size();
    }
    upload(MQ, Mp, mixed, true);
    for (int c = 0; c < 5; ++c) {
      upload_ell(mq_ell[c], Mp, off[c], off[c + 1] - off[c]);
    }
    std::vector<unsigned char> col(np);
    for (int c = 0; c < 5; ++c)
      for (int i = off[c]; i < off[c + 1]; ++i) col[i] = (unsigned char)c;
    mq_colour = alloc<unsigned char>(col.size());
    ETH_HIP(hipMemcpy(mq_colour, col.data(), col.size(), hipMemcpyHostToDevice));
    mq_perm = alloc<int>(perm.size());
    ETH_HIP(hipMemcpy(mq_perm, perm.data(), sizeof(int) * perm.size(), hipMemcpyHostToDevice));
  }
  // the bounding box of the pressure-mass solve: the absent elements must
  // be the corner e < hx, f < hy
  {
    box.ex = g.ex;
    box.ey = g.ey;
    box.h = g.h;
    int hx = 0, hy = 0;
    while (hx < g.ex && !g.elem_act[hx]) ++hx;
    while (hy < g.ey && !g.elem_act[(size_t)hy * g.ex]) ++hy;
    box.hx = hx;
    box.hy = hy;
    for (int f = 0; f < g.ey; ++f)
      for (int e = 0; e < g.ex; ++e)
        if ((g.elem_act[(size_t)f * g.ex + e] != 0) == (e < hx && f < hy))
          throw std::logic_error("step mesh: the absent elements are not a corner of the box");
    if (mq_box) {
      std::vector<int> bi((size_t)g.nk + g.n0);
      const long long nq = (long long)(g.ex + 1) * (g.ey + 1);
      for (int k = 0; k < g.nk; ++k) bi[k] = g.q1_J[k] * (g.ex + 1) + g.q1_I[k];
      for (int e = 0; e < g.n0; ++e) bi[(size_t)g.nk + e] = (int)(nq + (long long)g.el_y[e] * g.ex + g.el_x[e]);
      box_idx = alloc<int>(bi.size());
      ETH_HIP(hipMemcpy(box_idx, bi.data(), sizeof(int) * bi.size(), hipMemcpyHostToDevice));
      // absent entries are never written: zero them once
      const size_t bytes = (size_t)box.size() * (mixed ? sizeof(float) : sizeof(double));
      for (void** p : {&bx_r, &bx_d, &bx_z[0], &bx_z[1]}) {
        *p = allocT((size_t)box.size());
        ETH_HIP(hipMemset(*p, 0, bytes));
      }
      mq_box_tile = step_mq_tiles(box, 16) >= 128 ? 16 : 8;
      if (const char* e = std::getenv("ETH_STEP_MQ_TILE")) {
        const int t = std::atoi(e);
        if (t != 8 && t != 16) throw std::invalid_argument("ETH_STEP_MQ_TILE must be 8 or 16");
        mq_box_tile = t;
      }
    }
  }
  {
    std::vector<int> di;
    for (int c = 0; c < 2; ++c)
      for (int i = 0; i < g.nv; ++i)
        if (g.dirichlet[i]) di.push_back(c * g.nv + i);
    ndir = (int)di.size();
    dir_idx = alloc<int>(di.size());
    ETH_HIP(hipMemcpy(dir_idx, di.data(), sizeof(int) * di.size(), hipMemcpyHostToDevice));
  }
  // workspaces
  const long long n = N();
  kb = alloc<double>(n);
  kx = alloc<double>(n);
  ky = alloc<double>(n);
  kz = alloc<double>(n);
  kv = alloc<double>(n);
  kw = alloc<double>(n);
  kpb = alloc<double>(n);
  vb.resize(L);
  vt.resize(L);
  vx.resize(L);
  qb.resize(L);
  qt.resize(L);
  qx.resize(L);
  for (int l = 0; l < L; ++l) {
    const size_t nvl = 2 * (size_t)ms[l].nv, nkl = ms[l].nk;
    vb[l] = allocT(nvl);
    vt[l] = allocT(nvl);
    vx[l] = {allocT(nvl), allocT(nvl)};
    qb[l] = allocT(nkl);
    qt[l] = allocT(nkl);
    qx[l] = {allocT(nkl), allocT(nkl)};
  }
  q1x[0] = allocT(g.nk);
  q1x[1] = allocT(g.nk);
  const size_t np = (size_t)g.nk + g.n0;
  mr = allocT(np);
  mxx = allocT(np);
  md = allocT(np);
  msg = allocT(np);
  mres = allocT(np);
  fpart = alloc<double>(frame_project_blocks((int)np) + 1);
  p0part = alloc<double>(g.n0 / 1024 + 2);
  // FGMRES
  gV = alloc<double>((size_t)n * (gm_m + 1));
  gZ = alloc<double>((size_t)n * gm_m);
  gArr = alloc<double>((size_t)(gm_m + 1) * gm_m + 7 * 64);
  gpart = alloc<double>((size_t)64 * gmres_blocks(n));
  ghist = alloc<double>(hist_len);
  d_gm = alloc<GmresScalars>(1);
  ETH_HIP(hipHostMalloc((void**)&h_gm, sizeof(GmresScalars), hipHostMallocDefault));
  ETH_HIP(hipHostMalloc((void**)&h_red, sizeof(double) * 4, hipHostMallocDefault));
  red_part = alloc<double>(dot_blocks(n) + 1);
  red_res = alloc<double>(4);
  wind.assign(2 * (size_t)g.nv, 0.0);
  has_wind = false;
  assemble_wind();
}

// F on every level (injected wind, level viscosity), K, F_1 and the coarsest
// F inverse from the host wind
void StepProblem::assemble_wind() {
  Range range("eth_step_assemble_wind");
  const int L = (int)ms.size();
  double wmax = 0.0;
  for (int i = 0; i < ms[0].nv; ++i)
    wmax = std::max(wmax, std::sqrt(wind[i] * wind[i] + wind[ms[0].nv + i] * wind[ms[0].nv + i]));
  lnu.assign(L, d.nu);
  std::vector<double> w = wind;
  Csr Fc;
  for (int l = 0; l < L; ++l) {
    if (l > 0) w = step_inject_wind(w, ms[l - 1], ms[l]);
    if (d.gmg_peclet_max > 0.0 && has_wind) lnu[l] = std::max(d.nu, wmax * ms[l].h / (2.0 * d.gmg_peclet_max));
    const Csr Fl = step_assemble_F(ms[l], el[l], lnu[l], has_wind ? w.data() : nullptr, true);
    upload(F[l], Fl, mixed, true);
    if (l == L - 1) Fc = Fl;
  }
  // the Krylov operator carries the true viscosity whatever the level cap
  const Csr F0 = step_assemble_F(ms[0], el[0], d.nu, has_wind ? wind.data() : nullptr, true);
  upload(K, step_assemble_K(ms[0], F0, B), false, false);
  upload(F1, step_assemble_F1(ms[0], el[0], d.nu, has_wind ? wind.data() : nullptr, d.pcd_inflow_bc == 0), mixed,
         false);
  const std::vector<double> inv = dense_inverse(Fc);
  if (!Finv || nFc != Fc.rows) {
    nFc = Fc.rows;
    Finv = alloc<double>(inv.size());
  }
  ETH_HIP(hipMemcpy(Finv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice));
}

double StepProblem::norm(const double* v) {
  RedCtx rc{red_part, red_res, dot_blocks(N()), 1, 0, nullptr};
  launch_dot(N(), v, v, 0, 1, rc, no_gate(), st);
  ETH_HIP(hipMemcpyAsync(h_red, red_res, sizeof(double), hipMemcpyDeviceToHost, st));
  ETH_HIP(hipStreamSynchronize(st));
  return std::sqrt(h_red[0]);
}

// ---------------------------------------------------------------- V-cycles
template <typename T>
int StepProblem::cycle_F(int l, const int* gate) {
  const int nvl = ms[l].nv;
  T* b = static_cast<T*>(vb[l]);
  T* x0 = static_cast<T*>(vx[l][0]);
  T* x1 = static_cast<T*>(vx[l][1]);
  if (l == (int)ms.size() - 1) {
    launch_dense_apply<T>(Finv, nFc, b, nvl, x0, nvl, 2, gate, st);
    return 0;
  }
  const double w = d.gmg_omega;
  T* xs[2] = {x0, x1};
  launch_sell<T, T>(F[l], 3, (const T*)nullptr, nvl, b, nvl, x0, nvl, 2, w, 0.0, 0, gate, st);
  launch_sell<T, T>(F[l], 3, x0, nvl, b, nvl, x1, nvl, 2, w, 0.0, 0, gate, st);
  int cur = 1;
  T* t = static_cast<T*>(vt[l]);
  launch_sell<T, T>(F[l], 2, xs[cur], nvl, b, nvl, t, nvl, 2, 0.0, 0.0, 0, gate, st);
  const int nvc = ms[l + 1].nv;
  launch_sell<T, T>(R[l], 0, t, nvl, (const T*)nullptr, 0, static_cast<T*>(vb[l + 1]), nvc, 2, 0.0, 0.0, 0, gate,
                    st);
  const int c = cycle_F<T>(l + 1, gate);
  launch_sell<T, T>(P[l], 1, static_cast<const T*>(vx[l + 1][c]), nvc, (const T*)nullptr, 0, xs[cur], nvl, 2,
                    0.0, 0.0, 0, gate, st);
  for (int s = 0; s < 2; ++s) {
    launch_sell<T, T>(F[l], 3, xs[cur], nvl, b, nvl, xs[cur ^ 1], nvl, 2, w, 0.0, 0, gate, st);
    cur ^= 1;
  }
  return cur;
}

template <typename T>
void StepProblem::vcycle_F(const double* r, const double* sub, double* z, const int* gate) {
  const long long n2 = 2LL * nv();
  launch_vcombine<double, T>(n2, 1.0, r, -1.0, sub, static_cast<T*>(vb[0]), gate, st);
  const int c = cycle_F<T>(0, gate);
  launch_vcombine<T, double>(n2, 1.0, static_cast<const T*>(vx[0][c]), 0.0, nullptr, z, gate, st);
}

template <typename T>
int StepProblem::cycle_Ap(int l, const int* gate) {
  const int nkl = ms[l].nk;
  T* b = static_cast<T*>(qb[l]);
  T* xs[2] = {static_cast<T*>(qx[l][0]), static_cast<T*>(qx[l][1])};
  if (l == (int)ms.size() - 1) {
    launch_dense_apply<T>(Apinv, nAc, b, 0, xs[0], 0, 1, gate, st);
    return 0;
  }
  const auto& A = Ap[l];
  const auto& a = ap_a[l];
  const auto& be = ap_b[l];
  launch_sell<T, T>(A, 4, (const T*)nullptr, 0, b, 0, xs[0], 0, 1, be[0], 0.0, 0, gate, st);
  launch_sell<T, T>(A, 4, xs[0], 0, b, 0, xs[1], 0, 1, be[1], a[1], 2, gate, st);
  int cur = 1;
  T* t = static_cast<T*>(qt[l]);
  launch_sell<T, T>(A, 2, xs[cur], 0, b, 0, t, 0, 1, 0.0, 0.0, 0, gate, st);
  launch_sell<T, T>(Rq[l], 0, t, 0, (const T*)nullptr, 0, static_cast<T*>(qb[l + 1]), 0, 1, 0.0, 0.0, 0, gate, st);
  const int c = cycle_Ap<T>(l + 1, gate);
  launch_sell<T, T>(Pq[l], 1, static_cast<const T*>(qx[l + 1][c]), 0, (const T*)nullptr, 0, xs[cur], 0, 1, 0.0,
                    0.0, 0, gate, st);
  // post-smoothing: step 0 into the other array, step 1 back over the first
  launch_sell<T, T>(A, 4, xs[cur], 0, b, 0, xs[cur ^ 1], 0, 1, be[0], 0.0, 0, gate, st);
  launch_sell<T, T>(A, 4, xs[cur ^ 1], 0, b, 0, xs[cur], 0, 1, be[1], a[1], 1, gate, st);
  (void)nkl;
  return cur;
}

// stage-I preconditioner (PCD on the reduced system)
template <typename T>
void StepProblem::pcd(const double* r, double* z, const int* gate) {
  const int nk_ = nk(), nv2 = 2 * nv();
  const GmresScalars* gs = gate ? d_gm : nullptr;
  T* rp = static_cast<T*>(qt[0]);
  launch_vcombine<double, T>(nk_, 1.0, r + nv2, 0.0, nullptr, rp, gate, st);
  // Q_1^{-1} r_p: Chebyshev-Jacobi from zero
  T* q[2] = {static_cast<T*>(q1x[0]), static_cast<T*>(q1x[1])};
  launch_sell<T, T>(Q1, 4, (const T*)nullptr, 0, rp, 0, q[0], 0, 1, q1b[0], 0.0, 0, gate, st);
  int cur = 0;
  for (int k = 1; k < d.pcd_q1_steps; ++k) {
    launch_sell<T, T>(Q1, 4, q[cur], 0, rp, 0, q[cur ^ 1], 0, 1, q1b[k], q1a[k], k == 1 ? 2 : 1, gate, st);
    cur ^= 1;
  }
  // F_1 q, then A_p^{-1}
  launch_sell<T, T>(F1, 0, q[cur], 0, (const T*)nullptr, 0, static_cast<T*>(qb[0]), 0, 1, 0.0, 0.0, 0, gate, st);
  const int c = cycle_Ap<T>(0, gate);
  // z_p = [-x; 0] (z_u is written by the V-cycle below)
  launch_vcombine<T, double>(nk_, -1.0, static_cast<const T*>(qx[0][c]), 0.0, nullptr, z + nv2, gate, st);
  launch_gm_zero_range(z, 0, (long long)nv2 + nk_, n0(), 1, gs, st);
  // z_u = F^{-1}(r_u - B_1^T z_p)
  launch_sell<double, double>(Bt, 0, z + nv2, 0, nullptr, 0, kw, 0, 1, 0.0, 0.0, 0, gate, st);
  vcycle_F<T>(r, kw, z, gate);
}

template <typename T>
void StepProblem::mq_solve(const int* gate) {
  const int nk_ = nk(), n0_ = n0(), np = nk_ + n0_;
  T* r = static_cast<T*>(mr);
  T* x = static_cast<T*>(mxx);
  T* dd = static_cast<T*>(md);
  T* s = static_cast<T*>(msg);
  T* res = static_cast<T*>(mres);
  launch_frame_project(fpart, nk_, n0_, r, mixed, gate, st);
  // x_1 = d_0 = SGS(r) / theta;  x_{k+1} = x_k + d_k,  d_k = alpha_k d_{k-1} + beta_k SGS(r - M x_k);
  // the sweep from zero visits the colours 0, 1, 2, 3, 4, 3, 2, 1, 0
  for (int k = 0; k < d.mq_steps; ++k) {
    launch_sgs_enter<T, T>(MQ, mq_colour, k == 0 ? nullptr : x, r, res, s, gate, st);
    launch_ell_colour<T, T>(mq_ell[1], res, s, gate, st);
    launch_ell_colour<T, T>(mq_ell[2], res, s, gate, st);
    if (sgs_split) {
      launch_ell_colour<T, T>(mq_ell[3], res, s, gate, st);
      launch_ell_colour<T, T>(mq_ell[4], res, s, gate, st);
      launch_ell_colour<T, T>(mq_ell[3], res, s, gate, st);
    } else {
      launch_ell_middle<T, T>(mq_ell[3], mq_ell[4], res, s, gate, st);
    }
    launch_ell_colour<T, T>(mq_ell[2], res, s, gate, st);
    launch_ell_colour<T, T>(mq_ell[1], res, s, gate, st);
    launch_sgs_leave<T, T>(MQ, mq_colour, res, s, dd, x, mqa[k], mqb[k], k == 0 ? 1 : 0, gate, st);
  }
  (void)np;
  launch_frame_project(fpart, nk_, n0_, x, mixed, gate, st);
}

// The same solve on the bounding box: the projected input scattered to the
// box, one fused launch per Chebyshev step, the result gathered back and
// projected.
template <typename T>
void StepProblem::mq_solve_box(const int* gate) {
  const int nk_ = nk(), n0_ = n0(), np = nk_ + n0_;
  launch_frame_project(fpart, nk_, n0_, mr, mixed, gate, st);
  launch_permute<T, T>(np, box_idx, true, 1.0, static_cast<const T*>(mr), static_cast<T*>(bx_r), gate, st);
  for (int k = 0; k < d.mq_steps; ++k)
    launch_step_mq_fused<T>(box, mq_box_tile, static_cast<const T*>(bx_r), static_cast<const T*>(bx_z[k & 1]),
                            static_cast<T*>(bx_z[(k + 1) & 1]), static_cast<T*>(bx_d), mqa[k], mqb[k],
                            k == 0 ? 1 : 0, gate, st);
  launch_permute<T, T>(np, box_idx, false, 1.0, static_cast<const T*>(bx_z[d.mq_steps & 1]),
                       static_cast<T*>(mxx), gate, st);
  launch_frame_project(fpart, nk_, n0_, mxx, mixed, gate, st);
}

// stage-II preconditioner M_1
template <typename T>
void StepProblem::m1(const double* r, double* z, const int* gate) {
  const int nv2 = 2 * nv(), np = nk() + n0();
  if (mq_box) {
    launch_vcombine<double, T>(np, 1.0, r + nv2, 0.0, nullptr, static_cast<T*>(mr), gate, st);
    mq_solve_box<T>(gate);
    launch_vcombine<T, double>(np, -d.nu, static_cast<const T*>(mxx), 0.0, nullptr, z + nv2, gate, st);
  } else {
    launch_permute<double, T>(np, mq_perm, false, 1.0, r + nv2, static_cast<T*>(mr), gate, st);
    mq_solve<T>(gate);
    launch_permute<T, double>(np, mq_perm, true, -d.nu, static_cast<const T*>(mxx), z + nv2, gate, st);
  }
  launch_sell<double, double>(Bt, 0, z + nv2, 0, nullptr, 0, kw, 0, 1, 0.0, 0.0, 0, gate, st);
  vcycle_F<T>(r, kw, z, gate);
}

// ------------------------------------------------------------------ FGMRES
void StepProblem::arnoldi_steps(int kind, bool reduced, int j0, int j1) {
  const long long n = N();
  const int* gate = gm_gate();
  auto V = [&](int i) { return gV + (size_t)i * n; };
  auto Z = [&](int i) { return gZ + (size_t)i * n; };
  for (int j = j0; j < j1; ++j) {
    precond(kind, V(j), Z(j), gate);
    apply(Z(j), V(j + 1), gate);
    if (reduced) launch_gm_zero_range(V(j + 1), n, 2LL * nv() + nk(), n0(), 1, d_gm, st);
    launch_gm_mdot(n, j + 1, gV, V(j + 1), n, 1, gpart, d_gm, 0, st);
    launch_gm_maxpy(n, j + 1, gV, V(j + 1), n, 1, d_gm, 0, st);
    launch_gm_mdot(n, j + 1, gV, V(j + 1), n, 1, gpart, d_gm, 1, st);
    launch_gm_maxpy(n, j + 1, gV, V(j + 1), n, 1, d_gm, 1, st);
    launch_gm_norm_givens(n, j, V(j + 1), n, 1, gpart, d_gm, st);
    launch_gm_scale(n, V(j + 1), n, 1, d_gm, st);
  }
}

void StepProblem::arnoldi_steps_graph(int kind, bool reduced, int j0, int j1) {
  if (!gst) {
    ETH_HIP(hipStreamCreateWithFlags(&gst, hipStreamNonBlocking));
    ETH_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    ETH_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
  }
  hipStream_t caller = st;
  ETH_HIP(hipEventRecord(ev_fork, caller));
  ETH_HIP(hipStreamWaitEvent(gst, ev_fork, 0));
  st = gst;
  struct Restore {
    hipStream_t& s;
    hipStream_t v;
    ~Restore() { s = v; }
  } restore{st, caller};
  const std::array<int, 4> key{kind, reduced ? 1 : 0, j0, j1};
  auto it = graphs.find(key);
  if (it == graphs.end()) {
    hipGraph_t graph;
    ETH_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      arnoldi_steps(kind, reduced, j0, j1);
    } catch (...) {
      hipGraph_t discard;
      (void)hipStreamEndCapture(st, &discard);
      if (discard) (void)hipGraphDestroy(discard);
      throw;
    }
    ETH_HIP(hipStreamEndCapture(st, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    ETH_HIP(e);
    it = graphs.emplace(key, exec).first;
  }
  ETH_HIP(hipGraphLaunch(it->second, gst));
  ETH_HIP(hipEventRecord(ev_join, gst));
  ETH_HIP(hipStreamWaitEvent(caller, ev_join, 0));
}

void StepProblem::run_fgmres(int kind, bool reduced, const double* b, double* x, int m, int maxit, double atol,
                             bool use_graph) {
  const long long n = N();
  GmresScalars& G = *h_gm;
  std::memset(&G, 0, sizeof(G));
  G.target = atol;
  G.m = m;
  G.maxit = maxit;
  G.H = gArr;
  G.cs = gArr + (size_t)(gm_m + 1) * gm_m;
  G.sn = G.cs + 64;
  G.g = G.sn + 64;
  G.y = G.g + 64;
  G.h1 = G.y + 64;
  G.h2 = G.h1 + 64;
  G.hist = ghist;
  G.hist_len = hist_len;
  ETH_HIP(hipMemcpyAsync(d_gm, h_gm, sizeof(GmresScalars), hipMemcpyHostToDevice, st));
  auto op = [&](const double* in, double* out) {
    apply(in, out, nullptr);
    if (reduced) launch_gm_zero_range(out, n, 2LL * nv() + nk(), n0(), 1, nullptr, st);
  };
  for (int cycle = 0; cycle < 100000; ++cycle) {
    op(x, ky);
    launch_vcombine<double, double>(n, 1.0, b, -1.0, ky, gV, nullptr, st);
    launch_gm_beta(n, gV, n, 1, gpart, d_gm, st);
    launch_gm_scale(n, gV, n, 1, d_gm, st);
    for (int j0 = 0; j0 < m; j0 += 8) {
      const int j1 = std::min(j0 + 8, m);
      if (use_graph) arnoldi_steps_graph(kind, reduced, j0, j1);
      else arnoldi_steps(kind, reduced, j0, j1);
      if (j1 < m) {
        ETH_HIP(hipMemcpyAsync(h_gm, d_gm, sizeof(GmresScalars), hipMemcpyDeviceToHost, st));
        ETH_HIP(hipStreamSynchronize(st));
        if (!h_gm->active) break;
      }
    }
    launch_gm_finish(n, gZ, x, n, 1, d_gm, st);
    ETH_HIP(hipMemcpyAsync(h_gm, d_gm, sizeof(GmresScalars), hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    if (!(!h_gm->converged && h_gm->status >= 0 && h_gm->iters < maxit)) {
      op(x, ky);
      launch_vcombine<double, double>(n, 1.0, b, -1.0, ky, gV, nullptr, st);
      launch_gm_beta(n, gV, n, 1, gpart, d_gm, st);
      ETH_HIP(hipMemcpyAsync(h_gm, d_gm, sizeof(GmresScalars), hipMemcpyDeviceToHost, st));
      ETH_HIP(hipStreamSynchronize(st));
      break;
    }
  }
}

int StepProblem::solve(const eth_solve_opts& o, const double* b, double* x, eth_solve_info* info,
                       std::vector<double>* hist_out) {
  Range range("eth_step_solve");
  const double eta = o.rtol > 0 ? o.rtol : 1e-6;
  const int maxit = o.maxit > 0 ? o.maxit : 1000;
  const int m = o.restart > 0 ? o.restart : gm_m;
  if (m > gm_m) throw std::invalid_argument("restart exceeds the gmres_restart of the problem");
  const double c = o.c_factor > 0 ? o.c_factor : 10.0;
  const long long n = N();
  const int nv2 = 2 * nv();
  if (o.method == ETH_TWO_STAGE && !has_wind)
    throw std::runtime_error("unsupported:the two-stage PCD needs a wind (F_1 without convection is singular); "
                             "use ETH_FGMRES (M_1) for the Stokes operator");
  // Krylov right-hand side: Dirichlet rows zeroed
  launch_copy(n, b, n, kb, n, 1, st);
  hipLaunchKernelGGL(k_scatter_zero, dim3(nblk(ndir)), dim3(NT), 0, st, dir_idx, ndir, kb);
  ETH_LAUNCH_CHECK();
  const double bn = norm(kb);
  if (!std::isfinite(bn)) throw std::invalid_argument("right-hand side holds a NaN or Inf");
  {
    // consistency with null(K^T) = span{[0; k]}: k . b_p = 0 (for the lifted
    // right-hand side k . b_p = -(B^T k) . u_B = 0 exactly)
    const int nb = frame_project_blocks(nk() + n0());
    launch_frame_partials(fpart, nk(), n0(), kb + nv2, st);
    std::vector<double> part(nb);
    ETH_HIP(hipMemcpyAsync(part.data(), fpart, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    double kb_dot = 0.0;
    for (double v : part) kb_dot += v;
    const double kn = std::sqrt((double)(nk() + n0()));
    if (std::fabs(kb_dot) > 1e-10 * kn * std::max(bn, 1e-300))
      throw std::runtime_error("inconsistent:right-hand side not orthogonal to null(K^T): k . b_p = " +
                               std::to_string(kb_dot));
  }
  double r0 = bn;
  if (o.use_x0) {
    launch_copy(n, x, n, kx, n, 1, st);
    hipLaunchKernelGGL(k_scatter_zero, dim3(nblk(ndir)), dim3(NT), 0, st, dir_idx, ndir, kx);
    ETH_LAUNCH_CHECK();
    launch_copy(n, kx, n, kv, n, 1, st);   // kept: the result falls back to it
    apply(kx, ky, nullptr);
    launch_vcombine<double, double>(n, 1.0, kb, -1.0, ky, kz, nullptr, st);
    r0 = norm(kz);
  } else {
    launch_fill(n, 0.0, kx, n, 1, st);
  }
  std::vector<double> hist;
  auto take_hist = [&]() {
    if (!hist_out) return;
    std::vector<double> hb(hist_len);
    ETH_HIP(hipMemcpyAsync(hb.data(), ghist, sizeof(double) * hist_len, hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    const int k = std::min(h_gm->iters, hist_len - 1);
    for (int j = 0; j <= k; ++j) hist.push_back(bn > 0 ? hb[j] / bn : 0.0);
  };
  int it1 = 0;
  if (o.method == ETH_TWO_STAGE) {
    Range stage("stage I (reduced system, PCD)");
    launch_copy(n, kb, n, kz, n, 1, st);
    launch_gm_zero_range(kz, n, (long long)nv2 + nk(), n0(), 1, nullptr, st);
    launch_gm_zero_range(kx, n, (long long)nv2 + nk(), n0(), 1, nullptr, st);
    run_fgmres(2, true, kz, kx, m, maxit, c * eta * bn, o.use_graph != 0);
    it1 = h_gm->iters;
    take_hist();
  }
  {
    Range stage("stage II (full system, M_1)");
    run_fgmres(1, false, kb, kx, m, maxit, eta * bn, o.use_graph != 0);
    take_hist();
  }
  const bool noprog = h_gm->status >= 0 && h_gm->beta > r0 * (1.0 + 1e-12);
  if (noprog) {
    if (o.use_x0) launch_copy(n, kv, n, kx, n, 1, st);
    else launch_fill(n, 0.0, kx, n, 1, st);
  }
  launch_copy(n, kx, n, x, n, 1, st);
  hipLaunchKernelGGL(k_scatter_copy, dim3(nblk(ndir)), dim3(NT), 0, st, dir_idx, ndir, b, x);
  ETH_LAUNCH_CHECK();
  if (o.canonicalize) {
    const int nb = (n0() + 1023) / 1024;
    hipLaunchKernelGGL(k_p0_partial, dim3(nb), dim3(NT), 0, st, x + nv2 + nk(), n0(), p0part);
    ETH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_p0_shift, dim3(nblk((long long)nk() + n0())), dim3(NT), 0, st, x + nv2, nk(), n0(),
                       p0part, nb);
    ETH_LAUNCH_CHECK();
  }
  ETH_HIP(hipStreamSynchronize(st));
  int status = h_gm->status;
  if (status == kStOK && !h_gm->converged) status = ETH_WMAXIT;
  if (noprog) status = ETH_WNOPROGRESS;
  const double fin = noprog ? r0 : h_gm->beta;
  if (info) {
    info->status = status;
    info->iterations = h_gm->iters + it1;
    info->stage1_iterations = it1;
    info->rel_residual_est = bn > 0 ? fin / bn : 0.0;
    info->rel_residual_true = bn > 0 ? fin / bn : 0.0;
  }
  if (hist_out) *hist_out = hist;
  return status;
}

}  // namespace eth

// =============================================================================
// C ABI
// =============================================================================
struct eth_step {
  eth::StepProblem impl;
};

namespace {
thread_local std::string g_step_setup_error;

int sfail(eth_step* p, int code, const std::string& msg) {
  if (p) p->impl.err = msg;
  else g_step_setup_error = msg;
  return code;
}

template <typename F>
int sguard(eth_step* p, F&& f) {
  try {
    return f();
  } catch (const eth::HipError& e) {
    return sfail(p, ETH_EDEVICE, e.where + ": " + hipGetErrorString(e.err));
  } catch (const std::bad_alloc&) {
    return sfail(p, ETH_ENOMEM, "allocation failed");
  } catch (const std::invalid_argument& e) {
    return sfail(p, ETH_EINVAL, e.what());
  } catch (const std::runtime_error& e) {
    const std::string m = e.what();
    if (m.rfind("unsupported:", 0) == 0) return sfail(p, ETH_EUNSUPPORTED, m.substr(12));
    if (m.rfind("inconsistent:", 0) == 0) return sfail(p, ETH_EINCONSISTENT, m.substr(13));
    return sfail(p, ETH_EDEVICE, m);
  }
}

// host-side assembly of one named matrix (no device involved)
struct HostStep {
  std::vector<eth::StepMesh> ms;
  std::vector<eth::StepElem> el;
};
}  // namespace

extern "C" {

int eth_step_setup(const eth_step_desc* desc, eth_step** out) {
  if (!out) return sfail(nullptr, ETH_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc) return sfail(nullptr, ETH_EINVAL, "desc is NULL");
  eth_step* p = new (std::nothrow) eth_step();
  if (!p) return sfail(nullptr, ETH_ENOMEM, "host allocation failed");
  const int rc = sguard(p, [&] {
    p->impl.setup(*desc);
    return ETH_OK;
  });
  if (rc != ETH_OK) {
    g_step_setup_error = p->impl.err;
    delete p;
    return rc;
  }
  *out = p;
  return ETH_OK;
}

int eth_step_destroy(eth_step* p) {
  if (!p) return ETH_EINVAL;
  delete p;
  return ETH_OK;
}

int eth_step_sizes(const eth_step* p, int64_t* nv, int64_t* nk, int64_t* n0, int64_t* N) {
  if (!p) return ETH_EINVAL;
  const eth::StepMesh& g = p->impl.ms[0];
  if (nv) *nv = g.nv;
  if (nk) *nk = g.nk;
  if (n0) *n0 = g.n0;
  if (N) *N = g.N();
  return ETH_OK;
}

int eth_step_levels(const eth_step* p, int32_t* levels, int32_t* m_per_level, double* ap_lambdas) {
  if (!p) return ETH_EINVAL;
  const auto& P = p->impl;
  if (levels) *levels = (int32_t)P.ms.size();
  if (m_per_level)
    for (size_t l = 0; l < P.ms.size(); ++l) m_per_level[l] = P.ms[l].m;
  if (ap_lambdas)
    for (size_t l = 0; l < P.ap_lam.size(); ++l) ap_lambdas[l] = P.ap_lam[l];
  return ETH_OK;
}

int eth_step_set_wind(eth_step* p, const double* wind) {
  if (!p) return sfail(p, ETH_EINVAL, "NULL handle");
  return sguard(p, [&] {
    auto& P = p->impl;
    if (wind) {
      ETH_HIP(hipMemcpyAsync(P.wind.data(), wind, sizeof(double) * P.wind.size(), hipMemcpyDeviceToHost, P.st));
      ETH_HIP(hipStreamSynchronize(P.st));
      for (double v : P.wind)
        if (!std::isfinite(v)) throw std::invalid_argument("wind holds a NaN or Inf");
      P.has_wind = true;
    } else {
      std::fill(P.wind.begin(), P.wind.end(), 0.0);
      P.has_wind = false;
    }
    P.assemble_wind();
    return ETH_OK;
  });
}

int eth_step_rhs(eth_step* p, double* b) {
  if (!p || !b) return sfail(p, ETH_EINVAL, "NULL argument");
  return sguard(p, [&] {
    auto& P = p->impl;
    const eth::Csr Ff = eth::step_assemble_F(P.ms[0], P.el[0], P.d.nu, P.has_wind ? P.wind.data() : nullptr, false);
    const std::vector<double> h = eth::step_lift(P.ms[0], Ff, P.B, eth::step_inflow(P.ms[0]));
    ETH_HIP(hipMemcpyAsync(b, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, P.st));
    ETH_HIP(hipStreamSynchronize(P.st));
    return ETH_OK;
  });
}

int eth_step_apply(eth_step* p, const double* x, double* y) {
  if (!p || !x || !y) return sfail(p, ETH_EINVAL, "NULL argument");
  if (x == y) return sfail(p, ETH_EINVAL, "x and y must not alias");
  return sguard(p, [&] {
    p->impl.apply(x, y, nullptr);
    return ETH_OK;
  });
}

int eth_step_apply_preconditioner(eth_step* p, int32_t which, const double* r, double* z) {
  if (!p || !r || !z) return sfail(p, ETH_EINVAL, "NULL argument");
  if (r == z) return sfail(p, ETH_EINVAL, "r and z must not alias");
  if (which != 1 && which != 2) return sfail(p, ETH_EINVAL, "which must be 1 (M_1) or 2 (stage-I PCD)");
  return sguard(p, [&] {
    auto& P = p->impl;
    const long long n = P.N();
    eth::launch_copy(n, r, n, P.kv, n, 1, P.st);
    P.precond(which, P.kv, P.kz, nullptr);
    eth::launch_copy(n, P.kz, n, z, n, 1, P.st);
    return ETH_OK;
  });
}

int eth_step_solve(eth_step* p, const eth_solve_opts* opts, const double* b, double* x, eth_solve_info* info) {
  if (!p || !b || !x) return sfail(p, ETH_EINVAL, "NULL argument");
  if (b == x) return sfail(p, ETH_EINVAL, "b and x must not alias");
  eth_solve_opts o{};
  if (opts) {
    o = *opts;
  } else {
    o.canonicalize = 1;
    o.method = ETH_TWO_STAGE;
  }
  if (o.method != ETH_FGMRES && o.method != ETH_TWO_STAGE)
    return sfail(p, ETH_EUNSUPPORTED, "step problems are solved by FGMRES (M_1) or TWO_STAGE");
  if (o.maxit > 4096) return sfail(p, ETH_EINVAL, "maxit > 4096");
  if (o.residual_history && o.history_len < 1) return sfail(p, ETH_EINVAL, "history_len must be >= 1");
  return sguard(p, [&] {
    std::vector<double> hist;
    const int s = p->impl.solve(o, b, x, info, o.residual_history ? &hist : nullptr);
    if (o.residual_history)
      for (int j = 0; j < o.history_len; ++j) o.residual_history[j] = j < (int)hist.size() ? hist[j] : -1.0;
    return s;
  });
}

int eth_step_picard(eth_step* p, const eth_solve_opts* opts, int32_t steps, double* x, eth_solve_info* info) {
  if (!p || !x) return sfail(p, ETH_EINVAL, "NULL argument");
  if (steps < 0) return sfail(p, ETH_EINVAL, "steps must be >= 0");
  eth_solve_opts o{};
  if (opts) {
    o = *opts;
  } else {
    o.canonicalize = 1;
    o.method = ETH_TWO_STAGE;
  }
  if (o.method != ETH_FGMRES && o.method != ETH_TWO_STAGE)
    return sfail(p, ETH_EUNSUPPORTED, "step problems are solved by FGMRES (M_1) or TWO_STAGE");
  if (o.maxit > 4096) return sfail(p, ETH_EINVAL, "maxit > 4096");
  o.residual_history = nullptr;
  return sguard(p, [&] {
    auto& P = p->impl;
    const long long n = P.N();
    std::vector<double> bh;
    int worst = ETH_OK;
    auto rhs = [&]() {
      const eth::Csr Ff = eth::step_assemble_F(P.ms[0], P.el[0], P.d.nu, P.has_wind ? P.wind.data() : nullptr, false);
      bh = eth::step_lift(P.ms[0], Ff, P.B, eth::step_inflow(P.ms[0]));
      ETH_HIP(hipMemcpyAsync(P.kpb, bh.data(), sizeof(double) * n, hipMemcpyHostToDevice, P.st));
      ETH_HIP(hipStreamSynchronize(P.st));
    };
    // the Stokes start by M_1 (the PCD needs a wind), then Oseen steps whose
    // wind is the whole nodal velocity of the previous iterate
    std::fill(P.wind.begin(), P.wind.end(), 0.0);
    P.has_wind = false;
    P.assemble_wind();
    rhs();
    for (int k = 0; k <= steps; ++k) {
      eth_solve_opts ok = o;
      if (k == 0) {
        ok.method = ETH_FGMRES;
        ok.use_x0 = 0;
      } else {
        ok.use_x0 = 1;
      }
      const int s = P.solve(ok, P.kpb, x, info ? &info[k] : nullptr, nullptr);
      if (s < 0) return s;
      worst = std::max(worst, s);
      if (k == steps) break;
      ETH_HIP(hipMemcpyAsync(P.wind.data(), x, sizeof(double) * P.wind.size(), hipMemcpyDeviceToHost, P.st));
      ETH_HIP(hipStreamSynchronize(P.st));
      P.has_wind = true;
      P.assemble_wind();
      rhs();
    }
    return worst;
  });
}

const char* eth_step_last_error(const eth_step* p) {
  return p ? p->impl.err.c_str() : g_step_setup_error.c_str();
}

// Host-only inspection of the assembly (no device involved)
int eth_step_host_layout(int32_t m, int32_t length, int32_t channel, int64_t* sizes, int32_t* q2_ij,
                         int32_t* q1_ij, int32_t* el_ij, uint8_t* dirichlet) {
  try {
    eth::StepMesh g;
    g.build(m, length > 0 ? length : 5, channel != 0);
    if (sizes) {
      sizes[0] = g.nv;
      sizes[1] = g.nk;
      sizes[2] = g.n0;
      sizes[3] = g.N();
    }
    for (int i = 0; i < g.nv; ++i) {
      if (q2_ij) {
        q2_ij[2 * i] = g.q2_I[i];
        q2_ij[2 * i + 1] = g.q2_J[i];
      }
      if (dirichlet) dirichlet[i] = (uint8_t)g.dirichlet[i];
    }
    if (q1_ij)
      for (int i = 0; i < g.nk; ++i) {
        q1_ij[2 * i] = g.q1_I[i];
        q1_ij[2 * i + 1] = g.q1_J[i];
      }
    if (el_ij)
      for (int i = 0; i < g.n0; ++i) {
        el_ij[2 * i] = g.el_x[i];
        el_ij[2 * i + 1] = g.el_y[i];
      }
    return ETH_OK;
  } catch (const std::exception& e) {
    g_step_setup_error = e.what();
    return ETH_EINVAL;
  }
}

int eth_step_host_matrix(int32_t m, int32_t length, int32_t channel, double nu, const double* wind, int32_t which,
                         int64_t* rows, int64_t* cols, int64_t* nnz, int64_t* ptr, int32_t* col, double* val) {
  try {
    HostStep hs;
    const int Lm = length > 0 ? length : 5;
    hs.ms.resize(2);
    hs.el.resize(2);
    hs.ms[0].build(m, Lm, channel != 0);
    hs.el[0].build(hs.ms[0].h);
    const eth::StepMesh& g = hs.ms[0];
    const eth::StepElem& E = hs.el[0];
    eth::Csr A;
    switch (which) {
      case ETH_STEP_K: A = eth::step_assemble_K(g, eth::step_assemble_F(g, E, nu, wind, true), eth::step_assemble_B(g, E)); break;
      case ETH_STEP_MQ: A = eth::step_assemble_MQ(g, E); break;
      case ETH_STEP_Q1: A = eth::step_assemble_Q1(g, E); break;
      case ETH_STEP_F1: A = eth::step_assemble_F1(g, E, nu, wind, true); break;
      case ETH_STEP_AP: A = eth::step_assemble_Ap(g, E, eth::step_assemble_B(g, E)); break;
      case ETH_STEP_P:
      case ETH_STEP_PQ:
        if (m % 2) throw std::invalid_argument("m must be even for a prolongation");
        hs.ms[1].build(m / 2, Lm, channel != 0);
        A = which == ETH_STEP_P ? eth::step_q2_prolongation(g, hs.ms[1]) : eth::step_q1_prolongation(g, hs.ms[1]);
        break;
      case ETH_STEP_RHS: {
        const eth::Csr Ff = eth::step_assemble_F(g, E, nu, wind, false);
        const std::vector<double> b = eth::step_lift(g, Ff, eth::step_assemble_B(g, E), eth::step_inflow(g));
        A.rows = (int)b.size();
        A.cols = 1;
        A.ptr.resize(b.size() + 1);
        A.col.assign(b.size(), 0);
        A.val = b;
        for (size_t i = 0; i <= b.size(); ++i) A.ptr[i] = (int)i;
        break;
      }
      default: throw std::invalid_argument("unknown matrix");
    }
    if (rows) *rows = A.rows;
    if (cols) *cols = A.cols;
    if (nnz) *nnz = (int64_t)A.col.size();
    if (ptr)
      for (int i = 0; i <= A.rows; ++i) ptr[i] = A.ptr[i];
    if (col) std::copy(A.col.begin(), A.col.end(), col);
    if (val) std::copy(A.val.begin(), A.val.end(), val);
    return ETH_OK;
  } catch (const std::exception& e) {
    g_step_setup_error = e.what();
    return ETH_EINVAL;
  }
}

}  // extern "C"
