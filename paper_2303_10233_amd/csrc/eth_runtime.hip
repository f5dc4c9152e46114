// Runtime of libeth: problem set-up (multigrid hierarchy, coarse inverses,
// smoother bounds, workspaces), the block preconditioner, the MINRES driver
// with device-resident recurrences and optional hipGraph replay, and the C ABI
// declared in eth.h.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <vector>
#include <map>
#include <array>
#include <filesystem>
#include <fstream>
#include <mutex>
#include <sstream>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/eth.h"
#include "eth_kernels.h"

namespace eth {

constexpr int kDenseCoarseMax = 97 * 97;   // interior nodes of the densely solved coarsest level

// Phase ranges for timeline tools (rocprofv3 --marker-trace): set-up, each
// solve and each stage of one.  Without a tool attached a range costs a call.
struct PhaseRange {
  explicit PhaseRange(const char* name) { roctxRangePushA(name); }
  ~PhaseRange() { roctxRangePop(); }
};

// On-disk record of the choices set-up makes by timing, one "key value" line
// per choice.  The key names the device (architecture and compute units),
// the tuned kernel or launch pattern, the storage type, the mesh and the
// batch, so a later set-up of the same problem on the same kind of GPU reads
// the choice instead of timing it again.  ETH_TUNE_CACHE gives the file (an
// empty value disables the cache); default $HOME/.cache/eth_tune.txt.
struct TuneCache {
  static std::mutex& mu() {
    static std::mutex m;
    return m;
  }
  static std::string path() {
    if (const char* e = std::getenv("ETH_TUNE_CACHE")) return std::string(e);
    const char* h = std::getenv("HOME");
    return h ? std::string(h) + "/.cache/eth_tune.txt" : std::string();
  }
  static std::string device() {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::ostringstream o;
    o << prop.gcnArchName << "/" << prop.multiProcessorCount << "cu";
    std::string s = o.str();
    for (char& c : s)
      if (c == ' ') c = '_';
    return s;
  }
  static bool get(const std::string& key, std::string& val) {
    const std::string p = path();
    if (p.empty()) return false;
    std::lock_guard<std::mutex> lk(mu());
    std::ifstream f(p);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
      const size_t sp = line.rfind(' ');
      if (sp != std::string::npos && line.compare(0, sp, key) == 0 && sp == key.size()) {
        val = line.substr(sp + 1);   // the last record of a key wins
        found = true;
      }
    }
    return found;
  }
  static void put(const std::string& key, const std::string& val) {
    const std::string p = path();
    if (p.empty()) return;
    std::lock_guard<std::mutex> lk(mu());
    std::error_code ec;
    const std::filesystem::path fp(p);
    if (fp.has_parent_path()) std::filesystem::create_directories(fp.parent_path(), ec);
    std::ofstream f(p, std::ios::app);
    if (f) f << key << " " << val << "\n";
  }
};

thread_local std::string g_setup_error;

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Chebyshev polynomial smoother coefficients for degree d on [lo, hi]:
// step k: x_{k+1} = x_k + alpha_k (x_k - x_{k-1}) + beta_k D^{-1}(b - A x_k)
static void cheb_coefs(double lo, double hi, int d, std::vector<double>& alpha,
                       std::vector<double>& beta) {
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  alpha.assign(d, 0.0);
  beta.assign(d, 0.0);
  double rho = 1.0 / sigma;
  beta[0] = 1.0 / theta;
  for (int k = 1; k < d; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    alpha[k] = rn * rho;
    beta[k] = 2.0 * rn / delta;
    rho = rn;
  }
}

// largest eigenvalue of a symmetric tridiagonal matrix (Sturm bisection)
static double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int m = (int)a.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < m; ++i) {
      if (q == 0.0) q = 1e-300;
      q = a[i] - x - b[i - 1] * b[i - 1] / q;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= m) hi = mid;
    else lo = mid;
  }
  return hi;
}

// EST-MINRES: the harmonic Ritz values theta of the Lanczos process after k
// steps satisfy (T_k^2 + beta^2 e_k e_k^T) y = theta T_k y, T_k =
// tridiag(gamma_{j+1}, delta_j, gamma_{j+1}), beta = gamma_{k+1}.  With
// G = T_k^2 + beta^2 e_k e_k^T (symmetric positive definite) the values
// mu = 1/theta are the eigenvalues of the pencil T y = mu G y; the number of
// them below s equals the number of negative pivots of the symmetric
// pentadiagonal T - s G (Sylvester's law of inertia), so the most negative mu
// (the negative theta closest to zero) follows by bisection.  Returns false
// when there is no negative mu.
static bool most_negative_pencil_eig(const std::vector<double>& delta, const std::vector<double>& gam,
                                     double* mu_out) {
  const int k = (int)delta.size();
  auto t = [&](int i, int j) -> double {   // T_k entry
    if (i == j) return delta[i];
    if (j == i + 1 || i == j + 1) return gam[std::max(i, j)];   // gamma_{max+1} (0-based list)
    return 0.0;
  };
  auto gent = [&](int i, int j) -> double {   // (T^2 + beta^2 e_k e_k^T)_{ij}
    double s = 0.0;
    for (int l = std::max(0, std::max(i, j) - 1); l <= std::min(k - 1, std::min(i, j) + 1); ++l)
      s += t(i, l) * t(l, j);
    if (i == k - 1 && j == k - 1) s += gam[k] * gam[k];
    return s;
  };
  // the five diagonals of G
  std::vector<double> g0(k), g1(k, 0.0), g2(k, 0.0);
  for (int i = 0; i < k; ++i) {
    g0[i] = gent(i, i);
    if (i + 1 < k) g1[i] = gent(i, i + 1);
    if (i + 2 < k) g2[i] = gent(i, i + 2);
  }
  auto count_below = [&](double sgm) {
    // LDL^T of the band matrix C = T - sgm G (bandwidth 2), no pivoting
    std::vector<double> d(k), l1(k, 0.0), l2(k, 0.0);   // l1[i] = L(i, i-1), l2[i] = L(i, i-2)
    int neg = 0;
    double scale = 0.0;
    for (int i = 0; i < k; ++i) scale = std::max(scale, std::fabs(delta[i]) + std::fabs(sgm) * g0[i]);
    const double tiny = 1e-300 + 1e-14 * scale;
    for (int i = 0; i < k; ++i) {
      const double c0 = t(i, i) - sgm * g0[i];
      const double c1 = (i >= 1) ? t(i, i - 1) - sgm * g1[i - 1] : 0.0;   // C(i, i-1)
      const double c2 = (i >= 2) ? -sgm * g2[i - 2] : 0.0;                 // C(i, i-2)
      if (i >= 2) l2[i] = c2 / d[i - 2];
      if (i >= 1) {
        double v = c1;
        if (i >= 2) v -= l2[i] * d[i - 2] * l1[i - 1];
        l1[i] = v / d[i - 1];
      }
      double di = c0;
      if (i >= 1) di -= l1[i] * l1[i] * d[i - 1];
      if (i >= 2) di -= l2[i] * l2[i] * d[i - 2];
      if (std::fabs(di) < tiny) di = -tiny;
      d[i] = di;
      if (di < 0.0) ++neg;
    }
    return neg;
  };
  if (count_below(0.0) == 0) return false;
  double lo = -1.0;
  for (int it = 0; it < 400 && count_below(lo) > 0; ++it) lo *= 2.0;
  double hi = 0.0;
  for (int it = 0; it < 200; ++it) {   // the smallest eigenvalue lies in (lo, hi]
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= 1) hi = mid;
    else lo = mid;
  }
  *mu_out = hi;
  return true;
}

struct Problem {
  eth_problem_desc d{};
  Geo g{};
  hipStream_t st = nullptr;
  int max_batch = 1;
  long long ldw = 0;                 // internal stride of Krylov vectors
  bool mixed = false;
  bool oseen = false;
  std::string err;
  std::vector<void*> allocs;

  // velocity preconditioner
  std::vector<Geo> lv;               // multigrid levels (lv[0] finest)
  std::vector<double> lam;           // lambda_max(D^-1 A) per smoothing level
  std::vector<std::vector<double>> ca, cb;   // Chebyshev coefficients per level
  double* Ainv = nullptr;            // dense inverse on the coarsest level
  double* AinvT = nullptr;           // its transpose (Oseen: coarse solve with F^T)
  int coarse_ni = 0;
  double* dense_gbuf = nullptr;
  float *AinvF = nullptr, *AinvTF = nullptr;   // FP32 copies of the coarse inverses (mixed precision)
  std::vector<void*> vb, vx, vxo;    // per-level plane buffers (T)
  TailLevels tail{};                 // levels handled by the fused coarse V-cycle
  int tail_l0 = -1;                  // its first level (-1: per-level launches)

  // pressure preconditioner
  void *mq_r = nullptr, *mq_z = nullptr, *mq_t = nullptr, *mq_d = nullptr, *mq_d2 = nullptr;
  double* mq_coef = nullptr;         // batch
  double* mq_coef2 = nullptr;        // batch
  double kDk = 0.0, kk = 0.0;
  std::vector<double> mq_a, mq_b;    // Chebyshev coefficients for the SGS iteration
  // M_Q by P0 elimination: Q1 multigrid for S_k
  std::vector<Geo> slv;
  std::vector<double> slam;
  std::vector<std::vector<double>> sca, scb;
  std::vector<void*> sb, sx, sxo;
  double* sAinv = nullptr;
  int s_coarse_ni = 0;
  double* ssums = nullptr;
  bool fused_mq = true;              // one launch per Chebyshev step (ETH_DEBUG_UNFUSED_MQ=1: per colour)
  bool fused_q1 = true;              // the PCD's Q_1 solve in one launch (ETH_DEBUG_UNFUSED_Q1=1: per step)
  bool fused_aptail = true;          // A_p levels <= 32^2 in one launch (ETH_DEBUG_UNFUSED_APTAIL=1: per level)
  int aptail_max_n = 32;             // largest A_p level (elements per side) in that launch (ETH_APTAIL_MAX_N)
  // tile side of the fused Chebyshev step, chosen at set-up for batch 1
  // (lo) and for max_batch (hi)
  // variant of the fused Chebyshev step: tile side and steps per launch
  struct MqVariant {
    int tile = 32, steps = 1;
  };
  MqVariant mq_var_lo, mq_var_hi;
  MqVariant mq_variant_for(int batch) const {
    return (long long)batch * batch > max_batch ? mq_var_hi : mq_var_lo;
  }
  MqVariant tune_mq_variant(int batch);
  MqVariant cached_mq_variant(int batch);
  void tune_vcycle_fusion();
  int tuned_timed = 0, tuned_cached = 0;   // set-up choices timed / read from the cache
  template <typename T>
  void mq_chain(const MqVariant& v, T* rr, T* zz, T* tt, const double* r, long long ld, double* z,
                double scale, bool sink_out, bool project_in, int batch, Gate gate);
  ScaleState* d_scale = nullptr;     // [4] scale epilogue states

  // Krylov workspace
  double *kb = nullptr, *kx = nullptr, *ky = nullptr;
  double *kv[2] = {nullptr, nullptr}, *kz[2] = {nullptr, nullptr}, *kw[2] = {nullptr, nullptr};
  MinresScalars* d_ms = nullptr;
  MinresScalars* h_ms = nullptr;     // pinned host mirror
  double* d_hist = nullptr;
  double* d_hist_delta = nullptr;    // Lanczos delta_j / gamma_j of the last MINRES solve
  double* d_hist_gamma = nullptr;
  bool have_lanczos = false;
  int hist_len = 0;
  double* red_partials = nullptr;
  double* red_result = nullptr;      // batch * 4
  double* h_red = nullptr;           // pinned
  double* ub = nullptr;              // Dirichlet data (2 nv)

  // Oseen: velocity multigrid on F, PCD Q1 hierarchy, FGMRES workspace
  double* wind0 = nullptr;                  // internal copy of the finest nodal wind
  double* f_work = nullptr;                 // blocked Gauss-Jordan workspace of the coarse F
  double* pic_b = nullptr;                  // right-hand side of a Picard step (N)
  std::vector<double*> lwind, ldF;          // wind and diag(F) per velocity level
  std::vector<double> lnu;                  // viscosity of each F level (Peclet cap)
  std::vector<float*> lwindF;               // FP32 copy of each level's wind (mixed precision)
  // the wind of level l in the smoother's storage type
  template <typename T>
  const T* level_wind(int l) const {
    if constexpr (sizeof(T) == 4) {
      if (!lwindF[l]) throw std::logic_error("FP32 wind copy missing");
      return lwindF[l];
    } else {
      return lwind[l];
    }
  }
  std::vector<Geo> qlv;                     // Q1 levels of the A_p multigrid
  std::vector<double> qlam;
  std::vector<std::vector<double>> qca, qcb;
  std::vector<void*> qb, qx, qxo;
  std::vector<double*> qdAp;
  double* qAinv = nullptr;
  int q_coarse_ni = 0;
  void *pa = nullptr, *pb = nullptr, *pc = nullptr;   // PCD chain buffers [batch][n_k]
  double* q1sums = nullptr;
  std::vector<double> q1a, q1b;             // Chebyshev coefficients for Q_1 (Wathen interval)
  int gm_m = 0;
  double *gV = nullptr, *gZ = nullptr, *gArr = nullptr, *gpart = nullptr, *ghist = nullptr;
  GmresScalars* d_gm = nullptr;
  GmresScalars* h_gm = nullptr;
  std::vector<double> h_bnorm;

  // graph cache (keyed by batch); graphs are captured and replayed on the
  // internal stream gst, joined to the caller's stream with events
  hipGraphExec_t gexecs[2] = {nullptr, nullptr};   // 2 and graph_iters iterations
  int gexec_key[2] = {-1, -1};
  int graph_iters = 2;               // iterations per long replayed graph (ETH_GRAPH_ITERS)
  hipGraphExec_t iteration_graph(int batch, int iters);
  // captured Arnoldi chunks of FGMRES: (kind, reduced, transpose, batch, j0, j1) -> graph
  std::map<std::array<int, 6>, hipGraphExec_t> gm_graphs;
  hipStream_t gst = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // Stokes: the pressure block of the block-diagonal preconditioner runs on
  // pst concurrently with the velocity V-cycle (fork / join by events; inside
  // a captured graph the two become parallel branches)
  hipStream_t pst = nullptr;
  hipEvent_t ev_pf = nullptr, ev_pj = nullptr;
  bool own_stream = false;           // st was created by the library (ragged batches)

  template <typename T>
  T* alloc(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    allocs.push_back(p);
    // debug mode: every workspace starts as NaN (all bits set), so a read of
    // memory the code never wrote shows up in the results
    if (nan_fill && hipMemset(p, 0xFF, count * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    return static_cast<T*>(p);
  }
  bool nan_fill = false;             // ETH_DEBUG_NAN_FILL=1

  ~Problem() {
    for (auto& ge : gexecs)
      if (ge) (void)hipGraphExecDestroy(ge);
    for (auto& kv : gm_graphs) (void)hipGraphExecDestroy(kv.second);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_pf) (void)hipEventDestroy(ev_pf);
    if (ev_pj) (void)hipEventDestroy(ev_pj);
    if (pst) (void)hipStreamDestroy(pst);
    if (ev_poll) (void)hipEventDestroy(ev_poll);
    if (own_stream && st) (void)hipStreamDestroy(st);
    if (gst) (void)hipStreamDestroy(gst);
    for (void* p : allocs) (void)hipFree(p);
    if (h_ms) (void)hipHostFree(h_ms);
    if (h_red) (void)hipHostFree(h_red);
    if (h_gm) (void)hipHostFree(h_gm);
  }

  RedCtx red(int nblocks, int nvals, int epi, void* state, double* result = nullptr) {
    RedCtx rc{};
    rc.partials = red_partials;
    rc.result = result;
    rc.nblocks = nblocks;
    rc.nvals = nvals;
    rc.epi = epi;
    rc.epi_state = state;
    return rc;
  }
  Gate active_gate() const {
    return Gate{&d_ms[0].active, (int)(sizeof(MinresScalars) / sizeof(int))};
  }

  // K x (or K^T x) on the full layout
  void apply_op(int transpose, const double* x, double* y, long long ld, int batch, Gate gate,
                const RedCtx* dot, ClearFlag clear = no_clear()) {
    if (oseen)
      launch_apply_oseen(g, d.nu, d.wind, transpose, x, y, ld, batch, gate, dot, st, clear);
    else
      launch_apply_stokes(g, d.nu, x, y, ld, batch, gate, dot, st, clear);
  }

  // ---------------------------------------------------------------- setup
  void setup(const eth_problem_desc& desc);
  void build_velocity();
  void build_pressure();
  double lanczos_lambda_max(const Geo& g, int steps);

  // ------------------------------------------------------- preconditioner
  template <typename T>
  void vcycle(const double* r, double* z, long long ld, int batch, Gate gate);
  template <typename T>
  void mq_cheb(const double* r, double* z, long long ld, int batch, Gate gate, double scale,
               bool project_out = true);
  void mq_solve(const double* r, double* z, long long ld, int batch, Gate gate, double scale,
                bool project_out = true);
  void build_schur();
  template <typename T>
  void schur_vcycle(int batch, Gate gate);
  template <typename T>
  void mq_schur(const double* r, double* z, long long ld, int batch, Gate gate, double scale);
  // in_krylov: inside MINRES, where the k component of the pressure output
  // is left in place (see mq_cheb)
  void precond(const double* r, double* z, long long ld, int batch, Gate gate, bool in_krylov = false);

  // ------------------------------------------------------------ Oseen
  void build_oseen_velocity();
  void refresh_wind();
  int picard(const eth_solve_opts& o, int steps, const double* f_nodal, double* x,
             eth_solve_info* info);
  void build_pcd();
  void build_gmres();
  double lanczos_generic(long long len, const std::function<void(const double*, double*)>& apply,
                         const std::function<void(const double*, double*)>& dinv, int steps,
                         bool mean_zero);
  template <typename T>
  void vcycle_F(const double* r, const double* sub, double* z, long long ld, int batch, Gate gate,
                bool trans);
  template <typename T>
  void ap_vcycle(int batch, Gate gate);
  template <typename T>
  void pcd_schur(const double* r, double* z, long long ld, int batch, Gate gate, bool trans);
  // Q_1^{-1} b by pcd_q1_steps Chebyshev-Jacobi steps; returns the buffer holding it
  template <typename T>
  T* q1_inverse(T* b, T* cur, T* oth, int batch, Gate gate);
  // comparison Schur blocks (Sec. 3.1 two-field PCD, Sec. 3.2 LSC), one
  // right-hand side: z_p = -M_S^{-1} r_p with the pressure Laplacian
  // B M^{-1} B^T inverted by conjugate gradients on its range
  template <typename T>
  void schur2(const double* r, double* z, Gate gate);
  std::vector<double*> s2v;          // FP64 full-layout work vectors of schur2
  double dot1(const double* a, const double* b);
  void project_pressure(double* x);
  void lp_apply(const double* p, double* q);
  int lp_pinv(double* b, double* x);
  int lp_last_iters = 0;
  // kind 1: M_1, kind 2: stage-I PCD; kinds 3 and 4: the same for the
  // transposed system [F^T B^T; B 0] (velocity block F^T, Schur complement
  // S^T); r, z internal vectors (stride ldw)
  void precond_oseen(int kind, const double* r, double* z, int batch, Gate gate);
  Gate gm_gate() const {
    return Gate{&d_gm[0].active, (int)(sizeof(GmresScalars) / sizeof(int))};
  }
  // Arnoldi steps j0 .. j1-1 of the current FGMRES cycle (kernels only)
  void arnoldi_steps(int kind, bool reduced, bool transpose, int batch, int j0, int j1);
  // the same, replayed from a graph captured on first use
  void arnoldi_steps_graph(int kind, bool reduced, bool transpose, int batch, int j0, int j1);
  void run_fgmres(int kind, bool reduced, const double* b, double* x, int batch, int m, int maxit,
                  const std::vector<double>& atol, bool transpose = false, bool use_graph = false);
  int solve_oseen(const eth_solve_opts& o, const double* b, double* x, int batch, long long ld,
                  eth_solve_info* info, bool adjoint = false);

  // ---------------------------------------------------------------- solve
  // a MINRES solve split into phases, so that several problems can iterate
  // concurrently on their own streams (eth_batch_solve)
  struct MinresRun {
    eth_solve_opts o{};
    const double* b = nullptr;
    double* x = nullptr;
    int batch = 1;
    long long ld = 0;
    bool adjoint = false;
    double tol = 0.0, prev_rel = 1.0;
    int maxit = 0, done = 0, chunk = 8, prev_it = 0;
    bool use_graph = false;
    // FP64 defect-correction restarts (opts.refine) and the per-RHS record
    // kept across them: gamma_1 of the first start, iterations, the final
    // |eta| / gamma_1 and (when asked for) the residual history
    int refine_left = 0, runs = 0;
    std::vector<double> gamma0, rel;
    std::vector<int> iters;
    std::vector<std::vector<double>> hist;
  };
  void minres_end_of_run(MinresRun& R);
  void minres_restart(MinresRun& R);
  // per-RHS status of the right-hand sides b (0, ETH_EINCONSISTENT or
  // ETH_EINVAL); consistency = false checks finiteness only
  std::vector<int> check_rhs(const double* b, long long ld, int batch, bool consistency);
  double mq_sign = 1.0;              // -1 under ETH_DEBUG_NEGATE_MQ (indefinite preconditioner)
  bool fused_smooth = true;          // V(2,2) smoothing fused into restriction / correction launches
  bool fold_delta = true;            // the delta reduction finished inside the v update (ETH_DEBUG_FOLD_DELTA=0: separate launch)
  bool fold_wx = true;               // the w/x update made inside the next v update (ETH_DEBUG_FOLD_WX=0: own launch)
  hipEvent_t ev_poll = nullptr;
  // enqueue: also the first chunk of iterations (a joint batch graph runs
  // the iterations of every member itself)
  void minres_begin(MinresRun& R, bool enqueue = true);
  void minres_enqueue_chunk(MinresRun& R);
  // after the iterations have ended (scalars on the host): the book-keeping
  // and the output copies; false when an FP64 refinement restart was enqueued
  bool minres_conclude(MinresRun& R);
  // true once the iteration has ended and the output copies are enqueued;
  // block = false returns false at once while the last chunk still runs
  bool minres_poll(MinresRun& R, bool block);
  int minres_finish(MinresRun& R, eth_solve_info* info);
  void minres_iteration(int batch, int parity);
  void minres_flush_wx(int batch);
  int solve_minres(const eth_solve_opts& o, const double* b, double* x, int batch, long long ld,
                   eth_solve_info* info, bool adjoint = false);
  // Krylov RHS kb from b: boundary rows zeroed; for the adjoint also the
  // pressure block means removed (the part of g in null(K) has no adjoint)
  void load_rhs(const double* b, long long ld, int batch, bool adjoint);
  void run_iterations(int batch, int count, bool use_graph);
};

// ------------------------------------------------------------------------------
void Problem::setup(const eth_problem_desc& desc) {
  PhaseRange range("eth_setup");
  d = desc;
  if (const char* e = std::getenv("ETH_DEBUG_NAN_FILL")) nan_fill = (e[0] == '1');
  if (const char* e = std::getenv("ETH_DEBUG_FOLD_DELTA")) fold_delta = (e[0] != '0');
  if (const char* e = std::getenv("ETH_DEBUG_FOLD_WX")) fold_wx = (e[0] != '0');
  if (d.n < 2) throw std::invalid_argument("n must be >= 2");
  if (!(d.x1 > d.x0) || !(d.y1 > d.y0)) throw std::invalid_argument("empty domain");
  if (std::fabs((d.x1 - d.x0) - (d.y1 - d.y0)) > 1e-12 * (d.x1 - d.x0))
    throw std::invalid_argument("square domain required");
  if (!(d.nu > 0.0)) throw std::invalid_argument("nu must be > 0");
  if (d.kind != ETH_STOKES && d.kind != ETH_OSEEN) throw std::invalid_argument("invalid kind");
  if (d.kind == ETH_OSEEN && !d.wind) throw std::invalid_argument("Oseen needs a wind");
  if (d.corner_mode < 0 || d.corner_mode > 2) throw std::invalid_argument("corner_mode must be 0, 1 or 2");
  oseen = d.kind == ETH_OSEEN;
  if (d.mq_mode == 0) d.mq_mode = ETH_MQ_CHEB_SGS;
  if (d.mq_mode != ETH_MQ_DIAG && d.mq_mode != ETH_MQ_CHEB_SGS && d.mq_mode != ETH_MQ_SCHUR_GMG)
    throw std::invalid_argument("invalid mq_mode");
  if (d.mq_steps <= 0) d.mq_steps = 20;
  // lower end of the SGS-preconditioned M_Q interval: its smallest nonzero
  // eigenvalue decays like h^2; 0.4/n (at most 0.01) is the best of the oracle
  // sweeps at n = 128 and 256
  if (d.mq_cheb_lo <= 0.0) d.mq_cheb_lo = std::min(0.01, 0.4 / d.n);
  if (d.mq_cheb_hi <= 0.0) d.mq_cheb_hi = 1.0;
  if (!(d.mq_cheb_hi > d.mq_cheb_lo)) throw std::invalid_argument("mq interval empty");
  if (d.gmg_coarse_n <= 0) d.gmg_coarse_n = oseen ? 32 : 4;
  if (d.gmg_omega <= 0.0) d.gmg_omega = 0.7;
  if (d.gmg_peclet_max < 0.0) throw std::invalid_argument("gmg_peclet_max must be >= 0");
  if (d.oseen_schur < 0 || d.oseen_schur > 2) throw std::invalid_argument("oseen_schur must be 0, 1 or 2");
  if (d.oseen_schur != 0 && (d.kind != ETH_OSEEN || d.max_batch > 1))
    throw std::invalid_argument("oseen_schur needs an Oseen problem with max_batch 1");
  if (d.schur_cg_tol <= 0.0) d.schur_cg_tol = 1e-10;
  if (d.schur_cg_maxit <= 0) d.schur_cg_maxit = 2000;
  if (d.pcd_q1_steps <= 0) d.pcd_q1_steps = 10;
  if (d.gmres_restart <= 0) d.gmres_restart = 50;
  if (d.gmres_restart > 63) throw std::invalid_argument("gmres_restart must be <= 63");
  if (d.mq_tile != 0 && d.mq_tile != 8 && d.mq_tile != 16 && d.mq_tile != 24 && d.mq_tile != 32 &&
      d.mq_tile != 64)
    throw std::invalid_argument("mq_tile must be 0, 8, 16, 24, 32 or 64");
  if (d.mq_tile == 64 && d.precision != ETH_MIXED)
    throw std::invalid_argument("mq_tile 64 needs the FP32 preconditioner");
  if (d.mq_fuse_steps < 0 || d.mq_fuse_steps > 2) throw std::invalid_argument("mq_fuse_steps must be 0, 1 or 2");
  if (d.mq_fuse_steps == 2 &&
      ((d.mq_tile != 0 && d.mq_tile != 16 && d.mq_tile != 24) || d.precision != ETH_MIXED))
    throw std::invalid_argument("two Chebyshev steps per launch need mq_tile 16 or 24 and ETH_MIXED");
  if (d.gmg_degree <= 0) d.gmg_degree = 2;
  if (d.gmg_lo_frac <= 0.0) d.gmg_lo_frac = 0.3;
  if (d.gmg_hi_frac <= 0.0) d.gmg_hi_frac = 1.1;
  if (d.velocity_mode != ETH_VEL_GMG && d.velocity_mode != ETH_VEL_EXACT)
    throw std::invalid_argument("invalid velocity_mode");
  if (d.precision != ETH_FP64 && d.precision != ETH_MIXED)
    throw std::invalid_argument("invalid precision");
  mixed = d.precision == ETH_MIXED;
  // failure-path tests: a negated pressure block makes the Stokes
  // preconditioner indefinite, which MINRES reports as a breakdown
  if (const char* e = std::getenv("ETH_DEBUG_NEGATE_MQ")) mq_sign = (e[0] == '1') ? -1.0 : 1.0;
  if (const char* e = std::getenv("ETH_DEBUG_UNFUSED_MQ")) fused_mq = (e[0] != '1');
  if (const char* e = std::getenv("ETH_GRAPH_ITERS")) graph_iters = std::max(2, std::min(64, std::atoi(e) & ~1));
  if (const char* e = std::getenv("ETH_DEBUG_UNFUSED_Q1")) fused_q1 = (e[0] != '1');
  if (const char* e = std::getenv("ETH_DEBUG_UNFUSED_APTAIL")) fused_aptail = (e[0] != '1');
  if (const char* e = std::getenv("ETH_APTAIL_MAX_N")) aptail_max_n = std::max(2, std::min(32, std::atoi(e)));
  max_batch = d.max_batch > 0 ? d.max_batch : 1;
  st = static_cast<hipStream_t>(d.stream);
  ETH_HIP(hipEventCreateWithFlags(&ev_poll, hipEventDisableTiming));
  g = make_geo(d.n, (d.x1 - d.x0) / d.n);
  ldw = (g.N + 63) / 64 * 64;

  const size_t vec = (size_t)ldw * max_batch;
  kb = alloc<double>(vec);
  kx = alloc<double>(vec);
  ky = alloc<double>(vec);
  for (int i = 0; i < 2; ++i) {
    kv[i] = alloc<double>(vec);
    kz[i] = alloc<double>(vec);
    kw[i] = alloc<double>(vec);
  }
  d_ms = alloc<MinresScalars>(max_batch);
  ETH_HIP(hipHostMalloc((void**)&h_ms, sizeof(MinresScalars) * max_batch, hipHostMallocDefault));
  hist_len = 4097;
  d_hist = alloc<double>((size_t)hist_len * max_batch);
  d_hist_delta = alloc<double>((size_t)hist_len * max_batch);
  d_hist_gamma = alloc<double>((size_t)hist_len * max_batch);
  const int maxblocks =
      std::max(std::max(std::max(dot_blocks(g.N), saddle_blocks(g)), adjoint_blocks(g)), 4096);
  red_partials = alloc<double>((size_t)maxblocks * kMaxRedVals * max_batch);
  red_result = alloc<double>((size_t)kMaxRedVals * max_batch);
  ETH_HIP(hipHostMalloc((void**)&h_red, sizeof(double) * kMaxRedVals * max_batch, hipHostMallocDefault));
  ETH_HIP(hipMemsetAsync(d_ms, 0, sizeof(MinresScalars) * max_batch, st));
  ub = alloc<double>(2 * (size_t)g.nv);
  launch_dirichlet_lid(g, d.lid_u, d.corner_mode, ub, st);
  d_scale = alloc<ScaleState>(4);

  if (oseen) {
    wind0 = alloc<double>(2 * (size_t)g.nv);
    ETH_HIP(hipMemcpyAsync(wind0, d.wind, 2 * sizeof(double) * g.nv, hipMemcpyDeviceToDevice, st));
    d.wind = wind0;
    pic_b = alloc<double>(g.N);
    build_oseen_velocity();
    build_pcd();
    build_gmres();
    if (d.oseen_schur != 0)
      for (int i = 0; i < 7; ++i) {
        s2v.push_back(alloc<double>(ldw));
        ETH_HIP(hipMemsetAsync(s2v.back(), 0, sizeof(double) * ldw, st));
      }
  } else {
    build_velocity();
    // members of a ragged batch run concurrently with each other instead: a
    // second branch per member would only multiply the streams sharing the
    // few hardware queues
    if (!own_stream && !std::getenv("ETH_DEBUG_SERIAL_PRECOND")) {
      ETH_HIP(hipStreamCreateWithFlags(&pst, hipStreamNonBlocking));
      ETH_HIP(hipEventCreateWithFlags(&ev_pf, hipEventDisableTiming));
      ETH_HIP(hipEventCreateWithFlags(&ev_pj, hipEventDisableTiming));
    }
    if (d.velocity_mode == ETH_VEL_GMG) tune_vcycle_fusion();
  }
  build_pressure();
  ETH_HIP(hipStreamSynchronize(st));
}

double Problem::lanczos_lambda_max(const Geo& lg, int steps) {
  // PCG with Jacobi preconditioning on A x = b; the CG coefficients define the
  // Lanczos tridiagonal of D^{-1}A, whose largest Ritz value is returned.
  const size_t nv = lg.nv;
  double* r = alloc<double>(nv);
  double* z = alloc<double>(nv);
  double* p = alloc<double>(nv);
  double* q = alloc<double>(nv);
  std::vector<double> h(nv, 0.0);
  unsigned long long s = 0x9E3779B97F4A7C15ULL;
  for (int J = 1; J < lg.nq - 1; ++J)
    for (int I = 1; I < lg.nq - 1; ++I) {
      s = s * 6364136223846793005ULL + 1442695040888963407ULL;
      h[(size_t)J * lg.nq + I] = (double)((s >> 11) & ((1ULL << 53) - 1)) / (double)(1ULL << 53) - 0.5;
    }
  ETH_HIP(hipMemcpyAsync(r, h.data(), nv * sizeof(double), hipMemcpyHostToDevice, st));
  auto dot = [&](const double* a, const double* b) {
    RedCtx rc = red(dot_blocks((long long)nv), 1, EPI_NONE, nullptr, red_result);
    launch_dot((long long)nv, a, b, 0, 1, rc, no_gate(), st);
    ETH_HIP(hipMemcpyAsync(h_red, red_result, sizeof(double), hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    return h_red[0];
  };
  launch_plane_op(lg, 1, r, z, st);
  launch_copy((long long)nv, z, 0, p, 0, 1, st);
  double rz = dot(r, z);
  std::vector<double> al, be;
  for (int k = 0; k < steps; ++k) {
    launch_plane_op(lg, 0, p, q, st);
    const double pq = dot(p, q);
    if (!(pq > 0.0)) break;
    const double alpha = rz / pq;
    launch_axpby((long long)nv, -alpha, q, 1.0, r, 0, 1, st);
    launch_plane_op(lg, 1, r, z, st);
    const double rzn = dot(r, z);
    const double beta = rzn / rz;
    al.push_back(alpha);
    be.push_back(beta);
    launch_axpby((long long)nv, 1.0, z, beta, p, 0, 1, st);
    rz = rzn;
    if (!(rz > 0.0)) break;
  }
  const int m = (int)al.size();
  std::vector<double> ta(m), tb(m > 0 ? m - 1 : 0);
  for (int k = 0; k < m; ++k) {
    ta[k] = 1.0 / al[k] + (k > 0 ? be[k - 1] / al[k - 1] : 0.0);
    if (k + 1 < m) tb[k] = std::sqrt(be[k]) / al[k];
  }
  return m > 0 ? tridiag_max_eig(ta, tb) : 1.0;
}

void Problem::build_velocity() {
  lv.clear();
  if (d.velocity_mode == ETH_VEL_EXACT) {
    lv.push_back(g);
  } else {
    int n = d.n;
    double h = g.h;
    lv.push_back(g);
    while (n % 2 == 0 && n > d.gmg_coarse_n) {
      n /= 2;
      h *= 2.0;
      lv.push_back(make_geo(n, h));
    }
  }
  const Geo& gc = lv.back();
  coarse_ni = (gc.nq - 2) * (gc.nq - 2);
  // the coarsest level is solved with a dense inverse (FP64, and an FP32
  // copy in mixed precision): up to 97^2 interior nodes per component
  // (odd factor m <= 49 of n = m * 2^k), 0.7 GB for the FP64 matrix
  if (coarse_ni > kDenseCoarseMax)
    throw std::runtime_error("unsupported:coarsest mesh too large for the dense solve (n = m * 2^k needs odd m <= 49)");
  dense_gbuf = alloc<double>((size_t)2 * coarse_ni * max_batch);
  // dense inverse of the coarsest-level Laplacian (Gauss-Jordan, SPD, no pivoting)
  {
    const int ni = coarse_ni;
    double* work = alloc<double>(dense_inverse_work(ni));
    Ainv = alloc<double>((size_t)ni * ni);
    launch_dense_laplacian(gc, Ainv, ni, st);
    launch_dense_inverse(Ainv, ni, work, st);
    launch_symmetrize(Ainv, ni, st);
    if (mixed) {
      AinvF = alloc<float>((size_t)ni * ni);
      launch_to_float(Ainv, AinvF, (long long)ni * ni, st);
    }
  }
  const int L = (int)lv.size();
  lam.assign(std::max(L - 1, 0), 0.0);
  ca.assign(lam.size(), {});
  cb.assign(lam.size(), {});
  for (int l = 0; l + 1 < L; ++l) {
    lam[l] = d.gmg_lambda ? d.gmg_lambda[l] : lanczos_lambda_max(lv[l], 30);
    cheb_coefs(d.gmg_lo_frac * lam[l], d.gmg_hi_frac * lam[l], d.gmg_degree, ca[l], cb[l]);
  }
  vb.assign(L, nullptr);
  vx.assign(L, nullptr);
  vxo.assign(L, nullptr);
  if (L > 1) {
    for (int l = 0; l < L; ++l) {
      const size_t n = (size_t)2 * max_batch * lv[l].nv;
      if (mixed) {
        vb[l] = alloc<float>(n);
        vx[l] = alloc<float>(n);
        vxo[l] = alloc<float>(n);
        ETH_HIP(hipMemsetAsync(vb[l], 0, n * sizeof(float), st));
        ETH_HIP(hipMemsetAsync(vx[l], 0, n * sizeof(float), st));
        ETH_HIP(hipMemsetAsync(vxo[l], 0, n * sizeof(float), st));
      } else {
        vb[l] = alloc<double>(n);
        vx[l] = alloc<double>(n);
        vxo[l] = alloc<double>(n);
        ETH_HIP(hipMemsetAsync(vb[l], 0, n * sizeof(double), st));
        ETH_HIP(hipMemsetAsync(vx[l], 0, n * sizeof(double), st));
        ETH_HIP(hipMemsetAsync(vxo[l], 0, n * sizeof(double), st));
      }
    }
  }
  // fused coarse end of the V-cycle: from the first level below the finest
  // with at most 32 elements per side, when it fits in LDS and the coarsest
  // dense solve is small
  tail_l0 = -1;
  bool allow = true;
  if (const char* e = std::getenv("ETH_DEBUG_UNFUSED_VCYCLE")) allow = (e[0] != '1');
  int tail_max_n = 16;   // largest level (elements per side) inside the fused tail
  if (const char* e = std::getenv("ETH_TAIL_MAX_N")) tail_max_n = std::max(2, std::min(32, std::atoi(e)));
  int l0 = -1;
  for (int l = 1; l < L; ++l)
    if (lv[l].n <= tail_max_n) {
      l0 = l;
      break;
    }
  if (allow && l0 >= 1 && l0 <= L - 2 && L - l0 <= kTailMaxLevels && d.gmg_degree <= 4 && coarse_ni <= 289) {
    TailLevels t{};
    t.nlev = L - l0;
    t.deg = d.gmg_degree;
    for (int l = l0; l < L; ++l) {
      t.n[l - l0] = lv[l].n;
      if (l + 1 < L)
        for (int k = 0; k < d.gmg_degree; ++k) {
          t.ca[l - l0][k] = ca[l][k];
          t.cb[l - l0][k] = cb[l][k];
        }
    }
    const size_t lds = vcycle_tail_lds(t, mixed ? sizeof(float) : sizeof(double));
    const hipError_t e = mixed ? prepare_vcycle_tail<float>(lds) : prepare_vcycle_tail<double>(lds);
    if (lds <= 160 * 1024 && e == hipSuccess) {
      tail = t;
      tail_l0 = l0;
    } else {
      (void)hipGetLastError();
    }
  }
}

void Problem::build_pressure() {
  const double h2 = g.h * g.h;
  // k^T D^{-1} k and k^T k for the frame null vector k = [1; -1]
  double s = 0.0;
  for (int dd = 0; dd <= g.n; ++dd)
    for (int c = 0; c <= g.n; ++c) {
      const int mx = (c > 0) + (c < g.n), my = (dd > 0) + (dd < g.n);
      s += 36.0 / (h2 * 4.0 * mx * my);
    }
  s += (double)g.n0 / h2;
  kDk = s;
  kk = (double)g.nk + g.n0;
  mq_coef = alloc<double>(max_batch);
  mq_coef2 = alloc<double>(max_batch);
  ScaleState hs[4];
  hs[0] = ScaleState{mq_coef, 1.0 / kDk};
  hs[1] = ScaleState{mq_coef, 1.0 / kk};
  hs[2] = ScaleState{mq_coef2, 1.0 / kk};
  hs[3] = ScaleState{mq_coef, 1.0};
  ETH_HIP(hipMemcpyAsync(d_scale, hs, sizeof(hs), hipMemcpyHostToDevice, st));
  if (d.mq_mode == ETH_MQ_SCHUR_GMG) {
    const size_t n = (size_t)max_batch * (g.nk + g.n0);
    const size_t es = mixed ? sizeof(float) : sizeof(double);
    mq_r = alloc<char>(n * es);
    mq_z = alloc<char>(n * es);
    mq_t = alloc<char>(n * es);
    mq_d = alloc<char>(n * es);
    build_schur();
  }
  if (d.mq_mode == ETH_MQ_CHEB_SGS) {
    const size_t n = (size_t)max_batch * (g.nk + g.n0);
    const size_t es = mixed ? sizeof(float) : sizeof(double);
    mq_r = alloc<char>(n * es);
    mq_z = alloc<char>(n * es);
    mq_t = alloc<char>(n * es);
    mq_d = alloc<char>(n * es);
    mq_d2 = alloc<char>(n * es);
    // Chebyshev semi-iteration: step k uses a_k d_{k-1} + b_k s_k
    const double lo = d.mq_cheb_lo, hi = d.mq_cheb_hi;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    mq_a.assign(d.mq_steps, 0.0);
    mq_b.assign(d.mq_steps, 0.0);
    double rho = 1.0 / sigma;
    mq_b[0] = 1.0 / theta;
    for (int k = 1; k < d.mq_steps; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      mq_a[k] = rn * rho;
      mq_b[k] = 2.0 * rn / delta;
      rho = rn;
    }
    if (d.mq_tile != 0) {
      mq_var_lo.tile = mq_var_hi.tile = d.mq_tile;
      mq_var_lo.steps = mq_var_hi.steps = d.mq_fuse_steps > 0 ? d.mq_fuse_steps : 1;
    } else {
      mq_var_lo = cached_mq_variant(1);
      mq_var_hi = max_batch > 1 ? cached_mq_variant(max_batch) : mq_var_lo;
    }
  }
}

// tune_mq_variant through the set-up cache
Problem::MqVariant Problem::cached_mq_variant(int batch) {
  std::ostringstream k;
  k << TuneCache::device() << " mq_cheb_fused " << (mixed ? "f32" : "f64") << " n=" << g.n << " batch=" << batch
    << " steps=" << d.mq_steps << " fuse=" << d.mq_fuse_steps << " ctx=" << (pst != nullptr ? 1 : 0);
  std::string v;
  MqVariant r;
  if (TuneCache::get(k.str(), v) && std::sscanf(v.c_str(), "%dx%d", &r.tile, &r.steps) == 2 &&
      (r.tile == 8 || r.tile == 16 || r.tile == 24 || r.tile == 32 || (r.tile == 64 && mixed)) && (r.steps == 1 || r.steps == 2)) {
    ++tuned_cached;
    return r;
  }
  r = tune_mq_variant(batch);
  ++tuned_timed;
  TuneCache::put(k.str(), std::to_string(r.tile) + "x" + std::to_string(r.steps));
  return r;
}

// Launch pattern of the V(2,2) smoothing on the levels above the fused coarse
// end: the second pre-smoothing step inside the restriction's launch and the
// correction with both post-smoothing steps in one launch (fewer launches,
// wider halos), or one launch per step (narrower halos).  Timed on whole
// V-cycles at set-up, the choice kept in the set-up cache.
// ETH_DEBUG_UNFUSED_SMOOTH = 1 / 0 forces one launch per step / the fused form.
void Problem::tune_vcycle_fusion() {
  if (const char* e = std::getenv("ETH_DEBUG_UNFUSED_SMOOTH")) {
    fused_smooth = (e[0] != '1');
    return;
  }
  if (d.gmg_degree != 2 || lv.size() < 2 || (tail_l0 >= 0 && tail_l0 < 1)) return;
  std::ostringstream k;
  k << TuneCache::device() << " vcycle_smoothing " << (mixed ? "f32" : "f64") << " n=" << g.n
    << " batch=" << max_batch << " coarse=" << d.gmg_coarse_n;
  std::string v;
  if (TuneCache::get(k.str(), v) && (v == "fused" || v == "split")) {
    fused_smooth = v == "fused";
    ++tuned_cached;
    return;
  }
  ETH_HIP(hipMemsetAsync(kv[0], 0, (size_t)ldw * max_batch * sizeof(double), st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ETH_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    throw std::runtime_error("hipEventCreate failed");
  }
  float best[2] = {0.0f, 0.0f};
  try {
    auto cycle = [&](bool f) {
      fused_smooth = f;
      if (mixed) vcycle<float>(kv[0], kz[0], ldw, max_batch, no_gate());
      else vcycle<double>(kv[0], kz[0], ldw, max_batch, no_gate());
    };
    for (int f = 0; f < 2; ++f)
      for (int i = 0; i < 3; ++i) cycle(f == 1);
    for (int round = 0; round < 3; ++round)
      for (int f = 0; f < 2; ++f) {
        ETH_HIP(hipEventRecord(e0, st));
        for (int i = 0; i < 10; ++i) cycle(f == 1);
        ETH_HIP(hipEventRecord(e1, st));
        ETH_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        ETH_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (round == 0 || ms < best[f]) best[f] = ms;
      }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  fused_smooth = best[1] <= best[0];
  ++tuned_timed;
  TuneCache::put(k.str(), fused_smooth ? "fused" : "split");
}

// The fastest variant of the fused Chebyshev step (tile side, one or two
// steps per launch) for `batch` right-hand sides on this mesh: each candidate
// is timed with events on zeroed vectors, per Chebyshev step over a few
// launches, or, where the pressure solve runs beside the velocity V-cycle,
// per application of the whole preconditioner (a variant that is faster
// alone can hold more of the CUs the V-cycle shares).  Small meshes favour
// small tiles (more blocks in flight), large meshes large ones (less halo
// recomputation); two steps per launch trade a wider halo for half the
// launches.
Problem::MqVariant Problem::tune_mq_variant(int batch) {
  const size_t bytes = (size_t)max_batch * (g.nk + g.n0) * (mixed ? sizeof(float) : sizeof(double));
  ETH_HIP(hipMemsetAsync(mq_r, 0, bytes, st));
  ETH_HIP(hipMemsetAsync(mq_z, 0, bytes, st));
  ETH_HIP(hipMemsetAsync(mq_t, 0, bytes, st));
  ETH_HIP(hipMemsetAsync(mq_d, 0, bytes, st));
  ETH_HIP(hipMemsetAsync(mq_d2, 0, bytes, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ETH_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    throw std::runtime_error("hipEventCreate failed");
  }
  // candidates are timed in interleaved rounds after a common warm-up, and
  // each keeps its fastest round, so that a clock ramp at set-up does not
  // favour the later ones
  std::vector<MqVariant> cands;
  const int fs = d.mq_fuse_steps;
  for (int t : {8, 16, 24, 32, 64}) {
    if (t == 64 && !mixed) continue;
    if (fs != 2) cands.push_back(MqVariant{t, 1});
    if ((t == 16 || t == 24) && fs != 1 && d.mq_steps >= 2 && mixed) cands.push_back(MqVariant{t, 2});
  }
  if (cands.empty()) cands.push_back(MqVariant{16, 1});
  std::vector<float> best_ms(cands.size(), 0.0f);
  MqVariant best = cands[0];
  const MqVariant keep_lo = mq_var_lo, keep_hi = mq_var_hi;   // set per candidate in context
  try {
    auto launch = [&](const MqVariant& v) {
      if (mixed)
        launch_mq_cheb_fused<float>(g, (float*)mq_r, (float*)mq_z, (float*)mq_t, (float*)mq_d,
                                    v.steps == 2 ? (float*)mq_d2 : (float*)mq_d, 0.5, 0.1, 0.5, 0.1,
                                    v.steps, 0, batch, no_gate(), st, v.tile);
      else
        launch_mq_cheb_fused<double>(g, (double*)mq_r, (double*)mq_z, (double*)mq_t, (double*)mq_d,
                                     v.steps == 2 ? (double*)mq_d2 : (double*)mq_d, 0.5, 0.1, 0.5, 0.1,
                                     v.steps, 0, batch, no_gate(), st, v.tile);
    };
    const bool in_context = pst != nullptr && cands.size() > 1;
    if (in_context) ETH_HIP(hipMemsetAsync(kv[0], 0, (size_t)ldw * batch * sizeof(double), st));
    auto unit = [&](const MqVariant& v) {
      if (in_context) {
        mq_var_lo = mq_var_hi = v;
        precond(kv[0], kz[0], ldw, batch, no_gate(), true);
      } else {
        launch(v);
      }
    };
    const int warm = in_context ? 3 : 20, reps = in_context ? 8 : 10, rounds = in_context ? 5 : 3;
    for (const auto& v : cands)
      for (int i = 0; i < warm; ++i) unit(v);
    for (int round = 0; round < rounds; ++round)
      for (size_t c = 0; c < cands.size(); ++c) {
        ETH_HIP(hipEventRecord(e0, st));
        for (int i = 0; i < reps; ++i) unit(cands[c]);
        ETH_HIP(hipEventRecord(e1, st));
        ETH_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        ETH_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (!in_context) ms /= (float)cands[c].steps;
        if (round == 0 || ms < best_ms[c]) best_ms[c] = ms;
      }
    size_t bi = 0;
    for (size_t c = 1; c < cands.size(); ++c)
      if (best_ms[c] < best_ms[bi]) bi = c;
    // a near tie (within 2 %, the spread of repeated timings in context)
    // keeps the default variant, 16 x 16 tiles with one step per launch
    for (size_t c = 0; c < cands.size(); ++c)
      if (cands[c].tile == 16 && cands[c].steps == 1 && best_ms[c] <= 1.02f * best_ms[bi]) bi = c;
    best = cands[bi];
  } catch (...) {
    mq_var_lo = keep_lo;
    mq_var_hi = keep_hi;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  mq_var_lo = keep_lo;
  mq_var_hi = keep_hi;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

// The Chebyshev steps of the pressure-mass solve with the fused kernel: z
// ping-pongs between zz and tt (the result ends in zz), and d between mq_d and
// mq_d2 across two-step launches (which read d over their whole region).  The
// first launch takes r from the FP64 vectors with the input projection; with
// sink_out the last one writes scale * z to the FP64 vectors instead of zz.
template <typename T>
void Problem::mq_chain(const MqVariant& v, T* rr, T* zz, T* tt, const double* r, long long ld, double* z,
                       double scale, bool sink_out, bool project_in, int batch, Gate gate) {
  const int m = d.mq_steps;
  std::vector<int> per;   // Chebyshev steps of each launch
  for (int k = 0; k < m;) {
    const int s = (v.steps == 2 && k + 1 < m) ? 2 : 1;
    per.push_back(s);
    k += s;
  }
  const int nl = (int)per.size();
  T* zb[2] = {zz, tt};
  T* db[2] = {static_cast<T*>(mq_d), static_cast<T*>(mq_d2)};
  int zc = nl & 1, dc = 0;   // launch i reads zb[zc], writes zb[zc ^ 1]; zb[nl parity] ends in zz
  const MqSource src{r, ld, project_in ? mq_coef : nullptr};
  const MqSink sink{z, ld, scale};
  int k = 0;
  for (int i = 0; i < nl; ++i) {
    const bool last = i + 1 == nl;
    const int s = per[i];
    T* din = db[dc];
    T* dout = s == 2 ? db[dc ^ 1] : db[dc];
    launch_mq_cheb_fused<T>(g, rr, zb[zc], zb[zc ^ 1], din, dout, mq_a[k], mq_b[k],
                            s == 2 ? mq_a[k + 1] : 0.0, s == 2 ? mq_b[k + 1] : 0.0, s, k == 0, batch, gate,
                            st, s == 2 ? 16 : v.tile, k == 0 ? &src : nullptr,
                            last && sink_out ? &sink : nullptr);
    zc ^= 1;
    if (s == 2) dc ^= 1;
    k += s;
  }
}

// ---------------------------------------------------------------- V-cycle
template <typename T>
void Problem::vcycle(const double* r, double* z, long long ld, int batch, Gate gate) {
  const int L = (int)lv.size();
  const double sc = 1.0 / d.nu;
  if (L == 1) {
    launch_dense_solve<T>(lv[0], Ainv, AinvF, coarse_ni, nullptr, nullptr, 2 * batch, z, ld, sc, r, ld,
                          dense_gbuf, batch, gate, st);
    launch_zero_boundary(lv[0], z, ld, batch, st);
    return;
  }
  std::vector<T*> b(L), x(L), xo(L);
  for (int l = 0; l < L; ++l) {
    b[l] = static_cast<T*>(vb[l]);
    x[l] = static_cast<T*>(vx[l]);
    xo[l] = static_cast<T*>(vxo[l]);
  }
  const int np = 2 * batch;
  const int deg = d.gmg_degree;
  // V(2,2): the second pre-smoothing step rides in the restriction's launch
  // and the correction with both post-smoothing steps in one launch per level
  const bool fuse = fused_smooth && deg == 2;
  // finest level: b = r_u, first smoothing step from zero
  launch_vcycle_entry<T>(lv[0], r, ld, b[0], x[0], cb[0][0], batch, gate, st);
  // levels below `lstop` are handled by the fused coarse kernel when enabled
  const int lstop = tail_l0 >= 1 ? tail_l0 : L - 1;
  for (int l = 0; l < lstop; ++l) {
    const double beta_c = (l + 1 < L - 1) ? cb[l + 1][0] : 0.0;
    if (fuse) {
      launch_restrict_pre<T>(lv[l], lv[l + 1], b[l], x[l], xo[l], ca[l][1], cb[l][1], b[l + 1], x[l + 1],
                             beta_c, np, gate, st);
      std::swap(x[l], xo[l]);
      continue;
    }
    for (int k = 1; k < deg; ++k) {
      launch_cheb_step<T>(lv[l], b[l], x[l], xo[l], ca[l][k], cb[l][k], k == 1 ? 2 : 1, np,
                          nullptr, 0, 0.0, gate, batch, st);
      std::swap(x[l], xo[l]);
    }
    launch_restrict<T>(lv[l], lv[l + 1], b[l], x[l], b[l + 1], x[l + 1], beta_c, np, batch, gate, st);
  }
  if (tail_l0 >= 1)
    launch_vcycle_tail<T>(tail, Ainv, coarse_ni, b[lstop], x[lstop], np, gate, st);
  else
    launch_dense_solve<T>(lv[L - 1], Ainv, AinvF, coarse_ni, b[L - 1], x[L - 1], np, nullptr, 0, 0.0,
                          nullptr, 0, dense_gbuf, batch, gate, st);
  for (int l = lstop - 1; l >= 0; --l) {
    if (fuse) {
      launch_post2<T>(lv[l], lv[l + 1], b[l], x[l], x[l + 1], xo[l], ca[l][1], cb[l][0], cb[l][1], np,
                      l == 0 ? z : nullptr, ld, sc, gate, st);
      if (l > 0) std::swap(x[l], xo[l]);
      continue;
    }
    launch_prolong_add<T>(lv[l], lv[l + 1], x[l + 1], x[l], np, batch, gate, st);
    for (int k = 0; k < deg; ++k) {
      const bool last = (l == 0 && k == deg - 1);
      launch_cheb_step<T>(lv[l], b[l], x[l], xo[l], ca[l][k], cb[l][k], k == 0 ? 0 : 1, np,
                          last ? z : nullptr, ld, sc, gate, batch, st);
      if (!last) std::swap(x[l], xo[l]);
    }
  }
}

// project_out = false leaves out the final projection on k^perp: inside
// MINRES the output z only enters K z (B^T k = 0) and inner products with
// vectors whose pressure part is orthogonal to k (the pressure rows of K
// produce B u, and k^T B = 0), so every MINRES scalar is the same, and the k
// component that x picks up is removed with the pressure means at the end.
// For the same reason the fused path then also leaves out the input
// projection: the residual it is applied to is orthogonal to k already
// (b's pressure part is -B u_B, K's pressure rows are B u), so the
// projection would only remove rounding, at the price of a reduction and
// its finishing launch on the critical branch.
template <typename T>
void Problem::mq_cheb(const double* r, double* z, long long ld, int batch, Gate gate, double scale,
                      bool project_out) {
  T* rr = static_cast<T*>(mq_r);
  T* zz = static_cast<T*>(mq_z);
  T* tt = static_cast<T*>(mq_t);
  T* dd = static_cast<T*>(mq_d);
  const long long np = (long long)g.nk + g.n0;
  const int nbk = dot_blocks(np);
  RedCtx rin = red(nbk, 1, EPI_SCALE, &d_scale[1]);
  const bool project_in = project_out || !fused_mq;
  if (project_in) launch_mq_kdot<double>(g, r, ld, g.off_pk(), batch, rin, gate, st);
  if (fused_mq) {
    // ping-pong between mq_z and mq_t; the result ends in zz
    // step k reads zb[k&1] and writes zb[(k+1)&1]; the last step must write zz.
    // The first step takes r from the FP64 vectors with the input projection
    // (no separate projection launch).  k^T z of the output projection stays a
    // kernel of its own: reduced by the fused step, its summation order would
    // follow the tile side, which set-up picks by timing, and results would
    // then differ in the last bits between otherwise identical problems.
    mq_chain<T>(mq_variant_for(batch), rr, zz, tt, r, ld, z, scale, !project_out, project_in, batch, gate);
    if (!project_out) return;   // the last step wrote scale * z to the output
  } else {
    launch_mq_project_in<T>(g, r, ld, rr, zz, tt, dd, batch, mq_coef, gate, st);
    static const int order[9] = {0, 1, 2, 3, 4, 3, 2, 1, 0};
    for (int k = 0; k < d.mq_steps; ++k) {
      for (int c = 0; c < 9; ++c) launch_mq_colour<T>(g, rr, tt, order[c], batch, gate, st);
      launch_mq_cheb_combine<T>(g, tt, zz, dd, mq_a[k], mq_b[k], k == 0, batch, gate, st);
    }
  }
  RedCtx rout = red(nbk, 1, EPI_SCALE, &d_scale[2]);
  launch_mq_kdot<T>(g, zz, np, 0, batch, rout, gate, st);
  launch_mq_project_out<T>(g, zz, z, ld, batch, mq_coef2, scale, gate, st);
}

void Problem::mq_solve(const double* r, double* z, long long ld, int batch, Gate gate, double scale,
                       bool project_out) {
  if (d.mq_mode == ETH_MQ_DIAG) {
    const long long np = (long long)g.nk + g.n0;
    RedCtx rc = red(dot_blocks(np), 1, EPI_SCALE, &d_scale[0]);
    launch_mq_diag_dot(g, r, ld, batch, rc, gate, st);
    launch_mq_diag_apply(g, r, z, ld, batch, mq_coef, scale, gate, st);
  } else if (d.mq_mode == ETH_MQ_SCHUR_GMG) {
    if (mixed) mq_schur<float>(r, z, ld, batch, gate, scale);
    else mq_schur<double>(r, z, ld, batch, gate, scale);
  } else if (mixed) {
    mq_cheb<float>(r, z, ld, batch, gate, scale, project_out);
  } else {
    mq_cheb<double>(r, z, ld, batch, gate, scale, project_out);
  }
}

void Problem::build_schur() {
  slv.clear();
  slv.push_back(g);
  {
    int n = d.n;
    double h = g.h;
    while (n % 2 == 0 && n > 4) {
      n /= 2;
      h *= 2.0;
      slv.push_back(make_geo(n, h));
    }
  }
  const int LS = (int)slv.size();
  const double h2 = g.h * g.h;   // every level uses the finest h^2 (see k_schur.hip)
  const size_t es = mixed ? sizeof(float) : sizeof(double);
  sb.assign(LS, nullptr);
  sx.assign(LS, nullptr);
  sxo.assign(LS, nullptr);
  for (int l = 0; l < LS; ++l) {
    const size_t n = (size_t)max_batch * slv[l].nk * es;
    sb[l] = alloc<char>(n);
    sx[l] = alloc<char>(n);
    sxo[l] = alloc<char>(n);
  }
  slam.assign(std::max(LS - 1, 0), 0.0);
  sca.assign(slam.size(), {});
  scb.assign(slam.size(), {});
  for (int l = 0; l + 1 < LS; ++l) {
    const Geo ql = slv[l];
    double* inv = alloc<double>(ql.nk);
    launch_sk_diag_inv(ql, h2, inv, st);
    auto apply = [&, ql](const double* x, double* y) {
      launch_sk_op<double>(ql, h2, 0, nullptr, x, y, 0.0, 0.0, 0, 1, no_gate(), st);
    };
    auto dinv = [&, ql, inv](const double* x, double* y) {
      launch_copy(ql.nk, x, 0, y, 0, 1, st);
      launch_vmul(ql.nk, inv, y, st);
    };
    slam[l] = lanczos_generic(ql.nk, apply, dinv, 30, true);
    cheb_coefs(d.gmg_lo_frac * slam[l], d.gmg_hi_frac * slam[l], d.gmg_degree, sca[l], scb[l]);
  }
  // coarsest: inverse of S + s 1 1^T (s = mean diagonal / n_k)
  {
    const Geo& gc = slv.back();
    const int ni = gc.nk;
    if (ni > 4225) throw std::runtime_error("unsupported:coarsest Q1 mesh of the S_k multigrid too large");
    s_coarse_ni = ni;
    double* cols = alloc<double>((size_t)ni * ni);
    double* acols = alloc<double>((size_t)ni * ni);
    launch_unit_columns(cols, ni, st);
    launch_sk_op<double>(gc, h2, 0, nullptr, cols, acols, 0.0, 0.0, 0, ni, no_gate(), st);
    double* inv = alloc<double>(ni);
    launch_sk_diag_inv(gc, h2, inv, st);
    std::vector<double> hd(ni);
    ETH_HIP(hipMemcpyAsync(hd.data(), inv, ni * sizeof(double), hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    double mean = 0.0;
    for (double v : hd) mean += (1.0 / v) / ni;
    double* work = alloc<double>(dense_inverse_work(ni));
    sAinv = alloc<double>((size_t)ni * ni);
    launch_dense_sym_shift(acols, ni, mean / ni, sAinv, st);
    launch_dense_inverse(sAinv, ni, work, st);
    launch_symmetrize(sAinv, ni, st);
  }
  ssums = alloc<double>(max_batch);
}

// S_k^+ on sb[0] -> sx[0] (one V-cycle; mean projections by the caller)
template <typename T>
void Problem::schur_vcycle(int batch, Gate gate) {
  const int LS = (int)slv.size();
  const double h2 = g.h * g.h;
  std::vector<T*> b(LS), x(LS), xo(LS);
  for (int l = 0; l < LS; ++l) {
    b[l] = static_cast<T*>(sb[l]);
    x[l] = static_cast<T*>(sx[l]);
    xo[l] = static_cast<T*>(sxo[l]);
  }
  const int deg = d.gmg_degree;
  for (int l = 0; l + 1 < LS; ++l) {
    for (int k = 0; k < deg; ++k) {
      launch_sk_op<T>(slv[l], h2, 1, b[l], x[l], xo[l], sca[l][k], scb[l][k], k == 0 ? 0 : 1, batch, gate, st);
      std::swap(x[l], xo[l]);
    }
    launch_sk_op<T>(slv[l], h2, 2, b[l], x[l], xo[l], 0.0, 0.0, 0, batch, gate, st);
    launch_q1_restrict<T>(slv[l], slv[l + 1], xo[l], b[l + 1], x[l + 1], batch, gate, st);
  }
  launch_q1_dense_solve<T>(sAinv, s_coarse_ni, b[LS - 1], x[LS - 1], batch, gate, st);
  for (int l = LS - 2; l >= 0; --l) {
    launch_q1_prolong_add<T>(slv[l], slv[l + 1], x[l + 1], x[l], batch, gate, st);
    for (int k = 0; k < deg; ++k) {
      launch_sk_op<T>(slv[l], h2, 1, b[l], x[l], xo[l], sca[l][k], scb[l][k], k == 0 ? 0 : 1, batch, gate, st);
      std::swap(x[l], xo[l]);
    }
  }
  if (x[0] != static_cast<T*>(sx[0]))
    launch_q1_shift<T, T>(slv[0], x[0], slv[0].nk, 0, static_cast<T*>(sx[0]), slv[0].nk, 0, nullptr, 1.0,
                          batch, gate, st);
}

template <typename T>
void Problem::mq_schur(const double* r, double* z, long long ld, int batch, Gate gate, double scale) {
  T* rr = static_cast<T*>(mq_r);
  T* zz = static_cast<T*>(mq_z);
  T* tt = static_cast<T*>(mq_t);
  T* dd = static_cast<T*>(mq_d);
  const long long np = (long long)g.nk + g.n0;
  const long long nk = g.nk;
  const int nbk = dot_blocks(np);
  RedCtx rin = red(nbk, 1, EPI_SCALE, &d_scale[1]);
  launch_mq_kdot<double>(g, r, ld, g.off_pk(), batch, rin, gate, st);
  launch_mq_project_in<T>(g, r, ld, rr, zz, tt, dd, batch, mq_coef, gate, st);
  T* b0 = static_cast<T*>(sb[0]);
  T* x0 = static_cast<T*>(sx[0]);
  launch_schur_rhs<T>(g, rr, b0, x0, batch, gate, st);
  RedCtx rs = red(dot_blocks(nk), 1, EPI_NONE, nullptr, ssums);
  launch_q1_sum<T>(g, b0, rs, batch, gate, st);
  launch_q1_shift<T, T>(g, b0, nk, 0, b0, nk, 0, ssums, 1.0, batch, gate, st);
  schur_vcycle<T>(batch, gate);
  launch_q1_sum<T>(g, x0, rs, batch, gate, st);
  launch_q1_shift<T, T>(g, x0, nk, 0, x0, nk, 0, ssums, 1.0, batch, gate, st);
  launch_schur_p0<T>(g, rr, x0, zz, batch, gate, st);
  RedCtx rout = red(nbk, 1, EPI_SCALE, &d_scale[2]);
  launch_mq_kdot<T>(g, zz, np, 0, batch, rout, gate, st);
  launch_mq_project_out<T>(g, zz, z, ld, batch, mq_coef2, scale, gate, st);
}

void Problem::precond(const double* r, double* z, long long ld, int batch, Gate gate, bool in_krylov) {
  // the two diagonal blocks read disjoint parts of r and write disjoint parts
  // of z, and share no workspace
  if (pst) {
    ETH_HIP(hipEventRecord(ev_pf, st));
    ETH_HIP(hipStreamWaitEvent(pst, ev_pf, 0));
    {
      struct Restore {
        hipStream_t& s;
        hipStream_t v;
        ~Restore() { s = v; }
      } restore{st, st};
      st = pst;
      mq_solve(r, z, ld, batch, gate, mq_sign * d.nu, !in_krylov);
    }
    ETH_HIP(hipEventRecord(ev_pj, pst));
  } else {
    mq_solve(r, z, ld, batch, gate, mq_sign * d.nu, !in_krylov);
  }
  if (mixed) vcycle<float>(r, z, ld, batch, gate);
  else vcycle<double>(r, z, ld, batch, gate);
  if (pst) ETH_HIP(hipStreamWaitEvent(st, ev_pj, 0));
}

// ---------------------------------------------------------------- MINRES
// One iteration of alg:minres.  parity selects which buffers hold
// (v_j, v_{j-1}), (zhat_j, zhat_{j+1}) and (w_j, w_{j-1}).
//
// The w/x update that closes iteration j is made by the v update of
// iteration j + 1 (one launch fewer per iteration; the update reads only
// zhat_j, w_j, w_{j-1}, x and the Givens coefficients, which nothing in
// between touches).  Its pending flag (wx_todo, set by the Givens step) is
// then cleared by the gamma dot instead of the apply, and the update of the
// last iteration of a run is made by minres_flush_wx.
void Problem::minres_iteration(int batch, int parity) {
  const int a = parity, b = 1 - parity;
  double* v = kv[a];
  double* vp = kv[b];
  double* z = kz[a];
  double* zn = kz[b];
  double* w = kw[a];
  double* wp = kw[b];
  const Gate gate = active_gate();
  // the delta reduction of the apply is finished inside the v update (one
  // launch fewer on the iteration's critical path)
  RedCtx rd = red(saddle_blocks(g), 1, EPI_MINRES_DELTA, d_ms);
  rd.defer = fold_delta ? 1 : 0;
  const ClearFlag clear_wx{&d_ms[0].wx_todo, (int)(sizeof(MinresScalars) / sizeof(int))};
  launch_apply_stokes(g, d.nu, z, ky, ldw, batch, gate, &rd, st, fold_wx ? no_clear() : clear_wx);
  // the previous iteration's buffers: its zhat is kz[b], its w kw[b], its
  // w_{j-1} (overwritten by w_{j+1}) kw[a]
  const MinresWx prev = fold_wx ? MinresWx{kz[b], kw[a], kw[b], kx} : MinresWx{};
  launch_minres_v(g.N, ky, v, vp, ldw, batch, d_ms, st, fold_delta ? rd.partials : nullptr,
                  apply_blocks(g), prev);   // vp <- v_{j+1}
  precond(vp, zn, ldw, batch, gate, true);
  RedCtx rg = red(dot_blocks(g.N), 1, EPI_MINRES_GAMMA, d_ms);
  launch_dot(g.N, zn, vp, ldw, batch, rg, gate, st, fold_wx ? clear_wx : no_clear());
  if (!fold_wx) launch_minres_wx(g.N, z, wp, w, kx, ldw, batch, d_ms, st);   // wp <- w_{j+1}
}

// The w/x update of the last iteration of a run of minres_iteration calls
// (an even count, so its parity is 1), and its flag cleared, so that the
// next run starts with nothing pending.
void Problem::minres_flush_wx(int batch) {
  if (!fold_wx) return;
  launch_minres_wx(g.N, kz[1], kw[0], kw[1], kx, ldw, batch, d_ms, st);
  launch_clear_flag(ClearFlag{&d_ms[0].wx_todo, (int)(sizeof(MinresScalars) / sizeof(int))}, batch, st);
}

// The captured graph of `iters` (even) MINRES iterations for `batch`
// right-hand sides, captured on the current stream at first use.
hipGraphExec_t Problem::iteration_graph(int batch, int iters) {
  const int slot = iters == 2 ? 0 : 1;
  if (gexecs[slot] && gexec_key[slot] == batch * 1024 + iters) return gexecs[slot];
  if (gexecs[slot]) {
    ETH_HIP(hipGraphExecDestroy(gexecs[slot]));
    gexecs[slot] = nullptr;
  }
  hipGraph_t graph;
  ETH_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < iters; ++i) minres_iteration(batch, i & 1);
  ETH_HIP(hipStreamEndCapture(st, &graph));
  ETH_HIP(hipGraphInstantiate(&gexecs[slot], graph, nullptr, nullptr, 0));
  ETH_HIP(hipGraphDestroy(graph));
  gexec_key[slot] = batch * 1024 + iters;
  return gexecs[slot];
}

void Problem::run_iterations(int batch, int count, bool use_graph) {
  // `count` is even: the buffer roles repeat every two iterations
  if (!use_graph) {
    for (int i = 0; i < count; ++i) minres_iteration(batch, i & 1);
    minres_flush_wx(batch);
    return;
  }
  // long chunks replay a graph of graph_iters iterations, the rest one of two
  auto replay = [&](hipStream_t s) {
    int left = count;
    if (graph_iters > 2 && left >= graph_iters) {
      hipGraphExec_t gl = iteration_graph(batch, graph_iters);
      for (; left >= graph_iters; left -= graph_iters) ETH_HIP(hipGraphLaunch(gl, s));
    }
    if (left > 0) {
      hipGraphExec_t g2 = iteration_graph(batch, 2);
      for (; left > 0; left -= 2) ETH_HIP(hipGraphLaunch(g2, s));
    }
    minres_flush_wx(batch);   // on st == s
  };
  if (own_stream) {
    // a ragged-batch member captures and replays on its own stream: one
    // stream per member spreads the members evenly over the hardware queues
    replay(st);
    return;
  }
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
  replay(gst);
  ETH_HIP(hipEventRecord(ev_join, gst));
  ETH_HIP(hipStreamWaitEvent(caller, ev_join, 0));
}

void Problem::load_rhs(const double* b, long long ld, int batch, bool adjoint) {
  // Krylov RHS: b with the boundary rows zeroed (they carry Dirichlet data)
  launch_copy(g.N, b, ld, kb, ldw, batch, st);
  launch_zero_boundary(g, kb, ldw, batch, st);
  if (adjoint) {
    launch_pressure_sums(g, kb, ldw, batch, red_partials, red_result, st);
    launch_pressure_shift(g, kb, ldw, batch, red_result, st);
  }
}

void Problem::minres_begin(MinresRun& R, bool enqueue) {
  const eth_solve_opts& o = R.o;
  const int batch = R.batch;
  R.tol = o.rtol > 0 ? o.rtol : 1e-8;
  R.maxit = o.maxit > 0 ? o.maxit : 1000;
  R.use_graph = o.use_graph != 0;
  R.done = 0;
  R.chunk = 8;
  R.prev_rel = 1.0;
  R.prev_it = 0;
  R.refine_left = std::max(0, std::min(o.refine, 10));
  R.runs = 0;
  R.gamma0.assign(batch, 0.0);
  R.rel.assign(batch, 1.0);
  R.iters.assign(batch, 0);
  R.hist.assign(o.residual_history ? batch : 0, std::vector<double>());
  load_rhs(R.b, R.ld, batch, R.adjoint);
  // initial residual v1 = b - K x0
  if (o.use_x0) {
    launch_copy(g.N, R.x, R.ld, kx, ldw, batch, st);
    launch_zero_boundary(g, kx, ldw, batch, st);
    launch_apply_stokes(g, d.nu, kx, ky, ldw, batch, no_gate(), nullptr, st);
    launch_residual_init(g, kb, ky, kv[0], ldw, batch, st);
  } else {
    launch_fill(g.N, 0.0, kx, ldw, batch, st);
    launch_copy(g.N, kb, ldw, kv[0], ldw, batch, st);
  }
  launch_fill(g.N, 0.0, kv[1], ldw, batch, st);
  launch_fill(g.N, 0.0, kw[0], ldw, batch, st);
  launch_fill(g.N, 0.0, kw[1], ldw, batch, st);
  // scalar state
  for (int r = 0; r < batch; ++r) {
    MinresScalars& sc = h_ms[r];
    std::memset(&sc, 0, sizeof(sc));
    sc.tol = R.tol;
    sc.tol_abs = 0.0;
    sc.maxit = R.maxit;
    sc.hist = d_hist + (size_t)r * hist_len;
    sc.hist_delta = d_hist_delta + (size_t)r * hist_len;
    sc.hist_gamma = d_hist_gamma + (size_t)r * hist_len;
    sc.hist_len = hist_len;
    sc.active = 1;
  }
  have_lanczos = !R.adjoint;
  ETH_HIP(hipMemcpyAsync(d_ms, h_ms, sizeof(MinresScalars) * batch, hipMemcpyHostToDevice, st));
  // z1 = P^{-1} v1, gamma_1
  precond(kv[0], kz[0], ldw, batch, no_gate(), true);
  RedCtx ri = red(dot_blocks(g.N), 1, EPI_MINRES_INIT, d_ms);
  launch_dot(g.N, kz[0], kv[0], ldw, batch, ri, no_gate(), st);
  if (enqueue) minres_enqueue_chunk(R);
}

// enqueue R.chunk iterations, then the copy of the scalars to the host and
// the event that marks it
void Problem::minres_enqueue_chunk(MinresRun& R) {
  run_iterations(R.batch, R.chunk, R.use_graph);
  R.done += R.chunk;
  ETH_HIP(hipMemcpyAsync(h_ms, d_ms, sizeof(MinresScalars) * R.batch, hipMemcpyDeviceToHost, st));
  ETH_HIP(hipEventRecord(ev_poll, st));
}

bool Problem::minres_poll(MinresRun& R, bool block) {
  if (block) {
    ETH_HIP(hipEventSynchronize(ev_poll));
  } else {
    const hipError_t q = hipEventQuery(ev_poll);
    if (q == hipErrorNotReady) return false;
    ETH_HIP(q);
  }
  const int batch = R.batch;
  bool any = false;
  double worst_rel = 0.0;
  int it = 0;
  for (int r = 0; r < batch; ++r) {
    if (h_ms[r].active) {
      any = true;
      worst_rel = std::max(worst_rel, h_ms[r].rel);
      it = std::max(it, h_ms[r].iters);
    }
  }
  if (any && R.done < R.maxit + 2) {
    // iterate in chunks, predicting the remaining count from the recent rate
    int next = 8;
    if (it > R.prev_it && worst_rel > 0 && R.prev_rel > worst_rel) {
      const double rate = std::pow(worst_rel / R.prev_rel, 1.0 / (it - R.prev_it));
      if (rate < 1.0 && rate > 0.0) {
        const double rem = std::log(R.tol / worst_rel) / std::log(rate);
        next = (int)std::ceil(rem) + 1;
      } else {
        next = 16;
      }
    }
    next = std::max(2, std::min(next, 64));
    next += next & 1;
    R.prev_rel = worst_rel;
    R.prev_it = it;
    R.chunk = next;
    minres_enqueue_chunk(R);
    return false;
  }
  return minres_conclude(R);
}

bool Problem::minres_conclude(MinresRun& R) {
  const int batch = R.batch;
  minres_end_of_run(R);
  if (R.refine_left > 0) {
    // restart from x when every right-hand side met the recurrence's test
    // (no breakdown, no iteration limit) and one of them still iterated
    bool ok = true, iterated = false;
    for (int r = 0; r < batch; ++r) {
      ok = ok && h_ms[r].status == kStOK && !h_ms[r].active && R.iters[r] < R.maxit;
      iterated = iterated || h_ms[r].iters > 0;
    }
    if (ok && iterated) {
      --R.refine_left;
      minres_restart(R);
      return false;
    }
  }
  // output: x = interior solution + Dirichlet rows, canonical pressure
  launch_copy(g.N, kx, ldw, R.x, R.ld, batch, st);
  if (!R.adjoint) launch_copy_boundary(g, R.b, R.x, R.ld, batch, st);
  if (R.o.canonicalize) {
    launch_pressure_sums(g, R.x, R.ld, batch, red_partials, red_result, st);
    launch_pressure_shift(g, R.x, R.ld, batch, red_result, st);
  }
  return true;
}

// Book-keeping after one MINRES run (the first start or a restart) has
// ended: iterations, |eta| relative to the first start's gamma_1, history.
void Problem::minres_end_of_run(MinresRun& R) {
  const int batch = R.batch;
  std::vector<double> hbuf;
  if (!R.hist.empty()) {
    hbuf.resize((size_t)batch * hist_len);
    ETH_HIP(hipMemcpyAsync(hbuf.data(), d_hist, sizeof(double) * hbuf.size(), hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
  }
  for (int r = 0; r < batch; ++r) {
    const MinresScalars& sc = h_ms[r];
    if (R.runs == 0) R.gamma0[r] = sc.gamma1;
    const double scale = R.gamma0[r] > 0.0 ? sc.gamma1 / R.gamma0[r] : 0.0;
    R.iters[r] += sc.iters;
    R.rel[r] = sc.rel * scale;
    if (!R.hist.empty()) {
      const int k = std::min(sc.iters, hist_len - 1);
      for (int j = 0; j <= k; ++j) R.hist[r].push_back(hbuf[(size_t)r * hist_len + j] * scale);
    }
  }
  ++R.runs;
}

// FP64 defect correction: residual b - K x formed again from the current
// iterate, MINRES restarted on it with the absolute threshold
// rtol * gamma_1(first start); right-hand sides already below it stop at the
// start.  The Lanczos record of the first start is kept for EST-MINRES.
void Problem::minres_restart(MinresRun& R) {
  const int batch = R.batch;
  launch_apply_stokes(g, d.nu, kx, ky, ldw, batch, no_gate(), nullptr, st);
  launch_residual_init(g, kb, ky, kv[0], ldw, batch, st);
  launch_fill(g.N, 0.0, kv[1], ldw, batch, st);
  launch_fill(g.N, 0.0, kw[0], ldw, batch, st);
  launch_fill(g.N, 0.0, kw[1], ldw, batch, st);
  int most = 0;
  for (int r = 0; r < batch; ++r) {
    MinresScalars& sc = h_ms[r];
    std::memset(&sc, 0, sizeof(sc));
    sc.tol = R.tol;
    sc.tol_abs = std::max(R.tol * R.gamma0[r], 1e-300);
    sc.maxit = std::max(1, R.maxit - R.iters[r]);
    sc.hist = d_hist + (size_t)r * hist_len;
    sc.hist_len = hist_len;
    sc.active = 1;
    most = std::max(most, R.iters[r]);
  }
  ETH_HIP(hipMemcpyAsync(d_ms, h_ms, sizeof(MinresScalars) * batch, hipMemcpyHostToDevice, st));
  precond(kv[0], kz[0], ldw, batch, no_gate(), true);
  RedCtx ri = red(dot_blocks(g.N), 1, EPI_MINRES_INIT, d_ms);
  launch_dot(g.N, kz[0], kv[0], ldw, batch, ri, no_gate(), st);
  R.done = most;
  R.chunk = 8;
  R.prev_rel = 1.0;
  R.prev_it = 0;
  minres_enqueue_chunk(R);
}

std::vector<int> Problem::check_rhs(const double* b, long long ld, int batch, bool consistency) {
  // interior norm of b (boundary rows hold Dirichlet data) and the two
  // pressure-block sums
  launch_copy(g.N, b, ld, ky, ldw, batch, st);
  launch_zero_boundary(g, ky, ldw, batch, st);
  RedCtx rn = red(dot_blocks(g.N), 1, EPI_NONE, nullptr, red_result);
  launch_dot(g.N, ky, ky, ldw, batch, rn, no_gate(), st);
  ETH_HIP(hipMemcpyAsync(h_red, red_result, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
  ETH_HIP(hipStreamSynchronize(st));
  std::vector<double> nb2(h_red, h_red + batch);
  launch_pressure_sums(g, b, ld, batch, red_partials, red_result, st);
  ETH_HIP(hipMemcpyAsync(h_red, red_result, sizeof(double) * 2 * batch, hipMemcpyDeviceToHost, st));
  ETH_HIP(hipStreamSynchronize(st));
  std::vector<int> out(batch, ETH_OK);
  for (int r = 0; r < batch; ++r) {
    const double sk = h_red[2 * r], s0 = h_red[2 * r + 1];
    if (!std::isfinite(nb2[r]) || !std::isfinite(sk) || !std::isfinite(s0)) {
      out[r] = ETH_EINVAL;
      continue;
    }
    // Euclidean length of the projection of b onto null(K^T)
    const double pn = std::sqrt(sk * sk / g.nk + s0 * s0 / g.n0);
    if (consistency && pn > 1e-12 * std::sqrt(nb2[r])) out[r] = ETH_EINCONSISTENT;
  }
  return out;
}

int Problem::minres_finish(MinresRun& R, eth_solve_info* info) {
  const int batch = R.batch;
  std::vector<double> true_rel(batch, -1.0);
  if (R.o.true_residual) {
    launch_apply_stokes(g, d.nu, kx, ky, ldw, batch, no_gate(), nullptr, st);
    // kv[1] <- kb - K x (boundary rows zero)
    launch_residual_init(g, kb, ky, kv[1], ldw, batch, st);
    RedCtx r1 = red(dot_blocks(g.N), 1, EPI_NONE, nullptr, red_result);
    launch_dot(g.N, kv[1], kv[1], ldw, batch, r1, no_gate(), st);
    ETH_HIP(hipMemcpyAsync(h_red, red_result, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    std::vector<double> rr(h_red, h_red + batch);
    launch_dot(g.N, kb, kb, ldw, batch, r1, no_gate(), st);
    ETH_HIP(hipMemcpyAsync(h_red, red_result, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < batch; ++r)
      true_rel[r] = h_red[r] > 0 ? std::sqrt(rr[r] / h_red[r]) : 0.0;
  }
  ETH_HIP(hipStreamSynchronize(st));
  int worst = ETH_OK;
  for (int r = 0; r < batch; ++r) {
    const MinresScalars& sc = h_ms[r];
    int status = sc.status;
    if (status == kStOK && sc.active) status = ETH_WMAXIT;
    if (info) {
      info[r].status = status;
      info[r].iterations = R.runs ? R.iters[r] : sc.iters;
      info[r].stage1_iterations = 0;
      info[r].rel_residual_est = R.runs ? R.rel[r] : sc.rel;
      info[r].rel_residual_true = true_rel[r];
    }
    if (R.o.residual_history && R.o.history_len > 0) {
      double* out = R.o.residual_history + (size_t)r * R.o.history_len;
      const std::vector<double>* hv = R.hist.empty() ? nullptr : &R.hist[r];
      for (int j = 0; j < R.o.history_len; ++j)
        out[j] = (hv && j < (int)hv->size()) ? (*hv)[j] : -1.0;
    }
    if (status < 0) worst = std::min(worst, status);
    else if (worst >= 0) worst = std::max(worst, status);
  }
  return worst;
}

int Problem::solve_minres(const eth_solve_opts& o, const double* b, double* x, int batch,
                          long long ld, eth_solve_info* info, bool adjoint) {
  PhaseRange range(adjoint ? "eth_minres_adjoint" : "eth_minres");
  MinresRun R;
  R.o = o;
  R.b = b;
  R.x = x;
  R.batch = batch;
  R.ld = ld;
  R.adjoint = adjoint;
  minres_begin(R);
  while (!minres_poll(R, true)) {
  }
  return minres_finish(R, info);
}

// ============================================================================
// Oseen (Sec. 3)
// ============================================================================
double Problem::lanczos_generic(long long len,
                                const std::function<void(const double*, double*)>& apply,
                                const std::function<void(const double*, double*)>& dinv, int steps,
                                bool mean_zero) {
  // PCG (Jacobi) on A x = b; its coefficients give the Lanczos tridiagonal of
  // D^{-1}A, whose largest Ritz value is returned.
  double* r = alloc<double>(len);
  double* z = alloc<double>(len);
  double* p = alloc<double>(len);
  double* q = alloc<double>(len);
  std::vector<double> h(len);
  unsigned long long sd = 0x2545F4914F6CDD1DULL;
  double mean = 0.0;
  for (long long i = 0; i < len; ++i) {
    sd = sd * 6364136223846793005ULL + 1442695040888963407ULL;
    h[i] = (double)((sd >> 11) & ((1ULL << 53) - 1)) / (double)(1ULL << 53) - 0.5;
    mean += h[i];
  }
  if (mean_zero)
    for (auto& v : h) v -= mean / len;
  ETH_HIP(hipMemcpyAsync(r, h.data(), len * sizeof(double), hipMemcpyHostToDevice, st));
  auto dot = [&](const double* a, const double* b) {
    RedCtx rc = red(dot_blocks(len), 1, EPI_NONE, nullptr, red_result);
    launch_dot(len, a, b, 0, 1, rc, no_gate(), st);
    ETH_HIP(hipMemcpyAsync(h_red, red_result, sizeof(double), hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    return h_red[0];
  };
  dinv(r, z);
  launch_copy(len, z, 0, p, 0, 1, st);
  double rz = dot(r, z);
  std::vector<double> al, be;
  for (int k = 0; k < steps; ++k) {
    apply(p, q);
    const double pq = dot(p, q);
    if (!(pq > 0.0)) break;
    const double alpha = rz / pq;
    launch_axpby(len, -alpha, q, 1.0, r, 0, 1, st);
    dinv(r, z);
    const double rzn = dot(r, z);
    const double beta = rzn / rz;
    al.push_back(alpha);
    be.push_back(beta);
    launch_axpby(len, 1.0, z, beta, p, 0, 1, st);
    rz = rzn;
    if (!(rz > 0.0)) break;
  }
  const int m = (int)al.size();
  std::vector<double> ta(m), tb(m > 0 ? m - 1 : 0);
  for (int k = 0; k < m; ++k) {
    ta[k] = 1.0 / al[k] + (k > 0 ? be[k - 1] / al[k - 1] : 0.0);
    if (k + 1 < m) tb[k] = std::sqrt(be[k]) / al[k];
  }
  return m > 0 ? tridiag_max_eig(ta, tb) : 1.0;
}

void Problem::build_oseen_velocity() {
  lv.clear();
  lv.push_back(g);
  if (d.velocity_mode == ETH_VEL_GMG) {
    int n = d.n;
    double h = g.h;
    while (n % 2 == 0 && n > d.gmg_coarse_n) {
      n /= 2;
      h *= 2.0;
      lv.push_back(make_geo(n, h));
    }
  }
  const int L = (int)lv.size();
  lwind.assign(L, nullptr);
  ldF.assign(L, nullptr);
  lwind[0] = wind0;
  lwindF.assign(L, nullptr);
  for (int l = 0; l < L; ++l) {
    if (l > 0) lwind[l] = alloc<double>(2 * (size_t)lv[l].nv);
    ldF[l] = alloc<double>(lv[l].nv);
    if (mixed) lwindF[l] = alloc<float>(2 * (size_t)lv[l].nv);
  }
  const Geo& gc = lv.back();
  coarse_ni = (gc.nq - 2) * (gc.nq - 2);
  if (coarse_ni > kDenseCoarseMax)
    throw std::runtime_error("unsupported:coarsest mesh too large for the dense solve");
  dense_gbuf = alloc<double>((size_t)2 * coarse_ni * max_batch);
  f_work = alloc<double>(dense_inverse_work(coarse_ni));
  Ainv = alloc<double>((size_t)coarse_ni * coarse_ni);
  AinvT = alloc<double>((size_t)coarse_ni * coarse_ni);
  if (mixed) {
    AinvF = alloc<float>((size_t)coarse_ni * coarse_ni);
    AinvTF = alloc<float>((size_t)coarse_ni * coarse_ni);
  }
  refresh_wind();
  vb.assign(L, nullptr);
  vx.assign(L, nullptr);
  vxo.assign(L, nullptr);
  const size_t es = mixed ? sizeof(float) : sizeof(double);
  for (int l = 0; l < L; ++l) {
    const size_t n = (size_t)2 * max_batch * lv[l].nv * es;
    vb[l] = alloc<char>(n);
    vx[l] = alloc<char>(n);
    vxo[l] = alloc<char>(n);
    ETH_HIP(hipMemsetAsync(vb[l], 0, n, st));
    ETH_HIP(hipMemsetAsync(vx[l], 0, n, st));
    ETH_HIP(hipMemsetAsync(vxo[l], 0, n, st));
  }
}

// Everything of the Oseen preconditioners that depends on the wind: the wind
// of each multigrid level (injection), the diagonals of F per level and the
// dense inverse of the coarsest F (nonsymmetric, positive real: blocked
// Gauss-Jordan without pivoting) with its transpose.  F_1 of the PCD reads the finest wind
// when applied.  Allocates nothing.
void Problem::refresh_wind() {
  const int L = (int)lv.size();
  // level viscosities: nu, or with a Peclet cap max(nu, max|w| h_l / (2 cap))
  lnu.assign(L, d.nu);
  if (d.gmg_peclet_max > 0.0) {
    launch_wind_speed_max(g, wind0, red_result, st);
    double wmax = 0.0;
    ETH_HIP(hipMemcpyAsync(h_red, red_result, sizeof(double), hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    wmax = h_red[0];
    for (int l = 0; l < L; ++l) lnu[l] = std::max(d.nu, wmax * lv[l].h / (2.0 * d.gmg_peclet_max));
  }
  for (int l = 0; l < L; ++l) {
    if (l > 0) launch_inject_wind(g, lv[l], wind0, lwind[l], st);
    launch_cd_diag(lv[l], lwind[l], lnu[l], ldF[l], st);
    // the FP32 smoother rounds the wind to FP32 as it stages it: a rounded
    // copy gives the same values at half the bytes
    if (lwindF[l]) launch_to_float(lwind[l], lwindF[l], 2LL * lv[l].nv, st);
  }
  const int ni = coarse_ni;
  launch_fill((long long)ni * ni, 0.0, Ainv, 0, 1, st);
  launch_dense_convdiff(lv.back(), lwind[L - 1], lnu[L - 1], Ainv, ni, st);
  launch_dense_inverse(Ainv, ni, f_work, st);
  launch_transpose(Ainv, ni, AinvT, st);
  if (AinvF) {
    launch_to_float(Ainv, AinvF, (long long)ni * ni, st);
    launch_to_float(AinvT, AinvTF, (long long)ni * ni, st);
  }
}

void Problem::build_pcd() {
  // Q1 hierarchy for A_p (halve while even and > 4)
  qlv.clear();
  qlv.push_back(g);
  {
    int n = d.n;
    double h = g.h;
    while (n % 2 == 0 && n > 4) {
      n /= 2;
      h *= 2.0;
      qlv.push_back(make_geo(n, h));
    }
  }
  const int LQ = (int)qlv.size();
  const size_t es = mixed ? sizeof(float) : sizeof(double);
  qb.assign(LQ, nullptr);
  qx.assign(LQ, nullptr);
  qxo.assign(LQ, nullptr);
  qdAp.assign(LQ, nullptr);
  for (int l = 0; l < LQ; ++l) {
    const size_t n = (size_t)max_batch * qlv[l].nk * es;
    qb[l] = alloc<char>(n);
    qx[l] = alloc<char>(n);
    qxo[l] = alloc<char>(n);
    qdAp[l] = alloc<double>(qlv[l].nk);
    launch_ap_diag(qlv[l], qdAp[l], st);
  }
  qlam.assign(std::max(LQ - 1, 0), 0.0);
  qca.assign(qlam.size(), {});
  qcb.assign(qlam.size(), {});
  for (int l = 0; l + 1 < LQ; ++l) {
    const Geo ql = qlv[l];
    auto apply = [&, ql](const double* x, double* y) {
      launch_ap_op<double>(ql, 0, nullptr, x, y, 0.0, 0.0, 0, nullptr, 1, no_gate(), st);
    };
    // Jacobi scaling z = D^{-1} r with D = diag(A_p)
    double* inv = alloc<double>(ql.nk);
    {
      std::vector<double> hd(ql.nk);
      ETH_HIP(hipMemcpyAsync(hd.data(), qdAp[l], ql.nk * sizeof(double), hipMemcpyDeviceToHost, st));
      ETH_HIP(hipStreamSynchronize(st));
      for (auto& v : hd) v = 1.0 / v;
      ETH_HIP(hipMemcpyAsync(inv, hd.data(), ql.nk * sizeof(double), hipMemcpyHostToDevice, st));
    }
    auto dinv = [&, ql, inv](const double* x, double* y) {
      launch_copy(ql.nk, x, 0, y, 0, 1, st);
      launch_vmul(ql.nk, inv, y, st);
    };
    qlam[l] = lanczos_generic(ql.nk, apply, dinv, 30, true);
    cheb_coefs(d.gmg_lo_frac * qlam[l], d.gmg_hi_frac * qlam[l], d.gmg_degree, qca[l], qcb[l]);
  }
  // coarsest: inverse of A_p + s 1 1^T (s = mean diagonal / n_k), SPD
  {
    const Geo& gc = qlv.back();
    const int ni = gc.nk;
    if (ni > 4225)
      throw std::runtime_error("unsupported:coarsest Q1 mesh of the PCD multigrid too large");
    q_coarse_ni = ni;
    double* cols = alloc<double>((size_t)ni * ni);
    double* acols = alloc<double>((size_t)ni * ni);
    launch_unit_columns(cols, ni, st);
    launch_ap_op<double>(gc, 0, nullptr, cols, acols, 0.0, 0.0, 0, nullptr, ni, no_gate(), st);
    std::vector<double> hd(ni);
    ETH_HIP(hipMemcpyAsync(hd.data(), qdAp.back(), ni * sizeof(double), hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    double mean = 0.0;
    for (double v : hd) mean += v / ni;
    double* work = alloc<double>(dense_inverse_work(ni));
    qAinv = alloc<double>((size_t)ni * ni);
    launch_dense_sym_shift(acols, ni, mean / ni, qAinv, st);
    launch_dense_inverse(qAinv, ni, work, st);
    launch_symmetrize(qAinv, ni, st);
  }
  const size_t nq1 = (size_t)max_batch * g.nk * es;
  pa = alloc<char>(nq1);
  pb = alloc<char>(nq1);
  pc = alloc<char>(nq1);
  q1sums = alloc<double>(max_batch);
  cheb_coefs(0.25, 2.25, d.pcd_q1_steps, q1a, q1b);   // Wathen's interval for Q1 mass
}

void Problem::build_gmres() {
  gm_m = d.gmres_restart;
  const size_t vec = (size_t)ldw * max_batch;
  gV = alloc<double>(vec * (gm_m + 1));
  gZ = alloc<double>(vec * gm_m);
  const size_t per = (size_t)(gm_m + 1) * gm_m + 7 * 64;
  gArr = alloc<double>(per * max_batch);
  gpart = alloc<double>((size_t)64 * gmres_blocks(g.N) * max_batch);
  ghist = alloc<double>((size_t)hist_len * max_batch);
  d_gm = alloc<GmresScalars>(max_batch);
  ETH_HIP(hipHostMalloc((void**)&h_gm, sizeof(GmresScalars) * max_batch, hipHostMallocDefault));
  h_bnorm.assign(max_batch, 0.0);
}

template <typename T>
void Problem::vcycle_F(const double* r, const double* sub, double* z, long long ld, int batch,
                       Gate gate, bool trans) {
  const int tr = trans ? 1 : 0;
  const int L = (int)lv.size();
  std::vector<T*> b(L), x(L), xo(L);
  for (int l = 0; l < L; ++l) {
    b[l] = static_cast<T*>(vb[l]);
    x[l] = static_cast<T*>(vx[l]);
    xo[l] = static_cast<T*>(vxo[l]);
  }
  const int np = 2 * batch, deg = d.gmg_degree;
  const double om = d.gmg_omega;
  launch_vcycle_entry<T>(lv[0], r, ld, b[0], x[0], 0.0, batch, gate, st, sub);   // x = 0
  for (int l = 0; l + 1 < L; ++l) {
    for (int k = 0; k < deg; ++k) {
      launch_cd_step<T>(lv[l], level_wind<T>(l), ldF[l], lnu[l], b[l], x[l], xo[l], om, 0, np, nullptr, 0, 0.0,
                        gate, st, tr);
      std::swap(x[l], xo[l]);
    }
    launch_cd_step<T>(lv[l], level_wind<T>(l), ldF[l], lnu[l], b[l], x[l], xo[l], om, 1, np, nullptr, 0, 0.0,
                      gate, st, tr);
    launch_restrict<T>(lv[l], lv[l + 1], xo[l], nullptr, b[l + 1], x[l + 1], 0.0, np, batch, gate, st);
  }
  launch_dense_solve<T>(lv[L - 1], trans ? AinvT : Ainv, trans ? AinvTF : AinvF, coarse_ni, b[L - 1],
                        L == 1 ? nullptr : x[L - 1], np,
                        L == 1 ? z : nullptr, ld, 1.0, nullptr, 0, dense_gbuf, batch, gate, st);
  if (L == 1) {
    launch_zero_boundary(lv[0], z, ld, batch, st);
    return;
  }
  for (int l = L - 2; l >= 0; --l) {
    launch_prolong_add<T>(lv[l], lv[l + 1], x[l + 1], x[l], np, batch, gate, st);
    for (int k = 0; k < deg; ++k) {
      const bool last = (l == 0 && k == deg - 1);
      launch_cd_step<T>(lv[l], level_wind<T>(l), ldF[l], lnu[l], b[l], x[l], xo[l], om, 0, np,
                        last ? z : nullptr, ld, 1.0, gate, st, tr);
      if (!last) std::swap(x[l], xo[l]);
    }
  }
}

// A_p^+ on qb[0] -> qx[0] (one V-cycle; both input and output mean-projected
// by the caller)
template <typename T>
void Problem::ap_vcycle(int batch, Gate gate) {
  const int LQ = (int)qlv.size();
  std::vector<T*> b(LQ), x(LQ), xo(LQ);
  for (int l = 0; l < LQ; ++l) {
    b[l] = static_cast<T*>(qb[l]);
    x[l] = static_cast<T*>(qx[l]);
    xo[l] = static_cast<T*>(qxo[l]);
  }
  const int deg = d.gmg_degree;
  // levels from l0 (the first with n <= aptail_max_n) down are one launch per RHS
  int l0 = LQ;
  if (fused_aptail && deg <= 4 && LQ - 1 <= APT_L)
    for (int l = 0; l < LQ; ++l)
      if (qlv[l].n <= aptail_max_n) {
        l0 = l;
        break;
      }
  if (l0 < LQ && LQ - l0 > APT_L) l0 = LQ;
  const int lstop = l0 < LQ ? l0 : LQ - 1;   // per-level launches above lstop
  for (int l = 0; l < lstop; ++l) {
    for (int k = 0; k < deg; ++k) {
      launch_ap_op<T>(qlv[l], 1, b[l], x[l], xo[l], qca[l][k], qcb[l][k], k == 0 ? 0 : 1, qdAp[l],
                      batch, gate, st);
      std::swap(x[l], xo[l]);
    }
    launch_ap_op<T>(qlv[l], 2, b[l], x[l], xo[l], 0.0, 0.0, 0, qdAp[l], batch, gate, st);
    launch_q1_restrict<T>(qlv[l], qlv[l + 1], xo[l], b[l + 1], x[l + 1], batch, gate, st);
  }
  if (l0 < LQ) {
    ApTail tl{};
    tl.nlev = LQ - l0;
    tl.deg = deg;
    tl.ni = q_coarse_ni;
    tl.Ainv = qAinv;
    tl.off[0] = 0;
    for (int t = 0; t < tl.nlev; ++t) {
      const Geo& gq = qlv[l0 + t];
      tl.n[t] = gq.n;
      tl.h[t] = gq.h;
      tl.dAp[t] = qdAp[l0 + t];
      tl.off[t + 1] = tl.off[t] + (gq.n + 1) * (gq.n + 1);
      for (int k = 0; k < deg && t + 1 < tl.nlev; ++k) {
        tl.ca[t][k] = qca[l0 + t][k];
        tl.cb[t][k] = qcb[l0 + t][k];
      }
    }
    launch_ap_tail<T>(tl, b[l0], x[l0], batch, gate, st);
  } else {
    launch_q1_dense_solve<T>(qAinv, q_coarse_ni, b[LQ - 1], x[LQ - 1], batch, gate, st);
  }
  for (int l = std::min(l0, LQ - 1) - 1; l >= 0; --l) {
    launch_q1_prolong_add<T>(qlv[l], qlv[l + 1], x[l + 1], x[l], batch, gate, st);
    for (int k = 0; k < deg; ++k) {
      launch_ap_op<T>(qlv[l], 1, b[l], x[l], xo[l], qca[l][k], qcb[l][k], k == 0 ? 0 : 1, qdAp[l],
                      batch, gate, st);
      std::swap(x[l], xo[l]);
    }
  }
  // the result must end in qx[0]
  if (x[0] != static_cast<T*>(qx[0]))
    launch_q1_shift<T, T>(qlv[0], x[0], qlv[0].nk, 0, static_cast<T*>(qx[0]), qlv[0].nk, 0, nullptr, 1.0,
                          batch, gate, st);
}

// z_pk = -A_p^+ F_1 Q_1^{-1} r_pk (trans: the Schur approximation of the
// transposed system, z_pk = -Q_1^{-1} F_1^T A_p^+ r_pk); z_p0 is left alone
template <typename T>
void Problem::pcd_schur(const double* r, double* z, long long ld, int batch, Gate gate, bool trans) {
  T* A = static_cast<T*>(pa);
  T* B = static_cast<T*>(pb);
  T* C = static_cast<T*>(pc);
  T* qb0 = static_cast<T*>(qb[0]);
  T* qx0 = static_cast<T*>(qx[0]);
  const long long nk = g.nk;
  RedCtx rs = red(dot_blocks(nk), 1, EPI_NONE, nullptr, q1sums);
  // A_p^+ of A into the target, mean projection on input and output
  auto ap_pinv = [&](T* src, auto* dst, long long ldd, long long offd, double scale) {
    launch_q1_sum<T>(g, src, rs, batch, gate, st);
    launch_q1_shift<T, T>(g, src, nk, 0, qb0, nk, 0, q1sums, 1.0, batch, gate, st);
    launch_q1_shift<T, T>(g, src, nk, 0, qx0, nk, 0, nullptr, 0.0, batch, gate, st);
    ap_vcycle<T>(batch, gate);
    launch_q1_sum<T>(g, qx0, rs, batch, gate, st);
    launch_q1_shift<T, std::remove_pointer_t<decltype(dst)>>(g, qx0, nk, 0, dst, ldd, offd, q1sums, scale,
                                                            batch, gate, st);
  };
  auto q1_inv = [&](T* b, T* cur, T* oth) { return q1_inverse<T>(b, cur, oth, batch, gate); };
  launch_q1_shift<double, T>(g, r, ld, g.off_pk(), A, nk, 0, nullptr, 1.0, batch, gate, st);
  if (!trans) {
    T* q = q1_inv(A, B, C);
    launch_f1_apply<T>(g, wind0, d.nu, q, A, batch, gate, st, 0);
    ap_pinv(A, z, ld, g.off_pk(), -1.0);
  } else {
    ap_pinv(A, A, nk, 0, 1.0);
    launch_f1_apply<T>(g, wind0, d.nu, A, B, batch, gate, st, 1);
    T* q = q1_inv(B, C, A);
    launch_q1_shift<T, double>(g, q, nk, 0, z, ld, g.off_pk(), nullptr, -1.0, batch, gate, st);
  }
}

// Q_1^{-1} b: Chebyshev-Jacobi on [1/4, 9/4]
template <typename T>
T* Problem::q1_inverse(T* b, T* cur, T* oth, int batch, Gate gate) {
  if (fused_q1 && d.pcd_q1_steps <= 12) {   // every step in one launch, bit for bit the same
    Q1Cheb cc{};
    cc.steps = d.pcd_q1_steps;
    for (int k = 0; k < cc.steps; ++k) {
      cc.a[k] = q1a[k];
      cc.b[k] = q1b[k];
    }
    launch_q1mass_cheb_fused<T>(g, b, cur, cc, batch, gate, st);
    return cur;
  }
  launch_q1mass_cheb<T>(g, b, nullptr, cur, 0.0, q1b[0], 0, batch, gate, st);
  for (int k = 1; k < d.pcd_q1_steps; ++k) {
    launch_q1mass_cheb<T>(g, b, cur, oth, q1a[k], q1b[k], k == 1 ? 2 : 1, batch, gate, st);
    std::swap(cur, oth);
  }
  return cur;
}

double Problem::dot1(const double* a, const double* b) {
  RedCtx rc = red(dot_blocks(g.N), 1, EPI_NONE, nullptr, red_result);
  launch_dot(g.N, a, b, ldw, 1, rc, no_gate(), st);
  ETH_HIP(hipMemcpyAsync(h_red, red_result, sizeof(double), hipMemcpyDeviceToHost, st));
  ETH_HIP(hipStreamSynchronize(st));
  return h_red[0];
}

// remove the means of the Q1 and P0 blocks (the null space of B^T)
void Problem::project_pressure(double* x) {
  launch_pressure_sums(g, x, ldw, 1, red_partials, red_result, st);
  launch_pressure_shift(g, x, ldw, 1, red_result, st);
}

// q = [0; B M^{-1} B^T p_p] for p = [0; p_p] (M = diag of the velocity mass
// on the interior nodes): B^T and B from the saddle apply with nu = 0
void Problem::lp_apply(const double* p, double* q) {
  double* t = s2v[5];
  launch_apply_stokes(g, 0.0, p, t, ldw, 1, no_gate(), nullptr, st);
  launch_vel_minv(g, t, st);
  launch_apply_stokes(g, 0.0, t, q, ldw, 1, no_gate(), nullptr, st);
}

// x = (B M^{-1} B^T)^+ b by conjugate gradients on the range (b and x with
// zero velocity parts; b is projected first, x at the end): from x = 0 until
// ||r|| <= schur_cg_tol ||b||, at most schur_cg_maxit steps
int Problem::lp_pinv(double* b, double* x) {
  double *r = s2v[2], *p = s2v[3], *q = s2v[4];
  project_pressure(b);
  launch_fill(g.N, 0.0, x, ldw, 1, st);
  launch_copy(g.N, b, ldw, r, ldw, 1, st);
  launch_copy(g.N, b, ldw, p, ldw, 1, st);
  double rho = dot1(r, r);
  const double stop = d.schur_cg_tol * d.schur_cg_tol * rho;
  int it = 0;
  while (rho > stop && it < d.schur_cg_maxit) {
    lp_apply(p, q);
    const double pq = dot1(p, q);
    if (!(pq > 0.0)) break;
    const double alpha = rho / pq;
    launch_axpby(g.N, alpha, p, 1.0, x, ldw, 1, st);
    launch_axpby(g.N, -alpha, q, 1.0, r, ldw, 1, st);
    const double rn = dot1(r, r);
    launch_axpby(g.N, 1.0, r, rn / rho, p, ldw, 1, st);
    rho = rn;
    ++it;
  }
  project_pressure(x);
  return it;
}

template <typename T>
void Problem::schur2(const double* r, double* z, Gate gate) {
  double *b = s2v[0], *x = s2v[1], *t = s2v[5], *t2 = s2v[6];
  const long long np = (long long)g.nk + g.n0;
  launch_fill(g.N, 0.0, b, ldw, 1, st);
  if (d.oseen_schur == 1) {
    // [F_1 Q_1^{-1} r_k ; F_0 Q_0^{-1} r_0]  (Q_0 = h^2 I)
    T* A = static_cast<T*>(pa);
    T* B = static_cast<T*>(pb);
    T* C = static_cast<T*>(pc);
    launch_q1_shift<double, T>(g, r, ldw, g.off_pk(), A, g.nk, 0, nullptr, 1.0, 1, gate, st);
    T* q = q1_inverse<T>(A, B, C, 1, gate);
    launch_f1_apply<T>(g, wind0, d.nu, q, A, 1, gate, st, 0);
    launch_q1_shift<T, double>(g, A, g.nk, 0, b, ldw, g.off_pk(), nullptr, 1.0, 1, gate, st);
    launch_p0_cd_apply(g, wind0, d.nu, r + g.off_p0(), 1.0 / (g.h * g.h), b + g.off_p0(), st);
  } else {
    launch_copy(np, r + g.off_pk(), ldw, b + g.off_pk(), ldw, 1, st);
  }
  lp_last_iters = lp_pinv(b, x);
  if (d.oseen_schur == 2) {
    // LSC: the middle factor B M^{-1} F M^{-1} B^T, then the pressure Laplacian again
    launch_apply_stokes(g, 0.0, x, t, ldw, 1, no_gate(), nullptr, st);
    launch_vel_minv(g, t, st);
    launch_apply_oseen(g, d.nu, d.wind, 0, t, t2, ldw, 1, no_gate(), nullptr, st);
    launch_vel_minv(g, t2, st);
    launch_apply_stokes(g, 0.0, t2, b, ldw, 1, no_gate(), nullptr, st);
    lp_last_iters += lp_pinv(b, x);
  }
  launch_fill(np, 0.0, z + g.off_pk(), ldw, 1, st);
  launch_axpby(np, -1.0, x + g.off_pk(), 0.0, z + g.off_pk(), ldw, 1, st);
}

void Problem::precond_oseen(int kind, const double* r, double* z, int batch, Gate gate) {
  const GmresScalars* gs = (gate.p == gm_gate().p) ? d_gm : nullptr;
  const bool tr = (kind == 3 || kind == 4);
  if (kind == 2 || kind == 4) {
    if (mixed) pcd_schur<float>(r, z, ldw, batch, gate, tr);
    else pcd_schur<double>(r, z, ldw, batch, gate, tr);
    launch_gm_zero_range(z, ldw, g.off_p0(), g.n0, batch, gs, st);
  } else if (d.oseen_schur != 0) {
    if (kind == 3) throw std::runtime_error("unsupported:the transposed M_2 / M_3 preconditioner");
    if (batch != 1) throw std::runtime_error("unsupported:M_2 / M_3 take one right-hand side");
    if (mixed) schur2<float>(r, z, gate);
    else schur2<double>(r, z, gate);
  } else {
    mq_solve(r, z, ldw, batch, gate, -d.nu);
  }
  // z_u = F~^{-1}(r_u - B^T z_p): B^T z_p from the Stokes kernel with nu = 0
  launch_gm_zero_range(z, ldw, 0, 2LL * g.nv, batch, gs, st);
  launch_apply_stokes(g, 0.0, z, ky, ldw, batch, gate, nullptr, st);
  if (mixed) vcycle_F<float>(r, ky, z, ldw, batch, gate, tr);
  else vcycle_F<double>(r, ky, z, ldw, batch, gate, tr);
}

// Restarted FGMRES on the internal vectors b, x (stride ldw); kind selects
// the preconditioner (1: M_1, 2: PCD), reduced the stage-I operator (the p_0
// rows of K x are dropped).  atol: absolute tolerance per RHS.
void Problem::arnoldi_steps(int kind, bool reduced, bool transpose, int batch, int j0, int j1) {
  const Gate gate = gm_gate();
  const long long N = g.N;
  auto V = [&](int i) { return gV + (size_t)i * batch * ldw; };
  auto Z = [&](int i) { return gZ + (size_t)i * batch * ldw; };
  for (int j = j0; j < j1; ++j) {
    precond_oseen(kind, V(j), Z(j), batch, gate);
    apply_op(transpose ? 1 : 0, Z(j), V(j + 1), ldw, batch, gate, nullptr);
    if (reduced) launch_gm_zero_range(V(j + 1), ldw, g.off_p0(), g.n0, batch, d_gm, st);
    launch_gm_mdot(N, j + 1, gV, V(j + 1), ldw, batch, gpart, d_gm, 0, st);
    launch_gm_maxpy(N, j + 1, gV, V(j + 1), ldw, batch, d_gm, 0, st);
    launch_gm_mdot(N, j + 1, gV, V(j + 1), ldw, batch, gpart, d_gm, 1, st);
    launch_gm_maxpy(N, j + 1, gV, V(j + 1), ldw, batch, d_gm, 1, st);
    launch_gm_norm_givens(N, j, V(j + 1), ldw, batch, gpart, d_gm, st);
    launch_gm_scale(N, V(j + 1), ldw, batch, d_gm, st);
  }
}

void Problem::arnoldi_steps_graph(int kind, bool reduced, bool transpose, int batch, int j0, int j1) {
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
  const std::array<int, 6> key{kind, reduced ? 1 : 0, transpose ? 1 : 0, batch, j0, j1};
  auto it = gm_graphs.find(key);
  if (it == gm_graphs.end()) {
    hipGraph_t graph;
    ETH_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      arnoldi_steps(kind, reduced, transpose, batch, j0, j1);
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
    it = gm_graphs.emplace(key, exec).first;
  }
  ETH_HIP(hipGraphLaunch(it->second, gst));
  ETH_HIP(hipEventRecord(ev_join, gst));
  ETH_HIP(hipStreamWaitEvent(caller, ev_join, 0));
}

void Problem::run_fgmres(int kind, bool reduced, const double* b, double* x, int batch, int m,
                         int maxit, const std::vector<double>& atol, bool transpose, bool use_graph) {
  const size_t per = (size_t)(gm_m + 1) * gm_m + 7 * 64;
  for (int r = 0; r < batch; ++r) {
    GmresScalars& G = h_gm[r];
    std::memset(&G, 0, sizeof(G));
    G.target = atol[r];
    G.m = m;
    G.maxit = maxit;
    double* base = gArr + per * r;
    G.H = base;
    G.cs = base + (size_t)(gm_m + 1) * gm_m;
    G.sn = G.cs + 64;
    G.g = G.sn + 64;
    G.y = G.g + 64;
    G.h1 = G.y + 64;
    G.h2 = G.h1 + 64;
    G.hist = ghist + (size_t)hist_len * r;
    G.hist_len = hist_len;
  }
  ETH_HIP(hipMemcpyAsync(d_gm, h_gm, sizeof(GmresScalars) * batch, hipMemcpyHostToDevice, st));
  const Gate gate = gm_gate();
  const long long N = g.N;
  auto V = [&](int i) { return gV + (size_t)i * batch * ldw; };
  auto Z = [&](int i) { return gZ + (size_t)i * batch * ldw; };
  auto op = [&](const double* in, double* out, Gate gt) {
    apply_op(transpose ? 1 : 0, in, out, ldw, batch, gt, nullptr);
    if (reduced) launch_gm_zero_range(out, ldw, g.off_p0(), g.n0, batch, gt.p ? d_gm : nullptr, st);
  };
  for (int cycle = 0; cycle < 100000; ++cycle) {
    op(x, ky, no_gate());
    launch_residual_init(g, b, ky, V(0), ldw, batch, st);
    launch_gm_beta(N, V(0), ldw, batch, gpart, d_gm, st);
    launch_gm_scale(N, V(0), ldw, batch, d_gm, st);
    // chunks of 8 Arnoldi steps; steps after convergence are gated off on
    // the device, and the host looks at the flags between chunks
    for (int j0 = 0; j0 < m; j0 += 8) {
      const int j1 = std::min(j0 + 8, m);
      if (use_graph) arnoldi_steps_graph(kind, reduced, transpose, batch, j0, j1);
      else arnoldi_steps(kind, reduced, transpose, batch, j0, j1);
      if (j1 < m) {
        ETH_HIP(hipMemcpyAsync(h_gm, d_gm, sizeof(GmresScalars) * batch, hipMemcpyDeviceToHost, st));
        ETH_HIP(hipStreamSynchronize(st));
        bool any = false;
        for (int r = 0; r < batch; ++r) any = any || h_gm[r].active;
        if (!any) break;
      }
    }
    launch_gm_finish(N, gZ, x, ldw, batch, d_gm, st);
    ETH_HIP(hipMemcpyAsync(h_gm, d_gm, sizeof(GmresScalars) * batch, hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    bool more = false;
    for (int r = 0; r < batch; ++r) {
      const GmresScalars& G = h_gm[r];
      if (!G.converged && G.status >= 0 && G.iters < maxit) more = true;
    }
    if (!more) {
      // confirm with the true residual of the final iterate
      op(x, ky, no_gate());
      launch_residual_init(g, b, ky, V(0), ldw, batch, st);
      launch_gm_beta(N, V(0), ldw, batch, gpart, d_gm, st);
      ETH_HIP(hipMemcpyAsync(h_gm, d_gm, sizeof(GmresScalars) * batch, hipMemcpyDeviceToHost, st));
      ETH_HIP(hipStreamSynchronize(st));
      break;
    }
  }
}

int Problem::solve_oseen(const eth_solve_opts& o, const double* b, double* x, int batch, long long ld,
                         eth_solve_info* info, bool adjoint) {
  const double eta = o.rtol > 0 ? o.rtol : 1e-6;
  const int maxit = o.maxit > 0 ? o.maxit : 1000;
  const int m = o.restart > 0 ? o.restart : gm_m;
  if (m > gm_m) throw std::invalid_argument("restart exceeds the gmres_restart of the problem");
  const double c = o.c_factor > 0 ? o.c_factor : 10.0;
  load_rhs(b, ld, batch, adjoint);
  RedCtx rn = red(dot_blocks(g.N), 1, EPI_NONE, nullptr, red_result);
  launch_dot(g.N, kb, kb, ldw, batch, rn, no_gate(), st);
  ETH_HIP(hipMemcpyAsync(h_red, red_result, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
  ETH_HIP(hipStreamSynchronize(st));
  std::vector<double> bn(batch), r0(batch);
  for (int r = 0; r < batch; ++r) bn[r] = r0[r] = std::sqrt(h_red[r]);
  if (o.use_x0) {
    launch_copy(g.N, x, ld, kx, ldw, batch, st);
    launch_zero_boundary(g, kx, ldw, batch, st);
    // the initial guess and its residual: the result falls back to it when
    // the iteration ends worse (kw[1] is free outside MINRES)
    launch_copy(g.N, kx, ldw, kw[1], ldw, batch, st);
    apply_op(adjoint ? 1 : 0, kx, ky, ldw, batch, no_gate(), nullptr);
    launch_residual_init(g, kb, ky, kv[1], ldw, batch, st);
    launch_dot(g.N, kv[1], kv[1], ldw, batch, rn, no_gate(), st);
    ETH_HIP(hipMemcpyAsync(h_red, red_result, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < batch; ++r) r0[r] = std::sqrt(h_red[r]);
  } else {
    launch_fill(g.N, 0.0, kx, ldw, batch, st);
  }
  // residual history (host), stage by stage from the device record
  const bool want_hist = o.residual_history && o.history_len > 0;
  std::vector<std::vector<double>> hist(want_hist ? batch : 0);
  auto take_hist = [&]() {
    std::vector<double> hb((size_t)batch * hist_len);
    ETH_HIP(hipMemcpyAsync(hb.data(), ghist, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, st));
    ETH_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < batch; ++r) {
      const int k = std::min(h_gm[r].iters, hist_len - 1);
      for (int j = 0; j <= k; ++j) hist[r].push_back(bn[r] > 0 ? hb[(size_t)r * hist_len + j] / bn[r] : 0.0);
    }
  };
  std::vector<int> it1(batch, 0);
  PhaseRange range(adjoint ? "eth_fgmres_adjoint" : "eth_fgmres");
  if (o.method == ETH_TWO_STAGE) {
    PhaseRange stage("stage I (reduced system, PCD)");
    // stage I: reduced system [F B_1^T; B_1 0] (adjoint: its transpose), RHS
    // without the P0 rows
    launch_copy(g.N, kb, ldw, kv[0], ldw, batch, st);
    launch_gm_zero_range(kv[0], ldw, g.off_p0(), g.n0, batch, nullptr, st);
    launch_gm_zero_range(kx, ldw, g.off_p0(), g.n0, batch, nullptr, st);
    std::vector<double> a1(batch);
    for (int r = 0; r < batch; ++r) a1[r] = c * eta * bn[r];
    run_fgmres(adjoint ? 4 : 2, true, kv[0], kx, batch, m, maxit, a1, adjoint, o.use_graph != 0);
    for (int r = 0; r < batch; ++r) it1[r] = h_gm[r].iters;
    if (want_hist) take_hist();
  }
  std::vector<double> a2(batch);
  for (int r = 0; r < batch; ++r) a2[r] = eta * bn[r];
  // the M_2 / M_3 Schur blocks synchronise with the host inside (inner CG):
  // their Arnoldi steps run eagerly
  {
    PhaseRange stage("stage II (full system)");
    run_fgmres(adjoint ? 3 : 1, false, kb, kx, batch, m, std::max(1, maxit), a2, adjoint,
               o.use_graph != 0 && d.oseen_schur == 0);
  }
  if (want_hist) take_hist();
  // a result whose true residual exceeds that of the initial guess (the
  // preconditioner made no headway, e.g. a convection-dominated F beyond
  // what its multigrid smooths) falls back to the initial guess
  std::vector<char> noprog(batch, 0);
  for (int r = 0; r < batch; ++r) {
    if (h_gm[r].status < 0 || !(h_gm[r].beta > r0[r] * (1.0 + 1e-12))) continue;
    noprog[r] = 1;
    if (o.use_x0) launch_copy(g.N, kw[1] + (size_t)r * ldw, ldw, kx + (size_t)r * ldw, ldw, 1, st);
    else launch_fill(g.N, 0.0, kx + (size_t)r * ldw, ldw, 1, st);
  }
  // output
  launch_copy(g.N, kx, ldw, x, ld, batch, st);
  if (!adjoint) launch_copy_boundary(g, b, x, ld, batch, st);
  if (o.canonicalize) {
    launch_pressure_sums(g, x, ld, batch, red_partials, red_result, st);
    launch_pressure_shift(g, x, ld, batch, red_result, st);
  }
  ETH_HIP(hipStreamSynchronize(st));
  int worst = ETH_OK;
  for (int r = 0; r < batch; ++r) {
    const GmresScalars& G = h_gm[r];
    int status = G.status;
    if (status == kStOK && !G.converged) status = ETH_WMAXIT;
    const double fin = noprog[r] ? r0[r] : G.beta;
    if (noprog[r]) status = ETH_WNOPROGRESS;
    if (info) {
      info[r].status = status;
      info[r].iterations = G.iters + it1[r];
      info[r].stage1_iterations = it1[r];
      info[r].rel_residual_est = bn[r] > 0 ? fin / bn[r] : 0.0;
      info[r].rel_residual_true = bn[r] > 0 ? fin / bn[r] : 0.0;
    }
    if (want_hist) {
      double* out = o.residual_history + (size_t)r * o.history_len;
      for (int j = 0; j < o.history_len; ++j) out[j] = j < (int)hist[r].size() ? hist[r][j] : -1.0;
    }
    if (status < 0) worst = std::min(worst, status);
    else if (worst >= 0) worst = std::max(worst, status);
  }
  return worst;
}

// Picard (fixed-point) linearisation of the steady Navier-Stokes equations
// (Sec. 3: the wind of eq:generic-conv-diff is the velocity of the latest
// nonlinear iterate): each step takes the wind from the velocity of x, lifts
// the right-hand side with it and solves the Oseen system from x.
int Problem::picard(const eth_solve_opts& o, int steps, const double* f_nodal, double* x,
                    eth_solve_info* info) {
  eth_solve_opts os = o;
  os.use_x0 = 1;
  int worst = ETH_OK;
  for (int s = 0; s < steps; ++s) {
    ETH_HIP(hipMemcpyAsync(wind0, x, 2 * sizeof(double) * g.nv, hipMemcpyDeviceToDevice, st));
    refresh_wind();
    launch_lift_rhs(g, d.nu, wind0, ub, f_nodal, 2LL * g.nv, pic_b, g.N, 1, st);
    const int status = solve_oseen(os, pic_b, x, 1, g.N, info ? info + s : nullptr, false);
    if (status < 0) return status;
    worst = std::max(worst, status);
  }
  // the wind of the next step: the system a following solve sees
  if (steps > 0) {
    ETH_HIP(hipMemcpyAsync(wind0, x, 2 * sizeof(double) * g.nv, hipMemcpyDeviceToDevice, st));
    refresh_wind();
  }
  return worst;
}

}  // namespace eth

// =============================================================================
// C ABI
// =============================================================================
struct eth_problem {
  eth::Problem impl;
};

using eth::Problem;

static int fail(eth_problem* p, int code, const std::string& msg) {
  if (p) p->impl.err = msg;
  else eth::g_setup_error = msg;
  return code;
}

template <typename F>
static int guarded(eth_problem* p, F&& f) {
  try {
    return f();
  } catch (const eth::HipError& e) {
    return fail(p, ETH_EDEVICE, e.where + ": " + hipGetErrorString(e.err));
  } catch (const std::bad_alloc&) {
    return fail(p, ETH_ENOMEM, "device allocation failed");
  } catch (const std::invalid_argument& e) {
    return fail(p, ETH_EINVAL, e.what());
  } catch (const std::runtime_error& e) {
    const std::string m = e.what();
    if (m.rfind("unsupported:", 0) == 0) return fail(p, ETH_EUNSUPPORTED, m.substr(12));
    return fail(p, ETH_EDEVICE, m);
  }
}

static bool check_batch(eth_problem* p, int64_t batch, int64_t ld) {
  if (batch < 1 || batch > p->impl.max_batch) return false;
  if (batch > 1 && ld < p->impl.g.N) return false;
  return true;
}

extern "C" {

int eth_setup(const eth_problem_desc* desc, eth_problem** out) {
  if (!out) return fail(nullptr, ETH_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(nullptr, ETH_EINVAL, "desc is NULL");
  eth_problem* p = new (std::nothrow) eth_problem();
  if (!p) return fail(nullptr, ETH_ENOMEM, "host allocation failed");
  int rc;
  try {
    p->impl.setup(*desc);
    rc = ETH_OK;
  } catch (const eth::HipError& e) {
    rc = fail(nullptr, ETH_EDEVICE, e.where + ": " + hipGetErrorString(e.err));
  } catch (const std::bad_alloc&) {
    rc = fail(nullptr, ETH_ENOMEM, "device allocation failed");
  } catch (const std::invalid_argument& e) {
    rc = fail(nullptr, ETH_EINVAL, e.what());
  } catch (const std::runtime_error& e) {
    const std::string m = e.what();
    rc = (m.rfind("unsupported:", 0) == 0) ? fail(nullptr, ETH_EUNSUPPORTED, m.substr(12))
                                           : fail(nullptr, ETH_EDEVICE, m);
  }
  if (rc != ETH_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return ETH_OK;
}

int eth_destroy(eth_problem* p) {
  if (!p) return ETH_EINVAL;
  (void)hipStreamSynchronize(p->impl.st);
  delete p;
  return ETH_OK;
}

int64_t eth_vector_length(const eth_problem* p) { return p ? p->impl.g.N : -1; }

int eth_get_levels(const eth_problem* p, int32_t* levels, double* lambdas) {
  if (!p) return ETH_EINVAL;
  if (levels) *levels = (int32_t)p->impl.lv.size();
  if (lambdas)
    for (size_t i = 0; i < p->impl.lam.size(); ++i) lambdas[i] = p->impl.lam[i];
  return ETH_OK;
}

int eth_assemble_rhs(eth_problem* p, const double* f_nodal, int64_t ld_f, double* b,
                     int64_t batch, int64_t ld) {
  if (!p || !b) return fail(p, ETH_EINVAL, "NULL handle or b");
  if (!check_batch(p, batch, ld)) return fail(p, ETH_EINVAL, "invalid batch or ld");
  if (f_nodal && batch > 1 && ld_f < 2LL * p->impl.g.nv) return fail(p, ETH_EINVAL, "ld_f too small");
  return guarded(p, [&] {
    Problem& P = p->impl;
    eth::launch_lift_rhs(P.g, P.d.nu, P.oseen ? P.d.wind : nullptr, P.ub, f_nodal, ld_f, b, ld,
                         (int)batch, P.st);
    return ETH_OK;
  });
}

int eth_apply_operator(eth_problem* p, int transpose, const double* x, double* y, int64_t batch,
                       int64_t ld) {
  if (!p || !x || !y) return fail(p, ETH_EINVAL, "NULL argument");
  if (!check_batch(p, batch, ld)) return fail(p, ETH_EINVAL, "invalid batch or ld");
  if (x == y) return fail(p, ETH_EINVAL, "x and y must not alias");
  return guarded(p, [&] {
    Problem& P = p->impl;
    P.apply_op(transpose, x, y, ld, (int)batch, eth::no_gate(), nullptr);
    return ETH_OK;
  });
}

int eth_apply_preconditioner(eth_problem* p, int transpose, const double* r, double* z,
                             int64_t batch, int64_t ld) {
  if (!p || !r || !z) return fail(p, ETH_EINVAL, "NULL argument");
  if (!check_batch(p, batch, ld)) return fail(p, ETH_EINVAL, "invalid batch or ld");
  if (r == z) return fail(p, ETH_EINVAL, "r and z must not alias");
  return guarded(p, [&] {
    Problem& P = p->impl;
    if (P.oseen) {
      // the Oseen pieces work on the internal vector stride
      eth::launch_copy(P.g.N, r, ld, P.kv[0], P.ldw, (int)batch, P.st);
      P.precond_oseen(transpose ? 3 : 1, P.kv[0], P.kz[0], (int)batch, eth::no_gate());
      eth::launch_copy(P.g.N, P.kz[0], P.ldw, z, ld, (int)batch, P.st);
    } else {
      P.precond(r, z, ld, (int)batch, eth::no_gate());   // symmetric: transpose is the same
    }
    return ETH_OK;
  });
}

int eth_solve_adjoint(eth_problem* p, const eth_solve_opts* opts, const double* g, double* lambda,
                      int64_t batch, int64_t ld, eth_solve_info* info) {
  if (!p || !g || !lambda) return fail(p, ETH_EINVAL, "NULL argument");
  if (!check_batch(p, batch, ld)) return fail(p, ETH_EINVAL, "invalid batch or ld");
  if (g == lambda) return fail(p, ETH_EINVAL, "g and lambda must not alias");
  eth_solve_opts o{};
  if (opts) {
    o = *opts;
  } else {
    o.canonicalize = 1;
    o.method = p->impl.oseen ? ETH_TWO_STAGE : ETH_MINRES;
  }
  if (o.maxit > 4096) return fail(p, ETH_EINVAL, "maxit > 4096");
  if (o.residual_history && o.history_len < 1) return fail(p, ETH_EINVAL, "history_len must be >= 1");
  {
    bool finite = true;
    const int rc = guarded(p, [&] {
      for (int s : p->impl.check_rhs(g, ld, (int)batch, false)) finite = finite && s == ETH_OK;
      return ETH_OK;
    });
    if (rc != ETH_OK) return rc;
    if (!finite) return fail(p, ETH_EINVAL, "adjoint right-hand side holds a NaN or Inf");
  }
  if (p->impl.oseen) {
    if (o.method != ETH_FGMRES && o.method != ETH_TWO_STAGE)
      return fail(p, ETH_EUNSUPPORTED, "Oseen adjoints are solved by FGMRES or TWO_STAGE");
    return guarded(p, [&] { return p->impl.solve_oseen(o, g, lambda, (int)batch, ld, info, true); });
  }
  if (o.method != ETH_MINRES) return fail(p, ETH_EUNSUPPORTED, "only MINRES is available for Stokes");
  return guarded(p, [&] { return p->impl.solve_minres(o, g, lambda, (int)batch, ld, info, true); });
}

int eth_grad_forcing(eth_problem* p, const double* lambda, int64_t ld, double* dJdf, int64_t ld_f,
                     int64_t batch) {
  if (!p || !lambda || !dJdf) return fail(p, ETH_EINVAL, "NULL argument");
  if (!check_batch(p, batch, ld)) return fail(p, ETH_EINVAL, "invalid batch or ld");
  if (batch > 1 && ld_f < 2LL * p->impl.g.nv) return fail(p, ETH_EINVAL, "ld_f too small");
  return guarded(p, [&] {
    Problem& P = p->impl;
    eth::launch_velocity_mass(P.g, lambda, ld, nullptr, 0, 1, dJdf, ld_f, nullptr, (int)batch, P.st);
    return ETH_OK;
  });
}

int eth_grad_viscosity(eth_problem* p, const double* lambda, const double* x, double* dJdnu,
                       int64_t batch, int64_t ld) {
  if (!p || !lambda || !x || !dJdnu) return fail(p, ETH_EINVAL, "NULL argument");
  if (!check_batch(p, batch, ld)) return fail(p, ETH_EINVAL, "invalid batch or ld");
  return guarded(p, [&] {
    Problem& P = p->impl;
    eth::RedCtx rc = P.red(0, 1, eth::EPI_NONE, nullptr, dJdnu);
    eth::launch_grad_viscosity(P.g, lambda, ld, x, ld, rc, (int)batch, P.st);
    return ETH_OK;
  });
}

int eth_misfit(eth_problem* p, const double* x, const double* x_target, double* J, double* grad,
               int64_t batch, int64_t ld) {
  if (!p || !x || !x_target || !J) return fail(p, ETH_EINVAL, "NULL argument");
  if (!check_batch(p, batch, ld)) return fail(p, ETH_EINVAL, "invalid batch or ld");
  return guarded(p, [&] {
    Problem& P = p->impl;
    eth::RedCtx rc = P.red(0, 1, eth::EPI_NONE, nullptr, J);
    if (grad) {
      const long long np = (long long)P.g.nk + P.g.n0;
      eth::launch_fill(np, 0.0, grad + P.g.off_pk(), ld, (int)batch, P.st);
    }
    eth::launch_velocity_mass(P.g, x, ld, x_target, ld, 0, grad, ld, &rc, (int)batch, P.st);
    return ETH_OK;
  });
}

// ------------------------------------------------------------ ragged batches
}  // extern "C"

struct eth_batch {
  std::vector<eth_problem*> probs;
  hipStream_t caller = nullptr;
  hipEvent_t ev_in = nullptr;
  std::vector<hipEvent_t> ev_out;
  std::string err;
  // use_graph = 2: every member's iterations of one chunk in one captured
  // graph, replayed on jst (created at first use)
  hipStream_t jst = nullptr;
  hipEvent_t ev_fork = nullptr, ev_done = nullptr;
  hipGraphExec_t joint = nullptr;
  ~eth_batch() {
    if (jst) (void)hipStreamSynchronize(jst);
    for (auto* p : probs) {
      if (!p) continue;
      (void)hipStreamSynchronize(p->impl.st);
      delete p;
    }
    for (auto e : ev_out) (void)hipEventDestroy(e);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (joint) (void)hipGraphExecDestroy(joint);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_done) (void)hipEventDestroy(ev_done);
    if (jst) (void)hipStreamDestroy(jst);
  }
};

namespace {
constexpr int kJointChunk = 8;   // MINRES iterations per replay of the joint graph

// One graph holding kJointChunk MINRES iterations of every member, each on
// its own stream (captured by joining the member streams to a capture on
// jst with events), so one launch drives the whole ragged batch; members
// that have converged skip their kernels through their device flags.
void joint_graph(eth_batch* bt) {
  if (bt->joint) return;
  ETH_HIP(hipStreamCreateWithFlags(&bt->jst, hipStreamNonBlocking));
  ETH_HIP(hipEventCreateWithFlags(&bt->ev_fork, hipEventDisableTiming));
  ETH_HIP(hipEventCreateWithFlags(&bt->ev_done, hipEventDisableTiming));
  hipGraph_t graph;
  ETH_HIP(hipStreamBeginCapture(bt->jst, hipStreamCaptureModeThreadLocal));
  try {
    ETH_HIP(hipEventRecord(bt->ev_fork, bt->jst));
    for (size_t i = 0; i < bt->probs.size(); ++i) {
      Problem& P = bt->probs[i]->impl;
      ETH_HIP(hipStreamWaitEvent(P.st, bt->ev_fork, 0));
      P.run_iterations(1, kJointChunk, false);
      ETH_HIP(hipEventRecord(bt->ev_out[i], P.st));
      ETH_HIP(hipStreamWaitEvent(bt->jst, bt->ev_out[i], 0));
    }
  } catch (...) {
    hipGraph_t discard = nullptr;
    (void)hipStreamEndCapture(bt->jst, &discard);
    if (discard) (void)hipGraphDestroy(discard);
    throw;
  }
  ETH_HIP(hipStreamEndCapture(bt->jst, &graph));
  const hipError_t e = hipGraphInstantiate(&bt->joint, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  ETH_HIP(e);
}
}  // namespace

extern "C" {

int eth_batch_setup(const eth_problem_desc* descs, int32_t count, eth_batch** out) {
  if (!out) return fail(nullptr, ETH_EINVAL, "out is NULL");
  *out = nullptr;
  if (!descs || count < 1) return fail(nullptr, ETH_EINVAL, "descs is NULL or count < 1");
  for (int i = 0; i < count; ++i)
    if (descs[i].kind != ETH_STOKES)
      return fail(nullptr, ETH_EUNSUPPORTED, "ragged batches hold Stokes problems");
  std::unique_ptr<eth_batch> B(new (std::nothrow) eth_batch());
  if (!B) return fail(nullptr, ETH_ENOMEM, "host allocation failed");
  B->caller = static_cast<hipStream_t>(descs[0].stream);
  try {
    ETH_HIP(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
    for (int i = 0; i < count; ++i) {
      eth_problem_desc d = descs[i];
      // one Chebyshev step per launch unless asked: the two-step launch's
      // 832-thread blocks fill whole CUs, and members mixing the two variants
      // were measured to run one after another instead of together
      if (d.mq_fuse_steps == 0) d.mq_fuse_steps = 1;
      hipStream_t s = nullptr;
      ETH_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      d.stream = s;
      eth_problem* p = new eth_problem();
      p->impl.own_stream = true;   // set before setup: the stream is released with the problem
      p->impl.st = s;
      B->probs.push_back(p);
      p->impl.setup(d);
      hipEvent_t e = nullptr;
      ETH_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      B->ev_out.push_back(e);
    }
  } catch (const eth::HipError& e) {
    return fail(nullptr, ETH_EDEVICE, e.where + ": " + hipGetErrorString(e.err));
  } catch (const std::bad_alloc&) {
    return fail(nullptr, ETH_ENOMEM, "device allocation failed");
  } catch (const std::invalid_argument& e) {
    return fail(nullptr, ETH_EINVAL, e.what());
  } catch (const std::runtime_error& e) {
    const std::string m = e.what();
    return (m.rfind("unsupported:", 0) == 0) ? fail(nullptr, ETH_EUNSUPPORTED, m.substr(12))
                                             : fail(nullptr, ETH_EDEVICE, m);
  }
  *out = B.release();
  return ETH_OK;
}

int eth_batch_count(const eth_batch* b) { return b ? (int)b->probs.size() : -1; }

int eth_batch_problem(eth_batch* b, int32_t i, eth_problem** out) {
  if (!b || !out || i < 0 || i >= (int)b->probs.size()) return ETH_EINVAL;
  *out = b->probs[i];
  return ETH_OK;
}

int eth_batch_solve(eth_batch* bt, const eth_solve_opts* opts, const double* const* b, double* const* x,
                    eth_solve_info* infos) {
  if (!bt || !b || !x) return ETH_EINVAL;
  const int count = (int)bt->probs.size();
  for (int i = 0; i < count; ++i) {
    if (!b[i] || !x[i] || b[i] == x[i]) {
      bt->err = "NULL or aliased b/x";
      return ETH_EINVAL;
    }
  }
  eth_solve_opts o{};
  if (opts) o = *opts;
  else o.canonicalize = 1;
  if (o.method != ETH_MINRES || o.maxit > 4096) {
    bt->err = "ragged batches run MINRES with maxit <= 4096";
    return ETH_EINVAL;
  }
  if (o.use_graph == 2 && o.refine > 0) {
    bt->err = "the joint batch graph (use_graph = 2) takes no refinement restarts";
    return ETH_EUNSUPPORTED;
  }
  try {
    eth::PhaseRange range("eth_batch_solve");
    std::vector<Problem::MinresRun> runs(count);
    std::vector<char> done(count, 0);
    ETH_HIP(hipEventRecord(bt->ev_in, bt->caller));
    if (o.use_graph == 2) {
      // every member's set-up work on its stream, then one joint replay per
      // chunk on jst until no member is active
      joint_graph(bt);
      int maxit = 0;
      for (int i = 0; i < count; ++i) {
        Problem& P = bt->probs[i]->impl;
        ETH_HIP(hipStreamWaitEvent(P.st, bt->ev_in, 0));
        Problem::MinresRun& R = runs[i];
        R.o = o;
        R.b = b[i];
        R.x = x[i];
        R.batch = 1;
        R.ld = P.g.N;
        P.minres_begin(R, false);
        maxit = std::max(maxit, R.maxit);
        ETH_HIP(hipEventRecord(bt->ev_out[i], P.st));
        ETH_HIP(hipStreamWaitEvent(bt->jst, bt->ev_out[i], 0));
      }
      for (int it = 0; it < maxit + 2; it += kJointChunk) {
        ETH_HIP(hipGraphLaunch(bt->joint, bt->jst));
        for (int i = 0; i < count; ++i) {
          Problem& P = bt->probs[i]->impl;
          ETH_HIP(hipMemcpyAsync(P.h_ms, P.d_ms, sizeof(eth::MinresScalars), hipMemcpyDeviceToHost, bt->jst));
        }
        ETH_HIP(hipStreamSynchronize(bt->jst));
        bool any = false;
        for (int i = 0; i < count; ++i) any = any || bt->probs[i]->impl.h_ms[0].active;
        if (!any) break;
      }
      ETH_HIP(hipEventRecord(bt->ev_done, bt->jst));
      int worst = ETH_OK;
      for (int i = 0; i < count; ++i) {
        Problem& P = bt->probs[i]->impl;
        ETH_HIP(hipStreamWaitEvent(P.st, bt->ev_done, 0));
        (void)P.minres_conclude(runs[i]);
        const int st = P.minres_finish(runs[i], infos ? &infos[i] : nullptr);
        ETH_HIP(hipEventRecord(bt->ev_out[i], P.st));
        ETH_HIP(hipStreamWaitEvent(bt->caller, bt->ev_out[i], 0));
        if (st < 0) worst = std::min(worst, st);
        else if (worst >= 0) worst = std::max(worst, st);
      }
      return worst;
    }
    for (int i = 0; i < count; ++i) {
      Problem& P = bt->probs[i]->impl;
      ETH_HIP(hipStreamWaitEvent(P.st, bt->ev_in, 0));
      Problem::MinresRun& R = runs[i];
      R.o = o;
      R.b = b[i];
      R.x = x[i];
      R.batch = 1;
      R.ld = P.g.N;
      P.minres_begin(R);
    }
    int pending = count;
    while (pending > 0) {
      bool progress = false;
      for (int i = 0; i < count; ++i) {
        if (done[i]) continue;
        if (bt->probs[i]->impl.minres_poll(runs[i], false)) {
          done[i] = 1;
          --pending;
          progress = true;
        }
      }
      if (!progress) {
        // wait for the first unfinished problem; the others keep running
        for (int i = 0; i < count; ++i) {
          if (done[i]) continue;
          if (bt->probs[i]->impl.minres_poll(runs[i], true)) {
            done[i] = 1;
            --pending;
          }
          break;
        }
      }
    }
    int worst = ETH_OK;
    for (int i = 0; i < count; ++i) {
      Problem& P = bt->probs[i]->impl;
      const int st = P.minres_finish(runs[i], infos ? &infos[i] : nullptr);
      ETH_HIP(hipEventRecord(bt->ev_out[i], P.st));
      ETH_HIP(hipStreamWaitEvent(bt->caller, bt->ev_out[i], 0));
      if (st < 0) worst = std::min(worst, st);
      else if (worst >= 0) worst = std::max(worst, st);
    }
    return worst;
  } catch (const eth::HipError& e) {
    bt->err = e.where + ": " + hipGetErrorString(e.err);
    return ETH_EDEVICE;
  } catch (const std::exception& e) {
    bt->err = e.what();
    return ETH_EDEVICE;
  }
}

const char* eth_batch_last_error(const eth_batch* b) { return b ? b->err.c_str() : ""; }

int eth_batch_destroy(eth_batch* b) {
  if (!b) return ETH_EINVAL;
  delete b;
  return ETH_OK;
}

int eth_infsup_estimate(eth_problem* p, int64_t rhs, double* gamma2, double* theta, int32_t* steps) {
  if (!p || !gamma2) return fail(p, ETH_EINVAL, "NULL argument");
  Problem& P = p->impl;
  if (P.oseen) return fail(p, ETH_EUNSUPPORTED, "the inf-sup estimate belongs to MINRES (Stokes)");
  if (!P.have_lanczos) return fail(p, ETH_EINVAL, "no MINRES solve recorded yet");
  if (rhs < 0 || rhs >= P.max_batch) return fail(p, ETH_EINVAL, "invalid rhs index");
  return guarded(p, [&] {
    const int k = std::min(P.h_ms[rhs].iters, P.hist_len - 1);
    if (k < 1) throw std::invalid_argument("no Lanczos step recorded");
    std::vector<double> dl(k), gm(k + 1);
    ETH_HIP(hipMemcpyAsync(dl.data(), P.d_hist_delta + (size_t)rhs * P.hist_len, sizeof(double) * k,
                           hipMemcpyDeviceToHost, P.st));
    ETH_HIP(hipMemcpyAsync(gm.data(), P.d_hist_gamma + (size_t)rhs * P.hist_len, sizeof(double) * (k + 1),
                           hipMemcpyDeviceToHost, P.st));
    ETH_HIP(hipStreamSynchronize(P.st));
    double mu = 0.0;
    if (!eth::most_negative_pencil_eig(dl, gm, &mu))
      throw std::invalid_argument("no negative harmonic Ritz value yet");
    const double th = 1.0 / mu;
    *gamma2 = th * (th - 1.0);
    if (theta) *theta = th;
    if (steps) *steps = k;
    return ETH_OK;
  });
}

int eth_apply_pcd(eth_problem* p, int transpose, const double* r, double* z, int64_t batch,
                  int64_t ld) {
  if (!p || !r || !z) return fail(p, ETH_EINVAL, "NULL argument");
  if (!check_batch(p, batch, ld)) return fail(p, ETH_EINVAL, "invalid batch or ld");
  if (r == z) return fail(p, ETH_EINVAL, "r and z must not alias");
  if (!p->impl.oseen) return fail(p, ETH_EUNSUPPORTED, "PCD is built for Oseen problems only");
  return guarded(p, [&] {
    Problem& P = p->impl;
    eth::launch_copy(P.g.N, r, ld, P.kv[0], P.ldw, (int)batch, P.st);
    P.precond_oseen(transpose ? 4 : 2, P.kv[0], P.kz[0], (int)batch, eth::no_gate());
    eth::launch_copy(P.g.N, P.kz[0], P.ldw, z, ld, (int)batch, P.st);
    return ETH_OK;
  });
}

int eth_get_q1_levels(const eth_problem* p, int32_t* levels, double* lambdas) {
  if (!p) return ETH_EINVAL;
  const Problem& P = p->impl;
  const std::vector<eth::Geo>* lv = nullptr;
  const std::vector<double>* lam = nullptr;
  if (P.oseen) {
    lv = &P.qlv;
    lam = &P.qlam;
  } else if (!P.slv.empty()) {
    lv = &P.slv;
    lam = &P.slam;
  } else {
    return ETH_EUNSUPPORTED;
  }
  if (levels) *levels = (int32_t)lv->size();
  if (lambdas)
    for (size_t i = 0; i < lam->size(); ++i) lambdas[i] = (*lam)[i];
  return ETH_OK;
}

int eth_tuning_source(const eth_problem* p, int32_t* timed, int32_t* cached) {
  if (!p) return ETH_EINVAL;
  if (timed) *timed = p->impl.tuned_timed;
  if (cached) *cached = p->impl.tuned_cached;
  return ETH_OK;
}

int eth_get_mq_tile(const eth_problem* p, int32_t* tile_1, int32_t* tile_max, int32_t* steps_1,
                    int32_t* steps_max) {
  if (!p) return ETH_EINVAL;
  const Problem& P = p->impl;
  if (P.d.mq_mode != ETH_MQ_CHEB_SGS) return ETH_EUNSUPPORTED;
  if (tile_1) *tile_1 = P.mq_var_lo.tile;
  if (tile_max) *tile_max = P.mq_var_hi.tile;
  if (steps_1) *steps_1 = P.mq_var_lo.steps;
  if (steps_max) *steps_max = P.mq_var_hi.steps;
  return ETH_OK;
}

int eth_solve(eth_problem* p, const eth_solve_opts* opts, const double* b, double* x,
              int64_t batch, int64_t ld, eth_solve_info* info) {
  if (!p || !b || !x) return fail(p, ETH_EINVAL, "NULL argument");
  if (!check_batch(p, batch, ld)) return fail(p, ETH_EINVAL, "invalid batch or ld");
  if (b == x) return fail(p, ETH_EINVAL, "b and x must not alias");
  eth_solve_opts o{};
  if (opts) {
    o = *opts;
  } else {
    o.canonicalize = 1;
    o.method = p->impl.oseen ? ETH_TWO_STAGE : ETH_MINRES;
  }
  if (o.maxit > 4096) return fail(p, ETH_EINVAL, "maxit > 4096");
  if (o.residual_history && o.history_len < 1) return fail(p, ETH_EINVAL, "history_len must be >= 1");
  if (p->impl.oseen) {
    if (o.method != ETH_FGMRES && o.method != ETH_TWO_STAGE)
      return fail(p, ETH_EUNSUPPORTED, "Oseen systems are solved by FGMRES or TWO_STAGE");
  } else if (o.method != ETH_MINRES) {
    return fail(p, ETH_EUNSUPPORTED, "only MINRES is available for Stokes");
  }
  int bad = ETH_OK;
  const int rc = guarded(p, [&] {
    const std::vector<int> st = p->impl.check_rhs(b, ld, (int)batch, true);
    for (int r = 0; r < (int)batch; ++r) {
      if (st[r] != ETH_OK && (bad == ETH_OK || st[r] == ETH_EINVAL)) bad = st[r];
      if (info) info[r] = eth_solve_info{st[r], 0, 0, -1.0, -1.0};
    }
    return ETH_OK;
  });
  if (rc != ETH_OK) return rc;
  if (bad == ETH_EINVAL) return fail(p, ETH_EINVAL, "right-hand side holds a NaN or Inf");
  if (bad == ETH_EINCONSISTENT)
    return fail(p, ETH_EINCONSISTENT,
                "right-hand side not orthogonal to null(K^T): a pressure block of b does not sum to zero");
  if (p->impl.oseen) return guarded(p, [&] { return p->impl.solve_oseen(o, b, x, (int)batch, ld, info); });
  return guarded(p, [&] { return p->impl.solve_minres(o, b, x, (int)batch, ld, info); });
}

int eth_set_wind(eth_problem* p, const double* wind) {
  if (!p || !wind) return fail(p, ETH_EINVAL, "NULL argument");
  if (!p->impl.oseen) return fail(p, ETH_EUNSUPPORTED, "the problem has no wind (Stokes)");
  return guarded(p, [&] {
    Problem& P = p->impl;
    ETH_HIP(hipMemcpyAsync(P.wind0, wind, 2 * sizeof(double) * P.g.nv, hipMemcpyDeviceToDevice, P.st));
    P.refresh_wind();
    return ETH_OK;
  });
}

int eth_picard(eth_problem* p, const eth_solve_opts* opts, int32_t steps, const double* f_nodal,
               double* x, eth_solve_info* info) {
  if (!p || !x) return fail(p, ETH_EINVAL, "NULL argument");
  if (!p->impl.oseen) return fail(p, ETH_EUNSUPPORTED, "Picard steps need an Oseen problem");
  if (steps < 0) return fail(p, ETH_EINVAL, "steps must be >= 0");
  eth_solve_opts o{};
  if (opts) {
    o = *opts;
  } else {
    o.canonicalize = 1;
    o.method = ETH_TWO_STAGE;
  }
  if (o.maxit > 4096) return fail(p, ETH_EINVAL, "maxit > 4096");
  if (o.method != ETH_FGMRES && o.method != ETH_TWO_STAGE)
    return fail(p, ETH_EUNSUPPORTED, "Oseen systems are solved by FGMRES or TWO_STAGE");
  return guarded(p, [&] { return p->impl.picard(o, steps, f_nodal, x, info); });
}

int eth_profile_kernel(eth_problem* p, int kernel, int reps, int64_t batch, double* avg_ms,
                       double* bytes) {
  if (!p || !avg_ms || !bytes || reps < 1) return fail(p, ETH_EINVAL, "invalid argument");
  if (batch < 1 || batch > p->impl.max_batch) return fail(p, ETH_EINVAL, "invalid batch");
  return guarded(p, [&] {
    Problem& P = p->impl;
    const eth::Geo& g = P.g;
    const int B = (int)batch;
    const double N = (double)g.N;
    const double es = P.mixed ? 4.0 : 8.0;
    std::function<void()> launch;
    double by = 0.0;
    const eth::Gate gate = eth::no_gate();
    switch (kernel) {
      case ETH_K_SADDLE_APPLY: {
        launch = [&] {
          eth::RedCtx rd = P.red(eth::saddle_blocks(g), 1, eth::EPI_NONE, nullptr, P.red_result);
          eth::launch_apply_stokes(g, P.d.nu, P.kz[0], P.ky, P.ldw, B, gate, &rd, P.st);
        };
        by = 16.0 * N;
        break;
      }
      case ETH_K_CHEB_STEP:
      case ETH_K_RESTRICT:
      case ETH_K_PROLONG: {
        if (P.lv.size() < 2) throw std::runtime_error("unsupported:no multigrid hierarchy");
        const eth::Geo& gf = P.lv[0];
        const eth::Geo& gc = P.lv[1];
        const double vf = 2.0 * gf.nv, vc = 2.0 * gc.nv;
        if (kernel == ETH_K_CHEB_STEP) {
          launch = [&] {
            if (P.mixed)
              eth::launch_cheb_step<float>(gf, (float*)P.vb[0], (float*)P.vx[0], (float*)P.vxo[0],
                                           0.5, 0.1, 1, 2 * B, nullptr, 0, 0.0, gate, B, P.st);
            else
              eth::launch_cheb_step<double>(gf, (double*)P.vb[0], (double*)P.vx[0],
                                            (double*)P.vxo[0], 0.5, 0.1, 1, 2 * B, nullptr, 0, 0.0,
                                            gate, B, P.st);
          };
          by = 4.0 * es * vf;   // read b, x, x_prev; write x_new
        } else if (kernel == ETH_K_RESTRICT) {
          launch = [&] {
            if (P.mixed)
              eth::launch_restrict<float>(gf, gc, (float*)P.vb[0], (float*)P.vx[0],
                                          (float*)P.vb[1], (float*)P.vxo[1], 0.1, 2 * B, B, gate, P.st);
            else
              eth::launch_restrict<double>(gf, gc, (double*)P.vb[0], (double*)P.vx[0],
                                           (double*)P.vb[1], (double*)P.vxo[1], 0.1, 2 * B, B, gate,
                                           P.st);
          };
          by = 2.0 * es * vf + 2.0 * es * vc;
        } else {
          launch = [&] {
            if (P.mixed)
              eth::launch_prolong_add<float>(gf, gc, (float*)P.vx[1], (float*)P.vxo[0], 2 * B, B,
                                             gate, P.st);
            else
              eth::launch_prolong_add<double>(gf, gc, (double*)P.vx[1], (double*)P.vxo[0], 2 * B,
                                              B, gate, P.st);
          };
          by = es * vc + 2.0 * es * vf;
        }
        by *= B;
        break;
      }
      case ETH_K_MQ_CHEB_STEP: {
        if (!P.mq_r) throw std::runtime_error("unsupported:no Chebyshev-SGS workspace");
        const Problem::MqVariant v = P.mq_variant_for(B);
        launch = [&, v] {
          if (P.mixed)
            eth::launch_mq_cheb_fused<float>(g, (float*)P.mq_r, (float*)P.mq_z, (float*)P.mq_t,
                                             (float*)P.mq_d, v.steps == 2 ? (float*)P.mq_d2 : (float*)P.mq_d,
                                             0.5, 0.1, 0.5, 0.1, v.steps, 0, B, gate, P.st, v.tile);
          else
            eth::launch_mq_cheb_fused<double>(g, (double*)P.mq_r, (double*)P.mq_z, (double*)P.mq_t,
                                              (double*)P.mq_d,
                                              v.steps == 2 ? (double*)P.mq_d2 : (double*)P.mq_d, 0.5, 0.1,
                                              0.5, 0.1, v.steps, 0, B, gate, P.st, v.tile);
        };
        // one launch (of v.steps Chebyshev steps): read r, z_k, d; write
        // z_{k+v.steps}, d (pressure vectors of n_k + n_0)
        by = 5.0 * es * (g.nk + g.n0) * B;
        break;
      }
      case ETH_K_DOT: {
        launch = [&] {
          eth::RedCtx rc = P.red(eth::dot_blocks(g.N), 1, eth::EPI_NONE, nullptr, P.red_result);
          eth::launch_dot(g.N, P.kz[0], P.kv[0], P.ldw, B, rc, gate, P.st);
        };
        by = 16.0 * N * B;
        break;
      }
      case ETH_K_MINRES_V: {
        launch = [&] {
          eth::launch_minres_v(g.N, P.ky, P.kv[0], P.kw[0], P.ldw, B, P.d_ms, P.st);
        };
        by = 32.0 * N * B;
        break;
      }
      case ETH_K_MINRES_WX: {
        launch = [&] {
          eth::launch_minres_wx(g.N, P.kz[0], P.kw[0], P.kw[1], P.ky, P.ldw, B, P.d_ms, P.st);
        };
        by = 48.0 * N * B;
        break;
      }
      case ETH_K_OSEEN_APPLY: {
        if (!P.oseen) throw std::runtime_error("unsupported:not an Oseen problem");
        launch = [&] {
          eth::RedCtx rd = P.red(eth::saddle_blocks(g), 1, eth::EPI_NONE, nullptr, P.red_result);
          eth::launch_apply_oseen(g, P.d.nu, P.d.wind, 0, P.kz[0], P.ky, P.ldw, B, gate, &rd, P.st);
        };
        by = 16.0 * N * B + 16.0 * g.nv;   // x read, y written; the wind (2 planes) once
        break;
      }
      case ETH_K_CD_STEP: {
        if (!P.oseen || P.lv.empty()) throw std::runtime_error("unsupported:not an Oseen problem");
        const eth::Geo& gf = P.lv[0];
        launch = [&] {
          if (P.mixed)
            eth::launch_cd_step<float>(gf, P.level_wind<float>(0), P.ldF[0], P.lnu[0], (float*)P.vb[0], (float*)P.vx[0],
                                       (float*)P.vxo[0], P.d.gmg_omega, 0, 2 * B, nullptr, 0, 0.0, gate,
                                       P.st);
          else
            eth::launch_cd_step<double>(gf, P.lwind[0], P.ldF[0], P.lnu[0], (double*)P.vb[0],
                                        (double*)P.vx[0], (double*)P.vxo[0], P.d.gmg_omega, 0, 2 * B,
                                        nullptr, 0, 0.0, gate, P.st);
        };
        // per plane: read b, x, write x_new; the wind (2 planes, in the storage
        // type) and diag(F) (FP64) once
        by = 2.0 * B * 3.0 * es * gf.nv + (2.0 * es + 8.0) * gf.nv;
        break;
      }
      case ETH_K_GM_MDOT:
      case ETH_K_GM_MAXPY: {
        if (!P.oseen) throw std::runtime_error("unsupported:not an Oseen problem");
        const int nvec = std::max(1, P.gm_m / 2);   // the average Arnoldi position of a cycle
        const size_t per = (size_t)(P.gm_m + 1) * P.gm_m + 7 * 64;
        for (int r = 0; r < B; ++r) {
          eth::GmresScalars& G = P.h_gm[r];
          std::memset(&G, 0, sizeof(G));
          G.active = 1;
          G.m = P.gm_m;
          double* base = P.gArr + per * r;
          G.H = base;
          G.cs = base + (size_t)(P.gm_m + 1) * P.gm_m;
          G.sn = G.cs + 64;
          G.g = G.sn + 64;
          G.y = G.g + 64;
          G.h1 = G.y + 64;
          G.h2 = G.h1 + 64;
        }
        ETH_HIP(hipMemcpyAsync(P.d_gm, P.h_gm, sizeof(eth::GmresScalars) * B, hipMemcpyHostToDevice, P.st));
        ETH_HIP(hipMemsetAsync(P.gV, 0, sizeof(double) * P.ldw * B * (nvec + 1), P.st));
        double* w = P.gV + (size_t)nvec * B * P.ldw;
        if (kernel == ETH_K_GM_MDOT) {
          launch = [&, nvec, w] {
            eth::launch_gm_mdot(g.N, nvec, P.gV, w, P.ldw, B, P.gpart, P.d_gm, 0, P.st);
          };
          by = 8.0 * N * B * (nvec + 1);
        } else {
          eth::launch_gm_mdot(g.N, nvec, P.gV, w, P.ldw, B, P.gpart, P.d_gm, 0, P.st);
          launch = [&, nvec, w] { eth::launch_gm_maxpy(g.N, nvec, P.gV, w, P.ldw, B, P.d_gm, 0, P.st); };
          by = 8.0 * N * B * (nvec + 2);
        }
        break;
      }
      case ETH_K_COPY: {
        launch = [&] { eth::launch_copy(g.N, P.kz[0], P.ldw, P.kz[1], P.ldw, B, P.st); };
        by = 16.0 * N * B;   // read + write of N doubles per RHS: the calibration of byte counters
        break;
      }
      case ETH_K_SYNC_GRAPH:
      case ETH_K_SYNC_GRID: {
        // persistent kernel vs kernel boundaries: per step of a ring
        // dependency across one block per CU
        const int nb = eth::sync_probe_blocks();
        if ((long long)nb * 512 > P.ldw) throw std::invalid_argument("problem too small for the sync probe");
        double* buf = P.kz[1];
        ETH_HIP(hipMemsetAsync(buf, 0, sizeof(double) * 512 * nb, P.st));
        hipEvent_t e0, e1;
        ETH_HIP(hipEventCreate(&e0));
        ETH_HIP(hipEventCreate(&e1));
        float ms = 0.0f;
        if (kernel == ETH_K_SYNC_GRID) {
          eth::launch_grid_sync_rounds(buf, 4, P.st);   // warm-up
          ETH_HIP(hipEventRecord(e0, P.st));
          eth::launch_grid_sync_rounds(buf, reps, P.st);
          ETH_HIP(hipEventRecord(e1, P.st));
        } else {
          hipGraph_t graph;
          hipGraphExec_t exec;
          hipStream_t cs;
          ETH_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
          ETH_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
          for (int i = 0; i < reps; ++i) eth::launch_sync_step(buf, i, cs);
          ETH_HIP(hipStreamEndCapture(cs, &graph));
          ETH_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
          ETH_HIP(hipGraphLaunch(exec, P.st));   // warm-up
          ETH_HIP(hipEventRecord(e0, P.st));
          ETH_HIP(hipGraphLaunch(exec, P.st));
          ETH_HIP(hipEventRecord(e1, P.st));
          ETH_HIP(hipEventSynchronize(e1));
          ETH_HIP(hipGraphExecDestroy(exec));
          ETH_HIP(hipGraphDestroy(graph));
          ETH_HIP(hipStreamDestroy(cs));
        }
        ETH_HIP(hipEventSynchronize(e1));
        ETH_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *avg_ms = (double)ms / reps;
        *bytes = 16.0 * 256 * nb;
        return ETH_OK;
      }
      default:
        throw std::invalid_argument("unknown kernel id");
    }
    if (kernel == ETH_K_SADDLE_APPLY) by *= B;
    // keep the update kernels active (their gates read the MINRES flags)
    for (int r = 0; r < B; ++r) {
      P.h_ms[r].active = 1;
      P.h_ms[r].wx_todo = 1;
      P.h_ms[r].vy = 1.0;
    }
    ETH_HIP(hipMemcpyAsync(P.d_ms, P.h_ms, sizeof(eth::MinresScalars) * B, hipMemcpyHostToDevice, P.st));
    hipEvent_t e0, e1;
    ETH_HIP(hipEventCreate(&e0));
    ETH_HIP(hipEventCreate(&e1));
    launch();   // warm-up
    ETH_HIP(hipEventRecord(e0, P.st));
    for (int i = 0; i < reps; ++i) launch();
    ETH_HIP(hipEventRecord(e1, P.st));
    ETH_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    ETH_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
    *bytes = by;
    return ETH_OK;
  });
}

const char* eth_status_string(int status) {
  switch (status) {
    case ETH_OK: return "ok";
    case ETH_EINVAL: return "invalid argument";
    case ETH_EDEVICE: return "HIP runtime error";
    case ETH_ENOMEM: return "out of device memory";
    case ETH_EINCONSISTENT: return "inconsistent right-hand side";
    case ETH_EBREAKDOWN: return "Krylov breakdown";
    case ETH_EUNSUPPORTED: return "unsupported option";
    case ETH_WMAXIT: return "iteration limit reached";
    case ETH_WNOPROGRESS: return "no progress: the initial guess is returned";
    default: return "unknown status";
  }
}

const char* eth_last_error(const eth_problem* p) {
  return p ? p->impl.err.c_str() : eth::g_setup_error.c_str();
}

}  // extern "C"
