// Host launchers of the HIP kernels (one declaration per kernel family).
#pragma once
#include "eth_epilogue.h"
#include "eth_internal.h"

namespace eth {

// Per right-hand-side gate: a kernel skips RHS r when p && p[r*stride] == 0.
struct Gate {
  const int* p;
  int stride;  // in ints
  __device__ bool off(int r) const { return p && p[(long long)r * stride] == 0; }
};
inline Gate no_gate() { return Gate{nullptr, 0}; }

// Per right-hand-side flag cleared (set to 0) by block (0,0,r) of a kernel
// before anything else; used to retire the pending MINRES w/x update.
struct ClearFlag {
  int* p;
  int stride;  // in ints
  // for grids whose right-hand side r is blockIdx.z
  __device__ void apply(int r) const {
    if (p && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && threadIdx.y == 0)
      p[(long long)r * stride] = 0;
  }
};
inline ClearFlag no_clear() { return ClearFlag{nullptr, 0}; }

// ---------------- saddle-point operator (k_saddle.hip) ----------------------
// y = K x on the full layout, FP64.  mode 0: boundary velocity inputs are
// masked, boundary rows of y are 0.  Optional fused reduction of <y, x>.
int saddle_blocks(const Geo& g);
// node-parallel apply (k_apply.hip): wind == nullptr for Stokes; blocks per RHS
int apply_blocks(const Geo& g);
void launch_apply(const Geo& g, double nu, const double* wind, int transpose, const double* x, double* y,
                  long long ld, int batch, Gate gate, const RedCtx* dot, hipStream_t st,
                  ClearFlag clear = no_clear());
void launch_apply_stokes(const Geo& g, double nu, const double* x, double* y, long long ld,
                         int batch, Gate gate, const RedCtx* dot, hipStream_t st,
                         ClearFlag clear = no_clear());
// Oseen: y = [nu A + N(w)] u + B^T p, B u  (transpose: N -> N^T)
void launch_apply_oseen(const Geo& g, double nu, const double* wind, int transpose,
                        const double* x, double* y, long long ld, int batch, Gate gate,
                        const RedCtx* dot, hipStream_t st, ClearFlag clear = no_clear());
// b = lifted RHS: interior rows (M_v f)_I - (F u_B)_I, pressure rows -B u_B,
// boundary rows u_B.  ub: full-length velocity Dirichlet vector (2 nv).
void launch_lift_rhs(const Geo& g, double nu, const double* wind, const double* ub,
                     const double* f, long long ldf, double* b, long long ld, int batch,
                     hipStream_t st);
void launch_dirichlet_lid(const Geo& g, double lid_u, int corner_mode, double* ub,
                          hipStream_t st);

// ---------------- vector kernels (k_vector.hip) ------------------------------
// Second stage of a reduction (eth_reduce.h): totals of the block partials in
// block order, result and epilogue; nothing to do for a single block.  Every
// launcher of a reducing kernel calls it right after the kernel.
void launch_reduce_finish(const RedCtx& rc, int batch, Gate gate, hipStream_t st);
// (clear: a flag reset by the first block before the gate is read)
void launch_dot(long long n, const double* x, const double* y, long long ld, int batch,
                const RedCtx& rc, Gate gate, hipStream_t st, ClearFlag clear = no_clear());
// flag of every right-hand side = 0 (one small launch)
void launch_clear_flag(const ClearFlag& f, int batch, hipStream_t st);
int dot_blocks(long long n);
// y = a*x + b*y on [0,n)
void launch_axpby(long long n, double a, const double* x, double b, double* y, long long ld,
                  int batch, hipStream_t st);
void launch_copy(long long n, const double* x, long long ldx, double* y, long long ldy,
                 int batch, hipStream_t st);
void launch_fill(long long n, double v, double* y, long long ld, int batch, hipStream_t st);
// y *= d pointwise on [0,n) (one vector)
void launch_vmul(long long n, const double* d, double* y, hipStream_t st);
// zero the boundary velocity rows of a full-layout vector
void launch_zero_boundary(const Geo& g, double* y, long long ld, int batch, hipStream_t st);
// x boundary rows <- b boundary rows
void launch_copy_boundary(const Geo& g, const double* b, double* x, long long ld, int batch,
                          hipStream_t st);
// MINRES vector updates
// partials (may be null): nb > 1 block partials of <K zhat_j, zhat_j> whose
// finishing launch was deferred (RedCtx.defer); summed here with the delta
// epilogue
// wx (z null: none): the previous iteration's w/x update made in the same
// pass while its wx_todo flag is set (see launch_minres_wx)
struct MinresWx {
  const double* z = nullptr;
  double* wprev_io = nullptr;
  const double* w = nullptr;
  double* x = nullptr;
};
void launch_minres_v(long long n, const double* y, const double* v, double* vprev_io,
                     long long ld, int batch, MinresScalars* s, hipStream_t st,
                     const double* partials = nullptr, int nb = 0, MinresWx wx = MinresWx{});
void launch_minres_wx(long long n, const double* z, double* wprev_io, const double* w,
                      double* x, long long ld, int batch, const MinresScalars* s, hipStream_t st);
// v = b - y with boundary rows zeroed (initial residual)
void launch_residual_init(const Geo& g, const double* b, const double* y, double* v,
                          long long ld, int batch, hipStream_t st);
// pressure block sums (p_k, p_0) per RHS -> out[2*rhs + {0,1}]
void launch_pressure_sums(const Geo& g, const double* x, long long ld, int batch,
                          double* partials, double* out, hipStream_t st);
void launch_pressure_shift(const Geo& g, double* x, long long ld, int batch,
                           const double* sums, hipStream_t st);

// ---------------- geometric multigrid (k_gmg.hip) ---------------------------
// Scalar Q2 Laplacian planes: [batch][2 components][nq*nq], boundary zero.
template <typename T>
// has_prev: 0 none (alpha ignored), 1 x_prev in xo, 2 x_prev = 0
void launch_cheb_step(const Geo& g, const T* b, const T* x, T* xnew_io_prev, double alpha,
                      double beta, int has_prev, int nplanes, double* out64, long long ld64,
                      double out_scale, Gate gate, int batch, hipStream_t st);
// b = r_u - sub_u (sub may be null), x = beta D^{-1} b (Laplacian diagonal)
template <typename T>
void launch_vcycle_entry(const Geo& g, const double* r, long long ld, T* b, T* x,
                         double beta, int batch, Gate gate, hipStream_t st,
                         const double* sub = nullptr);
// xf == nullptr: bf already holds the fine residual
template <typename T>
void launch_restrict(const Geo& gf, const Geo& gc, const T* bf, const T* xf, T* bc, T* xc,
                     double beta_c, int nplanes, int batch, Gate gate, hipStream_t st);
template <typename T>
void launch_prolong_add(const Geo& gf, const Geo& gc, const T* xc, T* xf, int nplanes,
                        int batch, Gate gate, hipStream_t st);
// the second pre-smoothing step (has_prev 2, from x1 to x2, written to x2out
// on the fine nodes) fused with the restriction of the residual of x2
template <typename T>
void launch_restrict_pre(const Geo& gf, const Geo& gc, const T* bf, const T* x1, T* x2out, double alpha,
                         double beta, T* bc, T* xc, double beta_c, int nplanes, Gate gate, hipStream_t st);
// x0 = xold + P xc, then two Chebyshev steps (beta0; alpha1, beta1), result
// to xout (or out64 times out_scale)
template <typename T>
void launch_post2(const Geo& gf, const Geo& gc, const T* b, const T* xold, const T* xc, T* xout, double alpha1,
                  double beta0, double beta1, int nplanes, double* out64, long long ld64, double out_scale,
                  Gate gate, hipStream_t st);
// dense coarse solve: x = Ainv * b on the interior nodes of each plane, with
// the FP32 copy AinvF of the inverse when given; gbuf: 2*ni*batch doubles
template <typename T>
void launch_dense_solve(const Geo& g, const double* Ainv, const float* AinvF, int ni, const T* b,
                        T* x, int nplanes, double* out64, long long ld64, double out_scale,
                        const double* in64, long long ldin, double* gbuf, int batch, Gate gate,
                        hipStream_t st);
// the coarse end of a V-cycle in one launch (levels with at most 65^2 nodes,
// one block of 1024 threads per plane, all levels in LDS): tl.n[0] is the level
// whose b (restricted residual) and x (first Chebyshev step) are given in
// b0/x0; x0 receives the level's corrected iterate after post-smoothing
constexpr int kTailMaxLevels = 8;
struct TailLevels {
  int nlev;                          // levels in the tail, the last one solved densely
  int deg;                           // Chebyshev degree per side
  int n[kTailMaxLevels];             // elements per side of each level
  double ca[kTailMaxLevels][4], cb[kTailMaxLevels][4];   // Chebyshev coefficients
};
size_t vcycle_tail_lds(const TailLevels& tl, size_t elem);
template <typename T>
void launch_vcycle_tail(const TailLevels& tl, const double* Ainv, int ni, const T* b0, T* x0, int nplanes,
                        Gate gate, hipStream_t st);
template <typename T>
hipError_t prepare_vcycle_tail(size_t lds);   // allows the dynamic LDS size
// dense Laplacian of the interior nodes, and Gauss-Jordan inverse helpers
void launch_dense_laplacian(const Geo& g, double* A, int ni, hipStream_t st);
// setup helpers on one FP64 plane: mode 0: y = A x, mode 1: y = D^{-1} x
// (interior nodes; boundary 0)
void launch_plane_op(const Geo& g, int mode, const double* x, double* y, hipStream_t st);

// ---------------- pressure-mass solves (k_mq.hip) ----------------------------
// z = nu * bordered diag solve of r (pressure part of full-layout vectors)
void launch_mq_diag_dot(const Geo& g, const double* r, long long ld, int batch,
                        const RedCtx& rc, Gate gate, hipStream_t st);
void launch_mq_diag_apply(const Geo& g, const double* r, double* z, long long ld, int batch,
                          const double* lam, double scale, Gate gate, hipStream_t st);
// Chebyshev-SGS pieces on pressure vectors [batch][np] in T (np = nk + n0)
template <typename T>
void launch_mq_kdot(const Geo& g, const T* x, long long ldx, long long off, int batch,
                    const RedCtx& rc, Gate gate, hipStream_t st);
template <typename T>
void launch_mq_project_in(const Geo& g, const double* r, long long ld, T* rt, T* z, T* t, T* d,
                          int batch, const double* coef, Gate gate, hipStream_t st);
template <typename T>
void launch_mq_colour(const Geo& g, const T* r, T* t, int colour, int batch, Gate gate,
                      hipStream_t st);
template <typename T>
void launch_mq_cheb_combine(const Geo& g, T* t, T* z, T* d, double a, double b, int first,
                            int batch, Gate gate, hipStream_t st);
// one fused Chebyshev step (symmetric multicolour SGS sweep from zin + combine)
// on tiles of tile x tile Q1 nodes (16, 24, 32; 64 in FP32 only), or two steps
// (steps = 2, coefficients a, b then a2, b2; tile 16 or 24, din != dout).  src (first
// step, optional): r comes from the FP64 vectors projected by coef and is
// stored to the workspace r.  sink (last step, optional): the result goes,
// times scale, to the pressure part of FP64 vectors (zout and d untouched).
struct MqSource {
  const double* r;     // full FP64 vectors (pressure part at off_pk), null: none
  long long ld;
  const double* coef;  // [batch] coefficient of k removed from r, null: none
};
struct MqSink {
  double* out;         // full FP64 vectors (pressure part at off_pk), null: none
  long long ld;
  double scale;
};
template <typename T>
void launch_mq_cheb_fused(const Geo& g, T* r, const T* zin, T* zout, const T* din, T* dout, double a,
                          double b, double a2, double b2, int steps, int first, int batch, Gate gate,
                          hipStream_t st, int tile, const MqSource* src = nullptr,
                          const MqSink* sink = nullptr);
template <typename T>
void launch_mq_project_out(const Geo& g, const T* z, double* out, long long ld, int batch,
                           const double* coef, double scale, Gate gate, hipStream_t st);

// ---------------- Oseen preconditioner pieces (k_oseen.hip) ------------------
void launch_inject_wind(const Geo& gf, const Geo& gc, const double* wf, double* wc, hipStream_t st);
void launch_cd_diag(const Geo& g, const double* wind, double nu, double* dF, hipStream_t st);
// y = F_0 (scale x) on the n^2 elements (jump-based P0 convection-diffusion)
void launch_p0_cd_apply(const Geo& g, const double* wind, double nu, const double* x, double scale, double* y,
                        hipStream_t st);
// velocity part of a full vector times diag(M_v)^{-1} (interior nodes, else
// 0), pressure part zeroed
void launch_vel_minv(const Geo& g, double* x, hipStream_t st);
// synchronisation probes (one block of 256 threads per CU; buf >= 512 * CUs
// doubles): one step of a ring dependency per launch, or `rounds` steps in
// one cooperative launch separated by grid-wide barriers (one per step)
int sync_probe_blocks();
void launch_sync_step(double* buf, int round, hipStream_t st);
void launch_grid_sync_rounds(double* buf, int rounds, hipStream_t st);
// *out = max over the Q2 nodes of |w| (device scalar)
void launch_wind_speed_max(const Geo& g, const double* wind, double* out, hipStream_t st);
// the coarse F as a dense row-major ni x ni matrix (A zero on entry)
void launch_dense_convdiff(const Geo& g, const double* wind, double nu, double* A, int ni,
                           hipStream_t st);
// in-place inverse of a dense row-major matrix whose leading principal blocks
// are nonsingular (blocked Gauss-Jordan, no pivoting); work holds
// dense_inverse_work(ni) doubles (k_dense.hip)
size_t dense_inverse_work(int ni);
void launch_dense_inverse(double* A, int ni, double* work, hipStream_t st);
// A = (A + A^T) / 2 in place (the inverse of a symmetric matrix, against rounding)
void launch_symmetrize(double* A, int ni, hipStream_t st);
// f = (float)a, n values
void launch_to_float(const double* a, float* f, long long n, hipStream_t st);
// damped Jacobi step on F = nu A + N(w) (residual != 0: write b - F x instead;
// transpose != 0: F^T)
template <typename T>
void launch_cd_step(const Geo& g, const T* wind, const double* dF, double nu, const T* b,
                    const T* x, T* out, double omega, int residual, int nplanes, double* out64,
                    long long ld64, double out_scale, Gate gate, hipStream_t st, int transpose = 0);
// at = a^T for a dense ni x ni matrix
void launch_transpose(const double* a, int ni, double* at, hipStream_t st);
// the A_p multigrid from a level with n <= 32 down to the coarsest and back in
// one launch per RHS (levels, element sizes, diag(A_p) per level, Chebyshev
// coefficients per level and step, the coarsest bordered inverse)
constexpr int APT_L = 8;
struct ApTail {
  int nlev, deg, ni;
  int n[APT_L];
  int off[APT_L + 1];   // offset of each level's values in the kernel's LDS arrays
  double h[APT_L];
  const double* dAp[APT_L];
  double ca[APT_L][4], cb[APT_L][4];
  const double* Ainv;
};
template <typename T>
void launch_ap_tail(const ApTail& tl, const T* b0, T* x0, int batch, Gate gate, hipStream_t st);
// the whole Chebyshev-Jacobi solve for Q_1 in one launch (steps <= 12): x_1 =
// b[0] D^{-1} b, then x_{k+1} = x_k + a[k] (x_k - x_{k-1}) + b[k] D^{-1}(b - Q_1 x_k)
struct Q1Cheb {
  double a[12], b[12];
  int steps;
};
template <typename T>
void launch_q1mass_cheb_fused(const Geo& g, const T* b, T* out, const Q1Cheb& cc, int batch, Gate gate,
                              hipStream_t st);
template <typename T>
void launch_q1mass_cheb(const Geo& g, const T* b, const T* x, T* xo, double alpha, double beta,
                        int has_prev, int batch, Gate gate, hipStream_t st);
template <typename T>
void launch_f1_apply(const Geo& g, const double* wind, double nu, const T* x, T* y, int batch,
                     Gate gate, hipStream_t st, int transpose = 0);
// mode 0: out = A_p x; 1: Chebyshev step over out; 2: out = b - A_p x
template <typename T>
void launch_ap_op(const Geo& g, int mode, const T* b, const T* x, T* out, double alpha, double beta,
                  int has_prev, const double* dAp, int batch, Gate gate, hipStream_t st);
void launch_ap_diag(const Geo& g, double* dAp, hipStream_t st);
template <typename T>
void launch_q1_restrict(const Geo& gf, const Geo& gc, const T* rf, T* bc, T* xc, int batch, Gate gate,
                        hipStream_t st);
template <typename T>
void launch_q1_prolong_add(const Geo& gf, const Geo& gc, const T* xc, T* xf, int batch, Gate gate,
                           hipStream_t st);
template <typename T>
void launch_q1_sum(const Geo& g, const T* x, const RedCtx& rc, int batch, Gate gate, hipStream_t st);
// out = scale * (x - sums/nk) on Q1 vectors (strides/offsets select full-layout p_k parts)
template <typename TI, typename TO>
void launch_q1_shift(const Geo& g, const TI* x, long long ldx, long long offx, TO* out, long long ldo,
                     long long offo, const double* sums, double scale, int batch, Gate gate,
                     hipStream_t st);
void launch_unit_columns(double* cols, int ni, hipStream_t st);
void launch_dense_sym_shift(const double* cols, int ni, double shift, double* A, hipStream_t st);
template <typename T>
void launch_q1_dense_solve(const double* Ainv, int ni, const T* b, T* x, int batch, Gate gate,
                           hipStream_t st);

// ---------------- adjoint (k_adjoint.hip) -------------------------------------
// blocks of one RHS in the adjoint reductions (partials needed per value)
int adjoint_blocks(const Geo& g);
// e = x - xt (xt may be null; boundary nodes of e zeroed when mask_boundary),
// y = M_v e on all 2 nv velocity nodes (y may be null), and, with
// half_energy, result[rhs] = e^T M_v e / 2
void launch_velocity_mass(const Geo& g, const double* x, long long ldx, const double* xt, long long ldt,
                          int mask_boundary, double* y, long long ldy, const RedCtx* half_energy, int batch,
                          hipStream_t st);
// result[rhs] = -lambda_u^T (A u)_I with u the full velocity of x
void launch_grad_viscosity(const Geo& g, const double* lam, long long ldl, const double* x, long long ldx,
                           const RedCtx& rc, int batch, hipStream_t st);

// ---------------- M_Q by P0 elimination (k_schur.hip) --------------------------
// S_k on Q1 vectors [batch][nk] of a level, scaled by h2 (the finest h^2):
// mode 0: out = S x; 1: Chebyshev-Jacobi step over out; 2: out = b - S x
template <typename T>
void launch_sk_op(const Geo& g, double h2, int mode, const T* b, const T* x, T* out, double alpha, double beta,
                  int has_prev, int batch, Gate gate, hipStream_t st);
void launch_sk_diag_inv(const Geo& g, double h2, double* dinv, hipStream_t st);
// b = r_k - R^T Q_0^{-1} r_0 and x = 0 (r: projected pressure vectors)
template <typename T>
void launch_schur_rhs(const Geo& g, const T* r, T* bq, T* xq, int batch, Gate gate, hipStream_t st);
// z = [z_k; Q_0^{-1}(r_0 - R z_k)]
template <typename T>
void launch_schur_p0(const Geo& g, const T* r, const T* zk, T* z, int batch, Gate gate, hipStream_t st);

// ---------------- FGMRES (k_gmres.hip) ----------------------------------------
int gmres_blocks(long long N);
// partials: 64 * gmres_blocks(N) doubles per RHS.  Each reduction is a
// partial-sum kernel followed by a one-block-per-RHS finish kernel.
void launch_gm_mdot(long long N, int nv, const double* V, const double* w, long long ld, int batch,
                    double* partials, GmresScalars* S, int which, hipStream_t st);
void launch_gm_maxpy(long long N, int nv, const double* V, double* w, long long ld, int batch,
                     const GmresScalars* S, int which, hipStream_t st);
void launch_gm_norm_givens(long long N, int j, const double* w, long long ld, int batch, double* partials,
                           GmresScalars* S, hipStream_t st);
void launch_gm_scale(long long N, double* v, long long ld, int batch, const GmresScalars* S, hipStream_t st);
void launch_gm_beta(long long N, const double* v, long long ld, int batch, double* partials, GmresScalars* S,
                    hipStream_t st);
void launch_gm_finish(long long N, const double* Z, double* x, long long ld, int batch, GmresScalars* S,
                      hipStream_t st);
void launch_gm_zero_range(double* x, long long ld, long long off, long long count, int batch,
                          const GmresScalars* S, hipStream_t st);

}  // namespace eth
