// Flow over a step (Sec. 3, the inflow-outflow example): host-side mesh and
// assembly, and the device operators built from it.
//
// The domain is [-1, 0) x [0, 1] union [0, L] x [-1, 1] (or the channel
// [-1, L] x [0, 1]), divided into squares of side h = 1/m.  Unknowns are
// numbered over the nodes of the bounding box that belong to an element, row
// by row (y outer, x inner): the state vector is
//     [u_x (n_v) | u_y (n_v) | p_1 on the Q1 nodes (n_k) | p_0 per element (n_0)].
// Unlike the enclosed cavity, the geometry is not a single square, so the
// operators are assembled once on the host (per wind) and applied on the GPU
// as sliced-ELL sparse matrices; every Krylov iteration runs in kernels.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "eth_internal.h"

namespace eth {

// ---------------------------------------------------------------- host mesh
struct StepMesh {
  int m = 0, L = 0;
  bool channel = false;
  double h = 0.0, x0 = -1.0, y0 = -1.0;
  int ex = 0, ey = 0;         // elements of the bounding box along x, y
  int nqx = 0, nqy = 0;       // Q2 half-grid nodes of the bounding box
  std::vector<char> elem_act; // [ey][ex]
  std::vector<int> q2_index;  // [nqy][nqx] -> compact Q2 node or -1
  std::vector<int> q1_index;  // [ey+1][ex+1] -> compact Q1 node or -1
  std::vector<int> el_index;  // [ey][ex] -> compact element or -1
  std::vector<int> q2_I, q2_J, q1_I, q1_J, el_x, el_y;   // compact -> grid
  std::vector<char> dirichlet; // per compact Q2 node: wall or inflow
  int nv = 0, nk = 0, n0 = 0;
  long long N() const { return 2LL * nv + nk + n0; }
  void build(int m_, int L_, bool channel_);
  int q2(int I, int J) const { return (I < 0 || J < 0 || I >= nqx || J >= nqy) ? -1 : q2_index[(size_t)J * nqx + I]; }
  int q1(int I, int J) const {
    return (I < 0 || J < 0 || I > ex || J > ey) ? -1 : q1_index[(size_t)J * (ex + 1) + I];
  }
  bool active(int e, int f) const { return e >= 0 && f >= 0 && e < ex && f < ey && elem_act[(size_t)f * ex + e]; }
};

// Element matrices of an element of side h (Gauss quadrature, exact).
struct StepElem {
  double A[9][9], M[9][9], B1x[4][9], B1y[4][9], B0x[9], B0y[9], Qk[4][4], R[4], Q0, Kp[4][4];
  double Cx[9][9][9], Cy[9][9][9];      // N_T[i][j] = sum_m Cx[i][j][m] w_x,m + Cy w_y,m
  double Cpx[4][4][9], Cpy[4][4][9];    // the same for Q1 test / trial functions
  void build(double h);
};

// compressed sparse rows (host)
struct Csr {
  int rows = 0, cols = 0;
  std::vector<int> ptr, col;
  std::vector<double> val;
  double diag(int r) const;
};

// Row-by-row builder: every row keeps a short unsorted list of (column, value).
struct RowBuilder {
  int rows = 0, cols = 0;
  std::vector<std::vector<std::pair<int, double>>> r;
  RowBuilder(int nr, int nc) : rows(nr), cols(nc), r(nr) {}
  void add(int i, int j, double v);
  Csr finish(bool drop_zeros = false) const;
};

// Host assembly entry points (eth_step_asm.hip)
Csr step_assemble_F(const StepMesh& mesh, const StepElem& E, double nu, const double* wind, bool embed);
Csr step_assemble_B(const StepMesh& mesh, const StepElem& E);          // n_p x 2 n_v (all velocity columns)
Csr step_assemble_K(const StepMesh& mesh, const Csr& F, const Csr& B);  // N x N, Dirichlet rows / cols empty
Csr step_assemble_MQ(const StepMesh& mesh, const StepElem& E);
Csr step_assemble_Q1(const StepMesh& mesh, const StepElem& E);
Csr step_assemble_F1(const StepMesh& mesh, const StepElem& E, double nu, const double* wind, bool robin);
Csr step_assemble_Ap(const StepMesh& mesh, const StepElem& E, const Csr& B);
std::vector<double> step_velocity_mass_diag(const StepMesh& mesh, const StepElem& E);
Csr step_q2_prolongation(const StepMesh& fine, const StepMesh& coarse);
Csr step_q1_prolongation(const StepMesh& fine, const StepMesh& coarse);
Csr csr_transpose(const Csr& A);
std::vector<double> step_inject_wind(const std::vector<double>& w, const StepMesh& fine, const StepMesh& coarse);
std::vector<double> step_inflow(const StepMesh& mesh);   // 2 n_v Dirichlet vector
// lifted right-hand side: free rows -F u_B (both components), pressure rows
// -B u_B, Dirichlet rows u_B
std::vector<double> step_lift(const StepMesh& mesh, const Csr& Ffull, const Csr& B, const std::vector<double>& uB);
// sliced-ELL arrays of A (64 rows per slice, column-major in a slice, padding
// repeats a row's last column with value 0): slice offsets, columns, values
void sell_layout(const Csr& A, std::vector<int>& ptr, std::vector<int>& col, std::vector<double>& val);
// inverse of a small dense matrix (row-major), Gauss-Jordan with partial pivoting
std::vector<double> dense_inverse(const Csr& A);
// largest eigenvalue of D^{-1} A for symmetric positive definite A (Lanczos)
double lambda_max_dinv(const Csr& A, int steps = 60);

// --------------------------------------------------------------- device side
struct Sell {                 // sliced ELL: 64 rows per slice, column-major in a slice
  int rows = 0, cols = 0;
  int* ptr = nullptr;         // slices + 1 offsets (entries)
  int* col = nullptr;
  double* val = nullptr;
  float* valf = nullptr;      // FP32 copy (mixed precision), or null
  double* dinv = nullptr;     // 1 / diagonal (square matrices), or null
  float* dinvf = nullptr;
  long long stored = 0;       // entries incl. padding
};

// ELL block of one colour class of a colour-ordered matrix: rows
// [off, off + count), entry k of row i at k * count + i
struct Ell {
  int off = 0, count = 0, width = 0;
  int* col = nullptr;
  double* val = nullptr;
  float* valf = nullptr;
  double* dinv = nullptr;
  float* dinvf = nullptr;
};
template <typename V>
struct EllView {
  int off, count, width;
  const int* col;
  const V* val;
  const V* dinv;
};
template <typename V>
inline EllView<V> eview(const Ell& e);
template <>
inline EllView<double> eview<double>(const Ell& e) { return {e.off, e.count, e.width, e.col, e.val, e.dinv}; }
template <>
inline EllView<float> eview<float>(const Ell& e) { return {e.off, e.count, e.width, e.col, e.valf, e.dinvf}; }

template <typename V>
struct SellView {
  int rows;
  const int* ptr;
  const int* col;
  const V* val;
  const V* dinv;
};
template <typename V>
inline SellView<V> view(const Sell& s);
template <>
inline SellView<double> view<double>(const Sell& s) { return {s.rows, s.ptr, s.col, s.val, s.dinv}; }
template <>
inline SellView<float> view<float>(const Sell& s) { return {s.rows, s.ptr, s.col, s.valf, s.dinvf}; }

// Sparse kernels (k_sparse.hip).  Vectors: nvec of them, strides sx, sb, sy.
// mode 0: y = A x               mode 1: y += A x
// mode 2: y = b - A x           mode 3: y = x + w D^{-1}(b - A x)   (x == null: x = 0)
// mode 4: y = x + beta D^{-1}(b - A x) + alpha (x - yprev)   has_prev 1: yprev in y,
//         2: yprev = 0, 0: no alpha term (x == null: x = 0)
template <typename T, typename V>
void launch_sell(const Sell& A, int mode, const T* x, long long sx, const T* b, long long sb, T* y, long long sy,
                 int nvec, double w, double alpha, int has_prev, const int* gate, hipStream_t st);
// a Chebyshev step on M_Q based on multicolour SGS, in three parts:
// enter: res = r - M x (x null: r), s = D^{-1} res on colour 0, 0 elsewhere;
// the colour passes 1, 2, 3, 4, 3, 2, 1 (launch_ell_colour with b = res,
// or launch_ell_middle for 3, 4, 3);
// leave: the closing colour-0 pass, d = alpha d + beta s, x = x + d (x_zero: d)
template <typename T, typename V>
void launch_sgs_enter(const Sell& A, const unsigned char* colour, const T* x, const T* r, T* res, T* s,
                      const int* gate, hipStream_t st);
template <typename T, typename V>
void launch_sgs_leave(const Sell& A, const unsigned char* colour, const T* res, T* s, T* d, T* x, double alpha,
                      double beta, int x_zero, const int* gate, hipStream_t st);
// colour pass / the colour-3, element, colour-3 middle on ELL blocks of a
// colour-ordered matrix (b, x in the colour order)
template <typename T, typename V>
void launch_ell_colour(const Ell& E, const T* b, T* x, const int* gate, hipStream_t st);
template <typename T, typename V>
void launch_ell_middle(const Ell& E3, const Ell& E4, const T* b, T* x, const int* gate, hipStream_t st);
// The pressure-mass solve on the bounding box of the step (k_step_mq.hip):
// Q1 node (c, d) at d (ex + 1) + c, then element (e, f) at
// (ex + 1)(ey + 1) + f ex + e; the elements e < hx, f < hy are absent.
struct StepBox {
  int ex = 0, ey = 0, hx = 0, hy = 0;
  double h = 0.0;
  long long size() const { return (long long)(ex + 1) * (ey + 1) + (long long)ex * ey; }
};
// blocks of one launch with tile side `tile`
int step_mq_tiles(const StepBox& b, int tile);
// one Chebyshev step of the multicolour SGS semi-iteration on M_Q in one
// launch (tile 8 or 16 Q1 nodes per side of a block): from z_k = zin (not
// read when first) to z_{k+1} = zout, direction d updated in place
template <typename T>
void launch_step_mq_fused(const StepBox& b, int tile, const T* r, const T* zin, T* zout, T* d, double a, double bc,
                          int first, const int* gate, hipStream_t st);
// gather y[i] = a x[idx[i]] or scatter y[idx[i]] = a x[i], with type conversion
template <typename Ti, typename To>
void launch_permute(int n, const int* idx, bool scatter, double a, const Ti* x, To* y, const int* gate,
                    hipStream_t st);
// x = Ainv b (dense, FP64 matrix), nvec vectors of length n with strides
template <typename T>
void launch_dense_apply(const double* Ainv, int n, const T* b, long long sb, T* x, long long sx, int nvec,
                        const int* gate, hipStream_t st);
// y[i] = (To) (a * x[i] + c * z[i]) over n entries (z may be null)
template <typename Ti, typename To>
void launch_vcombine(long long n, double a, const Ti* x, double c, const Ti* z, To* y, const int* gate,
                     hipStream_t st);
// frame projection of a pressure vector p = [p_1 (nk) | p_0 (n0)] onto k^perp,
// k = [1; -1]: partial sums then p -= (k.p / (nk + n0)) k
void launch_frame_project(double* p_part_scratch, int nk, int n0, void* p, bool fp32, const int* gate,
                          hipStream_t st);
int frame_project_blocks(int np);
// block partial sums of k . p = sum(p_1) - sum(p_0) (FP64, frame_project_blocks(nk + n0) of them)
void launch_frame_partials(double* part, int nk, int n0, const double* p, hipStream_t st);

}  // namespace eth
