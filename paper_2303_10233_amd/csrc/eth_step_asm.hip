// Host-side mesh and finite-element assembly for the step domain (Sec. 3,
// the inflow-outflow example; bilinear forms of eq:stokes_fe and of the PCD
// matrices of Sec. 3.1).  Runs once per problem and per wind; the results go
// to the GPU as sliced-ELL matrices (eth_step.hip).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <stdexcept>
#include <thread>

#include "eth_step.h"

namespace eth {

// ------------------------------------------------------------------- mesh
namespace {
// elements along one axis whose closure holds grid line I: the Q2 half grid
// has odd lines inside one element, the Q1 grid none
int touching(int I, bool half, int out[2]) {
  if (half) {
    if (I % 2 == 0) {
      out[0] = I / 2 - 1;
      out[1] = I / 2;
      return 2;
    }
    out[0] = (I - 1) / 2;
    return 1;
  }
  out[0] = I - 1;
  out[1] = I;
  return 2;
}
}  // namespace

void StepMesh::build(int m_, int L_, bool channel_) {
  if (m_ < 1 || L_ < 1) throw std::invalid_argument("step mesh: m and length must be >= 1");
  m = m_;
  L = L_;
  channel = channel_;
  h = 1.0 / m;
  x0 = -1.0;
  y0 = channel ? 0.0 : -1.0;
  ex = (1 + L) * m;
  ey = channel ? m : 2 * m;
  elem_act.assign((size_t)ex * ey, 1);
  if (!channel)
    for (int f = 0; f < m; ++f)
      for (int e = 0; e < m; ++e) elem_act[(size_t)f * ex + e] = 0;   // the step
  nqx = 2 * ex + 1;
  nqy = 2 * ey + 1;
  auto flags = [&](int I, int J, bool half, bool& any, bool& all) {
    int tx[2], ty[2];
    const int nx = touching(I, half, tx), ny = touching(J, half, ty);
    any = false;
    all = true;
    for (int b = 0; b < ny; ++b)
      for (int a = 0; a < nx; ++a) {
        const bool ok = active(tx[a], ty[b]);
        any = any || ok;
        all = all && ok;
      }
  };
  q2_index.assign((size_t)nqx * nqy, -1);
  q2_I.clear();
  q2_J.clear();
  dirichlet.clear();
  for (int J = 0; J < nqy; ++J)
    for (int I = 0; I < nqx; ++I) {
      bool any, all;
      flags(I, J, true, any, all);
      if (!any) continue;
      q2_index[(size_t)J * nqx + I] = (int)q2_I.size();
      q2_I.push_back(I);
      q2_J.push_back(J);
      const bool outflow = I == nqx - 1 && J > 0 && J < nqy - 1;
      dirichlet.push_back((!all && !outflow) ? 1 : 0);
    }
  nv = (int)q2_I.size();
  q1_index.assign((size_t)(ex + 1) * (ey + 1), -1);
  q1_I.clear();
  q1_J.clear();
  for (int J = 0; J <= ey; ++J)
    for (int I = 0; I <= ex; ++I) {
      bool any, all;
      flags(I, J, false, any, all);
      if (!any) continue;
      q1_index[(size_t)J * (ex + 1) + I] = (int)q1_I.size();
      q1_I.push_back(I);
      q1_J.push_back(J);
    }
  nk = (int)q1_I.size();
  el_index.assign((size_t)ex * ey, -1);
  el_x.clear();
  el_y.clear();
  for (int f = 0; f < ey; ++f)
    for (int e = 0; e < ex; ++e) {
      if (!active(e, f)) continue;
      el_index[(size_t)f * ex + e] = (int)el_x.size();
      el_x.push_back(e);
      el_y.push_back(f);
    }
  n0 = (int)el_x.size();
}

// ---------------------------------------------------------- element matrices
namespace {
constexpr int NQ = 4;
void gauss4(double* x, double* w) {   // Gauss-Legendre on [0, 1], exact to degree 7
  const double t1 = 0.33998104358485626480, t2 = 0.86113631159405257522;
  const double w1 = 0.65214515486254614263, w2 = 0.34785484513745385737;
  x[0] = 0.5 * (1 - t2);
  x[1] = 0.5 * (1 - t1);
  x[2] = 0.5 * (1 + t1);
  x[3] = 0.5 * (1 + t2);
  w[0] = 0.5 * w2;
  w[1] = 0.5 * w1;
  w[2] = 0.5 * w1;
  w[3] = 0.5 * w2;
}
double q2v(int i, double t) { return i == 0 ? (1 - t) * (1 - 2 * t) : i == 1 ? 4 * t * (1 - t) : t * (2 * t - 1); }
double q2d(int i, double t) { return i == 0 ? 4 * t - 3 : i == 1 ? 4 - 8 * t : 4 * t - 1; }
double q1v(int a, double t) { return a == 0 ? 1 - t : t; }
double q1d(int a, double) { return a == 0 ? -1.0 : 1.0; }
}  // namespace

void StepElem::build(double h) {
  double xq[NQ], wq[NQ];
  gauss4(xq, wq);
  const double h2 = h * h;
  std::fill(&A[0][0], &A[0][0] + 81, 0.0);
  std::fill(&M[0][0], &M[0][0] + 81, 0.0);
  std::fill(&B1x[0][0], &B1x[0][0] + 36, 0.0);
  std::fill(&B1y[0][0], &B1y[0][0] + 36, 0.0);
  std::fill(B0x, B0x + 9, 0.0);
  std::fill(B0y, B0y + 9, 0.0);
  std::fill(&Qk[0][0], &Qk[0][0] + 16, 0.0);
  std::fill(R, R + 4, 0.0);
  std::fill(&Kp[0][0], &Kp[0][0] + 16, 0.0);
  std::fill(&Cx[0][0][0], &Cx[0][0][0] + 729, 0.0);
  std::fill(&Cy[0][0][0], &Cy[0][0][0] + 729, 0.0);
  std::fill(&Cpx[0][0][0], &Cpx[0][0][0] + 144, 0.0);
  std::fill(&Cpy[0][0][0], &Cpy[0][0][0] + 144, 0.0);
  Q0 = h2;
  for (int qy = 0; qy < NQ; ++qy)
    for (int qx = 0; qx < NQ; ++qx) {
      const double W = wq[qx] * wq[qy], s = xq[qx], t = xq[qy];
      double phi[9], px[9], py[9], psi[4], sx[4], sy[4];
      for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i) {
          phi[3 * j + i] = q2v(i, s) * q2v(j, t);
          px[3 * j + i] = q2d(i, s) * q2v(j, t);
          py[3 * j + i] = q2v(i, s) * q2d(j, t);
        }
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          psi[2 * b + a] = q1v(a, s) * q1v(b, t);
          sx[2 * b + a] = q1d(a, s) * q1v(b, t);
          sy[2 * b + a] = q1v(a, s) * q1d(b, t);
        }
      for (int i = 0; i < 9; ++i) {
        for (int j = 0; j < 9; ++j) {
          A[i][j] += W * (px[i] * px[j] + py[i] * py[j]);
          M[i][j] += W * h2 * phi[i] * phi[j];
          for (int k = 0; k < 9; ++k) {
            Cx[i][j][k] += W * h * phi[i] * px[j] * phi[k];
            Cy[i][j][k] += W * h * phi[i] * py[j] * phi[k];
          }
        }
        B0x[i] += -W * h * px[i];
        B0y[i] += -W * h * py[i];
      }
      for (int a = 0; a < 4; ++a) {
        for (int j = 0; j < 9; ++j) {
          B1x[a][j] += -W * h * psi[a] * px[j];
          B1y[a][j] += -W * h * psi[a] * py[j];
        }
        for (int b = 0; b < 4; ++b) {
          Qk[a][b] += W * h2 * psi[a] * psi[b];
          Kp[a][b] += W * (sx[a] * sx[b] + sy[a] * sy[b]);
          for (int k = 0; k < 9; ++k) {
            Cpx[a][b][k] += W * h * psi[a] * sx[b] * phi[k];
            Cpy[a][b][k] += W * h * psi[a] * sy[b] * phi[k];
          }
        }
        R[a] += W * h2 * psi[a];
      }
    }
}

// ----------------------------------------------------------------- sparse
double Csr::diag(int r) const {
  for (int k = ptr[r]; k < ptr[r + 1]; ++k)
    if (col[k] == r) return val[k];
  return 0.0;
}

void RowBuilder::add(int i, int j, double v) {
  auto& row = r[i];
  for (auto& e : row)
    if (e.first == j) {
      e.second += v;
      return;
    }
  row.emplace_back(j, v);
}

Csr RowBuilder::finish(bool drop_zeros) const {
  Csr A;
  A.rows = rows;
  A.cols = cols;
  A.ptr.assign(rows + 1, 0);
  size_t nnz = 0;
  for (int i = 0; i < rows; ++i) nnz += r[i].size();
  A.col.reserve(nnz);
  A.val.reserve(nnz);
  std::vector<std::pair<int, double>> row;
  for (int i = 0; i < rows; ++i) {
    row = r[i];
    std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    for (const auto& e : row) {
      if (drop_zeros && e.second == 0.0) continue;
      A.col.push_back(e.first);
      A.val.push_back(e.second);
    }
    A.ptr[i + 1] = (int)A.col.size();
  }
  return A;
}

Csr csr_transpose(const Csr& A) {
  Csr T;
  T.rows = A.cols;
  T.cols = A.rows;
  T.ptr.assign(T.rows + 1, 0);
  for (int c : A.col) T.ptr[c + 1]++;
  for (int i = 0; i < T.rows; ++i) T.ptr[i + 1] += T.ptr[i];
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  std::vector<int> next(T.ptr.begin(), T.ptr.end() - 1);
  for (int i = 0; i < A.rows; ++i)
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int p = next[A.col[k]]++;
      T.col[p] = i;
      T.val[p] = A.val[k];
    }
  return T;
}

// ------------------------------------------------------------------ assembly
namespace {
void elem_nodes(const StepMesh& g, int e, int f, int vel[9], int q1[4], int& p0) {
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < 3; ++i) vel[3 * j + i] = g.q2(2 * e + i, 2 * f + j);
  for (int b = 0; b < 2; ++b)
    for (int a = 0; a < 2; ++a) q1[2 * b + a] = g.q1(e + a, f + b);
  p0 = g.el_index[(size_t)f * g.ex + e];
}
}  // namespace

namespace {
// the elements of every Q2 node in ascending order (CSR over the nodes)
struct NodeElems {
  std::vector<int> ptr, el;
};
NodeElems node_elements(const StepMesh& g) {
  NodeElems ne;
  ne.ptr.assign((size_t)g.nv + 1, 0);
  int vel[9], q1[4], p0;
  for (int k = 0; k < g.n0; ++k) {
    elem_nodes(g, g.el_x[k], g.el_y[k], vel, q1, p0);
    for (int m = 0; m < 9; ++m) ne.ptr[(size_t)vel[m] + 1]++;
  }
  for (int i = 0; i < g.nv; ++i) ne.ptr[(size_t)i + 1] += ne.ptr[i];
  ne.el.resize(ne.ptr[g.nv]);
  std::vector<int> next(ne.ptr.begin(), ne.ptr.end() - 1);
  for (int k = 0; k < g.n0; ++k) {
    elem_nodes(g, g.el_x[k], g.el_y[k], vel, q1, p0);
    for (int m = 0; m < 9; ++m) ne.el[next[vel[m]]++] = k;
  }
  return ne;
}

// body(r0, r1) over contiguous blocks of rows on up to 16 host threads
// (one for small matrices; ETH_HOST_THREADS caps the count); blocks are
// independent
template <typename Body>
void parallel_rows(int rows, Body&& body) {
  unsigned nt = std::thread::hardware_concurrency();
  if (const char* e = std::getenv("ETH_HOST_THREADS")) nt = (unsigned)std::max(1, std::atoi(e));
  nt = std::max(1u, std::min(nt, 16u));
  if (rows < 8192) nt = 1;
  if (nt == 1) {
    body(0, rows);
    return;
  }
  std::vector<std::thread> th;
  const int per = (rows + (int)nt - 1) / (int)nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int r0 = (int)t * per, r1 = std::min(rows, r0 + per);
    if (r0 >= r1) break;
    th.emplace_back([&body, r0, r1] { body(r0, r1); });
  }
  for (auto& x : th) x.join();
}
}  // namespace

// F row by row: row i visits its elements in ascending order, so every entry
// sums its element contributions in the order of an element-by-element
// assembly; rows are filled on several host threads.
Csr step_assemble_F(const StepMesh& g, const StepElem& E, double nu, const double* wind, bool embed) {
  const NodeElems ne = node_elements(g);
  Csr A;
  A.rows = A.cols = g.nv;
  A.ptr.assign((size_t)g.nv + 1, 0);
  // row sizes first (a row's columns: the nodes of its elements, Dirichlet
  // ones left out in the embedded form), then the values into place
  std::vector<int> len(g.nv, 0);
  auto row_entries = [&](int i, std::vector<std::pair<int, double>>& row) {
    row.clear();
    if (embed && g.dirichlet[i]) {
      row.emplace_back(i, 1.0);
      return;
    }
    int vel[9], q1[4], p0;
    for (int q = ne.ptr[i]; q < ne.ptr[(size_t)i + 1]; ++q) {
      const int k = ne.el[q];
      elem_nodes(g, g.el_x[k], g.el_y[k], vel, q1, p0);
      double wx[9] = {0}, wy[9] = {0};
      if (wind)
        for (int m = 0; m < 9; ++m) {
          wx[m] = wind[vel[m]];
          wy[m] = wind[g.nv + vel[m]];
        }
      int li = 0;
      while (vel[li] != i) ++li;
      for (int j = 0; j < 9; ++j) {
        if (embed && g.dirichlet[vel[j]]) continue;
        double v = nu * E.A[li][j];
        if (wind)
          for (int m = 0; m < 9; ++m) v += E.Cx[li][j][m] * wx[m] + E.Cy[li][j][m] * wy[m];
        bool found = false;
        for (auto& e : row)
          if (e.first == vel[j]) {
            e.second += v;
            found = true;
            break;
          }
        if (!found) row.emplace_back(vel[j], v);
      }
    }
    std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  };
  parallel_rows(g.nv, [&](int r0, int r1) {
    std::vector<std::pair<int, double>> row;
    for (int i = r0; i < r1; ++i) {
      row_entries(i, row);
      len[i] = (int)row.size();
    }
  });
  for (int i = 0; i < g.nv; ++i) A.ptr[(size_t)i + 1] = A.ptr[i] + len[i];
  A.col.resize(A.ptr[g.nv]);
  A.val.resize(A.ptr[g.nv]);
  parallel_rows(g.nv, [&](int r0, int r1) {
    std::vector<std::pair<int, double>> row;
    for (int i = r0; i < r1; ++i) {
      row_entries(i, row);
      int o = A.ptr[i];
      for (const auto& e : row) {
        A.col[o] = e.first;
        A.val[o] = e.second;
        ++o;
      }
    }
  });
  return A;
}

Csr step_assemble_B(const StepMesh& g, const StepElem& E) {
  RowBuilder rb(g.nk + g.n0, 2 * g.nv);
  for (int k = 0; k < g.n0; ++k) {
    int vel[9], q1[4], p0;
    elem_nodes(g, g.el_x[k], g.el_y[k], vel, q1, p0);
    for (int j = 0; j < 9; ++j) {
      for (int a = 0; a < 4; ++a) {
        rb.add(q1[a], vel[j], E.B1x[a][j]);
        rb.add(q1[a], g.nv + vel[j], E.B1y[a][j]);
      }
      rb.add(g.nk + p0, vel[j], E.B0x[j]);
      rb.add(g.nk + p0, g.nv + vel[j], E.B0y[j]);
    }
  }
  return rb.finish();
}

Csr step_assemble_K(const StepMesh& g, const Csr& F, const Csr& B) {
  const int nv = g.nv, np = g.nk + g.n0;
  const long long N = g.N();
  const Csr Bt = csr_transpose(B);   // 2 nv x np
  Csr K;
  K.rows = K.cols = (int)N;
  K.ptr.assign(N + 1, 0);
  // row r of K: velocity rows (component c, node i) hold F's row i without
  // the Dirichlet columns, then B^T's row (none for a Dirichlet node);
  // pressure rows hold B's row without the Dirichlet velocity columns.
  // visit(r, emit) lists a row's entries in that order.
  auto visit = [&](int r, auto&& emit) {
    if (r < 2 * nv) {
      const int c = r / nv, i = r % nv;
      if (g.dirichlet[i]) return;
      for (int k = F.ptr[i]; k < F.ptr[i + 1]; ++k)
        if (!g.dirichlet[F.col[k]]) emit(c * nv + F.col[k], F.val[k]);
      for (int k = Bt.ptr[r]; k < Bt.ptr[r + 1]; ++k) emit(2 * nv + Bt.col[k], Bt.val[k]);
    } else {
      const int p = r - 2 * nv;
      for (int k = B.ptr[p]; k < B.ptr[p + 1]; ++k)
        if (!g.dirichlet[B.col[k] % nv]) emit(B.col[k], B.val[k]);
    }
  };
  std::vector<int> len((size_t)N, 0);
  parallel_rows((int)N, [&](int r0, int r1) {
    for (int r = r0; r < r1; ++r) {
      int n = 0;
      visit(r, [&](int, double) { ++n; });
      len[r] = n;
    }
  });
  for (long long r = 0; r < N; ++r) K.ptr[r + 1] = K.ptr[r] + len[r];
  K.col.resize(K.ptr[N]);
  K.val.resize(K.ptr[N]);
  parallel_rows((int)N, [&](int r0, int r1) {
    for (int r = r0; r < r1; ++r) {
      int o = K.ptr[r];
      visit(r, [&](int col, double v) {
        K.col[o] = col;
        K.val[o] = v;
        ++o;
      });
    }
  });
  (void)np;
  return K;
}

// Sliced-ELL layout of A: 64 rows per slice, a slice as wide as its longest
// row, entries column-major inside the slice (entry k of lane l at
// ptr[slice] + 64 k + l); a row's padding repeats its last column (0 for an
// empty row) with value 0.  Slices are filled on several host threads.
void sell_layout(const Csr& A, std::vector<int>& ptr, std::vector<int>& col, std::vector<double>& val) {
  const int slices = (A.rows + 63) / 64;
  ptr.assign((size_t)slices + 1, 0);
  std::vector<int> width(slices, 0);
  parallel_rows(slices, [&](int s0, int s1) {
    for (int sl = s0; sl < s1; ++sl) {
      int w = 0;
      for (int r = sl * 64; r < std::min(A.rows, sl * 64 + 64); ++r) w = std::max(w, A.ptr[r + 1] - A.ptr[r]);
      width[sl] = w;
    }
  });
  for (int sl = 0; sl < slices; ++sl) ptr[(size_t)sl + 1] = ptr[sl] + 64 * width[sl];
  const size_t tot = (size_t)ptr[slices];
  col.assign(tot, 0);
  val.assign(tot, 0.0);
  parallel_rows(slices, [&](int s0, int s1) {
    for (int sl = s0; sl < s1; ++sl) {
      const int w = width[sl];
      for (int lane = 0; lane < 64; ++lane) {
        const int r = sl * 64 + lane;
        const int len = r < A.rows ? A.ptr[r + 1] - A.ptr[r] : 0;
        int last = 0;
        for (int k = 0; k < w; ++k) {
          const size_t o = (size_t)ptr[sl] + (size_t)k * 64 + lane;
          if (k < len) {
            last = A.col[A.ptr[r] + k];
            val[o] = A.val[A.ptr[r] + k];
          }
          col[o] = last;
        }
      }
    }
  });
}

Csr step_assemble_MQ(const StepMesh& g, const StepElem& E) {
  RowBuilder rb(g.nk + g.n0, g.nk + g.n0);
  for (int k = 0; k < g.n0; ++k) {
    int vel[9], q1[4], p0;
    elem_nodes(g, g.el_x[k], g.el_y[k], vel, q1, p0);
    for (int a = 0; a < 4; ++a) {
      for (int b = 0; b < 4; ++b) rb.add(q1[a], q1[b], E.Qk[a][b]);
      rb.add(q1[a], g.nk + p0, E.R[a]);
      rb.add(g.nk + p0, q1[a], E.R[a]);
    }
    rb.add(g.nk + p0, g.nk + p0, E.Q0);
  }
  return rb.finish();
}

Csr step_assemble_Q1(const StepMesh& g, const StepElem& E) {
  RowBuilder rb(g.nk, g.nk);
  for (int k = 0; k < g.n0; ++k) {
    int vel[9], q1[4], p0;
    elem_nodes(g, g.el_x[k], g.el_y[k], vel, q1, p0);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) rb.add(q1[a], q1[b], E.Qk[a][b]);
  }
  return rb.finish();
}

// F_1 = nu int grad psi_j . grad psi_i + int (w . grad psi_j) psi_i, plus
// (robin) the inflow term - int_{x=-1} (w . n) psi_j psi_i ds = int w_x psi_j psi_i dy
Csr step_assemble_F1(const StepMesh& g, const StepElem& E, double nu, const double* wind, bool robin) {
  RowBuilder rb(g.nk, g.nk);
  for (int k = 0; k < g.n0; ++k) {
    int vel[9], q1[4], p0;
    elem_nodes(g, g.el_x[k], g.el_y[k], vel, q1, p0);
    double wx[9] = {0}, wy[9] = {0};
    if (wind)
      for (int m = 0; m < 9; ++m) {
        wx[m] = wind[vel[m]];
        wy[m] = wind[g.nv + vel[m]];
      }
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        double v = nu * E.Kp[a][b];
        for (int m = 0; m < 9; ++m) v += E.Cpx[a][b][m] * wx[m] + E.Cpy[a][b][m] * wy[m];
        rb.add(q1[a], q1[b], v);
      }
  }
  if (robin && wind) {
    double xq[NQ], wq[NQ];
    gauss4(xq, wq);
    for (int f = 0; f < g.ey; ++f) {
      if (!g.active(0, f)) continue;
      const int k0 = g.q1(0, f), k1 = g.q1(0, f + 1);
      double w3[3];
      for (int j = 0; j < 3; ++j) w3[j] = wind[g.q2(0, 2 * f + j)];
      const int kk[2] = {k0, k1};
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          double s = 0.0;
          for (int q = 0; q < NQ; ++q) {
            const double t = xq[q];
            const double w = w3[0] * q2v(0, t) + w3[1] * q2v(1, t) + w3[2] * q2v(2, t);
            s += wq[q] * w * q1v(a, t) * q1v(b, t);
          }
          rb.add(kk[a], kk[b], g.h * s);
        }
    }
  }
  return rb.finish();
}

std::vector<double> step_velocity_mass_diag(const StepMesh& g, const StepElem& E) {
  std::vector<double> d(g.nv, 0.0);
  for (int k = 0; k < g.n0; ++k) {
    int vel[9], q1[4], p0;
    elem_nodes(g, g.el_x[k], g.el_y[k], vel, q1, p0);
    for (int i = 0; i < 9; ++i) d[vel[i]] += E.M[i][i];
  }
  return d;
}

// A_p = B_1 diag(M_v)^{-1} B_1^T over the free velocity nodes
Csr step_assemble_Ap(const StepMesh& g, const StepElem& E, const Csr& B) {
  const std::vector<double> mv = step_velocity_mass_diag(g, E);
  Csr B1;
  B1.rows = g.nk;
  B1.cols = B.cols;
  B1.ptr.assign(B.ptr.begin(), B.ptr.begin() + g.nk + 1);
  B1.col.assign(B.col.begin(), B.col.begin() + B.ptr[g.nk]);
  B1.val.assign(B.val.begin(), B.val.begin() + B.ptr[g.nk]);
  const Csr Bt = csr_transpose(B1);   // 2 nv x nk
  RowBuilder rb(g.nk, g.nk);
  for (int c = 0; c < 2 * g.nv; ++c) {
    const int node = c % g.nv;
    if (g.dirichlet[node]) continue;
    const double s = 1.0 / mv[node];
    for (int a = Bt.ptr[c]; a < Bt.ptr[c + 1]; ++a)
      for (int b = Bt.ptr[c]; b < Bt.ptr[c + 1]; ++b) rb.add(Bt.col[a], Bt.col[b], Bt.val[a] * Bt.val[b] * s);
  }
  return rb.finish();
}

// coarse element holding a fine grid position given in units of a quarter
// (Q2 half grid of the fine mesh) or half (Q1) of a coarse element: the first
// active one of the (up to four) candidates whose closure holds the point
namespace {
bool coarse_cell(const StepMesh& c, int Ix, int Jy, int per, int& ex, int& ey, int& rx, int& ry) {
  const int bx = Ix / per, by = Jy / per;
  for (int dx = 0; dx >= -1; --dx)
    for (int dy = 0; dy >= -1; --dy) {
      const int cx = bx + dx, cy = by + dy;
      if (!c.active(cx, cy)) continue;
      if (Ix < per * cx || Ix > per * (cx + 1) || Jy < per * cy || Jy > per * (cy + 1)) continue;
      ex = cx;
      ey = cy;
      rx = Ix - per * cx;
      ry = Jy - per * cy;
      return true;
    }
  return false;
}
}  // namespace

Csr step_q2_prolongation(const StepMesh& f, const StepMesh& c) {
  RowBuilder rb(f.nv, c.nv);
  for (int i = 0; i < f.nv; ++i) {
    if (f.dirichlet[i]) continue;
    int ex, ey, rx, ry;
    if (!coarse_cell(c, f.q2_I[i], f.q2_J[i], 4, ex, ey, rx, ry))
      throw std::runtime_error("step prolongation: fine node outside the coarse mesh");
    const double sx = rx / 4.0, sy = ry / 4.0;
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) {
        const double w = q2v(a, sx) * q2v(b, sy);
        if (std::fabs(w) <= 1e-15) continue;
        const int j = c.q2(2 * ex + a, 2 * ey + b);
        if (c.dirichlet[j]) continue;
        rb.add(i, j, w);
      }
  }
  return rb.finish();
}

Csr step_q1_prolongation(const StepMesh& f, const StepMesh& c) {
  RowBuilder rb(f.nk, c.nk);
  for (int i = 0; i < f.nk; ++i) {
    int ex, ey, rx, ry;
    if (!coarse_cell(c, f.q1_I[i], f.q1_J[i], 2, ex, ey, rx, ry))
      throw std::runtime_error("step prolongation: fine node outside the coarse mesh");
    const double sx = rx / 2.0, sy = ry / 2.0;
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        const double w = q1v(a, sx) * q1v(b, sy);
        if (std::fabs(w) <= 1e-15) continue;
        rb.add(i, c.q1(ex + a, ey + b), w);
      }
  }
  return rb.finish();
}

std::vector<double> step_inject_wind(const std::vector<double>& w, const StepMesh& f, const StepMesh& c) {
  std::vector<double> out(2 * (size_t)c.nv);
  for (int i = 0; i < c.nv; ++i) {
    const int j = f.q2(2 * c.q2_I[i], 2 * c.q2_J[i]);
    out[i] = w[j];
    out[c.nv + i] = w[f.nv + j];
  }
  return out;
}

std::vector<double> step_inflow(const StepMesh& g) {
  std::vector<double> u(2 * (size_t)g.nv, 0.0);
  for (int i = 0; i < g.nv; ++i) {
    if (!g.dirichlet[i] || g.q2_I[i] != 0) continue;
    const double y = g.y0 + g.q2_J[i] * (g.h / 2);
    u[i] = 4.0 * y * (1.0 - y);
  }
  return u;
}

std::vector<double> step_lift(const StepMesh& g, const Csr& F, const Csr& B, const std::vector<double>& uB) {
  std::vector<double> b(g.N(), 0.0);
  for (int c = 0; c < 2; ++c)
    for (int i = 0; i < g.nv; ++i) {
      if (g.dirichlet[i]) {
        b[(size_t)c * g.nv + i] = uB[(size_t)c * g.nv + i];
        continue;
      }
      double s = 0.0;
      for (int k = F.ptr[i]; k < F.ptr[i + 1]; ++k) s += F.val[k] * uB[(size_t)c * g.nv + F.col[k]];
      b[(size_t)c * g.nv + i] = -s;
    }
  for (int p = 0; p < B.rows; ++p) {
    double s = 0.0;
    for (int k = B.ptr[p]; k < B.ptr[p + 1]; ++k) s += B.val[k] * uB[B.col[k]];
    b[2 * (size_t)g.nv + p] = -s;
  }
  return b;
}

std::vector<double> dense_inverse(const Csr& A) {
  const int n = A.rows;
  std::vector<double> a((size_t)n * n, 0.0), inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) a[(size_t)i * n + A.col[k]] += A.val[k];
    inv[(size_t)i * n + i] = 1.0;
  }
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)p * n + c])) p = r;
    if (a[(size_t)p * n + c] == 0.0) throw std::runtime_error("coarsest step operator is singular");
    if (p != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[(size_t)p * n + k], a[(size_t)c * n + k]);
        std::swap(inv[(size_t)p * n + k], inv[(size_t)c * n + k]);
      }
    const double d = 1.0 / a[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) {
      a[(size_t)c * n + k] *= d;
      inv[(size_t)c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
        inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
      }
    }
  }
  return inv;
}

// Lanczos on D^{-1/2} A D^{-1/2} from the vector of ones; the largest Ritz
// value by bisection on the Sturm sequence of the tridiagonal matrix
double lambda_max_dinv(const Csr& A, int steps) {
  const int n = A.rows;
  std::vector<double> s(n);
  for (int i = 0; i < n; ++i) s[i] = 1.0 / std::sqrt(A.diag(i));
  std::vector<double> v(n, 1.0 / std::sqrt((double)n)), vp(n, 0.0), w(n);
  std::vector<double> al, be;
  double beta = 0.0;
  for (int k = 0; k < std::min(steps, n); ++k) {
    for (int i = 0; i < n; ++i) {
      double t = 0.0;
      for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) t += A.val[q] * s[A.col[q]] * v[A.col[q]];
      w[i] = s[i] * t - beta * vp[i];
    }
    double a = 0.0;
    for (int i = 0; i < n; ++i) a += w[i] * v[i];
    for (int i = 0; i < n; ++i) w[i] -= a * v[i];
    double b = 0.0;
    for (int i = 0; i < n; ++i) b += w[i] * w[i];
    b = std::sqrt(b);
    al.push_back(a);
    if (b < 1e-14 * std::fabs(a)) break;
    be.push_back(b);
    for (int i = 0; i < n; ++i) {
      vp[i] = v[i];
      v[i] = w[i] / b;
    }
    beta = b;
  }
  const int m = (int)al.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {   // Gershgorin bounds
    const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(be[i]) : 0.0);
    lo = std::min(lo, al[i] - r);
    hi = std::max(hi, al[i] + r);
  }
  auto count_below = [&](double x) {   // eigenvalues < x
    int c = 0;
    double q = 1.0;
    for (int i = 0; i < m; ++i) {
      const double b2 = i > 0 ? be[i - 1] * be[i - 1] : 0.0;
      q = al[i] - x - (i > 0 ? b2 / q : 0.0);
      if (q == 0.0) q = 1e-300;
      if (q < 0.0) ++c;
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

}  // namespace eth
