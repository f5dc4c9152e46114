// Scalar work that runs in the last block of a reduction: the recurrences of
// preconditioned MINRES (alg:minres) kept on the device in FP64, so that an
// iteration needs no host round trip.
#pragma once
#include <hip/hip_runtime.h>

namespace eth {

enum Epilogue : int {
  EPI_NONE = 0,
  EPI_MINRES_INIT = 1,   // total = <z1, v1>            -> gamma_1
  EPI_MINRES_DELTA = 2,  // total = <K zhat_j, zhat_j>   -> delta_j, v-update coefficients
  EPI_MINRES_GAMMA = 3,  // total = <zhat_{j+1}, v_{j+1}> -> Givens step, w/x coefficients
  EPI_SCALE = 4,         // out[rhs] = total * scale
};

// Status codes mirrored from eth.h
constexpr int kStOK = 0;
constexpr int kStBreakdown = -5;
constexpr int kStMaxit = 1;

// Per right-hand side MINRES scalars.  zhat_j = P^{-1} v_j is kept
// unnormalised; z_j = zhat_j / gamma_j.
struct MinresScalars {
  double gamma, gamma_prev, gamma1, delta, eta;
  double c, c_prev, s, s_prev;
  double tol;
  double tol_abs;      // > 0: stop when |eta| <= tol_abs instead (refinement restarts)
  double vy, va, vb;   // v_{j+1} = vy*y - va*v_j - vb*v_{j-1},  y = K zhat_j
  double wz, wp, wc;   // w_{j+1} = wz*zhat_j - wp*w_{j-1} - wc*w_j
  double xc;           // x_j = x_{j-1} + xc*w_{j+1}
  double rel;          // |eta| / gamma_1
  int active;          // 1 while iterating
  int wx_todo;         // 1 when the w/x update of the last Givens step is pending
  int iters, maxit, status, hist_len;
  double* hist;        // |eta|/gamma_1 per iteration (device, hist_len entries)
  double* hist_delta;  // delta_j at j-1 (the Lanczos tridiagonal, for EST-MINRES)
  double* hist_gamma;  // gamma_j at j-1 (gamma_1 = ||r_0||_{P^{-1}} first)
};

// Per right-hand side FGMRES record (restart length m <= 63).
struct GmresScalars {
  double beta, target, res, inv;   // ||r_0||, absolute tolerance, |g_{j+1}|, 1/h_{j+1,j}
  int active;                      // Arnoldi steps of the current cycle still run
  int update;                      // the cycle-end solution update is due
  int converged, kend, iters, maxit, status, hist_len, m, pad;
  double *H, *cs, *sn, *g, *y, *h1, *h2, *hist;   // device arrays of this RHS
};

struct ScaleState {
  double* out;
  double scale;
};

__device__ inline void minres_init(MinresScalars& s, double g2) {
  if (!(g2 >= 0.0) || !isfinite(g2)) {
    s.status = kStBreakdown;
    s.active = 0;
    s.wx_todo = 0;
    return;
  }
  const double g = sqrt(g2);
  s.gamma = g;
  s.gamma1 = g;
  s.gamma_prev = 0.0;
  s.eta = g;
  s.c = s.c_prev = 1.0;
  s.s = s.s_prev = 0.0;
  s.iters = 0;
  s.rel = 1.0;
  s.wx_todo = 0;
  s.status = kStOK;
  s.active = (g > 0.0 && !(s.tol_abs > 0.0 && g <= s.tol_abs)) ? 1 : 0;
  if (s.hist && s.hist_len > 0) s.hist[0] = 1.0;
  if (s.hist_gamma && s.hist_len > 0) s.hist_gamma[0] = g;
}

__device__ inline void minres_delta(MinresScalars& s, double kzz) {
  const double g = s.gamma;
  const double delta = kzz / (g * g);
  s.delta = delta;
  s.vy = 1.0 / g;
  s.va = delta / g;
  s.vb = (s.iters > 0) ? g / s.gamma_prev : 0.0;   // gamma_0 v_0 term is zero at j = 1
  if (s.hist_delta && s.iters < s.hist_len) s.hist_delta[s.iters] = delta;
}

__device__ inline void minres_gamma(MinresScalars& s, double g2) {
  // tolerate rounding-level negatives once the Krylov space is exhausted
  if (g2 < 0.0 && g2 > -1e-28 * s.gamma1 * s.gamma1) g2 = 0.0;
  if (!(g2 >= 0.0) || !isfinite(g2)) {
    s.status = kStBreakdown;
    s.active = 0;
    s.wx_todo = 0;
    return;
  }
  const double gn = sqrt(g2);
  const double g = s.gamma, d = s.delta;
  // Column j of the extended Lanczos tridiagonal is (g above the diagonal,
  // d on it, gn below).  The rotations of steps j-2 (c_prev, s_prev) and j-1
  // (c, s) act on it first; a new rotation then annihilates gn.  The result
  // is column j of the QR factor R (rho on the diagonal, sigma and tau above)
  // and the next entries of the rotated right-hand side (eta).
  const double tau = s.s_prev * g;
  const double t = s.c_prev * g;
  const double sigma = s.c * t + s.s * d;
  const double diag = s.c * d - s.s * t;
  const double rho = sqrt(diag * diag + gn * gn);
  const double cn = diag / rho, sn = gn / rho;
  // search direction w_{j+1} = (zhat_j / g - sigma w_j - tau w_{j-1}) / rho
  s.wz = 1.0 / (g * rho);
  s.wp = tau / rho;
  s.wc = sigma / rho;
  s.xc = cn * s.eta;
  s.eta = -sn * s.eta;
  s.c_prev = s.c;
  s.c = cn;
  s.s_prev = s.s;
  s.s = sn;
  s.gamma_prev = g;
  s.gamma = gn;
  s.iters += 1;
  s.rel = fabs(s.eta) / s.gamma1;
  if (s.hist && s.iters < s.hist_len) s.hist[s.iters] = s.rel;
  if (s.hist_gamma && s.iters < s.hist_len) s.hist_gamma[s.iters] = gn;
  s.wx_todo = 1;
  if ((s.tol_abs > 0.0 ? fabs(s.eta) <= s.tol_abs : s.rel <= s.tol) || gn == 0.0) {
    s.active = 0;
  } else if (s.iters >= s.maxit) {
    s.active = 0;
    s.status = kStMaxit;
  }
}

__device__ inline void run_epilogue(int epi, void* state, int rhs, const double* tot) {
  switch (epi) {
    case EPI_MINRES_INIT:
      minres_init(static_cast<MinresScalars*>(state)[rhs], tot[0]);
      break;
    case EPI_MINRES_DELTA:
      minres_delta(static_cast<MinresScalars*>(state)[rhs], tot[0]);
      break;
    case EPI_MINRES_GAMMA:
      minres_gamma(static_cast<MinresScalars*>(state)[rhs], tot[0]);
      break;
    case EPI_SCALE: {
      ScaleState* st = static_cast<ScaleState*>(state);
      st->out[rhs] = tot[0] * st->scale;
      break;
    }
    default:
      break;
  }
}

}  // namespace eth
