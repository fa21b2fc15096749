// FP64 CPU oracle for batched iLQR trajectory optimisation.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark do.  It shares no code, header or constant with the
// HIP solver.
//
// What it computes (paper Sec. II, eq. 1; Sec. IV-B, eq. 7; Sec. IV-C):
//   min_{X,U} sum_{k<T} l(x_k,u_k) + l_T(x_T),  x_{k+1} = f(x_k,u_k),  x_0 given,
// solved per instance by iLQR: forward rollout, linearise/quadratise,
// eigenvalue-clip the state- and control-cost Hessians (eq. 7), backward
// Riccati sweep with a Cholesky of Q_uu, backtracking line search, a fixed
// iteration budget for the whole batch (Sec. IV-A), and afterwards the
// critic targets of Sec. II: the K-step partial cost-to-go V-bar for every
// state, its gradient V-bar_x from the backward (costate) pass, and the
// state K steps later.
//
// Plain on purpose: dense row-major loops, no blocking, no fusion, FP64
// throughout, compiled without floating-point contraction.  Dynamics
// Jacobians come from complex-step differentiation of f (a forward-mode
// automatic derivative, as the paper's pipeline obtains its derivatives by
// automatic differentiation, Sec. IV-C); cost gradients are written
// analytically and their Hessians are complex-step derivatives of those
// gradients.
//
// Readings of points the paper leaves open (listed in the design notes):
//   * clipped matrices: the running state-cost Hessian l_xx, the control-cost
//     Hessian l_uu and the terminal Hessian, every iteration, after
//     symmetrisation; eps default 1e-6.
//   * line search: alpha_j = beta^j (repeated multiplication from 1),
//     j = 0..trials-1, accept the first finite J_hat with J_hat < J.
//   * no accepted step: the instance is frozen with LS_FAILED (without the
//     Levenberg-Marquardt loop a retry would repeat the same step).
//   * tolerance mode: freeze with CONVERGED once an accepted step lowers J by
//     at most rtol*|J_old|.
//   * warm start: U0 (zero by default), X0 = rollout of U0.
//   * V-bar_x_k is the costate lambda_k of the final trajectory.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

using cd = std::complex<double>;

enum Kind { KIND_LQ = 0, KIND_PM = 1, KIND_P3 = 2, KIND_QUAD = 3 };

enum StatusBits : uint32_t {
  ST_CONVERGED = 1u,
  ST_MAX_ITER = 2u,
  ST_LS_FAILED = 4u,
  ST_NONFINITE = 8u,
  ST_CHOL_FAIL = 16u,
};

struct Sys {
  int kind = -1;
  int n = 0, m = 0;
  const double* p = nullptr;  // parameter vector
  // LQ views into p
  const double *A = nullptr, *B = nullptr, *Q = nullptr, *R = nullptr, *QT = nullptr, *xr = nullptr;
};

inline double re(double v) { return v; }
inline double re(const cd& v) { return v.real(); }

// ------------------------------------------------------------ small dense helpers
template <class S>
bool gauss_solve(int n, std::vector<S> M, S* rhs, int nrhs) {
  // Gaussian elimination without pivoting, for the SPD mass matrices only
  // (so it stays analytic for complex-step derivatives).  M is n x n row-major,
  // rhs is n x nrhs row-major and is overwritten by the solution.
  for (int c = 0; c < n; ++c) {
    S piv = M[c * n + c];
    if (re(piv) == 0.0) return false;
    for (int r = c + 1; r < n; ++r) {
      S f = M[r * n + c] / piv;
      for (int j = c; j < n; ++j) M[r * n + j] -= f * M[c * n + j];
      for (int j = 0; j < nrhs; ++j) rhs[r * nrhs + j] -= f * rhs[c * nrhs + j];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    for (int j = 0; j < nrhs; ++j) {
      S s = rhs[c * nrhs + j];
      for (int k = c + 1; k < n; ++k) s -= M[c * n + k] * rhs[k * nrhs + j];
      rhs[c * nrhs + j] = s / M[c * n + c];
    }
  }
  return true;
}

// ------------------------------------------------------------ point mass
// p = [dt, w_u, w_p, w_T, w_obs, g_x, g_y, (c_x, c_y, r) x 3]
// Semi-implicit Euler of a 2-D double integrator: v+ = v + dt u, p+ = p + dt v+.
template <class S>
void pm_dyn(const double* p, const S* x, const S* u, S* xn) {
  const double dt = p[0];
  S vx = x[2] + dt * u[0];
  S vy = x[3] + dt * u[1];
  xn[0] = x[0] + dt * vx;
  xn[1] = x[1] + dt * vy;
  xn[2] = vx;
  xn[3] = vy;
}

template <class S>
S pm_cost(const double* p, const S* x, const S* u) {
  S ex = x[0] - p[5], ey = x[1] - p[6];
  S l = p[1] * (u[0] * u[0] + u[1] * u[1]) + p[2] * (ex * ex + ey * ey);
  for (int i = 0; i < 3; ++i) {
    const double cx = p[7 + 3 * i], cy = p[8 + 3 * i], r = p[9 + 3 * i];
    S dx = x[0] - cx, dy = x[1] - cy;
    l += p[4] * std::exp(-(dx * dx + dy * dy) / (r * r));
  }
  return l;
}

template <class S>
void pm_cost_grad(const double* p, const S* x, const S* u, S* lx, S* lu) {
  lx[0] = 2.0 * p[2] * (x[0] - p[5]);
  lx[1] = 2.0 * p[2] * (x[1] - p[6]);
  lx[2] = 0.0;
  lx[3] = 0.0;
  for (int i = 0; i < 3; ++i) {
    const double cx = p[7 + 3 * i], cy = p[8 + 3 * i], r = p[9 + 3 * i];
    S dx = x[0] - cx, dy = x[1] - cy;
    S e = p[4] * std::exp(-(dx * dx + dy * dy) / (r * r));
    lx[0] += e * (-2.0 * dx / (r * r));
    lx[1] += e * (-2.0 * dy / (r * r));
  }
  lu[0] = 2.0 * p[1] * u[0];
  lu[1] = 2.0 * p[1] * u[1];
}

template <class S>
S pm_term(const double* p, const S* x) {
  S ex = x[0] - p[5], ey = x[1] - p[6];
  return p[3] * (ex * ex + ey * ey + x[2] * x[2] + x[3] * x[3]);
}

template <class S>
void pm_term_grad(const double* p, const S* x, S* lx) {
  lx[0] = 2.0 * p[3] * (x[0] - p[5]);
  lx[1] = 2.0 * p[3] * (x[1] - p[6]);
  lx[2] = 2.0 * p[3] * x[2];
  lx[3] = 2.0 * p[3] * x[3];
}

// ------------------------------------------------------------ planar 3-link arm
// p = [dt, m1, m2, m3, l1, l2, l3, w_u, w_ee, w_T, w_obs, p_x, p_y, c_x, c_y, r]
// Uniform rods (centre of mass at half length, inertia m l^2 / 12), relative
// joint angles, horizontal plane.  Mass matrix from link Jacobians,
// M = sum_i m_i Jv_i^T Jv_i + I_i Jw_i^T Jw_i, and the velocity-product term
// from the Christoffel symbols of M.
template <class S>
void p3_link_jac(const double* p, const S* q, int i, S Jv[2][3], S dJv[3][2][3]) {
  // Jv: d(com_i)/dq ; dJv[k]: d Jv / d q_k.
  const double* len = p + 4;
  S phi[3];
  phi[0] = q[0];
  phi[1] = q[0] + q[1];
  phi[2] = q[0] + q[1] + q[2];
  for (int c = 0; c < 3; ++c) {
    Jv[0][c] = 0.0;
    Jv[1][c] = 0.0;
    for (int k = 0; k < 3; ++k) { dJv[k][0][c] = 0.0; dJv[k][1][c] = 0.0; }
  }
  for (int j = 0; j <= i; ++j) {
    const double a = (j < i) ? len[j] : 0.5 * len[j];
    S s = std::sin(phi[j]), co = std::cos(phi[j]);
    // com_i contains a*(cos phi_j, sin phi_j); phi_j depends on q_0..q_j.
    for (int c = 0; c <= j; ++c) {
      Jv[0][c] += -a * s;
      Jv[1][c] += a * co;
      for (int k = 0; k <= j; ++k) {
        dJv[k][0][c] += -a * co;
        dJv[k][1][c] += -a * s;
      }
    }
  }
}

template <class S>
void p3_mass(const double* p, const S* q, S Mout[3][3], S dM[3][3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      Mout[a][b] = 0.0;
      for (int k = 0; k < 3; ++k) dM[k][a][b] = 0.0;
    }
  for (int i = 0; i < 3; ++i) {
    const double mi = p[1 + i], li = p[4 + i];
    const double Ii = mi * li * li / 12.0;
    S Jv[2][3], dJv[3][2][3];
    p3_link_jac(p, q, i, Jv, dJv);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        S v = Jv[0][a] * Jv[0][b] + Jv[1][a] * Jv[1][b];
        Mout[a][b] += mi * v;
        // angular velocity of link i is the sum of the first i+1 joint rates
        if (a <= i && b <= i) Mout[a][b] += Ii;
        for (int k = 0; k < 3; ++k) {
          S dv = dJv[k][0][a] * Jv[0][b] + Jv[0][a] * dJv[k][0][b] +
                 dJv[k][1][a] * Jv[1][b] + Jv[1][a] * dJv[k][1][b];
          dM[k][a][b] += mi * dv;
        }
      }
  }
}

template <class S>
void p3_accel(const double* p, const S* q, const S* qd, const S* tau, S* acc) {
  S M[3][3], dM[3][3][3];
  p3_mass(p, q, M, dM);
  S rhs[3];
  for (int i = 0; i < 3; ++i) {
    // c_i = sum_jk Gamma_ijk qd_j qd_k,
    // Gamma_ijk = 1/2 (dM_ij/dq_k + dM_ik/dq_j - dM_jk/dq_i)
    S ci = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        S g = 0.5 * (dM[k][i][j] + dM[j][i][k] - dM[i][j][k]);
        ci += g * qd[j] * qd[k];
      }
    rhs[i] = tau[i] - ci;
  }
  std::vector<S> Mv(9);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Mv[a * 3 + b] = M[a][b];
  gauss_solve<S>(3, Mv, rhs, 1);
  for (int i = 0; i < 3; ++i) acc[i] = rhs[i];
}

template <class S>
void p3_dyn(const double* p, const S* x, const S* u, S* xn) {
  const double dt = p[0];
  S acc[3];
  p3_accel<S>(p, x, x + 3, u, acc);
  for (int i = 0; i < 3; ++i) {
    xn[3 + i] = x[3 + i] + dt * acc[i];
    xn[i] = x[i] + dt * xn[3 + i];
  }
}

template <class S>
void p3_ee(const double* p, const S* q, S* ee, S J[2][3]) {
  const double* len = p + 4;
  S phi[3];
  phi[0] = q[0];
  phi[1] = q[0] + q[1];
  phi[2] = q[0] + q[1] + q[2];
  ee[0] = 0.0;
  ee[1] = 0.0;
  for (int c = 0; c < 3; ++c) { J[0][c] = 0.0; J[1][c] = 0.0; }
  for (int j = 0; j < 3; ++j) {
    S s = std::sin(phi[j]), co = std::cos(phi[j]);
    ee[0] += len[j] * co;
    ee[1] += len[j] * s;
    for (int c = 0; c <= j; ++c) {
      J[0][c] += -len[j] * s;
      J[1][c] += len[j] * co;
    }
  }
}

template <class S>
S p3_cost(const double* p, const S* x, const S* u) {
  S ee[2], J[2][3];
  p3_ee<S>(p, x, ee, J);
  S ex = ee[0] - p[11], ey = ee[1] - p[12];
  S dx = ee[0] - p[13], dy = ee[1] - p[14];
  const double r = p[15];
  return p[7] * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + p[8] * (ex * ex + ey * ey) +
         p[10] * std::exp(-(dx * dx + dy * dy) / (r * r));
}

template <class S>
void p3_cost_grad(const double* p, const S* x, const S* u, S* lx, S* lu) {
  S ee[2], J[2][3];
  p3_ee<S>(p, x, ee, J);
  S ex = ee[0] - p[11], ey = ee[1] - p[12];
  S dx = ee[0] - p[13], dy = ee[1] - p[14];
  const double r = p[15];
  S e = p[10] * std::exp(-(dx * dx + dy * dy) / (r * r));
  // d l / d ee
  S gx = 2.0 * p[8] * ex - 2.0 * e * dx / (r * r);
  S gy = 2.0 * p[8] * ey - 2.0 * e * dy / (r * r);
  for (int c = 0; c < 3; ++c) {
    lx[c] = J[0][c] * gx + J[1][c] * gy;
    lx[3 + c] = 0.0;
    lu[c] = 2.0 * p[7] * u[c];
  }
}

template <class S>
S p3_term(const double* p, const S* x) {
  S ee[2], J[2][3];
  p3_ee<S>(p, x, ee, J);
  S ex = ee[0] - p[11], ey = ee[1] - p[12];
  return p[9] * (ex * ex + ey * ey);
}

template <class S>
void p3_term_grad(const double* p, const S* x, S* lx) {
  S ee[2], J[2][3];
  p3_ee<S>(p, x, ee, J);
  S gx = 2.0 * p[9] * (ee[0] - p[11]);
  S gy = 2.0 * p[9] * (ee[1] - p[12]);
  for (int c = 0; c < 3; ++c) {
    lx[c] = J[0][c] * gx + J[1][c] * gy;
    lx[3 + c] = 0.0;
  }
}

// ------------------------------------------------------------ synthetic quadruped
// p = [dt, w_u, w_T, w_q, w_v, A(18x18), W1(18x18), W2(18x18), e(18), x_nom(37)]
// x = (q in R^19, v in R^18), u in R^12; with qb = q[0:18]:
//   M(q) = A^T A + diag(1 + 0.1 sin qb),  b = W1 sin qb + (W2 cos qb) .* v,
//   v+ = v + dt M^-1 (S u - b),  S = [0_{12x6} I_12]^T,
//   q+ = q + dt E v+,  E = [I_18; e^T].
constexpr int QOFF_A = 5, QOFF_W1 = QOFF_A + 324, QOFF_W2 = QOFF_W1 + 324,
              QOFF_E = QOFF_W2 + 324, QOFF_XN = QOFF_E + 18;

template <class S>
void quad_dyn(const double* p, const S* x, const S* u, S* xn) {
  const double dt = p[0];
  const double* A = p + QOFF_A;
  const double* W1 = p + QOFF_W1;
  const double* W2 = p + QOFF_W2;
  const double* e = p + QOFF_E;
  const S* q = x;
  const S* v = x + 19;
  std::vector<S> M(18 * 18);
  for (int a = 0; a < 18; ++a)
    for (int b = 0; b < 18; ++b) {
      double s = 0.0;
      for (int k = 0; k < 18; ++k) s += A[k * 18 + a] * A[k * 18 + b];
      M[a * 18 + b] = s;
    }
  for (int a = 0; a < 18; ++a) M[a * 18 + a] += 1.0 + 0.1 * std::sin(q[a]);
  S rhs[18];
  for (int i = 0; i < 18; ++i) {
    S b1 = 0.0, b2 = 0.0;
    for (int j = 0; j < 18; ++j) {
      b1 += W1[i * 18 + j] * std::sin(q[j]);
      b2 += W2[i * 18 + j] * std::cos(q[j]);
    }
    S bi = b1 + b2 * v[i];
    S su = (i >= 6) ? u[i - 6] : S(0.0);
    rhs[i] = su - bi;
  }
  gauss_solve<S>(18, M, rhs, 1);
  S last = 0.0;
  for (int i = 0; i < 18; ++i) {
    xn[19 + i] = v[i] + dt * rhs[i];
    xn[i] = q[i] + dt * xn[19 + i];
    last += e[i] * xn[19 + i];
  }
  xn[18] = q[18] + dt * last;
}

template <class S>
S quad_track(const double* p, const S* x) {
  const double* xn = p + QOFF_XN;
  S sq = 0.0, sv = 0.0;
  for (int i = 0; i < 19; ++i) sq += (x[i] - xn[i]) * (x[i] - xn[i]);
  for (int i = 19; i < 37; ++i) sv += (x[i] - xn[i]) * (x[i] - xn[i]);
  return p[3] * sq + p[4] * sv;
}

template <class S>
S quad_cost(const double* p, const S* x, const S* u) {
  S su = 0.0;
  for (int i = 0; i < 12; ++i) su += u[i] * u[i];
  return quad_track<S>(p, x) + p[1] * su;
}

template <class S>
void quad_cost_grad(const double* p, const S* x, const S* u, S* lx, S* lu) {
  const double* xn = p + QOFF_XN;
  for (int i = 0; i < 37; ++i) lx[i] = 2.0 * (i < 19 ? p[3] : p[4]) * (x[i] - xn[i]);
  for (int i = 0; i < 12; ++i) lu[i] = 2.0 * p[1] * u[i];
}

template <class S>
S quad_term(const double* p, const S* x) { return p[2] * quad_track<S>(p, x); }

template <class S>
void quad_term_grad(const double* p, const S* x, S* lx) {
  const double* xn = p + QOFF_XN;
  for (int i = 0; i < 37; ++i) lx[i] = 2.0 * p[2] * (i < 19 ? p[3] : p[4]) * (x[i] - xn[i]);
}

// ------------------------------------------------------------ linear-quadratic
// p = [n, m, A(nxn), B(nxm), Q(nxn), R(mxm), Q_T(nxn), x_ref(n)]
// f = A x + B u, l = (x-x_ref)^T Q (x-x_ref) + u^T R u, l_T with Q_T.
template <class S>
void lq_dyn(const Sys& s, const S* x, const S* u, S* xn) {
  for (int i = 0; i < s.n; ++i) {
    S v = 0.0;
    for (int j = 0; j < s.n; ++j) v += s.A[i * s.n + j] * x[j];
    for (int j = 0; j < s.m; ++j) v += s.B[i * s.m + j] * u[j];
    xn[i] = v;
  }
}

template <class S>
S quadform(int n, const double* Q, const S* a) {
  S v = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) v += a[i] * Q[i * n + j] * a[j];
  return v;
}

template <class S>
S lq_cost(const Sys& s, const S* x, const S* u) {
  std::vector<S> d(s.n);
  for (int i = 0; i < s.n; ++i) d[i] = x[i] - s.xr[i];
  return quadform<S>(s.n, s.Q, d.data()) + quadform<S>(s.m, s.R, u);
}

template <class S>
void lq_cost_grad(const Sys& s, const S* x, const S* u, S* lx, S* lu) {
  for (int i = 0; i < s.n; ++i) {
    S v = 0.0;
    for (int j = 0; j < s.n; ++j) v += (s.Q[i * s.n + j] + s.Q[j * s.n + i]) * (x[j] - s.xr[j]);
    lx[i] = v;
  }
  for (int i = 0; i < s.m; ++i) {
    S v = 0.0;
    for (int j = 0; j < s.m; ++j) v += (s.R[i * s.m + j] + s.R[j * s.m + i]) * u[j];
    lu[i] = v;
  }
}

template <class S>
S lq_term(const Sys& s, const S* x) {
  std::vector<S> d(s.n);
  for (int i = 0; i < s.n; ++i) d[i] = x[i] - s.xr[i];
  return quadform<S>(s.n, s.QT, d.data());
}

template <class S>
void lq_term_grad(const Sys& s, const S* x, S* lx) {
  for (int i = 0; i < s.n; ++i) {
    S v = 0.0;
    for (int j = 0; j < s.n; ++j) v += (s.QT[i * s.n + j] + s.QT[j * s.n + i]) * (x[j] - s.xr[j]);
    lx[i] = v;
  }
}

// ------------------------------------------------------------ dispatch
bool make_sys(int kind, const double* p, int np, Sys* s) {
  s->kind = kind;
  s->p = p;
  switch (kind) {
    case KIND_PM:
      if (np != 16) return false;
      s->n = 4; s->m = 2;
      return true;
    case KIND_P3:
      if (np != 16) return false;
      s->n = 6; s->m = 3;
      return true;
    case KIND_QUAD:
      if (np != QOFF_XN + 37) return false;
      s->n = 37; s->m = 12;
      return true;
    case KIND_LQ: {
      if (np < 2) return false;
      int n = (int)p[0], m = (int)p[1];
      if (n < 1 || m < 1 || n > 64 || m > 64) return false;
      if (np != 2 + 3 * n * n + n * m + m * m + n) return false;
      s->n = n; s->m = m;
      const double* c = p + 2;
      s->A = c; c += n * n;
      s->B = c; c += n * m;
      s->Q = c; c += n * n;
      s->R = c; c += m * m;
      s->QT = c; c += n * n;
      s->xr = c;
      return true;
    }
    default:
      return false;
  }
}

template <class S>
void dyn(const Sys& s, const S* x, const S* u, S* xn) {
  switch (s.kind) {
    case KIND_PM: pm_dyn<S>(s.p, x, u, xn); break;
    case KIND_P3: p3_dyn<S>(s.p, x, u, xn); break;
    case KIND_QUAD: quad_dyn<S>(s.p, x, u, xn); break;
    default: lq_dyn<S>(s, x, u, xn); break;
  }
}

template <class S>
S cost(const Sys& s, const S* x, const S* u) {
  switch (s.kind) {
    case KIND_PM: return pm_cost<S>(s.p, x, u);
    case KIND_P3: return p3_cost<S>(s.p, x, u);
    case KIND_QUAD: return quad_cost<S>(s.p, x, u);
    default: return lq_cost<S>(s, x, u);
  }
}

template <class S>
void cost_grad(const Sys& s, const S* x, const S* u, S* lx, S* lu) {
  switch (s.kind) {
    case KIND_PM: pm_cost_grad<S>(s.p, x, u, lx, lu); break;
    case KIND_P3: p3_cost_grad<S>(s.p, x, u, lx, lu); break;
    case KIND_QUAD: quad_cost_grad<S>(s.p, x, u, lx, lu); break;
    default: lq_cost_grad<S>(s, x, u, lx, lu); break;
  }
}

template <class S>
S term(const Sys& s, const S* x) {
  switch (s.kind) {
    case KIND_PM: return pm_term<S>(s.p, x);
    case KIND_P3: return p3_term<S>(s.p, x);
    case KIND_QUAD: return quad_term<S>(s.p, x);
    default: return lq_term<S>(s, x);
  }
}

template <class S>
void term_grad(const Sys& s, const S* x, S* lx) {
  switch (s.kind) {
    case KIND_PM: pm_term_grad<S>(s.p, x, lx); break;
    case KIND_P3: p3_term_grad<S>(s.p, x, lx); break;
    case KIND_QUAD: quad_term_grad<S>(s.p, x, lx); break;
    default: lq_term_grad<S>(s, x, lx); break;
  }
}

// ------------------------------------------------------------ derivatives
// Complex step: d f / d z_j = Im f(z + i h e_j) / h, exact to rounding for
// analytic f (no subtractive cancellation).
constexpr double CS_H = 1e-30;

void dyn_jac(const Sys& s, const double* x, const double* u, double* A, double* B) {
  const int n = s.n, m = s.m;
  std::vector<cd> xc(n), uc(m), out(n);
  for (int i = 0; i < n; ++i) xc[i] = x[i];
  for (int i = 0; i < m; ++i) uc[i] = u[i];
  for (int j = 0; j < n; ++j) {
    xc[j] = cd(x[j], CS_H);
    dyn<cd>(s, xc.data(), uc.data(), out.data());
    for (int i = 0; i < n; ++i) A[i * n + j] = out[i].imag() / CS_H;
    xc[j] = x[j];
  }
  for (int j = 0; j < m; ++j) {
    uc[j] = cd(u[j], CS_H);
    dyn<cd>(s, xc.data(), uc.data(), out.data());
    for (int i = 0; i < n; ++i) B[i * m + j] = out[i].imag() / CS_H;
    uc[j] = u[j];
  }
}

// First and second cost derivatives: lx, lu analytic; lxx, luu, lux by
// complex step of the analytic gradient.  lux is m x n.
void cost_derivs(const Sys& s, const double* x, const double* u, double* lx, double* lu,
                 double* lxx, double* luu, double* lux) {
  const int n = s.n, m = s.m;
  cost_grad<double>(s, x, u, lx, lu);
  std::vector<cd> xc(n), uc(m), gx(n), gu(m);
  for (int i = 0; i < n; ++i) xc[i] = x[i];
  for (int i = 0; i < m; ++i) uc[i] = u[i];
  for (int j = 0; j < n; ++j) {
    xc[j] = cd(x[j], CS_H);
    cost_grad<cd>(s, xc.data(), uc.data(), gx.data(), gu.data());
    for (int i = 0; i < n; ++i) lxx[i * n + j] = gx[i].imag() / CS_H;
    for (int i = 0; i < m; ++i) lux[i * n + j] = gu[i].imag() / CS_H;
    xc[j] = x[j];
  }
  for (int j = 0; j < m; ++j) {
    uc[j] = cd(u[j], CS_H);
    cost_grad<cd>(s, xc.data(), uc.data(), gx.data(), gu.data());
    for (int i = 0; i < m; ++i) luu[i * m + j] = gu[i].imag() / CS_H;
    uc[j] = u[j];
  }
}

void term_derivs(const Sys& s, const double* x, double* lx, double* lxx) {
  const int n = s.n;
  term_grad<double>(s, x, lx);
  std::vector<cd> xc(n), gx(n);
  for (int i = 0; i < n; ++i) xc[i] = x[i];
  for (int j = 0; j < n; ++j) {
    xc[j] = cd(x[j], CS_H);
    term_grad<cd>(s, xc.data(), gx.data());
    for (int i = 0; i < n; ++i) lxx[i * n + j] = gx[i].imag() / CS_H;
    xc[j] = x[j];
  }
}

// ------------------------------------------------------------ eigenvalue clipping (eq. 7)
// Cyclic Jacobi eigen-decomposition of a symmetric matrix: H = W diag(S) W^T.
void jacobi_eig(int n, const double* H, double* S, double* W) {
  std::vector<double> a(H, H + n * n);
  for (int i = 0; i < n * n; ++i) W[i] = 0.0;
  for (int i = 0; i < n; ++i) W[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a[i * n + j] * a[i * n + j];
        if (i != j) off += a[i * n + j] * a[i * n + j];
      }
    if (off == 0.0 || off <= 1e-32 * tot) break;
    for (int pi = 0; pi < n - 1; ++pi)
      for (int qi = pi + 1; qi < n; ++qi) {
        const double apq = a[pi * n + qi];
        if (apq == 0.0) continue;
        const double app = a[pi * n + pi], aqq = a[qi * n + qi];
        // rotation angle that zeroes a_pq (symmetric Schur decomposition)
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        for (int k = 0; k < n; ++k) {  // a <- a J   (columns p, q)
          const double akp = a[k * n + pi], akq = a[k * n + qi];
          a[k * n + pi] = c * akp - sn * akq;
          a[k * n + qi] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // a <- J^T a (rows p, q)
          const double apk = a[pi * n + k], aqk = a[qi * n + k];
          a[pi * n + k] = c * apk - sn * aqk;
          a[qi * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // W <- W J
          const double wkp = W[k * n + pi], wkq = W[k * n + qi];
          W[k * n + pi] = c * wkp - sn * wkq;
          W[k * n + qi] = sn * wkp + c * wkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) S[i] = a[i * n + i];
}

// Q_psd = sym(W diag(max(S, eps)) W^T) for the symmetric part of H.
void psd_clip(int n, const double* H, double eps, double* out) {
  std::vector<double> Hs(n * n), S(n), W(n * n), Qp(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Hs[i * n + j] = 0.5 * (H[i * n + j] + H[j * n + i]);
  jacobi_eig(n, Hs.data(), S.data(), W.data());
  for (int i = 0; i < n; ++i) S[i] = std::max(S[i], eps);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += W[i * n + k] * S[k] * W[j * n + k];
      Qp[i * n + j] = v;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[i * n + j] = 0.5 * (Qp[i * n + j] + Qp[j * n + i]);
}

// ------------------------------------------------------------ Cholesky of Q_uu
// Lower-triangular L with L L^T = A; false on a non-positive or non-finite pivot.
bool cholesky(int m, const double* A, double* L) {
  for (int i = 0; i < m * m; ++i) L[i] = 0.0;
  for (int j = 0; j < m; ++j) {
    double d = A[j * m + j];
    for (int k = 0; k < j; ++k) d -= L[j * m + k] * L[j * m + k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    const double ljj = std::sqrt(d);
    L[j * m + j] = ljj;
    for (int i = j + 1; i < m; ++i) {
      double v = A[i * m + j];
      for (int k = 0; k < j; ++k) v -= L[i * m + k] * L[j * m + k];
      L[i * m + j] = v / ljj;
    }
  }
  return true;
}

// Solve (L L^T) X = Bm for nrhs columns; Bm is m x nrhs row-major, overwritten.
void chol_solve(int m, const double* L, double* Bm, int nrhs) {
  for (int c = 0; c < nrhs; ++c) {
    for (int i = 0; i < m; ++i) {
      double v = Bm[i * nrhs + c];
      for (int k = 0; k < i; ++k) v -= L[i * m + k] * Bm[k * nrhs + c];
      Bm[i * nrhs + c] = v / L[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
      double v = Bm[i * nrhs + c];
      for (int k = i + 1; k < m; ++k) v -= L[k * m + i] * Bm[k * nrhs + c];
      Bm[i * nrhs + c] = v / L[i * m + i];
    }
  }
}

// ------------------------------------------------------------ control bound
// Bounded control step (eq. 1 keeps every control in [-u_max, u_max]): the
// minimiser d of 0.5 d'Hd + g'd subject to lo <= d <= hi, H symmetric
// positive definite (m x m, row-major), by the primal active-set method.
// On entry d holds the unconstrained minimiser -H^-1 g.  If it lies in the
// box it is the answer.  Otherwise its out-of-box components are clamped and
// held at their bounds (the working set), and the method alternates:
//  - if d is not yet the minimiser over the free components with the held
//    ones fixed (the face), compute that minimiser y and move from d towards
//    it until a free component meets a bound (the first such, lowest index on
//    ties, joins the working set) or, if none does, up to y;
//  - if d is the face's minimiser, compute the multiplier of every held
//    component (its gradient g + H d, with the sign flipped at an upper
//    bound); release the most negative one (lowest index on ties), or stop
//    when none is negative: d then satisfies the optimality conditions.
// At most 4m + 4 such steps are taken (a strictly convex problem needs fewer;
// d stays feasible either way).  held[i] = 1 for the components held at the
// end.  Returns false when a face's block of H cannot be factorised.
bool face_factor(int m, const double* H, const std::vector<char>& held, std::vector<int>& F,
                 std::vector<double>& LF) {
  F.clear();
  for (int i = 0; i < m; ++i)
    if (!held[i]) F.push_back(i);
  const int f = (int)F.size();
  std::vector<double> HF(f * f);
  for (int a = 0; a < f; ++a)
    for (int b = 0; b < f; ++b) HF[a * f + b] = H[F[a] * m + F[b]];
  LF.assign(f * f, 0.0);
  return f == 0 || cholesky(f, HF.data(), LF.data());
}

bool box_qp(int m, const double* H, const double* g, const double* lo, const double* hi, double* d,
            std::vector<char>& held) {
  held.assign(m, 0);
  bool inside = true;
  for (int i = 0; i < m; ++i) {
    if (std::isnan(d[i])) return true;  // reported by the caller's finiteness check
    inside = inside && d[i] >= lo[i] && d[i] <= hi[i];
  }
  if (inside) return true;
  std::vector<char> upper(m, 0);
  for (int i = 0; i < m; ++i) {
    if (d[i] < lo[i]) {
      d[i] = lo[i];
      held[i] = 1;
    } else if (d[i] > hi[i]) {
      d[i] = hi[i];
      held[i] = 1;
      upper[i] = 1;
    }
  }
  std::vector<int> F;
  std::vector<double> LF, y;
  bool at_min = false;
  for (int step = 0; step < 4 * m + 4; ++step) {
    if (!at_min) {
      if (!face_factor(m, H, held, F, LF)) return false;
      const int f = (int)F.size();
      if (f == 0) {
        at_min = true;
        continue;
      }
      // face minimiser: H_FF y_F = -(g_F + H_FW d_W)
      y.assign(f, 0.0);
      for (int a = 0; a < f; ++a) {
        double v = g[F[a]];
        for (int j = 0; j < m; ++j)
          if (held[j]) v += H[F[a] * m + j] * d[j];
        y[a] = -v;
      }
      chol_solve(f, LF.data(), y.data(), 1);
      double t_best = 1.0;
      int blocking = -1;
      bool blocking_upper = false;
      for (int a = 0; a < f; ++a) {
        const int i = F[a];
        const double dir = y[a] - d[i];
        double t = INFINITY;
        if (dir < 0.0) t = (lo[i] - d[i]) / dir;
        else if (dir > 0.0) t = (hi[i] - d[i]) / dir;
        if (t < t_best) {
          t_best = t;
          blocking = i;
          blocking_upper = dir > 0.0;
        }
      }
      if (blocking < 0) {
        for (int a = 0; a < f; ++a) d[F[a]] = y[a];
        at_min = true;
      } else {
        for (int a = 0; a < f; ++a) {
          const int i = F[a];
          if (i == blocking) continue;
          const double v = d[i] + t_best * (y[a] - d[i]);
          d[i] = v < lo[i] ? lo[i] : (v > hi[i] ? hi[i] : v);
        }
        d[blocking] = blocking_upper ? hi[blocking] : lo[blocking];
        held[blocking] = 1;
        upper[blocking] = blocking_upper;
      }
    } else {
      int release = -1;
      double most_negative = 0.0;
      for (int i = 0; i < m; ++i) {
        if (!held[i]) continue;
        double gr = g[i];
        for (int j = 0; j < m; ++j) gr += H[i * m + j] * d[j];
        const double mult = upper[i] ? -gr : gr;
        if (mult < most_negative) {
          most_negative = mult;
          release = i;
        }
      }
      if (release < 0) break;
      held[release] = 0;
      at_min = false;
    }
  }
  return true;
}

// ------------------------------------------------------------ one instance
struct Opts {
  int32_t max_iter;
  int32_t ls_trials;
  int32_t stop_mode;  // 0 fixed iterations, 1 relative-decrease tolerance
  int32_t lookahead;  // K of the K-step cost-to-go; <= 0 means the horizon
  double eps;
  double beta;
  double rtol;
  // regularization (Sec. IV-B): 0 eigenvalue clip (eq. 7); 1 Levenberg-Marquardt:
  // Hessians only symmetrised, Q_uu + mu I, mu raised by mu_factor and the
  // backward pass retried after a failed Cholesky or line search (up to
  // mu_max), lowered by mu_factor (not below mu0) after an accepted step
  int32_t reg;
  double mu0, mu_factor, mu_max;
  // control bound |u_k,i| <= umax (eq. 1); infinite: none
  double umax;
  // sensitivity probe, off by default: 1 rounds every quantity that the
  // mixed-precision form keeps in FP32 to FP32 where it is produced (see
  // solve_one); the arithmetic itself stays FP64
  int32_t round32;
};

// v rounded to FP32 and back when `on`
inline void to_f32(double* v, int len, bool on) {
  if (on)
    for (int i = 0; i < len; ++i) v[i] = (double)(float)v[i];
}

// the symmetric part of H (no clipping)
void sym_part(int n, const double* H, double* out) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[i * n + j] = 0.5 * (H[i * n + j] + H[j * n + i]);
}

bool all_finite(const double* v, int k) {
  for (int i = 0; i < k; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// J = sum_{k<T} l(x_k,u_k) + l_T(x_T), summed in index order; X = rollout of U.
double rollout(const Sys& s, int T, const double* x0, const double* U, double* X, bool r32 = false) {
  const int n = s.n, m = s.m;
  for (int i = 0; i < n; ++i) X[i] = x0[i];
  double J = 0.0;
  for (int k = 0; k < T; ++k) {
    J += cost<double>(s, X + k * n, U + k * m);
    dyn<double>(s, X + k * n, U + k * m, X + (k + 1) * n);
    to_f32(X + (k + 1) * n, n, r32);
  }
  J += term<double>(s, X + T * n);
  return J;
}

// Costate lambda_k = l_x + A_k^T lambda_{k+1} (lambda_T = d l_T / dx) and the
// control gradient g_k = l_u + B_k^T lambda_{k+1} of J along (X, U).
void costate(const Sys& s, int T, const double* X, const double* U, double* lam, double* g) {
  const int n = s.n, m = s.m;
  std::vector<double> A(n * n), B(n * m), lx(n), lu(m), lxx(n * n), luu(m * m), lux(m * n);
  term_grad<double>(s, X + T * n, lam + T * n);
  for (int k = T - 1; k >= 0; --k) {
    dyn_jac(s, X + k * n, U + k * m, A.data(), B.data());
    cost_grad<double>(s, X + k * n, U + k * m, lx.data(), lu.data());
    const double* ln = lam + (k + 1) * n;
    for (int i = 0; i < n; ++i) {
      double v = lx[i];
      for (int j = 0; j < n; ++j) v += A[j * n + i] * ln[j];
      lam[k * n + i] = v;
    }
    if (g)
      for (int i = 0; i < m; ++i) {
        double v = lu[i];
        for (int j = 0; j < n; ++j) v += B[j * m + i] * ln[j];
        g[k * m + i] = v;
      }
  }
}

// Critic targets of one trajectory (X, U): stage costs c_k and c_T, the
// K-step partial cost-to-go V_k = sum_{j=k}^{min(k+K,T)-1} c_j + [k+K >= T] c_T
// summed in index order, its gradient V_x,k = lambda_k (costate of the full
// tail cost), and x_{min(k+K,T)}.
void extract(const Sys& s, int T, const double* X, const double* U, int lookahead, double* Vbar, double* Vx,
             double* xK) {
  const int n = s.n, m = s.m;
  const int K = (lookahead <= 0) ? T : lookahead;
  if (Vbar) {
    std::vector<double> c(T + 1);
    for (int k = 0; k < T; ++k) c[k] = cost<double>(s, X + k * n, U + k * m);
    c[T] = term<double>(s, X + T * n);
    for (int k = 0; k <= T; ++k) {
      const int end = std::min(k + K, T);
      double v = 0.0;
      for (int t = k; t < end; ++t) v += c[t];
      if (k + K >= T) v += c[T];
      Vbar[k] = v;
    }
  }
  if (Vx) costate(s, T, X, U, Vx, nullptr);
  if (xK)
    for (int k = 0; k <= T; ++k) {
      const int t = std::min(k + K, T);
      for (int i = 0; i < n; ++i) xK[k * n + i] = X[t * n + i];
    }
}

struct Out {
  double* X;       // (T+1) x n
  double* U;       // T x m
  double* J;
  int32_t* iters;
  uint32_t* status;
  double* trace;   // max_iter+1 or null
  int32_t* jtrace; // max_iter or null: accepted j per iteration, -1 no step, -2 not run
  double* margin;  // max_iter or null: min over tried j of |J_hat - J| / |J|
  double* Vbar;    // T+1 or null
  double* Vx;      // (T+1) x n or null
  double* xK;      // (T+1) x n or null
  const int32_t* force_j;  // max_iter or null: replay these accepted j (-1 = none)
};

void solve_one(const Sys& s, int T, const double* x0_in, const double* U0, const Opts& o, Out r) {
  const int n = s.n, m = s.m;
  std::vector<double> X((T + 1) * n), U(T * m, 0.0), Xn((T + 1) * n), Un(T * m);
  std::vector<double> Kg(T * m * n), kf(T * m);
  if (U0) std::memcpy(U.data(), U0, sizeof(double) * T * m);
  const bool bounded = std::isfinite(o.umax);
  // controls are kept in [-umax, umax], the warm start included (NaN stays)
  auto clamp_u = [&](double v) { return v < -o.umax ? -o.umax : (v > o.umax ? o.umax : v); };
  if (bounded)
    for (auto& v : U) v = clamp_u(v);
  // the FP32-storage probe (round32): the initial state, the warm start, every
  // rolled-out state and control, the derivative blocks, the clipped Hessians,
  // P and p after each backward step and the gains are rounded to FP32
  const bool r32 = o.round32 != 0;
  std::vector<double> x0v(x0_in, x0_in + n);
  to_f32(x0v.data(), n, r32);
  to_f32(U.data(), T * m, r32);
  const double* x0 = x0v.data();
  double J = rollout(s, T, x0, U.data(), X.data(), r32);
  uint32_t status = 0;
  int iters = 0;
  bool frozen = false;
  if (!std::isfinite(J)) {
    status |= ST_NONFINITE;
    frozen = true;
  }
  if (r.trace) r.trace[0] = J;
  if (r.jtrace) for (int i = 0; i < o.max_iter; ++i) r.jtrace[i] = -2;
  if (r.margin) for (int i = 0; i < o.max_iter; ++i) r.margin[i] = INFINITY;

  std::vector<double> A(n * n), B(n * m), lx(n), lu(m), lxx(n * n), luu(m * m), lux(m * n);
  std::vector<double> Qc(n * n), Rc(m * m), P(n * n), p(n), PA(n * n), PB(n * m);
  std::vector<double> Qx(n), Qu(m), Qxx(n * n), Quu(m * m), Qux(m * n), L(m * m), rhs(m * (n + 1));
  std::vector<double> lo(m), hi(m), LF;
  std::vector<char> held;
  std::vector<int> F;

  const bool lm = o.reg == 1;
  double mu = o.mu0;

  // backward Riccati sweep about (X, U) with Levenberg-Marquardt parameter mu
  // (used only when lm); fills the gains Kg, kf; returns 0 or the failure's
  // status bit
  auto sweep = [&](double mu_) -> uint32_t {
    term_derivs(s, X.data() + T * n, p.data(), lxx.data());
    if (lm) sym_part(n, lxx.data(), P.data());
    else psd_clip(n, lxx.data(), o.eps, P.data());
    to_f32(p.data(), n, r32);
    to_f32(P.data(), n * n, r32);
    for (int k = T - 1; k >= 0; --k) {
      const double* xk = X.data() + k * n;
      const double* uk = U.data() + k * m;
      dyn_jac(s, xk, uk, A.data(), B.data());
      cost_derivs(s, xk, uk, lx.data(), lu.data(), lxx.data(), luu.data(), lux.data());
      to_f32(A.data(), n * n, r32);
      to_f32(B.data(), n * m, r32);
      to_f32(lx.data(), n, r32);
      to_f32(lu.data(), m, r32);
      if (lm) {
        sym_part(n, lxx.data(), Qc.data());
        sym_part(m, luu.data(), Rc.data());
      } else {
        psd_clip(n, lxx.data(), o.eps, Qc.data());
        psd_clip(m, luu.data(), o.eps, Rc.data());
      }
      to_f32(Qc.data(), n * n, r32);
      to_f32(Rc.data(), m * m, r32);
      // PA = P A, PB = P B
      for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
          double v = 0.0;
          for (int t = 0; t < n; ++t) v += P[i * n + t] * A[t * n + j];
          PA[i * n + j] = v;
        }
        for (int j = 0; j < m; ++j) {
          double v = 0.0;
          for (int t = 0; t < n; ++t) v += P[i * n + t] * B[t * m + j];
          PB[i * m + j] = v;
        }
      }
      for (int i = 0; i < n; ++i) {  // Q_x = l_x + A^T p ; Q_xx = Q + A^T P A
        double v = lx[i];
        for (int t = 0; t < n; ++t) v += A[t * n + i] * p[t];
        Qx[i] = v;
        for (int j = 0; j < n; ++j) {
          double w = Qc[i * n + j];
          for (int t = 0; t < n; ++t) w += A[t * n + i] * PA[t * n + j];
          Qxx[i * n + j] = w;
        }
      }
      for (int i = 0; i < m; ++i) {  // Q_u, Q_uu = R + B^T P B, Q_ux = l_ux + B^T P A
        double v = lu[i];
        for (int t = 0; t < n; ++t) v += B[t * m + i] * p[t];
        Qu[i] = v;
        for (int j = 0; j < m; ++j) {
          double w = Rc[i * m + j];
          for (int t = 0; t < n; ++t) w += B[t * m + i] * PB[t * m + j];
          Quu[i * m + j] = w;
        }
        for (int j = 0; j < n; ++j) {
          double w = lux[i * n + j];
          for (int t = 0; t < n; ++t) w += B[t * m + i] * PA[t * n + j];
          Qux[i * n + j] = w;
        }
      }
      if (lm)
        for (int i = 0; i < m; ++i) Quu[i * m + i] += mu_;
      if (!cholesky(m, Quu.data(), L.data())) return ST_CHOL_FAIL;
      // [K k] = -Q_uu^-1 [Q_ux Q_u]
      for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j) rhs[i * (n + 1) + j] = Qux[i * n + j];
        rhs[i * (n + 1) + n] = Qu[i];
      }
      chol_solve(m, L.data(), rhs.data(), n + 1);
      double* Kk = Kg.data() + k * m * n;
      double* kk = kf.data() + k * m;
      for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j) Kk[i * n + j] = -rhs[i * (n + 1) + j];
        kk[i] = -rhs[i * (n + 1) + n];
      }
      if (bounded) {
        // the step minimises the local model over the box u_k + d in
        // [-umax, umax]; held components get no feedback, the free ones the
        // feedback of their block of Q_uu
        for (int i = 0; i < m; ++i) {
          lo[i] = -o.umax - uk[i];
          hi[i] = o.umax - uk[i];
        }
        if (!box_qp(m, Quu.data(), Qu.data(), lo.data(), hi.data(), kk, held)) return ST_CHOL_FAIL;
        bool any = false;
        for (int i = 0; i < m; ++i) any = any || held[i];
        if (any) {
          if (!face_factor(m, Quu.data(), held, F, LF)) return ST_CHOL_FAIL;
          const int f = (int)F.size();
          std::vector<double> col(f);
          for (int j = 0; j < n; ++j) {
            for (int a = 0; a < f; ++a) col[a] = Qux[F[a] * n + j];
            if (f) chol_solve(f, LF.data(), col.data(), 1);
            for (int i = 0; i < m; ++i) Kk[i * n + j] = 0.0;
            for (int a = 0; a < f; ++a) Kk[F[a] * n + j] = -col[a];
          }
        }
      }
      if (!all_finite(Kk, m * n) || !all_finite(kk, m)) return ST_NONFINITE;
      // P = sym(Q_xx + Q_ux^T K), p = Q_x + Q_ux^T k
      for (int i = 0; i < n; ++i) {
        double v = Qx[i];
        for (int t = 0; t < m; ++t) v += Qux[t * n + i] * kk[t];
        p[i] = v;
        for (int j = 0; j < n; ++j) {
          double w = Qxx[i * n + j];
          for (int t = 0; t < m; ++t) w += Qux[t * n + i] * Kk[t * n + j];
          PA[i * n + j] = w;  // reuse as scratch
        }
      }
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) P[i * n + j] = 0.5 * (PA[i * n + j] + PA[j * n + i]);
      to_f32(Kk, m * n, r32);
      to_f32(kk, m, r32);
      to_f32(p.data(), n, r32);
      to_f32(P.data(), n * n, r32);
    }
    return 0u;
  };

  // backtracking line search of iteration it: returns the accepted j (or -1)
  // and the trial's cost in Jnew, the trial trajectory in (Xn, Un)
  auto line_search = [&](int it, double& Jnew) -> int {
    int accepted = -1;
    double alpha = 1.0;
    double margin = INFINITY;
    const int jmax = o.ls_trials;
    for (int j = 0; j < jmax; ++j) {
      if (r.force_j && r.force_j[it] >= 0 && j != r.force_j[it]) {
        alpha *= o.beta;
        continue;
      }
      if (r.force_j && r.force_j[it] < 0) break;
      for (int i = 0; i < n; ++i) Xn[i] = X[i];
      double Jh = 0.0;
      for (int k = 0; k < T; ++k) {
        const double* Kk = Kg.data() + k * m * n;
        const double* kk = kf.data() + k * m;
        for (int i = 0; i < m; ++i) {
          double v = U[k * m + i] + alpha * kk[i];
          for (int t = 0; t < n; ++t) v += Kk[i * n + t] * (Xn[k * n + t] - X[k * n + t]);
          Un[k * m + i] = bounded ? clamp_u(v) : v;
        }
        to_f32(Un.data() + k * m, m, r32);
        Jh += cost<double>(s, Xn.data() + k * n, Un.data() + k * m);
        dyn<double>(s, Xn.data() + k * n, Un.data() + k * m, Xn.data() + (k + 1) * n);
        to_f32(Xn.data() + (k + 1) * n, n, r32);
      }
      Jh += term<double>(s, Xn.data() + T * n);
      if (std::isfinite(Jh)) margin = std::min(margin, std::fabs(Jh - J) / std::max(std::fabs(J), 1e-300));
      const bool take = r.force_j ? std::isfinite(Jh) : (std::isfinite(Jh) && Jh < J);
      if (take) {
        accepted = j;
        Jnew = Jh;
        break;
      }
      alpha *= o.beta;
    }
    if (r.margin) r.margin[it] = margin;
    if (r.jtrace) r.jtrace[it] = accepted;
    return accepted;
  };

  for (int it = 0; it < o.max_iter && !frozen; ++it) {
    // one sweep and line search; the Levenberg-Marquardt variant raises mu and
    // retries after a failed Cholesky or line search while mu stays <= mu_max
    double Jnew = J;
    uint32_t fail = 0;
    for (;;) {
      const uint32_t bad = sweep(mu);
      if (bad) {
        if (lm && bad == ST_CHOL_FAIL && mu * o.mu_factor <= o.mu_max) {
          mu *= o.mu_factor;
          continue;
        }
        fail = bad;
        if (r.jtrace) r.jtrace[it] = -1;
        break;
      }
      if (line_search(it, Jnew) < 0) {
        if (lm && mu * o.mu_factor <= o.mu_max) {
          mu *= o.mu_factor;
          continue;
        }
        fail = ST_LS_FAILED;
      }
      break;
    }
    if (fail) {
      status |= fail;
      frozen = true;
      break;
    }
    if (lm) mu = std::max(mu / o.mu_factor, o.mu0);
    X.swap(Xn);
    U.swap(Un);
    const double Jold = J;
    J = Jnew;
    ++iters;
    if (r.trace) r.trace[it + 1] = J;
    if (o.stop_mode == 1 && (Jold - J) <= o.rtol * std::fabs(Jold)) {
      status |= ST_CONVERGED;
      frozen = true;
      break;
    }
  }
  if (!frozen) status |= ST_MAX_ITER;
  if (r.trace)
    for (int i = iters + 1; i <= o.max_iter; ++i) r.trace[i] = J;

  std::memcpy(r.X, X.data(), sizeof(double) * (T + 1) * n);
  std::memcpy(r.U, U.data(), sizeof(double) * T * m);
  *r.J = J;
  *r.iters = iters;
  *r.status = status;

  extract(s, T, X.data(), U.data(), o.lookahead, r.Vbar, r.Vx, r.xK);
}

thread_local char g_err[256];

}  // namespace

extern "C" {

struct orc_opts {
  int32_t max_iter;
  int32_t ls_trials;
  int32_t stop_mode;
  int32_t lookahead;
  double eps;
  double beta;
  double rtol;
  int32_t reg;
  double mu0, mu_factor, mu_max;
  double umax;
  int32_t round32;
};

const char* orc_last_error() { return g_err; }

int orc_dims(int kind, const double* p, int np, int* n, int* m) {
  Sys s;
  if (!make_sys(kind, p, np, &s)) return -1;
  *n = s.n;
  *m = s.m;
  return 0;
}

int orc_dyn(int kind, const double* p, int np, const double* x, const double* u, double* xn) {
  Sys s;
  if (!make_sys(kind, p, np, &s)) return -1;
  dyn<double>(s, x, u, xn);
  return 0;
}

int orc_dyn_jac(int kind, const double* p, int np, const double* x, const double* u, double* A,
                double* B) {
  Sys s;
  if (!make_sys(kind, p, np, &s)) return -1;
  dyn_jac(s, x, u, A, B);
  return 0;
}

int orc_cost(int kind, const double* p, int np, const double* x, const double* u, double* l) {
  Sys s;
  if (!make_sys(kind, p, np, &s)) return -1;
  *l = cost<double>(s, x, u);
  return 0;
}

int orc_cost_derivs(int kind, const double* p, int np, const double* x, const double* u,
                    double* lx, double* lu, double* lxx, double* luu, double* lux) {
  Sys s;
  if (!make_sys(kind, p, np, &s)) return -1;
  cost_derivs(s, x, u, lx, lu, lxx, luu, lux);
  return 0;
}

int orc_term(int kind, const double* p, int np, const double* x, double* l) {
  Sys s;
  if (!make_sys(kind, p, np, &s)) return -1;
  *l = term<double>(s, x);
  return 0;
}

int orc_term_derivs(int kind, const double* p, int np, const double* x, double* lx, double* lxx) {
  Sys s;
  if (!make_sys(kind, p, np, &s)) return -1;
  term_derivs(s, x, lx, lxx);
  return 0;
}

// Bounded control step (see box_qp): d in/out, held[m] out.
int orc_box_qp(int m, const double* H, const double* g, const double* lo, const double* hi, double* d,
               int32_t* held_out) {
  if (m < 1) return -1;
  std::vector<char> held;
  if (!box_qp(m, H, g, lo, hi, d, held)) return 1;
  for (int i = 0; i < m; ++i) held_out[i] = held[i];
  return 0;
}

int orc_psd_clip(int n, const double* H, double eps, double* out) {
  if (n < 1) return -1;
  psd_clip(n, H, eps, out);
  return 0;
}

int orc_eig(int n, const double* H, double* S, double* W) {
  if (n < 1) return -1;
  jacobi_eig(n, H, S, W);
  return 0;
}

int orc_p3_mass(const double* p, const double* q, double* M) {
  double Mm[3][3], dM[3][3][3];
  p3_mass<double>(p, q, Mm, dM);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) M[a * 3 + b] = Mm[a][b];
  return 0;
}

int orc_p3_ee(const double* p, const double* q, double* ee) {
  double J[2][3];
  p3_ee<double>(p, q, ee, J);
  return 0;
}

// ------------------------------------------------------------ networks
// The perceptron of the biased initial-state selection and the actor warm
// start (paper Sec. II, III): depth hidden layers of `width` units with
// activation act (0 tanh, 1 ELU, 2 ReLU), then a linear layer of out_dim
// units and the output map out_act (0 identity, 1 out_scale * tanh,
// 2 softplus).  Parameters (FP32, row-major, y = x W + b): W_0 [in][width],
// b_0, then depth - 1 times W_l [width][width], b_l, then W_out
// [width][out], b_out.  Evaluated here in FP64.
struct Net {
  int in_dim, width, depth, out_dim, act, out_act;
  double out_scale;
  const float* p;
};

double net_act(double z, int act) {
  if (act == 0) return std::tanh(z);
  if (act == 1) return z > 0.0 ? z : std::expm1(z);
  return z > 0.0 ? z : 0.0;
}

void net_eval(const Net& net, const double* x, double* y) {
  const int W = net.width;
  std::vector<double> h(W), g(W);
  const float* p = net.p;
  // input layer
  for (int j = 0; j < W; ++j) {
    double z = p[net.in_dim * W + j];
    for (int i = 0; i < net.in_dim; ++i) z += x[i] * (double)p[i * W + j];
    h[j] = net_act(z, net.act);
  }
  p += net.in_dim * W + W;
  for (int l = 1; l < net.depth; ++l) {
    for (int j = 0; j < W; ++j) {
      double z = p[W * W + j];
      for (int i = 0; i < W; ++i) z += h[i] * (double)p[i * W + j];
      g[j] = net_act(z, net.act);
    }
    h.swap(g);
    p += W * W + W;
  }
  for (int o = 0; o < net.out_dim; ++o) {
    double z = p[W * net.out_dim + o];
    for (int j = 0; j < W; ++j) z += h[j] * (double)p[j * net.out_dim + o];
    if (net.out_act == 1) z = net.out_scale * std::tanh(z);
    else if (net.out_act == 2) z = std::max(z, 0.0) + std::log1p(std::exp(-std::fabs(z)));
    y[o] = z;
  }
}

// y[b] = net(x[b]) for B rows.
int orc_mlp_forward(int in_dim, int width, int depth, int out_dim, int act, int out_act, double out_scale,
                    const float* params, int B, const double* x, double* y) {
  if (in_dim < 1 || width < 1 || depth < 1 || out_dim < 1) return -1;
  const Net net{in_dim, width, depth, out_dim, act, out_act, out_scale, params};
#pragma omp parallel for schedule(static)
  for (int b = 0; b < B; ++b) net_eval(net, x + (size_t)b * in_dim, y + (size_t)b * out_dim);
  return 0;
}

// Actor warm start: u_k = actor(x_k, tau_k), tau_k = (Tmax - T_b + k) / Tmax,
// x_{k+1} = f(x_k, u_k) for k < T_b; U [B][Tmax][m], X [B][Tmax+1][n], zero
// past the horizon (all zero for a horizon outside 1..Tmax).
int orc_actor_rollout(int kind, const double* p, int np, int in_dim, int width, int depth, int out_dim, int act,
                      int out_act, double out_scale, const float* params, int B, int Tmax, const int32_t* Tb,
                      const double* x0, double* U, double* X) {
  Sys s;
  if (!make_sys(kind, p, np, &s)) return -1;
  const int n = s.n, m = s.m;
  if (in_dim != n + 1 || out_dim != m) return -1;
  const Net net{in_dim, width, depth, out_dim, act, out_act, out_scale, params};
  std::memset(U, 0, sizeof(double) * (size_t)B * Tmax * m);
  std::memset(X, 0, sizeof(double) * (size_t)B * (Tmax + 1) * n);
#pragma omp parallel for schedule(static)
  for (int b = 0; b < B; ++b) {
    const int T = Tb ? Tb[b] : Tmax;
    if (T < 1 || T > Tmax) continue;
    double* Xb = X + (size_t)b * (Tmax + 1) * n;
    double* Ub = U + (size_t)b * Tmax * m;
    std::vector<double> in(n + 1);
    for (int i = 0; i < n; ++i) Xb[i] = x0[(size_t)b * n + i];
    for (int k = 0; k < T; ++k) {
      for (int i = 0; i < n; ++i) in[i] = Xb[k * n + i];
      in[n] = (double)(Tmax - T + k) / Tmax;
      net_eval(net, in.data(), Ub + k * m);
      dyn<double>(s, Xb + k * n, Ub + k * m, Xb + (k + 1) * n);
    }
  }
  return 0;
}

// Total cost of nb control sequences (each T x m) from one x0, in parallel.
int orc_rollout_costs(int kind, const double* p, int np, int T, const double* x0, int nb,
                      const double* U, double* J, int nthreads) {
  Sys s;
  if (!make_sys(kind, p, np, &s)) return -1;
  const int n = s.n, m = s.m;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
  {
    std::vector<double> X((T + 1) * n);
#pragma omp for schedule(static)
    for (int b = 0; b < nb; ++b) J[b] = rollout(s, T, x0, U + (size_t)b * T * m, X.data());
  }
  return 0;
}

// Rollout X, total cost J, costate lambda ((T+1) x n) and dJ/dU (T x m).
int orc_gradient(int kind, const double* p, int np, int T, const double* x0, const double* U,
                 double* X, double* J, double* lam, double* g) {
  Sys s;
  if (!make_sys(kind, p, np, &s)) return -1;
  *J = rollout(s, T, x0, U, X);
  costate(s, T, X, U, lam, g);
  return 0;
}

// Batched solve.  All arrays are host, row-major, padded to T_max:
// X[B][Tmax+1][n], U[B][Tmax][m], Vbar[B][Tmax+1], Vx/xK[B][Tmax+1][n],
// trace[B][max_iter+1], jtrace/margin/force_j[B][max_iter].  Optional ones may be null.
int orc_solve_batch(int kind, const double* p, int np, int B, int Tmax, const int32_t* Tb,
                    const double* x0, const double* U0, const orc_opts* opt, double* X, double* U,
                    double* J, int32_t* iters, uint32_t* status, double* Vbar, double* Vx,
                    double* xK, double* trace, int32_t* jtrace, double* margin,
                    const int32_t* force_j, int nthreads) {
  Sys s;
  if (!make_sys(kind, p, np, &s)) {
    std::snprintf(g_err, sizeof g_err, "bad system kind/params");
    return -1;
  }
  if (B < 0 || Tmax < 1 || !opt || opt->max_iter < 0 || opt->ls_trials < 0) {
    std::snprintf(g_err, sizeof g_err, "bad sizes/options");
    return -1;
  }
  const int n = s.n, m = s.m;
  Opts o{opt->max_iter, opt->ls_trials, opt->stop_mode, opt->lookahead, opt->eps, opt->beta, opt->rtol,
         opt->reg, opt->mu0, opt->mu_factor, opt->mu_max, opt->umax, opt->round32};
  const size_t sx = (size_t)(Tmax + 1) * n, su = (size_t)Tmax * m;
  std::memset(X, 0, sizeof(double) * sx * B);
  std::memset(U, 0, sizeof(double) * su * B);
  if (Vbar) std::memset(Vbar, 0, sizeof(double) * (Tmax + 1) * B);
  if (Vx) std::memset(Vx, 0, sizeof(double) * sx * B);
  if (xK) std::memset(xK, 0, sizeof(double) * sx * B);
  for (int b = 0; b < B; ++b)
    if (Tb && (Tb[b] < 1 || Tb[b] > Tmax)) {
      std::snprintf(g_err, sizeof g_err, "horizon out of range");
      return -1;
    }
#pragma omp parallel for schedule(dynamic) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
  for (int b = 0; b < B; ++b) {
    const int T = Tb ? Tb[b] : Tmax;
    std::vector<double> U0t;
    const double* u0 = nullptr;
    if (U0) {
      U0t.assign(U0 + (size_t)b * su, U0 + (size_t)b * su + (size_t)T * m);
      u0 = U0t.data();
    }
    Out r{X + b * sx, U + b * su, J + b, iters + b, status + b,
          trace ? trace + (size_t)b * (o.max_iter + 1) : nullptr,
          jtrace ? jtrace + (size_t)b * o.max_iter : nullptr,
          margin ? margin + (size_t)b * o.max_iter : nullptr,
          Vbar ? Vbar + (size_t)b * (Tmax + 1) : nullptr,
          Vx ? Vx + b * sx : nullptr,
          xK ? xK + b * sx : nullptr,
          force_j ? force_j + (size_t)b * o.max_iter : nullptr};
    solve_one(s, T, x0 + (size_t)b * n, u0, o, r);
  }
  return 0;
}

int orc_max_threads() { return omp_get_max_threads(); }

// Critic targets (V-bar[T+1], V-bar_x[T+1][n], x_K[T+1][n]) of a given
// trajectory, without re-simulating it.
int orc_extract(int kind, const double* p, int np, int T, const double* X, const double* U, int lookahead,
                double* Vbar, double* Vx, double* xK) {
  Sys s;
  if (!make_sys(kind, p, np, &s) || T < 1) return -1;
  extract(s, T, X, U, lookahead, Vbar, Vx, xK);
  return 0;
}

// Per-step dynamics residual max_i |x_{k+1,i} - f(x_k,u_k)_i| / (1 + |x_{k+1,i}|)
// and the total cost of a given trajectory (summed in index order).
int orc_check_trajectory(int kind, const double* p, int np, int T, const double* X, const double* U,
                         double* defect, double* J) {
  Sys s;
  if (!make_sys(kind, p, np, &s) || T < 1) return -1;
  const int n = s.n, m = s.m;
  std::vector<double> xn(n);
  double d = 0.0, c = 0.0;
  for (int k = 0; k < T; ++k) {
    dyn<double>(s, X + k * n, U + k * m, xn.data());
    for (int i = 0; i < n; ++i)
      d = std::max(d, std::fabs(X[(k + 1) * n + i] - xn[i]) / (1.0 + std::fabs(X[(k + 1) * n + i])));
    c += cost<double>(s, X + k * n, U + k * m);
  }
  c += term<double>(s, X + T * n);
  *defect = d;
  *J = c;
  return 0;
}

}  // extern "C"
