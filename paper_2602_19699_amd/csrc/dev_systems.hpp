// Device models of the OCP systems (paper Sec. II eq. 1): dynamics f, running
// cost l, terminal cost l_T, and their analytic derivatives (Jacobians f_x,
// f_u; gradients; Hessians, eigenvalue-clipped per Sec. IV-B eq. 7).
//
// Every model reads a device-resident block of doubles prepared on the host
// from the user's parameter vector (derived constants such as 1/r^2 or the
// arm's inertia products are folded in there).  The layout of each block is
// given beside each model.  Precision R is double (plain form) or float
// (mixed form).
#pragma once
#include "dev_common.hpp"

namespace cbic {

// ============================================================== point mass
// x = (p_x, p_y, v_x, v_y), u = (a_x, a_y); semi-implicit Euler
//   v+ = v + dt u,  p+ = p + dt v+.
// l = w_u |u|^2 + w_p |p - g|^2 + w_o sum_i exp(-|p - c_i|^2 / r_i^2),
// l_T = w_T (|p - g|^2 + |v|^2).
// Device block: [dt, w_u, w_p, w_T, w_o, g_x, g_y, (c_x, c_y, 1/r^2) x 3].
struct PointMass {
  static constexpr int N = 4, M = 2;
  static constexpr int NPRM = 16;
  static constexpr bool kNonNegCost = true;
  // the warm start records the obstacle bumps' share of its cost, which
  // predicts an instance's iteration count better than the total cost
  static constexpr bool kOrderCost = true;
  // a rollout step costs little next to the stores of GL trial trajectories:
  // the line search writes only alpha = 1 and re-rolls another accepted step
  static constexpr bool kOwnTrialBuffers = false;
  // two identical double integrators (one per plane axis) coupled only through
  // the position Hessian of the cost: the backward sweep splits by axis
  static constexpr bool kAxisPairs = true;
  // f_x and f_u do not depend on (x, u)
  static constexpr bool kConstJac = true;
  static constexpr bool kSemiImplicit = false;  // (constant Jacobians: nothing to factor)
  // structural nonzeros of f_x and f_u (A = [[I, dt I], [0, I]], B = [[dt^2 I], [dt I]])
  __host__ __device__ static constexpr bool a_nz(int i, int j) { return i == j || j == i + 2; }
  __host__ __device__ static constexpr bool b_nz(int i, int j) { return (i & 1) == j; }

  template <class R>
  struct Model {
    const double* __restrict__ p;

    CBIC_HD __forceinline__ void dyn(const R* x, const R* u, R* xn) const {
      const R dt = R(p[0]);
      const R vx = x[2] + dt * u[0];
      const R vy = x[3] + dt * u[1];
      xn[0] = x[0] + dt * vx;
      xn[1] = x[1] + dt * vy;
      xn[2] = vx;
      xn[3] = vy;
    }

    // the obstacle bump exp(-d2 / r_i^2): in FP32 the hardware base-2
    // exponential with log2(e) folded into the parameter (one multiply fewer)
    CBIC_HD __forceinline__ R bump(R d2, int i) const {
      if constexpr (sizeof(R) == 4) {
        return __builtin_amdgcn_exp2f(-d2 * float(p[9 + 3 * i] * 1.4426950408889634));
      } else {
        return dexp(-d2 * R(p[9 + 3 * i]));
      }
    }

    CBIC_HD __forceinline__ R cost(const R* x, const R* u) const {
      const R ex = x[0] - R(p[5]), ey = x[1] - R(p[6]);
      R l = R(p[1]) * (u[0] * u[0] + u[1] * u[1]) + R(p[2]) * (ex * ex + ey * ey);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const R dx = x[0] - R(p[7 + 3 * i]), dy = x[1] - R(p[8 + 3 * i]);
        l += R(p[4]) * bump(dx * dx + dy * dy, i);
      }
      return l;
    }

    // l as cost() computes it (the same operations in the same order), and in
    // nc the sum of the three unweighted bumps: the non-convex part of l
    CBIC_HD __forceinline__ R cost(const R* x, const R* u, R& nc) const {
      const R ex = x[0] - R(p[5]), ey = x[1] - R(p[6]);
      R l = R(p[1]) * (u[0] * u[0] + u[1] * u[1]) + R(p[2]) * (ex * ex + ey * ey);
      R b = R(0);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const R dx = x[0] - R(p[7 + 3 * i]), dy = x[1] - R(p[8 + 3 * i]);
        const R e = bump(dx * dx + dy * dy, i);
        l += R(p[4]) * e;
        b += e;
      }
      nc = b;
      return l;
    }

    CBIC_HD __forceinline__ R term(const R* x) const {
      const R ex = x[0] - R(p[5]), ey = x[1] - R(p[6]);
      return R(p[3]) * (ex * ex + ey * ey + x[2] * x[2] + x[3] * x[3]);
    }

    CBIC_HD __forceinline__ void jac(const R*, const R*, R A[N][N], R B[N][M]) const {
      const R dt = R(p[0]);
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) A[i][j] = (i == j) ? R(1) : (j == i + 2 ? dt : R(0));
      B[0][0] = dt * dt; B[0][1] = R(0);
      B[1][0] = R(0);    B[1][1] = dt * dt;
      B[2][0] = dt;      B[2][1] = R(0);
      B[3][0] = R(0);    B[3][1] = dt;
    }

    // gradient of l; if H != null also the clipped Hessians of l.
    CBIC_HD __forceinline__ void cost_derivs(const R* x, const R* u, R lx[N], R lu[M],
                                                R Q[N][N], R Ru[M][M], R eps, bool hess) const {
      const R wp2 = R(2) * R(p[2]);
      R gx = wp2 * (x[0] - R(p[5])), gy = wp2 * (x[1] - R(p[6]));
      R hxx = wp2, hxy = R(0), hyy = wp2;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const R ir2 = R(p[9 + 3 * i]);
        const R dx = x[0] - R(p[7 + 3 * i]), dy = x[1] - R(p[8 + 3 * i]);
        const R e = R(p[4]) * bump(dx * dx + dy * dy, i);
        const R e2 = R(-2) * e * ir2;
        gx += e2 * dx;
        gy += e2 * dy;
        if (hess) {
          const R e4 = R(4) * e * ir2 * ir2;
          hxx += e4 * dx * dx + e2;
          hxy += e4 * dx * dy;
          hyy += e4 * dy * dy + e2;
        }
      }
      lx[0] = gx; lx[1] = gy; lx[2] = R(0); lx[3] = R(0);
      lu[0] = R(2) * R(p[1]) * u[0];
      lu[1] = R(2) * R(p[1]) * u[1];
      if (hess) {
        clip_sym2(hxx, hxy, hyy, eps);
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int j = 0; j < N; ++j) Q[i][j] = R(0);
        Q[0][0] = hxx; Q[0][1] = hxy; Q[1][0] = hxy; Q[1][1] = hyy;
        Q[2][2] = dmax(R(0), eps);
        Q[3][3] = dmax(R(0), eps);
        const R ru = dmax(R(2) * R(p[1]), eps);
        Ru[0][0] = ru; Ru[0][1] = R(0); Ru[1][0] = R(0); Ru[1][1] = ru;
      }
    }

    // Per-step derivative block for the backward sweep, evaluated ahead of the
    // serial recursion: l_x (2 nonzero), clipped position Hessian (3), l_u (2).
    // Axis h's own entries are D[h] (position gradient), D[2 + 2h] (its
    // diagonal Hessian entry) and D[5 + h] (control gradient); D[3] is the
    // cross-axis Hessian entry.
    static constexpr int ND = 7;
    CBIC_HD __forceinline__ void pack_derivs(const R* x, const R* u, R* D, R eps) const {
      R lx[N], lu[M], Q[N][N], Ru[M][M];
      cost_derivs(x, u, lx, lu, Q, Ru, eps, true);
      D[0] = lx[0]; D[1] = lx[1];
      D[2] = Q[0][0]; D[3] = Q[0][1]; D[4] = Q[1][1];
      D[5] = lu[0]; D[6] = lu[1];
    }
    CBIC_HD __forceinline__ void unpack_derivs(const R* D, R A[N][N], R B[N][M], R lx[N], R lu[M], R Q[N][N],
                                               R Ru[M][M], R eps) const {
      jac(nullptr, nullptr, A, B);
      lx[0] = D[0]; lx[1] = D[1]; lx[2] = R(0); lx[3] = R(0);
      lu[0] = D[5]; lu[1] = D[6];
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) Q[i][j] = R(0);
      Q[0][0] = D[2]; Q[0][1] = D[3]; Q[1][0] = D[3]; Q[1][1] = D[4];
      Q[2][2] = dmax(R(0), eps);
      Q[3][3] = dmax(R(0), eps);
      const R ru = dmax(R(2) * R(p[1]), eps);
      Ru[0][0] = ru; Ru[0][1] = R(0); Ru[1][0] = R(0); Ru[1][1] = ru;
    }

    // constants of the per-axis Riccati step: dt, the clipped control Hessian
    // (2 w_u) and the clipped velocity Hessian (zero)
    CBIC_HD __forceinline__ R step_dt() const { return R(p[0]); }
    CBIC_HD __forceinline__ R ctrl_hess(R eps) const { return dmax(R(2) * R(p[1]), eps); }
    CBIC_HD __forceinline__ R vel_hess(R eps) const { return dmax(R(0), eps); }

    CBIC_HD __forceinline__ void term_derivs(const R* x, R lx[N], R Q[N][N], R eps, bool hess) const {
      const R w2 = R(2) * R(p[3]);
      lx[0] = w2 * (x[0] - R(p[5]));
      lx[1] = w2 * (x[1] - R(p[6]));
      lx[2] = w2 * x[2];
      lx[3] = w2 * x[3];
      if (hess) {
        const R d = dmax(w2, eps);
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int j = 0; j < N; ++j) Q[i][j] = (i == j) ? d : R(0);
      }
    }
  };
};

// ============================================================== planar 3-link arm
// x = (q_1..q_3, qd_1..qd_3) relative joint angles and rates, u = joint torques.
// In absolute angles phi = L q (L lower-triangular ones) the rod chain has
//   M_phi(phi)_jk = h_jk cos(phi_j - phi_k) + delta_jk I_j,
//   c_phi,j = sum_k h_jk sin(phi_j - phi_k) phidot_k^2,
// with h_jk = sum_{i >= max(j,k)} m_i a_ij a_ik (a_ij = l_j for j < i, l_i/2 for j = i),
// joint torques map as tau_phi = L^-T tau and qdd = L^-1 M_phi^-1 (tau_phi - c_phi).
// Semi-implicit Euler: qd+ = qd + dt qdd, q+ = q + dt qd+.
// l = w_u |tau|^2 + w_ee |ee - p_t|^2 + w_o exp(-|ee - c|^2 / r^2), l_T = w_T |ee - p_t|^2.
// Device block: [dt, d1, d2, d3, h12, h13, h23, l1, l2, l3, w_u, w_ee, w_T, w_o,
//                p_x, p_y, c_x, c_y, 1/r^2]   (d_j = h_jj + I_j)
struct Arm3 {
  static constexpr int N = 6, M = 3;
  static constexpr int NPRM = 19;
  static constexpr bool kNonNegCost = true;
  static constexpr bool kOrderCost = false;
  // a rollout step is expensive: every trial lane writes its own trajectory
  // so that an accepted step needs no second rollout
  static constexpr bool kOwnTrialBuffers = true;
  static constexpr bool kAxisPairs = false;
  static constexpr bool kConstJac = false;
  // q+ = q + dt qd+: the backward sweep takes the Jacobians in factored form
  static constexpr bool kSemiImplicit = true;
  __host__ __device__ static constexpr bool a_nz(int, int) { return true; }
  __host__ __device__ static constexpr bool b_nz(int, int) { return true; }

  template <class R>
  struct Model {
    const double* __restrict__ p;

    // absolute-angle sines/cosines and the pair terms cos/sin(phi_j - phi_k)
    struct Trig {
      R s[3], c[3];        // sin/cos phi_j
      R C12, S12, C13, S13, C23, S23;
    };

    CBIC_HD __forceinline__ void trig(const R* q, Trig& t) const {
      const R ph1 = q[0], ph2 = q[0] + q[1], ph3 = ph2 + q[2];
      dsincos(ph1, &t.s[0], &t.c[0]);
      dsincos(ph2, &t.s[1], &t.c[1]);
      dsincos(ph3, &t.s[2], &t.c[2]);
      // angle-difference identities
      t.C12 = t.c[0] * t.c[1] + t.s[0] * t.s[1];
      t.S12 = t.s[0] * t.c[1] - t.c[0] * t.s[1];
      t.C13 = t.c[0] * t.c[2] + t.s[0] * t.s[2];
      t.S13 = t.s[0] * t.c[2] - t.c[0] * t.s[2];
      t.C23 = t.c[1] * t.c[2] + t.s[1] * t.s[2];
      t.S23 = t.s[1] * t.c[2] - t.c[1] * t.s[2];
    }

    // inverse of the symmetric M_phi by its adjugate
    CBIC_HD __forceinline__ void minv(const Trig& t, R Mi[3][3]) const {
      const R m00 = R(p[1]), m11 = R(p[2]), m22 = R(p[3]);
      const R m01 = R(p[4]) * t.C12, m02 = R(p[5]) * t.C13, m12 = R(p[6]) * t.C23;
      const R c00 = m11 * m22 - m12 * m12;
      const R c01 = m02 * m12 - m01 * m22;
      const R c02 = m01 * m12 - m02 * m11;
      const R c11 = m00 * m22 - m02 * m02;
      const R c12 = m01 * m02 - m00 * m12;
      const R c22 = m00 * m11 - m01 * m01;
      const R idet = R(1) / (m00 * c00 + m01 * c01 + m02 * c02);
      Mi[0][0] = c00 * idet; Mi[0][1] = c01 * idet; Mi[0][2] = c02 * idet;
      Mi[1][0] = Mi[0][1];   Mi[1][1] = c11 * idet; Mi[1][2] = c12 * idet;
      Mi[2][0] = Mi[0][2];   Mi[2][1] = Mi[1][2];   Mi[2][2] = c22 * idet;
    }

    // phi-space acceleration
    CBIC_HD __forceinline__ void phiacc(const Trig& t, const R Mi[3][3], const R* qd, const R* u,
                                           R w[3], R a[3]) const {
      const R h12 = R(p[4]), h13 = R(p[5]), h23 = R(p[6]);
      w[0] = qd[0];
      w[1] = qd[0] + qd[1];
      w[2] = w[1] + qd[2];
      const R c0 = h12 * t.S12 * w[1] * w[1] + h13 * t.S13 * w[2] * w[2];
      const R c1 = -h12 * t.S12 * w[0] * w[0] + h23 * t.S23 * w[2] * w[2];
      const R c2 = -h13 * t.S13 * w[0] * w[0] - h23 * t.S23 * w[1] * w[1];
      const R r0 = (u[0] - u[1]) - c0, r1 = (u[1] - u[2]) - c1, r2 = u[2] - c2;
#pragma unroll
      for (int i = 0; i < 3; ++i) a[i] = Mi[i][0] * r0 + Mi[i][1] * r1 + Mi[i][2] * r2;
    }

    CBIC_HD __forceinline__ void dyn(const R* x, const R* u, R* xn) const {
      const R dt = R(p[0]);
      Trig t;
      trig(x, t);
      R Mi[3][3], w[3], a[3];
      minv(t, Mi);
      phiacc(t, Mi, x + 3, u, w, a);
      const R qdd[3] = {a[0], a[1] - a[0], a[2] - a[1]};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        xn[3 + i] = x[3 + i] + dt * qdd[i];
        xn[i] = x[i] + dt * xn[3 + i];
      }
    }

    CBIC_HD __forceinline__ R step_dt() const { return R(p[0]); }

    // Jacobians of the velocity update qd+ = qd + dt qdd: V = d qd+ / d(q, qd)
    // (3 x 6), W = d qd+ / d tau (3 x 3).  With q+ = q + dt qd+ the full
    // Jacobians are f_x = S + C V and f_u = C W, S = diag(I, 0), C = [dt I; I].
    CBIC_HD __forceinline__ void jac_v(const R* x, const R* u, R V[3][N], R W[3][M]) const {
      const R dt = R(p[0]);
      const R h12 = R(p[4]), h13 = R(p[5]), h23 = R(p[6]);
      Trig t;
      trig(x, t);
      R Mi[3][3], w[3], a[3];
      minv(t, Mi);
      phiacc(t, Mi, x + 3, u, w, a);
      // G = d(M_phi a + c_phi)/d phi (a, phidot held), Cv = d c_phi / d phidot
      R G[3][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
      auto pair = [&](int j, int k, R h, R C, R S) {
        const R ej = -h * S * a[k] + h * C * w[k] * w[k];
        const R ek = -h * S * a[j] - h * C * w[j] * w[j];
        G[j][j] += ej; G[j][k] -= ej;
        G[k][j] += ek; G[k][k] -= ek;
      };
      pair(0, 1, h12, t.C12, t.S12);
      pair(0, 2, h13, t.C13, t.S13);
      pair(1, 2, h23, t.C23, t.S23);
      R Cv[3][3];
      Cv[0][0] = R(0);                         Cv[0][1] = R(2) * h12 * t.S12 * w[1];   Cv[0][2] = R(2) * h13 * t.S13 * w[2];
      Cv[1][0] = R(-2) * h12 * t.S12 * w[0];   Cv[1][1] = R(0);                        Cv[1][2] = R(2) * h23 * t.S23 * w[2];
      Cv[2][0] = R(-2) * h13 * t.S13 * w[0];   Cv[2][1] = R(-2) * h23 * t.S23 * w[1];  Cv[2][2] = R(0);
      // D = -M_phi^-1 [G | Cv | L^-T]  (phi-space sensitivities)
      R Dq[3][3], Dv[3][3], Dt[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          Dq[i][j] = -(Mi[i][0] * G[0][j] + Mi[i][1] * G[1][j] + Mi[i][2] * G[2][j]);
          Dv[i][j] = -(Mi[i][0] * Cv[0][j] + Mi[i][1] * Cv[1][j] + Mi[i][2] * Cv[2][j]);
        }
#pragma unroll
      for (int i = 0; i < 3; ++i) {  // M_phi^-1 L^-T: columns e0, e1 - e0, e2 - e1
        Dt[i][0] = Mi[i][0];
        Dt[i][1] = Mi[i][1] - Mi[i][0];
        Dt[i][2] = Mi[i][2] - Mi[i][1];
      }
      // to joint space: right-multiply q-, qd-blocks by L, left-multiply all by L^-1
      R Aq[3][3], Av[3][3], At[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const R q2 = Dq[i][2], q1 = Dq[i][1] + q2, q0 = Dq[i][0] + q1;
        Dq[i][0] = q0; Dq[i][1] = q1; Dq[i][2] = q2;
        const R v2 = Dv[i][2], v1 = Dv[i][1] + v2, v0 = Dv[i][0] + v1;
        Dv[i][0] = v0; Dv[i][1] = v1; Dv[i][2] = v2;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        Aq[0][j] = Dq[0][j]; Aq[1][j] = Dq[1][j] - Dq[0][j]; Aq[2][j] = Dq[2][j] - Dq[1][j];
        Av[0][j] = Dv[0][j]; Av[1][j] = Dv[1][j] - Dv[0][j]; Av[2][j] = Dv[2][j] - Dv[1][j];
        At[0][j] = Dt[0][j]; At[1][j] = Dt[1][j] - Dt[0][j]; At[2][j] = Dt[2][j] - Dt[1][j];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const R id = (i == j) ? R(1) : R(0);
          V[i][j] = dt * Aq[i][j];
          V[i][3 + j] = id + dt * Av[i][j];
          W[i][j] = dt * At[i][j];
        }
    }

    CBIC_HD __forceinline__ void jac(const R* x, const R* u, R A[N][N], R B[N][M]) const {
      const R dt = R(p[0]);
      R V[3][N], W[3][M];
      jac_v(x, u, V, W);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
          A[i][j] = (i == j ? R(1) : R(0)) + dt * V[i][j];
          A[3 + i][j] = V[i][j];
        }
#pragma unroll
        for (int j = 0; j < M; ++j) {
          B[i][j] = dt * W[i][j];
          B[3 + i][j] = W[i][j];
        }
      }
    }

    // end effector, its joint Jacobian and the per-link terms for the Hessian
    CBIC_HD __forceinline__ void ee(const Trig& t, R e[2], R J[2][3]) const {
      const R l0 = R(p[7]), l1 = R(p[8]), l2 = R(p[9]);
      const R px[3] = {l0 * t.c[0], l1 * t.c[1], l2 * t.c[2]};
      const R py[3] = {l0 * t.s[0], l1 * t.s[1], l2 * t.s[2]};
      e[0] = px[0] + px[1] + px[2];
      e[1] = py[0] + py[1] + py[2];
      J[0][2] = -py[2];           J[1][2] = px[2];
      J[0][1] = J[0][2] - py[1];  J[1][1] = J[1][2] + px[1];
      J[0][0] = J[0][1] - py[0];  J[1][0] = J[1][1] + px[0];
    }

    CBIC_HD __forceinline__ R cost(const R* x, const R* u) const {
      Trig t;
      trig(x, t);
      R e[2], J[2][3];
      ee(t, e, J);
      const R ex = e[0] - R(p[14]), ey = e[1] - R(p[15]);
      const R dx = e[0] - R(p[16]), dy = e[1] - R(p[17]);
      return R(p[10]) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + R(p[11]) * (ex * ex + ey * ey) +
             R(p[13]) * dexp(-(dx * dx + dy * dy) * R(p[18]));
    }

    CBIC_HD __forceinline__ R term(const R* x) const {
      Trig t;
      trig(x, t);
      R e[2], J[2][3];
      ee(t, e, J);
      const R ex = e[0] - R(p[14]), ey = e[1] - R(p[15]);
      return R(p[12]) * (ex * ex + ey * ey);
    }

    // l_q = J^T g;  l_qq = J^T H_ee J + S,  S_bc = sum_{j >= max(b,c)} -g . ee_j
    CBIC_HD __forceinline__ void ee_derivs(const Trig& t, R gx, R gy, R hxx, R hxy, R hyy,
                                              R lq[3], R H[9], bool hess) const {
      R e[2], J[2][3];
      ee(t, e, J);
#pragma unroll
      for (int c = 0; c < 3; ++c) lq[c] = J[0][c] * gx + J[1][c] * gy;
      if (!hess) return;
      const R l0 = R(p[7]), l1 = R(p[8]), l2 = R(p[9]);
      const R w0 = -l0 * (gx * t.c[0] + gy * t.s[0]);
      const R w1 = -l1 * (gx * t.c[1] + gy * t.s[1]);
      const R w2 = -l2 * (gx * t.c[2] + gy * t.s[2]);
      const R sacc[3] = {w0 + w1 + w2, w1 + w2, w2};
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const R hb0 = hxx * J[0][b] + hxy * J[1][b];
        const R hb1 = hxy * J[0][b] + hyy * J[1][b];
#pragma unroll
        for (int c = b; c < 3; ++c) {
          const R v = hb0 * J[0][c] + hb1 * J[1][c] + sacc[c > b ? c : b];
          H[b * 3 + c] = v;
          H[c * 3 + b] = v;
        }
      }
    }

    CBIC_HD __forceinline__ void cost_derivs(const R* x, const R* u, R lx[N], R lu[M],
                                                R Q[N][N], R Ru[M][M], R eps, bool hess) const {
      Trig t;
      trig(x, t);
      R e[2], J[2][3];
      ee(t, e, J);
      const R ir2 = R(p[18]);
      const R ex = e[0] - R(p[14]), ey = e[1] - R(p[15]);
      const R dx = e[0] - R(p[16]), dy = e[1] - R(p[17]);
      const R ew = R(p[13]) * dexp(-(dx * dx + dy * dy) * ir2);
      const R wee2 = R(2) * R(p[11]);
      const R e2 = R(-2) * ew * ir2;
      const R gx = wee2 * ex + e2 * dx, gy = wee2 * ey + e2 * dy;
      const R e4 = R(4) * ew * ir2 * ir2;
      const R hxx = wee2 + e4 * dx * dx + e2, hxy = e4 * dx * dy, hyy = wee2 + e4 * dy * dy + e2;
      R lq[3], H[9];
      ee_derivs(t, gx, gy, hxx, hxy, hyy, lq, H, hess);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lx[c] = lq[c];
        lx[3 + c] = R(0);
        lu[c] = R(2) * R(p[10]) * u[c];
      }
      if (hess) {
        clip_sym3(H, eps);
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int j = 0; j < N; ++j) Q[i][j] = (i < 3 && j < 3) ? H[i * 3 + j] : R(0);
        const R ev = dmax(R(0), eps);
        Q[3][3] = ev; Q[4][4] = ev; Q[5][5] = ev;
        const R ru = dmax(R(2) * R(p[10]), eps);
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
          for (int j = 0; j < M; ++j) Ru[i][j] = (i == j) ? ru : R(0);
      }
    }

    // Per-step derivative block: the velocity-update Jacobians V (18) and W
    // (9), l_q (3), clipped q-block Hessian (6, upper triangle), l_u (3).
    static constexpr int ND = 39;
    CBIC_HD __forceinline__ void pack_derivs(const R* x, const R* u, R* D, R eps) const {
      R V[3][N], W[3][M], lx[N], lu[M], Q[N][N], Ru[M][M];
      jac_v(x, u, V, W);
      cost_derivs(x, u, lx, lu, Q, Ru, eps, true);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) D[i * N + j] = V[i][j];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) D[18 + i * M + j] = W[i][j];
      D[27] = lx[0]; D[28] = lx[1]; D[29] = lx[2];
      D[30] = Q[0][0]; D[31] = Q[0][1]; D[32] = Q[0][2]; D[33] = Q[1][1]; D[34] = Q[1][2]; D[35] = Q[2][2];
      D[36] = lu[0]; D[37] = lu[1]; D[38] = lu[2];
    }
    CBIC_HD __forceinline__ void unpack_derivs_si(const R* D, R V[3][N], R W[3][M], R lx[N], R lu[M], R Q[N][N],
                                                  R Ru[M][M], R eps) const {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) V[i][j] = D[i * N + j];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) W[i][j] = D[18 + i * M + j];
      lx[0] = D[27]; lx[1] = D[28]; lx[2] = D[29]; lx[3] = R(0); lx[4] = R(0); lx[5] = R(0);
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) Q[i][j] = R(0);
      Q[0][0] = D[30]; Q[0][1] = D[31]; Q[0][2] = D[32]; Q[1][1] = D[33]; Q[1][2] = D[34]; Q[2][2] = D[35];
      Q[1][0] = D[31]; Q[2][0] = D[32]; Q[2][1] = D[34];
      const R ev = dmax(R(0), eps);
      Q[3][3] = ev; Q[4][4] = ev; Q[5][5] = ev;
      lu[0] = D[36]; lu[1] = D[37]; lu[2] = D[38];
      const R ru = dmax(R(2) * R(p[10]), eps);
#pragma unroll
      for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) Ru[i][j] = (i == j) ? ru : R(0);
    }

    CBIC_HD __forceinline__ void term_derivs(const R* x, R lx[N], R Q[N][N], R eps, bool hess) const {
      Trig t;
      trig(x, t);
      R e[2], J[2][3];
      ee(t, e, J);
      const R wT2 = R(2) * R(p[12]);
      const R gx = wT2 * (e[0] - R(p[14])), gy = wT2 * (e[1] - R(p[15]));
      R lq[3], H[9];
      ee_derivs(t, gx, gy, wT2, R(0), wT2, lq, H, hess);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lx[c] = lq[c];
        lx[3 + c] = R(0);
      }
      if (hess) {
        clip_sym3(H, eps);
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int j = 0; j < N; ++j) Q[i][j] = (i < 3 && j < 3) ? H[i * 3 + j] : R(0);
        const R ev = dmax(R(0), eps);
        Q[3][3] = ev; Q[4][4] = ev; Q[5][5] = ev;
      }
    }
  };
};

// ============================================================== linear-quadratic
// f = A x + B u, l = (x - x_r)^T Q (x - x_r) + u^T R u, l_T with Q_T.
// Device block: [A (NxN), B (NxM), Qs, Rs, QTs, x_r, Qc, Rc, QTc] where
// Qs = Q + Q^T (the Hessian) and Qc = clip(Qs) etc. (clipped once on the host;
// the Hessians are constant).
template <int NN, int MM>
struct LinQuad {
  static constexpr int N = NN, M = MM;
  static constexpr int OA = 0, OB = OA + N * N, OQ = OB + N * M, OR = OQ + N * N, OQT = OR + M * M,
                       OXR = OQT + N * N, OQC = OXR + N, ORC = OQC + N * N, OQTC = ORC + M * M,
                       NPRM = OQTC + N * N;
  static constexpr bool kNonNegCost = false;
  static constexpr bool kOrderCost = false;
  static constexpr bool kOwnTrialBuffers = false;
  static constexpr bool kAxisPairs = false;
  static constexpr bool kConstJac = true;
  static constexpr bool kSemiImplicit = false;
  __host__ __device__ static constexpr bool a_nz(int, int) { return true; }
  __host__ __device__ static constexpr bool b_nz(int, int) { return true; }

  template <class R>
  struct Model {
    const double* __restrict__ p;
    static constexpr int ND = 0;  // constant derivatives: nothing to stage
    CBIC_HD __forceinline__ void pack_derivs(const R*, const R*, R*, R) const {}
    CBIC_HD __forceinline__ void unpack_derivs(const R*, R[N][N], R[N][M], R[N], R[M], R[N][N], R[M][M], R) const {}

    CBIC_HD __forceinline__ void dyn(const R* x, const R* u, R* xn) const {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        R v = R(0);
#pragma unroll
        for (int j = 0; j < N; ++j) v += R(p[OA + i * N + j]) * x[j];
#pragma unroll
        for (int j = 0; j < M; ++j) v += R(p[OB + i * M + j]) * u[j];
        xn[i] = v;
      }
    }

    CBIC_HD __forceinline__ R qform(int off, int n, const R* a) const {
      R v = R(0);
      for (int i = 0; i < n; ++i) {
        R w = R(0);
        for (int j = 0; j < n; ++j) w += R(p[off + i * n + j]) * a[j];
        v += a[i] * w;
      }
      return R(0.5) * v;
    }

    CBIC_HD __forceinline__ R cost(const R* x, const R* u) const {
      R d[N];
#pragma unroll
      for (int i = 0; i < N; ++i) d[i] = x[i] - R(p[OXR + i]);
      return qform(OQ, N, d) + qform(OR, M, u);
    }

    CBIC_HD __forceinline__ R term(const R* x) const {
      R d[N];
#pragma unroll
      for (int i = 0; i < N; ++i) d[i] = x[i] - R(p[OXR + i]);
      return qform(OQT, N, d);
    }

    CBIC_HD __forceinline__ void jac(const R*, const R*, R A[N][N], R B[N][M]) const {
#pragma unroll
      for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j < N; ++j) A[i][j] = R(p[OA + i * N + j]);
#pragma unroll
        for (int j = 0; j < M; ++j) B[i][j] = R(p[OB + i * M + j]);
      }
    }

    CBIC_HD __forceinline__ void cost_derivs(const R* x, const R* u, R lx[N], R lu[M],
                                                R Q[N][N], R Ru[M][M], R, bool hess) const {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        R v = R(0);
#pragma unroll
        for (int j = 0; j < N; ++j) v += R(p[OQ + i * N + j]) * (x[j] - R(p[OXR + j]));
        lx[i] = v;
      }
#pragma unroll
      for (int i = 0; i < M; ++i) {
        R v = R(0);
#pragma unroll
        for (int j = 0; j < M; ++j) v += R(p[OR + i * M + j]) * u[j];
        lu[i] = v;
      }
      if (hess) {
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int j = 0; j < N; ++j) Q[i][j] = R(p[OQC + i * N + j]);
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
          for (int j = 0; j < M; ++j) Ru[i][j] = R(p[ORC + i * M + j]);
      }
    }

    CBIC_HD __forceinline__ void term_derivs(const R* x, R lx[N], R Q[N][N], R, bool hess) const {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        R v = R(0);
#pragma unroll
        for (int j = 0; j < N; ++j) v += R(p[OQT + i * N + j]) * (x[j] - R(p[OXR + j]));
        lx[i] = v;
      }
      if (hess) {
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int j = 0; j < N; ++j) Q[i][j] = R(p[OQTC + i * N + j]);
      }
    }
  };
};

}  // namespace cbic
