// Lane-per-instance batched iLQR (paper Sec. II and IV): every lane of a
// 64-wide wavefront owns one TO instance and runs its whole solve with the
// small per-instance matrices (P, A, B, gains) in registers.  Trajectories and
// gains live in HBM slot-major, [slot][k][component] with each slot's block
// padded to whole 128-byte lines: the lanes of an instance's group load
// consecutive steps of that instance, so a group's load fills whole cache
// lines whatever the other groups of its wave are doing (an instance that has
// converged leaves no partly used lines behind).
//
// Three kernels share per-slot state in a workspace:
//   lane_init     warm start (U0 or zeros) and the initial rollout, J^0;
//   lane_iterate  up to G iLQR iterations (backward Riccati sweep with the
//                 eigenvalue-clipped Hessians of eq. 7 and a Cholesky of Q_uu,
//                 then the backtracking line search); resumable, so the same
//                 kernel serves one fused launch or a chain of G-iteration
//                 launches (graph-captured loops, serving);
//   lane_final    status, the critic targets of Sec. II (K-step cost-to-go,
//                 costate V_x, state after K steps) and the caller's AoS outputs.
//
// Precision R: double for the plain form; float for the mixed form, where the
// rollouts, derivatives and Riccati products run in FP32 while the Q_uu
// Cholesky, the gain solves, the cost sums and the line-search comparison stay
// in FP64.
#pragma once
#include "dev_common.hpp"

namespace cbic {

template <class R>
struct LaneState {
  // per-slot state, all [Bcap]
  int32_t* T;        // horizon
  int32_t* inst;     // caller's instance index of this slot
  double* J;         // current total cost
  int32_t* iters;    // accepted iterations
  uint32_t* status;  // status bits; nonzero = frozen
  int32_t* cur;      // which trajectory buffer holds the iterate (0/1)
  int32_t* work;     // [Bcap][4]: backward sweeps, rollout passes, rollout steps read, steps written
  double* mu;        // Levenberg-Marquardt parameter (that variant only)
  uint32_t* okey;    // iteration-order key (horizon, J^0 and the non-convex share of J^0
                     // where the system has one): orders the launches, never a result
  // trajectories and gains, step-major
  R* X;   // [nbuf][Bcap][xs]: x_k at k N; the iterate (buffer cur) and trial trajectories
  R* U;   // [nbuf][Bcap][us]: u_k at k M
  R* K;   // [Bcap][Ks]: K_k (M x N, row-major) at k M N
  R* kf;  // [Bcap][ks]: k_k at k M
  int Bcap, Tcap, nbuf;
  int xs, us, Ks, ks;  // per-slot strides (elements), whole cache lines
};

struct SolveParams {
  int32_t max_iter;
  int32_t ls_trials;
  int32_t stop_mode;
  int32_t lookahead;
  double eps;  // negative: no clipping
  double beta;
  double rtol;
  int32_t reg;  // 1: Levenberg-Marquardt (Q_uu + mu I, mu adapted per instance)
  double mu0, mu_fac, mu_max;
  double umax;  // control bound of eq. 1 (the BOX kernels; infinite otherwise)
};

template <class Sys, class R>
struct Lane {
  static constexpr int N = Sys::N, M = Sys::M;
  using Model = typename Sys::template Model<R>;

  __device__ static __forceinline__ R* xp(const LaneState<R>& w, int buf, int k, int s) {
    return w.X + (size_t(buf) * w.Bcap + s) * w.xs + k * N;
  }
  __device__ static __forceinline__ R* up(const LaneState<R>& w, int buf, int k, int s) {
    return w.U + (size_t(buf) * w.Bcap + s) * w.us + k * M;
  }
  __device__ static __forceinline__ R* Kp(const LaneState<R>& w, int k, int s) {
    return w.K + size_t(s) * w.Ks + k * (M * N);
  }
  __device__ static __forceinline__ R* kp(const LaneState<R>& w, int k, int s) {
    return w.kf + size_t(s) * w.ks + k * M;
  }

  template <int L>
  __device__ static __forceinline__ void ld(R (&dst)[L], const R* src) {
#pragma unroll
    for (int i = 0; i < L; ++i) dst[i] = src[i];
  }
  template <int L>
  __device__ static __forceinline__ void st(R* dst, const R (&src)[L]) {
#pragma unroll
    for (int i = 0; i < L; ++i) dst[i] = src[i];
  }

  // ------------------------------------------------------------------ backward
  // One Riccati step at time k from the step's derivatives; updates (P, p)
  // in place and writes K_k, k_k when `store`.  With BOX the control step
  // minimises the local model over the box |u_k + d| <= umax (eq. 1) and the
  // feedback rows of the components held at a bound are zero; u is the
  // iterate's control at step k.  Returns 0 or the status bit that freezes
  // the instance.
  template <bool BOX>
  __device__ static __forceinline__ uint32_t riccati_step(const LaneState<R>& w, int s, int k, const R (&A)[N][N],
                                                          const R (&B)[N][M], const R (&lx)[N], const R (&lu)[M],
                                                          const R (&Qc)[N][N], const R (&Rc)[M][M], R (&P)[N][N],
                                                          R (&p)[N], bool store, double mu, const R (&u)[M],
                                                          double umax) {
    // PA = P A, PB = P B  (structural zeros of A, B skipped at compile time)
    R PA[N][N], PB[N][M];
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        R v = R(0);
#pragma unroll
        for (int t = 0; t < N; ++t)
          if (Sys::a_nz(t, j)) v += P[i][t] * A[t][j];
        PA[i][j] = v;
      }
#pragma unroll
      for (int j = 0; j < M; ++j) {
        R v = R(0);
#pragma unroll
        for (int t = 0; t < N; ++t)
          if (Sys::b_nz(t, j)) v += P[i][t] * B[t][j];
        PB[i][j] = v;
      }
    }
    R Qx[N], Qu[M], Qxx[N][N], Qux[M][N];
    double Quu[M][M];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      R v = lx[i];
#pragma unroll
      for (int t = 0; t < N; ++t)
        if (Sys::a_nz(t, i)) v += A[t][i] * p[t];
      Qx[i] = v;
#pragma unroll
      for (int j = i; j < N; ++j) {
        R q = Qc[i][j];
#pragma unroll
        for (int t = 0; t < N; ++t)
          if (Sys::a_nz(t, i)) q += A[t][i] * PA[t][j];
        Qxx[i][j] = q;
      }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
      R v = lu[i];
#pragma unroll
      for (int t = 0; t < N; ++t)
        if (Sys::b_nz(t, i)) v += B[t][i] * p[t];
      Qu[i] = v;
#pragma unroll
      for (int j = i; j < M; ++j) {
        R q = Rc[i][j];
#pragma unroll
        for (int t = 0; t < N; ++t)
          if (Sys::b_nz(t, i)) q += B[t][i] * PB[t][j];
        Quu[i][j] = double(q);
      }
#pragma unroll
      for (int j = 0; j < N; ++j) {
        R q = R(0);
#pragma unroll
        for (int t = 0; t < N; ++t)
          if (Sys::b_nz(t, i)) q += B[t][i] * PA[t][j];
        Qux[i][j] = q;
      }
    }
    return gains_update<BOX>(w, s, k, Qx, Qu, Qxx, Quu, Qux, P, p, store, mu, u, umax);
  }

  // One Riccati step for a semi-implicit Euler system (q+ = q + dt v+, the
  // state (q, v) with NQ = N / 2 positions): the dynamics Jacobians factor as
  // A = S + C V and B = C W with S = diag(I, 0), C = [dt I; I] and V (NQ x N),
  // W (NQ x M) the Jacobians of the velocity update, so the products go
  // through P C, C^T P A and C^T P B (about 60 % of the dense count).
  template <bool BOX>
  __device__ static __forceinline__ uint32_t riccati_step_si(const LaneState<R>& w, int s, int k, R dt,
                                                             const R (&V)[N / 2][N], const R (&W)[N / 2][M],
                                                             const R (&lx)[N], const R (&lu)[M],
                                                             const R (&Qc)[N][N], const R (&Rc)[M][M],
                                                             R (&P)[N][N], R (&p)[N], bool store, double mu,
                                                             const R (&u)[M], double umax) {
    constexpr int NQ = N / 2;
    R PC[N][NQ];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int c = 0; c < NQ; ++c) PC[i][c] = dt * P[i][c] + P[i][NQ + c];
    R PA[N][N], PB[N][M];
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        R v = j < NQ ? P[i][j] : R(0);
#pragma unroll
        for (int c = 0; c < NQ; ++c) v += PC[i][c] * V[c][j];
        PA[i][j] = v;
      }
#pragma unroll
      for (int m = 0; m < M; ++m) {
        R v = R(0);
#pragma unroll
        for (int c = 0; c < NQ; ++c) v += PC[i][c] * W[c][m];
        PB[i][m] = v;
      }
    }
    R CPA[NQ][N], CPB[NQ][M], Cp[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
#pragma unroll
      for (int j = 0; j < N; ++j) CPA[c][j] = dt * PA[c][j] + PA[NQ + c][j];
#pragma unroll
      for (int m = 0; m < M; ++m) CPB[c][m] = dt * PB[c][m] + PB[NQ + c][m];
      Cp[c] = dt * p[c] + p[NQ + c];
    }
    R Qx[N], Qu[M], Qxx[N][N], Qux[M][N];
    double Quu[M][M];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      R v = lx[i] + (i < NQ ? p[i] : R(0));
#pragma unroll
      for (int c = 0; c < NQ; ++c) v += V[c][i] * Cp[c];
      Qx[i] = v;
#pragma unroll
      for (int j = i; j < N; ++j) {
        R q = Qc[i][j] + (i < NQ ? PA[i][j] : R(0));
#pragma unroll
        for (int c = 0; c < NQ; ++c) q += V[c][i] * CPA[c][j];
        Qxx[i][j] = q;
      }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      R v = lu[m];
#pragma unroll
      for (int c = 0; c < NQ; ++c) v += W[c][m] * Cp[c];
      Qu[m] = v;
#pragma unroll
      for (int n = m; n < M; ++n) {
        R q = Rc[m][n];
#pragma unroll
        for (int c = 0; c < NQ; ++c) q += W[c][m] * CPB[c][n];
        Quu[m][n] = double(q);
      }
#pragma unroll
      for (int j = 0; j < N; ++j) {
        R q = R(0);
#pragma unroll
        for (int c = 0; c < NQ; ++c) q += W[c][m] * CPA[c][j];
        Qux[m][j] = q;
      }
    }
    return gains_update<BOX>(w, s, k, Qx, Qu, Qxx, Quu, Qux, P, p, store, mu, u, umax);
  }

  // riccati_step_si split over a lane pair (lanes 2j, 2j + 1 of a group; h =
  // r & 1) for the 6-state, 3-control system: each lane forms the columns
  // J_h of P A, C^T P A, Q_xx, Q_ux, K and of the updated P (J_0 = {0, 2, 5},
  // J_1 = {1, 3, 4}: 10 and 11 entries of the upper triangle), the pair swaps
  // Q_ux and the new P (DPP), and the shared small terms (P C, P B, Q_uu, the
  // Cholesky, k, p) are formed by both.  Every entry comes from the same
  // formula as in riccati_step_si, so the results agree bit for bit with a
  // one-lane group.
  __device__ static __forceinline__ R psel(int h, R a, R b) { return h ? b : a; }
  template <bool BOX>
  __device__ static __forceinline__ uint32_t riccati_step_si_pair(const LaneState<R>& w, int s, int k, R dt,
                                                                  const R (&V)[N / 2][N], const R (&W)[N / 2][M],
                                                                  const R (&lx)[N], const R (&lu)[M],
                                                                  const R (&Qc)[N][N], const R (&Rc)[M][M],
                                                                  R (&P)[N][N], R (&p)[N], double mu,
                                                                  const R (&u)[M], double umax, int h) {
    static_assert(N == 6 && M == 3, "the column split is laid out for 6 states and 3 controls");
    constexpr int NQ = N / 2;
    constexpr int J0[3] = {0, 2, 5}, J1[3] = {1, 3, 4};
    constexpr int JN = 3;
    R PC[N][NQ];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int c = 0; c < NQ; ++c) PC[i][c] = dt * P[i][c] + P[i][NQ + c];
    // own columns of V
    R Vo[NQ][JN];
#pragma unroll
    for (int c = 0; c < NQ; ++c)
#pragma unroll
      for (int jj = 0; jj < JN; ++jj) Vo[c][jj] = psel(h, V[c][J0[jj]], V[c][J1[jj]]);
    R PAo[N][JN], PB[N][M];
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int jj = 0; jj < JN; ++jj) {
        R v = psel(h, J0[jj] < NQ ? P[i][J0[jj]] : R(0), J1[jj] < NQ ? P[i][J1[jj]] : R(0));
#pragma unroll
        for (int c = 0; c < NQ; ++c) v += PC[i][c] * Vo[c][jj];
        PAo[i][jj] = v;
      }
#pragma unroll
      for (int m = 0; m < M; ++m) {
        R v = R(0);
#pragma unroll
        for (int c = 0; c < NQ; ++c) v += PC[i][c] * W[c][m];
        PB[i][m] = v;
      }
    }
    R CPAo[NQ][JN], CPB[NQ][M], Cp[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
#pragma unroll
      for (int jj = 0; jj < JN; ++jj) CPAo[c][jj] = dt * PAo[c][jj] + PAo[NQ + c][jj];
#pragma unroll
      for (int m = 0; m < M; ++m) CPB[c][m] = dt * PB[c][m] + PB[NQ + c][m];
      Cp[c] = dt * p[c] + p[NQ + c];
    }
    R Qx[N], Qu[M];
    double Quu[M][M];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      R v = lx[i] + (i < NQ ? p[i] : R(0));
#pragma unroll
      for (int c = 0; c < NQ; ++c) v += V[c][i] * Cp[c];
      Qx[i] = v;
    }
    // Q_xx on the own columns, rows i <= j (slot (i, jj) is used where i <= J_h[jj])
    R Qxxo[N][JN];
#pragma unroll
    for (int jj = 0; jj < JN; ++jj) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        if (i > (J0[jj] > J1[jj] ? J0[jj] : J1[jj])) continue;
        R q = psel(h, Qc[i][J0[jj]], Qc[i][J1[jj]]) + (i < NQ ? PAo[i][jj] : R(0));
#pragma unroll
        for (int c = 0; c < NQ; ++c) q += V[c][i] * CPAo[c][jj];
        Qxxo[i][jj] = q;
      }
    }
    R Quxo[M][JN];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      R v = lu[m];
#pragma unroll
      for (int c = 0; c < NQ; ++c) v += W[c][m] * Cp[c];
      Qu[m] = v;
#pragma unroll
      for (int n = m; n < M; ++n) {
        R q = Rc[m][n];
#pragma unroll
        for (int c = 0; c < NQ; ++c) q += W[c][m] * CPB[c][n];
        Quu[m][n] = double(q);
      }
#pragma unroll
      for (int jj = 0; jj < JN; ++jj) {
        R q = R(0);
#pragma unroll
        for (int c = 0; c < NQ; ++c) q += W[c][m] * CPAo[c][jj];
        Quxo[m][jj] = q;
      }
    }
    // ---- gains (as gains_update, on the own columns)
    if (mu != 0.0)
#pragma unroll
      for (int i = 0; i < M; ++i) Quu[i][i] += mu;
    constexpr int NR = sizeof(R) == 4 ? 1 : 2;
    double Lc[M][M], invd[M];
    uint32_t bad = chol_fp64<M, NR>(Quu, Lc, invd) ? 0u : ST_CHOL_FAIL;
    R Ko[M][JN], kk[M];
    bool fin = true;
    bool solved = false;
    if constexpr (sizeof(R) == 4) {
      float lf[M][M], ivf[M];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        ivf[i] = float(invd[i]);
#pragma unroll
        for (int j = 0; j < M; ++j) lf[i][j] = float(Lc[i][j]);
      }
      auto solve = [&](float (&b)[M]) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
          float v = b[i];
#pragma unroll
          for (int k2 = 0; k2 < i; ++k2) v -= lf[i][k2] * b[k2];
          b[i] = v * ivf[i];
        }
#pragma unroll
        for (int i = M - 1; i >= 0; --i) {
          float v = b[i];
#pragma unroll
          for (int k2 = i + 1; k2 < M; ++k2) v += lf[k2][i] * b[k2];
          b[i] = v * -ivf[i];
        }
      };
      float col[M];
#pragma unroll
      for (int i = 0; i < M; ++i) col[i] = Qu[i];
      solve(col);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        kk[i] = col[i];
        fin = fin && dfinite(kk[i]);
      }
#pragma unroll
      for (int jj = 0; jj < JN; ++jj) {
#pragma unroll
        for (int i = 0; i < M; ++i) col[i] = Quxo[i][jj];
        solve(col);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          Ko[i][jj] = col[i];
          fin = fin && dfinite(Ko[i][jj]);
        }
      }
      solved = true;
      if constexpr (BOX) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
          const double d = double(kk[i]);
          solved = solved && d >= -umax - double(u[i]) && d <= umax - double(u[i]);
        }
        if (!solved) fin = true;
      }
    }
    if (!solved) {
      double col[M];
#pragma unroll
      for (int i = 0; i < M; ++i) col[i] = double(Qu[i]);
      chol_solve_neg_fp64<M>(Lc, invd, col);
      unsigned held = 0;
      if constexpr (BOX) {
        double g[M], lo[M], hi[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
          g[i] = double(Qu[i]);
          lo[i] = -umax - double(u[i]);
          hi[i] = umax - double(u[i]);
        }
        if (!box_qp<M, NR>(Quu, g, lo, hi, col, held, Lc, invd) && !bad) bad = ST_CHOL_FAIL;
      }
#pragma unroll
      for (int i = 0; i < M; ++i) {
        kk[i] = R(col[i]);
        fin = fin && dfinite(kk[i]);
      }
#pragma unroll
      for (int jj = 0; jj < JN; ++jj) {
#pragma unroll
        for (int i = 0; i < M; ++i) col[i] = ((held >> i) & 1u) ? 0.0 : double(Quxo[i][jj]);
        chol_solve_neg_fp64<M>(Lc, invd, col);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          Ko[i][jj] = R(col[i]);
          fin = fin && dfinite(Ko[i][jj]);
        }
      }
    }
    // the pair's finiteness check of its gains (the partner checked its own columns)
    fin = fin && (__builtin_amdgcn_mov_dpp(int(fin), 0xB1, 0xF, 0xF, true) != 0);
    if (!fin && !bad) bad = ST_NONFINITE;
    {
      // every lane stores its own columns of K and k
      R* dK = Kp(w, k, s);
#pragma unroll
      for (int i = 0; i < M; ++i)
#pragma unroll
        for (int jj = 0; jj < JN; ++jj) dK[i * N + (h ? J1[jj] : J0[jj])] = Ko[i][jj];
      st(kp(w, k, s), kk);
    }
    // Q_ux on all columns: own and the partner's
    R Quxp[M][JN];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int jj = 0; jj < JN; ++jj) Quxp[m][jj] = pair_swap(Quxo[m][jj]);
    R Qux[M][N];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int jj = 0; jj < JN; ++jj) {
        Qux[m][J0[jj]] = psel(h, Quxo[m][jj], Quxp[m][jj]);
        Qux[m][J1[jj]] = psel(h, Quxp[m][jj], Quxo[m][jj]);
      }
    // P = sym(Q_xx + Q_ux^T K) on the own columns, p = Q_x + Q_ux^T k
#pragma unroll
    for (int i = 0; i < N; ++i) {
      R v = Qx[i];
#pragma unroll
      for (int t = 0; t < M; ++t) v += Qux[t][i] * kk[t];
      p[i] = v;
    }
    R Po[N][JN];
#pragma unroll
    for (int jj = 0; jj < JN; ++jj)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        if (i > (J0[jj] > J1[jj] ? J0[jj] : J1[jj])) continue;
        R q = Qxxo[i][jj];
#pragma unroll
        for (int t = 0; t < M; ++t) q += Qux[t][i] * Ko[t][jj];
        Po[i][jj] = q;
      }
    // the partner's columns, then the full symmetric P
#pragma unroll
    for (int jj = 0; jj < JN; ++jj)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        if (i > (J0[jj] > J1[jj] ? J0[jj] : J1[jj])) continue;
        const R mine = Po[i][jj], other = pair_swap(Po[i][jj]);
        if (i <= J0[jj]) {
          const R v = psel(h, mine, other);
          P[i][J0[jj]] = v;
          P[J0[jj]][i] = v;
        }
        if (i <= J1[jj]) {
          const R v = psel(h, other, mine);
          P[i][J1[jj]] = v;
          P[J1[jj]][i] = v;
        }
      }
    return bad;
  }

  // The control step and the (P, p) update from the step's Q blocks (Q_xx
  // and Q_uu upper triangles): Cholesky of Q_uu (+ mu I in the
  // Levenberg-Marquardt variant) in FP64 (one Newton step on the reciprocal
  // pivots when the gains are FP32) and the gains; the checks are on the
  // gains as stored, so an FP32 overflow is caught as well.  Returns the first
  // failure's status bit (the step's results are then not used) without
  // leaving early, so the step has no branch.
  template <bool BOX>
  __device__ static __forceinline__ uint32_t gains_update(const LaneState<R>& w, int s, int k, const R (&Qx)[N],
                                                          const R (&Qu)[M], const R (&Qxx)[N][N],
                                                          double (&Quu)[M][M], const R (&Qux)[M][N], R (&P)[N][N],
                                                          R (&p)[N], bool store, double mu, const R (&u)[M],
                                                          double umax) {
    if (mu != 0.0)
#pragma unroll
      for (int i = 0; i < M; ++i) Quu[i][i] += mu;
    constexpr int NR = sizeof(R) == 4 ? 1 : 2;
    double Lc[M][M], invd[M];
    // a failure is recorded and the step runs on; the caller acts on it
    uint32_t bad = chol_fp64<M, NR>(Quu, Lc, invd) ? 0u : ST_CHOL_FAIL;
    R Kk[M][N], kk[M];
    bool fin = true;
    bool solved = false;
    if constexpr (sizeof(R) == 4) {
      // mixed form: the gains are stored in FP32, so their triangular solves
      // run in FP32 on the FP64 factor rounded to FP32 (a few ulps, as the
      // rounding of FP64 solves to FP32 would give).  With a bound, this
      // unconstrained step stands when it lies in the box (so a bound that
      // does not bind changes nothing); otherwise the FP64 box QP below runs
      float lf[M][M], ivf[M];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        ivf[i] = float(invd[i]);
#pragma unroll
        for (int j = 0; j < M; ++j) lf[i][j] = float(Lc[i][j]);
      }
      auto solve = [&](float (&b)[M]) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
          float v = b[i];
#pragma unroll
          for (int k2 = 0; k2 < i; ++k2) v -= lf[i][k2] * b[k2];
          b[i] = v * ivf[i];
        }
#pragma unroll
        for (int i = M - 1; i >= 0; --i) {
          float v = b[i];
#pragma unroll
          for (int k2 = i + 1; k2 < M; ++k2) v += lf[k2][i] * b[k2];
          b[i] = v * -ivf[i];
        }
      };
      float col[M];
#pragma unroll
      for (int i = 0; i < M; ++i) col[i] = Qu[i];
      solve(col);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        kk[i] = col[i];
        fin = fin && dfinite(kk[i]);
      }
#pragma unroll
      for (int j = 0; j < N; ++j) {
#pragma unroll
        for (int i = 0; i < M; ++i) col[i] = Qux[i][j];
        solve(col);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          Kk[i][j] = col[i];
          fin = fin && dfinite(Kk[i][j]);
        }
      }
      solved = true;
      if constexpr (BOX) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
          const double d = double(kk[i]);
          solved = solved && d >= -umax - double(u[i]) && d <= umax - double(u[i]);
        }
        if (!solved) fin = true;
      }
    }
    if (!solved) {
      double col[M];
#pragma unroll
      for (int i = 0; i < M; ++i) col[i] = double(Qu[i]);
      chol_solve_neg_fp64<M>(Lc, invd, col);
      unsigned held = 0;  // components held at a bound (BOX)
      if constexpr (BOX) {
        double g[M], lo[M], hi[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
          g[i] = double(Qu[i]);
          lo[i] = -umax - double(u[i]);
          hi[i] = umax - double(u[i]);
        }
        if (!box_qp<M, NR>(Quu, g, lo, hi, col, held, Lc, invd) && !bad) bad = ST_CHOL_FAIL;
      }
#pragma unroll
      for (int i = 0; i < M; ++i) {
        kk[i] = R(col[i]);
        fin = fin && dfinite(kk[i]);
      }
#pragma unroll
      for (int j = 0; j < N; ++j) {
#pragma unroll
        for (int i = 0; i < M; ++i) col[i] = ((held >> i) & 1u) ? 0.0 : double(Qux[i][j]);
        chol_solve_neg_fp64<M>(Lc, invd, col);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          Kk[i][j] = R(col[i]);
          fin = fin && dfinite(Kk[i][j]);
        }
      }
    }
    if (!fin && !bad) bad = ST_NONFINITE;
    if (store) {
      R* dK = Kp(w, k, s);
#pragma unroll
      for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) dK[i * N + j] = Kk[i][j];
      st(kp(w, k, s), kk);
    }
    // P = sym(Q_xx + Q_ux^T K), p = Q_x + Q_ux^T k
#pragma unroll
    for (int i = 0; i < N; ++i) {
      R v = Qx[i];
#pragma unroll
      for (int t = 0; t < M; ++t) v += Qux[t][i] * kk[t];
      p[i] = v;
#pragma unroll
      for (int j = i; j < N; ++j) {
        R q = Qxx[i][j];
#pragma unroll
        for (int t = 0; t < M; ++t) q += Qux[t][i] * Kk[t][j];
        P[i][j] = q;
        P[j][i] = q;
      }
    }
    return bad;
  }

  // ------------------------------------------------------------------ backward, axis pairs
  // For two identical double integrators, one per plane axis, coupled only
  // through the cross-axis entry of the cost's position Hessian (the point
  // mass; state (p_0, p_1, v_0, v_1)), A is a = [[1, dt], [0, 1]] and B is
  // b = (dt^2, dt) on each axis' (position, velocity) pair.  P is then held as
  // its diagonal blocks P_hh and its cross block, and one Riccati step splits
  // by axis: lanes 2j and 2j + 1 of a group take axis r & 1 each and swap
  // (DPP) the few values the other axis needs.  Everything the two lanes hold
  // in common comes from formulas that are symmetric in the two axes, so the
  // pair's copies agree bit for bit; the cross block of the update is
  // sym(Q_xx + Q_ux^T K), the mean of the pair's two products.  A one-lane
  // group runs both axes with the same formulas, so the result does not depend
  // on the group width.
  struct AxisP {
    R pp, pv, vv;          // diagonal block P_hh: (pos, pos), (pos, vel), (vel, vel)
    R xpp, xpv, xvp, xvv;  // cross block: rows this axis (pos, vel), columns the other axis
    R qp, qv;              // p on this axis: (pos, vel)
  };
  struct AxisQ {
    R s, qu, q01;              // b^T P_hh b, Q_u of this axis' control, b^T P_01 b
    R ga_p, ga_v, gb_p, gb_v;  // Q_ux on this axis' columns: this control's row, the other's
    R Qpp, Qpv, Qvv;           // Q_xx diagonal block
    R Xpp, Xpv, Xvp, Xvv;      // Q_xx cross block, this axis' orientation
    R Qxp, Qxv;                // Q_x
  };

  // the value held by the other lane of the pair (2j, 2j + 1): DPP quad_perm
  // [1, 0, 3, 2] (bound_ctrl set: never out of range here, and it lets the
  // swap fold into the instruction that uses it)
  __device__ static __forceinline__ float pair_swap(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
  }
  __device__ static __forceinline__ double pair_swap(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp(int(b), 0xB1, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), 0xB1, 0xF, 0xF, true);
    return __longlong_as_double(static_cast<long long>(static_cast<unsigned>(lo)) |
                                (static_cast<long long>(hi) << 32));
  }

  // the quantities of one axis that need only that axis' P blocks; lx, hd, hx,
  // lu: position gradient, diagonal and cross-axis position Hessian entries,
  // control gradient
  __device__ static __forceinline__ void axis_q(const AxisP& P, R dt, R dt2, R ev, R lx, R hd, R hx, R lu,
                                                AxisQ& q) {
    const R g0 = P.pp * dt2 + P.pv * dt;  // P_hh b
    const R g1 = P.pv * dt2 + P.vv * dt;
    q.s = g0 * dt2 + g1 * dt;
    q.ga_p = g0;
    q.ga_v = g0 * dt + g1;
    const R w0 = P.xpp * dt2 + P.xpv * dt;  // (cross block) b
    const R w1 = P.xvp * dt2 + P.xvv * dt;
    q.gb_p = w0;
    q.gb_v = w0 * dt + w1;
    q.q01 = dt2 * (P.xpp * dt2 + (P.xpv + P.xvp) * dt + P.xvv);
    q.qu = lu + (P.qp * dt2 + P.qv * dt);
    q.Qxp = lx + P.qp;
    q.Qxv = P.qp * dt + P.qv;
    q.Qpp = hd + P.pp;
    q.Qpv = P.pp * dt + P.pv;
    q.Qvv = ev + (q.Qpv * dt + (P.pv * dt + P.vv));
    q.Xpp = hx + P.xpp;
    q.Xpv = P.xpp * dt + P.xpv;
    q.Xvp = P.xpp * dt + P.xvp;
    q.Xvv = (P.xpp * dt + (P.xpv + P.xvp)) * dt + P.xvv;
  }

  // One Riccati step at time k on the axis blocks AP (both axes for GL = 1,
  // axis h otherwise) from the staged derivative block D (model layout: D[h]
  // position gradient, D[2 + 2h] diagonal and D[3] cross-axis position Hessian
  // entries, D[5 + h] control gradient).  ev, ru: the clipped velocity and
  // control Hessians.  Gains, the bounded step (BOX, u the iterate's control)
  // and the Levenberg-Marquardt shift as in riccati_step; with `store` (every
  // lane of the group) each lane writes its axis' gain columns.  Returns the
  // first failure's status bit; the step's results are then not used.
  template <int GL, bool BOX>
  __device__ static __forceinline__ uint32_t axis_step(const LaneState<R>& w, int s, int k, const R* D,
                                                       const R (&u)[M], AxisP (&AP)[GL == 1 ? 2 : 1], int h,
                                                       R dt, R dt2, R ev, R ru, bool store, double mu,
                                                       double umax) {
    static_assert(N == 4 && M == 2, "axis pairs: two axes of (position, velocity) and one control each");
    constexpr int NA = GL == 1 ? 2 : 1;
    AxisQ q[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const int ax = GL == 1 ? a : h;
      axis_q(AP[a], dt, dt2, ev, D[ax], D[2 + 2 * ax], D[3], D[5 + ax], q[a]);
    }
    // Q_uu and Q_u in control order
    const bool first0 = GL == 1 || h == 0;  // the lane's first axis is axis 0
    const R so = GL == 1 ? q[NA - 1].s : pair_swap(q[0].s);
    const R uo = GL == 1 ? q[NA - 1].qu : pair_swap(q[0].qu);
    const R S0 = first0 ? q[0].s : so, S1 = first0 ? so : q[0].s;
    const R U0 = first0 ? q[0].qu : uo, U1 = first0 ? uo : q[0].qu;
    double Quu[M][M];
    Quu[0][0] = double(ru + S0);
    Quu[0][1] = double(q[0].q01);
    Quu[1][0] = Quu[0][1];
    Quu[1][1] = double(ru + S1);
    // the Levenberg-Marquardt shift (zero otherwise: adding it changes no bit
    // of a diagonal that is not -0, and a -0 pivot fails either way)
    Quu[0][0] += mu;
    Quu[1][1] += mu;
    constexpr int NR = sizeof(R) == 4 ? 1 : 2;
    double Lc[M][M], invd[M];
    // a failure is recorded and the step runs on (the sweep stops at the end
    // of its chunk): no branch per step
    uint32_t bad = chol_fp64<M, NR>(Quu, Lc, invd) ? 0u : ST_CHOL_FAIL;
    // Q_ux on the lane's axes in control order: G[a][c][j], j = 0 position, 1 velocity
    R G[NA][M][2];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const bool a0 = GL == 1 ? a == 0 : h == 0;
      G[a][0][0] = a0 ? q[a].ga_p : q[a].gb_p;
      G[a][1][0] = a0 ? q[a].gb_p : q[a].ga_p;
      G[a][0][1] = a0 ? q[a].ga_v : q[a].gb_v;
      G[a][1][1] = a0 ? q[a].gb_v : q[a].ga_v;
    }
    R kk[M], Kc[NA][M][2];
    bool solved = false;
    if constexpr (sizeof(R) == 4) {
      // FP32 solves on the FP64 factor rounded to FP32 (as in riccati_step)
      float lf[M][M], ivf[M];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        ivf[i] = float(invd[i]);
#pragma unroll
        for (int j = 0; j < M; ++j) lf[i][j] = float(Lc[i][j]);
      }
      auto solve = [&](float (&b)[M]) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
          float v = b[i];
#pragma unroll
          for (int k2 = 0; k2 < i; ++k2) v -= lf[i][k2] * b[k2];
          b[i] = v * ivf[i];
        }
#pragma unroll
        for (int i = M - 1; i >= 0; --i) {
          float v = b[i];
#pragma unroll
          for (int k2 = i + 1; k2 < M; ++k2) v += lf[k2][i] * b[k2];
          b[i] = v * -ivf[i];
        }
      };
      float col[M] = {U0, U1};
      solve(col);
      kk[0] = col[0];
      kk[1] = col[1];
      solved = true;
      if constexpr (BOX) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
          const double d = double(kk[i]);
          solved = solved && d >= -umax - double(u[i]) && d <= umax - double(u[i]);
        }
      }
      if (solved) {
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            float c2[M] = {G[a][0][j], G[a][1][j]};
            solve(c2);
            Kc[a][0][j] = c2[0];
            Kc[a][1][j] = c2[1];
          }
      }
    }
    if (!solved) {
      double col[M] = {double(U0), double(U1)};
      chol_solve_neg_fp64<M>(Lc, invd, col);
      unsigned held = 0;
      if constexpr (BOX) {
        double g[M], lo[M], hi[M];
        g[0] = double(U0);
        g[1] = double(U1);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          lo[i] = -umax - double(u[i]);
          hi[i] = umax - double(u[i]);
        }
        if (!box_qp<M, NR>(Quu, g, lo, hi, col, held, Lc, invd) && !bad) bad = ST_CHOL_FAIL;
      }
      kk[0] = R(col[0]);
      kk[1] = R(col[1]);
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          double c2[M];
#pragma unroll
          for (int i = 0; i < M; ++i) c2[i] = ((held >> i) & 1u) ? 0.0 : double(G[a][i][j]);
          chol_solve_neg_fp64<M>(Lc, invd, c2);
          Kc[a][0][j] = R(c2[0]);
          Kc[a][1][j] = R(c2[1]);
        }
    }
    // the other axis' gain columns
    R Ko[NA][M][2];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int c = 0; c < M; ++c)
#pragma unroll
        for (int j = 0; j < 2; ++j) Ko[a][c][j] = GL == 1 ? Kc[NA - 1 - a][c][j] : pair_swap(Kc[a][c][j]);
    // all ten checked without branches (the pair checks the same values)
    bool fin = dfinite(kk[0]) & dfinite(kk[1]);
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
      for (int j = 0; j < 2; ++j) fin = fin & dfinite(Kc[0][c][j]) & dfinite(Ko[0][c][j]);
    if (!fin && !bad) bad = ST_NONFINITE;
    if (store) {
      // K row c over (p_0, p_1, v_0, v_1): every lane stores its own axis'
      // columns (the group's pairs store the same values at the same
      // addresses), so no lane waits on a branch
      R* dK = Kp(w, k, s);
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const int ax = GL == 1 ? a : h;
#pragma unroll
        for (int c = 0; c < M; ++c) {
          dK[c * N + ax] = Kc[a][c][0];
          dK[c * N + ax + 2] = Kc[a][c][1];
        }
      }
      st(kp(w, k, s), kk);
    }
    // Q_ux^T K on (this axis, other axis), then the update
    R S[NA][2][2];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) S[a][i][j] = G[a][0][i] * Ko[a][0][j] + G[a][1][i] * Ko[a][1][j];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      // the other axis' products, transposed into this axis' orientation
      R Tt[2][2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) Tt[i][j] = GL == 1 ? S[NA - 1 - a][j][i] : pair_swap(S[a][j][i]);
      AxisP& P = AP[a];
      const AxisQ& Q = q[a];
      P.pp = Q.Qpp + (G[a][0][0] * Kc[a][0][0] + G[a][1][0] * Kc[a][1][0]);
      P.pv = Q.Qpv + (G[a][0][0] * Kc[a][0][1] + G[a][1][0] * Kc[a][1][1]);
      P.vv = Q.Qvv + (G[a][0][1] * Kc[a][0][1] + G[a][1][1] * Kc[a][1][1]);
      P.xpp = Q.Xpp + R(0.5) * (S[a][0][0] + Tt[0][0]);
      P.xpv = Q.Xpv + R(0.5) * (S[a][0][1] + Tt[0][1]);
      P.xvp = Q.Xvp + R(0.5) * (S[a][1][0] + Tt[1][0]);
      P.xvv = Q.Xvv + R(0.5) * (S[a][1][1] + Tt[1][1]);
      P.qp = Q.Qxp + (G[a][0][0] * kk[0] + G[a][1][0] * kk[1]);
      P.qv = Q.Qxv + (G[a][0][1] * kk[0] + G[a][1][1] * kk[1]);
    }
    return bad;
  }

  __device__ static __forceinline__ void stage_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }

  // One Riccati sweep over the iterate in buffer `buf`; writes K_k, k_k.
  // For a model whose per-step derivatives are worth staging (ND > 0) the
  // sweep runs in chunks of C steps: the GL lanes of the group first evaluate
  // the derivative blocks of the chunk's steps in parallel into the group's
  // LDS area `stage` ([C][ND]), then every lane runs the (serial, redundant)
  // recursion over them; the (x_k, u_k) of the next chunk are loaded while the
  // recursion runs.  Every group width goes through the same code, so
  // results do not depend on the width.  Models with constant derivatives
  // (ND = 0) evaluate them per step, with (x_k, u_k) prefetched two steps ahead.
  //
  // With BOX the staged chunk also carries the controls u_k ([C][M] after the
  // derivative blocks) for the bounded control step.
  template <int GL, bool BOX>
  __device__ static uint32_t backward(const Model& mdl, const LaneState<R>& w, int s, int T, int buf, R eps,
                                      bool store, R* stage, int r, double mu, double umax) {
    constexpr int ND = Model::ND;
    constexpr bool staged = ND > 0;
    constexpr int C = staged ? GL * (ND <= 8 ? 2 : 1) : 1;
    R P[N][N], p[N];
    {
      R xT[N];
      ld(xT, xp(w, buf, T, s));
      mdl.term_derivs(xT, p, P, eps, true);
    }
    if constexpr (staged) {
      // axis-pair systems: the blocks of the terminal P, p for the lane's axes
      constexpr int NA = GL == 1 ? 2 : 1;
      const int h = GL == 1 ? 0 : (r & 1);
      AxisP AP[NA];
      R dt = R(0), dt2 = R(0), ev = R(0), ru = R(0);
      if constexpr (Sys::kSemiImplicit) dt = mdl.step_dt();
      if constexpr (Sys::kAxisPairs) {
        dt = mdl.step_dt();
        dt2 = dt * dt;
        ev = mdl.vel_hess(eps);
        ru = mdl.ctrl_hess(eps);
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          const bool one = (GL == 1 ? a : h) == 1;
          AP[a].pp = one ? P[1][1] : P[0][0];
          AP[a].pv = one ? P[1][3] : P[0][2];
          AP[a].vv = one ? P[3][3] : P[2][2];
          AP[a].xpp = one ? P[1][0] : P[0][1];
          AP[a].xpv = one ? P[1][2] : P[0][3];
          AP[a].xvp = one ? P[3][0] : P[2][1];
          AP[a].xvv = one ? P[3][2] : P[2][3];
          AP[a].qp = one ? p[1] : p[0];
          AP[a].qv = one ? p[3] : p[2];
        }
      }
      // (x_k, u_k) of the lane's steps of the next chunk are loaded while the
      // current chunk's recursion runs
      constexpr int PB = C / GL > 0 ? C / GL : 1;
      R px[PB][N], pu[PB][M];
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const int k = T - 1 - (r + q * GL);
        if (k >= 0) {
          ld(px[q], xp(w, buf, k, s));
          ld(pu[q], up(w, buf, k, s));
        }
      }
      uint32_t chunk_bad = 0;  // first failure in the chunk (axis-pair steps)
      for (int kc = T - 1; kc >= 0; kc -= C) {
#pragma unroll
        for (int q = 0; q < PB; ++q)
          if (kc - (r + q * GL) >= 0) {
            mdl.pack_derivs(px[q], pu[q], stage + (r + q * GL) * ND, eps);
            if constexpr (BOX) st(stage + C * ND + (r + q * GL) * M, pu[q]);
          }
#pragma unroll
        for (int q = 0; q < PB; ++q) {
          const int k = kc - C - (r + q * GL);
          if (k >= 0) {
            ld(px[q], xp(w, buf, k, s));
            ld(pu[q], up(w, buf, k, s));
          }
        }
        stage_sync();
        const int cn = kc + 1 < C ? kc + 1 : C;
        for (int q = 0; q < cn; ++q) {
          R uq[M] = {};
          if constexpr (BOX) ld(uq, stage + C * ND + q * M);
          if constexpr (Sys::kAxisPairs) {
            const uint32_t b =
                axis_step<GL, BOX>(w, s, kc - q, stage + q * ND, uq, AP, h, dt, dt2, ev, ru, true, mu, umax);
            if (!chunk_bad) chunk_bad = b;
          } else if constexpr (Sys::kSemiImplicit) {
            R V[N / 2][N], W[N / 2][M], lx[N], lu[M], Qc[N][N], Rc[M][M];
            mdl.unpack_derivs_si(stage + q * ND, V, W, lx, lu, Qc, Rc, eps);
            // every lane stores the gains (the group's lanes hold the same
            // values): no branch per step; a failure ends the sweep at the
            // end of the chunk
            uint32_t b;
            if constexpr (GL >= 2 && N == 6 && M == 3)
              b = riccati_step_si_pair<BOX>(w, s, kc - q, dt, V, W, lx, lu, Qc, Rc, P, p, mu, uq, umax, r & 1);
            else
              b = riccati_step_si<BOX>(w, s, kc - q, dt, V, W, lx, lu, Qc, Rc, P, p, true, mu, uq, umax);
            if (!chunk_bad) chunk_bad = b;
          } else {
            R A[N][N], B[N][M], lx[N], lu[M], Qc[N][N], Rc[M][M];
            mdl.unpack_derivs(stage + q * ND, A, B, lx, lu, Qc, Rc, eps);
            const uint32_t bad = riccati_step<BOX>(w, s, kc - q, A, B, lx, lu, Qc, Rc, P, p, store, mu, uq, umax);
            if (bad) return bad;
          }
        }
        stage_sync();
        if (chunk_bad) return chunk_bad;
      }
      return 0;
    }
    // unstaged: software prefetch of the next two steps' (x, u)
    R xn[N], un[M], xn2[N], un2[M];
    ld(xn, xp(w, buf, T - 1, s));
    ld(un, up(w, buf, T - 1, s));
    if (T > 1) {
      ld(xn2, xp(w, buf, T - 2, s));
      ld(un2, up(w, buf, T - 2, s));
    }
    for (int k = T - 1; k >= 0; --k) {
      R x[N], u[M];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        x[i] = xn[i];
        xn[i] = xn2[i];
      }
#pragma unroll
      for (int i = 0; i < M; ++i) {
        u[i] = un[i];
        un[i] = un2[i];
      }
      if (k > 1) {
        ld(xn2, xp(w, buf, k - 2, s));
        ld(un2, up(w, buf, k - 2, s));
      }
      R A[N][N], B[N][M], lx[N], lu[M], Qc[N][N], Rc[M][M];
      mdl.jac(x, u, A, B);
      mdl.cost_derivs(x, u, lx, lu, Qc, Rc, eps, true);
      const uint32_t bad = riccati_step<BOX>(w, s, k, A, B, lx, lu, Qc, Rc, P, p, store, mu, u, umax);
      if (bad) return bad;
    }
    return 0;
  }

  // ------------------------------------------------------------------ line search trial
  // Step record of the line-search stream: x_k, u_k, K_k, k_k, padded to 16 B.
  static constexpr int SW = N + M + M * N + M;
  static constexpr int SWP = (SW + 3) & ~3;
  // steps each lane loads per chunk
  static constexpr int PT = SWP * int(sizeof(R)) <= 64 ? 2 : 1;

  __device__ static __forceinline__ void load_step(const LaneState<R>& w, int buf, int k, int s, R (&v)[SW]) {
    const R* a = xp(w, buf, k, s);
    const R* b = up(w, buf, k, s);
    const R* c = Kp(w, k, s);
    const R* d = kp(w, k, s);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = a[i];
#pragma unroll
    for (int i = 0; i < M; ++i) v[N + i] = b[i];
#pragma unroll
    for (int i = 0; i < M * N; ++i) v[N + M + i] = c[i];
#pragma unroll
    for (int i = 0; i < M; ++i) v[N + M + M * N + i] = d[i];
  }
  __device__ static __forceinline__ void put_step(R* dst, const R (&v)[SW]) {
#pragma unroll
    for (int i = 0; i < SW; ++i) dst[i] = v[i];
  }

  // Closed-loop rollout with step alpha from the iterate in `buf`; returns
  // J_hat in FP64 (NaN-propagating).  With `write` the trial trajectory goes to
  // buffer `nb`.  With non-negative costs a trial stops at the end of the
  // chunk in which its partial sum reaches J: its total could only be
  // larger, so the accept/reject decision is unchanged; `steps` is the
  // number of steps up to that first failing one.  A stopped trial's J_hat
  // is then not its total (it is rejected either way), and a writing trial
  // may have written a few steps past it into a buffer that does not become
  // the iterate.
  //
  // The iterate's step records stream through the group's LDS ring `ring`
  // ([2][CT][SWP]) in chunks of CT = GL * PT steps: lane r loads steps
  // r, r + GL, ... of the next chunk from HBM while the current chunk is
  // rolled out, so the loads' latency is covered by a chunk of work.  The
  // group keeps streaming while any of its lanes is still rolling out.
  //
  // With BOX the trial's controls are clamped into [-umax, umax] (eq. 1).
  // REPLAY rolls out a step whose cost is already known only to write it:
  // the same controls and states, no costs (returns 0).
  template <int GL, bool BOX, bool REPLAY = false>
  __device__ static double trial(const Model& mdl, const LaneState<R>& w, int s, int T, int buf, int nb,
                                 R alpha, double Jcur, bool write, int& steps, R* ring, int r, int gbase,
                                 R umax) {
    constexpr int CT = GL * PT;
    const unsigned long long gmask = (GL >= 64) ? ~0ull : ((1ull << GL) - 1ull);
    R xh[N];
    ld(xh, xp(w, buf, 0, s));
    double Jh = 0.0;
    bool live = true;
    steps = T;
    R nxt[PT][SW];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const int k = r + q * GL;
      if (k < T) {
        load_step(w, buf, k, s, nxt[q]);
        put_step(ring + (r + q * GL) * SWP, nxt[q]);
      }
    }
    stage_sync();
    for (int kc = 0, c = 0; kc < T; kc += CT, ++c) {
      const R* cur = ring + (c & 1) * CT * SWP;
      R* nx = ring + ((c + 1) & 1) * CT * SWP;
      const bool more = kc + CT < T;
      if (more) {
#pragma unroll
        for (int q = 0; q < PT; ++q) {
          const int k = kc + CT + r + q * GL;
          if (k < T) load_step(w, buf, k, s, nxt[q]);
        }
      }
      if (live) {
        const int cn = T - kc < CT ? T - kc : CT;
        // the stop test is taken at the end of the chunk, so that no step
        // waits on the branch of the one before (steps past the first
        // failing one change neither the decision nor the counts)
        bool failed = false;
#pragma unroll 2
        for (int q = 0; q < cn; ++q) {
          const R* v = cur + q * SWP;
          const int k = kc + q;
          R dx[N], uh[M];
#pragma unroll
          for (int i = 0; i < N; ++i) dx[i] = xh[i] - v[i];
#pragma unroll
          for (int i = 0; i < M; ++i) {
            R u = v[N + i] + alpha * v[N + M + M * N + i];
#pragma unroll
            for (int j = 0; j < N; ++j) u += v[N + M + i * N + j] * dx[j];
            if constexpr (BOX) u = clamp_nan(u, umax);
            uh[i] = u;
          }
          if constexpr (!REPLAY) Jh += double(mdl.cost(xh, uh));
          R xn[N];
          mdl.dyn(xh, uh, xn);
#pragma unroll
          for (int i = 0; i < N; ++i) xh[i] = xn[i];
          if (write) {
            st(up(w, nb, k, s), uh);
            st(xp(w, nb, k + 1, s), xh);
          }
          if constexpr (Sys::kNonNegCost && !REPLAY) {
            const bool f = !(Jh < Jcur);
            steps = (f && !failed) ? k + 1 : steps;
            failed = failed || f;
          }
        }
        if (failed) live = false;
      }
      const unsigned long long any = (__ballot(live) >> gbase) & gmask;
      if (!any || !more) break;
#pragma unroll
      for (int q = 0; q < PT; ++q) {
        const int k = kc + CT + r + q * GL;
        if (k < T) put_step(nx + (r + q * GL) * SWP, nxt[q]);
      }
      stage_sync();
    }
    if constexpr (!REPLAY)
      if (live) Jh += double(mdl.term(xh));
    return Jh;
  }
};

struct FinalOut {
  double* X;      // [B][Tmax+1][N]
  double* U;      // [B][Tmax][M]
  double* J;      // [B]
  int32_t* iters;
  uint32_t* status;
  double* Vbar;   // [B][Tmax+1] or null
  double* Vx;     // [B][Tmax+1][N] or null
  double* xK;     // [B][Tmax+1][N] or null
  double* trace;  // [B][max_iter+1] or null
  int32_t* work;  // [B][2] or null
};

// ====================================================================== kernels
// Warm start and initial rollout, GL lanes per instance: group g initialises
// slot slots[g] (or g) from caller instance perm[g] (or g).  The rollout runs
// in chunks of GL steps; every lane of the group steps through the chunk (the
// dynamics are a few operations per step) and lane r keeps step kc + r: it
// evaluates that step's stage cost and writes its (u_k, x_{k+1}), so that the
// group's stores fill whole lines of the slot-major workspace.  The stage
// costs are added in index order.  The warm start's controls are clamped into
// [-umax, umax] (eq. 1; umax may be infinite).
template <class Sys, class R, int GL>
__global__ void __launch_bounds__(64) lane_init(const double* __restrict__ prm, LaneState<R> w, int nthreads,
                                                const int32_t* __restrict__ slots, int Tmax,
                                                const int32_t* __restrict__ Tin, const int32_t* __restrict__ perm,
                                                const double* __restrict__ x0, const double* __restrict__ U0,
                                                int max_iter, double* __restrict__ trace, double umax) {
  using LN = Lane<Sys, R>;
  constexpr int N = Sys::N, M = Sys::M;
  static_assert(GL >= 1 && GL <= 64 && (GL & (GL - 1)) == 0, "group width");
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int gi = tid / GL, r = tid & (GL - 1);
  if (gi >= nthreads) return;  // whole groups leave together
  const int gbase = (threadIdx.x & 63) & ~(GL - 1);
  const int s = slots ? slots[gi] : gi;
  const typename LN::Model mdl{prm};
  const int b = perm ? perm[gi] : gi;
  const int Tr = Tin ? Tin[b] : Tmax;
  const bool badT = Tr < 1 || Tr > Tmax || Tr > w.Tcap;
  const int T = badT ? 0 : Tr;  // an out-of-range horizon is never used as an index
  R x[N];
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = R(x0[size_t(b) * N + i]);
  for (int q = r; q < w.nbuf; q += GL) LN::st(LN::xp(w, q, 0, s), x);
  double J = 0.0;
  // a chunk's stage costs are gathered from their lanes at the chunk's end and
  // added to J after the next chunk's rollout (the same order of additions),
  // so that the rollout does not wait for the exchange
  double cprev[GL];
  int cnprev = 0;
  float oc = 0.f;  // this lane's steps' share of the iteration-order key
  for (int kc = 0; kc < T; kc += GL) {
    const int kr = kc + r;
    const int cn = T - kc < GL ? T - kc : GL;
    R ur[M], xr[N] = {}, xr1[N] = {};
#pragma unroll
    for (int i = 0; i < M; ++i)
      ur[i] = kr < T ? clamp_nan(U0 ? R(U0[(size_t(b) * Tmax + kr) * M + i]) : R(0), R(umax)) : R(0);
    // every lane steps through the whole chunk without a branch: past the
    // horizon the state stays at x_T (the extra steps are never kept)
#pragma unroll
    for (int q = 0; q < GL; ++q) {
      R u[M], xn[N];
#pragma unroll
      for (int i = 0; i < M; ++i) u[i] = GL == 1 ? ur[i] : __shfl(ur[i], gbase + q, 64);
      mdl.dyn(x, u, xn);
      const bool live = q < cn, mine = q == r;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        xr[i] = mine ? x[i] : xr[i];
        xr1[i] = mine ? xn[i] : xr1[i];
        x[i] = live ? xn[i] : x[i];
      }
    }
    double c = 0.0;
    if (r < cn) {
      if constexpr (Sys::kOrderCost) {
        R nc;
        c = double(mdl.cost(xr, ur, nc));
        oc += float(nc);
      } else {
        c = double(mdl.cost(xr, ur));
      }
      LN::st(LN::up(w, 0, kr, s), ur);
      LN::st(LN::xp(w, 0, kr + 1, s), xr1);
    }
#pragma unroll
    for (int q = 0; q < GL; ++q)
      if (q < cnprev) J += cprev[q];
#pragma unroll
    for (int q = 0; q < GL; ++q) cprev[q] = GL == 1 ? c : __shfl(c, gbase + q, 64);
    cnprev = cn;
  }
#pragma unroll
  for (int q = 0; q < GL; ++q)
    if (q < cnprev) J += cprev[q];
  // the group's sum of the order key (any order of additions: it only orders)
#pragma unroll
  for (int o = 1; o < GL; o <<= 1) oc += __shfl_xor(oc, o, 64);
  if (r != 0) return;
  J += double(mdl.term(x));
  uint32_t st = isfinite(J) ? 0u : ST_NONFINITE;
  if (badT) {
    st = ST_BAD_INPUT;
    J = __builtin_nan("");
  }
  if (st == 0 && max_iter <= 0) st = ST_MAX_ITER;
  w.T[s] = T;
  w.inst[s] = slots ? s : b;  // outputs of slot-addressed solves are indexed by slot
  w.J[s] = J;
  w.okey[s] = order_key(Tin != nullptr, T, J, oc, Tmax);
  w.iters[s] = 0;
  w.status[s] = st;
  w.cur[s] = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) w.work[4 * s + i] = 0;
  if (trace) trace[size_t(slots ? s : b) * (max_iter + 1)] = J;
}

template <class Sys, class R, int GL>
__device__ __forceinline__ void final_group(const double* __restrict__ prm, const LaneState<R>& w, int s, int b,
                                            int Ts, int buf, uint32_t st, double J, int iters,
                                            const int (&wk)[4], int r, int Tmax, int max_iter, int lookahead,
                                            const FinalOut& o);

// Up to `iters` iterations for every active slot, with GL lanes per instance.
// The GL lanes of a group run the backward sweep redundantly (identical
// arithmetic on identical data; the point mass splits each step over lane
// pairs by axis, and lanes holding the same gains all store them) and split
// the line search: in round q lane r tries alpha_j, j = q*GL + r.  The first
// j whose J_hat < J is taken (a wave ballot over the group), which is exactly
// the sequential rule.  Systems with their own trial buffers have every lane
// write its trial and the accepted lane's buffer becomes the iterate; the
// others write alpha = 1 while trying it and roll another accepted step out
// once more to write it.  `slots` (optional) maps the group index to a slot,
// for sparse slot sets.
//
// BOX selects the variant with the control bound of eq. 1 (sp.umax finite).
//
// FIN: the launch is the solve's last, and each group finalises its slot
// (final_group) as soon as it has stopped iterating, while other groups still
// iterate; every slot of the list is finalised, frozen ones included.
template <class Sys, class R, int GL, bool BOX, bool FIN = false>
__global__ void __launch_bounds__(64) lane_iterate(const double* __restrict__ prm, LaneState<R> w,
                                                   int nslots, const int32_t* __restrict__ slots,
                                                   SolveParams sp, int iters_this_launch, IterTrace tr,
                                                   int Tmax = 0, int lookahead = 0, FinalOut fo = {}) {
  using LN = Lane<Sys, R>;
  static_assert(GL >= 1 && GL <= 16 && (GL & (GL - 1)) == 0, "group width must be a power of two <= 16");
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int gi = tid / GL;
  const int r = tid & (GL - 1);
  if (gi >= nslots) return;  // whole groups leave together
  const int s = slots ? slots[gi] : gi;
  uint32_t st = w.status[s];
  if (st && !FIN) return;
  const bool lead = (r == 0);
  const int gbase = (threadIdx.x & 63) & ~(GL - 1);  // first lane of this group in the wave
  const typename LN::Model mdl{prm};
  // LDS staging area of the backward sweep's derivative blocks, per group
  constexpr int ND = LN::Model::ND;
  constexpr bool staged = ND > 0;
  constexpr int C = staged ? GL * (ND <= 8 ? 2 : 1) : 1;
  // one LDS area per group, shared by the backward sweep's derivative blocks
  // and the line search's step-record ring; the area stride is padded so that
  // the groups of a wave start on different banks
  constexpr int CT = GL * LN::PT;
  constexpr int DS = staged ? C * (ND + (BOX ? LN::M : 0)) : 0;
  constexpr int AREA = DS > 2 * CT * LN::SWP ? DS : 2 * CT * LN::SWP;
  constexpr int STRIDE = (AREA + 31) / 32 * 32 + 4;
  __shared__ __align__(16) R stage_mem[(64 / GL) * STRIDE];
  R* stage = stage_mem + (gbase / GL) * STRIDE;
  const int T = w.T[s];
  const int b = w.inst[s];
  double J = w.J[s];
  int iters = w.iters[s];
  int buf = w.cur[s];
  int nsweep = w.work[4 * s], npass = w.work[4 * s + 1], nread = w.work[4 * s + 2], nwrite = w.work[4 * s + 3];
  const R eps = R(sp.eps);
  const bool lm = sp.reg == 1;
  // the Levenberg-Marquardt parameter carries over between launches; a slot
  // that has not swept yet starts from mu0
  double mu = lm ? (nsweep == 0 ? sp.mu0 : w.mu[s]) : 0.0;
  for (int g = 0; g < iters_this_launch && st == 0; ++g) {
    if (iters >= sp.max_iter) {
      st = ST_MAX_ITER;
      break;
    }
    int acc = -1, nbuf_acc = buf;
    double Jn = J;
    uint32_t fail = 0;
    // one sweep and line search; in the Levenberg-Marquardt variant a failed
    // Cholesky or line search multiplies mu by mu_fac and retries while mu
    // stays within mu_max (the group's lanes decide alike)
    for (;;) {
      ++nsweep;
      const uint32_t bad = LN::template backward<GL, BOX>(mdl, w, s, T, buf, eps, lead, stage, r, mu, sp.umax);
      if (bad) {
        if (lm && bad == ST_CHOL_FAIL && mu * sp.mu_fac <= sp.mu_max) {
          mu *= sp.mu_fac;
          continue;
        }
        fail = bad;
        break;
      }
      acc = -1;
      nbuf_acc = buf;
      Jn = J;
      if constexpr (Sys::kOwnTrialBuffers) {
        // rounds of GL parallel trials; lane r of the group rolls out into its own
        // trajectory buffer, so the accepted trial is already written and becomes
        // the iterate (no second rollout); one call site of the rollout keeps the
        // register footprint down
        const int wb = (buf + 1 + r) % w.nbuf;  // never the iterate's buffer (GL < nbuf)
        for (int j0 = 0; j0 < sp.ls_trials && acc < 0; j0 += GL) {
          const int j = j0 + r;
          double Jh = __builtin_nan("");
          int steps = 0;
          if (j < sp.ls_trials) {
            double alpha = 1.0;
            for (int q = 0; q < j; ++q) alpha *= sp.beta;
            Jh = LN::template trial<GL, BOX>(mdl, w, s, T, buf, wb, R(alpha), J, true, steps, stage, r, gbase,
                                             R(sp.umax));
          }
          ++npass;
          // every lane writes what it rolled out; the lanes of a group read the
          // same data, so a round reads as many steps as its longest trial
          int total = steps, longest = steps;
#pragma unroll
          for (int o = 1; o < GL; o <<= 1) {
            total += __shfl_xor(total, o, 64);
            longest = max(longest, __shfl_xor(longest, o, 64));
          }
          nwrite += total;
          nread += longest;
          const bool ok = isfinite(Jh) && Jh < J;
          unsigned long long bits = __ballot(ok);
          bits = (bits >> gbase) & ((GL >= 64) ? ~0ull : ((1ull << GL) - 1ull));
          if (bits) {
            const int rs = __ffsll(bits) - 1;
            acc = j0 + rs;
            Jn = __shfl(Jh, gbase + rs, 64);
            nbuf_acc = (buf + 1 + rs) % w.nbuf;
          }
        }
      } else {
        // rounds of GL parallel trials, then (if the accepted step is not alpha = 1,
        // whose lane wrote while trying it) one replay of the accepted step
        // that writes it: the same controls and states, without the costs
        // (its J_hat is known from the round)
        for (int j0 = 0;;) {
          const int j = j0 + r;
          double Jh = __builtin_nan("");
          int steps = 0;
          if (j < sp.ls_trials) {
            double alpha = 1.0;
            for (int q = 0; q < j; ++q) alpha *= sp.beta;
            // alpha = 1 (j == 0) is written while it runs, as is every trial
            // of a one-lane group
            Jh = LN::template trial<GL, BOX>(mdl, w, s, T, buf, buf ^ 1, R(alpha), J, j == 0 || GL == 1, steps,
                                             stage, r, gbase, R(sp.umax));
          }
          ++npass;
          // the lanes of a group read the same data: a round moves as many steps
          // as its longest trial; only the alpha = 1 trial (or every trial of a
          // one-lane group) writes
          if (j0 == 0 || GL == 1) nwrite += (GL == 1) ? steps : __shfl(steps, gbase, 64);
          int longest = steps;
#pragma unroll
          for (int o = 1; o < GL; o <<= 1) longest = max(longest, __shfl_xor(longest, o, 64));
          nread += longest;
          const bool ok = isfinite(Jh) && Jh < J;
          unsigned long long bits = __ballot(ok);
          bits = (bits >> gbase) & ((1ull << GL) - 1);
          if (bits) {
            const int rs = __ffsll(bits) - 1;
            acc = j0 + rs;
            Jn = __shfl(Jh, gbase + rs, 64);
          }
          j0 += GL;
          if (acc == 0 || (acc > 0 && GL == 1) || (acc < 0 && j0 >= sp.ls_trials)) break;
          if (acc > 0) {
            // the group's lead lane writes the replay
            double alpha = 1.0;
            for (int q = 0; q < acc; ++q) alpha *= sp.beta;
            int rs = 0;
            LN::template trial<GL, BOX, true>(mdl, w, s, T, buf, buf ^ 1, R(alpha), __builtin_inf(), lead, rs,
                                              stage, r, gbase, R(sp.umax));
            ++npass;
            nread += rs;
            nwrite += rs;
            break;
          }
        }
        nbuf_acc = buf ^ 1;
      }
      if (acc < 0) {
        if (lm && mu * sp.mu_fac <= sp.mu_max) {
          mu *= sp.mu_fac;
          continue;
        }
        fail = ST_LS_FAILED;
      }
      break;
    }
    if (tr.j && lead) tr.j[size_t(b) * sp.max_iter + iters] = fail ? -1 : acc;
    if (fail) {
      st = fail;
      break;
    }
    if (lm) mu = fmax(mu / sp.mu_fac, sp.mu0);
    buf = nbuf_acc;
    const double Jold = J;
    J = Jn;
    ++iters;
    if (tr.J && lead) tr.J[size_t(b) * (sp.max_iter + 1) + iters] = J;
    if (sp.stop_mode == 1 && (Jold - J) <= sp.rtol * fabs(Jold)) {
      st = ST_CONVERGED;
      break;
    }
    if (iters >= sp.max_iter) st = ST_MAX_ITER;
  }
  if (lead) {
    w.J[s] = J;
    w.iters[s] = iters;
    w.status[s] = st;
    w.cur[s] = buf;
    w.work[4 * s] = nsweep;
    w.work[4 * s + 1] = npass;
    w.work[4 * s + 2] = nread;
    w.work[4 * s + 3] = nwrite;
    w.mu[s] = mu;
  }
  if constexpr (FIN) {
    const int wk[4] = {nsweep, npass, nread, nwrite};
    final_group<Sys, R, GL>(prm, w, s, b, T, buf, st, J, iters, wk, r, Tmax, sp.max_iter, lookahead, fo);
  }
}


// GL lanes per instance (one group of a wave): the lanes split the output
// copies and the stage costs by step; the costate recursion walks back over
// the final trajectory in every lane of the group, fed chunk by chunk by the
// group's lanes (a serial chain; lane 0 writes it), and lane 0 forms the
// cost-to-go sums from the stage costs the group wrote, after a wave barrier.
// The outputs of slot s by its group (lane r of GL): the slot's state (output
// index b, horizon Ts, iterate buffer, status, J, iterations, work counters)
// comes in registers, so that the iteration kernel can call this for its own
// group right after its last iteration.
template <class Sys, class R, int GL>
__device__ __forceinline__ void final_group(const double* __restrict__ prm, const LaneState<R>& w, int s, int b,
                                            int Ts, int buf, uint32_t st, double J, int iters,
                                            const int (&wk)[4], int r, int Tmax, int max_iter, int lookahead,
                                            const FinalOut& o) {
  using LN = Lane<Sys, R>;
  constexpr int N = Sys::N, M = Sys::M;
  static_assert(GL >= 1 && GL <= 64 && (GL & (GL - 1)) == 0, "group width");
  const bool lead = r == 0;
  const typename LN::Model mdl{prm};
  if (st == 0) st = ST_MAX_ITER;  // iteration budget ended without freezing
  // an instance with an invalid horizon gets all-zero trajectory outputs
  const int T = (st & ST_BAD_INPUT) ? -1 : Ts;
  if (lead) {
    o.J[b] = J;
    o.iters[b] = iters;
    o.status[b] = st;
    if (o.work)
#pragma unroll
      for (int i = 0; i < 4; ++i) o.work[4 * b + i] = wk[i];
  }
  if (o.trace)
    for (int i = iters + 1 + r; i <= max_iter; i += GL) o.trace[size_t(b) * (max_iter + 1) + i] = J;
  // copies, step k by lane k % GL; a lane issues the loads of CB of its
  // steps before their stores, so that it waits for memory once per batch
  double* Xo = o.X + size_t(b) * (Tmax + 1) * N;
  double* Uo = o.U + size_t(b) * Tmax * M;
  const int K = lookahead <= 0 ? T : lookahead;
  double* xo = o.xK ? o.xK + size_t(b) * (Tmax + 1) * N : nullptr;
  constexpr int CB = 4;
  for (int k0 = r; k0 <= Tmax; k0 += GL * CB) {
    R xv[CB][N], xkv[CB][N], uv[CB][M];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int k = k0 + c * GL;
      if (k <= T) {
        LN::ld(xv[c], LN::xp(w, buf, k, s));
        if (xo) LN::ld(xkv[c], LN::xp(w, buf, k + K < T ? k + K : T, s));
      }
      if (k < T) LN::ld(uv[c], LN::up(w, buf, k, s));
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int k = k0 + c * GL;
      if (k <= Tmax) {
        const bool in = k <= T;
#pragma unroll
        for (int i = 0; i < N; ++i) Xo[k * N + i] = in ? double(xv[c][i]) : 0.0;
        if (xo)
#pragma unroll
          for (int i = 0; i < N; ++i) xo[k * N + i] = in ? double(xkv[c][i]) : 0.0;
      }
      if (k < Tmax) {
        const bool in = k < T;
#pragma unroll
        for (int i = 0; i < M; ++i) Uo[k * M + i] = in ? double(uv[c][i]) : 0.0;
      }
    }
  }
  double* Vo = o.Vbar ? o.Vbar + size_t(b) * (Tmax + 1) : nullptr;
  double* Lo = o.Vx ? o.Vx + size_t(b) * (Tmax + 1) * N : nullptr;
  // zero past the horizon (everything for an invalid one)
  for (int k = (T < 0 ? 0 : T + 1) + r; k <= Tmax; k += GL) {
    if (Vo) Vo[k] = 0.0;
    if (Lo)
#pragma unroll
      for (int i = 0; i < N; ++i) Lo[size_t(k) * N + i] = 0.0;
  }
  if (T < 0 || (!Vo && !Lo)) return;
  // stage costs c_k (k < T), turned into cost-to-go sums below (written by
  // the costate walk's per-step pass where it has one)
  const bool costs_in_walk = Sys::kConstJac && Lo;
  const bool sums_in_walk = costs_in_walk && Vo && K >= T;
  if (Vo && !costs_in_walk)
    for (int k = r; k < T; k += GL) {
      R x[N], u[M];
      LN::ld(x, LN::xp(w, buf, k, s));
      LN::ld(u, LN::up(w, buf, k, s));
      Vo[k] = double(mdl.cost(x, u));
    }
  // costate lambda_T = d l_T/dx, lambda_k = l_x + A_k^T lambda_{k+1}
  // (unclipped first derivatives)
  R lam[N];
  R xT[N];
  LN::ld(xT, LN::xp(w, buf, T, s));
  {
    R Qd[N][N];
    mdl.term_derivs(xT, lam, Qd, R(0), false);
  }
  const double cT = double(mdl.term(xT));
  if (Lo) {
    if (lead)
#pragma unroll
      for (int i = 0; i < N; ++i) Lo[size_t(T) * N + i] = double(lam[i]);
    // the chain walks back in chunks of GL steps: lane q of the group loads
    // step kc - q (the next chunk is loaded while this one runs) and the chain
    // takes each step's (x, u) from its lane by a wave shuffle.  When f_x does
    // not depend on (x, u), lane q evaluates the cost gradient of its step for
    // the chunk at once and the chain takes that instead.
    const int gbase = (threadIdx.x & 63) & ~(GL - 1);
    R Ac[N][N] = {};
    if constexpr (Sys::kConstJac) {
      R Bc[N][M];
      mdl.jac(xT, nullptr, Ac, Bc);
    }
    // full cost-to-go as suffix sums in the walk's own (backward) order
    double vacc = cT, vmine = 0.0;
    R lmine[N] = {};
    if (sums_in_walk && lead) Vo[T] = cT;
    R xq[N] = {}, uq[M] = {}, xn[N] = {}, un[M] = {};
    if (T - 1 - r >= 0) {
      LN::ld(xq, LN::xp(w, buf, T - 1 - r, s));
      LN::ld(uq, LN::up(w, buf, T - 1 - r, s));
    }
    for (int kc = T - 1; kc >= 0; kc -= GL) {
      if (kc - GL - r >= 0) {
        LN::ld(xn, LN::xp(w, buf, kc - GL - r, s));
        LN::ld(un, LN::up(w, buf, kc - GL - r, s));
      }
      const int qn = kc + 1 < GL ? kc + 1 : GL;
      R lq[N] = {};
      double cq = 0.0;
      if constexpr (Sys::kConstJac) {
        if (kc - r >= 0) {
          R lu[M], Qd[N][N], Rd[M][M];
          mdl.cost_derivs(xq, uq, lq, lu, Qd, Rd, R(0), false);
          cq = double(mdl.cost(xq, uq));
          if (Vo && !sums_in_walk) Vo[kc - r] = cq;
        }
      }
      for (int q = 0; q < qn; ++q) {
        const int k = kc - q;
        R A[N][N], lx[N];
        if constexpr (Sys::kConstJac) {
#pragma unroll
          for (int i = 0; i < N; ++i) {
            lx[i] = __shfl(lq[i], gbase + q, 64);
#pragma unroll
            for (int j = 0; j < N; ++j) A[i][j] = Ac[i][j];
          }
          if (sums_in_walk) {
            vacc = __shfl(cq, gbase + q, 64) + vacc;
            if (q == r) vmine = vacc;
          }
        } else {
          R x[N], u[M];
#pragma unroll
          for (int i = 0; i < N; ++i) x[i] = __shfl(xq[i], gbase + q, 64);
#pragma unroll
          for (int i = 0; i < M; ++i) u[i] = __shfl(uq[i], gbase + q, 64);
          R B[N][M], lu[M], Qd[N][N], Rd[M][M];
          mdl.jac(x, u, A, B);
          mdl.cost_derivs(x, u, lx, lu, Qd, Rd, R(0), false);
        }
        R ln[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
          R v = lx[i];
#pragma unroll
          for (int t = 0; t < N; ++t)
            if (Sys::a_nz(t, i)) v += A[t][i] * lam[t];
          ln[i] = v;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) lam[i] = ln[i];
        // every lane walks the chain; lane q keeps step kc - q for the
        // chunk's stores below
        if (q == r)
#pragma unroll
          for (int i = 0; i < N; ++i) lmine[i] = ln[i];
      }
      // the chunk's costates (and cost-to-go) by the lanes of their steps:
      // contiguous stores instead of one lane's per-step pieces
      if (kc - r >= 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) Lo[size_t(kc - r) * N + i] = double(lmine[i]);
        if (sums_in_walk) Vo[kc - r] = vmine;
      }
#pragma unroll
      for (int i = 0; i < N; ++i) xq[i] = xn[i];
#pragma unroll
      for (int i = 0; i < M; ++i) uq[i] = un[i];
    }
  }
  if (Vo && !sums_in_walk) {
    // the group's stage costs are in Vo (global memory): complete the stores
    // and order them before lane 0's loads (workgroup-scope fences around a
    // wave barrier)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (lead) {
      if (K >= T) {
        // full cost-to-go: suffix sums, the stage costs loaded eight at a
        // time ahead of their updates (same summation order)
        double acc = cT;
        Vo[T] = cT;
        int k = T - 1;
        for (; k >= 7; k -= 8) {
          double c[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) c[j] = Vo[k - j];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            acc = c[j] + acc;
            Vo[k - j] = acc;
          }
        }
        for (; k >= 0; --k) {
          acc = Vo[k] + acc;
          Vo[k] = acc;
        }
      } else {
        // K-step window: V_k = sum_{j=k}^{min(k+K,T)-1} c_j + [k+K >= T] c_T, in index order
        Vo[T] = cT;
        for (int k = 0; k < T; ++k) {
          const int end = k + K < T ? k + K : T;
          double v = 0.0;
          for (int j = k; j < end; ++j) v += Vo[j];
          if (k + K >= T) v += cT;
          Vo[k] = v;  // reads only indices >= k, which still hold stage costs
        }
      }
    }
  }
}

// Finalisation kernel: one group of GL lanes per slot (whole groups past
// nslots leave).
template <class Sys, class R, int GL>
__global__ void __launch_bounds__(64) lane_final(const double* __restrict__ prm, LaneState<R> w, int nslots,
                                                 const int32_t* __restrict__ slots, int Tmax, int max_iter,
                                                 int lookahead, FinalOut o) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int gi = tid / GL, r = tid & (GL - 1);
  if (gi >= nslots) return;  // whole groups leave together
  const int s = slots ? slots[gi] : gi;
  const int wk[4] = {w.work[4 * s], w.work[4 * s + 1], w.work[4 * s + 2], w.work[4 * s + 3]};
  final_group<Sys, R, GL>(prm, w, s, w.inst[s], w.T[s], w.cur[s], w.status[s], w.J[s], w.iters[s], wk, r, Tmax,
                          max_iter, lookahead, o);
}

}  // namespace cbic
