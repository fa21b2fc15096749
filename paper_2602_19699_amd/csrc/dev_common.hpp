// Device-side helpers shared by the solver kernels: precision traits, small
// fixed-size linear algebra (Cholesky of Q_uu, triangular solves) and the
// eigenvalue clip of paper Sec. IV-B eq. 7 for 2x2 and 3x3 symmetric blocks.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

// Model and small linear-algebra helpers are pure arithmetic: they compile for
// the device and, for host-side tests of the same code, for the host.
#define CBIC_HD __host__ __device__

namespace cbic {

enum : uint32_t {
  ST_CONVERGED = 1u,
  ST_MAX_ITER = 2u,
  ST_LS_FAILED = 4u,
  ST_NONFINITE = 8u,
  ST_CHOL_FAIL = 16u,
  ST_BAD_INPUT = 32u,
};

// Optional per-iteration records of a solve, written by the iteration kernels
// into the caller's arrays (indexed by instance).
struct IterTrace {
  double* J;   // [B][max_iter + 1]: cost after each accepted iteration, or null
  int32_t* j;  // [B][max_iter]: accepted line-search index j (alpha = beta^j) of
               // each iteration, -1 where the iteration failed, or null
};

// ---------------------------------------------------------------- math by precision
// FP64 (the plain form) uses the correctly rounded library functions.  FP32
// (the mixed form's rollouts and derivatives, device only) uses the hardware
// exponential (a few ulp) and the hardware sine/cosine after an additive
// range reduction to [-pi, pi] (Cody and Waite's method: 2 pi split in two
// FP32 parts, the multiple subtracted with fused multiply-adds), which keeps
// the error near 2^-21 absolute whatever the angle; the hardware pair alone
// scales its argument by 1/(2 pi) in FP32 and so loses |v| 2^-24 of absolute
// accuracy, about 1e-4 at the joint angles a spinning arm reaches.  From
// |v| = 2^23 on, an FP32 angle holds no fraction of a radian and its sine has
// no meaning: the reduction returns NaN there, so that a rollout that spins
// up that far is non-finite, as its FP64 counterpart (which overflows on the
// way) is.
CBIC_HD __forceinline__ double dexp(double v) { return exp(v); }
__device__ __forceinline__ float dexp(float v) { return __expf(v); }
__device__ __forceinline__ float reduce_2pi(float v) {
  const float k = rintf(v * 0.159154943091895336f);  // nearest multiple of 2 pi
  const float r = fmaf(-k, 6.28318548202514648f, v);  // 2 pi rounded to FP32
  const float t = fmaf(-k, -1.74845553e-07f, r);      // 2 pi minus that rounding
  return fabsf(v) < 8388608.0f ? t : __builtin_nanf("");
}
CBIC_HD __forceinline__ double dsin(double v) { return sin(v); }
__device__ __forceinline__ float dsin(float v) { return __sinf(reduce_2pi(v)); }
CBIC_HD __forceinline__ double dcos(double v) { return cos(v); }
__device__ __forceinline__ float dcos(float v) { return __cosf(reduce_2pi(v)); }
CBIC_HD __forceinline__ void dsincos(double v, double* s, double* c) { sincos(v, s, c); }
__device__ __forceinline__ void dsincos(float v, float* s, float* c) { __sincosf(reduce_2pi(v), s, c); }
// the library sine/cosine in both precisions (measured faster than the
// hardware pair inside the quadruped's large kernel)
CBIC_HD __forceinline__ void dsincos_lib(double v, double* s, double* c) { sincos(v, s, c); }
__device__ __forceinline__ void dsincos_lib(float v, float* s, float* c) { sincosf(v, s, c); }
CBIC_HD __forceinline__ double dsqrt(double v) { return sqrt(v); }
CBIC_HD __forceinline__ float dsqrt(float v) { return sqrtf(v); }
CBIC_HD __forceinline__ bool dfinite(double v) { return isfinite(v); }
CBIC_HD __forceinline__ bool dfinite(float v) { return isfinite(v); }

template <class R>
CBIC_HD __forceinline__ R dmax(R a, R b) { return a > b ? a : b; }

// Squared relative off-diagonal size at which Jacobi rotations stop.
template <class R> struct JacobiTol;
template <> struct JacobiTol<double> { static constexpr double v = 1e-32; };
template <> struct JacobiTol<float> { static constexpr float v = 4e-15f; };

// ---------------------------------------------------------------- eigenvalue clip
// Clip of a symmetric 2x2 [[a,b],[b,c]]: eigenvalues below eps are raised to
// eps and the matrix is rebuilt.  Written as H + sum_{mu_i<eps} (eps-mu_i) v_i v_i^T,
// which leaves H bit-for-bit unchanged when no eigenvalue is clipped.
template <class R>
CBIC_HD __forceinline__ void clip_sym2(R& a, R& b, R& c, R eps) {
  if (eps < R(0)) return;  // a negative floor means no clipping (Levenberg-Marquardt variant)
  if (b == R(0)) {
    a = dmax(a, eps);
    c = dmax(c, eps);
    return;
  }
  const R half_tr = R(0.5) * (a + c);
  const R dh = R(0.5) * (a - c);
  const R rad = dsqrt(dh * dh + b * b);
  const R mu_lo = half_tr - rad, mu_hi = half_tr + rad;
  if (mu_lo >= eps) return;
  if (mu_hi < eps) {
    a = eps;
    b = R(0);
    c = eps;
    return;
  }
  // unit eigenvector of mu_lo, from the better-conditioned of two candidates
  R v0 = b, v1 = mu_lo - a;
  R w0 = mu_lo - c, w1 = b;
  if (v0 * v0 + v1 * v1 < w0 * w0 + w1 * w1) {
    v0 = w0;
    v1 = w1;
  }
  const R inv = R(1) / (v0 * v0 + v1 * v1);
  const R d = (eps - mu_lo) * inv;
  a += d * v0 * v0;
  b += d * v0 * v1;
  c += d * v1 * v1;
}

// Clip of a symmetric 3x3 (row-major h[9]).  Fast path: if H - eps I is
// positive definite (Cholesky succeeds) no eigenvalue is below eps and H is
// returned unchanged.  Otherwise cyclic Jacobi rotations give H = W S W^T and
// the clipped spectrum is recombined.
template <class R>
CBIC_HD __forceinline__ void clip_sym3(R h[9], R eps) {
  if (eps < R(0)) return;  // a negative floor means no clipping (Levenberg-Marquardt variant)
  {
    const R a00 = h[0] - eps, a11 = h[4] - eps, a22 = h[8] - eps;
    bool pd = a00 > R(0);
    if (pd) {
      const R l10 = h[3] / a00, l20 = h[6] / a00;
      const R d1 = a11 - l10 * h[3];
      pd = d1 > R(0);
      if (pd) {
        const R l21 = (h[7] - l20 * h[3]) / d1;
        const R d2 = a22 - l20 * h[6] - l21 * (h[7] - l20 * h[3]);
        pd = d2 > R(0);
      }
    }
    if (pd) return;
  }
  R a[3][3] = {{h[0], R(0.5) * (h[1] + h[3]), R(0.5) * (h[2] + h[6])},
               {R(0), h[4], R(0.5) * (h[5] + h[7])},
               {R(0), R(0), h[8]}};
  a[1][0] = a[0][1];
  a[2][0] = a[0][2];
  a[2][1] = a[1][2];
  R w[3][3] = {{R(1), R(0), R(0)}, {R(0), R(1), R(0)}, {R(0), R(0), R(1)}};
  for (int sweep = 0; sweep < 12; ++sweep) {
    const R off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const R dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (!(off > JacobiTol<R>::v * dia)) break;
#pragma unroll
    for (int pr = 0; pr < 3; ++pr) {
      const int p = pr == 2 ? 1 : 0;
      const int q = pr == 0 ? 1 : 2;
      const R apq = a[p][q];
      if (apq == R(0)) continue;
      const R tau = (a[q][q] - a[p][p]) / (R(2) * apq);
      const R t = (tau >= R(0) ? R(1) : R(-1)) / (fabs(tau) + dsqrt(R(1) + tau * tau));
      const R cs = R(1) / dsqrt(R(1) + t * t), sn = t * cs;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const R akp = a[k][p], akq = a[k][q];
        a[k][p] = cs * akp - sn * akq;
        a[k][q] = sn * akp + cs * akq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const R apk = a[p][k], aqk = a[q][k];
        a[p][k] = cs * apk - sn * aqk;
        a[q][k] = sn * apk + cs * aqk;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const R wkp = w[k][p], wkq = w[k][q];
        w[k][p] = cs * wkp - sn * wkq;
        w[k][q] = sn * wkp + cs * wkq;
      }
    }
  }
  const R s0 = dmax(a[0][0], eps), s1 = dmax(a[1][1], eps), s2 = dmax(a[2][2], eps);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const R v = w[i][0] * s0 * w[j][0] + w[i][1] * s1 * w[j][1] + w[i][2] * s2 * w[j][2];
      h[i * 3 + j] = v;
      h[j * 3 + i] = v;
    }
}

// ---------------------------------------------------------------- Cholesky (FP64)
// In-place lower Cholesky of the M x M symmetric matrix held in the upper
// triangle of a (a[i][j], j >= i).  Returns false on a non-positive or
// non-finite pivot.  L is returned in l[i][j], j <= i; diag holds 1/L_ii.
// NR Newton steps refine the reciprocal square roots: two give full FP64
// accuracy, one (relative error near 2^-44) suffices when the results are
// rounded to FP32.
template <int M, int NR = 2>
__device__ __forceinline__ bool chol_fp64(const double a[M][M], double l[M][M], double inv_diag[M]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double d = a[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= l[j][k] * l[j][k];
    ok = ok && (d > 0.0) && isfinite(d);
    // 1/sqrt(d) from the hardware estimate (relative error below 2^-22) and
    // Newton steps y <- y (3 - d y^2) / 2, each squaring the relative error;
    // sqrt(d) = d / sqrt(d)
    double inv = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < NR; ++it) inv = inv * (1.5 - 0.5 * d * inv * inv);
    const double ljj = d * inv;
    l[j][j] = ljj;
    inv_diag[j] = inv;
#pragma unroll
    for (int i = j + 1; i < M; ++i) {
      double v = a[j][i];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= l[i][k] * l[j][k];
      l[i][j] = v * inv;
    }
  }
  return ok;
}

// Solve (L L^T) y = b in place.
template <int M>
__device__ __forceinline__ void chol_solve_fp64(const double l[M][M], const double inv_diag[M], double b[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i) {
    double v = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= l[i][k] * b[k];
    b[i] = v * inv_diag[i];
  }
#pragma unroll
  for (int i = M - 1; i >= 0; --i) {
    double v = b[i];
#pragma unroll
    for (int k = i + 1; k < M; ++k) v -= l[k][i] * b[k];
    b[i] = v * inv_diag[i];
  }
}

// Solve (L L^T) y = b and return -y in b: the sign folds into the reciprocal
// diagonal of the back substitution (z = -y: z_i = (w_i + sum_k L_ki z_k) (-1/L_ii)),
// which rounds exactly as negating the solution would.
template <int M>
__device__ __forceinline__ void chol_solve_neg_fp64(const double l[M][M], const double inv_diag[M], double b[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i) {
    double v = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= l[i][k] * b[k];
    b[i] = v * inv_diag[i];
  }
#pragma unroll
  for (int i = M - 1; i >= 0; --i) {
    double v = b[i];
#pragma unroll
    for (int k = i + 1; k < M; ++k) v += l[k][i] * b[k];
    b[i] = v * -inv_diag[i];
  }
}

// Clamp into [-b, b], keeping NaN (a comparison with NaN is false).
template <class R>
__device__ __forceinline__ R clamp_nan(R v, R b) {
  return v < -b ? -b : (v > b ? b : v);
}
__device__ __forceinline__ double clamp_nan2(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Control step under the bound of eq. 1: minimise 0.5 d'Hd + g'd over
// lo <= d <= hi, H symmetric positive definite (upper triangle used, with its
// Cholesky factor lf/invf given), by a primal active-set method:
//   start from the unconstrained minimiser -H^-1 g; if it is in the box it is
//   the answer (W = 0, the factor is kept).  Otherwise clamp it into the box
//   and hold the clamped components at their bounds (the working set W, bit
//   i; bit i of `up` when at the upper bound), then repeat:
//   * not yet at the minimiser of the current face: solve for the free
//     components with W held, y_F = -H_FF^-1 (g_F + H_FW d_W), and move from
//     d towards y as far as the box allows; a component that reaches a bound
//     first (smallest step, lowest index on ties) joins W, otherwise d = y;
//   * at the face's minimiser: the multiplier of a held component is its
//     gradient g_i + (H d)_i, negated at an upper bound; if one is negative
//     (the most negative, lowest index on ties) it is released, otherwise d
//     is optimal.
// A strictly convex problem ends after finitely many steps; `cap` bounds them
// (the point reached is feasible either way).  The free block's factor goes
// to lf/invf (which hold H's factor on entry) with identity rows for the held
// components, so that
// -lf^-1 [Q_ux] gives the feedback rows of the free components and zero rows
// for the held ones.  Returns false when a free block does not factorise.
template <int M, int NR>
__device__ __forceinline__ bool box_qp(const double (&H)[M][M], const double (&g)[M], const double (&lo)[M],
                                       const double (&hi)[M], double (&d)[M], unsigned& W, double (&lf)[M][M],
                                       double (&invf)[M]) {
  constexpr unsigned ALL = (1u << M) - 1u;
  // on entry d = -H^-1 g (the unconstrained step) and lf/invf hold the factor
  // of H; both stay as they are when d is in the box or not a number (the
  // caller's finiteness check reports the latter)
  bool inside = true, nan = false;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    inside = inside && d[i] >= lo[i] && d[i] <= hi[i];
    nan = nan || !(d[i] == d[i]);
  }
  W = 0;
  if (inside || nan) return true;
  unsigned up = 0;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    if (d[i] < lo[i]) {
      d[i] = lo[i];
      W |= 1u << i;
    } else if (d[i] > hi[i]) {
      d[i] = hi[i];
      W |= 1u << i;
      up |= 1u << i;
    }
  }
  auto h = [&](int i, int j) { return i <= j ? H[i][j] : H[j][i]; };
  auto factor_face = [&]() -> bool {
    double hm[M][M];
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int j = i; j < M; ++j)
        hm[i][j] = ((W >> i) & 1u) || ((W >> j) & 1u) ? (i == j ? 1.0 : 0.0) : H[i][j];
    return chol_fp64<M, NR>(hm, lf, invf);
  };
  constexpr int cap = 4 * M + 4;
  bool at_min = false;
  for (int it = 0; it < cap; ++it) {
    if (!at_min) {
      if (W == ALL) {
        at_min = true;
        continue;
      }
      if (!factor_face()) return false;
      double y[M];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        double v = g[i];
#pragma unroll
        for (int j = 0; j < M; ++j)
          if ((W >> j) & 1u) v += h(i, j) * d[j];
        y[i] = ((W >> i) & 1u) ? 0.0 : -v;
      }
      chol_solve_fp64<M>(lf, invf, y);
      double alpha = 1.0;
      int blk = -1;
      bool bup = false;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        if ((W >> i) & 1u) continue;
        const double p = y[i] - d[i];
        if (p < 0.0) {
          const double t = (lo[i] - d[i]) / p;
          if (t < alpha) {
            alpha = t;
            blk = i;
            bup = false;
          }
        } else if (p > 0.0) {
          const double t = (hi[i] - d[i]) / p;
          if (t < alpha) {
            alpha = t;
            blk = i;
            bup = true;
          }
        }
      }
      if (blk < 0) {
#pragma unroll
        for (int i = 0; i < M; ++i)
          if (!((W >> i) & 1u)) d[i] = y[i];
        at_min = true;
      } else {
#pragma unroll
        for (int i = 0; i < M; ++i) {
          if ((W >> i) & 1u) continue;
          d[i] = i == blk ? (bup ? hi[i] : lo[i]) : clamp_nan2(d[i] + alpha * (y[i] - d[i]), lo[i], hi[i]);
        }
        W |= 1u << blk;
        up = bup ? (up | (1u << blk)) : (up & ~(1u << blk));
      }
    } else {
      int rel = -1;
      double lmin = 0.0;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        if (!((W >> i) & 1u)) continue;
        double gr = g[i];
#pragma unroll
        for (int j = 0; j < M; ++j) gr += h(i, j) * d[j];
        const double lam = ((up >> i) & 1u) ? -gr : gr;
        if (lam < lmin) {
          lmin = lam;
          rel = i;
        }
      }
      if (rel < 0) break;
      W &= ~(1u << rel);
      at_min = false;
    }
  }
  // the factor of the final face
  if (W == 0) return chol_fp64<M, NR>(H, lf, invf);
  if (W == ALL) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
#pragma unroll
      for (int j = 0; j < M; ++j) lf[i][j] = i == j ? 1.0 : 0.0;
      invf[i] = 1.0;
    }
    return true;
  }
  return factor_face();
}

// ------------------------------------------------------------------ iteration-order keys
// index of a positive float value in levels of 2^-(23 - sh) octaves, from its
// exponent and leading mantissa bits; 0 for values <= 0 or NaN (infinity
// takes the top index)
__device__ __forceinline__ uint32_t order_index(float v, int sh) {
  return v > 0.f ? (__float_as_uint(v) >> sh) + 1u : 0u;
}

// a slot's iteration-order key, written by the warm start.  Ragged batch: the
// horizon (clamped into [1, Tmax]) above the octave index of float(J^0).  One
// horizon: the quarter-octave index of float(J^0) above the half-octave index
// of o, the warm start's non-convex cost share.  Both indexes stay below 2^11.
__device__ __forceinline__ uint32_t order_key(bool ragged, int t, double J, float o, int Tmax) {
  if (ragged) {
    t = t < 1 ? 1 : (t > Tmax ? Tmax : t);
    return (uint32_t(t) << 11) | order_index(float(J), 23);
  }
  return (order_index(float(J), 21) << 11) | order_index(o, 22);
}

}  // namespace cbic
