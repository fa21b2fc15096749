// Workgroup-per-instance iLQR for the 37-state synthetic quadruped
// (q in R^19, v in R^18, u in R^12; paper Sec. II eq. 1 and Sec. IV).
//
// One 256-thread workgroup owns one instance.  The backward Riccati sweep
// keeps P, f_x, P f_x, f_u, P f_u, the gains and Q_ux in LDS and forms the
// products as 16 x 16 output tiles on the matrix cores (FP32 MFMA for the
// mixed form, FP64 MFMA for the plain one), the tiles spread over the four
// waves; Q_uu is factored in FP64 (wave 0, rows held by lanes, each pivot
// column broadcast from its lane through a scalar register) in both
// precisions.  The dynamics step needs a Cholesky of the 18 x 18 mass matrix
// M(q) = A^T A + diag(1 + 0.1 sin q); a wave does it with its lanes holding
// the rows.  The dynamics Jacobians do not depend on P, so the sweep
// evaluates them ahead of the recursion, CH steps at a time with every wave
// taking its own steps, into per-slot blocks in HBM that the recursion then
// reads back.  Line-search trials run one per wave: in
// round r wave w tries alpha_j with j = 4 r + w, and the first accepted j is
// taken, as in the sequential rule.  Trajectories and gains use the same
// step-major workspace as the lane schedule.
#include "lane_launch.hpp"

namespace cbic {
namespace quad {

constexpr int NQ = 19, NV = 18, N = 37, M = 12;
constexpr int LD = 40;   // row stride of 37-wide LDS matrices
constexpr int LDB = 13;  // row stride of 12-wide LDS matrices
constexpr int NT = 256;  // threads per workgroup
constexpr int NW = NT / 64;
constexpr int DB = N * (N + M);  // derivative block [f_x | f_u], row-major 37 x 49
constexpr int CH = 16;           // steps per chunk of precomputed derivative blocks

// device block: [dt, w_u, w_T, w_q, w_v, M0 = A^T A (18x18), W1, W2, e(18), x_nom(37)]
constexpr int O_DT = 0, O_WU = 1, O_WT = 2, O_WQ = 3, O_WV = 4, O_M0 = 5, O_W1 = O_M0 + 324,
              O_W2 = O_W1 + 324, O_E = O_W2 + 324, O_XN = O_E + 18, NPRM = O_XN + 37;

template <class R>
struct WaveScratch {
  R L[NV][NV + 1];  // Cholesky factor of M(q), lower, row-major
  R Li[NV];         // reciprocals of its diagonal
  R x[LD];          // state of this wave's rollout
  R xn[LD];         // next state
  R u[16];          // control
  R dx[LD];
  R s[NV], c[NV];   // sin, cos of q[0:18]
  R a[NV];          // acceleration M^-1 (S u - b)
  R w2c[NV];        // W2 cos q
};

template <class R>
struct Smem {
  using real = R;
  R M0[NV][NV + 1];
  R W1[NV][NV + 1];
  R W2[NV][NV + 1];
  R e[NV];
  R xnom[LD];
  R P[N][LD];   // value Hessian; Q_xx; the updated P
  R A[N][LD];   // f_x
  R PA[N][LD];  // P f_x; right-hand sides of the Jacobian solves; scratch
  R Bm[N][LDB]; // f_u
  // P f_u; once Q_uu is formed, the bounded step's copy of Q_uu and the
  // reciprocal pivots of its face factors live here (box_step)
  alignas(8) R PB[N][LDB];
  R Kg[M][LD];  // feedback gain (m x n)
  R Qux[M][LD];
  R p[LD], Qx[LD];
  R Qu[16], kk[16];
  double Quu[M][M + 1];
  double Lq[M][M + 1];
  double Lqi[M];  // reciprocals of the diagonal of Lq
  double wJ[NW];
  int wok[NW];
  int flag;
  unsigned Hq_held;  // components held at a bound by the bounded step
  WaveScratch<R> wv[NW];
};

// Shared memory of the kernels that need only the constants, one vector and
// the scratch of NWV waves (the initial rollout, the finalize): small enough
// for every instance of a CU's share of the batch to be resident at once
template <class R, int NWV>
struct WaveSmem {
  using real = R;
  R M0[NV][NV + 1];
  R W1[NV][NV + 1];
  R W2[NV][NV + 1];
  R e[NV];
  R xnom[LD];
  R p[LD];  // the finalize's costate
  WaveScratch<R> wv[NWV];
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// value of v in lane j (j uniform), read through a scalar register
__device__ __forceinline__ float bcast(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
// 1/sqrt(d) from the hardware estimate and Newton steps y <- y (3 - d y^2) / 2,
// each squaring the relative error: two in FP64, one in FP32 (the pivots of
// the Cholesky factors below are then d * (1/sqrt(d)), without a division)
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * (1.5 - 0.5 * d * y * y);
  return y * (1.5 - 0.5 * d * y * y);
}
__device__ __forceinline__ float rsqrt_nr(float d) {
  const float y = __builtin_amdgcn_rsqf(d);
  return y * (1.5f - 0.5f * d * y * y);
}

__device__ __forceinline__ double bcast(double v, int j) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, j);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), j);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <class R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------ constants
template <class S>
__device__ __forceinline__ void stage_constants(S& sm, const double* __restrict__ prm, int tid, int nt = NT) {
  using R = typename S::real;
  for (int i = tid; i < NV * NV; i += nt) {
    const int r = i / NV, c = i % NV;
    sm.M0[r][c] = R(prm[O_M0 + i]);
    sm.W1[r][c] = R(prm[O_W1 + i]);
    sm.W2[r][c] = R(prm[O_W2 + i]);
  }
  if (tid < NV) sm.e[tid] = R(prm[O_E + tid]);
  if (tid < N) sm.xnom[tid] = R(prm[O_XN + tid]);
}

// ------------------------------------------------------------------ wave-level dynamics
// One semi-implicit Euler step for wave scratch ws: reads ws.x and ws.u,
// writes ws.xn; leaves L (factor of M), a, sin/cos and W2 cos q in ws.
template <class R, class S>
__device__ __forceinline__ void wave_dyn(const S& sm, WaveScratch<R>& ws, R dt, int lane) {
  if (lane < NV) {
    R sn, cs;
    dsincos_lib(ws.x[lane], &sn, &cs);
    ws.s[lane] = sn;
    ws.c[lane] = cs;
  }
  wave_sync();
  const bool row = lane < NV;
  const int ri = row ? lane : 0;
  // M = A^T A + diag(1 + 0.1 sin q); Cholesky with the rows on lanes, the
  // pivot column broadcast from its lane
  R m[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) m[j] = row ? sm.M0[ri][j] : R(0);
#pragma unroll
  for (int j = 0; j < NV; ++j)
    if (j == lane) m[j] += R(1) + R(0.1) * ws.s[ri];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const R piv = bcast(m[j], j);
    const R inv = rsqrt_nr(piv);
    const R ljj = piv * inv;
    if (lane == 0) ws.Li[j] = inv;
    const R lij = (lane == j) ? ljj : (lane > j && row ? m[j] * inv : R(0));
    m[j] = lij;
#pragma unroll
    for (int k = j + 1; k < NV; ++k) {
      const R lkj = bcast(lij, k);
      m[k] -= lij * lkj;
    }
  }
  if (row)
#pragma unroll
    for (int j = 0; j < NV; ++j)
      if (j <= lane) ws.L[ri][j] = m[j];
  // bias forces and right-hand side r = S u - b
  R y = R(0);
  if (row) {
    R b1 = R(0), b2 = R(0);
#pragma unroll 3
    for (int j = 0; j < NV; ++j) {
      b1 += sm.W1[ri][j] * ws.s[j];
      b2 += sm.W2[ri][j] * ws.c[j];
    }
    ws.w2c[ri] = b2;
    const R b = b1 + b2 * ws.x[NQ + ri];
    y = (ri >= 6 ? ws.u[ri - 6] : R(0)) - b;
  }
  wave_sync();
  // L z = r (rows on lanes)
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const R yj = bcast(y, j) * ws.Li[j];
    if (lane == j) y = yj;
    else if (lane > j) y -= m[j] * yj;
  }
  // L^T a = z
#pragma unroll
  for (int j = NV - 1; j >= 0; --j) {
    const R zj = bcast(y, j) * ws.Li[j];
    if (lane == j) y = zj;
    else if (lane < j) y -= ws.L[j][ri] * zj;
  }
  R ev = R(0);
  if (row) {
    ws.a[ri] = y;
    const R vn = ws.x[NQ + ri] + dt * y;
    ws.xn[NQ + ri] = vn;
    ws.xn[ri] = ws.x[ri] + dt * vn;
    ev = sm.e[ri] * vn;
  }
  ev = wave_sum(ev);
  if (lane == 0) ws.xn[NV] = ws.x[NV] + dt * ev;
  wave_sync();
}

// running cost l(x, u) of the wave's (x, u); the same value in every lane
template <class R, class S>
__device__ __forceinline__ R wave_cost(const S& sm, const R* x, const R* u, const double* __restrict__ prm, int lane,
                       bool terminal) {
  R v = R(0);
  if (lane < N) {
    const R d = x[lane] - sm.xnom[lane];
    v = (lane < NQ ? R(prm[O_WQ]) : R(prm[O_WV])) * d * d;
    if (terminal) v *= R(prm[O_WT]);
  } else if (!terminal && lane < N + M) {
    const R uu = u[lane - N];
    v = R(prm[O_WU]) * uu * uu;
  }
  return wave_sum(v);
}

// ------------------------------------------------------------------ MFMA tiles
// One 16 x 16 output tile of C = Cin + op(A) op(B) (inner size Kd) by one wave
// with 16x16x4 matrix-core instructions: FP32 for the mixed form, FP64 for the
// plain one.  Lane l supplies A(i0 + l % 16, k0 + l / 16) and
// B(k0 + l / 16, j0 + l % 16) per step of 4; its result register r holds
// C(i0 + 4 (l / 16) + r, j0 + l % 16) in FP32 and C(i0 + l / 16 + 4 r,
// j0 + l % 16) in FP64.  Entries outside Mr x Nc x Kd enter as zeros and are
// not stored.
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef double mf_d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ mf_f4 mfma16(float a, float b, mf_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mf_d4 mfma16(double a, double b, mf_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <class R> struct MfAcc;
template <> struct MfAcc<float> {
  using type = mf_f4;
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};
template <> struct MfAcc<double> {
  using type = mf_d4;
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};

template <int Kd, bool TA, bool TB, class R>
__device__ __forceinline__ void mfma_tile(R* C, int ldc, const R* A, int lda, const R* Bp, int ldb, const R* Cin,
                                          int ldcin, int Mr, int Nc, int i0, int j0, int lane) {
  using V = typename MfAcc<R>::type;
  const int li = lane & 15, lk = lane >> 4;
  V acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + MfAcc<R>::row(lk, r), j = j0 + li;
    acc[r] = (Cin && i < Mr && j < Nc) ? Cin[i * ldcin + j] : R(0);
  }
  const int ia = i0 + li, jb = j0 + li;
#pragma unroll
  for (int k0 = 0; k0 < Kd; k0 += 4) {
    const int k = k0 + lk;
    const R a = (ia < Mr && k < Kd) ? (TA ? A[k * lda + ia] : A[ia * lda + k]) : R(0);
    const R b = (k < Kd && jb < Nc) ? (TB ? Bp[jb * ldb + k] : Bp[k * ldb + jb]) : R(0);
    acc = mfma16(a, b, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + MfAcc<R>::row(lk, r), j = j0 + li;
    if (i < Mr && j < Nc) C[i * ldc + j] = acc[r];
  }
}

// The same tile product handing each result to out(i, j, value) instead of
// storing it (no input accumulator).
template <int Kd, bool TA, bool TB, class R, class Out>
__device__ __forceinline__ void mfma_tile_out(Out&& out, const R* A, int lda, const R* Bp, int ldb, int Mr, int Nc,
                                              int i0, int j0, int lane) {
  using V = typename MfAcc<R>::type;
  const int li = lane & 15, lk = lane >> 4;
  V acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = R(0);
  const int ia = i0 + li, jb = j0 + li;
#pragma unroll
  for (int k0 = 0; k0 < Kd; k0 += 4) {
    const int k = k0 + lk;
    const R a = (ia < Mr && k < Kd) ? (TA ? A[k * lda + ia] : A[ia * lda + k]) : R(0);
    const R b = (k < Kd && jb < Nc) ? (TB ? Bp[jb * ldb + k] : Bp[k * ldb + jb]) : R(0);
    acc = mfma16(a, b, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + MfAcc<R>::row(lk, r), j = j0 + li;
    if (i < Mr && j < Nc) out(i, j, acc[r]);
  }
}

// ------------------------------------------------------------------ wave Jacobians
// [f_x | f_u] at (ws.x, ws.u) by one wave, after wave_dyn on that point (L, its
// reciprocal diagonal, a, sin/cos and W2 cos q in ws), written row-major
// (37 x 49) to dst.  Lane c < 48 owns column c of the right-hand sides
// (0..17 -dD/dq with a and v held, 18..35 -dD/dv, 36..47 the actuation S),
// solves it with M = L L^T in registers and writes the output column that
// depends on it: c for c < 18, c + 1 otherwise.  Lane 48 writes column 18
// (q_18 does not enter the dynamics; only the identity).
template <class R>
__device__ __forceinline__ void wave_jac(const Smem<R>& sm, const WaveScratch<R>& ws, R dt, int lane,
                                         R* __restrict__ dst) {
  if (lane < 48) {
    const int c = lane;
    R y[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      R v;
      if (c < NV) {
        v = -(sm.W1[i][c] * ws.c[c] - ws.x[NQ + i] * sm.W2[i][c] * ws.s[c]);
        if (i == c) v -= R(0.1) * ws.c[i] * ws.a[i];
      } else if (c < 2 * NV) {
        v = (c - NV == i) ? -ws.w2c[i] : R(0);
      } else {
        v = (c - 2 * NV + 6 == i) ? R(1) : R(0);
      }
      y[i] = v;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      R v0 = y[i], v1 = R(0);
#pragma unroll
      for (int k = 0; k < i; ++k) {
        if (k & 1) v1 += ws.L[i][k] * y[k];
        else v0 -= ws.L[i][k] * y[k];
      }
      y[i] = (v0 - v1) * ws.Li[i];
    }
#pragma unroll
    for (int i = NV - 1; i >= 0; --i) {
      R v0 = y[i], v1 = R(0);
#pragma unroll
      for (int k = i + 1; k < NV; ++k) {
        if (k & 1) v1 += ws.L[k][i] * y[k];
        else v0 -= ws.L[k][i] * y[k];
      }
      y[i] = (v0 - v1) * ws.Li[i];
    }
    // d v+_i / d (x, u)_col = [col is the velocity column i] + dt y_i; rows:
    // v+ (19..36), q+ = q + dt v+ (0..17), q_18+ = q_18 + dt e . v+
    const int col = c < NV ? c : c + 1;
    R se = R(0);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const R d = ((c >= NV && c < 2 * NV && c - NV == i) ? R(1) : R(0)) + dt * y[i];
      se += sm.e[i] * d;
      dst[(NQ + i) * (N + M) + col] = d;
      dst[i * (N + M) + col] = ((col == i) ? R(1) : R(0)) + dt * d;
    }
    dst[NV * (N + M) + col] = dt * se;
  } else if (lane == 48) {
#pragma unroll
    for (int r = 0; r < N; ++r) dst[r * (N + M) + NV] = (r == NV) ? R(1) : R(0);
  }
}

// ------------------------------------------------------------------ FP64 Cholesky of Q_uu and the gains
// Wave 0 factors Quu (rows on lanes); threads 0..37 solve for [K k].  The
// other waves run `side` meanwhile (work that needs none of the step's gains).
template <class R, class Side>
__device__ __forceinline__ bool gains(Smem<R>& sm, int tid, Side&& side) {
  if (tid >= 64) side();
  if (tid < 64) {
    const int lane = tid;
    const bool row = lane < M;
    const int ri = row ? lane : 0;
    double m[M];
#pragma unroll
    for (int j = 0; j < M; ++j) m[j] = row ? sm.Quu[min(ri, j)][max(ri, j)] : 0.0;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const double piv = bcast(m[j], j);
      ok = ok && (piv > 0.0) && isfinite(piv);
      const double inv = rsqrt_nr(piv);
      const double ljj = piv * inv;
      if (lane == 0) sm.Lqi[j] = inv;
      const double lij = (lane == j) ? ljj : (lane > j && row ? m[j] * inv : 0.0);
      m[j] = lij;
#pragma unroll
      for (int k = j + 1; k < M; ++k) m[k] -= lij * bcast(lij, k);
    }
    if (row)
#pragma unroll
      for (int j = 0; j < M; ++j) sm.Lq[ri][j] = m[j];
    if constexpr (sizeof(R) == 4) {
      // mixed form: the factor rounded to FP32 for the gain solves, in the
      // storage of Q_uu (read above, not needed again)
      float* lf = reinterpret_cast<float*>(&sm.Quu[0][0]);
      if (row)
#pragma unroll
        for (int j = 0; j < M; ++j) lf[ri * (M + 1) + j] = float(m[j]);
      wave_sync();  // the reciprocal pivots were stored by lane 0
      if (lane < M) lf[M * (M + 1) + lane] = float(sm.Lqi[lane]);
    }
    if (lane == 0) sm.flag = ok ? 0 : 1;
  }
  __syncthreads();
  if (sm.flag) return false;
  if constexpr (sizeof(R) == 4) {
    // mixed form: the gains are stored in FP32, so their triangular solves run
    // in FP32 on the FP64 factor rounded to FP32 (as in the lane kernels)
    if (tid <= N) {
      const float* lf = reinterpret_cast<const float*>(&sm.Quu[0][0]);
      const float* lfi = lf + M * (M + 1);
      float y[M];
#pragma unroll
      for (int i = 0; i < M; ++i) y[i] = tid < N ? sm.Qux[i][tid] : sm.Qu[i];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        float v0 = y[i], v1 = 0.0f;
#pragma unroll
        for (int k = 0; k < i; ++k) {
          if (k & 1) v1 += lf[i * (M + 1) + k] * y[k];
          else v0 -= lf[i * (M + 1) + k] * y[k];
        }
        y[i] = (v0 - v1) * lfi[i];
      }
#pragma unroll
      for (int i = M - 1; i >= 0; --i) {
        float v0 = y[i], v1 = 0.0f;
#pragma unroll
        for (int k = i + 1; k < M; ++k) {
          if (k & 1) v1 += lf[k * (M + 1) + i] * y[k];
          else v0 -= lf[k * (M + 1) + i] * y[k];
        }
        y[i] = (v0 - v1) * lfi[i];
      }
      bool fin = true;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        fin = fin && isfinite(y[i]);
        if (tid < N) sm.Kg[i][tid] = R(-y[i]);
        else sm.kk[i] = R(-y[i]);
      }
      if (!fin) sm.flag = 2;
    }
    __syncthreads();
    return sm.flag == 0;
  }
  if (tid <= N) {  // column tid of [Q_ux | Q_u]; the column lives in registers
    double y[M];
#pragma unroll
    for (int i = 0; i < M; ++i) y[i] = double(tid < N ? sm.Qux[i][tid] : sm.Qu[i]);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      double v0 = y[i], v1 = 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) {
        if (k & 1) v1 += sm.Lq[i][k] * y[k];
        else v0 -= sm.Lq[i][k] * y[k];
      }
      y[i] = (v0 - v1) * sm.Lqi[i];
    }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
      double v0 = y[i], v1 = 0.0;
#pragma unroll
      for (int k = i + 1; k < M; ++k) {
        if (k & 1) v1 += sm.Lq[k][i] * y[k];
        else v0 -= sm.Lq[k][i] * y[k];
      }
      y[i] = (v0 - v1) * sm.Lqi[i];
    }
    bool fin = true;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      fin = fin && isfinite(y[i]);
      if (tid < N) sm.Kg[i][tid] = R(-y[i]);
      else sm.kk[i] = R(-y[i]);
    }
    if (!fin) sm.flag = 2;
  }
  __syncthreads();
  return sm.flag == 0;
}

// ------------------------------------------------------------------ bounded control step (eq. 1)
// FP64 storage of the bounded step inside PB (free once Q_uu is formed):
// H = Q_uu [M][M + 1], then the reciprocal pivots of a face factor [M].
template <class R>
__device__ __forceinline__ double* box_H(Smem<R>& sm) {
  return reinterpret_cast<double*>(&sm.PB[0][0]);
}
static_assert(sizeof(double) * (M * (M + 1) + M) <= sizeof(float) * N * LDB, "box step storage fits PB");

// Wave-parallel Cholesky (rows on lanes, the pivot column broadcast from its
// lane) of the face of H with the components in W held: their rows and
// columns become identity.  Lane i < M keeps row i of the factor in f and
// stores it to Lf[i]; the reciprocal pivots go to Li (lane 0 writes).  False
// when a pivot is not positive or not finite.
__device__ __forceinline__ bool face_factor(const double* H, unsigned W, int lane, double (&f)[M],
                                            double (*Lf)[M + 1], double* Li) {
  const bool row = lane < M;
  const int ri = row ? lane : 0;
  const bool hr = (W >> ri) & 1u;
#pragma unroll
  for (int j = 0; j < M; ++j)
    f[j] = !row ? 0.0 : (hr || ((W >> j) & 1u)) ? (ri == j ? 1.0 : 0.0) : H[min(ri, j) * (M + 1) + max(ri, j)];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const double piv = bcast(f[j], j);
    ok = ok && (piv > 0.0) && isfinite(piv);
    const double inv = rsqrt_nr(piv);
    if (lane == 0) Li[j] = inv;
    const double lij = (lane == j) ? piv * inv : (lane > j && row ? f[j] * inv : 0.0);
    f[j] = lij;
#pragma unroll
    for (int k = j + 1; k < M; ++k) f[k] -= lij * bcast(lij, k);
  }
  if (row)
#pragma unroll
    for (int j = 0; j < M; ++j) Lf[ri][j] = f[j];
  wave_sync();
  return ok;
}

// (L L^T) y = b for the factor (rows on lanes in f, all rows in Lf) and its
// reciprocal pivots Li; lane i < M holds b_i on entry and y_i on return.
__device__ __forceinline__ double face_solve(const double (&f)[M], const double (*Lf)[M + 1], const double* Li,
                                             double y, int lane) {
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const double yj = bcast(y, j) * Li[j];
    if (lane == j) y = yj;
    else if (lane > j && lane < M) y -= f[j] * yj;
  }
  const int ri = lane < M ? lane : 0;
#pragma unroll
  for (int j = M - 1; j >= 0; --j) {
    const double zj = bcast(y, j) * Li[j];
    if (lane == j) y = zj;
    else if (lane < j) y -= Lf[j][ri] * zj;
  }
  return y;
}

// The control step under the bound (paper eq. 1) once gains() has formed the
// unconstrained gains: when the step k_k lies in the box [-umax - u_k,
// umax - u_k] it stands (so a bound that never binds changes nothing).
// Otherwise wave 0 minimises 0.5 d'Hd + Q_u'd over the box exactly in FP64 by
// the primal active-set method of the lane kernels (box_qp in dev_common.hpp):
// start from the clamped unconstrained minimiser, holding the clamped
// components; move towards the current face's minimiser until a free
// component meets a bound (smallest step, lowest index on ties), or at the
// face's minimiser release the held component with the most negative
// multiplier (lowest index on ties); at most 4 M + 4 steps.  The feedback rows
// of the held components are zero and the free ones come from the final
// face's factor: K = -[face factor]^-1 Q_ux with the held rows of Q_ux zeroed.
// Returns 0 or the status bit that freezes the instance.
template <class R>
__device__ uint32_t box_step(Smem<R>& sm, const WaveScratch<R>& w0, double umax, int tid) {
  double* H = box_H(sm);
  double* Li = H + M * (M + 1);
  if (tid < 64) {
    const int lane = tid;
    const bool row = lane < M;
    const int ri = row ? lane : 0;
    const double u = double(w0.u[ri]);
    const double lo = -umax - u, hi = umax - u;
    const double kk = double(sm.kk[ri]);
    const bool inside = !row || (kk >= lo && kk <= hi);
    unsigned W = 0, up = 0;
    bool ok = true;
    if (__ballot(!inside)) {
      constexpr unsigned ALL = (1u << M) - 1u;
      const double g = double(sm.Qu[ri]);
      // the unconstrained minimiser -H^-1 g in FP64 from the factor of H
      double f[M];
      ok = face_factor(H, 0u, lane, f, sm.Lq, Li);
      double d = face_solve(f, sm.Lq, Li, row ? -g : 0.0, lane);
      const bool dl = row && d < lo, dh = row && d > hi;
      d = dl ? lo : (dh ? hi : d);
      W = unsigned(__ballot(dl || dh)) & ALL;
      up = unsigned(__ballot(dh)) & ALL;
      bool at_min = false;
      for (int it = 0; it < 4 * M + 4 && ok; ++it) {
        if (!at_min) {
          if (W == ALL) {
            at_min = true;
            continue;
          }
          ok = face_factor(H, W, lane, f, sm.Lq, Li);
          if (!ok) break;
          const bool held = (W >> ri) & 1u;
          double v = g;
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const double dj = bcast(d, j);
            if ((W >> j) & 1u) v += H[min(ri, j) * (M + 1) + max(ri, j)] * dj;
          }
          const double y = face_solve(f, sm.Lq, Li, (row && !held) ? -v : 0.0, lane);
          // ratio test over the free components
          const double pdir = y - d;
          double t = __builtin_inf();
          if (row && !held) {
            if (pdir < 0.0) t = (lo - d) / pdir;
            else if (pdir > 0.0) t = (hi - d) / pdir;
          }
          double alpha = 1.0;
          int blk = -1;
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const double tj = bcast(t, j);
            if (tj < alpha) {
              alpha = tj;
              blk = j;
            }
          }
          if (blk < 0) {
            if (row && !held) d = y;
            at_min = true;
          } else {
            const bool bup = bcast(pdir, blk) > 0.0;
            if (row && !held)
              d = lane == blk ? (bup ? hi : lo) : clamp_nan2(d + alpha * (y - d), lo, hi);
            W |= 1u << blk;
            up = bup ? (up | (1u << blk)) : (up & ~(1u << blk));
          }
        } else {
          double gr = g;
#pragma unroll
          for (int j = 0; j < M; ++j) gr += H[min(ri, j) * (M + 1) + max(ri, j)] * bcast(d, j);
          const double lam = ((up >> ri) & 1u) ? -gr : gr;
          double lmin = 0.0;
          int rel = -1;
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const double lj = bcast(lam, j);
            if (((W >> j) & 1u) && lj < lmin) {
              lmin = lj;
              rel = j;
            }
          }
          if (rel < 0) break;
          W &= ~(1u << rel);
          at_min = false;
        }
      }
      // the final face's factor (to Lq, Lqi) and the step
      if (ok) ok = face_factor(H, W, lane, f, sm.Lq, Li);
      if (row) sm.kk[ri] = R(d);
      if (lane < M) sm.Lqi[lane] = Li[lane];
      if (lane == 0) sm.flag = ok ? 3 : 1;  // 3: the feedback rows are recomputed below
    } else if (lane == 0) {
      sm.flag = 0;
    }
    if (lane == 0) sm.Hq_held = W;
  }
  __syncthreads();
  if (sm.flag == 1) return ST_CHOL_FAIL;
  if (sm.flag == 0) return 0u;
  // feedback rows from the face factor (FP64), the held rows zero
  if (tid < N) {
    const unsigned W = sm.Hq_held;
    double y[M];
#pragma unroll
    for (int i = 0; i < M; ++i) y[i] = ((W >> i) & 1u) ? 0.0 : double(sm.Qux[i][tid]);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      double v = y[i];
#pragma unroll
      for (int k = 0; k < i; ++k) v -= sm.Lq[i][k] * y[k];
      y[i] = v * sm.Lqi[i];
    }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
      double v = y[i];
#pragma unroll
      for (int k = i + 1; k < M; ++k) v -= sm.Lq[k][i] * y[k];
      y[i] = v * sm.Lqi[i];
    }
    bool fin = true;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      sm.Kg[i][tid] = R(-y[i]);
      fin = fin && isfinite(sm.Kg[i][tid]);
    }
    if (tid < M) fin = fin && isfinite(sm.kk[tid]);
    if (!fin) sm.flag = 2;
  }
  __syncthreads();
  return sm.flag == 2 ? ST_NONFINITE : 0u;
}

template <class R>
struct QW {  // workspace accessors (the lane schedule's slot-major layout)
  static __device__ __forceinline__ R* xp(const LaneState<R>& w, int buf, int k, int s) {
    return w.X + (size_t(buf) * w.Bcap + s) * w.xs + k * N;
  }
  static __device__ __forceinline__ R* up(const LaneState<R>& w, int buf, int k, int s) {
    return w.U + (size_t(buf) * w.Bcap + s) * w.us + k * M;
  }
  static __device__ __forceinline__ R* Kp(const LaneState<R>& w, int k, int s) {
    return w.K + size_t(s) * w.Ks + k * (M * N);
  }
  static __device__ __forceinline__ R* kp(const LaneState<R>& w, int k, int s) {
    return w.kf + size_t(s) * w.ks + k * M;
  }
};

// ------------------------------------------------------------------ backward sweep
// BOX: the bounded control step of eq. 1 (umax); mu: the Levenberg-Marquardt
// shift of Q_uu (zero for the clipped form)
template <class R, bool BOX>
__device__ __forceinline__ uint32_t backward(Smem<R>& sm, const double* __restrict__ prm, const LaneState<R>& w, int s, int T,
                             int buf, R eps, int tid, R* __restrict__ blk, double mu, double umax) {
  using Q = QW<R>;
  const R dt = R(prm[O_DT]);
  const R wq = R(prm[O_WQ]), wv = R(prm[O_WV]), wu = R(prm[O_WU]), wT = R(prm[O_WT]);
  // terminal: P = clip(l_T,xx) (diagonal), p = l_T,x
  for (int i = tid; i < N * LD; i += NT) (&sm.P[0][0])[i] = R(0);
  __syncthreads();
  if (tid < N) {
    const R xv = Q::xp(w, buf, T, s)[tid];
    const R wi = (tid < NQ ? wq : wv) * wT;
    sm.p[tid] = R(2) * wi * (xv - sm.xnom[tid]);
    sm.P[tid][tid] = dmax(R(2) * wi, eps);
  }
  __syncthreads();
  const int wid = tid >> 6, lane = tid & 63;
  // Step kk's (x, u) go to the scratch of wave 2 + (kk & 1) (free between the
  // derivative pre-passes) and its derivative block to A, Bm, by the threads
  // from `first` on.  The first step of a chunk is staged by all threads after
  // the pre-pass; every other step by waves 1..3 while wave 0 factors the
  // previous step's Q_uu (A and Bm are not read again in a step once Q_uu is
  // formed).
  auto stage = [&](int kk, int first) {
    const int t = tid - first, nt = NT - first;
    if (t < 0) return;
    WaveScratch<R>& sx = sm.wv[2 + (kk & 1)];
    if (t < N) sx.x[t] = Q::xp(w, buf, kk, s)[t];
    if (t < M) sx.u[t] = Q::up(w, buf, kk, s)[t];
    const R* src = blk + ((T - 1 - kk) % CH) * DB;
    for (int i = t; i < DB; i += nt) {
      const int r = i / (N + M), c = i - r * (N + M);
      const R v = src[i];
      if (c < N) sm.A[r][c] = v;
      else sm.Bm[r][c - N] = v;
    }
  };
  for (int k = T - 1; k >= 0; --k) {
    const int q = (T - 1 - k) % CH;
    WaveScratch<R>& sx = sm.wv[2 + (k & 1)];
    if (q == 0) {
      // derivative blocks of the next CH steps, wave wid taking every fourth
      // step (they do not depend on P)
      WaveScratch<R>& wsw = sm.wv[wid];
      for (int qq = wid; qq < CH && k - qq >= 0; qq += NW) {
        if (lane < N) wsw.x[lane] = Q::xp(w, buf, k - qq, s)[lane];
        if (lane < M) wsw.u[lane] = Q::up(w, buf, k - qq, s)[lane];
        wave_sync();
        wave_dyn(sm, wsw, dt, lane);
        wave_jac(sm, wsw, dt, lane, blk + qq * DB);
        wave_sync();
      }
      __syncthreads();
      stage(k, 0);
      __syncthreads();
    }
    // PA = P A, PB = P B: nine 16 x 16 tiles of P A and three of P B; in the
    // same phase Q_x = l_x + A^T p and Q_u = l_u + B^T p (p is replaced only
    // after the gains) as four one-column tiles, the cost gradients (diagonal
    // Hessians) added to their results: sixteen tiles, four per wave
    for (int t = tid >> 6; t < 16; t += NW) {
      if (t < 9)
        mfma_tile<N, false, false>(&sm.PA[0][0], LD, &sm.P[0][0], LD, &sm.A[0][0], LD, (const R*)nullptr, 0, N, N,
                                   (t / 3) * 16, (t % 3) * 16, tid & 63);
      else if (t < 12)
        mfma_tile<N, false, false>(&sm.PB[0][0], LDB, &sm.P[0][0], LD, &sm.Bm[0][0], LDB, (const R*)nullptr, 0, N, M,
                                   (t - 9) * 16, 0, tid & 63);
      else if (t < 15)
        mfma_tile_out<N, true, false>(
            [&](int i, int, R v) { sm.Qx[i] = R(2) * (i < NQ ? wq : wv) * (sx.x[i] - sm.xnom[i]) + v; },
            &sm.A[0][0], LD, &sm.p[0], 1, N, 1, (t - 12) * 16, 0, tid & 63);
      else
        mfma_tile_out<N, true, false>([&](int i, int, R v) { sm.Qu[i] = R(2) * wu * sx.u[i] + v; }, &sm.Bm[0][0],
                                      LDB, &sm.p[0], 1, M, 1, 0, 0, tid & 63);
    }
    __syncthreads();
    // Q_xx = clip(l_xx) + A^T (P A) into P, Q_ux = B^T (P A): twelve tiles; Q_uu =
    // clip(l_uu) + B^T (P B) (+ mu I, the Levenberg-Marquardt shift, zero
    // otherwise: adding it changes no bit) in FP64 from a thirteenth
    for (int t = tid >> 6; t < 13; t += NW) {
      if (t < 9)
        mfma_tile<N, true, false>(&sm.P[0][0], LD, &sm.A[0][0], LD, &sm.PA[0][0], LD, (const R*)nullptr, 0, N, N,
                                  (t / 3) * 16, (t % 3) * 16, tid & 63);
      else if (t < 12)
        mfma_tile<N, true, false>(&sm.Qux[0][0], LD, &sm.Bm[0][0], LDB, &sm.PA[0][0], LD, (const R*)nullptr, 0, M, N,
                                  0, (t - 9) * 16, tid & 63);
      else
        mfma_tile_out<N, true, false>(
            [&](int i, int j, R v) {
              double q = double(v) + (i == j ? double(dmax(R(2) * wu, eps)) : 0.0);
              if (i == j) q += mu;
              sm.Quu[i][j] = q;
            },
            &sm.Bm[0][0], LDB, &sm.PB[0][0], LDB, M, M, 0, 0, tid & 63);
    }
    __syncthreads();
    if (tid < N) sm.P[tid][tid] += dmax(R(2) * (tid < NQ ? wq : wv), eps);
    if constexpr (BOX) {
      // Q_uu for the bounded step (gains() reuses its storage in the mixed form)
      if (tid < M * M) box_H(sm)[(tid / M) * (M + 1) + tid % M] = sm.Quu[tid / M][tid % M];
      __syncthreads();
    }
    if (!gains(sm, tid, [&] {
          if (k >= 1 && q + 1 < CH) stage(k - 1, 64);
        }))
      return sm.flag == 1 ? ST_CHOL_FAIL : ST_NONFINITE;
    if constexpr (BOX) {
      const uint32_t b = box_step(sm, sx, umax, tid);
      if (b) return b;
    }
    // store the gains
    {
      R* dK = Q::Kp(w, k, s);
      for (int i = tid; i < M * N; i += NT) dK[i] = sm.Kg[i / N][i % N];
      if (tid < M) Q::kp(w, k, s)[tid] = sm.kk[tid];
    }
    // C = Q_xx + Q_ux^T K into PA, p = Q_x + Q_ux^T k
    for (int t = tid >> 6; t < 9; t += NW)
      mfma_tile<M, true, false>(&sm.PA[0][0], LD, &sm.Qux[0][0], LD, &sm.Kg[0][0], LD, &sm.P[0][0], LD, N, N,
                                (t / 3) * 16, (t % 3) * 16, tid & 63);
    if (tid < N) {
      R v = sm.Qx[tid];
      for (int t = 0; t < M; ++t) v += sm.Qux[t][tid] * sm.kk[t];
      sm.p[tid] = v;
    }
    __syncthreads();
    // P = sym(C)
    for (int idx = tid; idx < N * N; idx += NT) {
      const int i = idx / N, j = idx % N;
      sm.P[i][j] = R(0.5) * (sm.PA[i][j] + sm.PA[j][i]);
    }
    __syncthreads();
  }
  return 0;
}

// ------------------------------------------------------------------ line-search trial (one wave)
// Closed-loop rollout of wave `wid` with step alpha; writes the trajectory
// when `write`; early stop once the partial cost reaches Jcur (costs >= 0).
// With BOX the trial's controls are clamped into [-umax, umax] (eq. 1).
template <class R, bool BOX>
__device__ __forceinline__ double wave_trial(Smem<R>& sm, const double* __restrict__ prm, const LaneState<R>& w, int s, int T,
                             int buf, R alpha, double Jcur, bool write, int lane, int wid, int& steps, R umax) {
  using Q = QW<R>;
  WaveScratch<R>& ws = sm.wv[wid];
  const R dt = R(prm[O_DT]);
  const int nb = buf ^ 1;
  if (lane < N) ws.x[lane] = Q::xp(w, buf, 0, s)[lane];
  wave_sync();
  double Jh = 0.0;
  steps = T;
  // the iterate's step data (x_k; lane (c, part): entries part, part + 4, ...
  // of row c of K_k; u_k and k_k for c) are loaded one step ahead of their use
  constexpr int KQ = (N + 3) / 4;
  const int c = lane >> 2, part = lane & 3;
  R xq = R(0), uq = R(0), kq = R(0), Kq[KQ];
  auto load = [&](int k) {
    if (lane < N) xq = Q::xp(w, buf, k, s)[lane];
    if (c < M) {
      const R* Kr = Q::Kp(w, k, s) + c * N;
#pragma unroll
      for (int q = 0; q < KQ; ++q) Kq[q] = part + 4 * q < N ? Kr[part + 4 * q] : R(0);
      if (part == 0) {
        uq = Q::up(w, buf, k, s)[c];
        kq = Q::kp(w, k, s)[c];
      }
    }
  };
  load(0);
  for (int k = 0; k < T; ++k) {
    const R xk = xq, uk = uq, kk = kq;
    R Kc[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) Kc[q] = Kq[q];
    if (k + 1 < T) load(k + 1);
    if (lane < N) ws.dx[lane] = ws.x[lane] - xk;
    wave_sync();
    {
      R acc = R(0);
      if (c < M) {
#pragma unroll
        for (int q = 0; q < KQ; ++q)
          if (part + 4 * q < N) acc += Kc[q] * ws.dx[part + 4 * q];
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      if (c < M && part == 0) {
        const R v = uk + alpha * kk + acc;
        ws.u[c] = BOX ? clamp_nan(v, umax) : v;
      }
    }
    wave_sync();
    Jh += double(wave_cost(sm, ws.x, ws.u, prm, lane, false));
    wave_dyn(sm, ws, dt, lane);
    if (write) {
      if (lane < M) Q::up(w, nb, k, s)[lane] = ws.u[lane];
      if (lane < N) Q::xp(w, nb, k + 1, s)[lane] = ws.xn[lane];
    }
    if (lane < N) ws.x[lane] = ws.xn[lane];
    wave_sync();
    if (!(Jh < Jcur)) {
      steps = k + 1;
      return Jh;
    }
  }
  Jh += double(wave_cost(sm, ws.x, ws.u, prm, lane, true));
  return Jh;
}

// ------------------------------------------------------------------ kernels
// Initial rollout: one wave per instance, a serial chain of T dynamics steps
template <class R>
__global__ void __launch_bounds__(64) quad_init(const double* __restrict__ prm, LaneState<R> w, int nthreads,
                                                 const int32_t* __restrict__ slots, int Tmax,
                                                 const int32_t* __restrict__ Tin, const int32_t* __restrict__ perm,
                                                 const double* __restrict__ x0, const double* __restrict__ U0,
                                                 int max_iter, double* __restrict__ trace, double umax) {
  using Q = QW<R>;
  __shared__ WaveSmem<R, 1> sm;
  const int g = blockIdx.x, tid = threadIdx.x;
  if (g >= nthreads) return;
  const int s = slots ? slots[g] : g;
  const int b = perm ? perm[g] : g;
  const int Tr = Tin ? Tin[b] : Tmax;
  const bool badT = Tr < 1 || Tr > Tmax || Tr > w.Tcap;
  const int T = badT ? 0 : Tr;
  stage_constants(sm, prm, tid, 64);
  __syncthreads();
  const int lane = tid;
  WaveScratch<R>& ws = sm.wv[0];
  const R dt = R(prm[O_DT]);
  if (lane < N) {
    const R v = R(x0[size_t(b) * N + lane]);
    ws.x[lane] = v;
    Q::xp(w, 0, 0, s)[lane] = v;
    Q::xp(w, 1, 0, s)[lane] = v;
  }
  wave_sync();
  double J = 0.0;
  for (int k = 0; k < T; ++k) {
    if (lane < M) {
      // the warm start is clamped into the box of eq. 1 (umax infinite: none)
      const R v = clamp_nan(U0 ? R(U0[(size_t(b) * Tmax + k) * M + lane]) : R(0), R(umax));
      ws.u[lane] = v;
      Q::up(w, 0, k, s)[lane] = v;
    }
    wave_sync();
    J += double(wave_cost(sm, ws.x, ws.u, prm, lane, false));
    wave_dyn(sm, ws, dt, lane);
    if (lane < N) {
      ws.x[lane] = ws.xn[lane];
      Q::xp(w, 0, k + 1, s)[lane] = ws.xn[lane];
    }
    wave_sync();
  }
  J += double(wave_cost(sm, ws.x, ws.u, prm, lane, true));
  if (lane == 0) {
    uint32_t st = isfinite(J) ? 0u : ST_NONFINITE;
    if (st == 0 && max_iter <= 0) st = ST_MAX_ITER;
    if (badT) {
      st = ST_BAD_INPUT;
      J = __builtin_nan("");
    }
    w.T[s] = T;
    w.inst[s] = slots ? s : b;
    w.J[s] = J;
    w.okey[s] = order_key(Tin != nullptr, T, J, 0.f, Tmax);  // no non-convex share: J^0 alone
    w.iters[s] = 0;
    w.status[s] = st;
    w.cur[s] = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) w.work[4 * s + i] = 0;
    if (trace) trace[size_t(slots ? s : b) * (max_iter + 1)] = J;
  }
}

template <class R, bool BOX, bool LM, int OCC>
// OCC: workgroups resident per CU the registers are sized for.  With 1 the
// kernel keeps its values in registers (one wave per SIMD); with 2 the
// registers are capped at 256 and some values spill, but the per-step chain is
// latency-bound and a second resident instance per CU hides more of it than
// the spills cost once the batch fills every CU (mixed, 1024 instances: -35 %;
// at most one instance per CU: +10 %; FP64 is slower with 2 at every size).
// BOX: the variant with the control bound of eq. 1 (sp.umax finite).  LM: the
// Levenberg-Marquardt variant (sp.reg = 1), in which a failed Cholesky or line search
// multiplies mu by mu_fac and retries the sweep while mu stays within mu_max;
// an accepted step divides it (not below mu0); mu carries over between launches.
__global__ void __launch_bounds__(NT, OCC) quad_iterate(const double* __restrict__ prm, LaneState<R> w, int nslots,
                                                    const int32_t* __restrict__ slots, SolveParams sp,
                                                    int iters_this_launch, IterTrace tr,
                                                    R* __restrict__ dblk) {
  __shared__ Smem<R> sm;
  const int g = blockIdx.x, tid = threadIdx.x;
  if (g >= nslots) return;
  const int s = slots ? slots[g] : g;
  uint32_t st = w.status[s];
  if (st) return;  // uniform over the workgroup
  const int lane = tid & 63, wid = tid >> 6;
  stage_constants(sm, prm, tid);
  __syncthreads();
  const int T = w.T[s];
  const int b = w.inst[s];
  double J = w.J[s];
  int iters = w.iters[s];
  int buf = w.cur[s];
  int nsweep = w.work[4 * s], npass = w.work[4 * s + 1], nread = w.work[4 * s + 2], nwrite = w.work[4 * s + 3];
  const R eps = R(sp.eps);
  constexpr bool lm = LM;
  double mu = lm ? (nsweep == 0 ? sp.mu0 : w.mu[s]) : 0.0;
  for (int it = 0; it < iters_this_launch && st == 0; ++it) {
    if (iters >= sp.max_iter) {
      st = ST_MAX_ITER;
      break;
    }
    int acc = -1;
    double Jn = J;
    uint32_t fail = 0;
    for (;;) {
      ++nsweep;
      const uint32_t bad = backward<R, BOX>(sm, prm, w, s, T, buf, eps, tid, dblk + size_t(s) * CH * DB, mu, sp.umax);
      if (bad) {
        if (lm && bad == ST_CHOL_FAIL && mu * sp.mu_fac <= sp.mu_max) {
          mu *= sp.mu_fac;
          continue;
        }
        fail = bad;
        break;
      }
      // line search: rounds of NW parallel trials, then (if the accepted step
      // is not alpha = 1, which wave 0 wrote while trying it) one commit
      // rollout; a single call site keeps the kernel's register footprint down
      acc = -1;
      Jn = J;
      bool commit = false;
      for (int j0 = 0;;) {
        const int j = commit ? acc : j0 + wid;
        const bool run = commit ? (wid == 0) : (j < sp.ls_trials);
        double Jh = __builtin_nan("");
        int steps = 0;
        if (run) {
          double alpha = 1.0;
          for (int q = 0; q < j; ++q) alpha *= sp.beta;
          Jh = wave_trial<R, BOX>(sm, prm, w, s, T, buf, R(alpha), commit ? __builtin_inf() : J, commit || j == 0,
                                  lane, wid, steps, R(sp.umax));
        }
        if (lane == 0) {
          sm.wJ[wid] = Jh;
          sm.wok[wid] = steps;
        }
        __syncthreads();
        ++npass;
        if (commit) {
          Jn = sm.wJ[0];
          nread += T;
          nwrite += T;
          __syncthreads();
          break;
        }
        int longest = 0;
        for (int q = 0; q < NW; ++q) {
          longest = max(longest, sm.wok[q]);
          const double v = sm.wJ[q];
          if (acc < 0 && j0 + q < sp.ls_trials && isfinite(v) && v < J) {
            acc = j0 + q;
            Jn = v;
          }
        }
        if (j0 == 0) nwrite += sm.wok[0];
        nread += longest;
        __syncthreads();
        j0 += NW;
        if (acc == 0 || (acc < 0 && j0 >= sp.ls_trials)) break;
        if (acc > 0) commit = true;
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
    if (tr.j && tid == 0) tr.j[size_t(b) * sp.max_iter + iters] = fail ? -1 : acc;
    if (fail) {
      st = fail;
      break;
    }
    if (lm) mu = fmax(mu / sp.mu_fac, sp.mu0);
    buf ^= 1;
    const double Jold = J;
    J = Jn;
    ++iters;
    if (tr.J && tid == 0) tr.J[size_t(b) * (sp.max_iter + 1) + iters] = J;
    if (sp.stop_mode == 1 && (Jold - J) <= sp.rtol * fabs(Jold)) {
      st = ST_CONVERGED;
      break;
    }
    if (iters >= sp.max_iter) st = ST_MAX_ITER;
  }
  if (tid == 0) {
    w.J[s] = J;
    w.iters[s] = iters;
    w.status[s] = st;
    w.cur[s] = buf;
    w.work[4 * s] = nsweep;
    w.work[4 * s + 1] = npass;
    w.work[4 * s + 2] = nread;
    w.work[4 * s + 3] = nwrite;
    if (lm) w.mu[s] = mu;
  }
}

template <class R>
__global__ void __launch_bounds__(NT, 2) quad_final(const double* __restrict__ prm, LaneState<R> w, int nslots,
                                                  const int32_t* __restrict__ slots, int Tmax, int max_iter,
                                                  int lookahead, FinalOut o, R* __restrict__ dblk) {
  using Q = QW<R>;
  __shared__ WaveSmem<R, NW> sm;
  const int g = blockIdx.x, tid = threadIdx.x;
  if (g >= nslots) return;
  const int s = slots ? slots[g] : g;
  const int b = w.inst[s];
  const int buf = w.cur[s];
  uint32_t st = w.status[s];
  if (st == 0) st = ST_MAX_ITER;
  const int T = (st & ST_BAD_INPUT) ? -1 : w.T[s];
  const double J = w.J[s];
  const int iters = w.iters[s];
  if (tid == 0) {
    o.J[b] = J;
    o.iters[b] = iters;
    o.status[b] = st;
    if (o.work)
      for (int i = 0; i < 4; ++i) o.work[4 * b + i] = w.work[4 * s + i];
  }
  if (o.trace)
    for (int i = iters + 1 + tid; i <= max_iter; i += NT) o.trace[size_t(b) * (max_iter + 1) + i] = J;
  double* Xo = o.X + size_t(b) * (Tmax + 1) * N;
  double* Uo = o.U + size_t(b) * Tmax * M;
  for (int idx = tid; idx < (Tmax + 1) * N; idx += NT) {
    const int k = idx / N, i = idx % N;
    Xo[idx] = k <= T ? double(Q::xp(w, buf, k, s)[i]) : 0.0;
  }
  for (int idx = tid; idx < Tmax * M; idx += NT) {
    const int k = idx / M, i = idx % M;
    Uo[idx] = k < T ? double(Q::up(w, buf, k, s)[i]) : 0.0;
  }
  const int K = lookahead <= 0 ? T : lookahead;
  if (o.xK) {
    double* xo = o.xK + size_t(b) * (Tmax + 1) * N;
    for (int idx = tid; idx < (Tmax + 1) * N; idx += NT) {
      const int k = idx / N, i = idx % N;
      xo[idx] = k <= T ? double(Q::xp(w, buf, (k + K < T ? k + K : T), s)[i]) : 0.0;
    }
  }
  double* Vo = o.Vbar ? o.Vbar + size_t(b) * (Tmax + 1) : nullptr;
  double* Lo = o.Vx ? o.Vx + size_t(b) * (Tmax + 1) * N : nullptr;
  if (T < 0) {
    if (Vo)
      for (int k = tid; k <= Tmax; k += NT) Vo[k] = 0.0;
    if (Lo)
      for (int idx = tid; idx < (Tmax + 1) * N; idx += NT) Lo[idx] = 0.0;
    return;
  }
  if (!Vo && !Lo) return;
  stage_constants(sm, prm, tid);
  __syncthreads();
  const R dt = R(prm[O_DT]);
  const R wq = R(prm[O_WQ]), wv = R(prm[O_WV]), wT = R(prm[O_WT]);
  WaveScratch<R>& w0 = sm.wv[0];
  // lambda_T = d l_T / dx
  if (tid < N) {
    w0.x[tid] = Q::xp(w, buf, T, s)[tid];
    const R wi = (tid < NQ ? wq : wv) * wT;
    sm.p[tid] = R(2) * wi * (w0.x[tid] - sm.xnom[tid]);
    if (Lo) Lo[size_t(T) * N + tid] = double(sm.p[tid]);
  }
  __syncthreads();
  if (Vo && tid < 64) {
    const double cT = double(wave_cost(sm, w0.x, w0.u, prm, tid, true));
    if (tid == 0) Vo[T] = cT;
  }
  __syncthreads();
  // costate lambda_k = l_x + f_x^T lambda_{k+1} through the adjoint of the
  // semi-implicit step instead of f_x itself: with
  // mu = lambda_v+ + dt E^T lambda_q+ and nu = M^-1 mu (M's factor from the
  // dynamics at (x_k, u_k); M is symmetric),
  //   f_x^T lambda+ = [lambda_q+ + dt g ; mu - dt (W2 cos q) . nu],
  //   g_j = -cos q_j (W1^T nu)_j + sin q_j (W2^T (nu . v))_j - 0.1 cos q_j a_j nu_j  (j < 18),
  // and nothing from the dynamics for q_18: one solve per step instead of the
  // 48 columns of [f_x | f_u].
  // The dynamics at a step (M's factor, accelerations, sin/cos) do not depend
  // on lambda: the four waves evaluate them for four steps at once (wave w
  // for step kc - w, with that step's stage cost), then wave 0 walks the four
  // steps.
  (void)dblk;
  {
    const int wid = tid >> 6, lane = tid & 63;
    const bool row = lane < NV;
    const int ri = row ? lane : 0;
    for (int kc = T - 1; kc >= 0; kc -= NW) {
      {
        const int k = kc - wid;
        WaveScratch<R>& ws = sm.wv[wid];
        if (k >= 0) {
          if (lane < N) ws.x[lane] = Q::xp(w, buf, k, s)[lane];
          if (lane < M) ws.u[lane] = Q::up(w, buf, k, s)[lane];
          wave_sync();
          if (Vo) {
            const double c = double(wave_cost(sm, ws.x, ws.u, prm, lane, false));
            if (lane == 0) Vo[k] = c;
          }
          if (Lo) wave_dyn(sm, ws, dt, lane);
        }
      }
      __syncthreads();
      if (Lo && wid == 0) {
        for (int q = 0; q < NW && kc - q >= 0; ++q) {
          const int k = kc - q;
          WaveScratch<R>& ws = sm.wv[q];
          // nu = M^-1 mu: L z = mu, then L^T nu = z (rows on lanes)
          R y = row ? sm.p[NQ + ri] + dt * (sm.p[ri] + sm.e[ri] * sm.p[NV]) : R(0);
#pragma unroll
          for (int j = 0; j < NV; ++j) {
            const R yj = bcast(y, j) * ws.Li[j];
            if (lane == j) y = yj;
            else if (lane > j) y -= ws.L[ri][j] * yj;
          }
#pragma unroll
          for (int j = NV - 1; j >= 0; --j) {
            const R zj = bcast(y, j) * ws.Li[j];
            if (lane == j) y = zj;
            else if (lane < j) y -= ws.L[j][ri] * zj;
          }
          if (row) ws.dx[ri] = y;
          wave_sync();
          R ln = R(0);
          if (lane < N) {
            ln = R(2) * (lane < NQ ? wq : wv) * (ws.x[lane] - sm.xnom[lane]);
            if (lane < NV) {
              R g1 = R(0), g2 = R(0);
#pragma unroll 6
              for (int i = 0; i < NV; ++i) {
                g1 += sm.W1[i][lane] * ws.dx[i];
                g2 += sm.W2[i][lane] * (ws.dx[i] * ws.x[NQ + i]);
              }
              const R gq = -ws.c[lane] * g1 + ws.s[lane] * g2 - R(0.1) * ws.c[lane] * ws.a[lane] * ws.dx[lane];
              ln += sm.p[lane] + dt * gq;
            } else if (lane == NV) {
              ln += sm.p[NV];
            } else {
              const int i = lane - NQ;
              const R mu = sm.p[lane] + dt * (sm.p[i] + sm.e[i] * sm.p[NV]);
              ln += mu - dt * ws.w2c[i] * ws.dx[i];
            }
          }
          wave_sync();  // every read of lambda_{k+1} is done before it is replaced
          if (lane < N) {
            sm.p[lane] = ln;
            Lo[size_t(k) * N + lane] = double(ln);
          }
          wave_sync();
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (Vo && tid == 0) {
    const double cT = Vo[T];
    if (K >= T) {
      double acc = cT;
      for (int k = T - 1; k >= 0; --k) {
        acc = Vo[k] + acc;
        Vo[k] = acc;
      }
    } else {
      for (int k = 0; k < T; ++k) {
        const int end = k + K < T ? k + K : T;
        double v = 0.0;
        for (int j = k; j < end; ++j) v += Vo[j];
        if (k + K >= T) v += cT;
        Vo[k] = v;
      }
    }
    for (int k = T + 1; k <= Tmax; ++k) Vo[k] = 0.0;
  }
  if (Lo)
    for (int idx = (T + 1) * N + tid; idx < (Tmax + 1) * N; idx += NT) Lo[idx] = 0.0;
}

template <class R>
struct QuadLaunch {
  // the lane layout, then per slot CH derivative blocks
  static size_t ws_bytes(int Bcap, int Tcap) {
    return lane_layout(N, M, int(sizeof(R)), Bcap, Tcap).total + size_t(Bcap) * CH * DB * sizeof(R);
  }
  static R* blocks(void* base, int Bcap, int Tcap) {
    return reinterpret_cast<R*>(static_cast<char*>(base) + lane_layout(N, M, int(sizeof(R)), Bcap, Tcap).total);
  }

  static hipError_t init(const double* prm, void* base, int Bcap, int Tcap, int nthreads, const int32_t* slots,
                         int Tmax, const int32_t* Tin, const int32_t* perm, const double* x0, const double* U0,
                         int max_iter, double* trace, double umax, hipStream_t st) {
    if (nthreads <= 0) return hipSuccess;
    auto w = lane_state<R>(base, N, M, Bcap, Tcap, 2);
    // one wave per instance (quad_init is built for 64-thread workgroups)
    hipLaunchKernelGGL(quad_init<R>, dim3(nthreads), dim3(64), 0, st, prm, w, nthreads, slots, Tmax, Tin, perm,
                       x0, U0, max_iter, trace, umax);
    return hipGetLastError();
  }

  // the bounded and Levenberg-Marquardt variants are kernels of their own, so
  // that the plain one keeps its register allocation and shared-memory footprint
  template <int OCC>
  static void launch_forms(bool box, bool lm, const double* prm, const LaneState<R>& w, int nthreads,
                           const int32_t* slots, const SolveParams& d, int G, const IterTrace& tr, R* blk,
                           hipStream_t st) {
    if (box && lm)
      hipLaunchKernelGGL((quad_iterate<R, true, true, OCC>), dim3(nthreads), dim3(NT), 0, st, prm, w, nthreads,
                         slots, d, G, tr, blk);
    else if (box)
      hipLaunchKernelGGL((quad_iterate<R, true, false, OCC>), dim3(nthreads), dim3(NT), 0, st, prm, w, nthreads,
                         slots, d, G, tr, blk);
    else if (lm)
      hipLaunchKernelGGL((quad_iterate<R, false, true, OCC>), dim3(nthreads), dim3(NT), 0, st, prm, w, nthreads,
                         slots, d, G, tr, blk);
    else
      hipLaunchKernelGGL((quad_iterate<R, false, false, OCC>), dim3(nthreads), dim3(NT), 0, st, prm, w, nthreads,
                         slots, d, G, tr, blk);
  }

  static hipError_t iterate(const double* prm, void* base, int Bcap, int Tcap, int nthreads,
                            const int32_t* slots, const SolveParamsH& sp, int G, int group, const IterTrace& tr,
                            hipStream_t st) {
    if (nthreads <= 0) return hipSuccess;
    auto w = lane_state<R>(base, N, M, Bcap, Tcap, 2);
    const SolveParams d = to_dev(sp);
    R* blk = blocks(base, Bcap, Tcap);
    const bool box = __builtin_isfinite(sp.umax), lm = sp.reg == 1;
    // group: workgroups per CU (2 only in FP32; FP64 always runs one per CU)
    if constexpr (sizeof(R) == 4) {
      if (group == 2) {
        launch_forms<2>(box, lm, prm, w, nthreads, slots, d, G, tr, blk, st);
        return hipGetLastError();
      }
    }
    launch_forms<1>(box, lm, prm, w, nthreads, slots, d, G, tr, blk, st);
    return hipGetLastError();
  }

  static hipError_t finalize(const double* prm, void* base, int Bcap, int Tcap, int nthreads,
                             const int32_t* slots, int Tmax, int max_iter, int lookahead, const FinalOutH& o,
                             hipStream_t st) {
    if (nthreads <= 0) return hipSuccess;
    auto w = lane_state<R>(base, N, M, Bcap, Tcap, 2);
    FinalOut fo{o.X, o.U, o.J, o.iters, o.status, o.Vbar, o.Vx, o.xK, o.trace, o.work};
    hipLaunchKernelGGL(quad_final<R>, dim3(nthreads), dim3(NT), 0, st, prm, w, nthreads, slots, Tmax, max_iter,
                       lookahead, fo, blocks(base, Bcap, Tcap));
    return hipGetLastError();
  }

  static const Launcher* get() {
    static const Launcher L{N, M, int(sizeof(R)), CBIC_SCHED_GROUP, &ws_bytes, &init, &iterate, &finalize,
                            size_t(CH) * DB * sizeof(R)};
    return &L;
  }
};

}  // namespace quad

const Launcher* launcher_quad(int precision) {
  return precision ? quad::QuadLaunch<float>::get() : quad::QuadLaunch<double>::get();
}

}  // namespace cbic
