// Host build of the solver's device models (the same header the kernels
// include) so that tests can compare each model term with the oracle on the
// CPU.  Test infrastructure only.
#include "../../paper_2602_19699_amd/csrc/dev_systems.hpp"
using namespace cbic;
template <class S> void ev(const double* prm, const double* x, const double* u, double eps, double* out) {
  constexpr int N = S::N, M = S::M;
  typename S::template Model<double> m{prm};
  double A[N][N], B[N][M], lx[N], lu[M], Q[N][N], R[M][M], xn[N];
  m.dyn(x, u, xn); m.jac(x, u, A, B); m.cost_derivs(x, u, lx, lu, Q, R, eps, true);
  double* o = out;
  for (int i = 0; i < N; ++i) *o++ = xn[i];
  for (int i = 0; i < N; ++i) for (int j = 0; j < N; ++j) *o++ = A[i][j];
  for (int i = 0; i < N; ++i) for (int j = 0; j < M; ++j) *o++ = B[i][j];
  *o++ = m.cost(x, u);
  for (int i = 0; i < N; ++i) *o++ = lx[i];
  for (int i = 0; i < M; ++i) *o++ = lu[i];
  for (int i = 0; i < N; ++i) for (int j = 0; j < N; ++j) *o++ = Q[i][j];
  for (int i = 0; i < M; ++i) for (int j = 0; j < M; ++j) *o++ = R[i][j];
  double tl[N], TQ[N][N];
  m.term_derivs(x, tl, TQ, eps, true);
  *o++ = m.term(x);
  for (int i = 0; i < N; ++i) *o++ = tl[i];
  for (int i = 0; i < N; ++i) for (int j = 0; j < N; ++j) *o++ = TQ[i][j];
}
// out: x+, A, B, l, l_x, l_u, clip(l_xx), clip(l_uu), l_T, l_T,x, clip(l_T,xx)
extern "C" void ev_pm(const double* p, const double* x, const double* u, double eps, double* o) { ev<PointMass>(p, x, u, eps, o); }
extern "C" void ev_arm(const double* p, const double* x, const double* u, double eps, double* o) { ev<Arm3>(p, x, u, eps, o); }
