// Host runtime: error reporting, workspace layouts, per-system device
// parameter blocks, the launcher table and the batched solve entry point.
#include "runtime.hpp"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>

namespace cbic {

const Launcher* launcher_point_mass(int precision);
const Launcher* launcher_lq(int n, int m, int precision);
const Launcher* launcher_arm(int precision);
const Launcher* launcher_quad(int precision);

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

const char* last_error() { return g_err; }

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

LaneLayout lane_layout(int N, int M, int elem, int Bcap, int Tcap, int nbuf) {
  LaneLayout L{};
  size_t o = 0;
  const size_t B = size_t(Bcap);
  L.T = o; o = align256(o + 4 * B);
  L.inst = o; o = align256(o + 4 * B);
  L.J = o; o = align256(o + 8 * B);
  L.iters = o; o = align256(o + 4 * B);
  L.status = o; o = align256(o + 4 * B);
  L.cur = o; o = align256(o + 4 * B);
  L.work = o; o = align256(o + 16 * B);
  L.mu = o; o = align256(o + 8 * B);
  L.okey = o; o = align256(o + 4 * B);
  // slot-major, each slot's block padded to whole cache lines
  L.X = o; o = align256(o + size_t(elem) * nbuf * B * lane_stride((Tcap + 1) * N, elem));
  L.U = o; o = align256(o + size_t(elem) * nbuf * B * lane_stride(Tcap * M, elem));
  L.K = o; o = align256(o + size_t(elem) * B * lane_stride(Tcap * M * N, elem));
  L.kf = o; o = align256(o + size_t(elem) * B * lane_stride(Tcap * M, elem));
  L.total = o;
  return L;
}

const Launcher* find_launcher(int kind, int n, int m, int precision, int schedule) {
  const Launcher* L = nullptr;
  switch (kind) {
    case CBIC_SYS_POINT_MASS: L = launcher_point_mass(precision); break;
    case CBIC_SYS_PLANAR3: L = launcher_arm(precision); break;
    case CBIC_SYS_LQ: L = launcher_lq(n, m, precision); break;
    case CBIC_SYS_QUAD_SYNTH: L = launcher_quad(precision); break;
    default: break;
  }
  if (L && schedule != 0 && L->schedule != schedule) return nullptr;
  return L;
}

int cu_count(int device) {
  static std::atomic<int> cache[64];
  if (device < 0 || device >= 64) return 256;
  int v = cache[device].load(std::memory_order_relaxed);
  if (v > 0) return v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || v <= 0) v = 256;
  cache[device].store(v, std::memory_order_relaxed);
  return v;
}

int default_group(int schedule, int B, int precision, int device) {
  if (schedule == CBIC_SCHED_GROUP) return (precision == CBIC_FP64 || B <= cu_count(device)) ? 1 : 2;
  int g = 1;
  while (g < 16 && long(B) * g * 2 <= 65536) g *= 2;
  return g;
}

int requested_group(const Launcher* L, const cbic_solve_opts* o) {
  return L->schedule == CBIC_SCHED_GROUP ? o->wg_per_cu : o->group_lanes;
}

// ------------------------------------------------------------------ host Jacobi (LQ Hessians)
// Symmetric eigen-decomposition by cyclic Jacobi rotations; used once per LQ
// system to clip its constant Hessians.
static void host_clip(int n, const double* H, double eps, double* out) {
  std::vector<double> a(n * n), v(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a[i * n + j] = 0.5 * (H[i * n + j] + H[j * n + i]);
  if (eps < 0.0) {  // no clipping (the Levenberg-Marquardt variant): symmetric part only
    for (int i = 0; i < n * n; ++i) out[i] = a[i];
    return;
  }
  for (int i = 0; i < n; ++i) v[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) (i == j ? dia : off) += a[i * n + j] * a[i * n + j];
    if (!(off > 1e-32 * dia)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (apq == 0.0) continue;
        const double th = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(1.0 + th * th));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double x = a[k * n + p], y = a[k * n + q];
          a[k * n + p] = c * x - s * y;
          a[k * n + q] = s * x + c * y;
        }
        for (int k = 0; k < n; ++k) {
          const double x = a[p * n + k], y = a[q * n + k];
          a[p * n + k] = c * x - s * y;
          a[q * n + k] = s * x + c * y;
        }
        for (int k = 0; k < n; ++k) {
          const double x = v[k * n + p], y = v[k * n + q];
          v[k * n + p] = c * x - s * y;
          v[k * n + q] = s * x + c * y;
        }
      }
  }
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += v[i * n + k] * std::max(a[k * n + k], eps) * v[j * n + k];
      out[i * n + j] = s;
      out[j * n + i] = s;
    }
}

// ------------------------------------------------------------------ device parameter blocks
static bool all_finite(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

bool build_device_block(const cbic_system* s, double eps, std::vector<double>& d) {
  const std::vector<double>& p = s->params;
  d.clear();
  switch (s->kind) {
    case CBIC_SYS_POINT_MASS: {
      d = {p[0], p[1], p[2], p[3], p[4], p[5], p[6]};
      for (int i = 0; i < 3; ++i) {
        d.push_back(p[7 + 3 * i]);
        d.push_back(p[8 + 3 * i]);
        d.push_back(1.0 / (p[9 + 3 * i] * p[9 + 3 * i]));
      }
      return true;
    }
    case CBIC_SYS_PLANAR3: {
      const double m1 = p[1], m2 = p[2], m3 = p[3], l1 = p[4], l2 = p[5], l3 = p[6];
      const double I1 = m1 * l1 * l1 / 12.0, I2 = m2 * l2 * l2 / 12.0, I3 = m3 * l3 * l3 / 12.0;
      const double h11 = m1 * l1 * l1 / 4.0 + (m2 + m3) * l1 * l1;
      const double h22 = m2 * l2 * l2 / 4.0 + m3 * l2 * l2;
      const double h33 = m3 * l3 * l3 / 4.0;
      const double h12 = (0.5 * m2 + m3) * l1 * l2;
      const double h13 = 0.5 * m3 * l1 * l3;
      const double h23 = 0.5 * m3 * l2 * l3;
      d = {p[0], h11 + I1, h22 + I2, h33 + I3, h12, h13, h23, l1, l2, l3,
           p[7], p[8], p[9], p[10], p[11], p[12], p[13], p[14], 1.0 / (p[15] * p[15])};
      return true;
    }
    case CBIC_SYS_LQ: {
      const int n = s->n, m = s->m;
      const double* A = p.data() + 2;
      const double* B = A + n * n;
      const double* Q = B + n * m;
      const double* R = Q + n * n;
      const double* QT = R + m * m;
      const double* xr = QT + n * n;
      std::vector<double> Qs(n * n), Rs(m * m), QTs(n * n), Qc(n * n), Rc(m * m), QTc(n * n);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          Qs[i * n + j] = Q[i * n + j] + Q[j * n + i];
          QTs[i * n + j] = QT[i * n + j] + QT[j * n + i];
        }
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Rs[i * m + j] = R[i * m + j] + R[j * m + i];
      host_clip(n, Qs.data(), eps, Qc.data());
      host_clip(m, Rs.data(), eps, Rc.data());
      host_clip(n, QTs.data(), eps, QTc.data());
      d.insert(d.end(), A, A + n * n);
      d.insert(d.end(), B, B + n * m);
      d.insert(d.end(), Qs.begin(), Qs.end());
      d.insert(d.end(), Rs.begin(), Rs.end());
      d.insert(d.end(), QTs.begin(), QTs.end());
      d.insert(d.end(), xr, xr + n);
      d.insert(d.end(), Qc.begin(), Qc.end());
      d.insert(d.end(), Rc.begin(), Rc.end());
      d.insert(d.end(), QTc.begin(), QTc.end());
      return true;
    }
    case CBIC_SYS_QUAD_SYNTH: {
      // same layout as the user's vector with A replaced by the constant part
      // of the mass matrix, A^T A
      d = p;
      const double* A = p.data() + 5;
      for (int a = 0; a < 18; ++a)
        for (int b = 0; b < 18; ++b) {
          double v = 0.0;
          for (int k = 0; k < 18; ++k) v += A[k * 18 + a] * A[k * 18 + b];
          d[5 + a * 18 + b] = v;
        }
      return true;
    }
    default:
      return false;
  }
}

bool make_device_block(cbic_system* s, double eps) { return build_device_block(s, eps, s->dev); }

bool validate_params(int kind, const double* p, size_t np, int* n, int* m) {
  if (!p) {
    set_error("params is NULL");
    return false;
  }
  if (!all_finite(p, np)) {
    set_error("params contain a non-finite value");
    return false;
  }
  switch (kind) {
    case CBIC_SYS_POINT_MASS:
      if (np != 16) { set_error("point mass needs 16 parameters, got %zu", np); return false; }
      if (!(p[0] > 0)) { set_error("dt must be > 0"); return false; }
      for (int i = 0; i < 3; ++i)
        if (!(p[9 + 3 * i] > 0)) { set_error("obstacle radius must be > 0"); return false; }
      *n = 4; *m = 2;
      return true;
    case CBIC_SYS_PLANAR3:
      if (np != 16) { set_error("planar arm needs 16 parameters, got %zu", np); return false; }
      if (!(p[0] > 0)) { set_error("dt must be > 0"); return false; }
      for (int i = 1; i < 7; ++i)
        if (!(p[i] > 0)) { set_error("link masses and lengths must be > 0"); return false; }
      if (!(p[15] > 0)) { set_error("obstacle radius must be > 0"); return false; }
      *n = 6; *m = 3;
      return true;
    case CBIC_SYS_QUAD_SYNTH:
      if (np != 5 + 3 * 324 + 18 + 37) { set_error("quadruped needs 1032 parameters, got %zu", np); return false; }
      if (!(p[0] > 0)) { set_error("dt must be > 0"); return false; }
      *n = 37; *m = 12;
      return true;
    case CBIC_SYS_LQ: {
      if (np < 2) { set_error("LQ parameter vector too short"); return false; }
      const double dn = p[0], dm = p[1];
      if (dn != std::floor(dn) || dm != std::floor(dm) || dn < 1 || dm < 1 || dn > 64 || dm > 64) {
        set_error("LQ dims must be integers in 1..64");
        return false;
      }
      const int nn = int(dn), mm = int(dm);
      const size_t need = 2 + 3 * size_t(nn) * nn + size_t(nn) * mm + size_t(mm) * mm + nn;
      if (np != need) { set_error("LQ with n=%d m=%d needs %zu parameters, got %zu", nn, mm, need, np); return false; }
      *n = nn; *m = mm;
      return true;
    }
    default:
      set_error("unknown system kind %d", kind);
      return false;
  }
}

}  // namespace cbic
