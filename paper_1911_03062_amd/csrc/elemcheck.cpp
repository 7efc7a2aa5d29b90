// Host build of the kernels' element math (projections.h) with a C ABI, so that the local
// step's per-triangle and per-hinge residuals can be checked on the CPU in both precisions.
#include <hip/hip_runtime.h>

#include "filters.h"
#include "projections.h"

using namespace npfem;

namespace {

template <typename T>
void tri(const double* p, const double* g, double area, double ws, double wa, double smin,
         double smax, double* out) {
  const Vec3<T> a = v3<T>(p[0], p[1], p[2]), b = v3<T>(p[3], p[4], p[5]), c = v3<T>(p[6], p[7], p[8]);
  Vec3<T> ra = v3<T>(0, 0, 0), rb = ra, rc = ra;
  triangle_residual<T>(a, b, c, (T)g[0], (T)g[1], (T)g[2], (T)g[3], (T)area, (T)ws, (T)wa,
                       (T)smin, (T)smax, ra, rb, rc);
  const Vec3<T> r[3] = {ra, rb, rc};
  for (int q = 0; q < 3; ++q) {
    out[3 * q] = r[q].x;
    out[3 * q + 1] = r[q].y;
    out[3 * q + 2] = r[q].z;
  }
}

template <typename T>
void hin(const double* p, const double* a, double rest, double wb, double* out) {
  Vec3<T> r[4] = {v3<T>(0, 0, 0), v3<T>(0, 0, 0), v3<T>(0, 0, 0), v3<T>(0, 0, 0)};
  hinge_residual<T>(v3<T>(p[0], p[1], p[2]), v3<T>(p[3], p[4], p[5]), v3<T>(p[6], p[7], p[8]),
                    v3<T>(p[9], p[10], p[11]), (T)a[1], (T)a[2], (T)a[3], (T)rest, (T)wb, r[0],
                    r[1], r[2], r[3]);
  for (int q = 0; q < 4; ++q) {
    out[3 * q] = r[q].x;
    out[3 * q + 1] = r[q].y;
    out[3 * q + 2] = r[q].z;
  }
}

template <typename T, int N>
double median_net(const double* vals, int k) {
  T a[N];
  for (int q = 0; q < N; ++q) a[q] = q < k ? (T)vals[q] : (T)__builtin_inf();
  return median_keys<N>(a, k);
}
template <typename T>
double median_any(const double* vals, int k) {
  if (k <= 8) return median_net<T, 8>(vals, k);
  if (k <= 16) return median_net<T, 16>(vals, k);
  return median_net<T, 32>(vals, k);
}

}  // namespace

extern "C" {
// p: [3][3] vertex positions a, b, c; g: (g_b0, g_b1, g_c0, g_c1); out: [3][3] contributions.
// Skalak triangle (p: [3][3], g: (g_b0, g_b1, g_c0, g_c1)): contributions to out [3][3],
// returns the energy A W.
double npfem_check_skalak(const double* p, const double* g, double area, double B, double C,
                          double* out, int precision) {
  if (precision == 64) {
    Vec3<double> r[3] = {v3<double>(0, 0, 0), v3<double>(0, 0, 0), v3<double>(0, 0, 0)};
    const double E = skalak_residual<double>(v3<double>(p[0], p[1], p[2]), v3<double>(p[3], p[4], p[5]),
                                             v3<double>(p[6], p[7], p[8]), g[0], g[1], g[2], g[3],
                                             area, B, C, r[0], r[1], r[2]);
    for (int q = 0; q < 3; ++q) { out[3 * q] = r[q].x; out[3 * q + 1] = r[q].y; out[3 * q + 2] = r[q].z; }
    return E;
  }
  Vec3<float> r[3] = {v3<float>(0, 0, 0), v3<float>(0, 0, 0), v3<float>(0, 0, 0)};
  const float E = skalak_residual<float>(v3<float>(p[0], p[1], p[2]), v3<float>(p[3], p[4], p[5]),
                                         v3<float>(p[6], p[7], p[8]), (float)g[0], (float)g[1],
                                         (float)g[2], (float)g[3], (float)area, (float)B, (float)C,
                                         r[0], r[1], r[2]);
  for (int q = 0; q < 3; ++q) { out[3 * q] = r[q].x; out[3 * q + 1] = r[q].y; out[3 * q + 2] = r[q].z; }
  return E;
}
void npfem_check_triangle(const double* p, const double* g, double area, double w_s, double w_a,
                          double s_min, double s_max, double* out, int precision) {
  if (precision == 64) tri<double>(p, g, area, w_s, w_a, s_min, s_max, out);
  else tri<float>(p, g, area, w_s, w_a, s_min, s_max, out);
}
// Position-based damping of one cell with the kernels' helpers: x, v [n][3]; out [n][3] damped
// velocities. Two passes in FP64 (centre of mass, then momentum and inertia), as the kernels.
void npfem_check_pbd(const double* x, const double* v, int n, double kappa, double* out) {
  double xc[3] = {0, 0, 0}, vc[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      xc[d] += x[3 * i + d];
      vc[d] += v[3 * i + d];
    }
  for (int d = 0; d < 3; ++d) {
    xc[d] /= n;
    vc[d] /= n;
  }
  double Isym[6] = {0, 0, 0, 0, 0, 0}, Lm[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i) {
    const double r[3] = {x[3 * i] - xc[0], x[3 * i + 1] - xc[1], x[3 * i + 2] - xc[2]};
    const double* u = v + 3 * i;
    Lm[0] += r[1] * u[2] - r[2] * u[1];
    Lm[1] += r[2] * u[0] - r[0] * u[2];
    Lm[2] += r[0] * u[1] - r[1] * u[0];
    const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    Isym[0] += rr - r[0] * r[0];
    Isym[1] += rr - r[1] * r[1];
    Isym[2] += rr - r[2] * r[2];
    Isym[3] -= r[0] * r[1];
    Isym[4] -= r[0] * r[2];
    Isym[5] -= r[1] * r[2];
  }
  double w[3];
  solve_sym3(Isym, Lm, w);
  for (int i = 0; i < n; ++i) {
    const Vec3<double> r = v3<double>(x[3 * i] - xc[0], x[3 * i + 1] - xc[1], x[3 * i + 2] - xc[2]);
    const Vec3<double> o = pbd_velocity<double>(v3<double>(v[3 * i], v[3 * i + 1], v[3 * i + 2]), r,
                                                v3<double>(vc[0], vc[1], vc[2]),
                                                v3<double>(w[0], w[1], w[2]), kappa);
    out[3 * i] = o.x;
    out[3 * i + 1] = o.y;
    out[3 * i + 2] = o.z;
  }
}
// Median of k (1..32) values with the kernels' sorting networks (8, 16 or 32 keys, the
// smallest that holds k) and middle selection, in the given precision.
double npfem_check_median(const double* vals, int k, int precision) {
  return precision == 64 ? median_any<double>(vals, k) : median_any<float>(vals, k);
}
// Median of k values by the kernels' rank selection (the path of wide rings).
double npfem_check_median_rank(const double* vals, int k, int precision) {
  if (precision == 64) return median_rank<double>(k, [&](int i) { return vals[i]; });
  return median_rank<float>(k, [&](int i) { return (float)vals[i]; });
}
// Number of 0/1 key vectors of length n (8 or 16) that the sorting network leaves unsorted
// (zero-one principle: a comparator network sorts every input iff it sorts all 0/1 inputs).
int npfem_check_sortnet01(int n) {
  int bad = 0;
  for (int m = 0; m < (1 << n); ++m) {
    if (n == 8) {
      float a[8];
      for (int q = 0; q < 8; ++q) a[q] = (float)((m >> q) & 1);
      sort_keys<8>(a);
      for (int q = 1; q < 8; ++q) bad += a[q - 1] > a[q];
    } else {
      float a[16];
      for (int q = 0; q < 16; ++q) a[q] = (float)((m >> q) & 1);
      sort_keys<16>(a);
      for (int q = 1; q < 16; ++q) bad += a[q - 1] > a[q];
    }
  }
  return bad;
}
// Velocity cap of one vector with the kernels' helper.
void npfem_check_cap(double* v, double v_max, int precision) {
  if (precision == 64) {
    cap_speed<double>(v[0], v[1], v[2], v_max);
    return;
  }
  float f[3] = {(float)v[0], (float)v[1], (float)v[2]};
  cap_speed<float>(f[0], f[1], f[2], (float)v_max);
  for (int q = 0; q < 3; ++q) v[q] = f[q];
}
// p: [4][3] positions i, j, k, l; a: stencil [4]; out: [4][3] contributions.
void npfem_check_hinge(const double* p, const double* a, double rest, double w_b, double* out,
                       int precision) {
  if (precision == 64) hin<double>(p, a, rest, w_b, out);
  else hin<float>(p, a, rest, w_b, out);
}
}
