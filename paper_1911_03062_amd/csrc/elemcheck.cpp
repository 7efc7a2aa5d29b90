// Host build of the kernels' element math (projections.h) with a C ABI, so that the local
// step's per-triangle and per-hinge residuals can be checked on the CPU in both precisions.
#include <hip/hip_runtime.h>

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

}  // namespace

extern "C" {
// p: [3][3] vertex positions a, b, c; g: (g_b0, g_b1, g_c0, g_c1); out: [3][3] contributions.
void npfem_check_triangle(const double* p, const double* g, double area, double w_s, double w_a,
                          double s_min, double s_max, double* out, int precision) {
  if (precision == 64) tri<double>(p, g, area, w_s, w_a, s_min, s_max, out);
  else tri<float>(p, g, area, w_s, w_a, s_min, s_max, out);
}
// p: [4][3] positions i, j, k, l; a: stencil [4]; out: [4][3] contributions.
void npfem_check_hinge(const double* p, const double* a, double rest, double w_b, double* out,
                       int precision) {
  if (precision == 64) hin<double>(p, a, rest, w_b, out);
  else hin<float>(p, a, rest, w_b, out);
}
}
