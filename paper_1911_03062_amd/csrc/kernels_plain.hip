// Plain one-cell-at-a-time form of the npFEM step: for one cell, a prediction kernel, then
// n_pd_iters pairs of (local, global) kernels, then a finalisation kernel, each a separate
// launch of one workgroup (2K + 2 launches per cell and step). Templated on precision; the
// FP64 instance runs the whole path in double.
//
// Step (supplementary material, npFEM subsection, implicit Euler and its quasi-Newton
// iteration): delta = x - x_n; delta^0 = y_n - x_n = h M~^-1 (M v_n + h F) (the prediction;
// h v_n + h^2 F/m without damping); iterate delta <- delta - L^-1 grad g(x_n + delta) with
// grad g = (M~/h^2) e + constraint residuals, e = delta - delta^0; then x_{n+1} = x_n + delta,
// v_{n+1} = delta / h. Rayleigh damping C = alpha M + beta K gives M~ = (1 + h alpha) M +
// h beta K: its prediction is one banded solve with M~'s factor, its gradient term
// (beta/h) K e a banded product. Positions inside the kernels are taken relative to the
// cell's first vertex, which leaves every difference, and the enclosed volume, unchanged.
#include <hip/hip_runtime.h>

#include "banded.h"
#include "npfem_internal.h"
#include "filters.h"
#include "projections.h"

namespace npfem {

namespace {

constexpr int kPlainThreads = 256;
constexpr int kMaxBand = 1024;

template <typename T>
struct PlainWork {
  // all arrays live in one device allocation, laid out by plain_layout()
  T* d0;      // [3][n] delta^0
  T* d;       // [3][n] delta^k
  T* r;       // [3][n] gradient of g
  T* gv;      // [3][n] volume gradient
  T* tcon;    // [m][3][3] triangle contributions to (a, b, c)
  T* tn;      // [m][3] twice the triangle area vector
  T* hcon;    // [e][4][3] hinge contributions
  T* dir;     // [3][n] search direction (Skalak membrane)
};

template <typename T>
__host__ __device__ inline PlainWork<T> plain_layout(void* base, int n, int m, int e) {
  T* p = reinterpret_cast<T*>(base);
  PlainWork<T> w;
  w.d0 = p; p += 3 * n;
  w.d = p; p += 3 * n;
  w.r = p; p += 3 * n;
  w.gv = p; p += 3 * n;
  w.tcon = p; p += 9 * m;
  w.tn = p; p += 3 * m;
  w.hcon = p; p += 12 * e;
  w.dir = p;
  return w;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0;
  const int nw = (blockDim.x + 63) / 64;
  for (int i = 0; i < nw; ++i) s += sh[i];   // same order in every thread
  return s;
}

template <typename T>
__device__ inline Vec3<T> cell_pos(const T* x, int64_t vt, int64_t off, const T* d, int n, int i) {
  return v3<T>((x[off + i] - x[off]) + d[i], (x[vt + off + i] - x[vt + off]) + d[n + i],
               (x[2 * vt + off + i] - x[2 * vt + off]) + d[2 * n + i]);
}

// delta^0 = h v_n + h^2 F/m, with v_n first damped (position-based damping) when kappa > 0:
// centre of mass and its velocity, then angular momentum and inertia about it (positions
// relative to the cell's first vertex, FP64 block sums), w = I^-1 L.
template <typename T>
__global__ void __launch_bounds__(kPlainThreads)
k_plain_predict(TypeParams p, const T* __restrict__ x, const T* __restrict__ v,
                const T* __restrict__ f, int64_t vt, int64_t off, void* work) {
  PlainWork<T> w = plain_layout<T>(work, p.n, p.m, p.e);
  const T h = T(p.h), h2m = T(p.h2_over_m);
  const int n = p.n;
  __shared__ double sh[8];
  auto xl = [&](int i) {
    return v3<T>(x[off + i] - x[off], x[vt + off + i] - x[vt + off],
                 x[2 * vt + off + i] - x[2 * vt + off]);
  };
  auto vel = [&](int i) { return v3<T>(v[off + i], v[vt + off + i], v[2 * vt + off + i]); };
  Vec3<T> vcm = v3<T>(0, 0, 0), xcm = vcm, om = vcm;
  const bool damp = p.kappa > 0.0;
  if (damp) {
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const Vec3<T> a = xl(i), b = vel(i);
      s[0] += a.x; s[1] += a.y; s[2] += a.z;
      s[3] += b.x; s[4] += b.y; s[5] += b.z;
    }
    double c[6];
    for (int k = 0; k < 6; ++k) c[k] = block_sum(s[k], sh) / n;
    double q[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // L (3), I (xx, yy, zz, xy, xz, yz)
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const Vec3<T> a = xl(i), b = vel(i);
      const double r0 = (double)a.x - c[0], r1 = (double)a.y - c[1], r2 = (double)a.z - c[2];
      q[0] += r1 * b.z - r2 * b.y;
      q[1] += r2 * b.x - r0 * b.z;
      q[2] += r0 * b.y - r1 * b.x;
      const double rr = r0 * r0 + r1 * r1 + r2 * r2;
      q[3] += rr - r0 * r0; q[4] += rr - r1 * r1; q[5] += rr - r2 * r2;
      q[6] -= r0 * r1; q[7] -= r0 * r2; q[8] -= r1 * r2;
    }
    double t[9];
    for (int k = 0; k < 9; ++k) t[k] = block_sum(q[k], sh);
    double wv[3];
    solve_sym3(t + 3, t, wv);
    xcm = v3<T>(T(c[0]), T(c[1]), T(c[2]));
    vcm = v3<T>(T(c[3]), T(c[4]), T(c[5]));
    om = v3<T>(T(wv[0]), T(wv[1]), T(wv[2]));
  }
  // Rayleigh damping with beta > 0: the right-hand side M (h v + h^2 F/m) of M~ delta^0 goes
  // to r for the solve that follows; otherwise delta^0 = (h v + h^2 F/m) / (1 + h alpha)
  const bool ray_solve = p.ray_k > 0.0;
  const T ph = T(p.pred_h), ph2m = T(p.pred_h2m), mm = T(p.mass);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    Vec3<T> vi = vel(i);
    if (damp) vi = pbd_velocity<T>(vi, xl(i) - xcm, vcm, om, T(p.kappa));
    const T vv[3] = {vi.x, vi.y, vi.z};
    for (int c = 0; c < 3; ++c) {
      if (ray_solve) {
        w.r[c * n + i] = mm * (h * vv[c] + h2m * f[c * vt + off + i]);
      } else {
        const T d0 = ph * vv[c] + ph2m * f[c * vt + off + i];
        w.d0[c * n + i] = d0;
        w.d[c * n + i] = d0;
      }
    }
  }
}

template <typename T>
struct PlainConst;
template <>
struct PlainConst<float> {
  static __device__ const float* G(const DevType& t) { return t.G32; }
  static __device__ const float* A(const DevType& t) { return t.A32; }
  static __device__ const float* coef(const DevType& t) { return t.coef32; }
  static __device__ const float* rest(const DevType& t) { return t.rest32; }
  static __device__ const float* cband(const DevType& t) { return t.cband32; }
  static __device__ const float* mband(const DevType& t) { return t.mband32; }
  static __device__ const float* kband(const DevType& t) { return t.kband32; }
};
template <>
struct PlainConst<double> {
  static __device__ const double* G(const DevType& t) { return t.G64; }
  static __device__ const double* A(const DevType& t) { return t.A64; }
  static __device__ const double* coef(const DevType& t) { return t.coef64; }
  static __device__ const double* rest(const DevType& t) { return t.rest64; }
  static __device__ const double* cband(const DevType& t) { return t.cband64; }
  static __device__ const double* mband(const DevType& t) { return t.mband64; }
  static __device__ const double* kband(const DevType& t) { return t.kband64; }
};

// Local step: projections of every constraint at x^k and assembly of grad g(x^k) into r,
// with the collision energies' w (x - p) when contacts are given (cp, cw: [3][V], [V]).
template <typename T>
__global__ void __launch_bounds__(kPlainThreads)
k_plain_local(const DevType* __restrict__ dtp, const T* __restrict__ x, int64_t vt, int64_t off,
              void* work, const T* __restrict__ cp, const T* __restrict__ cw) {
  const DevType& dt = *dtp;
  const TypeParams& p = dt.p;
  const int n = p.n, m = p.m, e = p.e;
  PlainWork<T> w = plain_layout<T>(work, n, m, e);
  const T* G = PlainConst<T>::G(dt);
  const T* A = PlainConst<T>::A(dt);
  const T* coef = PlainConst<T>::coef(dt);
  const T* rest = PlainConst<T>::rest(dt);
  __shared__ double sh[8];
  __shared__ double lam_sh;

  for (int t = threadIdx.x; t < m; t += blockDim.x) {
    const int a = dt.tri[3 * t], b = dt.tri[3 * t + 1], c = dt.tri[3 * t + 2];
    const Vec3<T> pa = cell_pos(x, vt, off, w.d, n, a);
    const Vec3<T> pb = cell_pos(x, vt, off, w.d, n, b);
    const Vec3<T> pc = cell_pos(x, vt, off, w.d, n, c);
    Vec3<T> ra = v3<T>(0, 0, 0), rb = ra, rc = ra;   // contributions are accumulated
    if (p.skalak)
      (void)skalak_residual<T>(pa, pb, pc, G[6 * t + 2], G[6 * t + 3], G[6 * t + 4], G[6 * t + 5],
                               A[t], T(p.w_s), T(p.w_a), ra, rb, rc);
    else
      triangle_residual<T>(pa, pb, pc, G[6 * t + 2], G[6 * t + 3], G[6 * t + 4], G[6 * t + 5],
                           A[t], T(p.w_s), T(p.w_a), T(p.s_min), T(p.s_max), ra, rb, rc);
    T* tc = w.tcon + 9 * t;
    tc[0] = ra.x; tc[1] = ra.y; tc[2] = ra.z;
    tc[3] = rb.x; tc[4] = rb.y; tc[5] = rb.z;
    tc[6] = rc.x; tc[7] = rc.y; tc[8] = rc.z;
    const Vec3<T> nt = cross3(pb - pa, pc - pa);
    w.tn[3 * t] = nt.x; w.tn[3 * t + 1] = nt.y; w.tn[3 * t + 2] = nt.z;
  }
  for (int h = threadIdx.x; h < e; h += blockDim.x) {
    const int* hv = dt.hinge + 4 * h;
    Vec3<T> ri = v3<T>(0, 0, 0), rj = ri, rk = ri, rl = ri;
    hinge_residual<T>(cell_pos(x, vt, off, w.d, n, hv[0]), cell_pos(x, vt, off, w.d, n, hv[1]),
                      cell_pos(x, vt, off, w.d, n, hv[2]), cell_pos(x, vt, off, w.d, n, hv[3]),
                      coef[4 * h + 1], coef[4 * h + 2], coef[4 * h + 3], rest[h], T(p.w_b),
                      ri, rj, rk, rl);
    T* hc = w.hcon + 12 * h;
    hc[0] = ri.x; hc[1] = ri.y; hc[2] = ri.z;
    hc[3] = rj.x; hc[4] = rj.y; hc[5] = rj.z;
    hc[6] = rk.x; hc[7] = rk.y; hc[8] = rk.z;
    hc[9] = rl.x; hc[10] = rl.y; hc[11] = rl.z;
  }
  __syncthreads();
  // volume gradient (1/6 of the summed doubled area vectors of the incident triangles),
  // V = 1/3 sum_i x_i . grad_i V and |grad V|^2, reduced in FP64
  double vpart = 0, gpart = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    T gx = 0, gy = 0, gz = 0;
    for (int s = dt.vt_off[i]; s < dt.vt_off[i + 1]; ++s) {
      const int t = dt.vt_list[s] / 3;
      gx += w.tn[3 * t]; gy += w.tn[3 * t + 1]; gz += w.tn[3 * t + 2];
    }
    gx *= T(1.0 / 6.0); gy *= T(1.0 / 6.0); gz *= T(1.0 / 6.0);
    w.gv[i] = gx; w.gv[n + i] = gy; w.gv[2 * n + i] = gz;
    const Vec3<T> pi = cell_pos(x, vt, off, w.d, n, i);
    vpart += (double)pi.x * (double)gx + (double)pi.y * (double)gy + (double)pi.z * (double)gz;
    gpart += (double)gx * (double)gx + (double)gy * (double)gy + (double)gz * (double)gz;
  }
  const double V = block_sum(vpart, sh) / 3.0;
  const double G2 = block_sum(gpart, sh);
  if (threadIdx.x == 0) lam_sh = G2 > 0 ? (p.V0 - V) / G2 : 0.0;
  __syncthreads();
  const T lam_w = T(lam_sh * p.w_v);
  const T ih2m = T(p.inv_h2m), ray_k = T(p.ray_k);
  const T* kb = PlainConst<T>::kband(dt);
  const int bw = p.bw, bs = bw + 1;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    for (int c = 0; c < 3; ++c) {
      T acc = ih2m * (w.d[c * n + i] - w.d0[c * n + i]);
      if (p.ray_k > 0.0) {   // Rayleigh: (beta/h) (K e)_i, K symmetric, lower band stored
        const T* dc = w.d + c * n;
        const T* d0c = w.d0 + c * n;
        T ke = 0;
        for (int k = 0; k <= bw && k <= i; ++k) ke += kb[i * bs + k] * (dc[i - k] - d0c[i - k]);
        for (int k = 1; k <= bw && i + k < n; ++k) ke += kb[(i + k) * bs + k] * (dc[i + k] - d0c[i + k]);
        acc += ray_k * ke;
      }
      for (int s = dt.vt_off[i]; s < dt.vt_off[i + 1]; ++s) acc += w.tcon[3 * dt.vt_list[s] + c];
      for (int s = dt.vh_off[i]; s < dt.vh_off[i + 1]; ++s) acc += w.hcon[3 * dt.vh_list[s] + c];
      acc -= lam_w * w.gv[c * n + i];
      if (cw != nullptr) {
        const T wc = cw[off + i];
        if (wc != T(0))   // x - p = (x_n - p) + delta
          acc += wc * ((x[c * vt + off + i] - cp[c * vt + off + i]) + w.d[c * n + i]);
      }
      w.r[c * n + i] = acc;
    }
  }
}

// Banded solve of r (three right-hand sides, one wave per coordinate, band products reduced
// across the wave). Global step (kSolveUpdate): L D = r with L's factor, then delta -= D.
// Prediction (kSolvePredict, Rayleigh damping with beta > 0): M~ D = r with M~'s factor,
// then delta^0 = delta = D. Direction (kSolveDirection, Skalak membrane): dir = -L^-1 r.
enum { kSolveUpdate = 0, kSolvePredict = 1, kSolveDirection = 2 };
template <typename T>
__global__ void __launch_bounds__(192)
k_plain_solve(const DevType* __restrict__ dtp, void* work, int mode) {
  const bool predict = mode == kSolvePredict;
  const DevType& dt = *dtp;
  const int n = dt.p.n, bw = dt.p.bw, bs = bw + 1;
  PlainWork<T> w = plain_layout<T>(work, n, dt.p.m, dt.p.e);
  const T* cb = predict ? PlainConst<T>::mband(dt) : PlainConst<T>::cband(dt);
  __shared__ T y[3][kMaxBand];
  const int c = threadIdx.x >> 6, lane = threadIdx.x & 63;
  T* yc = y[c];
  const T* rc = w.r + c * n;
  for (int i = 0; i < n; ++i) {
    T part = 0;
    const int kmax = bw < i ? bw : i;
    for (int k = lane + 1; k <= kmax; k += 64) part += cb[i * bs + k] * yc[i - k];
    const T s = wave_sum(part);
    const T yi = (rc[i] - s) / cb[i * bs];
    if (lane == 0) yc[i] = yi;
    __builtin_amdgcn_wave_barrier();
  }
  for (int i = n - 1; i >= 0; --i) {
    T part = 0;
    const int kmax = bw < (n - 1 - i) ? bw : (n - 1 - i);
    for (int k = lane + 1; k <= kmax; k += 64) part += cb[(i + k) * bs + k] * yc[i + k];
    const T s = wave_sum(part);
    const T xi = (yc[i] - s) / cb[i * bs];
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) yc[i] = xi;
    __builtin_amdgcn_wave_barrier();
  }
  if (predict) {
    for (int i = lane; i < n; i += 64) {
      w.d0[c * n + i] = yc[i];
      w.d[c * n + i] = yc[i];
    }
  } else if (mode == kSolveDirection) {
    for (int i = lane; i < n; i += 64) w.dir[c * n + i] = -yc[i];
  } else {
    for (int i = lane; i < n; i += 64) w.d[c * n + i] -= yc[i];
  }
}

// The same solves (kSolveUpdate, kSolveDirection) by the register-window substitution of
// banded.h: one wave, lanes 0-2 take the three coordinates (the factor through scalar loads,
// pending row sums in registers), then the whole wave applies the result.
template <typename T, int BW>
__global__ void __launch_bounds__(64)
k_plain_solve_band(const DevType* __restrict__ dtp, void* work, int mode) {
  const DevType& dt = *dtp;
  const int n = dt.p.n;
  PlainWork<T> w = plain_layout<T>(work, n, dt.p.m, dt.p.e);
  const int lane = threadIdx.x;
  if (lane < 3) band_solve_column<T, BW>(dt, w.r + lane * n, w.dir + lane * n);
  __threadfence_block();
  __syncthreads();
  if (mode == kSolveDirection) {
    for (int i = lane; i < 3 * n; i += 64) w.dir[i] = -w.dir[i];
  } else {
    for (int i = lane; i < 3 * n; i += 64) w.d[i] -= w.dir[i];
  }
}

template <typename T>
void launch_plain_solve(const DevType* dt_dev, const TypeParams& p, void* work, int mode,
                        hipStream_t s) {
  switch (p.band_w) {
#define NPFEM_CASE(W)                                                                            \
  case W:                                                                                        \
    hipLaunchKernelGGL((k_plain_solve_band<T, W>), dim3(1), dim3(64), 0, s, dt_dev, work, mode); \
    return;
    NPFEM_BAND_WINDOWS(NPFEM_CASE)
#undef NPFEM_CASE
    default:   // wider bands: the wave-reduction form
      hipLaunchKernelGGL(k_plain_solve<T>, dim3(1), dim3(192), 0, s, dt_dev, work, mode);
  }
}

// Skalak membrane: backtracking line search along dir from delta, one cell. g at step length
// a (positions x_n + delta + a dir): Skalak energies of the triangles, bending energies of the
// hinges (projections at that point), the volume energy (w_v/2)(V0 - V)^2/|grad V|^2, the
// inertia term (1 + h alpha)(m/2h^2)|delta + a dir - delta^0|^2 and the contact energies,
// all in FP64. The first a of 1, 1/2, ..., 2^-kMaxHalvings with
// g(a) <= g(0) + kArmijoC a grad g . dir is taken (the last one when none qualifies).
template <typename T>
__global__ void __launch_bounds__(kPlainThreads)
k_plain_linesearch(const DevType* __restrict__ dtp, const T* __restrict__ x, int64_t vt,
                   int64_t off, void* work, const T* __restrict__ cp, const T* __restrict__ cw) {
  const DevType& dt = *dtp;
  const TypeParams& p = dt.p;
  const int n = p.n, m = p.m, e = p.e;
  PlainWork<T> w = plain_layout<T>(work, n, m, e);
  const T* G = PlainConst<T>::G(dt);
  const T* A = PlainConst<T>::A(dt);
  const T* coef = PlainConst<T>::coef(dt);
  const T* rest = PlainConst<T>::rest(dt);
  __shared__ double sh[8];
  double sl = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    for (int c = 0; c < 3; ++c) sl += (double)w.r[c * n + i] * (double)w.dir[c * n + i];
  const double slope = block_sum(sl, sh);
  // positions x + a dir of the trial, cell-local, in FP64 from the stored values (exact up to
  // FP64 rounding: a is a power of two): near convergence a dir falls below the spacing of x
  // in FP32, and FP32 trial positions would equal x^k so that no halving could show the
  // decrease the test asks for
  auto pos = [&](int i, T a) {
    const double ad = (double)a;
    return v3<double>(((double)x[off + i] - (double)x[off]) + ((double)w.d[i] + ad * (double)w.dir[i]),
                      ((double)x[vt + off + i] - (double)x[vt + off]) +
                          ((double)w.d[n + i] + ad * (double)w.dir[n + i]),
                      ((double)x[2 * vt + off + i] - (double)x[2 * vt + off]) +
                          ((double)w.d[2 * n + i] + ad * (double)w.dir[2 * n + i]));
  };
  // g at step length a, every term in FP64
  auto energy = [&](T a) {
    const double ad = (double)a;
    double ee = 0;
    for (int t = threadIdx.x; t < m; t += blockDim.x)
      ee += skalak_energy<double>(pos(dt.tri[3 * t], a), pos(dt.tri[3 * t + 1], a), pos(dt.tri[3 * t + 2], a),
                                  (double)G[6 * t + 2], (double)G[6 * t + 3], (double)G[6 * t + 4],
                                  (double)G[6 * t + 5], (double)A[t], p.w_s, p.w_a);
    for (int h = threadIdx.x; h < e; h += blockDim.x) {
      const int* hv = dt.hinge + 4 * h;
      ee += hinge_energy<double>(pos(hv[0], a), pos(hv[1], a), pos(hv[2], a), pos(hv[3], a),
                                 (double)coef[4 * h + 1], (double)coef[4 * h + 2], (double)coef[4 * h + 3],
                                 (double)rest[h], p.w_b);
    }
    double vp = 0, gp = 0, em = 0, ec = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      // grad_i V = 1/6 sum of the doubled area vectors of the triangles around i
      Vec3<double> g = v3<double>(0.0, 0.0, 0.0);
      for (int s = dt.vt_off[i]; s < dt.vt_off[i + 1]; ++s) {
        const int t = dt.vt_list[s] / 3;
        const Vec3<double> pa = pos(dt.tri[3 * t], a), pb = pos(dt.tri[3 * t + 1], a);
        const Vec3<double> pc = pos(dt.tri[3 * t + 2], a);
        g = g + cross3(pb - pa, pc - pa);
      }
      g = g * (1.0 / 6.0);
      const Vec3<double> pi = pos(i, a);
      vp += dot3(pi, g);
      gp += dot3(g, g);
      const T wc = cw != nullptr ? cw[off + i] : T(0);
      for (int c = 0; c < 3; ++c) {
        const double dd = (double)w.d[c * n + i] + ad * (double)w.dir[c * n + i];
        const double dl = dd - (double)w.d0[c * n + i];
        em += dl * dl;
        if (wc != T(0)) {
          const double gd = ((double)x[c * vt + off + i] - (double)cp[c * vt + off + i]) + dd;
          ec += 0.5 * (double)wc * gd * gd;
        }
      }
    }
    const double E_el = block_sum(ee, sh);
    const double V = block_sum(vp, sh) / 3.0, G2 = block_sum(gp, sh);
    const double E_m = 0.5 * p.inv_h2m * block_sum(em, sh);
    const double E_c = block_sum(ec, sh);
    const double E_v = G2 > 0 ? 0.5 * p.w_v * (p.V0 - V) * (p.V0 - V) / G2 : 0.0;
    return E_el + E_m + E_v + E_c;
  };
  const double e0 = energy(T(0));
  T a = T(1);
  for (int h = 0; h <= kMaxHalvings; ++h) {
    if (energy(a) <= e0 + kArmijoC * (double)a * slope || h == kMaxHalvings) break;
    a *= T(0.5);
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    for (int c = 0; c < 3; ++c) w.d[c * n + i] += a * w.dir[c * n + i];
}

// Class test (not v - v == 0, which FMA contraction can turn into a product's rounding error).
template <typename T>
__device__ inline bool finite_val(T v) { return __builtin_isfinite(v); }

template <typename T>
__global__ void __launch_bounds__(kPlainThreads)
k_plain_finalize(const DevType* __restrict__ dtp, T* __restrict__ x, T* __restrict__ v,
                 int64_t vt, int64_t off, void* work, double* vol_area, int* flag) {
  const DevType& dt = *dtp;
  const TypeParams& p = dt.p;
  const int n = p.n, m = p.m;
  PlainWork<T> w = plain_layout<T>(work, n, m, p.e);
  __shared__ double sh[8];
  if (vol_area) {
    double vs = 0, as = 0;
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
      const Vec3<T> pa = cell_pos(x, vt, off, w.d, n, dt.tri[3 * t]);
      const Vec3<T> pb = cell_pos(x, vt, off, w.d, n, dt.tri[3 * t + 1]);
      const Vec3<T> pc = cell_pos(x, vt, off, w.d, n, dt.tri[3 * t + 2]);
      const Vec3<T> nt = cross3(pb - pa, pc - pa);
      vs += (double)pa.x * nt.x + (double)pa.y * nt.y + (double)pa.z * nt.z;
      as += sqrt((double)nt.x * nt.x + (double)nt.y * nt.y + (double)nt.z * nt.z);
    }
    const double V = block_sum(vs, sh) / 6.0;
    const double S = block_sum(as, sh) * 0.5;
    if (threadIdx.x == 0) {
      vol_area[0] = V;
      vol_area[1] = S;
    }
  }
  __syncthreads();
  const T ih = T(1) / T(p.h), v_max = T(p.v_max);
  bool bad = false;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    T vn[3];
    for (int c = 0; c < 3; ++c) {
      const T d = w.d[c * n + i];
      const T xn = x[c * vt + off + i] + d;
      vn[c] = d * ih;
      x[c * vt + off + i] = xn;
      bad |= !finite_val(xn);
    }
    cap_speed(vn[0], vn[1], vn[2], v_max);
    for (int c = 0; c < 3; ++c) {
      v[c * vt + off + i] = vn[c];
      bad |= !finite_val(vn[c]);
    }
  }
  if (bad) atomicOr(flag, 1);
}

template <typename T>
hipError_t plain_step_t(const DevType* dt_dev, const TypeParams& p, T* x, T* v, const T* f,
                        const T* cp, const T* cw, int64_t vt, int64_t off, int K, void* work,
                        double* vol_area, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_plain_predict<T>, dim3(1), dim3(kPlainThreads), 0, s, p, x, v, f, vt,
                     off, work);
  if (p.ray_k > 0.0)
    hipLaunchKernelGGL(k_plain_solve<T>, dim3(1), dim3(192), 0, s, dt_dev, work, (int)kSolvePredict);
  for (int k = 0; k < K; ++k) {
    hipLaunchKernelGGL(k_plain_local<T>, dim3(1), dim3(kPlainThreads), 0, s, dt_dev, x, vt, off,
                       work, cp, cw);
    if (p.skalak) {
      launch_plain_solve<T>(dt_dev, p, work, (int)kSolveDirection, s);
      hipLaunchKernelGGL(k_plain_linesearch<T>, dim3(1), dim3(kPlainThreads), 0, s, dt_dev, x, vt,
                         off, work, cp, cw);
    } else {
      launch_plain_solve<T>(dt_dev, p, work, (int)kSolveUpdate, s);
    }
  }
  hipLaunchKernelGGL(k_plain_finalize<T>, dim3(1), dim3(kPlainThreads), 0, s, dt_dev, x, v, vt,
                     off, work, vol_area, flag);
  return hipGetLastError();
}

}  // namespace

size_t plain_work_bytes(int precision, int n, int m, int e) {
  const size_t el = precision == 64 ? 8 : 4;
  return el * (15 * (size_t)n + 12 * (size_t)m + 12 * (size_t)e) + 256;
}

bool plain_supported(int n, int bw) { return n <= kMaxBand && bw < kMaxBand; }

hipError_t launch_plain_cell(int precision, const DevType* dt_dev, const TypeParams& p, void* x,
                             void* v, const void* f, const void* cp, const void* cw, int64_t vtot,
                             int64_t off, int K, void* work, double* vol_area, int* flag,
                             void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (precision == 64)
    return plain_step_t<double>(dt_dev, p, (double*)x, (double*)v, (const double*)f,
                                (const double*)cp, (const double*)cw, vtot, off, K, work, vol_area,
                                flag, s);
  return plain_step_t<float>(dt_dev, p, (float*)x, (float*)v, (const float*)f, (const float*)cp,
                             (const float*)cw, vtot, off, K, work, vol_area, flag, s);
}

}  // namespace npfem
