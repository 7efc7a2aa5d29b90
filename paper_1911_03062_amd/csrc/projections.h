// Device-side local step of the npFEM iteration: per-triangle strain/area and per-hinge
// bending residuals of the projective-dynamics constraint energies, templated on precision.
//
// Triangle (constraint energies A_t w/2 ||F - p||^2, F = sum_j x_j g_j^T, 3x2):
//   C = F^T F, s = |F0 x F1| = s1 s2, t = sqrt(tr C + 2 s) = s1 + s2,
//   disc = sqrt((c00 - c11)^2 + 4 c01^2) = s1^2 - s2^2,
//   polar factor R = F (F^T F)^(-1/2) = F [[c11 + s, -c01], [-c01, c00 + s]] / (s t),
//   stretch S = R^T F = (C + s I)/t with eigen-frame Q = [[cos 2a, sin 2a], [sin 2a, -cos 2a]]
//   (cos 2a, sin 2a) = (c00 - c11, 2 c01)/disc.
// Any symmetric 2x2 V diag(p, q) V^T in that frame equals (p+q)/2 I + (p-q)/2 Q, so the
// residual of both projections (strain: singular values clamped to [s_min, s_max]; area:
// (d, 1/d) nearest to (s1, s2)) is  F - p = R (alpha I + beta Q)  and the contribution to
// vertex j is  A_t R (w_s (S - S_s) + w_a (S - S_a)) g_j.  All "singular value minus target"
// differences are formed from a = s1 - 1, b = s2 - 1 and eps = d - 1 so that near the rest
// state no difference of two numbers close to one is taken twice.
//
// Area root: d minimises (d - s1)^2 + (1/d - s2)^2, i.e. solves d^4 - s1 d^3 + s2 d - 1 = 0;
// with d = 1 + eps, a = s1 - 1, b = s2 - 1 the quartic reads
//   (b - a) + eps (2 - 3a + b) + eps^2 (3 - 3a) + eps^3 (3 - a) + eps^4 = 0,
// solved by bracketed Newton for its largest root, started by one Halley step from
// sqrt(s1/s2) - 1 (which is exact when s1 = s2 <= 2).
#pragma once

#include <hip/hip_runtime.h>

namespace npfem {

template <typename T>
struct Vec3 {
  T x, y, z;
};

template <typename T>
__host__ __device__ __forceinline__ Vec3<T> v3(T x, T y, T z) { return {x, y, z}; }
template <typename T>
__host__ __device__ __forceinline__ Vec3<T> operator-(Vec3<T> a, Vec3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
__host__ __device__ __forceinline__ Vec3<T> operator+(Vec3<T> a, Vec3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T>
__host__ __device__ __forceinline__ Vec3<T> operator*(Vec3<T> a, T s) { return {a.x * s, a.y * s, a.z * s}; }
template <typename T>
__host__ __device__ __forceinline__ T dot3(Vec3<T> a, Vec3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__host__ __device__ __forceinline__ Vec3<T> cross3(Vec3<T> a, Vec3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// FP32 uses the hardware square root and reciprocal (v_sqrt_f32, v_rcp_f32, about 1 ulp)
// instead of the correctly rounded expansions; FP64 keeps IEEE sqrt and division. The host
// versions exist so that the same element math can be checked on the CPU.
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ float dsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ float drcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ float drsqrt(float v) { return __builtin_amdgcn_rsqf(v); }
#else
inline float dsqrt(float v) { return __builtin_sqrtf(v); }
inline float drcp(float v) { return 1.0f / v; }
inline float drsqrt(float v) { return 1.0f / __builtin_sqrtf(v); }
#endif
__host__ __device__ __forceinline__ double dsqrt(double v) { return __builtin_sqrt(v); }
__host__ __device__ __forceinline__ double drcp(double v) { return 1.0 / v; }
__host__ __device__ __forceinline__ double drsqrt(double v) { return 1.0 / __builtin_sqrt(v); }

template <typename T>
__host__ __device__ __forceinline__ T kRootTol();
template <>
__host__ __device__ __forceinline__ float kRootTol<float>() { return 2e-7f; }
template <>
__host__ __device__ __forceinline__ double kRootTol<double>() { return 4e-16; }

// F is taken as rank-deficient when s1 s2 <= this times s1^2 + s2^2 (about s2/s1): below it
// the computed s2 is dominated by the rounding of det C (noise near sqrt(eps) s1), so F S^-1
// would follow that noise, and s2 = 0 is the nearer value.
template <typename T>
__host__ __device__ __forceinline__ T kRankTol();
template <>
__host__ __device__ __forceinline__ float kRankTol<float>() { return 1e-3f; }
template <>
__host__ __device__ __forceinline__ double kRankTol<double>() { return 1e-7; }

// The area root's Halley start is kept without the safeguarded iteration when its step is at
// most this times (1 + eps) and both singular values lie within 0.3 of one: there the error
// after the step falls as the cube of the step (relative error below 1.3e-9 for steps up to
// 1e-3, measured against a bisected FP64 root over that square of singular values), well
// under the FP32 iteration's tolerance. Negative: never (FP64 keeps the iteration).
template <typename T>
__host__ __device__ __forceinline__ T kHalleyAccept();
template <>
__host__ __device__ __forceinline__ float kHalleyAccept<float>() { return 1e-3f; }
template <>
__host__ __device__ __forceinline__ double kHalleyAccept<double>() { return -1.0; }

template <typename T>
__host__ __device__ __forceinline__ T clamp_dev(T v, T lo, T hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Triangle residual contributions. Inputs: vertex positions pa, pb, pc (any common origin),
// rest gradients gb, gc (g_a = -g_b - g_c), rest area, weights. Outputs: contributions to
// the gradient of g at vertices a, b, c, added to ra, rb, rc.
//
// The polar factor is not formed: R = P A with P = F, A = adj(C + s I) / (s t) in the regular
// case (P = an orthonormal frame, A = I when F is rank deficient), so that the contribution
// to vertex j is A_t P (A T g_j) with the 2x2 matrix T = alpha I + beta Q.
template <typename T>
__host__ __device__ __forceinline__ void triangle_residual(Vec3<T> pa, Vec3<T> pb, Vec3<T> pc, T gb0,
                                                  T gb1, T gc0, T gc1, T area, T w_s, T w_a,
                                                  T s_min, T s_max, Vec3<T>& ra, Vec3<T>& rb,
                                                  Vec3<T>& rc) {
  const Vec3<T> e1 = pb - pa, e2 = pc - pa;
  // the rest frames in use make D_m upper triangular (g_c0 = 0); a literal zero here lets the
  // compiler drop those terms, which it may not do for x * 0 in general (NaN, signed zero)
  const bool lower0 = gc0 == T(0);
  const Vec3<T> F0 = lower0 ? e1 * gb0 : e1 * gb0 + e2 * gc0;
  const Vec3<T> F1 = e1 * gb1 + e2 * gc1;
  const T c00 = dot3(F0, F0), c01 = dot3(F0, F1), c11 = dot3(F1, F1);
  const T det2 = c00 * c11 - c01 * c01;            // |F0 x F1|^2 (Lagrange identity)
  const T s = dsqrt(det2 > T(0) ? det2 : T(0));    // s1 s2
  const T tr = c00 + c11;
  const T tt = dsqrt(tr + T(2) * s);               // s1 + s2
  const T dl = c00 - c11, of = T(2) * c01;
  const T disc = dsqrt(dl * dl + of * of);         // s1^2 - s2^2
  Vec3<T> P0, P1;
  T A00, A01, A11, a, b, rs;
  if (s > kRankTol<T>() * tr) {
    const T inv = drcp(s * tt);                    // 1 / (s t)
    P0 = F0;
    P1 = F1;
    A00 = (c11 + s) * inv;
    A01 = -c01 * inv;
    A11 = (c00 + s) * inv;
    const T half_diff = T(0.5) * disc * (inv * s);  // (s1 - s2)/2
    // (s1 + s2) - 2 = ((c00 - 1) + (c11 - 1) + 2 (s - 1)) / (s1 + s2 + 2); each bracket is
    // an exact subtraction for entries within a factor two of one
    const T tm2 = ((c00 - T(1)) + (c11 - T(1)) + T(2) * (s - T(1))) * drcp(tt + T(2));
    a = T(0.5) * tm2 + half_diff;
    b = T(0.5) * tm2 - half_diff;
    rs = drsqrt(s);                                // sqrt(s1 / s2) = s1 / sqrt(s)
  } else {
    // rank-deficient F = s1 u1 v1^T: the polar factor R = u1 v1^T + u2 v2^T with v1 the unit
    // eigenvector of C for its larger eigenvalue, u1 = F v1 / |F v1| and u2 any unit vector
    // orthogonal to u1 (the SVD's free completion); P holds R's columns R e1, R e2, and
    // F = 0 takes v1 = e1, u1 = e_x
    T ch = T(1), sh = T(0);   // v1 = (cos, sin) of half the angle of (dl, of)
    if (disc > T(0)) {
      const T qc = dl * drcp(disc);
      ch = dsqrt(clamp_dev(T(0.5) * (T(1) + qc), T(0), T(1)));
      sh = dsqrt(clamp_dev(T(0.5) * (T(1) - qc), T(0), T(1)));
      if (of < T(0)) sh = -sh;
    }
    Vec3<T> u1 = F0 * ch + F1 * sh;
    const T n1 = dsqrt(dot3(u1, u1));
    u1 = n1 > T(0) ? u1 * drcp(n1) : v3<T>(1, 0, 0);
    const Vec3<T> ax = (u1.x * u1.x < T(0.5)) ? v3<T>(1, 0, 0) : v3<T>(0, 1, 0);
    const Vec3<T> w = ax - u1 * dot3(u1, ax);
    const Vec3<T> u2 = w * drsqrt(dot3(w, w));
    P0 = u1 * ch - u2 * sh;   // v2 = (-sin, cos)
    P1 = u1 * sh + u2 * ch;
    A00 = T(1);
    A01 = T(0);
    A11 = T(1);
    a = dsqrt(tr) - T(1);
    b = T(-1);
    rs = T(0);
  }
  T q_c, q_s;
  if (disc > T(0)) {
    const T id = drcp(disc);
    q_c = dl * id;
    q_s = of * id;
  } else {
    q_c = T(1);
    q_s = T(0);
  }
  // strain: s - clamp(s) per singular value (the polar factor when s_min = s_max = 1; the
  // bounds are the same for all lanes, so this is a uniform branch)
  T ds1, ds2;
  if (s_min == T(1) && s_max == T(1)) {
    ds1 = a;
    ds2 = b;
  } else {
    ds1 = (a > s_max - T(1) ? a - (s_max - T(1)) : T(0)) + (a < s_min - T(1) ? a - (s_min - T(1)) : T(0));
    ds2 = (b > s_max - T(1) ? b - (s_max - T(1)) : T(0)) + (b < s_min - T(1) ? b - (s_min - T(1)) : T(0));
  }
  // area: eps = d - 1, the largest root of the shifted quartic. For s1 >= s2 exactly one
  // root has d >= 1 and it is the nearest area-preserving stretch; it lies in
  // [0, max(s1, 1)] in eps, where the quartic is <= 0 at the bottom and > 0 at the top.
  // Start: one Halley step from sqrt(s1/s2) - 1; then Newton, falling back to bisection
  // whenever a step leaves the bracket.
  const T s1 = T(1) + a;
  const T k0 = b - a, k1 = T(2) - T(3) * a + b, k2 = T(3) - T(3) * a, k3 = T(3) - a;
  T lo = T(0), hi = T(1) + (a > T(0) ? a : T(0));
  T eps = T(0.5) * hi;
  bool settled = false;
  if (rs > T(0)) {
    const T e0 = s1 * rs - T(1);
    const T f0 = k0 + e0 * (k1 + e0 * (k2 + e0 * (k3 + e0)));
    const T f1 = k1 + e0 * (T(2) * k2 + e0 * (T(3) * k3 + T(4) * e0));
    const T f2 = T(2) * k2 + e0 * (T(6) * k3 + T(12) * e0);
    const T den = T(2) * f1 * f1 - f0 * f2;
    eps = (den > T(0)) ? e0 - T(2) * f0 * f1 * drcp(den) : e0;
    const T st = eps - e0;
    settled = den > T(0) && (st < T(0) ? -st : st) <= kHalleyAccept<T>() * (T(1) + e0) &&
              a < T(0.3) && b > T(-0.3);   // b <= a: both within 0.3 of zero
  }
  settled = settled && eps >= lo && eps <= hi;
  eps = (eps >= lo && eps <= hi) ? eps : T(0.5) * (lo + hi);
  for (int it = 0; !settled && it < 40; ++it) {
    const T fv = k0 + eps * (k1 + eps * (k2 + eps * (k3 + eps)));
    const T fp = k1 + eps * (T(2) * k2 + eps * (T(3) * k3 + T(4) * eps));
    // an exact zero ends the iteration only where the quartic increases: for s1 = s2 > 2 the
    // start (eps = 0, t = 1) is a root where it decreases, a stationary point of the distance
    // that is not its minimiser, and the bisection goes on to the larger root
    if (fv == T(0) && fp > T(0)) break;
    if (fv > T(0)) hi = eps;
    else lo = eps;
    T nx = (fp > T(0)) ? eps - fv * drcp(fp) : T(-1);
    if (!(nx >= lo && nx <= hi)) nx = T(0.5) * (lo + hi);
    const T step = nx - eps;
    eps = nx;
    if ((step < T(0) ? -step : step) <= kRootTol<T>() * (T(1) + eps)) break;
  }
  const T ip = drcp(T(1) + eps);
  const T sum_a = (a + b) - eps * eps * ip;                    // (s1 + s2) - (d + 1/d)
  const T dif_a = (a - b) - eps * (T(2) + eps) * ip;           // (s1 - s2) - (d - 1/d)
  const T alpha = T(0.5) * area * (w_s * (ds1 + ds2) + w_a * sum_a);
  const T beta = T(0.5) * area * (w_s * (ds1 - ds2) + w_a * dif_a);
  // area T = area (alpha I + beta Q), K = A (area T) (A and T symmetric)
  const T t00 = alpha + beta * q_c, t01 = beta * q_s, t11 = alpha - beta * q_c;
  const T K00 = A00 * t00 + A01 * t01, K01 = A00 * t01 + A01 * t11;
  const T K10 = A01 * t00 + A11 * t01, K11 = A01 * t01 + A11 * t11;
  const T kb0 = K00 * gb0 + K01 * gb1, kb1 = K10 * gb0 + K11 * gb1;
  const T kc0 = lower0 ? K01 * gc1 : K00 * gc0 + K01 * gc1;
  const T kc1 = lower0 ? K11 * gc1 : K10 * gc0 + K11 * gc1;
  // contributions P k (b, c) and -(those two) (a, since g_a = -g_b - g_c), accumulated
  const T ka0 = -(kb0 + kc0), ka1 = -(kb1 + kc1);
  ra = ra + P0 * ka0 + P1 * ka1;
  rb = rb + P0 * kb0 + P1 * kb1;
  rc = rc + P0 * kc0 + P1 * kc1;
}

// Hinge residual: u = sum_q a_q x_q (written relative to x_i, since sum_q a_q = 0),
// p = r u/|u|, contribution w_b a_q (u - p) to vertex q (a_i = -(a_j + a_k + a_l)), added to
// ri, rj, rk, rl.
template <typename T>
__host__ __device__ __forceinline__ void hinge_residual(Vec3<T> pi, Vec3<T> pj, Vec3<T> pk, Vec3<T> pl,
                                               T a1, T a2, T a3, T rest, T w_b, Vec3<T>& ri,
                                               Vec3<T>& rj, Vec3<T>& rk, Vec3<T>& rl) {
  const Vec3<T> u = (pj - pi) * a1 + (pk - pi) * a2 + (pl - pi) * a3;
  const T nu2 = dot3(u, u);
  T fac = T(0);
  if (nu2 > T(0)) fac = w_b * (T(1) - rest * drsqrt(nu2));
  const Vec3<T> W = u * fac;
  const T a0 = -(a1 + a2 + a3);
  ri = ri + W * a0;
  rj = rj + W * a1;
  rk = rk + W * a2;
  rl = rl + W * a3;
}

// Bending energy of one hinge: (w_b/2) (|u| - r)^2, 0 for u = 0 (the projection is u then).
template <typename T>
__host__ __device__ __forceinline__ T hinge_energy(Vec3<T> pi, Vec3<T> pj, Vec3<T> pk, Vec3<T> pl,
                                                   T a1, T a2, T a3, T rest, T w_b) {
  const Vec3<T> u = (pj - pi) * a1 + (pk - pi) * a2 + (pl - pi) * a3;
  const T nu2 = dot3(u, u);
  if (!(nu2 > T(0))) return T(0);
  const T dd = dsqrt(nu2) - rest;
  return T(0.5) * w_b * dd * dd;
}

// Skalak membrane (Skalak et al. 1973) of one triangle: with F = [f0 f1] = sum_j x_j g_j^T,
// C = F^T F, I1 = tr C - 2, I2 = det C - 1, the energy A W with
// W = (B/4)(I1^2 + 2 I1 - 2 I2) + (C/4) I2^2 and the first Piola stress
// P = dW/dF = 2 F S, S = dW/dC = (B/2)(I1 + 1) 1 + (C I2 - B)/2 adj(C). Adds A P g_j to the
// vertex contributions (g_a = -g_b - g_c) and returns A W.
template <typename T>
__host__ __device__ __forceinline__ T skalak_residual(Vec3<T> pa, Vec3<T> pb, Vec3<T> pc, T gb0,
                                                      T gb1, T gc0, T gc1, T area, T B, T Cm,
                                                      Vec3<T>& ra, Vec3<T>& rb, Vec3<T>& rc) {
  const Vec3<T> e1 = pb - pa, e2 = pc - pa;
  const Vec3<T> f0 = e1 * gb0 + e2 * gc0, f1 = e1 * gb1 + e2 * gc1;
  const T c00 = dot3(f0, f0), c01 = dot3(f0, f1), c11 = dot3(f1, f1);
  const T I1 = (c00 - T(1)) + (c11 - T(1));
  const T I2 = c00 * c11 - c01 * c01 - T(1);
  const T W = T(0.25) * B * (I1 * I1 + T(2) * I1 - T(2) * I2) + T(0.25) * Cm * I2 * I2;
  const T sa = T(0.5) * B * (I1 + T(1)), sb = T(0.5) * (Cm * I2 - B);
  const T s00 = sa + sb * c11, s01 = -sb * c01, s11 = sa + sb * c00;
  const Vec3<T> p0 = (f0 * s00 + f1 * s01) * (T(2) * area);
  const Vec3<T> p1 = (f0 * s01 + f1 * s11) * (T(2) * area);
  const Vec3<T> kb = p0 * gb0 + p1 * gb1, kc = p0 * gc0 + p1 * gc1;
  rb = rb + kb;
  rc = rc + kc;
  ra = ra - kb - kc;
  return area * W;
}

// Skalak energy A W of one triangle alone (the value skalak_residual returns).
template <typename T>
__host__ __device__ __forceinline__ T skalak_energy(Vec3<T> pa, Vec3<T> pb, Vec3<T> pc, T gb0, T gb1,
                                                    T gc0, T gc1, T area, T B, T Cm) {
  const Vec3<T> e1 = pb - pa, e2 = pc - pa;
  const Vec3<T> f0 = e1 * gb0 + e2 * gc0, f1 = e1 * gb1 + e2 * gc1;
  const T c00 = dot3(f0, f0), c01 = dot3(f0, f1), c11 = dot3(f1, f1);
  const T I1 = (c00 - T(1)) + (c11 - T(1));
  const T I2 = c00 * c11 - c01 * c01 - T(1);
  const T W = T(0.25) * B * (I1 * I1 + T(2) * I1 - T(2) * I2) + T(0.25) * Cm * I2 * I2;
  return area * W;
}

// Position-based damping (Mueller et al. 2007): the angular velocity of a cell's rigid motion
// solves I w = L with the inertia tensor I = sum (|r|^2 1 - r r^T) and angular momentum
// L = sum r x v about the centre of mass (equal masses cancel). Isym = (xx, yy, zz, xy, xz, yz).
// Solved by the adjugate in FP64; a singular I (all vertices on a line) gives w = 0.
__host__ __device__ __forceinline__ void solve_sym3(const double Isym[6], const double Lm[3],
                                                    double w[3]) {
  const double a = Isym[0], b = Isym[1], c = Isym[2], d = Isym[3], e = Isym[4], f = Isym[5];
  // [[a, d, e], [d, b, f], [e, f, c]]
  const double c00 = b * c - f * f, c01 = e * f - d * c, c02 = d * f - b * e;
  const double c11 = a * c - e * e, c12 = d * e - a * f, c22 = a * b - d * d;
  const double det = a * c00 + d * c01 + e * c02;
  if (!(det > 0.0)) {
    w[0] = w[1] = w[2] = 0.0;
    return;
  }
  const double id = 1.0 / det;
  w[0] = (c00 * Lm[0] + c01 * Lm[1] + c02 * Lm[2]) * id;
  w[1] = (c01 * Lm[0] + c11 * Lm[1] + c12 * Lm[2]) * id;
  w[2] = (c02 * Lm[0] + c12 * Lm[1] + c22 * Lm[2]) * id;
}

// Damped velocity v + kappa (v_cm + w x r - v) of a vertex at r from the centre of mass.
template <typename T>
__host__ __device__ __forceinline__ Vec3<T> pbd_velocity(Vec3<T> v, Vec3<T> r, Vec3<T> vcm,
                                                         Vec3<T> w, T kappa) {
  const Vec3<T> rigid = vcm + cross3(w, r);
  return v + (rigid - v) * kappa;
}

}  // namespace npfem
