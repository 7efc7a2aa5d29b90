// Boundary filters of the fluid-structure coupling (Fluid-structure interaction subsection):
//   * the median filter of the external forces: every component of F_ext at a vertex is
//     replaced by the median of that component over the vertex and its one-ring neighbours
//     (the median of an even count is the mean of the two middle values);
//   * the velocity cap: a vertex velocity longer than v_max is scaled back to length v_max,
//     its direction kept (the truncation that keeps the immersed-boundary coupling stable).
// Host and device versions are the same code, so the CPU tests exercise what the kernels run.
#pragma once

#include <utility>

#include "projections.h"

namespace npfem {

// Batcher's odd-even merge sort for N (a power of two) keys as a list of compare-exchange
// pairs (lo[q], hi[q]); built at compile time and applied with constant indices, so a key
// array of a kernel stays in registers.
template <int N>
struct SortNet {
  int count = 0;
  unsigned char lo[N * N] = {};
  unsigned char hi[N * N] = {};
  constexpr SortNet() {
    for (int p = 1; p < N; p *= 2)
      for (int k = p; k >= 1; k /= 2)
        for (int j = k % p; j + k < N; j += 2 * k)
          for (int i = 0; i < k && i + j + k < N; ++i)
            if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) {
              lo[count] = (unsigned char)(i + j);
              hi[count] = (unsigned char)(i + j + k);
              ++count;
            }
  }
};

template <int N>
inline constexpr SortNet<N> kSortNet{};

__host__ __device__ __forceinline__ float kmin(float a, float b) { return __builtin_fminf(a, b); }
__host__ __device__ __forceinline__ float kmax(float a, float b) { return __builtin_fmaxf(a, b); }
__host__ __device__ __forceinline__ double kmin(double a, double b) { return __builtin_fmin(a, b); }
__host__ __device__ __forceinline__ double kmax(double a, double b) { return __builtin_fmax(a, b); }

template <int N, typename T, int... Q>
__host__ __device__ __forceinline__ void sort_net_apply(T (&a)[N], std::integer_sequence<int, Q...>) {
  ((void)([&] {
     constexpr int i = kSortNet<N>.lo[Q], j = kSortNet<N>.hi[Q];
     const T x = a[i], y = a[j];
     a[i] = kmin(x, y);
     a[j] = kmax(x, y);
   }()),
   ...);
}

// Sorts a[0..N) ascending (finite keys and +inf).
template <int N, typename T>
__host__ __device__ __forceinline__ void sort_keys(T (&a)[N]) {
  sort_net_apply<N>(a, std::make_integer_sequence<int, kSortNet<N>.count>{});
}

// The comparators of SortNet<N> that the two middle outputs (N/2 - 1, N/2) depend on, found
// by a backward pass from those outputs; a comparator whose min (max) output is not needed
// later keeps only its max (min).
template <int N>
struct MiddleNet {
  int count = 0;
  unsigned char lo[N * N] = {};
  unsigned char hi[N * N] = {};
  bool keep_min[N * N] = {};
  bool keep_max[N * N] = {};
  constexpr MiddleNet() {
    constexpr SortNet<N> full{};
    unsigned long long need = (1ull << (N / 2 - 1)) | (1ull << (N / 2));
    int m = 0;
    unsigned char rl[N * N] = {}, rh[N * N] = {};
    bool rmin[N * N] = {}, rmax[N * N] = {};
    for (int q = full.count - 1; q >= 0; --q) {
      const int i = full.lo[q], j = full.hi[q];
      const bool ni = (need >> i) & 1ull, nj = (need >> j) & 1ull;
      if (!ni && !nj) continue;
      rl[m] = (unsigned char)i;
      rh[m] = (unsigned char)j;
      rmin[m] = ni;
      rmax[m] = nj;
      ++m;
      need |= (1ull << i) | (1ull << j);
    }
    for (int q = 0; q < m; ++q) {
      lo[q] = rl[m - 1 - q];
      hi[q] = rh[m - 1 - q];
      keep_min[q] = rmin[m - 1 - q];
      keep_max[q] = rmax[m - 1 - q];
    }
    count = m;
  }
};

template <int N>
inline constexpr MiddleNet<N> kMiddleNet{};

template <int N, typename T, int... Q>
__host__ __device__ __forceinline__ void middle_net_apply(T (&a)[N], std::integer_sequence<int, Q...>) {
  ((void)([&] {
     constexpr int i = kMiddleNet<N>.lo[Q], j = kMiddleNet<N>.hi[Q];
     constexpr bool mn = kMiddleNet<N>.keep_min[Q], mx = kMiddleNet<N>.keep_max[Q];
     const T x = a[i], y = a[j];
     if (mn) a[i] = kmin(x, y);
     if (mx) a[j] = kmax(x, y);
   }()),
   ...);
}

// Median of the k members of a closed ring padded to N keys with floor((N - k) / 2) copies of
// -inf and the rest +inf: the padding puts the ring's middle at positions N/2 - 1 (odd k) or
// N/2 - 1 and N/2 (even k) of the sorted keys, so only the comparators feeding those two
// positions run. a is overwritten.
template <int N, typename T>
__host__ __device__ __forceinline__ T median_padded(T (&a)[N], int k) {
  middle_net_apply<N>(a, std::make_integer_sequence<int, kMiddleNet<N>.count>{});
  const T lo = a[N / 2 - 1], hi = a[N / 2];
  return (k & 1) ? lo : T(0.5) * (lo + hi);
}

// Median of the first k keys of a (1 <= k <= N); a[k..N) must hold +inf. Sorts a in place.
template <int N, typename T>
__host__ __device__ __forceinline__ T median_keys(T (&a)[N], int k) {
  sort_keys<N>(a);
  T lo = a[0], hi = a[0];
#pragma unroll
  for (int q = 1; q < N; ++q) {
    if (q == (k - 1) / 2) lo = a[q];
    if (q == k / 2) hi = a[q];
  }
  return (k & 1) ? hi : T(0.5) * (lo + hi);
}

// Median of k keys member(0..k) by rank selection, for rings too large for a network: the key
// at sorted position r is the member a with #{b < a} <= r < #{b <= a}. O(k^2) reads, exact,
// no per-lane key array.
template <typename T, typename Member>
__host__ __device__ __forceinline__ T median_rank(int k, Member member) {
  const int r_lo = (k - 1) / 2, r_hi = k / 2;
  T lo = T(0), hi = T(0);
  for (int i = 0; i < k; ++i) {
    const T a = member(i);
    int less = 0, leq = 0;
    for (int j = 0; j < k; ++j) {
      const T b = member(j);
      less += b < a;
      leq += b <= a;
    }
    if (less <= r_lo && r_lo < leq) lo = a;
    if (less <= r_hi && r_hi < leq) hi = a;
  }
  return (k & 1) ? hi : T(0.5) * (lo + hi);
}

// Velocity cap: (vx, vy, vz) scaled to length v_max when longer (v_max <= 0: no cap).
template <typename T>
__host__ __device__ __forceinline__ void cap_speed(T& vx, T& vy, T& vz, T v_max) {
  const T s2 = vx * vx + vy * vy + vz * vz;
  if (v_max > T(0) && s2 > v_max * v_max) {
    const T sc = v_max / dsqrt(s2);
    vx *= sc;
    vy *= sc;
    vz *= sc;
  }
}

}  // namespace npfem
