// Forward and back substitution of one right-hand side with a cell type's banded Cholesky
// factor L = C C^T (supplementary material, npFEM subsection: the constant, prefactored
// Hessian approximation shared by every cell of a type), one lane per column.
//
// The lane keeps the pending partial sums of the next BW rows in registers (a right-looking
// substitution): when y_i is known, row i + k (k = 1..BW) gains C[i+k][i] y_i. Unrolled over
// blocks of BW rows, the window's slots rotate by name, so no register moves. Every lane of a
// wave reads the same factor entries: from LDS (staged by the workgroup) or through the
// constant address space (scalar loads).
#pragma once

#include <hip/hip_runtime.h>

#include "npfem_internal.h"

namespace npfem {

template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

// The factor in the substitution's layouts, both padded with zeros to W = p.band_w entries off
// the diagonal: rows [n][W+1] holds C[i][i-k], cols [n][W+1] holds C[i+k][i] for k >= 1 and
// 1 / C[i][i] at k = 0.
template <typename T>
struct Band {
  static __device__ cptr<T> rows(const DevType& d);
  static __device__ cptr<T> cols(const DevType& d);
};
template <>
__device__ inline cptr<float> Band<float>::rows(const DevType& d) { return (cptr<float>)d.sband_rows32; }
template <>
__device__ inline cptr<double> Band<double>::rows(const DevType& d) { return (cptr<double>)d.sband_rows64; }
template <>
__device__ inline cptr<float> Band<float>::cols(const DevType& d) { return (cptr<float>)d.sband_cols32; }
template <>
__device__ inline cptr<double> Band<double>::cols(const DevType& d) { return (cptr<double>)d.sband_cols64; }

// Forward substitution C y = r for one column of n rows (out may be r), cols = the factor's
// column layout (through any pointer type: the constant address space, or LDS). Each block
// of BW right-hand sides is loaded ahead of the block's stores.
template <typename T, int BW, typename P>
__device__ __forceinline__ void band_forward(int n, P cols, const T* r, T* out) {
  constexpr int ld = BW + 1;
  T w[BW];
#pragma unroll
  for (int j = 0; j < BW; ++j) w[j] = T(0);
  for (int i0 = 0; i0 < n; i0 += BW) {
    T rb[BW];
#pragma unroll
    for (int j = 0; j < BW; ++j) rb[j] = i0 + j < n ? r[i0 + j] : T(0);
#pragma unroll
    for (int j = 0; j < BW; ++j) {
      const int i = i0 + j;
      if (i < n) {
        const P col = cols + (size_t)i * ld;
        const T y = (rb[j] - w[j]) * col[0];
        out[i] = y;
        w[j] = T(0);   // the slot now holds row i + BW
#pragma unroll
        for (int k = 1; k <= BW; ++k) w[(j + k) % BW] += col[k] * y;
      }
    }
  }
}

// Back substitution C^T x = y in place in out, rows = the factor's row layout, cols its
// column layout (for the reciprocal diagonal).
template <typename T, int BW, typename P>
__device__ __forceinline__ void band_backward(int n, P rows, P cols, T* out) {
  constexpr int ld = BW + 1;
  T w[BW];
#pragma unroll
  for (int j = 0; j < BW; ++j) w[j] = T(0);
  const int nb = (n + BW - 1) / BW * BW;   // rows nb - 1 ... 0 in blocks of BW
  for (int i0 = nb - 1; i0 >= 0; i0 -= BW) {
    T yb[BW];
#pragma unroll
    for (int j = 0; j < BW; ++j) yb[j] = i0 - j < n ? out[i0 - j] : T(0);
#pragma unroll
    for (int j = 0; j < BW; ++j) {
      const int i = i0 - j;
      if (i < n) {
        const P row = rows + (size_t)i * ld;
        const T x = (yb[j] - w[j]) * cols[(size_t)i * ld];
        out[i] = x;
        w[j] = T(0);
#pragma unroll
        for (int k = 1; k <= BW; ++k) w[(j + k) % BW] += row[k] * x;
      }
    }
  }
}

// out = L^-1 r for one column (out may be r); BW = the type's p.band_w; the factor through
// scalar loads.
template <typename T, int BW>
__device__ __forceinline__ void band_solve_column(const DevType& d, const T* r, T* out) {
  band_forward<T, BW>(d.p.n, Band<T>::cols(d), r, out);
  band_backward<T, BW>(d.p.n, Band<T>::rows(d), Band<T>::cols(d), out);
}

// Padded band widths the substitution is built for (8 k + 1, k = 1..8); p.band_w is one of
// them or 0.
#define NPFEM_BAND_WINDOWS(X) X(9) X(17) X(25) X(33) X(41) X(49) X(57) X(65)

}  // namespace npfem
