// Global step alone, sparse form: out = L^-1 r for every cell of one type by forward and back
// substitution with the type's banded Cholesky factor (the substitution of banded.h), one
// lane per right-hand side (cell, coordinate); all lanes of a launch share the type.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "banded.h"
#include "npfem_internal.h"

namespace npfem {

namespace {

constexpr int kGlobalThreads = 256;
constexpr size_t kBandLdsMax = 48 * 1024;   // stage the factor in LDS up to this size

// Lane t: coordinate t / n_cells, cell cells[t % n_cells] (consecutive lanes take consecutive
// cells of one coordinate). BW is the type's padded band width p.band_w. With LDS (the launch
// gives n (BW + 1) elements of dynamic LDS), the workgroup stages the factor's column layout
// for the forward pass, then its row layout for the back pass; without, the lanes read the
// factor by scalar loads.
template <typename T, int BW, bool LDS>
__global__ void __launch_bounds__(kGlobalThreads)
k_global_banded(const DevType* __restrict__ dtp, const int32_t* __restrict__ cells, int n_cells,
                const int64_t* __restrict__ offsets, int64_t vt, const T* r, T* out) {
  extern __shared__ __align__(16) unsigned char band_lds[];
  const DevType& d = *dtp;
  const int n = d.p.n;
  const int t = blockIdx.x * kGlobalThreads + threadIdx.x;
  const bool active = t < 3 * n_cells;
  int64_t base = 0;
  if (active) {
    const int coord = t / n_cells;
    base = (int64_t)coord * vt + offsets[cells[t - coord * n_cells]];
  }
  if (!LDS) {
    if (active) band_solve_column<T, BW>(d, r + base, out + base);
    return;
  }
  T* sb = reinterpret_cast<T*>(band_lds);
  const int len = n * (BW + 1);
  const T* gcols = (const T*)Band<T>::cols(d);
  const T* grows = (const T*)Band<T>::rows(d);
  for (int i = threadIdx.x; i < len; i += kGlobalThreads) sb[i] = gcols[i];
  __syncthreads();
  if (active) band_forward<T, BW>(n, (const T*)sb, r + base, out + base);
  __syncthreads();
  // the reciprocal diagonal of the column layout moves into the row layout's diagonal slot
  for (int i = threadIdx.x; i < len; i += kGlobalThreads)
    sb[i] = (i % (BW + 1)) == 0 ? gcols[i] : grows[i];
  __syncthreads();
  if (active) band_backward<T, BW>(n, (const T*)sb, (const T*)sb, out + base);
}

template <typename T>
hipError_t launch_t(int n, int band_w, const DevType* dt, const int32_t* cells, int n_cells,
                    const int64_t* offsets, int64_t vt, const T* r, T* out, hipStream_t s) {
  const dim3 grid((3 * n_cells + kGlobalThreads - 1) / kGlobalThreads);
  const size_t lds = (size_t)n * (band_w + 1) * sizeof(T);
  const bool use_lds = lds <= kBandLdsMax;
  switch (band_w) {
#define NPFEM_CASE(W)                                                                          \
  case W:                                                                                      \
    if (use_lds)                                                                               \
      hipLaunchKernelGGL((k_global_banded<T, W, true>), grid, dim3(kGlobalThreads), lds, s, dt, \
                         cells, n_cells, offsets, vt, r, out);                                 \
    else                                                                                       \
      hipLaunchKernelGGL((k_global_banded<T, W, false>), grid, dim3(kGlobalThreads), 0, s, dt, \
                         cells, n_cells, offsets, vt, r, out);                                 \
    return hipGetLastError();
    NPFEM_BAND_WINDOWS(NPFEM_CASE)
#undef NPFEM_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// Dense L^-1 of a type in the batch precision ([n][n], symmetric).
template <typename T>
__device__ inline const T* dense_linv(const DevType& d);
template <>
__device__ inline const float* dense_linv<float>(const DevType& d) { return d.linv32; }
template <>
__device__ inline const double* dense_linv<double>(const DevType& d) { return d.linv64; }

constexpr int kGemvCells = 4;                 // cells per workgroup
constexpr int kGemvCols = 3 * kGemvCells;     // right-hand sides per workgroup

// Global step alone, dense vector form: out = L^-1 r with the type's dense L^-1 (FP64-derived,
// in the batch precision) on the vector ALU, kGemvCells cells of one type per workgroup. The
// cells' kGemvCols right-hand sides are staged in LDS as [k][column] (every lane then reads the
// same words: broadcasts); thread t forms rows t, t + blockDim, ... as sums over k of
// L^-1[k][row] (= L^-1[row][k]) times the staged values, reading row k of L^-1 coalesced
// across the threads. out may be r: a workgroup stages its cells before it writes them.
template <typename T>
__global__ void __launch_bounds__(512)
k_global_gemv(const DevType* __restrict__ dtp, const int32_t* __restrict__ cells, int n_cells,
              const int64_t* __restrict__ offsets, int64_t vt, const T* r, T* out) {
  extern __shared__ __align__(16) unsigned char gemv_lds[];
  T* rs = reinterpret_cast<T*>(gemv_lds);
  __shared__ int64_t offs[kGemvCells];
  const DevType& d = *dtp;
  const int n = d.p.n;
  const T* Li = dense_linv<T>(d);
  const int c0 = blockIdx.x * kGemvCells;
  const int nc = min(kGemvCells, n_cells - c0);
  if (threadIdx.x < kGemvCells) offs[threadIdx.x] = (int)threadIdx.x < nc ? offsets[cells[c0 + threadIdx.x]] : 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n * kGemvCols; i += blockDim.x) {
    const int k = i / kGemvCols, col = i - k * kGemvCols, cell = col / 3, c = col - 3 * cell;
    rs[i] = cell < nc ? r[c * vt + offs[cell] + k] : T(0);
  }
  __syncthreads();
  for (int row = threadIdx.x; row < n; row += blockDim.x) {
    T acc[kGemvCols];
#pragma unroll
    for (int j = 0; j < kGemvCols; ++j) acc[j] = T(0);
#pragma unroll 4
    for (int k = 0; k < n; ++k) {
      const T a = Li[(size_t)k * n + row];
      const T* rk = rs + k * kGemvCols;
#pragma unroll
      for (int j = 0; j < kGemvCols; ++j) acc[j] += a * rk[j];
    }
#pragma unroll
    for (int j = 0; j < kGemvCols; ++j) {
      const int cell = j / 3, c = j - 3 * cell;
      if (cell < nc) out[c * vt + offs[cell] + row] = acc[j];
    }
  }
}

template <typename T>
hipError_t launch_gemv_t(int n, const DevType* dt, const int32_t* cells, int n_cells, const int64_t* offsets,
                         int64_t vt, const T* r, T* out, hipStream_t s) {
  // one thread per row up to 512 rows (whole waves), then rows loop
  const int threads = std::min(512, (n + 63) / 64 * 64);
  const dim3 grid((n_cells + kGemvCells - 1) / kGemvCells);
  const size_t lds = (size_t)n * kGemvCols * sizeof(T);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_global_gemv<T>, grid, dim3(threads), lds, s, dt, cells, n_cells, offsets, vt, r, out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_global_gemv(int precision, int n, const DevType* dt, const int32_t* cells, int n_cells,
                              const int64_t* offsets, int64_t vt, const void* r, void* out, void* stream) {
  if (n_cells == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (precision == 64)
    return launch_gemv_t<double>(n, dt, cells, n_cells, offsets, vt, static_cast<const double*>(r),
                                 static_cast<double*>(out), s);
  return launch_gemv_t<float>(n, dt, cells, n_cells, offsets, vt, static_cast<const float*>(r),
                              static_cast<float*>(out), s);
}

hipError_t launch_global_banded(int precision, int n, int band_w, const DevType* dt, const int32_t* cells,
                                int n_cells, const int64_t* offsets, int64_t vt, const void* r,
                                void* out, void* stream) {
  if (n_cells == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (precision == 64)
    return launch_t<double>(n, band_w, dt, cells, n_cells, offsets, vt, static_cast<const double*>(r),
                            static_cast<double*>(out), s);
  return launch_t<float>(n, band_w, dt, cells, n_cells, offsets, vt, static_cast<const float*>(r),
                         static_cast<float*>(out), s);
}

}  // namespace npfem
