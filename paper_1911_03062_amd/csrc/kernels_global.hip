// Global step alone, sparse form: out = L^-1 r for every cell of one type by forward and back
// substitution with the type's banded Cholesky factor (the substitution of banded.h), one
// lane per right-hand side (cell, coordinate); all lanes of a launch share the type.
#include <hip/hip_runtime.h>

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

}  // namespace

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
