// Median filter of the external forces over each vertex's one ring (Fluid-structure
// interaction subsection), for all cells of a batch.
//
// One workgroup per block of consecutive cells (whole cells only, at most kFilterMaxCells
// cells and, unless one cell is larger, kFilterMaxVerts vertices). The block's force columns
// are staged in LDS with coalesced loads; every neighbour of a vertex belongs to the same cell
// and so to the same block, which makes the filter safe in place (each block reads its whole
// range before it writes any of it). Per vertex the closed ring (vertex plus its neighbours) of
// each component goes through a sorting network in registers when it has at most N members
// (padded with +inf); the few wider rings are collected and done by rank selection in a second
// pass, so that one pole of high degree does not slow down a whole wave of ordinary vertices.
// Bytes per vertex: 3 components read + 3 written.
#include <hip/hip_runtime.h>

#include "filters.h"
#include "npfem_internal.h"

namespace npfem {
namespace {

template <typename T, int N>
__global__ void __launch_bounds__(kFilterThreads)
k_median_filter(const DevType* __restrict__ types, const int32_t* __restrict__ type_of,
                const int64_t* __restrict__ offsets, const FilterBlock* __restrict__ blocks,
                int64_t vt, const T* f, T* out) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int cell_start[kFilterMaxCells + 1];
  __shared__ const uint32_t* c_info[kFilterMaxCells];
  __shared__ const uint32_t* c_pairs[kFilterMaxCells];
  __shared__ int n_wide;
  const FilterBlock blk = blocks[blockIdx.x];
  const int64_t v0 = offsets[blk.cell0];
  const int tid = threadIdx.x;
  if (tid <= blk.count) cell_start[tid] = (int)(offsets[blk.cell0 + tid] - v0);
  if (tid < blk.count) {
    const DevType& d = types[type_of[blk.cell0 + tid]];
    c_info[tid] = d.ring_info;
    c_pairs[tid] = d.ring_pairs;
  }
  if (tid == 0) n_wide = 0;
  __syncthreads();
  const int nv = cell_start[blk.count];
  T* s = reinterpret_cast<T*>(smem);                    // [3][nv] staged forces
  int* wide = reinterpret_cast<int*>(s + 3 * nv);       // [nv] vertices left to pass 2
  for (int c = 0; c < 3; ++c)
    for (int u = tid; u < nv; u += kFilterThreads) s[c * nv + u] = f[c * vt + v0 + u];
  __syncthreads();
  // pass 1: closed rings of at most N members through the sorting network in registers; wider
  // rings (the poles of a latitude-longitude sphere, say) are listed for pass 2
  for (int u = tid; u < nv; u += kFilterThreads) {
    int cc = 0;
    while (u >= cell_start[cc + 1]) ++cc;   // u < nv = cell_start[count]: ends at cc < count
    const int base = cell_start[cc];
    const uint32_t info = c_info[cc][u - base];
    const int deg = (int)(info & 255u);
    if (deg + 1 > N) {
      wide[atomicAdd(&n_wide, 1)] = u;
      continue;
    }
    const uint32_t* pr = c_pairs[cc] + (info >> 8);
    // neighbour q is the second vertex of the q-th triangle of the ring (every neighbour of a
    // vertex of a closed, consistently oriented mesh is that once); missing slots point at u
    int nb[N - 1];
#pragma unroll
    for (int q = 0; q < N - 1; ++q) nb[q] = q < deg ? base + (int)(pr[q] & 0xffffu) : u;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T* sc = s + c * nv;
      T a[N];
      a[0] = sc[u];
#pragma unroll
      for (int q = 0; q < N - 1; ++q) {
        const T w = sc[nb[q]];
        a[q + 1] = q < deg ? w : T(__builtin_inf());
      }
      out[c * vt + v0 + u] = median_keys<N>(a, deg + 1);
    }
  }
  __syncthreads();
  // pass 2: the listed wide rings by rank selection over the staged values
  const int nw = n_wide;
  for (int l = tid; l < nw; l += kFilterThreads) {
    const int u = wide[l];
    int cc = 0;
    while (u >= cell_start[cc + 1]) ++cc;
    const int base = cell_start[cc];
    const uint32_t info = c_info[cc][u - base];
    const int deg = (int)(info & 255u);
    const uint32_t* pr = c_pairs[cc] + (info >> 8);
    for (int c = 0; c < 3; ++c) {
      const T* sc = s + c * nv;
      out[c * vt + v0 + u] = median_rank<T>(deg + 1, [&](int i) {
        return i == 0 ? sc[u] : sc[base + (int)(pr[i - 1] & 0xffffu)];
      });
    }
  }
}

template <typename T, int N>
hipError_t launch_t(const DevType* types, const int32_t* type_of, const int64_t* offsets,
                    const FilterBlock* blocks, int n_blocks, int64_t vt, const void* f, void* out,
                    size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL((k_median_filter<T, N>), dim3(n_blocks), dim3(kFilterThreads), lds_bytes, s,
                     types, type_of, offsets, blocks, vt, static_cast<const T*>(f),
                     static_cast<T*>(out));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_median_filter(int precision, int net_keys, const DevType* types,
                                const int32_t* type_of, const int64_t* offsets,
                                const FilterBlock* blocks, int n_blocks, int64_t vt,
                                const void* f, void* out, size_t lds_bytes, void* stream) {
  if (n_blocks == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (precision == 64)
    return net_keys == 8 ? launch_t<double, 8>(types, type_of, offsets, blocks, n_blocks, vt, f,
                                               out, lds_bytes, s)
                         : launch_t<double, 16>(types, type_of, offsets, blocks, n_blocks, vt, f,
                                                out, lds_bytes, s);
  return net_keys == 8 ? launch_t<float, 8>(types, type_of, offsets, blocks, n_blocks, vt, f, out,
                                            lds_bytes, s)
                       : launch_t<float, 16>(types, type_of, offsets, blocks, n_blocks, vt, f, out,
                                             lds_bytes, s);
}

}  // namespace npfem
