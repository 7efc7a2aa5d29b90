// Median filter of the external forces over each vertex's one ring (Fluid-structure
// interaction subsection), for all cells of a batch.
//
// One workgroup per block of consecutive cells (whole cells only, at most kFilterMaxCells
// cells and, unless one cell is larger, kFilterMaxVerts vertices), described by a header the
// host prepared. The block's forces are staged in LDS as one 4-value record per vertex
// (x, y, z, unused), each cell's records behind two pad records (-inf, +inf), so that one
// 16-byte LDS read fetches a neighbour's three components and every slot of the neighbour
// table (pad code or neighbour + 2) is a plain offset from the cell's first record. Every neighbour of a vertex belongs to the same cell and so
// to the same block, which makes the filter safe in place (each block reads its whole range
// before it writes any of it).
//
// Pass 1: closed rings of at most N members, padded evenly with -inf and +inf to N keys by
// the type's neighbour table, through the comparators of a sorting network that the two
// middle keys depend on. Pass 2: the few wider rings (the poles of a latitude-longitude
// sphere, say), one lane per vertex and component, through a kFilterWideKeys-key network, or
// rank selection beyond that. Bytes per vertex: 3 components read + 3 written.
#include <hip/hip_runtime.h>

#include "filters.h"
#include "npfem_internal.h"

namespace npfem {
namespace {

// Global-memory view of a pointer that went through LDS (and so lost its address space):
// global loads count only against vmcnt, flat loads also against the LDS counter.
template <typename P>
__device__ __forceinline__ const __attribute__((address_space(1))) P* as_global(const P* p) {
  return (const __attribute__((address_space(1))) P*)p;
}

// Neighbour-table row of a vertex: N / 2 dwords of 16-bit slots (N = 8: one 16-byte load).
template <int N>
__device__ __forceinline__ void load_row(const uint16_t* row, uint32_t (&w)[N / 2]) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const __attribute__((address_space(1))) u32x4* p = as_global(reinterpret_cast<const u32x4*>(row));
#pragma unroll
  for (int h = 0; h < N / 8; ++h) {
    const u32x4 v = p[h];
    w[4 * h] = v.x;
    w[4 * h + 1] = v.y;
    w[4 * h + 2] = v.z;
    w[4 * h + 3] = v.w;
  }
}

template <int N>
__device__ __forceinline__ int slot(const uint32_t (&w)[N / 2], int q) {
  return (int)((w[q >> 1] >> (16 * (q & 1))) & 0xffffu);
}

template <typename T>
struct alignas(4 * sizeof(T)) Rec {
  T x, y, z, w;
};

// Vertices per thread per chunk: every load of a chunk is issued before the first wait.
constexpr int kFilterIt = kFilterMaxVerts / kFilterThreads;
constexpr int kHeaderWords = (int)(sizeof(FilterBlock) / 4);
static_assert(kHeaderWords <= kFilterThreads, "one header word per lane");

// Cell of block-local vertex u: the largest c < count with start[c] <= u (branch-free binary
// search over the header in LDS).
__device__ __forceinline__ int cell_of(const int* start, int count, int u) {
  int c = 0;
#pragma unroll
  for (int step = kFilterMaxCells / 2; step >= 1; step >>= 1)
    if (c + step < count && start[c + step] <= u) c += step;
  return c;
}

template <typename T, int N>
__global__ void __launch_bounds__(kFilterThreads)
k_median_filter(const DevType* __restrict__ types, const FilterBlock* __restrict__ blocks,
                int64_t vt, const T* f, T* out) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ union {
    FilterBlock b;
    uint32_t w[kHeaderWords];
  } hdr;
  __shared__ const uint32_t* c_info[kFilterMaxCells];
  __shared__ const uint32_t* c_pairs[kFilterMaxCells];
  __shared__ int n_wide;
  const int tid = threadIdx.x;
  if (tid < kHeaderWords)
    hdr.w[tid] = as_global(reinterpret_cast<const uint32_t*>(blocks + blockIdx.x))[tid];
  if (tid == 0) n_wide = 0;
  __syncthreads();
  const int64_t v0 = hdr.b.v0;
  const int nv = hdr.b.nv;                              // >= 4: a block holds whole cells
  const int count = hdr.b.count;
  const int* cell_start = hdr.b.start;
  if (tid < count) {
    const DevType& d = types[hdr.b.type[tid]];
    c_info[tid] = d.ring_info;
    c_pairs[tid] = d.ring_pairs;
  }
  // records: cell c's pads at start[c] + 2c, its vertex j at start[c] + 2c + 2 + j
  Rec<T>* s = reinterpret_cast<Rec<T>*>(smem);
  int* wide = reinterpret_cast<int*>(s + nv + 2 * count);   // vertices left to pass 2
  if (tid < 2 * count) {
    const T p = (tid & 1) ? T(__builtin_inf()) : -T(__builtin_inf());
    s[cell_start[tid >> 1] + (tid & ~1) + (tid & 1)] = Rec<T>{p, p, p, p};
  }

  // The thread's vertices of chunk u0 are u0 + tid + 256 i. Per chunk: cell lookups (LDS
  // only), then every global load of the chunk back to back, then the LDS writes.
  constexpr int kChunk = kFilterIt * kFilterThreads;
  uint32_t rows[kFilterIt][N / 2];
  int bases[kFilterIt], selfs[kFilterIt];
  for (int u0 = 0; u0 < nv; u0 += kChunk) {
    int cells[kFilterIt];
    const uint16_t* rowp[kFilterIt];
#pragma unroll
    for (int i = 0; i < kFilterIt; ++i) {
      const int u = min(u0 + i * kFilterThreads + tid, nv - 1);
      const int c = cell_of(cell_start, count, u);
      cells[i] = c;
      rowp[i] = hdr.b.nb[c] + (size_t)(u - cell_start[c]) * N;
    }
    if (u0 == 0) {   // the first chunk's neighbour rows, in flight with its force loads
#pragma unroll
      for (int i = 0; i < kFilterIt; ++i) load_row<N>(rowp[i], rows[i]);
    }
    T r[3][kFilterIt];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i = 0; i < kFilterIt; ++i) {
        const int u = min(u0 + i * kFilterThreads + tid, nv - 1);
        r[c][i] = f[c * vt + v0 + u];
      }
#pragma unroll
    for (int i = 0; i < kFilterIt; ++i) {
      const int u = u0 + i * kFilterThreads + tid;
      if (u < nv) s[u + 2 * cells[i] + kNbBias] = Rec<T>{r[0][i], r[1][i], r[2][i], T(0)};
    }
  }
  __syncthreads();

  // pass 1
  for (int u0 = 0; u0 < nv; u0 += kChunk) {
#pragma unroll
    for (int i = 0; i < kFilterIt; ++i) {
      const int u = min(u0 + i * kFilterThreads + tid, nv - 1);
      const int c = cell_of(cell_start, count, u);
      bases[i] = cell_start[c] + 2 * c;                   // the cell's first record
      selfs[i] = u + 2 * c + kNbBias;                     // the vertex's own record
      if (u0 > 0) load_row<N>(hdr.b.nb[c] + (size_t)(u - cell_start[c]) * N, rows[i]);
    }
#pragma unroll
    for (int i = 0; i < kFilterIt; ++i) {
      const int u = u0 + i * kFilterThreads + tid;
      if (u >= nv) break;
      const int deg = slot<N>(rows[i], 0);
      if (deg + 1 > N) {
        wide[atomicAdd(&n_wide, 1)] = u;
        continue;
      }
      Rec<T> k[N];
      k[0] = s[selfs[i]];
#pragma unroll
      for (int q = 1; q < N; ++q) k[q] = s[bases[i] + slot<N>(rows[i], q)];
      T ax[N], ay[N], az[N];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        ax[q] = k[q].x;
        ay[q] = k[q].y;
        az[q] = k[q].z;
      }
      const int64_t o = v0 + u;
      out[o] = median_padded<N>(ax, deg + 1);
      out[vt + o] = median_padded<N>(ay, deg + 1);
      out[2 * vt + o] = median_padded<N>(az, deg + 1);
    }
  }
  __syncthreads();
  // pass 2: one lane per (listed vertex, component); the ring's neighbour loads are clamped
  // into the ring and all issued before the first wait
  const int nw3 = 3 * n_wide;
  for (int l = tid; l < nw3; l += kFilterThreads) {
    const int u = wide[l / 3], c = l % 3;
    int cw = 0;
    while (u >= cell_start[cw + 1]) ++cw;
    const int base = cell_start[cw];
    const uint32_t info = as_global(c_info[cw])[u - base];
    const int deg = (int)(info & 255u);
    const __attribute__((address_space(1))) uint32_t* pr = as_global(c_pairs[cw] + (info >> 8));
    const T* sc = reinterpret_cast<const T*>(s + base + 2 * cw + kNbBias) + c;   // component c
    T r;
    if (deg + 1 <= kFilterWideKeys) {
      uint32_t pq[kFilterWideKeys - 1];
#pragma unroll
      for (int q = 0; q < kFilterWideKeys - 1; ++q) pq[q] = pr[min(q, deg - 1)];
      T a[kFilterWideKeys];
      a[0] = sc[4 * (u - base)];
#pragma unroll
      for (int q = 0; q < kFilterWideKeys - 1; ++q) {
        const T x = sc[4 * (int)(pq[q] & 0xffffu)];
        a[q + 1] = q < deg ? x : T(__builtin_inf());
      }
      r = median_keys<kFilterWideKeys>(a, deg + 1);
    } else {
      r = median_rank<T>(deg + 1, [&](int i) {
        return i == 0 ? sc[4 * (u - base)] : sc[4 * (int)(pr[i - 1] & 0xffffu)];
      });
    }
    out[c * vt + v0 + u] = r;
  }
}

template <typename T, int N>
hipError_t launch_t(const DevType* types, const FilterBlock* blocks, int n_blocks, int64_t vt,
                    const void* f, void* out, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL((k_median_filter<T, N>), dim3(n_blocks), dim3(kFilterThreads), lds_bytes, s,
                     types, blocks, vt, static_cast<const T*>(f), static_cast<T*>(out));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_median_filter(int precision, int net_keys, const DevType* types,
                                const FilterBlock* blocks, int n_blocks, int64_t vt,
                                const void* f, void* out, size_t lds_bytes, void* stream) {
  if (n_blocks == 0) return hipSuccess;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (precision == 64)
    return net_keys == 8 ? launch_t<double, 8>(types, blocks, n_blocks, vt, f, out, lds_bytes, s)
                         : launch_t<double, 16>(types, blocks, n_blocks, vt, f, out, lds_bytes, s);
  return net_keys == 8 ? launch_t<float, 8>(types, blocks, n_blocks, vt, f, out, lds_bytes, s)
                       : launch_t<float, 16>(types, blocks, n_blocks, vt, f, out, lds_bytes, s);
}

}  // namespace npfem
