// Particle-in-kernel (PIK) contact detection: for every vertex of the batch, the closest
// vertex of another cell inside the interpolation kernel's sphere, and the projection point
// that the collision energy pulls the vertex towards (main text, near-contact handling;
// supplementary material, particle-in-kernel technique).
//
// A uniform grid of cell size c (slightly above the kernel radius r) is folded into a table
// of 2^k buckets by a periodic linear index, bucket = (ix mod 2^kx) + 2^kx ((iy mod 2^ky) +
// 2^ky (iz mod 2^kz)) with kx + ky + kz = k, so that neighbouring grid cells along x are
// consecutive buckets; a counting sort places every vertex's position and index in its
// bucket's range. Queries run in that bucket order (neighbouring lanes read nearly the same
// records). A vertex scans the grid cells around its own, one row along x at a time (one
// contiguous range of records unless the row wraps around the fold): every vertex within r
// lies in one of the 27, since |x_i - x_j| < r < c keeps the cell coordinates within one of
// each other, and cells whose box is a full cell size or more from the vertex are skipped
// (on average about 6 of the 27). Grid cells one fold period or more apart share buckets;
// their records only add candidates that the distance test rejects. The query writes its
// results in bucket order; a last pass puts them back in vertex order with coalesced writes.
//
// The choice of the neighbour is exact and independent of the order of the scan: squared
// distances in the batch precision, ((dx dx + dy dy) + dz dz) with every operation rounded
// (no fused multiply-add), strictly below r^2, smallest distance first and the smallest
// vertex index among equal distances.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <map>
#include <mutex>

#include "contacts.h"

namespace npfem {

// Workspace of the allocation-free detection. Each GPU that runs it holds its own copy of the
// array until the process ends; host code reaches it only through the device address that
// hipGetSymbolAddress returns for the current device (the name is a host-side stand-in).
static __device__ __align__(256) unsigned char scratch[kContactScratchBytes];

namespace {

constexpr int kContactThreads = 256;
constexpr double kCellOverRadius = 1.001;   // grid cell size / kernel radius
constexpr uint32_t kXcds = 8;               // accelerator complex dies (one L2 each)

template <typename T>
struct Entry {
  T x, y, z;
  int32_t j;
};

template <typename T>
struct Result {
  T px, py, pz, w;
};

__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ float sub_rn(float a, float b) { return __fsub_rn(a, b); }
__device__ __forceinline__ double sub_rn(double a, double b) { return __dsub_rn(a, b); }

// Periodic linear index of grid cell (ix, iy, iz); g = (kx, ky, kz) bit widths.
struct GridFold {
  uint32_t kx, ky, kz;
};

__device__ __forceinline__ uint32_t bucket_of(int ix, int iy, int iz, GridFold g) {
  const uint32_t bx = (uint32_t)ix & ((1u << g.kx) - 1u);
  const uint32_t by = (uint32_t)iy & ((1u << g.ky) - 1u);
  const uint32_t bz = (uint32_t)iz & ((1u << g.kz) - 1u);
  return bx | (by << g.kx) | (bz << (g.kx + g.ky));
}

template <typename T>
__device__ __forceinline__ int grid_coord(T v, T inv_c) {
  return (int)floor(v * inv_c);
}

__global__ void __launch_bounds__(kContactThreads) k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kContactThreads + threadIdx.x;
  if (i < n) p[i] = v;
}

// Runs of equal buckets among the lanes of a wave (consecutive vertices of a cell often share
// a grid cell): a lane learns the first lane of its run and the run's length, so that one
// atomic serves the run. Every lane of the wave takes part (inactive lanes carry b = ~0u).
struct Run {
  int head;    // first lane of the run
  int len;     // lanes in the run
};

__device__ __forceinline__ Run bucket_run(uint32_t b) {
  const int lane = (int)(threadIdx.x & 63u);
  const uint32_t prev = __shfl_up(b, 1, 64);
  const bool is_head = lane == 0 || prev != b;
  const uint64_t heads = __ballot(is_head);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);   // lanes 0..lane
  Run r;
  r.head = 63 - __clzll((long long)(heads & upto));
  const uint64_t after = heads & ~upto;
  r.len = (after ? (__ffsll((long long)after) - 1) : 64) - r.head;
  return r;
}

template <typename T>
__global__ void __launch_bounds__(kContactThreads)
    k_contact_count(const T* __restrict__ x, int64_t V, T inv_c, GridFold fold,
                    int32_t* __restrict__ bucket, uint32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * kContactThreads + threadIdx.x;
  const bool active = i < V;
  uint32_t b = ~0u;
  if (active) {
    b = bucket_of(grid_coord(x[i], inv_c), grid_coord(x[V + i], inv_c),
                  grid_coord(x[2 * V + i], inv_c), fold);
    bucket[i] = (int32_t)b;
  }
  const Run r = bucket_run(b);
  if (active && (int)(threadIdx.x & 63u) == r.head) atomicAdd(&count[b], (uint32_t)r.len);
}

// Counting-sort scatter: count[b] runs down to zero, so the table is clear for the next pass.
// The head of a run of equal buckets claims the run's slots with one atomic.
template <typename T>
__global__ void __launch_bounds__(kContactThreads)
    k_contact_scatter(const T* __restrict__ x, int64_t V, const int32_t* __restrict__ bucket,
                      const uint32_t* __restrict__ start, uint32_t* __restrict__ count,
                      Entry<T>* __restrict__ entries, int32_t* __restrict__ slot) {
  const int64_t i = (int64_t)blockIdx.x * kContactThreads + threadIdx.x;
  const bool active = i < V;
  const uint32_t b = active ? (uint32_t)bucket[i] : ~0u;
  const Run r = bucket_run(b);
  const int lane = (int)(threadIdx.x & 63u);
  uint32_t top = 0;   // count[b] before the run's claim: slots [top - len, top) are the run's
  if (active && lane == r.head) top = atomicSub(&count[b], (uint32_t)r.len);
  top = __shfl(top, r.head, 64);
  if (!active) return;
  const uint32_t pos = start[b] + top - (uint32_t)r.len + (uint32_t)(lane - r.head);
  Entry<T> e;
  e.x = x[i];
  e.y = x[V + i];
  e.z = x[2 * V + i];
  e.j = (int32_t)i;
  entries[pos] = e;
  slot[i] = (int32_t)pos;
}

template <typename T>
__global__ void __launch_bounds__(kContactThreads)
    k_contact_query(const DevType* __restrict__ types, const int64_t* __restrict__ offsets,
                    const int32_t* __restrict__ cell_of, const int32_t* __restrict__ type_of,
                    const T* __restrict__ x, int64_t V, T inv_c, GridFold fold,
                    const uint32_t* __restrict__ start, const Entry<T>* __restrict__ entries,
                    T r2, T sep, T weight, Result<T>* __restrict__ res) {
  // Workgroups go to the 8 XCDs round-robin (block b to XCD b mod 8); XCD x takes the x-th
  // contiguous eighth of the records, so that queries sharing rows of records share an L2.
  const uint32_t nb = gridDim.x, xcd = blockIdx.x % kXcds, idx = blockIdx.x / kXcds;
  const uint32_t per = nb / kXcds, rem = nb % kXcds;
  const uint32_t block = xcd * per + (xcd < rem ? xcd : rem) + idx;
  const int64_t q = (int64_t)block * kContactThreads + threadIdx.x;
  if (q >= V) return;
  // queries in bucket order: neighbouring lanes scan nearly the same rows of records
  const Entry<T> me = entries[q];
  const int64_t i = me.j;
  const T xi = me.x, yi = me.y, zi = me.z;
  const int ci = cell_of[i];
  const int64_t own0 = offsets[ci], own1 = offsets[ci + 1];   // the vertex's own cell
  const T ux = xi * inv_c, uy = yi * inv_c, uz = zi * inv_c;   // grid units
  const int gx = (int)floor(ux), gy = (int)floor(uy), gz = (int)floor(uz);
  const T fx = ux - (T)gx, fy = uy - (T)gy, fz = uz - (T)gz;
  T best = r2;
  int32_t bj = -1;
  auto scan = [&](uint32_t k0, uint32_t k1) {
    for (uint32_t k = k0; k < k1; ++k) {
      const Entry<T> e = entries[k];
      const T ex = sub_rn(e.x, xi), ey = sub_rn(e.y, yi), ez = sub_rn(e.z, zi);
      const T d2 = add_rn(add_rn(mul_rn(ex, ex), mul_rn(ey, ey)), mul_rn(ez, ez));
      if (d2 < r2 && (e.j < own0 || e.j >= own1) && (d2 < best || (d2 == best && e.j < bj))) {
        best = d2;
        bj = e.j;
      }
    }
  };
  // grid cells whose box lies a full cell (1.001 r) or more away hold no vertex within r
  // (the margin covers the rounding of the grid units); the cells of one row along x that
  // remain are consecutive buckets unless the row wraps around the fold
  for (int dz = -1; dz <= 1; ++dz) {
    const T cz = dz < 0 ? fz : (dz > 0 ? T(1) - fz : T(0));
    for (int dy = -1; dy <= 1; ++dy) {
      const T cy = dy < 0 ? fy : (dy > 0 ? T(1) - fy : T(0));
      const T row = cy * cy + cz * cz;
      if (row >= T(1)) continue;
      const int lo = (fx * fx + row < T(1)) ? -1 : 0;
      const int hi = ((T(1) - fx) * (T(1) - fx) + row < T(1)) ? 1 : 0;
      const uint32_t b_lo = bucket_of(gx + lo, gy + dy, gz + dz, fold);
      const uint32_t b_hi = bucket_of(gx + hi, gy + dy, gz + dz, fold);
      if (b_hi - b_lo == (uint32_t)(hi - lo)) {
        scan(start[b_lo], start[b_hi + 1]);
      } else {
        for (int dx = lo; dx <= hi; ++dx) {
          const uint32_t b = bucket_of(gx + dx, gy + dy, gz + dz, fold);
          scan(start[b], start[b + 1]);
        }
      }
    }
  }
  if (bj < 0) {
    res[q] = Result<T>{xi, yi, zi, T(0)};
    return;
  }
  // unit outward normal of the neighbour's cell at the neighbour: the sum of its incident
  // triangles' doubled area vectors (x_b - x_j) x (x_c - x_j), (j, b, c) counter-clockwise
  const int cj = cell_of[bj];
  const DevType& D = types[type_of[cj]];
  const int64_t off = offsets[cj];
  const int vj = (int)(bj - off);
  const T xj = x[bj], yj = x[V + bj], zj = x[2 * V + bj];
  const uint32_t info = D.ring_info[vj];
  const int roff = (int)(info >> 8), deg = (int)(info & 255u);
  T nx = T(0), ny = T(0), nz = T(0);
  for (int s = 0; s < deg; ++s) {
    const uint32_t pr = D.ring_pairs[roff + s];
    const int64_t b = off + (int64_t)(pr & 0xffffu), c = off + (int64_t)(pr >> 16);
    const T bx = x[b] - xj, by = x[V + b] - yj, bz = x[2 * V + b] - zj;
    const T cx = x[c] - xj, cy = x[V + c] - yj, cz = x[2 * V + c] - zj;
    nx += by * cz - bz * cy;
    ny += bz * cx - bx * cz;
    nz += bx * cy - by * cx;
  }
  const T s = sep / sqrt(nx * nx + ny * ny + nz * nz);
  res[q] = Result<T>{xj + s * nx, yj + s * ny, zj + s * nz, weight};
}

// Results back in vertex order: coalesced writes of contact_p [3][V] and contact_w [V].
template <typename T>
__global__ void __launch_bounds__(kContactThreads)
    k_contact_unpermute(int64_t V, const int32_t* __restrict__ slot,
                        const Result<T>* __restrict__ res, T* __restrict__ cp, T* __restrict__ cw) {
  const int64_t i = (int64_t)blockIdx.x * kContactThreads + threadIdx.x;
  if (i >= V) return;
  const Result<T> r = res[slot[i]];
  cp[i] = r.px;
  cp[V + i] = r.py;
  cp[2 * V + i] = r.pz;
  cw[i] = r.w;
}

// Cell of every vertex from the batch's vertex offsets (offsets[0] = 0 <= i < offsets[n_cells]
// = V): the last cell whose first vertex is at or before i.
__global__ void __launch_bounds__(kContactThreads)
    k_cell_of(const int64_t* __restrict__ offsets, int n_cells, int64_t V,
              int32_t* __restrict__ cell_of) {
  const int64_t i = (int64_t)blockIdx.x * kContactThreads + threadIdx.x;
  if (i >= V) return;
  int lo = 0, hi = n_cells;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offsets[mid] <= i) lo = mid;
    else hi = mid;
  }
  cell_of[i] = lo;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kContactThreads - 1) / kContactThreads); }

// Places the pieces of a workspace for V vertices at 256-byte aligned offsets from base (a
// null base only measures) and returns the bytes they span, 0 if the scan's size query fails.
// type_of is not placed: the caller supplies it.
size_t carve(ContactWork& w, char* base, int64_t V) {
  uint32_t nb = 1024;
  while ((int64_t)nb < 2 * V) nb <<= 1;
  size_t used = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + used : nullptr;
    used += (bytes + 255) & ~size_t(255);
    return p;
  };
  w.n_vertices = V;
  w.n_buckets = nb;
  w.cell_of = static_cast<int32_t*>(take(sizeof(int32_t) * (size_t)V));
  w.bucket = static_cast<int32_t*>(take(sizeof(int32_t) * (size_t)V));
  w.count = static_cast<uint32_t*>(take(sizeof(uint32_t) * ((size_t)nb + 1)));
  w.start = static_cast<uint32_t*>(take(sizeof(uint32_t) * ((size_t)nb + 1)));
  w.entries = take(sizeof(Entry<double>) * (size_t)V);   // large enough for either precision
  w.slot = static_cast<int32_t*>(take(sizeof(int32_t) * (size_t)V));
  w.results = take(sizeof(Result<double>) * (size_t)V);
  size_t scan = 0;
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, scan, w.count, w.start, (int)nb + 1) != hipSuccess)
    return 0;
  w.scan_bytes = scan;
  w.scan_tmp = take(scan > 0 ? scan : 1);
  return used;
}

// Device address of the scratch on the current device, looked up once per device.
hipError_t scratch_address(void** out) {
  static std::mutex mu;
  static std::map<int, void*> by_device;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = by_device.find(dev);
  if (it == by_device.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    it = by_device.emplace(dev, p).first;
  }
  *out = it->second;
  return hipSuccess;
}

template <typename T>
hipError_t detect(const DevType* types, const int64_t* offsets, ContactWork& w, const T* x,
                  double radius, double separation, double weight, T* cp, T* cw, hipStream_t s) {
  const int64_t V = w.n_vertices;
  const T inv_c = (T)(1.0 / (radius * kCellOverRadius));
  const T r = (T)radius;
  const T r2 = r * r;
  uint32_t k = 0;
  while ((1u << k) < w.n_buckets) ++k;
  GridFold fold;
  fold.kx = (k + 2) / 3;
  fold.ky = (k - fold.kx + 1) / 2;
  fold.kz = k - fold.kx - fold.ky;
  Entry<T>* entries = static_cast<Entry<T>*>(w.entries);
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(w.n_buckets + 1)), dim3(kContactThreads), 0, s,
                     w.count, (int64_t)w.n_buckets + 1, 0u);
  hipLaunchKernelGGL(k_contact_count<T>, dim3(blocks_for(V)), dim3(kContactThreads), 0, s, x, V,
                     inv_c, fold, w.bucket, w.count);
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(w.scan_tmp, w.scan_bytes, w.count, w.start,
                                                  (int)w.n_buckets + 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_contact_scatter<T>, dim3(blocks_for(V)), dim3(kContactThreads), 0, s, x, V,
                     w.bucket, w.start, w.count, entries, w.slot);
  hipLaunchKernelGGL(k_contact_query<T>, dim3(blocks_for(V)), dim3(kContactThreads), 0, s, types,
                     offsets, w.cell_of, w.type_of, x, V, inv_c, fold, w.start, entries, r2,
                     (T)separation, (T)weight, static_cast<Result<T>*>(w.results));
  hipLaunchKernelGGL(k_contact_unpermute<T>, dim3(blocks_for(V)), dim3(kContactThreads), 0, s, V,
                     w.slot, static_cast<const Result<T>*>(w.results), cp, cw);
  return hipGetLastError();
}

}  // namespace

hipError_t contact_work_alloc(ContactWork& w, int64_t n_vertices, int n_cells) {
  contact_work_free(w);
  uint32_t nb = 1024;
  while ((int64_t)nb < 2 * n_vertices) nb <<= 1;
  w.n_vertices = n_vertices;
  w.n_buckets = nb;
  const size_t entry_bytes = sizeof(Entry<double>);   // large enough for either precision
  hipError_t e = hipSuccess;
  if ((e = hipMalloc(&w.cell_of, sizeof(int32_t) * (size_t)n_vertices)) != hipSuccess ||
      (e = hipMalloc(&w.type_of, sizeof(int32_t) * (size_t)n_cells)) != hipSuccess ||
      (e = hipMalloc(&w.bucket, sizeof(int32_t) * (size_t)n_vertices)) != hipSuccess ||
      (e = hipMalloc(&w.count, sizeof(uint32_t) * ((size_t)nb + 1))) != hipSuccess ||
      (e = hipMalloc(&w.start, sizeof(uint32_t) * ((size_t)nb + 1))) != hipSuccess ||
      (e = hipMalloc(&w.entries, entry_bytes * (size_t)n_vertices)) != hipSuccess ||
      (e = hipMalloc(&w.slot, sizeof(int32_t) * (size_t)n_vertices)) != hipSuccess ||
      (e = hipMalloc(&w.results, sizeof(Result<double>) * (size_t)n_vertices)) != hipSuccess) {
    contact_work_free(w);
    return e;
  }
  e = hipcub::DeviceScan::ExclusiveSum(nullptr, w.scan_bytes, w.count, w.start, (int)nb + 1);
  if (e == hipSuccess) e = hipMalloc(&w.scan_tmp, w.scan_bytes > 0 ? w.scan_bytes : 1);
  if (e != hipSuccess) contact_work_free(w);
  return e;
}

size_t contact_noalloc_bytes(int64_t n_vertices) {
  ContactWork w;
  return carve(w, nullptr, n_vertices);
}

hipError_t launch_detect_contacts_noalloc(int precision, const DevType* types,
                                          const int64_t* offsets, int n_cells,
                                          const int32_t* type_of, int64_t n_vertices,
                                          const void* x, double radius, double separation,
                                          double weight, void* contact_p, void* contact_w,
                                          void* stream) {
  if (n_vertices == 0) return hipSuccess;
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return e;
  ContactWork w;   // a view of the scratch, never freed
  const size_t used = carve(w, static_cast<char*>(base), n_vertices);
  if (used == 0 || used > kContactScratchBytes) return hipErrorInvalidValue;
  w.type_of = const_cast<int32_t*>(type_of);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_cell_of, dim3(blocks_for(n_vertices)), dim3(kContactThreads), 0, s, offsets,
                     n_cells, n_vertices, w.cell_of);
  if (precision == 64)
    return detect<double>(types, offsets, w, static_cast<const double*>(x), radius, separation,
                          weight, static_cast<double*>(contact_p), static_cast<double*>(contact_w),
                          s);
  return detect<float>(types, offsets, w, static_cast<const float*>(x), radius, separation, weight,
                       static_cast<float*>(contact_p), static_cast<float*>(contact_w), s);
}

void contact_work_free(ContactWork& w) {
  for (void* p : {(void*)w.cell_of, (void*)w.type_of, (void*)w.bucket, (void*)w.count,
                  (void*)w.start, w.entries, (void*)w.slot, w.results, w.scan_tmp})
    if (p) (void)hipFree(p);
  w = ContactWork{};
}

hipError_t launch_detect_contacts(int precision, const DevType* types, const int64_t* offsets,
                                  ContactWork& w, const void* x, double radius, double separation,
                                  double weight, void* contact_p, void* contact_w, void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (w.n_vertices == 0) return hipSuccess;
  if (precision == 64)
    return detect<double>(types, offsets, w, static_cast<const double*>(x), radius, separation,
                          weight, static_cast<double*>(contact_p), static_cast<double*>(contact_w),
                          s);
  return detect<float>(types, offsets, w, static_cast<const float*>(x), radius, separation, weight,
                       static_cast<float*>(contact_p), static_cast<float*>(contact_w), s);
}

}  // namespace npfem
