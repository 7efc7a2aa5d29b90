// Launchers of the particle-in-kernel (PIK) contact detection kernels.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime_api.h>

#include "npfem_internal.h"

namespace npfem {

// Device workspace of one batch's contact detection, sized for V vertices.
struct ContactWork {
  int64_t n_vertices = 0;
  uint32_t n_buckets = 0;         // bucket table size: a power of two >= 2 V
  int32_t* cell_of = nullptr;     // [V] cell of each vertex
  int32_t* type_of = nullptr;     // [n_cells] type index of each cell
  int32_t* bucket = nullptr;      // [V] bucket of each vertex
  uint32_t* count = nullptr;      // [n_buckets] vertices per bucket (scatter cursor)
  uint32_t* start = nullptr;      // [n_buckets + 1] exclusive prefix sum of count
  void* entries = nullptr;        // [V] positions and vertex index, sorted by bucket
  int32_t* slot = nullptr;        // [V] sorted position of each vertex
  void* results = nullptr;        // [V] (p, w) of each record, in sorted order
  void* scan_tmp = nullptr;       // hipcub scan scratch
  size_t scan_bytes = 0;
};

// Allocates w for V vertices (cell_of / type_of filled by the caller afterwards).
hipError_t contact_work_alloc(ContactWork& w, int64_t n_vertices, int n_cells);
void contact_work_free(ContactWork& w);

// Allocation-free detection (npfem_detect_contacts_noalloc): the workspace is carved out of
// a static device array of kContactScratchBytes, one copy per GPU, instead of device memory
// allocated per batch. It serves batches of up to kNoAllocMaxVertices vertices.
constexpr size_t kContactScratchBytes = size_t(64) << 20;
constexpr int64_t kNoAllocMaxVertices = int64_t(1) << 19;

// Bytes of the workspace of a batch of V vertices in the scratch (both precisions, with the
// bucket scan's temporary storage), or 0 if the scan's size query fails.
size_t contact_noalloc_bytes(int64_t n_vertices);

// One detection pass on the scratch of the current device: cell_of is derived from the
// offsets on the device, type_of [n_cells] is the batch's device table. The first call on a
// device looks up the scratch's device address.
hipError_t launch_detect_contacts_noalloc(int precision, const DevType* types,
                                          const int64_t* offsets, int n_cells,
                                          const int32_t* type_of, int64_t n_vertices,
                                          const void* x, double radius, double separation,
                                          double weight, void* contact_p, void* contact_w,
                                          void* stream);

// One detection pass: fills contact_p [3][V] and contact_w [V] (precision 32 or 64).
hipError_t launch_detect_contacts(int precision, const DevType* types, const int64_t* offsets,
                                  ContactWork& w, const void* x, double radius, double separation,
                                  double weight, void* contact_p, void* contact_w, void* stream);

}  // namespace npfem
