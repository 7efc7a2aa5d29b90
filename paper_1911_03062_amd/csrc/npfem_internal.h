// Internal declarations shared by the host setup, the C ABI and the HIP kernels.
#pragma once

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/npfem.h"

namespace npfem {

// Per-vertex neighbour tables of the median filter for closed rings padded to N = 8 or 16 keys:
// slot 0 holds the degree, slots 1..N-1 the neighbours as cell-local index + 2, then the pads
// as codes 0 (-inf) and 1 (+inf): floor((N - 1 - degree) / 2) of code 0, the rest code 1 (rows
// of vertices whose closed ring exceeds N keys hold only the degree).
constexpr uint16_t kPadNeg = 0, kPadPos = 1, kNbBias = 2;

// ------------------------------------------------------------------------------------------
// Device-side records (plain structs, identical layout on host and device).
// ------------------------------------------------------------------------------------------

// One triangle slot of the per-wave round schedule (32 bytes). The vertex fields hold byte
// offsets (12 x vertex index) into a cell's LDS block of [vertex][xyz] floats, so that a lane
// adds its cell's base address and nothing else. A slot with orient == 0 (and area == 0) is
// empty. g_b, g_c are the rest-frame gradient vectors (g_a = -g_b - g_c); the rest frame makes
// D_m upper triangular, so g_c0 is always zero and not stored. The volume pass reads the first
// 16 bytes, the strain/area pass words 0-2 and 4-7.
struct TriRec {
  uint32_t a, b, c;   // 12 x vertex index
  float orient;       // +1 if (a, b, c) is a rotation of the mesh's (outward) order, -1 if
                      // not, 0 for an empty slot
  float area;
  float gb0, gb1, gc1;
};

// One hinge slot (32 bytes): edge (i, j), opposite vertices k, l (byte offsets as in TriRec),
// stencil a_e without a_i (a_i = -(a_j + a_k + a_l): the stencil sums to zero), rest norm.
// A slot with rest < 0 is empty.
struct HingeRec {
  uint32_t i, j, k, l;   // 12 x vertex index
  float a1, a2, a3;
  float rest;
};

// Element schedules of the fused form for one number of cells per wave (gw): slots = 64 / gw
// lanes per cell, rounds of vertex-disjoint elements.
struct FusedLayout {
  int gw = 0, slots = 0, tri_rounds = 0, hinge_rounds = 0;
  std::vector<TriRec> tri_sched;      // [tri_rounds][slots]
  std::vector<HingeRec> hinge_sched;  // [hinge_rounds][slots]
  int gather_slots = 0;
  std::vector<uint16_t> gather_sched; // [kMaxItems][64]: cell of the wave << 12 | vertex, or
                                      // kGatherEmpty; vertices by ring length, longest first
};

// Device copies of one fused layout's schedules.
struct LayoutDev {
  TriRec* tri = nullptr;
  HingeRec* hinge = nullptr;
  uint16_t* gather = nullptr;
};
constexpr uint16_t kGatherEmpty = 0xffff;

// Scalar parameters of a cell type as seen by the kernels.
struct TypeParams {
  int32_t n, m, e, bw;          // vertices, triangles, hinges, band width of L
  int32_t npad;                 // MFMA k rows per cell (fused): n rounded up to whole k steps
  int32_t cs;                   // LDS words per cell block (fused): 3 npad plus 3-15 pad words
  int32_t gw;                   // cells owned by one wave in a fused group
  int32_t slots;                // element slots per cell in a wave (64 / gw)
  int32_t tri_rounds, hinge_rounds;
  int32_t gather_slots;         // slots of the fused Skalak energy's ring gather (per lane)
  int32_t row_tiles;            // ceil(n / 16): MFMA row tiles of L^-1
  int32_t k_steps;              // MFMA k steps stored per L^-1 row tile: npad / 4 rounded
                                // up to whole kMfmaChunk chunks plus two chunks (zeros)
  int32_t skalak;               // membrane: 0 = PD constraints, 1 = Skalak energy
  int32_t band_w;               // window of the standalone banded substitution: the smallest
                                // 8 k + 1 >= bw (0: bw > 64, unsupported)
  int32_t linv_exp, pinv_exp;   // the fused global step's A tiles hold L^-1 (m M~^-1) times
                                // 2^exp
  double h, mass, inv_h2m;      // h, m, m / h^2
  double h2_over_m;             // h^2 / m
  double w_s, w_a, w_b, w_v;
  double s_min, s_max;
  double V0;
  double kappa;                 // position-based damping factor (0 = off)
  double v_max;                 // velocity cap (0 = off)
  double pred_h, pred_h2m;      // prediction without a solve: delta^0 = pred_h v + pred_h2m F
                                // (h and h^2/m over 1 + h alpha of Rayleigh damping)
  double ray_k;                 // beta / h of Rayleigh damping (0 = off): the gradient gains
                                // ray_k K e and the prediction solves with M~
  double ray_c;                 // fused form: c = ray_k / (1 + ray_k), the update's - c e
  double grad_mass;             // fused form: the gradient's coefficient of e
};

// Device copy of a cell type's constants. Pointers are device pointers.
struct DevType {
  TypeParams p;
  // vertex rings (fused form and median filter): the triangles (i, b, c) around each vertex i
  uint32_t* ring_info = nullptr;     // [n]: offset << 8 | degree
  uint32_t* ring_pairs = nullptr;    // [sum deg + kRingBatch]: b | c << 16 (then zero padding)
  uint16_t* ring_nb8 = nullptr;      // [n][8]: median-filter neighbour table, 8 keys
  uint16_t* ring_nb16 = nullptr;     // [n][16]: the same for 16 keys
  // fused form
  TriRec* tri_sched = nullptr;       // [tri_rounds][slots]
  HingeRec* hinge_sched = nullptr;   // [hinge_rounds][slots]
  uint16_t* gather_sched = nullptr;  // [kMaxItems][64] (fused Skalak energy)
  float* linv_tiles = nullptr;       // [row_tiles][k_steps / kMfmaChunk][512 words]: split
                                     // fp16 MFMA A operand of L^-1 2^linv_exp
  float* pinv_tiles = nullptr;       // m M~^-1 2^pinv_exp in the same form (Rayleigh beta > 0)
  // plain form (both precisions)
  int32_t* tri = nullptr;            // [m][3]
  int32_t* hinge = nullptr;          // [e][4]
  int32_t* vt_off = nullptr;         // [n+1] vertex -> (t*3 + j)
  int32_t* vt_list = nullptr;
  int32_t* vh_off = nullptr;         // [n+1] vertex -> (e*4 + q)
  int32_t* vh_list = nullptr;
  double* G64 = nullptr;  float* G32 = nullptr;          // [m][3][2]
  double* A64 = nullptr;  float* A32 = nullptr;          // [m]
  double* coef64 = nullptr; float* coef32 = nullptr;     // [e][4]
  double* rest64 = nullptr; float* rest32 = nullptr;     // [e]
  double* cband64 = nullptr; float* cband32 = nullptr;   // [n][bw+1]: C[i][i-k]
  double* mband64 = nullptr; float* mband32 = nullptr;   // [n][bw+1]: factor of M~ (Rayleigh)
  double* kband64 = nullptr; float* kband32 = nullptr;   // [n][bw+1]: K[i][i-k] (Rayleigh)
  // standalone global step (npfem_global_solve), banded factor padded to band_w:
  double* sband_rows64 = nullptr; float* sband_rows32 = nullptr;   // [n][band_w+1]: C[i][i-k]
  double* sband_cols64 = nullptr; float* sband_cols32 = nullptr;   // [n][band_w+1]: C[i+k][i],
                                                                   // k = 0: 1 / C[i][i]
  // standalone global step, dense vector form: L^-1 [n][n] (symmetric) in either precision
  double* linv64 = nullptr; float* linv32 = nullptr;
};

}  // namespace npfem

// ------------------------------------------------------------------------------------------
// Host objects behind the opaque C handles.
// ------------------------------------------------------------------------------------------

struct npfem_celltype {
  int n = 0, m = 0, e = 0, bw = 0;
  double h = 0, V0 = 0, area0 = 0, mass = 0;
  double w_s = 0, w_a = 0, w_b = 0, w_v = 0, s_min = 1, s_max = 1, kappa = 0;
  double v_max = 0;
  double alpha = 0, beta = 0;     // Rayleigh damping
  int membrane = 0;               // NPFEM_MEMBRANE_*
  std::vector<double> mband;      // [n][bw+1] banded Cholesky factor of M~ (beta > 0)
  std::vector<double> kband;      // [n][bw+1] lower band of K (beta > 0)
  std::vector<double> pinv;       // [n][n] m M~^-1 (beta > 0), the fused form's prediction
  std::vector<double> X;          // [n][3]
  std::vector<int32_t> tri;       // [m][3]
  std::vector<double> G;          // [m][3][2]
  std::vector<double> A;          // [m]
  std::vector<int32_t> hinge;     // [e][4]
  std::vector<double> coef;       // [e][4]
  std::vector<double> rest_norm;  // [e]
  std::vector<double> L;          // [n][n]
  std::vector<double> chol;       // [n][n] lower Cholesky factor
  std::vector<double> cband;      // [n][bw+1]
  std::vector<double> Linv;       // [n][n]
  std::vector<int32_t> vt_off, vt_list, vh_off, vh_list;
  std::vector<uint32_t> ring_info, ring_pairs;
  std::vector<uint16_t> ring_nb8, ring_nb16;  // [n][8], [n][16]
  // fused form: LDS column length and one element-schedule layout per feasible number of
  // cells per wave (largest first; layouts[0] is the default). gw, slots and the rounds
  // below describe layouts[0].
  int gw = 0, slots = 0, npad = 0, cs = 0, tri_rounds = 0, hinge_rounds = 0;
  std::vector<npfem::FusedLayout> layouts;
  bool fused_ok = false;
  std::string fused_reason;

  std::mutex mu;
  std::map<int, npfem::DevType*> dev;   // per HIP device: shared device data, layouts[0]
  // per HIP device, per layout: device copies of that layout's schedules
  std::map<int, std::vector<npfem::LayoutDev>> dev_sched;
  ~npfem_celltype();
};

namespace npfem {

void set_error(const std::string& msg);
npfem_status fail(npfem_status s, const std::string& msg);

// Host setup (setup.cpp).
npfem_status build_celltype(const npfem_mesh* mesh, const npfem_material* mat, double dt,
                            npfem_celltype* ct);

// Device upload of a cell type (device.cpp); returns the device copy for the current device.
npfem_status upload_celltype(npfem_celltype* ct, DevType** out);
void free_devtype(DevType* d);

constexpr int kFusedThreads = 256;          // 4 waves per workgroup
constexpr int kFusedWaves = 4;
constexpr int kMaxItems = 9;                // owner items per lane (cells x vertices / 64)
constexpr int kFusedLdsBudget = 52224;      // bytes of LDS per fused workgroup
// The fused kernel's residual blocks R start at this fixed word offset from the position
// blocks X (half the budget), so that one address per vertex serves both arrays (the offset
// goes into the LDS instruction's immediate field). X, and R with its damping words, must
// each fit in half the budget.
constexpr int kFusedRWords = kFusedLdsBudget / 8;
constexpr int kMaxGroupCells = 64;
constexpr int kMaxFusedGrid = 4096;         // workgroups of one fused launch (then they loop)

// One group of same-type cells processed by one fused workgroup.
struct FusedGroup {
  int32_t type;                  // index into the batch's type table
  int32_t count;                 // cells in the group (<= 4 * gw)
  int32_t cells[kMaxGroupCells]; // batch cell ids
};

constexpr int kMfmaChunk = 8;               // k steps per prefetched L^-1 chunk
constexpr double kArmijoC = 1e-4;           // Skalak line search: sufficient decrease
constexpr int kMaxHalvings = 8;             //   and step lengths 1, 1/2, ..., 1/256
constexpr int kSkalakMaxGw = 2;             // fused Skalak types: at most 2 cells per wave
constexpr int kSkalakMaxCells = kFusedWaves * kSkalakMaxGw;   // and per group
constexpr int kDampWords = 12;              // LDS floats per cell for position-based damping
constexpr int kRingBatch = 6;               // ring words loaded together (device copy padded by as many)
constexpr int kMaxTilesPerWave = 10;        // MFMA 16x16 output tiles held per wave (even)

// MFMA output tiles of the global step: each wave takes an equal share of the
// row_tiles x col_tiles tiles (row-major) and works on items of one or two neighbouring
// tiles, each item held in a pair of the kMaxTilesPerWave accumulator slots.
#ifdef __HIPCC__
#define NPFEM_HD __host__ __device__
#else
#define NPFEM_HD
#endif
// k row, within a chunk's 32 rows, of MFMA lane group g = lane / 16 at step j of the chunk:
// 2 j + {0, 16, 1, 17}[g]. The two groups of a half-wave read rows 16 apart (48 words: the
// other 16 banks).
inline NPFEM_HD constexpr int k_row_in_chunk(int g, int j) { return 2 * j + (g & 1) * 16 + (g >> 1); }
static_assert(kMfmaChunk == 8, "a chunk covers the 32 k rows of k_row_in_chunk's order");
// Number of work items the global step forms from the share [u0, u1) of the row-major tiles
// of a group with col_tiles column tiles (the kernel's pairing rule: two column tiles of one
// row tile, or two row tiles when there is one column tile).
inline NPFEM_HD int mfma_share_items(int col_tiles, int u0, int u1) {
  int items = 0;
  for (int u = u0; u < u1; ++items) {
    if (col_tiles >= 2) {
      const int ct = u % col_tiles;
      u += (ct + 1 < col_tiles && u + 1 < u1) ? 2 : 1;
    } else {
      u += (u + 1 < u1) ? 2 : 1;
    }
  }
  return items;
}

// Median filter of the external forces: one workgroup per block of consecutive whole cells.
constexpr int kFilterThreads = 256;
constexpr int kFilterMaxCells = 32;         // cells per block
constexpr int kFilterMaxVerts = 1024;       // vertices per block (a larger cell is alone)
constexpr int kFilterWideKeys = 32;         // network keys of the wide-ring pass
// Header of one block, read by the kernel with one load per lane.
struct FilterBlock {
  int64_t v0;                          // first vertex of the block in the batch
  int32_t count, nv;                   // cells, vertices
  const uint16_t* nb[kFilterMaxCells]; // each cell's neighbour table (device, 8 or 16 keys)
  int32_t start[kFilterMaxCells + 1];  // first vertex of each cell, relative to v0
  int16_t type[kFilterMaxCells];       // index of each cell's type in the batch's type table
  int32_t pad[2];
};
static_assert(sizeof(FilterBlock) % 16 == 0, "FilterBlock is read as whole dwords");

// Kernel launchers and sizes (kernels_plain.hip, kernels_fused.hip, kernels_filter.hip).
size_t plain_work_bytes(int precision, int n, int m, int e);
bool plain_supported(int n, int bw);
hipError_t launch_plain_cell(int precision, const DevType* dt_dev, const TypeParams& p, void* x,
                             void* v, const void* f, const void* cp, const void* cw, int64_t vtot,
                             int64_t off, int K, void* work, double* vol_area, int* flag,
                             void* stream);
hipError_t launch_fused_step(const DevType* types_dev, int n_types, const FusedGroup* groups,
                             const int* n_groups_dev, int max_groups, const int64_t* offsets,
                             int64_t vtot, float* x, float* v, const float* f, const float* cp,
                             const float* cw, int K, double* vol_area, int* flag, size_t lds_bytes,
                             bool extras, bool skalak, void* stream);
// Global step alone (npfem_global_solve), over one type's cells: dense L^-1 on the matrix cores
// (FP32), the dense L^-1 on the vector ALU or the banded substitution (either precision).
// Wide form of the dense global step over one type's cells: kWideMaxCells cells per workgroup
// unless their LDS cell blocks exceed 64 KB.
constexpr int kWideMaxCells = 16;
inline int wide_cells_per_block(int cs) {
  const int fit = (int)(65536 / ((size_t)cs * sizeof(float)));
  return fit < kWideMaxCells ? (fit < 1 ? 1 : fit) : kWideMaxCells;
}
hipError_t launch_global_dense_wide(const DevType* dt, int cs, const int32_t* cells, int n_cells,
                                    const int64_t* offsets, int64_t vtot, const float* r, float* out,
                                    void* stream);
hipError_t launch_global_gemv(int precision, int n, const DevType* dt, const int32_t* cells, int n_cells,
                              const int64_t* offsets, int64_t vt, const void* r, void* out, void* stream);
hipError_t launch_global_banded(int precision, int n, int band_w, const DevType* dt, const int32_t* cells,
                                int n_cells, const int64_t* offsets, int64_t vt, const void* r,
                                void* out, void* stream);
hipError_t launch_median_filter(int precision, int net_keys, const DevType* types,
                                const FilterBlock* blocks, int n_blocks, int64_t vt,
                                const void* f, void* out, size_t lds_bytes, void* stream);

}  // namespace npfem
