// C ABI of libnpfem: cell types, batches, the step entry point and error reporting.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "npfem_internal.h"
#include "contacts.h"

namespace npfem {

namespace {
thread_local std::string g_last_error;

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(NPFEM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

template <typename D, typename S>
npfem_status upload(D** dst, const std::vector<S>& src) {
  std::vector<D> tmp(src.begin(), src.end());
  if (tmp.empty()) tmp.resize(1);
  HIP_TRY(hipMalloc((void**)dst, tmp.size() * sizeof(D)));
  HIP_TRY(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(D), hipMemcpyHostToDevice));
  return NPFEM_OK;
}

template <typename D>
npfem_status upload_raw(D** dst, const D* src, size_t count) {
  HIP_TRY(hipMalloc((void**)dst, std::max<size_t>(count, 1) * sizeof(D)));
  if (count) HIP_TRY(hipMemcpy(*dst, src, count * sizeof(D), hipMemcpyHostToDevice));
  return NPFEM_OK;
}

#define NP_TRY(expr)                      \
  do {                                    \
    npfem_status s_ = (expr);             \
    if (s_ != NPFEM_OK) return s_;        \
  } while (0)

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

npfem_status fail(npfem_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

void free_devtype(DevType* d) {
  if (!d) return;
  // (schedules belong to the cell type's per-layout cache)
  void* ptrs[] = {d->ring_info, d->ring_pairs, d->ring_nb8, d->ring_nb16, d->linv_tiles, d->pinv_tiles,
                  d->tri,       d->hinge,       d->vt_off,    d->vt_list,    d->vh_off,
                  d->vh_list,   d->G64,         d->G32,       d->A64,        d->A32,
                  d->coef64,    d->coef32,      d->rest64,    d->rest32,     d->cband64,
                  d->cband32,   d->mband64,     d->mband32,   d->kband64,    d->kband32,
                  d->sband_rows64, d->sband_rows32, d->sband_cols64, d->sband_cols32,
                  d->linv64,    d->linv32};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete d;
}

// Device copies of layout li's schedules on device dev (uploaded once). Caller holds ct->mu.
npfem_status layout_schedules_locked(npfem_celltype* ct, int dev, int li, LayoutDev* out) {
  auto& v = ct->dev_sched[dev];
  if (v.empty()) v.assign(ct->layouts.size(), LayoutDev{});
  if (!v[li].tri) {
    const FusedLayout& lay = ct->layouts[li];
    LayoutDev d;
    npfem_status st = upload_raw(&d.tri, lay.tri_sched.data(), lay.tri_sched.size());
    if (st == NPFEM_OK) st = upload_raw(&d.hinge, lay.hinge_sched.data(), lay.hinge_sched.size());
    if (st == NPFEM_OK) st = upload_raw(&d.gather, lay.gather_sched.data(), lay.gather_sched.size());
    if (st != NPFEM_OK) {
      if (d.tri) (void)hipFree(d.tri);
      if (d.hinge) (void)hipFree(d.hinge);
      if (d.gather) (void)hipFree(d.gather);
      return st;
    }
    v[li] = d;
  }
  *out = v[li];
  return NPFEM_OK;
}

// Device copy of a cell type for the current device (created once, then shared).
npfem_status upload_celltype(npfem_celltype* ct, DevType** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(ct->mu);
  auto it = ct->dev.find(dev);
  if (it != ct->dev.end()) {
    *out = it->second;
    return NPFEM_OK;
  }
  DevType* d = new (std::nothrow) DevType();
  if (!d) return fail(NPFEM_E_NOMEM, "host allocation");
  TypeParams& p = d->p;
  p.n = ct->n; p.m = ct->m; p.e = ct->e; p.bw = ct->bw;
  p.npad = ct->npad; p.cs = ct->cs; p.gw = ct->gw; p.slots = ct->slots;
  p.tri_rounds = ct->tri_rounds; p.hinge_rounds = ct->hinge_rounds;
  p.gather_slots = ct->fused_ok ? ct->layouts[0].gather_slots : 0;
  p.row_tiles = (ct->n + 15) / 16;
  // whole chunks plus two zero chunks read by the global step's look-ahead loads
  p.k_steps = ((ct->npad / 4 + kMfmaChunk - 1) / kMfmaChunk + 2) * kMfmaChunk;
  p.skalak = 0;
  p.h = ct->h; p.mass = ct->mass;
  // Rayleigh damping: M~/h^2 = (1 + h alpha) m/h^2 I + (beta/h) K
  const double ma = 1.0 + ct->h * ct->alpha;
  p.inv_h2m = ma * ct->mass / (ct->h * ct->h);
  p.h2_over_m = ct->h * ct->h / ct->mass;
  p.ray_k = ct->beta / ct->h;
  p.skalak = ct->membrane == NPFEM_MEMBRANE_SKALAK ? 1 : 0;
  if (ct->beta > 0.0) {
    // the prediction is m M~^-1 (h v + h^2 F/m): the factor 1 / (1 + h alpha) is inside M~
    p.pred_h = ct->h;
    p.pred_h2m = p.h2_over_m;
  } else {
    p.pred_h = ct->h / ma;
    p.pred_h2m = p.h2_over_m / ma;
  }
  // fused form: with d = (1 + h alpha) m/h^2 + w_v and c = (beta/h) / (1 + beta/h),
  // (beta/h) K e = c (L e - d e), so the quasi-Newton update L^-1 grad g equals
  // L^-1 [(inv_h2m - c d) e + rest of grad g] + c e: the gradient takes grad_mass instead of
  // inv_h2m and the update subtracts c e
  p.ray_c = ct->beta > 0.0 ? p.ray_k / (1.0 + p.ray_k) : 0.0;
  p.grad_mass = p.inv_h2m - p.ray_c * (p.inv_h2m + ct->w_v);
  p.w_s = ct->w_s; p.w_a = ct->w_a; p.w_b = ct->w_b; p.w_v = ct->w_v;
  p.s_min = ct->s_min; p.s_max = ct->s_max; p.V0 = ct->V0; p.kappa = ct->kappa;
  p.v_max = ct->v_max;

  npfem_status st = NPFEM_OK;
  auto chk = [&](npfem_status s) { if (st == NPFEM_OK) st = s; };
  chk(upload(&d->tri, ct->tri));
  chk(upload(&d->hinge, ct->hinge));
  chk(upload(&d->vt_off, ct->vt_off));
  chk(upload(&d->vt_list, ct->vt_list));
  chk(upload(&d->vh_off, ct->vh_off));
  chk(upload(&d->vh_list, ct->vh_list));
  chk(upload(&d->G64, ct->G));   chk(upload(&d->G32, ct->G));
  chk(upload(&d->A64, ct->A));   chk(upload(&d->A32, ct->A));
  chk(upload(&d->coef64, ct->coef)); chk(upload(&d->coef32, ct->coef));
  chk(upload(&d->rest64, ct->rest_norm)); chk(upload(&d->rest32, ct->rest_norm));
  chk(upload(&d->cband64, ct->cband)); chk(upload(&d->cband32, ct->cband));
  // the standalone banded substitution's layouts of the factor, padded to its window
  p.band_w = 0;
  for (int w = 9; w <= 65; w += 8)
    if (ct->bw <= w) {
      p.band_w = w;
      break;
    }
  if (p.band_w > 0) {
    const int n = ct->n, bw = ct->bw, W = p.band_w;
    std::vector<double> rows((size_t)n * (W + 1), 0.0), cols((size_t)n * (W + 1), 0.0);
    for (int i = 0; i < n; ++i) {
      const double diag = ct->cband[(size_t)i * (bw + 1)];
      cols[(size_t)i * (W + 1)] = 1.0 / diag;
      rows[(size_t)i * (W + 1)] = diag;
      for (int k = 1; k <= bw; ++k) {
        if (i - k >= 0) rows[(size_t)i * (W + 1) + k] = ct->cband[(size_t)i * (bw + 1) + k];
        if (i + k < n) cols[(size_t)i * (W + 1) + k] = ct->cband[(size_t)(i + k) * (bw + 1) + k];
      }
    }
    chk(upload(&d->sband_rows64, rows)); chk(upload(&d->sband_rows32, rows));
    chk(upload(&d->sband_cols64, cols)); chk(upload(&d->sband_cols32, cols));
  }
  if (!ct->mband.empty()) {
    chk(upload(&d->mband64, ct->mband)); chk(upload(&d->mband32, ct->mband));
    chk(upload(&d->kband64, ct->kband)); chk(upload(&d->kband32, ct->kband));
  }
  // dense L^-1 for the standalone global step's vector form (both precisions)
  chk(upload(&d->linv64, ct->Linv)); chk(upload(&d->linv32, ct->Linv));
  // vertex rings: the fused form's volume gradient and the median filter (both forms)
  chk(upload(&d->ring_info, ct->ring_info));
  {
    std::vector<uint32_t> padded(ct->ring_pairs);
    padded.resize(padded.size() + kRingBatch, 0u);   // batched ring loads read past the last ring
    chk(upload(&d->ring_pairs, padded));
  }
  chk(upload(&d->ring_nb8, ct->ring_nb8));
  chk(upload(&d->ring_nb16, ct->ring_nb16));
  if (ct->fused_ok) {
    LayoutDev ld;
    chk(layout_schedules_locked(ct, dev, 0, &ld));
    d->tri_sched = ld.tri;
    d->hinge_sched = ld.hinge;
    d->gather_sched = ld.gather;
    // L^-1 as the split fp16 A operand of v_mfma_f32_16x16x32_f16: entries times 2^exp (exp
    // puts the largest magnitude in [2^13, 2^14)) as hi = fp16(a) and lo = fp16(a - hi), so
    // that hi + lo holds a to 22 significant bits (to 2^-25 absolute where lo is subnormal).
    // Row tile rt, chunk c (32 k rows), lane l, element i -> (row rt*16 + l%16, k row kr =
    // 4 s0 + k_row_in_chunk(l/16, i)), s0(c) = min(c C, KR - C) (C = kMfmaChunk, KR = npad / 4
    // >= C): each lane group reads its B rows in the order that keeps the global step's LDS
    // reads free of bank conflicts. A chunk is 512 words at word (rt KS + c C) 64: lane l's 8
    // hi values in words 4l..4l+3 (element i in half i % 2 of word 4l + i/2), then the lo
    // values in words 256 + 4l... The last chunk ends at the last row and overlaps the one
    // before it, so its rows below 4 c C are stored as zeros; the two chunks after the last
    // one are zero too (the kernel's look-ahead loads read them).
    const int RT = p.row_tiles, KS = p.k_steps, n = ct->n;
    const int KR = ct->npad / 4, C = kMfmaChunk, nch = (KR + C - 1) / C;
    auto tiles = [&](const std::vector<double>& dense, int32_t* exp_out) {
      double amax = 0.0;
      for (double a : dense) amax = std::max(amax, std::fabs(a));
      int ex = 0;
      if (amax > 0.0) std::frexp(amax, &ex);   // amax in [2^(ex-1), 2^ex)
      const int sh = amax > 0.0 ? 14 - ex : 0;
      *exp_out = sh;
      std::vector<uint16_t> halves((size_t)RT * KS * 64 * 2, 0);
      for (int rt = 0; rt < RT; ++rt)
        for (int c = 0; c < nch; ++c) {
          const int s0 = std::min(c * C, KR - C);
          uint16_t* chunk = halves.data() + ((size_t)rt * KS + (size_t)c * C) * 128;
          for (int l = 0; l < 64; ++l)
            for (int i = 0; i < C; ++i) {
              const int row = rt * 16 + (l & 15), kr = 4 * s0 + k_row_in_chunk(l >> 4, i);
              if (kr < 4 * c * C) continue;   // covered by the previous chunk
              if (row >= n || kr >= n) continue;
              const double a = std::ldexp(dense[(size_t)row * n + kr], sh);
              const _Float16 hi = (_Float16)a;
              const _Float16 lo = (_Float16)(a - (double)hi);
              std::memcpy(&chunk[8 * l + i], &hi, 2);
              std::memcpy(&chunk[512 + 8 * l + i], &lo, 2);
            }
        }
      return halves;
    };
    {
      const std::vector<uint16_t> t = tiles(ct->Linv, &p.linv_exp);
      chk(upload_raw(&d->linv_tiles, reinterpret_cast<const float*>(t.data()), t.size() / 2));
    }
    // Rayleigh damping with beta > 0: m M~^-1 in the same form, for the prediction
    if (!ct->pinv.empty()) {
      const std::vector<uint16_t> t = tiles(ct->pinv, &p.pinv_exp);
      chk(upload_raw(&d->pinv_tiles, reinterpret_cast<const float*>(t.data()), t.size() / 2));
    }
  }
  if (st != NPFEM_OK) {
    free_devtype(d);
    return st;
  }
  ct->dev[dev] = d;
  *out = d;
  return NPFEM_OK;
}

// The kernels' view of a cell type with layout li (fused form) on the current device.
npfem_status devtype_value(npfem_celltype* ct, int li, DevType* out) {
  DevType* base = nullptr;
  npfem_status st = upload_celltype(ct, &base);
  if (st != NPFEM_OK) return st;
  *out = *base;
  if (!ct->fused_ok) return NPFEM_OK;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(ct->mu);
  LayoutDev ld;
  st = layout_schedules_locked(ct, dev, li, &ld);
  if (st != NPFEM_OK) return st;
  out->tri_sched = ld.tri;
  out->hinge_sched = ld.hinge;
  out->gather_sched = ld.gather;
  const FusedLayout& lay = ct->layouts[li];
  out->p.gw = lay.gw;
  out->p.slots = lay.slots;
  out->p.tri_rounds = lay.tri_rounds;
  out->p.hinge_rounds = lay.hinge_rounds;
  out->p.gather_slots = lay.gather_slots;
  return NPFEM_OK;
}

}  // namespace npfem

using namespace npfem;

npfem_celltype::~npfem_celltype() {
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : dev) {
    (void)hipSetDevice(kv.first);
    free_devtype(kv.second);
  }
  for (auto& kv : dev_sched) {
    (void)hipSetDevice(kv.first);
    for (auto& p : kv.second) {
      if (p.tri) (void)hipFree(p.tri);
      if (p.hinge) (void)hipFree(p.hinge);
      if (p.gather) (void)hipFree(p.gather);
    }
  }
  (void)hipSetDevice(cur);
}

// A recorded sequence of steps (npfem_graph_create).
struct npfem_graph {
  int device = 0;
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  FusedGroup* d_groups = nullptr;   // the graph's own work list (fused form)
  int* d_count = nullptr;
  ~npfem_graph() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();   // replays may be in flight on any stream
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (capture) (void)hipStreamDestroy(capture);
    if (d_groups) (void)hipFree(d_groups);
    if (d_count) (void)hipFree(d_count);
    (void)hipSetDevice(cur);
  }
};

struct npfem_batch {
  int n_cells = 0, precision = 32, form = NPFEM_FORM_FUSED, device = 0;
  double dt = 0;
  std::vector<int64_t> offsets;
  std::vector<npfem_celltype*> types;
  std::vector<int> type_of;                 // per cell, index into types
  std::vector<int> layout_of;               // per type, index into its fused layouts
  std::vector<DevType*> dev_types;          // host pointers to per-type device copies
  DevType* d_types = nullptr;               // device array of DevType (by value)
  DevType** d_type_ptrs = nullptr;          // device pointers to each type's device DevType
  std::vector<DevType*> type_dev_structs;   // device DevType per type (plain form)
  // fused-form work lists: the list of all cells, plus a ring of two subset lists that
  // npfem_batch_set_active fills from pinned host staging; the kernel reads the group count
  // from device memory, so a captured step replays with whatever list is current
  FusedGroup* d_groups = nullptr;           // all cells
  int* d_count_all = nullptr;
  int n_groups = 0;                         // groups of the all-cells list (grid capacity)
  size_t list_capacity = 0;                 // groups the device lists can hold
  FusedGroup* d_ring[2] = {nullptr, nullptr};
  int* d_ring_count[2] = {nullptr, nullptr};
  FusedGroup* h_stage[2] = {nullptr, nullptr};
  int* h_stage_count[2] = {nullptr, nullptr};
  hipEvent_t ring_ev[2] = {nullptr, nullptr};
  int ring_cur = -1;                        // -1: the all-cells list is active
  std::vector<char> mark;
  int64_t* d_offsets = nullptr;
  int32_t* d_type_of = nullptr;             // per cell, index into types (device copy)
  int32_t* d_cells_by_type = nullptr;       // cell ids grouped by type (device)
  std::vector<int> type_first, type_count;  // each type's range in d_cells_by_type
  // median filter of the external forces: blocks of consecutive whole cells
  FilterBlock* d_filter_blocks = nullptr;
  int n_filter_blocks = 0;
  int filter_net = 8;                       // keys of the kernel's sorting network (8 or 16)
  size_t filter_lds = 0;
  std::string filter_reason;                // non-empty: the filter is unavailable
  size_t lds_bytes = 0;
  bool fused_extras = false;                // a type damps or caps velocities (kernel variant)
  bool fused_skalak = false;                // a type has the Skalak membrane (kernel variant)
  int solve_choice = -1;                    // NPFEM_SOLVE_AUTO's variant (-1: by form)
  void* work = nullptr;                     // plain-form workspace
  int* d_flag = nullptr;
  npfem::ContactWork contacts;              // contact detection workspace (first use)
  ~npfem_batch() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    if (d_types) (void)hipFree(d_types);
    for (DevType* p : type_dev_structs)
      if (p) (void)hipFree(p);
    if (d_groups) (void)hipFree(d_groups);
    if (d_count_all) (void)hipFree(d_count_all);
    for (int i = 0; i < 2; ++i) {
      if (ring_ev[i]) {
        (void)hipEventSynchronize(ring_ev[i]);
        (void)hipEventDestroy(ring_ev[i]);
      }
      if (d_ring[i]) (void)hipFree(d_ring[i]);
      if (d_ring_count[i]) (void)hipFree(d_ring_count[i]);
      if (h_stage[i]) (void)hipHostFree(h_stage[i]);
      if (h_stage_count[i]) (void)hipHostFree(h_stage_count[i]);
    }
    if (d_offsets) (void)hipFree(d_offsets);
    if (d_type_of) (void)hipFree(d_type_of);
    if (d_cells_by_type) (void)hipFree(d_cells_by_type);
    if (d_filter_blocks) (void)hipFree(d_filter_blocks);
    if (work) (void)hipFree(work);
    if (d_flag) (void)hipFree(d_flag);
    npfem::contact_work_free(contacts);
    (void)hipSetDevice(cur);
  }
};

namespace {

// Groups of up to 4*gw same-type cells, cells in the given order. Workgroups are dispatched
// in list order, so the types with the most vertices per cell (the longest groups) come first
// and the shorter groups fill the last, partial round of workgroups; equal sizes keep the
// types' order.
void build_groups(const npfem_batch* b, const int32_t* ids, int n, std::vector<FusedGroup>& out) {
  out.clear();
  const int nt = (int)b->types.size();
  std::vector<int> type_order(nt);
  for (int ti = 0; ti < nt; ++ti) type_order[ti] = ti;
  std::stable_sort(type_order.begin(), type_order.end(),
                   [&](int p, int q) { return b->types[p]->n > b->types[q]->n; });
  for (int ti : type_order) {
    const int cap = kFusedWaves * b->types[ti]->layouts[b->layout_of[ti]].gw;
    FusedGroup gcur{};
    gcur.type = ti;
    gcur.count = 0;
    for (int i = 0; i < n; ++i) {
      const int c = ids ? ids[i] : i;
      if (b->type_of[c] != ti) continue;
      gcur.cells[gcur.count++] = c;
      if (gcur.count == cap) {
        out.push_back(gcur);
        gcur.count = 0;
      }
    }
    if (gcur.count) out.push_back(gcur);
  }
}

void free_lists(npfem_batch* b) {
  if (b->d_groups) (void)hipFree(b->d_groups);
  b->d_groups = nullptr;
  for (int i = 0; i < 2; ++i) {
    if (b->ring_ev[i]) (void)hipEventSynchronize(b->ring_ev[i]);
    if (b->d_ring[i]) (void)hipFree(b->d_ring[i]);
    if (b->h_stage[i]) (void)hipHostFree(b->h_stage[i]);
    b->d_ring[i] = nullptr;
    b->h_stage[i] = nullptr;
  }
  b->list_capacity = 0;
}

// (Re)builds a fused-form batch's type table, all-cells work list, LDS size and list
// capacity for the types' current layouts and makes the all-cells list current. No step of
// the batch may be in flight.
npfem_status relayout(npfem_batch* b) {
  const int nt = (int)b->types.size();
  b->lds_bytes = 0;
  for (int ti = 0; ti < nt; ++ti) {
    npfem_celltype* t = b->types[ti];
    DevType v;
    npfem_status st = devtype_value(t, b->layout_of[ti], &v);
    if (st != NPFEM_OK) return st;
    HIP_TRY(hipMemcpy(b->d_types + ti, &v, sizeof(DevType), hipMemcpyHostToDevice));
    const int cap = kFusedWaves * t->layouts[b->layout_of[ti]].gw;
    // X blocks below kFusedRWords, R blocks from there, then the damping words
    const size_t per_cell = ((size_t)t->cs + (t->kappa > 0.0 ? kDampWords : 0)) * sizeof(float);
    b->lds_bytes = std::max(b->lds_bytes, kFusedRWords * sizeof(float) + (size_t)cap * per_cell);
  }
  std::vector<FusedGroup> groups;
  build_groups(b, nullptr, b->n_cells, groups);
  const size_t need = std::max<size_t>(groups.size(), 1);
  if (need > b->list_capacity) {
    free_lists(b);
    const size_t gbytes = need * sizeof(FusedGroup);
    if (hipMalloc((void**)&b->d_groups, gbytes) != hipSuccess)
      return fail(NPFEM_E_NOMEM, "device work list");
    for (int i = 0; i < 2; ++i)
      if (hipMalloc((void**)&b->d_ring[i], gbytes) != hipSuccess ||
          hipHostMalloc((void**)&b->h_stage[i], gbytes, hipHostMallocDefault) != hipSuccess)
        return fail(NPFEM_E_NOMEM, "active-list ring");
    b->list_capacity = need;
  }
  b->n_groups = (int)groups.size();
  if (b->n_groups)
    HIP_TRY(hipMemcpy(b->d_groups, groups.data(), groups.size() * sizeof(FusedGroup),
                      hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_count_all, &b->n_groups, sizeof(int), hipMemcpyHostToDevice));
  b->ring_cur = -1;
  return NPFEM_OK;
}

// Work list of the median filter: consecutive whole cells per block, at most kFilterMaxCells
// cells and kFilterMaxVerts vertices unless one cell alone is larger. The block's forces (and a
// list of its wide-ring vertices) are staged in LDS, so the largest block must fit in 64 KiB;
// otherwise the filter is unavailable for the batch, which the filter call reports. The
// network width is 8 keys (degree <= 7) when at most 1/32 of the vertices have wider closed
// rings, else 16; wider rings go to the kernel's rank-selection pass.
npfem_status build_filter_blocks(npfem_batch* b) {
  const int nt = (int)b->types.size();
  auto wide_count = [&](int ti, int keys) {
    int64_t w = 0;
    for (uint32_t info : b->types[ti]->ring_info) w += (int)(info & 255u) + 1 > keys;
    return w;
  };
  int64_t wide8 = 0;
  for (int c = 0; c < b->n_cells; ++c) wide8 += wide_count(b->type_of[c], 8);
  b->filter_net = 32 * wide8 <= b->offsets.back() ? 8 : 16;
  std::vector<int64_t> wide_of(nt);
  for (int ti = 0; ti < nt; ++ti) wide_of[ti] = wide_count(ti, b->filter_net);
  std::vector<FilterBlock> blocks;
  int64_t max_recs = 0, max_wide = 1;
  for (int c = 0; c < b->n_cells;) {
    FilterBlock blk{};
    blk.v0 = b->offsets[c];
    int64_t nv = 0, wide = 0;
    while (c < b->n_cells && blk.count < kFilterMaxCells) {
      const int64_t n = b->offsets[c + 1] - b->offsets[c];
      if (blk.count > 0 && nv + n > kFilterMaxVerts) break;
      blk.start[blk.count] = (int32_t)nv;
      blk.type[blk.count] = (int16_t)b->type_of[c];
      const DevType* dt = b->dev_types[b->type_of[c]];
      blk.nb[blk.count] = b->filter_net == 8 ? dt->ring_nb8 : dt->ring_nb16;
      nv += n;
      wide += wide_of[b->type_of[c]];
      ++blk.count;
      ++c;
    }
    blk.start[blk.count] = (int32_t)nv;
    blk.nv = (int32_t)nv;
    max_recs = std::max(max_recs, nv + 2 * blk.count);
    max_wide = std::max(max_wide, wide);
    blocks.push_back(blk);
  }
  // LDS: one record of 4 values per vertex plus two pad records (-inf, +inf) per cell, then
  // the list of wide-ring vertices
  const size_t el = b->precision == 64 ? 8 : 4;
  b->filter_lds = 4 * el * (size_t)max_recs + sizeof(int) * (size_t)max_wide;
  b->n_filter_blocks = (int)blocks.size();
  if (nt > 32767) b->filter_reason = "median filter: more than 32767 cell types";
  else if (b->filter_lds > 65536)
    b->filter_reason = "median filter: a cell's forces exceed 64 KiB of LDS";
  if (b->n_cells == 0) return NPFEM_OK;
  HIP_TRY(hipMalloc((void**)&b->d_filter_blocks, blocks.size() * sizeof(FilterBlock)));
  HIP_TRY(hipMemcpy(b->d_filter_blocks, blocks.data(), blocks.size() * sizeof(FilterBlock),
                    hipMemcpyHostToDevice));
  return NPFEM_OK;
}

}  // namespace

extern "C" {

const char* npfem_last_error(void) { return g_last_error.c_str(); }

npfem_status npfem_create_celltype(const npfem_mesh* mesh, const npfem_material* material,
                                   double dt, npfem_celltype** out) {
  if (!out) return fail(NPFEM_E_INVALID, "out is null");
  *out = nullptr;
  npfem_celltype* ct = new (std::nothrow) npfem_celltype();
  if (!ct) return fail(NPFEM_E_NOMEM, "host allocation");
  npfem_status s;
  try {
    s = build_celltype(mesh, material, dt, ct);
  } catch (const std::bad_alloc&) {
    s = fail(NPFEM_E_NOMEM, "host allocation during setup");
  }
  if (s != NPFEM_OK) {
    delete ct;
    return s;
  }
  *out = ct;
  g_last_error.clear();
  return NPFEM_OK;
}

void npfem_celltype_destroy(npfem_celltype* type) { delete type; }

npfem_status npfem_celltype_get_info(const npfem_celltype* t, npfem_celltype_info* out) {
  if (!t || !out) return fail(NPFEM_E_INVALID, "null argument");
  out->n_vertices = t->n;
  out->n_triangles = t->m;
  out->n_hinges = t->e;
  out->bandwidth = t->bw;
  out->rest_volume = t->V0;
  out->rest_area = t->area0;
  out->vertex_mass = t->mass;
  out->dt = t->h;
  out->tri_rounds = t->tri_rounds;
  out->hinge_rounds = t->hinge_rounds;
  return NPFEM_OK;
}

npfem_status npfem_celltype_get_matrix(const npfem_celltype* t, double* L_out) {
  if (!t || !L_out) return fail(NPFEM_E_INVALID, "null argument");
  std::memcpy(L_out, t->L.data(), t->L.size() * sizeof(double));
  return NPFEM_OK;
}

npfem_status npfem_batch_create(int32_t n_cells, npfem_celltype* const* type_of_cell,
                                int32_t precision, int32_t form, npfem_batch** out,
                                int64_t* vertex_offsets) {
  if (!out) return fail(NPFEM_E_INVALID, "out is null");
  *out = nullptr;
  if (n_cells < 0 || (n_cells > 0 && !type_of_cell)) return fail(NPFEM_E_INVALID, "bad cell list");
  if (precision != 32 && precision != 64) return fail(NPFEM_E_INVALID, "precision must be 32 or 64");
  if (form != NPFEM_FORM_PLAIN && form != NPFEM_FORM_FUSED) return fail(NPFEM_E_INVALID, "unknown form");
  if (form == NPFEM_FORM_FUSED && precision != 32)
    return fail(NPFEM_E_UNSUPPORTED, "the fused form computes in FP32");
  npfem_batch* b = new (std::nothrow) npfem_batch();
  if (!b) return fail(NPFEM_E_NOMEM, "host allocation");
  b->n_cells = n_cells;
  b->precision = precision;
  b->form = form;
  auto bail = [&](npfem_status s) { delete b; return s; };
  if (hipGetDevice(&b->device) != hipSuccess) return bail(fail(NPFEM_E_HIP, "hipGetDevice failed"));
  b->offsets.assign(n_cells + 1, 0);
  b->type_of.resize(n_cells);
  for (int c = 0; c < n_cells; ++c) {
    npfem_celltype* t = type_of_cell[c];
    if (!t) return bail(fail(NPFEM_E_INVALID, "null cell type"));
    auto it = std::find(b->types.begin(), b->types.end(), t);
    if (it == b->types.end()) {
      b->types.push_back(t);
      b->type_of[c] = (int)b->types.size() - 1;
    } else {
      b->type_of[c] = (int)(it - b->types.begin());
    }
    b->offsets[c + 1] = b->offsets[c] + t->n;
  }
  for (npfem_celltype* t : b->types) {
    b->fused_extras = b->fused_extras || t->kappa > 0.0 || t->v_max > 0.0 || t->beta > 0.0;
    b->fused_skalak = b->fused_skalak || t->membrane == NPFEM_MEMBRANE_SKALAK;
    if (b->dt == 0) b->dt = t->h;
    if (std::fabs(t->h - b->dt) > 1e-12 * b->dt)
      return bail(fail(NPFEM_E_DT, "cell types of one batch must share dt"));
    if (form == NPFEM_FORM_FUSED && !t->fused_ok)
      return bail(fail(NPFEM_E_UNSUPPORTED, t->fused_reason));
    if (form == NPFEM_FORM_PLAIN && !plain_supported(t->n, t->bw))
      return bail(fail(NPFEM_E_UNSUPPORTED, "plain form supports n <= 1024"));
    DevType* d = nullptr;
    npfem_status s = upload_celltype(t, &d);
    if (s != NPFEM_OK) return bail(s);
    b->dev_types.push_back(d);
  }
  if (vertex_offsets) std::memcpy(vertex_offsets, b->offsets.data(), (n_cells + 1) * sizeof(int64_t));

  const int nt = (int)b->types.size();
  if (hipMalloc((void**)&b->d_flag, sizeof(int)) != hipSuccess ||
      hipMemset(b->d_flag, 0, sizeof(int)) != hipSuccess)
    return bail(fail(NPFEM_E_NOMEM, "device flag"));
  if (nt > 0) {
    if (hipMalloc((void**)&b->d_types, nt * sizeof(DevType)) != hipSuccess)
      return bail(fail(NPFEM_E_NOMEM, "device type table"));
    for (int i = 0; i < nt; ++i)
      if (hipMemcpy(b->d_types + i, b->dev_types[i], sizeof(DevType), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(NPFEM_E_HIP, "type table copy"));
  }
  if (hipMalloc((void**)&b->d_offsets, (n_cells + 1) * sizeof(int64_t)) != hipSuccess ||
      hipMemcpy(b->d_offsets, b->offsets.data(), (n_cells + 1) * sizeof(int64_t),
                hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(NPFEM_E_NOMEM, "device offsets"));
  {
    std::vector<int32_t> type_of(b->type_of.begin(), b->type_of.end());
    std::vector<int32_t> by_type;
    by_type.reserve(n_cells);
    for (int ti = 0; ti < nt; ++ti) {
      b->type_first.push_back((int)by_type.size());
      for (int c = 0; c < n_cells; ++c)
        if (b->type_of[c] == ti) by_type.push_back(c);
      b->type_count.push_back((int)by_type.size() - b->type_first.back());
    }
    const size_t cb = std::max<size_t>(n_cells, 1) * sizeof(int32_t);
    if (hipMalloc((void**)&b->d_type_of, cb) != hipSuccess ||
        hipMalloc((void**)&b->d_cells_by_type, cb) != hipSuccess ||
        (n_cells > 0 && (hipMemcpy(b->d_type_of, type_of.data(), type_of.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice) != hipSuccess ||
                         hipMemcpy(b->d_cells_by_type, by_type.data(),
                                   by_type.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)))
      return bail(fail(NPFEM_E_NOMEM, "device cell types"));
  }
  {
    const npfem_status st = build_filter_blocks(b);
    if (st != NPFEM_OK) return bail(st);
  }
  if (form == NPFEM_FORM_PLAIN) {
    size_t wb = 0;
    for (npfem_celltype* t : b->types) wb = std::max(wb, plain_work_bytes(precision, t->n, t->m, t->e));
    if (wb && hipMalloc(&b->work, wb) != hipSuccess) return bail(fail(NPFEM_E_NOMEM, "plain workspace"));
  } else {
    b->layout_of.assign(nt, 0);
    if (hipMalloc((void**)&b->d_count_all, sizeof(int)) != hipSuccess)
      return bail(fail(NPFEM_E_NOMEM, "device work list"));
    for (int i = 0; i < 2; ++i)
      if (hipMalloc((void**)&b->d_ring_count[i], sizeof(int)) != hipSuccess ||
          hipHostMalloc((void**)&b->h_stage_count[i], sizeof(int), hipHostMallocDefault) != hipSuccess ||
          hipEventCreateWithFlags(&b->ring_ev[i], hipEventDisableTiming) != hipSuccess)
        return bail(fail(NPFEM_E_NOMEM, "active-list ring"));
    const npfem_status st = relayout(b);
    if (st != NPFEM_OK) return bail(st);
    b->mark.assign(n_cells, 0);
  }
  *out = b;
  g_last_error.clear();
  return NPFEM_OK;
}

void npfem_batch_destroy(npfem_batch* batch) { delete batch; }

int64_t npfem_batch_vertex_count(const npfem_batch* b) { return b ? b->offsets.back() : -1; }

}  // extern "C"

namespace {

// Makes `device` current for the guard's scope.
struct DeviceGuard {
  int prev = 0;
  explicit DeviceGuard(int device) {
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

npfem_status step_fused(npfem_batch* b, const FusedGroup* groups, const int* count, void* x,
                        void* v, const void* f, int32_t n_pd_iters, void* stream,
                        double* cell_volume_area, const void* cp = nullptr,
                        const void* cw = nullptr) {
  hipError_t e = launch_fused_step(b->d_types, (int)b->types.size(), groups, count, b->n_groups,
                                   b->d_offsets, b->offsets.back(), (float*)x, (float*)v,
                                   (const float*)f, (const float*)cp, (const float*)cw, n_pd_iters,
                                   cell_volume_area, b->d_flag, b->lds_bytes, b->fused_extras,
                                   b->fused_skalak,
                                   stream);
  if (e != hipSuccess) return fail(NPFEM_E_HIP, std::string("fused launch: ") + hipGetErrorString(e));
  return NPFEM_OK;
}

}  // namespace

extern "C" {

npfem_status npfem_step(npfem_batch* b, void* x, void* v, const void* f, double dt,
                        int32_t n_pd_iters, void* stream, double* cell_volume_area) {
  return npfem_step_contacts(b, x, v, f, dt, n_pd_iters, stream, cell_volume_area, nullptr,
                             nullptr);
}

npfem_status npfem_step_contacts(npfem_batch* b, void* x, void* v, const void* f, double dt,
                                 int32_t n_pd_iters, void* stream, double* cell_volume_area,
                                 const void* contact_p, const void* contact_w) {
  if (!b) return fail(NPFEM_E_INVALID, "batch is null");
  if (b->n_cells == 0) return NPFEM_OK;
  if (!x || !v || !f) return fail(NPFEM_E_INVALID, "null state or force buffer");
  if ((contact_p == nullptr) != (contact_w == nullptr))
    return fail(NPFEM_E_INVALID, "contact points and weights go together");
  if (n_pd_iters < 0) return fail(NPFEM_E_INVALID, "n_pd_iters < 0");
  if (!(std::fabs(dt - b->dt) <= 1e-12 * b->dt))
    return fail(NPFEM_E_DT, "dt differs from the cell types' factorised dt");
  const int64_t vtot = b->offsets.back();
  if (b->form == NPFEM_FORM_PLAIN) {
    const size_t el = b->precision == 64 ? 8 : 4;
    (void)el;
    for (int c = 0; c < b->n_cells; ++c) {
      const int ti = b->type_of[c];
      hipError_t e = launch_plain_cell(b->precision, b->d_types + ti, b->dev_types[ti]->p, x, v, f,
                                       contact_p, contact_w, vtot, b->offsets[c], n_pd_iters, b->work,
                                       cell_volume_area ? cell_volume_area + 2 * (int64_t)c : nullptr,
                                       b->d_flag, stream);
      if (e != hipSuccess) return fail(NPFEM_E_HIP, std::string("plain launch: ") + hipGetErrorString(e));
    }
    return NPFEM_OK;
  }
  const FusedGroup* groups = b->ring_cur < 0 ? b->d_groups : b->d_ring[b->ring_cur];
  const int* count = b->ring_cur < 0 ? b->d_count_all : b->d_ring_count[b->ring_cur];
  return step_fused(b, groups, count, x, v, f, n_pd_iters, stream, cell_volume_area, contact_p,
                    contact_w);
}

npfem_status npfem_batch_set_active(npfem_batch* b, const int32_t* cell_ids, int32_t n,
                                    void* stream) {
  if (!b) return fail(NPFEM_E_INVALID, "batch is null");
  if (b->form != NPFEM_FORM_FUSED)
    return fail(NPFEM_E_UNSUPPORTED, "active-cell lists need the fused form");
  if (!cell_ids || n < 0) {
    b->ring_cur = -1;
    return NPFEM_OK;
  }
  for (int i = 0; i < n; ++i) {
    const int c = cell_ids[i];
    if (c < 0 || c >= b->n_cells || b->mark[c]) {
      for (int j = 0; j < i; ++j) b->mark[cell_ids[j]] = 0;
      return fail(NPFEM_E_INVALID, "cell id out of range or repeated");
    }
    b->mark[c] = 1;
  }
  for (int i = 0; i < n; ++i) b->mark[cell_ids[i]] = 0;
  const int slot = b->ring_cur < 0 ? 0 : (b->ring_cur + 1) % 2;
  HIP_TRY(hipEventSynchronize(b->ring_ev[slot]));   // staging of this slot is free again
  std::vector<FusedGroup> groups;
  build_groups(b, cell_ids, n, groups);
  std::memcpy(b->h_stage[slot], groups.data(), groups.size() * sizeof(FusedGroup));
  *b->h_stage_count[slot] = (int)groups.size();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!groups.empty())
    HIP_TRY(hipMemcpyAsync(b->d_ring[slot], b->h_stage[slot], groups.size() * sizeof(FusedGroup),
                           hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b->d_ring_count[slot], b->h_stage_count[slot], sizeof(int),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(b->ring_ev[slot], s));
  b->ring_cur = slot;
  return NPFEM_OK;
}

npfem_status npfem_graph_create(npfem_batch* b, void* x, void* v, const void* const* f,
                                int32_t n_steps, double dt, int32_t n_pd_iters,
                                double* cell_volume_area, npfem_graph** out) {
  if (!out) return fail(NPFEM_E_INVALID, "out is null");
  *out = nullptr;
  if (!b || !x || !v || !f) return fail(NPFEM_E_INVALID, "null batch, state or force list");
  if (n_steps < 1) return fail(NPFEM_E_INVALID, "n_steps < 1");
  if (n_pd_iters < 0) return fail(NPFEM_E_INVALID, "n_pd_iters < 0");
  for (int s = 0; s < n_steps; ++s)
    if (!f[s]) return fail(NPFEM_E_INVALID, "null force buffer");
  if (!(std::fabs(dt - b->dt) <= 1e-12 * b->dt))
    return fail(NPFEM_E_DT, "dt differs from the cell types' factorised dt");
  DeviceGuard guard(b->device);
  npfem_graph* g = new (std::nothrow) npfem_graph();
  if (!g) return fail(NPFEM_E_NOMEM, "host allocation");
  g->device = b->device;
  auto bail = [&](npfem_status st) { delete g; return st; };
  const FusedGroup* groups = nullptr;
  const int* count = nullptr;
  if (b->form == NPFEM_FORM_FUSED && b->n_cells > 0) {
    // the graph's own copy of the current work list (group count included)
    const FusedGroup* src = b->ring_cur < 0 ? b->d_groups : b->d_ring[b->ring_cur];
    const int* src_count = b->ring_cur < 0 ? b->d_count_all : b->d_ring_count[b->ring_cur];
    const size_t gbytes = std::max<size_t>(b->n_groups, 1) * sizeof(FusedGroup);
    if (hipMalloc((void**)&g->d_groups, gbytes) != hipSuccess ||
        hipMalloc((void**)&g->d_count, sizeof(int)) != hipSuccess)
      return bail(fail(NPFEM_E_NOMEM, "graph work list"));
    // the source list may have been filled asynchronously: order the copies after it
    if (b->ring_cur >= 0 && hipEventSynchronize(b->ring_ev[b->ring_cur]) != hipSuccess)
      return bail(fail(NPFEM_E_HIP, "active-list event"));
    if (hipMemcpy(g->d_groups, src, gbytes, hipMemcpyDeviceToDevice) != hipSuccess ||
        hipMemcpy(g->d_count, src_count, sizeof(int), hipMemcpyDeviceToDevice) != hipSuccess)
      return bail(fail(NPFEM_E_HIP, "graph work list copy"));
    groups = g->d_groups;
    count = g->d_count;
  }
  if (hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(NPFEM_E_HIP, "capture stream"));
  if (hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return bail(fail(NPFEM_E_HIP, "begin capture"));
  npfem_status st = NPFEM_OK;
  for (int s = 0; s < n_steps && st == NPFEM_OK; ++s) {
    if (b->n_cells == 0) break;
    if (b->form == NPFEM_FORM_FUSED)
      st = step_fused(b, groups, count, x, v, f[s], n_pd_iters, g->capture, cell_volume_area);
    else
      st = npfem_step(b, x, v, f[s], dt, n_pd_iters, g->capture, cell_volume_area);
  }
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(g->capture, &graph);
  if (st != NPFEM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return bail(st);
  }
  if (ec != hipSuccess || !graph) return bail(fail(NPFEM_E_HIP, "end capture"));
  g->graph = graph;
  if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess)
    return bail(fail(NPFEM_E_HIP, "graph instantiate"));
  *out = g;
  g_last_error.clear();
  return NPFEM_OK;
}

npfem_status npfem_graph_launch(npfem_graph* g, void* stream) {
  if (!g || !g->exec) return fail(NPFEM_E_INVALID, "graph is null");
  HIP_TRY(hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream)));
  return NPFEM_OK;
}

void npfem_graph_destroy(npfem_graph* g) { delete g; }

int32_t npfem_celltype_cells_per_wave(const npfem_celltype* t, int32_t* out, int32_t max_out) {
  if (!t) return fail(NPFEM_E_INVALID, "type is null");
  const int n = (int)t->layouts.size();
  for (int i = 0; i < n && i < max_out; ++i)
    if (out) out[i] = t->layouts[i].gw;
  return n;
}

}  // extern "C"

namespace {

// Index of `type` among the batch's types, or -1.
int batch_type_index(const npfem_batch* b, const npfem_celltype* type) {
  for (size_t i = 0; i < b->types.size(); ++i)
    if (b->types[i] == type) return (int)i;
  return -1;
}

}  // namespace

extern "C" {

npfem_status npfem_batch_get_cells_per_wave(const npfem_batch* b, const npfem_celltype* type,
                                            int32_t* cells_per_wave) {
  if (!b || !type || !cells_per_wave) return fail(NPFEM_E_INVALID, "null argument");
  if (b->form != NPFEM_FORM_FUSED) return fail(NPFEM_E_UNSUPPORTED, "plain-form batch");
  const int ti = batch_type_index(b, type);
  if (ti < 0) return fail(NPFEM_E_INVALID, "type is not in the batch");
  *cells_per_wave = b->types[ti]->layouts[b->layout_of[ti]].gw;
  return NPFEM_OK;
}

npfem_status npfem_batch_set_cells_per_wave(npfem_batch* b, const npfem_celltype* type,
                                            int32_t cells_per_wave) {
  if (!b || !type) return fail(NPFEM_E_INVALID, "null argument");
  if (b->form != NPFEM_FORM_FUSED) return fail(NPFEM_E_UNSUPPORTED, "plain-form batch");
  const int ti = batch_type_index(b, type);
  if (ti < 0) return fail(NPFEM_E_INVALID, "type is not in the batch");
  const auto& lays = b->types[ti]->layouts;
  int li = -1;
  for (size_t i = 0; i < lays.size(); ++i)
    if (lays[i].gw == cells_per_wave) li = (int)i;
  if (li < 0) return fail(NPFEM_E_UNSUPPORTED, "cells_per_wave is not a layout of this type");
  DeviceGuard guard(b->device);
  HIP_TRY(hipDeviceSynchronize());   // the batch's lists may be in use by enqueued steps
  b->layout_of[ti] = li;
  return relayout(b);
}

npfem_status npfem_batch_autotune(npfem_batch* b, int32_t n_pd_iters, int32_t reps, void* stream) {
  if (!b) return fail(NPFEM_E_INVALID, "batch is null");
  if (b->form != NPFEM_FORM_FUSED) return fail(NPFEM_E_UNSUPPORTED, "plain-form batch");
  if (n_pd_iters < 1 || reps < 1) return fail(NPFEM_E_INVALID, "n_pd_iters and reps must be >= 1");
  if (b->n_cells == 0) return NPFEM_OK;
  DeviceGuard guard(b->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(hipDeviceSynchronize());
  // scratch state: every cell at its rest shape, at rest, under small pseudo-random forces
  const int64_t vt = b->offsets.back();
  std::vector<float> hx((size_t)3 * vt), hf((size_t)3 * vt);
  uint64_t rng = 0x9e3779b97f4a7c15ull;
  for (int c = 0; c < b->n_cells; ++c) {
    const npfem_celltype* t = b->types[b->type_of[c]];
    for (int i = 0; i < t->n; ++i)
      for (int d = 0; d < 3; ++d) {
        hx[(size_t)d * vt + b->offsets[c] + i] = (float)t->X[3 * i + d];
        rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;   // xorshift64
        hf[(size_t)d * vt + b->offsets[c] + i] = (float)((double)(rng >> 11) * 0x1.0p-53 - 0.5);
      }
  }
  float *x = nullptr, *v = nullptr, *f = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (x) (void)hipFree(x);
    if (v) (void)hipFree(v);
    if (f) (void)hipFree(f);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  const size_t bytes = (size_t)3 * vt * sizeof(float);
  if (hipMalloc((void**)&x, bytes) != hipSuccess || hipMalloc((void**)&v, bytes) != hipSuccess ||
      hipMalloc((void**)&f, bytes) != hipSuccess) {
    cleanup();
    return fail(NPFEM_E_NOMEM, "autotune scratch state");
  }
  if (hipMemcpy(x, hx.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(f, hf.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(v, 0, bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(NPFEM_E_HIP, "autotune setup");
  }
  npfem_status st = NPFEM_OK;
  for (int ti = 0; ti < (int)b->types.size() && st == NPFEM_OK; ++ti) {
    const int n_lay = (int)b->types[ti]->layouts.size();
    if (n_lay < 2) continue;
    std::vector<int32_t> ids;
    for (int c = 0; c < b->n_cells; ++c)
      if (b->type_of[c] == ti) ids.push_back(c);
    int best = b->layout_of[ti];
    float best_ms = 0.0f;
    for (int li = 0; li < n_lay && st == NPFEM_OK; ++li) {
      b->layout_of[ti] = li;
      st = relayout(b);
      if (st == NPFEM_OK) st = npfem_batch_set_active(b, ids.data(), (int32_t)ids.size(), stream);
      if (st == NPFEM_OK) st = npfem_step(b, x, v, f, b->dt, n_pd_iters, stream, nullptr);  // warm-up
      if (st != NPFEM_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) { st = fail(NPFEM_E_HIP, "event"); break; }
      for (int r = 0; r < reps && st == NPFEM_OK; ++r)
        st = npfem_step(b, x, v, f, b->dt, n_pd_iters, stream, nullptr);
      float ms = 0.0f;
      if (st == NPFEM_OK && (hipEventRecord(e1, s) != hipSuccess ||
                             hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = fail(NPFEM_E_HIP, "autotune timing");
      if (st == NPFEM_OK && (li == 0 || ms < best_ms)) {
        best = li;
        best_ms = ms;
      }
    }
    b->layout_of[ti] = best;
  }
  (void)hipStreamSynchronize(s);
  // the scratch steps may have set the non-finite flag: clear it, then restore all cells
  (void)hipMemset(b->d_flag, 0, sizeof(int));
  npfem_status st2 = relayout(b);
  // the global step alone (npfem_global_solve with NPFEM_SOLVE_AUTO): time both variants on
  // the whole batch with the chosen layouts, the scratch forces as right-hand sides
  if (st == NPFEM_OK && st2 == NPFEM_OK) {
    // every variant the batch supports (the matrix-core form needs a fused batch, the banded
    // one band widths up to 65); the fastest becomes NPFEM_SOLVE_AUTO's
    int best = -1;
    float best_ms = 0.0f;
    for (int variant : {NPFEM_SOLVE_DENSE, NPFEM_SOLVE_BANDED, NPFEM_SOLVE_GEMV}) {
      if (st != NPFEM_OK) break;
      if (variant == NPFEM_SOLVE_DENSE && b->form != NPFEM_FORM_FUSED) continue;
      npfem_status sv = npfem_global_solve(b, variant, f, v, stream);   // warm-up
      if (sv == NPFEM_E_UNSUPPORTED) {
        g_last_error.clear();
        continue;
      }
      st = sv;
      float ms = 0.0f;
      if (st == NPFEM_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(NPFEM_E_HIP, "event");
      for (int r = 0; r < reps && st == NPFEM_OK; ++r) st = npfem_global_solve(b, variant, f, v, stream);
      if (st == NPFEM_OK && (hipEventRecord(e1, s) != hipSuccess ||
                             hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = fail(NPFEM_E_HIP, "autotune timing");
      if (st == NPFEM_OK && (best < 0 || ms < best_ms)) {
        best = variant;
        best_ms = ms;
      }
    }
    if (st == NPFEM_OK && best >= 0) b->solve_choice = best;
  }
  (void)hipStreamSynchronize(s);
  cleanup();
  if (st != NPFEM_OK) return st;
  if (st2 == NPFEM_OK) g_last_error.clear();
  return st2;
}

npfem_status npfem_filter_forces(npfem_batch* b, const void* f_in, void* f_out, void* stream) {
  if (!b) return fail(NPFEM_E_INVALID, "batch is null");
  if (b->n_cells == 0) return NPFEM_OK;
  if (!f_in || !f_out) return fail(NPFEM_E_INVALID, "null force buffer");
  if (!b->filter_reason.empty()) return fail(NPFEM_E_UNSUPPORTED, b->filter_reason);
  DeviceGuard guard(b->device);
  const hipError_t e = launch_median_filter(b->precision, b->filter_net, b->d_types,
                                            b->d_filter_blocks, b->n_filter_blocks,
                                            b->offsets.back(), f_in, f_out, b->filter_lds, stream);
  if (e != hipSuccess) return fail(NPFEM_E_HIP, std::string("median filter launch: ") + hipGetErrorString(e));
  return NPFEM_OK;
}

// Vertex indices of the detection records are int32 and its bucket table (2^k >= 2 V
// buckets, uint32 counts) is scanned as one int-sized range.
constexpr int64_t kMaxContactVertices = int64_t(1) << 29;

npfem_status npfem_detect_contacts(npfem_batch* b, const void* x, double radius,
                                   double separation, double weight, void* contact_p,
                                   void* contact_w, void* stream) {
  if (!b) return fail(NPFEM_E_INVALID, "batch is null");
  if (!(radius > 0.0) || !std::isfinite(radius))
    return fail(NPFEM_E_INVALID, "radius must be finite and > 0");
  if (!(separation >= 0.0) || !std::isfinite(separation))
    return fail(NPFEM_E_INVALID, "separation must be finite and >= 0");
  if (!(weight >= 0.0) || !std::isfinite(weight))
    return fail(NPFEM_E_INVALID, "weight must be finite and >= 0");
  if (b->n_cells == 0) return NPFEM_OK;
  if (!x || !contact_p || !contact_w) return fail(NPFEM_E_INVALID, "null buffer");
  if (b->offsets.back() > kMaxContactVertices)
    return fail(NPFEM_E_UNSUPPORTED, "contact detection handles at most 2^29 vertices per batch");
  DeviceGuard guard(b->device);
  npfem::ContactWork& w = b->contacts;
  if (w.n_vertices == 0) {
    const int64_t V = b->offsets.back();
    if (npfem::contact_work_alloc(w, V, b->n_cells) != hipSuccess)
      return fail(NPFEM_E_NOMEM, "contact detection workspace");
    std::vector<int32_t> cell_of((size_t)V), type_of((size_t)b->n_cells);
    for (int c = 0; c < b->n_cells; ++c) {
      type_of[c] = b->type_of[c];
      for (int64_t i = b->offsets[c]; i < b->offsets[c + 1]; ++i) cell_of[(size_t)i] = c;
    }
    hipError_t e = hipMemcpy(w.cell_of, cell_of.data(), sizeof(int32_t) * cell_of.size(),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(w.type_of, type_of.data(), sizeof(int32_t) * type_of.size(),
                    hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      npfem::contact_work_free(w);
      return fail(NPFEM_E_HIP, std::string("contact tables: ") + hipGetErrorString(e));
    }
  }
  const hipError_t e = npfem::launch_detect_contacts(b->precision, b->d_types, b->d_offsets, w, x,
                                                     radius, separation, weight, contact_p,
                                                     contact_w, stream);
  if (e != hipSuccess) return fail(NPFEM_E_HIP, std::string("contact detection: ") + hipGetErrorString(e));
  return NPFEM_OK;
}

npfem_status npfem_detect_contacts_noalloc(npfem_batch* b, const void* x, double radius,
                                           double separation, double weight, void* contact_p,
                                           void* contact_w, void* stream) {
  if (!b) return fail(NPFEM_E_INVALID, "batch is null");
  if (!(radius > 0.0) || !std::isfinite(radius))
    return fail(NPFEM_E_INVALID, "radius must be finite and > 0");
  if (!(separation >= 0.0) || !std::isfinite(separation))
    return fail(NPFEM_E_INVALID, "separation must be finite and >= 0");
  if (!(weight >= 0.0) || !std::isfinite(weight))
    return fail(NPFEM_E_INVALID, "weight must be finite and >= 0");
  if (b->n_cells == 0) return NPFEM_OK;
  if (!x || !contact_p || !contact_w) return fail(NPFEM_E_INVALID, "null buffer");
  const int64_t V = b->offsets.back();
  if (V > npfem::kNoAllocMaxVertices)
    return fail(NPFEM_E_UNSUPPORTED, "npfem_detect_contacts_noalloc handles at most " +
                                         std::to_string(npfem::kNoAllocMaxVertices) +
                                         " vertices per batch (its static workspace is " +
                                         std::to_string(npfem::kContactScratchBytes >> 20) + " MiB)");
  const size_t need = npfem::contact_noalloc_bytes(V);
  if (need == 0 || need > npfem::kContactScratchBytes)
    return fail(NPFEM_E_UNSUPPORTED, "the static contact workspace is too small for this batch");
  DeviceGuard guard(b->device);
  const hipError_t e = npfem::launch_detect_contacts_noalloc(
      b->precision, b->d_types, b->d_offsets, b->n_cells, b->d_type_of, V, x, radius, separation,
      weight, contact_p, contact_w, stream);
  if (e != hipSuccess) return fail(NPFEM_E_HIP, std::string("contact detection: ") + hipGetErrorString(e));
  return NPFEM_OK;
}

npfem_status npfem_global_solve(npfem_batch* b, int32_t solve, const void* rhs, void* out,
                                void* stream) {
  if (!b) return fail(NPFEM_E_INVALID, "batch is null");
  if (solve != NPFEM_SOLVE_DENSE && solve != NPFEM_SOLVE_BANDED && solve != NPFEM_SOLVE_AUTO &&
      solve != NPFEM_SOLVE_GEMV)
    return fail(NPFEM_E_INVALID, "unknown global-step variant");
  if (solve == NPFEM_SOLVE_AUTO)
    solve = b->solve_choice >= 0 ? b->solve_choice
                                 : (b->form == NPFEM_FORM_FUSED ? NPFEM_SOLVE_DENSE : NPFEM_SOLVE_BANDED);
  if (b->n_cells == 0) return NPFEM_OK;
  if (!rhs || !out) return fail(NPFEM_E_INVALID, "null buffer");
  DeviceGuard guard(b->device);
  const int64_t V = b->offsets.back();
  const int nt = (int)b->types.size();
  if (solve == NPFEM_SOLVE_DENSE) {
    if (b->form != NPFEM_FORM_FUSED)
      return fail(NPFEM_E_UNSUPPORTED, "the dense global step needs a fused-form batch (FP32 L^-1)");
    for (int ti = 0; ti < nt; ++ti) {
      const hipError_t e = launch_global_dense_wide(b->d_types + ti, b->types[ti]->cs,
                                                    b->d_cells_by_type + b->type_first[ti], b->type_count[ti],
                                                    b->d_offsets, V, static_cast<const float*>(rhs),
                                                    static_cast<float*>(out), stream);
      if (e != hipSuccess) return fail(NPFEM_E_HIP, std::string("dense global step: ") + hipGetErrorString(e));
    }
    return NPFEM_OK;
  }
  if (solve == NPFEM_SOLVE_GEMV) {
    for (int ti = 0; ti < nt; ++ti) {
      const hipError_t e = launch_global_gemv(b->precision, b->dev_types[ti]->p.n, b->d_types + ti,
                                              b->d_cells_by_type + b->type_first[ti], b->type_count[ti],
                                              b->d_offsets, V, rhs, out, stream);
      if (e == hipErrorInvalidValue)
        return fail(NPFEM_E_UNSUPPORTED, "the dense vector global step stages at most 64 KiB per workgroup");
      if (e != hipSuccess) return fail(NPFEM_E_HIP, std::string("dense vector global step: ") + hipGetErrorString(e));
    }
    return NPFEM_OK;
  }
  for (int ti = 0; ti < nt; ++ti)
    if (b->dev_types[ti]->p.band_w == 0)
      return fail(NPFEM_E_UNSUPPORTED, "the banded global step handles band widths up to 65");
  for (int ti = 0; ti < nt; ++ti) {
    const hipError_t e = launch_global_banded(b->precision, b->dev_types[ti]->p.n,
                                              b->dev_types[ti]->p.band_w,
                                              b->d_types + ti, b->d_cells_by_type + b->type_first[ti],
                                              b->type_count[ti], b->d_offsets, V, rhs, out, stream);
    if (e != hipSuccess) return fail(NPFEM_E_HIP, std::string("banded global step: ") + hipGetErrorString(e));
  }
  return NPFEM_OK;
}

npfem_status npfem_batch_get_global_solve(const npfem_batch* b, int32_t* solve) {
  if (!b || !solve) return fail(NPFEM_E_INVALID, "null argument");
  *solve = b->solve_choice >= 0 ? b->solve_choice
                                : (b->form == NPFEM_FORM_FUSED ? NPFEM_SOLVE_DENSE : NPFEM_SOLVE_BANDED);
  return NPFEM_OK;
}

npfem_status npfem_batch_check(npfem_batch* b, void* stream) {
  if (!b) return fail(NPFEM_E_INVALID, "batch is null");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(hipStreamSynchronize(s));
  int flag = 0;
  HIP_TRY(hipMemcpy(&flag, b->d_flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) {
    HIP_TRY(hipMemset(b->d_flag, 0, sizeof(int)));
    return fail(NPFEM_E_NONFINITE, "a step produced a non-finite position or velocity");
  }
  return NPFEM_OK;
}

}  // extern "C"
