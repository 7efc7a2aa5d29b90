// Fused batched form of the npFEM step: every cell of the batch advanced by one launch.
//
// One workgroup (4 waves) takes a group of up to 4*gw cells of one type. Per cell, LDS holds
// the current positions X and the gradient/update R, FP32, vertex-interleaved
// [cell][vertex][xyz] with a cell stride of cs = 3 (mod 16) words (3 npad, npad >= n a
// multiple of 4, plus pad words); with the global step's k-row order each half-wave of an MFMA
// B-tile read then touches 32 distinct LDS banks.
// Each wave owns gw cells for everything except the global step:
//   prediction      delta^0 = h v + h^2 F/m, kept with delta and the cell-local rest of x_n
//                   in the owning lanes' registers (supplementary material, npFEM
//                   subsection: y_n with C = 0);
//   volume          grad_i V = 1/6 sum over incident triangles of their doubled area vector,
//                   accumulated into R over the triangle schedule, V = 1/6 sum_t x_a . N_t;
//                   V and |grad V|^2 summed per cell in FP64 over the cell's lanes;
//   local step      R = (m/h^2)(delta - delta^0) - k_vol lambda grad V, then every triangle
//                   and hinge adds its constraint residual; the schedule packs vertex-disjoint
//                   elements into rounds, so one wave updates R without atomics or barriers
//                   and the summation order is fixed (bitwise reproducible);
//   global step     D = -L^-1 R for all 3 * cells columns of the group at once as a product
//                   on the fp16 matrix cores (v_mfma_f32_16x16x32_f16) with split operands
//                   (hi + lo fp16 pairs, 22 significant bits, FP32 accumulation), A = L^-1
//                   tiles streamed from L2, B = R from LDS (split in place), both
//                   double-buffered; the 4 waves split the output tiles in pairs that share A;
//   update          delta += D (quasi-Newton step of the fourth displayed equation).
// Three workgroup barriers per iteration; everything else is wave-local.
#include <hip/hip_runtime.h>

#include "npfem_internal.h"
#include "filters.h"
#include "projections.h"

namespace npfem {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// Class test (not v - v == 0, which FMA contraction can turn into a product's rounding error).
__device__ __forceinline__ bool finite_f(float v) { return __builtin_isfinite(v); }

// Per-type constants are read through pointers stored in device memory; marking them as
// global-address-space pointers lets the compiler use global (not flat) loads.
template <typename P>
__device__ __forceinline__ const __attribute__((address_space(1))) P* gptr(const P* p) {
  return (const __attribute__((address_space(1))) P*)p;
}

typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u3 __attribute__((ext_vector_type(3)));

// Schedule records are read with loads of exactly the words a pass uses: a load whose result
// words are partly unused lets the register allocator reuse those words' registers, which
// then forces a wait for the load to land before the reuse. Records are loaded two rounds
// ahead of their use. A round's records start at a uniform address (scalar registers) and a
// lane's record sits at its slot's byte offset from there, so the loads take no vector
// address arithmetic.
struct TriHead {   // words 0-3 of a TriRec
  uint32_t a, b, c;
  float orient;
};
struct TriElem {   // words 0-2 and 4-7 of a TriRec
  uint32_t a, b, c;
  float area, gb0, gb1, gc1;
};
struct HingeElem { // a whole HingeRec
  uint32_t i, j, k, l;
  float a1, a2, a3, rest;
};

// Buffer resource over a per-type schedule (raw byte addressing, no range limit of note):
// a record load then takes the round's byte offset in a scalar register and the lane's slot
// offset in a vector register, with no address arithmetic in the vector ALU.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t sched_rsrc(const void* sched) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(sched), (short)0, 0x7fffffff,
                                           0x00020000);
}
__device__ __forceinline__ TriHead load_tri_head(__amdgpu_buffer_rsrc_t rs, int round, int S,
                                                 uint32_t slot_off) {
  static_assert(sizeof(TriRec) == 32 && sizeof(HingeRec) == 32, "32-byte records");
  const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, slot_off, round * S * 32, 0);
  return {v.x, v.y, v.z, __uint_as_float(v.w)};
}
__device__ __forceinline__ TriElem load_tri_elem(__amdgpu_buffer_rsrc_t rs, int round, int S,
                                                 uint32_t slot_off) {
  // a, b, c (orient unused here), then area, gb0, gb1, gc1
  const u3 v = __builtin_amdgcn_raw_buffer_load_b96(rs, slot_off, round * S * 32, 0);
  const u4 w = __builtin_amdgcn_raw_buffer_load_b128(rs, slot_off + 16u, round * S * 32, 0);
  return {v.x, v.y, v.z, __uint_as_float(w.x), __uint_as_float(w.y), __uint_as_float(w.z),
          __uint_as_float(w.w)};
}
__device__ __forceinline__ HingeElem load_hinge(__amdgpu_buffer_rsrc_t rs, int round, int S,
                                                uint32_t slot_off) {
  const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, slot_off, round * S * 32, 0);
  const u4 w = __builtin_amdgcn_raw_buffer_load_b128(rs, slot_off + 16u, round * S * 32, 0);
  return {v.x, v.y, v.z, v.w, __uint_as_float(w.x), __uint_as_float(w.y),
          __uint_as_float(w.z), __uint_as_float(w.w)};
}

// Split record loads for the rounds' two-stage pipeline: the vertex offsets of a round are
// loaded two rounds ahead of its arithmetic (its positions one round ahead), its
// coefficients one round ahead.
__device__ __forceinline__ u3 load_tri_offs(__amdgpu_buffer_rsrc_t rs, int round, int S,
                                            uint32_t slot_off) {
  return __builtin_amdgcn_raw_buffer_load_b96(rs, slot_off, round * S * 32, 0);
}
__device__ __forceinline__ float load_tri_orient(__amdgpu_buffer_rsrc_t rs, int round, int S,
                                                 uint32_t slot_off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, slot_off + 12u, round * S * 32, 0));
}
__device__ __forceinline__ u4 load_rec_hi(__amdgpu_buffer_rsrc_t rs, int round, int S,
                                          uint32_t slot_off) {   // words 4-7
  return __builtin_amdgcn_raw_buffer_load_b128(rs, slot_off + 16u, round * S * 32, 0);
}
__device__ __forceinline__ u4 load_hinge_offs(__amdgpu_buffer_rsrc_t rs, int round, int S,
                                              uint32_t slot_off) {
  return __builtin_amdgcn_raw_buffer_load_b128(rs, slot_off, round * S * 32, 0);
}

// x + a d with the product rounded on its own (no fused multiply-add): the Skalak line
// search's trial positions and the update that takes a trial must form the same values.
__device__ __forceinline__ float add_scaled(float x, float a, float d) {
#pragma clang fp contract(off)
  return x + a * d;
}

// A vertex's xyz in a cell block, from the block's base and the vertex's byte offset.
__device__ __forceinline__ float* vat(float* base, uint32_t byte_off) {
  return (float*)((char*)base + byte_off);
}
__device__ __forceinline__ const float* vat(const float* base, uint32_t byte_off) {
  return (const float*)((const char*)base + byte_off);
}

// Makes the packed owner-item codes opaque to the optimiser so that the per-item LDS
// addresses derived from them are recomputed where used instead of being hoisted out of the
// iteration loop and kept live in registers.
template <int NQ>
__device__ __forceinline__ void refresh_items(int (&item)[NQ]) {
#pragma unroll
  for (int it = 0; it < NQ; ++it) asm volatile("" : "+v"(item[it]));
}

__device__ __forceinline__ Vec3<float> ld3(const float* p) { return v3<float>(p[0], p[1], p[2]); }
__device__ __forceinline__ Vec3<double> to_d(Vec3<float> a) { return v3<double>(a.x, a.y, a.z); }
__device__ __forceinline__ void st3(float* p, Vec3<float> v) {
  p[0] = v.x;
  p[1] = v.y;
  p[2] = v.z;
}

typedef __attribute__((address_space(3))) float lfloat;

// Word offset of MFMA column col (3 cell + coord) of row 0; columns past the group's last
// read the first column of their tile (the same words as its lanes: no further LDS banks;
// their results are discarded).
__device__ __forceinline__ int col_base(int col, int ncols, int CS) {
  col = col < ncols ? col : (col & ~15);
  const int cell = col / 3;
  return cell * CS + (col - 3 * cell);
}

// The global step's product runs on the fp16 matrix cores with split operands: each FP32
// value x (scaled by a power of two) is carried as hi = fp16(x) and lo = fp16(x - hi), and
// A B = A_hi B_hi + A_hi B_lo + A_lo B_hi up to the dropped A_lo B_lo (2^-22 relative); the
// products of fp16 values are exact in the FP32 accumulator. Per 32 k rows and output tile,
// three v_mfma_f32_16x16x32_f16 issue in about 60 cycles (two accumulator chains; measured on
// gfx950) where eight v_mfma_f32_16x16x4_f32 take 256.
// Dynamic LDS of the fused kernels (cell blocks).
extern __shared__ float lds[];

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef const __attribute__((address_space(1))) u4 gu4;

// One k chunk (kMfmaChunk k steps = 32 k rows) of the split A operand from L2: the lane's 8 hi
// and 8 lo values (La: the row tile's first chunk plus the lane, in 16-byte units). A row tile
// stores its chunks plus two zero chunks, so every chunk load below is in bounds.
struct AChunk {
  u4 hi, lo;
};
__device__ __forceinline__ void load_a(AChunk& a, gu4* La, int c) {
  a.hi = La[c * 128];
  a.lo = La[c * 128 + 64];
}

// B words of chunk c: the lane's column at k rows 4 s0 + k_row_in_chunk(lane / 16, j), read
// at Rb[12 s0 + 6 j] (Rb includes the lane group's row offset). Chunks start at s0 =
// min(c kMfmaChunk, KR - kMfmaChunk): the last chunk is shifted back to end at the last row
// and overlaps its predecessor, whose rows hold zero A values in that chunk (as do the zero
// chunks after it). A lane's rows for j and j + 1 (j even) are rows r and r + 2 with r mod 4
// in {0, 1}, whose words hold the two hi values and the two lo values (split_b): the even
// words are the lane's 8 hi values, the odd words its 8 lo values, already in MFMA order.
template <bool TWO>
__device__ __forceinline__ void load_b(u4 (&b0)[2], u4 (&b1)[2], const lfloat* RbA, const lfloat* RbB,
                                       int c, int KR) {
  const int s0 = min(c * kMfmaChunk, KR - kMfmaChunk);
  const lfloat* pa = RbA + 12 * s0;
  const lfloat* pb = RbB + 12 * s0;
#pragma unroll
  for (int j = 0; j < kMfmaChunk; ++j) {
    b0[j & 1][j >> 1] = __float_as_uint(pa[3 * k_row_in_chunk(0, j)]);
    if (TWO) b1[j & 1][j >> 1] = __float_as_uint(pb[3 * k_row_in_chunk(0, j)]);
  }
}

// acc0 (and acc1 with TWO) += A B over one chunk, the small terms first.
template <bool TWO>
__device__ __forceinline__ void mma_chunk(const AChunk& a, const u4 (&b0)[2], const u4 (&b1)[2],
                                          f4& acc0, f4& acc1) {
  const h8 ah = __builtin_bit_cast(h8, a.hi), al = __builtin_bit_cast(h8, a.lo);
  const h8 b0h = __builtin_bit_cast(h8, b0[0]), b0l = __builtin_bit_cast(h8, b0[1]);
  if (TWO) {
    const h8 b1h = __builtin_bit_cast(h8, b1[0]), b1l = __builtin_bit_cast(h8, b1[1]);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, b0h, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, b1h, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, b0l, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, b1l, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, b0h, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, b1h, acc1, 0, 0, 0);
  } else {
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, b0h, acc0, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, b0l, acc0, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, b0h, acc0, 0, 0, 0);
  }
}

// D tiles of one A row tile: acc0 (and acc1 with TWO) += A x B over the chunks covering the k
// steps s < KR (KR >= kMfmaChunk). Two register sets alternate: while one chunk's MFMAs run,
// the next chunk's A values (from L2) and B words (from LDS) are in flight. The loads are the
// same on every pass (the last pass fetches a zero chunk), so each chunk waits only for its
// own operands.
template <bool TWO>
__device__ __forceinline__ void mfma_rows(gu4* La, const lfloat* RbA, const lfloat* RbB, int KR,
                                          f4& acc0, f4& acc1) {
  const int nch = (KR + kMfmaChunk - 1) / kMfmaChunk;
  // raised wave priority while the matrix cores work: the CU's other workgroups are in their
  // VALU-bound element rounds, and issuing this wave's loads and MFMAs first keeps both busy
  __builtin_amdgcn_s_setprio(1);
  AChunk aP, aQ;
  u4 bP0[2], bP1[2], bQ0[2], bQ1[2];
  load_a(aP, La, 0);
  load_b<TWO>(bP0, bP1, RbA, RbB, 0, KR);
  int c = 0;
  for (; c + 1 < nch; c += 2) {
    load_a(aQ, La, c + 1);
    load_b<TWO>(bQ0, bQ1, RbA, RbB, c + 1, KR);
    __builtin_amdgcn_sched_barrier(0);
    mma_chunk<TWO>(aP, bP0, bP1, acc0, acc1);
    __builtin_amdgcn_sched_barrier(0);
    load_a(aP, La, c + 2);
    load_b<TWO>(bP0, bP1, RbA, RbB, c + 2, KR);
    __builtin_amdgcn_sched_barrier(0);
    mma_chunk<TWO>(aQ, bQ0, bQ1, acc0, acc1);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (c < nch) mma_chunk<TWO>(aP, bP0, bP1, acc0, acc1);
  __builtin_amdgcn_s_setprio(0);
}

// D = -acc usc[cell] for output tile (rt, ct) into R (usc: the power of two that undoes the
// operands' scaling): lane holds rows rt*16 + 4 (lane/16) + r of column ct*16 + lane%16. R is
// the block at word r_off of the dynamic LDS (addressed from the array itself: a pointer held
// across the iteration would be a 64-bit generic one). With SL and slp (the Skalak line
// search), grad g . D of the tile's columns is added to slp[col] first: grad g is R's split
// B operand at these rows (a lane's rows row0..row0+3 hold the pairs (row0, row0 + 2) and
// (row0 + 1, row0 + 3) in their four words), times 2^-sc = usc 2^a_exp; the four lane
// groups of a column are summed in a fixed order, so the sums are reproducible.
template <bool SL = false>
__device__ __forceinline__ void write_tile(int r_off, f4 acc, int rt, int ct, int lane, int n,
                                           int ncols, int CS, const float* usc,
                                           double* slp = nullptr, int a_exp = 0) {
  // the lane index made opaque: the tile's addresses are recomputed here (a few VALU
  // instructions) instead of being hoisted out of the iteration loop and spilled
  int ln = lane;
  asm volatile("" : "+v"(ln));
  const int col = ct * 16 + (ln & 15);
  const int row0 = rt * 16 + 4 * (ln >> 4);
  double part = 0.0;
  if (col < ncols) {
    const int cell = col / 3;
    const float u = -usc[cell];
    lfloat* Rl = (lfloat*)lds + r_off;
    const int w = cell * CS + (col - 3 * cell) + 3 * row0;
    if (SL && slp != nullptr && row0 < n) {
      const uint32_t w0 = __float_as_uint(Rl[w]), w1 = __float_as_uint(Rl[w + 3]);
      const uint32_t w2 = __float_as_uint(Rl[w + 6]), w3 = __float_as_uint(Rl[w + 9]);
      auto hf = [](uint32_t bits) { return (float)__builtin_bit_cast(_Float16, (uint16_t)bits); };
      const float gs = ldexpf(usc[cell], a_exp);
      const float g[4] = {(hf(w0) + hf(w2)) * gs, (hf(w1) + hf(w3)) * gs,
                          (hf(w0 >> 16) + hf(w2 >> 16)) * gs, (hf(w1 >> 16) + hf(w3 >> 16)) * gs};
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (row0 + r < n) part += (double)g[r] * (double)(acc[r] * u);
    }
    if (row0 + 3 < n) {   // every row but those of the last row tile
#pragma unroll
      for (int r = 0; r < 4; ++r) Rl[w + 3 * r] = acc[r] * u;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (row0 + r < n) Rl[w + 3 * r] = acc[r] * u;
    }
  }
  if (SL && slp != nullptr) {
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (lane < 16 && col < ncols) slp[col] += part;
  }
}

// The product's B operand in place: x = R 2^sc (sc per cell putting the cell's largest |R| in
// [2^13, 2^14)) as hi = fp16(x) and lo = fp16(x - hi) (the difference is exact in FP32). Rows
// r and r + 2 with r mod 4 in {0, 1} are paired: word (r, coord) holds their hi values (r in
// the low half), word (r + 2, coord) their lo values, which is the order of the MFMA's B
// operand (load_b). Rows n..npad-1 count as zero (their words are not read as values).
// *usc = 2^-(sc + a_exp) undoes both operands' scaling. Lane mapping of the element phase:
// cell block Rc, S lanes per cell from slot s (all cells of the wave at once).
__device__ __forceinline__ void split_b(float* Rc, int n, int npad, int S, int s, bool ok, int a_exp,
                                        float* usc) {
  float m = 0.0f;
  if (ok)
    for (int vv = s; vv < n; vv += S) {
      const Vec3<float> r = ld3(Rc + 3 * vv);
      m = fmaxf(m, fmaxf(fabsf(r.x), fmaxf(fabsf(r.y), fabsf(r.z))));
    }
  for (int o = S >> 1; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  int ex = 0;
  (void)frexpf(m, &ex);   // m in [2^(ex-1), 2^ex)
  const int sc = m > 0.0f ? min(max(14 - ex, -100), 100) : 0;
  const float f = ldexpf(1.0f, sc);
  if (ok) {
    for (int p = s; p < npad / 2; p += S) {
      const int r = 4 * (p >> 1) + (p & 1);
      float* w0 = Rc + 3 * r;
      float* w1 = w0 + 6;   // row r + 2
      const bool ok0 = r < n, ok1 = r + 2 < n;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float x0 = ok0 ? w0[c] * f : 0.0f, x1 = ok1 ? w1[c] * f : 0.0f;
        const _Float16 h0 = (_Float16)x0, h1 = (_Float16)x1;
        const _Float16 l0 = (_Float16)(x0 - (float)h0), l1 = (_Float16)(x1 - (float)h1);
        w0[c] = __uint_as_float((uint32_t)__builtin_bit_cast(uint16_t, h0) |
                                ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16));
        w1[c] = __uint_as_float((uint32_t)__builtin_bit_cast(uint16_t, l0) |
                                ((uint32_t)__builtin_bit_cast(uint16_t, l1) << 16));
      }
    }
    if (s == 0) *usc = ldexpf(1.0f, -(sc + a_exp));
  }
}

// EXTRAS: some type of the batch has position-based damping, a velocity cap or Rayleigh
// damping with beta > 0, or the step has contacts (cp, cw: collision points [3][V] and
// weights [V]); without them the kernel is built without those code paths.
template <int NQ, bool EXTRAS, bool SKALAK>
__global__ void __launch_bounds__(kFusedThreads) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_fused_step(const DevType* __restrict__ types, const FusedGroup* __restrict__ groups,
             const int* __restrict__ n_groups_dev, const int64_t* __restrict__ offsets, int64_t vt,
             float* __restrict__ x, float* __restrict__ v, const float* __restrict__ f,
             const float* __restrict__ cp, const float* __restrict__ cw, int K,
             double* __restrict__ vol_area, int* __restrict__ flag) {
  __shared__ float lam_lds[kMaxGroupCells];
  __shared__ int64_t off_lds[kMaxGroupCells];
  __shared__ float usc_lds[kMaxGroupCells];   // per cell: undoes the product's operand scaling
  // Skalak line search, per cell: step length, accepted flag, g(x^k) and grad g . d
  __shared__ float ls_a[SKALAK ? kSkalakMaxCells : 1];
  __shared__ int ls_done[SKALAK ? kSkalakMaxCells : 1];
  __shared__ double ls_e0[SKALAK ? kSkalakMaxCells : 1], ls_slope[SKALAK ? kSkalakMaxCells : 1];
  // grad g . d per wave and MFMA column (3 cell + coord), summed in the product's write-back
  __shared__ double sl_part[SKALAK ? kFusedWaves : 1][SKALAK ? 3 * kSkalakMaxCells : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  const int n_groups = *n_groups_dev;
  for (int g = blockIdx.x; g < n_groups; g += gridDim.x) {
    const FusedGroup& grp = groups[g];
    const int count = grp.count;
    const DevType& T = types[grp.type];
    const int n = T.p.n, npad = T.p.npad, gw = T.p.gw, S = T.p.slots;
    const int G4 = kFusedWaves * gw;
    const int CS = T.p.cs;                   // words per cell block (3 npad + pad)
    float* X = lds;
    float* R = lds + kFusedRWords;   // fixed offset: one address per vertex serves X and R

    __syncthreads();   // the previous group's last reads of LDS are done
    for (int i = tid; i < G4 * CS; i += kFusedThreads) R[i] = 0.0f;

    // ---- owner items: (cell gc of this wave, vertex vi), q = lane + 64 * it, packed as
    //      vi | gc << 16; gc >= G4 marks an empty item
    int item[NQ];
#pragma unroll
    for (int it = 0; it < NQ; ++it) {
      const int q = lane + 64 * it;
      const int cw = q / n;
      const int gc = wave * gw + cw;
      item[it] = (cw < gw && gc < count) ? ((q - cw * n) | (gc << 16)) : (G4 << 16);
    }
#define ITEM_OK(it) ((item[it] >> 16) < G4)
#define ITEM_V(it) (item[it] & 0xffff)
#define ITEM_C(it) (item[it] >> 16)
#define ITEM_W(it) (ITEM_C(it) * CS + 3 * ITEM_V(it))   // word offset of the item's xyz
    // delta^0 = pred_h v + pred_h2m F (h v + h^2 F/m, over 1 + h alpha with Rayleigh alpha)
    const float h = (float)T.p.pred_h, h2m = (float)T.p.pred_h2m, ih2m = (float)T.p.inv_h2m;
    const float w_v = (float)T.p.w_v, ih = (float)(1.0 / T.p.h);
    if (tid < count) off_lds[tid] = offsets[grp.cells[tid]];
    __syncthreads();
    // element-phase lane mapping: cell cw = lane / S, slot s = lane % S
    const int e_cw = lane / S, e_s = lane - e_cw * S;
    const int e_gc = wave * gw + e_cw;
    const bool e_ok = e_gc < count;
    const uint32_t e_soff = 32u * (uint32_t)e_s;   // the lane's record within a round
    const __amdgpu_buffer_rsrc_t tri_rs = sched_rsrc(T.tri_sched);
    const __amdgpu_buffer_rsrc_t hinge_rs = sched_rsrc(T.hinge_sched);
    // e = delta - delta^0 is the only per-vertex state kept in registers; delta^0 is
    // recomputed from v and F when the step is written back. With position-based damping
    // each cell's centre of mass x_cm, its velocity v_cm, angular velocity w and first vertex
    // x_n[0] (kDampWords floats per cell after R) define the damped velocity used in delta^0.
    const bool damp = EXTRAS && T.p.kappa > 0.0;
    const float kappa = (float)T.p.kappa;
    const float v_max = (float)T.p.v_max;
    // Rayleigh damping with beta > 0: delta^0 = m M~^-1 (h v + h^2 F/m) is one more product on
    // the matrix cores (R = -(h v + h^2 F/m) first); delta^0 then waits in v for the
    // write-back (v_n has been read by then)
    const bool ray = EXTRAS && T.p.ray_c > 0.0;
    // Rayleigh in the iteration: grad g takes grad_mass instead of m/h^2 and the update
    // subtracts ray_c e (both the plain values for other types)
    const float gmass = EXTRAS ? (float)T.p.grad_mass : ih2m;
    const float ray_c = (float)T.p.ray_c;
    // Skalak types: the line search's slope grad g . d comes from the product's write-back
    // (grad g is R's split words there), its trial positions x + a d from X and R = d
    const bool sk = SKALAK && T.p.skalak;
    float* Dm = R + G4 * CS;
    float e[NQ][3];
#pragma unroll
    for (int it = 0; it < NQ; ++it) {
#pragma unroll
      for (int c = 0; c < 3; ++c) e[it][c] = 0.0f;
      if (ITEM_OK(it)) {
        const int64_t off = off_lds[ITEM_C(it)];
        const int vi = ITEM_V(it);
        float* Xv = X + ITEM_W(it);
        float* Rv = R + ITEM_W(it);
        // every input word loaded before the type's branches (a load whose value is used past a
        // branch is waited for there, one HBM round trip per item otherwise)
        float xi[3], x0[3], vv[3], ff[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          xi[c] = x[c * vt + off + vi];
          x0[c] = x[c * vt + off];
          vv[c] = v[c * vt + off + vi];
          ff[c] = f[c * vt + off + vi];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          // cell-local coordinates: positions relative to the cell's first vertex
          const float xl = xi[c] - x0[c];
          if (damp) {
            Xv[c] = xl;                       // x_n and v_n staged for the reductions
            Rv[c] = vv[c];
            if (vi == 0) Dm[kDampWords * ITEM_C(it) + 9 + c] = x0[c];
          } else if (ray) {
            Xv[c] = xl;
            Rv[c] = -(h * vv[c] + h2m * ff[c]);
          } else {
            Xv[c] = xl + (h * vv[c] + h2m * ff[c]);
          }
        }
      }
    }
    if (damp) {
      __builtin_amdgcn_wave_barrier();
      // per cell, over its lanes: centre of mass and its velocity, then angular momentum and
      // inertia about it (FP64 sums), w = I^-1 L; all cells of the wave at once
      const float* Xe0 = X + e_gc * CS;
      const float* Re0 = R + e_gc * CS;
      double sm[6] = {0, 0, 0, 0, 0, 0};
      if (e_ok)
        for (int vv = e_s; vv < n; vv += S) {
          const Vec3<float> a = ld3(Xe0 + 3 * vv), b = ld3(Re0 + 3 * vv);
          sm[0] += a.x; sm[1] += a.y; sm[2] += a.z;
          sm[3] += b.x; sm[4] += b.y; sm[5] += b.z;
        }
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        for (int o = S >> 1; o > 0; o >>= 1) sm[k] += __shfl_xor(sm[k], o, 64);
        sm[k] /= n;
      }
      double q[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // L (3), I (xx, yy, zz, xy, xz, yz)
      if (e_ok)
        for (int vv = e_s; vv < n; vv += S) {
          const Vec3<float> a = ld3(Xe0 + 3 * vv), b = ld3(Re0 + 3 * vv);
          const double r0 = (double)a.x - sm[0], r1 = (double)a.y - sm[1], r2 = (double)a.z - sm[2];
          q[0] += r1 * b.z - r2 * b.y;
          q[1] += r2 * b.x - r0 * b.z;
          q[2] += r0 * b.y - r1 * b.x;
          const double rr = r0 * r0 + r1 * r1 + r2 * r2;
          q[3] += rr - r0 * r0; q[4] += rr - r1 * r1; q[5] += rr - r2 * r2;
          q[6] -= r0 * r1; q[7] -= r0 * r2; q[8] -= r1 * r2;
        }
#pragma unroll
      for (int k = 0; k < 9; ++k)
        for (int o = S >> 1; o > 0; o >>= 1) q[k] += __shfl_xor(q[k], o, 64);
      if (e_ok && e_s == 0) {
        double wv[3];
        solve_sym3(q + 3, q, wv);
        float* d = Dm + kDampWords * e_gc;
        d[0] = (float)sm[0]; d[1] = (float)sm[1]; d[2] = (float)sm[2];
        d[3] = (float)sm[3]; d[4] = (float)sm[4]; d[5] = (float)sm[5];
        d[6] = (float)wv[0]; d[7] = (float)wv[1]; d[8] = (float)wv[2];
      }
      __builtin_amdgcn_wave_barrier();
      // delta^0 with the damped velocity; R back to zero
#pragma unroll
      for (int it = 0; it < NQ; ++it)
        if (ITEM_OK(it)) {
          const int64_t off = off_lds[ITEM_C(it)];
          const int vi = ITEM_V(it);
          float* Xv = X + ITEM_W(it);
          float* Rv = R + ITEM_W(it);
          const float* d = Dm + kDampWords * ITEM_C(it);
          const Vec3<float> xl = ld3(Xv);
          const Vec3<float> vd = pbd_velocity<float>(ld3(Rv), xl - v3<float>(d[0], d[1], d[2]),
                                                     v3<float>(d[3], d[4], d[5]),
                                                     v3<float>(d[6], d[7], d[8]), kappa);
          const float vdc[3] = {vd.x, vd.y, vd.z};
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float b = h * vdc[c] + h2m * f[c * vt + off + vi];
            if (ray) {
              Rv[c] = -b;
            } else {
              Xv[c] += b;
              Rv[c] = 0.0f;
            }
          }
        }
    }
    __syncthreads();   // R zeroed, X written

    const float* Xe = X + e_gc * CS;
    float* Re = R + e_gc * CS;
    const float w_s = (float)T.p.w_s, w_a = (float)T.p.w_a, w_b = (float)T.p.w_b;
    const float s_min = (float)T.p.s_min, s_max = (float)T.p.s_max;

    // MFMA output tiles of this wave: an equal share [u0, u1) of the RT x CT tiles in
    // row-major order, processed as pairs of neighbouring tiles (see the global step)
    const int RT = T.p.row_tiles, KS = T.p.k_steps, KR = npad / 4;
    const int ncols = 3 * count, CT = (ncols + 15) / 16;
    const int n_units = RT * CT;
    const int u0 = (n_units * wave) / kFusedWaves, u1 = (n_units * (wave + 1)) / kFusedWaves;

    // Products on the matrix cores: D = -A R for all 3 * cells columns of the group, A the
    // type's tiles (L^-1, or m M~^-1 for the Rayleigh prediction). Column col = 3 cell + coord,
    // row k = vertex: B(k, col) = R[cell][k][coord]. A work item is one tile or two
    // neighbouring tiles of the wave's share: with two or more column tiles, two column
    // tiles of one row tile (sharing every A fragment); with one column tile, two row tiles
    // (sharing B). Each wave holds its tiles in registers until every wave has read R, then
    // writes D over R.
    auto global_product = [&](const float* tiles) {
      f4 acc[kMaxTilesPerWave];
#pragma unroll
      for (int i = 0; i < kMaxTilesPerWave; ++i) acc[i] = f4{0.f, 0.f, 0.f, 0.f};
      int n_items = 0;
      {
        gu4* Lt = reinterpret_cast<gu4*>(gptr(tiles)) + lane;
        const int kq = lane >> 4;
        for (int u = u0; u < u1;) {
          f4 d0 = f4{0.f, 0.f, 0.f, 0.f}, d1 = f4{0.f, 0.f, 0.f, 0.f};
          if (CT >= 2) {
            const int rt = u / CT, ct = u - rt * CT;
            const lfloat* RbA = (const lfloat*)(R + col_base(ct * 16 + (lane & 15), ncols, CS) + 3 * k_row_in_chunk(kq, 0));
            if (ct + 1 < CT && u + 1 < u1) {
              const lfloat* RbB =
                  (const lfloat*)(R + col_base(ct * 16 + 16 + (lane & 15), ncols, CS) + 3 * k_row_in_chunk(kq, 0));
              mfma_rows<true>(Lt + (size_t)rt * KS * 16, RbA, RbB, KR, d0, d1);
              u += 2;
            } else {
              mfma_rows<false>(Lt + (size_t)rt * KS * 16, RbA, RbA, KR, d0, d1);
              u += 1;
            }
          } else {
            const lfloat* Rb = (const lfloat*)(R + col_base(lane & 15, ncols, CS) + 3 * k_row_in_chunk(kq, 0));
            mfma_rows<false>(Lt + (size_t)u * KS * 16, Rb, Rb, KR, d0, d1);
            if (u + 1 < u1) mfma_rows<false>(Lt + (size_t)(u + 1) * KS * 16, Rb, Rb, KR, d1, d0);
            u += (u + 1 < u1) ? 2 : 1;
          }
          // keep the item's tiles at the end of the held set (indices stay compile-time)
#pragma unroll
          for (int i = 0; i + 2 < kMaxTilesPerWave; ++i) acc[i] = acc[i + 2];
          acc[kMaxTilesPerWave - 2] = d0;
          acc[kMaxTilesPerWave - 1] = d1;
          ++n_items;
        }
      }
      __syncthreads();
      {
        // replay the item sequence to place the held tiles
        int u = u0;
#pragma unroll
        for (int q = 0; q < kMaxTilesPerWave / 2; ++q) {
          if (q >= kMaxTilesPerWave / 2 - n_items) {
            if (CT >= 2) {
              const int rt = u / CT, ct = u - rt * CT;
              write_tile(kFusedRWords, acc[2 * q], rt, ct, lane, n, ncols, CS, usc_lds);
              if (ct + 1 < CT && u + 1 < u1) {
                write_tile(kFusedRWords, acc[2 * q + 1], rt, ct + 1, lane, n, ncols, CS, usc_lds);
                u += 2;
              } else {
                u += 1;
              }
            } else {
              write_tile(kFusedRWords, acc[2 * q], u, 0, lane, n, ncols, CS, usc_lds);
              if (u + 1 < u1) write_tile(kFusedRWords, acc[2 * q + 1], u + 1, 0, lane, n, ncols, CS, usc_lds);
              u += (u + 1 < u1) ? 2 : 1;
            }
          }
        }
      }
    };

    if (ray) {   // delta^0 = m M~^-1 (h v + h^2 F/m): R holds its negated right-hand side
      split_b(Re, n, npad, S, e_s, e_ok, T.p.pinv_exp, &usc_lds[e_gc]);
      __syncthreads();
      global_product(T.pinv_tiles);
      __syncthreads();
      refresh_items(item);
#pragma unroll
      for (int it = 0; it < NQ; ++it)
        if (ITEM_OK(it)) {
          const int64_t off = off_lds[ITEM_C(it)];
          const int vi = ITEM_V(it);
          float* Rv = R + ITEM_W(it);
          float* Xv = X + ITEM_W(it);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float d0 = Rv[c];
            Xv[c] += d0;
            v[c * vt + off + vi] = d0;   // kept for the write-back
            Rv[c] = 0.0f;
          }
        }
      __syncthreads();
    }

    for (int k = 0; k < K; ++k) {
      // ---- volume constraint. R is zero here. Over the triangle rounds every triangle adds
      // its outward doubled area vector N_t = (x_b - x_a) x (x_c - x_a) (sign-corrected when
      // the schedule lists its vertices in reversed order) to R at its three vertices,
      // so that R_i = 6 grad_i V, and x_a . N_t (= 6 x its signed volume) to the lane's sum.
      double v6 = 0.0;
      {
        // Two-stage pipeline over the rounds, unrolled by two so that the A and B register
        // sets swap roles: while round r computes, the positions of round r + 1 (from its
        // offsets, loaded during round r - 1), its orientation and the offsets of round r + 2
        // are in flight, and round r's residual reads were issued before its arithmetic.
        // Reads of empty slots (vertex 0) and of cells past the group's count stay inside the
        // LDS blocks; only their writes are skipped.
        const int NR = T.p.tri_rounds;
        u3 o = load_tri_offs(tri_rs, 0, S, e_soff);
        float orA = load_tri_orient(tri_rs, 0, S, e_soff), orB;
        float *rA0, *rA1, *rA2, *rB0, *rB1, *rB2;
        Vec3<float> xA0, xA1, xA2, xB0, xB1, xB2;
        auto place = [&](int rr, float*& q0, float*& q1, float*& q2, Vec3<float>& p0,
                         Vec3<float>& p1, Vec3<float>& p2) {
          p0 = ld3(vat(Xe, o.x));
          p1 = ld3(vat(Xe, o.y));
          p2 = ld3(vat(Xe, o.z));
          q0 = vat(Re, o.x);
          q1 = vat(Re, o.y);
          q2 = vat(Re, o.z);
          __builtin_amdgcn_sched_barrier(0);   // o is consumed before it is reloaded
          o = load_tri_offs(tri_rs, min(rr + 1, NR - 1), S, e_soff);
        };
        auto work = [&](float orient, float* q0, float* q1, float* q2, const Vec3<float>& xa,
                        const Vec3<float>& xb, const Vec3<float>& xc) {
          const Vec3<float> oa = ld3(q0), ob = ld3(q1), oc = ld3(q2);
          __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the arithmetic
          // N_t and x_a . N_t in FP64 from the FP32 positions (differences of FP32 values are
          // exact in FP64); N_t enters the FP32 residual rounded once
          const Vec3<double> da = to_d(xa);
          const Vec3<double> ntd = cross3(to_d(xb) - da, to_d(xc) - da) * (double)orient;
          const Vec3<float> nt = v3<float>((float)ntd.x, (float)ntd.y, (float)ntd.z);
          if (e_ok && orient != 0.0f) {
            st3(q0, oa + nt);
            st3(q1, ob + nt);
            st3(q2, oc + nt);
            v6 += dot3(da, ntd);
          }
          __builtin_amdgcn_wave_barrier();
        };
        place(0, rA0, rA1, rA2, xA0, xA1, xA2);
        for (int r = 0; r < NR; r += 2) {
          place(r + 1, rB0, rB1, rB2, xB0, xB1, xB2);
          orB = load_tri_orient(tri_rs, min(r + 1, NR - 1), S, e_soff);
          work(orA, rA0, rA1, rA2, xA0, xA1, xA2);
          if (r + 1 < NR) {
            place(r + 2, rA0, rA1, rA2, xA0, xA1, xA2);
            orA = load_tri_orient(tri_rs, min(r + 2, NR - 1), S, e_soff);
            work(orB, rB0, rB1, rB2, xB0, xB1, xB2);
          }
        }
      }
      // |6 grad V|^2 of the cell: lane (cell, slot s) takes its vertices s, s + S, ...
      double g36 = 0.0;
      if (e_ok)
        for (int vv = e_s; vv < n; vv += S) {
          const Vec3<double> gv = to_d(ld3(Re + 3 * vv));
          g36 += dot3(gv, gv);
        }
      {
        // FP64 sums over the S lanes of each cell (all cells of the wave at once)
        double vs = v6, gs = g36;
        for (int o = S >> 1; o > 0; o >>= 1) {
          vs += __shfl_xor(vs, o, 64);
          gs += __shfl_xor(gs, o, 64);
        }
        // lambda = (V0 - V) / |grad V|^2 with V = vs / 6, |grad V|^2 = gs / 36; stored as
        // lambda / 6, the factor that multiplies R = 6 grad V
        if (e_ok && e_s == 0)
          lam_lds[e_gc] = (float)(gs > 0.0 ? (T.p.V0 - vs / 6.0) / gs * 6.0 : 0.0);
      }
      __builtin_amdgcn_wave_barrier();
      // ---- gradient of g: inertia + volume terms
      refresh_items(item);
#pragma unroll
      for (int it = 0; it < NQ; ++it)
        if (ITEM_OK(it)) {
          float* Rv = R + ITEM_W(it);
          const float lw = w_v * lam_lds[ITEM_C(it)];   // w_v lambda / 6
#pragma unroll
          for (int c = 0; c < 3; ++c) Rv[c] = gmass * e[it][c] - lw * Rv[c];
        }
      if (EXTRAS && cw != nullptr) {
        // collision energy w (x - p), x = x_n[0] + X. The weight, x_n[0] and p of three items
        // are loaded before any is used, every load unconditional (empty items read the first
        // vertex), and a zero weight selects no contribution: a load that a branch depends on
        // is waited for at once, which made every item an HBM round trip
#pragma unroll
        for (int i0 = 0; i0 < NQ; i0 += 3) {
          float wl[3], dl[3][3];
#pragma unroll
          for (int d = 0; d < 3; ++d)
            if (i0 + d < NQ) {
              const int it = i0 + d;
              const int64_t off = ITEM_OK(it) ? off_lds[ITEM_C(it)] : 0;
              const int64_t o = off + (ITEM_OK(it) ? ITEM_V(it) : 0);
              wl[d] = cw[o];
#pragma unroll
              for (int c = 0; c < 3; ++c) dl[d][c] = x[c * vt + off] - cp[c * vt + o];
            }
#pragma unroll
          for (int d = 0; d < 3; ++d)
            if (i0 + d < NQ && ITEM_OK(i0 + d)) {
              const int it = i0 + d;
              float* Rv = R + ITEM_W(it);
              const float* Xv = X + ITEM_W(it);
              const float w = wl[d];
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                const float t = w * (dl[d][c] + Xv[c]);
                Rv[c] += w != 0.0f ? t : 0.0f;
              }
            }
        }
      }
      __builtin_amdgcn_wave_barrier();
      // ---- triangle strain + area constraints
      {
        // pipelined and unrolled as the hinge rounds below
        const int NR = T.p.tri_rounds;
        u3 o = load_tri_offs(tri_rs, 0, S, e_soff);
        u4 cA = load_rec_hi(tri_rs, 0, S, e_soff), cB;     // area, gb0, gb1, gc1
        float *rA0, *rA1, *rA2, *rB0, *rB1, *rB2;
        Vec3<float> xA0, xA1, xA2, xB0, xB1, xB2;
        auto place = [&](int rr, float*& q0, float*& q1, float*& q2, Vec3<float>& p0,
                         Vec3<float>& p1, Vec3<float>& p2) {
          p0 = ld3(vat(Xe, o.x));
          p1 = ld3(vat(Xe, o.y));
          p2 = ld3(vat(Xe, o.z));
          q0 = vat(Re, o.x);
          q1 = vat(Re, o.y);
          q2 = vat(Re, o.z);
          __builtin_amdgcn_sched_barrier(0);   // o is consumed before it is reloaded
          o = load_tri_offs(tri_rs, min(rr + 1, NR - 1), S, e_soff);
        };
        auto work = [&](const u4& c, float* q0, float* q1, float* q2, const Vec3<float>& xa,
                        const Vec3<float>& xb, const Vec3<float>& xc) {
          __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the arithmetic
          const float area = __uint_as_float(c.x);
          if (e_ok && area > 0.0f) {
            Vec3<float> ra = ld3(q0), rb = ld3(q1), rcv = ld3(q2);
            if (SKALAK && sk)   // Skalak strain energy (B = w_s, C = w_a per unit rest area)
              (void)skalak_residual<float>(xa, xb, xc, __uint_as_float(c.y), __uint_as_float(c.z),
                                           0.0f, __uint_as_float(c.w), area, w_s, w_a, ra, rb, rcv);
            else
              triangle_residual<float>(xa, xb, xc, __uint_as_float(c.y), __uint_as_float(c.z), 0.0f,
                                       __uint_as_float(c.w), area, w_s, w_a, s_min, s_max, ra, rb,
                                       rcv);
            st3(q0, ra);
            st3(q1, rb);
            st3(q2, rcv);
          }
          __builtin_amdgcn_wave_barrier();
        };
        place(0, rA0, rA1, rA2, xA0, xA1, xA2);
        for (int r = 0; r < NR; r += 2) {
          place(r + 1, rB0, rB1, rB2, xB0, xB1, xB2);
          cB = load_rec_hi(tri_rs, min(r + 1, NR - 1), S, e_soff);
          work(cA, rA0, rA1, rA2, xA0, xA1, xA2);
          if (r + 1 < NR) {
            place(r + 2, rA0, rA1, rA2, xA0, xA1, xA2);
            cA = load_rec_hi(tri_rs, min(r + 2, NR - 1), S, e_soff);
            work(cB, rB0, rB1, rB2, xB0, xB1, xB2);
          }
        }
      }
      // ---- edge bending constraints
      {
        // Two-stage pipeline over the rounds, unrolled by two so that the A and B register
        // sets swap roles: while round r computes, the positions of round r + 1 (from its
        // offsets, loaded during round r - 1), its coefficients and the offsets of round r + 2
        // are in flight, and round r's residual reads were issued before its arithmetic.
        const int NR = T.p.hinge_rounds;
        u4 o = load_hinge_offs(hinge_rs, 0, S, e_soff);      // offsets of the round to place
        u4 cA = load_rec_hi(hinge_rs, 0, S, e_soff), cB;     // a1, a2, a3, rest
        float *rA0, *rA1, *rA2, *rA3, *rB0, *rB1, *rB2, *rB3;   // R addresses
        Vec3<float> xA0, xA1, xA2, xA3, xB0, xB1, xB2, xB3;
        // place round rr: positions and R addresses from o, then the offsets of round rr + 1
        auto place = [&](int rr, float*& q0, float*& q1, float*& q2, float*& q3, Vec3<float>& p0,
                         Vec3<float>& p1, Vec3<float>& p2, Vec3<float>& p3) {
          p0 = ld3(vat(Xe, o.x));
          p1 = ld3(vat(Xe, o.y));
          p2 = ld3(vat(Xe, o.z));
          p3 = ld3(vat(Xe, o.w));
          q0 = vat(Re, o.x);
          q1 = vat(Re, o.y);
          q2 = vat(Re, o.z);
          q3 = vat(Re, o.w);
          __builtin_amdgcn_sched_barrier(0);   // o is consumed before it is reloaded
          o = load_hinge_offs(hinge_rs, min(rr + 1, NR - 1), S, e_soff);
        };
        auto work = [&](const u4& c, float* q0, float* q1, float* q2, float* q3,
                        const Vec3<float>& xi, const Vec3<float>& xj, const Vec3<float>& xk,
                        const Vec3<float>& xl) {
          Vec3<float> ri = ld3(q0), rj = ld3(q1), rk = ld3(q2), rl = ld3(q3);
          __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the arithmetic
          const float a1 = __uint_as_float(c.x), a2 = __uint_as_float(c.y);
          const float a3 = __uint_as_float(c.z), rest = __uint_as_float(c.w);
          hinge_residual<float>(xi, xj, xk, xl, a1, a2, a3, rest, w_b, ri, rj, rk, rl);
          if (e_ok && rest >= 0.0f) {
            st3(q0, ri);
            st3(q1, rj);
            st3(q2, rk);
            st3(q3, rl);
          }
          __builtin_amdgcn_wave_barrier();
        };
        place(0, rA0, rA1, rA2, rA3, xA0, xA1, xA2, xA3);
        for (int r = 0; r < NR; r += 2) {
          place(r + 1, rB0, rB1, rB2, rB3, xB0, xB1, xB2, xB3);   // round r + 1 (clamped)
          cB = load_rec_hi(hinge_rs, min(r + 1, NR - 1), S, e_soff);
          work(cA, rA0, rA1, rA2, rA3, xA0, xA1, xA2, xA3);
          if (r + 1 < NR) {
            place(r + 2, rA0, rA1, rA2, rA3, xA0, xA1, xA2, xA3);
            cA = load_rec_hi(hinge_rs, min(r + 2, NR - 1), S, e_soff);
            work(cB, rB0, rB1, rB2, rB3, xB0, xB1, xB2, xB3);
          }
        }
      }
      split_b(Re, n, npad, S, e_s, e_ok, T.p.linv_exp, &usc_lds[e_gc]);
      __syncthreads();
      // ---- global step: D = -L^-1 R on the matrix cores (the product of global_product,
      //      written out here: through the lambda the loop spills one more register)
      f4 acc[kMaxTilesPerWave];
#pragma unroll
      for (int i = 0; i < kMaxTilesPerWave; ++i) acc[i] = f4{0.f, 0.f, 0.f, 0.f};
      int n_items = 0;
      {
        gu4* Lt = reinterpret_cast<gu4*>(gptr(T.linv_tiles)) + lane;
        const int kq = lane >> 4;
        for (int u = u0; u < u1;) {
          f4 d0 = f4{0.f, 0.f, 0.f, 0.f}, d1 = f4{0.f, 0.f, 0.f, 0.f};
          if (CT >= 2) {
            const int rt = u / CT, ct = u - rt * CT;
            const lfloat* RbA = (const lfloat*)(R + col_base(ct * 16 + (lane & 15), ncols, CS) + 3 * k_row_in_chunk(kq, 0));
            if (ct + 1 < CT && u + 1 < u1) {
              const lfloat* RbB =
                  (const lfloat*)(R + col_base(ct * 16 + 16 + (lane & 15), ncols, CS) + 3 * k_row_in_chunk(kq, 0));
              mfma_rows<true>(Lt + (size_t)rt * KS * 16, RbA, RbB, KR, d0, d1);
              u += 2;
            } else {
              mfma_rows<false>(Lt + (size_t)rt * KS * 16, RbA, RbA, KR, d0, d1);
              u += 1;
            }
          } else {
            const lfloat* Rb = (const lfloat*)(R + col_base(lane & 15, ncols, CS) + 3 * k_row_in_chunk(kq, 0));
            mfma_rows<false>(Lt + (size_t)u * KS * 16, Rb, Rb, KR, d0, d1);
            if (u + 1 < u1) mfma_rows<false>(Lt + (size_t)(u + 1) * KS * 16, Rb, Rb, KR, d1, d0);
            u += (u + 1 < u1) ? 2 : 1;
          }
          // keep the item's tiles at the end of the held set (indices stay compile-time)
#pragma unroll
          for (int i = 0; i + 2 < kMaxTilesPerWave; ++i) acc[i] = acc[i + 2];
          acc[kMaxTilesPerWave - 2] = d0;
          acc[kMaxTilesPerWave - 1] = d1;
          ++n_items;
        }
      }
      __syncthreads();
      // Skalak: this wave's grad g . d sums per column, filled by the write-back below
      double* slp = (SKALAK && sk) ? sl_part[wave] : nullptr;
      if (SKALAK && sk && lane < 3 * kSkalakMaxCells) sl_part[wave][lane] = 0.0;
      {
        // replay the item sequence to place the held tiles
        int u = u0;
#pragma unroll
        for (int q = 0; q < kMaxTilesPerWave / 2; ++q) {
          if (q >= kMaxTilesPerWave / 2 - n_items) {
            if (CT >= 2) {
              const int rt = u / CT, ct = u - rt * CT;
              write_tile<SKALAK>(kFusedRWords, acc[2 * q], rt, ct, lane, n, ncols, CS, usc_lds, slp, T.p.linv_exp);
              if (ct + 1 < CT && u + 1 < u1) {
                write_tile<SKALAK>(kFusedRWords, acc[2 * q + 1], rt, ct + 1, lane, n, ncols, CS, usc_lds, slp,
                                   T.p.linv_exp);
                u += 2;
              } else {
                u += 1;
              }
            } else {
              write_tile<SKALAK>(kFusedRWords, acc[2 * q], u, 0, lane, n, ncols, CS, usc_lds, slp, T.p.linv_exp);
              if (u + 1 < u1)
                write_tile<SKALAK>(kFusedRWords, acc[2 * q + 1], u + 1, 0, lane, n, ncols, CS, usc_lds, slp,
                                   T.p.linv_exp);
              u += (u + 1 < u1) ? 2 : 1;
            }
          }
        }
      }
      __syncthreads();
      if (SKALAK && sk) {
        // ---- line search along d = D (R), per cell and wave-local: the first step length a
        //      of 1, 1/2, ..., 2^-kMaxHalvings with g(x + a d) <= g(x) + kArmijoC a grad g . d
        //      (the last one when none qualifies), every sum in FP64
        const int lc0 = wave * gw;   // the wave's first cell in the group
        // per-cell sums over the owner items of the wave (every lane gets all of its cells')
        auto owner_sum = [&](double (&v)[kSkalakMaxGw]) {
#pragma unroll
          for (int q = 0; q < kSkalakMaxGw; ++q)
            for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
        };
        // g at x^k (trial false) or at x^k + a d, everything in FP64: the positions x + a d
        // from X and R = d (exact in FP64 up to its rounding: a is a power of two), delta -
        // delta^0 = e + a d, the element energies. Near convergence a d falls below the FP32
        // spacing of x, and a test on FP32 trial positions (which then equal x^k) could never
        // show the decrease it asks for; in FP64 the test resolves it as the paper's
        // formulation does. Returns the total of the lane's element cell.
        auto pos = [&](const float* xp, float a, bool trial) -> Vec3<double> {
          const Vec3<double> p = to_d(ld3(xp));
          if (!trial) return p;
          return p + to_d(ld3(xp + kFusedRWords)) * (double)a;
        };
        auto energy = [&](bool trial) -> double {
          double g2[kSkalakMaxGw], vx[kSkalakMaxGw], em[kSkalakMaxGw], ec[kSkalakMaxGw];
#pragma unroll
          for (int q = 0; q < kSkalakMaxGw; ++q) g2[q] = vx[q] = em[q] = ec[q] = 0.0;
          // volume terms over the gather schedule (the wave's vertices by ring length, 64 to a
          // slot): 6 grad_i V = sum over the triangles (i, b, c) around i of
          // (p_b - p_i) x (p_c - p_i) = sum of p_b x p_c (the remainder (sum of p_c - p_b) x p_i
          // vanishes on a closed star, where every neighbour is once a b and once a c). The ring
          // is stored in cyclic order (c of one pair is b of the next), so the walk reads each
          // neighbour once and loads b only where a star has several cycles. A lane's codes and
          // ring descriptors are loaded before any is used (a load that a branch depends on is
          // waited for at once); ring words come in batches of kRingBatch independent loads
          // (the array is padded by kRingBatch words, so a batch past the last ring stays in
          // bounds).
          {
            uint32_t code[NQ], info[NQ];
#pragma unroll
            for (int j = 0; j < NQ; ++j) code[j] = T.gather_sched[j * 64 + lane];
#pragma unroll
            for (int j = 0; j < NQ; ++j) info[j] = T.ring_info[code[j] == kGatherEmpty ? 0 : (code[j] & 0xfffu)];
#pragma unroll
            for (int j = 0; j < NQ; ++j) {
              const int lc = (int)(code[j] >> 12), vi = (int)(code[j] & 0xfffu);
              if (code[j] != kGatherEmpty && lc0 + lc < count) {
                const float* Pc = X + (lc0 + lc) * CS;
                const float a = trial ? ls_a[lc0 + lc] : 0.0f;
                const Vec3<double> dpi = pos(Pc + 3 * vi, a, trial);
                const int roff = (int)(info[j] >> 8), deg = (int)(info[j] & 255u);
                Vec3<double> gi = v3<double>(0.0, 0.0, 0.0);
                uint32_t prev_c = 0xffffffffu;
                Vec3<double> pprev = v3<double>(0.0, 0.0, 0.0);
                for (int q0 = 0; q0 < deg; q0 += kRingBatch) {
                  uint32_t prs[kRingBatch];
#pragma unroll
                  for (int jj = 0; jj < kRingBatch; ++jj) prs[jj] = T.ring_pairs[roff + q0 + jj];
#pragma unroll
                  for (int jj = 0; jj < kRingBatch; ++jj)
                    if (q0 + jj < deg) {
                      const uint32_t bb = prs[jj] & 0xffffu, cc = prs[jj] >> 16;
                      const Vec3<double> pb = bb == prev_c ? pprev : pos(Pc + 3 * (int)bb, a, trial);
                      const Vec3<double> pc = pos(Pc + 3 * (int)cc, a, trial);
                      gi = gi + cross3(pb, pc);
                      prev_c = cc;
                      pprev = pc;
                    }
                }
                const double g2i = dot3(gi, gi), vxi = dot3(dpi, gi);
#pragma unroll
                for (int q = 0; q < kSkalakMaxGw; ++q)
                  if (q == lc) {
                    g2[q] += g2i;
                    vx[q] += vxi;
                  }
              }
            }
          }
          // inertia and collision terms over the owner items
          refresh_items(item);
#pragma unroll
          for (int it = 0; it < NQ; ++it)
            if (ITEM_OK(it)) {
              const int lc = ITEM_C(it) - lc0, vi = ITEM_V(it);
              const float* Dv = R + ITEM_W(it);
              double emi = 0.0, eci = 0.0;
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                const double el = trial ? (double)e[it][c] + (double)ls_a[ITEM_C(it)] * (double)Dv[c] : (double)e[it][c];
                emi += el * el;
              }
              if (EXTRAS && cw != nullptr) {
                const int64_t off = off_lds[ITEM_C(it)];
                const float wc = cw[off + vi];
                if (wc != 0.0f) {
                  const float* Pc = X + ITEM_C(it) * CS;
                  const float a = trial ? ls_a[ITEM_C(it)] : 0.0f;
                  const Vec3<double> dpi = pos(Pc + 3 * vi, a, trial);
                  const double pic[3] = {dpi.x, dpi.y, dpi.z};
#pragma unroll
                  for (int c = 0; c < 3; ++c) {
                    const double gd = ((double)x[c * vt + off] - (double)cp[c * vt + off + vi]) + pic[c];
                    eci += 0.5 * (double)wc * gd * gd;
                  }
                }
              }
#pragma unroll
              for (int q = 0; q < kSkalakMaxGw; ++q)
                if (q == lc) {
                  em[q] += emi;
                  ec[q] += eci;
                }
            }
          owner_sum(g2);
          owner_sum(vx);
          owner_sum(em);
          owner_sum(ec);
          // element energies of the lane's cell: Skalak triangles and bending hinges, each
          // round's record loaded one round ahead
          double el = 0.0;
          if (e_ok) {
            const float* Pe = X + e_gc * CS;
            const float ae = trial ? ls_a[e_gc] : 0.0f;
            {
              const int NR = T.p.tri_rounds;
              u3 o = load_tri_offs(tri_rs, 0, S, e_soff);
              u4 c = load_rec_hi(tri_rs, 0, S, e_soff);
#pragma unroll 2
              for (int r = 0; r < NR; ++r) {
                const int rn = min(r + 1, NR - 1);
                const u3 on = load_tri_offs(tri_rs, rn, S, e_soff);
                const u4 cn = load_rec_hi(tri_rs, rn, S, e_soff);
                const float area = __uint_as_float(c.x);
                if (area > 0.0f)
                  el += skalak_energy<double>(pos(vat(Pe, o.x), ae, trial), pos(vat(Pe, o.y), ae, trial),
                                              pos(vat(Pe, o.z), ae, trial), (double)__uint_as_float(c.y),
                                              (double)__uint_as_float(c.z), 0.0,
                                              (double)__uint_as_float(c.w), (double)area, T.p.w_s, T.p.w_a);
                o = on;
                c = cn;
              }
            }
            {
              const int NR = T.p.hinge_rounds;
              u4 o = load_hinge_offs(hinge_rs, 0, S, e_soff);
              u4 c = load_rec_hi(hinge_rs, 0, S, e_soff);
#pragma unroll 2
              for (int r = 0; r < NR; ++r) {
                const int rn = min(r + 1, NR - 1);
                const u4 on = load_hinge_offs(hinge_rs, rn, S, e_soff);
                const u4 cn = load_rec_hi(hinge_rs, rn, S, e_soff);
                const float rest = __uint_as_float(c.w);
                if (rest >= 0.0f)
                  el += hinge_energy<double>(pos(vat(Pe, o.x), ae, trial), pos(vat(Pe, o.y), ae, trial),
                                             pos(vat(Pe, o.z), ae, trial), pos(vat(Pe, o.w), ae, trial),
                                             (double)__uint_as_float(c.x), (double)__uint_as_float(c.y),
                                             (double)__uint_as_float(c.z), (double)rest, T.p.w_b);
                o = on;
                c = cn;
              }
            }
          }
          for (int o = S >> 1; o > 0; o >>= 1) el += __shfl_xor(el, o, 64);
          // the lane's cell: volume energy (w_v/2)(V0 - V)^2 / |grad V|^2 with
          // V = sum p_i . grad_i V / 3 (homogeneity) and grad V = (6 grad V) / 6, inertia,
          // contacts
          double G2 = 0.0, V6 = 0.0, EM = 0.0, EC = 0.0;
#pragma unroll
          for (int q = 0; q < kSkalakMaxGw; ++q)
            if (q == e_cw) {
              G2 = g2[q];
              V6 = vx[q];
              EM = em[q];
              EC = ec[q];
            }
          const double V = V6 / 18.0, gv2 = G2 / 36.0;
          const double ev = gv2 > 0.0 ? 0.5 * T.p.w_v * (T.p.V0 - V) * (T.p.V0 - V) / gv2 : 0.0;
          return el + 0.5 * T.p.inv_h2m * EM + ev + EC;
        };
        {
          // g(x^k) at the stored (FP32) iterate: the accepted trial's FP64 positions were
          // rounded by the update
          const double e0 = energy(false);
          if (e_ok && e_s == 0) {
            // grad g . d of the cell: the waves' column sums in a fixed order
            double sl = 0.0;
            for (int w = 0; w < kFusedWaves; ++w)
#pragma unroll
              for (int c = 0; c < 3; ++c) sl += sl_part[w][3 * e_gc + c];
            ls_a[e_gc] = 1.0f;
            ls_done[e_gc] = 0;
            ls_e0[e_gc] = e0;
            ls_slope[e_gc] = sl;
          }
        }
        __builtin_amdgcn_wave_barrier();
        for (int h = 0; h <= kMaxHalvings; ++h) {
          const double et = energy(true);
          if (e_ok && e_s == 0 && !ls_done[e_gc]) {
            const float a = ls_a[e_gc];
            if (et <= ls_e0[e_gc] + kArmijoC * (double)a * ls_slope[e_gc] || h == kMaxHalvings) {
              ls_done[e_gc] = 1;
            } else {
              ls_a[e_gc] = 0.5f * a;
            }
          }
          __builtin_amdgcn_wave_barrier();
          int open = 0;
          for (int q = 0; q < gw; ++q)
            if (lc0 + q < count) open |= !ls_done[lc0 + q];
          if (!open) break;
        }
      }
      // ---- update: delta += D (registers), x^{k+1} = x^k + D (LDS); Skalak: a D
      refresh_items(item);
#pragma unroll
      for (int it = 0; it < NQ; ++it)
        if (ITEM_OK(it)) {
          float* Rv = R + ITEM_W(it);
          float* Xv = X + ITEM_W(it);
          const float a_ls = (SKALAK && sk) ? ls_a[ITEM_C(it)] : 1.0f;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if (SKALAK && sk) {
              e[it][c] = add_scaled(e[it][c], a_ls, Rv[c]);
              Xv[c] = add_scaled(Xv[c], a_ls, Rv[c]);
            } else {
              const float dd = EXTRAS ? Rv[c] - ray_c * e[it][c] : Rv[c];
              e[it][c] += dd;
              Xv[c] += dd;
            }
            Rv[c] = 0.0f;   // R starts the next iteration at zero
          }
        }
      __builtin_amdgcn_wave_barrier();
    }

    // ---- per-cell volume and area at x_{n+1}: over the triangle schedule, each lane sums
    //      x_a . N_t and |N_t| of its triangles in FP64 (N_t formed in FP64 from the FP32
    //      cell-local positions), then the S lanes of each cell are summed in FP64
    if (vol_area) {
      double vs = 0.0, as = 0.0;
      if (e_ok)
        for (int r = 0; r < T.p.tri_rounds; ++r) {
          const TriHead rc = load_tri_head(tri_rs, r, S, e_soff);
          if (rc.orient != 0.0f) {
            const Vec3<double> da = to_d(ld3(vat(Xe, rc.a)));
            const Vec3<double> db = to_d(ld3(vat(Xe, rc.b)));
            const Vec3<double> dc = to_d(ld3(vat(Xe, rc.c)));
            const Vec3<double> ntd = cross3(db - da, dc - da);
            vs += (double)rc.orient * dot3(da, ntd);
            as += __builtin_sqrt(dot3(ntd, ntd));
          }
        }
      for (int o = S >> 1; o > 0; o >>= 1) {
        vs += __shfl_xor(vs, o, 64);
        as += __shfl_xor(as, o, 64);
      }
      if (e_ok && e_s == 0) {
        vol_area[2 * (int64_t)grp.cells[e_gc]] = vs / 6.0;
        vol_area[2 * (int64_t)grp.cells[e_gc] + 1] = 0.5 * as;
      }
    }
    // ---- x_{n+1} = x_n + delta, v_{n+1} = delta / h capped at v_max, with delta = delta^0 + e
    //      (delta^0 recomputed exactly as at the start of the step; with damping the cell's
    //      first vertex x_n[0] comes from LDS, since its owner may already have overwritten it)
    refresh_items(item);
    bool bad = false;
#pragma unroll
    for (int it = 0; it < NQ; ++it)
      if (ITEM_OK(it)) {
        const int64_t off = off_lds[ITEM_C(it)];
        const int vi = ITEM_V(it);
        float vin[3], xin[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          vin[c] = v[c * vt + off + vi];
          xin[c] = x[c * vt + off + vi];
        }
        if (damp && !ray) {
          const float* d = Dm + kDampWords * ITEM_C(it);
          const Vec3<float> xl = v3<float>(xin[0] - d[9], xin[1] - d[10], xin[2] - d[11]);
          const Vec3<float> vd = pbd_velocity<float>(v3<float>(vin[0], vin[1], vin[2]),
                                                     xl - v3<float>(d[0], d[1], d[2]),
                                                     v3<float>(d[3], d[4], d[5]),
                                                     v3<float>(d[6], d[7], d[8]), kappa);
          vin[0] = vd.x; vin[1] = vd.y; vin[2] = vd.z;
        }
        float vn[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          // with Rayleigh beta, v holds delta^0 since the start of the step
          const float dl = ray ? vin[c] + e[it][c] : (h * vin[c] + h2m * f[c * vt + off + vi]) + e[it][c];
          const float xn = xin[c] + dl;
          vn[c] = dl * ih;
          x[c * vt + off + vi] = xn;
          bad |= !finite_f(xn);
        }
        if (EXTRAS) cap_speed(vn[0], vn[1], vn[2], v_max);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          v[c * vt + off + vi] = vn[c];
          bad |= !finite_f(vn[c]);
        }
      }
    if (bad) atomicOr(flag, 1);
#undef ITEM_OK
#undef ITEM_V
#undef ITEM_C
#undef ITEM_W
  }
}


// D = -acc usc[cell] of output tile (rt, ct) straight to out ([3][V] SoA): the lane's four
// rows row0..row0+3 of column col = 3 cell + coord are consecutive words of that plane.
__device__ __forceinline__ void store_tile(float* out, int64_t vt, f4 acc, int rt, int ct, int lane,
                                           int n, int ncols, const float* usc, const int64_t* off) {
  const int col = ct * 16 + (lane & 15);
  const int row0 = rt * 16 + 4 * (lane >> 4);
  if (col < ncols) {
    const int cell = col / 3;
    const float u = -usc[cell];
    float* o = out + (col - 3 * cell) * vt + off[cell] + row0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (row0 + r < n) o[r] = acc[r] * u;
  }
}

constexpr int kStageLoads = 26;   // right-hand-side loads per thread in flight (global step alone):
                                  // an RBC group of 8 cells in one batch

// Global step alone, wide form: out = L^-1 r for the cells of one type, up to kWideMaxCells
// per workgroup (bc, chosen per type so that bc cell blocks fit 64 KB of LDS), 3 bc columns in
// COLS column tiles. The right-hand sides are staged into the cell-block layout in LDS (rows
// n..npad-1 zero) and split as in the fused step (16 lanes per cell, four cells per wave); the
// staging issues kStageLoads loads per thread before any LDS store, every load unconditional
// from an in-range word (padding rows read row n - 1) and selected afterwards (a load under a
// branch is waited for at once), the element's (cell, coordinate, row) from a float-reciprocal
// division that is exact for every index and npad here. A work item is two row tiles times all COLS column tiles: each A chunk from L2 then
// feeds 6 COLS MFMAs and each B word read from LDS two row tiles, which keeps the operand
// traffic per MFMA within what a CU's L2 path and LDS deliver. The products of an
// accumulator run in the order of mma_chunk (the small terms first), as in the fused step.
// Every finished tile goes straight to HBM (its four rows are consecutive words of one
// coordinate plane); the block's right-hand sides are all in LDS by then, so out may alias r. The odd last row tile pairs with itself (computed twice,
// stored once).
template <int COLS>
__global__ void __launch_bounds__(kFusedThreads)
k_global_dense_wide(const DevType* __restrict__ tp, const int32_t* __restrict__ cells, int n_cells,
                    int bc, const int64_t* __restrict__ offsets, int64_t vt, const float* r, float* out) {
  __shared__ int64_t off_lds[kWideMaxCells];
  __shared__ float usc_lds[kWideMaxCells];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const DevType& T = *tp;
  const int n = T.p.n, npad = T.p.npad, CS = T.p.cs;
  const int c0 = blockIdx.x * bc;
  const int count = min(bc, n_cells - c0);
  float* R = lds;
  if (tid < count) off_lds[tid] = offsets[cells[c0 + tid]];
  __syncthreads();
  {
    const int total = count * 3 * npad;
    const float inv_npad = 1.0f / (float)npad;
    for (int i0 = tid; i0 < total; i0 += kFusedThreads * kStageLoads) {
      float val[kStageLoads];
      int dst[kStageLoads];
#pragma unroll
      for (int j = 0; j < kStageLoads; ++j) {
        const int i = i0 + j * kFusedThreads;
        const int ii = i < total ? i : 0;
        const int cc = (int)(((float)ii + 0.5f) * inv_npad);
        const int v = ii - cc * npad, cell = cc / 3, c = cc - 3 * cell;
        dst[j] = i < total ? cell * CS + 3 * v + c : -1;
        const float x = r[c * vt + off_lds[cell] + min(v, n - 1)];
        val[j] = (i < total && v < n) ? -x : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < kStageLoads; ++j)
        if (dst[j] >= 0) R[dst[j]] = val[j];
    }
  }
  __syncthreads();
  {
    const int e_cw = lane >> 4, e_s = lane & 15, e_gc = wave * 4 + e_cw;
    split_b(R + e_gc * CS, n, npad, 16, e_s, e_gc < count, T.p.linv_exp, &usc_lds[e_gc]);
  }
  __syncthreads();
  const int RT = T.p.row_tiles, KS = T.p.k_steps, KR = npad / 4;
  const int ncols = 3 * count;
  const int nch = (KR + kMfmaChunk - 1) / kMfmaChunk;
  gu4* Lt = reinterpret_cast<gu4*>(gptr(T.linv_tiles)) + lane;
  const int kq = lane >> 4;
  const lfloat* Rb[COLS];
#pragma unroll
  for (int ct = 0; ct < COLS; ++ct)
    Rb[ct] = (const lfloat*)(R + col_base(ct * 16 + (lane & 15), ncols, CS) + 3 * k_row_in_chunk(kq, 0));
  for (int ip = wave; 2 * ip < RT; ip += kFusedWaves) {
    const int rt0 = 2 * ip, rt1 = min(rt0 + 1, RT - 1);
    gu4* La0 = Lt + (size_t)rt0 * KS * 16;
    gu4* La1 = Lt + (size_t)rt1 * KS * 16;
    f4 acc[2][COLS];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int ct = 0; ct < COLS; ++ct) acc[q][ct] = f4{0.f, 0.f, 0.f, 0.f};
    AChunk aP0, aP1, aQ0, aQ1;
    u4 bP[COLS][2], bQ[COLS][2];
    auto loads = [&](AChunk& a0, AChunk& a1, u4 (&b)[COLS][2], int c) {
      load_a(a0, La0, c);
      load_a(a1, La1, c);
#pragma unroll
      for (int ct = 0; ct < COLS; ++ct) load_b<false>(b[ct], b[ct], Rb[ct], Rb[ct], c, KR);
    };
    auto mmas = [&](const AChunk& a0, const AChunk& a1, const u4 (&b)[COLS][2]) {
      const h8 a0h = __builtin_bit_cast(h8, a0.hi), a0l = __builtin_bit_cast(h8, a0.lo);
      const h8 a1h = __builtin_bit_cast(h8, a1.hi), a1l = __builtin_bit_cast(h8, a1.lo);
#pragma unroll
      for (int ct = 0; ct < COLS; ++ct) {
        const h8 bh = __builtin_bit_cast(h8, b[ct][0]);
        acc[0][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0l, bh, acc[0][ct], 0, 0, 0);
        acc[1][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1l, bh, acc[1][ct], 0, 0, 0);
      }
#pragma unroll
      for (int ct = 0; ct < COLS; ++ct) {
        const h8 bl = __builtin_bit_cast(h8, b[ct][1]);
        acc[0][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0h, bl, acc[0][ct], 0, 0, 0);
        acc[1][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1h, bl, acc[1][ct], 0, 0, 0);
      }
#pragma unroll
      for (int ct = 0; ct < COLS; ++ct) {
        const h8 bh = __builtin_bit_cast(h8, b[ct][0]);
        acc[0][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0h, bh, acc[0][ct], 0, 0, 0);
        acc[1][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1h, bh, acc[1][ct], 0, 0, 0);
      }
    };
    // two register sets alternate: while one chunk's MFMAs run, the next chunk's operands are
    // in flight; the loads past the last chunk fetch a zero chunk (A) or repeat the last (B)
    loads(aP0, aP1, bP, 0);
    int c = 0;
    for (; c + 1 < nch; c += 2) {
      loads(aQ0, aQ1, bQ, c + 1);
      __builtin_amdgcn_sched_barrier(0);
      mmas(aP0, aP1, bP);
      __builtin_amdgcn_sched_barrier(0);
      loads(aP0, aP1, bP, c + 2);
      __builtin_amdgcn_sched_barrier(0);
      mmas(aQ0, aQ1, bQ);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (c < nch) mmas(aP0, aP1, bP);
#pragma unroll
    for (int ct = 0; ct < COLS; ++ct) {
      store_tile(out, vt, acc[0][ct], rt0, ct, lane, n, ncols, usc_lds, off_lds);
      if (rt1 != rt0) store_tile(out, vt, acc[1][ct], rt1, ct, lane, n, ncols, usc_lds, off_lds);
    }
  }
}

}  // namespace

hipError_t launch_fused_step(const DevType* types_dev, int n_types, const FusedGroup* groups,
                             const int* n_groups_dev, int max_groups, const int64_t* offsets,
                             int64_t vtot, float* x, float* v, const float* f, const float* cp,
                             const float* cw, int K, double* vol_area, int* flag, size_t lds_bytes,
                             bool extras, bool skalak, void* stream) {
  (void)n_types;
  if (max_groups == 0) return hipSuccess;
  // one workgroup per group up to a few waves of the chip; beyond that workgroups loop
  const int grid = max_groups < kMaxFusedGrid ? max_groups : kMaxFusedGrid;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (skalak)
    hipLaunchKernelGGL((k_fused_step<kMaxItems, true, true>), dim3(grid), dim3(kFusedThreads),
                       lds_bytes, s, types_dev, groups, n_groups_dev, offsets, vtot, x, v, f, cp,
                       cw, K, vol_area, flag);
  else if (extras || cw != nullptr)
    hipLaunchKernelGGL((k_fused_step<kMaxItems, true, false>), dim3(grid), dim3(kFusedThreads),
                       lds_bytes, s, types_dev, groups, n_groups_dev, offsets, vtot, x, v, f, cp,
                       cw, K, vol_area, flag);
  else
    hipLaunchKernelGGL((k_fused_step<kMaxItems, false, false>), dim3(grid), dim3(kFusedThreads),
                       lds_bytes, s, types_dev, groups, n_groups_dev, offsets, vtot, x, v, f,
                       nullptr, nullptr, K, vol_area, flag);
  return hipGetLastError();
}

hipError_t launch_global_dense_wide(const DevType* dt, int cs, const int32_t* cells, int n_cells,
                                    const int64_t* offsets, int64_t vtot, const float* r, float* out,
                                    void* stream) {
  if (n_cells == 0) return hipSuccess;
  const int bc = wide_cells_per_block(cs);
  const int cols = (3 * bc + 15) / 16;
  const int grid = (n_cells + bc - 1) / bc;
  const size_t lds = (size_t)bc * cs * sizeof(float);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (cols >= 3)
    hipLaunchKernelGGL(k_global_dense_wide<3>, dim3(grid), dim3(kFusedThreads), lds, s, dt, cells, n_cells, bc,
                       offsets, vtot, r, out);
  else if (cols == 2)
    hipLaunchKernelGGL(k_global_dense_wide<2>, dim3(grid), dim3(kFusedThreads), lds, s, dt, cells, n_cells, bc,
                       offsets, vtot, r, out);
  else
    hipLaunchKernelGGL(k_global_dense_wide<1>, dim3(grid), dim3(kFusedThreads), lds, s, dt, cells, n_cells, bc,
                       offsets, vtot, r, out);
  return hipGetLastError();
}

}  // namespace npfem
