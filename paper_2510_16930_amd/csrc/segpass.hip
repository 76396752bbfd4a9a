// Segment passes for TTMcTC and the core on the gfx950 matrix cores, float32
// accumulation, in three operand precisions for the Kronecker products:
//   FP32: float32 factor rows, v_mfma_f32_16x16x4f32 (4 nonzeros per product);
//   BF16: bfloat16 factor copies, v_mfma_f32_16x16x16_bf16 (16 nonzeros);
//   FP16: float16 factor copies scaled by 2^15 (entries of a factor with
//         orthonormal columns are at most 1), v_mfma_f32_16x16x16_f16; the
//         value-times-row operand is scaled by a power of two chosen from
//         max|x| so it cannot overflow, and y is unscaled exactly afterwards.
// The product of y_i with the core (stage two) is float32 in all three.
//
// Both passes walk a copy of the nonzeros sorted by one mode n and, for every
// nonempty slice i (the index set I^(n)_i of Table 1), form
//     y_i = sum over nonzeros e of slice i of  x_e * (Kronecker over m != n of U^(m)(i_m^e, :)),
// the i-th row of Y_(n) with Y = X x_{-n} {U^T} (§4.1), without storing Y.
// Viewed as a matrix Y_i (rows: the Kronecker product of the first N-2 other
// modes, columns: the last other mode), Y_i = sum_e (x_e u_row^e)(u_col^e)^T is a
// product whose inner dimension is the slice's nonzeros, so it maps onto the
// matrix cores with 4 nonzeros per instruction: each group of 16 lanes gathers
// one nonzero's factor rows, row-contiguous (64 bytes per factor row at K=16).
//
//  - TTMcTC pass (mode n): A^(n)(i, :) = y_i G_(n)^T (definition in §4.1).
//    Finished y_i are staged in LDS, 16 slices at a time, and multiplied by
//    G_(n)^T on the matrix cores (the operand is kept in registers).
//  - Core pass (mode c): G_(c) = sum_i U^(c)(i, :)^T y_i, i.e. G = X x {U^T}
//    (§2.2) grouped by slices of mode c; run on the mode with the fewest
//    slices, so the per-slice outer product is negligible.
//
// Work split: the sorted nonzeros of a mode are cut into W contiguous ranges
// of equal nonzero count; slices crossing a range boundary produce partial
// rows that a fix-up kernel adds in range order. Every sum has a fixed order,
// so results are bitwise reproducible. Y_i may span several 16x16 blocks
// (rows > 16 or columns > 16); then each block is handled by its own wave of
// the workgroup and the TTMcTC partial products are added in LDS.
#include "passes.h"

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

namespace hoqri {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kRsrcWord3 = 0x00020000;  // raw buffer, gfx9 family
constexpr int YS = 260;                      // LDS floats per staged y_i block (256 + pad)
// finished slices staged per stage-two product (LDS per wave grows with it;
// 8 keeps several workgroups per CU also when a y_i spans several waves)
__host__ __device__ inline int stage_slots(int B) {
  (void)B;
  return 8;
}
constexpr int KIND_COMPLETE = 0, KIND_HEAD = 1, KIND_TAIL = 2;

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRsrcWord3);
}
// Raw buffer loads: an offset at or beyond the buffer size returns 0.
__device__ inline float ld_f(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline int32_t ld_i(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
__device__ inline i4 ld_i4(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0);
}

// Wave-uniform read of p[i] through the scalar cache (read-only data written
// before the launch): it is counted apart from the vector loads in flight, so
// waiting for it does not wait for them.
__device__ inline int32_t scalar_ld(const int32_t* p, int32_t i) {
  typedef const __attribute__((address_space(4))) int32_t* cptr;
  return ((cptr)p)[__builtin_amdgcn_readfirstlane(i)];
}

// Orders this wave's LDS writes before its later LDS reads (no cross-wave sync).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

typedef short s4 __attribute__((ext_vector_type(4)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef __bf16 b4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

constexpr int P_FP32 = 0, P_BF16 = 1, P_FP16 = 2;

__device__ inline uint32_t ld_u16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
}
// 16-bit factor entry (raw bits) to float32
template <int PREC>
__device__ inline float f16bits_to_f32(uint32_t b) {
  if constexpr (PREC == P_BF16) return __builtin_bit_cast(float, b << 16);
  else return (float)__builtin_bit_cast(_Float16, (unsigned short)b);
}
// one 16x16x16 product: a[t] (float32, rounded to nearest even here) against
// the packed 16-bit operand b
template <int PREC>
__device__ inline f4 mfma16v(const float* a, s4 b, f4 c) {
  if constexpr (PREC == P_BF16) {
    const b4 av = {(__bf16)a[0], (__bf16)a[1], (__bf16)a[2], (__bf16)a[3]};
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, av), b, c, 0, 0, 0);
  } else {
    const h4 av = {(_Float16)a[0], (_Float16)a[1], (_Float16)a[2], (_Float16)a[3]};
    return __builtin_amdgcn_mfma_f32_16x16x16f16(av, __builtin_bit_cast(h4, b), c, 0, 0, 0);
  }
}
// one 16x16x16 product: a[t] (float32, rounded to nearest even here) against
// b[t] (16-bit raw bits), k-slot 4g + t of lane group g
template <int PREC>
__device__ inline f4 mfma16(const float* a, const uint32_t* b, f4 c) {
  const s4 bv = {(short)b[0], (short)b[1], (short)b[2], (short)b[3]};
  if constexpr (PREC == P_BF16) {
    const b4 av = {(__bf16)a[0], (__bf16)a[1], (__bf16)a[2], (__bf16)a[3]};
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, av), bv, c, 0, 0, 0);
  } else {
    const h4 av = {(_Float16)a[0], (_Float16)a[1], (_Float16)a[2], (_Float16)a[3]};
    return __builtin_amdgcn_mfma_f32_16x16x16f16(av, __builtin_bit_cast(h4, bv), c, 0, 0, 0);
  }
}


__device__ inline int32_t range_lo(int64_t w, int64_t W, int64_t nnz) { return (int32_t)((w * nnz) / W); }

// The slices holding nonzeros e1 and e2: the largest s in [0, R) with
// seg_off[s] <= e (seg_off[0] = 0 <= e < nnz = seg_off[R]), both found by
// the whole wave at once (it must be converged): lanes 0..31 search for e1
// and lanes 32..63 for e2, 32-ary, each step one vector load of 32 evenly
// spaced probes of the current interval and a ballot, so a 1e6-slice table
// takes four load latencies instead of twenty dependent scalar loads per
// search.
__device__ inline void find_seg2(const int32_t* seg_off, int32_t R, int32_t e1, int32_t e2, int32_t* s1,
                                 int32_t* s2) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5, i = lane & 31;
  const int32_t e = half ? e2 : e1;
  int32_t lo = 0, hi = R;  // invariant: seg_off[lo] <= e < seg_off[hi]; uniform in each half
  while (__builtin_amdgcn_ballot_w64(hi - lo > 1) != 0) {
    const int64_t span = hi - lo;
    // probes lo + floor(span i / 32): nondecreasing in i and, when span <= 32,
    // every index of [lo, hi); seg_off increases, so the true lanes are a prefix
    const int32_t pr = lo + (int32_t)((span * i) >> 5);
    const bool le = i == 0 || (span > 1 && seg_off[pr] <= e);
    const uint64_t m = __builtin_amdgcn_ballot_w64(le);
    const uint32_t bits = (uint32_t)(half ? (m >> 32) : m);
    const int k = 31 - __builtin_clz(bits);  // last true lane of this half (lane 0 of it is true)
    if (span > 1) {
      const int32_t nlo = lo + (int32_t)((span * k) >> 5);
      hi = k == 31 ? hi : lo + (int32_t)((span * (k + 1)) >> 5);
      lo = nlo;
    }
  }
  *s1 = __builtin_amdgcn_readlane(lo, 0);
  *s2 = __builtin_amdgcn_readlane(lo, 32);
}

__device__ inline int32_t rd_lane(int32_t v, int32_t lane) { return __builtin_amdgcn_readlane(v, lane); }

// A window of the slice table in this wave's LDS: entry i holds seg_off[base+i]
// and seg_row[base+i] (64 entries). Reads use a wave-uniform address; the window
// lives in LDS so no loop-carried vector registers hold it.
struct SegWindow {
  int32_t* off;  // LDS [64]
  int32_t* row;  // LDS [64]
  int32_t base;
  __device__ void load(const SegArgs& a, int32_t b, int lane) {
    base = __builtin_amdgcn_readfirstlane(b);
    const int32_t i = base + lane;  // clamped, unconditional loads keep the control flow uniform
    const int32_t o = a.seg_off[i < a.R ? i : a.R];
    const int32_t r = a.seg_row[i < a.R ? i : a.R - 1];
    wave_sync();
    off[lane] = o;
    row[lane] = r;
    wave_sync();
  }
  __device__ int32_t get_off(int32_t s) const { return __builtin_amdgcn_readfirstlane(off[s - base]); }
  __device__ int32_t get_row(int32_t s) const { return __builtin_amdgcn_readfirstlane(row[s - base]); }
};

// Per-lane byte offsets of this lane's row / column inside the gathered factor
// rows, for block (rb, cb). Padded rows/columns read finite neighbouring data
// (or 0 beyond the buffer); their products land in padded entries of y_i that
// the stage-two operand zeroes and the core pass never stores.
template <int NM1, int PREC>
__device__ inline void lane_offsets(const SegArgs& a, int rb, int cb, int q, uint32_t* ka4, uint32_t* kb4,
                                    uint32_t* kc4) {
  const uint32_t es = PREC == P_FP32 ? 4u : 2u;  // bytes per factor entry
  const int r = 16 * rb + q;
  const int c = 16 * cb + q;
  if constexpr (NM1 == 3) {
    *ka4 = (uint32_t)(r / a.K1) * es;
    *kb4 = (uint32_t)(r % a.K1) * es;
  } else {
    *ka4 = (uint32_t)r * es;
    *kb4 = 0;
  }
  *kc4 = (uint32_t)c * es;
}

// Walks nonzeros [lo, hi) of the sorted stream (slices s_first..s_last, clipped
// to the range) and calls on_seg(s, row, y) when the clipped slice s is done;
// y holds this wave's 16x16 block of y_s as D[4g+v][q] in y[v].
//
// The stream is read in aligned blocks of 16 nonzeros. Inside a block the plan
// stores the nonzeros 4x4-transposed (physical 4g + t holds logical 4t + g), so
// the 16-byte load of lane group g returns its k-slot for all four sub-steps;
// sub-step t covers the 4 consecutive logical nonzeros 16b + 4t + (0..3), one
// matrix-core product each, accumulated in acc[t] (four independent chains).
// A block inside one slice takes 4 products; a block that a slice boundary cuts
// takes 4 masked products per slice it touches (lanes outside the slice give 0).
//
// Loads form a three-stage pipeline over three register sets rotated by
// renaming (the block loop is unrolled three times): while block b is
// multiplied, the factor rows of block b+2 and the index/value vectors of
// block b+3 are in flight. Loads complete in issue order, so each step issues
// the indices of b+3 before the rows of b+2 and waits only for loads issued
// two steps earlier.
template <int NM1>
struct PipeSet {
  float ga[4];     // row-factor part of the A operand (float32)
  uint32_t gb[4];  // column-factor entry: float32 bits, or 16-bit raw bits
};

// Lane n of each 16-lane row, broadcast to the whole row (DPP row_newbcast).
template <int N>
__device__ inline int32_t row_bcast(int32_t v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + N, 0xF, 0xF, false);
}
// The same broadcast folded into its consumer: with a zero old value the
// compiler merges the DPP move into the following VOP2 add or multiply.
template <int N>
__device__ inline uint32_t bcast_add(int32_t v, uint32_t k) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, v, 0x150 + N, 0xF, 0xF, false) + k;
}
template <int N>
__device__ inline float bcast_mul(int32_t v, float f) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, v, 0x150 + N, 0xF, 0xF, false)) * f;
}
// f(integral_constant<int, C>) for C = I .. N-1 (compile-time lane indices)
template <int I, int N, typename F>
__device__ inline void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}
template <int NM1, int PREC, typename OnSeg>
__device__ inline void walk_range(const SegArgs& a, int32_t lo, int32_t hi, int32_t s_first, int32_t s_last,
                                  uint32_t ka4, uint32_t kb4, uint32_t kc4, int lane, int32_t* wlds,
                                  OnSeg&& on_seg) {
  const int g = lane >> 4;
  // block records: 16 (NM1 + 1) dwords per 16 nonzeros; lane group g reads its
  // 4 (NM1 + 1) dwords (one per lane, the last lanes repeat the last dword)
  constexpr int GD = 4 * (NM1 + 1);
  const auto rRec = make_rsrc(a.rec, (uint32_t)a.nnz_pad * 4u * (NM1 + 1));
  const int qd = (lane & 15) < GD ? (lane & 15) : GD - 1;
  const uint32_t goff = (uint32_t)(g * GD + qd) * 4u;
  const auto rU0 = make_rsrc(a.U[0], a.Ubytes[0]);
  const auto rU1 = make_rsrc(a.U[1], NM1 >= 2 ? a.Ubytes[1] : 0u);
  const auto rU2 = make_rsrc(a.U[2], NM1 >= 3 ? a.Ubytes[2] : 0u);

  lo = __builtin_amdgcn_readfirstlane(lo);
  hi = __builtin_amdgcn_readfirstlane(hi);
  s_first = __builtin_amdgcn_readfirstlane(s_first);
  s_last = __builtin_amdgcn_readfirstlane(s_last);
  const int32_t b0 = lo >> 4;
  const int32_t nblk = ((hi - 1) >> 4) - b0 + 1;
  const int32_t bmax = (a.nnz_pad >> 4) - 1;

  // one dword per lane; the 16 lanes of group g then share the group's record
  // by row broadcasts (instead of every lane loading all of it)
  auto load_rec = [&](int32_t blk) -> int32_t {
    blk = blk <= bmax ? blk : bmax;
    return __builtin_amdgcn_raw_buffer_load_b32(rRec, goff, (uint32_t)blk * (64u * (NM1 + 1)), 0);
  };
  // The record holds the byte offset of a row's first 16-bit entry (twice the
  // element offset): the 16-bit copies add the lane's entry offset to the
  // broadcast value directly, the float32 factors first double it.
  auto gather = [&](int32_t rec, PipeSet<NM1>& S) {
    static_for<0, 4>([&](auto T) {
      constexpr int t = decltype(T)::value;
      if constexpr (PREC == P_FP32) {
        const uint32_t o0 = (uint32_t)row_bcast<t>(rec) << 1;
        if constexpr (NM1 == 1) {
          S.ga[t] = 1.f;
          S.gb[t] = __builtin_amdgcn_raw_buffer_load_b32(rU0, o0 + kc4, 0, 0);
        } else if constexpr (NM1 == 2) {
          const uint32_t o1 = (uint32_t)row_bcast<4 + t>(rec) << 1;
          S.ga[t] = ld_f(rU0, o0 + ka4);
          S.gb[t] = __builtin_amdgcn_raw_buffer_load_b32(rU1, o1 + kc4, 0, 0);
        } else {
          const uint32_t o1 = (uint32_t)row_bcast<4 + t>(rec) << 1;
          const uint32_t o2 = (uint32_t)row_bcast<8 + t>(rec) << 1;
          S.ga[t] = ld_f(rU0, o0 + ka4) * ld_f(rU1, o1 + kb4);
          S.gb[t] = __builtin_amdgcn_raw_buffer_load_b32(rU2, o2 + kc4, 0, 0);
        }
      } else {  // 16-bit copies: ka4 etc. hold 2 * k here
        if constexpr (NM1 == 1) {
          S.ga[t] = 1.f;
          S.gb[t] = ld_u16(rU0, bcast_add<t>(rec, kc4));
        } else if constexpr (NM1 == 2) {
          S.ga[t] = f16bits_to_f32<PREC>(ld_u16(rU0, bcast_add<t>(rec, ka4)));
          S.gb[t] = ld_u16(rU1, bcast_add<4 + t>(rec, kc4));
        } else {
          S.ga[t] = f16bits_to_f32<PREC>(ld_u16(rU0, bcast_add<t>(rec, ka4))) *
                    f16bits_to_f32<PREC>(ld_u16(rU1, bcast_add<4 + t>(rec, kb4)));
          S.gb[t] = ld_u16(rU2, bcast_add<8 + t>(rec, kc4));
        }
      }
    });
  };

  SegWindow win;
  win.off = wlds;
  win.row = wlds + 64;
  win.load(a, s_first, lane);
  int32_t s = s_first;
  int32_t seg_lo = lo;  // first slice is clipped at lo
  int32_t seg_hi = win.get_off(s_first + 1);
  seg_hi = __builtin_amdgcn_readfirstlane(seg_hi < hi ? seg_hi : hi);
  f4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
  bool done = false;

  // block `blk` with set C (current), set N2 (block blk+2: gather now);
  // set C then receives the indices of block blk+3. FP32: four products per
  // block (sub-steps t, chains acc[t]); 16-bit: one product per block, chain
  // acc[ci] (ci = position in the three-step unroll).
  auto step = [&](int32_t blk, int32_t crec, PipeSet<NM1>& C, int32_t nrec, PipeSet<NM1>& N2, const int ci) {
    float xa[4];
    uint32_t xb[4];
    static_for<0, 4>([&](auto T) {
      constexpr int t = decltype(T)::value;
      // FP16: the scale goes first, so no intermediate can exceed the bound
      if constexpr (PREC == P_FP16) {
        const float xv = bcast_mul<4 * NM1 + t>(crec, a.ascale);
        xa[t] = (NM1 == 1) ? xv : xv * C.ga[t];
      } else if constexpr (NM1 == 1) {
        xa[t] = __builtin_bit_cast(float, row_bcast<4 * NM1 + t>(crec));
      } else {
        xa[t] = bcast_mul<4 * NM1 + t>(crec, C.ga[t]);
      }
      xb[t] = C.gb[t];
    });
    gather(nrec, N2);
    const int32_t eb = blk * 16;  // uniform
    auto product = [&](const float* av) {
      if constexpr (PREC == P_FP32) {
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = mfma4(av[t], __builtin_bit_cast(float, xb[t]), acc[t]);
      } else {
        acc[ci] = mfma16<PREC>(av, xb, acc[ci]);
      }
    };
    if (__builtin_expect(seg_lo <= eb && seg_hi > eb + 16, 1)) {
      // the slice continues past this block
      product(xa);
    } else {
      // every slice touching the block: masked products (lanes outside give 0)
      while (!done && seg_lo < eb + 16) {
        float am[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int32_t e = eb + 4 * t + g;
          am[t] = (e >= seg_lo && e < seg_hi) ? xa[t] : 0.f;
        }
        product(am);
        if (seg_hi > eb + 16) break;  // continues into the next block
        // slice s ends in this block
        f4 y = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        if constexpr (PREC != P_FP32) y *= a.yscale;
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
        on_seg(s, win.get_row(s), y);
        s = s + 1;
        if (s > s_last) {
          done = true;
        } else {
          if (s + 1 - win.base >= 64) win.load(a, s, lane);
          seg_lo = win.get_off(s);
          const int32_t nx = win.get_off(s + 1);
          seg_hi = nx < hi ? nx : hi;
        }
      }
    }
  };

  // Three register sets of rows rotated by renaming and the records in
  // three groups of three blocks: the rows of block b + 2 are gathered at
  // block b, and the records of group i + 2 are loaded when group i starts,
  // so waiting for a gather's record does not drain the rows in flight
  // (vector loads complete in order); by the end of group i its waits have
  // covered the loads issued when it started, so the records move on
  // between groups without waiting.
  PipeSet<NM1> S0, S1, S2;
  int32_t qc[3], qn[3], qf[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) qc[j] = load_rec(b0 + j);
#pragma unroll
  for (int j = 0; j < 3; ++j) qn[j] = load_rec(b0 + 3 + j);
  __builtin_amdgcn_sched_barrier(0);
  gather(qc[0], S0);
  gather(qc[1], S1);
  __builtin_amdgcn_sched_barrier(0);
  for (int32_t ib = 0; ib < nblk; ib += 3) {
#pragma unroll
    for (int j = 0; j < 3; ++j) qf[j] = load_rec(b0 + ib + 6 + j);
    __builtin_amdgcn_sched_barrier(0);
    step(b0 + ib, qc[0], S0, qc[2], S2, 0);
    if (done || ib + 1 >= nblk) break;
    step(b0 + ib + 1, qc[1], S1, qn[0], S0, 1);
    if (done || ib + 2 >= nblk) break;
    step(b0 + ib + 2, qc[2], S2, qn[1], S1, 2);
    if (done) break;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      qc[j] = qn[j];
      qn[j] = qf[j];
    }
  }
}

// ---------------------------------------------------------------------------
// TTMcTC pass
// ---------------------------------------------------------------------------
// LDS of the TTMcTC pass (floats): staged y_i, cross-wave reduction (several
// tiles), slot table, slice-table windows.
__host__ __device__ inline int ttm_lds_floats(const SegArgs& a, int KN2) {
  const int multi = a.B > 1;
  return a.B * a.RPW * stage_slots(a.B) * YS + (multi ? a.RPW * a.B * KN2 * 256 : 0) + a.RPW * 32 +
         a.B * a.RPW * 128;
}

template <int NM1, int KN2, int PREC>
__device__ inline void ttm_body(const SegArgs& a, const int wg) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int rr = wv / a.B;
  const int b = wv - rr * a.B;
  const int rb = b / a.CB, cb = b - (b / a.CB) * a.CB;
  const int g = lane >> 4, q = lane & 15;
  const int32_t w = wg * a.RPW + rr;
  const bool multi = a.B > 1;

  const int SLOTS = stage_slots(a.B);
  float* ybat = lds + wv * (SLOTS * YS);
  float* red = lds + a.B * a.RPW * SLOTS * YS + rr * (a.B * KN2 * 256);
  int32_t* slot_base =
      reinterpret_cast<int32_t*>(lds + a.B * a.RPW * SLOTS * YS + (multi ? a.RPW * a.B * KN2 * 256 : 0));
  int32_t* slot_row = slot_base + rr * 32;
  int32_t* slot_kind = slot_row + 16;
  int32_t* wlds = slot_base + a.RPW * 32 + wv * 128;  // slice-table window of this wave

  // stage-two operand of this block, read from memory (L1/L2-resident: the
  // same few kilobytes for every workgroup): step u reads the contiguous
  // kilobyte gtl[(kb * 16 + u) * 256 ..], G_(n)^T[64 g + 4u + v][16 kb + q]
  const float* gtl = a.gtop + (size_t)b * KN2 * 4096 + lane * 4;

  uint32_t ka4, kb4, kc4;
  lane_offsets<NM1, PREC>(a, rb, cb, q, &ka4, &kb4, &kc4);
  if (w >= a.W) return;  // only when B == 1 (no workgroup barriers then)

  const int32_t lo = range_lo(w, a.W, a.nnz);
  const int32_t hi = range_lo(w + 1, a.W, a.nnz);
  int32_t s_first, s_last;
  find_seg2(a.seg_off, a.R, lo, hi - 1, &s_first, &s_last);
  const bool head_clip = a.seg_off[s_first] < lo;
  const bool tail_clip = a.seg_off[s_last + 1] > hi;
  if (b == 0 && lane == 0) {
    a.meta[w * 4 + 0] = s_first;
    a.meta[w * 4 + 1] = s_last;
    a.meta[w * 4 + 2] = (head_clip ? 1 : 0) | (tail_clip ? 2 : 0);
    a.meta[w * 4 + 3] = 0;
  }

  int slot = 0;
  // stage two: D[slot][kn] = sum_j' ybat[slot][j'] * G_(n)^T[j'][kn] for the staged slices
  auto stage_two = [&]() {
    if (!multi) wave_sync();
    f4 d[KN2];
#pragma unroll
    for (int kb = 0; kb < KN2; ++kb) d[kb] = f4{0.f, 0.f, 0.f, 0.f};
    // rows q >= SLOTS of the product are not used: they re-read staged rows
    const float* yrow = ybat + (q & (SLOTS - 1)) * YS + 64 * g;
#pragma unroll 4
    for (int u = 0; u < 16; ++u) {
      const f4 yv = *reinterpret_cast<const f4*>(yrow + 4 * u);
#pragma unroll
      for (int kb = 0; kb < KN2; ++kb) {
        const f4 gv = *reinterpret_cast<const f4*>(gtl + (kb * 16 + u) * 256);
#pragma unroll
        for (int v = 0; v < 4; ++v) d[kb] = mfma4(yv[v], gv[v], d[kb]);
      }
    }
    if (multi) {
#pragma unroll
      for (int kb = 0; kb < KN2; ++kb)
        *reinterpret_cast<f4*>(red + (b * KN2 + kb) * 256 + q * 16 + 4 * g) = d[kb];
      __syncthreads();
      if (b == 0) {
#pragma unroll
        for (int kb = 0; kb < KN2; ++kb) {
          f4 t = *reinterpret_cast<const f4*>(red + kb * 256 + q * 16 + 4 * g);
          for (int bb = 1; bb < a.B; ++bb)
            t += *reinterpret_cast<const f4*>(red + (bb * KN2 + kb) * 256 + q * 16 + 4 * g);
          d[kb] = t;
        }
      }
    }
    if (b == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int sl = 4 * g + v;
        if (sl < slot) {
          const int32_t row = slot_row[sl];
          const int kind = slot_kind[sl];
#pragma unroll
          for (int kb = 0; kb < KN2; ++kb) {
            const int kn = 16 * kb + q;
            if (kn < a.Kn) {
              const float val = d[kb][v];
              if (kind == KIND_COMPLETE) a.A[(size_t)row * a.Kn + kn] = val;
              else a.carry[((size_t)w * 2 + (kind == KIND_TAIL ? 1 : 0)) * 32 + kn] = val;
            }
          }
        }
      }
    }
    if (a.yrow) {
      // keep the staged y_s for the core of the updated factor: row by label
      // (slot_row: out_map is null here); a split slice leaves its partial per
      // range and zeros in its own row
      // (buffer stores: row bases in scalar registers, no per-lane 64-bit addresses)
      const size_t yrowf = (size_t)a.B * 256;
      const uint32_t vo = (uint32_t)(b * 256 + 4 * lane) * 4u;
      for (int sl = 0; sl < slot; ++sl) {
        const int32_t row = __builtin_amdgcn_readfirstlane(slot_row[sl]);
        const int kind = __builtin_amdgcn_readfirstlane(slot_kind[sl]);
        const i4 yv = __builtin_bit_cast(i4, *reinterpret_cast<const f4*>(ybat + sl * YS + 4 * lane));
        const auto own = make_rsrc(a.yrow + (size_t)row * yrowf, (uint32_t)(yrowf * 4));
        if (kind == KIND_COMPLETE) {
          __builtin_amdgcn_raw_buffer_store_b128(yv, own, vo, 0, 0);
        } else {
          const auto dst = make_rsrc(a.ycarry + ((size_t)w * 2 + (kind == KIND_TAIL ? 1 : 0)) * yrowf,
                                     (uint32_t)(yrowf * 4));
          __builtin_amdgcn_raw_buffer_store_b128(yv, dst, vo, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b128(i4{0, 0, 0, 0}, own, vo, 0, 0);
        }
      }
    }
    if (multi) __syncthreads();
    else wave_sync();
    slot = 0;
  };

  walk_range<NM1, PREC>(a, lo, hi, s_first, s_last, ka4, kb4, kc4, lane, wlds, [&](int32_t s, int32_t row, f4 y) {
    // stage y_s (column-major within the block: j' = c*16 + r)
    *reinterpret_cast<f4*>(ybat + slot * YS + q * 16 + 4 * g) = y;
    if (b == 0 && lane == 0) {
      int kind = KIND_COMPLETE;
      if (s == s_first && head_clip) kind = KIND_HEAD;
      else if (s == s_last && tail_clip) kind = KIND_TAIL;
      slot_row[slot] = a.out_map ? scalar_ld(a.out_map, row) : row;
      slot_kind[slot] = kind;
    }
    if (++slot == SLOTS) stage_two();
  });
  if (slot > 0) stage_two();
}

template <int NM1, int KN2, int PREC>
__global__ __launch_bounds__(512) void k_ttm(SegArgs a) {
  ttm_body<NM1, KN2, PREC>(a, blockIdx.x);
}

// The same pass held to 128 registers (four waves per SIMD) for the
// instances whose allocation lands above that: the 3-way FP32 pass fits
// without spilling; the 4-way passes spill a few registers and still run
// faster than at three waves per SIMD (their workgroups of up to 8 waves
// otherwise fit only once per CU).
template <int NM1, int KN2, int PREC>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_ttm_w4(SegArgs a) {
  ttm_body<NM1, KN2, PREC>(a, blockIdx.x);
}
template <int NM1, int KN2, int PREC>
constexpr bool ttm_hold4() {
  return (NM1 == 2 && KN2 == 1 && PREC == P_FP32) || NM1 == 3;
}

template <int NM1, int KN2, int PREC>
__global__ __launch_bounds__(512) void k_ttm_b(const SegArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  ttm_body<NM1, KN2, PREC>(d[r], blockIdx.x - first[r]);
}

// ---------------------------------------------------------------------------
// TTMcTC pass, BF16 form, for a y_i of 2 x 2 blocks (3-way tensors whose two
// other ranks both lie in 17..32): one wave computes all four 16x16 blocks of
// y_i, so every nonzero's record is read and its factor rows are gathered once
// per range instead of once per block and wave. Block (rb, cb) multiplies
// entries 16 rb + q of the first and 16 cb + q of the second other factor;
// lane group g holds the k-slots 4g + t as in walk_range. A finished y_i is
// staged in LDS in bfloat16 and multiplied by G_(n)^T (bfloat16 copy) on the
// matrix cores with float32 accumulation; the stored slice rows of Y_(n) are
// those same bfloat16 values (2 KB per slice at 32 x 32 instead of 4 KB), so
// the core of the updated factor sees exactly the y_i the product with the
// core saw.
// ---------------------------------------------------------------------------
constexpr int kYs22 = 1024 + 16;  // LDS entries per staged y_i (the pad puts slots 8 banks apart)
// Register sets of the block pipeline: while block b is multiplied, the rows
// of blocks b+1 .. b+kStages22-1 and the record of b+kStages22 are in flight.
constexpr int kStages22 = 4;
__host__ __device__ constexpr int ttm22_wave_bytes(int slots) { return slots * kYs22 * 2 + (2 * slots + 128) * 4; }

// PAIR (both other ranks even): lane q gathers one dword per row, entries
// 2q and 2q + 1, and block (rb, cb) takes entries 2r + rb of the first and
// 2c + cb of the second other factor (half the gather instructions; the
// stage-two operand and the core's scatter follow the same order). Otherwise
// lane q gathers entries q and 16 + q, one 16-bit load each.
template <bool PAIR, typename OnSeg>
__device__ inline void walk_range22(const SegArgs& a, int32_t lo, int32_t hi, int32_t s_first, int32_t s_last,
                                    uint32_t k2, int lane, int32_t* wlds, OnSeg&& on_seg) {
  constexpr int NM1 = 2;
  constexpr int GD = 4 * (NM1 + 1);
  const int g = lane >> 4;
  const auto rRec = make_rsrc(a.rec, (uint32_t)a.nnz_pad * 4u * (NM1 + 1));
  const int qd = (lane & 15) < GD ? (lane & 15) : GD - 1;
  const uint32_t goff = (uint32_t)(g * GD + qd) * 4u;
  const auto rU0 = make_rsrc(a.U[0], a.Ubytes[0]);
  const auto rU1 = make_rsrc(a.U[1], a.Ubytes[1]);

  lo = __builtin_amdgcn_readfirstlane(lo);
  hi = __builtin_amdgcn_readfirstlane(hi);
  s_first = __builtin_amdgcn_readfirstlane(s_first);
  s_last = __builtin_amdgcn_readfirstlane(s_last);
  const int32_t b0 = lo >> 4;
  const int32_t nblk = ((hi - 1) >> 4) - b0 + 1;
  const int32_t bmax = (a.nnz_pad >> 4) - 1;

  // raw bfloat16 entries of k-slots t = 0..3, one per register: packing them
  // where they are loaded would make the loop wait for loads still in flight
  // (PAIR: ga[0][t] / gb[0][t] hold both entries of the lane's dword)
  struct Set {
    int32_t rec;        // the block's record (unpaired gathers: kept with the rows)
    uint32_t ga[2][4];  // first other factor, entry 16 rb + q
    uint32_t gb[2][4];  // second other factor, entry 16 cb + q
  };
  auto load_rec = [&](int32_t blk) -> int32_t {
    blk = blk <= bmax ? blk : bmax;
    return __builtin_amdgcn_raw_buffer_load_b32(rRec, goff, (uint32_t)blk * (64u * (NM1 + 1)), 0);
  };
  // the record holds byte offsets of the rows; entries 16..31 sit 32 bytes on
  auto gather = [&](int32_t rec, Set& S) {
    static_for<0, 4>([&](auto T) {
      constexpr int t = decltype(T)::value;
      const uint32_t oa = bcast_add<t>(rec, k2);
      const uint32_t ob = bcast_add<4 + t>(rec, k2);
      if constexpr (PAIR) {
        S.ga[0][t] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rU0, oa, 0, 0);
        S.gb[0][t] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rU1, ob, 0, 0);
      } else {
        S.ga[0][t] = ld_u16(rU0, oa);
        S.ga[1][t] = ld_u16(rU0, oa + 32u);
        S.gb[0][t] = ld_u16(rU1, ob);
        S.gb[1][t] = ld_u16(rU1, ob + 32u);
      }
    });
  };

  SegWindow win;
  win.off = wlds;
  win.row = wlds + 64;
  win.load(a, s_first, lane);
  int32_t s = s_first;
  int32_t seg_lo = lo;
  int32_t seg_hi = win.get_off(s_first + 1);
  seg_hi = __builtin_amdgcn_readfirstlane(seg_hi < hi ? seg_hi : hi);
  f4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = f4{0.f, 0.f, 0.f, 0.f};
  bool done = false;

  // block blk (record crec, rows in C); the rows of block blk + 3 (record
  // nrec) go to N2; unpaired gathers: C first receives the record of block
  // blk + kStages22
  auto step = [&](int32_t blk, int32_t crec, Set& C, int32_t nrec, Set& N2) {
    // A operands (x U_a, rounded to bfloat16 once) of row blocks rb = 0, 1 and
    // B operands of column blocks 0, 1, both as two dwords of packed k-slots
    u2 pa[2];
    s4 xb0, xb1;
    if constexpr (PAIR) {
      float xa[2][4];
      static_for<0, 4>([&](auto T) {
        constexpr int t = decltype(T)::value;
        xb0[t] = (short)(C.gb[0][t] & 0xffffu);
        xb1[t] = (short)(C.gb[0][t] >> 16);
        xa[0][t] = bcast_mul<4 * NM1 + t>(crec, __builtin_bit_cast(float, C.ga[0][t] << 16));
        xa[1][t] = bcast_mul<4 * NM1 + t>(crec, __builtin_bit_cast(float, C.ga[0][t] & 0xffff0000u));
      });
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
        pa[rb] = __builtin_bit_cast(u2, b4{(__bf16)xa[rb][0], (__bf16)xa[rb][1], (__bf16)xa[rb][2], (__bf16)xa[rb][3]});
    } else {
      float xa[2][4];
      xb0 = s4{(short)C.gb[0][0], (short)C.gb[0][1], (short)C.gb[0][2], (short)C.gb[0][3]};
      xb1 = s4{(short)C.gb[1][0], (short)C.gb[1][1], (short)C.gb[1][2], (short)C.gb[1][3]};
      static_for<0, 4>([&](auto T) {
        constexpr int t = decltype(T)::value;
#pragma unroll
        for (int h = 0; h < 2; ++h) xa[h][t] = bcast_mul<4 * NM1 + t>(crec, f16bits_to_f32<P_BF16>(C.ga[h][t]));
      });
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
        pa[rb] = __builtin_bit_cast(u2, b4{(__bf16)xa[rb][0], (__bf16)xa[rb][1], (__bf16)xa[rb][2], (__bf16)xa[rb][3]});
    }
    if constexpr (!PAIR) C.rec = load_rec(blk + kStages22);
    gather(nrec, N2);
    const int32_t eb = blk * 16;
    auto product = [&](u2 m) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const s4 as = __builtin_bit_cast(s4, pa[rb] & m);
        acc[2 * rb + 0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as, xb0, acc[2 * rb + 0], 0, 0, 0);
        acc[2 * rb + 1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as, xb1, acc[2 * rb + 1], 0, 0, 0);
      }
    };
    if (__builtin_expect(seg_lo <= eb && seg_hi > eb + 16, 1)) {
      product(u2{0xffffffffu, 0xffffffffu});
    } else {
      while (!done && seg_lo < eb + 16) {
        // k-slot t of lane group g is nonzero eb + 4t + g: keep the 16-bit
        // halves of the slots inside the slice, zero the others
        uint32_t mk[2];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          const int32_t e0 = eb + 8 * d + g, e1 = e0 + 4;
          mk[d] = ((e0 >= seg_lo && e0 < seg_hi) ? 0x0000ffffu : 0u) | ((e1 >= seg_lo && e1 < seg_hi) ? 0xffff0000u : 0u);
        }
        product(u2{mk[0], mk[1]});
        if (seg_hi > eb + 16) break;
        on_seg(s, win.get_row(s), acc);
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = f4{0.f, 0.f, 0.f, 0.f};
        s = s + 1;
        if (s > s_last) {
          done = true;
        } else {
          if (s + 1 - win.base >= 64) win.load(a, s, lane);
          seg_lo = win.get_off(s);
          const int32_t nx = win.get_off(s + 1);
          seg_hi = nx < hi ? nx : hi;
        }
      }
    }
  };

  // Four register sets of rows rotated by renaming (the loop is unrolled
  // over them; every index is a constant); the rows of block b + 3 are
  // gathered at block b. Paired gathers: the records come in groups of four
  // blocks, and those of group i + 2 are loaded when group i starts, so a
  // gather's record arrived long before and waiting for it does not drain
  // the rows in flight (vector loads complete in order); by the end of group
  // i its waits have covered the loads issued when it started, so the
  // records move on between groups without waiting. Unpaired gathers (twice
  // the rows per set, no registers to spare): each set keeps its block's
  // record, loaded one block ahead of its gathers. The prologues issue in
  // their loop's own order, held by scheduling barriers.
  constexpr int NS = kStages22;
  static_assert(NS == 4, "the record groups have four blocks");
  Set S[NS];
  if constexpr (PAIR) {
    int32_t qc[4], qn[4], qf[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) qc[j] = load_rec(b0 + j);
#pragma unroll
    for (int j = 0; j < 4; ++j) qn[j] = load_rec(b0 + 4 + j);
    __builtin_amdgcn_sched_barrier(0);
    gather(qc[0], S[0]);
    gather(qc[1], S[1]);
    gather(qc[2], S[2]);
    __builtin_amdgcn_sched_barrier(0);
    for (int32_t ib = 0; ib < nblk; ib += NS) {
#pragma unroll
      for (int j = 0; j < 4; ++j) qf[j] = load_rec(b0 + ib + 8 + j);
      __builtin_amdgcn_sched_barrier(0);
      bool stop = false;
      static_for<0, NS>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (stop) return;
        step(b0 + ib + i, qc[i], S[i], i == 0 ? qc[3] : qn[i - 1], S[(i + NS - 1) % NS]);
        if (done || ib + i + 1 >= nblk) stop = true;
      });
      if (stop) break;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        qc[j] = qn[j];
        qn[j] = qf[j];
      }
    }
  } else {
    S[0].rec = load_rec(b0);
    S[1].rec = load_rec(b0 + 1);
    gather(S[0].rec, S[0]);
    static_for<2, NS>([&](auto I) {
      constexpr int i = decltype(I)::value;
      S[i].rec = load_rec(b0 + i);
      __builtin_amdgcn_sched_barrier(0);
      gather(S[i - 1].rec, S[i - 1]);
    });
    __builtin_amdgcn_sched_barrier(0);
    for (int32_t ib = 0; ib < nblk; ib += NS) {
      bool stop = false;
      static_for<0, NS>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if (stop) return;
        constexpr int pv = (i + NS - 1) % NS;
        step(b0 + ib + i, S[i].rec, S[i], S[pv].rec, S[pv]);
        if (done || ib + i + 1 >= nblk) stop = true;
      });
      if (stop) break;
    }
  }
}

// The pass itself: one wave per range. Finished slices go into a pool of
// the workgroup (two banks of 16 bfloat16 y_i in LDS); the wave that fills
// the 16th slot of a bank multiplies all 16 by the bfloat16 G_(n)^T on
// v_mfma_f32_16x16x32_bf16 (each of the 16 operand rows a slice) and stores
// their rows of A, so stage two reads the core operand once per 16 slices
// (a wave's own four staged slices used a quarter of each product and read
// it once per four).
// The core operand is gtop16[kb][32][lane][8] with
// gtop16[kb][8 b + u][lane][t] = G_(n)^T[256 b + 32 u + 8 (lane/16) + t][16 kb + lane%16]
// (inside block b, index c*16 + r), which k_prep_gtop writes for this pass;
// the workgroup first copies it into LDS (KN2 x 32 KB).
// Pool protocol (counters in LDS, atomics by lane 0):
//  claim idx = claims++: bank (idx / 16) % 2, slot idx % 16, round idx / 32;
//  wait until done[bank] == round (the bank's earlier rounds multiplied);
//  write y_i and its (row, kind, range) into the slot, then filled[bank]++;
//  the wave whose increment fills the bank multiplies it, sets filled = 0
//  and then done[bank] = round + 1.
// A claimed slot is written by its claimer right after its wait, and a wait
// is only for an earlier round of the same bank, so by induction over rounds
// every wait ends. The last wave of the workgroup to finish its range
// multiplies the partly filled bank. Waits are still bounded (kPoolSpin
// sleeps): past that a wave records a fault in *a.fault, tells the others to
// stop waiting, and goes on, so a fault in the protocol cannot hang the GPU.
constexpr int kPoolSlots = 16;
constexpr int kPoolSpin = 1 << 22;
struct PoolCounters {
  uint32_t claims, finished, filled[2], done[2], abort, pad;
};
__host__ __device__ constexpr int ttm22_pool_bytes() {
  return 2 * kPoolSlots * kYs22 * 2 + 2 * kPoolSlots * 3 * 4 + (int)sizeof(PoolCounters);
}
__host__ __device__ constexpr int ttm22_wave_bytes() { return 128 * 4; }  // the wave's slice-table window

__device__ inline uint32_t lds_fetch_add(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline uint32_t lds_load_acq(uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline void lds_store_rel(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int KN2, bool PAIR>
__device__ inline void ttm22_body(const SegArgs& a, const int wg) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int g = lane >> 4, q = lane & 15;
  const int32_t w = wg * a.RPW + wv;
  uint16_t* gl = reinterpret_cast<uint16_t*>(lds);
  char* pbase = reinterpret_cast<char*>(lds) + KN2 * 32768;
  uint16_t* pool = reinterpret_cast<uint16_t*>(pbase);                                 // [2][16][kYs22]
  int32_t* pmeta = reinterpret_cast<int32_t*>(pbase + 2 * kPoolSlots * kYs22 * 2);    // [2][16][3]
  PoolCounters* pc = reinterpret_cast<PoolCounters*>(pmeta + 2 * kPoolSlots * 3);
  int32_t* wlds = reinterpret_cast<int32_t*>(pbase + ttm22_pool_bytes()) + wv * 128;  // slice-table window
  {
    // eight 16-byte loads in flight per thread before their LDS stores
    const i4* src = reinterpret_cast<const i4*>(a.gtop);
    i4* dst = reinterpret_cast<i4*>(gl);
    const int nt = (int)blockDim.x;
    for (int base = 0; base < KN2 * 2048; base += 8 * nt) {
      i4 t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = base + (int)threadIdx.x + u * nt;
        t[u] = i < KN2 * 2048 ? src[i] : i4{0, 0, 0, 0};
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = base + (int)threadIdx.x + u * nt;
        if (i < KN2 * 2048) dst[i] = t[u];
      }
    }
    if (threadIdx.x == 0) *pc = PoolCounters{};
    __syncthreads();
  }
  if (w >= a.W) return;  // past the barrier: the waves meet only through the pool from here
  // waves of this workgroup that walk a range
  const int32_t nact = __builtin_amdgcn_readfirstlane(a.W - wg * a.RPW < a.RPW ? a.W - wg * a.RPW : a.RPW);

  const int32_t lo = range_lo(w, a.W, a.nnz);
  const int32_t hi = range_lo(w + 1, a.W, a.nnz);
  int32_t s_first, s_last;
  find_seg2(a.seg_off, a.R, lo, hi - 1, &s_first, &s_last);
  const bool head_clip = a.seg_off[s_first] < lo;
  const bool tail_clip = a.seg_off[s_last + 1] > hi;
  if (lane == 0) {
    a.meta[w * 4 + 0] = s_first;
    a.meta[w * 4 + 1] = s_last;
    a.meta[w * 4 + 2] = (head_clip ? 1 : 0) | (tail_clip ? 2 : 0);
    a.meta[w * 4 + 3] = 0;
  }
  const uint16_t* gt = gl + lane * 8;
  constexpr uint32_t yrowf = 1024;  // entries per stored row (4 blocks, bfloat16)

  // one atomic per wave (lane 0), result on every lane
  auto wave_add = [&](uint32_t* ctr) -> uint32_t {
    uint32_t r = 0;
    if (lane == 0) r = lds_fetch_add(ctr, 1u);
    return __builtin_amdgcn_readfirstlane(r);
  };
  auto pool_wait = [&](int bank, uint32_t round) {
    for (int spins = 0;; ++spins) {
      const uint32_t dn = __builtin_amdgcn_readfirstlane(lds_load_acq(&pc->done[bank]));
      const uint32_t ab = __builtin_amdgcn_readfirstlane(lds_load_acq(&pc->abort));
      if (dn >= round || ab != 0) break;
      if (spins >= kPoolSpin) {
        if (lane == 0) {
          lds_store_rel(&pc->abort, 1u);
          *a.fault = 1;
        }
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  };
  // stage two of the first n slots of a bank: D[slot][kn] = y_slot . G_(n)^T[:, kn]
  auto pool_product = [&](int bank, int n) {
    f4 d[KN2];
#pragma unroll
    for (int kb = 0; kb < KN2; ++kb) d[kb] = f4{0.f, 0.f, 0.f, 0.f};
    // lane group g takes the 8 consecutive indices 32 u + 8 g .. of each 32-wide
    // step u (v_mfma_f32_16x16x32_bf16 contracts a lane group's 8 entries of A
    // with the same group's 8 of B); rows of unfilled slots are not stored
    const uint16_t* yr = pool + (bank * kPoolSlots + q) * kYs22 + 8 * g;
    // fully unrolled: every LDS address is a base register plus an immediate
#pragma unroll
    for (int bu = 0; bu < 32; ++bu) {
      const b8 av = *reinterpret_cast<const b8*>(yr + 32 * bu);
#pragma unroll
      for (int kb = 0; kb < KN2; ++kb) {
        const b8 bv = *reinterpret_cast<const b8*>(gt + (kb * 32 + bu) * 512);
        d[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, d[kb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int sl = 4 * g + v;
      if (sl < n) {
        const int32_t* m = pmeta + (bank * kPoolSlots + sl) * 3;
        const int32_t row = m[0], kind = m[1], rw = m[2];
#pragma unroll
        for (int kb = 0; kb < KN2; ++kb) {
          const int kn = 16 * kb + q;
          if (kn < a.Kn) {
            const float val = d[kb][v];
            if (kind == KIND_COMPLETE) a.A[(size_t)row * a.Kn + kn] = val;
            else a.carry[((size_t)rw * 2 + (kind == KIND_TAIL ? 1 : 0)) * 32 + kn] = val;
          }
        }
      }
    }
  };

  walk_range22<PAIR>(a, lo, hi, s_first, s_last, (uint32_t)q * (PAIR ? 4u : 2u), lane, wlds,
                       [&](int32_t s, int32_t row, const f4* y) {
    int kind = KIND_COMPLETE;
    if (s == s_first && head_clip) kind = KIND_HEAD;
    else if (s == s_last && tail_clip) kind = KIND_TAIL;
    // y_s in bfloat16 (nearest even), block b at 256 b + c*16 + r
    u2 yb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const b4 v = {(__bf16)y[b].x, (__bf16)y[b].y, (__bf16)y[b].z, (__bf16)y[b].w};
      yb[b] = __builtin_bit_cast(u2, v);
    }
    if (a.yrow) {
      // the bfloat16 y_s for the core of the updated factor: row by label; a
      // split slice leaves its partial per range and zeros in its own row
      const uint32_t vo = (uint32_t)(q * 16 + 4 * g) * 2u;
      uint16_t* const yrow16 = reinterpret_cast<uint16_t*>(a.yrow);
      const auto own = make_rsrc(yrow16 + (size_t)row * yrowf, yrowf * 2u);
      if (kind == KIND_COMPLETE) {
#pragma unroll
        for (int b = 0; b < 4; ++b) __builtin_amdgcn_raw_buffer_store_b64(yb[b], own, vo + 512u * b, 0, 0);
      } else {
        uint16_t* const yc16 = reinterpret_cast<uint16_t*>(a.ycarry);
        const auto dst = make_rsrc(yc16 + ((size_t)w * 2 + (kind == KIND_TAIL ? 1 : 0)) * yrowf, yrowf * 2u);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          __builtin_amdgcn_raw_buffer_store_b64(yb[b], dst, vo + 512u * b, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b64(u2{0u, 0u}, own, vo + 512u * b, 0, 0);
        }
      }
    }
    // into the pool
    const uint32_t idx = wave_add(&pc->claims);
    const int bank = (int)((idx >> 4) & 1u), slot = (int)(idx & 15u);
    const uint32_t round = idx >> 5;
    pool_wait(bank, round);
    uint16_t* ys = pool + (bank * kPoolSlots + slot) * kYs22 + q * 16 + 4 * g;
#pragma unroll
    for (int b = 0; b < 4; ++b) *reinterpret_cast<u2*>(ys + 256 * b) = yb[b];
    if (lane == 0) {
      int32_t* m = pmeta + (bank * kPoolSlots + slot) * 3;
      m[0] = a.out_map ? scalar_ld(a.out_map, row) : row;
      m[1] = kind;
      m[2] = w;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // the slot's writes, every lane
    if (wave_add(&pc->filled[bank]) == kPoolSlots - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      pool_product(bank, kPoolSlots);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // every lane's reads of the bank
      if (lane == 0) {
        lds_store_rel(&pc->filled[bank], 0u);
        lds_store_rel(&pc->done[bank], round + 1);
      }
    }
  });
  // the last wave of the workgroup to finish multiplies the partly filled bank
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if (wave_add(&pc->finished) == (uint32_t)nact - 1) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint32_t c = __builtin_amdgcn_readfirstlane(lds_load_acq(&pc->claims));
    const int n = (int)(c & 15u);
    if (n > 0) pool_product((int)((c >> 4) & 1u), n);
  }
}

// One workgroup per CU: the core operand, the slice pool and up to 16 waves
// (four per SIMD: the pass fits in 128 registers).
constexpr int kMaxRpw22 = 16;

template <int KN2, bool PAIR>
__global__ __launch_bounds__(64 * kMaxRpw22) void k_ttm22(SegArgs a) {
  ttm22_body<KN2, PAIR>(a, blockIdx.x);
}
template <int KN2, bool PAIR>
__global__ __launch_bounds__(64 * kMaxRpw22) void k_ttm22_b(const SegArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  ttm22_body<KN2, PAIR>(d[r], blockIdx.x - first[r]);
}

// ---------------------------------------------------------------------------
// TTMcTC pass, 4-way tensors whose three other ranks are at most 16 (every
// operand form): y_i (K_a x K_b x K_c) is computed as accumulator tiles over (a, b), one
// per index c of the third other mode, four tiles per wave and ceil(K_c / 4)
// waves per range. Per k-slot a lane gathers one entry of each other factor's
// row (a = q, b = q, c = c0 + q for the wave's first tile c0); tile c
// multiplies x * U_a(., a) * U_c(., c) (the c entry broadcast from a lane of
// the lane group) by U_b(., b). A nonzero thus costs three gathers per lane
// and wave for four tiles of y_i, instead of three per 16x16 block of the
// (a K_b + b, c) layout. The waves of a range stage their tiles of finished
// y_i in LDS in float32, in the block layout of the other passes (blocks of
// 16 rows r = a K_b + b, columns c), store them from there as rows of Y_(n),
// and multiply them by G_(n)^T on the matrix cores, in bfloat16 in the 16-bit
// forms (float32 accumulation; bfloat16 keeps the range of y_i) and in
// float32 in the FP32 form, each wave over its own columns c, partial
// products added in LDS in a fixed order.
// ---------------------------------------------------------------------------
// c-tiles per wave: waves per range nw = ceil(K_c / 6), tiles per wave
// NC = ceil(K_c / nw) (4 to 6; fewer tiles than that still run 4)
constexpr int kMaxTiles4c = 6;
inline int tiles4c(int Kc, int* nw) {
  *nw = (Kc + kMaxTiles4c - 1) / kMaxTiles4c;
  const int nc = (Kc + *nw - 1) / *nw;
  return nc < 4 ? 4 : nc;
}

template <int PREC, int NC, typename OnSeg>
__device__ inline void walk_range4c(const SegArgs& a, int32_t lo, int32_t hi, int32_t s_first, int32_t s_last,
                                    uint32_t k2, uint32_t k2c, int lane, int32_t* wlds, OnSeg&& on_seg) {
  constexpr int NM1 = 3;
  constexpr int GD = 4 * (NM1 + 1);
  const int g = lane >> 4;
  const auto rRec = make_rsrc(a.rec, (uint32_t)a.nnz_pad * 4u * (NM1 + 1));
  const uint32_t goff = (uint32_t)(g * GD + (lane & 15)) * 4u;
  const auto rU0 = make_rsrc(a.U[0], a.Ubytes[0]);
  const auto rU1 = make_rsrc(a.U[1], a.Ubytes[1]);
  const auto rU2 = make_rsrc(a.U[2], a.Ubytes[2]);

  lo = __builtin_amdgcn_readfirstlane(lo);
  hi = __builtin_amdgcn_readfirstlane(hi);
  s_first = __builtin_amdgcn_readfirstlane(s_first);
  s_last = __builtin_amdgcn_readfirstlane(s_last);
  const int32_t b0 = lo >> 4;
  const int32_t nblk = ((hi - 1) >> 4) - b0 + 1;
  const int32_t bmax = (a.nnz_pad >> 4) - 1;

  // raw 16-bit entries of k-slots t = 0..3, one per register (see walk_range22)
  struct Set {
    uint32_t u0[4], u1[4], u2[4];
  };
  auto load_rec = [&](int32_t blk) -> int32_t {
    blk = blk <= bmax ? blk : bmax;
    return __builtin_amdgcn_raw_buffer_load_b32(rRec, goff, (uint32_t)blk * (64u * (NM1 + 1)), 0);
  };
  // records hold byte offsets of 16-bit rows (float32 rows: twice that)
  auto gather = [&](int32_t rec, Set& S) {
    static_for<0, 4>([&](auto T) {
      constexpr int t = decltype(T)::value;
      if constexpr (PREC == P_FP32) {
        const uint32_t o0 = (uint32_t)row_bcast<t>(rec) << 1, o1 = (uint32_t)row_bcast<4 + t>(rec) << 1,
                       o2 = (uint32_t)row_bcast<8 + t>(rec) << 1;
        S.u0[t] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rU0, o0 + k2, 0, 0);
        S.u1[t] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rU1, o1 + k2, 0, 0);
        S.u2[t] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rU2, o2 + k2c, 0, 0);
      } else {
        S.u0[t] = ld_u16(rU0, bcast_add<t>(rec, k2));
        S.u1[t] = ld_u16(rU1, bcast_add<4 + t>(rec, k2));
        S.u2[t] = ld_u16(rU2, bcast_add<8 + t>(rec, k2c));
      }
    });
  };

  SegWindow win;
  win.off = wlds;
  win.row = wlds + 64;
  win.load(a, s_first, lane);
  int32_t s = s_first;
  int32_t seg_lo = lo;
  int32_t seg_hi = win.get_off(s_first + 1);
  seg_hi = __builtin_amdgcn_readfirstlane(seg_hi < hi ? seg_hi : hi);
  f4 acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
  bool done = false;

  auto step = [&](int32_t blk, int32_t crec, Set& C, int32_t nrec, Set& N2) {
    float xa[4], uc[4];
    const s4 bv = {(short)C.u1[0], (short)C.u1[1], (short)C.u1[2], (short)C.u1[3]};
    static_for<0, 4>([&](auto T) {
      constexpr int t = decltype(T)::value;
      if constexpr (PREC == P_FP16) {
        // the scale goes first, so no intermediate can exceed the bound
        xa[t] = bcast_mul<4 * NM1 + t>(crec, a.ascale) * f16bits_to_f32<PREC>(C.u0[t]);
        uc[t] = f16bits_to_f32<PREC>(C.u2[t]);
      } else if constexpr (PREC == P_FP32) {
        xa[t] = bcast_mul<4 * NM1 + t>(crec, __builtin_bit_cast(float, C.u0[t]));
        uc[t] = __builtin_bit_cast(float, C.u2[t]);
      } else {
        xa[t] = bcast_mul<4 * NM1 + t>(crec, f16bits_to_f32<PREC>(C.u0[t]));
        uc[t] = f16bits_to_f32<PREC>(C.u2[t]);
      }
    });
    gather(nrec, N2);
    const int32_t eb = blk * 16;
    auto product = [&](const float* av) {
      if constexpr (PREC == P_FP16) {
        // packed half precision: x U_a(., a) rounded to float16 once, then one
        // packed product per pair of k-slots with the broadcast c entries
        const h2 xp0 = {(_Float16)av[0], (_Float16)av[1]}, xp1 = {(_Float16)av[2], (_Float16)av[3]};
        const int32_t up0 = (int32_t)(C.u2[0] | (C.u2[1] << 16)), up1 = (int32_t)(C.u2[2] | (C.u2[3] << 16));
        static_for<0, NC>([&](auto ci) {
          constexpr int c = decltype(ci)::value;
          const h2 a0 = xp0 * __builtin_bit_cast(h2, row_bcast<c>(up0));
          const h2 a1 = xp1 * __builtin_bit_cast(h2, row_bcast<c>(up1));
          const h4 ah = {a0.x, a0.y, a1.x, a1.y};
          acc[c] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah, __builtin_bit_cast(h4, bv), acc[c], 0, 0, 0);
        });
      } else if constexpr (PREC == P_FP32) {
        // float32: one v_mfma_f32_16x16x4f32 per k-slot t (k = lane group)
        static_for<0, NC>([&](auto ci) {
          constexpr int c = decltype(ci)::value;
#pragma unroll
          for (int t = 0; t < 4; ++t)
            acc[c] = mfma4(bcast_mul<c>(__builtin_bit_cast(int32_t, uc[t]), av[t]), __builtin_bit_cast(float, C.u1[t]),
                           acc[c]);
        });
      } else {
        static_for<0, NC>([&](auto ci) {
          constexpr int c = decltype(ci)::value;
          float ac[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) ac[t] = bcast_mul<c>(__builtin_bit_cast(int32_t, uc[t]), av[t]);
          acc[c] = mfma16v<PREC>(ac, bv, acc[c]);
        });
      }
    };
    if (__builtin_expect(seg_lo <= eb && seg_hi > eb + 16, 1)) {
      product(xa);
    } else {
      while (!done && seg_lo < eb + 16) {
        float am[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int32_t e = eb + 4 * t + g;
          am[t] = (e >= seg_lo && e < seg_hi) ? xa[t] : 0.f;
        }
        product(am);
        if (seg_hi > eb + 16) break;
        on_seg(s, win.get_row(s), acc);
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
        s = s + 1;
        if (s > s_last) {
          done = true;
        } else {
          if (s + 1 - win.base >= 64) win.load(a, s, lane);
          seg_lo = win.get_off(s);
          const int32_t nx = win.get_off(s + 1);
          seg_hi = nx < hi ? nx : hi;
        }
      }
    }
  };

  // records two groups of three blocks ahead of their gathers (see walk_range)
  Set S0, S1, S2;
  int32_t qc[3], qn[3], qf[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) qc[j] = load_rec(b0 + j);
#pragma unroll
  for (int j = 0; j < 3; ++j) qn[j] = load_rec(b0 + 3 + j);
  __builtin_amdgcn_sched_barrier(0);
  gather(qc[0], S0);
  gather(qc[1], S1);
  __builtin_amdgcn_sched_barrier(0);
  for (int32_t ib = 0; ib < nblk; ib += 3) {
#pragma unroll
    for (int j = 0; j < 3; ++j) qf[j] = load_rec(b0 + ib + 6 + j);
    __builtin_amdgcn_sched_barrier(0);
    step(b0 + ib, qc[0], S0, qc[2], S2);
    if (done || ib + 1 >= nblk) break;
    step(b0 + ib + 1, qc[1], S1, qn[0], S0);
    if (done || ib + 2 >= nblk) break;
    step(b0 + ib + 2, qc[2], S2, qn[1], S1);
    if (done) break;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      qc[j] = qn[j];
      qn[j] = qf[j];
    }
  }
}

constexpr int kSlots4c = 3;  // staged slices per stage-two product (six workgroups of two waves fit a CU)
__host__ __device__ constexpr int ttm4c_ys(int B) { return B * 256 + 4; }
// LDS of one range (workgroup of nw waves): staged slices, partial products
// of stage two, slot table, one slice-table window per wave.
__host__ __device__ constexpr int ttm4c_bytes(int B, int nw, int KN2) {
  return kSlots4c * ttm4c_ys(B) * 4 + nw * KN2 * 256 * 4 + 2 * kSlots4c * 4 + nw * 128 * 4;
}

// The pass: one workgroup of nw waves per range, NC c-tiles each. Stage two reads
// gtop16 in the layout of the 2 x 2-block pass generalised to B blocks
// ([kb][16 b + u][lane][t], u the column c inside block b), from memory:
// slices are long where this pass is used, so stage two is rare.
// CORE: the row-writing core pass of the same walk (the core mode's slice
// rows to a.yrow / a.ycarry for U^(c)T Y_(c); no product with a core).
template <int PREC, int NC, int KN2, bool CORE = false>
__device__ inline void ttm4c_body(const SegArgs& a, const int w) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int nw = blockDim.x >> 6;
  const int g = lane >> 4, q = lane & 15;
  const int B = a.B;
  const int YSB = ttm4c_ys(B);
  float* ybat = lds;
  float* red = lds + kSlots4c * YSB;
  int32_t* slot_row = reinterpret_cast<int32_t*>(red + nw * KN2 * 256);
  int32_t* slot_kind = slot_row + kSlots4c;
  int32_t* wlds = slot_kind + kSlots4c + wv * 128;
  // padded entries of the staged blocks are never written: zero them once
  for (int i = threadIdx.x; i < kSlots4c * YSB; i += blockDim.x) ybat[i] = 0.f;
  __syncthreads();

  const int32_t lo = range_lo(w, a.W, a.nnz);
  const int32_t hi = range_lo(w + 1, a.W, a.nnz);
  int32_t s_first, s_last;
  find_seg2(a.seg_off, a.R, lo, hi - 1, &s_first, &s_last);
  const bool head_clip = a.seg_off[s_first] < lo;
  const bool tail_clip = a.seg_off[s_last + 1] > hi;
  if (wv == 0 && lane == 0) {
    a.meta[w * 4 + 0] = s_first;
    a.meta[w * 4 + 1] = s_last;
    a.meta[w * 4 + 2] = (head_clip ? 1 : 0) | (tail_clip ? 2 : 0);
    a.meta[w * 4 + 3] = 0;
  }
  const int c0 = NC * wv;  // this wave's first column c
  const uint16_t* gt = reinterpret_cast<const uint16_t*>(a.gtop) + lane * 4;
  const float* gt32 = a.gtop + lane * 4;
  const uint32_t yrowf = (uint32_t)B * 256;
  const int K0 = a.K0, K1 = a.K1;
  const int cw = a.K2 - c0 < NC ? a.K2 - c0 : NC;  // columns of this wave

  int slot = 0;
  auto stage_two = [&]() {
    __syncthreads();  // every wave's tiles of the staged slices are in LDS
    if constexpr (!CORE) {
    f4 d[KN2];
#pragma unroll
    for (int kb = 0; kb < KN2; ++kb) d[kb] = f4{0.f, 0.f, 0.f, 0.f};
    const float* yr = ybat + (q % kSlots4c) * YSB + 4 * g;
    for (int b = 0; b < B; ++b) {
      for (int u = c0; u < c0 + cw; ++u) {
        const int bu = 16 * b + u;
        const f4 yv = *reinterpret_cast<const f4*>(yr + 16 * bu);
        if constexpr (PREC == P_FP32) {
          // float32 operand in the same order ([kb][16 b + u][lane][t]), one
          // v_mfma_f32_16x16x4f32 per t
#pragma unroll
          for (int kb = 0; kb < KN2; ++kb) {
            const f4 gv = *reinterpret_cast<const f4*>(gt32 + ((size_t)kb * 16 * B + bu) * 256);
#pragma unroll
            for (int t = 0; t < 4; ++t) d[kb] = mfma4(yv[t], gv[t], d[kb]);
          }
        } else {
          const b4 yb = {(__bf16)yv.x, (__bf16)yv.y, (__bf16)yv.z, (__bf16)yv.w};
          const s4 av = __builtin_bit_cast(s4, yb);
#pragma unroll
          for (int kb = 0; kb < KN2; ++kb) {
            const s4 gv = *reinterpret_cast<const s4*>(gt + ((size_t)kb * 16 * B + bu) * 256);
            d[kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, gv, d[kb], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int kb = 0; kb < KN2; ++kb) *reinterpret_cast<f4*>(red + (wv * KN2 + kb) * 256 + lane * 4) = d[kb];
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int kb = 0; kb < KN2; ++kb) {
        f4 t = d[kb];
        for (int w2 = 1; w2 < nw; ++w2) t += *reinterpret_cast<const f4*>(red + (w2 * KN2 + kb) * 256 + lane * 4);
        d[kb] = t;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int sl = 4 * g + v;
        if (sl < slot) {
          const int32_t row = slot_row[sl];
          const int kind = slot_kind[sl];
#pragma unroll
          for (int kb = 0; kb < KN2; ++kb) {
            const int kn = 16 * kb + q;
            if (kn < a.Kn) {
              const float val = d[kb][v];
              if (kind == KIND_COMPLETE) a.A[(size_t)row * a.Kn + kn] = val;
              else a.carry[((size_t)w * 2 + (kind == KIND_TAIL ? 1 : 0)) * 32 + kn] = val;
            }
          }
        }
      }
    }
    }  // !CORE
    if (a.yrow) {
      // the float32 y_s for the core of the updated factor (row by label; a
      // split slice leaves its partial per range and zeros in its own row);
      // the waves take the blocks in turn
      for (int sl = 0; sl < slot; ++sl) {
        const int32_t row = __builtin_amdgcn_readfirstlane(slot_row[sl]);
        const int kind = __builtin_amdgcn_readfirstlane(slot_kind[sl]);
        const auto own = make_rsrc(a.yrow + (size_t)row * yrowf, yrowf * 4u);
        const auto dst = make_rsrc(a.ycarry + ((size_t)w * 2 + (kind == KIND_TAIL ? 1 : 0)) * yrowf, yrowf * 4u);
        for (int b = wv; b < B; b += nw) {
          const uint32_t vo = (uint32_t)(b * 256 + 4 * lane) * 4u;
          const i4 yv = __builtin_bit_cast(i4, *reinterpret_cast<const f4*>(ybat + sl * YSB + b * 256 + 4 * lane));
          if (kind == KIND_COMPLETE) {
            __builtin_amdgcn_raw_buffer_store_b128(yv, own, vo, 0, 0);
          } else {
            __builtin_amdgcn_raw_buffer_store_b128(yv, dst, vo, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b128(i4{0, 0, 0, 0}, own, vo, 0, 0);
          }
        }
      }
    }
    __syncthreads();  // staged slices and the slot table are reused
    slot = 0;
  };

  constexpr uint32_t es = PREC == P_FP32 ? 4u : 2u;  // bytes per factor entry
  walk_range4c<PREC, NC>(a, lo, hi, s_first, s_last, (uint32_t)q * es, (uint32_t)(c0 + q) * es, lane, wlds,
                     [&](int32_t s, int32_t row, const f4* y) {
    // tile c0 + c, lane (g, q): y[a = 4g + v][b = q][c0 + c]; block row r = a K1 + b
    float* ys = ybat + slot * YSB;
    if (q < K1) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int av = 4 * g + v;
        if (av < K0) {
          const int r = av * K1 + q;
          float* yp = ys + (r >> 4) * 256 + (r & 15) + c0 * 16;
#pragma unroll
          for (int c = 0; c < NC; ++c)
            if (c < cw) yp[c * 16] = y[c][v] * a.yscale;
        }
      }
    }
    if (wv == 0 && lane == 0) {
      int kind = KIND_COMPLETE;
      if (s == s_first && head_clip) kind = KIND_HEAD;
      else if (s == s_last && tail_clip) kind = KIND_TAIL;
      slot_row[slot] = a.out_map ? scalar_ld(a.out_map, row) : row;
      slot_kind[slot] = kind;
    }
    if (++slot == kSlots4c) stage_two();
  });
  if (slot > 0) stage_two();
}

template <int PREC, int NC, int KN2>
__global__ __launch_bounds__(256) void k_ttm4c(SegArgs a) {
  ttm4c_body<PREC, NC, KN2>(a, blockIdx.x);
}
template <int PREC, int NC, int KN2>
__global__ __launch_bounds__(256) void k_ttm4c_b(const SegArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  ttm4c_body<PREC, NC, KN2>(d[r], blockIdx.x - first[r]);
}
template <int PREC, int NC>
__global__ __launch_bounds__(256) void k_core4c(SegArgs a) {
  ttm4c_body<PREC, NC, 1, true>(a, blockIdx.x);
}
template <int PREC, int NC>
__global__ __launch_bounds__(256) void k_core4c_b(const SegArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  ttm4c_body<PREC, NC, 1, true>(d[r], blockIdx.x - first[r]);
}

// Adds the partial rows of slices that cross range boundaries and writes them.
// One workgroup per range; only the owner of a split slice (the range where it
// starts, holding its tail partial) works: the head partials of the following
// ranges w0+1..w1 (thousands for the heaviest slices) are summed in float64 by
// thread groups (16 lanes per group when K_n <= 16, else 32) with a fixed
// stride and eight loads in flight, then the groups are added in order
// (deterministic).
__device__ inline void fix_body(const FixArgs& f, const int32_t w) {
  __shared__ double part[16][32];
  const int32_t* meta = f.meta;
  const float* carry = f.carry;
  const int32_t* seg_row = f.seg_row;
  const int32_t* seg_off = f.seg_off;
  const int32_t W = f.W, nnz = f.nnz, Kn = f.Kn;
  const int32_t* out_map = f.out_map;
  float* A = f.A;
  const int32_t s_first = meta[w * 4 + 0], s_last = meta[w * 4 + 1], flags = meta[w * 4 + 2];
  const bool head_clip = flags & 1, tail_clip = flags & 2;
  if (!(tail_clip && !(s_first == s_last && head_clip))) return;
  const int32_t s = s_last;
  // last range holding part of slice s: the largest w1 with w1 * nnz / W <= e_last
  const int64_t e_last = (int64_t)seg_off[s + 1] - 1;
  const int32_t w1 = (int32_t)(((e_last + 1) * (int64_t)W - 1) / nnz);
  const int gs = Kn <= 16 ? 16 : 32;  // lanes per group
  const int ng = 256 / gs;            // groups
  const int kn = threadIdx.x % gs, grp = threadIdx.x / gs;
  double acc = 0.0;
  if (kn < Kn) {
    // group grp adds ranges w+1+grp, w+1+grp+ng, ... in order, eight loads in flight
    int32_t w2 = w + 1 + grp;
    for (; w2 + 7 * ng <= w1; w2 += 8 * ng) {
      float c[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) c[i] = carry[((size_t)(w2 + i * ng) * 2 + 0) * 32 + kn];
#pragma unroll
      for (int i = 0; i < 8; ++i) acc += (double)c[i];
    }
    for (; w2 <= w1; w2 += ng) acc += (double)carry[((size_t)w2 * 2 + 0) * 32 + kn];
  }
  part[grp][kn] = acc;
  __syncthreads();
  if (threadIdx.x < gs && kn < Kn) {
    double t = (double)carry[((size_t)w * 2 + 1) * 32 + kn];
    for (int g2 = 0; g2 < ng; ++g2) t += part[g2][kn];
    const int32_t row = out_map ? out_map[seg_row[s]] : seg_row[s];
    A[(size_t)row * Kn + kn] = (float)t;
  }
}

__global__ __launch_bounds__(256) void k_fix_split(FixArgs f) { fix_body(f, blockIdx.x); }

__global__ __launch_bounds__(256) void k_fix_split_b(const FixArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  fix_body(d[r], blockIdx.x - first[r]);
}

// Zeroes the rows of empty slices: empty_row[r] (original order) or, with a
// null list, the contiguous label-order rows row0 .. row0+E-1.
__global__ void k_zero_rows(const int32_t* empty_row, int64_t row0, int64_t E, int32_t Kn, float* A) {
  const int64_t total = E * Kn;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / Kn;
    const int64_t row = empty_row ? empty_row[r] : row0 + r;
    A[(size_t)row * Kn + (t - r * Kn)] = 0.f;
  }
}


// gtop[b][kb][u][lane][v] = G_(n)^T[j'][kn] with j' = 64 (lane/16) + 4u + v
// inside block b (j' = c*16 + r), kn = 16 kb + lane%16; zero in padding. Step
// u of stage two reads one contiguous kilobyte (16 bytes per lane).
__device__ inline void prep_body(const PrepArgs& p, const int blk) {
  const int64_t total = (int64_t)p.B * p.KN2 * 4096;
  for (int64_t idx = blk * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)p.nblk * blockDim.x) {
    int lane = (int)((idx >> 2) & 63);
    int kb, b, jp;
    if (p.wide16 == 2) {
      // [kb][8 b + u][lane][t] (t < 8): index 32 u + 8 (lane/16) + t inside block b
      lane = (int)((idx >> 3) & 63);
      const int bu = (int)((idx >> 9) % (8 * p.B));
      kb = (int)(idx / (4096 * p.B));
      b = bu >> 3;
      jp = 32 * (bu & 7) + 8 * (lane >> 4) + (int)(idx & 7);
    } else if (p.wide16) {
      // [kb][16 b + u][lane][t]: index 16 u + 4 (lane/16) + t inside block b
      // (bfloat16; wide16 == 3: the same order in float32)
      const int bu = (int)((idx >> 8) % (16 * p.B));
      kb = (int)(idx / (4096 * p.B));
      b = bu >> 4;
      jp = 16 * (bu & 15) + 4 * (lane >> 4) + (int)(idx & 3);
    } else {
      const int t = (int)(((idx >> 8) & 15) * 4 + (idx & 3));
      const int64_t rest = idx >> 12;
      kb = (int)(rest % p.KN2);
      b = (int)(rest / p.KN2);
      jp = 64 * (lane >> 4) + t;
    }
    const int rb = b / p.CB, cb = b % p.CB;
    const int c = jp >> 4, r = jp & 15;
    // paired order of the 2 x 2-block pass: block (rb, cb) holds entries 2r + rb, 2c + cb
    const int rg = p.pair ? 2 * r + rb : 16 * rb + r, cg = p.pair ? 2 * c + cb : 16 * cb + c;
    const int kn = 16 * kb + (lane & 15);
    float v = 0.f;
    if (rg < p.krow && cg < p.kcol && kn < p.Kn) {
      int64_t flat = (int64_t)rg * p.kcol + cg;
      int64_t off = (int64_t)kn * p.gstride[p.mode];
      for (int m = p.nm1 - 1; m >= 0; --m) {
        const int64_t k = flat % p.Ko[m];
        flat /= p.Ko[m];
        off += k * p.gstride[p.om[m]];
      }
      v = p.G[off];
    }
    if (p.wide16 == 1 || p.wide16 == 2) reinterpret_cast<uint16_t*>(p.gtop)[idx] = __builtin_bit_cast(uint16_t, (__bf16)v);
    else p.gtop[idx] = v;
  }
}

__global__ void k_prep_gtop(PrepArgs p) { prep_body(p, blockIdx.x); }

__global__ void k_prep_gtop_b(const PrepArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  prep_body(d[r], blockIdx.x - first[r]);
}

// ---------------------------------------------------------------------------
// Core pass, row-writing form: y_i of every slice of the core mode c is
// written out (complete slices to their row of ybuf, partial rows of slices
// split across ranges to ycarry), then G_(c) = U^(c)T Y_(c) by a small product
// over the rows. Y_(c) has one row per nonempty slice of c (the mode with the
// fewest), so it is small; the walk itself keeps no partial G and needs LDS
// only for the slice-table window.
// ---------------------------------------------------------------------------
template <int NM1, int KN2, int PREC>
__device__ inline void core_rows_body(const SegArgs& a, const int wg) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int rr = wv / a.B;
  const int b = wv - rr * a.B;
  const int rb = b / a.CB, cb = b - (b / a.CB) * a.CB;
  const int g = lane >> 4, q = lane & 15;
  const int32_t w = wg * a.RPW + rr;
  int32_t* wlds = reinterpret_cast<int32_t*>(lds) + wv * 128;
  const size_t row = (size_t)a.B * 256;  // floats per slice row
  uint32_t ka4, kb4, kc4;
  lane_offsets<NM1, PREC>(a, rb, cb, q, &ka4, &kb4, &kc4);
  if (w >= a.W) return;  // only when B == 1 (no workgroup barriers)
  const int32_t lo = range_lo(w, a.W, a.nnz);
  const int32_t hi = range_lo(w + 1, a.W, a.nnz);
  int32_t s_first, s_last;
  find_seg2(a.seg_off, a.R, lo, hi - 1, &s_first, &s_last);
  const bool head_clip = a.seg_off[s_first] < lo;
  const bool tail_clip = a.seg_off[s_last + 1] > hi;
  if (b == 0 && lane == 0) {
    a.meta[w * 4 + 0] = s_first;
    a.meta[w * 4 + 1] = s_last;
    a.meta[w * 4 + 2] = (head_clip ? 1 : 0) | (tail_clip ? 2 : 0);
    a.meta[w * 4 + 3] = 0;
  }
  const int jo = b * 256 + q * 16 + 4 * g;  // this lane's 4 entries of the row (j' = c*16 + r)
  walk_range<NM1, PREC>(a, lo, hi, s_first, s_last, ka4, kb4, kc4, lane, wlds, [&](int32_t s, int32_t lrow, f4 y) {
    float* own = a.A + (size_t)lrow * row;
    float* dst = own;
    if (s == s_first && head_clip) dst = a.carry + ((size_t)w * 2 + 0) * row;
    else if (s == s_last && tail_clip) dst = a.carry + ((size_t)w * 2 + 1) * row;
    *reinterpret_cast<f4*>(dst + jo) = y;
    // a split slice's own row holds zeros (every range holding part of it
    // writes the same zeros); its partials enter the product from ycarry
    if (dst != own) *reinterpret_cast<f4*>(own + jo) = f4{0.f, 0.f, 0.f, 0.f};
  });
}

template <int NM1, int KN2, int PREC>
__global__ __launch_bounds__(512) void k_core_rows(SegArgs a) {
  core_rows_body<NM1, KN2, PREC>(a, blockIdx.x);
}

template <int NM1, int KN2, int PREC>
__global__ __launch_bounds__(512) void k_core_rows_b(const SegArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  core_rows_body<NM1, KN2, PREC>(d[r], blockIdx.x - first[r]);
}

// One block of 16 waves per (chunk, y-tile b): the partial product U^T Y over
// the chunk's rows on the matrix cores, 4 rows per product. The rows (the R
// complete slice rows, then the 2W split-slice partials) are taken in groups
// of 16; chunk c owns groups c, c + NC, c + 2 NC, ... of each part (NC =
// p.nchunk), so at any time the blocks read neighbouring groups rather than
// addresses a chunk length apart. Wave (rl, cq) takes columns
// j' = 64 cq .. 64 cq + 63 of tile b and every fourth of the chunk's groups,
// starting at rl: lane (g, q) loads entries 64 cq + 4q .. 4q+3 of row 4s + g
// of a group as one vector, and product c of a step takes component c, so its
// output column q stands for j' = 64 cq + 4q + c. The four row lanes' sums are
// added in order rl = 0, 1, 2, 3 (fixed order throughout).
// SPLIT (the 16-bit forms): each float32 operand is the sum of two bfloat16
// numbers (hi = nearest, lo = nearest of the rest, about 2^-16 relative) and a
// product of 16 rows takes three v_mfma_f32_16x16x16_bf16 (hi hi, hi lo,
// lo hi), k-slot 4g + t standing for row 4t + g, instead of four float32
// products of 4 rows.
// YB (rows stored in bfloat16 by the 2 x 2-block BF16 pass; with SPLIT): the
// row entries are exact bfloat16 operands, so a product of 16 rows takes two
// (hi y, lo y), and each lane loads 8 bytes per row instead of 16.
constexpr int kGemmThreads = 1024;
__device__ inline void split_bf16(const float* x, s4* hi, s4* lo) {
  const b4 h = {(__bf16)x[0], (__bf16)x[1], (__bf16)x[2], (__bf16)x[3]};
  const s4 hs = __builtin_bit_cast(s4, h);
  float r[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) r[t] = x[t] - __builtin_bit_cast(float, (uint32_t)(uint16_t)hs[t] << 16);
  const b4 l = {(__bf16)r[0], (__bf16)r[1], (__bf16)r[2], (__bf16)r[3]};
  *hi = hs;
  *lo = __builtin_bit_cast(s4, l);
}
// entry c (0..3) of 4 bfloat16 packed in two dwords, as raw bits
__device__ inline short bf16_part(u2 v, int c) {
  return (short)((c & 1) ? (v[c >> 1] >> 16) : (v[c >> 1] & 0xffffu));
}
template <int KTT, bool SPLIT, bool YB = false>
__device__ inline void core_gemm_body(const CoreGemmArgs& p, const int blk) {
  static_assert(!YB || SPLIT, "bfloat16 rows are read by the split products of the 16-bit forms");
  typedef typename std::conditional<YB, u2, f4>::type yv_t;
  constexpr int KTM = KTT == 0 ? 2 : KTT;
  __shared__ f4 red[3][4][KTM * 4][64];  // row lanes 1..3, column quarter, accumulator, lane
  // XCD-aware order: blocks are dealt to the eight XCDs in turn, and the B
  // tiles of a chunk (which read the same rows of U) get numbers 8 apart, so
  // they run on one XCD at about the same time and share its L2
  const int c_lo = blk & 7, rest = blk >> 3;
  const int c_hi = rest / p.B, b = rest - c_hi * p.B;
  const int chunk = 8 * c_hi + c_lo;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cq = wv & 3, rl = wv >> 2;
  const int g = lane >> 4, q = lane & 15;
  const size_t row = (size_t)p.B * 256;
  const int KT = KTT == 0 ? (p.KC >> 4) : KTT;
  f4 acc[KTM][4];
#pragma unroll
  for (int kt = 0; kt < KTM; ++kt)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[kt][c] = f4{0.f, 0.f, 0.f, 0.f};
  const int64_t NC = p.nchunk;
  const int64_t R = p.R;
  const int col = b * 256 + 64 * cq + 4 * q;
  auto product = [&](const yv_t* yv, float (*ua)[KTM]) {
    if constexpr (YB) {
      s4 yh[4];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        yh[c] = s4{bf16_part(yv[0], c), bf16_part(yv[1], c), bf16_part(yv[2], c), bf16_part(yv[3], c)};
#pragma unroll
      for (int kt = 0; kt < KTM; ++kt) {
        if (kt >= KT) continue;
        const float uc[4] = {ua[0][kt], ua[1][kt], ua[2][kt], ua[3][kt]};
        s4 uh, ul;
        split_bf16(uc, &uh, &ul);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          acc[kt][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(uh, yh[c], acc[kt][c], 0, 0, 0);
          acc[kt][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ul, yh[c], acc[kt][c], 0, 0, 0);
        }
      }
    } else if constexpr (SPLIT) {
      s4 yh[4], yl[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float yc[4] = {yv[0][c], yv[1][c], yv[2][c], yv[3][c]};
        split_bf16(yc, &yh[c], &yl[c]);
      }
#pragma unroll
      for (int kt = 0; kt < KTM; ++kt) {
        if (kt >= KT) continue;
        const float uc[4] = {ua[0][kt], ua[1][kt], ua[2][kt], ua[3][kt]};
        s4 uh, ul;
        split_bf16(uc, &uh, &ul);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          acc[kt][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(uh, yh[c], acc[kt][c], 0, 0, 0);
          acc[kt][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(uh, yl[c], acc[kt][c], 0, 0, 0);
          acc[kt][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ul, yh[c], acc[kt][c], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int kt = 0; kt < KTM; ++kt) {
          if (kt >= KT) continue;
          acc[kt][0] = mfma4(ua[st][kt], yv[st].x, acc[kt][0]);
          acc[kt][1] = mfma4(ua[st][kt], yv[st].y, acc[kt][1]);
          acc[kt][2] = mfma4(ua[st][kt], yv[st].z, acc[kt][2]);
          acc[kt][3] = mfma4(ua[st][kt], yv[st].w, acc[kt][3]);
        }
    }
  };
  // complete slice rows v < R (label v), groups j = chunk + NC (rl + 4i).
  // Loads go to clamped (valid) addresses and rows past R are masked only
  // after the barrier, so a group's loads are in flight together, and the
  // next group's loads are issued before a group's products.
  const int64_t NG = (R + 15) / 16;
  const yv_t yzero = {};
  // entries col .. col + 3 of stored row v (float32, or bfloat16 with YB)
  auto row_at = [&](const float* base, size_t v) -> yv_t {
    if constexpr (YB) return *reinterpret_cast<const u2*>(reinterpret_cast<const uint16_t*>(base) + v * row + col);
    else return *reinterpret_cast<const f4*>(base + v * row + col);
  };
  auto load_rows = [&](int64_t j, yv_t* y, float (*u)[KTM]) {
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int64_t v = 16 * j + 4 * st + g;
      const int64_t vv = v < R ? v : 0;
      y[st] = row_at(p.ybuf, (size_t)vv);
#pragma unroll
      for (int kt = 0; kt < KTM; ++kt) {
        const int k = 16 * kt + q;
        u[st][kt] = (kt < KT) ? p.Uc[(size_t)vv * p.Kc + (k < p.Kc ? k : 0)] : 0.f;
      }
    }
  };
  auto masked_product = [&](int64_t j, yv_t* y, float (*u)[KTM]) {
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const bool ok = j < NG && 16 * j + 4 * st + g < R;
      y[st] = ok ? y[st] : yzero;
#pragma unroll
      for (int kt = 0; kt < KTM; ++kt) u[st][kt] = (ok && 16 * kt + q < p.Kc) ? u[st][kt] : 0.f;
    }
    product(y, u);
  };
  yv_t yv[4], yn[4];
  float ua[4][KTM], un[4][KTM];
  const int64_t j0 = chunk + NC * rl, dj = 4 * NC;
  if (j0 < NG) {
    load_rows(j0, yv, ua);
    for (int64_t j = j0; j < NG; j += 2 * dj) {
      load_rows(j + dj, yn, un);
      __builtin_amdgcn_sched_barrier(0);
      masked_product(j, yv, ua);
      load_rows(j + 2 * dj, yv, ua);
      __builtin_amdgcn_sched_barrier(0);
      masked_product(j + dj, yn, un);
    }
  }
  // split-slice partials v = R + 2w + kind (head 0 / tail 1 of range w), when
  // valid; groups of 16 of them interleaved over the chunks the same way
  const int64_t NP = 2 * (int64_t)p.W;
  for (int64_t j = j0; 16 * j < NP; j += dj) {
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int64_t x = 16 * j + 4 * st + g;
      int32_t lab = -1;
      size_t src = 0;  // row of ycarry
      if (x < NP) {
        const int64_t w = x >> 1;
        const int kind = (int)(x & 1);
        const int32_t sf = p.ymeta[w * 4 + 0], sl = p.ymeta[w * 4 + 1], fl = p.ymeta[w * 4 + 2];
        const bool head = fl & 1;
        const bool tail = (fl & 2) && !(sf == sl && head);  // a slice clipped on both sides is a head
        if (kind == 0 ? head : tail) {
          src = (size_t)w * 2 + kind;
          lab = p.seg_row[kind == 0 ? sf : sl];
        }
      }
      yv[st] = lab >= 0 ? row_at(p.ycarry, src) : yzero;
#pragma unroll
      for (int kt = 0; kt < KTM; ++kt) {
        const int k = 16 * kt + q;
        const bool ok = lab >= 0 && kt < KT && k < p.Kc;
        ua[st][kt] = ok ? p.Uc[(size_t)lab * p.Kc + k] : 0.f;
      }
    }
    product(yv, ua);
  }
  // row lanes 1..3 hand their sums to row lane 0, which adds them in order
  if (rl > 0) {
#pragma unroll
    for (int kt = 0; kt < KTM; ++kt)
#pragma unroll
      for (int c = 0; c < 4; ++c) red[rl - 1][cq][kt * 4 + c][lane] = acc[kt][c];
  }
  __syncthreads();
  if (rl > 0) return;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int kt = 0; kt < KTM; ++kt)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[kt][c] += red[r][cq][kt * 4 + c][lane];
  // lane (g, q) holds D[kc = 16 kt + 4g + r][j' = 64 cq + 4q + c] in acc[kt][c][r]
  float* out = p.gpart + ((size_t)chunk * p.B + b) * p.KC * 256;
#pragma unroll
  for (int kt = 0; kt < KTM; ++kt) {
    if (kt >= KT) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kc = 16 * kt + 4 * g + r;
      *reinterpret_cast<f4*>(out + (size_t)kc * 256 + 64 * cq + 4 * q) =
          f4{acc[kt][0][r], acc[kt][1][r], acc[kt][2][r], acc[kt][3][r]};
    }
  }
}

// A from stored rows, one wave per 16-row group: lane (g, q) takes row q of
// the group and entries j' = 64 g + 4u + v of tile b (the stage-two operand's
// order), so the product is the TTMcTC pass's stage two with the rows read
// from memory: D(row 4g + v, kn = 16 kb + q) on every lane. Rows stored in
// bfloat16 (p.yb16) are widened exactly to float32.
__device__ inline void rows_a_body(const RowsAArgs& p, const int blk) {
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, q = lane & 15;
  const int64_t grp = (int64_t)blk * 4 + wv;
  if (grp >= p.groups) return;
  const size_t rowf = (size_t)p.B * 256;
  const int64_t R = p.R, NP = 2 * (int64_t)p.W;
  // where row x of the group comes from and goes to: complete rows v < R; then
  // the valid split-slice partials (head 0 / tail 1 of range w)
  // src: (buffer, entry offset of the row); dst: output row
  auto locate = [&](int64_t x, const float** src, size_t* soff, float** dst, int ld) -> bool {
    if (x < R) {
      *src = p.ybuf;
      *soff = (size_t)x * rowf;
      *dst = p.A + (size_t)(p.out_map ? p.out_map[x] : x) * ld;
      return true;
    }
    if (x >= R + NP) return false;
    const int64_t w = (x - R) >> 1;
    const int kind = (int)((x - R) & 1);
    const int32_t sf = p.ymeta[w * 4 + 0], sl = p.ymeta[w * 4 + 1], fl = p.ymeta[w * 4 + 2];
    const bool head = fl & 1;
    const bool tail = (fl & 2) && !(sf == sl && head);
    if (kind == 0 ? !head : !tail) return false;
    *src = p.ycarry;
    *soff = ((size_t)w * 2 + kind) * rowf;
    *dst = p.carry + ((size_t)w * 2 + kind) * 32;
    return true;
  };
  const float* src = p.ybuf;
  size_t soff = 0;
  float* dst = nullptr;
  const bool ok = locate(grp * 16 + q, &src, &soff, &dst, p.Kn);
  f4 d[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
  for (int b = 0; b < p.B; ++b) {
    const float* gtl = p.gtop + (size_t)b * p.KN2 * 4096 + lane * 4;
    const size_t yo = soff + b * 256 + 64 * g;
#pragma unroll 4
    for (int u = 0; u < 16; ++u) {
      f4 t;
      if (p.yb16) {
        const u2 h = *reinterpret_cast<const u2*>(reinterpret_cast<const uint16_t*>(src) + yo + 4 * u);
        t = f4{__builtin_bit_cast(float, h[0] << 16), __builtin_bit_cast(float, h[0] & 0xffff0000u),
               __builtin_bit_cast(float, h[1] << 16), __builtin_bit_cast(float, h[1] & 0xffff0000u)};
      } else {
        t = *reinterpret_cast<const f4*>(src + yo + 4 * u);
      }
      const f4 yv = ok ? t : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        if (kb >= p.KN2) break;
        const f4 gv = *reinterpret_cast<const f4*>(gtl + (kb * 16 + u) * 256);
#pragma unroll
        for (int v = 0; v < 4; ++v) d[kb] = mfma4(yv[v], gv[v], d[kb]);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float* s2;
    size_t o2;
    float* out;
    if (!locate(grp * 16 + 4 * g + v, &s2, &o2, &out, p.Kn)) continue;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const int kn = 16 * kb + q;
      if (kb < p.KN2 && kn < p.Kn) out[kn] = d[kb][v];
    }
  }
}

__global__ __launch_bounds__(256) void k_rows_a(RowsAArgs p) { rows_a_body(p, blockIdx.x); }

template <int KTT, bool SPLIT, bool YB>
__global__ __launch_bounds__(kGemmThreads) void k_core_gemm(CoreGemmArgs p) {
  core_gemm_body<KTT, SPLIT, YB>(p, blockIdx.x);
}

__global__ __launch_bounds__(kGemmThreads) void k_core_gemm_b(const CoreGemmArgs* d, const int32_t* first,
                                                              int count) {
  const int r = batch_item(first, count, blockIdx.x);
  core_gemm_body<0, false>(d[r], blockIdx.x - first[r]);
}

void launch_core_gemm(const CoreGemmArgs& m, int blocks, hipStream_t s) {
  if (m.yb16) {
    if (m.KC <= 16) hipLaunchKernelGGL((k_core_gemm<1, true, true>), dim3(blocks), dim3(kGemmThreads), 0, s, m);
    else hipLaunchKernelGGL((k_core_gemm<2, true, true>), dim3(blocks), dim3(kGemmThreads), 0, s, m);
  } else if (m.split) {
    if (m.KC <= 16) hipLaunchKernelGGL((k_core_gemm<1, true, false>), dim3(blocks), dim3(kGemmThreads), 0, s, m);
    else hipLaunchKernelGGL((k_core_gemm<2, true, false>), dim3(blocks), dim3(kGemmThreads), 0, s, m);
  } else {
    if (m.KC <= 16) hipLaunchKernelGGL((k_core_gemm<1, false, false>), dim3(blocks), dim3(kGemmThreads), 0, s, m);
    else hipLaunchKernelGGL((k_core_gemm<2, false, false>), dim3(blocks), dim3(kGemmThreads), 0, s, m);
  }
}

// ---------------------------------------------------------------------------
// Core pass
// ---------------------------------------------------------------------------
template <int NM1, int KN2, int PREC>
__device__ inline void core_body(const SegArgs& a, const int wg) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int rr = wv / a.B;
  const int b = wv - rr * a.B;
  const int rb = b / a.CB, cb = b - (b / a.CB) * a.CB;
  const int g = lane >> 4, q = lane & 15;
  const int32_t w = wg * a.RPW + rr;
  constexpr int KC = 16 * KN2;
  // this wave's partial G_(c)[kc][j'] for its block, in LDS (no loop-carried
  // registers): 16*KN2 x 256 floats, this lane owns j' = q*16 + 4g + 0..3
  float* gw = lds + wv * (KC * 256);
  int32_t* wlds = reinterpret_cast<int32_t*>(lds + a.RPW * a.B * (KC * 256)) + wv * 128;
  for (int k = 0; k < KC; ++k) *reinterpret_cast<f4*>(gw + k * 256 + q * 16 + 4 * g) = f4{0.f, 0.f, 0.f, 0.f};

  uint32_t ka4, kb4, kc4;
  lane_offsets<NM1, PREC>(a, rb, cb, q, &ka4, &kb4, &kc4);

  if (w < a.W) {
    const int32_t lo = range_lo(w, a.W, a.nnz);
    const int32_t hi = range_lo(w + 1, a.W, a.nnz);
    int32_t s_first, s_last;
    find_seg2(a.seg_off, a.R, lo, hi - 1, &s_first, &s_last);
    walk_range<NM1, PREC>(a, lo, hi, s_first, s_last, ka4, kb4, kc4, lane, wlds, [&](int32_t s, int32_t row, f4 y) {
      // G_(c) += U^(c)(row, :)^T y_s  (the row of U^(c) is wave-uniform: scalar loads)
      const float* urow = a.Uc + (size_t)__builtin_amdgcn_readfirstlane(row) * a.Kc;
      for (int k = 0; k < a.Kc; ++k) {
        const float u = urow[k];
        f4* dst = reinterpret_cast<f4*>(gw + k * 256 + q * 16 + 4 * g);
        *dst = *dst + u * y;
      }
    });
  }
  __syncthreads();
  // workgroup sum over its ranges (fixed order) for each block, one partial per block
  const int total = a.B * KC * 256;
  float* out = a.gpart + (size_t)wg * total;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int bb = t / (KC * 256), rest = t - bb * (KC * 256);
    float v = 0.f;
    for (int r2 = 0; r2 < a.RPW; ++r2) v += lds[(r2 * a.B + bb) * (KC * 256) + rest];
    out[t] = v;
  }
}

template <int NM1, int KN2, int PREC>
__global__ __launch_bounds__(512) void k_core(SegArgs a) {
  core_body<NM1, KN2, PREC>(a, blockIdx.x);
}

template <int NM1, int KN2, int PREC>
__global__ __launch_bounds__(512) void k_core_b(const SegArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  core_body<NM1, KN2, PREC>(d[r], blockIdx.x - first[r]);
}


// Sums the workgroup partials in order (float64), scatters into G (C order),
// and leaves per-block partial sums of squares for ||G||^2.
// 16 outputs per block of 1024 threads: thread (phase ph, output o) sums the
// partials of groups ph, ph + 64, ... in float64; the 64 phase sums are then
// added by a fixed tree. Output e = ((b * 16 KN2) + kc) * 256 + j' is scattered
// into the C-order core; the block's sum of squares goes to fpart[blk].
constexpr int kRedOut = 16;
constexpr int kRedThreads = 1024;
__device__ inline void red_body(const CoreRedArgs& p, const int blk) {
  __shared__ double sh[kRedThreads];
  const int total = p.B * 16 * p.KN2 * 256;
  const int o = threadIdx.x % kRedOut, ph = threadIdx.x / kRedOut;
  constexpr int NPH = kRedThreads / kRedOut;
  const int e = blk * kRedOut + o;
  double acc = 0.0;
  if (e < total)
    for (int gi = ph; gi < p.groups; gi += NPH) acc += (double)p.gpart[(size_t)gi * total + e];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = NPH / 2; st > 0; st >>= 1) {
    if (ph < st) sh[threadIdx.x] += sh[threadIdx.x + st * kRedOut];
    __syncthreads();
  }
  double sq = 0.0;
  if (threadIdx.x < kRedOut && e < total) {
    const double v = sh[threadIdx.x];
    // e = ((b * 16 KN2) + kc) * 256 + j', j' = c*16 + r within block b
    const int jp = e & 255;
    const int kc = (e >> 8) % (16 * p.KN2);
    const int b = (e >> 8) / (16 * p.KN2);
    const int rb = b / p.CB, cb = b % p.CB;
    const int rg = p.pair ? 2 * (jp & 15) + rb : 16 * rb + (jp & 15);
    const int cg = p.pair ? 2 * (jp >> 4) + cb : 16 * cb + (jp >> 4);
    if (rg < p.krow && cg < p.kcol && kc < p.Kc) {
      int64_t flat = (int64_t)rg * p.kcol + cg;
      int64_t off = (int64_t)kc * p.gstride[p.mode];
      for (int m = p.nm1 - 1; m >= 0; --m) {
        const int64_t k = flat % p.Ko[m];
        flat /= p.Ko[m];
        off += k * p.gstride[p.om[m]];
      }
      const float vf = (float)v;
      p.G[off] = vf;
      sq = (double)vf * (double)vf;
    }
  }
  __syncthreads();
  if (threadIdx.x < kRedOut) sh[threadIdx.x] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < kRedOut; ++i) t += sh[i];
    p.fpart[blk] = t;
  }
}

__global__ __launch_bounds__(1024) void k_core_reduce(CoreRedArgs p) { red_body(p, blockIdx.x); }

__global__ __launch_bounds__(1024) void k_core_reduce_b(const CoreRedArgs* d, const int32_t* first, int count) {
  const int r = batch_item(first, count, blockIdx.x);
  red_body(d[r], blockIdx.x - first[r]);
}

__device__ inline void sum_body(const SumArgs& a) {
  __shared__ double sh[256];
  const double* part = a.part;
  double* out = a.out;
  double acc = 0.0;
  for (int i = threadIdx.x; i < a.n; i += blockDim.x) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ void k_sum_f(SumArgs a) { sum_body(a); }

__global__ void k_sum_f_b(const SumArgs* d, const int32_t* first, int count) {
  sum_body(d[batch_item(first, count, blockIdx.x)]);
}

// ---------------------------------------------------------------------------
// Generic kernels: any order N <= 5 and any ranks <= 32, for the shapes the
// segment passes do not take (N = 5, or more than 8 16x16 tiles per y_i). They
// read the same block records and slice tables, in float32 with float32
// accumulation over a fixed order, and are sized for small tensors (one
// workgroup walks one slice).
// ---------------------------------------------------------------------------
struct GenArgs {
  const int32_t* rec;
  const int32_t* seg_off;
  const int32_t* seg_row;
  int32_t R, N, nm1;
  const float* U[kMaxOrder - 1];  // other modes ascending (label order)
  int32_t Ko[kMaxOrder - 1];
  int64_t gstride_o[kMaxOrder - 1];  // C-order strides of G along the other modes
  int64_t gstride_n;
  int32_t Kn;
  int64_t P;                          // prod of the other ranks
  const float* G;                     // TTMcTC: core
  float* A;                           // TTMcTC: output rows by label (or out_map)
  const int32_t* out_map;
  const float* Uc;                    // core: factor of the pass mode
  float* Gout;                        // core: C-order core
};

// Entry j' of a nonzero's Kronecker row (other modes ascending, last fastest):
// x times the product of its factor-row entries.
__device__ inline float gen_kron(const GenArgs& a, const int32_t* r, int t, int64_t jp) {
  const int N = a.N;
  float w = __int_as_float(r[4 * (N - 1) + t]);
  int64_t rem = jp;
  for (int c = a.nm1 - 1; c >= 0; --c) {
    const int k = (int)(rem % a.Ko[c]);
    rem /= a.Ko[c];
    w *= a.U[c][(int64_t)(r[4 * c + t] >> 1) + k];  // stored: 2 label * K_m
  }
  return w;
}

// y_s(j') for slice s, in the order of the slice's nonzeros
__device__ inline float gen_slice_y(const GenArgs& a, int32_t s, int64_t jp) {
  float y = 0.f;
  for (int32_t e = a.seg_off[s]; e < a.seg_off[s + 1]; ++e) {
    const int32_t* r = a.rec + (int64_t)(e >> 4) * 16 * a.N + (e & 3) * 4 * a.N;
    y += gen_kron(a, r, (e & 15) >> 2, jp);
  }
  return y;
}

// TTMcTC: one workgroup per slice; thread t takes j' = t, t + 256, ... and
// keeps partial sums of A(s, kn) = sum_j' y_s(j') G_(n)(kn, j'), reduced over
// the threads in a fixed tree.
__global__ __launch_bounds__(256) void k_ttm_generic(GenArgs a) {
  __shared__ float red[256];
  const int32_t s = blockIdx.x;
  float acc[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) acc[k] = 0.f;
  for (int64_t jp = threadIdx.x; jp < a.P; jp += 256) {
    const float y = gen_slice_y(a, s, jp);
    int64_t goff = 0, rem = jp;
    for (int c = a.nm1 - 1; c >= 0; --c) {
      goff += (rem % a.Ko[c]) * a.gstride_o[c];
      rem /= a.Ko[c];
    }
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if (k < a.Kn) acc[k] += y * a.G[goff + k * a.gstride_n];
  }
  const int32_t row = a.out_map ? a.out_map[a.seg_row[s]] : a.seg_row[s];
  for (int k = 0; k < a.Kn; ++k) {
    red[threadIdx.x] = acc[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.A[(int64_t)row * a.Kn + k] = red[0];
    __syncthreads();
  }
}

// Core: one thread per entry j' of G_(c); it walks every slice s and adds
// U^(c)(s, kc) y_s(j') for all kc (slices and nonzeros in stream order), so
// every core entry has one writer and a fixed order.
__global__ __launch_bounds__(256) void k_core_generic(GenArgs a) {
  const int64_t jp = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (jp >= a.P) return;
  float acc[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) acc[k] = 0.f;
  for (int32_t s = 0; s < a.R; ++s) {
    const float y = gen_slice_y(a, s, jp);
    const float* u = a.Uc + (int64_t)a.seg_row[s] * a.Kn;
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if (k < a.Kn) acc[k] += u[k] * y;
  }
  int64_t goff = 0, rem = jp;
  for (int c = a.nm1 - 1; c >= 0; --c) {
    goff += (rem % a.Ko[c]) * a.gstride_o[c];
    rem /= a.Ko[c];
  }
  for (int k = 0; k < a.Kn; ++k) a.Gout[goff + k * a.gstride_n] = acc[k];
}

// Split-Kronecker pass for modes beyond the segment passes (order 5, or more
// than 8 16x16 tiles of y_i): y_i as a matrix whose rows are the Kronecker
// product of the first other modes and whose columns that of the rest
// (yi_row_modes), cut into 16x16 tiles. One workgroup per nonempty slice;
// its 8 waves take the tiles in turn, and a tile is accumulated over the
// slice's nonzeros on the matrix cores, 4 nonzeros per v_mfma_f32_16x16x4f32:
// lane (g, q) supplies x_e times the row-mode factor entries of row 16 rb + q
// (A operand, nonzero 4s + g) and the column-mode factor entries of column
// 16 cb + q (B operand), so each Kronecker half is formed once per lane and
// nonzero instead of the whole row. BF16 form: 16 nonzeros per
// v_mfma_f32_16x16x16bf16_1k, lane group g forming nonzeros 4g .. 4g + 3 of
// the step, both operands rounded to bfloat16 (nearest even) from their
// float32 products, float32 accumulation. The finished tile is stored (in
// float32) as tile b of the slice's row of Y_(n) (entry c*16 + r, the segment
// passes' layout), from which A^(n) and the core follow as for stored slice
// rows.
struct GenRowsArgs {
  const int32_t* rec;
  const int32_t* seg_off;
  const int32_t* seg_row;
  int32_t R, N, nm1, nr;            // other modes, the first nr of which index the rows of y_i
  const float* U[kMaxOrder - 1];    // other modes ascending (label order)
  int32_t Ko[kMaxOrder - 1];
  int32_t krow, kcol, CB, B;
  float* ybuf;                      // [label][B * 256]
};
constexpr int kGenWaves = 8;
template <bool BF16>
__global__ __launch_bounds__(64 * kGenWaves) void k_gen_rows(GenRowsArgs a) {
  const int32_t s = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, q = lane & 15;
  const int32_t e_lo = a.seg_off[s], e_hi = a.seg_off[s + 1];
  float* yr = a.ybuf + (size_t)a.seg_row[s] * a.B * 256;
  const int N = a.N;
  for (int b = wv; b < a.B; b += kGenWaves) {
    const int rb = b / a.CB, cb = b - rb * a.CB;
    const int r = 16 * rb + q, c = 16 * cb + q;
    const bool rok = r < a.krow, cok = c < a.kcol;
    // this lane's entry of each other mode (padded rows / columns read entry 0)
    int ko[kMaxOrder - 1] = {0, 0, 0, 0};
    {
      int rem = rok ? r : 0;
      for (int m = a.nr - 1; m >= 0; --m) {
        ko[m] = rem % a.Ko[m];
        rem /= a.Ko[m];
      }
      rem = cok ? c : 0;
      for (int m = a.nm1 - 1; m >= a.nr; --m) {
        ko[m] = rem % a.Ko[m];
        rem /= a.Ko[m];
      }
    }
    // the two Kronecker halves of nonzero e for this lane (0 past the slice)
    auto halves = [&](int32_t e, float& av, float& bv) {
      av = 0.f;
      bv = 0.f;
      if (e < e_hi) {
        // record of nonzero e = 16 blk + 4 t + g': the row offsets 2 label * K_m and the value
        const int32_t* rp = a.rec + (size_t)(e >> 4) * 16 * N + (e & 3) * 4 * N;
        const int t = (e & 15) >> 2;
        float wa = __int_as_float(rp[4 * (N - 1) + t]);
        float wb = 1.f;
#pragma unroll
        for (int m = 0; m < kMaxOrder - 1; ++m) {
          if (m >= a.nm1) break;
          const float u = a.U[m][(int64_t)(rp[4 * m + t] >> 1) + ko[m]];  // stored: 2 label * K_m
          if (m < a.nr) wa *= u;
          else wb *= u;
        }
        av = rok ? wa : 0.f;
        bv = cok ? wb : 0.f;
      }
    };
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (BF16) {
#pragma unroll 2
      for (int32_t e0 = e_lo; e0 < e_hi; e0 += 16) {
        float av[4], bv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) halves(e0 + 4 * g + t, av[t], bv[t]);
        const b4 ab = {(__bf16)av[0], (__bf16)av[1], (__bf16)av[2], (__bf16)av[3]};
        const b4 bb = {(__bf16)bv[0], (__bf16)bv[1], (__bf16)bv[2], (__bf16)bv[3]};
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, ab), __builtin_bit_cast(s4, bb), acc,
                                                        0, 0, 0);
      }
    } else {
#pragma unroll 4
      for (int32_t e0 = e_lo; e0 < e_hi; e0 += 4) {
        float av, bv;
        halves(e0 + g, av, bv);
        acc = mfma4(av, bv, acc);
      }
    }
    // lane (g, q) holds rows 4g + v of column q of the tile: entry q*16 + 4g + v
    *reinterpret_cast<f4*>(yr + (size_t)b * 256 + q * 16 + 4 * g) = acc;
  }
}

// ||G||^2 in float64 by one workgroup (fixed order)
__global__ __launch_bounds__(256) void k_sumsq(const float* G, int64_t n, double* out) {
  __shared__ double sh[256];
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) t += (double)G[i] * (double)G[i];
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

struct PassGeom {
  int nm1;
  int om[kMaxOrder];
  int Ko[kMaxOrder];
  int krow, kcol, RB, CB, B;
};

PassGeom geom(const hoqri_plan* p, int mode) {
  PassGeom g{};
  g.nm1 = other_modes(p->N, mode, g.om);
  g.krow = 1;
  g.kcol = 1;
  for (int c = 0; c < g.nm1; ++c) g.Ko[c] = p->K[g.om[c]];
  const int nr = yi_row_modes(g.nm1);
  for (int c = 0; c < g.nm1; ++c) (c < nr ? g.krow : g.kcol) *= g.Ko[c];
  g.RB = (g.krow + 15) / 16;
  g.CB = (g.kcol + 15) / 16;
  g.B = g.RB * g.CB;
  return g;
}

bool fill_common(SegArgs& a, const hoqri_plan* p, int mode, const PassGeom& g, const Operands& op) {
  const ModeData& md = p->md[mode];
  const int es = op.prec == OP_FP32 ? 4 : 2;
  for (int c = 0; c < 3; ++c) {
    const int m = c < g.nm1 ? g.om[c] : g.om[0];
    a.U[c] = op.prec == OP_FP32 ? (const void*)op.U32[m] : (const void*)op.U16[m];
    a.Ubytes[c] = (uint32_t)(p->dims[m] * p->K[m] * es);
  }
  a.ascale = 1.f;
  a.yscale = 1.f;
  if (op.prec == OP_FP16 && !fp16_scales(p, g.nm1, &a.ascale, &a.yscale)) return false;
  a.rec = md.rec;
  a.fault = p->sc.status + 3;
  a.seg_off = md.seg_off;
  a.seg_row = md.seg_row;
  a.R = (int32_t)md.R;
  a.nnz = (int32_t)p->nnz;
  a.nnz_pad = (int32_t)((p->nnz + 15) / 16 * 16);
  a.B = g.B;
  a.RB = g.RB;
  a.CB = g.CB;
  a.K1 = g.nm1 >= 2 ? g.Ko[1] : 1;
  a.K0 = g.Ko[0];
  a.K2 = g.nm1 >= 3 ? g.Ko[2] : 1;
  return true;
}

// Key offset of the 2 x 2-block BF16 TTMcTC pass (core keys add 1000), and of
// the 4-way 16-bit pass with c-tiles (plus 1000 x the tiles per wave).
constexpr int kWideKey = 2000;
constexpr int kPairKey = 4000;  // the 2 x 2-block pass in paired order (added to kWideKey)
constexpr int kWide4Key = 10000;

// Kernel instances: one single-plan and one batched launch per
// (order, rank blocks, precision).
struct SegKernels {
  const void* ttm;
  const void* ttm_b;
  const void* core;
  const void* core_b;
  const void* rows;
  const void* rows_b;
};

template <int NM1, int KN2, int PREC>
SegKernels seg_kernels_t() {
  const void* ttm;
  if constexpr (ttm_hold4<NM1, KN2, PREC>()) ttm = (const void*)k_ttm_w4<NM1, KN2, PREC>;
  else ttm = (const void*)k_ttm<NM1, KN2, PREC>;
  return SegKernels{ttm,                                      (const void*)k_ttm_b<NM1, KN2, PREC>,
                    (const void*)k_core<NM1, KN2, PREC>,      (const void*)k_core_b<NM1, KN2, PREC>,
                    (const void*)k_core_rows<NM1, KN2, PREC>, (const void*)k_core_rows_b<NM1, KN2, PREC>};
}

template <int PREC>
bool seg_kernels_p(int nm1, int kn2, SegKernels* k) {
  switch (nm1 * 10 + kn2) {
    case 11: *k = seg_kernels_t<1, 1, PREC>(); return true;
    case 12: *k = seg_kernels_t<1, 2, PREC>(); return true;
    case 21: *k = seg_kernels_t<2, 1, PREC>(); return true;
    case 22: *k = seg_kernels_t<2, 2, PREC>(); return true;
    case 31: *k = seg_kernels_t<3, 1, PREC>(); return true;
    case 32: *k = seg_kernels_t<3, 2, PREC>(); return true;
    default: return false;
  }
}

template <int PREC, int NC>
bool seg_kernels_4c_n(int kn2, SegKernels* k) {
  k->rows = (const void*)k_core4c<PREC, NC>;
  k->rows_b = (const void*)k_core4c_b<PREC, NC>;
  if (kn2 == 1) {
    k->ttm = (const void*)k_ttm4c<PREC, NC, 1>;
    k->ttm_b = (const void*)k_ttm4c_b<PREC, NC, 1>;
  } else {
    k->ttm = (const void*)k_ttm4c<PREC, NC, 2>;
    k->ttm_b = (const void*)k_ttm4c_b<PREC, NC, 2>;
  }
  return true;
}

template <int PREC>
bool seg_kernels_4c(int nc, int kn2, SegKernels* k) {
  if (nc == 4) return seg_kernels_4c_n<PREC, 4>(kn2, k);
  if (nc == 5) return seg_kernels_4c_n<PREC, 5>(kn2, k);
  if (nc == 6) return seg_kernels_4c_n<PREC, 6>(kn2, k);
  return false;
}

bool seg_kernels(int key, SegKernels* k) {
  int nc4 = 0;  // c-tiles per wave of the 4-way c-tile pass
  if (key >= kWide4Key) {
    nc4 = (key - kWide4Key) / 1000;
    key %= 1000;
  }
  const bool pair = key >= kWideKey + kPairKey;
  if (pair) key -= kPairKey;
  const bool wide = key >= kWideKey;
  if (wide) key -= kWideKey;
  key %= 1000;
  const int nm1 = key / 100, kn2 = (key / 10) % 10, prec = key % 10;
  bool ok = false;
  if (prec == P_FP32) ok = seg_kernels_p<P_FP32>(nm1, kn2, k);
  else if (prec == P_BF16) ok = seg_kernels_p<P_BF16>(nm1, kn2, k);
  else if (prec == P_FP16) ok = seg_kernels_p<P_FP16>(nm1, kn2, k);
  if (ok && nc4 > 0) {
    if (nm1 != 3 || kn2 > 2) return false;
    if (prec == P_BF16) return seg_kernels_4c<P_BF16>(nc4, kn2, k);
    if (prec == P_FP16) return seg_kernels_4c<P_FP16>(nc4, kn2, k);
    if (prec == P_FP32) return seg_kernels_4c<P_FP32>(nc4, kn2, k);
    return false;
  }
  if (!ok || !wide) return ok;
  if (nm1 != 2 || prec != P_BF16) return false;
  if (pair) {
    k->ttm = kn2 == 1 ? (const void*)k_ttm22<1, true> : (const void*)k_ttm22<2, true>;
    k->ttm_b = kn2 == 1 ? (const void*)k_ttm22_b<1, true> : (const void*)k_ttm22_b<2, true>;
  } else {
    k->ttm = kn2 == 1 ? (const void*)k_ttm22<1, false> : (const void*)k_ttm22<2, false>;
    k->ttm_b = kn2 == 1 ? (const void*)k_ttm22_b<1, false> : (const void*)k_ttm22_b<2, false>;
  }
  return true;
}

// The 2 x 2-block pass takes the BF16 form of 3-way tensors whose two other
// ranks both lie in 17..32.
bool ttm_wide(const PassGeom& g, int prec) { return prec == OP_BF16 && g.nm1 == 2 && g.RB == 2 && g.CB == 2; }

// The 4-way c-tile pass takes every operand form when all three other ranks
// are at most 16 (every y_i then fits the staging of one range).
bool ttm_wide4(const PassGeom& g, int prec) {
  (void)prec;
  return g.nm1 == 3 && g.Ko[0] <= 16 && g.Ko[1] <= 16 && g.Ko[2] <= 16;
}

// Waves (ranges) per workgroup of that pass: as many as the LDS of one
// workgroup holds next to the core operand, at most kMaxRpw22.
int rpw22(int KN2) {
  static int lds_max = 0;
  if (lds_max == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 65536;
    lds_max = v;
  }
  int r = (lds_max - KN2 * 32768 - ttm22_pool_bytes()) / ttm22_wave_bytes();
  return r > kMaxRpw22 ? kMaxRpw22 : (r < 1 ? 1 : r);
}

hipError_t set_shmem(const void* k, size_t shmem) {
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
}

// Rounds to the 16-bit copy: bfloat16 (nearest even), or float16 of u * 2^15
// (nearest even). |u| <= 1 for a factor with orthonormal columns, so the
// float16 copy stays below 2^15 < 65504; an entry of magnitude 1.5 or more
// (or not finite) would leave that range or come from factors that are not
// orthonormal: it sets *range_flag (when given), which the callers read
// before any pass uses the copy.
__global__ void k_cast16(const float* __restrict__ U, int64_t n, uint16_t* __restrict__ Uh, int prec,
                         int32_t* range_flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float u = U[i];
    uint16_t b;
    if (prec == OP_BF16) {
      b = __builtin_bit_cast(uint16_t, (__bf16)u);
    } else {
      bad |= !(__builtin_fabsf(u) < 1.5f);
      b = __builtin_bit_cast(uint16_t, (_Float16)(u * 32768.f));
    }
    Uh[i] = b;
  }
  if (bad && range_flag) *range_flag = 1;
}

void g_strides(const hoqri_plan* p, int64_t* st) {
  int64_t s = 1;
  for (int m = p->N - 1; m >= 0; --m) {
    st[m] = s;
    s *= p->K[m];
  }
}

}  // namespace

// The 2 x 2-block pass gathers entry pairs (one dword) when both other ranks
// are even (every factor row then starts on a 4-byte boundary).
bool ttm_pair(const PassGeom& g) { return g.Ko[0] % 2 == 0 && g.Ko[1] % 2 == 0; }

int ttm_max_rpw(const hoqri_plan* p, int mode, int prec) {
  if (!segpass_supported(p, mode)) return 1;
  const PassGeom g = geom(p, mode);
  const int KN2 = (p->K[mode] + 15) / 16;
  if (ttm_wide(g, prec)) return rpw22(KN2);
  if (ttm_wide4(g, prec)) return 1;  // the c-tile pass takes one range per workgroup
  return g.B >= 8 ? 1 : 8 / g.B;     // 512 threads per workgroup
}

bool ttm_rows_bf16(const hoqri_plan* p, int mode, int prec) {
  return segpass_supported(p, mode) && ttm_wide(geom(p, mode), prec);
}

bool segpass_supported(const hoqri_plan* p, int mode) {
  PassGeom g = geom(p, mode);
  return g.nm1 <= 3 && g.B <= 8 && p->K[mode] <= 32;
}

bool fp16_scales(const hoqri_plan* p, int nm1, float* ascale, float* yscale) {
  // A operand of the FP16 form: x * ascale * (nm1 - 1 float16 copies, each
  // below 2^15 in magnitude) must stay below 60000; the product then carries
  // the factor ascale * 2^(15 nm1), removed exactly by yscale.
  const double mx = p->maxabs_x > 0 ? p->maxabs_x : 1.0;
  const int e = (int)std::floor(std::log2(60000.0 / mx) - 15.0 * (nm1 - 1));
  const int ec = e > 60 ? 60 : e;
  const int ey = -(15 * nm1 + ec);
  if (ec < -126 || ey < -126 || ey > 127) return false;
  *ascale = std::ldexp(1.0f, ec);
  *yscale = std::ldexp(1.0f, ey);
  return true;
}

hoqri_status launch_cast16(const float* U, int64_t rows, int32_t K, uint16_t* Uh, int prec, hipStream_t s,
                           int32_t* range_flag) {
  const int64_t n = rows * K;
  if (n <= 0) return HOQRI_OK;
  int64_t grid = (n + 255) / 256;
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(k_cast16, dim3((unsigned)grid), dim3(256), 0, s, U, n, Uh, prec, range_flag);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

hoqri_status prepare_ttm(hoqri_plan* p, int mode, const Operands& op, const float* G, float* A,
                         const int32_t* out_map, TtmJob* job, bool rows) {
  if (!segpass_supported(p, mode)) return HOQRI_ERR_UNSUPPORTED;
  if (rows && (!p->yfuse || out_map)) return HOQRI_ERR_UNSUPPORTED;
  const PassGeom g = geom(p, mode);
  const int KN2 = (p->K[mode] + 15) / 16;
  const ModeData& md = p->md[mode];
  *job = TtmJob{};
  const bool wide = ttm_wide(g, op.prec);
  const bool nc4 = ttm_wide4(g, op.prec);
  int nw4 = 1;  // waves per range of the c-tile pass
  const int tiles4 = nc4 ? tiles4c(g.Ko[2], &nw4) : 0;
  const bool pair = wide && ttm_pair(g);
  job->key = seg_key(g.nm1, KN2, op.prec) + (wide ? kWideKey : 0) + (pair ? kPairKey : 0) +
             (nc4 ? kWide4Key + 1000 * tiles4 : 0);
  // stage-two operand
  PrepArgs& pa = job->prep;
  pa.wide16 = wide ? 2 : (nc4 ? (op.prec == OP_FP32 ? 3 : 1) : 0);
  pa.pair = pair ? 1 : 0;
  pa.G = G;
  pa.gtop = p->sc.gtop;
  pa.B = g.B;
  pa.CB = g.CB;
  pa.KN2 = KN2;
  pa.krow = g.krow;
  pa.kcol = g.kcol;
  pa.Kn = p->K[mode];
  pa.mode = mode;
  pa.N = p->N;
  pa.nm1 = g.nm1;
  for (int c = 0; c < kMaxOrder - 1; ++c) {
    pa.om[c] = c < g.nm1 ? g.om[c] : 0;
    pa.Ko[c] = c < g.nm1 ? g.Ko[c] : 1;
  }
  g_strides(p, pa.gstride);
  const int64_t total = (int64_t)g.B * KN2 * 4096;
  pa.nblk = (int)((total + 255) / 256);
  job->prep_blocks = pa.nblk;
  // main pass
  SegArgs& a = job->seg;
  if (!fill_common(a, p, mode, g, op)) return HOQRI_ERR_UNSUPPORTED;
  int64_t W = md.ranges;
  if (W > p->nnz) W = p->nnz;
  a.W = (int32_t)W;
  a.RPW = wide ? rpw22(KN2) : nc4 ? 1 : (g.B == 1 ? 4 : 1);
  if (md.rpw > 0) a.RPW = std::min(md.rpw, ttm_max_rpw(p, mode, op.prec));
  a.gtop = p->sc.gtop;
  a.A = A;
  a.Kn = p->K[mode];
  a.carry = p->sc.carry;
  a.meta = p->sc.meta;
  a.out_map = out_map;
  a.yrow = rows ? p->sc.ybuf : nullptr;
  a.ycarry = rows ? p->sc.ycarry : nullptr;
  job->threads = wide ? 64 * a.RPW : nc4 ? 64 * nw4 : 64 * g.B * a.RPW;
  job->shmem = wide  ? (size_t)KN2 * 32768 + ttm22_pool_bytes() + (size_t)a.RPW * ttm22_wave_bytes()
               : nc4 ? (size_t)ttm4c_bytes(g.B, nw4, KN2)
                     : (size_t)ttm_lds_floats(a, KN2) * 4;
  job->seg_blocks = (a.W + a.RPW - 1) / a.RPW;
  // split slices
  FixArgs& f = job->fix;
  f.meta = p->sc.meta;
  f.carry = p->sc.carry;
  f.seg_row = md.seg_row;
  f.seg_off = md.seg_off;
  f.W = a.W;
  f.nnz = a.nnz;
  f.Kn = a.Kn;
  f.out_map = out_map;
  f.A = A;
  job->fix_blocks = a.W;
  SegKernels k;
  if (!seg_kernels(job->key, &k)) return HOQRI_ERR_UNSUPPORTED;
  return HOQRI_OK;
}

hoqri_status prepare_core(hoqri_plan* p, const Operands& op, float* G, double* f_out, CoreJob* job) {
  const int mode = p->core_mode;
  if (!segpass_supported(p, mode)) return HOQRI_ERR_UNSUPPORTED;
  const PassGeom g = geom(p, mode);
  const int KN2 = (p->K[mode] + 15) / 16;
  *job = CoreJob{};
  job->key = seg_key(g.nm1, KN2, op.prec);
  SegArgs& a = job->seg;
  if (!fill_common(a, p, mode, g, op)) return HOQRI_ERR_UNSUPPORTED;
  if (p->core_rows) {
    int64_t W = p->core_w;
    if (W > p->nnz) W = p->nnz;
    a.W = (int32_t)W;
    if (ttm_wide4(g, op.prec)) {
      // 16-bit forms of 4-way tensors: the c-tile walk writes the rows
      int nw4 = 1;
      const int tiles4 = tiles4c(g.Ko[2], &nw4);
      job->key += kWide4Key + 1000 * tiles4;
      a.RPW = 1;
      a.yrow = p->sc.ybuf;
      a.ycarry = p->sc.ycarry;
      a.meta = p->sc.ymeta;
      job->threads = 64 * nw4;
      job->shmem = (size_t)ttm4c_bytes(g.B, nw4, 1);
    } else {
      job->key += 1000;
      a.RPW = g.B == 1 ? 4 : 1;
      a.A = p->sc.ybuf;
      a.carry = p->sc.ycarry;
      a.meta = p->sc.ymeta;
      job->threads = 64 * g.B * a.RPW;
      job->shmem = (size_t)g.B * a.RPW * 128 * 4;
    }
    job->seg_blocks = (a.W + a.RPW - 1) / a.RPW;
    CoreGemmArgs& m = job->gemm;
    m.ybuf = p->sc.ybuf;
    m.ycarry = p->sc.ycarry;
    m.ymeta = p->sc.ymeta;
    m.seg_row = p->md[mode].seg_row;
    m.Uc = op.U32[mode];
    m.Kc = p->K[mode];
    m.KC = 16 * KN2;
    m.R = (int32_t)p->md[mode].R;
    m.W = a.W;
    m.B = g.B;
    m.gpart = p->sc.gpart;
    // a multiple of 8 (blocks go to the XCDs by chunk; empty chunks add zeros)
    const int64_t chunks = (((int64_t)m.R + 2 * (int64_t)m.W + kCoreChunk - 1) / kCoreChunk + 7) / 8 * 8;
    m.nchunk = (int32_t)chunks;
    job->gemm_blocks = (int)(chunks * g.B);
    CoreRedArgs& r = job->red;
    r.gpart = p->sc.gpart;
    r.groups = (int32_t)chunks;
    r.B = g.B;
    r.CB = g.CB;
    r.KN2 = KN2;
    r.krow = g.krow;
    r.kcol = g.kcol;
    r.Kc = p->K[mode];
    r.mode = mode;
    r.nm1 = g.nm1;
    for (int c = 0; c < kMaxOrder - 1; ++c) {
      r.om[c] = c < g.nm1 ? g.om[c] : 0;
      r.Ko[c] = c < g.nm1 ? g.Ko[c] : 1;
    }
    g_strides(p, r.gstride);
    r.G = G;
    r.fpart = p->sc.fpart;
    const int total = g.B * 16 * KN2 * 256;
    job->red_blocks = (total + kRedOut - 1) / kRedOut;
    job->sum.part = p->sc.fpart;
    job->sum.n = job->red_blocks;
    job->sum.out = f_out ? f_out : p->sc.f_dev;
    SegKernels k;
    if (!seg_kernels(job->key, &k)) return HOQRI_ERR_UNSUPPORTED;
    return HOQRI_OK;
  }
  // each wave keeps its partial (16*KN2 x 256 floats) in LDS: at most 160 KB per workgroup
  const int per_wave = 16 * KN2 * 256 * 4 + 128 * 4;
  int rpw = (160 * 1024) / (per_wave * g.B);
  if (rpw > 8) rpw = 8;
  if (rpw < 1) return HOQRI_ERR_UNSUPPORTED;
  a.RPW = rpw;
  int64_t groups = p->core_groups;
  int64_t W = groups * a.RPW;
  if (W > p->nnz) {
    W = p->nnz;
    groups = (W + a.RPW - 1) / a.RPW;
  }
  a.W = (int32_t)W;
  a.Uc = op.U32[mode];
  a.Kc = p->K[mode];
  a.gpart = p->sc.gpart;
  job->threads = 64 * g.B * a.RPW;
  job->shmem = (size_t)a.RPW * g.B * per_wave;
  job->seg_blocks = (int)groups;
  CoreRedArgs& r = job->red;
  r.gpart = p->sc.gpart;
  r.groups = (int32_t)groups;
  r.B = g.B;
  r.CB = g.CB;
  r.KN2 = KN2;
  r.krow = g.krow;
  r.kcol = g.kcol;
  r.Kc = p->K[mode];
  r.mode = mode;
  r.nm1 = g.nm1;
  for (int c = 0; c < kMaxOrder - 1; ++c) {
    r.om[c] = c < g.nm1 ? g.om[c] : 0;
    r.Ko[c] = c < g.nm1 ? g.Ko[c] : 1;
  }
  g_strides(p, r.gstride);
  r.G = G;
  r.fpart = p->sc.fpart;
  const int total = g.B * 16 * KN2 * 256;
  job->red_blocks = (total + kRedOut - 1) / kRedOut;
  job->sum.part = p->sc.fpart;
  job->sum.n = job->red_blocks;
  job->sum.out = f_out ? f_out : p->sc.f_dev;
  SegKernels k;
  if (!seg_kernels(job->key, &k)) return HOQRI_ERR_UNSUPPORTED;
  return HOQRI_OK;
}

namespace {
GenArgs gen_args(const hoqri_plan* p, int mode) {
  GenArgs a{};
  const ModeData& md = p->md[mode];
  a.rec = md.rec;
  a.seg_off = md.seg_off;
  a.seg_row = md.seg_row;
  a.R = (int32_t)md.R;
  a.N = p->N;
  int om[kMaxOrder];
  a.nm1 = other_modes(p->N, mode, om);
  int64_t st[kMaxOrder];
  g_strides(p, st);
  a.P = 1;
  for (int c = 0; c < a.nm1; ++c) {
    a.U[c] = p->sc.Up[om[c]];
    a.Ko[c] = p->K[om[c]];
    a.gstride_o[c] = st[om[c]];
    a.P *= p->K[om[c]];
  }
  a.gstride_n = st[mode];
  a.Kn = p->K[mode];
  return a;
}
}  // namespace

bool generic_supported(const hoqri_plan* p) {
  for (int n = 0; n < p->N; ++n)
    if (p->K[n] > 32) return false;
  return true;
}

// The split-Kronecker pass of mode `mode` (float32 or bfloat16 operands, from
// the float32 factors): the rows of Y_(mode) for every nonempty slice into the
// plan's slice-row buffer.
hoqri_status launch_gen_rows(hoqri_plan* p, int mode, int prec, hipStream_t s) {
  const PassGeom g = geom(p, mode);
  const ModeData& md = p->md[mode];
  GenRowsArgs a{};
  a.rec = md.rec;
  a.seg_off = md.seg_off;
  a.seg_row = md.seg_row;
  a.R = (int32_t)md.R;
  a.N = p->N;
  a.nm1 = g.nm1;
  a.nr = yi_row_modes(g.nm1);
  for (int c = 0; c < g.nm1; ++c) {
    a.U[c] = p->sc.Up[g.om[c]];
    a.Ko[c] = g.Ko[c];
  }
  a.krow = g.krow;
  a.kcol = g.kcol;
  a.CB = g.CB;
  a.B = g.B;
  a.ybuf = p->sc.ybuf;
  if (a.R > 0) {
    if (prec == OP_BF16) hipLaunchKernelGGL(k_gen_rows<true>, dim3((unsigned)a.R), dim3(64 * kGenWaves), 0, s, a);
    else hipLaunchKernelGGL(k_gen_rows<false>, dim3((unsigned)a.R), dim3(64 * kGenWaves), 0, s, a);
  }
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

// Stage-two operand (float32 order) of a mode that takes the split-Kronecker pass.
PrepArgs gen_prep(const hoqri_plan* p, int mode, const float* G) {
  const PassGeom g = geom(p, mode);
  PrepArgs pa{};
  pa.wide16 = 0;
  pa.pair = 0;
  pa.G = G;
  pa.gtop = p->sc.gtop;
  pa.B = g.B;
  pa.CB = g.CB;
  pa.KN2 = (p->K[mode] + 15) / 16;
  pa.krow = g.krow;
  pa.kcol = g.kcol;
  pa.Kn = p->K[mode];
  pa.mode = mode;
  pa.N = p->N;
  pa.nm1 = g.nm1;
  for (int c = 0; c < kMaxOrder - 1; ++c) {
    pa.om[c] = c < g.nm1 ? g.om[c] : 0;
    pa.Ko[c] = c < g.nm1 ? g.Ko[c] : 1;
  }
  g_strides(p, pa.gstride);
  const int64_t total = (int64_t)g.B * pa.KN2 * 4096;
  pa.nblk = (int)((total + 255) / 256);
  return pa;
}

// A^(mode) = Y_(mode) G_(mode)^T from the stored rows of a mode with no split
// slices (whole slices per workgroup), rows by label or through out_map.
hoqri_status gen_rows_a(hoqri_plan* p, int mode, const float* G, float* A, const int32_t* out_map, hipStream_t s) {
  const PrepArgs pa = gen_prep(p, mode, G);
  RowsAArgs r{};
  r.ybuf = p->sc.ybuf;
  r.ycarry = p->sc.ycarry;
  r.ymeta = p->sc.meta;
  r.gtop = p->sc.gtop;
  r.R = (int32_t)p->md[mode].R;
  r.W = 0;
  r.B = pa.B;
  r.KN2 = pa.KN2;
  r.Kn = p->K[mode];
  r.yb16 = 0;
  r.out_map = out_map;
  r.groups = ((int64_t)r.R + 15) / 16;
  r.A = A;
  r.carry = p->sc.carry;
  hipLaunchKernelGGL(k_prep_gtop, dim3(pa.nblk), dim3(256), 0, s, pa);
  if (r.groups > 0) hipLaunchKernelGGL(k_rows_a, dim3((unsigned)((r.groups + 3) / 4)), dim3(256), 0, s, r);
  const ModeData& md = p->md[mode];
  if (md.E > 0) {
    int64_t tot = md.E * p->K[mode];
    int grid = (int)((tot + 255) / 256 < 65536 ? (tot + 255) / 256 : 65536);
    hipLaunchKernelGGL(k_zero_rows, dim3(grid), dim3(256), 0, s, out_map ? md.empty_row : (const int32_t*)nullptr,
                       md.R, md.E, p->K[mode], A);
  }
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

hoqri_status launch_ttmctc(hoqri_plan* p, int mode, const Operands& op, const float* G, float* A,
                           const int32_t* out_map, hipStream_t s, bool rows) {
  if (!segpass_supported(p, mode)) {
    if (!generic_supported(p)) return HOQRI_ERR_UNSUPPORTED;
    if (p->yfuse && (op.prec == OP_FP32 || op.prec == OP_BF16)) {
      // split-Kronecker pass: the slice rows of Y_(mode), then A from them
      TimerScope ts(p, HOQRI_KERNEL_TTMCTC, s);
      HOQRI_TRY(launch_gen_rows(p, mode, op.prec, s));
      return gen_rows_a(p, mode, G, A, out_map, s);
    }
    if (op.prec != OP_FP32) return HOQRI_ERR_UNSUPPORTED;
    // generic scalar kernel (slice rows too large to store): no stored rows
    if (rows) return HOQRI_ERR_UNSUPPORTED;
    GenArgs a = gen_args(p, mode);
    a.G = G;
    a.A = A;
    a.out_map = out_map;
    TimerScope ts(p, HOQRI_KERNEL_TTMCTC, s);
    if (a.R > 0) hipLaunchKernelGGL(k_ttm_generic, dim3((unsigned)a.R), dim3(256), 0, s, a);
    const ModeData& md = p->md[mode];
    if (md.E > 0) {
      int64_t tot = md.E * p->K[mode];
      int grid = (int)((tot + 255) / 256 < 65536 ? (tot + 255) / 256 : 65536);
      hipLaunchKernelGGL(k_zero_rows, dim3(grid), dim3(256), 0, s, out_map ? md.empty_row : (const int32_t*)nullptr,
                         md.R, md.E, p->K[mode], A);
    }
    HOQRI_HIP_TRY(hipGetLastError());
    return HOQRI_OK;
  }
  TtmJob job;
  HOQRI_TRY(prepare_ttm(p, mode, op, G, A, out_map, &job, rows));
  SegKernels k;
  seg_kernels(job.key, &k);
  {
    TimerScope tp(p, HOQRI_KERNEL_FIXUP, s);
    hipLaunchKernelGGL(k_prep_gtop, dim3(job.prep_blocks), dim3(256), 0, s, job.prep);
    HOQRI_HIP_TRY(hipGetLastError());
  }
  {
    TimerScope ts(p, HOQRI_KERNEL_TTMCTC, s);
    HOQRI_HIP_TRY(set_shmem(k.ttm, job.shmem));
    void* args[] = {(void*)&job.seg};
    HOQRI_HIP_TRY(hipLaunchKernel(k.ttm, dim3(job.seg_blocks), dim3(job.threads), args, job.shmem, s));
  }
  TimerScope tf(p, HOQRI_KERNEL_FIXUP, s);
  hipLaunchKernelGGL(k_fix_split, dim3(job.fix_blocks), dim3(256), 0, s, job.fix);
  const ModeData& md = p->md[mode];
  if (md.E > 0) {
    int64_t tot = md.E * p->K[mode];
    int grid = (int)((tot + 255) / 256 < 65536 ? (tot + 255) / 256 : 65536);
    hipLaunchKernelGGL(k_zero_rows, dim3(grid), dim3(256), 0, s, out_map ? md.empty_row : (const int32_t*)nullptr,
                       md.R, md.E, p->K[mode], A);
  }
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

hoqri_status launch_core(hoqri_plan* p, const Operands& op, float* G, double* f_out, hipStream_t s) {
  if (!segpass_supported(p, p->core_mode)) {
    if (!generic_supported(p)) return HOQRI_ERR_UNSUPPORTED;
    if (p->yfuse && (op.prec == OP_FP32 || op.prec == OP_BF16)) {
      // split-Kronecker pass on the core mode, then G_(c) = U^(c)T Y_(c)
      YCoreJob job;
      {
        TimerScope ts(p, HOQRI_KERNEL_CORE, s);
        HOQRI_TRY(launch_gen_rows(p, p->core_mode, op.prec, s));
      }
      HOQRI_TRY(prepare_ycore(p, p->core_mode, G, f_out, &job, false, false));
      launch_core_gemm(job.gemm, job.gemm_blocks, s);
      hipLaunchKernelGGL(k_core_reduce, dim3(job.red_blocks), dim3(kRedThreads), 0, s, job.red);
      hipLaunchKernelGGL(k_sum_f, dim3(1), dim3(256), 0, s, job.sum);
      HOQRI_HIP_TRY(hipGetLastError());
      return HOQRI_OK;
    }
    if (op.prec != OP_FP32) return HOQRI_ERR_UNSUPPORTED;
    GenArgs a = gen_args(p, p->core_mode);
    a.Uc = op.U32[p->core_mode];
    a.Gout = G;
    int64_t PK = 1;
    for (int n = 0; n < p->N; ++n) PK *= p->K[n];
    TimerScope ts(p, HOQRI_KERNEL_CORE, s);
    hipLaunchKernelGGL(k_core_generic, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(256), 0, s, (const float*)G, PK, f_out ? f_out : p->sc.f_dev);
    HOQRI_HIP_TRY(hipGetLastError());
    return HOQRI_OK;
  }
  CoreJob job;
  HOQRI_TRY(prepare_core(p, op, G, f_out, &job));
  SegKernels k;
  seg_kernels(job.key, &k);
  {
    TimerScope ts(p, HOQRI_KERNEL_CORE, s);
    const void* kern = job.key >= 1000 ? k.rows : k.core;
    HOQRI_HIP_TRY(set_shmem(kern, job.shmem));
    void* args[] = {(void*)&job.seg};
    HOQRI_HIP_TRY(hipLaunchKernel(kern, dim3(job.seg_blocks), dim3(job.threads), args, job.shmem, s));
  }
  if (job.key >= 1000) launch_core_gemm(job.gemm, job.gemm_blocks, s);
  hipLaunchKernelGGL(k_core_reduce, dim3(job.red_blocks), dim3(kRedThreads), 0, s, job.red);
  hipLaunchKernelGGL(k_sum_f, dim3(1), dim3(256), 0, s, job.sum);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

// Core from the rows Y_(mode) that the last TTMcTC pass of `mode` stored and
// the updated factor U^(mode): G_(mode) = U^(mode)T Y_(mode). The rows (nonempty
// slices, then the split-slice partials) are cut into ycore_chunks(rows)
// chunks (at most kYChunks); partials are reduced in chunk order.
hoqri_status prepare_ycore(hoqri_plan* p, int mode, float* G, double* f_out, YCoreJob* job, bool split, bool yb16) {
  if (!p->yfuse) return HOQRI_ERR_UNSUPPORTED;
  const PassGeom g = geom(p, mode);
  const int KN2 = (p->K[mode] + 15) / 16;
  *job = YCoreJob{};
  int64_t W = p->md[mode].ranges;
  if (W > p->nnz) W = p->nnz;
  if (!segpass_supported(p, mode)) W = 0;  // the split-Kronecker pass keeps slices whole
  CoreGemmArgs& m = job->gemm;
  m.ybuf = p->sc.ybuf;
  m.ycarry = p->sc.ycarry;
  m.ymeta = p->sc.meta;
  m.seg_row = p->md[mode].seg_row;
  m.Uc = p->sc.Up[mode];
  m.Kc = p->K[mode];
  m.KC = 16 * KN2;
  m.R = (int32_t)p->md[mode].R;
  m.W = (int32_t)W;
  m.B = g.B;
  const int64_t chunks = ycore_chunks((int64_t)m.R + 2 * W);
  m.nchunk = (int32_t)chunks;
  m.split = (split || yb16) ? 1 : 0;
  m.yb16 = yb16 ? 1 : 0;
  m.gpart = p->sc.gpart;
  job->gemm_blocks = (int)(chunks * g.B);
  CoreRedArgs& r = job->red;
  r.gpart = p->sc.gpart;
  r.groups = (int32_t)chunks;
  r.B = g.B;
  r.CB = g.CB;
  r.KN2 = KN2;
  r.krow = g.krow;
  r.kcol = g.kcol;
  r.Kc = p->K[mode];
  r.mode = mode;
  r.nm1 = g.nm1;
  for (int c = 0; c < kMaxOrder - 1; ++c) {
    r.om[c] = c < g.nm1 ? g.om[c] : 0;
    r.Ko[c] = c < g.nm1 ? g.Ko[c] : 1;
  }
  g_strides(p, r.gstride);
  r.G = G;
  r.fpart = p->sc.fpart;
  r.pair = (yb16 && ttm_pair(g)) ? 1 : 0;  // the rows of the 2 x 2-block pass are in paired order
  const int total = g.B * 16 * KN2 * 256;
  job->red_blocks = (total + kRedOut - 1) / kRedOut;
  job->sum.part = p->sc.fpart;
  job->sum.n = job->red_blocks;
  job->sum.out = f_out ? f_out : p->sc.f_dev;
  return HOQRI_OK;
}

hoqri_status launch_ycore(hoqri_plan* p, int mode, float* G, double* f_out, hipStream_t s, bool split, bool yb16) {
  YCoreJob job;
  HOQRI_TRY(prepare_ycore(p, mode, G, f_out, &job, split, yb16));
  TimerScope ts(p, HOQRI_KERNEL_CORE, s);
  launch_core_gemm(job.gemm, job.gemm_blocks, s);
  hipLaunchKernelGGL(k_core_reduce, dim3(job.red_blocks), dim3(kRedThreads), 0, s, job.red);
  hipLaunchKernelGGL(k_sum_f, dim3(1), dim3(256), 0, s, job.sum);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

hoqri_status launch_rows_a(hoqri_plan* p, int mode, const float* G, float* A, hipStream_t s, bool yb16) {
  if (!segpass_supported(p, mode)) {
    if (!p->yfuse) return HOQRI_ERR_UNSUPPORTED;
    TimerScope ts(p, HOQRI_KERNEL_CORE, s);
    return gen_rows_a(p, mode, G, A, nullptr, s);
  }
  TtmJob job;  // for the stage-two operand and the fix-up of this mode's ranges
  const Operands op{OP_FP32, p->sc.Up, p->sc.Uh};
  HOQRI_TRY(prepare_ttm(p, mode, op, G, A, nullptr, &job, true));
  RowsAArgs r{};
  r.ybuf = p->sc.ybuf;
  r.ycarry = p->sc.ycarry;
  r.ymeta = p->sc.meta;
  r.gtop = p->sc.gtop;
  r.R = job.seg.R;
  r.W = job.seg.W;
  r.B = job.seg.B;
  r.KN2 = job.prep.KN2;
  r.Kn = p->K[mode];
  r.yb16 = yb16 ? 1 : 0;
  r.groups = ((int64_t)r.R + 2 * (int64_t)r.W + 15) / 16;
  r.A = A;
  r.carry = p->sc.carry;
  // k_rows_a reads the operand in the classic float32 order, whatever order
  // this mode's TTMcTC pass uses, with the rows' own entry order
  job.prep.wide16 = 0;
  job.prep.pair = (yb16 && ttm_pair(geom(p, mode))) ? 1 : 0;
  TimerScope ts(p, HOQRI_KERNEL_CORE, s);
  hipLaunchKernelGGL(k_prep_gtop, dim3(job.prep_blocks), dim3(256), 0, s, job.prep);
  hipLaunchKernelGGL(k_rows_a, dim3((unsigned)((r.groups + 3) / 4)), dim3(256), 0, s, r);
  hipLaunchKernelGGL(k_fix_split, dim3(job.fix_blocks), dim3(256), 0, s, job.fix);
  const ModeData& md = p->md[mode];
  if (md.E > 0) {
    int64_t tot = md.E * p->K[mode];
    int grid = (int)((tot + 255) / 256 < 65536 ? (tot + 255) / 256 : 65536);
    hipLaunchKernelGGL(k_zero_rows, dim3(grid), dim3(256), 0, s, (const int32_t*)nullptr, md.R, md.E, p->K[mode], A);
  }
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

// ---------------------------------------------------------------------------
// Batched launches (request server)
// ---------------------------------------------------------------------------
bool stage_ttm_group(const TtmJob* const* jobs, int n, Staging& st, TtmGroup* g) {
  if (n < 1 || n > 1024) return false;
  std::vector<PrepArgs> prep(n);
  std::vector<SegArgs> seg(n);
  std::vector<FixArgs> fix(n);
  std::vector<int32_t> nb_prep(n), nb_seg(n), nb_fix(n);
  for (int i = 0; i < n; ++i) {
    prep[i] = jobs[i]->prep;
    seg[i] = jobs[i]->seg;
    fix[i] = jobs[i]->fix;
    nb_prep[i] = jobs[i]->prep_blocks;
    nb_seg[i] = jobs[i]->seg_blocks;
    nb_fix[i] = jobs[i]->fix_blocks;
  }
  g->key = jobs[0]->key;
  g->threads = jobs[0]->threads;
  g->shmem = jobs[0]->shmem;
  return stage_table(st, prep.data(), nb_prep.data(), n, &g->prep) &&
         stage_table(st, seg.data(), nb_seg.data(), n, &g->seg) && stage_table(st, fix.data(), nb_fix.data(), n, &g->fix);
}

bool stage_core_group(const CoreJob* const* jobs, int n, Staging& st, CoreGroup* g) {
  if (n < 1 || n > 1024) return false;
  std::vector<SegArgs> seg(n);
  std::vector<CoreGemmArgs> gemm(n);
  std::vector<CoreRedArgs> red(n);
  std::vector<SumArgs> sum(n);
  std::vector<int32_t> nb_seg(n), nb_gemm(n), nb_red(n), ones(n);
  for (int i = 0; i < n; ++i) {
    seg[i] = jobs[i]->seg;
    gemm[i] = jobs[i]->gemm;
    red[i] = jobs[i]->red;
    sum[i] = jobs[i]->sum;
    nb_seg[i] = jobs[i]->seg_blocks;
    nb_gemm[i] = jobs[i]->gemm_blocks;
    nb_red[i] = jobs[i]->red_blocks;
    ones[i] = 1;
  }
  g->key = jobs[0]->key;
  g->threads = jobs[0]->threads;
  g->shmem = jobs[0]->shmem;
  g->gemm = BatchTable{nullptr, nullptr, 0, 0};
  if (g->key >= 1000 && !stage_table(st, gemm.data(), nb_gemm.data(), n, &g->gemm)) return false;
  return stage_table(st, seg.data(), nb_seg.data(), n, &g->seg) &&
         stage_table(st, red.data(), nb_red.data(), n, &g->red) && stage_table(st, sum.data(), ones.data(), n, &g->sum);
}

bool stage_ycore_group(const YCoreJob* const* jobs, int n, Staging& st, YCoreGroup* g) {
  if (n < 1 || n > 1024) return false;
  std::vector<CoreGemmArgs> gemm(n);
  std::vector<CoreRedArgs> red(n);
  std::vector<SumArgs> sum(n);
  std::vector<int32_t> nb_gemm(n), nb_red(n), ones(n);
  for (int i = 0; i < n; ++i) {
    gemm[i] = jobs[i]->gemm;
    red[i] = jobs[i]->red;
    sum[i] = jobs[i]->sum;
    nb_gemm[i] = jobs[i]->gemm_blocks;
    nb_red[i] = jobs[i]->red_blocks;
    ones[i] = 1;
  }
  return stage_table(st, gemm.data(), nb_gemm.data(), n, &g->gemm) &&
         stage_table(st, red.data(), nb_red.data(), n, &g->red) && stage_table(st, sum.data(), ones.data(), n, &g->sum);
}

hoqri_status launch_ycore_group(const YCoreGroup& g, hipStream_t s) {
  hipLaunchKernelGGL(k_core_gemm_b, dim3(g.gemm.blocks), dim3(kGemmThreads), 0, s, (const CoreGemmArgs*)g.gemm.descs,
                     g.gemm.first, g.gemm.count);
  hipLaunchKernelGGL(k_core_reduce_b, dim3(g.red.blocks), dim3(kRedThreads), 0, s, (const CoreRedArgs*)g.red.descs,
                     g.red.first, g.red.count);
  hipLaunchKernelGGL(k_sum_f_b, dim3(g.sum.blocks), dim3(256), 0, s, (const SumArgs*)g.sum.descs, g.sum.first,
                     g.sum.count);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

hoqri_status launch_ttm_group(const TtmGroup& g, hipStream_t s) {
  SegKernels k;
  if (!seg_kernels(g.key, &k)) return HOQRI_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(k_prep_gtop_b, dim3(g.prep.blocks), dim3(256), 0, s, (const PrepArgs*)g.prep.descs,
                     g.prep.first, g.prep.count);
  HOQRI_HIP_TRY(set_shmem(k.ttm_b, g.shmem));
  const SegArgs* d = (const SegArgs*)g.seg.descs;
  const int32_t* first = g.seg.first;
  int count = g.seg.count;
  void* args[] = {(void*)&d, (void*)&first, (void*)&count};
  HOQRI_HIP_TRY(hipLaunchKernel(k.ttm_b, dim3(g.seg.blocks), dim3(g.threads), args, g.shmem, s));
  hipLaunchKernelGGL(k_fix_split_b, dim3(g.fix.blocks), dim3(256), 0, s, (const FixArgs*)g.fix.descs, g.fix.first,
                     g.fix.count);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

hoqri_status launch_core_group(const CoreGroup& g, hipStream_t s) {
  SegKernels k;
  if (!seg_kernels(g.key, &k)) return HOQRI_ERR_UNSUPPORTED;
  const void* kern = g.key >= 1000 ? k.rows_b : k.core_b;
  HOQRI_HIP_TRY(set_shmem(kern, g.shmem));
  const SegArgs* d = (const SegArgs*)g.seg.descs;
  const int32_t* first = g.seg.first;
  int count = g.seg.count;
  void* args[] = {(void*)&d, (void*)&first, (void*)&count};
  HOQRI_HIP_TRY(hipLaunchKernel(kern, dim3(g.seg.blocks), dim3(g.threads), args, g.shmem, s));
  if (g.key >= 1000)
    hipLaunchKernelGGL(k_core_gemm_b, dim3(g.gemm.blocks), dim3(kGemmThreads), 0, s, (const CoreGemmArgs*)g.gemm.descs,
                       g.gemm.first, g.gemm.count);
  hipLaunchKernelGGL(k_core_reduce_b, dim3(g.red.blocks), dim3(kRedThreads), 0, s, (const CoreRedArgs*)g.red.descs,
                     g.red.first, g.red.count);
  hipLaunchKernelGGL(k_sum_f_b, dim3(g.sum.blocks), dim3(256), 0, s, (const SumArgs*)g.sum.descs, g.sum.first,
                     g.sum.count);
  HOQRI_HIP_TRY(hipGetLastError());
  return HOQRI_OK;
}

}  // namespace hoqri
