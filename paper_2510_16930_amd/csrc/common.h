// Internal declarations shared by the translation units of libhoqri.
// Everything here is an implementation detail behind include/hoqri.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/hoqri.h"

namespace hoqri {

constexpr int kMaxOrder = HOQRI_MAX_ORDER;
constexpr int kMaxRank = HOQRI_MAX_RANK;
constexpr int kWave = 64;
constexpr int kMaxSweeps = 4096;

// Status helpers -------------------------------------------------------------
#define HOQRI_HIP_TRY(expr)                                  \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return HOQRI_ERR_HIP;              \
  } while (0)

#define HOQRI_TRY(expr)                                      \
  do {                                                       \
    hoqri_status _s = (expr);                                \
    if (_s != HOQRI_OK) return _s;                           \
  } while (0)

// Per-mode data of a plan: the nonzeros stably sorted by their mode-n index,
// stored as structure of arrays, and the table of nonempty slices.
struct ModeData {
  // The nonzeros in mode-n sorted order as block records: for every block of
  // 16 nonzeros (e = 16b + 4t + g) and lane group g, N dwords-quads in turn:
  // for each other mode m' (ascending, mode n skipped) the byte offsets
  // 2 label(i_m) K_m of the nonzeros' factor rows in a 16-bit copy (4t+g,
  // t = 0..3; a float32 row starts at twice that), then their values
  // (float32 bits). rec[b][g][a][t], 16 N dwords per block; padding is zero.
  int32_t* rec;
  int32_t* seg_row;    // [R]   mode-n index of each nonempty slice (ascending)
  int32_t* seg_off;    // [R+1] first nonzero of each slice in sorted order
  int32_t* lab;        // [I_n] new label of original index i (descending slice size)
  int32_t* inv;        // [I_n] original index of label r
  int32_t* empty_row;  // [E]   original indices of the empty slices (= inv + R)
  int64_t R;           // number of nonempty slices
  int64_t E;           // number of empty slices (I_n - R)
  int32_t ranges;      // work ranges of the TTMcTC pass on this mode (tunable up to ranges_cap)
  int32_t ranges0;     // the library's own choice (plan creation)
  int32_t rpw;         // ranges per workgroup of the TTMcTC pass (0: the library's rule)
};

// Scratch regions used by the passes (all inside the caller's workspace).
struct Scratch {
  float* Up[kMaxOrder];  // factors with rows in the plan's label order
  uint16_t* Uh[kMaxOrder];  // 16-bit copies of Up (bfloat16, or float16 scaled by 2^15)
  float* A;            // max_n I_n * K_n floats: TTMcTC output inside hoqri_run
  float* G;            // prod K floats: the core inside hoqri_run
  float* gpart;        // core partials: core_groups * pad_core floats
  double* fpart;       // per-block partial sums of ||G||^2
  float* gtop;         // TTMcTC stage-two operand (core rearranged), <= 2 * pad floats
  float* carry;        // ranges_max * 2 * 32 floats: partial rows of split slices
  int32_t* meta;       // ranges_max * 4 ints
  double* orth_ws;     // CholeskyQR2 workspace (Gram partials, factors)
  int32_t* status;     // device status flags [4]: breakdown, skipped updates, FP16 range, slice-pool fault
  double* f_dev;       // scalars [64]
  double* fsweep;      // f after each sweep inside hoqri_run [kMaxSweeps + 1]
  double* gscr;        // gradient monitor: G_(n) G_(n)^T [32*32], block partials [4096], history
  float* ybuf;         // slice rows y_i: of the core mode [ybuf_rows][B_c * 256] (row-writing core
                       // pass), or of a TTMcTC pass's mode [R_n][B_n * 256] (stored rows)
  float* ycarry;       // their split-slice partials [ranges][2][B * 256]
  int32_t* ymeta;      // [core_w][4] (the TTMcTC pass keeps its range metadata in meta)
  size_t orth_ws_bytes;
};

}  // namespace hoqri

namespace hoqri {
// Optional per-kernel HIP-event timing of a plan's launches.
constexpr int kTimingKinds = 4;
constexpr int kTimingCap = 4096;
struct Timing {
  bool enabled = false;
  hipEvent_t* ev[kTimingKinds] = {nullptr, nullptr, nullptr, nullptr};  // 2 per launch
  int64_t count[kTimingKinds] = {0, 0, 0, 0};
};
}  // namespace hoqri

struct hoqri_plan {
  int32_t N;
  int64_t dims[hoqri::kMaxOrder];
  int32_t K[hoqri::kMaxOrder];
  int64_t nnz_in;      // coordinates given
  int64_t nnz;         // distinct coordinates after merging duplicates
  double normx2;       // ||X||^2 (float64)
  double maxabs_x;     // max |x| over the merged nonzeros
  int32_t core_mode;   // mode whose sorted copy the core pass reads (fewest slices)
  int32_t core_groups; // partials the core reduction sums
  int32_t core_rows;   // the core pass writes slice rows (see Layout)
  int64_t ybuf_rows;
  int32_t core_w;
  int32_t yfuse;       // TTMcTC passes can store Y_(n) and the core follows from it
  int32_t ranges_cap;  // most work ranges the range buffers (carries, metadata, row partials) hold
  hoqri::ModeData md[hoqri::kMaxOrder];
  hoqri::Scratch sc;
  void* ws;
  size_t ws_bytes;
  int32_t device;
  hoqri::Timing timing;
};

namespace hoqri {

// Layout of the workspace for a shape (computed on the host; sort temporary
// size needs the device). Offsets are 256-byte aligned.
struct Layout {
  size_t total;
  size_t persistent;   // plan data that lives until destroy
  size_t build_tmp;    // transient storage during plan creation
  size_t run_scratch;  // scratch of the passes (overlaps build_tmp)
  size_t sort_tmp;     // rocPRIM temporary storage
  int32_t ranges[kMaxOrder];
  int32_t ranges_cap;    // range buffers are sized for this many ranges (room for tuning)
  int32_t core_groups;   // partial blocks reduced by the core pass
  int32_t core_mode;     // mode whose sorted copy the core pass reads
  int32_t core_rows;     // nonzero: core pass writes slice rows y_i, then a small product with U^(c)
  int64_t ybuf_rows;     // rows of the slice-row buffer (>= nonempty slices of the core mode)
  int32_t core_w;        // work ranges of the row-writing core pass
  int32_t yfuse;         // every mode's TTMcTC pass can store its slice rows
  size_t ybuf_floats;    // slice-row buffer
  size_t ycarry_floats;  // its split-slice partials
  size_t gpart_floats;   // core partials
  size_t fpart_doubles;  // per-block partial sums of ||G||^2 of the core reduction (one per 16 entries)
};
constexpr int kCoreChunk = 64;  // rows per partial of the core product U^(c)T Y (core-mode pass)
constexpr int kYChunks = 128;  // most partials of the core product from stored rows
// Partials of the core product from stored rows for nv rows: one per 1024
// rows at least, a multiple of 8 (the product's blocks are spread over the
// eight XCDs by chunk), at most kYChunks.
inline int64_t ycore_chunks(int64_t nv) {
  int64_t c = (nv + 1023) / 1024;
  c = (c + 7) / 8 * 8;
  return c < kYChunks ? c : kYChunks;
}

hoqri_status compute_layout(int32_t N, const int64_t* dims, const int32_t* K, int64_t nnz, Layout* L);
hoqri_status validate_shape(int32_t N, const int64_t* dims, const int32_t* K, int64_t nnz);

// Segment-pass kernels (segpass.hip). Factors are in the plan's label order:
// U32 float32 (always; the core pass multiplies by its pass mode's factor in
// float32), U16 the 16-bit copies read by the BF16 / FP16 forms.
enum OperandPrec { OP_FP32 = 0, OP_BF16 = 1, OP_FP16 = 2 };
struct Operands {
  int prec;  // OperandPrec
  const float* const* U32;
  const uint16_t* const* U16;
};
hoqri_status launch_core(hoqri_plan* p, const Operands& op, float* G, double* f_out, hipStream_t s);
// out_map null: A rows in label order and rows R..I-1 zeroed; otherwise row r is
// written at out_map[r] (original order) and the empty slices' original rows
// are zeroed.
// rows: the pass also stores Y_(mode) for launch_ycore (requires yfuse).
hoqri_status launch_ttmctc(hoqri_plan* p, int mode, const Operands& op, const float* G, float* A,
                           const int32_t* out_map, hipStream_t s, bool rows = false);
// G = X x {U^T} from the rows Y_(mode) stored by the last TTMcTC pass of `mode`
// and the (updated) factor U^(mode) in the plan's scratch; ||G||^2 into *f_out.
hoqri_status launch_ycore(hoqri_plan* p, int mode, float* G, double* f_out, hipStream_t s, bool split = false,
                          bool yb16 = false);
// The TTMcTC pass of `mode` in operand form `prec` stores its slice rows in
// bfloat16 (the 2 x 2-block BF16 pass) rather than float32.
bool ttm_rows_bf16(const hoqri_plan* p, int mode, int prec);
// Most ranges per workgroup the TTMcTC pass of `mode` takes in form `prec`.
int ttm_max_rpw(const hoqri_plan* p, int mode, int prec);
// A = Y_(mode) G_(mode)^T from the rows stored by the last TTMcTC pass of
// `mode` (label order, rows of empty slices zeroed): one inner step of HOOI's
// orthogonal iteration when G = U^(mode)T Y_(mode).
hoqri_status launch_rows_a(hoqri_plan* p, int mode, const float* G, float* A, hipStream_t s, bool yb16 = false);
bool segpass_supported(const hoqri_plan* p, int mode);
// Modes the segment passes do not take use the generic kernels (float32
// operands; every rank <= 32).
bool generic_supported(const hoqri_plan* p);
// Power-of-two scales of the FP16 form for this plan (false: the values' range
// does not allow them; use another precision).
bool fp16_scales(const hoqri_plan* p, int nm1, float* ascale, float* yscale);
// Rounds rows [0, rows) of a float32 factor (K columns) to the 16-bit copy.
hoqri_status launch_cast16(const float* U, int64_t rows, int32_t K, uint16_t* Uh, int prec, hipStream_t s,
                           int32_t* range_flag = nullptr);

// Factor rows between the caller's order and the plan's label order (run.hip).
hoqri_status to_labels(hoqri_plan* p, const float* const* U, hipStream_t s);
hoqri_status from_labels(hoqri_plan* p, float* const* U, hipStream_t s);
// Zeroes the label-order rows of mode n's empty slices (rows R_n .. I_n-1).
hoqri_status zero_empty_rows(hoqri_plan* p, int n, hipStream_t s);
hoqri_status fill_i32(int32_t* x, int n, int32_t v, hipStream_t s);

// Riemannian gradient monitor (run.hip): ||2 (A - U G_(n) G_(n)^T)||_F^2 into *out.
hoqri_status launch_grad(hoqri_plan* p, int mode, const float* A, const float* U, const float* G, double* out,
                         hipStream_t s);
constexpr int kGradParts = 4096;

// CholeskyQR2 (orth.hip).
size_t orth_ws_bytes(int64_t rows, int32_t cols);
// Uh (optional): the 16-bit copy of the updated rows in form prec16, written
// by the apply kernel with them (what launch_cast16 would write).
hoqri_status launch_orth(int64_t rows, int32_t cols, const float* A, float* U, double* R,
                         int32_t* status, void* ws, size_t ws_bytes, hipStream_t s, bool sticky,
                         int32_t* skipped = nullptr, int64_t zero_to = 0, uint16_t* Uh = nullptr,
                         int prec16 = 0, int32_t* range_flag = nullptr);
hoqri_status launch_orth_err(int64_t rows, int32_t cols, const float* U, double* err_out, void* ws,
                             size_t ws_bytes, hipStream_t s);

// Records a start event on construction and a stop event on destruction when
// timing is enabled on the plan (no-op otherwise).
struct TimerScope {
  hoqri_plan* p;
  int kind;
  hipStream_t s;
  int64_t slot;
  TimerScope(hoqri_plan* plan, int k, hipStream_t st) : p(plan), kind(k), s(st), slot(-1) {
    if (p && p->timing.enabled && p->timing.count[kind] < kTimingCap) {
      slot = p->timing.count[kind]++;
      (void)hipEventRecord(p->timing.ev[kind][2 * slot], s);
    }
  }
  ~TimerScope() {
    if (slot >= 0) (void)hipEventRecord(p->timing.ev[kind][2 * slot + 1], s);
  }
};
void timing_release(hoqri_plan* p);

// Element offsets of the other modes of `mode` (ascending, mode skipped).
inline int other_modes(int N, int mode, int* out) {
  int c = 0;
  for (int m = 0; m < N; ++m)
    if (m != mode) out[c++] = m;
  return c;
}

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// y_i as a matrix whose rows are the first few other modes and whose columns
// are the rest (C order, so row-major in this matrix): the segment passes take
// the last other mode as the columns; four other modes (order 5) are split
// two and two, so both halves of the Kronecker product stay short.
inline int yi_row_modes(int nm1) { return nm1 >= 4 ? nm1 - 2 : nm1 - 1; }

}  // namespace hoqri
