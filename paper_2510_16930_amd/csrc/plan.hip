// Plan construction: index validation, merging of duplicate coordinates,
// ||X||^2, and for every mode n a copy of the nonzeros stably sorted by i_n
// together with the table of nonempty index sets I^(n)_{i_n} (Table 1).
//
// Integer and sort dominated; runs once per tensor. Sorting uses rocPRIM's
// stable radix sort; every other step is a small kernel of this file.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <new>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "common.h"

namespace hoqri {
namespace {

constexpr int kThreads = 256;

inline int grid_for(int64_t n, int threads = kThreads, int cap = 65536) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

int bits_for(uint64_t max_value_exclusive) {
  int b = 0;
  while (b < 64 && (uint64_t(1) << b) < max_value_exclusive) ++b;
  return b < 1 ? 1 : b;
}

struct KeyArgs {
  const int32_t* idx;
  int64_t nnz;
  int32_t N;
  int64_t dims[kMaxOrder];
  uint64_t stride[kMaxOrder];
};

// Range check of every coordinate and the C-order linear key of each nonzero.
__global__ void k_keys(KeyArgs a, uint64_t* keys, int32_t* pos, int32_t* err) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < a.nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t key = 0;
    bool bad = false;
    for (int m = 0; m < a.N; ++m) {
      int32_t i = a.idx[(int64_t)m * a.nnz + e];
      bad |= (i < 0) || ((int64_t)i >= a.dims[m]);
      key += (uint64_t)(i < 0 ? 0 : i) * a.stride[m];
    }
    if (bad) atomicOr(err, 1);
    keys[e] = key;
    pos[e] = (int32_t)e;
  }
}

template <typename T>
__global__ void k_head_flags(const T* keys, int64_t n, int32_t* head) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    head[e] = (e == 0 || keys[e] != keys[e - 1]) ? 1 : 0;
}

__global__ void k_count(const int32_t* head, const int32_t* scan, int64_t n, int64_t* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = (int64_t)scan[n - 1] + head[n - 1];
}

struct CoalesceArgs {
  const int32_t* idx;   // original coordinates [N][nnz_in]
  const float* vals;    // original values
  const uint64_t* keys; // sorted keys
  const int32_t* pos;   // original position of each sorted key
  const int32_t* head;
  const int32_t* uid;
  int64_t nnz_in;
  int32_t N;
  int32_t* cidx;        // [N][nnz_in] canonical coordinates (first nnz used)
  float* cval;
  double* vsq;
};

// One thread per run of equal keys: sums the run's values in sorted (= stable,
// input) order in float64, writes the canonical coordinate and value.
__global__ void k_coalesce(CoalesceArgs a) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < a.nnz_in;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (!a.head[e]) continue;
    double v = a.vals[a.pos[e]];
    for (int64_t f = e + 1; f < a.nnz_in && !a.head[f]; ++f) v += a.vals[a.pos[f]];
    int64_t j = a.uid[e];
    int32_t src = a.pos[e];
    for (int m = 0; m < a.N; ++m) a.cidx[(int64_t)m * a.nnz_in + j] = a.idx[(int64_t)m * a.nnz_in + src];
    float vf = (float)v;
    a.cval[j] = vf;
    a.vsq[j] = (double)vf * (double)vf;
  }
}

// Deterministic float64 sum: per-block partials, then one block in order.
__global__ void k_sum_partial(const double* x, const int64_t* n_dev, double* part) {
  __shared__ double sh[kThreads];
  int64_t n = *n_dev;
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    acc += x[e];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_final(const double* part, int nparts, double* out) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Per-block maxima of x (non-negative values, e.g. squares), then the maximum.
__global__ void k_max_partial(const double* x, const int64_t* n_dev, double* part) {
  __shared__ double sh[kThreads];
  int64_t n = *n_dev;
  double m = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, x[e]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_max_final(const double* part, int nparts, double* out) {
  __shared__ double sh[kThreads];
  double m = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = fmax(m, part[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Keys i_n in the order given by lperm; values are canonical positions.
__global__ void k_mode_keys_perm(const int32_t* cidx_n, const int32_t* lperm, int64_t nnz, uint32_t* k32,
                                 int32_t* perm) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz; j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = lperm[j];
    k32[j] = (uint32_t)cidx_n[c];
    perm[j] = c;
  }
}

__global__ void k_mode_keys(const int32_t* cidx_n, int64_t nnz, uint32_t* k32, int32_t* perm) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * blockDim.x) {
    k32[j] = (uint32_t)cidx_n[j];
    perm[j] = (int32_t)j;
  }
}

struct GatherArgs {
  const int32_t* cidx;   // [N][stride]
  const float* cval;
  const int32_t* perm;   // null = identity
  int64_t stride, nnz;
  int32_t N, mode;
  int32_t K[kMaxOrder];
  int32_t* rec;
  int32_t* modeidx;
  const int32_t* lab[kMaxOrder];  // label maps: stored offsets and slice rows use labels
};

// Mode-n sorted copy as block records (see ModeData::rec): nonzero
// j = 16b + 4t + g stores its other-mode factor row offsets at
// rec[b][g][c][t] (c-th other mode) and its value at rec[b][g][N-1][t]; a lane
// group of the segment passes reads its record with one dword per lane.
// Positions nnz .. nnz_pad-1 (padding to a multiple of 16) hold zeros.
__global__ void k_gather_mode(GatherArgs a) {
  const int64_t npad = (a.nnz + 15) / 16 * 16;
  const int N = a.N;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < npad;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = j >> 4;
    const int t = (int)((j & 15) >> 2), g = (int)(j & 3);
    int32_t* r = a.rec + b * 16 * N + g * 4 * N + t;
    if (j >= a.nnz) {
      for (int c = 0; c < N; ++c) r[4 * c] = 0;
      continue;
    }
    int64_t src = a.perm ? a.perm[j] : j;
    int c = 0;
    for (int m = 0; m < N; ++m) {
      const int32_t i = a.cidx[(int64_t)m * a.stride + src];
      if (m == a.mode) {
        a.modeidx[j] = i;  // original index: slice boundaries
      } else {
        r[4 * c++] = a.lab[m][i] * a.K[m] * 2;  // byte offset of the row in a 16-bit copy
      }
    }
    r[4 * (N - 1)] = __float_as_int(a.cval[src]);
  }
}

__global__ void k_segments(const int32_t* modeidx, const int32_t* head, const int32_t* sid, int64_t nnz,
                           const int32_t* lab, int32_t* seg_row, int32_t* seg_off, int64_t* R_out) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * blockDim.x) {
    if (head[j]) {
      seg_row[sid[j]] = lab[modeidx[j]];
      seg_off[sid[j]] = (int32_t)j;
    }
    if (j == nnz - 1) {
      int64_t R = (int64_t)sid[j] + head[j];
      seg_off[R] = (int32_t)nnz;
      *R_out = R;
    }
  }
}

// Slice sizes (degrees) of every mode-n index; integer atomics, exact. The
// lanes of a wave that hold the same index are counted together first (one
// atomic per distinct index per wave): a skewed mode sends a quarter of its
// nonzeros to one index, which per-lane atomics would serialise.
__global__ void k_degree(const int32_t* cidx_n, int64_t nnz, int32_t* deg) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // the loop runs the same number of times on every lane of a wave
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); base < nnz; base += stride) {
    const int64_t j = base + lane;
    const int32_t v = j < nnz ? cidx_n[j] : -1;
    uint64_t pending = __ballot(v >= 0);
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const int32_t lv = __builtin_amdgcn_readlane(v, leader);
      const uint64_t same = __ballot(v == lv) & pending;
      if (lane == leader) atomicAdd(&deg[lv], (int32_t)__popcll(same));
      pending &= ~same;
    }
  }
}

// Sort keys for the relabelling: larger degree first; the stable sort keeps
// equal degrees in index order.
__global__ void k_degree_keys(const int32_t* deg, int64_t In, uint32_t* key, int32_t* idx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < In; i += (int64_t)gridDim.x * blockDim.x) {
    key[i] = 0x7FFFFFFFu - (uint32_t)deg[i];
    idx[i] = (int32_t)i;
  }
}

struct LabKeyArgs {
  const int32_t* cidx;  // [N][stride]
  int64_t stride, nnz;
  int32_t N;
  const int32_t* lab[kMaxOrder];
  uint64_t lstride[kMaxOrder];
};

// C-order linear key of each nonzero's label coordinates; position as value.
__global__ void k_label_keys(LabKeyArgs a, uint64_t* keys, int32_t* pos) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < a.nnz; j += (int64_t)gridDim.x * blockDim.x) {
    uint64_t k = 0;
    for (int m = 0; m < a.N; ++m) k += (uint64_t)a.lab[m][a.cidx[(int64_t)m * a.stride + j]] * a.lstride[m];
    keys[j] = k;
    pos[j] = (int32_t)j;
  }
}

// lab[inv[r]] = r
__global__ void k_invert(const int32_t* inv, int64_t In, int32_t* lab) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < In; r += (int64_t)gridDim.x * blockDim.x)
    lab[inv[r]] = (int32_t)r;
}

__global__ void k_fill_i32(int32_t* x, int64_t n, int32_t v) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x)
    x[j] = v;
}

// Workspace carving ---------------------------------------------------------
struct Carver {
  char* base;
  size_t off;
  template <typename T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

size_t sort_tmp_bytes(int64_t nnz, int64_t Imax, hipError_t* err) {
  size_t b64 = 0, b32 = 0, bs = 0, bs2 = 0;
  *err = rocprim::radix_sort_pairs(nullptr, b64, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                                   (int32_t*)nullptr, (size_t)nnz, 0, 64, (hipStream_t)0);
  if (*err != hipSuccess) return 0;
  *err = rocprim::radix_sort_pairs(nullptr, b32, (uint32_t*)nullptr, (uint32_t*)nullptr, (int32_t*)nullptr,
                                   (int32_t*)nullptr, (size_t)(nnz > Imax ? nnz : Imax), 0, 32, (hipStream_t)0);
  if (*err != hipSuccess) return 0;
  *err = rocprim::exclusive_scan(nullptr, bs, (int32_t*)nullptr, (int32_t*)nullptr, 0, (size_t)nnz,
                                 rocprim::plus<int32_t>(), (hipStream_t)0);
  if (*err != hipSuccess) return 0;
  *err = rocprim::exclusive_scan(nullptr, bs2, (int32_t*)nullptr, (int32_t*)nullptr, 0, (size_t)Imax,
                                 rocprim::plus<int32_t>(), (hipStream_t)0);
  if (*err != hipSuccess) return 0;
  size_t m = b64;
  if (b32 > m) m = b32;
  if (bs > m) m = bs;
  if (bs2 > m) m = bs2;
  return align_up(m);
}

}  // namespace

hoqri_status validate_shape(int32_t N, const int64_t* dims, const int32_t* K, int64_t nnz) {
  if (N < 2 || N > kMaxOrder || !dims || !K) return HOQRI_ERR_ARG;
  if (nnz < 1 || nnz >= (int64_t(1) << 30)) return HOQRI_ERR_ARG;
  for (int n = 0; n < N; ++n)
    if (dims[n] < 1 || dims[n] >= (int64_t(1) << 31)) return HOQRI_ERR_ARG;
  // Duplicates are found by sorting C-order linear keys (uint64): the product
  // of the dims must not exceed 2^63, or distinct coordinates could share a key.
  unsigned __int128 cells = 1;
  for (int n = 0; n < N; ++n) {
    cells *= (unsigned __int128)dims[n];
    if (cells > ((unsigned __int128)1 << 63)) return HOQRI_ERR_UNSUPPORTED;
  }
  // A mode's block records (4 N bytes per nonzero, padded to 16 nonzeros) are
  // read through buffer descriptors with 32-bit byte offsets.
  if ((nnz + 15) / 16 * 16 * 4 * (int64_t)N >= (int64_t(1) << 32)) return HOQRI_ERR_UNSUPPORTED;
  for (int n = 0; n < N; ++n) {
    if (K[n] < 1 || K[n] > dims[n]) return HOQRI_ERR_RANK;
    int64_t other = 1;
    for (int m = 0; m < N; ++m)
      if (m != n) other *= K[m];
    if (K[n] > other) return HOQRI_ERR_RANK;
    if (K[n] > kMaxRank) return HOQRI_ERR_UNSUPPORTED;
    if (dims[n] * (int64_t)K[n] * 4 >= (int64_t(1) << 32)) return HOQRI_ERR_UNSUPPORTED;
  }
  return HOQRI_OK;
}

// Stage-two operand size (floats) of the TTMcTC pass on mode n and the core
// partial size (floats) of the core pass on mode n; see segpass.hip.
// Stage-two operand and core-partial sizes of mode n's segment pass (zero when
// the shape is beyond the passes: then mode n takes the generic kernels).
// Stage-two operand (any mode: the segment passes and the split-Kronecker
// pass's product from stored rows) and core-pass partials (segment passes).
static void pass_sizes(int32_t N, const int32_t* K, int n, size_t* gtop, size_t* gpart) {
  int om[kMaxOrder];
  int no = other_modes(N, n, om);
  const int nr = yi_row_modes(no);
  int64_t krow = 1, kcol = 1;
  for (int c = 0; c < no; ++c) (c < nr ? krow : kcol) *= K[om[c]];
  int64_t RB = (krow + 15) / 16, CB = (kcol + 15) / 16;
  int64_t B = RB * CB;
  int64_t KN2 = (K[n] + 15) / 16;
  const bool seg = B <= 8 && K[n] <= 32 && no <= 3;
  *gtop = K[n] <= 32 ? (size_t)(B * KN2 * 4096) : 0;
  *gpart = seg ? (size_t)(B * 256 * 16 * KN2) : 0;
}

// Work ranges of a pass: about 3072 nonzeros each on large tensors; smaller
// tensors are cut finer (down to 128 nonzeros) so that up to 2048 waves share
// the work instead of a few dozen walking long ranges.
static int32_t choose_ranges(int64_t nnz) {
  int64_t w = nnz / 3072;
  const int64_t fine = std::min<int64_t>(nnz / 128, 2048);
  if (w < fine) w = fine;
  if (w < 1) w = 1;
  if (w > 16384) w = 16384;
  return (int32_t)w;
}

static int32_t choose_core_groups(int64_t nnz, int64_t B) {
  int64_t g = nnz / 16384;
  int64_t cap = B >= 4 ? 256 : 512;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int32_t)g;
}

hoqri_status compute_layout(int32_t N, const int64_t* dims, const int32_t* K, int64_t nnz, Layout* L) {
  HOQRI_TRY(validate_shape(N, dims, K, nnz));
  int64_t Imax = 0, IKmax = 0, PK = 1;
  for (int n = 0; n < N; ++n) {
    if (dims[n] > Imax) Imax = dims[n];
    if (dims[n] * K[n] > IKmax) IKmax = dims[n] * K[n];
    PK *= K[n];
  }
  hipError_t e;
  size_t stmp = sort_tmp_bytes(nnz, Imax, &e);
  if (e != hipSuccess) return HOQRI_ERR_HIP;

  Carver c{nullptr, 0};
  // persistent
  const int64_t npad = (nnz + 15) / 16 * 16;
  for (int n = 0; n < N; ++n) {
    c.take<int32_t>(npad * N);  // block records
    int64_t rmax = dims[n] < nnz ? dims[n] : nnz;
    c.take<int32_t>(rmax);
    c.take<int32_t>(rmax + 1);
    c.take<int32_t>(dims[n]);  // lab
    c.take<int32_t>(dims[n]);  // inv
  }
  size_t persistent = c.off;
  // build temporaries
  Carver b{nullptr, 0};
  b.take<uint64_t>(nnz);
  b.take<uint64_t>(nnz);
  b.take<int32_t>(nnz);
  b.take<int32_t>(nnz);
  b.take<int32_t>(nnz);
  b.take<int32_t>(nnz);
  b.take<int32_t>((size_t)N * nnz);
  b.take<float>(nnz);
  b.take<double>(nnz);
  b.take<int32_t>(nnz);
  b.take<int32_t>(Imax);
  b.take<int32_t>(Imax);
  b.take<uint32_t>(Imax);
  b.take<uint32_t>(Imax);
  b.take<double>(65536);
  b.take<int64_t>(64);
  b.take<char>(stmp);
  size_t build = b.off;
  // run scratch
  size_t gtop_max = 0, gpart = 0;
  int64_t Bcore = 1;
  for (int n = 0; n < N; ++n) {
    size_t g1, g2;
    pass_sizes(N, K, n, &g1, &g2);
    if (g1 > gtop_max) gtop_max = g1;
    if (g2 > gpart) gpart = g2;
    int om[kMaxOrder];
    int no = other_modes(N, n, om);
    int64_t krow = 1;
    for (int q = 0; q < no - 1; ++q) krow *= K[om[q]];
    int64_t B = ((krow + 15) / 16) * ((K[om[no - 1]] + 15) / 16);
    if (B <= 8 && B > Bcore) Bcore = B;
  }
  int32_t groups = choose_core_groups(nnz, Bcore);
  int32_t rmax = 0;
  for (int n = 0; n < N; ++n) {
    L->ranges[n] = choose_ranges(nnz);
    if (L->ranges[n] > rmax) rmax = L->ranges[n];
  }
  // the range buffers leave room for a tuner to double the ranges (up to 16384)
  rmax = (int32_t)std::min<int64_t>(std::min<int64_t>(2 * (int64_t)rmax, std::max<int32_t>(rmax, 16384)), nnz);
  if (rmax < 1) rmax = 1;
  L->ranges_cap = rmax;
  // core mode, from the shape alone: cost ~ nnz / K_n (Kronecker work) plus an
  // upper bound min(I_n, nnz) of its nonempty slices (per-slice work)
  int cm = 0;
  double best = 0;
  for (int n = 0; n < N; ++n) {
    const double cost = (double)nnz / K[n] + (double)(dims[n] < nnz ? dims[n] : nnz);
    if (n == 0 || cost < best) {
      cm = n;
      best = cost;
    }
  }
  L->core_mode = cm;
  // row-writing core pass when its row buffer stays small next to the
  // nonzero streams (otherwise per-wave partials in LDS)
  {
    int om[kMaxOrder];
    const int no = other_modes(N, cm, om);
    int64_t krow = 1;
    for (int q = 0; q < no - 1; ++q) krow *= K[om[q]];
    const int64_t Bc = ((krow + 15) / 16) * ((K[om[no - 1]] + 15) / 16);
    const int64_t KC = 16 * ((K[cm] + 15) / 16);
    const int64_t rows = dims[cm] < nnz ? dims[cm] : nnz;
    const int64_t ybytes = rows * Bc * 256 * 4;
    const int64_t stream = nnz * 4 * N;
    int64_t w = nnz / 4096;
    const int64_t fine = std::min<int64_t>(nnz / 128, 2048);  // as choose_ranges
    if (w < fine) w = fine;
    if (w < 1) w = 1;
    if (w > 8192) w = 8192;
    L->core_rows = (Bc <= 8 && ybytes <= std::max<int64_t>(2 * stream, 16 << 20)) ? 1 : 0;
    L->ybuf_rows = L->core_rows ? rows : 0;
    L->core_w = L->core_rows ? (int32_t)w : 0;
    if (L->core_rows) {
      // a multiple of 8: the product's blocks are spread over the XCDs by chunk
      const int64_t chunks = ((rows + 2 * w + kCoreChunk - 1) / kCoreChunk + 7) / 8 * 8;
      groups = (int32_t)chunks;
      gpart = (size_t)(Bc * KC * 256);
    }
  }
  L->core_groups = groups;
  // stored slice rows: every mode's TTMcTC pass keeps Y_(n) (rows bounded by
  // min(I_n, nnz)) when every mode's tiles fit the pass kernels
  size_t ybuf_f = 0, ycarry_f = 0, gpart_f = (size_t)groups * gpart;
  if (L->core_rows) {
    const size_t row = gpart / (16 * ((K[L->core_mode] + 15) / 16));  // B_c * 256
    ybuf_f = (size_t)L->ybuf_rows * row;
    ycarry_f = (size_t)L->core_w * 2 * row;
  }
  L->yfuse = 1;
  {
    // every mode's pass stores its slice rows: the segment passes (at most 8
    // tiles of y_i, split slices leave partials) or the split-Kronecker pass
    // (whole slices), as long as the largest mode's rows (float32 layout)
    // stay within max(4 x one mode's nonzero stream, 16 GiB): a 1e6-row mode
    // with 1024-entry rows takes 4 GiB
    size_t yrows = 0, yrow = 0, ygp = 0, ybig = 0;
    for (int n = 0; n < N; ++n) {
      int om[kMaxOrder];
      const int no = other_modes(N, n, om);
      const int nr = yi_row_modes(no);
      int64_t krow = 1, kcol = 1;
      for (int q = 0; q < no; ++q) (q < nr ? krow : kcol) *= K[om[q]];
      const int64_t Bn = ((krow + 15) / 16) * ((kcol + 15) / 16);
      if (K[n] > 32) L->yfuse = 0;
      const bool seg = Bn <= 8 && no <= 3;
      const size_t rows = (size_t)(dims[n] < nnz ? dims[n] : nnz);
      const size_t chunks = seg ? (size_t)kYChunks : (size_t)ycore_chunks((int64_t)rows);
      yrows = std::max(yrows, rows);
      yrow = std::max(yrow, (size_t)Bn * 256);
      ybig = std::max(ybig, rows * (size_t)Bn * 256 * 4);
      ygp = std::max(ygp, chunks * Bn * 16 * ((K[n] + 15) / 16) * 256);
    }
    if (ybig > std::max<size_t>((size_t)4 * (size_t)nnz * 4 * N, (size_t)16 << 30)) L->yfuse = 0;
    if (L->yfuse) {
      ybuf_f = std::max(ybuf_f, yrows * yrow);
      ycarry_f = std::max(ycarry_f, (size_t)std::max<int32_t>(rmax, L->core_w) * 2 * yrow);
      gpart_f = std::max(gpart_f, ygp);
    }
  }
  L->ybuf_floats = ybuf_f;
  L->ycarry_floats = ycarry_f;
  L->gpart_floats = gpart_f;
  // the core reduction writes one float64 partial per 16 entries of G_(n)'s
  // padded tile layout: B_n 16 ceil(K_n/16) 256 / 16 for the mode reduced
  {
    size_t fp = 4096;
    for (int n = 0; n < N; ++n) {
      int om[kMaxOrder];
      const int no = other_modes(N, n, om);
      const int nr = yi_row_modes(no);
      int64_t krow = 1, kcol = 1;
      for (int q = 0; q < no; ++q) (q < nr ? krow : kcol) *= K[om[q]];
      const size_t Bn = (size_t)(((krow + 15) / 16) * ((kcol + 15) / 16));
      fp = std::max(fp, Bn * (size_t)((K[n] + 15) / 16) * 256);
    }
    L->fpart_doubles = fp;
  }
  int64_t IKsum = 0;
  for (int n = 0; n < N; ++n) IKsum += dims[n] * K[n];
  Carver r{nullptr, 0};
  for (int n = 0; n < N; ++n) r.take<float>(dims[n] * K[n]);  // row-relabelled factors
  for (int n = 0; n < N; ++n) r.take<uint16_t>(dims[n] * K[n]);  // their 16-bit copies
  r.take<float>(IKmax);                 // A
  r.take<float>(PK);                    // G
  r.take<float>(gpart_f);               // core partials
  r.take<double>(L->fpart_doubles);     // fpart
  r.take<float>(gtop_max);              // stage-two operand
  r.take<float>((size_t)rmax * 2 * 32); // carries
  r.take<int32_t>((size_t)rmax * 4);    // range metadata
  size_t ow = orth_ws_bytes(Imax, kMaxRank);
  r.take<char>(ow);
  r.take<int32_t>(64);                  // status
  r.take<double>(64);                   // scalars
  r.take<double>(kMaxSweeps + 1);       // f after each sweep
  r.take<double>(kMaxRank * kMaxRank + kGradParts + (size_t)kMaxSweeps * kMaxOrder);  // gradient monitor
  r.take<float>(ybuf_f);                // slice rows
  r.take<float>(ycarry_f);              // split-slice partials
  r.take<int32_t>((size_t)L->core_w * 4);  // core-pass range metadata
  size_t run = r.off;
  L->persistent = persistent;
  L->build_tmp = build;
  L->run_scratch = run;
  L->sort_tmp = stmp;
  L->total = persistent + (build > run ? build : run);
  return HOQRI_OK;
}

}  // namespace hoqri

using namespace hoqri;

extern "C" hoqri_status hoqri_plan_workspace_size(int32_t order, const int64_t* dims, const int32_t* ranks,
                                                  int64_t nnz, size_t* bytes) {
  if (!bytes) return HOQRI_ERR_ARG;
  Layout L;
  HOQRI_TRY(compute_layout(order, dims, ranks, nnz, &L));
  *bytes = L.total;
  return HOQRI_OK;
}

static hoqri_status build_plan(hoqri_plan* p, const int32_t* d_idx, const float* d_vals, hipStream_t s,
                               const Layout& L) {
  const int N = p->N;
  const int64_t nnz_in = p->nnz_in;
  int64_t Imax = 0;
  for (int n = 0; n < N; ++n)
    if (p->dims[n] > Imax) Imax = p->dims[n];

  // persistent region
  Carver c{(char*)p->ws, 0};
  const int64_t npad_in = (nnz_in + 15) / 16 * 16;
  for (int n = 0; n < N; ++n) {
    ModeData& md = p->md[n];
    md.rec = c.take<int32_t>(npad_in * N);
    int64_t rmax = p->dims[n] < nnz_in ? p->dims[n] : nnz_in;
    md.seg_row = c.take<int32_t>(rmax);
    md.seg_off = c.take<int32_t>(rmax + 1);
    md.lab = c.take<int32_t>(p->dims[n]);
    md.inv = c.take<int32_t>(p->dims[n]);
  }
  // build temporaries (after the persistent region)
  Carver b{(char*)p->ws + L.persistent, 0};
  uint64_t* keys = b.take<uint64_t>(nnz_in);
  uint64_t* keys_s = b.take<uint64_t>(nnz_in);
  int32_t* pos = b.take<int32_t>(nnz_in);
  int32_t* pos_s = b.take<int32_t>(nnz_in);
  int32_t* head = b.take<int32_t>(nnz_in);
  int32_t* uid = b.take<int32_t>(nnz_in);
  int32_t* cidx = b.take<int32_t>((size_t)N * nnz_in);
  float* cval = b.take<float>(nnz_in);
  double* vsq = b.take<double>(nnz_in);
  int32_t* modeidx = b.take<int32_t>(nnz_in);
  int32_t* flag_i = b.take<int32_t>(Imax);
  int32_t* scan_i = b.take<int32_t>(Imax);
  uint32_t* lkey = b.take<uint32_t>(Imax);
  uint32_t* lkey_s = b.take<uint32_t>(Imax);
  double* dpart = b.take<double>(65536);
  int64_t* small = b.take<int64_t>(64);
  void* stmp = b.take<char>(L.sort_tmp);
  int32_t* err = (int32_t*)(small + 32);

  // 1. keys + range check
  KeyArgs ka{};
  ka.idx = d_idx;
  ka.nnz = nnz_in;
  ka.N = N;
  uint64_t stride = 1;
  for (int m = N - 1; m >= 0; --m) {
    ka.dims[m] = p->dims[m];
    ka.stride[m] = stride;
    stride *= (uint64_t)p->dims[m];
  }
  HOQRI_HIP_TRY(hipMemsetAsync(err, 0, sizeof(int32_t), s));
  k_keys<<<grid_for(nnz_in), kThreads, 0, s>>>(ka, keys, pos, err);
  HOQRI_HIP_TRY(hipGetLastError());
  int32_t herr = 0;
  HOQRI_HIP_TRY(hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HOQRI_HIP_TRY(hipStreamSynchronize(s));
  if (herr) return HOQRI_ERR_INDEX;

  // 2. sort by linear key (stable), merge duplicates
  size_t tb = L.sort_tmp;
  int keybits = bits_for(stride);
  HOQRI_HIP_TRY(rocprim::radix_sort_pairs(stmp, tb, keys, keys_s, pos, pos_s, (size_t)nnz_in, 0, keybits, s));
  k_head_flags<<<grid_for(nnz_in), kThreads, 0, s>>>(keys_s, nnz_in, head);
  tb = L.sort_tmp;
  HOQRI_HIP_TRY(rocprim::exclusive_scan(stmp, tb, head, uid, 0, (size_t)nnz_in, rocprim::plus<int32_t>(), s));
  k_count<<<1, 1, 0, s>>>(head, uid, nnz_in, small);
  CoalesceArgs ca{d_idx, d_vals, keys_s, pos_s, head, uid, nnz_in, N, cidx, cval, vsq};
  k_coalesce<<<grid_for(nnz_in), kThreads, 0, s>>>(ca);
  int np = grid_for(nnz_in, kThreads, 1024);
  k_sum_partial<<<np, kThreads, 0, s>>>(vsq, small, dpart);
  k_sum_final<<<1, kThreads, 0, s>>>(dpart, np, (double*)(small + 1));
  k_max_partial<<<np, kThreads, 0, s>>>(vsq, small, dpart);
  k_max_final<<<1, kThreads, 0, s>>>(dpart, np, (double*)(small + 16));
  HOQRI_HIP_TRY(hipGetLastError());
  int64_t hsmall[17];
  HOQRI_HIP_TRY(hipMemcpyAsync(hsmall, small, 17 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HOQRI_HIP_TRY(hipStreamSynchronize(s));
  const int64_t nnz = hsmall[0];
  double nx2, mx2;
  std::memcpy(&nx2, &hsmall[1], sizeof(double));
  std::memcpy(&mx2, &hsmall[16], sizeof(double));
  p->nnz = nnz;
  p->normx2 = nx2;
  p->maxabs_x = std::sqrt(mx2);

  // 3. label every mode's indices by descending slice size (ties by index):
  //    factor rows are kept in label order inside the passes, so hot rows are
  //    contiguous in memory and empty slices take the last labels; the sorted
  //    streams below keep the original index order, so heavy and light slices
  //    stay mixed along each stream
  for (int n = 0; n < N; ++n) {
    ModeData& md = p->md[n];
    const int64_t In = p->dims[n];
    const int32_t* cn = cidx + (int64_t)n * nnz_in;
    k_fill_i32<<<grid_for(In), kThreads, 0, s>>>(flag_i, In, 0);
    k_degree<<<grid_for(nnz), kThreads, 0, s>>>(cn, nnz, flag_i);
    k_degree_keys<<<grid_for(In), kThreads, 0, s>>>(flag_i, In, lkey, scan_i);
    tb = L.sort_tmp;
    HOQRI_HIP_TRY(rocprim::radix_sort_pairs(stmp, tb, lkey, lkey_s, scan_i, md.inv, (size_t)In, 0, 31, s));
    k_invert<<<grid_for(In), kThreads, 0, s>>>(md.inv, In, md.lab);
    HOQRI_HIP_TRY(hipGetLastError());
  }

  // 4. order the merged nonzeros by their label coordinates (C order): inside
  //    every slice of every mode the nonzeros then come hot rows first, grouped
  //    by row, which is what the gathers of the segment passes want
  int32_t* lperm = reinterpret_cast<int32_t*>(vsq);  // the squares are summed already: reuse their storage
  {
    LabKeyArgs la{};
    la.cidx = cidx;
    la.stride = nnz_in;
    la.nnz = nnz;
    la.N = N;
    uint64_t st = 1;
    for (int m = N - 1; m >= 0; --m) {
      la.lab[m] = p->md[m].lab;
      la.lstride[m] = st;
      st *= (uint64_t)p->dims[m];
    }
    k_label_keys<<<grid_for(nnz), kThreads, 0, s>>>(la, keys, pos);
    tb = L.sort_tmp;
    HOQRI_HIP_TRY(rocprim::radix_sort_pairs(stmp, tb, keys, keys_s, pos, lperm, (size_t)nnz, 0, bits_for(st), s));
  }

  // 5. per mode: stable sort of that order by the original i_n (slice order
  //    stays the original index order), sorted copy (labels), slice table
  uint32_t* k32 = reinterpret_cast<uint32_t*>(keys);
  uint32_t* k32s = reinterpret_cast<uint32_t*>(keys_s);
  for (int n = 0; n < N; ++n) {
    ModeData& md = p->md[n];
    k_mode_keys_perm<<<grid_for(nnz), kThreads, 0, s>>>(cidx + (int64_t)n * nnz_in, lperm, nnz, k32, pos);
    tb = L.sort_tmp;
    HOQRI_HIP_TRY(rocprim::radix_sort_pairs(stmp, tb, k32, k32s, pos, pos_s, (size_t)nnz, 0,
                                            bits_for((uint64_t)p->dims[n]), s));
    const int32_t* perm = pos_s;
    GatherArgs ga{};
    ga.cidx = cidx;
    ga.cval = cval;
    ga.perm = perm;
    for (int m = 0; m < N; ++m) ga.lab[m] = p->md[m].lab;
    ga.stride = nnz_in;
    ga.nnz = nnz;
    ga.N = N;
    ga.mode = n;
    for (int m = 0; m < N; ++m) ga.K[m] = p->K[m];
    ga.rec = md.rec;
    ga.modeidx = modeidx;
    k_gather_mode<<<grid_for(nnz + 16), kThreads, 0, s>>>(ga);
    k_head_flags<<<grid_for(nnz), kThreads, 0, s>>>(modeidx, nnz, head);
    tb = L.sort_tmp;
    HOQRI_HIP_TRY(rocprim::exclusive_scan(stmp, tb, head, uid, 0, (size_t)nnz, rocprim::plus<int32_t>(), s));
    k_segments<<<grid_for(nnz), kThreads, 0, s>>>(modeidx, head, uid, nnz, md.lab, md.seg_row, md.seg_off,
                                                    small + 2 + n);
    HOQRI_HIP_TRY(hipGetLastError());
  }
  int64_t Rh[kMaxOrder];
  HOQRI_HIP_TRY(hipMemcpyAsync(Rh, small + 2, N * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HOQRI_HIP_TRY(hipStreamSynchronize(s));
  for (int n = 0; n < N; ++n) {
    p->md[n].R = Rh[n];
    p->md[n].E = p->dims[n] - Rh[n];
    p->md[n].empty_row = p->md[n].inv + Rh[n];  // original indices of the empty slices
    p->md[n].ranges = L.ranges[n];
    p->md[n].ranges0 = L.ranges[n];
    p->md[n].rpw = 0;
  }
  p->ranges_cap = L.ranges_cap;
  p->core_mode = L.core_mode;
  p->core_groups = L.core_groups;
  p->core_rows = L.core_rows;
  p->ybuf_rows = L.ybuf_rows;
  p->core_w = L.core_w;
  p->yfuse = L.yfuse;
  return HOQRI_OK;
}

static void carve_scratch(hoqri_plan* p, const Layout& L) {
  int64_t IKmax = 0, PK = 1, Imax = 0;
  for (int n = 0; n < p->N; ++n) {
    if (p->dims[n] * p->K[n] > IKmax) IKmax = p->dims[n] * p->K[n];
    if (p->dims[n] > Imax) Imax = p->dims[n];
    PK *= p->K[n];
  }
  size_t gtop_max = 0;
  for (int n = 0; n < p->N; ++n) {
    size_t g1, g2;
    pass_sizes(p->N, p->K, n, &g1, &g2);
    if (g1 > gtop_max) gtop_max = g1;
  }
  const int32_t rmax = L.ranges_cap;
  Carver r{(char*)p->ws + L.persistent, 0};
  for (int n = 0; n < p->N; ++n) p->sc.Up[n] = r.take<float>(p->dims[n] * p->K[n]);
  for (int n = 0; n < p->N; ++n) p->sc.Uh[n] = r.take<uint16_t>(p->dims[n] * p->K[n]);
  p->sc.A = r.take<float>(IKmax);
  p->sc.G = r.take<float>(PK);
  p->sc.gpart = r.take<float>(L.gpart_floats);
  p->sc.fpart = r.take<double>(L.fpart_doubles);
  p->sc.gtop = r.take<float>(gtop_max);
  p->sc.carry = r.take<float>((size_t)rmax * 2 * 32);
  p->sc.meta = r.take<int32_t>((size_t)rmax * 4);
  size_t ow = orth_ws_bytes(Imax, kMaxRank);
  p->sc.orth_ws = (double*)r.take<char>(ow);
  p->sc.orth_ws_bytes = ow;
  p->sc.status = r.take<int32_t>(64);
  p->sc.f_dev = r.take<double>(64);
  p->sc.fsweep = r.take<double>(kMaxSweeps + 1);
  p->sc.gscr = r.take<double>(kMaxRank * kMaxRank + kGradParts + (size_t)kMaxSweeps * kMaxOrder);
  p->sc.ybuf = r.take<float>(L.ybuf_floats);
  p->sc.ycarry = r.take<float>(L.ycarry_floats);
  p->sc.ymeta = r.take<int32_t>((size_t)L.core_w * 4);
}

extern "C" hoqri_status hoqri_plan_create(hoqri_plan** plan, int32_t order, const int64_t* dims,
                                          const int32_t* ranks, int64_t nnz, const int32_t* d_idx,
                                          const float* d_vals, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (!plan || !dims || !ranks || !d_idx || !d_vals || !d_ws) return HOQRI_ERR_ARG;
  *plan = nullptr;
  Layout L;
  HOQRI_TRY(compute_layout(order, dims, ranks, nnz, &L));
  if (ws_bytes < L.total) return HOQRI_ERR_NOMEM;
  hoqri_plan* p = new (std::nothrow) hoqri_plan();
  if (!p) return HOQRI_ERR_NOMEM;
  p->N = order;
  for (int n = 0; n < order; ++n) {
    p->dims[n] = dims[n];
    p->K[n] = ranks[n];
  }
  p->nnz_in = nnz;
  p->ws = d_ws;
  p->ws_bytes = ws_bytes;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return HOQRI_ERR_HIP;
  }
  hoqri_status st = build_plan(p, d_idx, d_vals, stream, L);
  if (st != HOQRI_OK) {
    delete p;
    return st;
  }
  carve_scratch(p, L);
  *plan = p;
  return HOQRI_OK;
}

extern "C" hoqri_status hoqri_plan_info(const hoqri_plan* p, int64_t* nnz_coalesced, double* norm_x2,
                                        int64_t* R) {
  if (!p) return HOQRI_ERR_ARG;
  if (nnz_coalesced) *nnz_coalesced = p->nnz;
  if (norm_x2) *norm_x2 = p->normx2;
  if (R)
    for (int n = 0; n < p->N; ++n) R[n] = p->md[n].R;
  return HOQRI_OK;
}

extern "C" void hoqri_plan_destroy(hoqri_plan* p) {
  if (!p) return;
  timing_release(p);
  delete p;
}

extern "C" const char* hoqri_status_string(hoqri_status s) {
  switch (s) {
    case HOQRI_OK: return "ok";
    case HOQRI_ERR_ARG: return "invalid argument";
    case HOQRI_ERR_INDEX: return "coordinate out of range";
    case HOQRI_ERR_RANK: return "invalid rank";
    case HOQRI_ERR_BREAKDOWN: return "rank-deficient update (Cholesky breakdown)";
    case HOQRI_ERR_NOMEM: return "workspace too small";
    case HOQRI_ERR_HIP: return "HIP runtime error";
    case HOQRI_ERR_UNSUPPORTED: return "shape not supported";
  }
  return "unknown status";
}
