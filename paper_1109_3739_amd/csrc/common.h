// Internal helpers shared by the HIP sources of libspx: error handling,
// scratch allocation, wave-level primitives and semiring arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <initializer_list>
#include <string>
#include <vector>

#include "spx.h"

namespace spx {

constexpr int kWave = 64;

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);

struct Status {
  int code = SPX_OK;
  bool ok() const { return code == SPX_OK; }
};

#define SPX_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::spx::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
      return SPX_EDEVICE;                                                          \
    }                                                                              \
  } while (0)

#define SPX_TRY(expr)          \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != SPX_OK) return rc_; \
  } while (0)

inline int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

// ---------------------------------------------------------------- scratch
// Device buffers taken from the context's allocator (or hipMalloc) and
// released when the owning object is destroyed.
// Output buffers of the one-shot entry points: from ctx->alloc (hipMalloc
// without one).  Unless keep() is called, the destructor releases them, so an
// entry point that fails half way leaves nothing behind.
class OutAlloc {
 public:
  explicit OutAlloc(const spx_ctx* ctx) : ctx_(ctx) {}
  ~OutAlloc();
  int get(size_t bytes, void** out);
  void keep() { got_.clear(); }

 private:
  const spx_ctx* ctx_;
  std::vector<void*> got_;
};

class Scratch {
 public:
  explicit Scratch(const spx_ctx* ctx);
  ~Scratch();
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  // Returns SPX_OK and sets *out (256-byte aligned), or SPX_ENOMEM.
  int get(size_t bytes, void** out);
  template <typename T>
  int get_n(size_t count, T** out) {
    void* p = nullptr;
    int rc = get(count * sizeof(T) + 16, &p);
    *out = static_cast<T*>(p);
    return rc;
  }
  // One allocation carved into several arrays (each 256-byte aligned), so
  // that a plan's arrays of one phase cost a single allocator call.
  struct Part {
    void** out;
    size_t bytes;
  };
  template <typename T>
  static Part part(T** out, int64_t count) {
    return {reinterpret_cast<void**>(out), (size_t)(count > 0 ? count : 0) * sizeof(T) + 16};
  }
  int get_many(std::initializer_list<Part> parts);
  void release_all();
  hipStream_t stream() const { return stream_; }

 private:
  static constexpr size_t kArenaSmall = 256 << 10;  // requests up to this size share blocks
  static constexpr size_t kArenaBlock = 2 << 20;
  int raw_alloc(size_t bytes, void** out);
  spx_ctx ctx_;
  hipStream_t stream_;
  std::vector<void*> bufs_;
  char* arena_ = nullptr;
  size_t arena_used_ = 0, arena_size_ = 0;
};

inline hipStream_t stream_of(const spx_ctx* ctx) { return ctx ? (hipStream_t)ctx->stream : (hipStream_t)0; }

int device_cu_count();

// Kernel fills (used instead of hipMemsetAsync so that work enqueued by the
// library can be captured into a HIP graph).
int fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t stream);
int fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream);
// Zeroes up to kMaxZeroRuns runs of 8-byte words with one launch.
constexpr int kMaxZeroRuns = 8;
struct ZeroRun {
  void* p;
  int64_t words;
};
int zero_words(hipStream_t stream, std::initializer_list<ZeroRun> runs);

// Reads device scalars of 4 or 8 bytes (4-byte ones zero-extended), or
// runs of `count` of them, at most kMaxReadRanges runs and kMaxReadWords
// words in all, with one kernel that writes them to this thread's pinned
// host words, and waits for the stream: one launch instead of a copy per
// scalar.  out[] receives the words in the order given.
constexpr int kMaxReadRanges = 12;
constexpr int kMaxReadWords = 64;
struct DevWord {
  const void* p;
  int bytes;
  int count = 1;
};
int read_device_words(hipStream_t stream, const DevWord* words, int nwords, int64_t* out);
inline int read_device_words(hipStream_t stream, std::initializer_list<DevWord> words, int64_t* out) {
  return read_device_words(stream, words.begin(), (int)words.size(), out);
}

// A second stream of the calling host thread on the current device (default
// priority), for a launch that may run beside the work of the caller's
// stream: side_fork makes it wait for what `st` holds so far, side_join
// makes `st` wait for what was enqueued on it since.  Created on first use
// and destroyed when the thread ends.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  ~SideStream();
};
int side_fork(hipStream_t st, SideStream** out);
int side_join(SideStream* ss, hipStream_t st);

// Joins a forked side stream back into `st` when it goes out of scope, so
// that an early error return still leaves no side work unordered with the
// caller's stream; join() does it at a chosen point and reports errors.
struct SideJoin {
  SideStream* ss = nullptr;
  hipStream_t st = nullptr;
  int join() {
    SideStream* s = ss;
    ss = nullptr;
    return s ? side_join(s, st) : SPX_OK;
  }
  ~SideJoin() {
    if (ss) (void)side_join(ss, st);
  }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t next_pow2(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}
inline unsigned grid_for(int64_t items, int per_block, int64_t cap = 1 << 30) {
  int64_t g = ceil_div(items, per_block);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// Reads element i of a column-pointer array of either index type.
__device__ __forceinline__ int64_t load_ptr(const void* p, int32_t ptr_t, int64_t i) {
  return ptr_t == SPX_PTR_I64 ? reinterpret_cast<const int64_t*>(p)[i]
                              : (int64_t) reinterpret_cast<const int32_t*>(p)[i];
}
__device__ __forceinline__ void store_ptr(void* p, int32_t ptr_t, int64_t i, int64_t v) {
  if (ptr_t == SPX_PTR_I64)
    reinterpret_cast<int64_t*>(p)[i] = v;
  else
    reinterpret_cast<int32_t*>(p)[i] = (int32_t)v;
}

// ---------------------------------------------------------------- waves
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T t = __shfl_xor(v, o);
    v = t > v ? t : v;
  }
  return v;
}

// Value moved by the DPP control CTRL with rows outside ROW_MASK (and lanes
// without a source) reading 0.  32- or 64-bit integers.
template <int CTRL, int ROW_MASK, typename T>
__device__ __forceinline__ T dpp_move(T v) {
  if constexpr (sizeof(T) == 4) {
    return (T)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
  } else {
    static_assert(sizeof(T) == 8, "32- or 64-bit integers");
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xF, false);
    return (T)(((uint64_t)hi << 32) | lo);
  }
}

// Inclusive prefix sum over the 64 lanes (all active): shifts by 1, 2, 4, 8
// inside each 16-lane row, then the last lane of rows 0 and 2 is added into
// rows 1 and 3, and lane 31 into rows 2 and 3.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  static_assert(__is_integral(T), "integer scans");
  v += dpp_move<0x111, 0xF>(v);  // row_shr:1
  v += dpp_move<0x112, 0xF>(v);  // row_shr:2
  v += dpp_move<0x114, 0xF>(v);  // row_shr:4
  v += dpp_move<0x118, 0xF>(v);  // row_shr:8
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31
  return v;
}

// Value held by lane (lane ^ j), j a power of two below 64, without the LDS
// permute path: j = 1, 2 are quad permutes (DPP); j = 4 a half-row mirror
// (lane -> lane ^ 7) followed by a quad reversal (^ 3); j = 8 a rotation of
// each 16-lane row by 8; j = 16 and 32 the gfx950 lane swaps, which return
// every row pair (half pair) as [even, even] and [odd, odd], so a lane takes
// the copy of the other row.  The source lane must be active; j must be a
// constant after unrolling (the switch folds away).
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t v, int j) {
  switch (j) {
    case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    case 4: {
      const int m = __builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);
      return (uint32_t)__builtin_amdgcn_update_dpp(0, m, 0x1B, 0xF, 0xF, false);
    }
    case 8: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);
    case 16: {
      const auto s = __builtin_amdgcn_permlane16_swap(v, v, false, false);
      return (__lane_id() & 16) ? s[0] : s[1];
    }
    default: {
      const auto s = __builtin_amdgcn_permlane32_swap(v, v, false, false);
      return (__lane_id() & 32) ? s[0] : s[1];
    }
  }
}
__device__ __forceinline__ uint64_t xor_lane(uint64_t v, int j) {
  const uint32_t lo = xor_lane_u32((uint32_t)v, j), hi = xor_lane_u32((uint32_t)(v >> 32), j);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int j) { return xor_lane_u32(v, j); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Claims one slot of a global counter for every lane with `pred` set, with a
// single atomic per wave (lanes not taking part must still be active or have
// left the loop together).  Returns the lane's slot (undefined without pred).
__device__ __forceinline__ unsigned long long wave_claim(unsigned long long* ctr, bool pred) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return 0;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader);
  return base + (unsigned long long)__popcll(mask & lanemask_lt());
}

// Exclusive block-wide prefix sum of one value per thread; `red` is LDS
// scratch of at least blockDim.x/64 + 1 entries.  Returns the exclusive
// prefix and writes the block total to *total (all threads).
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* red, T* total) {
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  T incl = wave_incl_scan(v);
  if (lane == kWave - 1) red[wid] = incl;
  __syncthreads();
  if (wid == 0) {
    T w = lane < nw ? red[lane] : T(0);
    T wi = wave_incl_scan(w);
    if (lane < nw) red[lane] = wi - w;
    if (lane == nw - 1) red[nw] = wi;
  }
  __syncthreads();
  T res = red[wid] + incl - v;
  *total = red[nw];
  __syncthreads();
  return res;
}

// The same with one barrier: every wave adds up the totals of the waves
// before it.  `red` must not be written again before the workgroup's next
// barrier (callers place one between two scans).
template <typename T>
__device__ __forceinline__ T block_excl_scan1(T v, T* red, T* total) {
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const T incl = wave_incl_scan(v);
  if (lane == kWave - 1) red[wid] = incl;
  __syncthreads();
  T before = T(0), all = T(0);
  for (int k = 0; k < nw; ++k) {
    const T x = red[k];
    if (k < wid) before += x;
    all += x;
  }
  *total = all;
  return before + incl - v;
}

// ---------------------------------------------------------------- semirings
// mul: product of A(i,k) and B(k,j); add: combine into an accumulator;
// lds_acc: atomic combine into LDS; ident: value of an untouched slot.
// ident is the exact neutral element of add, so that a slot started from it
// and combined with the products ends where a fold started from the first
// product ends (Algorithm 1 starts each accumulator from its first product).
// For floating-point (+,x) that is -0.0, not +0.0: -0 + x = x for every x,
// including x = -0, whereas +0 + (-0) = +0 would lose the sign of a sum of
// negative zeros.
template <int SR, typename T>
struct Semiring;

template <typename T>
struct Semiring<SPX_PLUS_TIMES, T> {
  static constexpr bool kUsesA = true, kUsesB = true;
  __device__ static T mul(T a, T b) { return a * b; }
  __device__ static T add(T acc, T x) { return acc + x; }
  __device__ static T ident() { return -T(0); }
  __device__ static void lds_acc(T* p, T x) {
    __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};
template <>
struct Semiring<SPX_PLUS_TIMES, int64_t> {
  static constexpr bool kUsesA = true, kUsesB = true;
  __device__ static int64_t mul(int64_t a, int64_t b) { return (int64_t)((uint64_t)a * (uint64_t)b); }
  __device__ static int64_t add(int64_t acc, int64_t x) { return (int64_t)((uint64_t)acc + (uint64_t)x); }
  __device__ static int64_t ident() { return 0; }
  __device__ static void lds_acc(int64_t* p, int64_t x) {
    __hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(p), (unsigned long long)x, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

template <typename T>
__device__ __forceinline__ T pos_inf();
template <>
__device__ __forceinline__ float pos_inf<float>() { return __builtin_huge_valf(); }
template <>
__device__ __forceinline__ double pos_inf<double>() { return __builtin_huge_val(); }
template <>
__device__ __forceinline__ int64_t pos_inf<int64_t>() { return INT64_MAX; }

template <typename T>
struct MinAcc {
  __device__ static T add(T acc, T x) { return x < acc ? x : acc; }
  __device__ static T ident() { return pos_inf<T>(); }
  __device__ static void lds_acc(T* p, T x) {
    __hip_atomic_fetch_min(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

template <typename T>
struct Semiring<SPX_MIN_PLUS, T> : MinAcc<T> {
  static constexpr bool kUsesA = true, kUsesB = true;
  __device__ static T mul(T a, T b) { return a + b; }
};
template <>
struct Semiring<SPX_MIN_PLUS, int64_t> : MinAcc<int64_t> {
  static constexpr bool kUsesA = true, kUsesB = true;
  __device__ static int64_t mul(int64_t a, int64_t b) { return (int64_t)((uint64_t)a + (uint64_t)b); }
};
template <typename T>
struct Semiring<SPX_SELECT2ND, T> : MinAcc<T> {
  static constexpr bool kUsesA = false, kUsesB = true;
  __device__ static T mul(T, T b) { return b; }
};
template <typename T>
struct Semiring<SPX_SELECT1ST, T> : MinAcc<T> {
  static constexpr bool kUsesA = true, kUsesB = false;
  __device__ static T mul(T a, T) { return a; }
};

// Pattern-only marker type for OR_AND.
struct NoVal {};

}  // namespace spx
