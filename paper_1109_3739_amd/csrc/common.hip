// Error reporting, scratch allocation and small fill kernels of libspx.
#include "common.h"

#include <cstdlib>
#include <mutex>

namespace spx {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

// Allocation fault injection for tests of the error paths.  SPX_FAULT set
// to "alloc:N" makes the N-th device allocation request of the library
// fail (1-based, counted from the moment the variable took its current
// value); "alloc:N+" makes that request and every later one fail.  Unset or
// any other value: no faults.  Both the plans' scratch and the one-shot
// entry points' outputs count.
static bool fault_injected() {
  static std::mutex mu;
  static std::string spec;
  static long long count = 0;
  const char* env = getenv("SPX_FAULT");
  const std::string cur = env ? env : "";
  std::lock_guard<std::mutex> lock(mu);
  if (cur != spec) {
    spec = cur;
    count = 0;
  }
  if (spec.compare(0, 6, "alloc:") != 0) return false;
  char* end = nullptr;
  const long long n = strtoll(spec.c_str() + 6, &end, 10);
  if (end == spec.c_str() + 6 || n < 1) return false;
  const bool and_later = *end == '+';
  ++count;
  return and_later ? count >= n : count == n;
}

Scratch::Scratch(const spx_ctx* ctx) : stream_(stream_of(ctx)) {
  if (ctx)
    ctx_ = *ctx;
  else
    ctx_ = spx_ctx{};
}

Scratch::~Scratch() { release_all(); }

int Scratch::raw_alloc(size_t bytes, void** out) {
  void* p = nullptr;
  if (fault_injected()) return fail(SPX_ENOMEM, "allocation failed (injected by SPX_FAULT)");
  if (ctx_.alloc) {
    p = ctx_.alloc(bytes, ctx_.user);
    if (!p) return fail(SPX_ENOMEM, "allocation callback failed for " + std::to_string(bytes) + " bytes");
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(SPX_ENOMEM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
    }
  }
  bufs_.push_back(p);
  *out = p;
  return SPX_OK;
}

int Scratch::get(size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) bytes = 16;
  bytes = (bytes + 255) & ~(size_t)255;
  if (bytes > kArenaSmall) return raw_alloc(bytes, out);
  // small buffers are cut from shared blocks (one allocation call per block)
  if (arena_used_ + bytes > arena_size_) {
    void* blk = nullptr;
    const int rc = raw_alloc(kArenaBlock, &blk);
    if (rc != SPX_OK) return rc;
    arena_ = static_cast<char*>(blk);
    arena_used_ = 0;
    arena_size_ = kArenaBlock;
  }
  *out = arena_ + arena_used_;
  arena_used_ += bytes;
  return SPX_OK;
}

void Scratch::release_all() {
  for (void* p : bufs_) {
    if (ctx_.alloc) {
      if (ctx_.free) ctx_.free(p, ctx_.user);
    } else {
      (void)hipFree(p);
    }
  }
  bufs_.clear();
  arena_ = nullptr;
  arena_used_ = arena_size_ = 0;
}

OutAlloc::~OutAlloc() {
  for (void* p : got_) {
    if (ctx_ && ctx_->alloc) {
      if (ctx_->free) ctx_->free(p, ctx_->user);
    } else {
      (void)hipFree(p);
    }
  }
}

int OutAlloc::get(size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) bytes = 16;
  void* p = nullptr;
  if (fault_injected()) return fail(SPX_ENOMEM, "allocation of an output buffer failed (injected by SPX_FAULT)");
  if (ctx_ && ctx_->alloc) {
    p = ctx_->alloc(bytes, ctx_->user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (!p) return fail(SPX_ENOMEM, "allocation of an output buffer failed (" + std::to_string(bytes) + " bytes)");
  got_.push_back(p);
  *out = p;
  return SPX_OK;
}

int device_cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
  return cus;
}

int Scratch::get_many(std::initializer_list<Part> parts) {
  size_t total = 0;
  for (const Part& q : parts) total += (q.bytes + 255) & ~(size_t)255;
  void* base = nullptr;
  SPX_TRY(get(total, &base));
  char* c = static_cast<char*>(base);
  for (const Part& q : parts) {
    *q.out = c;
    c += (q.bytes + 255) & ~(size_t)255;
  }
  return SPX_OK;
}

struct WordList {
  const void* p[kMaxReadRanges];
  int32_t bytes[kMaxReadRanges];
  int32_t count[kMaxReadRanges];
  int32_t n;
};

__global__ void k_read_words(WordList w, int64_t* dst) {
  const int i = threadIdx.x;
  int base = 0;
  for (int r = 0; r < w.n; ++r) {
    if (i < base + w.count[r]) {
      const int k = i - base;
      dst[i] = w.bytes[r] == 4 ? (int64_t) static_cast<const uint32_t*>(w.p[r])[k]
                               : static_cast<const int64_t*>(w.p[r])[k];
      return;
    }
    base += w.count[r];
  }
}

int read_device_words(hipStream_t stream, const DevWord* words, int nwords, int64_t* out) {
  constexpr int kMaxDev = 64;
  // per thread and device, allocated on first use and kept for the process
  static thread_local int64_t* host[kMaxDev] = {};
  static thread_local int64_t* mapped[kMaxDev] = {};  // the same words' device address
  if (nwords > kMaxReadRanges) return fail(SPX_EINVAL, "read_device_words: too many runs");
  WordList w{};
  int total = 0;
  for (int r = 0; r < nwords; ++r) {
    const DevWord& d = words[r];
    w.p[w.n] = d.p;
    w.bytes[w.n] = d.bytes;
    w.count[w.n] = d.count;
    total += d.count;
    ++w.n;
  }
  if (total > kMaxReadWords) return fail(SPX_EINVAL, "read_device_words: too many words");
  int dev = 0;
  SPX_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDev) return fail(SPX_EDEVICE, "device id out of the supported range");
  if (!host[dev]) {
    void* h = nullptr;
    SPX_HIP(hipHostMalloc(&h, kMaxReadWords * sizeof(int64_t), hipHostMallocCoherent | hipHostMallocMapped));
    void* d = nullptr;
    SPX_HIP(hipHostGetDevicePointer(&d, h, 0));
    host[dev] = static_cast<int64_t*>(h);
    mapped[dev] = static_cast<int64_t*>(d);
  }
  k_read_words<<<1, kMaxReadWords, 0, stream>>>(w, mapped[dev]);
  SPX_HIP(hipGetLastError());
  SPX_HIP(hipStreamSynchronize(stream));
  for (int i = 0; i < total; ++i) out[i] = host[dev][i];
  return SPX_OK;
}

SideStream::~SideStream() {
  if (join) (void)hipEventDestroy(join);
  if (fork) (void)hipEventDestroy(fork);
  if (s) (void)hipStreamDestroy(s);
}

int side_fork(hipStream_t st, SideStream** out) {
  constexpr int kMaxDev = 64;
  static thread_local SideStream per_dev[kMaxDev];
  int dev = 0;
  SPX_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDev) return fail(SPX_EDEVICE, "device id out of the supported range");
  SideStream& ss = per_dev[dev];
  if (!ss.s) {
    if (!ss.fork) SPX_HIP(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming));
    if (!ss.join) SPX_HIP(hipEventCreateWithFlags(&ss.join, hipEventDisableTiming));
    SPX_HIP(hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking));
  }
  SPX_HIP(hipEventRecord(ss.fork, st));
  SPX_HIP(hipStreamWaitEvent(ss.s, ss.fork, 0));
  *out = &ss;
  return SPX_OK;
}

int side_join(SideStream* ss, hipStream_t st) {
  SPX_HIP(hipEventRecord(ss->join, ss->s));
  SPX_HIP(hipStreamWaitEvent(st, ss->join, 0));
  return SPX_OK;
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

int fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t stream) {
  if (n <= 0) return SPX_OK;
  k_fill<int64_t><<<grid_for(n, 256, 4096), 256, 0, stream>>>(p, n, v);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

struct ZeroList {
  int64_t* p[kMaxZeroRuns];
  int64_t end[kMaxZeroRuns];  // inclusive prefix of the runs' lengths
  int n;
};

__global__ void k_zero_words(ZeroList z) {
  const int64_t total = z.end[z.n - 1];
  int r = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    while (i >= z.end[r]) ++r;  // i only grows, so r does too
    z.p[r][i - (r ? z.end[r - 1] : 0)] = 0;
  }
}

int zero_words(hipStream_t stream, std::initializer_list<ZeroRun> runs) {
  if (runs.size() > (size_t)kMaxZeroRuns) return fail(SPX_EINVAL, "zero_words: too many runs");
  ZeroList z{};
  int64_t total = 0;
  for (const ZeroRun& r : runs) {
    if (r.words <= 0) continue;
    total += r.words;
    z.p[z.n] = static_cast<int64_t*>(r.p);
    z.end[z.n] = total;
    ++z.n;
  }
  if (total == 0) return SPX_OK;
  k_zero_words<<<grid_for(total, 256, 4096), 256, 0, stream>>>(z);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

int fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream) {
  if (n <= 0) return SPX_OK;
  k_fill<uint32_t><<<grid_for(n, 256, 4096), 256, 0, stream>>>(p, n, v);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

}  // namespace spx

extern "C" const char* spx_last_error(void) { return spx::g_last_error.c_str(); }

extern "C" const char* spx_version(void) { return "spx 0.1 (gfx950)"; }
