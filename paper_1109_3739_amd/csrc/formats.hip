// CSC <-> DCSC conversion and canonical-form checks (Section 3.2: DCSC drops
// the repeated column pointers of empty columns and lists the ids of the
// nonempty columns in JC; IR and NUM are the same arrays as in CSC).
#include <algorithm>
#include <mutex>
#include <string>

#include "common.h"
#include "operand.h"
#include "plan.h"
#include "scan.h"

namespace spx {

struct NonemptyCol {
  Operand A;
  __device__ int64_t operator()(int64_t j) const { return slot_begin(A, j + 1) > slot_begin(A, j) ? 1 : 0; }
};

// Nonempty column j becomes entry zoff[j] of jc / cp.  Entries at or beyond
// the output's capacity `cap` (its nzc) are not written; nzc_out (if given)
// receives the number of nonempty columns.
__global__ void k_to_dcsc(Operand A, const int64_t* zoff, int32_t* jc, void* cp, int32_t ptr_t, int64_t cap,
                          int64_t* nzc_out) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < A.n; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = slot_begin(A, j), e = slot_begin(A, j + 1);
    if (e > s && zoff[j] < cap) {
      jc[zoff[j]] = (int32_t)j;
      store_ptr(cp, ptr_t, zoff[j], s);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (zoff[A.n] <= cap) store_ptr(cp, ptr_t, zoff[A.n], A.nnz);
    if (nzc_out) *nzc_out = zoff[A.n];
  }
}

// cp[j] = start of column j = DCSC pointer of the first stored column >= j.
__global__ void k_to_csc(Operand A, void* cp, int32_t ptr_t) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= A.n; j += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = A.nzc;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)A.jc[mid] < j)
        lo = mid + 1;
      else
        hi = mid;
    }
    store_ptr(cp, ptr_t, j, slot_begin(A, lo));
  }
}

// Canonical form: cp[0] = 0, cp[last] = nnz, cp nondecreasing, rows in
// [0, m) strictly increasing per stored column, DCSC jc strictly increasing
// in [0, n) with nonempty columns only.
__global__ void k_check(Operand A, int64_t nslots, unsigned* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nslots; t += stride) {
    const int64_t s = slot_begin(A, t), e = slot_begin(A, t + 1);
    if (e < s || s < 0 || e > A.nnz) {
      atomicOr(bad, 1u);
      continue;
    }
    if (A.fmt == SPX_DCSC) {
      const int32_t c = A.jc[t];
      if (c < 0 || c >= A.n || (t > 0 && A.jc[t - 1] >= c) || e == s) atomicOr(bad, 2u);
    }
    int32_t prev = -1;
    for (int64_t i = s; i < e; ++i) {
      const int32_t r = A.ir[i];
      if (r <= prev || r >= A.m) {
        atomicOr(bad, 4u);
        break;
      }
      prev = r;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (slot_begin(A, 0) != 0 || slot_begin(A, nslots) != A.nnz) atomicOr(bad, 8u);
  }
}

}  // namespace spx

using namespace spx;

extern "C" int spx_count_nonempty(const spx_ctx* ctx, const spx_mat* A, int64_t* nzc) {
  SPX_TRY(check_mat(A, "A"));
  if (!nzc) return fail(SPX_EINVAL, "nzc is NULL");
  if (A->fmt == SPX_DCSC) {
    *nzc = A->nzc;
    return SPX_OK;
  }
  hipStream_t st = stream_of(ctx);
  Scratch scr(ctx);
  int64_t* zoff = nullptr;
  SPX_TRY(scr.get_n(A->n + 1, &zoff));
  SPX_TRY(exclusive_scan(NonemptyCol{make_operand(A)}, A->n, zoff, scr, st));
  SPX_HIP(hipMemcpyAsync(nzc, zoff + A->n, 8, hipMemcpyDeviceToHost, st));
  SPX_HIP(hipStreamSynchronize(st));
  return SPX_OK;
}

extern "C" int spx_csc_to_dcsc(const spx_ctx* ctx, const spx_mat* A, spx_mat* out) {
  SPX_TRY(check_mat(A, "A"));
  if (A->fmt != SPX_CSC) return fail(SPX_EINVAL, "A must be CSC");
  if (!out || !out->cp || (out->nzc > 0 && !out->jc)) return fail(SPX_EINVAL, "out buffers missing");
  if (out->ptr_t != SPX_PTR_I32 && out->ptr_t != SPX_PTR_I64) return fail(SPX_EINVAL, "bad out ptr_t");
  if (out->ptr_t == SPX_PTR_I32 && A->nnz >= (1ll << 31)) return fail(SPX_EOVERFLOW, "nnz needs I64 pointers");
  hipStream_t st = stream_of(ctx);
  Scratch scr(ctx);
  int64_t* zoff = nullptr;
  SPX_TRY(scr.get_n(A->n + 1, &zoff));
  const Operand a = make_operand(A);
  SPX_TRY(exclusive_scan(NonemptyCol{a}, A->n, zoff, scr, st));
  k_to_dcsc<<<grid_for(std::max<int64_t>(A->n, 1), 256, 65536), 256, 0, st>>>(a, zoff, out->jc, out->cp, out->ptr_t,
                                                                                out->nzc, nullptr);
  SPX_HIP(hipGetLastError());
  // the scratch (zoff) must outlive the kernel: wait before it is released
  SPX_HIP(hipStreamSynchronize(st));
  out->m = A->m;
  out->n = A->n;
  out->nnz = A->nnz;
  out->fmt = SPX_DCSC;
  out->val_t = A->val_t;
  out->ir = A->ir;
  out->num = A->num;
  return SPX_OK;
}

extern "C" int spx_dcsc_to_csc(const spx_ctx* ctx, const spx_mat* A, spx_mat* out) {
  SPX_TRY(check_mat(A, "A"));
  if (A->fmt != SPX_DCSC) return fail(SPX_EINVAL, "A must be DCSC");
  if (!out || !out->cp) return fail(SPX_EINVAL, "out buffers missing");
  if (out->ptr_t != SPX_PTR_I32 && out->ptr_t != SPX_PTR_I64) return fail(SPX_EINVAL, "bad out ptr_t");
  if (out->ptr_t == SPX_PTR_I32 && A->nnz >= (1ll << 31)) return fail(SPX_EOVERFLOW, "nnz needs I64 pointers");
  hipStream_t st = stream_of(ctx);
  k_to_csc<<<grid_for(A->n + 1, 256, 65536), 256, 0, st>>>(make_operand(A), out->cp, out->ptr_t);
  SPX_HIP(hipGetLastError());
  out->m = A->m;
  out->n = A->n;
  out->nnz = A->nnz;
  out->nzc = 0;
  out->fmt = SPX_CSC;
  out->val_t = A->val_t;
  out->jc = nullptr;
  out->ir = A->ir;
  out->num = A->num;
  return SPX_OK;
}

extern "C" int spx_check(const spx_ctx* ctx, const spx_mat* A, int32_t* ok) {
  SPX_TRY(check_mat(A, "A"));
  if (!ok) return fail(SPX_EINVAL, "ok is NULL");
  hipStream_t st = stream_of(ctx);
  Scratch scr(ctx);
  unsigned* bad = nullptr;
  SPX_TRY(scr.get_n(4, &bad));
  SPX_TRY(fill_u32(bad, 1, 0, st));
  const Operand a = make_operand(A);
  const int64_t ns = nslots_of(a);
  k_check<<<grid_for(std::max<int64_t>(ns, 1), 256, 65536), 256, 0, st>>>(a, ns, bad);
  SPX_HIP(hipGetLastError());
  unsigned h = 0;
  SPX_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, st));
  SPX_HIP(hipStreamSynchronize(st));
  *ok = h == 0;
  return SPX_OK;
}

// ==================================================================== no allocation
// CSC -> DCSC for callers that cannot allocate device memory (code under
// HIP graph capture, serving loops, harnesses that forbid hipMalloc).  Its
// scratch -- the offsets of the nonempty columns and the scan's block sums --
// lives in the file-scope device array `scratch` below, which every GPU the
// library runs on holds until the process ends.  In host code the array's
// name is only a host-side stand-in: its device address is looked up once
// per device (hipGetSymbolAddress, with that device current) and only that
// address is passed to kernels.
namespace {

constexpr int64_t kNoAllocMaxCols = 1ll << 22;  // columns of A accepted
// offsets [n+1] int64, then the scan's block sums (two int64 per block of
// kScanTile columns at the first level, fewer at the next), 256-byte aligned
constexpr size_t kNoAllocScratchBytes = (size_t)(kNoAllocMaxCols + 1) * 8 + (1u << 20);

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call for that device).
int scratch_on_current_device(void** out) {
  int dev = -1;
  SPX_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SPX_EDEVICE, "device id out of the supported range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SPX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(SPX_EDEVICE, "no device address for the static scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SPX_OK;
}

// Bump allocator over a fixed device buffer (same interface as Scratch).
class FixedScratch {
 public:
  FixedScratch(void* base, size_t bytes) : base_(static_cast<char*>(base)), size_(bytes) {}
  int get(size_t bytes, void** out) {
    *out = nullptr;
    bytes = (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255;
    if (used_ + bytes > size_) return fail(SPX_ENOMEM, "static scratch exhausted");
    *out = base_ + used_;
    used_ += bytes;
    return SPX_OK;
  }
  template <typename T>
  int get_n(size_t count, T** out) {
    void* p = nullptr;
    const int rc = get(count * sizeof(T) + 16, &p);
    *out = static_cast<T*>(p);
    return rc;
  }

 private:
  char* base_;
  size_t size_;
  size_t used_ = 0;
};

}  // namespace

extern "C" int spx_csc_to_dcsc_noalloc(const spx_ctx* ctx, const spx_mat* A, spx_mat* out, int64_t* nzc_dev) {
  SPX_TRY(check_mat(A, "A"));
  if (A->fmt != SPX_CSC) return fail(SPX_EINVAL, "A must be CSC");
  if (A->n > kNoAllocMaxCols)
    return fail(SPX_EINVAL, "A has " + std::to_string(A->n) + " columns; the no-allocation conversion takes at most " +
                                std::to_string(kNoAllocMaxCols));
  if (!out || !out->cp || (out->nzc > 0 && !out->jc)) return fail(SPX_EINVAL, "out buffers missing");
  if (out->nzc < 0) return fail(SPX_EINVAL, "out->nzc (capacity) is negative");
  if (out->ptr_t != SPX_PTR_I32 && out->ptr_t != SPX_PTR_I64) return fail(SPX_EINVAL, "bad out ptr_t");
  if (out->ptr_t == SPX_PTR_I32 && A->nnz >= (1ll << 31)) return fail(SPX_EOVERFLOW, "nnz needs I64 pointers");
  void* base = nullptr;
  SPX_TRY(scratch_on_current_device(&base));
  hipStream_t st = stream_of(ctx);
  FixedScratch scr(base, kNoAllocScratchBytes);
  int64_t* zoff = nullptr;
  SPX_TRY(scr.get_n(A->n + 1, &zoff));
  const Operand a = make_operand(A);
  // every scratch word the kernels read is written first by the scan, so
  // nothing left by an earlier call needs clearing
  SPX_TRY(exclusive_scan(NonemptyCol{a}, A->n, zoff, scr, st));
  k_to_dcsc<<<grid_for(std::max<int64_t>(A->n, 1), 256, 65536), 256, 0, st>>>(a, zoff, out->jc, out->cp, out->ptr_t,
                                                                                out->nzc, nzc_dev);
  SPX_HIP(hipGetLastError());
  out->m = A->m;
  out->n = A->n;
  out->nnz = A->nnz;
  out->fmt = SPX_DCSC;
  out->val_t = A->val_t;
  out->ir = A->ir;
  out->num = A->num;
  return SPX_OK;
}
