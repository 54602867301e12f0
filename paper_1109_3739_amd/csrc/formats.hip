// CSC <-> DCSC conversion and canonical-form checks (Section 3.2: DCSC drops
// the repeated column pointers of empty columns and lists the ids of the
// nonempty columns in JC; IR and NUM are the same arrays as in CSC).
#include <algorithm>

#include "common.h"
#include "operand.h"
#include "plan.h"
#include "scan.h"

namespace spx {

struct NonemptyCol {
  Operand A;
  __device__ int64_t operator()(int64_t j) const { return slot_begin(A, j + 1) > slot_begin(A, j) ? 1 : 0; }
};

__global__ void k_to_dcsc(Operand A, const int64_t* zoff, int32_t* jc, void* cp, int32_t ptr_t) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < A.n; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = slot_begin(A, j), e = slot_begin(A, j + 1);
    if (e > s) {
      jc[zoff[j]] = (int32_t)j;
      store_ptr(cp, ptr_t, zoff[j], s);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) store_ptr(cp, ptr_t, zoff[A.n], A.nnz);
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
  k_to_dcsc<<<grid_for(std::max<int64_t>(A->n, 1), 256, 65536), 256, 0, st>>>(a, zoff, out->jc, out->cp, out->ptr_t);
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
