// Device-side view of a CSC / DCSC operand and column lookup (Section 3.2:
// DCSC keeps only nonempty columns; the AUX array indexes them).
#pragma once

#include "common.h"

namespace spx {

struct Operand {
  int64_t m, n, nnz, nzc;
  int32_t fmt, ptr_t, val_t, pad;
  const int32_t* jc;
  const void* cp;
  const int32_t* ir;
  const void* num;
};

inline Operand make_operand(const spx_mat* X) {
  Operand o;
  o.m = X->m;
  o.n = X->n;
  o.nnz = X->nnz;
  o.nzc = X->nzc;
  o.fmt = X->fmt;
  o.ptr_t = X->ptr_t;
  o.val_t = X->val_t;
  o.pad = 0;
  o.jc = X->jc;
  o.cp = X->cp;
  o.ir = X->ir;
  o.num = X->num;
  return o;
}

// Stored columns ("slots"): all n columns of a CSC matrix, the nzc nonempty
// ones of a DCSC matrix.
__host__ __device__ inline int64_t nslots_of(const Operand& X) { return X.fmt == SPX_DCSC ? X.nzc : X.n; }

__device__ __forceinline__ int64_t slot_begin(const Operand& X, int64_t t) { return load_ptr(X.cp, X.ptr_t, t); }
__device__ __forceinline__ int64_t slot_col(const Operand& X, int64_t t) {
  return X.fmt == SPX_DCSC ? (int64_t)X.jc[t] : t;
}

// AUX index of a DCSC matrix: aux[c] = first position in jc with
// jc >= c*chunk (c = 0..naux), chunk = ceil(n / nzc).  A column k is then
// searched in jc[aux[k/chunk], aux[k/chunk+1]), about one entry on average.
static __global__ void k_build_aux(const int32_t* jc, int64_t nzc, int64_t chunk, int64_t naux, int64_t* aux) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c > naux) return;
  const int64_t key = c * chunk;
  int64_t lo = 0, hi = nzc;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)jc[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  aux[c] = lo;
}

// Range [a0, a1) of column k of X in X.ir (empty if a DCSC X has no column k).
__device__ __forceinline__ void column_range(const Operand& X, const int64_t* aux, int64_t chunk, int64_t k, int64_t& a0,
                                             int64_t& a1) {
  a0 = a1 = 0;
  if (X.fmt == SPX_CSC) {
    a0 = load_ptr(X.cp, X.ptr_t, k);
    a1 = load_ptr(X.cp, X.ptr_t, k + 1);
    return;
  }
  const int64_t c = k / chunk;
  int64_t lo = aux[c], hi = aux[c + 1];
  const int64_t end = hi;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (X.jc[mid] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo < end && X.jc[lo] == k) {
    a0 = load_ptr(X.cp, X.ptr_t, lo);
    a1 = load_ptr(X.cp, X.ptr_t, lo + 1);
  }
}

// As column_range, also giving the slot of column k (-1 if not stored).
__device__ __forceinline__ int64_t column_slot(const Operand& X, const int64_t* aux, int64_t chunk, int64_t k) {
  if (X.fmt == SPX_CSC) return k;
  const int64_t c = k / chunk;
  int64_t lo = aux[c], hi = aux[c + 1];
  const int64_t end = hi;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (X.jc[mid] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < end && X.jc[lo] == k) ? lo : -1;
}

// Builds the AUX index of a DCSC operand into scratch (no-op for CSC).
int build_aux(const Operand& X, Scratch& scr, hipStream_t st, int64_t** aux, int64_t* chunk);

}  // namespace spx
