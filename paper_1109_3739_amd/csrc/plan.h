// Plan objects shared by the entry points of libspx.  A plan owns the
// device scratch of one operation between its plan and exec calls.
#pragma once

#include <memory>

#include "common.h"

struct spx_plan {
  spx_plan(const spx_ctx* c, int k) : kind(k), scratch(c) {
    if (c) ctx = *c;
  }
  virtual ~spx_plan() {}
  int kind;
  spx_ctx ctx{};
  spx::Scratch scratch;
};

namespace spx {

enum { kPlanGemm = 1, kPlanSpref = 2, kPlanSpasgn = 3, kPlanBatch = 4, kPlanExtAdd = 5, kPlanSum = 6, kPlanContract = 7 };

// Validates a descriptor (dimensions, codes, non-NULL buffers).
int check_mat(const spx_mat* X, const char* name);

// Bytes per value of a value type (0 for BOOL).
inline int value_size(int32_t vt) {
  switch (vt) {
    case SPX_VAL_F32: return 4;
    case SPX_VAL_F64: return 8;
    case SPX_VAL_I64: return 8;
    default: return 0;
  }
}

// Copies `vb` bytes (0, 4 or 8) of element `src` of `from` to element `dst` of `to`.
__device__ __forceinline__ void copy_value(const void* from, int64_t src, void* to, int64_t dst, int vb) {
  if (vb == 8)
    reinterpret_cast<uint64_t*>(to)[dst] = reinterpret_cast<const uint64_t*>(from)[src];
  else if (vb == 4)
    reinterpret_cast<uint32_t*>(to)[dst] = reinterpret_cast<const uint32_t*>(from)[src];
}

// Device pointer to the output column offsets of a SpGEMM plan (one entry
// per stored column of B plus the total), valid while the plan lives.
const int64_t* gemm_plan_offsets(const spx_plan* plan);

// The SpGEMM plan inside a stage-sum plan (plan->kind == kPlanSum).
const spx_plan* sum_plan_inner(const spx_plan* plan);

// The SpGEMM plan inside a contraction plan (plan->kind == kPlanContract).
const spx_plan* contract_plan_inner(const spx_plan* plan);

}  // namespace spx

