// Graph contraction / restriction C = S_r * A * S_c^T as one SpGEMM pass
// (Section 5.3.2: restriction operators and the triple product S A S^T;
// Section 6: a triple-product primitive that forms no intermediate).
//
// S_r (m' x m) has one unit entry per column, S_r(row_agg(u), u); S_c
// (n' x n) likewise with col_agg.  Every stored A(u,v) then contributes
// exactly one product, to C(row_agg(u), col_agg(v)):
//     C = S_r * A * S_c^T = A_r * S_c^T,
// where A_r is A with its row ids replaced by row_agg (same columns, same
// values).  A non-decreasing row_agg keeps A_r's columns sorted (with
// repeated row ids), which is all the SpGEMM kernels need: they only take
// lower bounds over a column's rows, and their accumulators merge repeated
// rows as they merge rows reached from several columns.  So the triple
// product is one symbolic and one numeric pass over A; neither S_r * A nor
// A * S_c^T is formed, and both parenthesizations give this same pass.
// S_c^T (n x n') lists in column J the vertices v with col_agg(v) = J in
// ascending order, with value one of the semiring (1 for PLUS_TIMES, 0 for
// MIN_PLUS, pattern for SELECT1ST and OR_AND).
#include <algorithm>
#include <vector>

#include "common.h"
#include "operand.h"
#include "plan.h"
#include "scan.h"
#include "sort.h"

namespace spx {

struct ContractPlan : spx_plan {
  explicit ContractPlan(const spx_ctx* c) : spx_plan(c, kPlanContract) {}
  ~ContractPlan() override {
    if (gemm) spx_plan_destroy(gemm);
  }
  int32_t* air = nullptr;  // A's row ids through row_agg
  int64_t* scp = nullptr;  // S_c^T: [n'+1] pointers, [n] rows, [n] values
  int32_t* sir = nullptr;
  void* snum = nullptr;
  spx_plan* gemm = nullptr;
};

// err bit 1: an aggregate id out of range; bit 2: row_agg decreases somewhere.
__global__ void k_check_agg(const int32_t* agg, int64_t n, int64_t bound, unsigned* err, unsigned need_sorted) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = agg[v];
    if (a < 0 || a >= bound) atomicOr(err, 1u);
    if (v + 1 < n && agg[v + 1] < a) atomicOr(err, need_sorted ? 2u : 4u);
  }
}

__global__ void k_map_rows(const int32_t* ir, int64_t nnz, const int32_t* agg, int32_t* out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = agg[ir[e]];
}

__global__ void k_count_agg(const int32_t* agg, int64_t n, int64_t* cnt) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[agg[v]]), 1ull);
}

// Rows of S_c^T when col_agg is non-decreasing: vertex v sits at position v.
__global__ void k_iota(int32_t* out, int64_t n) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    out[v] = (int32_t)v;
}

__global__ void k_agg_keys(const int32_t* agg, int64_t n, uint64_t* keys) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    keys[v] = ((uint64_t)(uint32_t)agg[v] << 32) | (uint32_t)v;
}

__global__ void k_key_low(const uint64_t* keys, int64_t n, int32_t* out) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    out[v] = (int32_t)(uint32_t)keys[v];
}

template <typename T>
__global__ void k_fill_value(T* p, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace spx

using namespace spx;

extern "C" int spx_contract_plan(const spx_ctx* ctx, const spx_mat* A, const int32_t* row_agg, int64_t m_coarse,
                                 const int32_t* col_agg, int64_t n_coarse, int32_t semiring, int32_t c_fmt,
                                 const spx_tuning* tuning, spx_plan** plan, int64_t* nnz_c, int64_t* nzc_c) {
  if (!plan) return fail(SPX_EINVAL, "plan is NULL");
  *plan = nullptr;
  SPX_TRY(check_mat(A, "A"));
  const int64_t m = A->m, n = A->n;
  if (!row_agg) m_coarse = m;
  if (!col_agg) n_coarse = n;
  if (m_coarse < 0 || n_coarse < 0 || m_coarse >= (1ll << 31) || n_coarse >= (1ll << 31))
    return fail(SPX_EINVAL, "bad coarse dimensions");
  if ((row_agg && m > 0 && m_coarse == 0) || (col_agg && n > 0 && n_coarse == 0))
    return fail(SPX_EINVAL, "a nonempty side needs at least one aggregate");
  if (semiring != SPX_PLUS_TIMES && semiring != SPX_MIN_PLUS && semiring != SPX_SELECT1ST && semiring != SPX_OR_AND)
    return fail(SPX_EUNSUPPORTED, "contraction takes PLUS_TIMES, MIN_PLUS, SELECT1ST or OR_AND");
  if ((semiring == SPX_PLUS_TIMES || semiring == SPX_MIN_PLUS) && A->val_t == SPX_VAL_BOOL)
    return fail(SPX_EUNSUPPORTED, "PLUS_TIMES / MIN_PLUS contraction needs A's values");
  if (ctx && ctx->validate) {
    int32_t ok = 0;
    SPX_TRY(spx_check(ctx, A, &ok));
    if (!ok) return fail(SPX_EINVAL, "A is not canonical");
  }
  auto* P = new ContractPlan(ctx);
  std::unique_ptr<ContractPlan> guard(P);
  hipStream_t st = stream_of(ctx);
  Scratch& scr = P->scratch;
  unsigned* err = nullptr;
  SPX_TRY(scr.get_n(4, &err));
  SPX_TRY(fill_u32(err, 1, 0, st));
  if (row_agg && m > 0) {
    k_check_agg<<<grid_for(m, 256, 4096), 256, 0, st>>>(row_agg, m, m_coarse, err, 1u);
    SPX_HIP(hipGetLastError());
  }
  unsigned cerr_h = 0;
  unsigned* cerr = err + 1;
  SPX_TRY(fill_u32(cerr, 1, 0, st));
  if (col_agg && n > 0) {
    k_check_agg<<<grid_for(n, 256, 4096), 256, 0, st>>>(col_agg, n, n_coarse, cerr, 0u);
    SPX_HIP(hipGetLastError());
  }
  unsigned err_h = 0;
  SPX_HIP(hipMemcpyAsync(&err_h, err, 4, hipMemcpyDeviceToHost, st));
  SPX_HIP(hipMemcpyAsync(&cerr_h, cerr, 4, hipMemcpyDeviceToHost, st));
  SPX_HIP(hipStreamSynchronize(st));
  if ((err_h | cerr_h) & 1u) return fail(SPX_EINVAL, "an aggregate id is out of range");
  if (err_h & 2u) return fail(SPX_EUNSUPPORTED, "row_agg must be non-decreasing");
  const bool col_sorted = !(cerr_h & 4u);

  // left operand: A with mapped rows (A's pointers and values)
  spx_mat Ar = *A;
  if (row_agg) {
    SPX_TRY(scr.get_n(std::max<int64_t>(A->nnz, 1), &P->air));
    if (A->nnz > 0) {
      k_map_rows<<<grid_for(A->nnz, 256, 65536), 256, 0, st>>>(A->ir, A->nnz, row_agg, P->air);
      SPX_HIP(hipGetLastError());
    }
    Ar.ir = P->air;
    Ar.m = m_coarse;
  }
  // right operand: S_c^T in CSC
  const bool pattern_s = semiring == SPX_SELECT1ST || semiring == SPX_OR_AND;
  const int32_t s_vt = pattern_s ? SPX_VAL_BOOL : A->val_t;
  SPX_TRY(scr.get_n(n_coarse + 1, &P->scp));
  SPX_TRY(scr.get_n(std::max<int64_t>(n, 1), &P->sir));
  if (!pattern_s) SPX_TRY(scr.get(std::max<int64_t>(n, 1) * value_size(s_vt), &P->snum));
  if (col_agg) {
    int64_t* cnt = nullptr;
    SPX_TRY(scr.get_n(std::max<int64_t>(n_coarse, 1), &cnt));
    SPX_TRY(fill_i64(cnt, n_coarse, 0, st));
    if (n > 0) {
      k_count_agg<<<grid_for(n, 256, 4096), 256, 0, st>>>(col_agg, n, cnt);
      SPX_HIP(hipGetLastError());
    }
    SPX_TRY(exclusive_scan(LoadI64{cnt}, n_coarse, P->scp, scr, st));
    if (n > 0 && col_sorted) {
      k_iota<<<grid_for(n, 256, 65536), 256, 0, st>>>(P->sir, n);
      SPX_HIP(hipGetLastError());
    } else if (n > 0) {
      uint64_t* keys = nullptr;
      SPX_TRY(scr.get_n(sort_capacity(n), &keys));
      k_agg_keys<<<grid_for(n, 256, 65536), 256, 0, st>>>(col_agg, n, keys);
      SPX_HIP(hipGetLastError());
      SPX_TRY(sort_u64(keys, n, st));
      k_key_low<<<grid_for(n, 256, 65536), 256, 0, st>>>(keys, n, P->sir);
      SPX_HIP(hipGetLastError());
    }
  } else {  // S_c = I: scp[j] = j, sir[v] = v
    int64_t* ones = nullptr;
    SPX_TRY(scr.get_n(std::max<int64_t>(n, 1), &ones));
    SPX_TRY(fill_i64(ones, n, 1, st));
    SPX_TRY(exclusive_scan(LoadI64{ones}, n, P->scp, scr, st));
    if (n > 0) {
      k_iota<<<grid_for(n, 256, 65536), 256, 0, st>>>(P->sir, n);
      SPX_HIP(hipGetLastError());
    }
  }
  if (!pattern_s && n > 0) {
    if (s_vt == SPX_VAL_F32)
      k_fill_value<float><<<grid_for(n, 256, 65536), 256, 0, st>>>(static_cast<float*>(P->snum), n,
                                                                   semiring == SPX_PLUS_TIMES ? 1.0f : 0.0f);
    else if (s_vt == SPX_VAL_F64)
      k_fill_value<double><<<grid_for(n, 256, 65536), 256, 0, st>>>(static_cast<double*>(P->snum), n,
                                                                    semiring == SPX_PLUS_TIMES ? 1.0 : 0.0);
    else
      k_fill_value<int64_t><<<grid_for(n, 256, 65536), 256, 0, st>>>(static_cast<int64_t*>(P->snum), n,
                                                                     semiring == SPX_PLUS_TIMES ? 1 : 0);
    SPX_HIP(hipGetLastError());
  }
  spx_mat Sc{};
  Sc.m = n;
  Sc.n = n_coarse;
  Sc.nnz = n;
  Sc.fmt = SPX_CSC;
  Sc.ptr_t = SPX_PTR_I64;
  Sc.val_t = s_vt;
  Sc.cp = P->scp;
  Sc.ir = P->sir;
  Sc.num = P->snum;
  spx_ctx c2 = ctx ? *ctx : spx_ctx{};
  c2.validate = 0;  // A_r repeats row ids inside a column by design
  SPX_TRY(spx_spgemm_plan(&c2, &Ar, &Sc, semiring, c_fmt, tuning, &P->gemm, nnz_c, nzc_c));
  *plan = guard.release();
  return SPX_OK;
}

extern "C" int spx_contract_exec(spx_plan* plan, spx_mat* C) {
  if (!plan || plan->kind != kPlanContract) return fail(SPX_EINVAL, "not a contraction plan");
  return spx_spgemm_exec(static_cast<ContractPlan*>(plan)->gemm, C);
}

namespace spx {
const spx_plan* contract_plan_inner(const spx_plan* plan) { return static_cast<const ContractPlan*>(plan)->gemm; }
}  // namespace spx
