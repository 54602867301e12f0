// Batched SpGEMM: C_i = A_i * B_i for many products in one pass.
//
// The batch is the single product  [A_1 A_2 ... A_n] * blockdiag(B_1, ..., B_n)
// = [C_1 C_2 ... C_n]: column j of block i of the right operand only has
// rows inside block i's range, so it only meets the columns of A_i.  Left
// operands passed more than once (the same arrays) enter the concatenation
// once, and every B_i that uses them points at that block.  The
// concatenated operands are built once by the plan (patterns) and refreshed
// by every exec (values, unless the callers' value arrays already lie back to
// back in batch order: then they are read in place); the symbolic phase, the binning and the persistent
// numeric launches of the ordinary SpGEMM then run over the work items of
// all products together.  C_i are views into caller-owned pools.
#include <algorithm>
#include <map>
#include <tuple>
#include <cstring>
#include <vector>

#include "common.h"
#include "plan.h"

namespace spx {

struct BatchDesc {
  const void* acp;
  const int32_t* air;
  const void* anum;
  const void* bcp;
  const int32_t* bir;
  const void* bnum;
  int32_t a_ptr_t, b_ptr_t;
};

struct BatchPlan : spx_plan {
  explicit BatchPlan(const spx_ctx* c) : spx_plan(c, kPlanBatch) {}
  ~BatchPlan() override {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (gemm) spx_plan_destroy(gemm);
  }
  int32_t count = 0;
  int32_t count_a = 0;  // distinct left operands
  int32_t vt_c = 0;
  int vb_a = 0, vb_b = 0, vb_c = 0;
  std::vector<int64_t> m_h, n_h, acol_h, anz_h, bcol_h, bnz_h, cnz_h;  // bases, count+1 entries
  BatchDesc* desc = nullptr;
  int64_t *acol = nullptr, *anz = nullptr, *bcol = nullptr, *bnz = nullptr;
  int64_t* acolp = nullptr;  // per product: first column of its left operand's block
  int64_t* acp = nullptr;
  int32_t* air = nullptr;
  void* anum = nullptr;
  int64_t* bcp = nullptr;
  int32_t* bir = nullptr;
  void* bnum = nullptr;
  int64_t* ccp = nullptr;  // column pointers of [C_1 ... C_n]
  spx_plan* gemm = nullptr;
  int64_t nnz_total = 0, cp_total = 0, mmax = 0;
  bool anum_in_place = false, bnum_in_place = false;  // anum / bnum alias the callers' arrays
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

__device__ __forceinline__ int find_block(const int64_t* base, int count, int64_t x) {
  int lo = 0, hi = count;  // last i with base[i] <= x
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Concatenation of one array of every product.  Product i is handled by the
// workgroups with blockIdx.y == i (mod gridDim.y), which stride over its
// elements, so no element searches for its product.
//   kCatAIr / kCatBIr: row indices (B's rows move to block i's column range
//   of A); kCatANum / kCatBNum: values; kCatACp / kCatBCp: column pointers,
//   cp[c] = nnz base of block i + its own cp (the final entry is written
//   separately).
enum CatKind { kCatAIr, kCatBIr, kCatANum, kCatBNum, kCatACp, kCatBCp };

__global__ void k_cat(const BatchDesc* d, int count, const int64_t* nzb, const int64_t* colb, const int64_t* acolb,
                      int kind, int vb, void* out) {
  for (int i = blockIdx.y; i < count; i += gridDim.y) {
    const bool cp = kind == kCatACp || kind == kCatBCp;
    const int64_t base = cp ? colb[i] : nzb[i];
    const int64_t len = (cp ? colb[i + 1] : nzb[i + 1]) - base;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < len; k += (int64_t)gridDim.x * blockDim.x) {
      switch (kind) {
        case kCatAIr: static_cast<int32_t*>(out)[base + k] = d[i].air[k]; break;
        case kCatBIr: static_cast<int32_t*>(out)[base + k] = (int32_t)(d[i].bir[k] + acolb[i]); break;
        case kCatANum: copy_value(d[i].anum, k, out, base + k, vb); break;
        case kCatBNum: copy_value(d[i].bnum, k, out, base + k, vb); break;
        case kCatACp: static_cast<int64_t*>(out)[base + k] = nzb[i] + load_ptr(d[i].acp, d[i].a_ptr_t, k); break;
        default: static_cast<int64_t*>(out)[base + k] = nzb[i] + load_ptr(d[i].bcp, d[i].b_ptr_t, k); break;
      }
    }
  }
}

// Largest per-product length of a prefix array (count + 1 entries).
static int64_t max_len(const std::vector<int64_t>& pre) {
  int64_t m = 0;
  for (size_t i = 1; i < pre.size(); ++i) m = std::max(m, pre[i] - pre[i - 1]);
  return m;
}

static void launch_cat(BatchPlan* P, int kind, const int64_t* nzb, const int64_t* colb, int vb, void* out,
                       int64_t max_len, hipStream_t st) {
  const int n = (kind == kCatAIr || kind == kCatANum || kind == kCatACp) ? P->count_a : P->count;
  const unsigned gy = (unsigned)std::min<int64_t>(n, 65535);
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(max_len, 256 * 4), 64));
  k_cat<<<dim3(gx, gy), 256, 0, st>>>(P->desc, n, nzb, colb, P->acolp, kind, vb, out);
}

// Per-product column pointers (relative to the product's first entry).
__global__ void k_batch_cp(const int64_t* ccp, const int64_t* bcol, int count, int64_t total, int64_t* cp_pool) {
  // entry x of the pool: product i owns [bcol[i] + i, bcol[i+1] + i + 1)
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = count;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (bcol[mid] + mid <= x)
        lo = mid;
      else
        hi = mid;
    }
    const int64_t j = x - (bcol[lo] + lo);
    cp_pool[x] = ccp[bcol[lo] + j] - ccp[bcol[lo]];
  }
}

__global__ void k_gather_i64(const int64_t* src, const int64_t* idx, int n, int64_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = src[idx[i]];
}

// Start of the concatenation when every nonempty value array of the batch
// already lies at its concatenated offset from one address (nz holds the
// entry offsets, count + 1 of them), else null.  The outputs of an earlier
// batch are views into one pool in batch order, so a batch that takes them
// as its right operands reads their values in place instead of copying them.
static void* in_place_base(const std::vector<const void*>& ptrs, const std::vector<int64_t>& nz, int vb) {
  uintptr_t base = 0;
  bool any = false;
  for (size_t i = 0; i < ptrs.size(); ++i) {
    if (nz[i + 1] == nz[i]) continue;  // an empty operand is never read
    const uintptr_t b = reinterpret_cast<uintptr_t>(ptrs[i]) - (uintptr_t)(nz[i] * vb);
    if (!ptrs[i] || (any && b != base)) return nullptr;
    base = b;
    any = true;
  }
  return any ? reinterpret_cast<void*>(base) : nullptr;
}

static int run_exec(BatchPlan* P, int64_t* cp_pool, int32_t* ir_pool, void* num_pool, hipStream_t st) {
  const int64_t anz = P->anz_h[P->count_a], bnz = P->bnz_h[P->count];
  if (P->vb_a && anz > 0 && !P->anum_in_place) {
    launch_cat(P, kCatANum, P->anz, P->acol, P->vb_a, P->anum, max_len(P->anz_h), st);
    SPX_HIP(hipGetLastError());
  }
  if (P->vb_b && bnz > 0 && !P->bnum_in_place) {
    launch_cat(P, kCatBNum, P->bnz, P->bcol, P->vb_b, P->bnum, max_len(P->bnz_h), st);
    SPX_HIP(hipGetLastError());
  }
  spx_mat C{};
  C.m = P->mmax;
  C.n = P->bcol_h[P->count];
  C.fmt = SPX_CSC;
  C.ptr_t = SPX_PTR_I64;
  C.val_t = P->vt_c;
  C.cp = P->ccp;
  C.ir = ir_pool;
  C.num = num_pool;
  SPX_TRY(spx_spgemm_exec(P->gemm, &C));
  k_batch_cp<<<grid_for(P->cp_total, 256, 65536), 256, 0, st>>>(P->ccp, P->bcol, P->count, P->cp_total, cp_pool);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

static void fill_outputs(BatchPlan* P, int64_t* cp_pool, int32_t* ir_pool, void* num_pool, spx_mat* C) {
  for (int i = 0; i < P->count; ++i) {
    spx_mat& c = C[i];
    std::memset(&c, 0, sizeof(c));
    c.m = P->m_h[i];
    c.n = P->n_h[i];
    c.nnz = P->cnz_h[i + 1] - P->cnz_h[i];
    c.fmt = SPX_CSC;
    c.ptr_t = SPX_PTR_I64;
    c.val_t = P->vt_c;
    c.cp = cp_pool + P->bcol_h[i] + i;
    c.ir = ir_pool + P->cnz_h[i];
    c.num = P->vb_c ? (void*)((char*)num_pool + P->cnz_h[i] * P->vb_c) : nullptr;
  }
}

}  // namespace spx

using namespace spx;

extern "C" int spx_batch_plan(const spx_ctx* ctx, int32_t count, const spx_mat* A, const spx_mat* B, int32_t semiring,
                              const spx_tuning* tuning, spx_plan** plan, int64_t* nnz_total, int64_t* cp_total) {
  if (!plan) return fail(SPX_EINVAL, "plan is NULL");
  *plan = nullptr;
  if (count <= 0 || !A || !B) return fail(SPX_EINVAL, "empty batch");
  for (int i = 0; i < count; ++i) {
    SPX_TRY(check_mat(&A[i], "A[i]"));
    SPX_TRY(check_mat(&B[i], "B[i]"));
    if (A[i].fmt != SPX_CSC || B[i].fmt != SPX_CSC) return fail(SPX_EUNSUPPORTED, "batched operands must be CSC");
    if (A[i].n != B[i].m) return fail(SPX_EINVAL, "inner dimensions differ in product " + std::to_string(i));
    if (A[i].val_t != A[0].val_t || B[i].val_t != B[0].val_t)
      return fail(SPX_EINVAL, "all A_i (and all B_i) must share one value type");
  }
  auto* P = new BatchPlan(ctx);
  std::unique_ptr<BatchPlan> guard(P);
  hipStream_t st = stream_of(ctx);
  Scratch& scr = P->scratch;
  P->count = count;
  P->vb_a = value_size(A[0].val_t);
  P->vb_b = value_size(B[0].val_t);
  for (auto* v : {&P->m_h, &P->n_h}) v->resize(count);
  for (auto* v : {&P->bcol_h, &P->bnz_h, &P->cnz_h}) v->assign(count + 1, 0);
  // distinct left operands (entry u of the descriptors holds the u-th one;
  // the B fields of entry i hold product i)
  std::vector<BatchDesc> hd(count);
  std::vector<int64_t> acolp_h(count);
  std::map<std::tuple<const void*, const void*, const void*, int64_t, int64_t, int64_t, int32_t>, int> seen;
  P->acol_h.assign(1, 0);
  P->anz_h.assign(1, 0);
  for (int i = 0; i < count; ++i) {
    P->m_h[i] = A[i].m;
    P->n_h[i] = B[i].n;
    P->mmax = std::max(P->mmax, A[i].m);
    const auto key = std::make_tuple((const void*)A[i].cp, (const void*)A[i].ir, (const void*)A[i].num, A[i].m,
                                     A[i].n, A[i].nnz, A[i].ptr_t);
    auto it = seen.find(key);
    int u;
    if (it == seen.end()) {
      u = (int)seen.size();
      seen.emplace(key, u);
      hd[u].acp = A[i].cp;
      hd[u].air = A[i].ir;
      hd[u].anum = A[i].num;
      hd[u].a_ptr_t = A[i].ptr_t;
      P->acol_h.push_back(P->acol_h.back() + A[i].n);
      P->anz_h.push_back(P->anz_h.back() + A[i].nnz);
    } else {
      u = it->second;
    }
    acolp_h[i] = P->acol_h[u];
    P->bcol_h[i + 1] = P->bcol_h[i] + B[i].n;
    P->bnz_h[i + 1] = P->bnz_h[i] + B[i].nnz;
    hd[i].bcp = B[i].cp;
    hd[i].bir = B[i].ir;
    hd[i].bnum = B[i].num;
    hd[i].b_ptr_t = B[i].ptr_t;
  }
  P->count_a = (int32_t)seen.size();
  const int na = P->count_a;
  const int64_t ka = P->acol_h[na], anz = P->anz_h[na], nb = P->bcol_h[count], bnz = P->bnz_h[count];
  if (ka >= (1ll << 31) || nb >= (1ll << 31)) return fail(SPX_EUNSUPPORTED, "batch too large (2^31 columns)");
  SPX_TRY(scr.get_n(count, &P->desc));
  for (auto* pp : {&P->acol, &P->anz}) SPX_TRY(scr.get_n(na + 1, pp));
  for (auto* pp : {&P->bcol, &P->bnz}) SPX_TRY(scr.get_n(count + 1, pp));
  SPX_TRY(scr.get_n(count, &P->acolp));
  SPX_HIP(hipMemcpyAsync(P->desc, hd.data(), sizeof(BatchDesc) * count, hipMemcpyHostToDevice, st));
  SPX_HIP(hipMemcpyAsync(P->acol, P->acol_h.data(), 8 * (na + 1), hipMemcpyHostToDevice, st));
  SPX_HIP(hipMemcpyAsync(P->anz, P->anz_h.data(), 8 * (na + 1), hipMemcpyHostToDevice, st));
  SPX_HIP(hipMemcpyAsync(P->acolp, acolp_h.data(), 8 * count, hipMemcpyHostToDevice, st));
  SPX_HIP(hipMemcpyAsync(P->bcol, P->bcol_h.data(), 8 * (count + 1), hipMemcpyHostToDevice, st));
  SPX_HIP(hipMemcpyAsync(P->bnz, P->bnz_h.data(), 8 * (count + 1), hipMemcpyHostToDevice, st));
  SPX_TRY(scr.get_n(ka + 1, &P->acp));
  SPX_TRY(scr.get_n(std::max<int64_t>(anz, 1), &P->air));
  SPX_TRY(scr.get_n(nb + 1, &P->bcp));
  SPX_TRY(scr.get_n(std::max<int64_t>(bnz, 1), &P->bir));
  SPX_TRY(scr.get_n(nb + 1, &P->ccp));
  // values: read in place when the callers' arrays already form the
  // concatenation, else copied by every exec into the plan's own arrays
  if (P->vb_a && anz > 0) {
    std::vector<const void*> ap(na);
    for (int u = 0; u < na; ++u) ap[u] = hd[u].anum;
    P->anum = in_place_base(ap, P->anz_h, P->vb_a);
    P->anum_in_place = P->anum != nullptr;
  }
  if (P->vb_b && bnz > 0) {
    std::vector<const void*> bp(count);
    for (int i = 0; i < count; ++i) bp[i] = hd[i].bnum;
    P->bnum = in_place_base(bp, P->bnz_h, P->vb_b);
    P->bnum_in_place = P->bnum != nullptr;
  }
  if (P->vb_a && !P->anum_in_place) SPX_TRY(scr.get(std::max<int64_t>(anz, 1) * P->vb_a, &P->anum));
  if (P->vb_b && !P->bnum_in_place) SPX_TRY(scr.get(std::max<int64_t>(bnz, 1) * P->vb_b, &P->bnum));
  // patterns of the concatenated operands (values are copied by every exec)
  launch_cat(P, kCatACp, P->anz, P->acol, 0, P->acp, max_len(P->acol_h), st);
  launch_cat(P, kCatBCp, P->bnz, P->bcol, 0, P->bcp, max_len(P->bcol_h), st);
  SPX_TRY(fill_i64(P->acp + ka, 1, anz, st));
  SPX_TRY(fill_i64(P->bcp + nb, 1, bnz, st));
  if (anz > 0) launch_cat(P, kCatAIr, P->anz, P->acol, 0, P->air, max_len(P->anz_h), st);
  if (bnz > 0) launch_cat(P, kCatBIr, P->bnz, P->bcol, 0, P->bir, max_len(P->bnz_h), st);
  SPX_HIP(hipGetLastError());
  spx_mat Ac{}, Bc{};
  Ac.m = P->mmax;
  Ac.n = ka;
  Ac.nnz = anz;
  Ac.fmt = SPX_CSC;
  Ac.ptr_t = SPX_PTR_I64;
  Ac.val_t = A[0].val_t;
  Ac.cp = P->acp;
  Ac.ir = P->air;
  Ac.num = P->anum;
  Bc.m = ka;
  Bc.n = nb;
  Bc.nnz = bnz;
  Bc.fmt = SPX_CSC;
  Bc.ptr_t = SPX_PTR_I64;
  Bc.val_t = B[0].val_t;
  Bc.cp = P->bcp;
  Bc.ir = P->bir;
  Bc.num = P->bnum;
  int64_t nnz = 0, nzc = 0;
  spx_ctx c2 = ctx ? *ctx : spx_ctx{};
  c2.validate = 0;
  SPX_TRY(spx_spgemm_plan(&c2, &Ac, &Bc, semiring, SPX_CSC, tuning, &P->gemm, &nnz, &nzc));
  spx_plan_info info;
  SPX_TRY(spx_plan_get_info(P->gemm, &info));
  (void)info;
  // output nnz base of every product: the offsets of its first column
  int64_t* cb = nullptr;
  SPX_TRY(scr.get_n(count + 1, &cb));
  k_gather_i64<<<grid_for(count + 1, 256), 256, 0, st>>>(gemm_plan_offsets(P->gemm), P->bcol, count + 1, cb);
  SPX_HIP(hipGetLastError());
  SPX_HIP(hipMemcpyAsync(P->cnz_h.data(), cb, 8 * (count + 1), hipMemcpyDeviceToHost, st));
  SPX_HIP(hipStreamSynchronize(st));
  P->vt_c = semiring == SPX_OR_AND ? SPX_VAL_BOOL
            : semiring == SPX_SELECT2ND ? B[0].val_t
            : A[0].val_t;
  P->vb_c = value_size(P->vt_c);
  P->nnz_total = nnz;
  P->cp_total = nb + count;
  if (nnz_total) *nnz_total = nnz;
  if (cp_total) *cp_total = P->cp_total;
  *plan = guard.release();
  return SPX_OK;
}

static int batch_args(spx_plan* plan, int64_t* cp_pool, int32_t* ir_pool, void* num_pool, spx_mat* C, BatchPlan** out) {
  if (!plan || plan->kind != kPlanBatch) return fail(SPX_EINVAL, "not a batch plan");
  auto* P = static_cast<BatchPlan*>(plan);
  if (!cp_pool || !C || (P->nnz_total > 0 && (!ir_pool || (P->vb_c && !num_pool))))
    return fail(SPX_EINVAL, "batch output pools missing");
  *out = P;
  return SPX_OK;
}

extern "C" int spx_batch_exec(spx_plan* plan, int64_t* cp_pool, int32_t* ir_pool, void* num_pool, spx_mat* C) {
  BatchPlan* P = nullptr;
  SPX_TRY(batch_args(plan, cp_pool, ir_pool, num_pool, C, &P));
  SPX_TRY(run_exec(P, cp_pool, ir_pool, num_pool, stream_of(&P->ctx)));
  fill_outputs(P, cp_pool, ir_pool, num_pool, C);
  return SPX_OK;
}

extern "C" int spx_batch_capture(spx_plan* plan, int64_t* cp_pool, int32_t* ir_pool, void* num_pool, spx_mat* C) {
  BatchPlan* P = nullptr;
  SPX_TRY(batch_args(plan, cp_pool, ir_pool, num_pool, C, &P));
  if (P->ctx.profile) return fail(SPX_EINVAL, "capture needs a plan without profiling events");
  hipStream_t st = stream_of(&P->ctx);
  if (!st) return fail(SPX_EINVAL, "capture needs a non-null stream");
  if (P->gexec) {
    (void)hipGraphExecDestroy(P->gexec);
    P->gexec = nullptr;
  }
  if (P->graph) {
    (void)hipGraphDestroy(P->graph);
    P->graph = nullptr;
  }
  SPX_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const int rc = run_exec(P, cp_pool, ir_pool, num_pool, st);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (rc != SPX_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(SPX_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  P->graph = g;
  SPX_HIP(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
  fill_outputs(P, cp_pool, ir_pool, num_pool, C);
  return SPX_OK;
}

extern "C" int spx_batch_replay(spx_plan* plan) {
  if (!plan || plan->kind != kPlanBatch) return fail(SPX_EINVAL, "not a batch plan");
  auto* P = static_cast<BatchPlan*>(plan);
  if (!P->gexec) return fail(SPX_EINVAL, "no captured graph");
  SPX_HIP(hipGraphLaunch(P->gexec, stream_of(&P->ctx)));
  return SPX_OK;
}

extern "C" int spx_batch_spgemm(const spx_ctx* ctx, int32_t count, const spx_mat* A, const spx_mat* B,
                                int32_t semiring, const spx_tuning* tuning, spx_mat* C) {
  if (!C) return fail(SPX_EINVAL, "C is NULL");
  spx_plan* plan = nullptr;
  int64_t nnz_total = 0, cp_total = 0;
  SPX_TRY(spx_batch_plan(ctx, count, A, B, semiring, tuning, &plan, &nnz_total, &cp_total));
  std::unique_ptr<spx_plan> guard(plan);
  auto* P = static_cast<BatchPlan*>(plan);
  OutAlloc oa(ctx);
  void *cp = nullptr, *ir = nullptr, *num = nullptr;
  SPX_TRY(oa.get((size_t)cp_total * 8, &cp));
  SPX_TRY(oa.get((size_t)std::max<int64_t>(nnz_total, 1) * 4, &ir));
  if (P->vb_c) SPX_TRY(oa.get((size_t)std::max<int64_t>(nnz_total, 1) * P->vb_c, &num));
  SPX_TRY(spx_batch_exec(plan, static_cast<int64_t*>(cp), static_cast<int32_t*>(ir), num, C));
  oa.keep();
  return SPX_OK;
}
