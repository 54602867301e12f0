// Sparse SUMMA stage accumulation on one GPU (Section 3.3, Algorithm 2).
//
// On a sqrt(p) x sqrt(p) grid, processor (i,j) accumulates
// C_ij = C_ij + A_ik * B_kj over the stages k.  When all stage blocks of one
// processor are resident in HBM, the stages are one product over a longer
// inner dimension:
//     sum_k A_k * B_k = [A_1 A_2 ... A_K] * [B_1; B_2; ...; B_K].
// Every output column then gathers the products of all stages into one LDS
// accumulator (the accumulators of the stage products stay live across the
// stages), so no partial C_ij is written, re-read or merged.
//
// The plan builds the two concatenated patterns once:
//   * left:  DCSC, m x sum(b_k); the nonempty columns of every A_k, moved to
//            the stage's column range (its row ids and values are A_k's,
//            one after the other);
//   * right: CSC, sum(b_k) x n; column j lists B_1(:,j), B_2(:,j) + b_1, ...
//            in stage order, so rows stay ascending.
// and a SpGEMM plan over them.  Exec copies the values of the stage blocks
// into the concatenations and runs the SpGEMM numeric phase.
#include <algorithm>
#include <vector>

#include "common.h"
#include "operand.h"
#include "plan.h"
#include "scan.h"

namespace spx {

struct SumPlan : spx_plan {
  explicit SumPlan(const spx_ctx* c) : spx_plan(c, kPlanSum) {}
  ~SumPlan() override {
    if (gemm) spx_plan_destroy(gemm);
  }
  int32_t count = 0;
  int vb_a = 0, vb_b = 0;
  std::vector<Operand> a_h, b_h;      // the stage blocks
  std::vector<int64_t> anz_h, bnz_h;  // nnz bases of the stages (count+1)
  Operand* a_d = nullptr;
  Operand* b_d = nullptr;
  int64_t* bnzb = nullptr;   // [count+1] nnz bases of the B_k
  int64_t* slotb = nullptr;  // [count+1] slot bases of the A_k
  int64_t* colb = nullptr;   // [count+1] column bases of the A_k (= row bases of the B_k)
  int64_t* anzb = nullptr;   // [count+1] nnz bases of the A_k
  int32_t* ajc = nullptr;
  int64_t* acp = nullptr;
  int32_t* air = nullptr;
  void* anum = nullptr;
  int64_t* bcp = nullptr;
  int32_t* bir = nullptr;
  void* bnum = nullptr;
  int64_t* bmap = nullptr;  // position in the right concatenation of every B_k entry
  spx_plan* gemm = nullptr;
};

__device__ __forceinline__ int stage_of(const int64_t* base, int count, int64_t x) {
  int lo = 0, hi = count;  // last k with base[k] <= x
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// 1 for a nonempty slot of the concatenated left operand (slot i of all stages).
struct LoadNonempty {
  const Operand* a;
  const int64_t* slotb;
  int count;
  __device__ int64_t operator()(int64_t i) const {
    const int k = stage_of(slotb, count, i);
    const int64_t t = i - slotb[k];
    return slot_begin(a[k], t + 1) > slot_begin(a[k], t);
  }
};

// Writes the DCSC column ids and pointers of the left concatenation.
__global__ void k_sum_left(const Operand* a, const int64_t* slotb, const int64_t* colb, const int64_t* anzb,
                           const int64_t* pos, int count, int32_t* jc, int64_t* cp) {
  for (int k = blockIdx.y; k < count; k += gridDim.y) {
    const Operand X = a[k];
    const int64_t ns = slotb[k + 1] - slotb[k];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ns; t += (int64_t)gridDim.x * blockDim.x) {
      const int64_t s0 = slot_begin(X, t);
      if (slot_begin(X, t + 1) == s0) continue;
      const int64_t p = pos[slotb[k] + t];
      jc[p] = (int32_t)(colb[k] + slot_col(X, t));
      cp[p] = anzb[k] + s0;
    }
  }
}

// Column lengths of the right concatenation (B_k share the n columns).
__global__ void k_sum_right_count(Operand X, int64_t* cnt) {
  const int64_t ns = nslots_of(X);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ns; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t len = slot_begin(X, t + 1) - slot_begin(X, t);
    if (len > 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[slot_col(X, t)]), (unsigned long long)len);
  }
}

// Appends B_k's columns (rows moved down by the stage's row base) at each
// column's cursor.  One wave per slot; stages run one launch after the
// other, so every column's cursor has one writer per launch.
__global__ void __launch_bounds__(256) k_sum_right_place(Operand X, int64_t rowb, int64_t* cur, int32_t* ir,
                                                         int64_t* map) {
  const int64_t ns = nslots_of(X);
  const int lane = threadIdx.x % kWave;
  const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t t = w0; t < ns; t += nw) {
    const int64_t s0 = slot_begin(X, t), s1 = slot_begin(X, t + 1);
    if (s1 == s0) continue;
    const int64_t j = slot_col(X, t);
    const int64_t dst = cur[j];
    for (int64_t e = s0 + lane; e < s1; e += kWave) {
      ir[dst + (e - s0)] = (int32_t)(X.ir[e] + rowb);
      map[e] = dst + (e - s0);
    }
    if (lane == 0) cur[j] = dst + (s1 - s0);
  }
}

// Values of the right concatenation: stage k scatters through its map.
__global__ void k_sum_right_vals(const Operand* b, const int64_t* bnzb, const int64_t* map, int count, int vb,
                                 void* out) {
  for (int k = blockIdx.y; k < count; k += gridDim.y) {
    const int64_t len = bnzb[k + 1] - bnzb[k];
    const void* src = b[k].num;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x)
      copy_value(src, e, out, map[bnzb[k] + e], vb);
  }
}

const spx_plan* sum_plan_inner(const spx_plan* plan) { return static_cast<const SumPlan*>(plan)->gemm; }

}  // namespace spx

using namespace spx;

extern "C" int spx_spgemm_sum_plan(const spx_ctx* ctx, int32_t count, const spx_mat* A, const spx_mat* B,
                                   int32_t semiring, int32_t c_fmt, const spx_tuning* tuning, spx_plan** plan,
                                   int64_t* nnz_c, int64_t* nzc_c) {
  if (!plan) return fail(SPX_EINVAL, "plan is NULL");
  *plan = nullptr;
  if (count < 1 || !A || !B) return fail(SPX_EINVAL, "need count >= 1 stage blocks");
  int64_t inner = 0, anz = 0, bnz = 0, slots = 0;
  for (int k = 0; k < count; ++k) {
    SPX_TRY(check_mat(&A[k], "A_k"));
    SPX_TRY(check_mat(&B[k], "B_k"));
    if (A[k].m != A[0].m || B[k].n != B[0].n) return fail(SPX_EINVAL, "stage blocks must share m (A) and n (B)");
    if (A[k].n != B[k].m) return fail(SPX_EINVAL, "inner dimensions of a stage differ");
    if (A[k].val_t != A[0].val_t || B[k].val_t != B[0].val_t)
      return fail(SPX_EINVAL, "stage blocks must share value types");
    inner += A[k].n;
    anz += A[k].nnz;
    bnz += B[k].nnz;
  }
  if (inner >= (1ll << 31)) return fail(SPX_EUNSUPPORTED, "the summed inner dimension must be below 2^31");
  if (ctx && ctx->validate) {
    for (int k = 0; k < count; ++k) {
      int32_t ok = 0;
      SPX_TRY(spx_check(ctx, &A[k], &ok));
      if (!ok) return fail(SPX_EINVAL, "A_k is not canonical");
      SPX_TRY(spx_check(ctx, &B[k], &ok));
      if (!ok) return fail(SPX_EINVAL, "B_k is not canonical");
    }
  }
  auto* P = new SumPlan(ctx);
  std::unique_ptr<SumPlan> guard(P);
  hipStream_t st = stream_of(ctx);
  Scratch& scr = P->scratch;
  P->count = count;
  P->vb_a = value_size(A[0].val_t);
  P->vb_b = value_size(B[0].val_t);
  const int64_t m = A[0].m, n = B[0].n;
  std::vector<int64_t> slotb(count + 1, 0), colb(count + 1, 0);
  P->anz_h.assign(count + 1, 0);
  P->bnz_h.assign(count + 1, 0);
  for (int k = 0; k < count; ++k) {
    P->a_h.push_back(make_operand(&A[k]));
    P->b_h.push_back(make_operand(&B[k]));
    slotb[k + 1] = slotb[k] + nslots_of(P->a_h[k]);
    colb[k + 1] = colb[k] + A[k].n;
    P->anz_h[k + 1] = P->anz_h[k] + A[k].nnz;
    P->bnz_h[k + 1] = P->bnz_h[k] + B[k].nnz;
  }
  slots = slotb[count];
  // stage tables on the device (the host vectors live as long as the plan)
  SPX_TRY(scr.get_n(count, &P->a_d));
  SPX_TRY(scr.get_n(count + 1, &P->slotb));
  SPX_TRY(scr.get_n(count + 1, &P->colb));
  SPX_TRY(scr.get_n(count + 1, &P->anzb));
  SPX_TRY(scr.get_n(count, &P->b_d));
  SPX_TRY(scr.get_n(count + 1, &P->bnzb));
  SPX_HIP(hipMemcpyAsync(P->a_d, P->a_h.data(), sizeof(Operand) * count, hipMemcpyHostToDevice, st));
  SPX_HIP(hipMemcpyAsync(P->b_d, P->b_h.data(), sizeof(Operand) * count, hipMemcpyHostToDevice, st));
  SPX_HIP(hipMemcpyAsync(P->bnzb, P->bnz_h.data(), 8 * (count + 1), hipMemcpyHostToDevice, st));
  std::vector<int64_t> tables(3 * (count + 1));
  std::copy(slotb.begin(), slotb.end(), tables.begin());
  std::copy(colb.begin(), colb.end(), tables.begin() + (count + 1));
  std::copy(P->anz_h.begin(), P->anz_h.end(), tables.begin() + 2 * (count + 1));
  SPX_HIP(hipMemcpyAsync(P->slotb, tables.data(), 8 * (count + 1), hipMemcpyHostToDevice, st));
  SPX_HIP(hipMemcpyAsync(P->colb, tables.data() + (count + 1), 8 * (count + 1), hipMemcpyHostToDevice, st));
  SPX_HIP(hipMemcpyAsync(P->anzb, tables.data() + 2 * (count + 1), 8 * (count + 1), hipMemcpyHostToDevice, st));

  // left concatenation (DCSC)
  int64_t* pos = nullptr;
  SPX_TRY(scr.get_n(slots + 1, &pos));
  SPX_TRY(exclusive_scan(LoadNonempty{P->a_d, P->slotb, count}, slots, pos, scr, st));
  int64_t nzc_a = 0;
  SPX_HIP(hipMemcpyAsync(&nzc_a, pos + slots, 8, hipMemcpyDeviceToHost, st));
  SPX_HIP(hipStreamSynchronize(st));  // tables and nzc_a are read below
  SPX_TRY(scr.get_n(std::max<int64_t>(nzc_a, 1), &P->ajc));
  SPX_TRY(scr.get_n(nzc_a + 1, &P->acp));
  SPX_TRY(scr.get_n(std::max<int64_t>(anz, 1), &P->air));
  if (P->vb_a) SPX_TRY(scr.get(std::max<int64_t>(anz, 1) * P->vb_a, &P->anum));
  if (slots > 0) {
    const unsigned gy = (unsigned)std::min<int>(count, 64);
    int64_t widest = 0;
    for (const Operand& X : P->a_h) widest = std::max(widest, nslots_of(X));
    dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(widest, 256), 1024)), gy);
    k_sum_left<<<grid, 256, 0, st>>>(P->a_d, P->slotb, P->colb, P->anzb, pos, count, P->ajc, P->acp);
    SPX_HIP(hipGetLastError());
  }
  SPX_TRY(fill_i64(P->acp + nzc_a, 1, anz, st));
  for (int k = 0; k < count; ++k)
    if (A[k].nnz > 0)
      SPX_HIP(hipMemcpyAsync(P->air + P->anz_h[k], A[k].ir, 4 * A[k].nnz, hipMemcpyDeviceToDevice, st));

  // right concatenation (CSC)
  int64_t* cnt = nullptr;
  int64_t* cur = nullptr;
  SPX_TRY(scr.get_n(std::max<int64_t>(n, 1), &cnt));
  SPX_TRY(scr.get_n(n + 1, &P->bcp));
  SPX_TRY(scr.get_n(n + 1, &cur));
  SPX_TRY(scr.get_n(std::max<int64_t>(bnz, 1), &P->bir));
  SPX_TRY(scr.get_n(std::max<int64_t>(bnz, 1), &P->bmap));
  if (P->vb_b) SPX_TRY(scr.get(std::max<int64_t>(bnz, 1) * P->vb_b, &P->bnum));
  SPX_TRY(fill_i64(cnt, n, 0, st));
  for (int k = 0; k < count; ++k) {
    const int64_t ns = nslots_of(P->b_h[k]);
    if (ns == 0 || B[k].nnz == 0) continue;
    k_sum_right_count<<<grid_for(ns, 256, 4096), 256, 0, st>>>(P->b_h[k], cnt);
    SPX_HIP(hipGetLastError());
  }
  SPX_TRY(exclusive_scan(LoadI64{cnt}, n, P->bcp, scr, st));
  SPX_HIP(hipMemcpyAsync(cur, P->bcp, 8 * (n + 1), hipMemcpyDeviceToDevice, st));
  for (int k = 0; k < count; ++k) {
    const int64_t ns = nslots_of(P->b_h[k]);
    if (ns == 0 || B[k].nnz == 0) continue;
    k_sum_right_place<<<grid_for(ns * kWave, 256, 8192), 256, 0, st>>>(P->b_h[k], colb[k], cur, P->bir,
                                                                        P->bmap + P->bnz_h[k]);
    SPX_HIP(hipGetLastError());
  }

  // one SpGEMM over the concatenations
  spx_mat Ac{}, Bc{};
  Ac.m = m;
  Ac.n = inner;
  Ac.nnz = anz;
  Ac.nzc = nzc_a;
  Ac.fmt = SPX_DCSC;
  Ac.ptr_t = SPX_PTR_I64;
  Ac.val_t = A[0].val_t;
  Ac.jc = P->ajc;
  Ac.cp = P->acp;
  Ac.ir = P->air;
  Ac.num = P->anum;
  Bc.m = inner;
  Bc.n = n;
  Bc.nnz = bnz;
  Bc.fmt = SPX_CSC;
  Bc.ptr_t = SPX_PTR_I64;
  Bc.val_t = B[0].val_t;
  Bc.cp = P->bcp;
  Bc.ir = P->bir;
  Bc.num = P->bnum;
  spx_ctx c2 = ctx ? *ctx : spx_ctx{};
  c2.validate = 0;
  SPX_TRY(spx_spgemm_plan(&c2, &Ac, &Bc, semiring, c_fmt, tuning, &P->gemm, nnz_c, nzc_c));
  *plan = guard.release();
  return SPX_OK;
}

extern "C" int spx_spgemm_sum_exec(spx_plan* plan, spx_mat* C) {
  if (!plan || plan->kind != kPlanSum) return fail(SPX_EINVAL, "not a stage-sum plan");
  auto* P = static_cast<SumPlan*>(plan);
  hipStream_t st = stream_of(&P->ctx);
  if (P->vb_a) {
    for (int k = 0; k < P->count; ++k) {
      const int64_t len = P->anz_h[k + 1] - P->anz_h[k];
      if (len > 0)
        SPX_HIP(hipMemcpyAsync(static_cast<char*>(P->anum) + P->anz_h[k] * P->vb_a, P->a_h[k].num, len * P->vb_a,
                               hipMemcpyDeviceToDevice, st));
    }
  }
  if (P->vb_b && P->bnz_h[P->count] > 0) {
    int64_t widest = 0;
    for (int k = 0; k < P->count; ++k) widest = std::max(widest, P->bnz_h[k + 1] - P->bnz_h[k]);
    dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(widest, 256), 2048)),
              (unsigned)std::min<int>(P->count, 64));
    k_sum_right_vals<<<grid, 256, 0, st>>>(P->b_d, P->bnzb, P->bmap, P->count, P->vb_b, P->bnum);
    SPX_HIP(hipGetLastError());
  }
  return spx_spgemm_exec(P->gemm, C);
}
