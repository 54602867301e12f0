// SpAsgn C = A with A(I,J) = B (Section 4.1).
//
// The paper forms C = A + R*B*Q - S*A*T, replacing the subtraction by an
// elementwise product of A with the negated pattern of S*A*T so that no
// additive inverse is needed.  The two terms have disjoint patterns: the
// masked A keeps the entries (i, j) with i not in I or j not in J, and
// R*B*Q places B(p,q) at (I(p), J(q)).  So C is a union with no semiring
// addition, computed here per column:
//   * columns j not in J: copied from A unchanged (streamed in tiles);
//   * columns j in J: A(:,j) minus the rows in I, merged with the rows
//     I(p) of B(:,q), q = last position of j in J.
// Repeated indices: the last occurrence in I (and J) wins, as sequential
// assignment would leave it (the selection matrices are built from last
// occurrences, and S, T are 0/1 patterns).
#include <algorithm>

#include "common.h"
#include "operand.h"
#include "plan.h"
#include "scan.h"

namespace spx {

constexpr int kAsgnMaxInsert = 4096;  // inserted rows per column handled in LDS
constexpr int64_t kCopyTile = 4096;   // A entries per copy workgroup

struct SpasgnPlan : spx_plan {
  explicit SpasgnPlan(const spx_ctx* c) : spx_plan(c, kPlanSpasgn) {}
  Operand A{}, B{};
  const int32_t* I = nullptr;
  const int32_t* J = nullptr;
  int64_t lenI = 0, lenJ = 0, nnz = 0, nmod = 0, ndrop = 0;
  int32_t* lastI = nullptr;  // [m] last p with I(p) = i, or -1
  int32_t* lastJ = nullptr;  // [n]
  int64_t* cnt = nullptr;    // [n]
  int64_t* off = nullptr;    // [n+1] = C.cp
  int32_t* mod = nullptr;    // [n] modified columns
  int64_t* dcnt = nullptr;   // [nmod] dropped entries per modified column
  int64_t* doff = nullptr;   // [nmod+1]
  int32_t* drows = nullptr;  // [ndrop] rows of the dropped entries
  unsigned* err = nullptr;
  unsigned long long* nmod_d = nullptr;
};

__global__ void k_last_occ(const int32_t* v, int64_t len, int64_t bound, int32_t* last, unsigned* err, unsigned bit) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < len; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = v[p];
    if (x < 0 || x >= bound)
      atomicOr(err, bit);
    else
      atomicMax(&last[x], (int32_t)p);
  }
}

// Unmodified columns keep their length; modified ones are listed.
__global__ void k_asgn_cols(Operand A, const int32_t* lastJ, int64_t* cnt, int32_t* mod, unsigned long long* nmod) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < A.n; j += (int64_t)gridDim.x * blockDim.x) {
    if (lastJ[j] < 0) {
      cnt[j] = slot_begin(A, j + 1) - slot_begin(A, j);
    } else {
      cnt[j] = 0;
      mod[atomicAdd(nmod, 1ull)] = (int32_t)j;
    }
  }
}

// Per modified column: kept A entries, dropped ones, inserted B entries.
__global__ void __launch_bounds__(256) k_asgn_mod_count(Operand A, Operand B, const int32_t* I, const int32_t* lastI,
                                                        const int32_t* lastJ, const int32_t* mod, int64_t nmod,
                                                        int64_t* cnt, int64_t* dcnt, unsigned* err) {
  __shared__ int64_t red[256 / kWave + 1];
  for (int64_t u = blockIdx.x; u < nmod; u += gridDim.x) {
    const int32_t j = mod[u];
    const int64_t a0 = slot_begin(A, j), a1 = slot_begin(A, j + 1);
    const int32_t q = lastJ[j];
    const int64_t b0 = slot_begin(B, q), b1 = slot_begin(B, q + 1);
    int64_t kept = 0, ins = 0;
    for (int64_t e = a0 + threadIdx.x; e < a1; e += blockDim.x) kept += lastI[A.ir[e]] < 0;
    for (int64_t e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
      const int32_t p = B.ir[e];
      ins += lastI[I[p]] == p;
    }
    int64_t tk, ti;
    block_excl_scan(kept, red, &tk);
    block_excl_scan(ins, red, &ti);
    if (threadIdx.x == 0) {
      cnt[j] = tk + ti;
      dcnt[u] = (a1 - a0) - tk;
      if (ti > kAsgnMaxInsert) atomicOr(err, 4u);
    }
  }
}

// Copies the unmodified columns: each workgroup takes a tile of A's
// entries, finds their columns by binary search over A's pointers and
// writes them at C's offsets.
__global__ void __launch_bounds__(256) k_asgn_copy(Operand A, const int32_t* lastJ, const int64_t* off, int vb,
                                                   int32_t* cir, void* cnum) {
  __shared__ int64_t s_range[2];
  const int64_t nt = (A.nnz + kCopyTile - 1) / kCopyTile;
  for (int64_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const int64_t e0 = tile * kCopyTile;
    const int64_t e1 = e0 + kCopyTile < A.nnz ? e0 + kCopyTile : A.nnz;
    if (threadIdx.x < 2) {
      // column of entry e0 (resp. e1-1): last j with cp[j] <= e
      const int64_t e = threadIdx.x == 0 ? e0 : e1 - 1;
      int64_t lo = 0, hi = A.n;  // find first j with cp[j+1] > e
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (slot_begin(A, mid + 1) <= e)
          lo = mid + 1;
        else
          hi = mid;
      }
      s_range[threadIdx.x] = lo;
    }
    __syncthreads();
    const int64_t j0 = s_range[0], j1 = s_range[1];
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      int64_t lo = j0, hi = j1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (slot_begin(A, mid + 1) <= e)
          lo = mid + 1;
        else
          hi = mid;
      }
      const int64_t j = lo;
      if (lastJ[j] >= 0) continue;
      const int64_t o = off[j] + (e - slot_begin(A, j));
      cir[o] = A.ir[e];
      copy_value(A.num, e, cnum, o, vb);
    }
    __syncthreads();
  }
}

// Modified columns: merge the kept A entries (rows not in I, ascending) with
// the inserted rows I(p) (sorted here), by merge-path positions.
__global__ void __launch_bounds__(256) k_asgn_mod_fill(Operand A, Operand B, const int32_t* I, const int32_t* lastI,
                                                       const int32_t* lastJ, const int32_t* mod, int64_t nmod,
                                                       const int64_t* off, const int64_t* doff, int32_t* drows,
                                                       int vb, int32_t* cir, void* cnum) {
  __shared__ uint64_t s_key[kAsgnMaxInsert];
  __shared__ int64_t s_src[kAsgnMaxInsert];
  __shared__ int64_t red[256 / kWave + 1];
  for (int64_t u = blockIdx.x; u < nmod; u += gridDim.x) {
    const int32_t j = mod[u];
    const int64_t a0 = slot_begin(A, j), a1 = slot_begin(A, j + 1);
    const int32_t q = lastJ[j];
    const int64_t b0 = slot_begin(B, q), b1 = slot_begin(B, q + 1);
    const int64_t cbase = off[j];
    // 1. inserted entries (row, source) -> LDS, sorted by row
    int64_t nins = 0;
    for (int64_t ec = b0; ec < b1; ec += blockDim.x) {
      const int64_t e = ec + threadIdx.x;
      int64_t take = 0;
      int32_t row = 0;
      if (e < b1) {
        const int32_t p = B.ir[e];
        row = I[p];
        take = lastI[row] == p;
      }
      int64_t tot;
      const int64_t ex = block_excl_scan(take, red, &tot);
      if (take && nins + ex < kAsgnMaxInsert) {
        s_key[nins + ex] = ((uint64_t)(uint32_t)row << 32) | (uint32_t)(nins + ex);
        s_src[nins + ex] = e;
      }
      nins += tot;
    }
    if (nins > kAsgnMaxInsert) nins = kAsgnMaxInsert;
    int p2 = 1;
    while (p2 < nins) p2 <<= 1;
    for (int s = (int)nins + threadIdx.x; s < p2; s += blockDim.x) s_key[s] = ~0ull;
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int t = threadIdx.x; t < (p2 >> 1); t += blockDim.x) {
          const int lo = 2 * t - (t & (jj - 1));
          const int hi = lo + jj;
          const bool asc = (lo & k) == 0;
          const uint64_t x = s_key[lo], y = s_key[hi];
          if ((x > y) == asc) {
            s_key[lo] = y;
            s_key[hi] = x;
          }
        }
        __syncthreads();
      }
    }
    // 2. kept A entries: position = kept rank + inserted rows below; dropped rows listed
    int64_t kept_run = 0, drop_run = 0;
    const int64_t dbase = doff[u];
    for (int64_t ec = a0; ec < a1; ec += blockDim.x) {
      const int64_t e = ec + threadIdx.x;
      int64_t keep = 0, drop = 0;
      int32_t row = 0;
      if (e < a1) {
        row = A.ir[e];
        keep = lastI[row] < 0;
        drop = !keep;
      }
      int64_t tk, td;
      const int64_t xk = block_excl_scan(keep, red, &tk);
      const int64_t xd = block_excl_scan(drop, red, &td);
      if (keep) {
        int lo = 0, hi = (int)nins;  // inserted rows < row
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if ((int32_t)(s_key[mid] >> 32) < row)
            lo = mid + 1;
          else
            hi = mid;
        }
        const int64_t o = cbase + kept_run + xk + lo;
        cir[o] = row;
        copy_value(A.num, e, cnum, o, vb);
      }
      if (drop) drows[dbase + drop_run + xd] = row;
      kept_run += tk;
      drop_run += td;
    }
    __threadfence_block();
    __syncthreads();
    // 3. inserted entries: position = rank + kept rows below
    const int32_t* acol = A.ir + a0;
    const int32_t alen = (int32_t)(a1 - a0);
    for (int s = threadIdx.x; s < nins; s += blockDim.x) {
      const uint64_t key = s_key[s];
      const int32_t row = (int32_t)(key >> 32);
      int32_t lo = 0, hi = alen;  // A rows < row
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (acol[mid] < row)
          lo = mid + 1;
        else
          hi = mid;
      }
      int64_t dlo = 0, dhi = drop_run;  // dropped rows < row
      while (dlo < dhi) {
        const int64_t mid = (dlo + dhi) >> 1;
        if (drows[dbase + mid] < row)
          dlo = mid + 1;
        else
          dhi = mid;
      }
      const int64_t o = cbase + s + (lo - dlo);
      cir[o] = row;
      copy_value(B.num, s_src[key & 0xffffffffu], cnum, o, vb);
    }
    __syncthreads();
  }
}

__global__ void k_asgn_write_cp(const int64_t* off, int64_t n, void* cp, int32_t ptr_t) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= n; j += (int64_t)gridDim.x * blockDim.x)
    store_ptr(cp, ptr_t, j, off[j]);
}

}  // namespace spx

using namespace spx;

extern "C" int spx_spasgn_plan(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J,
                               int64_t lenJ, const spx_mat* B, spx_plan** plan, int64_t* nnz_c) {
  if (!plan) return fail(SPX_EINVAL, "plan is NULL");
  *plan = nullptr;
  SPX_TRY(check_mat(A, "A"));
  SPX_TRY(check_mat(B, "B"));
  if (A->fmt != SPX_CSC || B->fmt != SPX_CSC) return fail(SPX_EUNSUPPORTED, "SpAsgn takes CSC operands");
  if (lenI < 0 || lenJ < 0 || lenI >= (1ll << 31) || lenJ >= (1ll << 31)) return fail(SPX_EINVAL, "bad index length");
  if (B->m != lenI || B->n != lenJ) return fail(SPX_EINVAL, "B must be lenI x lenJ");
  if (A->val_t != B->val_t) return fail(SPX_EINVAL, "A and B must have the same value type");
  if ((lenI > 0 && !I) || (lenJ > 0 && !J)) return fail(SPX_EINVAL, "index vector is NULL");
  if (ctx && ctx->validate) {
    int32_t ok = 0;
    SPX_TRY(spx_check(ctx, A, &ok));
    if (!ok) return fail(SPX_EINVAL, "A is not canonical");
    SPX_TRY(spx_check(ctx, B, &ok));
    if (!ok) return fail(SPX_EINVAL, "B is not canonical");
  }
  auto* P = new SpasgnPlan(ctx);
  std::unique_ptr<SpasgnPlan> guard(P);
  hipStream_t st = stream_of(ctx);
  Scratch& scr = P->scratch;
  P->A = make_operand(A);
  P->B = make_operand(B);
  P->I = I;
  P->J = J;
  P->lenI = lenI;
  P->lenJ = lenJ;
  const int64_t m = A->m, n = A->n;
  const int cus = device_cu_count();
  SPX_TRY(scr.get_n(4, &P->err));
  SPX_TRY(fill_u32(P->err, 1, 0, st));
  SPX_TRY(scr.get_n(1, &P->nmod_d));
  SPX_TRY(fill_i64((int64_t*)P->nmod_d, 1, 0, st));
  SPX_TRY(scr.get_n(std::max<int64_t>(m, 1), &P->lastI));
  SPX_TRY(scr.get_n(std::max<int64_t>(n, 1), &P->lastJ));
  SPX_TRY(fill_u32((uint32_t*)P->lastI, m, 0xffffffffu, st));
  SPX_TRY(fill_u32((uint32_t*)P->lastJ, n, 0xffffffffu, st));
  if (lenI > 0) {
    k_last_occ<<<grid_for(lenI, 256, 4096), 256, 0, st>>>(I, lenI, m, P->lastI, P->err, 1u);
    SPX_HIP(hipGetLastError());
  }
  if (lenJ > 0) {
    k_last_occ<<<grid_for(lenJ, 256, 4096), 256, 0, st>>>(J, lenJ, n, P->lastJ, P->err, 2u);
    SPX_HIP(hipGetLastError());
  }
  SPX_TRY(scr.get_n(std::max<int64_t>(n, 1), &P->cnt));
  SPX_TRY(scr.get_n(n + 1, &P->off));
  SPX_TRY(scr.get_n(std::max<int64_t>(n, 1), &P->mod));
  if (n > 0) {
    k_asgn_cols<<<grid_for(n, 256, 65536), 256, 0, st>>>(P->A, P->lastJ, P->cnt, P->mod, P->nmod_d);
    SPX_HIP(hipGetLastError());
  }
  unsigned long long nmod_h = 0;
  unsigned err_h = 0;
  SPX_HIP(hipMemcpyAsync(&nmod_h, P->nmod_d, 8, hipMemcpyDeviceToHost, st));
  SPX_HIP(hipMemcpyAsync(&err_h, P->err, 4, hipMemcpyDeviceToHost, st));
  SPX_HIP(hipStreamSynchronize(st));
  if (err_h & 1u) return fail(SPX_EINVAL, "I has an index outside [0, m)");
  if (err_h & 2u) return fail(SPX_EINVAL, "J has an index outside [0, n)");
  P->nmod = (int64_t)nmod_h;
  SPX_TRY(scr.get_n(std::max<int64_t>(P->nmod, 1), &P->dcnt));
  SPX_TRY(scr.get_n(P->nmod + 1, &P->doff));
  if (P->nmod > 0) {
    k_asgn_mod_count<<<(unsigned)std::min<int64_t>(P->nmod, (int64_t)cus * 8), 256, 0, st>>>(
        P->A, P->B, I, P->lastI, P->lastJ, P->mod, P->nmod, P->cnt, P->dcnt, P->err);
    SPX_HIP(hipGetLastError());
  }
  SPX_TRY(exclusive_scan(LoadI64{P->cnt}, n, P->off, scr, st));
  SPX_TRY(exclusive_scan(LoadI64{P->dcnt}, P->nmod, P->doff, scr, st));
  int64_t tail[2] = {0, 0};
  SPX_HIP(hipMemcpyAsync(&tail[0], P->off + n, 8, hipMemcpyDeviceToHost, st));
  SPX_HIP(hipMemcpyAsync(&tail[1], P->doff + P->nmod, 8, hipMemcpyDeviceToHost, st));
  SPX_HIP(hipMemcpyAsync(&err_h, P->err, 4, hipMemcpyDeviceToHost, st));
  SPX_HIP(hipStreamSynchronize(st));
  if (err_h & 4u) return fail(SPX_EUNSUPPORTED, "a column of B inserts more than 4096 rows");
  P->nnz = tail[0];
  P->ndrop = tail[1];
  SPX_TRY(scr.get_n(std::max<int64_t>(P->ndrop, 1), &P->drows));
  if (nnz_c) *nnz_c = P->nnz;
  *plan = guard.release();
  return SPX_OK;
}

extern "C" int spx_spasgn_exec(spx_plan* plan, spx_mat* C) {
  if (!plan || plan->kind != kPlanSpasgn) return fail(SPX_EINVAL, "not a SpAsgn plan");
  auto* P = static_cast<SpasgnPlan*>(plan);
  if (!C) return fail(SPX_EINVAL, "C is NULL");
  if (C->m != P->A.m || C->n != P->A.n || C->fmt != SPX_CSC) return fail(SPX_EINVAL, "C must be m x n CSC");
  if (C->val_t != P->A.val_t) return fail(SPX_EINVAL, "C's value type must be A's");
  if (C->ptr_t == SPX_PTR_I32 && P->nnz >= (1ll << 31)) return fail(SPX_EOVERFLOW, "nnz(C) needs I64 pointers");
  if (!C->cp || (P->nnz > 0 && (!C->ir || (C->val_t != SPX_VAL_BOOL && !C->num))))
    return fail(SPX_EINVAL, "C buffers missing");
  C->nnz = P->nnz;
  C->nzc = 0;
  hipStream_t st = stream_of(&P->ctx);
  const int vb = value_size(P->A.val_t);
  const int cus = device_cu_count();
  if (P->A.nnz > 0) {
    const int64_t tiles = ceil_div(P->A.nnz, kCopyTile);
    k_asgn_copy<<<(unsigned)std::min<int64_t>(tiles, (int64_t)cus * 8), 256, 0, st>>>(P->A, P->lastJ, P->off, vb,
                                                                                       C->ir, C->num);
    SPX_HIP(hipGetLastError());
  }
  if (P->nmod > 0) {
    k_asgn_mod_fill<<<(unsigned)std::min<int64_t>(P->nmod, (int64_t)cus * 2), 256, 0, st>>>(
        P->A, P->B, P->I, P->lastI, P->lastJ, P->mod, P->nmod, P->off, P->doff, P->drows, vb, C->ir, C->num);
    SPX_HIP(hipGetLastError());
  }
  k_asgn_write_cp<<<grid_for(P->A.n + 1, 256, 65536), 256, 0, st>>>(P->off, P->A.n, C->cp, C->ptr_t);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}
