// Graph contraction / restriction C = S_r * A * S_c^T as one SpGEMM pass
// (Section 5.3.2: restriction operators and the triple product S A S^T;
// Section 6: a triple-product primitive that forms no intermediate).
//
// S_r (m' x m) has one unit entry per column, S_r(row_agg(u), u); S_c
// (n' x n) likewise with col_agg.  Every stored A(u,v) then contributes
// exactly one product, to C(row_agg(u), col_agg(v)):
//     C = S_r * A * S_c^T = A_r * S_c^T,
// where A_r is A with its row ids replaced by row_agg (same columns, same
// values).  The SpGEMM kernels need each column's rows non-decreasing (they
// only take lower bounds over a column's rows, and their accumulators merge
// repeated rows as they merge rows reached from several columns).  A
// non-decreasing row_agg keeps A's order; any other map has the plan sort
// each column of A_r by mapped row and keep the permutation, through which
// every exec gathers A's values.  So the triple product is one symbolic and
// one numeric pass over A; neither S_r * A nor A * S_c^T is formed, and both
// parenthesizations give this same pass.
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
  int32_t* air = nullptr;  // A's row ids through row_agg (sorted within each column)
  int64_t* aperm = nullptr;  // unsorted row_agg: source entry of each entry of A_r
  void* anum = nullptr;      // and A's values in that order (refreshed by exec)
  const void* src_num = nullptr;
  int64_t nnz = 0;
  int vb = 0;
  int64_t* scp = nullptr;  // S_c^T: [n'+1] pointers, [n] rows, [n] values
  int32_t* sir = nullptr;
  void* snum = nullptr;
  spx_plan* gemm = nullptr;
};

// err bit 1: an aggregate id out of range; bit 2 (row map) or 4 (column
// map): the map decreases somewhere.  Flags are gathered per thread and
// combined per wave, so an unsorted map costs one atomic per wave.
__global__ void k_check_agg(const int32_t* agg, int64_t n, int64_t bound, unsigned* err, unsigned need_sorted) {
  unsigned flags = 0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = agg[v];
    if (a < 0 || a >= bound) flags |= 1u;
    if (v + 1 < n && agg[v + 1] < a) flags |= need_sorted ? 2u : 4u;
  }
  const uint64_t m1 = __ballot((flags & 1u) != 0), m2 = __ballot((flags & 6u) != 0);
  if (lane_id() == 0 && (m1 | m2)) atomicOr(err, (m1 ? 1u : 0u) | (m2 ? (need_sorted ? 2u : 4u) : 0u));
}

__global__ void k_map_rows(const int32_t* ir, int64_t nnz, const int32_t* agg, int32_t* out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = agg[ir[e]];
}

// Runs of equal aggregate ids in a wave (consecutive vertices often share
// an aggregate): a lane heads a run when its id differs from the lane
// before it, and the head's atomic counts (or claims slots for) the whole
// run.  The valid lanes of a wave (v < n) are a prefix of it.
struct AggRun {
  int32_t a;      // this lane's aggregate, -1 past the end
  bool head;
  int len;        // run length (heads)
  int head_lane;  // the head of this lane's run (valid lanes)
};
__device__ __forceinline__ AggRun agg_run(const int32_t* agg, int64_t v, int64_t n) {
  const int lane = lane_id();
  AggRun R;
  R.a = v < n ? agg[v] : -1;
  const int32_t prev = __shfl_up(R.a, 1);
  R.head = R.a >= 0 && (lane == 0 || prev != R.a);
  const uint64_t hm = __ballot(R.head);
  const int nvalid = __popcll(__ballot(R.a >= 0));
  const uint64_t later = lane < 63 ? hm >> (lane + 1) : 0ull;
  R.len = later ? __ffsll((long long)later) : nvalid - lane;
  const uint64_t upto = hm & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
  R.head_lane = upto ? 63 - __clzll((long long)upto) : 0;
  return R;
}

__global__ void k_count_agg(const int32_t* agg, int64_t n, int64_t* cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x - lane_id(); w < n; w += stride) {
    const AggRun R = agg_run(agg, w + lane_id(), n);
    if (R.head) atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[R.a]), (unsigned long long)R.len);
  }
}

// Rows of S_c^T when col_agg is non-decreasing: vertex v sits at position v.
__global__ void k_iota(int32_t* out, int64_t n) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    out[v] = (int32_t)v;
}

// Vertices into their aggregate's column of S_c^T (any order inside a column;
// the column sort puts them in ascending order).
__global__ void k_scatter_agg(const int32_t* agg, int64_t n, const int64_t* scp, unsigned* cur, int32_t* sir) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x - lane_id(); w < n; w += stride) {
    const int64_t v = w + lane_id();
    const AggRun R = agg_run(agg, v, n);
    unsigned base = 0;
    if (R.head) base = atomicAdd(&cur[R.a], (unsigned)R.len);
    base = __shfl(base, R.head_lane);
    if (R.a >= 0) sir[scp[R.a] + base + (unsigned)(lane_id() - R.head_lane)] = (int32_t)v;
  }
}

__global__ void k_agg_keys(const int32_t* agg, int64_t n, uint64_t* keys) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    keys[v] = ((uint64_t)(uint32_t)agg[v] << 32) | (uint32_t)v;
}

__global__ void k_key_low(const uint64_t* keys, int64_t n, int32_t* out) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    out[v] = (int32_t)(uint32_t)keys[v];
}

// Sorting the columns of A_r by mapped row (unsorted row_agg), or the columns
// of S_c^T by row (row_agg NULL; in place, no permutation).  Groups of
// G lanes sort one stored column of at most G entries each ((row, position)
// keys in registers): G = 8 takes every column and lists the longer ones,
// G = 64 takes that list and lists the columns above 64 entries for
// k_sort_cols_block.  A sort is a chain of lane exchanges, so short groups
// and 32-bit keys (K = uint32_t: the row above log2(G) position bits, when
// the rows fit) keep the chain short.  Each group loads U columns before it
// sorts any of them, so the loads of U columns overlap.
constexpr int kColSortMax = 4096;  // longest column the plan sorts (LDS bitonic)

template <int G, int U, typename K>
__global__ void k_sort_cols_group(Operand A, const int32_t* row_agg, const int32_t* list_in,
                                  const unsigned long long* nlist_in, int32_t* ir_r, int64_t* perm, int32_t* list_out,
                                  unsigned long long* nlist_out) {
  constexpr int kPosBits = G == 8 ? 3 : (G == 16 ? 4 : (G == 32 ? 5 : 6));
  constexpr int kShift = sizeof(K) == 4 ? kPosBits : 32;
  const int gl = lane_id() & (G - 1);
  const int64_t n = list_in ? (int64_t)*nlist_in : nslots_of(A);
  const int64_t g0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int64_t ng = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t i = g0; i < n; i += U * ng) {
    int64_t t[U], a0[U], len[U];
    int32_t key_row[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t idx = i + u * ng;
      t[u] = idx < n ? (list_in ? (int64_t)list_in[idx] : idx) : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a0[u] = t[u] >= 0 ? slot_begin(A, t[u]) : 0;
      len[u] = t[u] >= 0 ? slot_begin(A, t[u] + 1) - a0[u] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) key_row[u] = gl < len[u] && len[u] <= G ? A.ir[a0[u] + gl] : 0;
    if (row_agg) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (gl < len[u] && len[u] <= G) key_row[u] = row_agg[key_row[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (t[u] < 0) continue;  // uniform in the group
      if (len[u] > G) {
        if (gl == 0) list_out[atomicAdd(nlist_out, 1ull)] = (int32_t)t[u];
        continue;
      }
      K key = gl < len[u] ? (K)(((K)(uint32_t)key_row[u] << kShift) | (K)gl) : ~(K)0;
#pragma unroll
      for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
          const K other = xor_lane(key, j);
          const bool up = (gl & k) == 0, lower = (gl & j) == 0;
          const K mn = other < key ? other : key, mx = other < key ? key : other;
          key = (lower == up) ? mn : mx;
        }
      }
      if (gl < len[u]) {
        ir_r[a0[u] + gl] = (int32_t)(key >> kShift);
        if (perm) perm[a0[u] + gl] = a0[u] + (int64_t)(key & (((K)1 << kShift) - 1));
      }
    }
  }
}

// Launches the group tiers over every column of A; columns longer than 64
// entries are listed in `longs` (count in nl[1]).  nl[0..1] must be zero.
// `max_row` bounds the sort keys' rows (exclusive).
static int sort_cols_groups(const Operand& A, const int32_t* row_agg, int64_t ns, int64_t max_row, int32_t* ir_r,
                            int64_t* perm, int32_t* mids, int32_t* longs, unsigned long long* nl, hipStream_t st) {
  const unsigned g8 = grid_for(ns * 8 / 2, 256, 65536);
  if (max_row <= (1ll << 29))
    k_sort_cols_group<8, 2, uint32_t><<<g8, 256, 0, st>>>(A, row_agg, nullptr, nullptr, ir_r, perm, mids, nl);
  else
    k_sort_cols_group<8, 2, uint64_t><<<g8, 256, 0, st>>>(A, row_agg, nullptr, nullptr, ir_r, perm, mids, nl);
  SPX_HIP(hipGetLastError());
  const unsigned g64 = (unsigned)device_cu_count() * 16;
  if (max_row <= (1ll << 26))
    k_sort_cols_group<kWave, 1, uint32_t><<<g64, 256, 0, st>>>(A, row_agg, mids, nl, ir_r, perm, longs, nl + 1);
  else
    k_sort_cols_group<kWave, 1, uint64_t><<<g64, 256, 0, st>>>(A, row_agg, mids, nl, ir_r, perm, longs, nl + 1);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

// Columns above kColSortMax entries are listed in `huge` (count *nhuge) for
// one global sort each, or, without a list, flagged in err (bit 8).
__global__ void __launch_bounds__(256) k_sort_cols_block(Operand A, const int32_t* row_agg, const int32_t* longs,
                                                         const unsigned long long* nlong, int32_t* ir_r, int64_t* perm,
                                                         unsigned* err, int32_t* huge, unsigned long long* nhuge) {
  __shared__ uint64_t s[kColSortMax];
  const int64_t nl = (int64_t)*nlong;
  for (int64_t i = blockIdx.x; i < nl; i += gridDim.x) {
    const int32_t t = longs[i];
    const int64_t a0 = slot_begin(A, t), a1 = slot_begin(A, t + 1);
    const int len = (int)(a1 - a0);
    if (a1 - a0 > kColSortMax) {  // uniform
      if (threadIdx.x == 0) {
        if (huge)
          huge[atomicAdd(nhuge, 1ull)] = t;
        else
          atomicOr(err, 8u);
      }
      continue;
    }
    int p2 = 1;
    while (p2 < len) p2 <<= 1;
    for (int j = threadIdx.x; j < p2; j += blockDim.x) {
      uint64_t key = ~0ull;
      if (j < len) {
        const int32_t r = A.ir[a0 + j];
        key = ((uint64_t)(uint32_t)(row_agg ? row_agg[r] : r) << 32) | (uint32_t)j;
      }
      s[j] = key;
    }
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int x = threadIdx.x; x < (p2 >> 1); x += blockDim.x) {
          const int lo = 2 * x - (x & (jj - 1));
          const int hi = lo + jj;
          const bool asc = (lo & k) == 0;
          const uint64_t a = s[lo], b = s[hi];
          if ((a > b) == asc) {
            s[lo] = b;
            s[hi] = a;
          }
        }
        __syncthreads();
      }
    }
    for (int j = threadIdx.x; j < len; j += blockDim.x) {
      ir_r[a0 + j] = (int32_t)(s[j] >> 32);
      if (perm) perm[a0 + j] = a0 + (int64_t)(uint32_t)s[j];
    }
    __syncthreads();
  }
}

// First position and length of each listed column.
__global__ void k_col_extents(Operand A, const int32_t* cols, int64_t n, int64_t* ext) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a0 = slot_begin(A, cols[i]);
    ext[2 * i] = a0;
    ext[2 * i + 1] = slot_begin(A, cols[i] + 1) - a0;
  }
}

// (mapped row, position) keys of one column, and their sorted order written
// back as the column's rows and value permutation.
__global__ void k_col_keys(const int32_t* ir, int64_t a0, int64_t len, const int32_t* row_agg, uint64_t* keys) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < len; j += (int64_t)gridDim.x * blockDim.x)
    keys[j] = ((uint64_t)(uint32_t)row_agg[ir[a0 + j]] << 32) | (uint32_t)j;
}
__global__ void k_col_unkey(const uint64_t* keys, int64_t a0, int64_t len, int32_t* ir_r, int64_t* perm) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < len; j += (int64_t)gridDim.x * blockDim.x) {
    ir_r[a0 + j] = (int32_t)(keys[j] >> 32);
    perm[a0 + j] = a0 + (int64_t)(uint32_t)keys[j];
  }
}

__global__ void k_gather_values(const int64_t* perm, int64_t n, const void* src, int vb, void* dst) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    if (vb == 8)
      static_cast<uint64_t*>(dst)[e] = static_cast<const uint64_t*>(src)[perm[e]];
    else
      static_cast<uint32_t*>(dst)[e] = static_cast<const uint32_t*>(src)[perm[e]];
  }
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
  const bool row_sorted = !(err_h & 2u);
  const bool col_sorted = !(cerr_h & 4u);

  // left operand: A with mapped rows (A's pointers and values)
  spx_mat Ar = *A;
  if (row_agg) {
    SPX_TRY(scr.get_n(std::max<int64_t>(A->nnz, 1), &P->air));
    if (row_sorted) {
      if (A->nnz > 0) {
        k_map_rows<<<grid_for(A->nnz, 256, 65536), 256, 0, st>>>(A->ir, A->nnz, row_agg, P->air);
        SPX_HIP(hipGetLastError());
      }
    } else if (A->nnz > 0) {
      // sort every column by mapped row; values follow through the permutation
      const Operand Ao = make_operand(A);
      const int64_t ns = nslots_of(Ao);
      int32_t *mids = nullptr, *longs = nullptr;
      unsigned long long* nl = nullptr;  // [0] columns above 8 entries, [1] above 64, [2] above 4096
      SPX_TRY(scr.get_n(std::max<int64_t>(A->nnz, 1), &P->aperm));
      SPX_TRY(scr.get_n(std::max<int64_t>(ns, 1), &mids));
      SPX_TRY(scr.get_n(std::max<int64_t>(ns, 1), &longs));
      SPX_TRY(scr.get_n(3, &nl));
      SPX_TRY(fill_i64(reinterpret_cast<int64_t*>(nl), 3, 0, st));
      SPX_TRY(sort_cols_groups(Ao, row_agg, ns, m_coarse, P->air, P->aperm, mids, longs, nl, st));
      // columns above the LDS sort: listed in mids (free again once the
      // 64-lane tier has run), then one global sort each
      int32_t* huge = mids;
      k_sort_cols_block<<<(unsigned)device_cu_count() * 4, 256, 0, st>>>(Ao, row_agg, longs, nl + 1, P->air, P->aperm,
                                                                        err, huge, nl + 2);
      SPX_HIP(hipGetLastError());
      unsigned long long nhuge = 0;
      SPX_HIP(hipMemcpyAsync(&nhuge, nl + 2, 8, hipMemcpyDeviceToHost, st));
      SPX_HIP(hipStreamSynchronize(st));
      if (nhuge > 0) {
        int64_t* ext = nullptr;
        SPX_TRY(scr.get_n(2 * (int64_t)nhuge, &ext));
        k_col_extents<<<grid_for((int64_t)nhuge, 256, 1024), 256, 0, st>>>(Ao, huge, (int64_t)nhuge, ext);
        SPX_HIP(hipGetLastError());
        std::vector<int64_t> ext_h(2 * nhuge);
        SPX_HIP(hipMemcpyAsync(ext_h.data(), ext, ext_h.size() * 8, hipMemcpyDeviceToHost, st));
        SPX_HIP(hipStreamSynchronize(st));
        int64_t maxlen = 0;
        for (size_t i = 0; i < nhuge; ++i) maxlen = std::max(maxlen, ext_h[2 * i + 1]);
        uint64_t* keys = nullptr;
        SPX_TRY(scr.get_n(sort_capacity(maxlen), &keys));
        for (size_t i = 0; i < nhuge; ++i) {
          const int64_t a0 = ext_h[2 * i], len = ext_h[2 * i + 1];
          k_col_keys<<<grid_for(len, 256, 4096), 256, 0, st>>>(A->ir, a0, len, row_agg, keys);
          SPX_HIP(hipGetLastError());
          SPX_TRY(sort_u64(keys, len, st));
          k_col_unkey<<<grid_for(len, 256, 4096), 256, 0, st>>>(keys, a0, len, P->air, P->aperm);
          SPX_HIP(hipGetLastError());
        }
      }
      P->vb = value_size(A->val_t);
      P->nnz = A->nnz;
      P->src_num = A->num;
      if (P->vb) {
        SPX_TRY(scr.get(A->nnz * P->vb, &P->anum));
        Ar.num = P->anum;
      }
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
      // counting scatter into the aggregates' columns, then each column sorted
      unsigned* cur = nullptr;
      int32_t *mids = nullptr, *longs = nullptr;
      unsigned long long* nl = nullptr;
      SPX_TRY(scr.get_n(std::max<int64_t>(n_coarse, 1), &cur));
      SPX_TRY(scr.get_n(std::max<int64_t>(n_coarse, 1), &mids));
      SPX_TRY(scr.get_n(std::max<int64_t>(n_coarse, 1), &longs));
      SPX_TRY(scr.get_n(2, &nl));
      SPX_TRY(fill_u32(cur, n_coarse, 0, st));
      SPX_TRY(fill_i64(reinterpret_cast<int64_t*>(nl), 2, 0, st));
      SPX_TRY(fill_u32(err, 1, 0, st));
      k_scatter_agg<<<grid_for(n, 256, 65536), 256, 0, st>>>(col_agg, n, P->scp, cur, P->sir);
      SPX_HIP(hipGetLastError());
      Operand So{};
      So.m = n;
      So.n = n_coarse;
      So.nnz = n;
      So.fmt = SPX_CSC;
      So.ptr_t = SPX_PTR_I64;
      So.val_t = SPX_VAL_BOOL;
      So.cp = P->scp;
      So.ir = P->sir;
      SPX_TRY(sort_cols_groups(So, nullptr, n_coarse, n, P->sir, nullptr, mids, longs, nl, st));
      k_sort_cols_block<<<(unsigned)device_cu_count() * 4, 256, 0, st>>>(So, nullptr, longs, nl + 1, P->sir, nullptr,
                                                                        err, nullptr, nullptr);
      SPX_HIP(hipGetLastError());
      SPX_HIP(hipMemcpyAsync(&err_h, err, 4, hipMemcpyDeviceToHost, st));
      SPX_HIP(hipStreamSynchronize(st));
      if (err_h & 8u) {  // an aggregate above 4096 vertices: one global sort of (aggregate, vertex) keys
        uint64_t* keys = nullptr;
        SPX_TRY(scr.get_n(sort_capacity(n), &keys));
        k_agg_keys<<<grid_for(n, 256, 65536), 256, 0, st>>>(col_agg, n, keys);
        SPX_HIP(hipGetLastError());
        SPX_TRY(sort_u64(keys, n, st));
        k_key_low<<<grid_for(n, 256, 65536), 256, 0, st>>>(keys, n, P->sir);
        SPX_HIP(hipGetLastError());
      }
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
  auto* P = static_cast<ContractPlan*>(plan);
  if (P->aperm && P->vb && P->nnz > 0) {  // A's current values in the sorted order
    k_gather_values<<<grid_for(P->nnz, 256, 65536), 256, 0, stream_of(&P->ctx)>>>(P->aperm, P->nnz, P->src_num,
                                                                                   P->vb, P->anum);
    SPX_HIP(hipGetLastError());
  }
  return spx_spgemm_exec(P->gemm, C);
}

namespace spx {
const spx_plan* contract_plan_inner(const spx_plan* plan) { return static_cast<const ContractPlan*>(plan)->gemm; }
}  // namespace spx
