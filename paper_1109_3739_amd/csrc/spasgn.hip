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
//
// Extend-add C = A + R B Q (Section 4.1: SpAsgn without the S A T term) is
// computed with the same column split.  Without the mask nothing of A is
// dropped; a repeated index lands several B entries on one position, where
// the semiring sum combines them.  Each modified column sorts its landing
// entries by (row, position in B), so a row's values are added to A's value
// in B's storage order.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "operand.h"
#include "plan.h"
#include "scan.h"

namespace spx {

constexpr int kAsgnMaxInsert = 4096;  // inserted rows per column handled in LDS; larger ("huge")
                                      // columns sort their keys in global memory
// Columns with at most this many inserted (landing) entries take one wave and
// a small LDS area; the others go to a list served by 256-thread workgroups.
constexpr int kAsgnSmall = 64;
// Extend-add: modified columns with more A entries than this have their A
// entries placed by the tiles (spread over the whole device) rather than by
// the one workgroup that handles the column.
constexpr int64_t kEaLongA = 1024;

// ---------------------------------------------------------------- helpers
// Pointers of a DCSC operand expanded to CSC (cp[j] = start of column j);
// rows and values stay the operand's.
__global__ void k_dcsc_to_csc_ptr(Operand X, int64_t* cp) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= X.n; j += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = X.nzc;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)X.jc[mid] < j)
        lo = mid + 1;
      else
        hi = mid;
    }
    cp[j] = slot_begin(X, lo);
  }
}

// The operand as CSC: a DCSC operand gets CSC pointers from `scr`.
int csc_view(const spx_mat* X, Scratch& scr, hipStream_t st, Operand* out) {
  *out = make_operand(X);
  if (X->fmt != SPX_DCSC) return SPX_OK;
  int64_t* cp = nullptr;
  SPX_TRY(scr.get_n(X->n + 1, &cp));
  k_dcsc_to_csc_ptr<<<grid_for(X->n + 1, 256, 65536), 256, 0, st>>>(*out, cp);
  SPX_HIP(hipGetLastError());
  out->fmt = SPX_CSC;
  out->ptr_t = SPX_PTR_I64;
  out->cp = cp;
  out->jc = nullptr;
  out->nzc = 0;
  return SPX_OK;
}

// Ascending bitonic sort of keys[0, p2) in global memory by the calling
// workgroup (p2 a power of two >= kAsgnMaxInsert; the caller pads past the
// keys with ~0).  Stages whose partner distance is below the LDS tile run in
// `tile` (kAsgnMaxInsert keys), the others over global memory.
__device__ void wg_sort_global(uint64_t* keys, int64_t p2, uint64_t* tile) {
  constexpr int64_t T = kAsgnMaxInsert;
  // whole tiles: every stage with k <= T, direction by the tile's position
  for (int64_t base = 0; base < p2; base += T) {
    for (int i = threadIdx.x; i < T; i += blockDim.x) tile[i] = keys[base + i];
    __syncthreads();
    for (int64_t k = 2; k <= T; k <<= 1) {
      for (int64_t j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < T / 2; i += blockDim.x) {
          const int lo = 2 * i - (i & (int)(j - 1));
          const int hi = lo + (int)j;
          const bool asc = ((base + lo) & k) == 0;
          const uint64_t x = tile[lo], y = tile[hi];
          if ((x > y) == asc) {
            tile[lo] = y;
            tile[hi] = x;
          }
        }
        __syncthreads();
      }
    }
    for (int i = threadIdx.x; i < T; i += blockDim.x) keys[base + i] = tile[i];
    __syncthreads();
  }
  for (int64_t k = 2 * T; k <= p2; k <<= 1) {
    for (int64_t j = k >> 1; j >= T; j >>= 1) {  // partners in different tiles
      __threadfence_block();
      for (int64_t i = threadIdx.x; i < p2 / 2; i += blockDim.x) {
        const int64_t lo = 2 * i - (i & (j - 1));
        const int64_t hi = lo + j;
        const bool asc = (lo & k) == 0;
        const uint64_t x = keys[lo], y = keys[hi];
        if ((x > y) == asc) {
          keys[lo] = y;
          keys[hi] = x;
        }
      }
      __threadfence_block();
      __syncthreads();
    }
    for (int64_t base = 0; base < p2; base += T) {  // the rest of merge step k inside each tile
      for (int i = threadIdx.x; i < T; i += blockDim.x) tile[i] = keys[base + i];
      __syncthreads();
      const bool asc = (base & k) == 0;
      for (int j = (int)T >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < T / 2; i += blockDim.x) {
          const int lo = 2 * i - (i & (j - 1));
          const int hi = lo + j;
          const uint64_t x = tile[lo], y = tile[hi];
          if ((x > y) == asc) {
            tile[lo] = y;
            tile[hi] = x;
          }
        }
        __syncthreads();
      }
      for (int i = threadIdx.x; i < T; i += blockDim.x) keys[base + i] = tile[i];
      __threadfence_block();
      __syncthreads();
    }
  }
}

// Extend-add's key segments: a huge column's as HugeCap; a long A column's
// (flag set) max(keys, 1); 0 for the others and past *len.
struct EaSeg {
  const int64_t* n;
  const int32_t* flag;
  const unsigned long long* len;
  __device__ int64_t operator()(int64_t w) const {
    if (w >= (int64_t)*len) return 0;
    const int64_t c = n[w];
    if (c > kAsgnMaxInsert) {
      int64_t p = kAsgnMaxInsert;
      while (p < c) p <<= 1;
      return p;
    }
    return flag[w] ? (c > 0 ? c : 1) : 0;
  }
};

// Smallest power of two >= max(n, kAsgnMaxInsert) for a huge column, 0 for others.
struct HugeCap {
  const int64_t* n;        // per list entry: its number of keys
  const int32_t* list;     // list entry -> index into n (NULL: identity)
  const unsigned long long* len;  // entries at or past *len count 0 (NULL: none)
  __device__ int64_t operator()(int64_t w) const {
    if (len && w >= (int64_t)*len) return 0;
    const int64_t c = n[list ? list[w] : w];
    if (c <= kAsgnMaxInsert) return 0;
    int64_t p = kAsgnMaxInsert;
    while (p < c) p <<= 1;
    return p;
  }
};

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
  int32_t* drows = nullptr;  // [ndrop] rows of the dropped entries, ascending per column
  int64_t* icnt = nullptr;   // [nmod] inserted entries per modified column
  int64_t* kbase = nullptr;  // [nmod] start of the column's B column (its keys sit at ikeys[kbase ..])
  uint64_t* ikeys = nullptr; // [nnz(B)] sorted (row, position in B's column) keys of the inserted entries
  int32_t* big = nullptr;    // modified columns (indices into mod) whose B column exceeds a wave
  unsigned long long* nbig_d = nullptr;
  int64_t nbig = 0;
  int64_t* hoff = nullptr;   // [nbig+1] key segment of each big column (0 length unless huge)
  uint64_t* hkeys = nullptr; // huge columns' padded key segments, sorted in place
  int64_t nhuge_keys = 0;
  int64_t* tmod = nullptr;    // [ntiles+1] modified columns before each tile (k_copy_tiles)
  int64_t ntiles = 0;
  int64_t* lastseg = nullptr; // [ntiles] dropped entries of each tile's last column
  int64_t* colb = nullptr;    // [nmod] A's entry range of each modified column
  int64_t* cole = nullptr;
  int64_t* runshift = nullptr;  // [nmod+1] output shift of the unmodified run before modified column u
  int64_t* mshift = nullptr;    // [nmod] off[j] - cp[j] of modified column u
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

// Unmodified columns keep their length (modified ones are counted later);
// *modent (when given) accumulates the entries of the modified columns.
__global__ void k_asgn_cols(Operand A, const int32_t* lastJ, int64_t* cnt, unsigned long long* modent) {
  int64_t mine = 0;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < A.n; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t len = slot_begin(A, j + 1) - slot_begin(A, j);
    const bool m = lastJ[j] >= 0;
    cnt[j] = m ? 0 : len;
    mine += m ? len : 0;
  }
  if (modent) {  // one atomic per workgroup
    __shared__ int64_t red[256 / kWave];
    mine = wave_sum(mine);
    if (lane_id() == 0) red[threadIdx.x / kWave] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t t = 0;
      for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += red[w];
      if (t) atomicAdd(modent, (unsigned long long)t);
    }
  }
}

// 1 for a column that receives B's entries.
struct LoadModified {
  const int32_t* lastJ;
  __device__ int64_t operator()(int64_t j) const { return lastJ[j] >= 0; }
};

// The modified columns in ascending order, compacted in place of a scan:
// block b of kScanTile columns starts at carry[b] (the scanned block counts
// of the modified flags; null for a single block), ranks its own flags with
// a block scan and writes its columns.  The last thread of the last block
// leaves the total in *nmod.  Items are taken kScanItems consecutive per
// thread, as by k_scan_apply.
__global__ void __launch_bounds__(kScanThreads) k_list_modified(const int32_t* lastJ, int64_t n, const int64_t* carry,
                                                                int32_t* mod, unsigned long long* nmod) {
  __shared__ int64_t red[kScanThreads / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  bool f[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    f[k] = base + k < n && lastJ[base + k] >= 0;
    s += f[k];
  }
  int64_t total;
  int64_t run = block_excl_scan(s, red, &total) + (carry ? carry[blockIdx.x] : 0);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (f[k]) mod[run++] = (int32_t)(base + k);
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == blockDim.x - 1) *nmod = (unsigned long long)run;
}

// Lists the modified columns and leaves their number in *nmod.
int list_modified(const Operand& A, const int32_t* lastJ, int64_t* cnt, int32_t* mod, unsigned long long* nmod,
                  unsigned long long* modent, Scratch& scr, hipStream_t st) {
  const int64_t n = A.n;
  if (n == 0) return fill_i64(reinterpret_cast<int64_t*>(nmod), 1, 0, st);
  k_asgn_cols<<<grid_for(n, 256, (int64_t)device_cu_count() * 4), 256, 0, st>>>(A, lastJ, cnt, modent);
  SPX_HIP(hipGetLastError());
  const int64_t nblocks = ceil_div(n, kScanTile);
  int64_t* carry = nullptr;
  if (nblocks > 1) {
    int64_t* sums = nullptr;
    SPX_TRY(scr.get_n(nblocks, &sums));
    SPX_TRY(scr.get_n(nblocks + 1, &carry));
    k_scan_reduce<LoadModified><<<(unsigned)nblocks, kScanThreads, 0, st>>>(LoadModified{lastJ}, n, sums);
    SPX_HIP(hipGetLastError());
    SPX_TRY(exclusive_scan(LoadI64{sums}, nblocks, carry, scr, st));
  }
  k_list_modified<<<(unsigned)nblocks, kScanThreads, 0, st>>>(lastJ, n, carry, mod, nmod);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

// Ascending bitonic sort of one 64-bit key per lane over the whole wave
// (every lane active), by lane exchanges.
__device__ __forceinline__ uint64_t wave_sort_u64(uint64_t key) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      const uint64_t other = xor_lane(key, jj);
      const bool up = (lane & k) == 0, lower = (lane & jj) == 0;
      const uint64_t mn = other < key ? other : key, mx = other < key ? key : other;
      key = lower == up ? mn : mx;
    }
  }
  return key;
}

// Ascending bitonic sort of s[0, n) in LDS (n <= kAsgnMaxInsert), padded with ~0.
__device__ __forceinline__ void lds_sort_keys(uint64_t* s, int n) {
  int p2 = 1;
  while (p2 < n) p2 <<= 1;
  for (int t = n + threadIdx.x; t < p2; t += blockDim.x) s[t] = ~0ull;
  __syncthreads();
  for (int k = 2; k <= p2; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int t = threadIdx.x; t < (p2 >> 1); t += blockDim.x) {
        const int lo = 2 * t - (t & (jj - 1));
        const int hi = lo + jj;
        const bool asc = (lo & k) == 0;
        const uint64_t x = s[lo], y = s[hi];
        if ((x > y) == asc) {
          s[lo] = y;
          s[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

// Number of rows < row in the sorted column col[0, len).
__device__ __forceinline__ int64_t rows_below(const int32_t* col, int64_t len, int32_t row) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[mid] < row)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Keys (row << 32 | position in B(:,q)) of a modified column's inserted
// entries (B entries whose row index is the last occurrence in I), in B's
// order, compacted by block scans; writes the first `cap` of them to
// `keys` and returns their number.  Called by the whole workgroup.
template <class KeyPtr>
__device__ __forceinline__ int64_t asgn_insert_keys(const Operand& B, const int32_t* I, const int32_t* lastI,
                                                    int64_t b0, int64_t b1, KeyPtr keys, int64_t cap,
                                                    int64_t* red) {
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
    if (take && nins + ex < cap) keys[nins + ex] = ((uint64_t)(uint32_t)row << 32) | (uint32_t)(e - b0);
    nins += tot;
  }
  return nins;
}

// --------------------------------------------------- merged-order tiles of A
// A's entries and the modified columns are processed together in one
// balanced order.  In A's storage order, modified column u is placed right
// after its last entry, at merged position end(u) + u with
// end(u) = cp[mod[u] + 1]; each workgroup takes kTileItems consecutive items
// of that merged order.  tmod[t] = the number of modified columns placed
// before item t * kTileItems, so tile t holds A's entries
// [t*T - tmod[t], (t+1)*T - tmod[t+1]) and meets modified columns tmod[t] ..
// tmod[t+1] (T = kTileItems): at most T + 1 of them, staged in LDS with
// their entry ranges relative to the tile.  An entry's staged index is the
// number of staged columns ending at or before it (a binary search in LDS):
// the entry lies inside that column when the column begins at or before
// it, else in the run of unmodified columns before it.
constexpr int kTileItems = 1024;
constexpr int kTileThreads = 256;
constexpr int kTilePer = kTileItems / kTileThreads;

// tmod[t] for t = 0..nt: modified column u owns the merged positions
// (end(u-1) + u - 1, end(u) + u], and the tile starts among them.  Also
// records each modified column's entry range [colb[u], cole[u]).
__global__ void k_copy_tiles(Operand A, const int32_t* mod, int64_t nmod, int64_t nt, int64_t* tmod, int64_t* colb,
                             int64_t* cole) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u <= nmod; u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t lo = u == 0 ? 0 : slot_begin(A, (int64_t)mod[u - 1] + 1) + u;
    int64_t hi = INT64_MAX;
    if (u < nmod) {
      const int64_t c = mod[u];
      const int64_t e = slot_begin(A, c + 1);
      colb[u] = slot_begin(A, c);
      cole[u] = e;
      hi = e + u;
    }
    for (int64_t t = (lo + kTileItems - 1) / kTileItems; t <= nt && t * kTileItems <= hi; ++t) tmod[t] = u;
  }
}

// Number of merged-order tiles of A with nmod modified columns.
inline int64_t tile_count(const Operand& A, int64_t nmod) { return ceil_div(A.nnz + nmod, (int64_t)kTileItems); }

// tmod[0..nt], colb and cole[0..nmod) are the caller's.
int copy_tiles(const Operand& A, const int32_t* mod, int64_t nmod, int64_t nt, int64_t* tmod, int64_t* colb,
               int64_t* cole, hipStream_t st) {
  k_copy_tiles<<<grid_for(nmod + 1, 256, 65536), 256, 0, st>>>(A, mod, nmod, nt, tmod, colb, cole);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

struct TileSpan {
  int64_t us, ue;  // modified columns tmod[t] .. tmod[t+1]
  int64_t es, ee;  // A's entries [es, ee)
  int32_t nst;     // staged columns us .. us + nst - 1 (those below nmod)
};

__device__ __forceinline__ TileSpan tile_span(const Operand& A, int64_t nmod, const int64_t* tmod, int64_t t) {
  TileSpan s;
  s.us = tmod[t];
  s.ue = tmod[t + 1];
  s.es = t * kTileItems - s.us;
  s.ee = std::min<int64_t>((t + 1) * kTileItems - s.ue, A.nnz);
  s.nst = (int32_t)(std::min<int64_t>(s.ue, nmod - 1) - s.us + 1);
  return s;
}


// Entry position relative to the tile, clamped to [0, kTileItems] (which
// keeps every comparison with an in-tile position).
__device__ __forceinline__ int32_t tile_rel(int64_t pos, int64_t es) {
  return (int32_t)std::min<int64_t>(std::max<int64_t>(pos - es, 0), kTileItems);
}

// Staged columns ending at or before in-tile position x.
template <typename P>
__device__ __forceinline__ int32_t staged_rank(const P* s_end, int32_t nst, int32_t x) {
  int32_t lo = 0, hi = nst;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (s_end[mid] <= x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// ------------------------------------------------ SpAsgn's modified columns
// An entry of A in modified column j is dropped when its row is in I, else
// kept.  Its kept rank in the column is its position there minus the
// dropped entries before it: the merged-order tile counts those among its
// own entries with a scan and, for a column begun in earlier tiles, adds
// their dropped counts of it (recorded per tile by the plan's count pass).
// A kept entry lands at off[j] + kept rank + the inserted rows below it (a
// binary search in the column's sorted inserted keys); a dropped one records
// its row at its rank in the column's list of dropped rows (ascending, as
// A's rows are).  The inserted entry of sorted rank s and row r lands at
// off[j] + s + (A's rows below r) - (dropped rows below r).

// Count pass over the tiles: dropped entries per modified column (dcnt,
// accumulated atomically, zero on entry) and, per tile, those of the last
// column it meets (lastseg; 0 when that column starts after the tile).
__global__ void __launch_bounds__(kTileThreads) k_asgn_drop_count(Operand A, const int32_t* lastI,
                                                                  const int64_t* colb, const int64_t* cole,
                                                                  int64_t nmod, const int64_t* tmod, int64_t nt,
                                                                  unsigned long long* dcnt, int64_t* lastseg) {
  __shared__ int32_t s_beg[kTileItems + 1];
  __shared__ int32_t s_end[kTileItems + 1];
  __shared__ int32_t s_cnt[kTileItems + 1];
  for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const TileSpan sp = tile_span(A, nmod, tmod, t);
    for (int32_t i = threadIdx.x; i < sp.nst; i += kTileThreads) {
      s_beg[i] = tile_rel(colb[sp.us + i], sp.es);
      s_end[i] = tile_rel(cole[sp.us + i], sp.es);
      s_cnt[i] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) {
      const int32_t x = threadIdx.x + k * kTileThreads;
      if (sp.es + x < sp.ee) {
        const int32_t lo = staged_rank(s_end, sp.nst, x);
        if (lo < sp.nst && s_beg[lo] <= x && lastI[A.ir[sp.es + x]] >= 0) atomicAdd(&s_cnt[lo], 1);
      }
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < sp.nst; i += kTileThreads)
      if (s_cnt[i]) atomicAdd(&dcnt[sp.us + i], (unsigned long long)s_cnt[i]);
    if (threadIdx.x == 0) lastseg[t] = sp.ue < nmod ? s_cnt[sp.ue - sp.us] : 0;
    __syncthreads();
  }
}

// Ascending bitonic sort of one 64-bit key per lane within each 16-lane
// group of the wave (every lane active).
__device__ __forceinline__ uint64_t group16_sort_u64(uint64_t key) {
  const int gl = lane_id() & 15;
#pragma unroll
  for (int k = 2; k <= 16; k <<= 1) {
#pragma unroll
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      const uint64_t other = xor_lane(key, jj);
      const bool up = (gl & k) == 0, lower = (gl & jj) == 0;
      const uint64_t mn = other < key ? other : key, mx = other < key ? key : other;
      key = lower == up ? mn : mx;
    }
  }
  return key;
}

// Per modified column: the inserted entries (B entries whose row index is
// the last occurrence in I), their count icnt, the column's output length
// cnt[j] = nnz(A(:,j)) - dropped + inserted, and B's column start kbase.
// A wave takes four columns at a time, one per 16-lane group: a B column of
// at most 16 entries has its keys (row << 32 | position in the B column)
// sorted within the group and stored at ikeys[kbase ..].  The others are
// then taken by the whole wave, one by one: up to 64 entries sorted across
// the wave, longer ones counted and put on the big list (sorted by
// k_asgn_big_keys or, past kAsgnMaxInsert, k_asgn_huge_keys).
__global__ void __launch_bounds__(256) k_asgn_keys(Operand A, Operand B, const int32_t* I, const int32_t* lastI,
                                                   const int32_t* lastJ, const int32_t* mod, int64_t nmod,
                                                   const unsigned long long* dcnt, int64_t* icnt, int64_t* kbase,
                                                   uint64_t* ikeys, int64_t* cnt, int32_t* big,
                                                   unsigned long long* nbig) {
  const int lane = lane_id(), g = lane >> 4, gl = lane & 15;
  const int64_t wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave));
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t base = wave * 4; base < nmod; base += nwaves * 4) {
    const int64_t u = base + g;
    const bool has = u < nmod;
    int32_t j = 0;
    int64_t b0 = 0, b1 = 0;
    if (has) {
      j = mod[u];
      const int32_t q = lastJ[j];
      b0 = slot_begin(B, q);
      b1 = slot_begin(B, q + 1);
    }
    const bool small = has && b1 - b0 <= 16;
    uint64_t key = ~0ull;
    if (small && gl < b1 - b0) {
      const int32_t p = B.ir[b0 + gl];
      const int32_t row = I[p];
      if (lastI[row] == p) key = ((uint64_t)(uint32_t)row << 32) | (uint32_t)gl;
    }
    const int ins_g = __popcll((__ballot(key != ~0ull) >> (g * 16)) & 0xffffull);
    key = group16_sort_u64(key);
    if (small) {
      if (gl < ins_g) ikeys[b0 + gl] = key;
      if (gl == 0) {
        icnt[u] = ins_g;
        kbase[u] = b0;
        cnt[j] = slot_begin(A, j + 1) - slot_begin(A, j) - (int64_t)dcnt[u] + ins_g;
      }
    }
    uint64_t rest = __ballot(has && !small && gl == 0);
    while (rest) {  // uniform
      const int64_t v = base + (__ffsll((unsigned long long)rest) - 1) / 16;
      rest &= rest - 1;
      const int32_t jv = mod[v];
      const int32_t q = lastJ[jv];
      const int64_t c0 = slot_begin(B, q), c1 = slot_begin(B, q + 1);
      int64_t ins = 0;
      if (c1 - c0 <= kWave) {
        uint64_t kv = ~0ull;
        if (lane < c1 - c0) {
          const int32_t p = B.ir[c0 + lane];
          const int32_t row = I[p];
          if (lastI[row] == p) kv = ((uint64_t)(uint32_t)row << 32) | (uint32_t)lane;
        }
        ins = __popcll(__ballot(kv != ~0ull));
        kv = wave_sort_u64(kv);
        if (lane < ins) ikeys[c0 + lane] = kv;
      } else {
        for (int64_t ec = c0; ec < c1; ec += kWave) {
          const int64_t e = ec + lane;
          bool take = false;
          if (e < c1) {
            const int32_t p = B.ir[e];
            take = lastI[I[p]] == p;
          }
          ins += __popcll(__ballot(take));
        }
      }
      if (lane == 0) {
        icnt[v] = ins;
        kbase[v] = c0;
        cnt[jv] = slot_begin(A, jv + 1) - slot_begin(A, jv) - (int64_t)dcnt[v] + ins;
        if (c1 - c0 > kWave) big[atomicAdd(nbig, 1ull)] = (int32_t)v;
      }
    }
  }
}

// Big-list columns with at most kAsgnMaxInsert inserted entries: keys
// compacted and sorted in LDS, then stored at ikeys[kbase ..].
__global__ void __launch_bounds__(256) k_asgn_big_keys(Operand B, const int32_t* I, const int32_t* lastI,
                                                       const int32_t* lastJ, const int32_t* mod, const int32_t* big,
                                                       int64_t nbig, const int64_t* icnt, uint64_t* ikeys) {
  __shared__ uint64_t s_key[kAsgnMaxInsert];
  __shared__ int64_t red[256 / kWave + 1];
  for (int64_t w = blockIdx.x; w < nbig; w += gridDim.x) {
    const int64_t u = big[w];
    if (icnt[u] > kAsgnMaxInsert) continue;  // uniform: a huge column
    const int32_t q = lastJ[mod[u]];
    const int64_t b0 = slot_begin(B, q);
    const int64_t nins = asgn_insert_keys(B, I, lastI, b0, slot_begin(B, q + 1), s_key, kAsgnMaxInsert, red);
    lds_sort_keys(s_key, (int)nins);
    for (int64_t s = threadIdx.x; s < nins; s += blockDim.x) ikeys[b0 + s] = s_key[s];
    __syncthreads();
  }
}

// Huge columns (more than kAsgnMaxInsert inserted rows), at plan time: each
// workgroup writes one column's keys into its segment of hkeys, pads the
// segment to its power-of-two length, sorts it in global memory and stores
// the sorted keys at ikeys[kbase ..].
__global__ void __launch_bounds__(256) k_asgn_huge_keys(Operand B, const int32_t* I, const int32_t* lastI,
                                                        const int32_t* lastJ, const int32_t* mod, const int32_t* big,
                                                        int64_t nbig, const int64_t* icnt, const int64_t* hoff,
                                                        uint64_t* hkeys, uint64_t* ikeys) {
  __shared__ uint64_t s_tile[kAsgnMaxInsert];
  __shared__ int64_t red[256 / kWave + 1];
  for (int64_t w = blockIdx.x; w < nbig; w += gridDim.x) {
    const int64_t p2 = hoff[w + 1] - hoff[w];
    if (p2 == 0) continue;  // uniform: not a huge column
    const int64_t u = big[w];
    const int32_t q = lastJ[mod[u]];
    const int64_t b0 = slot_begin(B, q);
    uint64_t* seg = hkeys + hoff[w];
    const int64_t nins = asgn_insert_keys(B, I, lastI, b0, slot_begin(B, q + 1), seg, p2, red);
    for (int64_t s = nins + threadIdx.x; s < p2; s += blockDim.x) seg[s] = ~0ull;
    __threadfence_block();
    __syncthreads();
    wg_sort_global(seg, p2, s_tile);
    for (int64_t s = threadIdx.x; s < nins; s += blockDim.x) ikeys[b0 + s] = seg[s];
    __syncthreads();
  }
}

// Output shifts for the fill tiles: runshift[u] = off[c0] - cp[c0] for the
// run of unmodified columns c0 = mod[u-1] + 1 .. mod[u] - 1, and
// mshift[u] = off[mod[u]] - cp[mod[u]].
__global__ void k_asgn_shifts(Operand A, const int32_t* mod, int64_t nmod, const int64_t* off, const int64_t* colb,
                              int64_t* runshift, int64_t* mshift) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u <= nmod; u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c0 = u == 0 ? 0 : (int64_t)mod[u - 1] + 1;
    runshift[u] = off[c0] - slot_begin(A, c0);
    if (u < nmod) mshift[u] = off[mod[u]] - colb[u];
  }
}

// Fill pass over the tiles: unmodified runs are copied with their output
// shift; entries of modified columns are kept or dropped as described above.
template <int VB>
__global__ void __launch_bounds__(kTileThreads) k_asgn_fill(Operand A, const int32_t* lastI, const int64_t* colb,
                                                            const int64_t* cole, const int64_t* runshift,
                                                            const int64_t* mshift, int64_t nmod, const int64_t* tmod,
                                                            int64_t nt, const int64_t* lastseg,
                                                            const int64_t* icnt, const int64_t* kbase,
                                                            const uint64_t* ikeys, const int64_t* doff,
                                                            int32_t* drows, int32_t* cir, void* cnum) {
  using V = typename std::conditional<VB == 8, uint64_t, uint32_t>::type;
  constexpr int kWaves = kTileThreads / kWave;
  __shared__ int16_t s_beg[kTileItems + 1];
  __shared__ int16_t s_end[kTileItems + 1];
  __shared__ int16_t s_dbase[kTileItems + 1];   // dropped entries of the tile before the column's first
  __shared__ int64_t s_shift[kTileItems + 1];   // output shift of the run before staged column i
  __shared__ int64_t s_mshift[kTileItems + 1];  // off[c] - cp[c] of staged column i
  __shared__ int32_t s_wt[kTilePer][kWaves];    // dropped entries per wave and round
  __shared__ int64_t s_red[kWaves];
  __shared__ int64_t s_a0;
  const V* anum = static_cast<const V*>(A.num);
  V* out = static_cast<V*>(cnum);
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const TileSpan sp = tile_span(A, nmod, tmod, t);
    for (int64_t i = threadIdx.x; i <= sp.ue - sp.us; i += kTileThreads) {
      const int64_t r = sp.us + i;
      s_shift[i] = runshift[r];
      if (i < sp.nst) {
        const int64_t cb = colb[r];
        s_beg[i] = (int16_t)tile_rel(cb, sp.es);
        s_end[i] = (int16_t)tile_rel(cole[r], sp.es);
        s_mshift[i] = mshift[r];
        if (i == 0) s_a0 = cb;
      }
    }
    __syncthreads();
    // dropped entries of the first staged column in the tiles before this one
    int64_t dprev = 0;
    if (sp.nst > 0 && s_a0 < sp.es) {  // uniform
      int64_t part = 0;
      for (int64_t tt = (s_a0 + sp.us) / kTileItems + threadIdx.x; tt < t; tt += kTileThreads) part += lastseg[tt];
      part = wave_sum(part);
      if (lane == 0) s_red[wid] = part;
      __syncthreads();
      for (int w = 0; w < kWaves; ++w) dprev += s_red[w];
    }
    int32_t lo[kTilePer], row[kTilePer], ex[kTilePer];
    bool inmod[kTilePer], drop[kTilePer];
    V val[kTilePer];
    int64_t nkey[kTilePer];
    const uint64_t* keys[kTilePer];
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) {
      const int32_t x = threadIdx.x + k * kTileThreads;
      const bool valid = sp.es + x < sp.ee;
      lo[k] = valid ? staged_rank(s_end, sp.nst, x) : 0;
      inmod[k] = valid && lo[k] < sp.nst && s_beg[lo[k]] <= x;
      row[k] = valid ? A.ir[sp.es + x] : -1;
      if (VB && valid) val[k] = anum[sp.es + x];
      nkey[k] = 0;
      keys[k] = ikeys;
      if (inmod[k]) {  // the column's inserted keys, for kept entries
        nkey[k] = icnt[sp.us + lo[k]];
        keys[k] = ikeys + kbase[sp.us + lo[k]];
      }
    }
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) {
      drop[k] = inmod[k] && lastI[row[k]] >= 0;
      const uint64_t m = __ballot(drop[k]);
      ex[k] = __popcll(m & lanemask_lt());
      if (lane == 0) s_wt[k][wid] = __popcll(m);
    }
    __syncthreads();
    int32_t base = 0;
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) {
      int32_t before = 0, tot = 0;
      for (int w = 0; w < kWaves; ++w) {
        before += w < wid ? s_wt[k][w] : 0;
        tot += s_wt[k][w];
      }
      ex[k] += base + before;  // dropped entries of the tile before this one
      base += tot;
      const int32_t x = threadIdx.x + k * kTileThreads;
      if (inmod[k] && x == s_beg[lo[k]]) s_dbase[lo[k]] = (int16_t)ex[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) {
      if (row[k] < 0) continue;
      const int64_t e = sp.es + threadIdx.x + k * kTileThreads;
      int64_t dst;
      if (!inmod[k]) {
        dst = e + s_shift[lo[k]];
      } else {
        const int64_t db = ex[k] - s_dbase[lo[k]] + (lo[k] == 0 ? dprev : 0);
        const int64_t u = sp.us + lo[k];
        if (drop[k]) {
          drows[doff[u] + db] = row[k];
          continue;
        }
        // inserted rows below this row
        int64_t a = 0, b = nkey[k];
        while (a < b) {
          const int64_t mid = (a + b) >> 1;
          if ((int32_t)(keys[k][mid] >> 32) < row[k])
            a = mid + 1;
          else
            b = mid;
        }
        dst = e + s_mshift[lo[k]] - db + a;
      }
      __builtin_nontemporal_store(row[k], &cir[dst]);  // C is written once: streaming stores
      if (VB) __builtin_nontemporal_store(val[k], &out[dst]);
    }
    __syncthreads();
  }
}

// One inserted entry: key of sorted rank s in modified column u.
__device__ __forceinline__ void asgn_insert_one(const Operand& A, const Operand& B, const int32_t* mod, int64_t u,
                                                int64_t s, const int64_t* kbase, const uint64_t* ikeys,
                                                const int64_t* off, const int64_t* doff, const int32_t* drows, int vb,
                                                int32_t* cir, void* cnum) {
  const int32_t j = mod[u];
  const int64_t a0 = slot_begin(A, j), alen = slot_begin(A, j + 1) - a0;
  const int64_t d0 = doff[u], dlen = doff[u + 1] - d0;
  const int64_t kb = kbase[u];
  const uint64_t key = ikeys[kb + s];
  const int32_t r = (int32_t)(key >> 32);
  const int64_t o = off[j] + s + rows_below(A.ir + a0, alen, r) - rows_below(drows + d0, dlen, r);
  cir[o] = r;
  copy_value(B.num, kb + (int64_t)(key & 0xffffffffu), cnum, o, vb);
}

// Inserted entries of the columns with at most 64: a wave takes four
// columns at a time, one per 16-lane group (lane s of the group takes the
// key of rank s); a column above 16 then takes the whole wave.
__global__ void __launch_bounds__(256) k_asgn_insert(Operand A, Operand B, const int32_t* mod, int64_t nmod,
                                                     const int64_t* icnt, const int64_t* kbase,
                                                     const uint64_t* ikeys, const int64_t* off, const int64_t* doff,
                                                     const int32_t* drows, int vb, int32_t* cir, void* cnum) {
  const int lane = lane_id(), g = lane >> 4, gl = lane & 15;
  const int64_t wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave));
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t base = wave * 4; base < nmod; base += nwaves * 4) {
    const int64_t u = base + g;
    const int64_t n = u < nmod ? icnt[u] : 0;
    if (n <= 16 && gl < n) asgn_insert_one(A, B, mod, u, gl, kbase, ikeys, off, doff, drows, vb, cir, cnum);
    uint64_t rest = __ballot(n > 16 && n <= kAsgnSmall && gl == 0);
    while (rest) {  // uniform
      const int64_t v = base + (__ffsll((unsigned long long)rest) - 1) / 16;
      rest &= rest - 1;
      if (lane < icnt[v]) asgn_insert_one(A, B, mod, v, lane, kbase, ikeys, off, doff, drows, vb, cir, cnum);
    }
  }
}

// Inserted entries of the big-list columns above 64: one workgroup each.
__global__ void __launch_bounds__(256) k_asgn_insert_big(Operand A, Operand B, const int32_t* mod, const int32_t* big,
                                                         int64_t nbig, const int64_t* icnt, const int64_t* kbase,
                                                         const uint64_t* ikeys, const int64_t* off,
                                                         const int64_t* doff, const int32_t* drows, int vb,
                                                         int32_t* cir, void* cnum) {
  for (int64_t w = blockIdx.x; w < nbig; w += gridDim.x) {
    const int64_t u = big[w];
    const int64_t n = icnt[u];
    if (n <= kAsgnSmall) continue;  // uniform: k_asgn_insert's column
    for (int64_t s = threadIdx.x; s < n; s += blockDim.x)
      asgn_insert_one(A, B, mod, u, s, kbase, ikeys, off, doff, drows, vb, cir, cnum);
  }
}

int launch_asgn_fill(const SpasgnPlan* P, int vb, int32_t* cir, void* cnum, hipStream_t st) {
  if (P->ntiles == 0) return SPX_OK;
  const unsigned grid = (unsigned)std::min<int64_t>(P->ntiles, (int64_t)device_cu_count() * 32);
#define SPX_ASGN_FILL(VB)                                                                                          \
  k_asgn_fill<VB><<<grid, kTileThreads, 0, st>>>(P->A, P->lastI, P->colb, P->cole, P->runshift, P->mshift,       \
                                                 P->nmod, P->tmod, P->ntiles, P->lastseg, P->icnt, P->kbase,      \
                                                 P->ikeys, P->doff, P->drows, cir, cnum)
  if (vb == 8)
    SPX_ASGN_FILL(8);
  else if (vb == 4)
    SPX_ASGN_FILL(4);
  else
    SPX_ASGN_FILL(0);
#undef SPX_ASGN_FILL
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

__global__ void k_asgn_write_cp(const int64_t* off, int64_t n, void* cp, int32_t ptr_t) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= n; j += (int64_t)gridDim.x * blockDim.x)
    store_ptr(cp, ptr_t, j, off[j]);
}

// ------------------------------------------------------------ extend-add
struct ExtAddPlan : spx_plan {
  explicit ExtAddPlan(const spx_ctx* c) : spx_plan(c, kPlanExtAdd) {}
  Operand A{}, B{};
  const int32_t* I = nullptr;
  int64_t lenI = 0, lenJ = 0, nnz = 0, nmod = 0;
  int32_t sr = 0;
  int32_t* lastJ = nullptr;  // [n] >= 0 for the columns that receive B entries
  int32_t* qcnt = nullptr;   // [n] number of q with J(q) = j
  int64_t* qoff = nullptr;   // [n+1]
  int32_t* qlist = nullptr;  // [lenJ] the q of each column, grouped by column
  int64_t* cnt = nullptr;    // [n]
  int64_t* off = nullptr;    // [n+1] = C.cp
  int32_t* mod = nullptr;    // [n] modified columns
  int32_t* rest = nullptr;   // modified columns (indices into mod) beyond k_ea_wave's reach
  unsigned long long* nrest_d = nullptr;
  int64_t nrest = 0;
  int32_t* big = nullptr;    // those above kAsgnSmall landing entries
  unsigned long long* nbig_d = nullptr;
  int64_t nbig = 0;
  int64_t* hcnt = nullptr;   // [nmod] per big-list entry: landing entries of a huge column, else 0
  int64_t* hoff = nullptr;   // [nmod+1] key segment of each big-list entry (0 length unless huge)
  uint64_t* hkeys = nullptr; // sorted (row, position in B) keys of the huge columns
  int32_t* hhead = nullptr;  // per segment column, hoff[w] + w .. : distinct-row heads
  int32_t* hnin = nullptr;   // and new-row counts
  int32_t* hlong = nullptr;  // [nmod] per big-list entry: 1 for a long A column (its A entries go to the tiles)
  int64_t* hnu = nullptr;    // [nmod] per segment column: distinct landing rows
  int32_t* lw = nullptr;     // [nmod] per modified column: its big-list entry if long, else -1
  int64_t nhuge_keys = 0;
  int64_t* tmod = nullptr;    // [ntiles+1] modified columns before each copy tile (k_copy_tiles)
  int64_t ntiles = 0;
  int64_t* colb = nullptr;    // [nmod] A's entry range of each modified column
  int64_t* cole = nullptr;
  unsigned* err = nullptr;
  unsigned long long* nmod_d = nullptr;
};

__global__ void k_check_range(const int32_t* v, int64_t len, int64_t bound, unsigned* err, unsigned bit) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < len; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = v[p];
    if (x < 0 || x >= bound) atomicOr(err, bit);
  }
}

__global__ void k_count_q(const int32_t* J, int64_t lenJ, int64_t n, int32_t* qcnt) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < lenJ; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = J[q];
    if (j >= 0 && j < n) atomicAdd(&qcnt[j], 1);
  }
}

// Groups the q by column (any order inside a group: the sort keys of the
// column kernel fix the order of the landing entries).  Leaves qcnt at zero.
__global__ void k_scatter_q(const int32_t* J, int64_t lenJ, const int64_t* qoff, int32_t* qcnt, int32_t* qlist) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < lenJ; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = J[q];
    qlist[qoff[j] + atomicSub(&qcnt[j], 1) - 1] = (int32_t)q;
  }
}

struct LoadI32 {
  const int32_t* p;
  __device__ int64_t operator()(int64_t i) const { return p[i]; }
};

// One modified column j of extend-add from its landing entries, given as
// keys (I(p) << 32 | e), e the entry's position in B, sorted ascending in
// `keys` (LDS or global), with scratch `head` and `nin` of nins + 1 entries:
//   1. the distinct rows are listed (first key of each) and looked up in A(:,j);
//   2. count pass: nnz(C(:,j)) = nnz(A(:,j)) + distinct rows not in A(:,j);
//      fill pass: A's entries move down by the new rows below them and add
//      the values landing on their row; each new row takes the sum of its
//      landing values.  Sums run in key order (B's storage order).
// Called by the whole workgroup.
template <bool kFill, bool kVals, typename T, class Acc, class KeyPtr, class IdxPtr>
__device__ __forceinline__ int64_t ea_column_body(const Operand& A, int32_t j, KeyPtr keys, int64_t nins,
                                                  IdxPtr head, IdxPtr nin, int64_t* red, int64_t* cnt,
                                                  const int64_t* off, const T* bnum, int32_t* cir, T* cnum,
                                                  bool skip_a = false) {
  const T* anum = static_cast<const T*>(A.num);
  const int64_t a0 = slot_begin(A, j), a1 = slot_begin(A, j + 1);
  const int32_t* acol = A.ir + a0;
  const int64_t alen = a1 - a0;
  // distinct rows
  int64_t nu = 0;
  for (int64_t tc = 0; tc < nins; tc += blockDim.x) {
    const int64_t t = tc + threadIdx.x;
    int64_t hd = 0;
    if (t < nins) hd = t == 0 || (keys[t] >> 32) != (keys[t - 1] >> 32);
    int64_t tot;
    const int64_t ex = block_excl_scan(hd, red, &tot);
    if (hd) head[nu + ex] = (int32_t)t;
    nu += tot;
  }
  if (threadIdx.x == 0) head[nu] = (int32_t)nins;
  __threadfence_block();
  __syncthreads();
  // which distinct rows A(:,j) lacks
  int64_t nnew = 0;
  for (int64_t kc = 0; kc < nu; kc += blockDim.x) {
    const int64_t k = kc + threadIdx.x;
    int64_t fresh = 0;
    if (k < nu) {
      const int32_t row = (int32_t)(keys[head[k]] >> 32);
      const int64_t at = rows_below(acol, alen, row);
      fresh = !(at < alen && acol[at] == row);
    }
    int64_t tot;
    const int64_t ex = block_excl_scan(fresh, red, &tot);
    if (k < nu) nin[k] = (int32_t)(nnew + ex);
    nnew += tot;
  }
  if (threadIdx.x == 0) nin[nu] = (int32_t)nnew;
  __threadfence_block();
  __syncthreads();
  if (!kFill) {
    if (threadIdx.x == 0) cnt[j] = alen + nnew;
    return nu;
  }
  const int64_t cbase = off[j];
  // A's entries (a long column's go through the tiles instead)
  for (int64_t t = skip_a ? alen : threadIdx.x; t < alen; t += blockDim.x) {
    const int32_t row = acol[t];
    int64_t lo = 0, hi = nu;  // distinct landing rows < row
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int32_t)(keys[head[mid]] >> 32) < row)
        lo = mid + 1;
      else
        hi = mid;
    }
    const int64_t o = cbase + t + nin[lo];
    cir[o] = row;
    if (kVals) {
      T acc = anum[a0 + t];
      if (lo < nu && (int32_t)(keys[head[lo]] >> 32) == row)
        for (int64_t h = head[lo]; h < head[lo + 1]; ++h) acc = Acc::add(acc, bnum[(uint32_t)keys[h]]);
      cnum[o] = acc;
    }
  }
  // new rows
  for (int64_t k = threadIdx.x; k < nu; k += blockDim.x) {
    if (nin[k + 1] == nin[k]) continue;  // A(:,j) stores this row
    const int32_t row = (int32_t)(keys[head[k]] >> 32);
    const int64_t o = cbase + nin[k] + rows_below(acol, alen, row);
    cir[o] = row;
    if (kVals) {
      T acc = bnum[(uint32_t)keys[head[k]]];
      for (int64_t h = head[k] + 1; h < head[k + 1]; ++h) acc = Acc::add(acc, bnum[(uint32_t)keys[h]]);
      cnum[o] = acc;
    }
  }
  __syncthreads();
  return nu;
}

// Keys (I(p) << 32 | e) of the entries of every B(:,q) with J(q) = j that
// land in column j, the first `cap` of them written to `keys`; returns their
// number.  Called by the whole workgroup.
template <class KeyPtr>
__device__ __forceinline__ int64_t ea_landing_keys(const Operand& B, const int32_t* I, int32_t j, const int64_t* qoff,
                                                   const int32_t* qlist, KeyPtr keys, int64_t cap) {
  int64_t nins = 0;
  for (int64_t t = qoff[j]; t < qoff[j + 1]; ++t) {
    const int32_t q = qlist[t];
    const int64_t b0 = slot_begin(B, q), b1 = slot_begin(B, q + 1);
    for (int64_t e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
      const int64_t slot = nins + (e - b0);
      if (slot < cap) keys[slot] = ((uint64_t)(uint32_t)I[B.ir[e]] << 32) | (uint32_t)e;
    }
    nins += b1 - b0;
  }
  return nins;
}

// One modified column of extend-add per group of G lanes (G = 16 or 64, the
// group aligned in the wave), done in registers: lane l of the group holds
// A(:,j)'s l-th entry and the l-th landing key (I(p) << 32 | e), the keys
// sorted within the group.  The first lane of each distinct landing row
// finds the row among A's (lane reads): its output position is A's rows
// below it plus the new rows below it, and it sums the row's landing values
// in key order onto A's value, or onto the first landing value for a new
// row.  A's entries that receive nothing move down by the new rows below
// them.  `keep` (per group) says whether the group's results are written:
// every lane runs the exchanges.  Count pass: nnz(C(:,j)); fill pass: the
// entries.
template <int G, bool kFill, bool kVals, typename T, class Acc>
__device__ __forceinline__ void ea_group_column(const Operand& A, const Operand& B, bool keep, int32_t j,
                                                int64_t a0, int alen, int nk, uint64_t key, int64_t* cnt,
                                                const int64_t* off, int32_t* cir, T* cnum) {
  const T* anum = static_cast<const T*>(A.num);
  const T* bnum = static_cast<const T*>(B.num);
  const int lane = lane_id();
  const int gl = lane & (G - 1), gb = lane & ~(G - 1);
  const uint64_t gbits = G == 64 ? ~0ull : ((1ull << G) - 1);
  const int32_t arow = gl < alen ? A.ir[a0 + gl] : 0x7fffffff;
  key = G == 64 ? wave_sort_u64(key) : group16_sort_u64(key);
  const int32_t krow = (int32_t)(key >> 32);  // lane gl < nk: the gl-th landing row
  const int32_t prev = __shfl(krow, gl == 0 ? lane : lane - 1);
  const bool head = gl < nk && (gl == 0 || prev != krow);
  int at = 0;  // A rows below krow
  bool found = false;
  for (int t = 0; t < (G == kWave ? alen : G); ++t) {  // the whole wave: a uniform bound and lane reads
    const int32_t r = G == kWave ? __builtin_amdgcn_readlane(arow, t) : __shfl(arow, gb + t);
    if (t < alen) {
      at += r < krow ? 1 : 0;
      found = found || r == krow;
    }
  }
  const uint64_t fm = (__ballot(head && !found) >> gb) & gbits;  // the group's new rows, bit gl
  if (!kFill) {
    if (keep && gl == 0) cnt[j] = alen + __popcll(fm);
    return;
  }
  const int64_t cbase = keep ? off[j] : 0;
  // A's entries that receive no landing value
  bool landed = false;
  int fbelow = 0;  // new rows below arow
  for (int t = 0; t < (G == kWave ? nk : G); ++t) {
    const int32_t r = G == kWave ? __builtin_amdgcn_readlane(krow, t) : __shfl(krow, gb + t);
    if (t < nk) {
      landed = landed || r == arow;
      fbelow += ((fm >> t) & 1ull) && r < arow ? 1 : 0;
    }
  }
  if (keep && gl < alen && !landed) {
    const int64_t o = cbase + gl + fbelow;
    cir[o] = arow;
    if (kVals) cnum[o] = anum[a0 + gl];
  }
  // one entry per distinct landing row
  const uint64_t hm = (__ballot(head) >> gb) & gbits;
  const uint64_t after = gl == G - 1 ? 0ull : hm >> (gl + 1);
  const int glen = head ? (after ? __ffsll((unsigned long long)after) : nk - gl) : 0;
  const uint64_t below = gl == 0 ? 0ull : (fm & ((1ull << gl) - 1));
  if (keep && head) cir[cbase + at + __popcll(below)] = krow;
  if (kVals) {
    const T bv = gl < nk ? bnum[(uint32_t)key] : T(0);
    T acc = found && keep ? anum[a0 + at] : bv;
    int gmax = glen;
    for (int s = 1; s < kWave; s <<= 1) gmax = max(gmax, __shfl_xor(gmax, s));
    for (int d = 0; d < gmax; ++d) {
      const T v = __shfl(bv, gb + ((gl + d) & (G - 1)));
      if (d < glen && (found || d > 0)) acc = Acc::add(acc, v);
    }
    if (keep && head) cnum[cbase + at + __popcll(below)] = acc;
  }
}

// Landing keys of column j for a group of G lanes: lane gl takes the gl-th
// landing entry (B columns q with J(q) = j, in list order); returns the
// number of landing entries (counting stops once above G).
template <int G>
__device__ __forceinline__ int64_t ea_group_keys(const Operand& B, const int32_t* I, const int32_t* qlist, int64_t q0,
                                                 int64_t q1, uint64_t* key) {
  const int gl = lane_id() & (G - 1);
  int64_t nins = 0;
  *key = ~0ull;
  for (int64_t t = q0; t < q1 && nins <= G; ++t) {
    const int32_t q = qlist[t];
    const int64_t b0 = slot_begin(B, q), len = slot_begin(B, q + 1) - b0;
    if (nins + len <= G && gl >= nins && gl < nins + len) {
      const int64_t e = b0 + (gl - nins);
      *key = ((uint64_t)(uint32_t)I[B.ir[e]] << 32) | (uint32_t)e;
    }
    nins += len;
  }
  return nins;
}

// Modified columns whose A column and landing entries fit in registers: a
// wave takes four columns at a time, one per 16-lane group; a column that
// does not fit 16 then takes the whole wave (64), and one that does not fit
// 64 goes, in the count pass, to the `rest` list for the LDS kernels (the
// fill pass skips it).
template <bool kFill, bool kVals, typename T, class Acc>
__global__ void __launch_bounds__(256) k_ea_wave(Operand A, Operand B, const int32_t* I, const int32_t* mod,
                                                 int64_t nmod, const int64_t* qoff, const int32_t* qlist,
                                                 int64_t* cnt, const int64_t* off, int32_t* rest,
                                                 unsigned long long* nrest, int32_t* cir, T* cnum) {
  const int lane = lane_id(), g = lane >> 4, gl = lane & 15;
  const int64_t wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave));
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t base = wave * 4; base < nmod; base += nwaves * 4) {
    const int64_t u = base + g;
    const bool has = u < nmod;
    int32_t j = 0;
    int64_t a0 = 0, a1 = 0, q0 = 0, q1 = 0;
    if (has) {
      j = mod[u];
      a0 = slot_begin(A, j);
      a1 = slot_begin(A, j + 1);
      q0 = qoff[j];
      q1 = qoff[j + 1];
    }
    uint64_t key;
    const int64_t nins = ea_group_keys<16>(B, I, qlist, q0, q1, &key);
    const bool small = has && a1 - a0 <= 16 && nins <= 16;
    ea_group_column<16, kFill, kVals, T, Acc>(A, B, small, j, a0, small ? (int)(a1 - a0) : 0,
                                             small ? (int)nins : 0, key, cnt, off, cir, cnum);
    uint64_t more = __ballot(has && !small && gl == 0);
    while (more) {  // uniform: the whole wave per remaining column
      const int64_t v = base + (__ffsll((unsigned long long)more) - 1) / 16;
      more &= more - 1;
      const int32_t jv = mod[v];
      const int64_t b0 = slot_begin(A, jv), b1 = slot_begin(A, jv + 1);
      uint64_t kv;
      const int64_t nv = ea_group_keys<kWave>(B, I, qlist, qoff[jv], qoff[jv + 1], &kv);
      if (b1 - b0 > kWave || nv > kWave) {  // uniform: an LDS kernel's column
        if (!kFill && lane == 0) rest[atomicAdd(nrest, 1ull)] = (int32_t)v;
        continue;
      }
      ea_group_column<kWave, kFill, kVals, T, Acc>(A, B, true, jv, b0, (int)(b1 - b0), (int)nv, kv, cnt, off, cir,
                                                  cnum);
    }
  }
}

// One workgroup per modified column j (grid-stride over the list) whose
// landing entries fit CAP and whose A column has at most kEaLongA entries:
// the keys are sorted in LDS, then ea_column_body.  The
// one-wave variant (CAP = kAsgnSmall) serves the rest list of k_ea_wave; in
// the count pass it hands larger columns to the `big` list, which the
// 256-thread variant (CAP = kAsgnMaxInsert) then serves (list lengths read
// from *nlist_d in the count pass); in its count pass that variant records, per list entry,
// the landing entries of a column above CAP or with a long A column in hcnt
// (0 for the others), and such ("segment") columns are done by k_ea_huge,
// with a long column's A entries left to the tiles (k_ea_tiles).
template <bool kFill, bool kVals, int CAP, typename T, class Acc>
__global__ void __launch_bounds__(256) k_ea_column(Operand A, Operand B, const int32_t* I, const int32_t* mod,
                                                   const int32_t* list, const unsigned long long* nlist_d,
                                                   int64_t nlist_h, const int64_t* qoff, const int32_t* qlist,
                                                   int64_t* cnt, const int64_t* off, int32_t* big,
                                                   unsigned long long* nbig, int64_t* hcnt, int32_t* hlong,
                                                   int32_t* lw, int32_t* cir, T* cnum) {
  __shared__ uint64_t s_key[CAP];
  __shared__ int32_t s_head[CAP + 1];  // sorted position of each distinct row's first key
  __shared__ int32_t s_nin[CAP + 1];   // distinct rows before k that A(:,j) lacks
  __shared__ int64_t red[256 / kWave + 1];
  const T* bnum = static_cast<const T*>(B.num);
  const int64_t nl = nlist_d ? (int64_t)*nlist_d : nlist_h;
  for (int64_t w = blockIdx.x; w < nl; w += gridDim.x) {
    const int64_t u = list ? list[w] : w;
    const int32_t j = mod[u];
    const bool long_a = slot_begin(A, j + 1) - slot_begin(A, j) > kEaLongA;
    const int64_t nins = ea_landing_keys(B, I, j, qoff, qlist, s_key, CAP);
    if (!kFill && CAP == kAsgnMaxInsert && threadIdx.x == 0) {
      hcnt[w] = nins > CAP || long_a ? nins : 0;
      hlong[w] = long_a ? 1 : 0;
      if (long_a) lw[u] = (int32_t)w;
    }
    if (nins > CAP || long_a) {  // uniform: a segment column (k_ea_huge), listed by the one-wave variant
      if (!kFill && CAP < kAsgnMaxInsert && threadIdx.x == 0) big[atomicAdd(nbig, 1ull)] = (int32_t)u;
      __syncthreads();
      continue;
    }
    lds_sort_keys(s_key, (int)nins);
    ea_column_body<kFill, kVals, T, Acc>(A, j, s_key, nins, s_head, s_nin, red, cnt, off, bnum, cir, cnum);
  }
}

// Segment columns, at plan time: each workgroup writes one column's keys
// into its segment of hkeys.  A huge column's (more than kAsgnMaxInsert
// landing entries) is padded to its power-of-two length and sorted in
// global memory; a long A column's fewer keys are sorted in LDS (segment of
// max(keys, 1) entries).
__global__ void __launch_bounds__(256) k_ea_huge_keys(Operand B, const int32_t* I, const int32_t* mod,
                                                      const int32_t* big, int64_t nbig, const int64_t* qoff,
                                                      const int32_t* qlist, const int64_t* hoff, uint64_t* hkeys) {
  __shared__ uint64_t s_tile[kAsgnMaxInsert];
  for (int64_t w = blockIdx.x; w < nbig; w += gridDim.x) {
    const int64_t p2 = hoff[w + 1] - hoff[w];
    if (p2 == 0) continue;  // uniform: not a segment column
    uint64_t* seg = hkeys + hoff[w];
    if (p2 < kAsgnMaxInsert) {  // a long A column's few keys: sorted in LDS
      const int64_t nins = ea_landing_keys(B, I, mod[big[w]], qoff, qlist, s_tile, kAsgnMaxInsert);
      __syncthreads();
      lds_sort_keys(s_tile, (int)nins);
      for (int64_t s = threadIdx.x; s < p2; s += blockDim.x) seg[s] = s_tile[s];
      __syncthreads();
      continue;
    }
    const int64_t nins = ea_landing_keys(B, I, mod[big[w]], qoff, qlist, seg, p2);
    for (int64_t s = nins + threadIdx.x; s < p2; s += blockDim.x) seg[s] = ~0ull;
    __threadfence_block();
    __syncthreads();
    wg_sort_global(seg, p2, s_tile);
  }
}

// Segment columns, count (plan) or fill (exec) pass: ea_column_body over
// the sorted global keys; head and nin take hoff[w] + w .. + p2 + 1 of
// hhead and hnin, and the count pass records the distinct rows in hnu.  The
// fill pass leaves a long A column's entries to the tiles.
template <bool kFill, bool kVals, typename T, class Acc>
__global__ void __launch_bounds__(256) k_ea_huge(Operand A, Operand B, const int32_t* mod, const int32_t* big,
                                                 int64_t nbig, const int64_t* hcnt, const int64_t* hoff,
                                                 const uint64_t* hkeys, int32_t* hhead, int32_t* hnin,
                                                 const int32_t* hlong, int64_t* hnu, int64_t* cnt,
                                                 const int64_t* off, int32_t* cir, T* cnum) {
  __shared__ int64_t red[256 / kWave + 1];
  const T* bnum = static_cast<const T*>(B.num);
  for (int64_t w = blockIdx.x; w < nbig; w += gridDim.x) {
    if (hoff[w + 1] == hoff[w]) continue;  // uniform: not a segment column
    const int64_t seg = hoff[w] + w;
    const int64_t nu = ea_column_body<kFill, kVals, T, Acc>(A, mod[big[w]], hkeys + hoff[w], hcnt[w], hhead + seg,
                                                            hnin + seg, red, cnt, off, bnum, cir, cnum,
                                                            kFill && hlong[w]);
    if (!kFill && threadIdx.x == 0) hnu[w] = nu;
  }
}

// Extend-add's tiles (the merged order above): an entry in the run before
// staged column i moves by that run's output shift; an entry of a long
// modified column (big-list entry lw[u] >= 0) keeps its place among A's
// rows and moves by the new rows below it, found in the column's sorted
// distinct landing rows (segment w: keys, heads, new-row counts), and adds
// the landing values of its own row in key order.  The other modified
// columns' entries are left to the column kernels.
template <bool kVals, typename T, class Acc>
__global__ void __launch_bounds__(kTileThreads) k_ea_tiles(Operand A, Operand B, const int32_t* mod, int64_t nmod,
                                                           const int64_t* tmod, int64_t nt, const int64_t* off,
                                                           const int32_t* lw, const int64_t* hoff,
                                                           const uint64_t* hkeys, const int32_t* hhead,
                                                           const int32_t* hnin, const int64_t* hnu, int32_t* cir,
                                                           T* cnum) {
  __shared__ int16_t s_beg[kTileItems + 1];
  __shared__ int16_t s_end[kTileItems + 1];
  __shared__ int32_t s_lw[kTileItems + 1];
  __shared__ int64_t s_shift[kTileItems + 1];  // output shift of the run before staged column i
  __shared__ int64_t s_mo[kTileItems + 1];     // off[c] - cp[c] of a long staged column
  const T* anum = static_cast<const T*>(A.num);
  const T* bnum = static_cast<const T*>(B.num);
  for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const TileSpan sp = tile_span(A, nmod, tmod, t);
    for (int64_t i = threadIdx.x; i <= sp.ue - sp.us; i += kTileThreads) {
      const int64_t r = sp.us + i;
      const int64_t c0 = r == 0 ? 0 : (int64_t)mod[r - 1] + 1;
      s_shift[i] = off[c0] - slot_begin(A, c0);
      if (i < sp.nst) {
        const int64_t c = mod[r];
        const int64_t cb = slot_begin(A, c);
        s_beg[i] = (int16_t)tile_rel(cb, sp.es);
        s_end[i] = (int16_t)tile_rel(slot_begin(A, c + 1), sp.es);
        s_lw[i] = lw[r];
        s_mo[i] = off[c] - cb;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) {
      const int32_t x = threadIdx.x + k * kTileThreads;
      const int64_t e = sp.es + x;
      if (e >= sp.ee) continue;
      const int32_t lo = staged_rank(s_end, sp.nst, x);
      const bool inmod = lo < sp.nst && s_beg[lo] <= x;
      if (!inmod) {
        const int64_t dst = e + s_shift[lo];
        __builtin_nontemporal_store(A.ir[e], &cir[dst]);  // C is written once: streaming stores
        if (kVals) __builtin_nontemporal_store(anum[e], &cnum[dst]);
        continue;
      }
      const int32_t w = s_lw[lo];
      if (w < 0) continue;  // a column kernel's entry
      const int32_t row = A.ir[e];
      const uint64_t* keys = hkeys + hoff[w];
      const int64_t seg = hoff[w] + w;
      const int32_t* head = hhead + seg;
      const int64_t nu = hnu[w];
      int64_t a = 0, b = nu;  // distinct landing rows below this row
      while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if ((int32_t)(keys[head[mid]] >> 32) < row)
          a = mid + 1;
        else
          b = mid;
      }
      const int64_t dst = e + s_mo[lo] + hnin[seg + a];
      cir[dst] = row;
      if (kVals) {
        T acc = anum[e];
        if (a < nu && (int32_t)(keys[head[a]] >> 32) == row)
          for (int64_t h = head[a]; h < head[a + 1]; ++h) acc = Acc::add(acc, bnum[(uint32_t)keys[h]]);
        cnum[dst] = acc;
      }
    }
    __syncthreads();
  }
}

// The register kernel over all modified columns, the one-wave LDS variant
// over the rest list, then the 256-thread variant over the big list (list
// lengths are on the device in the count pass; the fill pass knows them from
// the plan).  `huge`: the huge columns' kernel instead.
template <bool kFill, bool kVals, typename T, class Acc>
int launch_ea(const ExtAddPlan* P, int32_t* cir, void* cnum, hipStream_t st, bool huge) {
  const int cus = device_cu_count();
  T* out = static_cast<T*>(cnum);
  if (huge) {
    if (P->nhuge_keys > 0) {
      k_ea_huge<kFill, kVals, T, Acc><<<(unsigned)std::min<int64_t>(P->nbig, (int64_t)cus * 2), 256, 0, st>>>(
          P->A, P->B, P->mod, P->big, P->nbig, P->hcnt, P->hoff, P->hkeys, P->hhead, P->hnin, P->hlong, P->hnu,
          P->cnt, P->off, cir, out);
      SPX_HIP(hipGetLastError());
    }
    return SPX_OK;
  }
  if (kFill && P->ntiles > 0) {  // unmodified runs and the long columns' A entries
    k_ea_tiles<kVals, T, Acc><<<(unsigned)std::min<int64_t>(P->ntiles, (int64_t)cus * 32), kTileThreads, 0, st>>>(
        P->A, P->B, P->mod, P->nmod, P->tmod, P->ntiles, P->off, P->lw, P->hoff, P->hkeys, P->hhead, P->hnin, P->hnu,
        cir, out);
    SPX_HIP(hipGetLastError());
  }
  if (P->nmod == 0) return SPX_OK;
  k_ea_wave<kFill, kVals, T, Acc><<<(unsigned)std::min<int64_t>(ceil_div(P->nmod, (int64_t)16), (int64_t)cus * 16),
                                     256, 0, st>>>(P->A, P->B, P->I, P->mod, P->nmod, P->qoff, P->qlist, P->cnt,
                                                   P->off, P->rest, P->nrest_d, cir, out);
  SPX_HIP(hipGetLastError());
  if (!kFill || P->nrest > 0) {
    const int64_t grid = kFill ? std::min<int64_t>(P->nrest, (int64_t)cus * 32) : (int64_t)cus * 32;
    k_ea_column<kFill, kVals, kAsgnSmall, T, Acc><<<(unsigned)grid, 64, 0, st>>>(
        P->A, P->B, P->I, P->mod, P->rest, kFill ? nullptr : P->nrest_d, P->nrest, P->qoff, P->qlist, P->cnt,
        P->off, P->big, P->nbig_d, P->hcnt, P->hlong, P->lw, cir, out);
    SPX_HIP(hipGetLastError());
  }
  if (!kFill || P->nbig > 0) {
    const int64_t grid = kFill ? std::min<int64_t>(P->nbig, (int64_t)cus * 4) : (int64_t)cus * 4;
    k_ea_column<kFill, kVals, kAsgnMaxInsert, T, Acc><<<(unsigned)grid, 256, 0, st>>>(
        P->A, P->B, P->I, P->mod, P->big, kFill ? nullptr : P->nbig_d, P->nbig, P->qoff, P->qlist, P->cnt, P->off,
        P->big, P->nbig_d, P->hcnt, P->hlong, P->lw, cir, out);
    SPX_HIP(hipGetLastError());
  }
  return SPX_OK;
}

template <bool kFill>
int dispatch_ea(const ExtAddPlan* P, int32_t* cir, void* cnum, hipStream_t st, bool huge) {
  const int32_t vt = P->A.val_t;
  if (vt == SPX_VAL_BOOL || P->sr == SPX_OR_AND)
    return launch_ea<kFill, false, float, MinAcc<float>>(P, cir, nullptr, st, huge);
  const bool plus = P->sr == SPX_PLUS_TIMES;
  switch (vt) {
    case SPX_VAL_F32:
      return plus ? launch_ea<kFill, true, float, Semiring<SPX_PLUS_TIMES, float>>(P, cir, cnum, st, huge)
                  : launch_ea<kFill, true, float, MinAcc<float>>(P, cir, cnum, st, huge);
    case SPX_VAL_F64:
      return plus ? launch_ea<kFill, true, double, Semiring<SPX_PLUS_TIMES, double>>(P, cir, cnum, st, huge)
                  : launch_ea<kFill, true, double, MinAcc<double>>(P, cir, cnum, st, huge);
    default:
      return plus ? launch_ea<kFill, true, int64_t, Semiring<SPX_PLUS_TIMES, int64_t>>(P, cir, cnum, st, huge)
                  : launch_ea<kFill, true, int64_t, MinAcc<int64_t>>(P, cir, cnum, st, huge);
  }
}

}  // namespace spx

using namespace spx;

extern "C" int spx_spasgn_plan(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J,
                               int64_t lenJ, const spx_mat* B, spx_plan** plan, int64_t* nnz_c) {
  if (!plan) return fail(SPX_EINVAL, "plan is NULL");
  *plan = nullptr;
  SPX_TRY(check_mat(A, "A"));
  SPX_TRY(check_mat(B, "B"));
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
  SPX_TRY(csc_view(A, scr, st, &P->A));  // DCSC operands get CSC pointers
  SPX_TRY(csc_view(B, scr, st, &P->B));
  P->I = I;
  P->J = J;
  P->lenI = lenI;
  P->lenJ = lenJ;
  const int64_t m = A->m, n = A->n;
  const int cus = device_cu_count();
  SPX_TRY(scr.get_many({Scratch::part(&P->err, 4), Scratch::part(&P->nmod_d, 2), Scratch::part(&P->lastI, m),
                        Scratch::part(&P->lastJ, n), Scratch::part(&P->cnt, n), Scratch::part(&P->off, n + 1),
                        Scratch::part(&P->mod, n)}));
  SPX_TRY(fill_u32(P->err, 1, 0, st));
  SPX_TRY(fill_i64((int64_t*)P->nmod_d, 2, 0, st));  // modified columns, their entries
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
  SPX_TRY(list_modified(P->A, P->lastJ, P->cnt, P->mod, P->nmod_d, P->nmod_d + 1, scr, st));
  int64_t h1[3] = {0, 0, 0};
  SPX_TRY(read_device_words(st, {{P->nmod_d, 8}, {P->err, 4}, {P->nmod_d + 1, 8}}, h1));
  if (h1[1] & 1) return fail(SPX_EINVAL, "I has an index outside [0, m)");
  if (h1[1] & 2) return fail(SPX_EINVAL, "J has an index outside [0, n)");
  P->nmod = h1[0];
  const int64_t nm = P->nmod;
  P->ntiles = tile_count(P->A, nm);
  // dropped entries are at most the modified columns' entries
  SPX_TRY(scr.get_many({Scratch::part(&P->tmod, P->ntiles + 1), Scratch::part(&P->colb, nm),
                        Scratch::part(&P->cole, nm), Scratch::part(&P->drows, h1[2]),
                        Scratch::part(&P->dcnt, nm), Scratch::part(&P->lastseg, P->ntiles),
                        Scratch::part(&P->doff, nm + 1), Scratch::part(&P->icnt, nm), Scratch::part(&P->kbase, nm),
                        Scratch::part(&P->ikeys, P->B.nnz), Scratch::part(&P->big, nm),
                        Scratch::part(&P->hoff, nm + 1), Scratch::part(&P->nbig_d, 1),
                        Scratch::part(&P->runshift, nm + 1), Scratch::part(&P->mshift, nm)}));
  SPX_TRY(copy_tiles(P->A, P->mod, nm, P->ntiles, P->tmod, P->colb, P->cole, st));
  SPX_TRY(fill_i64(P->dcnt, P->nmod, 0, st));
  if (P->nmod > 0 && P->ntiles > 0) {
    k_asgn_drop_count<<<(unsigned)std::min<int64_t>(P->ntiles, (int64_t)cus * 32), kTileThreads, 0, st>>>(
        P->A, P->lastI, P->colb, P->cole, P->nmod, P->tmod, P->ntiles,
        reinterpret_cast<unsigned long long*>(P->dcnt), P->lastseg);
    SPX_HIP(hipGetLastError());
  }
  SPX_TRY(fill_i64((int64_t*)P->nbig_d, 1, 0, st));
  if (P->nmod > 0) {
    k_asgn_keys<<<(unsigned)std::min<int64_t>(ceil_div(P->nmod, (int64_t)16), (int64_t)cus * 16), 256, 0, st>>>(
        P->A, P->B, I, P->lastI, P->lastJ, P->mod, P->nmod, reinterpret_cast<const unsigned long long*>(P->dcnt),
        P->icnt, P->kbase, P->ikeys, P->cnt, P->big, P->nbig_d);
    SPX_HIP(hipGetLastError());
  }
  SPX_TRY(exclusive_scan(LoadI64{P->cnt}, n, P->off, scr, st));
  SPX_TRY(exclusive_scan(LoadI64{P->dcnt}, P->nmod, P->doff, scr, st));
  // key segments of the huge columns (big-list order; entries past nbig are empty)
  SPX_TRY(exclusive_scan(HugeCap{P->icnt, P->big, P->nbig_d}, P->nmod, P->hoff, scr, st));
  k_asgn_shifts<<<grid_for(P->nmod + 1, 256, 65536), 256, 0, st>>>(P->A, P->mod, P->nmod, P->off, P->colb,
                                                                   P->runshift, P->mshift);
  SPX_HIP(hipGetLastError());
  int64_t tail[4] = {0, 0, 0, 0};
  SPX_TRY(read_device_words(st, {{P->off + n, 8}, {P->doff + P->nmod, 8}, {P->nbig_d, 8}, {P->hoff + P->nmod, 8}},
                            tail));
  P->nnz = tail[0];
  P->ndrop = tail[1];
  P->nbig = tail[2];
  P->nhuge_keys = tail[3];
  if (P->nbig > 0) {
    k_asgn_big_keys<<<(unsigned)std::min<int64_t>(P->nbig, (int64_t)cus * 4), 256, 0, st>>>(
        P->B, I, P->lastI, P->lastJ, P->mod, P->big, P->nbig, P->icnt, P->ikeys);
    SPX_HIP(hipGetLastError());
  }
  if (P->nhuge_keys > 0) {
    SPX_TRY(scr.get_n(P->nhuge_keys, &P->hkeys));
    k_asgn_huge_keys<<<(unsigned)std::min<int64_t>(P->nbig, (int64_t)cus * 2), 256, 0, st>>>(
        P->B, I, P->lastI, P->lastJ, P->mod, P->big, P->nbig, P->icnt, P->hoff, P->hkeys, P->ikeys);
    SPX_HIP(hipGetLastError());
  }
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
  SPX_TRY(launch_asgn_fill(P, vb, C->ir, C->num, st));
  if (P->nmod > 0) {
    k_asgn_insert<<<(unsigned)std::min<int64_t>(ceil_div(P->nmod, (int64_t)16), (int64_t)cus * 16), 256, 0, st>>>(
        P->A, P->B, P->mod, P->nmod, P->icnt, P->kbase, P->ikeys, P->off, P->doff, P->drows, vb, C->ir, C->num);
    SPX_HIP(hipGetLastError());
  }
  if (P->nbig > 0) {
    k_asgn_insert_big<<<(unsigned)std::min<int64_t>(P->nbig, (int64_t)cus * 4), 256, 0, st>>>(
        P->A, P->B, P->mod, P->big, P->nbig, P->icnt, P->kbase, P->ikeys, P->off, P->doff, P->drows, vb, C->ir,
        C->num);
    SPX_HIP(hipGetLastError());
  }
  k_asgn_write_cp<<<grid_for(P->A.n + 1, 256, 65536), 256, 0, st>>>(P->off, P->A.n, C->cp, C->ptr_t);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

extern "C" int spx_extend_add_plan(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI,
                                   const int32_t* J, int64_t lenJ, const spx_mat* B, int32_t semiring,
                                   spx_plan** plan, int64_t* nnz_c) {
  if (!plan) return fail(SPX_EINVAL, "plan is NULL");
  *plan = nullptr;
  SPX_TRY(check_mat(A, "A"));
  SPX_TRY(check_mat(B, "B"));
  if (lenI < 0 || lenJ < 0 || lenI >= (1ll << 31) || lenJ >= (1ll << 31)) return fail(SPX_EINVAL, "bad index length");
  if (B->m != lenI || B->n != lenJ) return fail(SPX_EINVAL, "B must be lenI x lenJ");
  if (A->val_t != B->val_t) return fail(SPX_EINVAL, "A and B must have the same value type");
  if (semiring < SPX_PLUS_TIMES || semiring > SPX_SELECT1ST) return fail(SPX_EINVAL, "unknown semiring");
  if (semiring == SPX_OR_AND && A->val_t != SPX_VAL_BOOL)
    return fail(SPX_EUNSUPPORTED, "OR_AND extend-add takes pattern-only (BOOL) operands");
  if (B->nnz >= (1ll << 32)) return fail(SPX_EUNSUPPORTED, "nnz(B) must be below 2^32");
  if ((lenI > 0 && !I) || (lenJ > 0 && !J)) return fail(SPX_EINVAL, "index vector is NULL");
  if (ctx && ctx->validate) {
    int32_t ok = 0;
    SPX_TRY(spx_check(ctx, A, &ok));
    if (!ok) return fail(SPX_EINVAL, "A is not canonical");
    SPX_TRY(spx_check(ctx, B, &ok));
    if (!ok) return fail(SPX_EINVAL, "B is not canonical");
  }
  auto* P = new ExtAddPlan(ctx);
  std::unique_ptr<ExtAddPlan> guard(P);
  hipStream_t st = stream_of(ctx);
  Scratch& scr = P->scratch;
  SPX_TRY(csc_view(A, scr, st, &P->A));  // DCSC operands get CSC pointers
  SPX_TRY(csc_view(B, scr, st, &P->B));
  P->I = I;
  P->lenI = lenI;
  P->lenJ = lenJ;
  P->sr = semiring;
  const int64_t m = A->m, n = A->n;
  SPX_TRY(scr.get_many({Scratch::part(&P->err, 4), Scratch::part(&P->nmod_d, 1), Scratch::part(&P->lastJ, n),
                        Scratch::part(&P->qcnt, n), Scratch::part(&P->cnt, n), Scratch::part(&P->off, n + 1),
                        Scratch::part(&P->mod, n), Scratch::part(&P->qoff, n + 1),
                        Scratch::part(&P->qlist, lenJ)}));
  SPX_TRY(fill_u32(P->err, 1, 0, st));
  SPX_TRY(fill_i64((int64_t*)P->nmod_d, 1, 0, st));
  SPX_TRY(fill_u32((uint32_t*)P->lastJ, n, 0xffffffffu, st));
  SPX_TRY(fill_u32((uint32_t*)P->qcnt, n, 0u, st));
  if (lenI > 0) {
    k_check_range<<<grid_for(lenI, 256, 4096), 256, 0, st>>>(I, lenI, m, P->err, 1u);
    SPX_HIP(hipGetLastError());
  }
  if (lenJ > 0) {
    k_last_occ<<<grid_for(lenJ, 256, 4096), 256, 0, st>>>(J, lenJ, n, P->lastJ, P->err, 2u);
    SPX_HIP(hipGetLastError());
    k_count_q<<<grid_for(lenJ, 256, 4096), 256, 0, st>>>(J, lenJ, n, P->qcnt);
    SPX_HIP(hipGetLastError());
  }
  SPX_TRY(list_modified(P->A, P->lastJ, P->cnt, P->mod, P->nmod_d, nullptr, scr, st));
  int64_t h1[2] = {0, 0};
  SPX_TRY(read_device_words(st, {{P->nmod_d, 8}, {P->err, 4}}, h1));
  if (h1[1] & 1) return fail(SPX_EINVAL, "I has an index outside [0, m)");
  if (h1[1] & 2) return fail(SPX_EINVAL, "J has an index outside [0, n)");
  P->nmod = h1[0];
  P->ntiles = tile_count(P->A, P->nmod);
  SPX_TRY(scr.get_many({Scratch::part(&P->tmod, P->ntiles + 1), Scratch::part(&P->colb, P->nmod),
                        Scratch::part(&P->cole, P->nmod)}));
  SPX_TRY(copy_tiles(P->A, P->mod, P->nmod, P->ntiles, P->tmod, P->colb, P->cole, st));
  SPX_TRY(exclusive_scan(LoadI32{P->qcnt}, n, P->qoff, scr, st));
  if (lenJ > 0) {
    k_scatter_q<<<grid_for(lenJ, 256, 4096), 256, 0, st>>>(J, lenJ, P->qoff, P->qcnt, P->qlist);
    SPX_HIP(hipGetLastError());
  }
  SPX_TRY(scr.get_many({Scratch::part(&P->rest, P->nmod), Scratch::part(&P->big, P->nmod),
                        Scratch::part(&P->hcnt, P->nmod), Scratch::part(&P->hoff, P->nmod + 1),
                        Scratch::part(&P->nbig_d, 2), Scratch::part(&P->hlong, P->nmod),
                        Scratch::part(&P->lw, P->nmod)}));
  SPX_TRY(fill_u32(reinterpret_cast<uint32_t*>(P->lw), P->nmod, 0xffffffffu, st));
  P->nrest_d = P->nbig_d + 1;
  SPX_TRY(fill_i64((int64_t*)P->nbig_d, 2, 0, st));
  if (P->nmod > 0) SPX_TRY(dispatch_ea<false>(P, nullptr, nullptr, st, false));
  // key segments of the huge columns (big-list order; entries past nbig are empty)
  SPX_TRY(exclusive_scan(EaSeg{P->hcnt, P->hlong, P->nbig_d}, P->nmod, P->hoff, scr, st));
  {
    int64_t h[3] = {0, 0, 0};
    SPX_TRY(read_device_words(st, {{P->nbig_d, 8}, {P->nbig_d + 1, 8}, {P->hoff + P->nmod, 8}}, h));
    P->nbig = h[0];
    P->nrest = h[1];
    P->nhuge_keys = h[2];
  }
  if (P->nhuge_keys > 0) {
    if (P->nhuge_keys >= (1ll << 31)) return fail(SPX_EUNSUPPORTED, "landing entries of the large columns exceed 2^31");
    SPX_TRY(scr.get_many({Scratch::part(&P->hkeys, P->nhuge_keys), Scratch::part(&P->hhead, P->nhuge_keys + P->nbig),
                          Scratch::part(&P->hnin, P->nhuge_keys + P->nbig), Scratch::part(&P->hnu, P->nbig)}));
    const int cus = device_cu_count();
    k_ea_huge_keys<<<(unsigned)std::min<int64_t>(P->nbig, (int64_t)cus * 2), 256, 0, st>>>(
        P->B, I, P->mod, P->big, P->nbig, P->qoff, P->qlist, P->hoff, P->hkeys);
    SPX_HIP(hipGetLastError());
    SPX_TRY(dispatch_ea<false>(P, nullptr, nullptr, st, true));
  }
  SPX_TRY(exclusive_scan(LoadI64{P->cnt}, n, P->off, scr, st));
  int64_t total = 0;
  SPX_TRY(read_device_words(st, {{P->off + n, 8}}, &total));
  P->nnz = total;
  if (nnz_c) *nnz_c = P->nnz;
  *plan = guard.release();
  return SPX_OK;
}

extern "C" int spx_extend_add_exec(spx_plan* plan, spx_mat* C) {
  if (!plan || plan->kind != kPlanExtAdd) return fail(SPX_EINVAL, "not an extend-add plan");
  auto* P = static_cast<ExtAddPlan*>(plan);
  if (!C) return fail(SPX_EINVAL, "C is NULL");
  if (C->m != P->A.m || C->n != P->A.n || C->fmt != SPX_CSC) return fail(SPX_EINVAL, "C must be m x n CSC");
  if (C->val_t != P->A.val_t) return fail(SPX_EINVAL, "C's value type must be A's");
  if (C->ptr_t == SPX_PTR_I32 && P->nnz >= (1ll << 31)) return fail(SPX_EOVERFLOW, "nnz(C) needs I64 pointers");
  if (!C->cp || (P->nnz > 0 && (!C->ir || (C->val_t != SPX_VAL_BOOL && !C->num))))
    return fail(SPX_EINVAL, "C buffers missing");
  C->nnz = P->nnz;
  C->nzc = 0;
  hipStream_t st = stream_of(&P->ctx);
  SPX_TRY(dispatch_ea<true>(P, C->ir, C->num, st, false));  // tiles, then the column kernels
  if (P->nmod > 0) SPX_TRY(dispatch_ea<true>(P, C->ir, C->num, st, true));
  k_asgn_write_cp<<<grid_for(P->A.n + 1, 256, 65536), 256, 0, st>>>(P->off, P->A.n, C->cp, C->ptr_t);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

// One-shot forms: plan, output buffers from ctx->alloc, exec, plan destroyed.
static int one_shot_csc(const spx_ctx* ctx, spx_plan* plan, int64_t nnz, const spx_mat* A,
                        int (*exec)(spx_plan*, spx_mat*), spx_mat* C) {
  std::unique_ptr<spx_plan> guard(plan);
  OutAlloc oa(ctx);
  spx_mat out{};
  out.m = A->m;
  out.n = A->n;
  out.fmt = SPX_CSC;
  out.ptr_t = SPX_PTR_I64;
  out.val_t = A->val_t;
  const int vb = value_size(A->val_t);
  SPX_TRY(oa.get((size_t)(A->n + 1) * 8, &out.cp));
  SPX_TRY(oa.get((size_t)std::max<int64_t>(nnz, 1) * 4, reinterpret_cast<void**>(&out.ir)));
  if (vb) SPX_TRY(oa.get((size_t)std::max<int64_t>(nnz, 1) * vb, &out.num));
  SPX_TRY(exec(plan, &out));
  oa.keep();
  *C = out;
  return SPX_OK;
}

extern "C" int spx_spasgn(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J,
                          int64_t lenJ, const spx_mat* B, spx_mat* C) {
  if (!C) return fail(SPX_EINVAL, "C is NULL");
  spx_plan* plan = nullptr;
  int64_t nnz = 0;
  SPX_TRY(spx_spasgn_plan(ctx, A, I, lenI, J, lenJ, B, &plan, &nnz));
  return one_shot_csc(ctx, plan, nnz, A, spx_spasgn_exec, C);
}

extern "C" int spx_extend_add(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J,
                              int64_t lenJ, const spx_mat* B, int32_t semiring, spx_mat* C) {
  if (!C) return fail(SPX_EINVAL, "C is NULL");
  spx_plan* plan = nullptr;
  int64_t nnz = 0;
  SPX_TRY(spx_extend_add_plan(ctx, A, I, lenI, J, lenJ, B, semiring, &plan, &nnz));
  return one_shot_csc(ctx, plan, nnz, A, spx_extend_add_exec, C);
}
