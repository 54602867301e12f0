// SpRef B = A(I,J) (Section 4) as the selection-matrix product R*A*Q, with
// R = sparse(1:len(I), I, 1) and Q = sparse(J, 1:len(J), 1).
//
// The product is evaluated right to left, R*(A*Q), and fused:
//   * A*Q: column q of A*Q is column J(q) of A (Q has one nonzero per column),
//     so it is a gather of A's columns -- no arithmetic;
//   * R*(AQ): R has one nonzero per row, so every entry (i, v) of column q
//     is copied to the rows p with I(p) = i.  The transpose of R in
//     compressed form (for each row index i the ascending list of p with
//     I(p) = i) is built once by sorting the pairs (I(p), p).
// Every output entry receives exactly one product (flops(R*A) = nnz(R*A)),
// so there is no semiring addition and the values are copied bit for bit.
// Rows of each output column are put in ascending p order by a wave-wide
// sort (<= 64 entries), an LDS bitonic sort (<= 4096), or, for longer
// columns, by scanning p in order and probing A(:,J(q)) by binary search.
#include <algorithm>

#include "common.h"
#include "operand.h"
#include "plan.h"
#include "scan.h"

namespace spx {

constexpr int kRefSmall = 64;
constexpr int kRefMedium = 4096;
enum { kClsEmpty = 0, kClsSmall = 1, kClsMedium = 2, kClsLarge = 3, kNumCls = 4 };

struct SprefPlan : spx_plan {
  explicit SprefPlan(const spx_ctx* c) : spx_plan(c, kPlanSpref) {}
  Operand A{};
  const int32_t* I = nullptr;
  const int32_t* J = nullptr;
  int64_t lenI = 0, lenJ = 0, nnz = 0;
  int64_t* rptr = nullptr;   // [m+1] start of row index i in rpos
  int32_t* rpos = nullptr;   // [lenI] positions p grouped by I(p), ascending
  int64_t* qa0 = nullptr;    // [lenJ] start of A(:,J(q))
  int32_t* qlen = nullptr;   // [lenJ] its length
  int64_t* cnt = nullptr;    // [lenJ] nnz(B(:,q))
  int64_t* off = nullptr;    // [lenJ+1]
  int32_t* list = nullptr;   // [lenJ] columns grouped by class
  int64_t* clsoff = nullptr; // [kNumCls+1]
  int64_t clsoff_h[kNumCls + 1] = {};
  int64_t nwide = 0;         // columns gathering more than kRefWide entries of A
  int32_t* wide = nullptr;   // [lenJ] those columns (the first nwide entries)
  unsigned* err = nullptr;
};

// Range checks of I (against m, error bit 1) and J (against n, bit 2) in one pass.
__global__ void k_check_index(const int32_t* I, int64_t lenI, int64_t m, const int32_t* J, int64_t lenJ, int64_t n,
                              unsigned* err) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < lenI + lenJ;
       x += (int64_t)gridDim.x * blockDim.x) {
    const bool in_i = x < lenI;
    const int32_t v = in_i ? I[x] : J[x - lenI];
    if (v < 0 || v >= (in_i ? m : n)) atomicOr(err, in_i ? 1u : 2u);
  }
}

__global__ void k_row_hist(const int32_t* I, int64_t lenI, int64_t m, unsigned* rcnt) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < lenI; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = I[p];
    if (i >= 0 && i < m) atomicAdd(&rcnt[i], 1u);
  }
}

struct LoadU32 {
  const unsigned* p;
  __device__ int64_t operator()(int64_t i) const { return (int64_t)p[i]; }
};

// Transpose of R: the positions p of each row index i = I(p), ascending,
// at rpos[rptr[i] ..].  A counting scatter fills each row's slots in any
// order (its count in rcnt runs down to zero), then every row sorts its
// own slots: rows of at most kRowShort positions by one thread in place,
// longer ones by a workgroup (LDS bitonic sort up to kRowLds positions,
// else one ordered pass over I that keeps the positions of that row).
constexpr int64_t kRowShort = 16;
constexpr int kRowLds = 4096;

__global__ void k_scatter_rows(const int32_t* I, int64_t lenI, int64_t m, const int64_t* rptr, unsigned* rcnt,
                               int32_t* rpos) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < lenI; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = I[p];
    if (i >= 0 && i < m) rpos[rptr[i] + atomicSub(&rcnt[i], 1u) - 1] = (int32_t)p;
  }
}

__global__ void k_sort_rows(const int64_t* rptr, int64_t m, int32_t* rpos, int32_t* longs,
                            unsigned long long* nlong) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r0 = rptr[i], r1 = rptr[i + 1];
    if (r1 - r0 > kRowShort) {
      longs[atomicAdd(nlong, 1ull)] = (int32_t)i;
      continue;
    }
    for (int64_t a = r0 + 1; a < r1; ++a) {  // insertion sort
      const int32_t x = rpos[a];
      int64_t b = a - 1;
      while (b >= r0 && rpos[b] > x) {
        rpos[b + 1] = rpos[b];
        --b;
      }
      rpos[b + 1] = x;
    }
  }
}

__global__ void __launch_bounds__(256) k_sort_long_rows(const int32_t* I, int64_t lenI, const int64_t* rptr,
                                                        const int32_t* longs, const unsigned long long* nlong,
                                                        int32_t* rpos) {
  __shared__ uint32_t s[kRowLds];
  __shared__ int64_t red[256 / kWave + 1];
  const int64_t n = (int64_t)*nlong;
  for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
    const int32_t i = longs[w];
    const int64_t r0 = rptr[i], len = rptr[i + 1] - r0;
    if (len <= kRowLds) {  // uniform
      int p2 = 1;
      while (p2 < len) p2 <<= 1;
      for (int t = threadIdx.x; t < p2; t += blockDim.x) s[t] = t < len ? (uint32_t)rpos[r0 + t] : 0xffffffffu;
      __syncthreads();
      for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
          for (int t = threadIdx.x; t < (p2 >> 1); t += blockDim.x) {
            const int lo = 2 * t - (t & (j - 1));
            const int hi = lo + j;
            const bool asc = (lo & k) == 0;
            const uint32_t x = s[lo], y = s[hi];
            if ((x > y) == asc) {
              s[lo] = y;
              s[hi] = x;
            }
          }
          __syncthreads();
        }
      }
      for (int t = threadIdx.x; t < len; t += blockDim.x) rpos[r0 + t] = (int32_t)s[t];
      __syncthreads();
    } else {
      int64_t run = 0;
      for (int64_t pc = 0; pc < lenI; pc += blockDim.x) {
        const int64_t p = pc + threadIdx.x;
        const int64_t f = p < lenI && I[p] == i;
        int64_t tot;
        const int64_t ex = block_excl_scan(f, red, &tot);
        if (f) rpos[r0 + run + ex] = (int32_t)p;
        run += tot;
      }
    }
  }
}

// Columns gathering more entries of A than this are counted (and, with at
// most kRefMedium outputs, extracted) by 1024-thread workgroups, so that a
// hub column of A is not left to one wave or one small workgroup.
constexpr int32_t kRefWide = 4096;

// Where each gathered column A(:,J(q)) starts and how long it is; columns
// longer than kRefWide are also appended to the wide list.
__global__ void k_col_info(Operand A, const int64_t* aux, int64_t chunk, const int32_t* J, int64_t lenJ, int64_t* qa0,
                           int32_t* qlen, int32_t* wide, unsigned long long* nwide) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < lenJ; q += (int64_t)gridDim.x * blockDim.x) {
    int64_t a0 = 0, a1 = 0;
    const int32_t k = J[q];
    if (k >= 0 && k < A.n) column_range(A, aux, chunk, k, a0, a1);
    qa0[q] = a0;
    qlen[q] = (int32_t)(a1 - a0);
    if (a1 - a0 > kRefWide) wide[atomicAdd(nwide, 1ull)] = (int32_t)q;
  }
}

// nnz(B(:,q)) = sum over the entries (i, v) of A(:,J(q)) of |{p : I(p) = i}|;
// one wave per column.  Also classifies the column.

// Output class of a column with s outputs gathering al entries of A (a wide
// column with few outputs still goes to the workgroup path).
__device__ __forceinline__ int ref_class(int64_t s, int32_t al) {
  return s == 0 ? kClsEmpty : (s <= kRefSmall && al <= kRefWide) ? kClsSmall : s <= kRefMedium ? kClsMedium : kClsLarge;
}

__global__ void k_ref_count(const Operand A, const int64_t* qa0, const int32_t* qlen, const int64_t* rptr, int64_t lenJ,
                            int64_t* cnt, unsigned long long* clscount) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  unsigned long long n0 = 0, n1 = 0, n2 = 0, n3 = 0;  // class counts of this wave's columns
  for (int64_t q = wave; q < lenJ; q += nw) {
    const int64_t a0 = qa0[q];
    const int32_t al = qlen[q];
    if (al > kRefWide) continue;  // uniform: k_ref_count_wide's column
    int64_t s = 0;
    for (int32_t e0 = 0; e0 < al; e0 += 4 * kWave) {  // four rows in flight per lane
      int32_t i[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int32_t e = e0 + k * kWave + lane;
        i[k] = e < al ? A.ir[a0 + e] : -1;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (i[k] >= 0) s += rptr[i[k] + 1] - rptr[i[k]];
    }
    s = wave_sum(s);
    const int c = ref_class(s, al);
    n0 += c == kClsEmpty;
    n1 += c == kClsSmall;
    n2 += c == kClsMedium;
    n3 += c == kClsLarge;
    if (lane == 0) cnt[q] = s;
  }
  __shared__ unsigned long long s_cls[kNumCls];  // the workgroup's class counts
  if (threadIdx.x < kNumCls) s_cls[threadIdx.x] = 0;
  __syncthreads();
  if (lane == 0) {
    if (n0) atomicAdd(&s_cls[kClsEmpty], n0);
    if (n1) atomicAdd(&s_cls[kClsSmall], n1);
    if (n2) atomicAdd(&s_cls[kClsMedium], n2);
    if (n3) atomicAdd(&s_cls[kClsLarge], n3);
  }
  __syncthreads();
  if (threadIdx.x < kNumCls && s_cls[threadIdx.x]) atomicAdd(&clscount[threadIdx.x], s_cls[threadIdx.x]);
}

// The wide columns' counts: one 1024-thread workgroup per column, four rows
// in flight per thread.
__global__ void __launch_bounds__(1024) k_ref_count_wide(const Operand A, const int64_t* qa0, const int32_t* qlen,
                                                         const int64_t* rptr, const int32_t* wide,
                                                         const unsigned long long* nwide, int64_t* cnt,
                                                         unsigned long long* clscount) {
  __shared__ int64_t red[1024 / kWave + 1];
  const int64_t n = (int64_t)*nwide;
  for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
    const int32_t q = wide[w];
    const int64_t a0 = qa0[q];
    const int32_t al = qlen[q];
    int64_t s = 0;
    for (int32_t e0 = 0; e0 < al; e0 += 4 * (int32_t)blockDim.x) {
      int32_t i[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int32_t e = e0 + k * (int32_t)blockDim.x + (int32_t)threadIdx.x;
        i[k] = e < al ? A.ir[a0 + e] : -1;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (i[k] >= 0) s += rptr[i[k] + 1] - rptr[i[k]];
    }
    int64_t tot;
    block_excl_scan(s, red, &tot);
    if (threadIdx.x == 0) {
      cnt[q] = tot;
      atomicAdd(&clscount[ref_class(tot, al)], 1ull);
    }
  }
}

// Columns grouped by class (any order inside a class).  A thread takes
// kClsPer consecutive columns; the class counts of a thread are packed in
// 16-bit fields, so one workgroup scan ranks every column in its class and
// one atomic per class and workgroup claims the workgroup's slots.  Every
// workgroup derives the class offsets from the counts itself; the first one
// also stores them (clsoff, kNumCls + 1 entries).  fill must be zero.
constexpr int kClsPer = 8;
__global__ void __launch_bounds__(256) k_cls_fill(const int64_t* cnt, const int32_t* qlen, int64_t lenJ,
                                                  const unsigned long long* clscount, int64_t* clsoff,
                                                  unsigned long long* fill, int32_t* list) {
  __shared__ uint64_t red[256 / kWave + 1];
  __shared__ unsigned long long s_base[kNumCls];
  __shared__ int64_t s_off[kNumCls + 1];
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int c = 0; c < kNumCls; ++c) {
      s_off[c] = run;
      run += (int64_t)clscount[c];
    }
    s_off[kNumCls] = run;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x <= kNumCls) clsoff[threadIdx.x] = s_off[threadIdx.x];
  for (int64_t q0 = (int64_t)blockIdx.x * 256 * kClsPer; q0 < lenJ; q0 += (int64_t)gridDim.x * 256 * kClsPer) {
    const int64_t qt = q0 + (int64_t)threadIdx.x * kClsPer;
    int c[kClsPer];
    uint64_t mine = 0;
#pragma unroll
    for (int k = 0; k < kClsPer; ++k) {
      c[k] = qt + k < lenJ ? ref_class(cnt[qt + k], qlen[qt + k]) : -1;
      if (c[k] >= 0) mine += 1ull << (16 * c[k]);
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan(mine, red, &tot);
    if (threadIdx.x < kNumCls) {
      const unsigned long long n = (tot >> (16 * threadIdx.x)) & 0xffffull;
      s_base[threadIdx.x] = n ? atomicAdd(&fill[threadIdx.x], n) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kClsPer; ++k) {
      if (c[k] < 0) continue;
      const int64_t slot = (int64_t)s_base[c[k]] + (int64_t)((ex >> (16 * c[k])) & 0xffffull);
      list[s_off[c[k]] + slot] = (int32_t)(qt + k);
      ex += 1ull << (16 * c[k]);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t wave_sort_keys(uint64_t key) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint64_t other = xor_lane(key, j);
      const bool up = (lane & k) == 0;
      const bool lower = (lane & j) == 0;
      const uint64_t mn = other < key ? other : key;
      const uint64_t mx = other < key ? key : other;
      key = (lower == up) ? mn : mx;
    }
  }
  return key;
}

// Columns with at most 64 entries: one wave gathers (p, source) pairs into
// LDS, sorts them by p across its lanes and writes the column.
__global__ void __launch_bounds__(256) k_ref_small(Operand A, const int64_t* qa0, const int32_t* qlen,
                                                   const int64_t* rptr, const int32_t* rpos, const int32_t* list,
                                                   const int64_t* clsoff, const int64_t* off, int vb, int32_t* bir,
                                                   void* bnum) {
  __shared__ int32_t s_p[4][kWave];
  __shared__ int64_t s_e[4][kWave];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t beg = clsoff[kClsSmall], end = clsoff[kClsSmall + 1];
  for (int64_t pos = beg + (int64_t)blockIdx.x * 4 + w; pos < end; pos += (int64_t)gridDim.x * 4) {
    const int32_t q = list[pos];
    const int64_t a0 = qa0[q];
    const int32_t al = qlen[q];
    int total = 0;
    for (int32_t ec = 0; ec < al; ec += kWave) {
      const int32_t e = ec + lane;
      int32_t i = 0;
      int rc = 0;
      if (e < al) {
        i = A.ir[a0 + e];
        rc = (int)(rptr[i + 1] - rptr[i]);
      }
      const int incl = wave_incl_scan(rc);
      const int excl = incl - rc;
      for (int r = 0; r < rc; ++r) {
        const int slot = total + excl + r;
        if (slot < kWave) {
          s_p[w][slot] = rpos[rptr[i] + r];
          s_e[w][slot] = a0 + e;
        }
      }
      total += __shfl(incl, kWave - 1);
    }
    if (total > kWave) total = kWave;
    wsync();
    uint64_t key = lane < total ? ((uint64_t)(uint32_t)s_p[w][lane] << 32) | (uint32_t)lane : ~0ull;
    key = wave_sort_keys(key);
    if (lane < total) {
      const int slot = (int)(key & 0xffffffffu);
      const int64_t o = off[q] + lane;
      bir[o] = (int32_t)(key >> 32);
      copy_value(A.num, s_e[w][slot], bnum, o, vb);
    }
    wsync();
  }
}

// Columns with at most 4096 entries: one workgroup, LDS bitonic sort.  The
// 256-thread variant walks the medium class list and leaves out its wide
// columns; the 1024-thread variant walks the list of wide columns (nwide
// entries) and takes those of the medium class, so its workgroups share the
// wide columns evenly.
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_ref_medium(Operand A, const int64_t* qa0, const int32_t* qlen,
                                                      const int64_t* rptr, const int32_t* rpos, const int32_t* list,
                                                      const int32_t* wide, int64_t nwide, const int64_t* clsoff,
                                                      const int64_t* cnt, const int64_t* off, int vb, int32_t* bir,
                                                      void* bnum) {
  constexpr bool kWide = BLOCK > 256;
  __shared__ uint64_t s_key[kRefMedium];
  __shared__ int64_t s_e[kRefMedium];
  __shared__ int64_t red[BLOCK / kWave + 1];
  const int64_t beg = kWide ? 0 : clsoff[kClsMedium], end = kWide ? nwide : clsoff[kClsMedium + 1];
  for (int64_t pos = beg + blockIdx.x; pos < end; pos += gridDim.x) {
    const int32_t q = kWide ? wide[pos] : list[pos];
    const int64_t a0 = qa0[q];
    const int32_t al = qlen[q];
    const int64_t c64 = cnt[q];
    // uniform: a column of the other variant (or, in the wide list, of another class)
    if (kWide ? (c64 == 0 || c64 > kRefMedium) : al > kRefWide) continue;
    const int c = (int)c64;
    int64_t total = 0;
    // four consecutive gathered entries per thread and round, their loads in flight together
    for (int32_t ec = 0; ec < al; ec += 4 * (int32_t)blockDim.x) {
      const int32_t e0 = ec + 4 * (int32_t)threadIdx.x;
      int32_t i[4];
      int64_t rb[4], rc[4];
      int64_t mine = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) i[k] = e0 + k < al ? A.ir[a0 + e0 + k] : -1;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        rb[k] = i[k] >= 0 ? rptr[i[k]] : 0;
        rc[k] = i[k] >= 0 ? rptr[i[k] + 1] - rb[k] : 0;
        mine += rc[k];
      }
      int64_t ctot;
      int64_t slot = total + block_excl_scan(mine, red, &ctot);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        for (int64_t r = 0; r < rc[k]; ++r, ++slot) {
          if (slot < kRefMedium) {
            s_key[slot] = ((uint64_t)(uint32_t)rpos[rb[k] + r] << 32) | (uint32_t)slot;
            s_e[slot] = a0 + e0 + k;
          }
        }
      }
      total += ctot;
    }
    int p2 = 64;
    while (p2 < c) p2 <<= 1;
    for (int s = c + threadIdx.x; s < p2; s += blockDim.x) s_key[s] = ~0ull;
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int t = threadIdx.x; t < (p2 >> 1); t += blockDim.x) {
          const int lo = 2 * t - (t & (j - 1));
          const int hi = lo + j;
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
    for (int s = threadIdx.x; s < c; s += blockDim.x) {
      const uint64_t k = s_key[s];
      const int64_t o = off[q] + s;
      bir[o] = (int32_t)(k >> 32);
      copy_value(A.num, s_e[k & 0xffffffffu], bnum, o, vb);
    }
    __syncthreads();
  }
}

// Long columns: walk p = 0..lenI-1 in order; B(p,q) exists iff row I(p)
// is stored in A(:,J(q)) (binary search).  Output is in p order directly.
__global__ void __launch_bounds__(1024) k_ref_large(Operand A, const int64_t* qa0, const int32_t* qlen,
                                                    const int32_t* I, int64_t lenI, const int32_t* list,
                                                    const int64_t* clsoff, const int64_t* off, int vb, int32_t* bir,
                                                    void* bnum) {
  __shared__ int64_t red[1024 / kWave + 1];
  const int64_t beg = clsoff[kClsLarge], end = clsoff[kClsLarge + 1];
  for (int64_t pos = beg + blockIdx.x; pos < end; pos += gridDim.x) {
    const int32_t q = list[pos];
    const int64_t a0 = qa0[q];
    const int32_t al = qlen[q];
    const int32_t* col = A.ir + a0;
    int64_t run = off[q];
    for (int64_t pc = 0; pc < lenI; pc += blockDim.x) {
      const int64_t p = pc + threadIdx.x;
      int64_t found = -1;
      if (p < lenI) {
        const int32_t i = I[p];
        int32_t lo = 0, hi = al;
        while (lo < hi) {
          const int32_t mid = (lo + hi) >> 1;
          if (col[mid] < i)
            lo = mid + 1;
          else
            hi = mid;
        }
        if (lo < al && col[lo] == i) found = a0 + lo;
      }
      int64_t ctot;
      const int64_t excl = block_excl_scan((int64_t)(found >= 0), red, &ctot);
      if (found >= 0) {
        bir[run + excl] = (int32_t)p;
        copy_value(A.num, found, bnum, run + excl, vb);
      }
      run += ctot;
    }
  }
}

__global__ void k_write_cp(const int64_t* off, int64_t n, void* cp, int32_t ptr_t) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= n; j += (int64_t)gridDim.x * blockDim.x)
    store_ptr(cp, ptr_t, j, off[j]);
}

}  // namespace spx

using namespace spx;

extern "C" int spx_spref_plan(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J,
                              int64_t lenJ, spx_plan** plan, int64_t* nnz_b) {
  if (!plan) return fail(SPX_EINVAL, "plan is NULL");
  *plan = nullptr;
  SPX_TRY(check_mat(A, "A"));
  if (lenI < 0 || lenJ < 0 || lenI >= (1ll << 31) || lenJ >= (1ll << 31)) return fail(SPX_EINVAL, "bad index length");
  if ((lenI > 0 && !I) || (lenJ > 0 && !J)) return fail(SPX_EINVAL, "index vector is NULL");
  if (A->m > (1ll << 30)) return fail(SPX_EUNSUPPORTED, "SpRef needs m <= 2^30 (dense row map)");
  if (ctx && ctx->validate) {
    int32_t ok = 0;
    SPX_TRY(spx_check(ctx, A, &ok));
    if (!ok) return fail(SPX_EINVAL, "A is not canonical");
  }
  auto* P = new SprefPlan(ctx);
  std::unique_ptr<SprefPlan> guard(P);
  hipStream_t st = stream_of(ctx);
  Scratch& scr = P->scratch;
  P->A = make_operand(A);
  P->I = I;
  P->J = J;
  P->lenI = lenI;
  P->lenJ = lenJ;
  const int64_t m = A->m;
  const int cus = device_cu_count();
  unsigned* rcnt = nullptr;
  unsigned long long *clscount = nullptr, *fill = nullptr, *nlong = nullptr;
  int32_t* longs = nullptr;  // rows with more than kRowShort positions (at most lenI / 17)
  SPX_TRY(scr.get_many({Scratch::part(&nlong, 2), Scratch::part(&longs, lenI / (kRowShort + 1) + 1),
                        Scratch::part(&P->wide, lenJ),
                        Scratch::part(&P->err, 4), Scratch::part(&rcnt, m + 1), Scratch::part(&P->rptr, m + 1),
                        Scratch::part(&P->rpos, lenI), Scratch::part(&P->qa0, lenJ), Scratch::part(&P->qlen, lenJ),
                        Scratch::part(&P->cnt, lenJ), Scratch::part(&P->off, lenJ + 1), Scratch::part(&P->list, lenJ),
                        Scratch::part(&P->clsoff, kNumCls + 1), Scratch::part(&clscount, kNumCls),
                        Scratch::part(&fill, kNumCls)}));
  // error bits, long rows and wide columns, class counts and fills; the class
  // offsets stay zero when J is empty (k_cls_fill writes them otherwise)
  SPX_TRY(zero_words(st, {{P->err, 2}, {nlong, 2}, {clscount, kNumCls}, {fill, kNumCls}, {P->clsoff, kNumCls + 1}}));
  unsigned long long* nwide = nlong + 1;
  if (lenI + lenJ > 0) {
    k_check_index<<<grid_for(lenI + lenJ, 256, 4096), 256, 0, st>>>(I, lenI, m, J, lenJ, A->n, P->err);
    SPX_HIP(hipGetLastError());
  }
  // transpose of R: rows of I grouped by index, positions ascending
  SPX_TRY(fill_u32(rcnt, m + 1, 0, st));
  if (lenI > 0) {
    k_row_hist<<<grid_for(lenI, 256, 4096), 256, 0, st>>>(I, lenI, m, rcnt);
    SPX_HIP(hipGetLastError());
  }
  SPX_TRY(exclusive_scan(LoadU32{rcnt}, m, P->rptr, scr, st));
  if (lenI > 0) {
    k_scatter_rows<<<grid_for(lenI, 256, 4096), 256, 0, st>>>(I, lenI, m, P->rptr, rcnt, P->rpos);
    SPX_HIP(hipGetLastError());
    k_sort_rows<<<grid_for(m, 256, 4096), 256, 0, st>>>(P->rptr, m, P->rpos, longs, nlong);
    SPX_HIP(hipGetLastError());
    k_sort_long_rows<<<(unsigned)(cus * 2), 256, 0, st>>>(I, lenI, P->rptr, longs, nlong, P->rpos);
    SPX_HIP(hipGetLastError());
  }
  // A*Q: the columns J(q) of A
  int64_t *aux = nullptr, chunk = 1;
  SPX_TRY(build_aux(P->A, scr, st, &aux, &chunk));
  if (lenJ > 0) {
    k_col_info<<<grid_for(lenJ, 256, 4096), 256, 0, st>>>(P->A, aux, chunk, J, lenJ, P->qa0, P->qlen, P->wide,
                                                          nwide);
    SPX_HIP(hipGetLastError());
    k_ref_count_wide<<<(unsigned)(cus * 2), 1024, 0, st>>>(P->A, P->qa0, P->qlen, P->rptr, P->wide, nwide, P->cnt,
                                                           clscount);
    SPX_HIP(hipGetLastError());
    k_ref_count<<<grid_for(lenJ * kWave, 256, (int64_t)cus * 8), 256, 0, st>>>(P->A, P->qa0, P->qlen, P->rptr, lenJ,
                                                                                P->cnt, clscount);
    SPX_HIP(hipGetLastError());
  }
  if (lenJ > 0) {
    k_cls_fill<<<grid_for(lenJ, 256 * kClsPer, 4096), 256, 0, st>>>(P->cnt, P->qlen, lenJ, clscount, P->clsoff,
                                                                     fill, P->list);
    SPX_HIP(hipGetLastError());
  }
  SPX_TRY(exclusive_scan(LoadI64{P->cnt}, lenJ, P->off, scr, st));
  int64_t h[kNumCls + 4] = {};
  SPX_TRY(read_device_words(st, {{P->clsoff, 8, kNumCls + 1}, {P->off + lenJ, 8}, {P->err, 4}, {nwide, 8}}, h));
  if (h[kNumCls + 2] & 1) return fail(SPX_EINVAL, "I has an index outside [0, m)");
  if (h[kNumCls + 2] & 2) return fail(SPX_EINVAL, "J has an index outside [0, n)");
  for (int c = 0; c <= kNumCls; ++c) P->clsoff_h[c] = h[c];
  P->nwide = h[kNumCls + 3];
  const int64_t nnz = h[kNumCls + 1];
  P->nnz = nnz;
  if (nnz_b) *nnz_b = nnz;
  *plan = guard.release();
  return SPX_OK;
}

extern "C" int spx_spref_exec(spx_plan* plan, spx_mat* B) {
  if (!plan || plan->kind != kPlanSpref) return fail(SPX_EINVAL, "not a SpRef plan");
  auto* P = static_cast<SprefPlan*>(plan);
  if (!B) return fail(SPX_EINVAL, "B is NULL");
  if (B->m != P->lenI || B->n != P->lenJ || B->fmt != SPX_CSC) return fail(SPX_EINVAL, "B must be lenI x lenJ CSC");
  if (B->val_t != P->A.val_t) return fail(SPX_EINVAL, "B's value type must be A's");
  if (B->ptr_t == SPX_PTR_I32 && P->nnz >= (1ll << 31)) return fail(SPX_EOVERFLOW, "nnz(B) needs I64 pointers");
  if (!B->cp || (P->nnz > 0 && (!B->ir || (B->val_t != SPX_VAL_BOOL && !B->num))))
    return fail(SPX_EINVAL, "B buffers missing");
  B->nnz = P->nnz;
  B->nzc = 0;
  hipStream_t st = stream_of(&P->ctx);
  const int vb = value_size(P->A.val_t);
  const int cus = device_cu_count();
  const int64_t* co = P->clsoff_h;
  // the wide medium columns' few workgroups run beside the other classes
  SideJoin side{nullptr, st};
  if (co[kClsMedium + 1] > co[kClsMedium] && P->nwide > 0) {
    SPX_TRY(side_fork(st, &side.ss));
    k_ref_medium<1024><<<(unsigned)std::min<int64_t>(P->nwide, (int64_t)cus * 2), 1024, 0, side.ss->s>>>(
        P->A, P->qa0, P->qlen, P->rptr, P->rpos, P->list, P->wide, P->nwide, P->clsoff, P->cnt, P->off, vb, B->ir,
        B->num);
    SPX_HIP(hipGetLastError());
  }
  if (co[kClsSmall + 1] > co[kClsSmall]) {
    k_ref_small<<<grid_for(co[kClsSmall + 1] - co[kClsSmall], 4, (int64_t)cus * 16), 256, 0, st>>>(
        P->A, P->qa0, P->qlen, P->rptr, P->rpos, P->list, P->clsoff, P->off, vb, B->ir, B->num);
    SPX_HIP(hipGetLastError());
  }
  if (co[kClsMedium + 1] > co[kClsMedium]) {
    k_ref_medium<256><<<grid_for(co[kClsMedium + 1] - co[kClsMedium], 1, (int64_t)cus * 2), 256, 0, st>>>(
        P->A, P->qa0, P->qlen, P->rptr, P->rpos, P->list, P->wide, P->nwide, P->clsoff, P->cnt, P->off, vb, B->ir,
        B->num);
    SPX_HIP(hipGetLastError());
  }
  if (co[kClsLarge + 1] > co[kClsLarge]) {
    k_ref_large<<<grid_for(co[kClsLarge + 1] - co[kClsLarge], 1, (int64_t)cus * 2), 1024, 0, st>>>(
        P->A, P->qa0, P->qlen, P->I, P->lenI, P->list, P->clsoff, P->off, vb, B->ir, B->num);
    SPX_HIP(hipGetLastError());
  }
  SPX_TRY(side.join());
  k_write_cp<<<grid_for(P->lenJ + 1, 256, 65536), 256, 0, st>>>(P->off, P->lenJ, B->cp, B->ptr_t);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

extern "C" int spx_spref(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J,
                         int64_t lenJ, spx_mat* B) {
  if (!B) return fail(SPX_EINVAL, "B is NULL");
  spx_plan* plan = nullptr;
  int64_t nnz = 0;
  SPX_TRY(spx_spref_plan(ctx, A, I, lenI, J, lenJ, &plan, &nnz));
  std::unique_ptr<spx_plan> guard(plan);
  OutAlloc oa(ctx);
  spx_mat out{};
  out.m = lenI;
  out.n = lenJ;
  out.fmt = SPX_CSC;
  out.ptr_t = SPX_PTR_I64;
  out.val_t = A->val_t;
  const int vb = value_size(A->val_t);
  SPX_TRY(oa.get((size_t)(lenJ + 1) * 8, &out.cp));
  SPX_TRY(oa.get((size_t)std::max<int64_t>(nnz, 1) * 4, reinterpret_cast<void**>(&out.ir)));
  if (vb) SPX_TRY(oa.get((size_t)std::max<int64_t>(nnz, 1) * vb, &out.num));
  SPX_TRY(spx_spref_exec(plan, &out));
  oa.keep();
  *B = out;
  return SPX_OK;
}
