// CPU oracle for the sparse kernels.  TEST INFRASTRUCTURE ONLY: the library
// never calls, links or loads this file; tests, the smoke check and the
// benchmark's CPU-baseline leg do.
//
// Plain, slow, obviously correct implementations of what the GPU path
// computes, written from the paper (Buluc & Gilbert, "Parallel Sparse
// Matrix-Matrix Multiplication and Indexing: Implementation and
// Experiments"):
//
//   * SpGEMM C = A*B over a semiring: the column-wise formulation of
//     Gustavson's algorithm (Section 3, Algorithm 1) with a dense sparse
//     accumulator (SPA: value array, occupied flags, list of occupied rows;
//     caption of Figure 1).  Column j of C is the semiring sum, over the
//     nonzeros B(k,j) in ascending k, of A(:,k) "times" B(k,j).
//   * SpRef B = A(I,J): the definition of Section 4 -- B(p,q) = A(I(p),J(q))
//     for every p, q, respecting the order (and repeats) of I and J --
//     evaluated by direct loops, not through products.
//   * SpAsgn A(I,J) = B: the result of Section 4.1 (C = A + R B Q - S A T,
//     with the subtraction replaced by an elementwise mask that drops the
//     pattern of A(I,J)); repeated indices resolved so that the last
//     occurrence wins, evaluated by direct loops.
//   * Extend-add A(I,J) = A(I,J) + B: SpAsgn without the S A T term
//     (Section 4.1), i.e. C = A + R B Q.  R and Q are the selection
//     matrices of SpAsgn, so a repeated index makes several B entries land
//     on one position, where the semiring sum combines them.  Evaluated by
//     direct loops: each output value starts from A's value (if stored) and
//     adds the landing B values in B's storage order (column q ascending,
//     then row p ascending).
//   * CSC -> DCSC compression (Section 3.2): keep only the nonempty columns,
//     with JC listing their ids.
//
// Conventions: 0-based indices, CSC with int64 column pointers and int32
// row indices, rows strictly increasing inside a column on input and
// output.  Structural semantics: an output entry exists iff at least one
// product contributes to it, whatever its value.  Compile with
// -ffp-contract=off so that a*b+c is two rounded operations.
//
// parity unpinned: none (every routine is pinned by tests/test_oracle_*.py).

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>
#include <type_traits>
#include <omp.h>

namespace {

enum Semiring { PLUS_TIMES = 0, MIN_PLUS = 1, SELECT2ND = 2, OR_AND = 3, SELECT1ST = 4 };
enum VType { F32 = 0, F64 = 1, I64 = 2, BOOL = 3 };

// ---- semiring arithmetic ---------------------------------------------------
// "mul" is the semiring product of A(i,k) and B(k,j); "add" combines a new
// product into an existing accumulator value.
template <typename T> struct PlusTimes {
  static T mul(T a, T b) { return a * b; }
  static T add(T acc, T x) { return acc + x; }
};
template <> struct PlusTimes<int64_t> {  // two's-complement wrap-around
  static int64_t mul(int64_t a, int64_t b) { return (int64_t)((uint64_t)a * (uint64_t)b); }
  static int64_t add(int64_t acc, int64_t x) { return (int64_t)((uint64_t)acc + (uint64_t)x); }
};
template <typename T> struct MinPlus {
  static T mul(T a, T b) { return a + b; }
  static T add(T acc, T x) { return x < acc ? x : acc; }
};
template <> struct MinPlus<int64_t> {
  static int64_t mul(int64_t a, int64_t b) { return (int64_t)((uint64_t)a + (uint64_t)b); }
  static int64_t add(int64_t acc, int64_t x) { return x < acc ? x : acc; }
};
// select-second: the product is B's value, the sum keeps the smallest value.
template <typename T> struct Select2nd {
  static T mul(T, T b) { return b; }
  static T add(T acc, T x) { return x < acc ? x : acc; }
};
template <typename T> struct Select1st {
  static T mul(T a, T) { return a; }
  static T add(T acc, T x) { return x < acc ? x : acc; }
};

// ---- SpGEMM: Algorithm 1 with a dense SPA ----------------------------------
// One output column.  `val`, `occ` are dense arrays of length m owned by the
// calling thread; `list` collects the occupied rows in first-touch order.
template <typename T, typename Op>
int64_t spa_column(int64_t j, const int64_t* acp, const int32_t* air, const T* anum,
                   const int64_t* bcp, const int32_t* bir, const T* bnum,
                   std::vector<T>& val, std::vector<char>& occ, std::vector<int32_t>& list,
                   int32_t* out_ir, T* out_num) {
  list.clear();
  for (int64_t q = bcp[j]; q < bcp[j + 1]; ++q) {  // B(k,j) != 0, ascending k
    const int32_t k = bir[q];
    const T b = bnum ? bnum[q] : T(1);
    for (int64_t p = acp[k]; p < acp[k + 1]; ++p) {  // C(:,j) += A(:,k) * B(k,j)
      const int32_t i = air[p];
      const T a = anum ? anum[p] : T(1);
      const T x = Op::mul(a, b);
      if (!occ[i]) {
        occ[i] = 1;
        val[i] = x;
        list.push_back(i);
      } else {
        val[i] = Op::add(val[i], x);
      }
    }
  }
  std::sort(list.begin(), list.end());
  const int64_t cnt = (int64_t)list.size();
  for (int64_t t = 0; t < cnt; ++t) {
    const int32_t i = list[t];
    if (out_ir) out_ir[t] = i;
    if (out_num) out_num[t] = val[i];
    occ[i] = 0;  // reset the SPA for the next column
  }
  return cnt;
}

template <typename T, typename Op>
void spgemm_run(int64_t m, const int64_t* acp, const int32_t* air, const T* anum, const int64_t* bcp,
                const int32_t* bir, const T* bnum, int64_t ncols, const int64_t* cols, int64_t* counts,
                const int64_t* offs, int32_t* cir, T* cnum, int nthreads) {
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<T> val((size_t)m);
    std::vector<char> occ((size_t)m, 0);
    std::vector<int32_t> list;
#pragma omp for schedule(dynamic, 16)
    for (int64_t t = 0; t < ncols; ++t) {
      const int64_t j = cols ? cols[t] : t;
      int32_t* oi = cir ? cir + offs[t] : nullptr;
      T* ov = cnum ? cnum + offs[t] : nullptr;
      const int64_t c = spa_column<T, Op>(j, acp, air, anum, bcp, bir, bnum, val, occ, list, oi, ov);
      if (counts) counts[t] = c;
    }
  }
}

template <typename T>
int spgemm_typed(int sr, int64_t m, const int64_t* acp, const int32_t* air, const void* anum,
                 const int64_t* bcp, const int32_t* bir, const void* bnum, int64_t ncols, const int64_t* cols,
                 int64_t* counts, const int64_t* offs, int32_t* cir, void* cnum, int nthreads) {
  const T* a = (const T*)anum;
  const T* b = (const T*)bnum;
  T* c = (T*)cnum;
  switch (sr) {
    case PLUS_TIMES: spgemm_run<T, PlusTimes<T>>(m, acp, air, a, bcp, bir, b, ncols, cols, counts, offs, cir, c, nthreads); return 0;
    case MIN_PLUS: spgemm_run<T, MinPlus<T>>(m, acp, air, a, bcp, bir, b, ncols, cols, counts, offs, cir, c, nthreads); return 0;
    case SELECT2ND: spgemm_run<T, Select2nd<T>>(m, acp, air, a, bcp, bir, b, ncols, cols, counts, offs, cir, c, nthreads); return 0;
    case SELECT1ST: spgemm_run<T, Select1st<T>>(m, acp, air, a, bcp, bir, b, ncols, cols, counts, offs, cir, c, nthreads); return 0;
    default: return -1;
  }
}

// ---- Extend-add by direct loops ---------------------------------------------
// One column j of C = A + R B Q: the stored A(:,j) entries, then every stored
// B(p,q) with J(q) = j in B's storage order, are listed with their target row;
// a stable sort by row keeps that order among entries of one row, and each
// run of one row is folded left to right with the semiring sum `Add`.
template <typename T, typename Add>
void extend_add_typed(int64_t m, int64_t n, const int64_t* acp, const int32_t* air, const T* anum,
                      const int32_t* I, const std::vector<std::vector<int64_t>>& qs_of, const int64_t* bcp,
                      const int32_t* bir, const T* bnum, int64_t* counts, const int64_t* offs, int32_t* cir,
                      T* cnum, int nthreads) {
  (void)m;
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<std::pair<int32_t, int64_t>> col;  // (row, source): >= 0 A position, < 0 B position -(e+1)
#pragma omp for schedule(dynamic, 256)
    for (int64_t j = 0; j < n; ++j) {
      col.clear();
      for (int64_t e = acp[j]; e < acp[j + 1]; ++e) col.emplace_back(air[e], e);
      for (int64_t q : qs_of[j])
        for (int64_t e = bcp[q]; e < bcp[q + 1]; ++e) col.emplace_back(I[bir[e]], -(e + 1));
      std::stable_sort(col.begin(), col.end(),
                       [](const std::pair<int32_t, int64_t>& x, const std::pair<int32_t, int64_t>& y) {
                         return x.first < y.first;
                       });
      int64_t out = 0;
      for (size_t t = 0; t < col.size();) {
        size_t u = t + 1;
        while (u < col.size() && col[u].first == col[t].first) ++u;
        if (cir) {
          cir[offs[j] + out] = col[t].first;
          if (cnum) {
            auto value = [&](int64_t s) { return s >= 0 ? anum[s] : bnum[-s - 1]; };
            T acc = value(col[t].second);
            for (size_t k = t + 1; k < u; ++k) acc = Add::add(acc, value(col[k].second));
            cnum[offs[j] + out] = acc;
          }
        }
        ++out;
        t = u;
      }
      if (counts) counts[j] = out;
    }
  }
}

// ---- Checking a computed product column by column -------------------------
// Recomputes columns [j0, j1) of C = A*B with the SPA of Algorithm 1 (the
// same spa_column as oracle_spgemm) and compares them with a given block of
// columns: gcp[0 .. j1-j0] are its column pointers (gcp[0] is the position of
// column j0 in gir / gnum), gir its rows, gnum its values (NULL: pattern).
// A column matches when its row list is identical and every value matches:
// bitwise when rtol <= 0 or for integers; otherwise |g - r| <= rtol * |r| and,
// where the oracle's value is a zero, the same zero (sign included).
// Returns the number of columns that differ; *first_bad receives the
// smallest such column (or -1).
template <typename T>
bool value_matches(T g, T r, double rtol) {
  if constexpr (std::is_floating_point<T>::value) {
    if (rtol > 0 && r != T(0)) {
      const double d = (double)g - (double)r;
      const double lim = rtol * ((double)r < 0 ? -(double)r : (double)r);
      return (d < 0 ? -d : d) <= lim;  // false for NaN
    }
  }
  return std::memcmp(&g, &r, sizeof(T)) == 0;
}

template <typename T, typename Op>
int64_t check_run(int64_t m, const int64_t* acp, const int32_t* air, const T* anum, const int64_t* bcp,
                  const int32_t* bir, const T* bnum, int64_t j0, int64_t j1, const int64_t* gcp, const int32_t* gir,
                  const T* gnum, double rtol, int64_t* first_bad, int nthreads) {
  int64_t nbad = 0, first = -1;
#pragma omp parallel num_threads(nthreads) reduction(+ : nbad)
  {
    std::vector<T> val((size_t)m);
    std::vector<char> occ((size_t)m, 0);
    std::vector<int32_t> list, rir;
    std::vector<T> rnum;
    int64_t my_first = -1;
#pragma omp for schedule(dynamic, 16)
    for (int64_t j = j0; j < j1; ++j) {
      const int64_t len = gcp[j - j0 + 1] - gcp[j - j0];
      const int64_t at = gcp[j - j0] - gcp[0];
      rir.resize((size_t)m > 0 ? (size_t)m : 1);
      rnum.resize(gnum ? rir.size() : 0);
      const int64_t c = spa_column<T, Op>(j, acp, air, anum, bcp, bir, bnum, val, occ, list, rir.data(),
                                          gnum ? rnum.data() : nullptr);
      bool ok = c == len;
      for (int64_t t = 0; ok && t < c; ++t) ok = gir[at + t] == rir[t];
      for (int64_t t = 0; ok && gnum && t < c; ++t) ok = value_matches<T>(gnum[at + t], rnum[t], rtol);
      if (!ok) {
        ++nbad;
        if (my_first < 0 || j < my_first) my_first = j;
      }
    }
#pragma omp critical
    if (my_first >= 0 && (first < 0 || my_first < first)) first = my_first;
  }
  if (first_bad) *first_bad = first;
  return nbad;
}

template <typename T>
int64_t check_typed(int sr, int64_t m, const int64_t* acp, const int32_t* air, const void* anum,
                    const int64_t* bcp, const int32_t* bir, const void* bnum, int64_t j0, int64_t j1,
                    const int64_t* gcp, const int32_t* gir, const void* gnum, double rtol, int64_t* first_bad,
                    int nthreads) {
  const T* a = (const T*)anum;
  const T* b = (const T*)bnum;
  const T* g = (const T*)gnum;
  switch (sr) {
    case PLUS_TIMES: return check_run<T, PlusTimes<T>>(m, acp, air, a, bcp, bir, b, j0, j1, gcp, gir, g, rtol, first_bad, nthreads);
    case MIN_PLUS: return check_run<T, MinPlus<T>>(m, acp, air, a, bcp, bir, b, j0, j1, gcp, gir, g, rtol, first_bad, nthreads);
    case SELECT2ND: return check_run<T, Select2nd<T>>(m, acp, air, a, bcp, bir, b, j0, j1, gcp, gir, g, rtol, first_bad, nthreads);
    case SELECT1ST: return check_run<T, Select1st<T>>(m, acp, air, a, bcp, bir, b, j0, j1, gcp, gir, g, rtol, first_bad, nthreads);
    default: return -1;
  }
}

}  // namespace

extern "C" {

// Column counts and (optionally) the columns themselves of C = A*B.
//   m        rows of A (and C)
//   acp/air  A in CSC; anum: A's values (NULL = pattern / ignored)
//   bcp/bir  B in CSC; bnum: B's values
//   ncols, cols  which columns of C to compute (cols NULL = 0..ncols-1)
//   counts   [ncols] out, nnz of each requested column (may be NULL)
//   offs     [ncols] start of each requested column in cir/cnum (fill pass)
//   cir/cnum out arrays (NULL to skip); cnum's type is `vt`
// Value typing: PLUS_TIMES and MIN_PLUS need A and B of type vt;
// SELECT2ND takes B's values (anum ignored); SELECT1ST takes A's;
// OR_AND is pattern only (vt = BOOL).  Returns 0, or -1 on a bad code.
int oracle_spgemm(int sr, int vt, int64_t m, const int64_t* acp, const int32_t* air, const void* anum,
                  const int64_t* bcp, const int32_t* bir, const void* bnum, int64_t ncols, const int64_t* cols,
                  int64_t* counts, const int64_t* offs, int32_t* cir, void* cnum, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (sr == OR_AND || vt == BOOL) {  // pattern only: any instantiation computes the pattern
    return spgemm_typed<double>(PLUS_TIMES, m, acp, air, nullptr, bcp, bir, nullptr, ncols, cols, counts, offs,
                                cir, nullptr, nthreads);
  }
  switch (vt) {
    case F32: return spgemm_typed<float>(sr, m, acp, air, anum, bcp, bir, bnum, ncols, cols, counts, offs, cir, cnum, nthreads);
    case F64: return spgemm_typed<double>(sr, m, acp, air, anum, bcp, bir, bnum, ncols, cols, counts, offs, cir, cnum, nthreads);
    case I64: return spgemm_typed<int64_t>(sr, m, acp, air, anum, bcp, bir, bnum, ncols, cols, counts, offs, cir, cnum, nthreads);
    default: return -1;
  }
}

// Compares columns [j0, j1) of a computed C = A*B with the oracle's (see
// check_run).  Same operand conventions as oracle_spgemm.  Returns the number
// of differing columns, or -1 for an unsupported semiring / type.
int64_t oracle_spgemm_check(int sr, int vt, int64_t m, const int64_t* acp, const int32_t* air, const void* anum,
                            const int64_t* bcp, const int32_t* bir, const void* bnum, int64_t j0, int64_t j1,
                            const int64_t* gcp, const int32_t* gir, const void* gnum, double rtol,
                            int64_t* first_bad, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (sr == OR_AND || vt == BOOL)
    return check_typed<double>(PLUS_TIMES, m, acp, air, nullptr, bcp, bir, nullptr, j0, j1, gcp, gir, nullptr, 0.0,
                               first_bad, nthreads);
  switch (vt) {
    case F32: return check_typed<float>(sr, m, acp, air, anum, bcp, bir, bnum, j0, j1, gcp, gir, gnum, rtol, first_bad, nthreads);
    case F64: return check_typed<double>(sr, m, acp, air, anum, bcp, bir, bnum, j0, j1, gcp, gir, gnum, rtol, first_bad, nthreads);
    case I64: return check_typed<int64_t>(sr, m, acp, air, anum, bcp, bir, bnum, j0, j1, gcp, gir, gnum, 0.0, first_bad, nthreads);
    default: return -1;
  }
}

// ---- SpRef by direct indexing ---------------------------------------------
// B = A(I,J): B(p,q) = A(I(p), J(q)).  inv[i] lists, ascending, every p with
// I(p) = i, so a row index that appears several times in I is replicated.
// counts[q] = nnz(B(:,q)); fill pass writes rows p ascending and values
// (element size `vbytes`, 0 = pattern only).
int oracle_spref(int64_t m, const int64_t* acp, const int32_t* air, const void* anum, int vbytes, int64_t lenI,
                 const int32_t* I, int64_t lenJ, const int32_t* J, int64_t* counts, const int64_t* offs,
                 int32_t* bir, void* bnum, int nthreads) {
  for (int64_t p = 0; p < lenI; ++p)
    if (I[p] < 0 || I[p] >= m) return -1;
  std::vector<int64_t> start((size_t)m + 1, 0);
  for (int64_t p = 0; p < lenI; ++p) start[(size_t)I[p] + 1]++;
  for (int64_t i = 0; i < m; ++i) start[i + 1] += start[i];
  std::vector<int64_t> pos(start.begin(), start.end() - 1);
  std::vector<int32_t> inv((size_t)lenI);
  for (int64_t p = 0; p < lenI; ++p) inv[pos[I[p]]++] = (int32_t)p;  // ascending p per i
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<std::pair<int32_t, int64_t>> col;  // (p, source position in A)
#pragma omp for schedule(dynamic, 64)
    for (int64_t q = 0; q < lenJ; ++q) {
      col.clear();
      const int32_t jq = J[q];
      for (int64_t e = acp[jq]; e < acp[jq + 1]; ++e) {
        const int32_t i = air[e];
        for (int64_t t = start[i]; t < start[i + 1]; ++t) col.emplace_back(inv[t], e);
      }
      std::sort(col.begin(), col.end());
      if (counts) counts[q] = (int64_t)col.size();
      if (bir) {
        for (size_t t = 0; t < col.size(); ++t) {
          bir[offs[q] + t] = col[t].first;
          if (bnum && vbytes)
            std::memcpy((char*)bnum + (offs[q] + t) * vbytes, (const char*)anum + col[t].second * vbytes, vbytes);
        }
      }
    }
  }
  return 0;
}

// ---- SpAsgn by direct loops -------------------------------------------------
// C = A with the block A(I,J) replaced by B (lenI x lenJ, CSC).  UI, UJ are
// the sets of indices in I and J; lastI[i] is the last p with I(p) = i.
// C = { A(i,j) : not (i in UI and j in UJ) }
//   u { (I(p), J(q)) <- B(p,q) : p = lastI[I(p)], q = lastJ[J(q)], B(p,q) stored }
int oracle_spasgn(int64_t m, int64_t n, const int64_t* acp, const int32_t* air, const void* anum, int vbytes,
                  int64_t lenI, const int32_t* I, int64_t lenJ, const int32_t* J, const int64_t* bcp,
                  const int32_t* bir, const void* bnum, int64_t* counts, const int64_t* offs, int32_t* cir,
                  void* cnum, int nthreads) {
  std::vector<int64_t> lastI((size_t)m, -1), lastJ((size_t)n, -1);
  for (int64_t p = 0; p < lenI; ++p) {
    if (I[p] < 0 || I[p] >= m) return -1;
    lastI[I[p]] = p;
  }
  for (int64_t q = 0; q < lenJ; ++q) {
    if (J[q] < 0 || J[q] >= n) return -1;
    lastJ[J[q]] = q;
  }
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
  {
    // (row, source): source >= 0 -> A position, source < 0 -> B position -(s+1)
    std::vector<std::pair<int32_t, int64_t>> col;
#pragma omp for schedule(dynamic, 256)
    for (int64_t j = 0; j < n; ++j) {
      col.clear();
      const bool jin = lastJ[j] >= 0;
      for (int64_t e = acp[j]; e < acp[j + 1]; ++e) {
        const int32_t i = air[e];
        if (jin && lastI[i] >= 0) continue;  // inside the assigned block: dropped
        col.emplace_back(i, e);
      }
      if (jin) {
        const int64_t q = lastJ[j];
        for (int64_t e = bcp[q]; e < bcp[q + 1]; ++e) {
          const int32_t p = bir[e];
          if (lastI[I[p]] != p) continue;  // an earlier occurrence of a repeated row index
          col.emplace_back(I[p], -(e + 1));
        }
      }
      std::sort(col.begin(), col.end());
      if (counts) counts[j] = (int64_t)col.size();
      if (cir) {
        for (size_t t = 0; t < col.size(); ++t) {
          cir[offs[j] + t] = col[t].first;
          if (cnum && vbytes) {
            const int64_t s = col[t].second;
            const void* src = s >= 0 ? (const char*)anum + s * vbytes : (const char*)bnum + (-s - 1) * vbytes;
            std::memcpy((char*)cnum + (offs[j] + t) * vbytes, src, vbytes);
          }
        }
      }
    }
  }
  return 0;
}

// ---- Extend-add C = A + R B Q (Section 4.1, SpAsgn without S A T) ----------
// Semiring `sr` chooses the sum: + for PLUS_TIMES, min for MIN_PLUS,
// SELECT2ND and SELECT1ST; OR_AND or vt = BOOL give the pattern only.
// counts[j] = nnz(C(:,j)); the fill pass (offs, cir, cnum non-NULL) writes
// rows ascending.  Returns -1 for an index out of range.
int oracle_extend_add(int sr, int vt, int64_t m, int64_t n, const int64_t* acp, const int32_t* air,
                      const void* anum, int64_t lenI, const int32_t* I, int64_t lenJ, const int32_t* J,
                      const int64_t* bcp, const int32_t* bir, const void* bnum, int64_t* counts,
                      const int64_t* offs, int32_t* cir, void* cnum, int nthreads) {
  for (int64_t p = 0; p < lenI; ++p)
    if (I[p] < 0 || I[p] >= m) return -1;
  std::vector<std::vector<int64_t>> qs_of((size_t)n);
  for (int64_t q = 0; q < lenJ; ++q) {
    if (J[q] < 0 || J[q] >= n) return -1;
    qs_of[J[q]].push_back(q);
  }
  if (nthreads < 1) nthreads = 1;
  if (sr == OR_AND || vt == BOOL) {
    extend_add_typed<double, PlusTimes<double>>(m, n, acp, air, nullptr, I, qs_of, bcp, bir, nullptr, counts,
                                                offs, cir, nullptr, nthreads);
    return 0;
  }
  const bool plus = sr == PLUS_TIMES;
  switch (vt) {
    case F32:
      if (plus)
        extend_add_typed<float, PlusTimes<float>>(m, n, acp, air, (const float*)anum, I, qs_of, bcp, bir,
                                                  (const float*)bnum, counts, offs, cir, (float*)cnum, nthreads);
      else
        extend_add_typed<float, MinPlus<float>>(m, n, acp, air, (const float*)anum, I, qs_of, bcp, bir,
                                                (const float*)bnum, counts, offs, cir, (float*)cnum, nthreads);
      return 0;
    case F64:
      if (plus)
        extend_add_typed<double, PlusTimes<double>>(m, n, acp, air, (const double*)anum, I, qs_of, bcp, bir,
                                                    (const double*)bnum, counts, offs, cir, (double*)cnum, nthreads);
      else
        extend_add_typed<double, MinPlus<double>>(m, n, acp, air, (const double*)anum, I, qs_of, bcp, bir,
                                                  (const double*)bnum, counts, offs, cir, (double*)cnum, nthreads);
      return 0;
    case I64:
      if (plus)
        extend_add_typed<int64_t, PlusTimes<int64_t>>(m, n, acp, air, (const int64_t*)anum, I, qs_of, bcp, bir,
                                                      (const int64_t*)bnum, counts, offs, cir, (int64_t*)cnum,
                                                      nthreads);
      else
        extend_add_typed<int64_t, MinPlus<int64_t>>(m, n, acp, air, (const int64_t*)anum, I, qs_of, bcp, bir,
                                                    (const int64_t*)bnum, counts, offs, cir, (int64_t*)cnum,
                                                    nthreads);
      return 0;
    default: return -2;
  }
}

// ---- CSC -> DCSC (Section 3.2) -----------------------------------------------
// Returns nzc; when jc/dcp are non-NULL fills JC (ids of nonempty columns,
// ascending) and the compressed pointers CP (nzc+1 entries).
int64_t oracle_csc_to_dcsc(int64_t n, const int64_t* cp, int32_t* jc, int64_t* dcp) {
  int64_t nzc = 0;
  for (int64_t j = 0; j < n; ++j) {
    if (cp[j + 1] > cp[j]) {
      if (jc) {
        jc[nzc] = (int32_t)j;
        dcp[nzc] = cp[j];
      }
      ++nzc;
    }
  }
  if (dcp) dcp[nzc] = cp[n];
  return nzc;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
