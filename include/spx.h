/*
 * spx -- sparse matrix-matrix multiplication, indexing and assignment on one
 * AMD Instinct MI355X (gfx950).
 *
 * The operations follow Buluc & Gilbert, "Parallel Sparse Matrix-Matrix
 * Multiplication and Indexing: Implementation and Experiments":
 *   C = A*B over a semiring            Section 3, Algorithm 1 (column-wise SpGEMM)
 *   B = A(I,J)           (SpRef)       Section 4; computed as R*(A*Q)
 *   C = A with A(I,J) = B (SpAsgn)     Section 4.1 (A + R B Q, minus the pattern of S A T)
 *   A(I,J) = A(I,J) + B  (extend-add)  Section 4.1 (A + R B Q)
 *   C = sum_k A_k*B_k    (stage sum)   Section 3.3, Algorithm 2 (one processor's SUMMA stages)
 *   C = S_r*A*S_c^T      (contraction) Section 5.3.2 restriction, as one SpGEMM pass
 *   CSC <-> DCSC                       Section 3.2
 *
 * Conventions for every entry point
 *   - All matrix and index arrays are DEVICE pointers, 0-based.
 *   - Canonical form: inside each column the row ids in `ir` are strictly
 *     increasing (no duplicates); in DCSC `jc` is strictly increasing and
 *     lists nonempty columns only.  Non-canonical input gives undefined
 *     results unless ctx->validate is set (then SPX_EINVAL).
 *   - Structural semantics: an output entry exists iff at least one product
 *     contributes to it; values equal to zero are kept.
 *   - The caller owns inputs, outputs and plans.  A plan keeps pointers to
 *     its inputs: they must stay alive and unchanged until the plan's last
 *     exec call has completed on the stream.
 *   - All device work is enqueued on ctx->stream.  Plan calls synchronise
 *     that stream once (to read back output sizes); exec calls do not.
 *   - Every call returns SPX_OK or an error code; spx_last_error() gives a
 *     thread-local message.  On error, output buffers are left untouched
 *     unless the code is SPX_EDEVICE.
 */
#ifndef SPX_H
#define SPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
enum {
  SPX_OK = 0,
  SPX_EINVAL = 1,       /* bad descriptor, dimension mismatch, index out of range */
  SPX_ENOMEM = 2,       /* the allocation callback (or hipMalloc) failed */
  SPX_EOVERFLOW = 3,    /* a count does not fit the requested pointer type */
  SPX_EUNSUPPORTED = 4, /* semiring / value-type combination not provided */
  SPX_EDEVICE = 5       /* a HIP runtime call failed */
};
/* Fault injection for tests of the error paths: with the environment
 * variable SPX_FAULT set to "alloc:N", the N-th device allocation the
 * library makes (plan scratch and one-shot outputs, counted from the moment
 * the variable took its current value) fails as SPX_ENOMEM; "alloc:N+"
 * fails that allocation and every later one.  An entry point that fails
 * releases what it had allocated and leaves its outputs untouched. */

/* ---- descriptors ----------------------------------------------------- */
enum { SPX_CSC = 0, SPX_DCSC = 1 };                 /* storage format (Section 3.2) */
enum { SPX_PTR_I32 = 0, SPX_PTR_I64 = 1 };          /* element type of cp */
enum { SPX_VAL_F32 = 0, SPX_VAL_F64 = 1, SPX_VAL_I64 = 2, SPX_VAL_BOOL = 3 };

/* Semirings (Section 2: matrices over a semiring (S, +, x)).
 *   PLUS_TIMES  ordinary (+, x); int64 wraps around (two's complement)
 *   MIN_PLUS    x = +, + = min        (tropical; shortest two-hop paths)
 *   SELECT2ND   x returns B's value, + keeps the minimum; A may be BOOL
 *   SELECT1ST   x returns A's value, + keeps the minimum; B may be BOOL
 *   OR_AND      boolean; pattern only, no values                        */
enum { SPX_PLUS_TIMES = 0, SPX_MIN_PLUS = 1, SPX_SELECT2ND = 2, SPX_OR_AND = 3, SPX_SELECT1ST = 4 };

/* A sparse matrix in CSC or DCSC.
 *   m, n   dimensions (each < 2^31)
 *   nnz    stored entries
 *   nzc    DCSC: number of nonempty columns = length of jc (ignored for CSC)
 *   jc     DCSC only: [nzc] ids of the nonempty columns, strictly increasing
 *   cp     [n+1] (CSC) or [nzc+1] (DCSC) of type ptr_t, cp[0] = 0, cp[last] = nnz
 *   ir     [nnz] int32 row ids
 *   num    [nnz] values of type val_t; not read or written for SPX_VAL_BOOL  */
typedef struct spx_mat {
  int64_t m, n, nnz, nzc;
  int32_t fmt, ptr_t, val_t, reserved;
  int32_t* jc;
  void* cp;
  int32_t* ir;
  void* num;
} spx_mat;

/* Execution context.
 *   stream    hipStream_t to enqueue on (NULL: the null stream)
 *   alloc     device allocator for scratch (and one-shot outputs); NULL: hipMalloc
 *   free      matching free; called with the pointer alloc returned
 *   user      passed to alloc / free
 *   validate  nonzero: check that inputs are canonical before computing
 *   profile   nonzero: plans record HIP events around their kernel groups
 *             (read with spx_plan_get_times)                              */
typedef struct spx_ctx {
  void* stream;
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
  int32_t validate;
  int32_t profile;
} spx_ctx;

/* Tuning knobs of the SpGEMM kernels (NULL = built-in defaults, which
 * spx_default_tuning() returns).  Output columns are binned by their
 * number of multiplications mu (an upper bound on their output size):
 *   tiny_max         mu <= tiny_max (<= 64): formed by one 64-lane wave that
 *                    sorts the column's products
 *   hash_count_max   mu <= hash_count_max (<= 16384): exact count through an
 *                    LDS hash table; larger columns through an LDS bitmap
 *   single_part_max  power of two in [64, 4096]: columns with mu at most this
 *                    are accumulated as one part (LDS hash or bitmap sized
 *                    for it); larger columns are cut into row-range parts
 *   part_lds_bytes   LDS budget of one part of a larger column
 *   *_threads        workgroup sizes (multiples of 64, at most 1024) of the
 *                    hash count, bitmap count, multi-part and single-part
 *                    numeric kernels
 *   bitmap_chunk_log2  rows per work item of the bitmap count (log2); 0: one
 *                    chunk per row slice, at most 2^18 rows
 *   xcd_slices       the row space is cut into this many slices (parts never
 *                    straddle one); workgroup w serves slice w mod xcd_slices
 *                    first, so each XCD's L2 holds one slice of A (1: off)
 *   bitmap_store_mb  HBM (MiB) the plan may hold to keep the row bitmaps of
 *                    the bitmap-counted columns from the count to the numeric
 *                    phase, which then reads them instead of gathering those
 *                    rows again; 0: off.  Above the cap, or if the allocation
 *                    fails, the numeric phase recomputes them.
 *   range_chunk      B entries per range set-up round of the multi-part
 *                    launch: 256, 512, or 0 = chosen per product (512 when the
 *                    cut columns would make more than one set-up per two
 *                    multiplications, as with a tall-skinny B); 512 costs
 *                    5 KiB of the part budget and is skipped if a dense row
 *                    block would then no longer fit.
 *   bucket_parts     1: every part of a cut column visits only the B entries
 *                    whose A column has rows in the part's range (lists built
 *                    by the plan, one entry per B entry and part reached);
 *                    -1: parts walk all of their column's B entries; 0: lists
 *                    when range set-ups would outnumber multiplications 3 to
 *                    2 (a very tall-skinny B).
 *   force_off64      1: gather A's rows and values through 64-bit positions
 *                    even when A has fewer than 2^29 entries (the path that
 *                    larger operands take); 0: 32-bit byte offsets when they
 *                    fit.                                                    */
typedef struct spx_tuning {
  int32_t tiny_max;
  int32_t hash_count_max;
  int32_t single_part_max;
  int32_t part_lds_bytes;
  int32_t count_threads;
  int32_t bitmap_threads;
  int32_t part_threads;
  int32_t single_threads;
  int32_t bitmap_chunk_log2;
  int32_t xcd_slices;
  int32_t bitmap_store_mb;
  int32_t range_chunk;
  int32_t bucket_parts;
  int32_t force_off64;
} spx_tuning;

/* Statistics of a SpGEMM plan, available once the plan call returned. */
typedef struct spx_plan_info {
  int64_t mults;          /* total number of multiplications (sum over columns) */
  int64_t nnz;            /* nnz(C) */
  int64_t nzc;            /* nonempty columns of C */
  int64_t cols_empty, cols_tiny, cols_medium, cols_heavy;
  int64_t heavy_parts;    /* row-range parts (every non-tiny nonempty column has >= 1) */
  int64_t nnz_tiny;       /* entries of C formed by the one-wave path */
  int64_t nnz_multi;      /* entries of C in parts of columns cut into row ranges */
  int64_t multi_parts;    /* number of those parts (the first heavy_parts launch) */
} spx_plan_info;

/* Device time of the kernel groups of the last plan / exec calls of a
 * SpGEMM plan created with ctx->profile set (milliseconds, HIP events on
 * the plan's stream; 0 when a group did not run).                       */
typedef struct spx_times {
  float symbolic_ms;       /* plan: lookup, counts, binning, exact sizes, scans, parts */
  float numeric_parts_ms;  /* exec: all parts (LDS bitmap / hash accumulation) */
  float numeric_multi_ms;  /* exec: the launch over parts of columns cut into row ranges */
  float numeric_tiny_ms;   /* exec: columns formed by one wave */
  float pointers_ms;       /* exec: column pointers of C */
} spx_times;

typedef struct spx_plan spx_plan;

/* ---- SpGEMM: C = A*B over a semiring (Algorithm 1) --------------------
 * spx_spgemm_plan: validates A (m x k) and B (k x n), runs the symbolic
 *   phase on the device and returns nnz(C) and the number of nonempty
 *   columns nzc(C).  Both operands may be CSC or DCSC.  c_fmt selects the
 *   output format.  Values: PLUS_TIMES and MIN_PLUS need A and B of one
 *   value type (F32, F64 or I64); SELECT2ND takes B's type, SELECT1ST A's;
 *   OR_AND produces a pattern (C.val_t = BOOL).
 * spx_spgemm_exec: fills C.  The caller sets C->m, n, fmt (= c_fmt),
 *   ptr_t, val_t and provides buffers: cp [n+1] or [nzc+1] of ptr_t,
 *   jc [nzc] (DCSC), ir [nnz], num [nnz] (unless BOOL).  SPX_EOVERFLOW if
 *   ptr_t is I32 and nnz >= 2^31.  Several execs of one plan are allowed.
 * spx_spgemm: one shot; C's buffers come from ctx->alloc (free them with
 *   ctx->free, or hipFree when ctx->alloc is NULL).                      */
int spx_spgemm_plan(const spx_ctx* ctx, const spx_mat* A, const spx_mat* B, int32_t semiring, int32_t c_fmt,
                    const spx_tuning* tuning, spx_plan** plan, int64_t* nnz_c, int64_t* nzc_c);
int spx_spgemm_exec(spx_plan* plan, spx_mat* C);
int spx_spgemm(const spx_ctx* ctx, const spx_mat* A, const spx_mat* B, int32_t semiring, int32_t c_fmt,
               spx_mat* C);
int spx_plan_get_info(const spx_plan* plan, spx_plan_info* info);
/* Waits for the recorded events and reports their elapsed times. */
int spx_plan_get_times(spx_plan* plan, spx_times* times);
void spx_plan_destroy(spx_plan* plan);
void spx_default_tuning(spx_tuning* tuning);

/* ---- Sparse SUMMA stage accumulation: C = sum_k A_k*B_k (Algorithm 2) ---
 * One processor's output block of Sparse SUMMA (Section 3.3): over the
 * stages k < count it accumulates C = C + A_k*B_k with the semiring's sum.
 * With every stage block resident, the stages are computed as the single
 * product [A_1 ... A_K] * [B_1; ...; B_K]: each output column accumulates
 * the products of all stages at once, and no partial C is written.
 * spx_spgemm_sum_plan: A and B are arrays of `count` >= 1 descriptors,
 *   A_k m x b_k and B_k b_k x n (CSC or DCSC, sum of b_k below 2^31); all
 *   A_k (and all B_k) share one value type; the semiring rules of
 *   spx_spgemm_plan apply.  Copies the blocks' patterns into the plan
 *   (about 12 bytes per stored entry plus 8 per column of the stacked
 *   right operand), runs the symbolic phase and returns nnz(C) and nzc(C).
 * spx_spgemm_sum_exec: refreshes the values from A_k.num / B_k.num
 *   (patterns must be unchanged) and fills C as spx_spgemm_exec does.
 * spx_plan_get_info / spx_plan_get_times report the inner product.
 * An output entry exists iff some stage contributes a product to it; the
 * order of the floating-point sums is unspecified, as in spx_spgemm.     */
int spx_spgemm_sum_plan(const spx_ctx* ctx, int32_t count, const spx_mat* A, const spx_mat* B, int32_t semiring,
                        int32_t c_fmt, const spx_tuning* tuning, spx_plan** plan, int64_t* nnz_c, int64_t* nzc_c);
int spx_spgemm_sum_exec(spx_plan* plan, spx_mat* C);

/* ---- Graph contraction / restriction: C = S_r*A*S_c^T (Section 5.3.2) ---
 * S_r (m_coarse x m) has the single unit entry S_r(row_agg[u], u) in every
 * column u, and S_c (n_coarse x n) likewise with col_agg; a NULL map makes
 * that side the identity (its coarse dimension is then ignored).  So
 * C(I,J) is the semiring sum of the stored A(u,v) with row_agg[u] = I and
 * col_agg[v] = J (restriction of order r: agg[v] = v / r; graph
 * contraction: S*A*S^T with one map for both sides).  The triple product
 * is one SpGEMM pass over A and forms neither S_r*A nor A*S_c^T (Section 6
 * asks for such a primitive).
 * Maps may be in any order; values must lie in [0, coarse dimension)
 * (SPX_EINVAL).  A non-decreasing row_agg keeps A's entry order; any other
 * row_agg makes the plan sort every column of A by mapped row (in
 * registers or LDS up to 4096 entries, longer columns by one global sort
 * each; 12 more bytes per entry of A) and every exec gather A's values in
 * that order.  Semirings: PLUS_TIMES (sums, S entries 1) and MIN_PLUS
 * (minima, S entries 0) on A's value type; SELECT1ST (minimum of A's
 * values) and OR_AND (pattern) with any A.  The plan keeps A's pointers and
 * values (patterns must stay unchanged; values may change between execs)
 * plus 4 bytes per entry of A for the mapped row ids.
 * spx_contract_exec fills C (m_coarse x n_coarse) as spx_spgemm_exec does;
 * spx_plan_get_info / spx_plan_get_times report the inner product.       */
int spx_contract_plan(const spx_ctx* ctx, const spx_mat* A, const int32_t* row_agg, int64_t m_coarse,
                      const int32_t* col_agg, int64_t n_coarse, int32_t semiring, int32_t c_fmt,
                      const spx_tuning* tuning, spx_plan** plan, int64_t* nnz_c, int64_t* nzc_c);
int spx_contract_exec(spx_plan* plan, spx_mat* C);

/* ---- Batched SpGEMM: C_i = A_i*B_i for i < count ------------------------
 * All products of a batch run through one symbolic pass and one persistent
 * numeric launch: the batch is computed as the single product
 * [A_1 ... A_n] * blockdiag(B_1, ..., B_n) = [C_1 ... C_n] (Algorithm 1
 * applied to a block-diagonal right operand), so work items of every
 * product share the device work lists.
 * spx_batch_plan: A and B are arrays of `count` CSC descriptors (A_i m_i x k_i,
 *   B_i k_i x n_i); all A_i (and all B_i) share one value type and the
 *   semiring rules of spx_spgemm_plan apply.  Copies the operands' patterns
 *   into the plan, runs the symbolic phase (one synchronisation) and returns
 *   the total nnz of all C_i and the total length of their column pointers
 *   (sum of n_i + 1).
 * spx_batch_exec: refreshes the operand values from A_i.num / B_i.num
 *   (patterns must be unchanged), runs the numeric phase and fills C[i]:
 *   C[i].cp points into cp_pool (int64, cp_total entries), C[i].ir / num into
 *   ir_pool / num_pool (nnz_total entries); the caller owns the pools, which
 *   must not overlap any operand.  When the distinct A_i.num (or all B_i.num)
 *   lie back to back in batch order in one allocation -- as the C_i of an
 *   earlier batch do -- they are read in place rather than copied, so they
 *   must stay allocated for as long as the plan is executed.
 * spx_batch_capture / spx_batch_replay: record spx_batch_exec with the given
 *   pools into a HIP graph once, then launch it on the plan's stream (values
 *   may change between replays).                                           */
int spx_batch_plan(const spx_ctx* ctx, int32_t count, const spx_mat* A, const spx_mat* B, int32_t semiring,
                   const spx_tuning* tuning, spx_plan** plan, int64_t* nnz_total, int64_t* cp_total);
int spx_batch_exec(spx_plan* plan, int64_t* cp_pool, int32_t* ir_pool, void* num_pool, spx_mat* C);
int spx_batch_capture(spx_plan* plan, int64_t* cp_pool, int32_t* ir_pool, void* num_pool, spx_mat* C);
int spx_batch_replay(spx_plan* plan);
/* spx_batch_spgemm: one shot (plan, pools, exec, plan destroyed).  The three
 * pools come from ctx->alloc (hipMalloc without one) and begin at C[0].cp,
 * C[0].ir and C[0].num (NULL for a pattern result); the caller frees those
 * three pointers with ctx->free (hipFree).  tuning may be NULL.  Returns
 * once the work is enqueued on ctx->stream.                               */
int spx_batch_spgemm(const spx_ctx* ctx, int32_t count, const spx_mat* A, const spx_mat* B, int32_t semiring,
                     const spx_tuning* tuning, spx_mat* C);

/* ---- SpRef: B = A(I,J) (Section 4) ------------------------------------
 * B(p,q) = A(I(p), J(q)) for p < lenI, q < lenJ, respecting the order of I
 * and J; repeated indices replicate rows / columns.  A is CSC or DCSC,
 * I and J are device int32 arrays (any order, repeats allowed).  The
 * product R*(A*Q) is formed right to left: A*Q gathers the columns J,
 * R selects and reorders rows; every output entry receives exactly one
 * product, so values are copied bit for bit.
 * spx_spref_plan returns nnz(B); spx_spref_exec fills B (CSC, lenI x lenJ,
 * caller-allocated: cp [lenJ+1], ir [nnz], num [nnz]).  SPX_EINVAL if an
 * index is out of range (checked on the device during the plan).
 * spx_spref_exec may put the columns that gather more than 4096 entries of
 * A on a second stream of the calling host thread (created on first use);
 * that work is joined back into ctx->stream by an event before the call
 * returns, so everything enqueued on ctx->stream afterwards sees it.      */
int spx_spref_plan(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J,
                   int64_t lenJ, spx_plan** plan, int64_t* nnz_b);
int spx_spref_exec(spx_plan* plan, spx_mat* B);
/* One shot: B's buffers (CSC, int64 cp, A's value type) come from
 * ctx->alloc (hipMalloc without one); free B->cp, B->ir, B->num with
 * ctx->free (hipFree).  Nothing stays allocated on error.                 */
int spx_spref(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J, int64_t lenJ,
              spx_mat* B);

/* ---- SpAsgn: C = A with the submatrix A(I,J) replaced by B (Section 4.1)
 * A is m x n and B is lenI x lenJ, each CSC or DCSC (a DCSC operand's
 * pointers are expanded to CSC in the plan's scratch; rows and values are
 * read in place).  Functional: A is not modified.  C keeps every A(i,j)
 * with i not in I or j not in J, and takes C(I(p), J(q)) = B(p,q) for the
 * stored B(p,q); entries of A(I,J) that B does not store are removed.  A
 * repeated index resolves to its last occurrence in I (or J), as in
 * sequential assignment.  A and B must have the same value type.  Any
 * number of rows may be inserted into one column: columns above 4096
 * inserted rows have their entries sorted in global memory by the plan.
 * spx_spasgn_plan returns nnz(C); spx_spasgn_exec fills C (CSC, m x n,
 * caller-allocated: cp [n+1], ir [nnz], num [nnz]).                      */
int spx_spasgn_plan(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J,
                    int64_t lenJ, const spx_mat* B, spx_plan** plan, int64_t* nnz_c);
int spx_spasgn_exec(spx_plan* plan, spx_mat* C);
/* One shot, with C's buffers from ctx->alloc as for spx_spref.             */
int spx_spasgn(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J, int64_t lenJ,
               const spx_mat* B, spx_mat* C);

/* ---- Extend-add: A(I,J) = A(I,J) + B (Section 4.1) ----------------------
 * SpAsgn without the S*A*T term: C = A + R*B*Q, with R and Q SpAsgn's
 * selection matrices (R(I(p), p) = 1, Q(q, J(q)) = 1).  Functional: A is
 * not modified.  C keeps every stored A entry and every position
 * (I(p), J(q)) of a stored B(p,q); where several of these meet (A stores
 * the position, or I or J repeats an index) their values are combined with
 * the semiring's sum: + for PLUS_TIMES, min for MIN_PLUS, SELECT2ND and
 * SELECT1ST.  The sum starts from A's value (if stored) and adds the B
 * values in B's storage order (column q ascending, then row p ascending),
 * so results do not depend on scheduling.  OR_AND takes pattern-only (BOOL)
 * operands; BOOL operands give the pattern union under any semiring.
 * A and B are CSC or DCSC with the same value type; B is lenI x lenJ with
 * nnz(B) < 2^32; I and J are device int32 arrays (any order, repeats
 * allowed).  Any number of B entries may land in one column of C: columns
 * above 4096 landing entries are sorted in global memory by the plan
 * (SPX_EUNSUPPORTED only if those columns' entries total 2^31 or more).
 * spx_extend_add_plan returns nnz(C) (SPX_EINVAL for an index out of range);
 * spx_extend_add_exec fills C (CSC, m x n, value type of A, caller-allocated:
 * cp [n+1], ir [nnz], num [nnz]).                                         */
int spx_extend_add_plan(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J,
                        int64_t lenJ, const spx_mat* B, int32_t semiring, spx_plan** plan, int64_t* nnz_c);
int spx_extend_add_exec(spx_plan* plan, spx_mat* C);
/* One shot, with C's buffers from ctx->alloc as for spx_spref.             */
int spx_extend_add(const spx_ctx* ctx, const spx_mat* A, const int32_t* I, int64_t lenI, const int32_t* J,
                   int64_t lenJ, const spx_mat* B, int32_t semiring, spx_mat* C);

/* ---- formats (Section 3.2) ----------------------------------------------
 * spx_count_nonempty: nzc of a CSC matrix (synchronises the stream).
 * spx_csc_to_dcsc: writes out->jc [nzc] and out->cp [nzc+1] (ptr_t of
 *   out) for the CSC matrix A; out->ir / out->num are set to A's arrays
 *   (DCSC shares them with CSC).  out->nzc must hold spx_count_nonempty's
 *   result.
 * spx_dcsc_to_csc: writes out->cp [n+1] for the DCSC matrix A; ir / num
 *   are shared likewise.                                                 */
int spx_count_nonempty(const spx_ctx* ctx, const spx_mat* A, int64_t* nzc);
int spx_csc_to_dcsc(const spx_ctx* ctx, const spx_mat* A, spx_mat* out);
int spx_dcsc_to_csc(const spx_ctx* ctx, const spx_mat* A, spx_mat* out);

/* spx_csc_to_dcsc_noalloc: spx_csc_to_dcsc for callers that cannot allocate
 *   device memory -- code under HIP graph capture, tight serving loops,
 *   harnesses that forbid hipMalloc.  It calls no allocator (neither
 *   ctx->alloc nor hipMalloc) and does not synchronise the stream: its
 *   scratch is a static device array of the library (about 33 MiB per GPU,
 *   held until the process ends), so A may have at most 2^22 columns
 *   (SPX_EINVAL beyond).  out->nzc is the capacity of out->jc ([nzc]) and
 *   out->cp ([nzc+1]) and must be the number of nonempty columns of A;
 *   entries beyond it are not written.  nzc_dev (device int64, may be NULL)
 *   receives the number of nonempty columns.  All calls on one GPU share the
 *   static array: calls that overlap on one GPU (other streams or threads)
 *   race and must be ordered by the caller.                              */
int spx_csc_to_dcsc_noalloc(const spx_ctx* ctx, const spx_mat* A, spx_mat* out, int64_t* nzc_dev);

/* Checks that A is canonical (pointers monotone, rows in range and
 * strictly increasing per column, jc strictly increasing and in range).
 * *ok = 1 or 0.  Synchronises the stream.                                */
int spx_check(const spx_ctx* ctx, const spx_mat* A, int32_t* ok);

/* Thread-local message describing the last error of this thread. */
const char* spx_last_error(void);

/* Library version string. */
const char* spx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPX_H */
