/*
 * nbgrb.h -- C ABI of a nonblocking GraphBLAS subset for AMD Instinct MI355X
 * (gfx950), built around the fused PageRank iteration of
 * "Julia GraphBLAS with Nonblocking Execution" (Costanza, Mattson, Kimmerer,
 * Brock).
 *
 * Execution model (paper, Section II "Nonblocking execution"):
 *   - GrB_init(GrB_BLOCKING): every operation runs as its own GPU kernel
 *     and its output is materialised before the next operation is issued.
 *   - GrB_init(GrB_NONBLOCKING): operations are validated and recorded as
 *     nodes of a DAG (Section III-A, "General approach"; Fig. 3 shows the
 *     node kept for mxv).  Nothing runs until a wait or a value read forces
 *     it; then the pending DAG is pattern-matched onto fused kernels and
 *     intermediates that no handle can reach any more are never written
 *     (the "elide unneeded objects" of Section II).  Results equal blocking
 *     mode up to floating-point reassociation.
 *
 * Device and stream: all work is enqueued on one HIP stream (GrM_set_stream;
 * the null stream by default).  "Complete" means complete in stream order:
 * later work on that stream sees the result.  Calls that hand a value to
 * the host (GrB_Scalar_extractElement_FP64, GrB_Vector_reduce_FP64, the
 * *_export_* calls into host memory, GrM_pagerank's iteration count)
 * synchronise the stream.
 *
 * Memory: every pointer argument documented as "device" must be device
 * memory on the current HIP device; "host" pointers are ordinary host
 * memory.  Imports copy the caller's data; exports copy out.  The library
 * owns all storage behind its handles and frees it in *_free or
 * GrB_finalize.  Device memory comes from the allocator installed with
 * GrM_set_allocator (hipMalloc/hipFree when none is installed), cached by
 * exact size and reused in stream order.
 *
 * Errors: every call returns a GrB_Info.  API errors (null pointers,
 * uninitialised handles, size or type mismatches, unsupported operator
 * combinations) are detected eagerly in both modes and leave all objects
 * unchanged.  Execution errors (GrB_OUT_OF_MEMORY, GrB_PANIC on a HIP
 * failure) surface at the call that executes the work: the operation itself
 * in blocking mode, the forcing call in nonblocking mode.  GrM_error()
 * returns a text describing the last error of the calling thread.
 * Non-convergence of an iterative algorithm is not an error.
 *
 * Threads: one context per process; the library is not thread-safe.
 */
#ifndef NBGRB_H
#define NBGRB_H

#include <stdbool.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef uint64_t GrB_Index;

/* Return codes, numbered as in the GraphBLAS C API specification 2.x. */
typedef enum {
  GrB_SUCCESS = 0,
  GrB_NO_VALUE = 1,
  GrB_UNINITIALIZED_OBJECT = -1,
  GrB_NULL_POINTER = -2,
  GrB_INVALID_VALUE = -3,
  GrB_INVALID_INDEX = -4,
  GrB_DOMAIN_MISMATCH = -5,
  GrB_DIMENSION_MISMATCH = -6,
  GrB_OUTPUT_NOT_EMPTY = -7,
  GrB_NOT_IMPLEMENTED = -8,
  GrB_PANIC = -101,
  GrB_OUT_OF_MEMORY = -102,
  GrB_INSUFFICIENT_SPACE = -103,
  GrB_INVALID_OBJECT = -104,
  GrB_INDEX_OUT_OF_BOUNDS = -105,
  GrB_EMPTY_OBJECT = -106
} GrB_Info;

/* Execution modes (Section II of the paper). */
typedef enum { GrB_NONBLOCKING = 0, GrB_BLOCKING = 1 } GrB_Mode;

/* GrB_COMPLETE: the object's value is computed (in stream order).
 * GrB_MATERIALIZE: additionally it is held in storage, not as a pending
 * node.  Both force the pending DAG in nonblocking mode. */
typedef enum { GrB_COMPLETE = 0, GrB_MATERIALIZE = 1 } GrB_WaitMode;

/* Opaque handles. */
typedef struct GB_Type_opaque *GrB_Type;
typedef struct GB_UnaryOp_opaque *GrB_UnaryOp;
typedef struct GB_BinaryOp_opaque *GrB_BinaryOp;
typedef struct GB_Monoid_opaque *GrB_Monoid;
typedef struct GB_Semiring_opaque *GrB_Semiring;
typedef struct GB_Descriptor_opaque *GrB_Descriptor;
typedef struct GB_Vector_opaque *GrB_Vector;
typedef struct GB_Matrix_opaque *GrB_Matrix;
typedef struct GB_Scalar_opaque *GrB_Scalar;

/* ------------------------------------------------------------------------
 * Built-in types and operators.  User-defined (host) functions cannot run
 * in a GPU kernel, so the operator set is closed; the paper's anonymous
 * functions map onto it as follows (Fig. 6):
 *   (x, y) -> abs(x - y)            GrM_ABSDIFF_*
 *   (_, x) -> x  (mxv multiply)     GrM_PLUS_SECOND_SEMIRING_*
 *   x / d with d = max(outdeg,1)/damping   GrB_DIV_* (eWiseMult)
 * ---------------------------------------------------------------------- */
extern GrB_Type GrB_BOOL, GrB_INT32, GrB_FP32, GrB_FP64;
/* bfloat16 (upper half of binary32, rounded to nearest even): storage type
 * of network activations only (GrM_GNN_new); not a vector type. */
extern GrB_Type GrM_BF16;

extern GrB_UnaryOp GrB_IDENTITY_FP32, GrB_IDENTITY_FP64;
extern GrB_UnaryOp GrB_ABS_FP32, GrB_ABS_FP64;
extern GrB_UnaryOp GrB_AINV_FP32, GrB_AINV_FP64; /* -x */
extern GrB_UnaryOp GrB_MINV_FP32, GrB_MINV_FP64; /* 1/x */
/* 1/x where x != 0, else 0: the inverse out-degree with dangling -> 0. */
extern GrB_UnaryOp GrM_MINV_OR_ZERO_FP32, GrM_MINV_OR_ZERO_FP64;

extern GrB_BinaryOp GrB_PLUS_FP32, GrB_PLUS_FP64;
extern GrB_BinaryOp GrB_MINUS_FP32, GrB_MINUS_FP64;
extern GrB_BinaryOp GrB_TIMES_FP32, GrB_TIMES_FP64;
extern GrB_BinaryOp GrB_DIV_FP32, GrB_DIV_FP64;
extern GrB_BinaryOp GrB_MAX_FP32, GrB_MAX_FP64;
extern GrB_BinaryOp GrB_MIN_FP32, GrB_MIN_FP64;
extern GrB_BinaryOp GrB_FIRST_FP32, GrB_FIRST_FP64;
extern GrB_BinaryOp GrB_SECOND_FP32, GrB_SECOND_FP64;
extern GrB_BinaryOp GrM_ABSDIFF_FP32, GrM_ABSDIFF_FP64; /* |x - y| */

extern GrB_Monoid GrB_PLUS_MONOID_FP32, GrB_PLUS_MONOID_FP64;

/* Semirings accepted by GrB_mxv.  The matrices built by this
 * library are patterns whose stored values are all 1 (iso-valued), so
 * plus-times and plus-second compute the same product. */
extern GrB_Semiring GrB_PLUS_TIMES_SEMIRING_FP32, GrB_PLUS_TIMES_SEMIRING_FP64;
extern GrB_Semiring GrM_PLUS_SECOND_SEMIRING_FP32, GrM_PLUS_SECOND_SEMIRING_FP64;

/* Descriptors: NULL (defaults), or any combination of R (replace: positions
 * the mask does not allow lose their entry instead of keeping the output's
 * old one), S (structural mask: a present mask entry allows its position
 * whatever its value; otherwise the value must be nonzero) and C
 * (complement the mask). */
extern GrB_Descriptor GrB_DESC_C, GrB_DESC_S, GrB_DESC_SC, GrB_DESC_R, GrB_DESC_RC, GrB_DESC_RS,
    GrB_DESC_RSC;

/* ------------------------------------------------------------------------
 * Context
 * ---------------------------------------------------------------------- */

/* Start the library in the given mode.  GrB_INVALID_VALUE for an unknown
 * mode; GrB_INVALID_VALUE if already initialised; GrB_PANIC if no HIP
 * device is usable. */
GrB_Info GrB_init(GrB_Mode mode);

/* Wait for all queued work, free every object and cached buffer. */
GrB_Info GrB_finalize(void);

GrB_Info GrM_get_mode(GrB_Mode *mode);

/* Switch the execution mode of the running context (project extension):
 * pending work is forced first.  Lets one process compare blocking and
 * nonblocking execution on the same objects. */
GrB_Info GrM_set_mode(GrB_Mode mode);

/* Text of the last error (never NULL; empty when there was none). */
const char *GrM_error(void);

/* Stream all work is enqueued on (a hipStream_t).  The previous stream is
 * synchronised first, so cached buffers are never shared across streams
 * without ordering. */
GrB_Info GrM_set_stream(void *hip_stream);

/* Device allocator callbacks: alloc(bytes, ctx) returns device memory or
 * NULL; release(ptr, ctx) frees it.  Pass NULLs to return to hipMalloc /
 * hipFree.  Only allowed while no object holds device memory
 * (GrB_INVALID_VALUE otherwise). */
GrB_Info GrM_set_allocator(void *(*alloc)(size_t bytes, void *ctx),
                           void (*release)(void *ptr, void *ctx), void *ctx);

/* Test hook: make the k-th device allocation from now on fail (k >= 1);
 * k = 0 disables.  The failure surfaces as GrB_OUT_OF_MEMORY at the call
 * that executes the work. */
GrB_Info GrM_fail_allocation_after(int64_t k);

/* Counters since GrB_init or the last reset: kernels launched, fused
 * PageRank-iteration launches, plan-cache hits and misses, number of
 * intermediates that were never materialised. */
typedef struct {
  int64_t kernels;
  int64_t fused_launches;
  int64_t plan_hits;
  int64_t plan_misses;
  int64_t elided_nodes;
  int64_t forced_waits;
  int64_t ewise_fused;      /* generated elementwise-tree launches */
  int64_t ewise_ops;        /* operations those launches covered */
  int64_t jit_compiles;     /* generated kernels compiled */
  int64_t jit_disk_hits;    /* ... loaded from the code cache directory */
  int64_t jit_memory_hits;  /* ... found already loaded */
  int64_t mxv_push;         /* mxv with missing entries driven by u's entries */
  int64_t mxv_pull;         /* ... driven by the rows of A */
  int64_t out_full;         /* results with missing entries possible, stored full */
  int64_t out_bitset;       /* ... stored as bitsets */
  int64_t out_sparse;       /* ... stored sparse */
  int64_t index_loops;      /* elementwise loops driven by a sparse input's entries */
  int64_t range_loops;      /* ... over the whole index range */
  int64_t device_allocs;    /* device buffers handed out, from the cache or the allocator */
} GrM_Stats;
GrB_Info GrM_get_stats(GrM_Stats *stats);
GrB_Info GrM_reset_stats(void);

/* Nonblocking fusion level: 0 fuses only the PageRank-iteration pattern;
 * 1 (default) also runs every needed elementwise result together with the
 * pending elementwise intermediates below it (eWiseAdd, eWiseMult, apply
 * with or without a bound scalar; FP32/FP64 results, FP32/FP64/INT32
 * inputs; up to 24 operations, 12 input vectors and 6 scalars) as one
 * kernel generated for the tree's signature.  Generated kernels are
 * compiled with hipRTC once per process and their code objects kept in the
 * directory NBGRB_CODE_CACHE (default $HOME/.cache/nbgrb), keyed by the
 * source they were compiled from.  Results equal the per-operation
 * kernels' bit for bit. */
GrB_Info GrM_set_fusion(int level);
/* Unload every generated kernel of this process (the directory stays). */
GrB_Info GrM_code_cache_clear(void);

/* ------------------------------------------------------------------------
 * Scalars.  Values live on the device as FP64 whatever the declared type.
 * ---------------------------------------------------------------------- */
GrB_Info GrB_Scalar_new(GrB_Scalar *s, GrB_Type type);
GrB_Info GrB_Scalar_free(GrB_Scalar *s);
GrB_Info GrB_Scalar_setElement_FP64(GrB_Scalar s, double x);
/* Forces the scalar and copies its value to *x (synchronises).
 * GrB_NO_VALUE if the scalar has never been assigned. */
GrB_Info GrB_Scalar_extractElement_FP64(double *x, GrB_Scalar s);
/* Complete s (as GrB_Vector_wait; Section III: reading a scalar's value,
 * as Fig. 6 does with the residual in its loop test, also forces it). */
GrB_Info GrB_Scalar_wait(GrB_Scalar s, GrB_WaitMode mode);
/* out = alpha * in + beta, recorded like any other operation (project
 * extension: it expresses the teleport constant (1-d)/n + d*D/n from the
 * dangling mass D without a host round trip). */
GrB_Info GrM_Scalar_affine(GrB_Scalar out, double alpha, GrB_Scalar in, double beta);

/* ------------------------------------------------------------------------
 * Vectors.  All vectors are full (dense): every index holds a value, as the
 * FullVector of the paper (Section III-A, Fig. 4).
 * ---------------------------------------------------------------------- */

/* New vector of length n (n >= 1) holding zeros.  type FP32, FP64 or INT32. */
GrB_Info GrB_Vector_new(GrB_Vector *v, GrB_Type type, GrB_Index n);
GrB_Info GrB_Vector_free(GrB_Vector *v);
/* w = u (a new reference to u's value; no copy is made). */
GrB_Info GrB_Vector_dup(GrB_Vector *w, GrB_Vector u);
GrB_Info GrB_Vector_size(GrB_Index *n, GrB_Vector v);
GrB_Info GrM_Vector_type(GrB_Type *t, GrB_Vector v);
/* Complete v: run whatever pending work it depends on (nonblocking mode).
 * Defined by: the wait method that materialises an object (Section III,
 * and Section III-C: the point where the pending method tree is matched,
 * looked up in the cache by its signature and run); Fig. 6 calls it on the
 * new rank vector every iteration.  In blocking mode a no-op. */
GrB_Info GrB_Vector_wait(GrB_Vector v, GrB_WaitMode mode);

/* Every entry := value (the paper's GrBVector(n, value) constructor,
 * Fig. 6).  Kept iso-valued -- one value, no storage -- until an operation
 * needs it stored. */
GrB_Info GrM_Vector_fill(GrB_Vector v, double value);

/* Copy n entries of the vector's type from device memory src_dev. */
GrB_Info GrM_Vector_import_dense(GrB_Vector v, const void *src_dev, GrB_Index n);
/* Force v and copy its n entries (vector's type) to device memory dst_dev. */
GrB_Info GrM_Vector_export_dense(void *dst_dev, GrB_Index n, GrB_Vector v);
/* Force and materialise v; *ptr receives the device address of its
 * storage, valid until v is next modified or freed.  Read-only. */
GrB_Info GrM_Vector_device_pointer(const void **ptr, GrB_Vector v);

/* ------------------------------------------------------------------------
 * Matrices: CSR patterns with int32 row pointers and column indices (the
 * paper uses 32-bit indices throughout its experiments, Section IV), so
 * nnz < 2^31 and dimensions < 2^31.  Stored values are all 1.
 * ---------------------------------------------------------------------- */

GrB_Info GrB_Matrix_new(GrB_Matrix *A, GrB_Type type, GrB_Index nrows, GrB_Index ncols);
GrB_Info GrB_Matrix_free(GrB_Matrix *A);
GrB_Info GrB_Matrix_nrows(GrB_Index *n, GrB_Matrix A);
GrB_Info GrB_Matrix_ncols(GrB_Index *n, GrB_Matrix A);
GrB_Info GrB_Matrix_nvals(GrB_Index *nvals, GrB_Matrix A);
GrB_Info GrB_Matrix_wait(GrB_Matrix A, GrB_WaitMode mode);

/* Replace A's content by the CSR pattern (rowptr_dev[nrows+1],
 * col_dev[nnz], device, int32).  rowptr must start at 0, be
 * non-decreasing and end at nnz; columns must lie in [0, ncols), with no
 * column repeated within a row (any order).  The arrays are copied.
 * GrB_INVALID_VALUE on a malformed pattern (checked on the device). */
GrB_Info GrM_Matrix_import_CSR(GrB_Matrix A, const int32_t *rowptr_dev,
                               const int32_t *col_dev, GrB_Index nnz);

/* Copy A's CSR pattern to device memory (rowptr_dev[nrows+1], col_dev[nnz]). */
GrB_Info GrM_Matrix_export_CSR(int32_t *rowptr_dev, int32_t *col_dev, GrB_Matrix A);

/* A := the n x n pattern with an entry (src[e], dst[e]) for every edge e
 * (device arrays of length nedges).  Duplicate edges are merged; self-loops
 * are dropped when drop_self is true.  Rows are sources, each row's columns
 * ascending.  GrB_INDEX_OUT_OF_BOUNDS if an endpoint is >= n. */
GrB_Info GrM_Matrix_build_edges(GrB_Matrix A, const uint32_t *src_dev,
                                const uint32_t *dst_dev, GrB_Index nedges,
                                bool drop_self);

/* Dense matrices (the second operand and the result of GrB_mxm).  A
 * matrix made by GrB_Matrix_new(type FP32 or FP64, nrows, ncols) becomes
 * dense by this import: nrows x ncols values of A's type, row-major (row i
 * at src_dev + i*ncols), copied from device memory.  nrows and ncols must
 * be A's (GrB_DIMENSION_MISMATCH otherwise).  A dense matrix is accepted
 * only by GrB_mxm (as B, and as C, which it overwrites), the export below,
 * GrB_Matrix_free / nrows / ncols / nvals / wait and the pattern imports
 * that replace its content; every other call that takes a matrix rejects
 * it with GrB_INVALID_VALUE.
 * Defined by: the matrix operand of the GraphBLAS operations the paper
 * records (Section II); the paper itself only multiplies by vectors. */
GrB_Info GrM_Matrix_import_dense(GrB_Matrix A, const void *src_dev, GrB_Index nrows, GrB_Index ncols);
/* Copy a dense matrix's nrows x ncols values (row-major, its type) to
 * device memory.  GrB_INVALID_VALUE if A holds a pattern. */
GrB_Info GrM_Matrix_export_dense(void *dst_dev, GrB_Matrix A);

/* C := A (+.*) B with A a CSR pattern (nrows x ncols) and B dense
 * (ncols x k, 1 <= k <= 64): C(i, c) = sum over the entries j of row i of
 * B(j, c), every row of B read as one k-wide vector.  C becomes dense
 * nrows x k (C must have been made nrows x k); the types of B, C and the
 * semiring must agree (FP32 or FP64).  Mask, accum and desc must be NULL
 * (GrB_NOT_IMPLEMENTED otherwise), as must k > 64; semirings are
 * plus-times or plus-second (equal on a pattern).  Runs at once in both
 * modes: no vector operation is pending on matrices.  Empty rows give 0.
 * Defined by: the GraphBLAS mxm operation (Section II's operations on
 * matrix objects), restricted to the sparse x dense product that batches k
 * right-hand sides of the mxv of Fig. 6 -- the product behind batched
 * personalised PageRank (GrM_ppr_batch fuses the same product with its
 * epilogue and never materialises it). */
GrB_Info GrB_mxm(GrB_Matrix C, GrB_Matrix Mask, GrB_BinaryOp accum, GrB_Semiring op,
                 GrB_Matrix A, GrB_Matrix B, GrB_Descriptor desc);

/* C := A^T (GraphBLAS transpose with no mask and no accumulator; mask and
 * accum must be NULL).  C must be ncols(A) x nrows(A).  Each row of C lists
 * its columns in ascending order. */
GrB_Info GrB_transpose(GrB_Matrix C, GrB_Matrix Mask, GrB_BinaryOp accum,
                       GrB_Matrix A, GrB_Descriptor desc);

/* deg := number of stored entries in each row of A (deg has nrows(A)
 * entries; type INT32, FP32 or FP64).  With A the adjacency pattern this is
 * the out-degree vector the paper's PageRank takes as input (Fig. 6). */
GrB_Info GrM_Matrix_row_degree(GrB_Vector deg, GrB_Matrix A);

/* R-MAT edge list (Chakrabarti, Zhan & Faloutsos 2004) written to device
 * arrays src_dev[nedges], dst_dev[nedges].  Edge e chooses a quadrant at
 * each of `scale` levels, most significant bit first, from draw
 * k = e*scale + level of a SplitMix64 stream (Steele, Lea & Flood 2014)
 * seeded with `seed`, as u = (draw >> 11) * 2^-53: u < t_a -> no bit,
 * u < t_ab -> destination bit, u < t_abc -> source bit, else both.  The
 * library only uses this to produce inputs; it is not part of any
 * GraphBLAS operation.  GrB_INVALID_VALUE unless 1 <= scale <= 31. */
GrB_Info GrM_rmat_edges(uint32_t *src_dev, uint32_t *dst_dev, int scale,
                        GrB_Index nedges, uint64_t seed, double t_a,
                        double t_ab, double t_abc);

/* Web-shaped synthetic graph: a stand-in for the crawl the paper measures
 * on (Section IV: 50.6M pages, 1.95B links, with strong locality and a
 * high mean degree), generated vertex by vertex from a SplitMix64 stream
 * seeded with `seed`.  All arithmetic is on unsigned 64-bit integers.
 * With D(c, r) = (c << 52) / ((r >> 12) + 1) (a Pareto-like draw:
 * P(D >= x) ~ c / x for x >= c) and draw(key) the stream's draw number key:
 *   vertex u: a = draw(u<<18 | 0x3FFFC), b = draw(u<<18 | 0x3FFFD);
 *     out-degree k_u = 0 if (a >> 48) < p_zero,
 *     else min(kmax, D(kmin, b));
 *   link j < k_u of u: r = draw(u<<18 | j<<2), q = draw(u<<18 | j<<2 | 1),
 *     t = r >> 48;
 *     t < p_home:            v = u & ~(2^h - 1), h = 6 + (r & 15)
 *                            (the first page of an enclosing aligned block);
 *     t < p_home + p_local:  d = min(n - 1, D(max(local_min, k_u), q)),
 *                            v = (u - d) mod n if bit 4 of r is set,
 *                            else (u + d) mod n;
 *     otherwise:             i = (D(hub, q) - hub) mod n,
 *                            v = (perm_a * i + perm_b) mod n.
 * Links are emitted as (u, v) in order of u, then j; self-loops and repeats
 * are kept (GrM_Matrix_build_edges drops and merges them).
 * Probabilities p_* are in units of 2^-16.  Requirements (else
 * GrB_INVALID_VALUE): 1 <= n < 2^32; 1 <= kmin <= kmax <= 4095;
 * 1 <= local_min, hub <= 4095; p_zero + p_home + p_local <= 65536;
 * perm_a coprime with n (so that i -> v is a bijection).
 * Call with src_dev == NULL to get the number of links in *nedges; then
 * with device arrays of at least `capacity` entries each
 * (GrB_INSUFFICIENT_SPACE if capacity < the count).  Temporary device
 * memory: 16 bytes per vertex plus the scan's workspace. */
typedef struct {
  int32_t kmin, kmax;               /* out-degree draw */
  int32_t p_zero, p_home, p_local;  /* units of 2^-16 */
  int32_t local_min;                /* smallest local link distance scale */
  int32_t hub;                      /* popularity scale of global links */
  uint32_t perm_a, perm_b;          /* vertex permutation of global links */
} GrM_WebModel;

GrB_Info GrM_web_edges(uint32_t *src_dev, uint32_t *dst_dev, GrB_Index capacity,
                       GrB_Index *nedges, GrB_Index n, uint64_t seed,
                       const GrM_WebModel *model);

/* ------------------------------------------------------------------------
 * Vectors with missing entries (Section III-A: a vector is stored full,
 * as a bitset or sparse).  A vector made by GrB_Vector_new, the import and
 * fill calls is full.  Operations on vectors with missing entries follow
 * the GraphBLAS meaning: eWiseMult keeps the positions present in both
 * inputs, eWiseAdd those present in either (op where both are, else the
 * present value), apply keeps the input's positions, reduce sums the
 * present values, and mxv gives w(i) where row i of A meets at least one
 * present u(j) -- except that a u with every entry present gives a w with
 * every entry present (an empty row holds 0, as the paper's mxv with the
 * initial value 0).  A mask restricts the positions an mxv or assign
 * writes (see the descriptors).  How a result is stored and which loop
 * computes it are chosen by naive fill-ratio estimates made when the
 * operation is recorded (Section III-D): the product of the inputs' fills
 * for eWiseMult, their union for eWiseAdd, 1 - (1 - f)^L for mxv with mean
 * row length L, times the mask's allowed share.  The choice never changes a
 * result beyond the order of a floating-point sum.  Calls that need every
 * entry present (the dense import/export calls, the PageRank drivers and
 * their vectors, fused PageRank passes) fail with GrB_INVALID_VALUE on a
 * vector that has missing entries.
 * ---------------------------------------------------------------------- */

typedef enum { GrM_FULL = 0, GrM_BITSET = 1, GrM_SPARSE = 2 } GrM_Format;

/* Number of present entries (forces the vector). */
GrB_Info GrB_Vector_nvals(GrB_Index *nvals, GrB_Vector v);
/* Remove every entry. */
GrB_Info GrB_Vector_clear(GrB_Vector v);
/* w := the entries (indices[k], values[k]), k < nvals, from host arrays;
 * repeated indices are combined with dup (GrB_INVALID_VALUE if dup is
 * NULL), GrB_INDEX_OUT_OF_BOUNDS for an index >= size(w).  The type of the
 * values must be w's. */
GrB_Info GrB_Vector_build_FP32(GrB_Vector w, const GrB_Index *indices, const float *values,
                               GrB_Index nvals, GrB_BinaryOp dup);
GrB_Info GrB_Vector_build_FP64(GrB_Vector w, const GrB_Index *indices, const double *values,
                               GrB_Index nvals, GrB_BinaryOp dup);
GrB_Info GrB_Vector_build_INT32(GrB_Vector w, const GrB_Index *indices, const int32_t *values,
                                GrB_Index nvals, GrB_BinaryOp dup);
/* The present entries into host arrays in ascending index order; *n holds
 * their capacity on entry (GrB_INSUFFICIENT_SPACE if below nvals) and the
 * count on return.  Values are converted to the function's type. */
GrB_Info GrB_Vector_extractTuples_FP32(GrB_Index *indices, float *values, GrB_Index *n, GrB_Vector v);
GrB_Info GrB_Vector_extractTuples_FP64(GrB_Index *indices, double *values, GrB_Index *n, GrB_Vector v);
GrB_Info GrB_Vector_extractTuples_INT32(GrB_Index *indices, int32_t *values, GrB_Index *n, GrB_Vector v);
/* w<mask> = x at every position (indices must be NULL, i.e. GrB_ALL, and
 * ni = size(w)); positions the mask does not allow keep w's old entries
 * unless the descriptor says replace.  accum must be NULL. */
GrB_Info GrB_Vector_assign_FP32(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, float x,
                                const GrB_Index *indices, GrB_Index ni, GrB_Descriptor desc);
GrB_Info GrB_Vector_assign_FP64(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, double x,
                                const GrB_Index *indices, GrB_Index ni, GrB_Descriptor desc);
GrB_Info GrB_Vector_assign_INT32(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, int32_t x,
                                 const GrB_Index *indices, GrB_Index ni, GrB_Descriptor desc);
/* How v is stored now (forces it). */
GrB_Info GrM_Vector_format(GrM_Format *fmt, GrB_Vector v);
/* 0 (default): estimates choose the storage of results with missing
 * entries; 1: always bitset; 2: always sparse.  Results are the same. */
GrB_Info GrM_set_format_policy(int policy);

/* ------------------------------------------------------------------------
 * Operations (GraphBLAS C API forms, destructive output as in the C
 * specification; the paper's Julia methods return new nodes instead,
 * Section III-A).  mask and accum must be NULL unless stated.  Output
 * vectors are overwritten entirely.  Operand types must equal the
 * operator's type (INT32 inputs are accepted and converted by the unary
 * apply forms).
 * ---------------------------------------------------------------------- */

/* w<mask> = A (+.*) u.  A is nrows x ncols, u has ncols entries, w nrows.
 * With every entry of u present an empty row gives the monoid identity 0;
 * otherwise see "Vectors with missing entries".  mask may be NULL; accum
 * must be NULL.
 * Defined by: the paper's mxv method (Section III-A, Fig. 3: identity,
 * add and multiply operators over a matrix and a vector) as the PageRank
 * loop uses it (Fig. 6: identity 0, add +, multiply "second" over the
 * transposed adjacency).  On a pattern matrix plus-second and plus-times
 * agree.  In nonblocking mode this is the anchor the matcher fuses with the
 * elementwise operations around it (Section II, Section IV). */
GrB_Info GrB_mxv(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum,
                 GrB_Semiring op, GrB_Matrix A, GrB_Vector u, GrB_Descriptor desc);

/* w(i) = op(u(i), v(i)).  For full vectors the union (eWiseAdd) and the
 * intersection (eWiseMult) of the patterns coincide.
 * Defined by: ewise_mult of Figs. 1 and 2 (the elementwise product whose
 * generated loop the paper shows) and the ewise_mult / ewise_add calls of
 * the PageRank loop (Fig. 6: the division by the degree vector, the
 * teleport addition and the absolute difference behind the residual). */
GrB_Info GrB_Vector_eWiseMult_BinaryOp(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum,
                                       GrB_BinaryOp op, GrB_Vector u, GrB_Vector v,
                                       GrB_Descriptor desc);
GrB_Info GrB_Vector_eWiseAdd_BinaryOp(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum,
                                      GrB_BinaryOp op, GrB_Vector u, GrB_Vector v,
                                      GrB_Descriptor desc);

/* w(i) = op(u(i)).
 * Defined by: the apply method (Fig. 2's inner apply, Fig. 4's iterator
 * form of it, Section III-B). */
GrB_Info GrB_Vector_apply(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum,
                          GrB_UnaryOp op, GrB_Vector u, GrB_Descriptor desc);
/* w(i) = op(s, u(i)) and w(i) = op(u(i), s) with a host scalar s.
 * Defined by: an elementwise operation with an iso-valued vector (Section
 * III-B: vectors whose entries all hold one value); Fig. 6 builds the
 * teleport term as such a vector and adds it with ewise_add. */
GrB_Info GrB_Vector_apply_BinaryOp1st_FP64(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum,
                                           GrB_BinaryOp op, double s, GrB_Vector u,
                                           GrB_Descriptor desc);
GrB_Info GrB_Vector_apply_BinaryOp2nd_FP64(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum,
                                           GrB_BinaryOp op, GrB_Vector u, double s,
                                           GrB_Descriptor desc);
/* w(i) = op(u(i), s) with s a (possibly pending) GrB_Scalar.
 * Defined by: the same iso-vector form with the value held by a scalar
 * object (Fig. 6 keeps the residual in a GraphBLAS scalar); a pending
 * scalar stays on the device, so the dangling share of the uniform
 * PageRank variant never goes through the host. */
GrB_Info GrB_Vector_apply_BinaryOp2nd_Scalar(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum,
                                             GrB_BinaryOp op, GrB_Vector u, GrB_Scalar s,
                                             GrB_Descriptor desc);

/* s = sum of u (plus monoid only), accumulated in FP64.  The _Scalar form
 * is recorded lazily; the _FP64 form forces and synchronises.
 * Defined by: the reduce of the PageRank loop (Fig. 6: the plus reduction
 * of the absolute differences that gives the residual, read through the
 * scalar in the loop test).  The paper accumulates in FP32; this library
 * accumulates in FP64. */
GrB_Info GrB_Vector_reduce_Monoid_Scalar(GrB_Scalar s, GrB_BinaryOp accum, GrB_Monoid monoid,
                                         GrB_Vector u, GrB_Descriptor desc);
GrB_Info GrB_Vector_reduce_FP64(double *s, GrB_BinaryOp accum, GrB_Monoid monoid,
                                GrB_Vector u, GrB_Descriptor desc);

/* s = sum of u(i) over the i selected by the value mask `mask` (mask(i) !=
 * 0), or by its complement when desc is GrB_DESC_C.  Project extension: the
 * C API's reduce takes no mask.  With mask = the inverse out-degree vector
 * and GrB_DESC_C this is the dangling mass sum_{outdeg(j)=0} u(j). */
GrB_Info GrM_Vector_reduce_masked_Scalar(GrB_Scalar s, GrB_Vector mask, GrB_Monoid monoid,
                                         GrB_Vector u, GrB_Descriptor desc);

/* ------------------------------------------------------------------------
 * PageRank drivers.  They issue the operations above (so the nonblocking
 * matcher and the plan cache are on their path) and add device-side loop
 * control so the host reads the residual only every `check_every`
 * iterations (GrM_pagerank and GrM_ppr queue two more iterations behind
 * each read, so the device keeps working while the host decides);
 * iterations past convergence are skipped on the device, so the iteration
 * count is the same as with a check after every pass.
 * ---------------------------------------------------------------------- */

typedef enum { GrM_DANGLING_DROP = 0, GrM_DANGLING_UNIFORM = 1 } GrM_Dangling;

/* PageRank of the graph whose transposed adjacency pattern is AT (n x n),
 * with out-degrees outdeg (n entries, any numeric type), following the loop
 * of Fig. 6: w = x .* (damping ./ outdeg); s = AT (+.second) w;
 * r = c + s; rho = sum |x - r|; repeat while iterations < itermax and
 * rho > tol (rho = 1 before the first pass).  GrM_DANGLING_DROP uses
 * c = (1-damping)/n as the paper does; GrM_DANGLING_UNIFORM uses
 * c = (1-damping)/n + damping * D/n with D the rank held by vertices of
 * out-degree 0, so the ranks sum to one.  r (FP32 or FP64, n entries)
 * receives the result and fixes the arithmetic type; the residual and D
 * are accumulated in FP64.  x0 is the start vector (NULL: every entry 1/n).
 * *iters = passes performed, *resid = last rho.  check_every >= 1. */
GrB_Info GrM_pagerank(GrB_Vector r, int *iters, double *resid, GrB_Matrix AT,
                      GrB_Vector outdeg, double damping, double tol, int itermax,
                      GrM_Dangling dangling, GrB_Vector x0, int check_every);

/* Personalised PageRank: as GrM_pagerank with the uniform 1/n teleport
 * replaced by the distribution `teleport` (r's type, entries summing to
 * one, typically 1/|S| on a seed set S):  r = s + (1-damping) v, plus, in
 * GrM_DANGLING_UNIFORM, damping * D * v (the dangling mass returns to the
 * seeds).  x0 = NULL starts from the teleport vector. */
GrB_Info GrM_ppr(GrB_Vector r, int *iters, double *resid, GrB_Matrix AT, GrB_Vector outdeg,
                 GrB_Vector teleport, double damping, double tol, int itermax,
                 GrM_Dangling dangling, GrB_Vector x0, int check_every);

/* Batched personalised PageRank of k seed sets (1 <= k <= 64), iterated
 * together as one sparse x dense product per pass.  Seed set q is
 * seed_vtx[seed_ptr[q] : seed_ptr[q+1]] (host int32 arrays; non-empty,
 * distinct vertices in [0, n)); its teleport vector is 1/|S_q| on the set.
 * Column q follows GrM_ppr exactly (start = teleport vector, the dangling
 * mass returns to the seeds in GrM_DANGLING_UNIFORM), with the residual and
 * dangling mass of every column in FP64, and stops where GrM_ppr would:
 * at the first pass whose residual is <= tol, or after itermax passes.  A
 * stopped column keeps the ranks of that pass (later passes carry them
 * forward unchanged); as columns stop, the product narrows to the running
 * ones (multiples of 16 columns), and the last eight or fewer finish as
 * single-vector solves, so the passes of the slowest sets cost less than
 * full-width passes.  X (device, n x k
 * row-major, `type` FP32 or FP64) receives in column q the ranks of the
 * pass column q stopped at; *iters the passes of the longest-running
 * column; col_iters[q] (host, may be NULL) the pass at which column q's
 * residual first was <= tol (-1 if never within itermax); col_resid[q]
 * (host, may be NULL) column q's residual at its last pass (1 when no
 * pass ran).
 * Defined by: the loop of Fig. 6 with the mxv over one vector replaced by
 * the product with k of them (one per seed set). */
GrB_Info GrM_ppr_batch(void *X, GrB_Type type, int k, const int32_t *seed_ptr,
                       const int32_t *seed_vtx, GrB_Matrix AT, GrB_Vector outdeg, double damping,
                       double tol, int itermax, GrM_Dangling dangling, int check_every, int *iters,
                       int *col_iters, double *col_resid);

/* Personalised PageRank of nsets seed sets through k column slots
 * (1 <= k <= 64) of the batched pass: the first k sets start together; a
 * column stops at the first pass whose residual is <= tol (frozen there)
 * or after itermax passes, and at the next check (every check_every
 * passes) its ranks are written out and the column restarts with the next
 * set, so one pass serves up to k queries.  Once no set is waiting and at
 * most half the columns still run, the product narrows to them.
 * Seed sets as in GrM_ppr_batch.  X (device, nsets x n of `type` FP32 or
 * FP64) receives set q's ranks at X + q n in the original numbering;
 * set_iters[q] (host, may be NULL) the pass at which its residual first
 * was <= tol (-1 if never within itermax), set_passes[q] the passes it ran
 * (its ranks are that iterate: set_iters[q] when it converged, else
 * itermax), set_resid[q] its residual at that pass.  Each set's ranks
 * equal GrM_ppr's after set_passes[q] passes. */
GrB_Info GrM_ppr_stream(void *X, GrB_Type type, int nsets, const int32_t *seed_ptr,
                        const int32_t *seed_vtx, GrB_Matrix AT, GrB_Vector outdeg, double damping,
                        double tol, int itermax, GrM_Dangling dangling, int k, int check_every,
                        int *set_iters, int *set_passes, double *set_resid);

/* ------------------------------------------------------------------------
 * Many independent graphs in one launch.  A multigraph packs copies of
 * ngraphs transposed adjacency patterns AT[g] (square; each graph's
 * out-degrees are the column counts of its AT) with their vertices
 * renumbered by decreasing out-degree.  GrM_pagerank_many then solves the
 * global PageRank of every graph (the loop of GrM_pagerank, uniform start,
 * each graph stopping at its own residual <= tol or itermax passes) in one
 * persistent kernel, captured in a HIP graph on first use for a given
 * (type, damping, tol, itermax, dangling, X) and replayed afterwards.
 * X (device, total vertices entries of `type`) receives the ranks of graph
 * g at offsets voff[g] .. voff[g+1] in the graph's original numbering;
 * iters / resid (host arrays of ngraphs, may be NULL) receive each graph's
 * passes and last residual (reading them synchronises, and reports
 * GrB_PANIC if a team of workgroups gave up waiting for a member).
 *
 * Graphs much larger than the mean share of one compute unit are solved
 * by a team of up to GrM_set_many_team_max workgroups (default 8; 1 solves
 * every graph with one workgroup), sized when the multigraph is created.
 * ---------------------------------------------------------------------- */
typedef struct GB_Multigraph_opaque *GrM_Multigraph;
GrB_Info GrM_set_many_team_max(int max_team);
/* Test hook for the failure path, for callers that test error handling: a
 * team member gives up a barrier wait after `ticks` of the 100 MHz wall
 * clock (default 1e9, ten seconds), flags the launch and exits; the next
 * GrM_pagerank_many that reads iters or resid then returns GrB_PANIC.  The
 * limit is part of the captured launch's key. */
GrB_Info GrM_set_many_team_wait(unsigned long long ticks);
GrB_Info GrM_Multigraph_new(GrM_Multigraph *mg, int ngraphs, const GrB_Matrix *AT);
GrB_Info GrM_Multigraph_free(GrM_Multigraph *mg);
/* voff: host array of ngraphs + 1 vertex offsets. */
GrB_Info GrM_Multigraph_offsets(int64_t *voff, GrM_Multigraph mg);
GrB_Info GrM_pagerank_many(void *X, GrB_Type type, GrM_Multigraph mg, double damping, double tol,
                           int itermax, GrM_Dangling dangling, int *iters, double *resid);

/* ------------------------------------------------------------------------
 * Tile plans.  The row-parallel kernels (mxv and the fused PageRank pass)
 * walk a plan of row tiles built once per matrix and configuration on the
 * host (the analogue of the paper's compiled-kernel cache keyed by a method
 * signature, Section III-C):
 *   kernel       0: one workgroup per tile; 1: one wavefront per tile;
 *                2: stripes of rows (kernel 2 below); 3: the same stripes
 *                in two phases (kernel 3 below)
 *   lds_entries  entries a tile stages in LDS (kernel 0: 1024, 2048 or 4096;
 *                kernel 1: 512)
 *   lds_rows     rows per tile (kernel 0: 512 with 1024 entries, else 1024;
 *                kernel 1: 256)
 *   long_row     rows with more entries get a tile of their own
 *                (1 <= long_row <= chunk)
 *   chunk        rows with more entries than this are split into chunks
 *                of this size reduced by several workgroups
 *                (long_row <= chunk <= lds_entries)
 *   grid         persistent workgroups (0: 8 per compute unit)
 * Kernel 2 (FP32 ranks only; other types run kernel 1) cuts the rows into
 * stripes of at most 8064 rows whose sums stay in LDS while the columns
 * are visited in blocks of 12288: a stripe loads the blocks holding the
 * most of its entries into LDS one at a time (at most hot/12288 of them,
 * only blocks holding at least long_row of its entries, 1024 when long_row
 * is 0, and only among the first 16383 blocks when there are more than
 * 16384) and gathers its other entries from memory.
 * Row sums are exact 64-bit fixed-point sums of the FP32 terms scaled by
 * 2^F, F = 62 - ceil(log2(sum |w|)), rounded once to FP32, so
 * they do not depend on the order of accumulation; the truncation of each
 * term to the fixed-point grid adds at most (row length) * 2^-F to a row
 * sum.  chunk 1 reads a stripe's packed entries with the nontemporal cache
 * hint (any other value: the default policy); lds_entries, lds_rows and
 * xcd_split are ignored; grid is the number of workgroups (0: one per
 * compute unit).  Matrices with 2^30 or
 * more columns or 2^31 or more entries run kernel 1 instead.
 * Kernel 3 is kernel 2 with the gathers replaced by a first phase: a list
 * of the stripes' other entries ordered by column block streams each block
 * of the vector through LDS and writes every entry's value into its slot,
 * and the pass then reads those values in sequence.  Same parameters, same
 * exact sums (bit-identical results to kernel 2), two launches per pass,
 * and 10 more bytes per gathered entry held with the plan (its slot and
 * its column within the block, in place of its column).
 * The choice never changes results beyond floating-point reassociation.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t kernel;   /* 0: workgroup tiles; 1: wavefront tiles (lds_entries 512,
                       lds_rows 256, 1024-thread workgroups); 2: row stripes
                       with their densest column blocks in LDS (FP32 only;
                       see below); 3: kernel 2 in two phases */
  int32_t lds_entries;
  int32_t lds_rows;
  int32_t long_row;
  int32_t chunk;
  int32_t grid;
  int32_t hot;      /* kernel 1: leading entries of the gathered vector kept in
                       LDS (clamped to what fits); kernels 2 and 3: columns
                       a stripe may hold in LDS (whole blocks of 12288, 0:
                       63 blocks) */
  int32_t relabel;  /* GrM_pagerank: 1 runs on a copy of the matrix with the
                       vertices renumbered by decreasing out-degree (built once
                       and cached with the matrix), so the most gathered values
                       come first; 0 runs on the matrix as given */
  int32_t xcd_split; /* 1: the tile list is cut into 8 contiguous ranges and
                       workgroup b works only in range b mod 8 (the XCD the
                       hardware places it on), so each XCD's L2 serves one
                       region of the matrix; 0: tiles interleaved over all
                       workgroups.  Ignored when grid is not a multiple of 8 */
} GrM_PlanConfig;

/* Use cfg for A's kernels computing in `type` (FP32 or FP64); NULL goes
 * back to the default.  GrB_INVALID_VALUE for an unsupported geometry. */
GrB_Info GrM_Matrix_plan_set(GrB_Matrix A, GrB_Type type, const GrM_PlanConfig *cfg);
/* The configuration A's kernels computing in `type` would use now. */
GrB_Info GrM_Matrix_plan_get(GrM_PlanConfig *cfg, GrB_Matrix A, GrB_Type type);

/* Autotuner: time candidate plan configurations of the fused PageRank pass
 * on AT (a few fixed-length GrM_pagerank runs each, with outdeg as its
 * out-degree vector, computing in `type`), install the fastest for AT and
 * return it in *chosen (and its time per pass in *us_per_pass, or -1 when
 * it came from the cache).  cache_path (may be NULL) names a text file of
 * earlier choices keyed by the matrix signature (dimension, entries,
 * longest row, value type, compute units): a hit installs the stored
 * choice without timing; a miss appends the new choice.  Candidates only
 * differ in speed, never beyond rounding in results. */
GrB_Info GrM_autotune_pagerank(GrM_PlanConfig *chosen, double *us_per_pass, GrB_Matrix AT,
                               GrB_Vector outdeg, GrB_Type type, const char *cache_path);

/* ------------------------------------------------------------------------
 * Learned warm start for personalised PageRank.  A network predicts the
 * start vector x0 of GrM_ppr for one seed set S on a graph given as A
 * (rows = sources) and A^T (both square n x n, the same pattern), from 11
 * features per vertex v:
 *   x[0] = 1 if v in S, x[1] = log(1 + indeg v), x[2] = log(1 + outdeg v),
 *   x[2+t] = log(1 + n c_t(v) / W), t = 1..8,
 * where c_t(v) counts the W random walkers at v after step t: walker w
 * starts at S[w mod |S|]; at step t, with u from draw 4(8w + t - 1) of the
 * SplitMix64 stream of `seed` (top 53 bits, scaled to [0,1)), it restarts at
 * S[r mod |S|] (r = the next draw) when u < 1 - damping or its vertex has no
 * out-edge, else follows out-edge r mod outdeg (r = the draw after that).
 * The walkers' distribution after t steps is the t-th personalised
 * PageRank iterate from the teleport start.  Network (parameter vector
 * theta of GRM_GNN_NPARAMS FP32 values in this order: W1s[64][11],
 * W1n[64][11], b1[64], w2s[64], w2n[64], b2):
 *   m_v = mean of x over in-neighbours (0 without any)
 *   h_v = ReLU(W1s x_v + W1n m_v + b1)
 *   z_v = w2s . h_v + b2 + mean over in-neighbours u of w2n . h_u
 *   x0  = softmax(z), or the teleport vector (1/|S| on S) when z has a
 *         non-finite value or the normaliser is not finite and positive.
 * Training minimises KL(x* || x0) for target ranks x*.  Activations (x, m,
 * h) are stored in the network's activation type (GrB_FP32 or GrM_BF16),
 * weights in FP32, sums accumulated in FP32, weight gradients and the
 * softmax normaliser in FP64.  The calls enqueue on the library stream; a
 * network keeps work space for the graph it was last used with.
 * ---------------------------------------------------------------------- */
#define GRM_GNN_FEATURES 11
#define GRM_GNN_HIDDEN 64
#define GRM_GNN_NPARAMS 1601
typedef struct GB_GNN_opaque *GrM_GNN;
/* New network: Glorot-uniform weights from the SplitMix64 stream of
 * init_seed (draw i for parameter i), zero biases, Adam state cleared. */
GrB_Info GrM_GNN_new(GrM_GNN *net, GrB_Type act, uint64_t init_seed);
GrB_Info GrM_GNN_free(GrM_GNN *net);
/* theta: host array of GRM_GNN_NPARAMS floats (set also clears Adam). */
GrB_Info GrM_GNN_set_params(GrM_GNN net, const float *theta);
GrB_Info GrM_GNN_get_params(GrM_GNN net, float *theta);
/* grad: host array of GRM_GNN_NPARAMS doubles, the accumulated gradient. */
GrB_Info GrM_GNN_get_grad(GrM_GNN net, double *grad);
/* Device pointer and element count of a work buffer of the last graph
 * (synchronises): 0 walk counts (INT32, 8 x n), 1 features x, 2 means m
 * (activation type, n x 16 row-major, columns 11..15 zero), 3 hidden h (n
 * x 64), 4 a = w2s.h + b2, 5 q = w2n.h, 6 z, 7 x0, 8 dL/dq (FP32, n). */
GrB_Info GrM_GNN_buffer(GrM_GNN net, int which, void **ptr, int64_t *count);
/* Features of seed set seeds[0:nseeds) (host, distinct, in [0, n)) with
 * `walkers` walks (1 <= walkers <= 2^26) at `damping`. */
GrB_Info GrM_gnn_features(GrM_GNN net, GrB_Matrix A, GrB_Matrix AT, const int32_t *seeds, int nseeds,
                          int walkers, double damping, uint64_t seed);
/* z and x0 from the current features; *fell_back (may be NULL; reading it
 * synchronises) is 1 when x0 is the teleport vector. */
GrB_Info GrM_gnn_forward(GrM_GNN net, GrB_Matrix A, GrB_Matrix AT, int *fell_back);
/* Gradient of KL(x* || x0) after GrM_gnn_forward: x_star (device FP32,
 * element v at x_star[v * stride]) is the target; the gradient replaces
 * (accumulate 0) or adds to (1) the network's gradient; *loss (may be
 * NULL; reading it synchronises) receives the KL value. */
GrB_Info GrM_gnn_backward(GrM_GNN net, GrB_Matrix A, GrB_Matrix AT, const float *x_star, int64_t stride,
                          int accumulate, double *loss);
/* Adam step (Kingma & Ba, 2015, with bias correction) on grad * grad_scale. */
GrB_Info GrM_gnn_adam_step(GrM_GNN net, double lr, double beta1, double beta2, double eps, double grad_scale);
/* Features + forward, then x0 (FP32 or FP64 vector of length n) = the
 * prediction: a start vector for GrM_ppr. */
GrB_Info GrM_gnn_predict_x0(GrB_Vector x0, GrM_GNN net, GrB_Matrix A, GrB_Matrix AT, const int32_t *seeds,
                            int nseeds, int walkers, double damping, uint64_t seed, int *fell_back);

/* ------------------------------------------------------------------------
 * Bandwidth probe: dst_dev[0:bytes) = src_dev[0:bytes) with a streaming
 * copy kernel (bytes a multiple of 16, pointers 16-byte aligned).
 * ---------------------------------------------------------------------- */
GrB_Info GrM_stream_copy(void *dst_dev, const void *src_dev, size_t bytes);

/* Per-launch timing of fused PageRank kernels (HIP events recorded around
 * every fused launch on the library stream while enabled).  GrM_timing_read
 * synchronises, returns the summed duration and the number of launches
 * recorded since the previous read, and drops those records.  The count
 * includes passes the device loop guard turned into no-ops (a driver
 * enqueues check_every passes between host checks). */
GrB_Info GrM_timing_enable(bool on);
GrB_Info GrM_timing_read(double *total_ms, int64_t *launches);

/* ------------------------------------------------------------------------
 * Allocation-free sum, for callers that cannot allocate device memory (code
 * under stream capture, serving loops, hosts that forbid allocation).
 *
 * *sum_dev = the sum of x_dev[0:n) in FP64, enqueued on the library stream.
 * Same kernel, grid and summation order as GrB_Vector_reduce_FP64 on a full
 * vector holding the same n values, so the two give bit-identical sums.
 *   sum_dev  device, one double, written (not accumulated into);
 *   x_dev    device, n values of `type` (GrB_FP32 or GrB_FP64), read only;
 *            may be NULL when n == 0 (the sum is then 0);
 *   n        at most GRM_NOALLOC_MAX_N.
 * The call allocates nothing and does not synchronise.  Its scratch (one
 * FP64 partial per workgroup, at most 1024, and a completion ticket: 8.4 KB)
 * is a static device array that every call on a device shares; GrB_init
 * locates this device's copy.  Two calls that overlap on one device (other
 * streams or host threads) race on it and give wrong sums; calls in stream
 * order are safe.  Errors: GrB_NULL_POINTER (sum_dev, type, or x_dev with
 * n > 0), GrB_DOMAIN_MISMATCH (type not FP32/FP64), GrB_INVALID_VALUE
 * (n > GRM_NOALLOC_MAX_N), GrB_PANIC (launch failure).
 * ---------------------------------------------------------------------- */
#define GRM_NOALLOC_MAX_N (1ull << 40)
GrB_Info GrM_reduce_dense_noalloc(double *sum_dev, const void *x_dev, GrB_Type type, GrB_Index n);

#ifdef __cplusplus
}
#endif

#endif /* NBGRB_H */
