// Internal interface between the runtime (DAG, matcher, plans) and the
// gfx950 kernels.  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nbgrb {

// Value type codes of dense vector storage.
// T_BF16 is a storage type of network activations only.
enum TypeCode : int { T_BOOL = 0, T_INT32 = 1, T_FP32 = 2, T_FP64 = 3, T_BF16 = 4 };

inline size_t type_size(int t) {
  switch (t) {
    case T_BOOL: return 1;
    case T_BF16: return 2;
    case T_INT32: return 4;
    case T_FP32: return 4;
    default: return 8;
  }
}

// Closed operator set.
enum UnOp : int { U_IDENTITY = 0, U_ABS, U_AINV, U_MINV, U_MINV_OR_ZERO };
enum BinOp : int {
  B_PLUS = 0, B_MINUS, B_TIMES, B_DIV, B_MAX, B_MIN, B_FIRST, B_SECOND, B_ABSDIFF
};

// Device-side loop control of an iterative driver.  Kernels launched while
// a guard is installed return at once when `active` is 0; the reduction
// that produces the guarded residual updates it.
struct GuardDev {
  int active;       // 1 while another pass is wanted
  int iters;        // passes completed
  double rho;       // last residual
  double rho_prev;  // the one before (lets the host predict how many more)
  double tol;
  int itermax;
  int bad;          // set when a residual or dangling mass was not finite
};

// Scalar operand: value = dev ? alpha * (*dev) + beta : beta.
struct ScalarArg {
  const double* dev;
  double alpha;
  double beta;
};

// Dense operand of an elementwise kernel: storage of type `type`, or an
// iso value when p == nullptr.
struct Operand {
  const void* p;
  int type;
  double iso;
};

// Reduction target: the result goes to *out (FP64); if `guard` is set the
// reduction also advances the guard with its result.
struct ReduceOut {
  double* out;
  GuardDev* guard;
};

// Scratch of a deterministic two-level reduction (per-block partials + a
// ticket for the last block).  `partials` holds 2 * nblocks doubles.
struct RedScratch {
  double* partials;
  unsigned* ticket;  // zero before the launch; the last block resets it
};

// ------------------------------------------------------------------ tiles
// Row tiles of a CSR pattern for the row-parallel kernels (built once per
// matrix and tile geometry on the host).
//   STREAM tile  : {row0, nrows > 0, e0, ne}  rows [row0,row0+nrows), their
//                  ne entries start at e0; staged through LDS.
//   CHUNK tile   : {k, -(h+1), e0, ne} chunk k of hub row h; the block
//                  that completes the last chunk finishes the row.
// Every tile holds at most the kernel's LDS entry budget of entries.
// HubInfo h: {row, nchunks, first partial slot, first entry}.
struct TilePlanDev {
  const int4* tiles;
  int ntiles;
  const int4* hubs;
  int nhubs;
  int nparts;  // total chunk partial slots
  int xcd;     // 1: one contiguous tile range per XCD (workgroup b on XCD b mod 8)
};

// Epilogue of the fused PageRank pass, per row i with row sum s:
//   mode PLAIN : s_out[i] = s
//   mode PR    : r = tele(i) + s, tele(i) = tele_vec ? tele_vec[i] (* c when
//                tele_scaled) : c,
//                c = (T)(c.alpha * (*c.dev) + c.beta) or (T)c.beta;
//                r_out[i] = r; rho += |x_old[i] - r| (FP64);
//                w_out[i] = memo_div ? r / dvec[i] : r * dvec[i];
//                D += r where the mask selects i (FP64).
enum EpiMode : int { EPI_PLAIN = 0, EPI_PR = 1 };

template <typename T>
struct FusedArgs {
  const int* rowptr;
  const int* col;
  const T* w;  // gathered vector
  int nrows;
  int ncols;   // length of w
  int mode;
  T* s_out;
  T* r_out;
  const T* x_old;     // residual against this vector (nullptr: none)
  const T* dvec;      // prescale vector for the memo / the dvec mask
  T* w_out;           // memo output (nullptr: none)
  int memo_div;
  int do_D;
  int mask_is_dvec;   // mask = dvec (value mask)
  Operand mask;       // otherwise this vector
  int mask_comp;      // complement the mask
  const T* tele_vec;  // per-row teleport (nullptr: scalar c)
  int tele_scaled;    // teleport = tele_vec[i] * c instead of tele_vec[i]
  ScalarArg c;
  ReduceOut rho_out;
  ReduceOut D_out;
};

struct FusedScratch {
  double* wg_part;    // 2 per workgroup: (rho, D) partials
  double* hub_sum;    // one slot per hub chunk: chunk row sums
  int* hub_cnt;       // per hub: chunks finished (zero; the finisher resets)
  double* hub_red;    // 2 per hub: (rho, D) of the hub row
  unsigned* ticket;   // zero; the last workgroup resets it
};

// Geometry of the row-parallel kernels.
constexpr int FUSED_BLOCK = 256;

// ------------------------------------------------------------ launchers
// All launchers enqueue on `s` and return the launch status.

// Fused PageRank pass / plain SpMV over a tile plan.  grid = persistent
// workgroup count; tiles are assigned round-robin, so the per-workgroup
// partials are summed in a fixed order.  lds_entries = STREAM tile entry
// budget the plan was built for; lds_rows = its row budget.
hipError_t launch_fused_f32(const TilePlanDev& plan, const FusedArgs<float>& a,
                            const FusedScratch& scr, int grid, int lds_entries, int lds_rows,
                            const GuardDev* guard, hipStream_t s);
hipError_t launch_fused_f64(const TilePlanDev& plan, const FusedArgs<double>& a,
                            const FusedScratch& scr, int grid, int lds_entries, int lds_rows,
                            const GuardDev* guard, hipStream_t s);

// Wave-tiled fused pass: tiles of at most 512 entries and 256 rows, one
// wavefront each, 1024-thread workgroups (grid = persistent workgroups),
// the first hot_n entries of the gathered vector held in LDS (clamped to
// wave_hot_max(type)).
constexpr int WAVE_TILE_ENTRIES = 512;
constexpr int WAVE_TILE_ROWS = 256;
hipError_t launch_fused_wave_f32(const TilePlanDev& plan, const FusedArgs<float>& a,
                                 const FusedScratch& scr, int grid, int hot_n,
                                 const GuardDev* guard, hipStream_t s);
hipError_t launch_fused_wave_f64(const TilePlanDev& plan, const FusedArgs<double>& a,
                                 const FusedScratch& scr, int grid, int hot_n,
                                 const GuardDev* guard, hipStream_t s);
int wave_hot_max(int type);

// Stripe-blocked fused pass (FP32 only).  Rows of the pattern are cut into
// stripes of at most STRIPE_RMAX rows, one workgroup of STRIPE_BLOCK threads
// per stripe at a time, row sums in LDS as 64-bit fixed point; columns into
// blocks of STRIPE_HB values of the gathered vector, the `nb` blocks that
// hold most of a stripe's entries (listed ascending in blk) loaded into LDS
// in turn.  Blocks at or past STRIPE_MAXBLK - 1 are never loaded (one bin
// counts them all when the layout is built).
//   hot words   : (row in stripe + 1) << 16 | column in the block, one
//                 segment per (stripe, LDS block), sorted by row, padded to
//                 a multiple of 8 with zero words;
//   cold pairs  : column (uint32) and row in stripe + 1 (uint16) of the
//                 stripe's other entries, sorted by row, padded the same way.
// Row slot 0 takes the padding entries and is never read.
constexpr int STRIPE_BLOCK = 1024;
constexpr int STRIPE_RMAX = 8064;
constexpr int STRIPE_HB = 12288;
constexpr int STRIPE_NBMAX = 63;  // segment starts 0..nb sit one per lane of a wavefront
constexpr int STRIPE_K = 8;  // consecutive entries per lane
constexpr int STRIPE_MAXBLK = 16384;

struct StripeDesc {
  int r0, nrows, nb, cold_n;    // rows [r0, r0 + nrows); LDS blocks; padded cold entries
  long long hot_base, cold_base;  // first hot word / cold pair of the stripe
  int seg[STRIPE_NBMAX + 1];    // hot segment of LDS block b: [seg[b], seg[b+1]) after hot_base
  int blk[STRIPE_NBMAX];        // column block of LDS block b (ascending)
  int pad[1];
};
static_assert(sizeof(StripeDesc) == 544, "stripe descriptor layout");

struct StripePlanDev {
  const StripeDesc* desc;
  const unsigned* hot;
  const unsigned* cold_col;       // gathered plan: column of each gathered entry
  const float* cold_val;          // two-phase plan: its value, filled before the pass
  const unsigned short* cold_row;
  const int* wg_off;   // workgroup g runs wg_list[wg_off[g] .. wg_off[g+1])
  const int* wg_list;
  double* wg_sum;      // per-workgroup sum |w'| (scratch)
  int nstripes;
  int maxlen;          // longest row
};

// Two-phase stripe plan: the stripes' gathered entries, listed by column
// block and then by their slot in the stripes' arrays.  Chunk c covers list
// entries [start, end) of column block blk; entry e's value is
// w[blk * STRIPE_HB + (src[e] & 0x3FFF)] and goes to slot pos(e).  Slots
// are stored per run: a run is a stretch of the list whose slots are
// consecutive; bit 15 of src[e] marks the first entry of a run, and run r
// starts at slot run_pos[r].  Chunks are cut into sub-chunks of
// FILL_SUB entries, each starting a run; sub-chunk j of chunk c has run
// index sub_run[c.sub0 + j] at its first entry.
constexpr unsigned FILL_SUB = 2048;
struct ColdChunk {
  int blk;
  unsigned start, end, sub0;
};
struct ColdFillDev {
  const unsigned short* src;
  const unsigned* run_pos;
  const unsigned* sub_run;
  const ColdChunk* chunk;
  float* val;
  int nchunks;
};
// Fills val for the pass that gathers w (ncols values).  Skipped when the
// guard is inactive.
hipError_t launch_cold_fill_f32(const ColdFillDev& f, const float* w, int ncols, const GuardDev* guard,
                                hipStream_t s);

// The fused pass over a stripe plan.  wsum_in: sum |w| of the gathered
// vector (sets the fixed-point scale; a non-finite value makes every row sum
// NaN).  wsum_out (may be null): receives sum |w'| of the pre-scaled copy
// written.  grid must be the plan's workgroup count.  nt_streams: the
// packed entries (LDS-block words, gathered columns and rows) are read with
// the nontemporal hint, which keeps them from displacing the gathered
// vector in the caches.
// prefilled: the plan is two-phase (values of the gathered entries are
// read from p.cold_val, filled by launch_cold_fill_f32 for this pass).
hipError_t launch_fused_stripe_f32(const StripePlanDev& p, const FusedArgs<float>& a, const double* wsum_in,
                                   double* wsum_out, const FusedScratch& scr, int grid, bool nt_streams,
                                   bool prefilled, const GuardDev* guard, hipStream_t s);
// *out = sum |x[i]| in FP64 (deterministic).
hipError_t launch_abssum_f32(const float* x, int64_t n, double* out, RedScratch scr, const GuardDev* guard,
                             hipStream_t s);

// Elementwise: out[i] = f(a[i], b[i]) computed in `ct` (T_FP32 / T_FP64).
//   kind 0: binary op(a, b); 1: unary op(a); 2: op(s, a); 3: op(a, s)
enum EwKind : int { EW_BINARY = 0, EW_UNARY = 1, EW_BIND1ST = 2, EW_BIND2ND = 3 };
hipError_t launch_ewise(int64_t n, int ct, int kind, int op, Operand a, Operand b,
                        ScalarArg sc, void* out, int out_type, const GuardDev* guard,
                        hipStream_t s);

// Deterministic sum of x (selected by mask when use_mask) into out.out.
constexpr int REDUCE_BLOCK = 256;
constexpr int REDUCE_GRID = 1024;
hipError_t launch_reduce(int64_t n, Operand x, int use_mask, Operand mask, int mask_comp,
                         ReduceOut out, RedScratch scr, const GuardDev* guard, hipStream_t s);

// out[0:n) = v converted to `type`.
hipError_t launch_fill(void* out, int type, int64_t n, double v, hipStream_t s);
// *dst = v (one double).
hipError_t launch_set_scalar(double* dst, double v, hipStream_t s);
// Copy with conversion between storage types.
hipError_t launch_convert(const void* src, int src_type, void* dst, int dst_type, int64_t n,
                          hipStream_t s);
// Guard := {active, 0 iterations, rho, tol, itermax}.
hipError_t launch_guard_init(GuardDev* g, int active, double tol, int itermax, hipStream_t s);
// Zero n bytes with a kernel (no memset node, safe under graph capture).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// R-MAT edges, one thread per edge.
hipError_t launch_rmat(uint32_t* src, uint32_t* dst, int scale, int64_t nedges, uint64_t seed,
                       double ta, double tab, double tabc, hipStream_t s);

// Streaming copy probe (bytes multiple of 16).
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// Row degree deg[i] = rowptr[i+1] - rowptr[i] written as `type`.
hipError_t launch_row_degree(const int* rowptr, int64_t n, void* deg, int type, hipStream_t s);

// CSR validity check: flag[0] != 0 afterwards if rowptr is not a valid
// non-decreasing 0..nnz sequence or a column is outside [0, ncols).
hipError_t launch_check_csr(const int* rowptr, int64_t nrows, const int* col, int64_t nnz,
                            int64_t ncols, int* flag, hipStream_t s);

// ------------------------------------------------------------ batched PPR
// One pass of k-column personalised PageRank over the wavefront-tile plan
// (spmm.hip).  x_old / w / x_new / w_new are n x k row-major.  Seeds are
// given sorted by vertex (seed_v ascending; seed_c its column, seed_w its
// weight 1/|S_c|).  d_prev[c] is the previous dangling mass of column c
// (nullptr: no redistribution); the teleport factor of column c is
// c_beta + c_alpha * d_prev[c].  hub_sum holds 64 slots per chunk,
// hub_red and wg_part 128 per hub / workgroup.
struct SpmmArgs {
  const int* rowptr;
  const int* col;
  int k;
  const void* w;
  unsigned w_bytes;       // size of w in bytes when below 4 GiB (buffer-addressed pass), else 0
  const int* tile_seed;   // per tile: first vertex-sorted seed at or after the tile's first row
  const void* x_old;
  const void* dvec;
  void* x_new;
  void* w_new;
  const int* seed_v;
  const int* seed_c;
  const double* seed_w;
  int nseeds;
  const double* d_prev;
  double c_alpha, c_beta;
  double* rho_out;  // k
  double* d_out;    // k
  int* hit;         // k: first pass with rho_c <= hit_tol (-1 before)
  double hit_tol;
  GuardDev* guard;
  double* hub_sum;
  int* hub_cnt;
  double* hub_red;
  double* wg_part;
  unsigned* ticket;
  // plain product (GrB_mxm): x_new = A (+.second) W and nothing else -- no
  // teleport, pre-scaled copy, residual or dangling mass; x_old, dvec,
  // seeds, tile_seed, the reductions and the guard are not used
  int plain;
  // the buffer-addressed pass leaves rows with no entries and no seed
  // untouched; the caller guarantees their x and w are zero in both the
  // input and the output buffers (every column)
  int skip_empty;
};
constexpr int SPMM_BLOCK = 1024;
hipError_t launch_spmm_ppr(const TilePlanDev& plan, const SpmmArgs& a, int type, int grid,
                           const GuardDev* guard, hipStream_t s);
hipError_t launch_spmm_tile_seed(const TilePlanDev& plan, const int* seed_v, int nseeds, int* out, hipStream_t s);
// Columns c with bit c of `cols` set: x_new = V, w_new = V .* d (both must
// be zero there beforehand), d_out = D0, hit = -1; other columns untouched.
hipError_t launch_spmm_init(const SpmmArgs& a, int type, const int* by_col_ptr, const int* by_col_v,
                            const double* by_col_w, uint64_t cols, hipStream_t s);
// Zero columns `cols` (bit mask) of the n x k arrays x and w.
hipError_t launch_spmm_zero_columns(void* x, void* w, int type, int64_t n, int k, uint64_t cols, hipStream_t s);
// For every column c with bit c of `cols` set: out[c][i * ld] =
// in[(idx ? idx[i] : i) * k + c], i < n (columns of the n x k array in
// vertex order), with in = in1 when bit c of from1 is set, else in0.
struct ColumnOutputs {
  void* out[64];
  int64_t ld;
};
hipError_t launch_spmm_columns_out(const void* in0, const void* in1, uint64_t from1, int type, const int* idx,
                                   int64_t n, int k, uint64_t cols, const ColumnOutputs& outs, hipStream_t s);
// Vector c < nc (n values at ins.in[c]) into column ins.dst[c] of the
// n-row array `out` whose rows are ins.ld values apart (0 <= dst < ld).
struct ColumnInputs {
  const void* in[64];
  int64_t dst[64];
  int64_t ld;
};
hipError_t launch_columns_in(const ColumnInputs& ins, int nc, int type, int64_t n, void* out, hipStream_t s);
// New column j < k2 of the n x k2 array x2 = column map.c[j] of the n x k
// array x (map.c[j] < 0: zeros), w2 = x2 .* dvec (dvec: n entries of the
// same type); d2[j] = d[map.c[j]] (0 when empty); hit[j] = -1 for a mapped
// column, 0 (frozen) otherwise, j < 64.
struct ColumnMap {
  int c[64];
};
hipError_t launch_spmm_compact(const void* x, const void* dvec, const double* d, void* x2, void* w2, double* d2,
                               int* hit, int type, int64_t n, int k, int k2, const ColumnMap& map, hipStream_t s);
// x[idx[j]] = v for j < cnt (x of `type` FP32 or FP64).
hipError_t launch_scatter_value(void* x, int type, const int* idx, int cnt, double v, hipStream_t s);
// out row i = in row idx[i] (n rows of k values).
hipError_t launch_rows_permute(const void* in, int type, const int* idx, void* out, int64_t n, int k,
                               hipStream_t s);

// ------------------------------------------------------------ many graphs
// One problem of the persistent many-graph launch (many.hip): n vertices,
// row pointers at rowptr + roff (n + 1 local offsets), columns at
// col + eoff, vertex arrays at + voff; lpr lanes reduce one row.
struct ManyGraph {
  int n, m, lpr, nlong;   // nlong rows longer than MANY_LONG_ROW entries
  int64_t voff, eoff, roff, loff;
  int team;               // workgroups solving this graph together, 1..MANY_MAX_TEAM
  int pad_;
};
constexpr int MANY_MAX_TEAM = 8;
// Rows with more entries are summed by the whole workgroup, not by one
// lane group, so no lane accumulates more than this many terms serially.
constexpr int MANY_LONG_ROW = 256;
struct ManyArgs {
  const ManyGraph* graphs;
  const int* queue;   // graph * MANY_MAX_TEAM + member: teams first, then single graphs, largest first
  int* queue_next;    // reset to 0 by the launch
  unsigned* team_bar;   // per graph: team arrivals, reset to 0 by the launch
  double* team_part;    // per graph: [barrier parity][member][residual, dangling]
  int* team_err;        // bit 0: a team member waited too long; bit 1: a residual was not finite (reset by the launch)
  unsigned long long team_wait_ticks;  // give-up limit of a team wait, in 100 MHz wall-clock ticks
  int ngraphs;
  int nslots;         // queue entries: one per team member, one per single graph
  const int* rowptr;
  const int* col;
  const int* deg;     // out-degree per vertex (execution numbering)
  const int* inv;     // per graph: position of original vertex v
  const int* longrows;  // per graph at loff: its long rows, ascending
  void* xa;
  void* xb;
  void* wa;
  void* wb;
  void* out;          // ranks in the original numbering
  int* iters;
  double* resid;
  double damping, tol;
  int itermax, uniform;
};
// Queue, barrier and error reset + the persistent kernel (grid workgroups of
// 1024 threads; the team slots at the head of the queue must number at most grid).
hipError_t launch_pr_many(const ManyArgs& a, int type, int grid, hipStream_t s);

// ------------------------------------------------------------ graph build
// (graph_build.hip) Sort-based construction of a CSR pattern from an edge
// list.  Temporary device memory comes from `alloc` / `release`.
typedef void* (*AllocFn)(size_t bytes, void* ctx);
typedef void (*ReleaseFn)(void* p, void* ctx);

// Builds rowptr (n+1) and col (capacity nedges) from (src,dst); *nnz gets
// the number of distinct edges.  bad_flag[0] is set if an endpoint >= n.
// Synchronises `s` once to read the count back.
hipError_t build_csr_from_edges(int64_t n, const uint32_t* src, const uint32_t* dst,
                                int64_t nedges, bool drop_self, int* rowptr, int* col,
                                int64_t* nnz, int* bad_flag, AllocFn alloc, ReleaseFn release,
                                void* actx, hipStream_t s);

// Transpose of an nrows x ncols pattern: rowptrT (ncols+1), colT (nnz).
hipError_t transpose_csr(int64_t nrows, int64_t ncols, const int* rowptr, const int* col,
                         int64_t nnz, int* rowptrT, int* colT, AllocFn alloc,
                         ReleaseFn release, void* actx, hipStream_t s);

// cnt[col[e]] += 1 for every entry (cnt zeroed by the caller).
hipError_t launch_column_count(const int* col, int64_t nnz, int* cnt, hipStream_t s);
// Vertex order by decreasing column count of an n x n pattern (ties by
// increasing id): order[k] = vertex at position k, inv[v] = position of v.
hipError_t degree_order(int64_t n, const int* col, int64_t nnz, int* order, int* inv, AllocFn alloc,
                        ReleaseFn release, void* actx, hipStream_t s);
// The pattern with rows and columns renumbered by inv (both sorted again).
hipError_t permute_csr(int64_t n, const int* rowptr, const int* col, int64_t nnz, const int* inv,
                       int* rowptr2, int* col2, AllocFn alloc, ReleaseFn release, void* actx,
                       hipStream_t s);
// out[i] = in[0] + ... + in[i] for i < n (unsigned, wrapping).  Synchronises `s`.
hipError_t scan_u32_inclusive(const unsigned* in, unsigned* out, int64_t n, AllocFn alloc, ReleaseFn release,
                              void* actx, hipStream_t s);
// Sorts n (key, value) pairs by key bits [0, end_bit) (stable); the inputs
// are left as they were.  Synchronises `s`.
hipError_t sort_pairs_u64_u16(const uint64_t* keys_in, uint64_t* keys_out, const uint16_t* vals_in,
                              uint16_t* vals_out, int64_t n, unsigned end_bit, AllocFn alloc,
                              ReleaseFn release, void* actx, hipStream_t s);
// out[k] = in[idx[k]] for k < n, storage type `type`.
hipError_t launch_permute(const void* in, int type, const int* idx, void* out, int64_t n, hipStream_t s);

}  // namespace nbgrb
