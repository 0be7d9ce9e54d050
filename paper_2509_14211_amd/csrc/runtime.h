// Host-side runtime of the nonblocking GraphBLAS library: device memory,
// versioned objects, the DAG of pending operations and its scheduler.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.h"
#include "../../include/nbgrb.h"

namespace nbgrb {

// Internal error carrying a GraphBLAS return code; caught at the C ABI.
struct GrbError {
  GrB_Info info;
  std::string msg;
};

[[noreturn]] void fail(GrB_Info info, const std::string& msg);
void hip_check(hipError_t e, const char* what);

// ------------------------------------------------------------ device memory

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf();
};
using BufP = std::shared_ptr<DevBuf>;

// Allocate from the size-keyed cache (or the allocator on a miss).
BufP dev_alloc(size_t bytes);

// ------------------------------------------------------------ operators

struct OpInfo {
  int kind;  // 0 unary, 1 binary
  int op;
  int type;
};

// ------------------------------------------------------------ matrices

struct Plan;
struct MatData;
using MatP = std::shared_ptr<MatData>;

// The same pattern with vertices renumbered by decreasing out-degree
// (column count): order[k] = old vertex at position k, inv[v] = position
// of old vertex v.
struct Relabeled {
  MatP A;
  BufP order, inv;
};

struct MatData {
  uint64_t id = 0;
  int64_t nrows = 0, ncols = 0, nnz = 0;
  BufP rowptr, col;
  std::map<std::tuple<int, int, int, int, int, int, int>, std::shared_ptr<Plan>> plans;
  std::shared_ptr<Relabeled> relabeled;
  std::shared_ptr<MatData> transposed;  // built on demand for push-style mxv
  BufP long_rows;                       // rows longer than SV_LONG_ROW, for the pull mxv (on demand)
  int64_t nlong = -1;                   // their count; -1 until computed
  // A dense matrix (the operand and result of GrB_mxm) holds nrows x ncols
  // values of type dense_type, row-major, in `dense`, and no pattern.
  BufP dense;
  int dense_type = -1;
};

// Kernel family of a plan.
enum KernelKind : int { K_BLOCK = 0, K_WAVE = 1, K_STRIPE = 2, K_STRIPE2 = 3 };
inline bool is_stripe(int kernel) { return kernel == K_STRIPE || kernel == K_STRIPE2; }

// Tile plan of one matrix for the row-parallel kernels.
struct PlanConfig {
  int kernel = K_BLOCK;    // block-tiled or wave-tiled pass
  int lds_entries = 2048;  // STREAM tile entry budget
  int lds_rows = 1024;     // STREAM tile row budget
  int long_row = 2048;     // rows longer than this get a tile of their own;
                           // stripe kernel: fewest entries that make a stripe load a block
  int chunk = 2048;        // rows longer than this are split in chunks (<= lds_entries)
  int grid = 0;            // persistent workgroups (0: from the device)
  int hot = 0;             // wave kernel: leading gathered entries kept in LDS;
                           // stripe kernel: leading columns in LDS blocks (0: all 32 blocks)
  int relabel = 0;         // drivers: run on the degree-renumbered copy
  int xcd = 0;             // tiles split into one contiguous range per XCD
};

struct Plan {
  PlanConfig cfg;
  int ntiles = 0, nhubs = 0, nparts = 0;
  int nstream = 0, nlong = 0, nchunk = 0;
  BufP tiles, hubs, hub_sum, hub_cnt, hub_red;
  TilePlanDev dev{};
  // stripe plan (K_STRIPE, K_STRIPE2)
  BufP st_desc, st_hot, st_ccol, st_crow, st_wgoff, st_wglist, st_wgsum, st_mass;
  int st_nstripes = 0;
  int64_t st_hot_entries = 0, st_cold_entries = 0;  // padded
  StripePlanDev st_dev{};
  // two-phase stripe plan (K_STRIPE2): the gathered entries' values, and
  // the list that fills them block by block
  BufP st_cval, st_pasrc, st_prun, st_psub, st_pachunk;
  ColdFillDev st_fill{};
};

// Builds the stripe layout of A into plan (plan.cfg set; rp = A's row
// pointers on the host).
void build_stripe_plan(const MatP& A, Plan& plan, const std::vector<int>& rp);

std::shared_ptr<Plan> get_plan(const MatP& A, const PlanConfig& cfg);
PlanConfig default_plan_config(const MatP& A, int value_type);

// ------------------------------------------------------------ DAG nodes

enum NodeKind : int {
  N_DENSE = 0,   // materialised vector (storage or iso value)
  N_EWISE,       // w = op(a, b)
  N_APPLY_U,     // w = op(a)
  N_APPLY_B1,    // w = op(k, a)
  N_APPLY_B2,    // w = op(a, k)
  N_APPLY_B2S,   // w = op(a, scalar s)
  N_MXV,         // w = A (+.*) a
  N_REDUCE,      // scalar = sum a
  N_REDUCE_MASK, // scalar = sum a(mask)
  N_SCALAR,      // materialised scalar
  N_AFFINE,      // scalar = alpha * s + beta
  N_ASSIGN,      // w<mask> = k (GrB_ALL), old value in b
};

// Storage of a materialised vector (Section III-A: full, bitset and sparse
// vectors).  FULL: every entry present, values in buf (or iso).  BITSET:
// values in buf (n entries, 0 where absent) and one presence byte per entry
// in bits.  SPARSE: nvals ascending int32 positions in idx, their values in
// buf.
enum VecFormat : int { F_FULL = 0, F_BITSET = 1, F_SPARSE = 2 };

// Output format policy: estimates choose (default), or every vector with a
// missing entry is stored as a bitset / sparse vector (results are the same
// either way; the policy only exists to show it).
enum FormatPolicy : int { FP_ESTIMATE = 0, FP_BITSET = 1, FP_SPARSE = 2 };

struct Node;
using NodeP = std::shared_ptr<Node>;

struct Node {
  uint64_t id = 0;
  NodeKind kind = N_DENSE;
  int type = T_FP64;   // value type
  int64_t n = 0;       // vector length (0 for scalars)
  bool scalar = false;
  NodeP a, b, s, mask;
  bool mask_comp = false;
  MatP A;
  int op = 0;
  double k = 0.0, alpha = 1.0, beta = 0.0;

  bool done = false;
  bool pending = false;    // recorded in nonblocking mode, not yet run
  BufP buf;                // storage (vectors) / one double (scalars)
  bool iso = false;        // materialised vector with one value, no storage
  double iso_val = 0.0;
  bool has_value = true;   // scalars: false until assigned
  int handles = 0;         // user handles pointing here
  bool guard_watch = false;  // this scalar advances the loop guard

  // Vectors with missing entries.  `sparse_path` is decided when the node
  // is recorded: set when an input may have missing entries or a mask
  // restricts the output; such nodes run on the kernels of
  // vectors-with-missing-entries and never join a fused dense group.
  // `est` is the naive metadata estimate of the fraction of present
  // entries (Section III-D).
  int fmt = F_FULL;
  BufP bits, idx;
  int64_t nvals = -1;
  bool sparse_path = false;
  double est = 1.0;
  bool mask_struct = false, replace = false;
  bool set_union = false;  // N_EWISE: eWiseAdd (union of the entries) rather than eWiseMult

  // Pre-scaled copy of this vector (value .* dvec or ./ dvec) produced as a
  // side output by the fused pass, keyed by operator and dvec node id.
  BufP memo;
  BufP memo_sum;  // sum |memo| (FP64), when the pass that wrote the memo computed it
  int memo_op = -1;
  uint64_t memo_dvec = 0;

  ~Node();
};

// ------------------------------------------------------------ handles

constexpr uint32_t MAGIC_VEC = 0x56454331u;
constexpr uint32_t MAGIC_SCA = 0x53434131u;
constexpr uint32_t MAGIC_MAT = 0x4d415431u;
constexpr uint32_t MAGIC_FREED = 0xdeadbeefu;

}  // namespace nbgrb

struct GB_Type_opaque {
  int code;
};
struct GB_UnaryOp_opaque {
  int op;
  int type;
};
struct GB_BinaryOp_opaque {
  int op;
  int type;
};
struct GB_Monoid_opaque {
  int op;
  int type;
};
struct GB_Semiring_opaque {
  int add;
  int mul;
  int type;
};
struct GB_Descriptor_opaque {
  bool mask_comp;
  bool mask_struct;
  bool replace;
};
struct GB_Vector_opaque {
  uint32_t magic;
  int type;
  int64_t n;
  nbgrb::NodeP node;
};
struct GB_Scalar_opaque {
  uint32_t magic;
  int type;
  nbgrb::NodeP node;
};
struct GB_Matrix_opaque {
  uint32_t magic;
  int type;
  int64_t nrows, ncols;
  nbgrb::MatP data;
};

namespace nbgrb {

// ------------------------------------------------------------ context

struct Stats {
  int64_t kernels = 0, fused = 0, plan_hits = 0, plan_misses = 0, elided = 0, waits = 0;
  int64_t ewise_fused = 0;   // generated elementwise-tree launches
  int64_t ewise_ops = 0;     // operations they covered
  int64_t jit_compiles = 0, jit_disk_hits = 0, jit_memory_hits = 0;
  int64_t mxv_push = 0, mxv_pull = 0;        // sparse-path mxv by loop driver
  int64_t out_full = 0, out_bitset = 0, out_sparse = 0;  // sparse-path output formats
  int64_t index_loops = 0, range_loops = 0;  // sparse-path elementwise loop drivers
  int64_t device_allocs = 0;  // device buffers handed out (cache hits included)
};

struct Ctx {
  bool init = false;
  GrB_Mode mode = GrB_NONBLOCKING;
  hipStream_t stream = nullptr;
  int device = 0;
  int cus = 256;
  void* (*alloc)(size_t, void*) = nullptr;
  void (*release)(void*, void*) = nullptr;
  void* actx = nullptr;
  int64_t fail_after = 0;  // 0: off
  int64_t live_bytes = 0;
  std::map<size_t, std::vector<void*>> cache;
  std::vector<std::weak_ptr<Node>> pending;
  uint64_t next_id = 1;
  Stats stats;
  // scratch shared by all reductions / fused passes on the stream
  BufP red_part, red_ticket, fused_part, fused_ticket;
  int fused_part_cap = 0;
  GuardDev* guard = nullptr;  // installed loop guard (device)
  // timing of fused launches
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  std::vector<hipEvent_t> event_pool;
  // 0: only the PageRank pattern is fused; 1: pending elementwise trees are
  // also fused into generated kernels
  int fusion = 1;
  int format_policy = FP_ESTIMATE;
  // largest team of workgroups per graph in the many-graph launch
  int many_team_max = 8;
  // give-up limit of a team barrier wait (100 MHz wall-clock ticks)
  unsigned long long many_wait_ticks = 1000000000ull;
  // plan configuration override chosen by the autotuner (per matrix id)
  std::map<std::pair<uint64_t, int>, PlanConfig> tuned;
  // two pinned host slots for copies of the loop guard, each with the event
  // that marks its copy done (created on first use)
  GuardDev* guard_snap = nullptr;
  hipEvent_t guard_snap_ev[2] = {nullptr, nullptr};
  // pinned host copy of a batched PPR check (per-column hit pass and
  // residual, and the guard) and the event that marks it done
  void* ppr_snap = nullptr;
  hipEvent_t ppr_snap_ev = nullptr;
  // damping ./ outdeg in execution order, per (execution matrix, out-degree
  // vector node, damping bits, type)
  std::map<std::tuple<uint64_t, uint64_t, uint64_t, int>, NodeP> dinv_cache;
};

Ctx& ctx();
void require_init();
void* raw_alloc(size_t bytes);
void raw_release(void* p);

NodeP new_node(NodeKind k, int type, int64_t n, bool scalar);
void set_vec(GB_Vector_opaque* v, NodeP node);
void set_sca(GB_Scalar_opaque* s, NodeP node);

// Record (nonblocking) or run (blocking) a node.
void submit(const NodeP& node);
// Run all pending work of the DAG (nonblocking mode).
void force_all();
// Make sure `node` is computed and (for vectors) held in storage.
void materialize(const NodeP& node);

// Scalar operand of a kernel for a scalar node (folds a pending affine).
ScalarArg scalar_arg(const NodeP& s);
Operand operand_of(const NodeP& v);

void launch_mark(bool fused);
// Finds this device's copy of the allocation-free entry point's static
// scratch array (the device must be current); once per device.
void noalloc_setup(int device, hipStream_t s);

// Scratch of the deterministic reduction kernel on the context stream.
RedScratch reduce_scratch();

// Text returned by GrM_error() for the calling thread.
void set_error_text(const std::string& msg);

// Cache-backed allocator callbacks for the graph builders.
void* cache_alloc(size_t bytes, void* ctx);
void cache_release(void* p, void* ctx);

// s = A (+.second) w over the pattern of A (dense FP32/FP64 w and s of the
// same type), run now on the context stream with the matrix's plan.
void mxv_now(const MatP& A, int type, const void* w, void* s_out);

// Kernel `name` of a generated HIP source, compiled for the device once per
// process (and cached on disk across processes).
hipFunction_t jit_kernel(const std::string& key, const std::string& source, const char* name);
// Unload every generated module (the disk cache stays).
void jit_clear();

// Degree-renumbered copy of a square pattern (built once, then cached).
std::shared_ptr<Relabeled> get_relabeled(const MatP& A);

// Transposed pattern of A (built once, then cached with A).
MatP get_transposed(const MatP& A);

// Vectors with missing entries: decide the sparse path and the fill
// estimate of a node from its inputs (called when it is recorded), run such
// a node, and the checks of the dense paths.
void annotate(const NodeP& node);
void exec_sparse_node(const NodeP& node);
// Fail unless the done vector has every entry present.
void require_full(const NodeP& v, const char* what);
// Present entries of a done vector: count, then host copies.
int64_t vec_nvals(const NodeP& v);
void vec_tuples(const NodeP& v, int64_t* idx, void* vals, int out_type);

}  // namespace nbgrb
