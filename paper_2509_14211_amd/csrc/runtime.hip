// Runtime of the nonblocking GraphBLAS library.
//
// Nonblocking execution (paper, Section II; Section III-A "General
// approach"): every operation builds a Node that refers to the nodes of its
// inputs, the output handle is re-pointed to the new node, and nothing runs
// until a wait or a host read.  Then force_all() takes the pending nodes in
// program order.  A pending node that no handle and no other node refers to
// any more has already been destroyed: it is elided without running.  For
// the rest, the matcher looks for the PageRank-iteration shape
//     mxv(A, w)  ->  + teleport  ->  { |x - r| -> sum ,  masked sum }
// and runs it as one fused pass; intermediates that only feed the pass are
// never written.  A needed elementwise result and the elementwise
// intermediates below it run as one generated kernel.  Everything else runs
// one kernel per node, which is also exactly what blocking mode does at
// every call.
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <sstream>

namespace nbgrb {

static Ctx g_ctx;
Ctx& ctx() { return g_ctx; }

[[noreturn]] void fail(GrB_Info info, const std::string& msg) { throw GrbError{info, msg}; }

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory) fail(GrB_OUT_OF_MEMORY, std::string(what) + ": out of device memory");
  fail(GrB_PANIC, std::string(what) + ": " + hipGetErrorString(e));
}

void require_init() {
  if (!g_ctx.init) fail(GrB_PANIC, "GrB_init has not been called");
}

// ------------------------------------------------------------ memory

void* raw_alloc(size_t bytes) {
  Ctx& c = g_ctx;
  if (c.fail_after > 0 && --c.fail_after == 0) {
    c.fail_after = -1;  // the test hook fired: the caller must not retry
    return nullptr;
  }
  void* p = nullptr;
  if (c.alloc) {
    p = c.alloc(bytes, c.actx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  return p;
}

void raw_release(void* p) {
  Ctx& c = g_ctx;
  if (!p) return;
  if (c.release)
    c.release(p, c.actx);
  else
    (void)hipFree(p);
}

static size_t round_bytes(size_t b) {
  if (b < 256) return 256;
  return (b + 255) & ~(size_t)255;
}

BufP dev_alloc(size_t bytes) {
  Ctx& c = g_ctx;
  c.stats.device_allocs++;
  const size_t rb = round_bytes(bytes);
  auto it = c.cache.find(rb);
  void* p = nullptr;
  if (it != c.cache.end() && !it->second.empty()) {
    p = it->second.back();
    it->second.pop_back();
  } else {
    p = raw_alloc(rb);
    if (!p) {
      // give cached blocks back and retry once
      for (auto& kv : c.cache)
        for (void* q : kv.second) raw_release(q);
      c.cache.clear();
      if (c.fail_after == 0) p = raw_alloc(rb);
      if (c.fail_after < 0) c.fail_after = 0;  // one failure per arming of the hook
      if (!p) fail(GrB_OUT_OF_MEMORY, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
  }
  auto b = std::make_shared<DevBuf>();
  b->p = p;
  b->bytes = rb;
  c.live_bytes += (int64_t)rb;
  return b;
}

// Buffers of 2 GiB or more (one-off temporaries of the large builders)
// go straight back to the allocator instead of the size-keyed cache, which
// would keep them for an exact-size reuse that rarely comes.
constexpr size_t CACHE_MAX_BYTES = (size_t)2 << 30;

DevBuf::~DevBuf() {
  if (!p) return;
  Ctx& c = g_ctx;
  c.live_bytes -= (int64_t)bytes;
  if (c.init && bytes < CACHE_MAX_BYTES)
    c.cache[bytes].push_back(p);  // reused in stream order
  else
    raw_release(p);
}

// ------------------------------------------------------------ nodes

Node::~Node() {
  if (pending && !done) g_ctx.stats.elided++;
}

NodeP new_node(NodeKind k, int type, int64_t n, bool scalar) {
  auto p = std::make_shared<Node>();
  p->id = g_ctx.next_id++;
  p->kind = k;
  p->type = type;
  p->n = n;
  p->scalar = scalar;
  return p;
}

void set_vec(GB_Vector_opaque* v, NodeP node) {
  if (v->node) v->node->handles--;
  v->node = std::move(node);
  if (v->node) v->node->handles++;
}

void set_sca(GB_Scalar_opaque* s, NodeP node) {
  if (s->node) s->node->handles--;
  s->node = std::move(node);
  if (s->node) s->node->handles++;
}

void launch_mark(bool fused) {
  g_ctx.stats.kernels++;
  if (fused) g_ctx.stats.fused++;
}

Operand operand_of(const NodeP& v) {
  require_full(v, "this operation");
  Operand o{};
  if (v->iso) {
    o.p = nullptr;
    o.type = v->type;
    o.iso = v->iso_val;
  } else {
    o.p = v->buf->p;
    o.type = v->type;
    o.iso = 0.0;
  }
  return o;
}

static void exec_node(const NodeP& node);

ScalarArg scalar_arg(const NodeP& s) {
  if (s->kind == N_AFFINE && !s->done) {
    // fold alpha * in + beta into the consumer
    ScalarArg in = scalar_arg(s->s);
    ScalarArg r{};
    r.dev = in.dev;
    r.alpha = s->alpha * in.alpha;
    r.beta = s->alpha * in.beta + s->beta;
    return r;
  }
  if (!s->done) exec_node(s);
  if (!s->has_value) fail(GrB_EMPTY_OBJECT, "scalar operand has no value");
  ScalarArg r{};
  r.dev = (const double*)s->buf->p;
  r.alpha = 1.0;
  r.beta = 0.0;
  return r;
}

// ------------------------------------------------------------ scratch

RedScratch reduce_scratch() {
  Ctx& c = g_ctx;
  if (!c.red_part) {
    c.red_part = dev_alloc(sizeof(double) * REDUCE_GRID);
    c.red_ticket = dev_alloc(256);
    hip_check(launch_zero(c.red_ticket->p, 256, c.stream), "zero reduce ticket");
    launch_mark(false);
  }
  return RedScratch{(double*)c.red_part->p, (unsigned*)c.red_ticket->p};
}

static void fused_scratch_ensure(int grid) {
  Ctx& c = g_ctx;
  if (!c.fused_ticket) {
    c.fused_ticket = dev_alloc(256);
    hip_check(launch_zero(c.fused_ticket->p, 256, c.stream), "zero fused ticket");
    launch_mark(false);
  }
  if (grid > c.fused_part_cap) {
    c.fused_part = dev_alloc(sizeof(double) * 2 * (size_t)grid);
    c.fused_part_cap = grid;
  }
}

// ------------------------------------------------------------ temporaries

// Temporary buffers of the graph builders come from the buffer cache.
static std::map<void*, BufP>& tmp_bufs() {
  static std::map<void*, BufP> m;
  return m;
}

void* cache_alloc(size_t bytes, void*) {
  try {
    BufP b = dev_alloc(bytes);
    void* p = b->p;
    tmp_bufs()[p] = b;
    return p;
  } catch (const GrbError&) {
    return nullptr;
  }
}

void cache_release(void* p, void*) { tmp_bufs().erase(p); }

std::shared_ptr<Relabeled> get_relabeled(const MatP& A) {
  if (A->relabeled) return A->relabeled;
  if (A->nrows != A->ncols) fail(GrB_DIMENSION_MISMATCH, "relabeling needs a square matrix");
  Ctx& c = g_ctx;
  const int64_t n = A->nrows;
  auto r = std::make_shared<Relabeled>();
  r->order = dev_alloc(sizeof(int) * (size_t)n);
  r->inv = dev_alloc(sizeof(int) * (size_t)n);
  hip_check(degree_order(n, A->col ? (const int*)A->col->p : nullptr, A->nnz, (int*)r->order->p,
                         (int*)r->inv->p, cache_alloc, cache_release, nullptr, c.stream),
            "degree order");
  auto m = std::make_shared<MatData>();
  m->id = c.next_id++;
  m->nrows = n;
  m->ncols = n;
  m->nnz = A->nnz;
  m->rowptr = dev_alloc(sizeof(int) * (size_t)(n + 1));
  if (A->nnz > 0) m->col = dev_alloc(sizeof(int) * (size_t)A->nnz);
  hip_check(permute_csr(n, (const int*)A->rowptr->p, A->col ? (const int*)A->col->p : nullptr, A->nnz,
                        (const int*)r->inv->p, (int*)m->rowptr->p, m->col ? (int*)m->col->p : nullptr,
                        cache_alloc, cache_release, nullptr, c.stream),
            "relabel");
  launch_mark(false);
  r->A = m;
  A->relabeled = r;
  return r;
}

// ------------------------------------------------------------ plans

static int device_cus() { return g_ctx.cus; }

PlanConfig default_plan_config(const MatP& A, int value_type) {
  auto it = g_ctx.tuned.find({A->id, value_type});
  if (it != g_ctx.tuned.end()) return it->second;
  PlanConfig c;
  c.lds_entries = 2048;
  c.lds_rows = 1024;
  c.long_row = 2048;
  c.chunk = 2048;
  c.grid = device_cus() * 8;
  return c;
}

std::shared_ptr<Plan> get_plan(const MatP& A, const PlanConfig& cfg0) {
  PlanConfig cfg = cfg0;
  if (cfg.kernel == K_WAVE && (uint64_t)A->ncols * sizeof(double) > 0xFFFFFFFFull) {
    // the wave kernel addresses the gathered vector with 32-bit byte offsets
    cfg.kernel = K_BLOCK;
    cfg.lds_entries = 2048;
    cfg.lds_rows = 1024;
    cfg.long_row = 2048;
    cfg.chunk = 2048;
    cfg.grid = 0;
    cfg.hot = 0;
  }
  if (is_stripe(cfg.kernel) && (A->ncols >= ((int64_t)1 << 30) || A->nnz >= ((int64_t)1 << 31))) {
    // beyond the stripe layout's 32-bit offsets: the wave plan
    cfg.kernel = K_WAVE;
    cfg.hot = wave_hot_max(T_FP32);
    cfg.long_row = WAVE_TILE_ENTRIES;
    cfg.chunk = WAVE_TILE_ENTRIES;
    cfg.grid = 0;
  }
  if (cfg.kernel == K_WAVE) {
    cfg.lds_entries = WAVE_TILE_ENTRIES;
    cfg.lds_rows = WAVE_TILE_ROWS;
  }
  const bool stripe = is_stripe(cfg.kernel);
  if (stripe) {
    // geometry is fixed by the kernel; hot caps the LDS blocks, long_row is
    // the fewest entries that make a stripe load a block, chunk 1 reads the
    // packed entries with the nontemporal hint
    cfg.lds_entries = 0;
    cfg.lds_rows = 0;
    cfg.chunk = cfg.chunk == 1 ? 1 : 0;
    cfg.xcd = 0;
    if (cfg.hot <= 0 || cfg.hot > STRIPE_NBMAX * STRIPE_HB) cfg.hot = STRIPE_NBMAX * STRIPE_HB;
    cfg.hot = std::max(1, cfg.hot / STRIPE_HB) * STRIPE_HB;
    if (cfg.long_row <= 0) cfg.long_row = 1024;
  }
  if (cfg.grid <= 0) cfg.grid = (cfg.kernel == K_WAVE || stripe) ? device_cus() : device_cus() * 8;
  if (cfg.grid % 8 != 0) cfg.xcd = 0;
  auto key = std::make_tuple(cfg.kernel, stripe ? cfg.hot : cfg.lds_entries, cfg.lds_rows, cfg.long_row,
                             cfg.chunk, cfg.grid, cfg.xcd);
  auto it = A->plans.find(key);
  if (it != A->plans.end()) {
    g_ctx.stats.plan_hits++;
    return it->second;
  }
  g_ctx.stats.plan_misses++;
  if (!stripe && (cfg.long_row < 1 || cfg.chunk < cfg.long_row || cfg.chunk > cfg.lds_entries ||
                  cfg.lds_rows < 1))
    fail(GrB_INVALID_VALUE, "bad tile plan configuration");
  Ctx& c = g_ctx;
  const int64_t n = A->nrows;
  std::vector<int> rp((size_t)n + 1);
  hip_check(hipMemcpyAsync(rp.data(), A->rowptr->p, sizeof(int) * (n + 1), hipMemcpyDeviceToHost,
                           c.stream),
            "copy row pointers");
  hip_check(hipStreamSynchronize(c.stream), "sync");

  auto plan = std::make_shared<Plan>();
  plan->cfg = cfg;
  if (stripe) {
    build_stripe_plan(A, *plan, rp);
    A->plans[key] = plan;
    return plan;
  }
  std::vector<int4> tiles;
  std::vector<int4> hubs;
  int nparts = 0;
  int64_t cur0 = -1;  // first row of the open STREAM tile
  auto flush = [&](int64_t end) {
    if (cur0 >= 0 && end > cur0) {
      tiles.push_back(make_int4((int)cur0, (int)(end - cur0), rp[cur0], rp[end] - rp[cur0]));
      plan->nstream++;
    }
    cur0 = -1;
  };
  for (int64_t i = 0; i < n; ++i) {
    const int len = rp[i + 1] - rp[i];
    if (len > cfg.long_row) {
      flush(i);
      if (len <= cfg.chunk) {
        // a STREAM tile of its own
        tiles.push_back(make_int4((int)i, 1, rp[i], len));
        plan->nlong++;
      } else {
        const int h = (int)hubs.size();
        const int nch = (len + cfg.chunk - 1) / cfg.chunk;
        hubs.push_back(make_int4((int)i, nch, nparts, rp[i]));
        for (int k = 0; k < nch; ++k) {
          const int e0 = rp[i] + k * cfg.chunk;
          const int ne = std::min(cfg.chunk, rp[i + 1] - e0);
          tiles.push_back(make_int4(k, -(h + 1), e0, ne));
          plan->nchunk++;
        }
        nparts += nch;
      }
      continue;
    }
    if (cur0 >= 0 && ((i - cur0) + 1 > cfg.lds_rows || (rp[i + 1] - rp[cur0]) > cfg.lds_entries))
      flush(i);
    if (cur0 < 0) cur0 = i;
  }
  flush(n);
  plan->ntiles = (int)tiles.size();
  plan->nhubs = (int)hubs.size();
  plan->nparts = nparts;
  if (!tiles.empty()) {
    plan->tiles = dev_alloc(sizeof(int4) * tiles.size());
    hip_check(hipMemcpyAsync(plan->tiles->p, tiles.data(), sizeof(int4) * tiles.size(),
                             hipMemcpyHostToDevice, c.stream),
              "upload tiles");
  }
  if (!hubs.empty()) {
    plan->hubs = dev_alloc(sizeof(int4) * hubs.size());
    hip_check(hipMemcpyAsync(plan->hubs->p, hubs.data(), sizeof(int4) * hubs.size(),
                             hipMemcpyHostToDevice, c.stream),
              "upload hubs");
    plan->hub_sum = dev_alloc(sizeof(double) * (size_t)nparts);
    plan->hub_cnt = dev_alloc(sizeof(int) * hubs.size());
    plan->hub_red = dev_alloc(sizeof(double) * 2 * hubs.size());
    hip_check(launch_zero(plan->hub_cnt->p, sizeof(int) * hubs.size(), c.stream), "zero hub counters");
    launch_mark(false);
  }
  // host vectors must outlive the async copies
  hip_check(hipStreamSynchronize(c.stream), "sync");
  plan->dev.tiles = plan->tiles ? (const int4*)plan->tiles->p : nullptr;
  plan->dev.ntiles = plan->ntiles;
  plan->dev.hubs = plan->hubs ? (const int4*)plan->hubs->p : nullptr;
  plan->dev.nhubs = plan->nhubs;
  plan->dev.nparts = nparts;
  plan->dev.xcd = cfg.xcd;
  A->plans[key] = plan;
  return plan;
}

// ------------------------------------------------------------ fused launch

struct FusedSpec {
  int type = T_FP64;
  const void* w = nullptr;
  int mode = EPI_PLAIN;
  void* s_out = nullptr;
  void* r_out = nullptr;
  const void* x_old = nullptr;
  const void* dvec = nullptr;
  void* w_out = nullptr;
  int memo_div = 0;
  int do_D = 0;
  int mask_is_dvec = 0;
  Operand mask{};
  int mask_comp = 0;
  const void* tele_vec = nullptr;
  int tele_scaled = 0;
  ScalarArg c{nullptr, 0.0, 0.0};
  ReduceOut rho{nullptr, nullptr};
  ReduceOut D{nullptr, nullptr};
  // stripe plans: sum |w| of the gathered vector if known, and where to
  // put sum |w_out|
  const double* wsum_in = nullptr;
  double* wsum_out = nullptr;
};

static hipEvent_t pooled_event() {
  Ctx& c = g_ctx;
  if (!c.event_pool.empty()) {
    hipEvent_t e = c.event_pool.back();
    c.event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  hip_check(hipEventCreate(&e), "event create");
  return e;
}

// Returns whether f.wsum_out was written.
static bool run_fused(const MatP& A, const FusedSpec& f, const PlanConfig* cfg_override = nullptr) {
  Ctx& c = g_ctx;
  PlanConfig cfg = cfg_override ? *cfg_override : default_plan_config(A, f.type);
  if (is_stripe(cfg.kernel) && f.type != T_FP32) {
    // the stripe kernel's fixed-point sums serve FP32 ranks only
    cfg.kernel = K_WAVE;
    cfg.hot = wave_hot_max(f.type);
    cfg.long_row = WAVE_TILE_ENTRIES;
    cfg.chunk = WAVE_TILE_ENTRIES;
    cfg.grid = 0;
  }
  auto plan = get_plan(A, cfg);
  const bool stripe = is_stripe(plan->cfg.kernel);
  if (!stripe) {
    // the hot slice is w[0, hot): never more than the gathered vector holds
    int64_t hot = cfg.hot < 0 ? 0 : cfg.hot;
    if (hot > A->ncols) hot = A->ncols;
    if (hot > wave_hot_max(f.type)) hot = wave_hot_max(f.type);
    plan->cfg.hot = (int)hot;
  }
  fused_scratch_ensure(plan->cfg.grid);
  FusedScratch scr{};
  scr.wg_part = (double*)c.fused_part->p;
  scr.hub_sum = plan->hub_sum ? (double*)plan->hub_sum->p : nullptr;
  scr.hub_cnt = plan->hub_cnt ? (int*)plan->hub_cnt->p : nullptr;
  scr.hub_red = plan->hub_red ? (double*)plan->hub_red->p : nullptr;
  scr.ticket = (unsigned*)c.fused_ticket->p;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = c.timing && f.mode == EPI_PR;
  if (timed) {
    e0 = pooled_event();
    e1 = pooled_event();
    hip_check(hipEventRecord(e0, c.stream), "event record");
  }
  hipError_t e;
  bool wrote_wsum = false;
  const bool wave = plan->cfg.kernel == K_WAVE;
  // no more workgroups than there is tile work: the block kernel takes tiles
  // per workgroup, the wave kernel per wavefront (16 per workgroup); a small
  // matrix would otherwise pay for dispatching thousands of idle workgroups
  const int ntl = std::max(1, plan->dev.ntiles);
  const int grid = std::max(1, std::min(plan->cfg.grid, wave ? (ntl + 15) / 16 : ntl));
  if (f.type == T_FP32) {
    FusedArgs<float> a{};
    a.rowptr = (const int*)A->rowptr->p;
    a.col = A->col ? (const int*)A->col->p : nullptr;
    a.w = (const float*)f.w;
    a.nrows = (int)A->nrows;
    a.ncols = (int)A->ncols;
    a.mode = f.mode;
    a.s_out = (float*)f.s_out;
    a.r_out = (float*)f.r_out;
    a.x_old = (const float*)f.x_old;
    a.dvec = (const float*)f.dvec;
    a.w_out = (float*)f.w_out;
    a.memo_div = f.memo_div;
    a.do_D = f.do_D;
    a.mask_is_dvec = f.mask_is_dvec;
    a.mask = f.mask;
    a.mask_comp = f.mask_comp;
    a.tele_vec = (const float*)f.tele_vec;
    a.tele_scaled = f.tele_scaled;
    a.c = f.c;
    a.rho_out = f.rho;
    a.D_out = f.D;
    if (stripe) {
      const double* wsum_in = f.wsum_in;
      double* mass = (double*)plan->st_mass->p;
      if (!wsum_in) {
        // no bound carried over from the pass that wrote w: measure it
        hip_check(launch_abssum_f32(a.w, A->ncols, mass, reduce_scratch(), c.guard, c.stream), "sum |w|");
        launch_mark(false);
        wsum_in = mass;
        // the pass timer covers the fused kernel alone
        if (timed) hip_check(hipEventRecord(e0, c.stream), "event record");
      }
      const bool two_phase = plan->cfg.kernel == K_STRIPE2;
      if (two_phase) {
        // phase one: the values of the stripes' gathered entries, streamed
        // block by block
        hip_check(launch_cold_fill_f32(plan->st_fill, a.w, a.ncols, c.guard, c.stream), "fill gathered values");
        launch_mark(false);
      }
      e = launch_fused_stripe_f32(plan->st_dev, a, wsum_in, f.wsum_out, scr, plan->cfg.grid, plan->cfg.chunk == 1,
                                  two_phase, c.guard, c.stream);
      wrote_wsum = f.wsum_out != nullptr && a.w_out != nullptr;
    } else {
      e = wave ? launch_fused_wave_f32(plan->dev, a, scr, grid, plan->cfg.hot, c.guard, c.stream)
               : launch_fused_f32(plan->dev, a, scr, grid, plan->cfg.lds_entries,
                                  plan->cfg.lds_rows, c.guard, c.stream);
    }
  } else {
    FusedArgs<double> a{};
    a.rowptr = (const int*)A->rowptr->p;
    a.col = A->col ? (const int*)A->col->p : nullptr;
    a.w = (const double*)f.w;
    a.nrows = (int)A->nrows;
    a.ncols = (int)A->ncols;
    a.mode = f.mode;
    a.s_out = (double*)f.s_out;
    a.r_out = (double*)f.r_out;
    a.x_old = (const double*)f.x_old;
    a.dvec = (const double*)f.dvec;
    a.w_out = (double*)f.w_out;
    a.memo_div = f.memo_div;
    a.do_D = f.do_D;
    a.mask_is_dvec = f.mask_is_dvec;
    a.mask = f.mask;
    a.mask_comp = f.mask_comp;
    a.tele_vec = (const double*)f.tele_vec;
    a.tele_scaled = f.tele_scaled;
    a.c = f.c;
    a.rho_out = f.rho;
    a.D_out = f.D;
    e = wave ? launch_fused_wave_f64(plan->dev, a, scr, grid, plan->cfg.hot, c.guard, c.stream)
             : launch_fused_f64(plan->dev, a, scr, grid, plan->cfg.lds_entries,
                                plan->cfg.lds_rows, c.guard, c.stream);
  }
  hip_check(e, "fused pass launch");
  if (timed) {
    hip_check(hipEventRecord(e1, c.stream), "event record");
    c.events.push_back({e0, e1});
  }
  launch_mark(f.mode == EPI_PR);
  return wrote_wsum;
}

// Plain (blocking) mxv: s = A (+.*) w.
static void run_mxv_plain(const MatP& A, int type, const void* w, void* s_out) {
  FusedSpec f;
  f.type = type;
  f.w = w;
  f.mode = EPI_PLAIN;
  f.s_out = s_out;
  run_fused(A, f);
}

void mxv_now(const MatP& A, int type, const void* w, void* s_out) { run_mxv_plain(A, type, w, s_out); }

// Public hook for the autotuner and tests: one fused pass with an explicit
// plan configuration.
void run_fused_with(const MatP& A, const FusedSpec& f, const PlanConfig& cfg) {
  (void)run_fused(A, f, &cfg);
}

// ------------------------------------------------------------ single nodes

static void release_inputs(Node& n) {
  n.a.reset();
  n.b.reset();
  n.s.reset();
  n.mask.reset();
  n.A.reset();
}

static BufP vec_storage(const Node& n) { return dev_alloc(type_size(n.type) * (size_t)n.n); }

// Materialise an iso vector into storage.
static void store_iso(const NodeP& v) {
  if (!v->iso) return;
  Ctx& c = g_ctx;
  BufP b = vec_storage(*v);
  hip_check(launch_fill(b->p, v->type, v->n, v->iso_val, c.stream), "fill");
  launch_mark(false);
  v->buf = b;
  v->iso = false;
}

static void ensure_done(const NodeP& x) {
  if (x && !x->done) exec_node(x);
}

static void exec_node(const NodeP& np) {
  Node& n = *np;
  if (n.done) return;
  Ctx& c = g_ctx;
  ensure_done(n.a);
  ensure_done(n.b);
  if (n.kind != N_APPLY_B2S) ensure_done(n.s);
  ensure_done(n.mask);
  if (n.sparse_path) {
    exec_sparse_node(np);
    n.done = true;
    release_inputs(n);
    return;
  }
  switch (n.kind) {
    case N_EWISE: {
      BufP out = vec_storage(n);
      hip_check(launch_ewise(n.n, n.type, EW_BINARY, n.op, operand_of(n.a), operand_of(n.b),
                             ScalarArg{nullptr, 0.0, 0.0}, out->p, n.type, c.guard, c.stream),
                "ewise");
      launch_mark(false);
      n.buf = out;
      break;
    }
    case N_APPLY_U:
    case N_APPLY_B1:
    case N_APPLY_B2:
    case N_APPLY_B2S: {
      const int ct = (n.type == T_FP32) ? T_FP32 : T_FP64;
      ScalarArg sc{nullptr, 0.0, n.k};
      if (n.kind == N_APPLY_B2S) sc = scalar_arg(n.s);
      const int kind = n.kind == N_APPLY_U ? EW_UNARY : n.kind == N_APPLY_B1 ? EW_BIND1ST : EW_BIND2ND;
      BufP out = vec_storage(n);
      hip_check(launch_ewise(n.n, ct, kind, n.op, operand_of(n.a), Operand{nullptr, ct, 0.0}, sc,
                             out->p, n.type, c.guard, c.stream),
                "apply");
      launch_mark(false);
      n.buf = out;
      break;
    }
    case N_MXV: {
      store_iso(n.a);
      BufP out = vec_storage(n);
      run_mxv_plain(n.A, n.type, n.a->buf->p, out->p);
      n.buf = out;
      break;
    }
    case N_REDUCE:
    case N_REDUCE_MASK: {
      BufP out = dev_alloc(sizeof(double));
      ReduceOut ro{(double*)out->p, n.guard_watch ? c.guard : nullptr};
      const bool masked = n.kind == N_REDUCE_MASK;
      hip_check(launch_reduce(n.a->n, operand_of(n.a), masked ? 1 : 0,
                              masked ? operand_of(n.mask) : Operand{nullptr, T_FP64, 0.0},
                              n.mask_comp ? 1 : 0, ro, reduce_scratch(), c.guard, c.stream),
                "reduce");
      launch_mark(false);
      n.buf = out;
      n.has_value = true;
      break;
    }
    case N_AFFINE: {
      const ScalarArg in = scalar_arg(n.s);
      BufP out = dev_alloc(sizeof(double));
      // out = second(_, alpha * in + beta) on one element
      const ScalarArg sa{in.dev, n.alpha * in.alpha, n.alpha * in.beta + n.beta};
      hip_check(launch_ewise(1, T_FP64, EW_BIND2ND, B_SECOND, Operand{nullptr, T_FP64, 0.0},
                             Operand{nullptr, T_FP64, 0.0}, sa, out->p, T_FP64, c.guard, c.stream),
                "scalar affine");
      launch_mark(false);
      n.buf = out;
      n.has_value = true;
      break;
    }
    default:
      break;
  }
  n.done = true;
  release_inputs(n);
}

// ------------------------------------------------------------ matcher

namespace {

using Consumers = std::map<const Node*, std::vector<NodeP>>;

bool is_dense_of(const NodeP& v, int type) {
  return v && v->done && !v->iso && v->fmt == F_FULL && v->type == type;
}

// The mxv anchor of a PageRank-iteration group and the nodes it absorbs.
struct PRMatch {
  NodeP M, E, T, R, DR, RT;
  NodeP W;
  NodeP X;        // vector whose memo the pass gathers (W = X op DV)
  NodeP DV;       // pre-scale vector
  int memo_op = -1;
  bool gather_memo = false;
  FusedSpec spec;
};

bool only_consumer(const Consumers& cons, const Node* n, const Node* user) {
  auto it = cons.find(n);
  if (it == cons.end()) return false;
  return it->second.size() == 1 && it->second[0].get() == user;
}

bool match_pr(const NodeP& M, const Consumers& cons, PRMatch& m) {
  const int T = M->type;
  if (T != T_FP32 && T != T_FP64) return false;
  if (M->handles > 0) return false;
  auto cit = cons.find(M.get());
  if (cit == cons.end() || cit->second.size() != 1) return false;
  NodeP E = cit->second[0];
  if (E->type != T || E->done || E->sparse_path) return false;
  m.M = M;
  m.E = E;
  FusedSpec& f = m.spec;
  f.type = T;
  f.mode = EPI_PR;
  // teleport form
  if (E->kind == N_APPLY_B2S && E->op == B_PLUS && E->a == M) {
    m.spec.c = scalar_arg(E->s);  // folds a pending affine of a done scalar
  } else if ((E->kind == N_APPLY_B2 || E->kind == N_APPLY_B1) && E->op == B_PLUS && E->a == M) {
    f.c = ScalarArg{nullptr, 0.0, E->k};
  } else if (E->kind == N_EWISE && E->op == B_PLUS && (E->a == M || E->b == M)) {
    NodeP RT = E->a == M ? E->b : E->a;
    if (RT->type != T) return false;
    if (RT->done) {
      if (RT->fmt != F_FULL) return false;
      if (RT->iso)
        f.c = ScalarArg{nullptr, 0.0, RT->iso_val};
      else
        f.tele_vec = RT->buf->p;
    } else if ((RT->kind == N_APPLY_B2S || RT->kind == N_APPLY_B2) && RT->op == B_TIMES &&
               RT->handles == 0 && only_consumer(cons, RT.get(), E.get()) && is_dense_of(RT->a, T)) {
      // teleport v .* c with a (possibly pending) scalar c: folded per row
      f.tele_vec = RT->a->buf->p;
      f.tele_scaled = 1;
      f.c = RT->kind == N_APPLY_B2S ? scalar_arg(RT->s) : ScalarArg{nullptr, 0.0, RT->k};
      m.RT = RT;
    } else {
      return false;
    }
  } else {
    return false;
  }
  // residual and dangling reductions hanging off E
  auto eit = cons.find(E.get());
  if (eit != cons.end()) {
    for (const NodeP& u : eit->second) {
      if (u->sparse_path) continue;
      if (!m.T && u->kind == N_EWISE && u->op == B_ABSDIFF && u->handles == 0 && !u->done) {
        NodeP X = u->a == E ? u->b : u->a;
        if (!(u->a == E || u->b == E) || !is_dense_of(X, T)) continue;
        auto tit = cons.find(u.get());
        if (tit == cons.end() || tit->second.size() != 1) continue;
        NodeP R = tit->second[0];
        if (R->kind != N_REDUCE || R->a != u || R->done || R->sparse_path) continue;
        m.T = u;
        m.R = R;
        f.x_old = X->buf->p;
      } else if (!m.DR && u->kind == N_REDUCE_MASK && u->a == E && !u->done && u->mask &&
                 u->mask->done) {
        m.DR = u;
      }
    }
  }
  return true;
}

}  // namespace

// ------------------------------------------------------------ generated elementwise fusion
//
// A pending elementwise operation whose result is needed, together with the
// pending elementwise intermediates below it that nothing else uses, runs as
// one generated kernel: the tree is printed as HIP source (one statement per
// operation, each result rounded to its node's type exactly as the per-op
// kernel would store it, no contraction), compiled once per signature and
// launched over the vector.  Leaves are the vectors and scalars the tree
// reads.

namespace {

constexpr int EW_MAX_LEAVES = 12, EW_MAX_SCALARS = 6, EW_MAX_OPS = 24;

// Argument block of every generated elementwise kernel (the generated
// source declares the same struct).
struct EwArgs {
  const void* in[EW_MAX_LEAVES];
  double iso[EW_MAX_LEAVES];
  const double* sdev[EW_MAX_SCALARS];
  double salpha[EW_MAX_SCALARS];
  double sbeta[EW_MAX_SCALARS];
  const int* active;
  void* out;
  long long n;
};

bool ew_kind(const Node& n) {
  return (n.kind == N_EWISE || n.kind == N_APPLY_U || n.kind == N_APPLY_B1 || n.kind == N_APPLY_B2 ||
          n.kind == N_APPLY_B2S) &&
         (n.type == T_FP32 || n.type == T_FP64);
}

const char* ctype(int t) { return t == T_FP32 ? "float" : t == T_FP64 ? "double" : "int"; }

struct EwTree {
  std::vector<NodeP> ops;      // post-order, root last
  std::vector<NodeP> leaves;   // vectors read
  std::vector<NodeP> scalars;  // scalar operands
  std::map<const Node*, std::string> var;
  bool ok = true;
};

// Add x (an operation of the tree) and, below it, the pending elementwise
// intermediates used only by it; everything else becomes a leaf.
void ew_collect(const NodeP& x, const Consumers& cons, EwTree& t) {
  auto operand = [&](const NodeP& v) {
    if (!t.ok || t.var.count(v.get())) return;
    const bool inner = !v->done && v->handles == 0 && ew_kind(*v) && v->n == x->n &&
                       only_consumer(cons, v.get(), x.get());
    if (inner) {
      ew_collect(v, cons, t);
      return;
    }
    if (v->type != T_FP32 && v->type != T_FP64 && v->type != T_INT32) {
      t.ok = false;
      return;
    }
    t.var[v.get()] = "l" + std::to_string(t.leaves.size());
    t.leaves.push_back(v);
  };
  operand(x->a);
  if (x->kind == N_EWISE) operand(x->b);
  if (x->kind == N_APPLY_B2S && !t.var.count(x->s.get())) {
    t.var[x->s.get()] = "s" + std::to_string(t.scalars.size());
    t.scalars.push_back(x->s);
  }
  t.var[x.get()] = "v" + std::to_string(t.ops.size());
  t.ops.push_back(x);
  if ((int)t.leaves.size() > EW_MAX_LEAVES || (int)t.scalars.size() > EW_MAX_SCALARS ||
      (int)t.ops.size() > EW_MAX_OPS)
    t.ok = false;
}

std::string binop_expr(int op, const std::string& x, const std::string& y) {
  switch (op) {
    case B_PLUS: return "(" + x + " + " + y + ")";
    case B_MINUS: return "(" + x + " - " + y + ")";
    case B_TIMES: return "(" + x + " * " + y + ")";
    case B_DIV: return "(" + x + " / " + y + ")";
    case B_MAX: return "(" + x + " > " + y + " ? " + x + " : " + y + ")";
    case B_MIN: return "(" + x + " < " + y + " ? " + x + " : " + y + ")";
    case B_FIRST: return x;
    case B_SECOND: return y;
    default: return "fabs(" + x + " - " + y + ")";  // B_ABSDIFF
  }
}

std::string unop_expr(int op, const std::string& T, const std::string& x) {
  switch (op) {
    case U_IDENTITY: return x;
    case U_ABS: return "fabs(" + x + ")";
    case U_AINV: return "(-" + x + ")";
    case U_MINV: return "((" + T + ")1 / " + x + ")";
    default: return "(" + x + " != (" + T + ")0 ? (" + T + ")1 / " + x + " : (" + T + ")0)";  // U_MINV_OR_ZERO
  }
}

// HIP source of the tree; operands of each operation are first converted
// to its type, as the per-op kernel converts what it loads.
std::string ew_source(const EwTree& t) {
  std::ostringstream s;
  s << "struct EwArgs { const void* in[" << EW_MAX_LEAVES << "]; double iso[" << EW_MAX_LEAVES
    << "]; const double* sdev[" << EW_MAX_SCALARS << "]; double salpha[" << EW_MAX_SCALARS << "]; double sbeta["
    << EW_MAX_SCALARS << "]; const int* active; void* out; long long n; };\n";
  s << "__device__ __forceinline__ void elem(const EwArgs& a, long long i";
  for (size_t j = 0; j < t.scalars.size(); ++j) s << ", double s" << j;
  s << ") {\n";
  for (size_t j = 0; j < t.leaves.size(); ++j) {
    const Node& v = *t.leaves[j];
    if (v.done && v.iso)
      s << "  const double l" << j << " = a.iso[" << j << "];\n";
    else
      s << "  const " << ctype(v.type) << " l" << j << " = ((const " << ctype(v.type) << "*)a.in[" << j
        << "])[i];\n";
  }
  for (const NodeP& o : t.ops) {
    const std::string T = ctype(o->type);
    auto cv = [&](const NodeP& x) { return "(" + T + ")" + t.var.at(x.get()); };
    std::string e;
    switch (o->kind) {
      case N_EWISE: e = binop_expr(o->op, cv(o->a), cv(o->b)); break;
      case N_APPLY_U: e = unop_expr(o->op, T, cv(o->a)); break;
      case N_APPLY_B1: {
        std::ostringstream k;
        k.precision(17);
        k << "(" << T << ")" << std::scientific << o->k;
        e = binop_expr(o->op, k.str(), cv(o->a));
        break;
      }
      case N_APPLY_B2: {
        std::ostringstream k;
        k.precision(17);
        k << "(" << T << ")" << std::scientific << o->k;
        e = binop_expr(o->op, cv(o->a), k.str());
        break;
      }
      default: e = binop_expr(o->op, cv(o->a), "(" + T + ")" + t.var.at(o->s.get())); break;  // N_APPLY_B2S
    }
    s << "  const " << T << " " << t.var.at(o.get()) << " = " << e << ";\n";
  }
  const NodeP& root = t.ops.back();
  s << "  ((" << ctype(root->type) << "*)a.out)[i] = " << t.var.at(root.get()) << ";\n}\n";
  s << "extern \"C\" __global__ void __launch_bounds__(256) nbgrb_ewise(EwArgs a) {\n";
  s << "  if (a.active && *a.active == 0) return;\n";
  for (size_t j = 0; j < t.scalars.size(); ++j)
    s << "  const double s" << j << " = a.sdev[" << j << "] ? __builtin_fma(a.salpha[" << j << "], *a.sdev[" << j
      << "], a.sbeta[" << j << "]) : a.sbeta[" << j << "];\n";
  std::string sargs;
  for (size_t j = 0; j < t.scalars.size(); ++j) sargs += ", s" + std::to_string(j);
  s << "  const long long stride = (long long)gridDim.x * 256;\n";
  s << "  long long i = (long long)blockIdx.x * 256 + threadIdx.x;\n";
  s << "  for (; i + 3 * stride < a.n; i += 4 * stride) {\n";
  for (int u = 0; u < 4; ++u) s << "    elem(a, i + " << u << " * stride" << sargs << ");\n";
  s << "  }\n  for (; i < a.n; i += stride) elem(a, i" << sargs << ");\n}\n";
  return s.str();
}

void run_ew_tree(EwTree& t) {
  Ctx& c = g_ctx;
  const NodeP root = t.ops.back();
  for (const NodeP& v : t.leaves) ensure_done(v);
  EwArgs args{};
  for (size_t j = 0; j < t.leaves.size(); ++j) {
    const Node& v = *t.leaves[j];
    args.in[j] = v.iso ? nullptr : v.buf->p;
    args.iso[j] = v.iso ? v.iso_val : 0.0;
  }
  for (size_t j = 0; j < t.scalars.size(); ++j) {
    const ScalarArg sa = scalar_arg(t.scalars[j]);
    args.sdev[j] = sa.dev;
    args.salpha[j] = sa.alpha;
    args.sbeta[j] = sa.beta;
  }
  const std::string src = ew_source(t);
  hipFunction_t fn = jit_kernel(src, src, "nbgrb_ewise");
  BufP out = vec_storage(*root);
  args.active = c.guard ? &c.guard->active : nullptr;
  args.out = out->p;
  args.n = root->n;
  if (root->n > 0) {
    int64_t g = (root->n + 1023) / 1024;
    if (g > 16384) g = 16384;
    void* params[] = {&args};
    hip_check(hipModuleLaunchKernel(fn, (unsigned)g, 1, 1, 256, 1, 1, 0, c.stream, params, nullptr),
              "generated elementwise kernel");
    launch_mark(false);
  }
  c.stats.ewise_fused++;
  c.stats.ewise_ops += (int64_t)t.ops.size();
  for (const NodeP& o : t.ops) {
    o->done = true;
    if (o != root) release_inputs(*o);
  }
  root->buf = out;
  release_inputs(*root);
}

// Fuse the elementwise tree rooted at r if it has two operations or more.
bool try_ew_fusion(const NodeP& r, const Consumers& cons) {
  if (g_ctx.fusion < 1 || r->done || !ew_kind(*r)) return false;
  EwTree t;
  ew_collect(r, cons, t);
  if (!t.ok || t.ops.size() < 2) return false;
  run_ew_tree(t);
  return true;
}

}  // namespace

// Run the matched group as one fused pass.
static void run_pr_group(PRMatch& m, const Consumers& cons) {
  Ctx& c = g_ctx;
  FusedSpec& f = m.spec;
  const int T = f.type;
  NodeP M = m.M, E = m.E;
  // operand gathered by the pass
  NodeP W = M->a;
  bool memo_hit = false;
  NodeP X, DV;
  int wop = -1;
  if (W->kind == N_EWISE && (W->op == B_TIMES || W->op == B_DIV) && !W->done) {
    // w = x .* dv or x ./ dv with a materialised pre-scale vector
    if (W->a && W->b && W->a->done && is_dense_of(W->b, T)) {
      X = W->a;
      DV = W->b;
      wop = W->op;
      if (X->memo && X->memo_op == wop && X->memo_dvec == DV->id && W->handles == 0 &&
          only_consumer(cons, W.get(), M.get()))
        memo_hit = true;
    }
  }
  if (memo_hit) {
    f.w = X->memo->p;
    if (X->memo_sum) f.wsum_in = (const double*)X->memo_sum->p;
    W->done = true;  // elided: never written
    release_inputs(*W);
  } else {
    exec_node(W);
    store_iso(W);
    f.w = W->buf->p;
  }
  // side output for the next pass: r .* dv (or ./ dv)
  BufP memo, memo_sum;
  if (DV) {
    memo = dev_alloc(type_size(T) * (size_t)E->n);
    memo_sum = dev_alloc(sizeof(double));
    f.dvec = DV->buf->p;
    f.w_out = memo->p;
    f.wsum_out = (double*)memo_sum->p;
    f.memo_div = wop == B_DIV ? 1 : 0;
  }
  // E is stored when a handle or a node outside the group reads it
  BufP rbuf = dev_alloc(type_size(T) * (size_t)E->n);
  f.r_out = rbuf->p;
  // reductions
  BufP rho_buf, d_buf;
  if (m.R) {
    rho_buf = dev_alloc(sizeof(double));
    f.rho = ReduceOut{(double*)rho_buf->p, m.R->guard_watch ? c.guard : nullptr};
  }
  if (m.DR) {
    d_buf = dev_alloc(sizeof(double));
    f.D = ReduceOut{(double*)d_buf->p, m.DR->guard_watch ? c.guard : nullptr};
    f.do_D = 1;
    f.mask_comp = m.DR->mask_comp ? 1 : 0;
    if (DV && m.DR->mask == DV && !DV->iso) {
      f.mask_is_dvec = 1;
    } else {
      store_iso(m.DR->mask);
      f.mask = operand_of(m.DR->mask);
    }
  }
  const bool wrote_sum = run_fused(M->A, f);
  // bookkeeping
  M->done = true;
  release_inputs(*M);
  E->done = true;
  E->buf = rbuf;
  E->iso = false;
  if (DV) {
    E->memo = memo;
    E->memo_sum = wrote_sum ? memo_sum : nullptr;
    E->memo_op = wop;
    E->memo_dvec = DV->id;
  }
  release_inputs(*E);
  if (m.T) {
    m.T->done = true;
    release_inputs(*m.T);
  }
  if (m.RT) {
    m.RT->done = true;  // folded into the pass, never stored
    release_inputs(*m.RT);
  }
  if (m.R) {
    m.R->done = true;
    m.R->buf = rho_buf;
    m.R->has_value = true;
    release_inputs(*m.R);
  }
  if (m.DR) {
    m.DR->done = true;
    m.DR->buf = d_buf;
    m.DR->has_value = true;
    release_inputs(*m.DR);
  }
  g_ctx.stats.elided += 1 + (m.T ? 1 : 0) + (memo_hit ? 1 : 0);
}

void force_all() {
  Ctx& c = g_ctx;
  std::vector<NodeP> live;
  live.reserve(c.pending.size());
  for (auto& w : c.pending)
    if (auto p = w.lock())
      if (!p->done) live.push_back(p);
  c.pending.clear();
  if (live.empty()) return;
  Consumers cons;
  auto add = [&](const NodeP& x, const NodeP& user) {
    if (x && !x->done) cons[x.get()].push_back(user);
  };
  for (const NodeP& p : live) {
    add(p->a, p);
    add(p->b, p);
    add(p->s, p);
    add(p->mask, p);
  }
  for (const NodeP& p : live) {
    if (p->done) continue;
    if (p->kind == N_MXV && !p->sparse_path) {
      PRMatch m;
      bool ok = false;
      try {
        ok = match_pr(p, cons, m);
      } catch (const GrbError&) {
        ok = false;
      }
      if (ok) {
        run_pr_group(m, cons);
        continue;
      }
    }
    // A node no handle refers to is an intermediate: it runs on demand when
    // a consumer needs it, is absorbed by a fused group, or (a scalar
    // affine) is folded into its consumer -- or it is never needed.
    if (p->handles == 0) continue;
    if (!p->sparse_path && try_ew_fusion(p, cons)) continue;
    // a reduction of an elementwise tree: the tree as one kernel first
    if ((p->kind == N_REDUCE || p->kind == N_REDUCE_MASK) && !p->sparse_path && p->a && !p->a->done &&
        p->a->handles == 0 && only_consumer(cons, p->a.get(), p.get()))
      try_ew_fusion(p->a, cons);
    exec_node(p);
  }
}

void submit(const NodeP& node) {
  Ctx& c = g_ctx;
  annotate(node);
  if (c.mode == GrB_BLOCKING) {
    exec_node(node);
  } else {
    node->pending = true;
    c.pending.push_back(node);
  }
}

void materialize(const NodeP& node) {
  if (!node->done) {
    g_ctx.stats.waits++;
    force_all();
  }
  if (!node->done) exec_node(node);
}

}  // namespace nbgrb
