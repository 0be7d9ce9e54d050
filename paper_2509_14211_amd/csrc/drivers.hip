// C entry points of the iterative drivers (declared in include/nbgrb.h):
// PageRank and personalised PageRank as recorded GraphBLAS loops
// (GrM_pagerank, GrM_ppr), the batched and streamed personalised solvers
// over the SpMM pass (GrM_ppr_batch, GrM_ppr_stream), and many graphs in one
// persistent launch (GrM_Multigraph_*, GrM_pagerank_many).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "abi_util.h"

using namespace nbgrb;

extern "C" {

// ------------------------------------------------------------ PageRank

// d = damping ./ outdeg (0 where outdeg = 0) in the execution order of
// A_exec (the out-degree vector permuted by rl when the plan renumbers),
// materialised.  Solves on the same matrix, out-degree vector, damping and
// type share it: the context keeps the last few.
static NodeP damping_over_outdeg(const MatP& A_exec, const std::shared_ptr<Relabeled>& rl,
                                 GB_Vector_opaque* dego, int T, double damping) {
  Ctx& c = ctx();
  uint64_t dbits = 0;
  std::memcpy(&dbits, &damping, sizeof dbits);
  const auto key = std::make_tuple(A_exec->id, dego->node->id, dbits, T);
  auto it = c.dinv_cache.find(key);
  if (it != c.dinv_cache.end()) return it->second;
  const int64_t n = dego->n;
  GB_Vector_opaque deg_exec{MAGIC_VEC, dego->type, n, nullptr};
  set_vec(&deg_exec, rl ? permuted(dego->node, rl->order) : dego->node);
  GB_Vector_opaque dinv{MAGIC_VEC, T, n, nullptr};
  rec_unop(&dinv, U_MINV_OR_ZERO, &deg_exec);
  rec_bind(&dinv, B_TIMES, &dinv, damping, true);
  set_vec(&deg_exec, nullptr);
  materialize(dinv.node);
  require_full(dinv.node, "the PageRank out-degree vector");
  store_if_iso(dinv.node);
  NodeP d = dinv.node;
  set_vec(&dinv, nullptr);
  if (c.dinv_cache.size() >= 4) c.dinv_cache.erase(c.dinv_cache.begin());
  c.dinv_cache[key] = d;
  return d;
}

// The context's two pinned guard-copy slots and their events.
static GuardDev* guard_snapshots() {
  Ctx& c = ctx();
  if (!c.guard_snap) {
    void* p = nullptr;
    hip_check(hipHostMalloc(&p, 2 * sizeof(GuardDev), hipHostMallocDefault), "pinned guard slots");
    c.guard_snap = (GuardDev*)p;
  }
  for (auto& e : c.guard_snap_ev)
    if (!e) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  return c.guard_snap;
}

static GrB_Info pagerank_impl(GrB_Vector r, int* iters, double* resid, GrB_Matrix AT, GrB_Vector outdeg,
                              GrB_Vector teleport, double damping, double tol, int itermax,
                              GrM_Dangling dangling, GrB_Vector x0, int check_every) {
  Ctx& c = ctx();
  GuardDev* saved_guard = c.guard;
  BufP gbuf;
  API_BEGIN
  require_init();
  GB_Vector_opaque* ro = vec(r, "r");
  need(iters, "iters");
  need(resid, "resid");
  GB_Matrix_opaque* ao = mat(AT, "AT");
  GB_Vector_opaque* dego = vec(outdeg, "outdeg");
  GB_Vector_opaque* xo = x0 ? vec(x0, "x0") : nullptr;
  GB_Vector_opaque* vo = teleport ? vec(teleport, "teleport") : nullptr;
  float_type(ro->type, "r");
  const int T = ro->type;
  const int64_t n = ao->nrows;
  if (ao->ncols != n || ro->n != n || dego->n != n || (xo && xo->n != n) || (vo && vo->n != n))
    fail(GrB_DIMENSION_MISMATCH, "pagerank dimensions");
  if (vo && vo->type != T) fail(GrB_DOMAIN_MISMATCH, "teleport vector must have r's type");
  if (dangling != GrM_DANGLING_DROP && dangling != GrM_DANGLING_UNIFORM) fail(GrB_INVALID_VALUE, "dangling mode");
  if (check_every < 1 || itermax < 0 || !(damping >= 0.0 && damping < 1.0) || std::isnan(tol))
    fail(GrB_INVALID_VALUE, "pagerank parameters");
  if (c.guard) fail(GrB_INVALID_VALUE, "an iterative driver is already running");
  const bool uniform = dangling == GrM_DANGLING_UNIFORM;
  const double tele = (1.0 - damping) / (double)n;

  // Execution matrix: AT itself, or its copy with vertices renumbered by
  // decreasing out-degree (the teleport vector is uniform, so the method is
  // unchanged; vectors are permuted in and out).
  const PlanConfig pc = default_plan_config(ao->data, T);
  std::shared_ptr<Relabeled> rl;
  GB_Matrix_opaque A_exec{MAGIC_MAT, ao->type, n, n, ao->data};
  if (pc.relabel) {
    rl = get_relabeled(ao->data);
    A_exec.data = rl->A;
    PlanConfig sub = pc;
    sub.relabel = 0;
    c.tuned[{rl->A->id, T}] = sub;
  }

  // d = damping ./ outdeg (0 where outdeg = 0)
  GB_Vector_opaque dinv{MAGIC_VEC, T, n, nullptr};
  set_vec(&dinv, damping_over_outdeg(A_exec.data, rl, dego, T, damping));

  // personalised teleport distribution (permuted like every vector)
  GB_Vector_opaque v{MAGIC_VEC, T, n, nullptr};
  if (vo) {
    set_vec(&v, rl ? permuted(vo->node, rl->order) : vo->node);
    materialize(v.node);
    require_full(v.node, "the teleport vector");
    store_if_iso(v.node);
  }

  GB_Vector_opaque x{MAGIC_VEC, T, n, nullptr};
  if (!xo && vo) {
    set_vec(&x, v.node);
  } else if (xo) {
    if (xo->type == T)
      set_vec(&x, xo->node);
    else
      rec_unop(&x, U_IDENTITY, xo);
    materialize(x.node);
    if (rl) set_vec(&x, permuted(x.node, rl->order));
  } else {
    set_vec(&x, iso_node(T, n, 1.0 / (double)n));
  }
  materialize(x.node);
  require_full(x.node, "the start vector");
  store_if_iso(x.node);

  GB_Scalar_opaque D{MAGIC_SCA, T_FP64, nullptr};
  if (uniform) rec_reduce(&D, &x, &dinv, true, false);

  gbuf = dev_alloc(sizeof(GuardDev));
  hip_check(launch_guard_init((GuardDev*)gbuf->p, (1.0 > tol && itermax > 0) ? 1 : 0, tol, itermax, c.stream),
            "guard init");
  launch_mark(false);
  c.guard = (GuardDev*)gbuf->p;

  // hist[i]: the iterate after pass base + i
  std::vector<NodeP> hist{x.node};
  int64_t base = 0;
  GuardDev hg{};
  int enq = 0;  // passes enqueued (never beyond itermax: the guard would only skip them)
  auto enqueue = [&](int count) {
    for (int j = 0; j < count; ++j) {
      GB_Vector_opaque w{MAGIC_VEC, T, n, nullptr}, s{MAGIC_VEC, T, n, nullptr};
      GB_Vector_opaque rn{MAGIC_VEC, T, n, nullptr}, t{MAGIC_VEC, T, n, nullptr};
      GB_Scalar_opaque cs{MAGIC_SCA, T_FP64, nullptr}, rho{MAGIC_SCA, T_FP64, nullptr};
      GB_Scalar_opaque Dn{MAGIC_SCA, T_FP64, nullptr};
      rec_ewise(&w, B_TIMES, &x, &dinv, false);     // w = x .* d
      rec_mxv(&s, &A_exec, &w, nullptr, nullptr); // s = AT (+.second) w
      GB_Vector_opaque vt{MAGIC_VEC, T, n, nullptr};
      if (vo) {                                     // r = s + v .* c
        if (uniform) {                              //   c = (1-d) + d D
          rec_affine(&cs, damping, &D, 1.0 - damping);
          rec_bind_scalar(&vt, B_TIMES, &v, &cs);
        } else {                                    //   c = 1-d
          rec_bind(&vt, B_TIMES, &v, 1.0 - damping, false);
        }
        rec_ewise(&rn, B_PLUS, &s, &vt, true);
        set_vec(&vt, nullptr);
      } else if (uniform) {                         // r = c + s, c = (1-d)/n + d D/n
        rec_affine(&cs, damping / (double)n, &D, tele);
        rec_bind_scalar(&rn, B_PLUS, &s, &cs);
      } else {
        rec_bind(&rn, B_PLUS, &s, tele, false);
      }
      rec_ewise(&t, B_ABSDIFF, &x, &rn, true);      // t = |x - r|
      rec_reduce(&rho, &t, nullptr, false, true);   // rho = sum t  (advances the guard)
      if (uniform) rec_reduce(&Dn, &rn, &dinv, true, false);  // D = sum r(outdeg = 0)
      // only r, rho and D stay reachable: w, s, t and c become intermediates
      set_vec(&w, nullptr);
      set_vec(&s, nullptr);
      set_vec(&t, nullptr);
      set_sca(&cs, nullptr);
      materialize(rn.node);
      set_vec(&x, rn.node);
      if (uniform) set_sca(&D, Dn.node);
      hist.push_back(rn.node);
      set_vec(&rn, nullptr);
      set_sca(&rho, nullptr);
      set_sca(&Dn, nullptr);
    }
    enq += count;
  };
  // The guard is copied to pinned host memory after each batch, and a few
  // more passes are queued behind the copy before the host waits for it:
  // the device works through them while the host reads the guard and
  // queues the next batch, instead of waiting for the host.  Passes queued
  // past convergence are skipped by the guard.
  constexpr int AHEAD = 2;
  GuardDev* snap = guard_snapshots();
  int slot = 0;
  auto snapshot = [&]() {
    hip_check(hipMemcpyAsync(&snap[slot], c.guard, sizeof(GuardDev), hipMemcpyDeviceToHost, c.stream),
              "read guard");
    hip_check(hipEventRecord(c.guard_snap_ev[slot], c.stream), "event record");
  };
  enqueue(check_every < itermax ? check_every : itermax);
  snapshot();
  for (;;) {
    enqueue(std::min(AHEAD, itermax - enq));
    hip_check(hipEventSynchronize(c.guard_snap_ev[slot]), "wait for the guard");
    hg = snap[slot];
    if (!hg.active) break;
    // passes before hg.iters are done with
    const int64_t drop = (int64_t)hg.iters - base;
    if (drop > 0 && drop < (int64_t)hist.size()) {
      hist.erase(hist.begin(), hist.begin() + drop);
      base = hg.iters;
    }
    // The residual contracts about geometrically: predict the passes still
    // needed from the last two residuals (at least 1, at most what itermax
    // allows); an underestimate only costs one more check.
    int need = check_every;
    if (hg.rho_prev > 0.0 && hg.rho > 0.0 && hg.rho < hg.rho_prev && tol > 0.0) {
      const double q = hg.rho / hg.rho_prev;
      const double pn = std::log(tol / hg.rho) / std::log(q);
      if (pn > 0.0 && pn < 1e6) need = (int)std::ceil(pn);
      if (need < 1) need = 1;
    }
    // beyond the passes already queued after hg.iters
    int next = need - (enq - hg.iters);
    if (next > itermax - enq) next = itermax - enq;
    if (next > 0) enqueue(next);
    slot ^= 1;
    snapshot();
  }
  if (hg.bad) fail(GrB_PANIC, "pagerank: a residual or dangling mass was not finite (NaN or Inf in the iterate)");
  const int64_t idx = (int64_t)hg.iters - base;
  if (idx < 0 || idx >= (int64_t)hist.size()) fail(GrB_PANIC, "loop guard out of step");
  c.guard = saved_guard;
  NodeP result = hist[(size_t)idx];
  set_vec(ro, rl ? permuted(result, rl->inv) : result);
  hist.clear();
  set_vec(&x, nullptr);
  set_vec(&v, nullptr);
  set_vec(&dinv, nullptr);
  set_sca(&D, nullptr);
  *iters = hg.iters;
  *resid = hg.rho;
  }
  catch (const GrbError& e) {
    c.guard = saved_guard;
    api_error() = e.msg;
    return e.info;
  }
  catch (const std::exception& e) {
    c.guard = saved_guard;
    api_error() = e.what();
    return GrB_PANIC;
  }
  return GrB_SUCCESS;
}

GrB_Info GrM_pagerank(GrB_Vector r, int* iters, double* resid, GrB_Matrix AT, GrB_Vector outdeg, double damping,
                      double tol, int itermax, GrM_Dangling dangling, GrB_Vector x0, int check_every) {
  return pagerank_impl(r, iters, resid, AT, outdeg, nullptr, damping, tol, itermax, dangling, x0, check_every);
}

GrB_Info GrM_ppr(GrB_Vector r, int* iters, double* resid, GrB_Matrix AT, GrB_Vector outdeg, GrB_Vector teleport,
                 double damping, double tol, int itermax, GrM_Dangling dangling, GrB_Vector x0, int check_every) {
  if (!teleport) {
    api_error() = "teleport is NULL";
    return GrB_NULL_POINTER;
  }
  return pagerank_impl(r, iters, resid, AT, outdeg, teleport, damping, tol, itermax, dangling, x0, check_every);
}

// ------------------------------------------------------------ batched PPR

namespace {

struct PprSeed {
  int v, c;
  double w;
};

// A batch with at most this many columns still running finishes them as
// single-vector solves.  A gathered row narrower than a 128-byte cache line
// costs a whole line, so a product pass of 8 columns costs about as much as
// one of 16 and more than 8 single-vector passes.
constexpr int PPR_TAIL_COLUMNS = 8;

// Width of the product once `live` columns still run: whole 64-byte FP32
// row sectors, at least 16 columns (gathered four entries per load).
inline int ppr_narrow_width(int live) { return live > 16 ? (live + 15) / 16 * 16 : 16; }

// Seed sets seed_vtx[seed_ptr[q] : seed_ptr[q+1]], q < nsets: non-empty,
// distinct vertices in [0, n).
void check_seed_sets(int nsets, const int32_t* seed_ptr, const int32_t* seed_vtx, int64_t n) {
  need(seed_ptr, "seed_ptr");
  need(seed_vtx, "seed_vtx");
  if (seed_ptr[0] != 0) fail(GrB_INVALID_VALUE, "seed_ptr[0] must be 0");
  for (int q = 0; q < nsets; ++q)
    if (seed_ptr[q + 1] <= seed_ptr[q]) fail(GrB_INVALID_VALUE, "every seed set must be non-empty");
  for (int q = 0; q < nsets; ++q) {
    std::vector<int> s(seed_vtx + seed_ptr[q], seed_vtx + seed_ptr[q + 1]);
    std::sort(s.begin(), s.end());
    for (size_t i = 0; i < s.size(); ++i) {
      if (s[i] < 0 || s[i] >= n) fail(GrB_INDEX_OUT_OF_BOUNDS, "seed vertex out of range");
      if (i > 0 && s[i] == s[i - 1]) fail(GrB_INVALID_VALUE, "repeated seed vertex in a set");
    }
  }
}

// Device state of k personalised PageRank columns iterated together by the
// SpMM pass: the execution matrix (degree-renumbered copy when the plan
// asks for it), its wave tile plan, d = damping ./ outdeg, the two
// alternating n x k iterate / pre-scaled buffers, the per-column FP64
// residual and dangling mass, and the vertex-sorted seed table.
struct PprColumns {
  int64_t n = 0;
  int T = T_FP32, k = 0;
  std::shared_ptr<Relabeled> rl;
  MatP A_exec;
  std::vector<int> inv_host;
  std::shared_ptr<Plan> plan;
  GB_Vector_opaque dinv{MAGIC_VEC, T_FP32, 0, nullptr};
  size_t vbytes = 0;
  BufP Xb[2], Wb[2], Db[2], rho, hit, hub_sum, hub_cnt, hub_red, wg_part, ticket, gbuf, tile_seed, sv, sc, sw;
  SpmmArgs a{};
  int grid = 0;
  bool uniform = true;
  // the next pass stores every row: after a start or a narrowing, the
  // output buffers do not yet hold zeros in the rows the pass may skip
  bool full_next = true;

  ~PprColumns() { set_vec(&dinv, nullptr); }

  void setup(GB_Matrix_opaque* ao, GB_Vector_opaque* dego, int type, int kk, double damping, double tol,
             bool unif) {
    Ctx& c = ctx();
    n = ao->nrows;
    T = type;
    k = kk;
    uniform = unif;
    const PlanConfig pc = default_plan_config(ao->data, T);
    A_exec = ao->data;
    if (pc.relabel) {
      rl = get_relabeled(ao->data);
      A_exec = rl->A;
      inv_host.resize((size_t)n);
      hip_check(hipMemcpyAsync(inv_host.data(), rl->inv->p, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost,
                               c.stream),
                "copy permutation");
      hip_check(hipStreamSynchronize(c.stream), "sync");
    }
    PlanConfig wp;
    wp.kernel = K_WAVE;
    wp.lds_entries = WAVE_TILE_ENTRIES;
    wp.lds_rows = WAVE_TILE_ROWS;
    wp.long_row = (pc.kernel == K_WAVE) ? pc.long_row : WAVE_TILE_ENTRIES;
    wp.chunk = WAVE_TILE_ENTRIES;
    wp.grid = c.cus * 2;
    plan = get_plan(A_exec, wp);
    // the SpMM kernels assume wavefront tiles (at most 256 rows, 512 entries)
    if (plan->cfg.kernel != K_WAVE) fail(GrB_NOT_IMPLEMENTED, "batched PPR: too many vertices for the wavefront tile plan");
    grid = plan->cfg.grid;

    // d = damping ./ outdeg (0 for dangling), in execution order
    dinv.type = T;
    dinv.n = n;
    set_vec(&dinv, damping_over_outdeg(A_exec, rl, dego, T, damping));

    vbytes = type_size(T) * (size_t)n * (size_t)k;
    for (int i = 0; i < 2; ++i) {
      Xb[i] = dev_alloc(vbytes);
      Wb[i] = dev_alloc(vbytes);
      Db[i] = dev_alloc(sizeof(double) * 64);
    }
    rho = dev_alloc(sizeof(double) * 64);
    hit = dev_alloc(sizeof(int) * 64);
    hub_sum = dev_alloc(sizeof(double) * 64 * (size_t)std::max(plan->nparts, 1));
    hub_cnt = dev_alloc(sizeof(int) * (size_t)std::max(plan->nhubs, 1));
    hub_red = dev_alloc(sizeof(double) * 128 * (size_t)std::max(plan->nhubs, 1));
    wg_part = dev_alloc(sizeof(double) * 128 * (size_t)grid);
    ticket = dev_alloc(256);
    gbuf = dev_alloc(sizeof(GuardDev));
    tile_seed = dev_alloc(sizeof(int) * (size_t)std::max(plan->dev.ntiles, 1));
    hip_check(launch_zero(hub_cnt->p, sizeof(int) * (size_t)std::max(plan->nhubs, 1), c.stream), "zero");
    hip_check(launch_zero(ticket->p, 256, c.stream), "zero");
    hip_check(launch_zero(Xb[0]->p, vbytes, c.stream), "zero");
    hip_check(launch_zero(Wb[0]->p, vbytes, c.stream), "zero");
    hip_check(launch_zero(Db[0]->p, sizeof(double) * 64, c.stream), "zero");
    hip_check(launch_zero(rho->p, sizeof(double) * 64, c.stream), "zero");
    for (int i = 0; i < 6; ++i) launch_mark(false);

    a.rowptr = (const int*)A_exec->rowptr->p;
    a.col = A_exec->col ? (const int*)A_exec->col->p : nullptr;
    a.k = k;
    a.w_bytes = vbytes < 0xFFFFFF00ull ? (unsigned)vbytes : 0u;
    a.dvec = dinv.node->buf->p;
    a.c_alpha = damping;
    a.c_beta = 1.0 - damping;
    a.rho_out = (double*)rho->p;
    a.hit = (int*)hit->p;
    a.hit_tol = tol;
    a.hub_sum = (double*)hub_sum->p;
    a.hub_cnt = (int*)hub_cnt->p;
    a.hub_red = (double*)hub_red->p;
    a.wg_part = (double*)wg_part->p;
    a.ticket = (unsigned*)ticket->p;
    a.tile_seed = (const int*)tile_seed->p;
  }

  int exec_vertex(int v) const { return rl ? inv_host[(size_t)v] : v; }

  BufP upload(const void* h, size_t bytes) {
    BufP b = dev_alloc(std::max<size_t>(bytes, 16));
    if (bytes) hip_check(hipMemcpyAsync(b->p, h, bytes, hipMemcpyHostToDevice, ctx().stream), "upload");
    return b;
  }

  // Teleport table of the columns in use: seeds (execution numbering)
  // sorted by vertex, then column; each tile's first seed.
  void set_seeds(std::vector<PprSeed> seeds) {
    std::sort(seeds.begin(), seeds.end(),
              [](const PprSeed& x, const PprSeed& y) { return x.v != y.v ? x.v < y.v : x.c < y.c; });
    const int ns = (int)seeds.size();
    std::vector<int> v(ns), cc(ns);
    std::vector<double> w(ns);
    for (int i = 0; i < ns; ++i) {
      v[i] = seeds[i].v;
      cc[i] = seeds[i].c;
      w[i] = seeds[i].w;
    }
    sv = upload(v.data(), sizeof(int) * ns);
    sc = upload(cc.data(), sizeof(int) * ns);
    sw = upload(w.data(), sizeof(double) * ns);
    a.seed_v = (const int*)sv->p;
    a.seed_c = (const int*)sc->p;
    a.seed_w = (const double*)sw->p;
    a.nseeds = ns;
    hip_check(launch_spmm_tile_seed(plan->dev, a.seed_v, ns, (int*)tile_seed->p, ctx().stream), "tile seeds");
    launch_mark(false);
  }

  // Start columns `cols` (their seeds listed by column in seeds_by_col) in
  // buffer set `cur`: x = v, w = v .* d, D = dangling seed mass, hit = -1.
  // `zeroed`: those columns of set `cur` are zero already (set 0 is, right
  // after setup).
  void start_columns(uint64_t cols, int cur, const std::vector<PprSeed>& seeds_by_col, bool zeroed = false) {
    Ctx& c = ctx();
    if (!zeroed) hip_check(launch_spmm_zero_columns(Xb[cur]->p, Wb[cur]->p, T, n, k, cols, c.stream), "zero columns");
    std::vector<int> ptr(k + 1, 0), v;
    std::vector<double> w;
    for (int col = 0; col < k; ++col) {
      for (const PprSeed& s : seeds_by_col)
        if (s.c == col) {
          v.push_back(s.v);
          w.push_back(s.w);
        }
      ptr[col + 1] = (int)v.size();
    }
    BufP dp = upload(ptr.data(), sizeof(int) * (k + 1)), dv = upload(v.data(), sizeof(int) * v.size());
    BufP dw = upload(w.data(), sizeof(double) * w.size());
    SpmmArgs ia = a;
    ia.x_new = Xb[cur]->p;
    ia.w_new = Wb[cur]->p;
    ia.d_out = (double*)Db[cur]->p;
    hip_check(launch_spmm_init(ia, T, (const int*)dp->p, (const int*)dv->p, (const double*)dw->p, cols, c.stream),
              "ppr init");
    launch_mark(false);
    launch_mark(false);
    full_next = true;
  }

  // Columns `cols` to their outputs: column c of the iterate from buffer
  // set 1 when bit c of from1 is set, else from set 0 (a converged column
  // is frozen in the buffer of the pass it converged in), in vertex order.
  void output(uint64_t cols, uint64_t from1, const ColumnOutputs& outs) {
    if (!cols) return;
    hip_check(launch_spmm_columns_out(Xb[0]->p, Xb[1]->p, from1, T, rl ? (const int*)rl->inv->p : nullptr, n, k,
                                      cols, outs, ctx().stream),
              "columns out");
    launch_mark(false);
  }

  // Narrows the iterate after pass `pass` to k2 columns: new column j is old
  // column keep[j] (j < keep.size()), the rest are empty and frozen.  The
  // product's cost follows k, so once most columns have converged the
  // remaining passes gather k2-wide rows instead of k-wide ones.  The
  // caller renumbers the seed table.
  void narrow(int pass, const std::vector<int>& keep, int k2) {
    const int cur = pass & 1;
    ColumnMap map;
    for (int j = 0; j < 64; ++j) map.c[j] = j < (int)keep.size() ? keep[(size_t)j] : -1;
    hip_check(launch_spmm_compact(Xb[cur]->p, a.dvec, (const double*)Db[cur]->p, Xb[cur ^ 1]->p,
                                  Wb[cur ^ 1]->p, (double*)Db[cur ^ 1]->p, (int*)hit->p, T, n, k, k2, map,
                                  ctx().stream),
              "narrow columns");
    launch_mark(false);
    // the narrowed copy becomes the iterate of pass `pass`
    std::swap(Xb[0], Xb[1]);
    std::swap(Wb[0], Wb[1]);
    std::swap(Db[0], Db[1]);
    k = k2;
    a.k = k2;
    const size_t used = type_size(T) * (size_t)n * (size_t)k2;
    a.w_bytes = used < 0xFFFFFF00ull ? (unsigned)used : 0u;
    full_next = true;
  }

  // One pass from buffer set (pass-1)&1 into pass&1.
  void run_pass(int pass) {
    Ctx& c = ctx();
    const int in = (pass - 1) & 1, out = pass & 1;
    a.w = Wb[in]->p;
    a.x_old = Xb[in]->p;
    a.x_new = Xb[out]->p;
    a.w_new = Wb[out]->p;
    a.d_prev = uniform ? (const double*)Db[in]->p : nullptr;
    a.d_out = (double*)Db[out]->p;
    // rows with no entries and no seed stay zero in both buffer sets once a
    // pass has stored every row of the current layout and seeds
    a.skip_empty = full_next ? 0 : 1;
    full_next = false;
    hip_check(launch_spmm_ppr(plan->dev, a, T, grid, a.guard, c.stream), "ppr pass");
    launch_mark(true);
  }

  // The per-column converged pass and residual and the guard after the
  // passes queued so far: copied into pinned host memory with one wait.
  void read_state(std::vector<int>& hh, std::vector<double>& rr, GuardDev& hg) {
    struct Snap {
      int hit[64];
      double rho[64];
      GuardDev g;
    };
    Ctx& c = ctx();
    if (!c.ppr_snap) {
      void* p = nullptr;
      hip_check(hipHostMalloc(&p, sizeof(Snap), hipHostMallocDefault), "pinned check slot");
      c.ppr_snap = p;
    }
    if (!c.ppr_snap_ev) hip_check(hipEventCreateWithFlags(&c.ppr_snap_ev, hipEventDisableTiming), "event");
    Snap* sn = (Snap*)c.ppr_snap;
    hip_check(hipMemcpyAsync(sn->hit, hit->p, sizeof(int) * 64, hipMemcpyDeviceToHost, c.stream), "copy");
    hip_check(hipMemcpyAsync(sn->rho, rho->p, sizeof(double) * 64, hipMemcpyDeviceToHost, c.stream), "copy");
    hip_check(hipMemcpyAsync(&sn->g, c.guard, sizeof(GuardDev), hipMemcpyDeviceToHost, c.stream), "read guard");
    hip_check(hipEventRecord(c.ppr_snap_ev, c.stream), "event record");
    hip_check(hipEventSynchronize(c.ppr_snap_ev), "wait for the check");
    hh.assign(sn->hit, sn->hit + 64);
    rr.assign(sn->rho, sn->rho + 64);
    hg = sn->g;
  }
};

}  // namespace

GrB_Info GrM_ppr_batch(void* X, GrB_Type type, int k, const int32_t* seed_ptr, const int32_t* seed_vtx,
                       GrB_Matrix AT, GrB_Vector outdeg, double damping, double tol, int itermax,
                       GrM_Dangling dangling, int check_every, int* iters, int* col_iters, double* col_resid) {
  Ctx& c = ctx();
  GuardDev* saved_guard = c.guard;
  API_BEGIN
  require_init();
  need(X, "X");
  need(type, "type");
  need(iters, "iters");
  GB_Matrix_opaque* ao = mat(AT, "AT");
  GB_Vector_opaque* dego = vec(outdeg, "outdeg");
  const int T = type->code;
  float_type(T, "type");
  const int64_t n = ao->nrows;
  if (ao->ncols != n || dego->n != n) fail(GrB_DIMENSION_MISMATCH, "ppr_batch dimensions");
  if (k < 1 || k > 64) fail(GrB_INVALID_VALUE, "k must be in [1, 64]");
  if (dangling != GrM_DANGLING_DROP && dangling != GrM_DANGLING_UNIFORM) fail(GrB_INVALID_VALUE, "dangling mode");
  if (check_every < 1 || itermax < 0 || !(damping >= 0.0 && damping < 1.0) || std::isnan(tol))
    fail(GrB_INVALID_VALUE, "ppr_batch parameters");
  if (c.guard) fail(GrB_INVALID_VALUE, "an iterative driver is already running");
  check_seed_sets(k, seed_ptr, seed_vtx, n);

  PprColumns pc;
  pc.setup(ao, dego, T, k, damping, tol, dangling == GrM_DANGLING_UNIFORM);
  std::vector<PprSeed> seeds;
  for (int q = 0; q < k; ++q) {
    const double w = 1.0 / (double)(seed_ptr[q + 1] - seed_ptr[q]);
    for (int e = seed_ptr[q]; e < seed_ptr[q + 1]; ++e) seeds.push_back({pc.exec_vertex(seed_vtx[e]), q, w});
  }
  pc.set_seeds(seeds);
  pc.start_columns(k == 64 ? ~0ull : ((1ull << k) - 1ull), 0, seeds, true);
  hip_check(launch_guard_init((GuardDev*)pc.gbuf->p, (1.0 > tol && itermax > 0) ? 1 : 0, tol, itermax, c.stream),
            "guard init");
  launch_mark(false);
  c.guard = (GuardDev*)pc.gbuf->p;
  pc.a.guard = c.guard;

  // col_set[c]: the seed set in column c (-1: none).  Each column stops at
  // the pass its own residual first reaches tol (the pass kernel freezes it
  // there and every later pass carries its ranks forward unchanged, so the
  // buffer set of the last pass holds every column), and column q ends
  // where a single-vector solve of set q would.  Finished columns go to a
  // column-major staging copy (set q at stage + q n, vertex order), written
  // in whole lines, when the product narrows and at the end; X is written
  // once, whole rows at a time, at the very end.
  const size_t vb = type_size(T) * (size_t)n;
  BufP stage = dev_alloc(vb * (size_t)k);
  std::vector<int> col_set((size_t)k);
  for (int q = 0; q < k; ++q) col_set[(size_t)q] = q;
  int live = k;
  uint64_t frozen = 0;  // converged, not yet staged
  bool tail = false;
  ColumnOutputs outs{};
  outs.ld = 1;
  auto out_of = [&](uint64_t cols, int at_pass) {
    for (int col = 0; col < pc.k; ++col)
      if ((cols >> col) & 1ull) outs.out[col] = (char*)stage->p + vb * (size_t)col_set[(size_t)col];
    pc.output(cols, (at_pass & 1) ? cols : 0ull, outs);
  };
  std::vector<int> hh(64, -1);
  std::vector<double> rr(64, 1.0);
  GuardDev hg{};
  int pass = 0, batch = check_every;
  for (;;) {
    for (int j = 0; j < batch; ++j) pc.run_pass(++pass);
    pc.read_state(hh, rr, hg);
    if (hg.bad) break;
    for (int col = 0; col < pc.k; ++col) {
      const int q = col_set[(size_t)col];
      if (q < 0 || ((frozen >> col) & 1ull) || hh[(size_t)col] < 0) continue;
      frozen |= 1ull << col;
      if (col_iters) col_iters[q] = hh[(size_t)col];
      if (col_resid) col_resid[q] = rr[(size_t)col];
      --live;
    }
    if (!hg.active) break;
    if (live <= PPR_TAIL_COLUMNS) {
      tail = true;
      break;
    }
    // narrow to the live columns once that is narrower
    const int k2 = ppr_narrow_width(live);
    if (k2 < pc.k) {
      out_of(frozen, hg.iters);
      for (int col = 0; col < pc.k; ++col)
        if ((frozen >> col) & 1ull) col_set[(size_t)col] = -1;
      frozen = 0;
      std::vector<int> keep, newpos((size_t)pc.k, -1), set2((size_t)k2, -1);
      for (int col = 0; col < pc.k; ++col)
        if (col_set[(size_t)col] >= 0) {
          newpos[(size_t)col] = (int)keep.size();
          set2[keep.size()] = col_set[(size_t)col];
          keep.push_back(col);
        }
      std::vector<PprSeed> kept;
      for (const PprSeed& sd : seeds)
        if (newpos[(size_t)sd.c] >= 0) kept.push_back({sd.v, newpos[(size_t)sd.c], sd.w});
      pc.narrow(hg.iters, keep, k2);
      seeds.swap(kept);
      pc.set_seeds(seeds);
      col_set.swap(set2);
    }
    // at most check_every passes between checks (fewer when the slowest
    // column is predicted to finish sooner); once columns start to
    // converge, every second pass, so the product narrows soon after
    int next = check_every;
    if (hg.rho_prev > 0.0 && hg.rho > 0.0 && hg.rho < hg.rho_prev && tol > 0.0) {
      const double need_passes = std::log(tol / hg.rho) / std::log(hg.rho / hg.rho_prev);
      if (need_passes > 0.0 && need_passes < (double)next) next = (int)std::ceil(need_passes);
    }
    if (live < k && next > 2) next = 2;
    if (next > itermax - hg.iters) next = itermax - hg.iters;
    if (next < 1) next = 1;
    batch = next;
  }
  c.guard = saved_guard;
  if (hg.bad) fail(GrB_PANIC, "ppr_batch: a column's residual or dangling mass was not finite");
  // the converged columns not yet staged
  out_of(frozen, hg.iters);
  uint64_t rest = 0;
  for (int col = 0; col < pc.k; ++col)
    if (col_set[(size_t)col] >= 0 && !((frozen >> col) & 1ull)) rest |= 1ull << col;
  const int done_passes = hg.iters;
  int max_passes = hg.iters;
  // source of every column of X: its staged copy, or a tail solve's result
  ColumnInputs ins{};
  ins.ld = k;
  for (int q = 0; q < k; ++q) {
    ins.in[q] = (const char*)stage->p + vb * (size_t)q;
    ins.dst[q] = q;
  }
  std::vector<int> tcols;
  if (tail && itermax > done_passes)
    for (int col = 0; col < pc.k; ++col)
      if ((rest >> col) & 1ull) tcols.push_back(col);
  const int nt = (int)tcols.size();
  std::vector<GB_Vector_opaque> xv((size_t)nt, GB_Vector_opaque{MAGIC_VEC, T, n, nullptr});
  std::vector<GB_Vector_opaque> rv((size_t)nt, GB_Vector_opaque{MAGIC_VEC, T, n, nullptr});
  auto release = [&]() {
    for (int i = 0; i < nt; ++i) {
      set_vec(&xv[(size_t)i], nullptr);
      set_vec(&rv[(size_t)i], nullptr);
    }
  };
  try {
    if (nt > 0) {
      // The few columns still running continue one by one as single-vector
      // solves (GrM_ppr) from their current iterate: that pass costs a small
      // fraction of even a one-column SpMM pass.  Their iterate, teleport
      // vector and dangling mass define the next pass completely, so column
      // q still ends where a single-vector solve of set q from the start
      // would.  Every tail column's current iterate, in the original
      // numbering, comes out in one sweep over the operand.
      ColumnOutputs xo{};
      xo.ld = 1;
      for (int i = 0; i < nt; ++i) {
        NodeP xn = new_node(N_DENSE, T, n, false);
        xn->buf = dev_alloc(vb);
        xn->done = true;
        xo.out[tcols[(size_t)i]] = xn->buf->p;
        set_vec(&xv[(size_t)i], xn);
      }
      pc.output(rest, (done_passes & 1) ? rest : 0ull, xo);
      for (int i = 0; i < nt; ++i) {
        const int q = col_set[(size_t)tcols[(size_t)i]];
        GB_Vector_opaque tv{MAGIC_VEC, T, n, nullptr};
        NodeP tn = new_node(N_DENSE, T, n, false);
        tn->buf = dev_alloc(vb);
        hip_check(launch_zero(tn->buf->p, vb, c.stream), "zero");
        const int ns = seed_ptr[q + 1] - seed_ptr[q];
        BufP sidx = pc.upload(seed_vtx + seed_ptr[q], sizeof(int) * (size_t)ns);
        hip_check(launch_scatter_value(tn->buf->p, T, (const int*)sidx->p, ns, 1.0 / (double)ns, c.stream),
                  "seeds");
        launch_mark(false);
        tn->done = true;
        set_vec(&tv, tn);
        int it = 0;
        double res = 1.0;
        c.guard = saved_guard;
        const GrB_Info info = pagerank_impl((GrB_Vector)&rv[(size_t)i], &it, &res, AT, outdeg, (GrB_Vector)&tv,
                                            damping, tol, itermax - done_passes, dangling,
                                            (GrB_Vector)&xv[(size_t)i], check_every);
        set_vec(&tv, nullptr);
        if (info != GrB_SUCCESS) fail(info, "ppr_batch: " + api_error());
        set_vec(&xv[(size_t)i], nullptr);  // its start vector is no longer needed
        materialize(rv[(size_t)i].node);
        require_full(rv[(size_t)i].node, "a batched PPR column");
        ins.in[q] = rv[(size_t)i].node->buf->p;
        const bool conv = res <= tol;
        if (col_iters) col_iters[q] = conv ? done_passes + it : -1;
        if (col_resid) col_resid[q] = res;
        max_passes = std::max(max_passes, done_passes + it);
      }
    } else {
      // columns that did not converge within itermax (or ran no pass):
      // their current iterate
      for (int col = 0; col < pc.k; ++col) {
        if (!((rest >> col) & 1ull)) continue;
        const int q = col_set[(size_t)col];
        if (col_iters) col_iters[q] = -1;
        if (col_resid) col_resid[q] = hg.iters == 0 ? 1.0 : rr[(size_t)col];
      }
      out_of(rest, hg.iters);
    }
    // every column into X, whole rows at a time
    hip_check(launch_columns_in(ins, k, T, n, X, c.stream), "columns in");
    launch_mark(false);
    hip_check(hipStreamSynchronize(c.stream), "sync");
  } catch (...) {
    release();
    throw;
  }
  release();
  *iters = max_passes;
  }
  catch (const GrbError& e) {
    c.guard = saved_guard;
    api_error() = e.msg;
    return e.info;
  }
  catch (const std::exception& e) {
    c.guard = saved_guard;
    api_error() = e.what();
    return GrB_PANIC;
  }
  return GrB_SUCCESS;
}

GrB_Info GrM_ppr_stream(void* X, GrB_Type type, int nsets, const int32_t* seed_ptr, const int32_t* seed_vtx,
                        GrB_Matrix AT, GrB_Vector outdeg, double damping, double tol, int itermax,
                        GrM_Dangling dangling, int k, int check_every, int* set_iters, int* set_passes,
                        double* set_resid) {
  Ctx& c = ctx();
  GuardDev* saved_guard = c.guard;
  API_BEGIN
  require_init();
  need(X, "X");
  need(type, "type");
  GB_Matrix_opaque* ao = mat(AT, "AT");
  GB_Vector_opaque* dego = vec(outdeg, "outdeg");
  const int T = type->code;
  float_type(T, "type");
  const int64_t n = ao->nrows;
  if (ao->ncols != n || dego->n != n) fail(GrB_DIMENSION_MISMATCH, "ppr_stream dimensions");
  if (nsets < 1) fail(GrB_INVALID_VALUE, "nsets must be >= 1");
  if (k < 1 || k > 64) fail(GrB_INVALID_VALUE, "k must be in [1, 64]");
  if (dangling != GrM_DANGLING_DROP && dangling != GrM_DANGLING_UNIFORM) fail(GrB_INVALID_VALUE, "dangling mode");
  if (check_every < 1 || itermax < 1 || !(damping >= 0.0 && damping < 1.0) || std::isnan(tol))
    fail(GrB_INVALID_VALUE, "ppr_stream parameters");
  if (c.guard) fail(GrB_INVALID_VALUE, "an iterative driver is already running");
  check_seed_sets(nsets, seed_ptr, seed_vtx, n);
  if (k > nsets) k = nsets;

  PprColumns pc;
  pc.setup(ao, dego, T, k, damping, tol, dangling == GrM_DANGLING_UNIFORM);
  // the device guard only counts passes here (it never stops them)
  hip_check(launch_guard_init((GuardDev*)pc.gbuf->p, 1, -1.0, INT32_MAX, c.stream), "guard init");
  launch_mark(false);
  c.guard = (GuardDev*)pc.gbuf->p;
  pc.a.guard = c.guard;

  // slot_set[c]: the set in column c (-1: free), started after slot_start[c]
  // passes.  A column stops at the pass its residual first reaches tol (the
  // pass kernel freezes it there) or after itermax passes; it is written out
  // at the next check and the column restarts with the next set.  Once no
  // set is waiting and at most half the columns are live, the rest are
  // narrowed.
  std::vector<int> slot_set((size_t)k, -1), slot_start((size_t)k, 0);
  std::vector<PprSeed> active;  // seeds of the columns in use
  int next_set = 0, pass = 0, live = 0;
  auto set_seeds_of = [&](int q, int col, std::vector<PprSeed>& out) {
    const double w = 1.0 / (double)(seed_ptr[q + 1] - seed_ptr[q]);
    for (int e = seed_ptr[q]; e < seed_ptr[q + 1]; ++e) out.push_back({pc.exec_vertex(seed_vtx[e]), col, w});
  };
  // fill the free slots with the next sets, starting them in buffer set `cur`
  auto refill = [&](int cur, uint64_t freed) {
    // drop the seeds of retired columns, then hand free columns the next sets
    active.erase(std::remove_if(active.begin(), active.end(),
                                [&](const PprSeed& sd) { return slot_set[(size_t)sd.c] < 0; }),
                 active.end());
    uint64_t cols = 0;
    std::vector<PprSeed> fresh;
    for (int col = 0; col < pc.k && next_set < nsets; ++col) {
      if (slot_set[(size_t)col] >= 0) continue;
      slot_set[(size_t)col] = next_set;
      slot_start[(size_t)col] = pass;
      set_seeds_of(next_set, col, fresh);
      cols |= 1ull << col;
      ++next_set;
      ++live;
    }
    active.insert(active.end(), fresh.begin(), fresh.end());
    pc.set_seeds(active);
    pc.start_columns(cols | freed, cur, fresh);
  };
  refill(0, 0);
  std::vector<int> hh(64);
  std::vector<double> rr(64);
  ColumnOutputs outs{};
  outs.ld = 1;
  while (live > 0) {
    // up to check_every passes, never past a column's itermax
    int batch = check_every;
    for (int col = 0; col < pc.k; ++col)
      if (slot_set[(size_t)col] >= 0) batch = std::min(batch, itermax - (pass - slot_start[(size_t)col]));
    for (int j = 0; j < std::max(batch, 1); ++j) pc.run_pass(++pass);
    GuardDev hg{};
    pc.read_state(hh, rr, hg);
    if (hg.bad) fail(GrB_PANIC, "ppr_stream: a column's residual or dangling mass was not finite");
    const int cur = pass & 1;
    uint64_t retired = 0, from1 = 0;
    for (int col = 0; col < pc.k; ++col) {
      const int q = slot_set[(size_t)col];
      if (q < 0) continue;
      const int done = pass - slot_start[(size_t)col];
      const int h = hh[(size_t)col];
      const bool conv = h >= 0;
      if (!conv && done < itermax) continue;
      // retire: the iterate of the pass it converged in (frozen since), or
      // after itermax passes the current one
      retired |= 1ull << col;
      if ((conv ? h : pass) & 1) from1 |= 1ull << col;
      outs.out[col] = (char*)X + type_size(T) * (size_t)n * (size_t)q;
      if (set_iters) set_iters[q] = conv ? h - slot_start[(size_t)col] : -1;
      if (set_passes) set_passes[q] = conv ? h - slot_start[(size_t)col] : done;
      if (set_resid) set_resid[q] = rr[(size_t)col];
      slot_set[(size_t)col] = -1;
      --live;
    }
    pc.output(retired, from1, outs);
    // freed columns restart with new sets (or are zeroed) while sets wait
    if (retired && next_set < nsets) refill(cur, retired);
    if (next_set >= nsets && live > 0 && live <= pc.k / 2) {
      int k2 = 1;
      while (k2 < live) k2 <<= 1;
      std::vector<int> keep, newpos((size_t)pc.k, -1), set2((size_t)k2, -1), start2((size_t)k2, 0);
      for (int col = 0; col < pc.k; ++col)
        if (slot_set[(size_t)col] >= 0) {
          newpos[(size_t)col] = (int)keep.size();
          set2[keep.size()] = slot_set[(size_t)col];
          start2[keep.size()] = slot_start[(size_t)col];
          keep.push_back(col);
        }
      std::vector<PprSeed> kept;
      for (const PprSeed& sd : active)
        if (newpos[(size_t)sd.c] >= 0) kept.push_back({sd.v, newpos[(size_t)sd.c], sd.w});
      pc.narrow(pass, keep, k2);
      active.swap(kept);
      pc.set_seeds(active);
      slot_set.swap(set2);
      slot_start.swap(start2);
    }
  }
  c.guard = saved_guard;
  hip_check(hipStreamSynchronize(c.stream), "sync");
  }
  catch (const GrbError& e) {
    c.guard = saved_guard;
    api_error() = e.msg;
    return e.info;
  }
  catch (const std::exception& e) {
    c.guard = saved_guard;
    api_error() = e.what();
    return GrB_PANIC;
  }
  return GrB_SUCCESS;
}

// ------------------------------------------------------------ sparse x dense

GrB_Info GrB_mxm(GrB_Matrix C, GrB_Matrix Mask, GrB_BinaryOp accum, GrB_Semiring op, GrB_Matrix A, GrB_Matrix B,
                 GrB_Descriptor desc) {
  API_BEGIN
  require_init();
  GB_Matrix_opaque* co = mat_any(C, "C");
  GB_Matrix_opaque* ao = mat(A, "A");
  GB_Matrix_opaque* bo = mat_any(B, "B");
  need(op, "semiring");
  if (Mask) fail(GrB_NOT_IMPLEMENTED, "GrB_mxm: masks are not supported");
  if (accum) fail(GrB_NOT_IMPLEMENTED, "GrB_mxm: accumulators are not supported");
  if (desc) fail(GrB_NOT_IMPLEMENTED, "GrB_mxm: descriptors are not supported");
  if (!bo->data->dense) fail(GrB_NOT_IMPLEMENTED, "GrB_mxm: B must be dense (GrM_Matrix_import_dense)");
  if (op->add != B_PLUS || (op->mul != B_TIMES && op->mul != B_SECOND))
    fail(GrB_NOT_IMPLEMENTED, "GrB_mxm: only plus-times / plus-second semirings");
  const int T = op->type;
  float_type(T, "semiring");
  if (bo->data->dense_type != T || co->type != T) fail(GrB_DOMAIN_MISMATCH, "GrB_mxm: B, C and the semiring differ in type");
  if (ao->ncols != bo->nrows || co->nrows != ao->nrows || co->ncols != bo->ncols)
    fail(GrB_DIMENSION_MISMATCH, "GrB_mxm dimensions");
  const int64_t n = ao->nrows;
  const int k = (int)bo->ncols;
  if (k < 1 || k > 64) fail(GrB_NOT_IMPLEMENTED, "GrB_mxm: B may have at most 64 columns");
  Ctx& c = ctx();
  const MatP& Am = ao->data;

  // the wavefront tile plan of A (lane c of a wavefront owns column c)
  PlanConfig wp;
  wp.kernel = K_WAVE;
  wp.lds_entries = WAVE_TILE_ENTRIES;
  wp.lds_rows = WAVE_TILE_ROWS;
  wp.long_row = WAVE_TILE_ENTRIES;
  wp.chunk = WAVE_TILE_ENTRIES;
  wp.grid = c.cus * 2;
  auto plan = get_plan(Am, wp);
  if (plan->cfg.kernel != K_WAVE)
    fail(GrB_NOT_IMPLEMENTED, "GrB_mxm: A has too many columns for the wavefront tile plan (2^29 or more)");

  auto m = std::make_shared<MatData>();
  m->id = c.next_id++;
  m->nrows = n;
  m->ncols = k;
  m->dense_type = T;
  const size_t obytes = type_size(T) * (size_t)n * (size_t)k;
  m->dense = dev_alloc(obytes);
  const size_t bbytes = type_size(T) * (size_t)bo->nrows * (size_t)k;
  BufP hub_sum = dev_alloc(sizeof(double) * 64 * (size_t)std::max(plan->nparts, 1));
  BufP hub_cnt = dev_alloc(sizeof(int) * (size_t)std::max(plan->nhubs, 1));
  BufP hub_red = dev_alloc(sizeof(double) * 128 * (size_t)std::max(plan->nhubs, 1));
  hip_check(launch_zero(hub_cnt->p, sizeof(int) * (size_t)std::max(plan->nhubs, 1), c.stream), "zero");
  launch_mark(false);
  SpmmArgs a{};
  a.rowptr = (const int*)Am->rowptr->p;
  a.col = Am->col ? (const int*)Am->col->p : nullptr;
  a.k = k;
  a.w = bo->data->dense->p;
  // the buffer-addressed pass needs every operand below 4 GiB
  a.w_bytes = std::max(bbytes, obytes) < 0xFFFFFF00ull ? (unsigned)std::max(bbytes, obytes) : 0u;
  a.x_new = m->dense->p;
  a.hub_sum = (double*)hub_sum->p;
  a.hub_cnt = (int*)hub_cnt->p;
  a.hub_red = (double*)hub_red->p;
  a.plain = 1;
  // no more workgroups than tiles can use (16 wavefronts each)
  const int grid = std::max(1, std::min(plan->cfg.grid, (std::max(plan->dev.ntiles, 1) + 15) / 16));
  if (plan->dev.ntiles > 0) {
    hip_check(launch_spmm_ppr(plan->dev, a, T, grid, nullptr, c.stream), "mxm");
    launch_mark(false);
  } else {
    hip_check(launch_zero(m->dense->p, obytes, c.stream), "zero");
    launch_mark(false);
  }
  co->data = m;
  API_END
}

// ------------------------------------------------------------ many graphs

struct GB_Multigraph_opaque {
  uint32_t magic;
  int ngraphs;
  int64_t nv, ne;
  std::vector<int64_t> voff;
  int nslots = 0;
  BufP graphs, queue, qnext, rowptr, col, deg, inv, longrows, xa, xb, wa, wb, iters, resid, team_bar, team_part, team_err;
  std::vector<std::shared_ptr<MatData>> keep;  // relabeled copies stay alive
  struct Exec {
    int type;
    double damping, tol;
    int itermax, uniform;
    void* out;
    unsigned long long wait_ticks;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<Exec> execs;
  hipStream_t aux = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};
static constexpr uint32_t MAGIC_MULTI = 0x4d554c54u;

static void multigraph_release(GB_Multigraph_opaque* m) {
  for (auto& e : m->execs) {
    (void)hipGraphExecDestroy(e.exec);
    (void)hipGraphDestroy(e.graph);
  }
  m->execs.clear();
  if (m->ev0) (void)hipEventDestroy(m->ev0);
  if (m->ev1) (void)hipEventDestroy(m->ev1);
  if (m->aux) (void)hipStreamDestroy(m->aux);
}

GrB_Info GrM_Multigraph_new(GrM_Multigraph* mg, int ngraphs, const GrB_Matrix* AT) {
  GB_Multigraph_opaque* m = nullptr;
  API_BEGIN
  require_init();
  need(mg, "mg");
  need(AT, "AT");
  if (ngraphs < 1) fail(GrB_INVALID_VALUE, "ngraphs must be >= 1");
  Ctx& c = ctx();
  std::vector<std::shared_ptr<Relabeled>> rls;
  std::vector<ManyGraph> gs((size_t)ngraphs);
  int64_t nv = 0, ne = 0, nr = 0;
  for (int g = 0; g < ngraphs; ++g) {
    GB_Matrix_opaque* a = mat(AT[g], "AT[g]");
    if (a->nrows != a->ncols) fail(GrB_DIMENSION_MISMATCH, "graphs must be square");
    rls.push_back(get_relabeled(a->data));
    const MatData& r = *rls.back()->A;
    ManyGraph& G = gs[(size_t)g];
    G.n = (int)r.nrows;
    G.m = (int)r.nnz;
    const double avg = r.nrows > 0 ? (double)r.nnz / (double)r.nrows : 0.0;
    int lpr = 1;
    while (lpr * 2 <= avg && lpr < 32) lpr *= 2;
    G.lpr = lpr;
    G.nlong = 0;
    G.loff = 0;
    G.team = 1;
    G.pad_ = 0;
    G.voff = nv;
    G.eoff = ne;
    G.roff = nr;
    nv += r.nrows;
    ne += r.nnz;
    nr += r.nrows + 1;
  }
  if (ne > (int64_t)INT32_MAX * 4) fail(GrB_INVALID_VALUE, "too many entries");
  // rows too long for one lane group, per graph
  std::vector<int> longrows;
  for (int g = 0; g < ngraphs; ++g) {
    const MatData& r = *rls[(size_t)g]->A;
    std::vector<int> rp((size_t)r.nrows + 1);
    hip_check(hipMemcpyAsync(rp.data(), r.rowptr->p, sizeof(int) * rp.size(), hipMemcpyDeviceToHost, c.stream),
              "copy row pointers");
    hip_check(hipStreamSynchronize(c.stream), "sync");
    ManyGraph& G = gs[(size_t)g];
    G.loff = (int64_t)longrows.size();
    for (int64_t i = 0; i < r.nrows; ++i)
      if (rp[(size_t)i + 1] - rp[(size_t)i] > MANY_LONG_ROW) longrows.push_back((int)i);
    G.nlong = (int)((int64_t)longrows.size() - G.loff);
  }
  m = new GB_Multigraph_opaque();
  m->magic = MAGIC_MULTI;
  m->ngraphs = ngraphs;
  m->nv = nv;
  m->ne = ne;
  m->graphs = dev_alloc(sizeof(ManyGraph) * gs.size());
  m->rowptr = dev_alloc(sizeof(int) * (size_t)nr);
  m->col = dev_alloc(sizeof(int) * (size_t)std::max<int64_t>(ne, 1));
  m->deg = dev_alloc(sizeof(int) * (size_t)nv);
  m->inv = dev_alloc(sizeof(int) * (size_t)nv);
  for (BufP* b : {&m->xa, &m->xb, &m->wa, &m->wb}) *b = dev_alloc(sizeof(double) * (size_t)nv);
  m->iters = dev_alloc(sizeof(int) * (size_t)ngraphs);
  m->resid = dev_alloc(sizeof(double) * (size_t)ngraphs);
  m->qnext = dev_alloc(256);
  hip_check(launch_fill(m->deg->p, T_INT32, nv, 0.0, c.stream), "fill");
  launch_mark(false);
  for (int g = 0; g < ngraphs; ++g) {
    const ManyGraph& G = gs[(size_t)g];
    const MatData& r = *rls[(size_t)g]->A;
    hip_check(hipMemcpyAsync((int*)m->rowptr->p + G.roff, r.rowptr->p, sizeof(int) * (size_t)(G.n + 1),
                             hipMemcpyDeviceToDevice, c.stream), "pack");
    if (G.m > 0) {
      hip_check(hipMemcpyAsync((int*)m->col->p + G.eoff, r.col->p, sizeof(int) * (size_t)G.m,
                               hipMemcpyDeviceToDevice, c.stream), "pack");
      hip_check(launch_column_count((const int*)r.col->p, G.m, (int*)m->deg->p + G.voff, c.stream), "degrees");
      launch_mark(false);
    }
    hip_check(hipMemcpyAsync((int*)m->inv->p + G.voff, rls[(size_t)g]->inv->p, sizeof(int) * (size_t)G.n,
                             hipMemcpyDeviceToDevice, c.stream), "pack");
    m->voff.push_back(G.voff);
    m->keep.push_back(rls[(size_t)g]->A);
  }
  m->voff.push_back(nv);
  std::vector<int> order((size_t)ngraphs);
  for (int g = 0; g < ngraphs; ++g) order[(size_t)g] = g;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return gs[(size_t)a].m > gs[(size_t)b].m; });
  // Teams: a graph gets about one workgroup per mean per-CU share of all
  // edges (at most many_team_max).  Team slots lead the queue and number at
  // most the grid (one workgroup per compute unit), so every member of
  // every team starts at once.
  {
    const double share = std::max(1.0, (double)ne / (double)c.cus);
    int used = 0;
    for (int g : order) {
      ManyGraph& G = gs[(size_t)g];
      int t = (int)std::llround((double)G.m / share);
      t = std::max(1, std::min(t, std::min(c.many_team_max, MANY_MAX_TEAM)));
      if (t > 1 && used + t > c.cus) t = 1;
      if (t > 1) used += t;
      G.team = t;
    }
  }
  std::stable_partition(order.begin(), order.end(), [&](int g) { return gs[(size_t)g].team > 1; });
  std::vector<int> slots;
  for (int g : order)
    for (int k = 0; k < gs[(size_t)g].team; ++k) slots.push_back(g * MANY_MAX_TEAM + k);
  m->nslots = (int)slots.size();
  m->team_bar = dev_alloc(sizeof(unsigned) * (size_t)ngraphs);
  m->team_part = dev_alloc(sizeof(double) * 4 * MANY_MAX_TEAM * (size_t)ngraphs);
  m->team_err = dev_alloc(sizeof(int));
  m->queue = dev_alloc(sizeof(int) * slots.size());
  m->longrows = dev_alloc(sizeof(int) * std::max<size_t>(longrows.size(), 1));
  if (!longrows.empty())
    hip_check(hipMemcpyAsync(m->longrows->p, longrows.data(), sizeof(int) * longrows.size(), hipMemcpyHostToDevice,
                             c.stream), "upload");
  hip_check(hipMemcpyAsync(m->graphs->p, gs.data(), sizeof(ManyGraph) * gs.size(), hipMemcpyHostToDevice, c.stream),
            "upload");
  hip_check(hipMemcpyAsync(m->queue->p, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice, c.stream),
            "upload");
  hip_check(hipStreamSynchronize(c.stream), "sync");
  hip_check(hipStreamCreateWithFlags(&m->aux, hipStreamNonBlocking), "stream");
  hip_check(hipEventCreateWithFlags(&m->ev0, hipEventDisableTiming), "event");
  hip_check(hipEventCreateWithFlags(&m->ev1, hipEventDisableTiming), "event");
  *mg = m;
  m = nullptr;
  }
  catch (const GrbError& e) {
    if (m) {
      multigraph_release(m);
      delete m;
    }
    api_error() = e.msg;
    return e.info;
  }
  catch (const std::exception& e) {
    api_error() = e.what();
    return GrB_PANIC;
  }
  return GrB_SUCCESS;
}

GrB_Info GrM_Multigraph_free(GrM_Multigraph* mg) {
  API_BEGIN
  if (!mg || !*mg) return GrB_SUCCESS;
  GB_Multigraph_opaque* m = *mg;
  if (m->magic != MAGIC_MULTI) fail(GrB_UNINITIALIZED_OBJECT, "not a multigraph");
  (void)hipStreamSynchronize(ctx().stream);
  if (m->aux) (void)hipStreamSynchronize(m->aux);
  multigraph_release(m);
  m->magic = MAGIC_FREED;
  delete m;
  *mg = nullptr;
  API_END
}

GrB_Info GrM_Multigraph_offsets(int64_t* voff, GrM_Multigraph mg) {
  API_BEGIN
  need(voff, "voff");
  need(mg, "mg");
  if (mg->magic != MAGIC_MULTI) fail(GrB_UNINITIALIZED_OBJECT, "not a multigraph");
  for (size_t i = 0; i < mg->voff.size(); ++i) voff[i] = mg->voff[i];
  API_END
}

GrB_Info GrM_pagerank_many(void* X, GrB_Type type, GrM_Multigraph mg, double damping, double tol, int itermax,
                           GrM_Dangling dangling, int* iters, double* resid) {
  API_BEGIN
  require_init();
  need(X, "X");
  need(type, "type");
  need(mg, "mg");
  if (mg->magic != MAGIC_MULTI) fail(GrB_UNINITIALIZED_OBJECT, "not a multigraph");
  const int T = type->code;
  float_type(T, "type");
  if (dangling != GrM_DANGLING_DROP && dangling != GrM_DANGLING_UNIFORM) fail(GrB_INVALID_VALUE, "dangling mode");
  if (itermax < 0 || !(damping >= 0.0 && damping < 1.0) || std::isnan(tol))
    fail(GrB_INVALID_VALUE, "pagerank parameters");
  Ctx& c = ctx();
  const int uniform = dangling == GrM_DANGLING_UNIFORM ? 1 : 0;
  GB_Multigraph_opaque::Exec* ex = nullptr;
  for (auto& e : mg->execs)
    if (e.type == T && e.damping == damping && e.tol == tol && e.itermax == itermax && e.uniform == uniform &&
        e.out == X && e.wait_ticks == c.many_wait_ticks)
      ex = &e;
  if (!ex) {
    ManyArgs a{};
    a.graphs = (const ManyGraph*)mg->graphs->p;
    a.queue = (const int*)mg->queue->p;
    a.queue_next = (int*)mg->qnext->p;
    a.ngraphs = mg->ngraphs;
    a.nslots = mg->nslots;
    a.team_bar = (unsigned*)mg->team_bar->p;
    a.team_part = (double*)mg->team_part->p;
    a.team_err = (int*)mg->team_err->p;
    a.team_wait_ticks = c.many_wait_ticks;
    a.rowptr = (const int*)mg->rowptr->p;
    a.col = (const int*)mg->col->p;
    a.deg = (const int*)mg->deg->p;
    a.inv = (const int*)mg->inv->p;
    a.longrows = (const int*)mg->longrows->p;
    a.xa = mg->xa->p;
    a.xb = mg->xb->p;
    a.wa = mg->wa->p;
    a.wb = mg->wb->p;
    a.out = X;
    a.iters = (int*)mg->iters->p;
    a.resid = (double*)mg->resid->p;
    a.damping = damping;
    a.tol = tol;
    a.itermax = itermax;
    a.uniform = uniform;
    GB_Multigraph_opaque::Exec e{T, damping, tol, itermax, uniform, X, c.many_wait_ticks, nullptr, nullptr};
    hip_check(hipStreamBeginCapture(mg->aux, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t le = launch_pr_many(a, T, c.cus, mg->aux);
    hipGraph_t gph = nullptr;
    hipError_t ce = hipStreamEndCapture(mg->aux, &gph);
    hip_check(le, "many-graph launch");
    hip_check(ce, "end capture");
    e.graph = gph;
    hip_check(hipGraphInstantiate(&e.exec, gph, nullptr, nullptr, 0), "instantiate");
    mg->execs.push_back(e);
    ex = &mg->execs.back();
  }
  // order the replay after the library stream's work, and later work after it
  hip_check(hipEventRecord(mg->ev0, c.stream), "record");
  hip_check(hipStreamWaitEvent(mg->aux, mg->ev0, 0), "wait");
  hip_check(hipGraphLaunch(ex->exec, mg->aux), "graph launch");
  hip_check(hipEventRecord(mg->ev1, mg->aux), "record");
  hip_check(hipStreamWaitEvent(c.stream, mg->ev1, 0), "wait");
  launch_mark(true);
  if (iters)
    hip_check(hipMemcpyAsync(iters, mg->iters->p, sizeof(int) * (size_t)mg->ngraphs, hipMemcpyDeviceToHost, c.stream),
              "copy");
  if (resid)
    hip_check(hipMemcpyAsync(resid, mg->resid->p, sizeof(double) * (size_t)mg->ngraphs, hipMemcpyDeviceToHost,
                             c.stream),
              "copy");
  int team_err = 0;
  if (iters || resid)
    hip_check(hipMemcpyAsync(&team_err, mg->team_err->p, sizeof(int), hipMemcpyDeviceToHost, c.stream), "copy");
  if (iters || resid) hip_check(hipStreamSynchronize(c.stream), "sync");
  if (team_err & 1) fail(GrB_PANIC, "a team of workgroups gave up waiting for a member");
  if (team_err & 2) fail(GrB_PANIC, "pagerank_many: a graph's residual was not finite");
  API_END
}

GrB_Info GrM_set_many_team_wait(unsigned long long ticks) {
  API_BEGIN
  require_init();
  ctx().many_wait_ticks = ticks;
  API_END
}

GrB_Info GrM_set_many_team_max(int max_team) {
  API_BEGIN
  require_init();
  if (max_team < 1 || max_team > MANY_MAX_TEAM) fail(GrB_INVALID_VALUE, "max_team must be 1..8");
  ctx().many_team_max = max_team;
  API_END
}

}  // extern "C"
