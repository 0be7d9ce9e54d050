// C ABI entry points (declared in include/nbgrb.h) for the context, the
// objects and the operations; the iterative drivers are in drivers.hip.
// Each call validates its arguments eagerly, then records (nonblocking) or
// runs (blocking) the operation through the runtime.  Internal errors are
// C++ exceptions that are turned into GrB_Info codes here.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "abi_util.h"

using namespace nbgrb;

// ------------------------------------------------------------ built-ins

static GB_Type_opaque t_bool{T_BOOL}, t_int32{T_INT32}, t_fp32{T_FP32}, t_fp64{T_FP64}, t_bf16{T_BF16};
GrB_Type GrB_BOOL = &t_bool, GrB_INT32 = &t_int32, GrB_FP32 = &t_fp32, GrB_FP64 = &t_fp64, GrM_BF16 = &t_bf16;

#define UNOP(NAME, OP, T)                  \
  static GB_UnaryOp_opaque u_##NAME{OP, T}; \
  GrB_UnaryOp NAME = &u_##NAME;
UNOP(GrB_IDENTITY_FP32, U_IDENTITY, T_FP32)
UNOP(GrB_IDENTITY_FP64, U_IDENTITY, T_FP64)
UNOP(GrB_ABS_FP32, U_ABS, T_FP32)
UNOP(GrB_ABS_FP64, U_ABS, T_FP64)
UNOP(GrB_AINV_FP32, U_AINV, T_FP32)
UNOP(GrB_AINV_FP64, U_AINV, T_FP64)
UNOP(GrB_MINV_FP32, U_MINV, T_FP32)
UNOP(GrB_MINV_FP64, U_MINV, T_FP64)
UNOP(GrM_MINV_OR_ZERO_FP32, U_MINV_OR_ZERO, T_FP32)
UNOP(GrM_MINV_OR_ZERO_FP64, U_MINV_OR_ZERO, T_FP64)

#define BINOP(NAME, OP, T)                   \
  static GB_BinaryOp_opaque b_##NAME{OP, T}; \
  GrB_BinaryOp NAME = &b_##NAME;
BINOP(GrB_PLUS_FP32, B_PLUS, T_FP32)
BINOP(GrB_PLUS_FP64, B_PLUS, T_FP64)
BINOP(GrB_MINUS_FP32, B_MINUS, T_FP32)
BINOP(GrB_MINUS_FP64, B_MINUS, T_FP64)
BINOP(GrB_TIMES_FP32, B_TIMES, T_FP32)
BINOP(GrB_TIMES_FP64, B_TIMES, T_FP64)
BINOP(GrB_DIV_FP32, B_DIV, T_FP32)
BINOP(GrB_DIV_FP64, B_DIV, T_FP64)
BINOP(GrB_MAX_FP32, B_MAX, T_FP32)
BINOP(GrB_MAX_FP64, B_MAX, T_FP64)
BINOP(GrB_MIN_FP32, B_MIN, T_FP32)
BINOP(GrB_MIN_FP64, B_MIN, T_FP64)
BINOP(GrB_FIRST_FP32, B_FIRST, T_FP32)
BINOP(GrB_FIRST_FP64, B_FIRST, T_FP64)
BINOP(GrB_SECOND_FP32, B_SECOND, T_FP32)
BINOP(GrB_SECOND_FP64, B_SECOND, T_FP64)
BINOP(GrM_ABSDIFF_FP32, B_ABSDIFF, T_FP32)
BINOP(GrM_ABSDIFF_FP64, B_ABSDIFF, T_FP64)

static GB_Monoid_opaque m_plus32{B_PLUS, T_FP32}, m_plus64{B_PLUS, T_FP64};
GrB_Monoid GrB_PLUS_MONOID_FP32 = &m_plus32, GrB_PLUS_MONOID_FP64 = &m_plus64;

static GB_Semiring_opaque s_pt32{B_PLUS, B_TIMES, T_FP32}, s_pt64{B_PLUS, B_TIMES, T_FP64};
static GB_Semiring_opaque s_ps32{B_PLUS, B_SECOND, T_FP32}, s_ps64{B_PLUS, B_SECOND, T_FP64};
GrB_Semiring GrB_PLUS_TIMES_SEMIRING_FP32 = &s_pt32, GrB_PLUS_TIMES_SEMIRING_FP64 = &s_pt64;
GrB_Semiring GrM_PLUS_SECOND_SEMIRING_FP32 = &s_ps32, GrM_PLUS_SECOND_SEMIRING_FP64 = &s_ps64;

static GB_Descriptor_opaque d_comp{true, false, false}, d_s{false, true, false}, d_sc{true, true, false},
    d_r{false, false, true}, d_rc{true, false, true}, d_rs{false, true, true}, d_rsc{true, true, true};
GrB_Descriptor GrB_DESC_C = &d_comp;
GrB_Descriptor GrB_DESC_S = &d_s;
GrB_Descriptor GrB_DESC_SC = &d_sc;
GrB_Descriptor GrB_DESC_R = &d_r;
GrB_Descriptor GrB_DESC_RC = &d_rc;
GrB_Descriptor GrB_DESC_RS = &d_rs;
GrB_Descriptor GrB_DESC_RSC = &d_rsc;

// ------------------------------------------------------------ errors

namespace nbgrb {

std::string& api_error() {
  static thread_local std::string text;
  return text;
}

}  // namespace nbgrb

void nbgrb::set_error_text(const std::string& msg) { api_error() = msg; }


void nbgrb::need(const void* p, const char* what) {
  if (!p) fail(GrB_NULL_POINTER, std::string(what) + " is NULL");
}

GB_Vector_opaque* nbgrb::vec(GrB_Vector v, const char* what) {
  need(v, what);
  if (v->magic != MAGIC_VEC) fail(GrB_UNINITIALIZED_OBJECT, std::string(what) + " is not a vector");
  return v;
}

GB_Scalar_opaque* nbgrb::sca(GrB_Scalar s, const char* what) {
  need(s, what);
  if (s->magic != MAGIC_SCA) fail(GrB_UNINITIALIZED_OBJECT, std::string(what) + " is not a scalar");
  return s;
}

GB_Matrix_opaque* nbgrb::mat_any(GrB_Matrix A, const char* what) {
  need(A, what);
  if (A->magic != MAGIC_MAT) fail(GrB_UNINITIALIZED_OBJECT, std::string(what) + " is not a matrix");
  return A;
}

GB_Matrix_opaque* nbgrb::mat(GrB_Matrix A, const char* what) {
  mat_any(A, what);
  if (A->data && A->data->dense)
    fail(GrB_INVALID_VALUE, std::string(what) + " holds dense values; only GrB_mxm's second operand and output, "
                                                "GrM_Matrix_export_dense and the size queries take a dense matrix");
  return A;
}

void nbgrb::no_mask_accum(const void* mask, const void* accum) {
  if (mask) fail(GrB_NOT_IMPLEMENTED, "masks are not supported by this operation");
  if (accum) fail(GrB_NOT_IMPLEMENTED, "accumulators are not supported");
}

void nbgrb::float_type(int t, const char* what) {
  if (t != T_FP32 && t != T_FP64) fail(GrB_DOMAIN_MISMATCH, std::string(what) + " must be FP32 or FP64");
}

bool nbgrb::desc_comp(GrB_Descriptor d) { return d && d->mask_comp; }
bool nbgrb::desc_struct(GrB_Descriptor d) { return d && d->mask_struct; }
bool nbgrb::desc_replace(GrB_Descriptor d) { return d && d->replace; }

// ------------------------------------------------------------ recording

namespace nbgrb {

NodeP iso_node(int type, int64_t n, double v) {
  NodeP p = new_node(N_DENSE, type, n, false);
  p->done = true;
  p->iso = true;
  p->iso_val = v;
  return p;
}

void rec_ewise(GB_Vector_opaque* w, int op, GB_Vector_opaque* u, GB_Vector_opaque* v, bool set_union) {
  NodeP p = new_node(N_EWISE, w->type, w->n, false);
  p->a = u->node;
  p->b = v->node;
  p->op = op;
  p->set_union = set_union;
  submit(p);
  set_vec(w, p);
}

void rec_unop(GB_Vector_opaque* w, int op, GB_Vector_opaque* u) {
  NodeP p = new_node(N_APPLY_U, w->type, w->n, false);
  p->a = u->node;
  p->op = op;
  submit(p);
  set_vec(w, p);
}

void rec_bind(GB_Vector_opaque* w, int op, GB_Vector_opaque* u, double k, bool first) {
  NodeP p = new_node(first ? N_APPLY_B1 : N_APPLY_B2, w->type, w->n, false);
  p->a = u->node;
  p->op = op;
  p->k = k;
  submit(p);
  set_vec(w, p);
}

void rec_bind_scalar(GB_Vector_opaque* w, int op, GB_Vector_opaque* u, GB_Scalar_opaque* s) {
  NodeP p = new_node(N_APPLY_B2S, w->type, w->n, false);
  p->a = u->node;
  p->s = s->node;
  p->op = op;
  submit(p);
  set_vec(w, p);
}

void rec_mxv(GB_Vector_opaque* w, GB_Matrix_opaque* A, GB_Vector_opaque* u, GB_Vector_opaque* mask,
             GrB_Descriptor desc) {
  NodeP p = new_node(N_MXV, w->type, w->n, false);
  p->A = A->data;
  p->a = u->node;
  if (mask) {
    p->mask = mask->node;
    p->mask_comp = desc_comp(desc);
    p->mask_struct = desc_struct(desc);
    p->replace = desc_replace(desc);
    if (!p->replace) p->b = w->node;  // positions the mask forbids keep w's entries
  }
  submit(p);
  set_vec(w, p);
}

void rec_assign(GB_Vector_opaque* w, GB_Vector_opaque* mask, double x, GrB_Descriptor desc) {
  NodeP p = new_node(N_ASSIGN, w->type, w->n, false);
  p->k = x;
  if (mask) {
    p->mask = mask->node;
    p->mask_comp = desc_comp(desc);
    p->mask_struct = desc_struct(desc);
  }
  p->replace = desc_replace(desc);
  if (!p->replace && mask) p->b = w->node;
  submit(p);
  set_vec(w, p);
}

void rec_reduce(GB_Scalar_opaque* s, GB_Vector_opaque* u, GB_Vector_opaque* mask, bool comp,
                bool watch) {
  NodeP p = new_node(mask ? N_REDUCE_MASK : N_REDUCE, T_FP64, 0, true);
  p->a = u->node;
  if (mask) {
    p->mask = mask->node;
    p->mask_comp = comp;
  }
  p->guard_watch = watch;
  submit(p);
  set_sca(s, p);
}

void rec_affine(GB_Scalar_opaque* out, double alpha, GB_Scalar_opaque* in, double beta) {
  NodeP p = new_node(N_AFFINE, T_FP64, 0, true);
  p->s = in->node;
  p->alpha = alpha;
  p->beta = beta;
  submit(p);
  set_sca(out, p);
}

void store_if_iso(const NodeP& v) {
  if (!v->iso) return;
  BufP b = dev_alloc(type_size(v->type) * (size_t)v->n);
  hip_check(launch_fill(b->p, v->type, v->n, v->iso_val, ctx().stream), "fill");
  launch_mark(false);
  v->buf = b;
  v->iso = false;
}

MatP new_matdata(int64_t nrows, int64_t ncols) {
  auto m = std::make_shared<MatData>();
  m->id = ctx().next_id++;
  m->nrows = nrows;
  m->ncols = ncols;
  m->nnz = 0;
  m->rowptr = dev_alloc(sizeof(int) * (size_t)(nrows + 1));
  hip_check(launch_fill(m->rowptr->p, T_INT32, nrows + 1, 0.0, ctx().stream), "fill");
  launch_mark(false);
  return m;
}

// out[k] = v[idx[k]] as a new materialised node (iso vectors stay iso).
NodeP permuted(const NodeP& v, const BufP& idx) {
  materialize(v);
  require_full(v, "a relabeled run");
  if (v->iso) return iso_node(v->type, v->n, v->iso_val);
  NodeP p = new_node(N_DENSE, v->type, v->n, false);
  p->buf = dev_alloc(type_size(v->type) * (size_t)v->n);
  hip_check(launch_permute(v->buf->p, v->type, (const int*)idx->p, p->buf->p, v->n, ctx().stream), "permute");
  launch_mark(false);
  p->done = true;
  return p;
}

int read_flag(const BufP& f) {
  int h = 0;
  hip_check(hipMemcpyAsync(&h, f->p, sizeof(int), hipMemcpyDeviceToHost, ctx().stream), "copy flag");
  hip_check(hipStreamSynchronize(ctx().stream), "sync");
  return h;
}

}  // namespace

extern "C" {

// ------------------------------------------------------------ context

GrB_Info GrB_init(GrB_Mode mode) {
  API_BEGIN
  Ctx& c = ctx();
  if (c.init) fail(GrB_INVALID_VALUE, "already initialised");
  if (mode != GrB_BLOCKING && mode != GrB_NONBLOCKING) fail(GrB_INVALID_VALUE, "unknown mode");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    fail(GrB_PANIC, "no HIP device");
  }
  hip_check(hipGetDevice(&c.device), "get device");
  hipDeviceProp_t prop;
  hip_check(hipGetDeviceProperties(&prop, c.device), "device properties");
  c.cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c.mode = mode;
  c.stream = nullptr;
  noalloc_setup(c.device, nullptr);
  c.stats = Stats{};
  c.init = true;
  API_END
}

GrB_Info GrB_finalize(void) {
  API_BEGIN
  Ctx& c = ctx();
  if (!c.init) return GrB_SUCCESS;
  (void)hipStreamSynchronize(c.stream);
  c.pending.clear();
  c.red_part.reset();
  c.red_ticket.reset();
  c.fused_part.reset();
  c.fused_ticket.reset();
  c.fused_part_cap = 0;
  c.guard = nullptr;
  for (auto& e : c.events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  c.events.clear();
  for (auto e : c.event_pool) (void)hipEventDestroy(e);
  c.event_pool.clear();
  for (auto& e : c.guard_snap_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (c.guard_snap) (void)hipHostFree(c.guard_snap);
  c.guard_snap = nullptr;
  if (c.ppr_snap_ev) (void)hipEventDestroy(c.ppr_snap_ev);
  c.ppr_snap_ev = nullptr;
  if (c.ppr_snap) (void)hipHostFree(c.ppr_snap);
  c.ppr_snap = nullptr;
  c.tuned.clear();
  c.dinv_cache.clear();
  c.init = false;
  for (auto& kv : c.cache)
    for (void* p : kv.second) raw_release(p);
  c.cache.clear();
  API_END
}

GrB_Info GrM_get_mode(GrB_Mode* mode) {
  API_BEGIN
  require_init();
  need(mode, "mode");
  *mode = ctx().mode;
  API_END
}

GrB_Info GrM_set_mode(GrB_Mode mode) {
  API_BEGIN
  require_init();
  if (mode != GrB_BLOCKING && mode != GrB_NONBLOCKING) fail(GrB_INVALID_VALUE, "unknown mode");
  force_all();
  ctx().mode = mode;
  API_END
}

const char* GrM_error(void) { return api_error().c_str(); }

GrB_Info GrM_set_stream(void* hip_stream) {
  API_BEGIN
  require_init();
  Ctx& c = ctx();
  force_all();
  hip_check(hipStreamSynchronize(c.stream), "sync old stream");
  c.stream = (hipStream_t)hip_stream;
  API_END
}

GrB_Info GrM_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*), void* actx) {
  API_BEGIN
  require_init();
  Ctx& c = ctx();
  if ((alloc == nullptr) != (release == nullptr)) fail(GrB_NULL_POINTER, "give both callbacks or neither");
  force_all();
  hip_check(hipStreamSynchronize(c.stream), "sync");
  for (auto& kv : c.cache)
    for (void* p : kv.second) raw_release(p);
  c.cache.clear();
  if (c.live_bytes != 0) fail(GrB_INVALID_VALUE, "objects still hold device memory");
  c.alloc = alloc;
  c.release = release;
  c.actx = actx;
  API_END
}

GrB_Info GrM_fail_allocation_after(int64_t k) {
  API_BEGIN
  require_init();
  if (k < 0) fail(GrB_INVALID_VALUE, "k < 0");
  Ctx& c = ctx();
  c.fail_after = k;
  if (k > 0) {
    // force fresh allocations so the countdown is seen
    for (auto& kv : c.cache)
      for (void* p : kv.second) raw_release(p);
    c.cache.clear();
  }
  API_END
}

GrB_Info GrM_get_stats(GrM_Stats* s) {
  API_BEGIN
  require_init();
  need(s, "stats");
  const Stats& t = ctx().stats;
  s->kernels = t.kernels;
  s->fused_launches = t.fused;
  s->plan_hits = t.plan_hits;
  s->plan_misses = t.plan_misses;
  s->elided_nodes = t.elided;
  s->forced_waits = t.waits;
  s->ewise_fused = t.ewise_fused;
  s->ewise_ops = t.ewise_ops;
  s->jit_compiles = t.jit_compiles;
  s->jit_disk_hits = t.jit_disk_hits;
  s->jit_memory_hits = t.jit_memory_hits;
  s->mxv_push = t.mxv_push;
  s->mxv_pull = t.mxv_pull;
  s->out_full = t.out_full;
  s->out_bitset = t.out_bitset;
  s->out_sparse = t.out_sparse;
  s->index_loops = t.index_loops;
  s->range_loops = t.range_loops;
  s->device_allocs = t.device_allocs;
  API_END
}

GrB_Info GrM_set_fusion(int level) {
  API_BEGIN
  require_init();
  if (level < 0 || level > 1) fail(GrB_INVALID_VALUE, "fusion level must be 0 or 1");
  force_all();
  ctx().fusion = level;
  API_END
}

GrB_Info GrM_code_cache_clear(void) {
  API_BEGIN
  require_init();
  hip_check(hipStreamSynchronize(ctx().stream), "sync");
  jit_clear();
  API_END
}

GrB_Info GrM_reset_stats(void) {
  API_BEGIN
  require_init();
  ctx().stats = Stats{};
  API_END
}

// ------------------------------------------------------------ scalars

GrB_Info GrB_Scalar_new(GrB_Scalar* s, GrB_Type type) {
  API_BEGIN
  require_init();
  need(s, "scalar");
  need(type, "type");
  auto* o = new GB_Scalar_opaque{MAGIC_SCA, type->code, nullptr};
  NodeP p = new_node(N_SCALAR, T_FP64, 0, true);
  p->done = true;
  p->has_value = false;
  set_sca(o, p);
  *s = o;
  API_END
}

GrB_Info GrB_Scalar_free(GrB_Scalar* s) {
  API_BEGIN
  if (!s || !*s) return GrB_SUCCESS;
  GB_Scalar_opaque* o = sca(*s, "scalar");
  set_sca(o, nullptr);
  o->magic = MAGIC_FREED;
  delete o;
  *s = nullptr;
  API_END
}

GrB_Info GrB_Scalar_setElement_FP64(GrB_Scalar s, double x) {
  API_BEGIN
  require_init();
  GB_Scalar_opaque* o = sca(s, "scalar");
  NodeP p = new_node(N_SCALAR, T_FP64, 0, true);
  p->buf = dev_alloc(sizeof(double));
  hip_check(launch_set_scalar((double*)p->buf->p, x, ctx().stream), "set scalar");
  launch_mark(false);
  p->done = true;
  set_sca(o, p);
  API_END
}

GrB_Info GrB_Scalar_extractElement_FP64(double* x, GrB_Scalar s) {
  API_BEGIN
  require_init();
  need(x, "x");
  GB_Scalar_opaque* o = sca(s, "scalar");
  materialize(o->node);
  if (!o->node->has_value) return GrB_NO_VALUE;
  double h = 0.0;
  hip_check(hipMemcpyAsync(&h, o->node->buf->p, sizeof(double), hipMemcpyDeviceToHost, ctx().stream),
            "copy scalar");
  hip_check(hipStreamSynchronize(ctx().stream), "sync");
  *x = h;
  API_END
}

GrB_Info GrB_Scalar_wait(GrB_Scalar s, GrB_WaitMode mode) {
  API_BEGIN
  require_init();
  GB_Scalar_opaque* o = sca(s, "scalar");
  if (mode != GrB_COMPLETE && mode != GrB_MATERIALIZE) fail(GrB_INVALID_VALUE, "wait mode");
  materialize(o->node);
  API_END
}

GrB_Info GrM_Scalar_affine(GrB_Scalar out, double alpha, GrB_Scalar in, double beta) {
  API_BEGIN
  require_init();
  GB_Scalar_opaque* o = sca(out, "out");
  GB_Scalar_opaque* i = sca(in, "in");
  rec_affine(o, alpha, i, beta);
  API_END
}

// ------------------------------------------------------------ vectors

GrB_Info GrB_Vector_new(GrB_Vector* v, GrB_Type type, GrB_Index n) {
  API_BEGIN
  require_init();
  need(v, "vector");
  need(type, "type");
  if (n < 1 || n > (GrB_Index)INT32_MAX) fail(GrB_INVALID_VALUE, "vector length must be in [1, 2^31)");
  if (type->code == T_BOOL || type->code == T_BF16)
    fail(GrB_NOT_IMPLEMENTED, "BOOL and BF16 vectors are not supported");
  auto* o = new GB_Vector_opaque{MAGIC_VEC, type->code, (int64_t)n, nullptr};
  set_vec(o, iso_node(type->code, (int64_t)n, 0.0));
  *v = o;
  API_END
}

GrB_Info GrB_Vector_free(GrB_Vector* v) {
  API_BEGIN
  if (!v || !*v) return GrB_SUCCESS;
  GB_Vector_opaque* o = vec(*v, "vector");
  set_vec(o, nullptr);
  o->magic = MAGIC_FREED;
  delete o;
  *v = nullptr;
  API_END
}

GrB_Info GrB_Vector_dup(GrB_Vector* w, GrB_Vector u) {
  API_BEGIN
  require_init();
  need(w, "w");
  GB_Vector_opaque* uo = vec(u, "u");
  auto* o = new GB_Vector_opaque{MAGIC_VEC, uo->type, uo->n, nullptr};
  set_vec(o, uo->node);
  *w = o;
  API_END
}

GrB_Info GrB_Vector_size(GrB_Index* n, GrB_Vector v) {
  API_BEGIN
  need(n, "n");
  *n = (GrB_Index)vec(v, "vector")->n;
  API_END
}

GrB_Info GrM_Vector_type(GrB_Type* t, GrB_Vector v) {
  API_BEGIN
  need(t, "t");
  switch (vec(v, "vector")->type) {
    case T_INT32: *t = GrB_INT32; break;
    case T_FP32: *t = GrB_FP32; break;
    case T_FP64: *t = GrB_FP64; break;
    default: *t = GrB_BOOL; break;
  }
  API_END
}

GrB_Info GrB_Vector_wait(GrB_Vector v, GrB_WaitMode mode) {
  API_BEGIN
  require_init();
  GB_Vector_opaque* o = vec(v, "vector");
  if (mode != GrB_COMPLETE && mode != GrB_MATERIALIZE) fail(GrB_INVALID_VALUE, "wait mode");
  materialize(o->node);
  API_END
}

GrB_Info GrM_Vector_fill(GrB_Vector v, double value) {
  API_BEGIN
  require_init();
  GB_Vector_opaque* o = vec(v, "vector");
  set_vec(o, iso_node(o->type, o->n, value));
  API_END
}

GrB_Info GrM_Vector_import_dense(GrB_Vector v, const void* src, GrB_Index n) {
  API_BEGIN
  require_init();
  GB_Vector_opaque* o = vec(v, "vector");
  need(src, "src");
  if ((int64_t)n != o->n) fail(GrB_DIMENSION_MISMATCH, "length differs from the vector's");
  NodeP p = new_node(N_DENSE, o->type, o->n, false);
  p->buf = dev_alloc(type_size(o->type) * (size_t)o->n);
  hip_check(hipMemcpyAsync(p->buf->p, src, type_size(o->type) * (size_t)o->n,
                           hipMemcpyDeviceToDevice, ctx().stream),
            "import");
  p->done = true;
  set_vec(o, p);
  API_END
}

GrB_Info GrM_Vector_export_dense(void* dst, GrB_Index n, GrB_Vector v) {
  API_BEGIN
  require_init();
  GB_Vector_opaque* o = vec(v, "vector");
  need(dst, "dst");
  if ((int64_t)n != o->n) fail(GrB_DIMENSION_MISMATCH, "length differs from the vector's");
  materialize(o->node);
  const NodeP& p = o->node;
  require_full(p, "the dense export");
  if (p->iso) {
    hip_check(launch_fill(dst, o->type, o->n, p->iso_val, ctx().stream), "export fill");
    launch_mark(false);
  } else {
    hip_check(hipMemcpyAsync(dst, p->buf->p, type_size(o->type) * (size_t)o->n,
                             hipMemcpyDeviceToDevice, ctx().stream),
              "export");
  }
  API_END
}

GrB_Info GrM_Vector_device_pointer(const void** ptr, GrB_Vector v) {
  API_BEGIN
  require_init();
  need(ptr, "ptr");
  GB_Vector_opaque* o = vec(v, "vector");
  materialize(o->node);
  require_full(o->node, "a device pointer");
  store_if_iso(o->node);
  *ptr = o->node->buf->p;
  API_END
}

// ------------------------------------------------------------ matrices

GrB_Info GrB_Matrix_new(GrB_Matrix* A, GrB_Type type, GrB_Index nrows, GrB_Index ncols) {
  API_BEGIN
  require_init();
  need(A, "matrix");
  need(type, "type");
  if (nrows < 1 || ncols < 1 || nrows > (GrB_Index)INT32_MAX - 1 || ncols > (GrB_Index)INT32_MAX - 1)
    fail(GrB_INVALID_VALUE, "dimensions must be in [1, 2^31-1)");
  auto* o = new GB_Matrix_opaque{MAGIC_MAT, type->code, (int64_t)nrows, (int64_t)ncols, nullptr};
  o->data = new_matdata((int64_t)nrows, (int64_t)ncols);
  *A = o;
  API_END
}

GrB_Info GrB_Matrix_free(GrB_Matrix* A) {
  API_BEGIN
  if (!A || !*A) return GrB_SUCCESS;
  GB_Matrix_opaque* o = mat_any(*A, "matrix");
  o->data.reset();
  o->magic = MAGIC_FREED;
  delete o;
  *A = nullptr;
  API_END
}

GrB_Info GrB_Matrix_nrows(GrB_Index* n, GrB_Matrix A) {
  API_BEGIN
  need(n, "n");
  *n = (GrB_Index)mat_any(A, "A")->nrows;
  API_END
}

GrB_Info GrB_Matrix_ncols(GrB_Index* n, GrB_Matrix A) {
  API_BEGIN
  need(n, "n");
  *n = (GrB_Index)mat_any(A, "A")->ncols;
  API_END
}

GrB_Info GrB_Matrix_nvals(GrB_Index* nvals, GrB_Matrix A) {
  API_BEGIN
  need(nvals, "nvals");
  GB_Matrix_opaque* o = mat_any(A, "A");
  *nvals = o->data->dense ? (GrB_Index)(o->nrows * o->ncols) : (GrB_Index)o->data->nnz;
  API_END
}

GrB_Info GrM_Matrix_import_dense(GrB_Matrix A, const void* src, GrB_Index nrows, GrB_Index ncols) {
  API_BEGIN
  require_init();
  GB_Matrix_opaque* o = mat_any(A, "A");
  need(src, "src");
  float_type(o->type, "A");
  if ((int64_t)nrows != o->nrows || (int64_t)ncols != o->ncols)
    fail(GrB_DIMENSION_MISMATCH, "dense import must fill the whole matrix (nrows x ncols of GrB_Matrix_new)");
  Ctx& c = ctx();
  auto m = std::make_shared<MatData>();
  m->id = c.next_id++;
  m->nrows = o->nrows;
  m->ncols = o->ncols;
  m->nnz = 0;
  m->dense_type = o->type;
  const size_t bytes = type_size(o->type) * (size_t)o->nrows * (size_t)o->ncols;
  m->dense = dev_alloc(bytes);
  hip_check(hipMemcpyAsync(m->dense->p, src, bytes, hipMemcpyDeviceToDevice, c.stream), "import dense");
  o->data = m;
  API_END
}

GrB_Info GrM_Matrix_export_dense(void* dst, GrB_Matrix A) {
  API_BEGIN
  require_init();
  GB_Matrix_opaque* o = mat_any(A, "A");
  need(dst, "dst");
  if (!o->data->dense) fail(GrB_INVALID_VALUE, "A holds a pattern, not dense values");
  const size_t bytes = type_size(o->data->dense_type) * (size_t)o->nrows * (size_t)o->ncols;
  hip_check(hipMemcpyAsync(dst, o->data->dense->p, bytes, hipMemcpyDeviceToDevice, ctx().stream), "export dense");
  API_END
}

GrB_Info GrB_Matrix_wait(GrB_Matrix A, GrB_WaitMode mode) {
  API_BEGIN
  require_init();
  mat_any(A, "A");
  if (mode != GrB_COMPLETE && mode != GrB_MATERIALIZE) fail(GrB_INVALID_VALUE, "wait mode");
  API_END
}

GrB_Info GrM_Matrix_import_CSR(GrB_Matrix A, const int32_t* rowptr, const int32_t* col, GrB_Index nnz) {
  API_BEGIN
  require_init();
  GB_Matrix_opaque* o = mat_any(A, "A");
  need(rowptr, "rowptr");
  if (nnz > 0) need(col, "col");
  if (nnz > (GrB_Index)INT32_MAX) fail(GrB_INVALID_VALUE, "nnz must be < 2^31");
  Ctx& c = ctx();
  auto m = std::make_shared<MatData>();
  m->id = c.next_id++;
  m->nrows = o->nrows;
  m->ncols = o->ncols;
  m->nnz = (int64_t)nnz;
  m->rowptr = dev_alloc(sizeof(int) * (size_t)(o->nrows + 1));
  hip_check(hipMemcpyAsync(m->rowptr->p, rowptr, sizeof(int) * (size_t)(o->nrows + 1),
                           hipMemcpyDeviceToDevice, c.stream),
            "import rowptr");
  if (nnz > 0) {
    m->col = dev_alloc(sizeof(int) * (size_t)nnz);
    hip_check(hipMemcpyAsync(m->col->p, col, sizeof(int) * (size_t)nnz, hipMemcpyDeviceToDevice, c.stream),
              "import col");
  }
  BufP flag = dev_alloc(sizeof(int));
  hip_check(launch_fill(flag->p, T_INT32, 1, 0.0, c.stream), "fill");
  hip_check(launch_check_csr((const int*)m->rowptr->p, m->nrows, m->col ? (const int*)m->col->p : nullptr,
                             m->nnz, m->ncols, (int*)flag->p, c.stream),
            "check csr");
  launch_mark(false);
  launch_mark(false);
  if (read_flag(flag) != 0) fail(GrB_INVALID_VALUE, "malformed CSR pattern");
  o->data = m;
  API_END
}

GrB_Info GrM_Matrix_export_CSR(int32_t* rowptr, int32_t* col, GrB_Matrix A) {
  API_BEGIN
  require_init();
  GB_Matrix_opaque* o = mat(A, "A");
  need(rowptr, "rowptr");
  const MatP& m = o->data;
  if (m->nnz > 0) need(col, "col");
  Ctx& c = ctx();
  hip_check(hipMemcpyAsync(rowptr, m->rowptr->p, sizeof(int) * (size_t)(m->nrows + 1),
                           hipMemcpyDeviceToDevice, c.stream),
            "export rowptr");
  if (m->nnz > 0)
    hip_check(hipMemcpyAsync(col, m->col->p, sizeof(int) * (size_t)m->nnz, hipMemcpyDeviceToDevice, c.stream),
              "export col");
  API_END
}

GrB_Info GrM_Matrix_build_edges(GrB_Matrix A, const uint32_t* src, const uint32_t* dst, GrB_Index nedges,
                                bool drop_self) {
  API_BEGIN
  require_init();
  GB_Matrix_opaque* o = mat_any(A, "A");
  if (o->nrows != o->ncols) fail(GrB_DIMENSION_MISMATCH, "edge lists build square matrices");
  if (nedges > 0) {
    need(src, "src");
    need(dst, "dst");
  }
  if (nedges > (GrB_Index)INT32_MAX) fail(GrB_INVALID_VALUE, "at most 2^31-1 edges");
  Ctx& c = ctx();
  const int64_t n = o->nrows;
  auto m = std::make_shared<MatData>();
  m->id = c.next_id++;
  m->nrows = n;
  m->ncols = n;
  m->rowptr = dev_alloc(sizeof(int) * (size_t)(n + 1));
  BufP colbuf = nedges > 0 ? dev_alloc(sizeof(int) * (size_t)nedges) : nullptr;
  BufP flag = dev_alloc(sizeof(int));
  hip_check(launch_fill(flag->p, T_INT32, 1, 0.0, c.stream), "fill");
  int64_t nnz = 0;
  hip_check(build_csr_from_edges(n, src, dst, (int64_t)nedges, drop_self, (int*)m->rowptr->p,
                                 colbuf ? (int*)colbuf->p : nullptr, &nnz, (int*)flag->p, cache_alloc,
                                 cache_release, nullptr, c.stream),
            "build CSR");
  launch_mark(false);
  if (read_flag(flag) != 0) fail(GrB_INDEX_OUT_OF_BOUNDS, "edge endpoint >= n");
  m->nnz = nnz;
  if (nnz > 0) {
    // shrink the column array to nnz
    m->col = dev_alloc(sizeof(int) * (size_t)nnz);
    hip_check(hipMemcpyAsync(m->col->p, colbuf->p, sizeof(int) * (size_t)nnz, hipMemcpyDeviceToDevice,
                             c.stream),
              "copy col");
  }
  o->data = m;
  API_END
}

GrB_Info GrB_transpose(GrB_Matrix C, GrB_Matrix Mask, GrB_BinaryOp accum, GrB_Matrix A, GrB_Descriptor desc) {
  API_BEGIN
  require_init();
  (void)desc;
  GB_Matrix_opaque* co = mat(C, "C");
  GB_Matrix_opaque* ao = mat(A, "A");
  no_mask_accum(Mask, accum);
  if (co->nrows != ao->ncols || co->ncols != ao->nrows) fail(GrB_DIMENSION_MISMATCH, "C must be ncols(A) x nrows(A)");
  Ctx& c = ctx();
  const MatP& a = ao->data;
  auto m = std::make_shared<MatData>();
  m->id = c.next_id++;
  m->nrows = a->ncols;
  m->ncols = a->nrows;
  m->nnz = a->nnz;
  m->rowptr = dev_alloc(sizeof(int) * (size_t)(m->nrows + 1));
  if (a->nnz > 0) m->col = dev_alloc(sizeof(int) * (size_t)a->nnz);
  hip_check(transpose_csr(a->nrows, a->ncols, (const int*)a->rowptr->p, a->col ? (const int*)a->col->p : nullptr,
                          a->nnz, (int*)m->rowptr->p, m->col ? (int*)m->col->p : nullptr, cache_alloc,
                          cache_release, nullptr, c.stream),
            "transpose");
  launch_mark(false);
  co->data = m;
  API_END
}

GrB_Info GrM_Matrix_row_degree(GrB_Vector deg, GrB_Matrix A) {
  API_BEGIN
  require_init();
  GB_Vector_opaque* d = vec(deg, "deg");
  GB_Matrix_opaque* a = mat(A, "A");
  if (d->n != a->nrows) fail(GrB_DIMENSION_MISMATCH, "deg must have nrows(A) entries");
  NodeP p = new_node(N_DENSE, d->type, d->n, false);
  p->buf = dev_alloc(type_size(d->type) * (size_t)d->n);
  hip_check(launch_row_degree((const int*)a->data->rowptr->p, a->nrows, p->buf->p, d->type, ctx().stream),
            "row degree");
  launch_mark(false);
  p->done = true;
  set_vec(d, p);
  API_END
}

GrB_Info GrM_rmat_edges(uint32_t* src, uint32_t* dst, int scale, GrB_Index nedges, uint64_t seed, double ta,
                        double tab, double tabc) {
  API_BEGIN
  require_init();
  if (scale < 1 || scale > 31) fail(GrB_INVALID_VALUE, "scale must be in [1, 31]");
  if (nedges > 0) {
    need(src, "src");
    need(dst, "dst");
  }
  hip_check(launch_rmat(src, dst, scale, (int64_t)nedges, seed, ta, tab, tabc, ctx().stream), "rmat");
  launch_mark(false);
  API_END
}

// ------------------------------------------------------------ operations

GrB_Info GrB_mxv(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_Semiring op, GrB_Matrix A, GrB_Vector u,
                 GrB_Descriptor desc) {
  API_BEGIN
  require_init();
  (void)desc;
  GB_Vector_opaque* wo = vec(w, "w");
  GB_Vector_opaque* uo = vec(u, "u");
  GB_Matrix_opaque* ao = mat(A, "A");
  need(op, "semiring");
  if (accum) fail(GrB_NOT_IMPLEMENTED, "accumulators are not supported");
  GB_Vector_opaque* mo = mask ? vec(mask, "mask") : nullptr;
  if (mo && mo->n != wo->n) fail(GrB_DIMENSION_MISMATCH, "mask length");
  if (ao->ncols != uo->n || ao->nrows != wo->n) fail(GrB_DIMENSION_MISMATCH, "mxv dimensions");
  if (op->add != B_PLUS || (op->mul != B_TIMES && op->mul != B_SECOND))
    fail(GrB_NOT_IMPLEMENTED, "only plus-times / plus-second semirings");
  if (op->type != wo->type || op->type != uo->type) fail(GrB_DOMAIN_MISMATCH, "mxv types");
  rec_mxv(wo, ao, uo, mo, desc);
  API_END
}

static GrB_Info ewise_common(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_BinaryOp op, GrB_Vector u,
                             GrB_Vector v, bool set_union) {
  API_BEGIN
  require_init();
  GB_Vector_opaque* wo = vec(w, "w");
  GB_Vector_opaque* uo = vec(u, "u");
  GB_Vector_opaque* vo = vec(v, "v");
  need(op, "op");
  no_mask_accum(mask, accum);
  if (uo->n != wo->n || vo->n != wo->n) fail(GrB_DIMENSION_MISMATCH, "vector lengths differ");
  float_type(op->type, "operator");
  if (op->type != wo->type || op->type != uo->type || op->type != vo->type)
    fail(GrB_DOMAIN_MISMATCH, "operand types differ from the operator's");
  rec_ewise(wo, op->op, uo, vo, set_union);
  API_END
}

GrB_Info GrB_Vector_eWiseMult_BinaryOp(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_BinaryOp op,
                                       GrB_Vector u, GrB_Vector v, GrB_Descriptor desc) {
  (void)desc;
  return ewise_common(w, mask, accum, op, u, v, false);
}

GrB_Info GrB_Vector_eWiseAdd_BinaryOp(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_BinaryOp op,
                                      GrB_Vector u, GrB_Vector v, GrB_Descriptor desc) {
  (void)desc;
  return ewise_common(w, mask, accum, op, u, v, true);
}

GrB_Info GrB_Vector_apply(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_UnaryOp op, GrB_Vector u,
                          GrB_Descriptor desc) {
  API_BEGIN
  require_init();
  (void)desc;
  GB_Vector_opaque* wo = vec(w, "w");
  GB_Vector_opaque* uo = vec(u, "u");
  need(op, "op");
  no_mask_accum(mask, accum);
  if (uo->n != wo->n) fail(GrB_DIMENSION_MISMATCH, "vector lengths differ");
  if (op->type != wo->type) fail(GrB_DOMAIN_MISMATCH, "output type differs from the operator's");
  rec_unop(wo, op->op, uo);
  API_END
}

static GrB_Info bind_common(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_BinaryOp op, GrB_Vector u,
                            double s, bool first) {
  API_BEGIN
  require_init();
  GB_Vector_opaque* wo = vec(w, "w");
  GB_Vector_opaque* uo = vec(u, "u");
  need(op, "op");
  no_mask_accum(mask, accum);
  if (uo->n != wo->n) fail(GrB_DIMENSION_MISMATCH, "vector lengths differ");
  float_type(op->type, "operator");
  if (op->type != wo->type || op->type != uo->type) fail(GrB_DOMAIN_MISMATCH, "operand types");
  rec_bind(wo, op->op, uo, s, first);
  API_END
}

GrB_Info GrB_Vector_apply_BinaryOp1st_FP64(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_BinaryOp op,
                                           double s, GrB_Vector u, GrB_Descriptor desc) {
  (void)desc;
  return bind_common(w, mask, accum, op, u, s, true);
}

GrB_Info GrB_Vector_apply_BinaryOp2nd_FP64(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_BinaryOp op,
                                           GrB_Vector u, double s, GrB_Descriptor desc) {
  (void)desc;
  return bind_common(w, mask, accum, op, u, s, false);
}

GrB_Info GrB_Vector_apply_BinaryOp2nd_Scalar(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_BinaryOp op,
                                             GrB_Vector u, GrB_Scalar s, GrB_Descriptor desc) {
  API_BEGIN
  require_init();
  (void)desc;
  GB_Vector_opaque* wo = vec(w, "w");
  GB_Vector_opaque* uo = vec(u, "u");
  GB_Scalar_opaque* so = sca(s, "s");
  need(op, "op");
  no_mask_accum(mask, accum);
  if (uo->n != wo->n) fail(GrB_DIMENSION_MISMATCH, "vector lengths differ");
  float_type(op->type, "operator");
  if (op->type != wo->type || op->type != uo->type) fail(GrB_DOMAIN_MISMATCH, "operand types");
  if (so->node->done && !so->node->has_value) fail(GrB_EMPTY_OBJECT, "scalar has no value");
  rec_bind_scalar(wo, op->op, uo, so);
  API_END
}

GrB_Info GrB_Vector_reduce_Monoid_Scalar(GrB_Scalar s, GrB_BinaryOp accum, GrB_Monoid monoid, GrB_Vector u,
                                         GrB_Descriptor desc) {
  API_BEGIN
  require_init();
  (void)desc;
  GB_Scalar_opaque* so = sca(s, "s");
  GB_Vector_opaque* uo = vec(u, "u");
  need(monoid, "monoid");
  if (accum) fail(GrB_NOT_IMPLEMENTED, "accumulators are not supported");
  if (monoid->op != B_PLUS) fail(GrB_NOT_IMPLEMENTED, "only the plus monoid");
  float_type(uo->type, "u");
  rec_reduce(so, uo, nullptr, false, false);
  API_END
}

GrB_Info GrB_Vector_reduce_FP64(double* s, GrB_BinaryOp accum, GrB_Monoid monoid, GrB_Vector u,
                                GrB_Descriptor desc) {
  API_BEGIN
  require_init();
  (void)desc;
  need(s, "s");
  GB_Vector_opaque* uo = vec(u, "u");
  need(monoid, "monoid");
  if (accum) fail(GrB_NOT_IMPLEMENTED, "accumulators are not supported");
  if (monoid->op != B_PLUS) fail(GrB_NOT_IMPLEMENTED, "only the plus monoid");
  float_type(uo->type, "u");
  GB_Scalar_opaque tmp{MAGIC_SCA, T_FP64, nullptr};
  rec_reduce(&tmp, uo, nullptr, false, false);
  NodeP node = tmp.node;
  materialize(node);
  double h = 0.0;
  hip_check(hipMemcpyAsync(&h, node->buf->p, sizeof(double), hipMemcpyDeviceToHost, ctx().stream), "copy");
  hip_check(hipStreamSynchronize(ctx().stream), "sync");
  set_sca(&tmp, nullptr);
  *s = h;
  API_END
}

GrB_Info GrM_Vector_reduce_masked_Scalar(GrB_Scalar s, GrB_Vector mask, GrB_Monoid monoid, GrB_Vector u,
                                         GrB_Descriptor desc) {
  API_BEGIN
  require_init();
  GB_Scalar_opaque* so = sca(s, "s");
  GB_Vector_opaque* uo = vec(u, "u");
  GB_Vector_opaque* mo = vec(mask, "mask");
  need(monoid, "monoid");
  if (monoid->op != B_PLUS) fail(GrB_NOT_IMPLEMENTED, "only the plus monoid");
  if (mo->n != uo->n) fail(GrB_DIMENSION_MISMATCH, "mask length");
  float_type(uo->type, "u");
  rec_reduce(so, uo, mo, desc_comp(desc), false);
  API_END
}

// ------------------------------------------------------------ plans

static bool plan_geometry_ok(const GrM_PlanConfig& c, int type) {
  if (c.kernel != K_BLOCK && c.kernel != K_WAVE && !is_stripe(c.kernel)) return false;
  if (c.hot < 0 || (c.relabel != 0 && c.relabel != 1) || (c.xcd_split != 0 && c.xcd_split != 1)) return false;
  if (is_stripe(c.kernel))  // fixed geometry; FP32 ranks only
    return type == T_FP32 && c.long_row >= 0 && c.grid >= 0 && c.grid <= (1 << 20);
  const bool lds_ok = c.kernel == K_WAVE
                          ? (c.lds_entries == WAVE_TILE_ENTRIES && c.lds_rows == WAVE_TILE_ROWS)
                          : ((c.lds_entries == 1024 && c.lds_rows == 512) ||
                             (c.lds_entries == 2048 && c.lds_rows == 1024) ||
                             (c.lds_entries == 4096 && c.lds_rows == 1024));
  return lds_ok && c.long_row >= 1 && c.long_row <= c.chunk && c.chunk <= c.lds_entries &&
         c.grid >= 0 && c.grid <= (1 << 20);
}

GrB_Info GrM_Matrix_plan_set(GrB_Matrix A, GrB_Type type, const GrM_PlanConfig* cfg) {
  API_BEGIN
  require_init();
  GB_Matrix_opaque* ao = mat(A, "A");
  need(type, "type");
  float_type(type->code, "type");
  auto key = std::make_pair(ao->data->id, type->code);
  if (!cfg) {
    ctx().tuned.erase(key);
  } else {
    if (!plan_geometry_ok(*cfg, type->code)) fail(GrB_INVALID_VALUE, "unsupported tile plan geometry");
    PlanConfig pc;
    pc.kernel = cfg->kernel;
    pc.hot = cfg->hot;
    pc.relabel = cfg->relabel;
    pc.xcd = cfg->xcd_split;
    pc.lds_entries = cfg->lds_entries;
    pc.lds_rows = cfg->lds_rows;
    pc.long_row = cfg->long_row;
    pc.chunk = cfg->chunk;
    pc.grid = cfg->grid;
    ctx().tuned[key] = pc;
  }
  API_END
}

GrB_Info GrM_Matrix_plan_get(GrM_PlanConfig* cfg, GrB_Matrix A, GrB_Type type) {
  API_BEGIN
  require_init();
  need(cfg, "cfg");
  GB_Matrix_opaque* ao = mat(A, "A");
  need(type, "type");
  float_type(type->code, "type");
  PlanConfig pc = default_plan_config(ao->data, type->code);
  cfg->kernel = pc.kernel;
  cfg->hot = pc.hot;
  cfg->relabel = pc.relabel;
  cfg->xcd_split = pc.xcd;
  cfg->lds_entries = pc.lds_entries;
  cfg->lds_rows = pc.lds_rows;
  cfg->long_row = pc.long_row;
  cfg->chunk = pc.chunk;
  cfg->grid = pc.grid;
  API_END
}

// ------------------------------------------------------------ probe / timing

GrB_Info GrM_stream_copy(void* dst, const void* src, size_t bytes) {
  API_BEGIN
  require_init();
  need(dst, "dst");
  need(src, "src");
  hip_check(launch_stream_copy(dst, src, bytes, ctx().stream), "stream copy");
  launch_mark(false);
  API_END
}

GrB_Info GrM_timing_enable(bool on) {
  API_BEGIN
  require_init();
  ctx().timing = on;
  API_END
}

GrB_Info GrM_timing_read(double* total_ms, int64_t* launches) {
  API_BEGIN
  require_init();
  need(total_ms, "total_ms");
  need(launches, "launches");
  Ctx& c = ctx();
  hip_check(hipStreamSynchronize(c.stream), "sync");
  double tot = 0.0;
  for (auto& e : c.events) {
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, e.first, e.second), "elapsed");
    tot += ms;
    c.event_pool.push_back(e.first);
    c.event_pool.push_back(e.second);
  }
  *launches = (int64_t)c.events.size();
  c.events.clear();
  *total_ms = tot;
  API_END
}

}  // extern "C"
