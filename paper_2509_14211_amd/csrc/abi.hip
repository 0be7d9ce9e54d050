// C ABI entry points (declared in include/nbgrb.h).  Each call validates
// its arguments eagerly, then records (nonblocking) or runs (blocking) the
// operation through the runtime.  Internal errors are C++ exceptions that
// are turned into GrB_Info codes here.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "runtime.h"

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

static GB_Descriptor_opaque d_comp{true};
GrB_Descriptor GrB_DESC_C = &d_comp;

// ------------------------------------------------------------ errors

static thread_local std::string g_err;

void nbgrb::set_error_text(const std::string& msg) { g_err = msg; }

#define API_BEGIN \
  try {           \
    g_err.clear();
#define API_END                                      \
  }                                                  \
  catch (const GrbError& e) {                        \
    g_err = e.msg;                                   \
    return e.info;                                   \
  }                                                  \
  catch (const std::bad_alloc&) {                    \
    g_err = "host allocation failed";                \
    return GrB_OUT_OF_MEMORY;                        \
  }                                                  \
  catch (const std::exception& e) {                  \
    g_err = e.what();                                \
    return GrB_PANIC;                                \
  }                                                  \
  return GrB_SUCCESS;

static void need(const void* p, const char* what) {
  if (!p) fail(GrB_NULL_POINTER, std::string(what) + " is NULL");
}

static GB_Vector_opaque* vec(GrB_Vector v, const char* what) {
  need(v, what);
  if (v->magic != MAGIC_VEC) fail(GrB_UNINITIALIZED_OBJECT, std::string(what) + " is not a vector");
  return v;
}

static GB_Scalar_opaque* sca(GrB_Scalar s, const char* what) {
  need(s, what);
  if (s->magic != MAGIC_SCA) fail(GrB_UNINITIALIZED_OBJECT, std::string(what) + " is not a scalar");
  return s;
}

static GB_Matrix_opaque* mat(GrB_Matrix A, const char* what) {
  need(A, what);
  if (A->magic != MAGIC_MAT) fail(GrB_UNINITIALIZED_OBJECT, std::string(what) + " is not a matrix");
  return A;
}

static void no_mask_accum(const void* mask, const void* accum) {
  if (mask) fail(GrB_NOT_IMPLEMENTED, "masks are not supported by this operation");
  if (accum) fail(GrB_NOT_IMPLEMENTED, "accumulators are not supported");
}

static void float_type(int t, const char* what) {
  if (t != T_FP32 && t != T_FP64) fail(GrB_DOMAIN_MISMATCH, std::string(what) + " must be FP32 or FP64");
}

static bool desc_comp(GrB_Descriptor d) { return d && d->mask_comp; }

// ------------------------------------------------------------ recording

namespace {

NodeP iso_node(int type, int64_t n, double v) {
  NodeP p = new_node(N_DENSE, type, n, false);
  p->done = true;
  p->iso = true;
  p->iso_val = v;
  return p;
}

void rec_ewise(GB_Vector_opaque* w, int op, GB_Vector_opaque* u, GB_Vector_opaque* v) {
  NodeP p = new_node(N_EWISE, w->type, w->n, false);
  p->a = u->node;
  p->b = v->node;
  p->op = op;
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

void rec_mxv(GB_Vector_opaque* w, GB_Matrix_opaque* A, GB_Vector_opaque* u) {
  NodeP p = new_node(N_MXV, w->type, w->n, false);
  p->A = A->data;
  p->a = u->node;
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
  c.tuned.clear();
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

const char* GrM_error(void) { return g_err.c_str(); }

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
  GB_Matrix_opaque* o = mat(*A, "matrix");
  o->data.reset();
  o->magic = MAGIC_FREED;
  delete o;
  *A = nullptr;
  API_END
}

GrB_Info GrB_Matrix_nrows(GrB_Index* n, GrB_Matrix A) {
  API_BEGIN
  need(n, "n");
  *n = (GrB_Index)mat(A, "A")->nrows;
  API_END
}

GrB_Info GrB_Matrix_ncols(GrB_Index* n, GrB_Matrix A) {
  API_BEGIN
  need(n, "n");
  *n = (GrB_Index)mat(A, "A")->ncols;
  API_END
}

GrB_Info GrB_Matrix_nvals(GrB_Index* nvals, GrB_Matrix A) {
  API_BEGIN
  need(nvals, "nvals");
  *nvals = (GrB_Index)mat(A, "A")->data->nnz;
  API_END
}

GrB_Info GrB_Matrix_wait(GrB_Matrix A, GrB_WaitMode mode) {
  API_BEGIN
  require_init();
  mat(A, "A");
  if (mode != GrB_COMPLETE && mode != GrB_MATERIALIZE) fail(GrB_INVALID_VALUE, "wait mode");
  API_END
}

GrB_Info GrM_Matrix_import_CSR(GrB_Matrix A, const int32_t* rowptr, const int32_t* col, GrB_Index nnz) {
  API_BEGIN
  require_init();
  GB_Matrix_opaque* o = mat(A, "A");
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
  GB_Matrix_opaque* o = mat(A, "A");
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
  no_mask_accum(mask, accum);
  if (ao->ncols != uo->n || ao->nrows != wo->n) fail(GrB_DIMENSION_MISMATCH, "mxv dimensions");
  if (op->add != B_PLUS || (op->mul != B_TIMES && op->mul != B_SECOND))
    fail(GrB_NOT_IMPLEMENTED, "only plus-times / plus-second semirings");
  if (op->type != wo->type || op->type != uo->type) fail(GrB_DOMAIN_MISMATCH, "mxv types");
  rec_mxv(wo, ao, uo);
  API_END
}

static GrB_Info ewise_common(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_BinaryOp op, GrB_Vector u,
                             GrB_Vector v) {
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
  rec_ewise(wo, op->op, uo, vo);
  API_END
}

GrB_Info GrB_Vector_eWiseMult_BinaryOp(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_BinaryOp op,
                                       GrB_Vector u, GrB_Vector v, GrB_Descriptor desc) {
  (void)desc;
  return ewise_common(w, mask, accum, op, u, v);
}

GrB_Info GrB_Vector_eWiseAdd_BinaryOp(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, GrB_BinaryOp op,
                                      GrB_Vector u, GrB_Vector v, GrB_Descriptor desc) {
  (void)desc;
  return ewise_common(w, mask, accum, op, u, v);
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

// ------------------------------------------------------------ PageRank

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

  GB_Vector_opaque deg_exec{MAGIC_VEC, dego->type, n, nullptr};
  set_vec(&deg_exec, rl ? permuted(dego->node, rl->order) : dego->node);

  // d = damping ./ outdeg (0 where outdeg = 0)
  GB_Vector_opaque dinv{MAGIC_VEC, T, n, nullptr};
  rec_unop(&dinv, U_MINV_OR_ZERO, &deg_exec);
  rec_bind(&dinv, B_TIMES, &dinv, damping, true);
  set_vec(&deg_exec, nullptr);
  materialize(dinv.node);
  store_if_iso(dinv.node);

  // personalised teleport distribution (permuted like every vector)
  GB_Vector_opaque v{MAGIC_VEC, T, n, nullptr};
  if (vo) {
    set_vec(&v, rl ? permuted(vo->node, rl->order) : vo->node);
    materialize(v.node);
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
  store_if_iso(x.node);

  GB_Scalar_opaque D{MAGIC_SCA, T_FP64, nullptr};
  if (uniform) rec_reduce(&D, &x, &dinv, true, false);

  gbuf = dev_alloc(sizeof(GuardDev));
  hip_check(launch_guard_init((GuardDev*)gbuf->p, (1.0 > tol && itermax > 0) ? 1 : 0, tol, itermax, c.stream),
            "guard init");
  launch_mark(false);
  c.guard = (GuardDev*)gbuf->p;

  std::vector<NodeP> hist{x.node};
  int64_t base = 0;
  GuardDev hg{};
  int batch = check_every;
  for (;;) {
    for (int j = 0; j < batch; ++j) {
      GB_Vector_opaque w{MAGIC_VEC, T, n, nullptr}, s{MAGIC_VEC, T, n, nullptr};
      GB_Vector_opaque rn{MAGIC_VEC, T, n, nullptr}, t{MAGIC_VEC, T, n, nullptr};
      GB_Scalar_opaque cs{MAGIC_SCA, T_FP64, nullptr}, rho{MAGIC_SCA, T_FP64, nullptr};
      GB_Scalar_opaque Dn{MAGIC_SCA, T_FP64, nullptr};
      rec_ewise(&w, B_TIMES, &x, &dinv);            // w = x .* d
      rec_mxv(&s, &A_exec, &w);                     // s = AT (+.second) w
      GB_Vector_opaque vt{MAGIC_VEC, T, n, nullptr};
      if (vo) {                                     // r = s + v .* c
        if (uniform) {                              //   c = (1-d) + d D
          rec_affine(&cs, damping, &D, 1.0 - damping);
          rec_bind_scalar(&vt, B_TIMES, &v, &cs);
        } else {                                    //   c = 1-d
          rec_bind(&vt, B_TIMES, &v, 1.0 - damping, false);
        }
        rec_ewise(&rn, B_PLUS, &s, &vt);
        set_vec(&vt, nullptr);
      } else if (uniform) {                         // r = c + s, c = (1-d)/n + d D/n
        rec_affine(&cs, damping / (double)n, &D, tele);
        rec_bind_scalar(&rn, B_PLUS, &s, &cs);
      } else {
        rec_bind(&rn, B_PLUS, &s, tele, false);
      }
      rec_ewise(&t, B_ABSDIFF, &x, &rn);            // t = |x - r|
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
    hip_check(hipMemcpyAsync(&hg, c.guard, sizeof(GuardDev), hipMemcpyDeviceToHost, c.stream), "read guard");
    hip_check(hipStreamSynchronize(c.stream), "sync");
    if (!hg.active) break;
    base += (int64_t)hist.size() - 1;
    NodeP last = hist.back();
    hist.assign(1, last);
    // The residual contracts about geometrically: predict the passes still
    // needed from the last two residuals (at least 1, at most what itermax
    // allows); an underestimate only costs one more check.
    int next = check_every;
    if (hg.rho_prev > 0.0 && hg.rho > 0.0 && hg.rho < hg.rho_prev && tol > 0.0) {
      const double q = hg.rho / hg.rho_prev;
      const double need = std::log(tol / hg.rho) / std::log(q);
      if (need > 0.0 && need < 1e6) next = (int)std::ceil(need);
      if (next < 1) next = 1;
    }
    if (next > itermax - hg.iters) next = itermax - hg.iters;
    if (next < 1) next = 1;
    batch = next;
  }
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
    g_err = e.msg;
    return e.info;
  }
  catch (const std::exception& e) {
    c.guard = saved_guard;
    g_err = e.what();
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
    g_err = "teleport is NULL";
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
    grid = plan->cfg.grid;

    // d = damping ./ outdeg (0 for dangling), in execution order
    GB_Vector_opaque deg_exec{MAGIC_VEC, dego->type, n, nullptr};
    set_vec(&deg_exec, rl ? permuted(dego->node, rl->order) : dego->node);
    dinv.type = T;
    dinv.n = n;
    rec_unop(&dinv, U_MINV_OR_ZERO, &deg_exec);
    rec_bind(&dinv, B_TIMES, &dinv, damping, true);
    set_vec(&deg_exec, nullptr);
    materialize(dinv.node);
    store_if_iso(dinv.node);

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
  void start_columns(uint64_t cols, int cur, const std::vector<PprSeed>& seeds_by_col) {
    Ctx& c = ctx();
    hip_check(launch_spmm_zero_columns(Xb[cur]->p, Wb[cur]->p, T, n, k, cols, c.stream), "zero columns");
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
    hip_check(launch_spmm_ppr(plan->dev, a, T, grid, a.guard, c.stream), "ppr pass");
    launch_mark(true);
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
  pc.start_columns(k == 64 ? ~0ull : ((1ull << k) - 1ull), 0, seeds);
  hip_check(launch_guard_init((GuardDev*)pc.gbuf->p, (1.0 > tol && itermax > 0) ? 1 : 0, tol, itermax, c.stream),
            "guard init");
  launch_mark(false);
  c.guard = (GuardDev*)pc.gbuf->p;
  pc.a.guard = c.guard;

  GuardDev hg{};
  int pass = 0, batch = check_every;
  for (;;) {
    for (int j = 0; j < batch; ++j) pc.run_pass(++pass);
    hip_check(hipMemcpyAsync(&hg, c.guard, sizeof(GuardDev), hipMemcpyDeviceToHost, c.stream), "read guard");
    hip_check(hipStreamSynchronize(c.stream), "sync");
    if (!hg.active) break;
    int next = check_every;
    if (hg.rho_prev > 0.0 && hg.rho > 0.0 && hg.rho < hg.rho_prev && tol > 0.0) {
      const double need_passes = std::log(tol / hg.rho) / std::log(hg.rho / hg.rho_prev);
      if (need_passes > 0.0 && need_passes < 1e6) next = (int)std::ceil(need_passes);
    }
    if (next > itermax - hg.iters) next = itermax - hg.iters;
    if (next < 1) next = 1;
    batch = next;
  }
  c.guard = saved_guard;
  const BufP& res = pc.Xb[hg.iters & 1];
  if (pc.rl)
    hip_check(launch_rows_permute(res->p, T, (const int*)pc.rl->inv->p, X, n, k, c.stream), "unpermute");
  else
    hip_check(hipMemcpyAsync(X, res->p, pc.vbytes, hipMemcpyDeviceToDevice, c.stream), "copy out");
  std::vector<int> hh(64);
  std::vector<double> rr(64);
  hip_check(hipMemcpyAsync(hh.data(), pc.hit->p, sizeof(int) * 64, hipMemcpyDeviceToHost, c.stream), "copy");
  hip_check(hipMemcpyAsync(rr.data(), pc.rho->p, sizeof(double) * 64, hipMemcpyDeviceToHost, c.stream), "copy");
  hip_check(hipStreamSynchronize(c.stream), "sync");
  if (col_iters)
    for (int q = 0; q < k; ++q) col_iters[q] = hg.iters == 0 ? -1 : hh[q];
  if (col_resid)
    for (int q = 0; q < k; ++q) col_resid[q] = hg.iters == 0 ? 1.0 : rr[q];
  *iters = hg.iters;
  }
  catch (const GrbError& e) {
    c.guard = saved_guard;
    g_err = e.msg;
    return e.info;
  }
  catch (const std::exception& e) {
    c.guard = saved_guard;
    g_err = e.what();
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

  std::vector<int> slot_set(k, -1), slot_start(k, 0);
  std::vector<PprSeed> active;  // seeds of the columns in use
  int next_set = 0, pass = 0, live = 0;
  auto set_seeds_of = [&](int q, int col, std::vector<PprSeed>& out) {
    const double w = 1.0 / (double)(seed_ptr[q + 1] - seed_ptr[q]);
    for (int e = seed_ptr[q]; e < seed_ptr[q + 1]; ++e) out.push_back({pc.exec_vertex(seed_vtx[e]), col, w});
  };
  // fill the free slots with the next sets, starting them in buffer set `cur`
  auto refill = [&](int cur, uint64_t freed) {
    // drop the seeds of retired columns, then hand free columns the next sets
    active.erase(std::remove_if(active.begin(), active.end(), [&](const PprSeed& s) { return slot_set[s.c] < 0; }),
                 active.end());
    uint64_t cols = 0;
    std::vector<PprSeed> fresh;
    for (int col = 0; col < k && next_set < nsets; ++col) {
      if (slot_set[col] >= 0) continue;
      slot_set[col] = next_set;
      slot_start[col] = pass;
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
  while (live > 0) {
    // up to check_every passes, never past a column's itermax
    int batch = check_every;
    for (int col = 0; col < k; ++col)
      if (slot_set[col] >= 0) batch = std::min(batch, itermax - (pass - slot_start[col]));
    for (int j = 0; j < std::max(batch, 1); ++j) pc.run_pass(++pass);
    hip_check(hipMemcpyAsync(hh.data(), pc.hit->p, sizeof(int) * 64, hipMemcpyDeviceToHost, c.stream), "copy");
    hip_check(hipMemcpyAsync(rr.data(), pc.rho->p, sizeof(double) * 64, hipMemcpyDeviceToHost, c.stream), "copy");
    hip_check(hipStreamSynchronize(c.stream), "sync");
    const int cur = pass & 1;
    uint64_t retired = 0;
    ColumnOutputs outs{};
    for (int col = 0; col < k; ++col) {
      const int q = slot_set[col];
      if (q < 0) continue;
      const int done = pass - slot_start[col];
      const bool conv = hh[col] >= 0;
      if (!conv && done < itermax) continue;
      // retire: the column's current iterate goes to set q's output
      retired |= 1ull << col;
      outs.out[col] = (char*)X + type_size(T) * (size_t)n * (size_t)q;
      if (set_iters) set_iters[q] = conv ? hh[col] - slot_start[col] : -1;
      if (set_passes) set_passes[q] = done;
      if (set_resid) set_resid[q] = rr[col];
      slot_set[col] = -1;
      --live;
    }
    if (retired) {
      hip_check(launch_spmm_columns_out(pc.Xb[cur]->p, T, pc.rl ? (const int*)pc.rl->inv->p : nullptr, n, k, retired,
                                        outs, c.stream),
                "columns out");
      launch_mark(false);
      // freed columns stop contributing (zeroed) or restart with new sets
      refill(cur, retired);
    }
  }
  c.guard = saved_guard;
  hip_check(hipStreamSynchronize(c.stream), "sync");
  }
  catch (const GrbError& e) {
    c.guard = saved_guard;
    g_err = e.msg;
    return e.info;
  }
  catch (const std::exception& e) {
    c.guard = saved_guard;
    g_err = e.what();
    return GrB_PANIC;
  }
  return GrB_SUCCESS;
}

// ------------------------------------------------------------ many graphs

struct GB_Multigraph_opaque {
  uint32_t magic;
  int ngraphs;
  int64_t nv, ne;
  std::vector<int64_t> voff;
  BufP graphs, queue, qnext, rowptr, col, deg, inv, longrows, xa, xb, wa, wb, iters, resid;
  std::vector<std::shared_ptr<MatData>> keep;  // relabeled copies stay alive
  struct Exec {
    int type;
    double damping, tol;
    int itermax, uniform;
    void* out;
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
  m->queue = dev_alloc(sizeof(int) * order.size());
  m->longrows = dev_alloc(sizeof(int) * std::max<size_t>(longrows.size(), 1));
  if (!longrows.empty())
    hip_check(hipMemcpyAsync(m->longrows->p, longrows.data(), sizeof(int) * longrows.size(), hipMemcpyHostToDevice,
                             c.stream), "upload");
  hip_check(hipMemcpyAsync(m->graphs->p, gs.data(), sizeof(ManyGraph) * gs.size(), hipMemcpyHostToDevice, c.stream),
            "upload");
  hip_check(hipMemcpyAsync(m->queue->p, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice, c.stream),
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
    g_err = e.msg;
    return e.info;
  }
  catch (const std::exception& e) {
    g_err = e.what();
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
        e.out == X)
      ex = &e;
  if (!ex) {
    ManyArgs a{};
    a.graphs = (const ManyGraph*)mg->graphs->p;
    a.queue = (const int*)mg->queue->p;
    a.queue_next = (int*)mg->qnext->p;
    a.ngraphs = mg->ngraphs;
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
    GB_Multigraph_opaque::Exec e{T, damping, tol, itermax, uniform, X, nullptr, nullptr};
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
  if (iters || resid) hip_check(hipStreamSynchronize(c.stream), "sync");
  API_END
}

// ------------------------------------------------------------ plans

static bool plan_geometry_ok(const GrM_PlanConfig& c) {
  if (c.kernel != K_BLOCK && c.kernel != K_WAVE) return false;
  if (c.hot < 0 || (c.relabel != 0 && c.relabel != 1)) return false;
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
    if (!plan_geometry_ok(*cfg)) fail(GrB_INVALID_VALUE, "unsupported tile plan geometry");
    PlanConfig pc;
    pc.kernel = cfg->kernel;
    pc.hot = cfg->hot;
    pc.relabel = cfg->relabel;
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
