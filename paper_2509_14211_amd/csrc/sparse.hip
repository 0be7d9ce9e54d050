// Vectors with missing entries (Section III-A: sparse, bitset and full
// vectors) and the naive fill-ratio estimators that choose their storage
// and the loop driver of each operation (Section III-D).
//
// Every operation whose inputs may have missing entries, or whose output a
// mask restricts, runs here instead of on the dense kernels.  Its result is
// computed into a bitset (values plus one presence byte per entry, with a
// count of present entries) and then stored by the estimate made when the
// operation was recorded: full when every entry turned out present, sparse
// (sorted positions and their values) when the estimated fill is below
// 1/16, else bitset.  The estimates only choose storage and loop drivers;
// the result is the same whatever they say (up to the order of a sum).
//
// Loop drivers: eWiseMult runs over the entries of a sparse input when that
// input is the sparser one, else over the whole range; eWiseAdd runs over
// the entries of its inputs when both are sparse and the union is estimated
// sparse; mxv is driven by the entries of u (push: each present u(j) is
// added into the rows of column j, through the transposed pattern) when u
// is sparse with fill below 1/32, else by the rows of A (pull).
#include <hip/hip_runtime.h>
#include <rocprim/device/device_select.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "abi_util.h"
#include "device_util.h"
#include "kernels.h"
#include "ops_device.h"
#include "runtime.h"

namespace nbgrb {

namespace {

constexpr int SV_BLOCK = 256;
constexpr double SPARSE_BELOW = 1.0 / 16;  // estimated fill below which outputs are stored sparse
constexpr double PUSH_BELOW = 1.0 / 32;    // fill of a sparse u below which mxv is driven by u
constexpr int SV_LONG_ROW = 2048;          // pull mxv: longer rows get a workgroup of their own

int sv_grid(int64_t n) {
  int64_t g = (n + SV_BLOCK * 4 - 1) / (SV_BLOCK * 4);
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  return (int)g;
}

// ------------------------------------------------------------ device side

// Values (n entries, or an iso value) and presence (nullptr: all present).
struct VView {
  Operand val;
  const uint8_t* bits;
};

struct MaskView {
  VView v;
  int use, comp, structural;
};

__device__ __forceinline__ bool present(const VView& v, int64_t i) { return !v.bits || v.bits[i] != 0; }

__device__ __forceinline__ bool allowed(const MaskView& m, int64_t i) {
  if (!m.use) return true;
  const bool a = present(m.v, i) && (m.structural || nonzero_at(m.v.val, i));
  return a != (m.comp != 0);
}

// Counts are kept in COUNT_SLOTS counters, one per 128-byte line, and
// summed when read.
constexpr int COUNT_SLOTS = 64, COUNT_STRIDE = 16;

// Adds the counts of all threads of the block to its counter slot with one
// atomic per block (every thread of the block calls it, once, at the end of
// the kernel): counting per wavefront and loop step on one address
// serialised tens of thousands of atomics.
__device__ __forceinline__ void count_add(unsigned long long mine, unsigned long long* cnt) {
  __shared__ unsigned long long part[SV_BLOCK / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < SV_BLOCK / 64; ++w) t += part[w];
    if (t) atomicAdd(cnt + (blockIdx.x % COUNT_SLOTS) * COUNT_STRIDE, t);
  }
}

enum SvMode : int { SV_MULT = 0, SV_ADD = 1, SV_UNARY = 2, SV_BIND1 = 3, SV_BIND2 = 4, SV_COPY = 5 };

template <typename T>
__device__ __forceinline__ T sv_value(int mode, int op, T x, T y, T k) {
  switch (mode) {
    case SV_UNARY: return apply_unop<T>(op, x);
    case SV_BIND1: return apply_binop<T>(op, k, x);
    case SV_BIND2: return apply_binop<T>(op, x, k);
    case SV_COPY: return x;
    default: return apply_binop<T>(op, x, y);
  }
}

// Whole-range loop: out(i) from a(i), b(i) with the presence rule of the mode.
template <typename T>
__global__ void sv_range_kernel(int64_t n, int mode, int op, VView a, VView b, ScalarArg s, int out_type, void* out,
                                uint8_t* obits, unsigned long long* cnt) {
  unsigned long long mine = 0;
  const T k = (T)scalar_value(s);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i0 = base - threadIdx.x; i0 < n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    bool p = false;
    T v = (T)0;
    if (i < n) {
      const bool pa = present(a, i);
      const bool pb = (mode == SV_MULT || mode == SV_ADD) && present(b, i);
      if (mode == SV_MULT) {
        p = pa && pb;
        if (p) v = apply_binop<T>(op, load_as<T>(a.val, i), load_as<T>(b.val, i));
      } else if (mode == SV_ADD) {
        p = pa || pb;
        if (pa && pb) v = apply_binop<T>(op, load_as<T>(a.val, i), load_as<T>(b.val, i));
        else if (pa) v = load_as<T>(a.val, i);
        else if (pb) v = load_as<T>(b.val, i);
      } else {
        p = pa;
        if (p) v = sv_value<T>(mode, op, load_as<T>(a.val, i), (T)0, k);
      }
      store_as<T>(out, out_type, i, v);
      obits[i] = p ? 1 : 0;
    }
    mine += p ? 1ull : 0ull;
  }
  count_add(mine, cnt);
}

// Loop over the nnz entries (positions idx, values aval) of a sparse input:
//   SV_MULT     out(i) = op(a, b(i)) where b(i) is present (swap: op(b(i), a))
//   SV_ADD      second input of an index-driven union: out(i) = op(out(i), a)
//               (swap: op(a, out(i))) where out(i) is present, else a
//   apply modes out(i) = f(a)
// out / obits start zeroed (SV_ADD: holding the first input).
template <typename T>
__global__ void sv_index_kernel(int64_t nnz, const int* __restrict__ idx, Operand aval, int mode, int op, int swap,
                                VView b, ScalarArg s, int out_type, void* out, uint8_t* obits) {
  const T k = (T)scalar_value(s);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    const int64_t i = idx[e];
    const T x = load_as<T>(aval, e);
    if (mode == SV_MULT) {
      if (!present(b, i)) continue;
      const T y = load_as<T>(b.val, i);
      store_as<T>(out, out_type, i, swap ? apply_binop<T>(op, y, x) : apply_binop<T>(op, x, y));
      obits[i] = 1;
    } else if (mode == SV_ADD) {
      T v = x;
      if (obits[i]) {
        const Operand o{out, out_type, 0.0};
        const T y = load_as<T>(o, i);
        v = swap ? apply_binop<T>(op, x, y) : apply_binop<T>(op, y, x);
      }
      store_as<T>(out, out_type, i, v);
      obits[i] = 1;
    } else {
      store_as<T>(out, out_type, i, sv_value<T>(mode, op, x, (T)0, k));
      obits[i] = 1;
    }
  }
}

// Pull mxv: GROUP lanes per row, rows the mask forbids keep the old entry
// (keep_old) or none.  A full u makes every allowed row present.
template <typename T, int GROUP>
__global__ void sv_mxv_pull_kernel(int64_t nrows, const int* __restrict__ rowptr, const int* __restrict__ col,
                                   VView u, int u_full, MaskView m, VView old, int keep_old, T* out, uint8_t* obits,
                                   unsigned long long* cnt) {
  unsigned long long mine = 0;
  const int lane = threadIdx.x & (GROUP - 1);
  const int64_t groups = (int64_t)gridDim.x * (blockDim.x / GROUP);
  const int64_t g0 = (int64_t)blockIdx.x * (blockDim.x / GROUP) + threadIdx.x / GROUP;
  // every lane runs the same number of rounds so the wavefront-wide count
  // and shuffles see all lanes
  const int64_t rounds = (nrows + groups - 1) / groups;
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t i = g0 + r * groups;
    // rows longer than SV_LONG_ROW belong to sv_mxv_pull_long_kernel
    const bool row_ok = i < nrows && rowptr[i + 1] - rowptr[i] <= SV_LONG_ROW;
    const bool allow = row_ok && allowed(m, i);
    T s = (T)0;
    bool hit = false;
    if (allow) {
      const int e1 = rowptr[i + 1];
      for (int e = rowptr[i] + lane; e < e1; e += GROUP) {
        const int j = col[e];
        if (present(u, j)) {
          s += load_as<T>(u.val, j);
          hit = true;
        }
      }
    }
#pragma unroll
    for (int o = GROUP / 2; o > 0; o >>= 1) {
      s += __shfl_xor(s, o, 64);
      hit = __shfl_xor((int)hit, o, 64) != 0 || hit;
    }
    bool p = false;
    if (row_ok && lane == 0) {
      if (allow) {
        p = hit || u_full;
        out[i] = p ? s : (T)0;
      } else {
        p = keep_old && present(old, i);
        out[i] = p ? load_as<T>(old.val, i) : (T)0;
      }
      obits[i] = p ? 1 : 0;
    }
    mine += p ? 1ull : 0ull;
  }
  count_add(mine, cnt);
}

// Pull mxv of the rows longer than SV_LONG_ROW (list `rows`): one
// workgroup per row, four loads in flight per thread, the sum and the
// presence combined in a fixed order, the rest as in the pull kernel.
template <typename T>
__global__ __launch_bounds__(SV_BLOCK) void sv_mxv_pull_long_kernel(const int* __restrict__ rows,
                                                                    const int* __restrict__ rowptr,
                                                                    const int* __restrict__ col, VView u, int u_full,
                                                                    MaskView m, VView old, int keep_old, T* out,
                                                                    uint8_t* obits, unsigned long long* cnt) {
  __shared__ T ssum[SV_BLOCK / 64];
  __shared__ int shit[SV_BLOCK / 64];
  const int64_t i = rows[blockIdx.x];
  const bool allow = allowed(m, i);
  T s = (T)0;
  int hit = 0;
  if (allow) {
    const int e0 = rowptr[i], e1 = rowptr[i + 1];
    for (int e = e0 + (int)threadIdx.x; e < e1; e += 4 * SV_BLOCK) {
      int j[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) j[k] = col[min(e + k * SV_BLOCK, e1 - 1)];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (e + k * SV_BLOCK < e1 && present(u, j[k])) {
          s += load_as<T>(u.val, j[k]);
          hit = 1;
        }
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o, 64);
    hit |= __shfl_xor(hit, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    ssum[threadIdx.x >> 6] = s;
    shit[threadIdx.x >> 6] = hit;
  }
  __syncthreads();
  bool p = false;
  if (threadIdx.x == 0) {
    T t = (T)0;
    int h = 0;
    for (int w = 0; w < SV_BLOCK / 64; ++w) {
      t += ssum[w];
      h |= shit[w];
    }
    if (allow) {
      p = h || u_full;
      out[i] = p ? t : (T)0;
    } else {
      p = keep_old && present(old, i);
      out[i] = p ? load_as<T>(old.val, i) : (T)0;
    }
    obits[i] = p ? 1 : 0;
  }
  count_add(p ? 1ull : 0ull, cnt);
}

// Push mxv: one wavefront per present u(j) adds it into the rows i of
// column j (row j of the transposed pattern) that the mask allows.
template <typename T>
__global__ void sv_mxv_push_kernel(int64_t nnz, const int* __restrict__ uidx, Operand uval,
                                   const int* __restrict__ rowptrT, const int* __restrict__ colT, MaskView m, T* out,
                                   uint8_t* obits) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t k = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; k < nnz; k += waves) {
    const int j = uidx[k];
    const T v = load_as<T>(uval, k);
    const int e1 = rowptrT[j + 1];
    for (int e = rowptrT[j] + lane; e < e1; e += 64) {
      const int i = colT[e];
      if (!allowed(m, i)) continue;
      atomicAdd(out + i, v);
      obits[i] = 1;
    }
  }
}

// After a push: positions the mask forbids keep the old entry (or none).
template <typename T>
__global__ void sv_keep_old_kernel(int64_t n, MaskView m, VView old, int keep_old, T* out, uint8_t* obits,
                                   unsigned long long* cnt) {
  unsigned long long mine = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    bool p = false;
    if (i < n) {
      if (!allowed(m, i)) {
        const bool k = keep_old && present(old, i);
        out[i] = k ? load_as<T>(old.val, i) : (T)0;
        obits[i] = k ? 1 : 0;
      }
      p = obits[i] != 0;
    }
    mine += p ? 1ull : 0ull;
  }
  count_add(mine, cnt);
}

// w(i) = x where the mask allows, else the old entry unless replace.
template <typename T>
__global__ void sv_assign_kernel(int64_t n, double x, MaskView m, VView old, int keep_old, int out_type, void* out,
                                 uint8_t* obits, unsigned long long* cnt) {
  unsigned long long mine = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    bool p = false;
    if (i < n) {
      T v = (T)0;
      if (allowed(m, i)) {
        p = true;
        v = (T)x;
      } else if (keep_old && present(old, i)) {
        p = true;
        v = load_as<T>(old.val, i);
      }
      store_as<T>(out, out_type, i, v);
      obits[i] = p ? 1 : 0;
    }
    mine += p ? 1ull : 0ull;
  }
  count_add(mine, cnt);
}

// sparse -> bitset: out and bits must start zeroed.
__global__ void sv_scatter_kernel(int64_t nnz, const int* __restrict__ idx, Operand vals, int out_type, void* out,
                                  uint8_t* bits) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    const int64_t i = idx[e];
    store_as<double>(out, out_type, i, load_as<double>(vals, e));
    bits[i] = 1;
  }
}

// Presence of u and the reduce mask together, as a BOOL selector.
__global__ void sv_select_kernel(int64_t n, VView u, MaskView m, uint8_t* sel) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    sel[i] = (present(u, i) && allowed(m, i)) ? 1 : 0;
}

__global__ void sv_present_at_kernel(const uint8_t* bits, int64_t i, int* out) { *out = bits[i]; }

// ------------------------------------------------------------ host side

struct Held {
  VView v{};
  std::vector<BufP> keep;
};

BufP alloc_bytes(size_t b) { return dev_alloc(b < 4 ? 4 : b); }

constexpr size_t COUNT_BYTES = sizeof(unsigned long long) * COUNT_SLOTS * COUNT_STRIDE;

unsigned long long* new_counter(BufP& holder) {
  holder = alloc_bytes(COUNT_BYTES);
  hip_check(launch_zero(holder->p, COUNT_BYTES, ctx().stream), "zero counter");
  launch_mark(false);
  return (unsigned long long*)holder->p;
}

int64_t read_counter(const BufP& holder) {
  unsigned long long h[COUNT_SLOTS * COUNT_STRIDE];
  hip_check(hipMemcpyAsync(h, holder->p, COUNT_BYTES, hipMemcpyDeviceToHost, ctx().stream), "copy count");
  hip_check(hipStreamSynchronize(ctx().stream), "sync");
  unsigned long long t = 0;
  for (int k = 0; k < COUNT_SLOTS; ++k) t += h[k * COUNT_STRIDE];
  return (int64_t)t;
}

// Bitset storage (values of `type` and presence bytes) of the sparse node x.
void scatter_to_bitset(const Node& x, int type, BufP& vals, BufP& bits) {
  Ctx& c = ctx();
  vals = alloc_bytes(type_size(type) * (size_t)x.n);
  bits = alloc_bytes((size_t)x.n);
  hip_check(launch_zero(vals->p, type_size(type) * (size_t)x.n, c.stream), "zero");
  hip_check(launch_zero(bits->p, (size_t)x.n, c.stream), "zero");
  if (x.nvals > 0) {
    hipLaunchKernelGGL(sv_scatter_kernel, dim3(sv_grid(x.nvals)), dim3(SV_BLOCK), 0, c.stream, x.nvals,
                       (const int*)x.idx->p, Operand{x.buf->p, x.type, 0.0}, type, vals->p, (uint8_t*)bits->p);
    hip_check(hipGetLastError(), "scatter");
  }
  launch_mark(false);
}

// Whole-range view of a done vector (a sparse one is scattered first).
Held view_of(const NodeP& x) {
  Held h;
  if (x->fmt == F_FULL) {
    h.v.val = x->iso ? Operand{nullptr, x->type, x->iso_val} : Operand{x->buf->p, x->type, 0.0};
    h.v.bits = nullptr;
    if (!x->iso) h.keep.push_back(x->buf);
  } else if (x->fmt == F_BITSET) {
    h.v.val = Operand{x->buf->p, x->type, 0.0};
    h.v.bits = (const uint8_t*)x->bits->p;
    h.keep = {x->buf, x->bits};
  } else {
    BufP vals, bits;
    scatter_to_bitset(*x, x->type, vals, bits);
    h.v.val = Operand{vals->p, x->type, 0.0};
    h.v.bits = (const uint8_t*)bits->p;
    h.keep = {vals, bits};
  }
  return h;
}

struct HeldMask {
  MaskView m{};
  Held h;
};

HeldMask mask_of(const NodeP& mask, bool comp, bool structural) {
  HeldMask r;
  if (!mask) return r;
  r.h = view_of(mask);
  r.m.v = r.h.v;
  r.m.use = 1;
  r.m.comp = comp ? 1 : 0;
  r.m.structural = structural ? 1 : 0;
  return r;
}

// Store a computed bitset result in the node in the format its estimate
// (or the policy) asks for.
void finish(Node& n, const BufP& vals, const BufP& bits, int64_t count) {
  Ctx& c = ctx();
  n.nvals = count;
  n.iso = false;
  if (count == n.n) {
    n.fmt = F_FULL;
    n.buf = vals;
    n.bits.reset();
    n.idx.reset();
    c.stats.out_full++;
    return;
  }
  const bool sparse = c.format_policy == FP_SPARSE || (c.format_policy == FP_ESTIMATE && n.est < SPARSE_BELOW);
  if (!sparse) {
    n.fmt = F_BITSET;
    n.buf = vals;
    n.bits = bits;
    n.idx.reset();
    c.stats.out_bitset++;
    return;
  }
  BufP idx = alloc_bytes(sizeof(int) * (size_t)count);
  BufP out = alloc_bytes(type_size(n.type) * (size_t)count);
  BufP dcount = alloc_bytes(sizeof(unsigned int));
  const uint8_t* flags = (const uint8_t*)bits->p;
  const size_t nn = (size_t)n.n;
  auto select_into = [&](auto input, auto output) {
    size_t tb = 0;
    hip_check(rocprim::select(nullptr, tb, input, flags, output, (unsigned int*)dcount->p, nn, c.stream),
              "select size");
    BufP tmp = alloc_bytes(tb);
    hip_check(rocprim::select(tmp->p, tb, input, flags, output, (unsigned int*)dcount->p, nn, c.stream), "select");
    launch_mark(false);
    hip_check(hipStreamSynchronize(c.stream), "sync");  // tmp is released on return
  };
  select_into(rocprim::counting_iterator<int>(0), (int*)idx->p);
  switch (n.type) {
    case T_INT32: select_into((const int*)vals->p, (int*)out->p); break;
    case T_FP32: select_into((const float*)vals->p, (float*)out->p); break;
    default: select_into((const double*)vals->p, (double*)out->p); break;
  }
  n.fmt = F_SPARSE;
  n.idx = idx;
  n.buf = out;
  n.bits.reset();
  c.stats.out_sparse++;
}

int compute_type(int t) { return t == T_FP32 ? T_FP32 : T_FP64; }

template <typename F>
void by_type(int t, F f) {
  if (t == T_FP32) f(float(0));
  else f(double(0));
}

void exec_ewise(Node& n) {
  Ctx& c = ctx();
  const int ct = compute_type(n.type);
  BufP vals = alloc_bytes(type_size(n.type) * (size_t)n.n);
  BufP bits = alloc_bytes((size_t)n.n);
  BufP cntb;
  unsigned long long* cnt = new_counter(cntb);
  const bool binary = n.kind == N_EWISE;
  const int mode = binary ? (n.set_union ? SV_ADD : SV_MULT)
                          : n.kind == N_APPLY_U ? SV_UNARY : n.kind == N_APPLY_B1 ? SV_BIND1 : SV_BIND2;
  ScalarArg sc{nullptr, 0.0, n.k};
  if (n.kind == N_APPLY_B2S) sc = scalar_arg(n.s);
  const NodeP& A = n.a;
  const NodeP& B = n.b;
  auto fill_of = [](const NodeP& x) { return x->fmt == F_FULL ? 1.0 : (double)x->nvals / (double)std::max<int64_t>(1, x->n); };
  // index-driven loops
  bool index = false;
  if (mode == SV_MULT) {
    const bool as = A->fmt == F_SPARSE, bs = B->fmt == F_SPARSE;
    if (as || bs) {
      const bool drive_a = as && (!bs || fill_of(A) <= fill_of(B));
      const NodeP& D = drive_a ? A : B;
      const NodeP& O = drive_a ? B : A;
      Held ho = view_of(O);
      hip_check(launch_zero(vals->p, type_size(n.type) * (size_t)n.n, c.stream), "zero");
      hip_check(launch_zero(bits->p, (size_t)n.n, c.stream), "zero");
      by_type(ct, [&](auto z) {
        using T = decltype(z);
        if (D->nvals > 0)
          hipLaunchKernelGGL(sv_index_kernel<T>, dim3(sv_grid(D->nvals)), dim3(SV_BLOCK), 0, c.stream, D->nvals,
                             (const int*)D->idx->p, Operand{D->buf->p, D->type, 0.0}, mode, n.op, drive_a ? 0 : 1,
                             ho.v, sc, n.type, vals->p, (uint8_t*)bits->p);
      });
      hip_check(hipGetLastError(), "ewise index");
      index = true;
    }
  } else if (mode == SV_ADD) {
    if (A->fmt == F_SPARSE && B->fmt == F_SPARSE && n.est < SPARSE_BELOW) {
      BufP av, ab;
      scatter_to_bitset(*A, n.type, av, ab);
      vals = av;
      bits = ab;
      by_type(ct, [&](auto z) {
        using T = decltype(z);
        if (B->nvals > 0)
          hipLaunchKernelGGL(sv_index_kernel<T>, dim3(sv_grid(B->nvals)), dim3(SV_BLOCK), 0, c.stream, B->nvals,
                             (const int*)B->idx->p, Operand{B->buf->p, B->type, 0.0}, SV_ADD, n.op, 0,
                             VView{Operand{nullptr, n.type, 0.0}, nullptr}, sc, n.type, vals->p, (uint8_t*)bits->p);
      });
      hip_check(hipGetLastError(), "ewise index");
      index = true;
    }
  } else if (A->fmt == F_SPARSE) {
    hip_check(launch_zero(vals->p, type_size(n.type) * (size_t)n.n, c.stream), "zero");
    hip_check(launch_zero(bits->p, (size_t)n.n, c.stream), "zero");
    by_type(ct, [&](auto z) {
      using T = decltype(z);
      if (A->nvals > 0)
        hipLaunchKernelGGL(sv_index_kernel<T>, dim3(sv_grid(A->nvals)), dim3(SV_BLOCK), 0, c.stream, A->nvals,
                           (const int*)A->idx->p, Operand{A->buf->p, A->type, 0.0}, mode, n.op, 0,
                           VView{Operand{nullptr, n.type, 0.0}, nullptr}, sc, n.type, vals->p, (uint8_t*)bits->p);
    });
    hip_check(hipGetLastError(), "apply index");
    index = true;
  }
  int64_t count;
  if (index) {
    c.stats.index_loops++;
    // count the present entries
    HeldMask none;
    by_type(ct, [&](auto z) {
      using T = decltype(z);
      (void)z;
      hipLaunchKernelGGL(sv_range_kernel<T>, dim3(sv_grid(n.n)), dim3(SV_BLOCK), 0, c.stream, n.n, (int)SV_COPY, 0,
                         VView{Operand{vals->p, n.type, 0.0}, (const uint8_t*)bits->p}, VView{}, ScalarArg{nullptr, 0, 0},
                         n.type, vals->p, (uint8_t*)bits->p, cnt);
    });
    hip_check(hipGetLastError(), "count");
  } else {
    c.stats.range_loops++;
    Held ha = view_of(A);
    Held hb;
    if (binary) hb = view_of(B);
    by_type(ct, [&](auto z) {
      using T = decltype(z);
      hipLaunchKernelGGL(sv_range_kernel<T>, dim3(sv_grid(n.n)), dim3(SV_BLOCK), 0, c.stream, n.n, mode, n.op, ha.v,
                         hb.v, sc, n.type, vals->p, (uint8_t*)bits->p, cnt);
    });
    hip_check(hipGetLastError(), "ewise range");
  }
  launch_mark(false);
  count = read_counter(cntb);
  finish(n, vals, bits, count);
}

// Rows of A longer than SV_LONG_ROW (computed once per matrix, on the host
// from its row pointers).
int64_t long_rows_of(const MatP& A) {
  if (A->nlong >= 0) return A->nlong;
  Ctx& c = ctx();
  std::vector<int> rp((size_t)A->nrows + 1);
  hip_check(hipMemcpyAsync(rp.data(), A->rowptr->p, sizeof(int) * rp.size(), hipMemcpyDeviceToHost, c.stream),
            "copy row pointers");
  hip_check(hipStreamSynchronize(c.stream), "sync");
  std::vector<int> rows;
  for (int64_t i = 0; i < A->nrows; ++i)
    if (rp[(size_t)i + 1] - rp[(size_t)i] > SV_LONG_ROW) rows.push_back((int)i);
  A->long_rows = alloc_bytes(sizeof(int) * std::max<size_t>(rows.size(), 1));
  if (!rows.empty()) {
    hip_check(hipMemcpyAsync(A->long_rows->p, rows.data(), sizeof(int) * rows.size(), hipMemcpyHostToDevice, c.stream),
              "upload long rows");
    hip_check(hipStreamSynchronize(c.stream), "sync");
  }
  A->nlong = (int64_t)rows.size();
  return A->nlong;
}

void exec_mxv(Node& n) {
  Ctx& c = ctx();
  const NodeP& U = n.a;
  const MatP& A = n.A;
  BufP vals = alloc_bytes(type_size(n.type) * (size_t)n.n);
  BufP bits = alloc_bytes((size_t)n.n);
  BufP cntb;
  unsigned long long* cnt = new_counter(cntb);
  HeldMask hm = mask_of(n.mask, n.mask_comp, n.mask_struct);
  Held hold;
  const bool keep_old = n.mask && !n.replace && n.b;
  if (keep_old) hold = view_of(n.b);
  const double fill_u = U->fmt == F_FULL ? 1.0 : (double)U->nvals / (double)std::max<int64_t>(1, U->n);
  const bool push = U->fmt == F_SPARSE && fill_u < PUSH_BELOW && A->nnz > 0;
  if (push) {
    c.stats.mxv_push++;
    MatP AT = get_transposed(A);
    hip_check(launch_zero(vals->p, type_size(n.type) * (size_t)n.n, c.stream), "zero");
    hip_check(launch_zero(bits->p, (size_t)n.n, c.stream), "zero");
    by_type(n.type, [&](auto z) {
      using T = decltype(z);
      if (U->nvals > 0) {
        const int64_t blocks = std::min<int64_t>(65535, (U->nvals + 3) / 4);
        hipLaunchKernelGGL(sv_mxv_push_kernel<T>, dim3((int)blocks), dim3(SV_BLOCK), 0, c.stream, U->nvals,
                           (const int*)U->idx->p, Operand{U->buf->p, U->type, 0.0}, (const int*)AT->rowptr->p,
                           (const int*)AT->col->p, hm.m, (T*)vals->p, (uint8_t*)bits->p);
        hip_check(hipGetLastError(), "mxv push");
      }
      hipLaunchKernelGGL(sv_keep_old_kernel<T>, dim3(sv_grid(n.n)), dim3(SV_BLOCK), 0, c.stream, n.n, hm.m, hold.v,
                         keep_old ? 1 : 0, (T*)vals->p, (uint8_t*)bits->p, cnt);
      hip_check(hipGetLastError(), "mxv keep");
    });
  } else {
    c.stats.mxv_pull++;
    Held hu = view_of(U);
    const int u_full = U->fmt == F_FULL ? 1 : 0;
    const int* rp = (const int*)A->rowptr->p;
    const int* col = A->col ? (const int*)A->col->p : nullptr;
    const int64_t nlong = long_rows_of(A);
    by_type(n.type, [&](auto z) {
      using T = decltype(z);
      hipLaunchKernelGGL((sv_mxv_pull_kernel<T, 8>), dim3(sv_grid(n.n * 8)), dim3(SV_BLOCK), 0, c.stream, n.n, rp,
                         col, hu.v, u_full, hm.m, hold.v, keep_old ? 1 : 0, (T*)vals->p, (uint8_t*)bits->p, cnt);
      if (nlong > 0)
        hipLaunchKernelGGL(sv_mxv_pull_long_kernel<T>, dim3((unsigned)nlong), dim3(SV_BLOCK), 0, c.stream,
                           (const int*)A->long_rows->p, rp, col, hu.v, u_full, hm.m, hold.v, keep_old ? 1 : 0,
                           (T*)vals->p, (uint8_t*)bits->p, cnt);
    });
    hip_check(hipGetLastError(), "mxv pull");
  }
  launch_mark(false);
  finish(n, vals, bits, read_counter(cntb));
}

void exec_assign(Node& n) {
  Ctx& c = ctx();
  BufP vals = alloc_bytes(type_size(n.type) * (size_t)n.n);
  BufP bits = alloc_bytes((size_t)n.n);
  BufP cntb;
  unsigned long long* cnt = new_counter(cntb);
  HeldMask hm = mask_of(n.mask, n.mask_comp, n.mask_struct);
  Held hold;
  const bool keep_old = !n.replace && n.b;
  if (keep_old) hold = view_of(n.b);
  by_type(compute_type(n.type), [&](auto z) {
    using T = decltype(z);
    hipLaunchKernelGGL(sv_assign_kernel<T>, dim3(sv_grid(n.n)), dim3(SV_BLOCK), 0, c.stream, n.n, n.k, hm.m, hold.v,
                       keep_old ? 1 : 0, n.type, vals->p, (uint8_t*)bits->p, cnt);
  });
  hip_check(hipGetLastError(), "assign");
  launch_mark(false);
  finish(n, vals, bits, read_counter(cntb));
}

void exec_reduce(Node& n) {
  Ctx& c = ctx();
  BufP out = dev_alloc(sizeof(double));
  ReduceOut ro{(double*)out->p, n.guard_watch ? c.guard : nullptr};
  const NodeP& U = n.a;
  const bool masked = n.kind == N_REDUCE_MASK;
  if (!masked && U->fmt == F_SPARSE) {
    hip_check(launch_reduce(U->nvals, Operand{U->buf->p, U->type, 0.0}, 0, Operand{nullptr, T_FP64, 0.0}, 0, ro,
                            reduce_scratch(), c.guard, c.stream),
              "reduce");
  } else {
    Held hu = view_of(U);
    BufP sel = alloc_bytes((size_t)U->n);
    HeldMask hm;
    if (masked) {
      // the dense masked reduce tests the mask's values; keep that reading
      hm = mask_of(n.mask, n.mask_comp, false);
    }
    hipLaunchKernelGGL(sv_select_kernel, dim3(sv_grid(U->n)), dim3(SV_BLOCK), 0, c.stream, U->n, hu.v, hm.m,
                       (uint8_t*)sel->p);
    hip_check(hipGetLastError(), "select");
    hip_check(launch_reduce(U->n, hu.v.val, 1, Operand{sel->p, T_BOOL, 0.0}, 0, ro, reduce_scratch(), c.guard,
                            c.stream),
              "reduce");
    hip_check(hipStreamSynchronize(c.stream), "sync");  // sel and the views are released on return
  }
  launch_mark(false);
  n.buf = out;
  n.has_value = true;
}

double fill_of(const NodeP& x) {
  if (!x) return 1.0;
  if (x->done) return x->fmt == F_FULL ? 1.0 : (double)x->nvals / (double)std::max<int64_t>(1, x->n);
  return x->est;
}

bool maybe_missing(const NodeP& x) { return x && (x->done ? x->fmt != F_FULL : x->sparse_path); }

}  // namespace

// ------------------------------------------------------------ runtime hooks

void annotate(const NodeP& p) {
  Node& n = *p;
  const double fa = fill_of(n.a), fb = fill_of(n.b);
  auto masked_fill = [&](double f) {
    if (!n.mask) return f;
    const double fm = fill_of(n.mask);
    const double allow = n.mask_comp ? 1.0 - fm : fm;
    const double old = (n.b && !n.replace) ? fill_of(n.b) : 0.0;
    return f * allow + old * (1.0 - allow);
  };
  switch (n.kind) {
    case N_EWISE:
      n.sparse_path = maybe_missing(n.a) || maybe_missing(n.b);
      n.est = n.set_union ? fa + fb - fa * fb : fa * fb;  // independent positions
      break;
    case N_APPLY_U:
    case N_APPLY_B1:
    case N_APPLY_B2:
    case N_APPLY_B2S:
      n.sparse_path = maybe_missing(n.a);
      n.est = fa;
      break;
    case N_MXV: {
      n.sparse_path = maybe_missing(n.a) || n.mask != nullptr;
      double f = 1.0;
      if (maybe_missing(n.a) && n.A && n.A->nrows > 0) {
        // a row of mean length L meets no present entry with probability (1-fa)^L
        const double L = (double)n.A->nnz / (double)n.A->nrows;
        f = 1.0 - std::pow(1.0 - std::min(1.0, fa), L);
      }
      n.est = masked_fill(f);
      break;
    }
    case N_ASSIGN:
      n.sparse_path = true;
      n.est = masked_fill(1.0);
      break;
    case N_REDUCE:
    case N_REDUCE_MASK:
      n.sparse_path = maybe_missing(n.a) || maybe_missing(n.mask);
      break;
    default:
      break;
  }
  n.est = std::min(1.0, std::max(0.0, n.est));
}

void exec_sparse_node(const NodeP& np) {
  Node& n = *np;
  switch (n.kind) {
    case N_EWISE:
    case N_APPLY_U:
    case N_APPLY_B1:
    case N_APPLY_B2:
    case N_APPLY_B2S: exec_ewise(n); break;
    case N_MXV: exec_mxv(n); break;
    case N_ASSIGN: exec_assign(n); break;
    case N_REDUCE:
    case N_REDUCE_MASK: exec_reduce(n); break;
    default: fail(GrB_PANIC, "operation without a sparse form");
  }
}

void require_full(const NodeP& v, const char* what) {
  if (v->fmt != F_FULL)
    fail(GrB_INVALID_VALUE, std::string(what) + " needs a vector with every entry present");
}

int64_t vec_nvals(const NodeP& v) { return v->fmt == F_FULL ? v->n : v->nvals; }

void vec_tuples(const NodeP& v, int64_t* idx, void* vals, int out_type) {
  Ctx& c = ctx();
  const int64_t nv = vec_nvals(v);
  std::vector<int> hidx;
  BufP dvals;
  if (v->fmt == F_SPARSE) {
    hidx.resize((size_t)nv);
    if (nv) hip_check(hipMemcpyAsync(hidx.data(), v->idx->p, sizeof(int) * (size_t)nv, hipMemcpyDeviceToHost, c.stream),
                      "copy indices");
    dvals = v->buf;
  } else {
    std::vector<uint8_t> hb;
    if (v->fmt == F_BITSET) {
      hb.resize((size_t)v->n);
      hip_check(hipMemcpyAsync(hb.data(), v->bits->p, (size_t)v->n, hipMemcpyDeviceToHost, c.stream), "copy bits");
      hip_check(hipStreamSynchronize(c.stream), "sync");
    }
    for (int64_t i = 0; i < v->n; ++i)
      if (hb.empty() || hb[(size_t)i]) hidx.push_back((int)i);
    store_if_iso(v);
    dvals = v->buf;
  }
  // values converted to out_type on the device, then copied
  const int64_t m = v->fmt == F_SPARSE ? nv : v->n;
  BufP conv = alloc_bytes(type_size(out_type) * (size_t)std::max<int64_t>(m, 1));
  if (m) {
    hip_check(launch_convert(dvals->p, v->type, conv->p, out_type, m, c.stream), "convert");
    launch_mark(false);
  }
  std::vector<char> h(type_size(out_type) * (size_t)std::max<int64_t>(m, 1));
  if (m) hip_check(hipMemcpyAsync(h.data(), conv->p, type_size(out_type) * (size_t)m, hipMemcpyDeviceToHost, c.stream),
                   "copy values");
  hip_check(hipStreamSynchronize(c.stream), "sync");
  const size_t ts = type_size(out_type);
  for (int64_t k = 0; k < nv; ++k) {
    idx[k] = hidx[(size_t)k];
    const int64_t src = v->fmt == F_SPARSE ? k : hidx[(size_t)k];
    std::memcpy((char*)vals + ts * (size_t)k, h.data() + ts * (size_t)src, ts);
  }
}

MatP get_transposed(const MatP& A) {
  if (A->transposed) return A->transposed;
  Ctx& c = ctx();
  auto m = std::make_shared<MatData>();
  m->id = c.next_id++;
  m->nrows = A->ncols;
  m->ncols = A->nrows;
  m->nnz = A->nnz;
  m->rowptr = dev_alloc(sizeof(int) * (size_t)(m->nrows + 1));
  if (A->nnz > 0) m->col = dev_alloc(sizeof(int) * (size_t)A->nnz);
  hip_check(transpose_csr(A->nrows, A->ncols, (const int*)A->rowptr->p, A->col ? (const int*)A->col->p : nullptr,
                          A->nnz, (int*)m->rowptr->p, m->col ? (int*)m->col->p : nullptr, cache_alloc, cache_release,
                          nullptr, c.stream),
            "transpose");
  launch_mark(false);
  A->transposed = m;
  return m;
}

}  // namespace nbgrb

// ------------------------------------------------------------ C entry points

using namespace nbgrb;

namespace {

template <typename T>
T host_binop(int op, T x, T y) {
  switch (op) {
    case B_PLUS: return x + y;
    case B_MINUS: return x - y;
    case B_TIMES: return x * y;
    case B_DIV: return x / y;
    case B_MAX: return x > y ? x : y;
    case B_MIN: return x < y ? x : y;
    case B_FIRST: return x;
    case B_SECOND: return y;
    default: return x > y ? x - y : y - x;  // B_ABSDIFF
  }
}

template <typename T>
void build_vector(GrB_Vector w, const GrB_Index* indices, const T* values, GrB_Index nv, GrB_BinaryOp dup,
                  int type) {
  require_init();
  GB_Vector_opaque* o = vec(w, "w");
  if (o->type != type) fail(GrB_DOMAIN_MISMATCH, "value type differs from the vector's");
  if (nv > 0) {
    need(indices, "indices");
    need(values, "values");
  }
  if (dup && dup->type != type) fail(GrB_DOMAIN_MISMATCH, "dup operator type");
  std::vector<size_t> order((size_t)nv);
  std::iota(order.begin(), order.end(), (size_t)0);
  for (size_t k = 0; k < (size_t)nv; ++k)
    if (indices[k] >= (GrB_Index)o->n) fail(GrB_INDEX_OUT_OF_BOUNDS, "index >= vector size");
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return indices[a] < indices[b]; });
  std::vector<int> idx;
  std::vector<T> val;
  idx.reserve((size_t)nv);
  val.reserve((size_t)nv);
  for (size_t k : order) {
    if (!idx.empty() && idx.back() == (int)indices[k]) {
      if (!dup) fail(GrB_INVALID_VALUE, "repeated index and no dup operator");
      val.back() = host_binop<T>(dup->op, val.back(), values[k]);
    } else {
      idx.push_back((int)indices[k]);
      val.push_back(values[k]);
    }
  }
  Ctx& c = ctx();
  const int64_t count = (int64_t)idx.size();
  NodeP p = new_node(N_DENSE, type, o->n, false);
  p->done = true;
  p->nvals = count;
  p->fmt = F_SPARSE;
  p->idx = alloc_bytes(sizeof(int) * (size_t)count);
  p->buf = alloc_bytes(sizeof(T) * (size_t)count);
  if (count) {
    hip_check(hipMemcpyAsync(p->idx->p, idx.data(), sizeof(int) * (size_t)count, hipMemcpyHostToDevice, c.stream),
              "copy indices");
    hip_check(hipMemcpyAsync(p->buf->p, val.data(), sizeof(T) * (size_t)count, hipMemcpyHostToDevice, c.stream),
              "copy values");
  }
  const double fill = (double)count / (double)o->n;
  const bool sparse = c.format_policy == FP_SPARSE || (c.format_policy == FP_ESTIMATE && fill < SPARSE_BELOW);
  if (count == o->n || !sparse) {
    BufP vals, bits;
    scatter_to_bitset(*p, type, vals, bits);
    p->buf = vals;
    p->idx.reset();
    if (count == o->n) {
      p->fmt = F_FULL;
    } else {
      p->fmt = F_BITSET;
      p->bits = bits;
    }
  }
  // the host arrays are read by the copies above before this returns
  hip_check(hipStreamSynchronize(c.stream), "sync");
  set_vec(o, p);
}

template <typename T>
void extract_tuples(GrB_Index* indices, T* values, GrB_Index* n, GrB_Vector v, int type) {
  require_init();
  need(n, "n");
  GB_Vector_opaque* o = vec(v, "v");
  materialize(o->node);
  const int64_t nv = vec_nvals(o->node);
  if ((GrB_Index)nv > *n) fail(GrB_INSUFFICIENT_SPACE, "arrays are shorter than the number of entries");
  if (nv > 0) {
    need(indices, "indices");
    need(values, "values");
  }
  std::vector<int64_t> idx((size_t)std::max<int64_t>(nv, 1));
  vec_tuples(o->node, idx.data(), values, type);
  for (int64_t k = 0; k < nv; ++k) indices[k] = (GrB_Index)idx[(size_t)k];
  *n = (GrB_Index)nv;
}

void assign_scalar(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, double x, const GrB_Index* indices,
                   GrB_Index ni, GrB_Descriptor desc) {
  require_init();
  GB_Vector_opaque* wo = vec(w, "w");
  if (accum) fail(GrB_NOT_IMPLEMENTED, "accumulators are not supported");
  if (indices) fail(GrB_NOT_IMPLEMENTED, "only GrB_ALL (NULL) indices");
  if (ni != (GrB_Index)wo->n) fail(GrB_DIMENSION_MISMATCH, "ni must equal the vector size");
  GB_Vector_opaque* mo = mask ? vec(mask, "mask") : nullptr;
  if (mo && mo->n != wo->n) fail(GrB_DIMENSION_MISMATCH, "mask length");
  rec_assign(wo, mo, x, desc);
}

}  // namespace

extern "C" {

GrB_Info GrB_Vector_nvals(GrB_Index* nvals, GrB_Vector v) {
  API_BEGIN
  require_init();
  need(nvals, "nvals");
  GB_Vector_opaque* o = vec(v, "v");
  materialize(o->node);
  *nvals = (GrB_Index)vec_nvals(o->node);
  API_END
}

GrB_Info GrB_Vector_clear(GrB_Vector v) {
  API_BEGIN
  require_init();
  GB_Vector_opaque* o = vec(v, "v");
  NodeP p = new_node(N_DENSE, o->type, o->n, false);
  p->done = true;
  p->fmt = F_SPARSE;
  p->nvals = 0;
  p->idx = alloc_bytes(4);
  p->buf = alloc_bytes(8);
  set_vec(o, p);
  API_END
}

GrB_Info GrB_Vector_build_FP32(GrB_Vector w, const GrB_Index* indices, const float* values, GrB_Index nvals,
                               GrB_BinaryOp dup) {
  API_BEGIN
  build_vector<float>(w, indices, values, nvals, dup, T_FP32);
  API_END
}

GrB_Info GrB_Vector_build_FP64(GrB_Vector w, const GrB_Index* indices, const double* values, GrB_Index nvals,
                               GrB_BinaryOp dup) {
  API_BEGIN
  build_vector<double>(w, indices, values, nvals, dup, T_FP64);
  API_END
}

GrB_Info GrB_Vector_build_INT32(GrB_Vector w, const GrB_Index* indices, const int32_t* values, GrB_Index nvals,
                                GrB_BinaryOp dup) {
  API_BEGIN
  if (dup) fail(GrB_NOT_IMPLEMENTED, "INT32 vectors are built without a dup operator");
  build_vector<int32_t>(w, indices, values, nvals, nullptr, T_INT32);
  API_END
}

GrB_Info GrB_Vector_extractTuples_FP32(GrB_Index* indices, float* values, GrB_Index* n, GrB_Vector v) {
  API_BEGIN
  extract_tuples<float>(indices, values, n, v, T_FP32);
  API_END
}

GrB_Info GrB_Vector_extractTuples_FP64(GrB_Index* indices, double* values, GrB_Index* n, GrB_Vector v) {
  API_BEGIN
  extract_tuples<double>(indices, values, n, v, T_FP64);
  API_END
}

GrB_Info GrB_Vector_extractTuples_INT32(GrB_Index* indices, int32_t* values, GrB_Index* n, GrB_Vector v) {
  API_BEGIN
  extract_tuples<int32_t>(indices, values, n, v, T_INT32);
  API_END
}

GrB_Info GrB_Vector_assign_FP32(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, float x, const GrB_Index* indices,
                                GrB_Index ni, GrB_Descriptor desc) {
  API_BEGIN
  assign_scalar(w, mask, accum, (double)x, indices, ni, desc);
  API_END
}

GrB_Info GrB_Vector_assign_FP64(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, double x,
                                const GrB_Index* indices, GrB_Index ni, GrB_Descriptor desc) {
  API_BEGIN
  assign_scalar(w, mask, accum, x, indices, ni, desc);
  API_END
}

GrB_Info GrB_Vector_assign_INT32(GrB_Vector w, GrB_Vector mask, GrB_BinaryOp accum, int32_t x,
                                 const GrB_Index* indices, GrB_Index ni, GrB_Descriptor desc) {
  API_BEGIN
  assign_scalar(w, mask, accum, (double)x, indices, ni, desc);
  API_END
}

GrB_Info GrM_Vector_format(GrM_Format* fmt, GrB_Vector v) {
  API_BEGIN
  require_init();
  need(fmt, "fmt");
  GB_Vector_opaque* o = vec(v, "v");
  materialize(o->node);
  *fmt = o->node->fmt == F_FULL ? GrM_FULL : o->node->fmt == F_BITSET ? GrM_BITSET : GrM_SPARSE;
  API_END
}

GrB_Info GrM_set_format_policy(int policy) {
  API_BEGIN
  require_init();
  if (policy < FP_ESTIMATE || policy > FP_SPARSE) fail(GrB_INVALID_VALUE, "policy must be 0, 1 or 2");
  ctx().format_policy = policy;
  API_END
}

}  // extern "C"
