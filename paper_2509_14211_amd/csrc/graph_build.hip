// Sort-based CSR construction on the GPU: edge list -> 64-bit (row, col)
// keys -> rocPRIM radix sort -> unique -> row pointers by binary search.
// The same path builds a transpose from the (col, row) keys of an existing
// pattern.  Everything here is integer work, so the result is exact.
#include <cstring>
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

#include "kernels.h"

namespace nbgrb {

namespace {

constexpr int GB_BLOCK = 256;

int gb_grid(int64_t n) {
  int64_t g = (n + GB_BLOCK * 4 - 1) / (GB_BLOCK * 4);
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  return (int)g;
}

int bit_width_u64(uint64_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

// key = src << 32 | dst; dropped edges get key = n << 32 (sorts after every
// valid key and is stripped after the unique pass).
__global__ void edge_keys_kernel(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                                 int64_t nedges, int64_t n, int drop_self,
                                 uint64_t* __restrict__ keys, int* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t sentinel = (uint64_t)n << 32;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nedges; e += stride) {
    const uint32_t s = src[e], d = dst[e];
    uint64_t k = ((uint64_t)s << 32) | (uint64_t)d;
    if ((int64_t)s >= n || (int64_t)d >= n) {
      atomicOr(bad, 1);
      k = sentinel;
    } else if (drop_self && s == d) {
      k = sentinel;
    }
    keys[e] = k;
  }
}

// key = col << 32 | row for every entry of a CSR pattern; the row of entry
// e is found by binary search in rowptr.
__global__ void transpose_keys_kernel(const int* __restrict__ rowptr, int64_t nrows,
                                      const int* __restrict__ col, int64_t nnz,
                                      uint64_t* __restrict__ keys) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    // largest row r with rowptr[r] <= e
    int64_t lo = 0, hi = nrows;  // invariant rowptr[lo] <= e < rowptr[hi]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)rowptr[mid] <= e) lo = mid; else hi = mid;
    }
    keys[e] = ((uint64_t)(uint32_t)col[e] << 32) | (uint64_t)lo;
  }
}

// rowptr[r] = number of sorted keys whose high word is < r, r in [0, n];
// col[k] = low word of key k.
__global__ void keys_to_csr_kernel(const uint64_t* __restrict__ keys, int64_t nkeys, int64_t n,
                                   int* __restrict__ rowptr, int* __restrict__ col) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t r = tid; r <= n; r += stride) {
    const uint64_t target = (uint64_t)r << 32;
    int64_t lo = 0, hi = nkeys;  // first index with keys[idx] >= target
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < target) lo = mid + 1; else hi = mid;
    }
    rowptr[r] = (int)lo;
  }
  for (int64_t k = tid; k < nkeys; k += stride) col[k] = (int)(uint32_t)(keys[k] & 0xFFFFFFFFull);
}

struct Scoped {
  AllocFn alloc;
  ReleaseFn release;
  void* ctx;
  void* p = nullptr;
  Scoped(AllocFn a, ReleaseFn r, void* c, size_t bytes) : alloc(a), release(r), ctx(c) {
    p = bytes ? alloc(bytes, ctx) : nullptr;
  }
  ~Scoped() {
    if (p) release(p, ctx);
  }
  bool ok(size_t bytes) const { return bytes == 0 || p != nullptr; }
};

// Sort keys[0:nkeys) (bits [0, end_bit)) into out, unique them into keys,
// return the unique count in *count.
hipError_t sort_unique(uint64_t* keys, uint64_t* out, int64_t nkeys, unsigned end_bit,
                       int64_t* count, AllocFn alloc, ReleaseFn release, void* actx,
                       hipStream_t s) {
  size_t sort_bytes = 0, uniq_bytes = 0;
  hipError_t e = rocprim::radix_sort_keys(nullptr, sort_bytes, keys, out, (size_t)nkeys, 0u,
                                          end_bit, s);
  if (e != hipSuccess) return e;
  e = rocprim::unique(nullptr, uniq_bytes, out, keys, (unsigned long long*)nullptr, (size_t)nkeys,
                      rocprim::equal_to<uint64_t>(), s);
  if (e != hipSuccess) return e;
  const size_t tmp_bytes = (sort_bytes > uniq_bytes ? sort_bytes : uniq_bytes) + 256;
  Scoped tmp(alloc, release, actx, tmp_bytes);
  if (!tmp.ok(tmp_bytes)) return hipErrorOutOfMemory;
  unsigned long long* dcount = (unsigned long long*)tmp.p;
  void* work = (char*)tmp.p + 256;
  size_t wb = tmp_bytes - 256;
  e = rocprim::radix_sort_keys(work, wb, keys, out, (size_t)nkeys, 0u, end_bit, s);
  if (e != hipSuccess) return e;
  wb = tmp_bytes - 256;
  e = rocprim::unique(work, wb, out, keys, dcount, (size_t)nkeys, rocprim::equal_to<uint64_t>(),
                      s);
  if (e != hipSuccess) return e;
  unsigned long long hcount = 0;
  e = hipMemcpyAsync(&hcount, dcount, sizeof(hcount), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  *count = (int64_t)hcount;
  return hipSuccess;
}

}  // namespace

hipError_t build_csr_from_edges(int64_t n, const uint32_t* src, const uint32_t* dst,
                                int64_t nedges, bool drop_self, int* rowptr, int* col,
                                int64_t* nnz, int* bad_flag, AllocFn alloc, ReleaseFn release,
                                void* actx, hipStream_t s) {
  *nnz = 0;
  if (nedges == 0) return launch_fill(rowptr, T_INT32, n + 1, 0.0, s);
  Scoped kbuf(alloc, release, actx, (size_t)nedges * 16);
  if (!kbuf.ok(1)) return hipErrorOutOfMemory;
  uint64_t* keys = (uint64_t*)kbuf.p;
  uint64_t* out = keys + nedges;
  hipLaunchKernelGGL(edge_keys_kernel, dim3(gb_grid(nedges)), dim3(GB_BLOCK), 0, s, src, dst,
                     nedges, n, drop_self ? 1 : 0, keys, bad_flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned end_bit = 32u + (unsigned)bit_width_u64((uint64_t)n);
  int64_t u = 0;
  e = sort_unique(keys, out, nedges, end_bit, &u, alloc, release, actx, s);
  if (e != hipSuccess) return e;
  // strip the sentinel (it sorts last; unique keeps at most one copy)
  if (u > 0) {
    uint64_t last = 0;
    e = hipMemcpyAsync(&last, keys + (u - 1), 8, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if ((last >> 32) >= (uint64_t)n) --u;
  }
  hipLaunchKernelGGL(keys_to_csr_kernel, dim3(gb_grid(n + 1 > u ? n + 1 : u)), dim3(GB_BLOCK), 0,
                     s, keys, u, n, rowptr, col);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  *nnz = u;
  return hipSuccess;
}

hipError_t transpose_csr(int64_t nrows, int64_t ncols, const int* rowptr, const int* col,
                         int64_t nnz, int* rowptrT, int* colT, AllocFn alloc,
                         ReleaseFn release, void* actx, hipStream_t s) {
  if (nnz == 0) return launch_fill(rowptrT, T_INT32, ncols + 1, 0.0, s);
  Scoped kbuf(alloc, release, actx, (size_t)nnz * 16);
  if (!kbuf.ok(1)) return hipErrorOutOfMemory;
  uint64_t* keys = (uint64_t*)kbuf.p;
  uint64_t* out = keys + nnz;
  hipLaunchKernelGGL(transpose_keys_kernel, dim3(gb_grid(nnz)), dim3(GB_BLOCK), 0, s, rowptr,
                     nrows, col, nnz, keys);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned end_bit = 32u + (unsigned)bit_width_u64((uint64_t)ncols);
  int64_t u = 0;
  e = sort_unique(keys, out, nnz, end_bit, &u, alloc, release, actx, s);
  if (e != hipSuccess) return e;
  if (u != nnz) return hipErrorInvalidValue;  // duplicate entries in the input pattern
  hipLaunchKernelGGL(keys_to_csr_kernel, dim3(gb_grid(ncols + 1 > nnz ? ncols + 1 : nnz)),
                     dim3(GB_BLOCK), 0, s, keys, nnz, ncols, rowptrT, colT);
  return hipGetLastError();
}

namespace {

__global__ void column_count_kernel(const int* __restrict__ col, int64_t nnz, int* __restrict__ cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride)
    atomicAdd(&cnt[col[e]], 1);
}

// key = (2^32 - 1 - count) << 32 | v: ascending keys = decreasing count,
// ties by increasing vertex id.
__global__ void degree_keys_kernel(const int* __restrict__ cnt, int64_t n, uint64_t* __restrict__ keys) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    keys[v] = ((uint64_t)(0xFFFFFFFFu - (uint32_t)cnt[v]) << 32) | (uint64_t)v;
}

__global__ void order_from_keys_kernel(const uint64_t* __restrict__ keys, int64_t n, int* __restrict__ order,
                                       int* __restrict__ inv) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    const int v = (int)(uint32_t)(keys[k] & 0xFFFFFFFFull);
    order[k] = v;
    inv[v] = (int)k;
  }
}

// key = inv[row] << 32 | inv[col] for every entry of a square pattern.
__global__ void permute_keys_kernel(const int* __restrict__ rowptr, int64_t n, const int* __restrict__ col,
                                    int64_t nnz, const int* __restrict__ inv, uint64_t* __restrict__ keys) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)rowptr[mid] <= e) lo = mid; else hi = mid;
    }
    keys[e] = ((uint64_t)(uint32_t)inv[lo] << 32) | (uint64_t)(uint32_t)inv[col[e]];
  }
}

}  // namespace

hipError_t launch_column_count(const int* col, int64_t nnz, int* cnt, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(column_count_kernel, dim3(gb_grid(nnz)), dim3(GB_BLOCK), 0, s, col, nnz, cnt);
  return hipGetLastError();
}

hipError_t degree_order(int64_t n, const int* col, int64_t nnz, int* order, int* inv, AllocFn alloc,
                        ReleaseFn release, void* actx, hipStream_t s) {
  Scoped cbuf(alloc, release, actx, (size_t)n * sizeof(int));
  Scoped kbuf(alloc, release, actx, (size_t)n * 16);
  if (!cbuf.ok(1) || !kbuf.ok(1)) return hipErrorOutOfMemory;
  int* cnt = (int*)cbuf.p;
  uint64_t* keys = (uint64_t*)kbuf.p;
  uint64_t* out = keys + n;
  hipError_t e = launch_fill(cnt, T_INT32, n, 0.0, s);
  if (e != hipSuccess) return e;
  if (nnz > 0) {
    hipLaunchKernelGGL(column_count_kernel, dim3(gb_grid(nnz)), dim3(GB_BLOCK), 0, s, col, nnz, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(degree_keys_kernel, dim3(gb_grid(n)), dim3(GB_BLOCK), 0, s, cnt, n, keys);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  size_t tb = 0;
  e = rocprim::radix_sort_keys(nullptr, tb, keys, out, (size_t)n, 0u, 64u, s);
  if (e != hipSuccess) return e;
  Scoped tmp(alloc, release, actx, tb + 256);
  if (!tmp.ok(1)) return hipErrorOutOfMemory;
  e = rocprim::radix_sort_keys(tmp.p, tb, keys, out, (size_t)n, 0u, 64u, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(order_from_keys_kernel, dim3(gb_grid(n)), dim3(GB_BLOCK), 0, s, out, n, order, inv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipStreamSynchronize(s);  // scoped temporaries are released on return
}

hipError_t scan_u32_inclusive(const unsigned* in, unsigned* out, int64_t n, AllocFn alloc, ReleaseFn release,
                              void* actx, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  size_t tb = 0;
  hipError_t e = rocprim::inclusive_scan(nullptr, tb, in, out, (size_t)n, rocprim::plus<unsigned>(), s);
  if (e != hipSuccess) return e;
  Scoped tmp(alloc, release, actx, tb + 256);
  if (!tmp.ok(1)) return hipErrorOutOfMemory;
  e = rocprim::inclusive_scan(tmp.p, tb, in, out, (size_t)n, rocprim::plus<unsigned>(), s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);  // the scoped temporary is released on return
}

hipError_t sort_pairs_u64_u16(const uint64_t* keys_in, uint64_t* keys_out, const uint16_t* vals_in,
                              uint16_t* vals_out, int64_t n, unsigned end_bit, AllocFn alloc,
                              ReleaseFn release, void* actx, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  size_t tb = 0;
  hipError_t e = rocprim::radix_sort_pairs(nullptr, tb, keys_in, keys_out, vals_in, vals_out, (size_t)n, 0u,
                                           end_bit, s);
  if (e != hipSuccess) return e;
  Scoped tmp(alloc, release, actx, tb + 256);
  if (!tmp.ok(1)) return hipErrorOutOfMemory;
  e = rocprim::radix_sort_pairs(tmp.p, tb, keys_in, keys_out, vals_in, vals_out, (size_t)n, 0u, end_bit, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);  // the scoped temporary is released on return
}

hipError_t permute_csr(int64_t n, const int* rowptr, const int* col, int64_t nnz, const int* inv,
                       int* rowptr2, int* col2, AllocFn alloc, ReleaseFn release, void* actx,
                       hipStream_t s) {
  if (nnz == 0) return launch_fill(rowptr2, T_INT32, n + 1, 0.0, s);
  Scoped kbuf(alloc, release, actx, (size_t)nnz * 16);
  if (!kbuf.ok(1)) return hipErrorOutOfMemory;
  uint64_t* keys = (uint64_t*)kbuf.p;
  uint64_t* out = keys + nnz;
  hipLaunchKernelGGL(permute_keys_kernel, dim3(gb_grid(nnz)), dim3(GB_BLOCK), 0, s, rowptr, n, col, nnz,
                     inv, keys);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned end_bit = 32u + (unsigned)bit_width_u64((uint64_t)n);
  int64_t u = 0;
  e = sort_unique(keys, out, nnz, end_bit, &u, alloc, release, actx, s);
  if (e != hipSuccess) return e;
  if (u != nnz) return hipErrorInvalidValue;
  hipLaunchKernelGGL(keys_to_csr_kernel, dim3(gb_grid(n + 1 > nnz ? n + 1 : nnz)), dim3(GB_BLOCK), 0, s,
                     keys, nnz, n, rowptr2, col2);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace nbgrb
