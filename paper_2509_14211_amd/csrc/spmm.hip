// Batched personalised PageRank as one sparse x dense product per pass.
//
// k <= 64 seed sets are iterated together: the operand is the n x k
// row-major matrix W (one row per vertex, one column per seed set), so each
// gathered neighbour is one coalesced k-wide row and lane c of a wavefront
// owns column c.  The pass fuses, per column, the same steps as the
// single-vector pass: the product, the teleport to the column's seeds
// (v_c = 1/|S_c| on S_c, scaled by (1-d) + d D_c when dangling mass is
// redistributed), the new ranks, their pre-scaled copy for the next pass,
// and the FP64 residual and dangling mass of every column.  Tiles come from
// the wavefront-tile plan of the matrix; hub rows are split into chunks
// whose k-wide partial sums are combined by the wavefront finishing the
// last chunk.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace nbgrb {

namespace {

constexpr int SB = 1024;   // threads per workgroup
constexpr int SNW = SB / 64;

template <typename V>
__device__ __forceinline__ void put(V* p, V v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename V>
__device__ __forceinline__ V get(const V* p) {
  return __hip_atomic_load(const_cast<V*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void drain() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Row sum of row entries [e0, e1) for this lane's column.
template <typename T>
__device__ __forceinline__ T row_gather(const int* __restrict__ col, const T* __restrict__ W, int k,
                                        int lane, bool on, int e0, int e1) {
  T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int e = e0;
  for (; e + 7 < e1; e += 8) {
    int j[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) j[u] = col[e + u];
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = on ? W[(int64_t)j[u] * k + lane] : (T)0;
    a0 += v[0] + v[4];
    a1 += v[1] + v[5];
    a2 += v[2] + v[6];
    a3 += v[3] + v[7];
  }
  for (; e < e1; ++e) {
    const int j = col[e];
    a0 += on ? W[(int64_t)j * k + lane] : (T)0;
  }
  return (a0 + a1) + (a2 + a3);
}

// First index in the vertex-sorted seed list with vertex >= v.
__device__ __forceinline__ int seed_lower_bound(const SpmmArgs& p, int v) {
  int lo = 0, hi = p.nseeds;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (p.seed_v[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ void spmm_epilogue(const SpmmArgs& p, int i, T s, int lane, bool on, T cfac,
                                              int& sp, double& rho, double& dm) {
  T tele = 0;
  while (sp < p.nseeds && p.seed_v[sp] == i) {
    if (p.seed_c[sp] == lane) tele += (T)p.seed_w[sp] * cfac;
    ++sp;
  }
  if (!on) return;
  const int64_t at = (int64_t)i * p.k + lane;
  const T r = s + tele;
  const T xo = __builtin_nontemporal_load((const T*)p.x_old + at);
  const T dv = ((const T*)p.dvec)[i];
  __builtin_nontemporal_store(r, (T*)p.x_new + at);
  ((T*)p.w_new)[at] = r * dv;
  rho += fabs((double)xo - (double)r);
  if (dv == (T)0) dm += (double)r;
}

template <typename T>
__global__ __launch_bounds__(SB) void spmm_ppr_kernel(TilePlanDev plan, SpmmArgs p, const GuardDev* guard) {
  if (guard && guard->active == 0) return;
  __shared__ double sr[SNW][64];
  __shared__ double sd[SNW][64];
  __shared__ int sflag;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const bool on = lane < p.k;
  const T* W = (const T*)p.w;
  // teleport factor of this lane's column: (1-d) + d D_c, or (1-d)
  T cfac = (T)0;
  if (on) cfac = (T)(p.c_beta + (p.d_prev ? p.c_alpha * p.d_prev[lane] : 0.0));
  double rho = 0.0, dm = 0.0;

  const int nwaves = (int)gridDim.x * SNW;
  for (int t = (int)blockIdx.x * SNW + wv; t < plan.ntiles; t += nwaves) {
    const int4 td = plan.tiles[t];
    if (td.y > 0) {
      const int row0 = td.x, nr = td.y;
      int sp = seed_lower_bound(p, row0);
      int e = p.rowptr[row0];
      for (int r = 0; r < nr; ++r) {
        const int e1 = p.rowptr[row0 + r + 1];
        const T s = row_gather<T>(p.col, W, p.k, lane, on, e, e1);
        spmm_epilogue<T>(p, row0 + r, s, lane, on, cfac, sp, rho, dm);
        e = e1;
      }
    } else {
      const int h = -td.y - 1;
      const int4 hub = plan.hubs[h];  // {row, nchunks, slot0, -}
      const T part = row_gather<T>(p.col, W, p.k, lane, on, td.z, td.z + td.w);
      if (on) put(&p.hub_sum[(int64_t)(hub.z + td.x) * 64 + lane], (double)part);
      drain();
      int last = 0;
      if (lane == 0) last = __hip_atomic_fetch_add(&p.hub_cnt[h], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                            hub.y - 1;
      last = __shfl(last, 0, 64);
      if (last) {
        T s = 0;
        for (int q = 0; q < hub.y; ++q) s += on ? (T)get(&p.hub_sum[(int64_t)(hub.z + q) * 64 + lane]) : (T)0;
        int sp = seed_lower_bound(p, hub.x);
        double hr = 0.0, hd = 0.0;
        spmm_epilogue<T>(p, hub.x, s, lane, on, cfac, sp, hr, hd);
        put(&p.hub_red[(int64_t)h * 128 + lane], hr);
        put(&p.hub_red[(int64_t)h * 128 + 64 + lane], hd);
        if (lane == 0) put(&p.hub_cnt[h], 0);
      }
    }
  }

  // per-column partials: wavefronts in order, then workgroups in order
  sr[wv][lane] = rho;
  sd[wv][lane] = dm;
  __syncthreads();
  if (tid < 64) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < SNW; ++w) {
      a += sr[w][tid];
      b += sd[w][tid];
    }
    put(&p.wg_part[(int64_t)blockIdx.x * 128 + tid], a);
    put(&p.wg_part[(int64_t)blockIdx.x * 128 + 64 + tid], b);
  }
  drain();
  __syncthreads();
  if (tid == 0) sflag = __hip_atomic_fetch_add(p.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                        gridDim.x - 1;
  __syncthreads();
  if (!sflag) return;
  if (tid < 64) {
    double a = 0.0, b = 0.0;
    for (int g = 0; g < (int)gridDim.x; ++g) {
      a += get(&p.wg_part[(int64_t)g * 128 + tid]);
      b += get(&p.wg_part[(int64_t)g * 128 + 64 + tid]);
    }
    for (int h = 0; h < plan.nhubs; ++h) {
      a += get(&p.hub_red[(int64_t)h * 128 + tid]);
      b += get(&p.hub_red[(int64_t)h * 128 + 64 + tid]);
    }
    sr[0][tid] = tid < p.k ? a : 0.0;
    sd[0][tid] = b;
  }
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    const int it = p.guard ? p.guard->iters + 1 : 0;
    for (int c = 0; c < p.k; ++c) {
      p.rho_out[c] = sr[0][c];
      p.d_out[c] = sd[0][c];
      if (sr[0][c] > mx) mx = sr[0][c];
      if (p.hit && p.hit[c] < 0 && p.guard && sr[0][c] <= p.guard->tol) p.hit[c] = it;
    }
    if (p.guard) {
      GuardDev* g = p.guard;
      g->rho_prev = g->rho;
      g->rho = mx;
      g->iters = it;
      g->active = (mx > g->tol && it < g->itermax) ? 1 : 0;
    }
    put(p.ticket, 0u);
  }
}

// x0 / w0 / D0 of the batch: x0 = V (seed weights), w0 = V .* d,
// D0_c = sum of the seed weights of column c on dangling vertices.
template <typename T>
__global__ void spmm_init_kernel(SpmmArgs p, const int* __restrict__ by_col_ptr,
                                 const int* __restrict__ by_col_v, const double* __restrict__ by_col_w) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= p.k) return;
  double D = 0.0;
  for (int q = by_col_ptr[c]; q < by_col_ptr[c + 1]; ++q) {
    const int v = by_col_v[q];
    const T wv = (T)by_col_w[q];
    const T dv = ((const T*)p.dvec)[v];
    ((T*)p.x_new)[(int64_t)v * p.k + c] = wv;
    ((T*)p.w_new)[(int64_t)v * p.k + c] = wv * dv;
    if (dv == (T)0) D += (double)wv;
  }
  p.d_out[c] = D;
  if (p.hit) p.hit[c] = -1;
}

__global__ void rows_permute_kernel(const void* __restrict__ in, int type, const int* __restrict__ idx,
                                    void* __restrict__ out, int64_t n, int k) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t total = n * k;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
    const int64_t i = q / k, c = q - i * k;
    const int64_t src = (int64_t)idx[i] * k + c;
    if (type == T_FP32)
      ((float*)out)[q] = ((const float*)in)[src];
    else
      ((double*)out)[q] = ((const double*)in)[src];
  }
}

}  // namespace

hipError_t launch_spmm_ppr(const TilePlanDev& plan, const SpmmArgs& a, int type, int grid,
                           const GuardDev* guard, hipStream_t s) {
  if (grid <= 0 || a.k < 1 || a.k > 64) return hipErrorInvalidValue;
  if (type == T_FP32)
    hipLaunchKernelGGL(spmm_ppr_kernel<float>, dim3(grid), dim3(SB), 0, s, plan, a, guard);
  else
    hipLaunchKernelGGL(spmm_ppr_kernel<double>, dim3(grid), dim3(SB), 0, s, plan, a, guard);
  return hipGetLastError();
}

hipError_t launch_spmm_init(const SpmmArgs& a, int type, const int* by_col_ptr, const int* by_col_v,
                            const double* by_col_w, hipStream_t s) {
  if (type == T_FP32)
    hipLaunchKernelGGL(spmm_init_kernel<float>, dim3(1), dim3(64), 0, s, a, by_col_ptr, by_col_v, by_col_w);
  else
    hipLaunchKernelGGL(spmm_init_kernel<double>, dim3(1), dim3(64), 0, s, a, by_col_ptr, by_col_v, by_col_w);
  return hipGetLastError();
}

hipError_t launch_rows_permute(const void* in, int type, const int* idx, void* out, int64_t n, int k,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n * k + 1023) / 1024;
  if (g > 16384) g = 16384;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(rows_permute_kernel, dim3((int)g), dim3(256), 0, s, in, type, idx, out, n, k);
  return hipGetLastError();
}

}  // namespace nbgrb
