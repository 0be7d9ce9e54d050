// Web-shaped synthetic graph generator.
//
// The paper measures on a web crawl with strong locality and a high mean
// degree (Section IV).  This generator produces a graph of that shape,
// vertex by vertex and link by link, from a counter-based SplitMix64 stream:
// every link depends only on (seed, u, j), so the whole edge list is made in
// parallel and any single row can be regenerated on its own.  Only unsigned
// 64-bit integer arithmetic is used, so every implementation of the same
// definition produces the same bits.
//
// Three kinds of links:
//  * home links to the first page of an aligned block around u (a site's
//    front page at one of 16 levels of the address hierarchy);
//  * local links at a heavy-tailed distance d >= max(local_min, k_u) on
//    either side of u (pages of one site link to each other);
//  * global links to a popular page: a Pareto-like index scattered over
//    the vertex range by an affine bijection.
// Out-degrees follow a truncated Pareto-like law with a share of pages
// having no out-links at all.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_scan.hpp>

#include "abi_util.h"
#include "device_util.h"
#include "kernels.h"

namespace nbgrb {

namespace {

constexpr int WG_BLOCK = 256;

struct WebDev {
  uint64_t n, seed;
  uint64_t kmin, kmax, p_zero, p_home, p_local_end, local_min, hub, perm_a, perm_b;
};

// (c << 52) / ((r >> 12) + 1): at least c, P(value >= x) close to c / x.
__device__ __forceinline__ uint64_t pareto_draw(uint64_t c, uint64_t r) {
  return (c << 52) / ((r >> 12) + 1ull);
}

__device__ __forceinline__ uint64_t web_degree(const WebDev& m, uint64_t u) {
  const uint64_t a = splitmix_draw(m.seed, (u << 18) | 0x3FFFCull);
  if ((a >> 48) < m.p_zero) return 0;
  const uint64_t k = pareto_draw(m.kmin, splitmix_draw(m.seed, (u << 18) | 0x3FFFDull));
  return k < m.kmax ? k : m.kmax;
}

__device__ __forceinline__ uint64_t web_target(const WebDev& m, uint64_t u, uint64_t j, uint64_t ku) {
  const uint64_t key = (u << 18) | (j << 2);
  const uint64_t r = splitmix_draw(m.seed, key);
  const uint64_t t = r >> 48;
  if (t < m.p_home) return u & ~((1ull << (6 + (r & 15))) - 1ull);
  const uint64_t q = splitmix_draw(m.seed, key | 1ull);
  if (t < m.p_local_end) {
    uint64_t d = pareto_draw(ku > m.local_min ? ku : m.local_min, q);
    if (d > m.n - 1) d = m.n - 1;
    return ((r >> 4) & 1ull) ? (u + m.n - d) % m.n : (u + d) % m.n;
  }
  const uint64_t i = (pareto_draw(m.hub, q) - m.hub) % m.n;
  return (m.perm_a * i + m.perm_b) % m.n;
}

__global__ void web_degree_kernel(WebDev m, int64_t* __restrict__ deg, int64_t* __restrict__ off) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t0 == 0) off[0] = 0;
  for (int64_t u = t0; u < (int64_t)m.n; u += stride) deg[u] = (int64_t)web_degree(m, (uint64_t)u);
}

// Link e belongs to the vertex u with off[u] <= e < off[u+1] (binary
// search over the n+1 offsets) and is its link j = e - off[u].
__global__ void web_edge_kernel(WebDev m, const int64_t* __restrict__ off, int64_t nedges,
                                uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t n = (int64_t)m.n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nedges; e += stride) {
    int64_t lo = 0, hi = n;  // off[lo] <= e < off[hi]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (off[mid] <= e) lo = mid; else hi = mid;
    }
    const uint64_t ku = (uint64_t)(off[lo + 1] - off[lo]);
    src[e] = (uint32_t)lo;
    dst[e] = (uint32_t)web_target(m, (uint64_t)lo, (uint64_t)(e - off[lo]), ku);
  }
}

int web_grid(int64_t items) {
  int64_t g = (items + WG_BLOCK * 4 - 1) / (WG_BLOCK * 4);
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  return (int)g;
}

uint64_t gcd_u64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace

}  // namespace nbgrb

using namespace nbgrb;

extern "C" {

GrB_Info GrM_web_edges(uint32_t* src, uint32_t* dst, GrB_Index capacity, GrB_Index* nedges, GrB_Index n,
                       uint64_t seed, const GrM_WebModel* model) {
  API_BEGIN
  require_init();
  need(nedges, "nedges");
  need(model, "model");
  const GrM_WebModel& M = *model;
  if (n < 1 || n > 0xFFFFFFFFull) fail(GrB_INVALID_VALUE, "n must be in [1, 2^32)");
  if (M.kmin < 1 || M.kmax < M.kmin || M.kmax > 4095) fail(GrB_INVALID_VALUE, "need 1 <= kmin <= kmax <= 4095");
  if (M.local_min < 1 || M.local_min > 4095 || M.hub < 1 || M.hub > 4095)
    fail(GrB_INVALID_VALUE, "local_min and hub must be in [1, 4095]");
  if (M.p_zero < 0 || M.p_home < 0 || M.p_local < 0 ||
      (int64_t)M.p_zero + M.p_home + M.p_local > 65536)
    fail(GrB_INVALID_VALUE, "probabilities must be >= 0 and sum to at most 65536");
  if (gcd_u64(M.perm_a, n) != 1) fail(GrB_INVALID_VALUE, "perm_a must be coprime with n");
  *nedges = 0;
  WebDev d{};
  d.n = n;
  d.seed = seed;
  d.kmin = (uint64_t)M.kmin;
  d.kmax = (uint64_t)M.kmax;
  d.p_zero = (uint64_t)M.p_zero;
  d.p_home = (uint64_t)M.p_home;
  d.p_local_end = (uint64_t)M.p_home + (uint64_t)M.p_local;
  d.local_min = (uint64_t)M.local_min;
  d.hub = (uint64_t)M.hub;
  d.perm_a = M.perm_a;
  d.perm_b = M.perm_b;
  Ctx& c = ctx();
  BufP deg = dev_alloc(sizeof(int64_t) * (size_t)n);
  BufP off = dev_alloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* dp = (int64_t*)deg->p;
  int64_t* op = (int64_t*)off->p;
  hipLaunchKernelGGL(web_degree_kernel, dim3(web_grid((int64_t)n)), dim3(WG_BLOCK), 0, c.stream, d, dp, op);
  hip_check(hipGetLastError(), "web degrees");
  launch_mark(false);
  size_t tb = 0;
  hip_check(rocprim::inclusive_scan(nullptr, tb, dp, op + 1, (size_t)n, rocprim::plus<int64_t>(), c.stream),
            "scan size");
  {
    BufP tmp = dev_alloc(tb + 256);
    hip_check(rocprim::inclusive_scan(tmp->p, tb, dp, op + 1, (size_t)n, rocprim::plus<int64_t>(), c.stream),
              "scan");
    launch_mark(false);
    int64_t total = 0;
    hip_check(hipMemcpyAsync(&total, op + n, sizeof(total), hipMemcpyDeviceToHost, c.stream), "copy count");
    hip_check(hipStreamSynchronize(c.stream), "sync");
    *nedges = (GrB_Index)total;
  }
  if (!src && !dst) return GrB_SUCCESS;
  need(src, "src");
  need(dst, "dst");
  if (capacity < *nedges) fail(GrB_INSUFFICIENT_SPACE, "capacity is below the number of links");
  if (*nedges > 0) {
    hipLaunchKernelGGL(web_edge_kernel, dim3(web_grid((int64_t)*nedges)), dim3(WG_BLOCK), 0, c.stream, d, op,
                       (int64_t)*nedges, src, dst);
    hip_check(hipGetLastError(), "web links");
    launch_mark(false);
  }
  // the temporaries are released on return: the stream must be past them
  hip_check(hipStreamSynchronize(c.stream), "sync");
  API_END
}

}  // extern "C"
