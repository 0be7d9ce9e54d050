// Learned warm start for personalised PageRank: random-walk features, a
// two-layer mean-aggregation graph network, its gradient and Adam, and the
// C entry points that drive them (declared in include/nbgrb.h).
//
// Per vertex v with seed set S:
//   x_v  = [1{v in S}, log(1+indeg), log(1+outdeg), log(1 + n c_t(v)/W), t=1..8]
//          (c_t = walkers at v after t steps of W walks with restart to S)
//   m_v  = mean of x_u over in-neighbours u (0 without any)
//   h_v  = ReLU(W1s x_v + W1n m_v + b1)                         (11 -> 64)
//   a_v  = w2s . h_v + b2,  q_v = w2n . h_v
//   z_v  = a_v + mean of q_u over in-neighbours                 (64 -> 1)
//   x0   = softmax(z), or the teleport vector when that is not a finite
//          positive distribution.
// Weights are FP32, activations (x, m, h) are stored as FP32 or BF16, sums
// are accumulated in FP32 (weight gradients and the softmax normaliser in
// FP64).
//
// Layer 1 is one pass over the wavefront tile plan of A^T: lanes 0..15
// gather the 16-wide (11 used) feature rows of the in-neighbours, and at
// the end of each row all 64 lanes (one per hidden unit) apply the dense
// layer with the row's features broadcast from scalar registers, so the
// 11 -> 64 contraction never leaves the gather kernel.  It is small (22
// terms per output) and bound by the gather, so it runs on the vector ALUs
// rather than as a separate matrix-core GEMM with an extra round trip of
// the aggregated features.  Layer 2 projects to one value per vertex first
// and aggregates that value with the library's mxv.  The backward pass
// walks A (out-neighbours) with the same mxv for the aggregation's adjoint
// and accumulates the weight gradients per lane in FP64 with fixed-order
// reductions, so every result is bitwise reproducible.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "device_util.h"
#include "runtime.h"

namespace nbgrb {
namespace {

constexpr int GNF = 11;   // features
constexpr int GF = 16;    // stored feature row width (padded)
constexpr int GH = 64;    // hidden units
constexpr int GSTEPS = 8; // walk steps
constexpr int NPARAM = 2 * GH * GNF + 3 * GH + 1;
constexpr int OFF_W1S = 0, OFF_W1N = GH * GNF, OFF_B1 = 2 * GH * GNF, OFF_W2S = OFF_B1 + GH,
              OFF_W2N = OFF_W2S + GH, OFF_B2 = OFF_W2N + GH;
constexpr int GB = 1024;  // threads per workgroup of the graph kernels
constexpr int GNW = GB / 64;

// bfloat16 storage: the upper half of an IEEE binary32 value, rounded to
// nearest even (NaN stays NaN).
struct bf16 {
  uint16_t v;
};
__device__ __forceinline__ float act_to_f(float x) { return x; }
__device__ __forceinline__ float act_to_f(bf16 x) { return __uint_as_float((uint32_t)x.v << 16); }
template <typename A>
__device__ __forceinline__ A act_from_f(float x);
template <>
__device__ __forceinline__ float act_from_f<float>(float x) {
  return x;
}
template <>
__device__ __forceinline__ bf16 act_from_f<bf16>(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return bf16{(uint16_t)((u >> 16) | 0x40u)};
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16{(uint16_t)(u >> 16)};
}

template <typename V>
__device__ __forceinline__ V wsum(V v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ void lds_fence_wave() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// --------------------------------------------------------------- features

// One thread per walker; counts[(t-1) n + v] += 1 for its vertex after step t.
// Draw key(w, t, j) = 4 (8 w + t - 1) + j: j = 0 decides restart (u < 1 - d,
// or a vertex without out-edges), j = 1 picks the restart seed, j = 2 the
// out-edge.
__global__ void gnn_walk_kernel(const int* __restrict__ rowptr, const int* __restrict__ col,
                                const int* __restrict__ seeds, int ns, int walkers, double damping,
                                uint64_t seed, int* __restrict__ counts, int64_t n) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= walkers) return;
  int pos = seeds[w % ns];
  const double restart = 1.0 - damping;
  for (int t = 1; t <= GSTEPS; ++t) {
    const uint64_t key = ((uint64_t)w * GSTEPS + (uint64_t)(t - 1)) * 4ull;
    const double u = draw_unit(splitmix_draw(seed, key));
    const int lo = rowptr[pos], d = rowptr[pos + 1] - lo;
    if (u < restart || d == 0)
      pos = seeds[(int)(splitmix_draw(seed, key + 1) % (uint64_t)ns)];
    else
      pos = col[lo + (int)(splitmix_draw(seed, key + 2) % (uint64_t)d)];
    atomicAdd(&counts[(int64_t)(t - 1) * n + pos], 1);
  }
}

template <typename A>
__global__ void gnn_features_kernel(int64_t n, const int* __restrict__ rowptrA, const int* __restrict__ rowptrT,
                                    const int* __restrict__ counts, int walkers, A* __restrict__ X) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  A f[GF];
  f[0] = act_from_f<A>(0.f);
  f[1] = act_from_f<A>((float)log1p((double)(rowptrT[v + 1] - rowptrT[v])));
  f[2] = act_from_f<A>((float)log1p((double)(rowptrA[v + 1] - rowptrA[v])));
#pragma unroll
  for (int t = 0; t < GSTEPS; ++t)
    f[3 + t] = act_from_f<A>((float)log1p((double)n * (double)counts[(int64_t)t * n + v] / (double)walkers));
#pragma unroll
  for (int k = GNF; k < GF; ++k) f[k] = act_from_f<A>(0.f);
#pragma unroll
  for (int k = 0; k < GF; ++k) X[v * GF + k] = f[k];
}

template <typename A>
__global__ void gnn_seed_flag_kernel(const int* __restrict__ seeds, int ns, A* __restrict__ X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) X[(int64_t)seeds[i] * GF] = act_from_f<A>(1.f);
}

// --------------------------------------------------------------- layer 1

struct L1Args {
  const int* rowptr;  // CSR(A^T): in-neighbours of each row
  const int* col;
  int n;
  const void* X;
  void* M;
  void* H;
  float* a;
  float* q;
  const float* theta;
  float* hub_sum;  // 16 partial sums per chunk slot
  int* hub_cnt;    // chunks finished per hub (zero; the finisher resets)
};

// This lane's row of the layer weights (lane = hidden unit).
struct L1W {
  float w1s[GNF], w1n[GNF];
  float b1, w2s, w2n, b2;
};

template <typename A>
struct L1Bufs {
  __amdgpu_buffer_rsrc_t x, m, h;
  unsigned voff;  // feature column of lanes 0..15 (others re-read column 0)
};

// Row i of layer 1 from its in-neighbour feature sum s (lanes 0..15), its
// in-degree len and its own features xv (lanes 0..15).
template <typename A>
__device__ __forceinline__ void l1_finish(const L1Args& p, const L1W& w, const L1Bufs<A>& b, int i, float s,
                                          int len, float xv, int lane) {
  const float m = len > 0 ? s / (float)len : 0.f;
  const A mA = act_from_f<A>(m);
  const float mr = act_to_f(mA);
  const unsigned frow = (unsigned)i * (unsigned)(GF * sizeof(A));
  if (lane < GF) buf_store<A>(b.m, mA, b.voff, frow);
  float pre = w.b1;
#pragma unroll
  for (int k = 0; k < GNF; ++k) pre += w.w1s[k] * lane_value(xv, k) + w.w1n[k] * lane_value(mr, k);
  // ReLU that keeps NaN (so a broken network reaches the fallback)
  const A hA = act_from_f<A>(pre > 0.f || __builtin_isnan(pre) ? pre : 0.f);
  const float h = act_to_f(hA);
  buf_store<A>(b.h, hA, (unsigned)lane * (unsigned)sizeof(A), (unsigned)i * (unsigned)(GH * sizeof(A)));
  const float av = wsum(w.w2s * h), qv = wsum(w.w2n * h);
  if (lane == 0) {
    p.a[i] = av + w.b2;
    p.q[i] = qv;
  }
}

template <typename A>
__global__ __launch_bounds__(GB) void gnn_layer1_kernel(TilePlanDev plan, L1Args p) {
  constexpr int TR = WAVE_TILE_ROWS, U = 16;
  __shared__ int srp[GNW][TR + 1];
  const int tid = threadIdx.x, wv = wave_uniform(tid >> 6), lane = tid & 63;
  L1W w;
#pragma unroll
  for (int k = 0; k < GNF; ++k) {
    w.w1s[k] = p.theta[OFF_W1S + lane * GNF + k];
    w.w1n[k] = p.theta[OFF_W1N + lane * GNF + k];
  }
  w.b1 = p.theta[OFF_B1 + lane];
  w.w2s = p.theta[OFF_W2S + lane];
  w.w2n = p.theta[OFF_W2N + lane];
  w.b2 = wave_uniform(p.theta[OFF_B2]);
  constexpr unsigned RB = GF * sizeof(A);  // feature row bytes
  L1Bufs<A> b;
  b.voff = lane < GF ? (unsigned)lane * (unsigned)sizeof(A) : 0u;
  b.x = buf_rsrc(p.X, (unsigned)p.n * RB);
  b.m = buf_rsrc(p.M, (unsigned)p.n * RB);
  b.h = buf_rsrc(p.H, (unsigned)p.n * (unsigned)(GH * sizeof(A)));
  int* wrp = srp[wv];

  const int nwaves = (int)gridDim.x * GNW;
  for (int t = (int)blockIdx.x * GNW + wv; t < plan.ntiles; t += nwaves) {
    const int4 td = tile_desc(plan.tiles, t);
    const int e0 = td.z, ne = td.w;
    int colv = lane < ne ? p.col[e0 + lane] : 0;
    if (td.y > 0) {
      const int row0 = td.x, nr = td.y;
      for (int qq = lane; qq <= nr; qq += 64) wrp[qq] = p.rowptr[row0 + qq] - e0;
      lds_fence_wave();
      int r = 0, rbeg = 0;
      int rend = wave_uniform(wrp[1]);
      float acc = 0.f;
      float xv = act_to_f(buf_load<A>(b.x, b.voff, (unsigned)row0 * RB));
      for (int c0 = 0; c0 < ne; c0 += 64) {
        const int cn = c0 + 64 + lane;
        const int coln = cn < ne ? p.col[e0 + cn] : 0;
#pragma unroll
        for (int hh = 0; hh < 64; hh += U) {
          const int base = c0 + hh;
          if (base >= ne) break;
          float v[U];
#pragma unroll
          for (int u = 0; u < U; ++u)
            v[u] = act_to_f(buf_load<A>(b.x, b.voff, (unsigned)lane_value(colv, hh + u) * RB));
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int e = base + u;
            if (e < ne) {
              while (e == rend) {
                l1_finish<A>(p, w, b, row0 + r, acc, rend - rbeg, xv, lane);
                acc = 0.f;
                ++r;
                rbeg = rend;
                rend = wave_uniform(wrp[r + 1]);
                xv = act_to_f(buf_load<A>(b.x, b.voff, (unsigned)(row0 + r) * RB));
              }
              acc += v[u];
            }
          }
        }
        colv = coln;
      }
      while (r < nr) {  // the last row with entries, then empty rows
        l1_finish<A>(p, w, b, row0 + r, acc, rend - rbeg, xv, lane);
        acc = 0.f;
        ++r;
        if (r < nr) {
          rbeg = rend;
          rend = wave_uniform(wrp[r + 1]);
          xv = act_to_f(buf_load<A>(b.x, b.voff, (unsigned)(row0 + r) * RB));
        }
      }
      lds_fence_wave();  // the next tile rewrites wrp
    } else {
      // one chunk of hub row h: its 16 partial sums, then the last chunk to
      // finish adds them in chunk order and runs the row
      const int h = -td.y - 1;
      float acc = 0.f;
      for (int c0 = 0; c0 < ne; c0 += 64) {
        const int cn = c0 + 64 + lane;
        const int coln = cn < ne ? p.col[e0 + cn] : 0;
#pragma unroll
        for (int hh = 0; hh < 64; hh += U) {
          const int base = c0 + hh;
          if (base >= ne) break;
          float v[U];
#pragma unroll
          for (int u = 0; u < U; ++u)
            v[u] = act_to_f(buf_load<A>(b.x, b.voff, (unsigned)lane_value(colv, hh + u) * RB));
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (base + u < ne) acc += v[u];
        }
        colv = coln;
      }
      const int4 hub = tile_desc(plan.hubs, h);  // {row, nchunks, slot0, -}
      if (lane < GF) publish(&p.hub_sum[(int64_t)(hub.z + td.x) * GF + lane], acc);
      wait_stores();
      int last = 0;
      if (lane == 0) last = counter_add(&p.hub_cnt[h]) == hub.y - 1;
      last = __shfl(last, 0, 64);
      if (last) {
        float s = 0.f;
        for (int c = 0; c < hub.y; ++c)
          s += lane < GF ? consume(&p.hub_sum[(int64_t)(hub.z + c) * GF + lane]) : 0.f;
        const int len = wave_uniform(p.rowptr[hub.x + 1] - p.rowptr[hub.x]);
        const float xv = act_to_f(buf_load<A>(b.x, b.voff, (unsigned)hub.x * RB));
        l1_finish<A>(p, w, b, hub.x, s, len, xv, lane);
        if (lane == 0) publish(&p.hub_cnt[h], 0);
      }
    }
  }
}

// --------------------------------------------------------------- layer 2 and softmax

struct HeadCtrl {
  float zmax;
  int bad;         // a non-finite z, or a normaliser that is not finite and > 0
  double total;    // sum of exp(z - zmax)
  double inv;      // 1 / total
  double loss;     // KL(x* || x0) of the last backward pass
};

template <typename V, int B>
__device__ __forceinline__ V block_reduce(V v, V* red, bool is_max) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const V u = __shfl_xor(v, o, 64);
    v = is_max ? (u > v ? u : v) : v + u;
  }
  if (l == 0) red[w] = v;
  __syncthreads();
  V r = red[0];
  for (int i = 1; i < B / 64; ++i) r = is_max ? (red[i] > r ? red[i] : r) : r + red[i];
  __syncthreads();
  return r;
}

// z = a + (A^T q) / indeg; per-block max and a non-finite flag.
__global__ __launch_bounds__(256) void gnn_head_z_kernel(int64_t n, const float* __restrict__ a,
                                                         const float* __restrict__ s, const int* __restrict__ rowptrT,
                                                         float* __restrict__ z, float* __restrict__ part_max,
                                                         HeadCtrl* ctrl) {
  __shared__ float red[4];
  float mx = -INFINITY;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int len = rowptrT[i + 1] - rowptrT[i];
    const float zi = a[i] + (len > 0 ? s[i] / (float)len : 0.f);
    z[i] = zi;
    if (!isfinite(zi)) bad = true;
    mx = fmaxf(mx, zi);
  }
  if (bad) atomicOr(&ctrl->bad, 1);
  const float bm = block_reduce<float, 256>(mx, red, true);
  if (threadIdx.x == 0) part_max[blockIdx.x] = bm;
}

// e = exp(z - zmax) into x0; per-block FP64 sums.
__global__ __launch_bounds__(256) void gnn_head_exp_kernel(int64_t n, const float* __restrict__ z,
                                                           float* __restrict__ x0, double* __restrict__ part_sum,
                                                           const HeadCtrl* ctrl) {
  __shared__ double red[4];
  const float zmax = ctrl->zmax;
  double sum = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float e = expf(z[i] - zmax);
    x0[i] = e;
    sum += (double)e;
  }
  const double bs = block_reduce<double, 256>(sum, red, false);
  if (threadIdx.x == 0) part_sum[blockIdx.x] = bs;
}

// One workgroup: the max (stage 0) or the normaliser (stage 1) over the
// block partials, in block order.
__global__ __launch_bounds__(1024) void gnn_head_reduce_kernel(int stage, int nparts, const float* part_max,
                                                               const double* part_sum, HeadCtrl* ctrl) {
  __shared__ float rf[16];
  __shared__ double rd[16];
  if (stage == 0) {
    float mx = -INFINITY;
    for (int i = threadIdx.x; i < nparts; i += 1024) mx = fmaxf(mx, part_max[i]);
    const float m = block_reduce<float, 1024>(mx, rf, true);
    if (threadIdx.x == 0) ctrl->zmax = m;
  } else {
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 1024) s += part_sum[i];
    const double t = block_reduce<double, 1024>(s, rd, false);
    if (threadIdx.x == 0) {
      ctrl->total = t;
      const bool ok = !ctrl->bad && isfinite(t) && t > 0.0 && isfinite(ctrl->zmax);
      if (!ok) ctrl->bad = 1;
      ctrl->inv = ok ? 1.0 / t : 0.0;
    }
  }
}

// x0 = e / total, or 0 before the teleport scatter when the output is unusable.
__global__ void gnn_head_norm_kernel(int64_t n, float* __restrict__ x0, const HeadCtrl* ctrl) {
  const int bad = ctrl->bad;
  const double inv = ctrl->inv;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x0[i] = bad ? 0.f : (float)((double)x0[i] * inv);
}

__global__ void gnn_teleport_kernel(const int* __restrict__ seeds, int ns, float* __restrict__ x0,
                                    const HeadCtrl* ctrl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns && ctrl->bad) x0[seeds[i]] = (float)(1.0 / (double)ns);
}

// --------------------------------------------------------------- backward

// gz = x0 - x*, t = gz / indeg (0 without in-neighbours), and per-block
// FP64 partials of KL(x* || x0).
__global__ __launch_bounds__(256) void gnn_gradz_kernel(int64_t n, const float* __restrict__ x0,
                                                        const float* __restrict__ xs, int64_t stride,
                                                        const int* __restrict__ rowptrT, float* __restrict__ gz,
                                                        float* __restrict__ tv, double* __restrict__ part_loss) {
  __shared__ double red[4];
  double loss = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float xi = x0[i], si = xs[i * stride];
    const float g = xi - si;
    const int len = rowptrT[i + 1] - rowptrT[i];
    gz[i] = g;
    tv[i] = len > 0 ? g / (float)len : 0.f;
    if (si > 0.f) loss += (double)si * (log((double)si) - log((double)xi));
  }
  const double b = block_reduce<double, 256>(loss, red, false);
  if (threadIdx.x == 0) part_loss[blockIdx.x] = b;
}

__global__ __launch_bounds__(1024) void gnn_loss_reduce_kernel(int nparts, const double* part_loss, HeadCtrl* ctrl) {
  __shared__ double rd[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 1024) s += part_loss[i];
  const double t = block_reduce<double, 1024>(s, rd, false);
  if (threadIdx.x == 0) ctrl->loss = t;
}

// Weight gradients: each wavefront takes vertices round-robin and
// accumulates, lane j = hidden unit j, its row of every gradient in FP64.
// The waves of a workgroup are combined in wave order in LDS and each
// workgroup writes its partial; gnn_wgrad_final adds them in order.
template <typename A>
__global__ __launch_bounds__(GB) void gnn_wgrad_kernel(int64_t n, const void* __restrict__ Xv,
                                                       const void* __restrict__ Mv, const void* __restrict__ Hv,
                                                       const float* __restrict__ gz, const float* __restrict__ gq,
                                                       const float* __restrict__ theta, double* __restrict__ part) {
  __shared__ double red[NPARAM];
  const int tid = threadIdx.x, wv = wave_uniform(tid >> 6), lane = tid & 63;
  const A* X = (const A*)Xv;
  const A* M = (const A*)Mv;
  const A* H = (const A*)Hv;
  const float w2s = theta[OFF_W2S + lane], w2n = theta[OFF_W2N + lane];
  double gw1s[GNF], gw1n[GNF];
#pragma unroll
  for (int k = 0; k < GNF; ++k) gw1s[k] = gw1n[k] = 0.0;
  double gb1 = 0.0, gw2s = 0.0, gw2n = 0.0, gb2 = 0.0;
  const int64_t nw = (int64_t)gridDim.x * GNW;
  for (int64_t v = (int64_t)blockIdx.x * GNW + wv; v < n; v += nw) {
    const float h = act_to_f(H[v * GH + lane]);
    const float xk = lane < GF ? act_to_f(X[v * GF + lane]) : 0.f;
    const float mk = lane < GF ? act_to_f(M[v * GF + lane]) : 0.f;
    const float ga = wave_uniform(gz[v]), gqv = wave_uniform(gq[v]);
    gw2s += (double)ga * (double)h;
    gw2n += (double)gqv * (double)h;
    gb2 += (double)ga;
    const float gh = ga * w2s + gqv * w2n;
    const double gp = h > 0.f ? (double)gh : 0.0;
    gb1 += gp;
#pragma unroll
    for (int k = 0; k < GNF; ++k) {
      gw1s[k] += gp * (double)lane_value(xk, k);
      gw1n[k] += gp * (double)lane_value(mk, k);
    }
  }
  for (int w = 0; w < GNW; ++w) {
    if (wv == w) {
#pragma unroll
      for (int k = 0; k < GNF; ++k) {
        double* a1 = &red[OFF_W1S + lane * GNF + k];
        double* a2 = &red[OFF_W1N + lane * GNF + k];
        *a1 = (w == 0 ? 0.0 : *a1) + gw1s[k];
        *a2 = (w == 0 ? 0.0 : *a2) + gw1n[k];
      }
      red[OFF_B1 + lane] = (w == 0 ? 0.0 : red[OFF_B1 + lane]) + gb1;
      red[OFF_W2S + lane] = (w == 0 ? 0.0 : red[OFF_W2S + lane]) + gw2s;
      red[OFF_W2N + lane] = (w == 0 ? 0.0 : red[OFF_W2N + lane]) + gw2n;
      if (lane == 0) red[OFF_B2] = (w == 0 ? 0.0 : red[OFF_B2]) + gb2;
    }
    __syncthreads();
  }
  for (int i = tid; i < NPARAM; i += GB) part[(int64_t)blockIdx.x * NPARAM + i] = red[i];
}

__global__ void gnn_wgrad_final_kernel(int nparts, const double* __restrict__ part, double* __restrict__ grad,
                                       int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * NPARAM + i];
  grad[i] = accumulate ? grad[i] + s : s;
}

// Adam (Kingma & Ba, 2015) on grad * scale, step t >= 1, in FP64.
__global__ void gnn_adam_kernel(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                                const double* __restrict__ grad, int64_t t, double lr, double b1, double b2,
                                double eps, double scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  const double g = grad[i] * scale;
  const double mi = b1 * (double)m[i] + (1.0 - b1) * g;
  const double vi = b2 * (double)v[i] + (1.0 - b2) * g * g;
  m[i] = (float)mi;
  v[i] = (float)vi;
  const double mh = mi / (1.0 - pow(b1, (double)t));
  const double vh = vi / (1.0 - pow(b2, (double)t));
  theta[i] = (float)((double)theta[i] - lr * mh / (sqrt(vh) + eps));
}

__global__ void gnn_to_vector_kernel(int64_t n, const float* __restrict__ x0, void* out, int type) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (type == T_FP32)
      ((float*)out)[i] = x0[i];
    else
      ((double*)out)[i] = (double)x0[i];
  }
}

int blocks_for(int64_t n, int threads, int cap) {
  int64_t b = (n + threads - 1) / threads;
  if (b > cap) b = cap;
  return b < 1 ? 1 : (int)b;
}

}  // namespace
}  // namespace nbgrb

// ============================================================= host side

using namespace nbgrb;

static constexpr uint32_t MAGIC_GNN = 0x474e4e31u;  // "GNN1"
static constexpr int HEAD_PARTS = 1024;             // partial slots of the head reductions

struct GB_GNN_opaque {
  uint32_t magic = MAGIC_GNN;
  int act = T_FP32;
  BufP theta, adam_m, adam_v, grad;
  int64_t adam_t = 0;
  // work space of the graph last used
  int64_t n = 0;
  uint64_t graph_id = 0;
  bool have_features = false, have_forward = false;
  BufP counts, X, M, H, a, q, s, z, x0, gz, tv, gq, seeds, ctrl, part_max, part_sum, part_w, hub_sum, hub_cnt;
  int nseeds = 0;
  int hub_slots = 0, hub_hubs = 0;
};

namespace {

#define GNN_BEGIN try {
#define GNN_END                            \
  }                                        \
  catch (const GrbError& e) {              \
    set_error_text(e.msg);                 \
    return e.info;                         \
  }                                        \
  catch (const std::bad_alloc&) {          \
    set_error_text("host allocation failed"); \
    return GrB_OUT_OF_MEMORY;              \
  }                                        \
  catch (const std::exception& e) {        \
    set_error_text(e.what());              \
    return GrB_PANIC;                      \
  }                                        \
  return GrB_SUCCESS;

GB_GNN_opaque* net_of(GrM_GNN net) {
  if (!net) fail(GrB_NULL_POINTER, "network is NULL");
  if (net->magic != MAGIC_GNN) fail(GrB_UNINITIALIZED_OBJECT, "not a network");
  return net;
}

MatP mat_of(GrB_Matrix A, const char* what) {
  if (!A) fail(GrB_NULL_POINTER, std::string(what) + " is NULL");
  if (A->magic != MAGIC_MAT) fail(GrB_UNINITIALIZED_OBJECT, std::string(what) + " is not a matrix");
  return A->data;
}

// A (rows = sources) and A^T of one square graph.
void check_pair(const MatP& A, const MatP& AT) {
  if (A->nrows != A->ncols || AT->nrows != AT->ncols || A->nrows != AT->nrows)
    fail(GrB_DIMENSION_MISMATCH, "A and A^T must be square and of the same size");
  if (A->nnz != AT->nnz) fail(GrB_DIMENSION_MISMATCH, "A and A^T must have the same number of entries");
  if (A->nrows * (int64_t)(GH * sizeof(float)) >= (int64_t)0xFFFFFF00ll)
    fail(GrB_INVALID_VALUE, "graph too large for the network's 32-bit buffer offsets");
}

void ensure_graph(GB_GNN_opaque* g, const MatP& A, const MatP& AT) {
  check_pair(A, AT);
  const int64_t n = AT->nrows;
  if (g->n == n && g->graph_id == AT->id && g->X) return;
  const size_t as = type_size(g->act);
  g->n = n;
  g->graph_id = AT->id;
  g->have_features = g->have_forward = false;
  g->counts = dev_alloc(sizeof(int) * GSTEPS * (size_t)n);
  g->X = dev_alloc(as * GF * (size_t)n);
  g->M = dev_alloc(as * GF * (size_t)n);
  g->H = dev_alloc(as * GH * (size_t)n);
  for (BufP* b : {&g->a, &g->q, &g->s, &g->z, &g->x0, &g->gz, &g->tv, &g->gq}) *b = dev_alloc(sizeof(float) * (size_t)n);
}

PlanConfig layer1_plan_config() {
  PlanConfig wp;
  wp.kernel = K_WAVE;
  wp.lds_entries = WAVE_TILE_ENTRIES;
  wp.lds_rows = WAVE_TILE_ROWS;
  wp.long_row = WAVE_TILE_ENTRIES;
  wp.chunk = WAVE_TILE_ENTRIES;
  wp.grid = ctx().cus * 2;
  return wp;
}

void run_layer1(GB_GNN_opaque* g, const MatP& AT) {
  Ctx& c = ctx();
  auto plan = get_plan(AT, layer1_plan_config());
  if (plan->nparts > g->hub_slots) {
    g->hub_sum = dev_alloc(sizeof(float) * GF * (size_t)plan->nparts);
    g->hub_slots = plan->nparts;
  }
  if (!g->hub_cnt || plan->nhubs > g->hub_hubs) {
    g->hub_hubs = std::max(plan->nhubs, 1);
    g->hub_cnt = dev_alloc(sizeof(int) * (size_t)g->hub_hubs);
    hip_check(launch_zero(g->hub_cnt->p, sizeof(int) * (size_t)g->hub_hubs, c.stream), "zero");
    launch_mark(false);
  }
  L1Args p{};
  p.rowptr = (const int*)AT->rowptr->p;
  p.col = AT->col ? (const int*)AT->col->p : nullptr;
  p.n = (int)g->n;
  p.X = g->X->p;
  p.M = g->M->p;
  p.H = g->H->p;
  p.a = (float*)g->a->p;
  p.q = (float*)g->q->p;
  p.theta = (const float*)g->theta->p;
  p.hub_sum = g->hub_sum ? (float*)g->hub_sum->p : nullptr;
  p.hub_cnt = (int*)g->hub_cnt->p;
  if (plan->dev.ntiles > 0) {
    if (g->act == T_FP32)
      hipLaunchKernelGGL(gnn_layer1_kernel<float>, dim3(plan->cfg.grid), dim3(GB), 0, c.stream, plan->dev, p);
    else
      hipLaunchKernelGGL(gnn_layer1_kernel<bf16>, dim3(plan->cfg.grid), dim3(GB), 0, c.stream, plan->dev, p);
    hip_check(hipGetLastError(), "layer 1");
    launch_mark(false);
  }
}

void run_head(GB_GNN_opaque* g, const MatP& AT) {
  Ctx& c = ctx();
  const int64_t n = g->n;
  if (!g->ctrl) {
    g->ctrl = dev_alloc(sizeof(HeadCtrl));
    g->part_max = dev_alloc(sizeof(float) * HEAD_PARTS);
    g->part_sum = dev_alloc(sizeof(double) * HEAD_PARTS);
  }
  mxv_now(AT, T_FP32, g->q->p, g->s->p);
  HeadCtrl* ctrl = (HeadCtrl*)g->ctrl->p;
  hip_check(launch_zero(ctrl, sizeof(HeadCtrl), c.stream), "zero");
  const int nb = blocks_for(n, 256, HEAD_PARTS);
  hipLaunchKernelGGL(gnn_head_z_kernel, dim3(nb), dim3(256), 0, c.stream, n, (const float*)g->a->p,
                     (const float*)g->s->p, (const int*)AT->rowptr->p, (float*)g->z->p, (float*)g->part_max->p,
                     ctrl);
  hipLaunchKernelGGL(gnn_head_reduce_kernel, dim3(1), dim3(1024), 0, c.stream, 0, nb, (const float*)g->part_max->p,
                     (const double*)g->part_sum->p, ctrl);
  hipLaunchKernelGGL(gnn_head_exp_kernel, dim3(nb), dim3(256), 0, c.stream, n, (const float*)g->z->p,
                     (float*)g->x0->p, (double*)g->part_sum->p, (const HeadCtrl*)ctrl);
  hipLaunchKernelGGL(gnn_head_reduce_kernel, dim3(1), dim3(1024), 0, c.stream, 1, nb, (const float*)g->part_max->p,
                     (const double*)g->part_sum->p, ctrl);
  hipLaunchKernelGGL(gnn_head_norm_kernel, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, c.stream, n,
                     (float*)g->x0->p, (const HeadCtrl*)ctrl);
  hipLaunchKernelGGL(gnn_teleport_kernel, dim3(blocks_for(g->nseeds, 256, 1 << 20)), dim3(256), 0, c.stream,
                     (const int*)g->seeds->p, g->nseeds, (float*)g->x0->p, (const HeadCtrl*)ctrl);
  hip_check(hipGetLastError(), "head");
  for (int i = 0; i < 7; ++i) launch_mark(false);
}

int read_bad(GB_GNN_opaque* g) {
  HeadCtrl h{};
  hip_check(hipMemcpyAsync(&h, g->ctrl->p, sizeof(h), hipMemcpyDeviceToHost, ctx().stream), "read head");
  hip_check(hipStreamSynchronize(ctx().stream), "sync");
  return h.bad;
}

// Glorot-uniform weights from the SplitMix64 stream (draw i -> parameter
// i), zero biases.
uint64_t host_splitmix(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void upload_params(GB_GNN_opaque* g, const float* host) {
  Ctx& c = ctx();
  hip_check(hipMemcpyAsync(g->theta->p, host, sizeof(float) * NPARAM, hipMemcpyHostToDevice, c.stream), "params");
  hip_check(launch_zero(g->adam_m->p, sizeof(float) * NPARAM, c.stream), "zero");
  hip_check(launch_zero(g->adam_v->p, sizeof(float) * NPARAM, c.stream), "zero");
  hip_check(launch_zero(g->grad->p, sizeof(double) * NPARAM, c.stream), "zero");
  for (int i = 0; i < 3; ++i) launch_mark(false);
  g->adam_t = 0;
  hip_check(hipStreamSynchronize(c.stream), "sync");
}

}  // namespace

extern "C" {

GrB_Info GrM_GNN_new(GrM_GNN* net, GrB_Type act, uint64_t init_seed) {
  GNN_BEGIN
  require_init();
  if (!net || !act) fail(GrB_NULL_POINTER, "NULL argument");
  if (act->code != T_FP32 && act->code != T_BF16) fail(GrB_DOMAIN_MISMATCH, "activations must be FP32 or BF16");
  auto* g = new GB_GNN_opaque();
  g->act = act->code;
  g->theta = dev_alloc(sizeof(float) * NPARAM);
  g->adam_m = dev_alloc(sizeof(float) * NPARAM);
  g->adam_v = dev_alloc(sizeof(float) * NPARAM);
  g->grad = dev_alloc(sizeof(double) * NPARAM);
  std::vector<float> th(NPARAM, 0.f);
  const double lim1 = std::sqrt(6.0 / (GNF + GH)), lim2 = std::sqrt(6.0 / (GH + 1));
  for (int i = 0; i < NPARAM; ++i) {
    const double u = (double)(host_splitmix(init_seed, (uint64_t)i) >> 11) * 0x1.0p-53;
    if (i < OFF_B1) th[i] = (float)((2.0 * u - 1.0) * lim1);
    else if (i >= OFF_W2S && i < OFF_B2) th[i] = (float)((2.0 * u - 1.0) * lim2);
  }
  upload_params(g, th.data());
  *net = g;
  GNN_END
}

GrB_Info GrM_GNN_free(GrM_GNN* net) {
  GNN_BEGIN
  if (!net || !*net) return GrB_SUCCESS;
  if ((*net)->magic != MAGIC_GNN) fail(GrB_UNINITIALIZED_OBJECT, "not a network");
  if (ctx().init) hip_check(hipStreamSynchronize(ctx().stream), "sync");
  (*net)->magic = 0;
  delete *net;
  *net = nullptr;
  GNN_END
}

GrB_Info GrM_GNN_set_params(GrM_GNN net, const float* theta) {
  GNN_BEGIN
  require_init();
  GB_GNN_opaque* g = net_of(net);
  if (!theta) fail(GrB_NULL_POINTER, "theta is NULL");
  upload_params(g, theta);
  g->have_forward = false;
  GNN_END
}

GrB_Info GrM_GNN_get_params(GrM_GNN net, float* theta) {
  GNN_BEGIN
  require_init();
  GB_GNN_opaque* g = net_of(net);
  if (!theta) fail(GrB_NULL_POINTER, "theta is NULL");
  hip_check(hipMemcpyAsync(theta, g->theta->p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, ctx().stream), "copy");
  hip_check(hipStreamSynchronize(ctx().stream), "sync");
  GNN_END
}

GrB_Info GrM_GNN_get_grad(GrM_GNN net, double* grad) {
  GNN_BEGIN
  require_init();
  GB_GNN_opaque* g = net_of(net);
  if (!grad) fail(GrB_NULL_POINTER, "grad is NULL");
  hip_check(hipMemcpyAsync(grad, g->grad->p, sizeof(double) * NPARAM, hipMemcpyDeviceToHost, ctx().stream), "copy");
  hip_check(hipStreamSynchronize(ctx().stream), "sync");
  GNN_END
}

GrB_Info GrM_GNN_buffer(GrM_GNN net, int which, void** ptr, int64_t* count) {
  GNN_BEGIN
  require_init();
  GB_GNN_opaque* g = net_of(net);
  if (!ptr) fail(GrB_NULL_POINTER, "ptr is NULL");
  if (!g->X) fail(GrB_INVALID_OBJECT, "no graph has been used with this network");
  const int64_t n = g->n;
  struct B {
    BufP b;
    int64_t c;
  };
  B tab[] = {{g->counts, GSTEPS * n}, {g->X, GF * n}, {g->M, GF * n}, {g->H, GH * n}, {g->a, n},
             {g->q, n}, {g->z, n}, {g->x0, n}, {g->gq, n}};
  if (which < 0 || which >= (int)(sizeof(tab) / sizeof(tab[0]))) fail(GrB_INVALID_VALUE, "unknown buffer");
  hip_check(hipStreamSynchronize(ctx().stream), "sync");
  *ptr = tab[which].b->p;
  if (count) *count = tab[which].c;
  GNN_END
}

GrB_Info GrM_gnn_features(GrM_GNN net, GrB_Matrix A, GrB_Matrix AT, const int32_t* seeds, int nseeds, int walkers,
                          double damping, uint64_t seed) {
  GNN_BEGIN
  require_init();
  GB_GNN_opaque* g = net_of(net);
  const MatP a = mat_of(A, "A"), at = mat_of(AT, "AT");
  if (!seeds) fail(GrB_NULL_POINTER, "seeds is NULL");
  if (nseeds < 1) fail(GrB_INVALID_VALUE, "the seed set is empty");
  if (walkers < 1 || walkers > (1 << 26)) fail(GrB_INVALID_VALUE, "walkers must be in [1, 2^26]");
  if (!(damping >= 0.0 && damping <= 1.0)) fail(GrB_INVALID_VALUE, "damping must be in [0, 1]");
  ensure_graph(g, a, at);
  std::vector<int> s(seeds, seeds + nseeds);
  std::vector<int> sorted(s);
  std::sort(sorted.begin(), sorted.end());
  if (sorted.front() < 0 || sorted.back() >= g->n) fail(GrB_INVALID_INDEX, "seed vertex out of range");
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) fail(GrB_INVALID_VALUE, "repeated seed");
  Ctx& c = ctx();
  if (!g->seeds || g->nseeds < nseeds) g->seeds = dev_alloc(sizeof(int) * (size_t)nseeds);
  g->nseeds = nseeds;
  hip_check(hipMemcpyAsync(g->seeds->p, s.data(), sizeof(int) * (size_t)nseeds, hipMemcpyHostToDevice, c.stream),
            "seeds");
  const int64_t n = g->n;
  hip_check(launch_zero(g->counts->p, sizeof(int) * GSTEPS * (size_t)n, c.stream), "zero");
  hipLaunchKernelGGL(gnn_walk_kernel, dim3((walkers + 255) / 256), dim3(256), 0, c.stream,
                     (const int*)a->rowptr->p, a->col ? (const int*)a->col->p : nullptr, (const int*)g->seeds->p,
                     nseeds, walkers, damping, seed, (int*)g->counts->p, n);
  const int fb = (int)((n + 255) / 256);
  if (g->act == T_FP32) {
    hipLaunchKernelGGL(gnn_features_kernel<float>, dim3(fb), dim3(256), 0, c.stream, n, (const int*)a->rowptr->p,
                       (const int*)at->rowptr->p, (const int*)g->counts->p, walkers, (float*)g->X->p);
    hipLaunchKernelGGL(gnn_seed_flag_kernel<float>, dim3((nseeds + 255) / 256), dim3(256), 0, c.stream,
                       (const int*)g->seeds->p, nseeds, (float*)g->X->p);
  } else {
    hipLaunchKernelGGL(gnn_features_kernel<bf16>, dim3(fb), dim3(256), 0, c.stream, n, (const int*)a->rowptr->p,
                       (const int*)at->rowptr->p, (const int*)g->counts->p, walkers, (bf16*)g->X->p);
    hipLaunchKernelGGL(gnn_seed_flag_kernel<bf16>, dim3((nseeds + 255) / 256), dim3(256), 0, c.stream,
                       (const int*)g->seeds->p, nseeds, (bf16*)g->X->p);
  }
  hip_check(hipGetLastError(), "features");
  for (int i = 0; i < 4; ++i) launch_mark(false);
  g->have_features = true;
  g->have_forward = false;
  GNN_END
}

GrB_Info GrM_gnn_forward(GrM_GNN net, GrB_Matrix A, GrB_Matrix AT, int* fell_back) {
  GNN_BEGIN
  require_init();
  GB_GNN_opaque* g = net_of(net);
  const MatP a = mat_of(A, "A"), at = mat_of(AT, "AT");
  check_pair(a, at);
  if (!g->have_features || g->graph_id != at->id) fail(GrB_INVALID_OBJECT, "run GrM_gnn_features on this graph first");
  run_layer1(g, at);
  run_head(g, at);
  g->have_forward = true;
  if (fell_back) *fell_back = read_bad(g);
  GNN_END
}

GrB_Info GrM_gnn_backward(GrM_GNN net, GrB_Matrix A, GrB_Matrix AT, const float* x_star, int64_t stride,
                          int accumulate, double* loss) {
  GNN_BEGIN
  require_init();
  GB_GNN_opaque* g = net_of(net);
  const MatP a = mat_of(A, "A"), at = mat_of(AT, "AT");
  check_pair(a, at);
  if (!x_star) fail(GrB_NULL_POINTER, "x_star is NULL");
  if (stride < 1) fail(GrB_INVALID_VALUE, "stride must be >= 1");
  if (!g->have_forward || g->graph_id != at->id) fail(GrB_INVALID_OBJECT, "run GrM_gnn_forward on this graph first");
  Ctx& c = ctx();
  const int64_t n = g->n;
  const int nb = blocks_for(n, 256, HEAD_PARTS);
  hipLaunchKernelGGL(gnn_gradz_kernel, dim3(nb), dim3(256), 0, c.stream, n, (const float*)g->x0->p, x_star, stride,
                     (const int*)at->rowptr->p, (float*)g->gz->p, (float*)g->tv->p, (double*)g->part_sum->p);
  hipLaunchKernelGGL(gnn_loss_reduce_kernel, dim3(1), dim3(1024), 0, c.stream, nb, (const double*)g->part_sum->p,
                     (HeadCtrl*)g->ctrl->p);
  launch_mark(false);
  launch_mark(false);
  mxv_now(a, T_FP32, g->tv->p, g->gq->p);
  const int wb = c.cus;
  if (!g->part_w) g->part_w = dev_alloc(sizeof(double) * NPARAM * (size_t)wb);
  if (g->act == T_FP32)
    hipLaunchKernelGGL(gnn_wgrad_kernel<float>, dim3(wb), dim3(GB), 0, c.stream, n, g->X->p, g->M->p, g->H->p,
                       (const float*)g->gz->p, (const float*)g->gq->p, (const float*)g->theta->p,
                       (double*)g->part_w->p);
  else
    hipLaunchKernelGGL(gnn_wgrad_kernel<bf16>, dim3(wb), dim3(GB), 0, c.stream, n, g->X->p, g->M->p, g->H->p,
                       (const float*)g->gz->p, (const float*)g->gq->p, (const float*)g->theta->p,
                       (double*)g->part_w->p);
  hipLaunchKernelGGL(gnn_wgrad_final_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, c.stream, wb,
                     (const double*)g->part_w->p, (double*)g->grad->p, accumulate ? 1 : 0);
  hip_check(hipGetLastError(), "backward");
  launch_mark(false);
  launch_mark(false);
  if (loss) {
    HeadCtrl h{};
    hip_check(hipMemcpyAsync(&h, g->ctrl->p, sizeof(h), hipMemcpyDeviceToHost, c.stream), "read loss");
    hip_check(hipStreamSynchronize(c.stream), "sync");
    *loss = h.loss;
  }
  GNN_END
}

GrB_Info GrM_gnn_adam_step(GrM_GNN net, double lr, double beta1, double beta2, double eps, double grad_scale) {
  GNN_BEGIN
  require_init();
  GB_GNN_opaque* g = net_of(net);
  if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    fail(GrB_INVALID_VALUE, "Adam needs lr > 0, 0 <= beta < 1 and eps > 0");
  ++g->adam_t;
  hipLaunchKernelGGL(gnn_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, ctx().stream, (float*)g->theta->p,
                     (float*)g->adam_m->p, (float*)g->adam_v->p, (const double*)g->grad->p, g->adam_t, lr, beta1,
                     beta2, eps, grad_scale);
  hip_check(hipGetLastError(), "adam");
  launch_mark(false);
  g->have_forward = false;
  GNN_END
}

GrB_Info GrM_gnn_predict_x0(GrB_Vector x0, GrM_GNN net, GrB_Matrix A, GrB_Matrix AT, const int32_t* seeds,
                            int nseeds, int walkers, double damping, uint64_t seed, int* fell_back) {
  GNN_BEGIN
  require_init();
  if (!x0) fail(GrB_NULL_POINTER, "x0 is NULL");
  if (x0->magic != MAGIC_VEC) fail(GrB_UNINITIALIZED_OBJECT, "x0 is not a vector");
  if (x0->type != T_FP32 && x0->type != T_FP64) fail(GrB_DOMAIN_MISMATCH, "x0 must be FP32 or FP64");
  GrB_Info info = GrM_gnn_features(net, A, AT, seeds, nseeds, walkers, damping, seed);
  if (info != GrB_SUCCESS) return info;
  info = GrM_gnn_forward(net, A, AT, fell_back);
  if (info != GrB_SUCCESS) return info;
  GB_GNN_opaque* g = net_of(net);
  if (x0->n != g->n) fail(GrB_DIMENSION_MISMATCH, "x0 length differs from the graph's");
  NodeP p = new_node(N_DENSE, x0->type, x0->n, false);
  p->buf = dev_alloc(type_size(x0->type) * (size_t)x0->n);
  hipLaunchKernelGGL(gnn_to_vector_kernel, dim3(blocks_for(g->n, 256, 4096)), dim3(256), 0, ctx().stream, g->n,
                     (const float*)g->x0->p, p->buf->p, x0->type);
  hip_check(hipGetLastError(), "x0 copy");
  launch_mark(false);
  p->done = true;
  set_vec(x0, p);
  GNN_END
}

}  // extern "C"
