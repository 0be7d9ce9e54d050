// Many independent PageRank problems in one persistent launch.
//
// Every workgroup (1024 threads, one per compute unit) takes work from a
// queue: first the graphs large enough to be solved by a team of
// workgroups (one queue slot per member), then whole graphs, largest first.
// A single workgroup runs the fused pass on its graph until the graph's own
// residual reaches the tolerance and never waits for another workgroup.
// The members of a team split the rows of every pass between them and meet
// at a barrier of their own after it: they publish their residual and
// dangling partial sums, wait until every member has arrived, and add the
// partials in member order, so every member takes the same loop decision.
// Team slots come first and number at most the grid, so every member is
// running when the first barrier is reached; a wait still gives up after a
// bounded time (ten seconds unless set lower) and flags the launch as
// failed instead of hanging.
// Inside a graph the vertices are numbered by decreasing out-degree, so the
// leading slice of the gathered vector -- all of it for graphs up to the LDS
// capacity -- is kept in LDS and refreshed after every pass.  Rows are
// reduced by groups of lanes (a power of two per graph from its mean
// degree) with shuffles, rows longer than MANY_LONG_ROW by one wavefront
// each; the residual and the dangling mass are summed in FP64 in a fixed
// order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "device_util.h"
#include "kernels.h"

namespace nbgrb {

namespace {

constexpr int MB = 1024;
constexpr int MNW = MB / 64;

template <typename T>
struct ManyLds;
template <>
struct ManyLds<float> {
  static constexpr int H = 36864;  // 144 KiB
};
template <>
struct ManyLds<double> {
  static constexpr int H = 18432;  // 144 KiB
};

template <typename V>
__device__ __forceinline__ V wsum(V v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-tree sum over the workgroup, returned to every thread.
__device__ __forceinline__ double bsum(double v, double* red, double* out) {
  v = wsum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < MNW; ++i) s += red[i];
    *out = s;
  }
  __syncthreads();
  const double r = *out;
  __syncthreads();
  return r;
}

// Thread 0: wait until *bar reaches target; false, with *err set, when the
// wait runs out (after `ticks` of the 100 MHz wall clock).
__device__ bool team_wait(unsigned* bar, unsigned target, int* err, uint64_t ticks) {
  const uint64_t t0 = wall_clock64();
  while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (wall_clock64() - t0 > ticks) {
      __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

// Team barrier (every thread calls it): this workgroup's global writes are
// released, its arrival counted, and once all members have arrived their
// writes are acquired (which also drops this compute unit's stale cached
// lines of the shared vectors).  False when the wait ran out.
__device__ bool team_sync(unsigned* bar, unsigned target, int* err, uint64_t ticks, int* sflag) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    *sflag = team_wait(bar, target, err, ticks) ? 1 : 0;
  }
  __syncthreads();
  const bool ok = *sflag != 0;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok;
}

template <typename T>
__global__ __launch_bounds__(MB) void pr_many_kernel(ManyArgs p) {
  constexpr int HM = ManyLds<T>::H;
  constexpr int RPG = 4;  // rows per lane group and step (register budget)
  __shared__ T hot[HM];
  __shared__ double red[MNW];
  __shared__ double bcast;
  __shared__ int sq, sflag;
  const int tid = threadIdx.x;

  for (;;) {
    if (tid == 0) sq = __hip_atomic_fetch_add(p.queue_next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int q = sq;
    __syncthreads();
    if (q >= p.nslots) break;
    const int gi = p.queue[q] / MANY_MAX_TEAM, mk = p.queue[q] % MANY_MAX_TEAM;
    const ManyGraph G = p.graphs[gi];
    const int team = G.team;
    unsigned* bar = p.team_bar + gi;
    double* part = p.team_part + (int64_t)gi * (4 * MANY_MAX_TEAM);
    unsigned gen = 0;
    const int n = G.n;
    const int* rp = p.rowptr + G.roff;
    const int* col = p.col + G.eoff;
    const int* deg = p.deg + G.voff;
    T* xa = (T*)p.xa + G.voff;
    T* xb = (T*)p.xb + G.voff;
    T* wa = (T*)p.wa + G.voff;
    T* wb = (T*)p.wb + G.voff;
    const int H = n < HM ? n : HM;
    const int lpr = G.lpr;
    const int groups = MB / lpr;
    const int grp = tid / lpr, sub = tid & (lpr - 1);
    const T dmp = (T)p.damping;

    // start: x = 1/n, w = x .* d, D = mass on dangling vertices (every
    // member computes D and its slice itself, and stores its share of x, w)
    double dl = 0.0;
    const T x0 = (T)(1.0 / (double)n);
    for (int i = tid; i < n; i += MB) {
      const int dg = deg[i];
      const T dv = dg > 0 ? dmp * ((T)1 / (T)dg) : (T)0;
      const T wv = x0 * dv;
      if ((i / MB) % team == mk) {
        xa[i] = x0;
        wa[i] = wv;
      }
      if (i < H) hot[i] = wv;
      if (dg == 0) dl += (double)x0;
    }
    double D = bsum(dl, red, &bcast);
    if (team > 1 && !team_sync(bar, ++gen * (unsigned)team, p.team_err, p.team_wait_ticks, &sflag)) return;
    double rho = 1.0;
    int it = 0;
    T* xc = xa;
    T* xn = xb;
    T* wc = wa;
    T* wn = wb;
    while (it < p.itermax && rho > p.tol) {
      const double cd = (1.0 - p.damping) / (double)n + (p.uniform ? p.damping * D / (double)n : 0.0);
      const T c = (T)cd;
      double rl = 0.0, dn = 0.0;
      // RPG rows per lane group and step: their row bounds, old ranks and
      // degrees, then their column indices and gathers, are issued together
      // (out-of-range lanes load nothing), so one step waits for a few
      // memory latencies instead of a few per row
      const __amdgpu_buffer_rsrc_t rrp = buf_rsrc(rp, (unsigned)(n + 1) * 4u);
      const __amdgpu_buffer_rsrc_t rcol = buf_rsrc(col, (unsigned)G.m * 4u);
      const __amdgpu_buffer_rsrc_t rw = buf_rsrc(wc, (unsigned)n * (unsigned)sizeof(T));
      const __amdgpu_buffer_rsrc_t rx = buf_rsrc(xc, (unsigned)n * (unsigned)sizeof(T));
      const __amdgpu_buffer_rsrc_t rdg = buf_rsrc(deg, (unsigned)n * 4u);
      for (int base = mk * groups * RPG; base < n; base += team * groups * RPG) {
        int lo[RPG], len[RPG], dg[RPG];
        T xo[RPG], s[RPG];
#pragma unroll
        for (int k = 0; k < RPG; ++k) {
          const int row = base + grp + k * groups;
          const unsigned off = row < n ? (unsigned)row * 4u : BUF_SKIP;
          lo[k] = buf_load<int>(rrp, off);
          len[k] = buf_load<int>(rrp, off, 4u);
          dg[k] = buf_load<int>(rdg, off);
          xo[k] = buf_load<T>(rx, row < n ? (unsigned)row * (unsigned)sizeof(T) : BUF_SKIP);
        }
        int maxlen = 0;
#pragma unroll
        for (int k = 0; k < RPG; ++k) {
          len[k] -= lo[k];
          // long rows: second phase
          if (base + grp + k * groups >= n || len[k] > MANY_LONG_ROW) len[k] = -1;
          maxlen = len[k] > maxlen ? len[k] : maxlen;
          s[k] = 0;
        }
        for (int t = sub; t < maxlen; t += lpr) {
          int j[RPG];
#pragma unroll
          for (int k = 0; k < RPG; ++k) j[k] = buf_load<int>(rcol, t < len[k] ? (unsigned)(lo[k] + t) * 4u : BUF_SKIP);
#pragma unroll
          for (int k = 0; k < RPG; ++k) {
            const bool v = t < len[k];
            const bool h = j[k] < H;
            const T g = buf_load<T>(rw, v && !h ? (unsigned)j[k] * (unsigned)sizeof(T) : BUF_SKIP);
            const T hv = hot[h ? j[k] : 0];
            if (v) s[k] += h ? hv : g;
          }
        }
#pragma unroll
        for (int k = 0; k < RPG; ++k) {
          T sk = s[k];
          for (int o = lpr >> 1; o > 0; o >>= 1) sk += __shfl_xor(sk, o, 64);
          const int row = base + grp + k * groups;
          if (sub == 0 && len[k] >= 0) {
            const T r = c + sk;
            const T dv = dg[k] > 0 ? dmp * ((T)1 / (T)dg[k]) : (T)0;
            xn[row] = r;
            wn[row] = r * dv;
            rl += fabs((double)xo[k] - (double)r);
            if (dg[k] == 0) dn += (double)r;
          }
        }
      }
      // long rows: one wavefront per row, sixteen rows at a time, four
      // loads per lane in flight; the row's sum is a fixed tree
      {
        const int wv = tid >> 6, lane = tid & 63;
        for (int lq = wv + MNW * mk; lq < G.nlong; lq += MNW * team) {
          const int row = p.longrows[G.loff + lq];
          const int e0 = rp[row], e1 = rp[row + 1];
          T sl = 0;
          for (int e = e0 + lane; e < e1; e += 256) {
            int j[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) j[k] = buf_load<int>(rcol, e + 64 * k < e1 ? (unsigned)(e + 64 * k) * 4u : BUF_SKIP);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const bool v = e + 64 * k < e1;
              const bool h = j[k] < H;
              const T g = buf_load<T>(rw, v && !h ? (unsigned)j[k] * (unsigned)sizeof(T) : BUF_SKIP);
              const T hv = hot[h ? j[k] : 0];
              if (v) sl += h ? hv : g;
            }
          }
          sl = wsum(sl);
          if (lane == 0) {
            const T r = c + sl;
            const T xo = xc[row];
            const int dg = deg[row];
            const T dv = dg > 0 ? dmp * ((T)1 / (T)dg) : (T)0;
            xn[row] = r;
            wn[row] = r * dv;
            rl += fabs((double)xo - (double)r);
            if (dg == 0) dn += (double)r;
          }
        }
      }
      __syncthreads();  // every row of the pass is written
      const double brl = bsum(rl, red, &bcast);
      const double bdn = bsum(dn, red, &bcast);
      if (team == 1) {
        rho = brl;
        D = bdn;
      } else {
        // partials in the slot of this barrier's parity: a member can only
        // overwrite it after every member has read it (two barriers later)
        double* pp = part + (int64_t)((gen + 1) & 1) * (2 * MANY_MAX_TEAM);
        if (tid == 0) {
          publish(&pp[2 * mk], brl);
          publish(&pp[2 * mk + 1], bdn);
        }
        if (!team_sync(bar, ++gen * (unsigned)team, p.team_err, p.team_wait_ticks, &sflag)) return;
        double a0 = 0.0, a1 = 0.0;
        for (int u = 0; u < team; ++u) {
          a0 += consume(&pp[2 * u]);
          a1 += consume(&pp[2 * u + 1]);
        }
        rho = a0;
        D = a1;
      }
      ++it;
      // the next pass gathers the new pre-scaled vector
      for (int i = tid; i < H; i += MB) hot[i] = wn[i];
      __syncthreads();
      T* t = xc;
      xc = xn;
      xn = t;
      t = wc;
      wc = wn;
      wn = t;
    }
    // ranks back in the graph's original numbering
    T* out = (T*)p.out + G.voff;
    const int* inv = p.inv + G.voff;
    for (int v = tid; v < n; v += MB)
      if ((v / MB) % team == mk) out[v] = xc[inv[v]];
    if (tid == 0 && mk == 0) {
      p.iters[gi] = it;
      p.resid[gi] = rho;
      // a residual that is not finite ended this graph's loop (a NaN
      // compares false with the tolerance): flag it (bit 1) for the driver
      if (!__builtin_isfinite(rho)) __hip_atomic_fetch_or(p.team_err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

__global__ void queue_reset_kernel(int* q, unsigned* bar, int ngraphs, int* err) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ngraphs; i += gridDim.x * blockDim.x) bar[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *q = 0;
    *err = 0;
  }
}

}  // namespace

hipError_t launch_pr_many(const ManyArgs& a, int type, int grid, hipStream_t s) {
  if (grid <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(queue_reset_kernel, dim3((a.ngraphs + 255) / 256), dim3(256), 0, s, a.queue_next, a.team_bar,
                     a.ngraphs, a.team_err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (type == T_FP32)
    hipLaunchKernelGGL(pr_many_kernel<float>, dim3(grid), dim3(MB), 0, s, a);
  else
    hipLaunchKernelGGL(pr_many_kernel<double>, dim3(grid), dim3(MB), 0, s, a);
  return hipGetLastError();
}

}  // namespace nbgrb
