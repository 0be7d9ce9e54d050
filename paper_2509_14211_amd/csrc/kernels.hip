// gfx950 kernels of the nonblocking GraphBLAS PageRank path.
//
// The central kernel is the fused PageRank pass (paper, Fig. 6: the
// ewise_mult, mxv and ewise_add that the nonblocking DAG materialises at
// wait(r), plus the absdiff/reduce pair behind rdiff(), here also the
// dangling-mass reduction), run over a tile plan of the transposed
// adjacency pattern:
//   * STREAM tiles (runs of short rows) gather their entries' operand
//     values into LDS with coalesced, non-temporal column reads, then reduce
//     each row from LDS with a power-of-two group of lanes per row chosen
//     from the tile's row count, finishing with cross-lane shuffles;
//   * CHUNK tiles split a hub row over several workgroups; the workgroup
//     that completes the last chunk adds the chunk sums in chunk order and
//     finishes the row.
// The per-row epilogue applies the teleport/dangling constant, writes the
// new rank, the pre-scaled copy the next pass gathers, and accumulates the
// L1 residual and the dangling mass in FP64.  Partials are combined in a
// fixed order by the last workgroup, so results are bitwise reproducible.
//
// Cross-workgroup hand-off (hub chunks, workgroup partials) publishes values
// with device-scope atomic stores, waits for their completion, then bumps a
// counter; readers use device-scope atomic loads.  This avoids L2
// write-back / invalidate fences in the middle of the pass.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "device_util.h"
#include "kernels.h"
#include "ops_device.h"

namespace nbgrb {

// ------------------------------------------------------------------ helpers

template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the block in a fixed tree; the result is valid in thread 0.
template <typename V, int B>
__device__ __forceinline__ V block_sum(V v, V* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  V r = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < B / 64; ++i) r += red[i];
  }
  __syncthreads();
  return r;
}

// ---------------------------------------------------------- fused PR pass

template <typename T>
__device__ __forceinline__ void pr_epilogue(const FusedArgs<T>& a, int i, T s, T c, double& rho,
                                            double& dm) {
  if (a.mode == EPI_PLAIN) {
    a.s_out[i] = s;
    return;
  }
  const T tele = a.tele_vec ? (a.tele_scaled ? a.tele_vec[i] * c : a.tele_vec[i]) : c;
  const T r = tele + s;
  if (a.r_out) __builtin_nontemporal_store(r, a.r_out + i);
  if (a.x_old) rho += fabs((double)__builtin_nontemporal_load(a.x_old + i) - (double)r);
  T dv = (T)0;
  if (a.dvec) dv = __builtin_nontemporal_load(a.dvec + i);
  if (a.w_out) a.w_out[i] = a.memo_div ? r / dv : r * dv;
  if (a.do_D) {
    const bool m = a.mask_is_dvec ? (dv != (T)0) : nonzero_at(a.mask, i);
    if (m != (a.mask_comp != 0)) dm += (double)r;
  }
}

// Registers a thread holds for one tile before its gathers: column indices
// of its entries, the tile's row pointers and, for the PageRank epilogue,
// x_old and d of its rows.  Loading them for the next tile while the
// current one is reduced hides one memory round trip per tile.
template <typename T, int KE, int KP, int KR>
struct TileRegs {
  int4 td;
  int ci[KE];
  int rp[KP];
  T xo[KR];
  T dv[KR];
};

template <typename T, int B, int KE, int KP, int KR>
__device__ __forceinline__ void tile_prefetch(const TilePlanDev& plan, const FusedArgs<T>& a,
                                              int t, bool pr, TileRegs<T, KE, KP, KR>& R) {
  const int tid = threadIdx.x;
  R.td = plan.tiles[t];
  const int4 d = R.td;
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int e = tid + k * B;
    R.ci[k] = e < d.w ? __builtin_nontemporal_load(a.col + d.z + e) : 0;
  }
  if (d.y > 0) {
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int r = tid + k * B;
      R.rp[k] = r <= d.y ? a.rowptr[d.x + r] : 0;
    }
    if (pr) {
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int r = tid + k * B;
        const bool ok = r < d.y;
        R.xo[k] = (ok && a.x_old) ? __builtin_nontemporal_load(a.x_old + d.x + r) : (T)0;
        R.dv[k] = (ok && a.dvec) ? __builtin_nontemporal_load(a.dvec + d.x + r) : (T)0;
      }
    }
  }
}

// Epilogue with x_old and d already loaded.
template <typename T>
__device__ __forceinline__ void pr_epilogue_pre(const FusedArgs<T>& a, int i, T s, T c, T xo, T dv,
                                                double& rho, double& dm) {
  if (a.mode == EPI_PLAIN) {
    a.s_out[i] = s;
    return;
  }
  const T tele = a.tele_vec ? (a.tele_scaled ? a.tele_vec[i] * c : a.tele_vec[i]) : c;
  const T r = tele + s;
  if (a.r_out) __builtin_nontemporal_store(r, a.r_out + i);
  if (a.x_old) rho += fabs((double)xo - (double)r);
  if (a.w_out) a.w_out[i] = a.memo_div ? r / dv : r * dv;
  if (a.do_D) {
    const bool m = a.mask_is_dvec ? (dv != (T)0) : nonzero_at(a.mask, i);
    if (m != (a.mask_comp != 0)) dm += (double)r;
  }
}

// Tiles a worker runs: first, end and stride.  Workers are workgroups
// (per_wg = 1) or the per_wg wavefronts of each workgroup (slot = wavefront).
// With plan.xcd the tile list is cut into 8 contiguous ranges and workgroup
// b works in range b mod 8 -- the XCD that workgroup is dispatched to -- so
// the rows, and with them the neighbouring columns, that one XCD's L2 sees
// stay in one region of the matrix.
struct TileWalk {
  int t, end, step;
};

__device__ __forceinline__ TileWalk tile_walk(const TilePlanDev& plan, int slot, int per_wg) {
  const int G = (int)gridDim.x, b = (int)blockIdx.x;
  if (plan.xcd && (G & 7) == 0) {
    const int x = b & 7, j = b >> 3;
    const int lo = (int)((int64_t)plan.ntiles * x / 8);
    const int hi = (int)((int64_t)plan.ntiles * (x + 1) / 8);
    return {lo + j * per_wg + slot, hi, (G >> 3) * per_wg};
  }
  return {b * per_wg + slot, plan.ntiles, G * per_wg};
}

template <typename T, int ET, int RT>
__global__ __launch_bounds__(FUSED_BLOCK) void fused_pr_kernel(TilePlanDev plan, FusedArgs<T> a,
                                                               FusedScratch scr,
                                                               const GuardDev* guard) {
  constexpr int B = FUSED_BLOCK;
  constexpr int KE = ET / B;                 // entries per thread
  constexpr int KP = (RT + 1 + B - 1) / B;   // row pointers per thread
  constexpr int KR = (RT + B - 1) / B;       // epilogue rows per thread
  if (guard && guard->active == 0) return;

  __shared__ T sval[ET];
  __shared__ int srp[RT + 1];
  __shared__ T sres[RT];
  __shared__ double sred[B / 64];
  __shared__ T sredT[B / 64];
  __shared__ int sflag;

  const int tid = threadIdx.x;
  const bool pr = a.mode == EPI_PR;
  T c = (T)0;
  if (pr) c = (T)scalar_value(a.c);
  double rho = 0.0, dm = 0.0;

  TileRegs<T, KE, KP, KR> R;
  const TileWalk tw = tile_walk(plan, 0, 1);
  int t = tw.t;
  if (t < tw.end) tile_prefetch<T, B>(plan, a, t, pr, R);
  for (; t < tw.end; t += tw.step) {
    // gathers of the current tile
    const int4 cur = R.td;
    T val[KE];
#pragma unroll
    for (int k = 0; k < KE; ++k) val[k] = (tid + k * B < cur.w) ? a.w[R.ci[k]] : (T)0;
    int crp[KP];
    T cxo[KR], cdv[KR];
#pragma unroll
    for (int k = 0; k < KP; ++k) crp[k] = R.rp[k];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      cxo[k] = R.xo[k];
      cdv[k] = R.dv[k];
    }
    // next tile's independent loads go out while this one is reduced
    const int tn = t + tw.step;
    if (tn < tw.end) tile_prefetch<T, B>(plan, a, tn, pr, R);

    if (cur.y > 0) {
      // ---- rows [row0, row0 + nr) staged through LDS
      const int row0 = cur.x, nr = cur.y, e0 = cur.z, ne = cur.w;
#pragma unroll
      for (int k = 0; k < KE; ++k)
        if (tid + k * B < ne) sval[tid + k * B] = val[k];
#pragma unroll
      for (int k = 0; k < KP; ++k)
        if (tid + k * B <= nr) srp[tid + k * B] = crp[k] - e0;
      __syncthreads();
      const int q = B / nr;
      const int lpr = q >= 64 ? 64 : q >= 32 ? 32 : q >= 16 ? 16 : q >= 8 ? 8 : q >= 4 ? 4 : q >= 2 ? 2 : 1;
      const int slots = B / lpr;
      const int grp = tid / lpr, lane = tid & (lpr - 1);
      const int rounds = (nr + slots - 1) / slots;
      for (int rd = 0; rd < rounds; ++rd) {
        const int rr = rd * slots + grp;
        T v = 0;
        if (rr < nr) {
          const int hi = srp[rr + 1];
          for (int k = srp[rr] + lane; k < hi; k += lpr) v += sval[k];
        }
        for (int o = lpr >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0 && rr < nr) sres[rr] = v;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int r = tid + k * B;
        if (r < nr) pr_epilogue_pre(a, row0 + r, sres[r], c, cxo[k], cdv[k], rho, dm);
      }
      // the next tile writes sval/srp before its first barrier and sres only
      // after it, so no barrier is needed here
    } else {
      // ---- one chunk of hub row h
      T part = 0;
#pragma unroll
      for (int k = 0; k < KE; ++k) part += val[k];
      const T tot = block_sum<T, B>(part, sredT);
      const int h = -cur.y - 1;
      const int4 hub = plan.hubs[h];  // {row, nchunks, slot0, -}
      if (tid == 0) {
        publish(&scr.hub_sum[hub.z + cur.x], (double)tot);
        wait_stores();
        sflag = counter_add(&scr.hub_cnt[h]) == hub.y - 1;
      }
      __syncthreads();
      if (sflag) {
        // This block finished the hub's last chunk: add the chunk sums
        // (fixed tree over chunk order) and finish the row.
        T s = 0;
        for (int k = tid; k < hub.y; k += B) s += (T)consume(&scr.hub_sum[hub.z + k]);
        s = block_sum<T, B>(s, sredT);
        if (tid == 0) {
          double hr = 0.0, hd = 0.0;
          pr_epilogue(a, hub.x, s, c, hr, hd);
          publish(&scr.hub_red[2 * h], hr);
          publish(&scr.hub_red[2 * h + 1], hd);
          publish(&scr.hub_cnt[h], 0);
        }
      }
      __syncthreads();
    }
  }

  const bool reduce = pr && (a.rho_out.out || a.D_out.out || a.rho_out.guard);
  if (!reduce) return;

  const double br = block_sum<double, B>(rho, sred);
  const double bd = block_sum<double, B>(dm, sred);
  if (tid == 0) {
    publish(&scr.wg_part[2 * blockIdx.x], br);
    publish(&scr.wg_part[2 * blockIdx.x + 1], bd);
    wait_stores();
    const unsigned prev = ticket_add(scr.ticket);
    sflag = prev == gridDim.x - 1;
  }
  __syncthreads();
  if (!sflag) return;

  // Last workgroup: partials in workgroup order, then hub rows in order.
  double pr_ = 0.0, pd = 0.0;
  for (int k = tid; k < (int)gridDim.x; k += B) {
    pr_ += consume(&scr.wg_part[2 * k]);
    pd += consume(&scr.wg_part[2 * k + 1]);
  }
  for (int h = tid; h < plan.nhubs; h += B) {
    pr_ += consume(&scr.hub_red[2 * h]);
    pd += consume(&scr.hub_red[2 * h + 1]);
  }
  const double tr = block_sum<double, B>(pr_, sred);
  const double tdm = block_sum<double, B>(pd, sred);
  if (tid == 0) {
    if (a.rho_out.out) *a.rho_out.out = tr;
    if (a.D_out.out) *a.D_out.out = tdm;
    if (a.rho_out.guard) guard_advance(a.rho_out.guard, tr, a.do_D ? tdm : 0.0);
    publish(scr.ticket, 0u);
  }
}

template <typename T, int ET, int RT>
static hipError_t launch_fused_t(const TilePlanDev& plan, const FusedArgs<T>& a,
                                 const FusedScratch& scr, int grid, const GuardDev* guard,
                                 hipStream_t s) {
  hipLaunchKernelGGL((fused_pr_kernel<T, ET, RT>), dim3(grid), dim3(FUSED_BLOCK), 0, s, plan, a,
                     scr, guard);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_fused_dispatch(const TilePlanDev& plan, const FusedArgs<T>& a,
                                        const FusedScratch& scr, int grid, int lds_entries,
                                        int lds_rows, const GuardDev* guard, hipStream_t s) {
  if (grid <= 0) return hipErrorInvalidValue;
  if (lds_entries == 1024 && lds_rows == 512)
    return launch_fused_t<T, 1024, 512>(plan, a, scr, grid, guard, s);
  if (lds_entries == 2048 && lds_rows == 1024)
    return launch_fused_t<T, 2048, 1024>(plan, a, scr, grid, guard, s);
  if (lds_entries == 4096 && lds_rows == 1024)
    return launch_fused_t<T, 4096, 1024>(plan, a, scr, grid, guard, s);
  return hipErrorInvalidValue;
}

hipError_t launch_fused_f32(const TilePlanDev& plan, const FusedArgs<float>& a,
                            const FusedScratch& scr, int grid, int lds_entries, int lds_rows,
                            const GuardDev* guard, hipStream_t s) {
  return launch_fused_dispatch<float>(plan, a, scr, grid, lds_entries, lds_rows, guard, s);
}

hipError_t launch_fused_f64(const TilePlanDev& plan, const FusedArgs<double>& a,
                            const FusedScratch& scr, int grid, int lds_entries, int lds_rows,
                            const GuardDev* guard, hipStream_t s) {
  return launch_fused_dispatch<double>(plan, a, scr, grid, lds_entries, lds_rows, guard, s);
}

// ---------------------------------------------------------- wave-tiled pass
//
// Same pass over a plan of smaller tiles (at most WE entries and WR rows),
// each processed by one wavefront on its own: no workgroup barrier inside
// the tile loop, so the 16 wavefronts of a workgroup overlap each other's
// memory and LDS phases freely.  One 1024-thread workgroup per compute unit
// also keeps the first `hot` entries of the gathered vector in LDS for all
// its wavefronts; with vertices numbered by decreasing out-degree those are
// the most gathered values, served from LDS instead of the L2.

template <typename T>
struct WaveLds;
template <>
struct WaveLds<float> {
  static constexpr int HMAX = 32704;  // 127.75 KiB: with the entry staging, 159.9 KiB of LDS
};
template <>
struct WaveLds<double> {
  static constexpr int HMAX = 12224;  // 95.5 KiB: with the entry staging, 159.6 KiB of LDS
};

constexpr int WAVE_BLOCK = 1024;
constexpr int WAVE_WE = 512;
constexpr int WAVE_WR = 256;

template <typename T, int POL, int KE, int KP, int KR>
__device__ __forceinline__ void wave_prefetch(const TilePlanDev& plan, const FusedArgs<T>& a, int t,
                                              bool pr, int lane, TileRegs<T, KE, KP, KR>& R) {
  R.td = tile_desc(plan.tiles, t);
  const int4 d = R.td;
  // cache policy POL of these streams: the nontemporal hint keeps them out
  // of the gathered vector's way in L2 but slows the loads themselves; it
  // pays once the gathered vector is much larger than L2
  const __amdgpu_buffer_rsrc_t rc = buf_rsrc(a.col + d.z, (unsigned)d.w * 4u);
#pragma unroll
  for (int k = 0; k < KE; ++k) R.ci[k] = buf_load<int, POL>(rc, (unsigned)(lane + 64 * k) * 4u);
  if (d.y > 0) {
    const __amdgpu_buffer_rsrc_t rr = buf_rsrc(a.rowptr + d.x, (unsigned)(d.y + 1) * 4u);
#pragma unroll
    for (int k = 0; k < KP; ++k) R.rp[k] = buf_load<int, 0>(rr, (unsigned)(lane + 64 * k) * 4u);
    if (pr) {
      const unsigned rows = (unsigned)d.y * (unsigned)sizeof(T);
      const __amdgpu_buffer_rsrc_t rx = buf_rsrc(a.x_old ? a.x_old + d.x : nullptr, a.x_old ? rows : 0u);
      const __amdgpu_buffer_rsrc_t rd = buf_rsrc(a.dvec ? a.dvec + d.x : nullptr, a.dvec ? rows : 0u);
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const unsigned off = (unsigned)(lane + 64 * k) * (unsigned)sizeof(T);
        R.xo[k] = buf_load<T, POL>(rx, off);
        R.dv[k] = buf_load<T, POL>(rd, off);
      }
    }
  }
}

__device__ __forceinline__ void wave_lds_fence() {
  // order this wavefront's LDS writes before its later LDS reads by other lanes
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Entries of the tile whose column indices R holds: hot-slice hits from LDS,
// the rest gathered from memory.
// Entries past the tile's end hold column 0 (the index loads return zero
// there) and their values are never used.
template <typename T, int KE>
__device__ __forceinline__ void wave_gather(__amdgpu_buffer_rsrc_t rw, const T* hot, int H,
                                            const int (&ci)[KE], T (&val)[KE]) {
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int c = ci[k];
    const bool h = c < H;
    const T g = buf_load<T, 0>(rw, h ? BUF_SKIP : (unsigned)c * (unsigned)sizeof(T));
    const T hv = hot[h ? c : 0];
    val[k] = h ? hv : g;
  }
}

// Row sums and epilogues of one tile whose entries are in val.  Only the
// entries go through LDS: row bounds come from the row-pointer registers
// by cross-lane reads, and row sums stay in registers (at most four
// rounds), so the LDS left over holds a larger slice of the gathered
// vector.
template <typename T, int KE, int KP, int KR>
__device__ __forceinline__ void wave_process(const TilePlanDev& plan, const FusedArgs<T>& a,
                                             const FusedScratch& scr, int lane, T c, const int4 cur,
                                             const T (&val)[KE], const int (&crp)[KP], const T (&cxo)[KR],
                                             const T (&cdv)[KR], T* wval, double& rho, double& dm) {
  static_assert(KR <= 4, "row sums are held in four registers");
  if (cur.y > 0) {
    const int row0 = cur.x, nr = cur.y, e0 = cur.z, ne = cur.w;
#pragma unroll
    for (int k = 0; k < KE; ++k)
      if (lane + 64 * k < ne) wval[lane + 64 * k] = val[k];
    wave_lds_fence();
    // rows of up to 64/nr entries get a power-of-two group of lanes each;
    // with more than 64 rows one lane sums row lane + 64 rd in round rd
    const int q = 64 / nr;
    const int lpr = q >= 64 ? 64 : q >= 32 ? 32 : q >= 16 ? 16 : q >= 8 ? 8 : q >= 4 ? 4 : q >= 2 ? 2 : 1;
    const int slots = 64 / lpr;
    const int grp = lane / lpr, sub = lane & (lpr - 1);
    const int rounds = (nr + slots - 1) / slots;
    T res[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
    for (int rd = 0; rd < 4; ++rd) {
      if (rd < rounds) {
        // rows rd*slots .. rd*slots+slots-1 lie in one register of row
        // pointers: crp[rd] when lpr == 1, else (one round) crp[0].  Only
        // constant indices, so the register arrays are never addressed.
        const int rr = rd * slots + grp;
        const int k = lpr == 1 ? rd : 0;
        const int here = lpr == 1 ? crp[rd] : crp[0];
        const int next = lpr == 1 ? crp[rd + 1 < KP ? rd + 1 : KP - 1] : crp[1];
        const int lo = __shfl(here, rr & 63, 64) - e0;
        const int hiA = __shfl(here, (rr + 1) & 63, 64);
        const int hiB = __shfl(next, (rr + 1) & 63, 64);
        const int hi = (((rr + 1) >> 6) != k ? hiB : hiA) - e0;
        T v = 0;
        if (rr < nr)
          for (int e = lo + sub; e < hi; e += lpr) v += wval[e];
        for (int o = lpr >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        res[rd] = v;
      }
    }
    // with one round the sum of row r sits in lane r*lpr; with several
    // (lpr == 1) row lane + 64k is in this lane's res[k]
    const T first = __shfl(res[0], (lane * lpr) & 63, 64);
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int r = lane + 64 * k;
      const T s = lpr == 1 ? res[k] : first;
      if (r < nr) pr_epilogue_pre(a, row0 + r, s, c, cxo[k], cdv[k], rho, dm);
    }
    wave_lds_fence();  // wval is rewritten by the next tile
  } else {
    // one chunk of hub row h
    T part = 0;
#pragma unroll
    for (int k = 0; k < KE; ++k)
      if (lane + 64 * k < cur.w) part += val[k];
    part = wave_sum(part);
    const int h = -cur.y - 1;
    const int4 hub = tile_desc(plan.hubs, h);  // {row, nchunks, slot0, -}
    int last = 0;
    if (lane == 0) {
      publish(&scr.hub_sum[hub.z + cur.x], (double)part);
      wait_stores();
      last = counter_add(&scr.hub_cnt[h]) == hub.y - 1;
    }
    last = __shfl(last, 0, 64);
    if (last) {
      T s = 0;
      for (int k = lane; k < hub.y; k += 64) s += (T)consume(&scr.hub_sum[hub.z + k]);
      s = wave_sum(s);
      if (lane == 0) {
        double hr = 0.0, hd = 0.0;
        pr_epilogue(a, hub.x, s, c, hr, hd);
        publish(&scr.hub_red[2 * h], hr);
        publish(&scr.hub_red[2 * h + 1], hd);
        publish(&scr.hub_cnt[h], 0);
        // Any wavefront of the workgroup may finish a hub, but only thread
        // 0 waits for its own stores before the workgroup takes its ticket:
        // the hub row's partials must be complete before this wavefront
        // reaches the workgroup barrier that precedes the ticket.
        wait_stores();
      }
    }
  }
}

// Tiles of one wavefront are software-pipelined: while tile i is reduced,
// the gathers of tile i+1 and the column indices (and row pointers and
// epilogue inputs) of tile i+2 are in flight.  Loads are issued in the
// order [indices of i+2][gathers of i+1], so waiting for either never waits
// for the other.  FP64 keeps one tile in flight (register budget).
template <typename T, int POL>
__global__ __launch_bounds__(WAVE_BLOCK) void fused_wave_kernel(TilePlanDev plan, FusedArgs<T> a,
                                                                FusedScratch scr, int hot_n,
                                                                const GuardDev* guard) {
  constexpr int B = WAVE_BLOCK;
  constexpr int NW = B / 64;
  constexpr int WE = WAVE_WE, WR = WAVE_WR;
  constexpr int KE = WE / 64, KP = (WR + 1 + 63) / 64, KR = WR / 64;
  constexpr int HMAX = WaveLds<T>::HMAX;
  constexpr bool PIPE = sizeof(T) == 4;
  if (guard && guard->active == 0) return;

  __shared__ __attribute__((aligned(16))) T hot[HMAX];
  __shared__ T sval[NW][WE];
  __shared__ double sred[B / 64];
  __shared__ int sflag;

  const int tid = threadIdx.x;
  const int wv = wave_uniform(tid >> 6), lane = tid & 63;
  const bool pr = a.mode == EPI_PR;
  T c = (T)0;
  if (pr) c = (T)scalar_value(a.c);
  double rho = 0.0, dm = 0.0;

  const int H = hot_n < HMAX ? hot_n : HMAX;
  {
    // the slice in 16-byte pieces, every load issued before the first LDS
    // store, so the fill costs about one memory latency
    constexpr int HV = (int)((HMAX * sizeof(T) + 16 * B - 1) / (16 * B));
    const int nvec = (int)((H * sizeof(T)) / 16);
    const uint4* src = (const uint4*)a.w;
    if (nvec > 0) {
      uint4 tmp[HV];
#pragma unroll
      for (int j = 0; j < HV; ++j) tmp[j] = src[min(tid + j * B, nvec - 1)];
#pragma unroll
      for (int j = 0; j < HV; ++j)
        if (tid + j * B < nvec) ((uint4*)hot)[tid + j * B] = tmp[j];
    }
    for (int k = (int)(nvec * 16 / sizeof(T)) + tid; k < H; k += B) hot[k] = a.w[k];
  }
  __syncthreads();
  const __amdgpu_buffer_rsrc_t rw = buf_rsrc(a.w, (unsigned)a.ncols * (unsigned)sizeof(T));

  T* wval = sval[wv];
  const TileWalk tw = tile_walk(plan, wv, NW);
  const int nwaves = tw.step, tend = tw.end;
  int t = tw.t;
  if (PIPE) {
    if (t < tend) {
      // three register sets rotate through the roles (reduce, gather,
      // prefetch), unrolled by three so no set is ever copied: a copy of a
      // register with a load in flight would wait for every older load.
      TileRegs<T, KE, KP, KR> X, Y, Z;
      T vX[KE], vY[KE], vZ[KE];
      const int last = tend - 1;
      wave_prefetch<T, POL>(plan, a, t, pr, lane, X);
      wave_prefetch<T, POL>(plan, a, min(t + nwaves, last), pr, lane, Y);
      wave_gather<T, KE>(rw, hot, H, X.ci, vX);
      auto step = [&](int tt, TileRegs<T, KE, KP, KR>& P, T (&vP)[KE], TileRegs<T, KE, KP, KR>& G, T (&vG)[KE],
                      TileRegs<T, KE, KP, KR>& F) {
        wave_prefetch<T, POL>(plan, a, min(tt + 2 * nwaves, last), pr, lane, F);
        wave_gather<T, KE>(rw, hot, H, G.ci, vG);
        wave_process<T>(plan, a, scr, lane, c, P.td, vP, P.rp, P.xo, P.dv, wval, rho, dm);
      };
      for (;;) {
        step(t, X, vX, Y, vY, Z);
        t += nwaves;
        if (t >= tend) break;
        step(t, Y, vY, Z, vZ, X);
        t += nwaves;
        if (t >= tend) break;
        step(t, Z, vZ, X, vX, Y);
        t += nwaves;
        if (t >= tend) break;
      }
    }
  } else {
    TileRegs<T, KE, KP, KR> R;
    if (t < tend) wave_prefetch<T, POL>(plan, a, t, pr, lane, R);
    for (; t < tend; t += nwaves) {
      T val[KE];
      wave_gather<T, KE>(rw, hot, H, R.ci, val);
      const int4 cur = R.td;
      int crp[KP];
      T cxo[KR], cdv[KR];
#pragma unroll
      for (int k = 0; k < KP; ++k) crp[k] = R.rp[k];
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        cxo[k] = R.xo[k];
        cdv[k] = R.dv[k];
      }
      const int tn = t + nwaves;
      if (tn < tend) wave_prefetch<T, POL>(plan, a, tn, pr, lane, R);
      wave_process<T>(plan, a, scr, lane, c, cur, val, crp, cxo, cdv, wval, rho, dm);
    }
  }

  const bool reduce = pr && (a.rho_out.out || a.D_out.out || a.rho_out.guard);
  if (!reduce) return;

  const double br = block_sum<double, B>(rho, sred);
  const double bd = block_sum<double, B>(dm, sred);
  if (tid == 0) {
    publish(&scr.wg_part[2 * blockIdx.x], br);
    publish(&scr.wg_part[2 * blockIdx.x + 1], bd);
    wait_stores();
    sflag = ticket_add(scr.ticket) == gridDim.x - 1;
  }
  __syncthreads();
  if (!sflag) return;
  double pr_ = 0.0, pd = 0.0;
  for (int k = tid; k < (int)gridDim.x; k += B) {
    pr_ += consume(&scr.wg_part[2 * k]);
    pd += consume(&scr.wg_part[2 * k + 1]);
  }
  for (int h = tid; h < plan.nhubs; h += B) {
    pr_ += consume(&scr.hub_red[2 * h]);
    pd += consume(&scr.hub_red[2 * h + 1]);
  }
  const double tr = block_sum<double, B>(pr_, sred);
  const double tdm = block_sum<double, B>(pd, sred);
  if (tid == 0) {
    if (a.rho_out.out) *a.rho_out.out = tr;
    if (a.D_out.out) *a.D_out.out = tdm;
    if (a.rho_out.guard) guard_advance(a.rho_out.guard, tr, a.do_D ? tdm : 0.0);
    publish(scr.ticket, 0u);
  }
}

// Gathered vectors larger than the L2 of all XCDs together (32 MiB) read the
// streams with the nontemporal hint (measured: 3% faster at 134 MB, 2%
// slower at 17 MB).
constexpr int64_t WAVE_NT_ABOVE = 32ll << 20;

template <typename T>
static hipError_t launch_fused_wave_t(const TilePlanDev& plan, const FusedArgs<T>& a, const FusedScratch& scr,
                                      int grid, int hot_n, const GuardDev* guard, hipStream_t s) {
  if (grid <= 0) return hipErrorInvalidValue;
  if ((int64_t)a.ncols * (int64_t)sizeof(T) > WAVE_NT_ABOVE)
    hipLaunchKernelGGL((fused_wave_kernel<T, CP_NT>), dim3(grid), dim3(WAVE_BLOCK), 0, s, plan, a, scr, hot_n, guard);
  else
    hipLaunchKernelGGL((fused_wave_kernel<T, 0>), dim3(grid), dim3(WAVE_BLOCK), 0, s, plan, a, scr, hot_n, guard);
  return hipGetLastError();
}

hipError_t launch_fused_wave_f32(const TilePlanDev& plan, const FusedArgs<float>& a,
                                 const FusedScratch& scr, int grid, int hot_n,
                                 const GuardDev* guard, hipStream_t s) {
  return launch_fused_wave_t<float>(plan, a, scr, grid, hot_n, guard, s);
}

hipError_t launch_fused_wave_f64(const TilePlanDev& plan, const FusedArgs<double>& a,
                                 const FusedScratch& scr, int grid, int hot_n,
                                 const GuardDev* guard, hipStream_t s) {
  return launch_fused_wave_t<double>(plan, a, scr, grid, hot_n, guard, s);
}

int wave_hot_max(int type) { return type == T_FP32 ? WaveLds<float>::HMAX : WaveLds<double>::HMAX; }

// ---------------------------------------------------------- elementwise

constexpr int EW_BLOCK = 256;

template <typename T>
__global__ __launch_bounds__(EW_BLOCK) void ewise_kernel(int64_t n, int kind, int op, Operand a,
                                                         Operand b, ScalarArg sc, void* out,
                                                         int out_type, const GuardDev* guard) {
  if (guard && guard->active == 0) return;
  const T sv = (T)scalar_value(sc);
  const int64_t stride = (int64_t)gridDim.x * EW_BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * EW_BLOCK + threadIdx.x; i < n; i += stride) {
    const T x = load_as<T>(a, i);
    T r;
    switch (kind) {
      case EW_BINARY: r = apply_binop<T>(op, x, load_as<T>(b, i)); break;
      case EW_UNARY: r = apply_unop<T>(op, x); break;
      case EW_BIND1ST: r = apply_binop<T>(op, sv, x); break;
      default: r = apply_binop<T>(op, x, sv); break;
    }
    store_as<T>(out, out_type, i, r);
  }
}

// Dense same-type fast path: four elements in flight per thread.
template <typename T>
__global__ __launch_bounds__(EW_BLOCK) void ewise_fast_kernel(int64_t n, int kind, int op,
                                                              const T* __restrict__ a, T aiso,
                                                              const T* __restrict__ b, T biso,
                                                              ScalarArg sc, T* __restrict__ out,
                                                              const GuardDev* guard) {
  if (guard && guard->active == 0) return;
  const T sv = (T)scalar_value(sc);
  const int64_t stride = (int64_t)gridDim.x * EW_BLOCK;
  int64_t i = (int64_t)blockIdx.x * EW_BLOCK + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    T x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = a ? a[i + u * stride] : aiso;
    if (kind == EW_BINARY) {
#pragma unroll
      for (int u = 0; u < 4; ++u) y[u] = b ? b[i + u * stride] : biso;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      T r;
      switch (kind) {
        case EW_BINARY: r = apply_binop<T>(op, x[u], y[u]); break;
        case EW_UNARY: r = apply_unop<T>(op, x[u]); break;
        case EW_BIND1ST: r = apply_binop<T>(op, sv, x[u]); break;
        default: r = apply_binop<T>(op, x[u], sv); break;
      }
      out[i + u * stride] = r;
    }
  }
  for (; i < n; i += stride) {
    const T x = a ? a[i] : aiso;
    T r;
    switch (kind) {
      case EW_BINARY: r = apply_binop<T>(op, x, b ? b[i] : biso); break;
      case EW_UNARY: r = apply_unop<T>(op, x); break;
      case EW_BIND1ST: r = apply_binop<T>(op, sv, x); break;
      default: r = apply_binop<T>(op, x, sv); break;
    }
    out[i] = r;
  }
}

static int ew_grid(int64_t n, int per_thread) {
  int64_t g = (n + (int64_t)EW_BLOCK * per_thread - 1) / ((int64_t)EW_BLOCK * per_thread);
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  return (int)g;
}

hipError_t launch_ewise(int64_t n, int ct, int kind, int op, Operand a, Operand b, ScalarArg sc,
                        void* out, int out_type, const GuardDev* guard, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const bool a_ok = !a.p || a.type == ct;
  const bool b_ok = kind != EW_BINARY || !b.p || b.type == ct;
  if (a_ok && b_ok && out_type == ct && (ct == T_FP32 || ct == T_FP64)) {
    const int g = ew_grid(n, 4);
    if (ct == T_FP32)
      hipLaunchKernelGGL(ewise_fast_kernel<float>, dim3(g), dim3(EW_BLOCK), 0, s, n, kind, op,
                         (const float*)a.p, (float)a.iso, (const float*)b.p, (float)b.iso, sc,
                         (float*)out, guard);
    else
      hipLaunchKernelGGL(ewise_fast_kernel<double>, dim3(g), dim3(EW_BLOCK), 0, s, n, kind, op,
                         (const double*)a.p, a.iso, (const double*)b.p, b.iso, sc,
                         (double*)out, guard);
    return hipGetLastError();
  }
  const int g = ew_grid(n, 2);
  if (ct == T_FP32)
    hipLaunchKernelGGL(ewise_kernel<float>, dim3(g), dim3(EW_BLOCK), 0, s, n, kind, op, a, b, sc,
                       out, out_type, guard);
  else
    hipLaunchKernelGGL(ewise_kernel<double>, dim3(g), dim3(EW_BLOCK), 0, s, n, kind, op, a, b,
                       sc, out, out_type, guard);
  return hipGetLastError();
}

// ---------------------------------------------------------- reduction

__global__ __launch_bounds__(REDUCE_BLOCK) void reduce_kernel(int64_t n, Operand x, int use_mask,
                                                              Operand mask, int mask_comp,
                                                              ReduceOut out, RedScratch scr,
                                                              const GuardDev* guard) {
  constexpr int B = REDUCE_BLOCK;
  if (guard && guard->active == 0) return;
  __shared__ double sred[B / 64];
  __shared__ int sflag;
  const int tid = threadIdx.x;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * B;
  for (int64_t i = (int64_t)blockIdx.x * B + tid; i < n; i += stride) {
    if (use_mask && (nonzero_at(mask, i) == (mask_comp != 0))) continue;
    acc += load_as<double>(x, i);
  }
  const double b = block_sum<double, B>(acc, sred);
  if (tid == 0) {
    publish(&scr.partials[blockIdx.x], b);
    wait_stores();
    sflag = ticket_add(scr.ticket) == gridDim.x - 1;
  }
  __syncthreads();
  if (!sflag) return;
  double p = 0.0;
  for (int k = tid; k < (int)gridDim.x; k += B) p += consume(&scr.partials[k]);
  const double tot = block_sum<double, B>(p, sred);
  if (tid == 0) {
    if (out.out) *out.out = tot;
    if (out.guard) guard_advance(out.guard, tot);
    publish(scr.ticket, 0u);
  }
}

hipError_t launch_reduce(int64_t n, Operand x, int use_mask, Operand mask, int mask_comp,
                         ReduceOut out, RedScratch scr, const GuardDev* guard, hipStream_t s) {
  int64_t g = (n + REDUCE_BLOCK * 4 - 1) / (REDUCE_BLOCK * 4);
  if (g < 1) g = 1;
  if (g > REDUCE_GRID) g = REDUCE_GRID;
  hipLaunchKernelGGL(reduce_kernel, dim3((int)g), dim3(REDUCE_BLOCK), 0, s, n, x, use_mask, mask,
                     mask_comp, out, scr, guard);
  return hipGetLastError();
}

// ---------------------------------------------------------- small kernels

__global__ void fill_kernel(void* out, int type, int64_t n, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    store_as<double>(out, type, i, v);
}

hipError_t launch_fill(void* out, int type, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(ew_grid(n, 4)), dim3(EW_BLOCK), 0, s, out, type, n, v);
  return hipGetLastError();
}

__global__ void set_scalar_kernel(double* dst, double v) { *dst = v; }

hipError_t launch_set_scalar(double* dst, double v, hipStream_t s) {
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, s, dst, v);
  return hipGetLastError();
}

__global__ void convert_kernel(Operand src, void* dst, int dst_type, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (dst_type == T_FP32)
      ((float*)dst)[i] = load_as<float>(src, i);
    else
      store_as<double>(dst, dst_type, i, load_as<double>(src, i));
  }
}

hipError_t launch_convert(const void* src, int src_type, void* dst, int dst_type, int64_t n,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  Operand o{src, src_type, 0.0};
  hipLaunchKernelGGL(convert_kernel, dim3(ew_grid(n, 4)), dim3(EW_BLOCK), 0, s, o, dst, dst_type,
                     n);
  return hipGetLastError();
}

__global__ void guard_init_kernel(GuardDev* g, int active, double tol, int itermax) {
  g->active = active;
  g->iters = 0;
  g->rho = 1.0;
  g->rho_prev = 0.0;
  g->tol = tol;
  g->itermax = itermax;
  g->bad = 0;
}

hipError_t launch_guard_init(GuardDev* g, int active, double tol, int itermax, hipStream_t s) {
  hipLaunchKernelGGL(guard_init_kernel, dim3(1), dim3(1), 0, s, g, active, tol, itermax);
  return hipGetLastError();
}

__global__ void zero_kernel(uint8_t* p, size_t bytes) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t words = bytes / 4;
  uint32_t* w = (uint32_t*)p;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) w[i] = 0u;
  for (size_t i = words * 4 + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes;
       i += stride)
    p[i] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (((uintptr_t)p & 3u) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_kernel, dim3(ew_grid((int64_t)(bytes / 4 + 1), 4)), dim3(EW_BLOCK), 0, s,
                     (uint8_t*)p, bytes);
  return hipGetLastError();
}

// ---------------------------------------------------------- R-MAT

__global__ void rmat_kernel(uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int scale,
                            int64_t nedges, uint64_t seed, double ta, double tab, double tabc) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nedges; e += stride) {
    uint32_t su = 0, dv = 0;
    uint64_t k = (uint64_t)e * (uint64_t)scale;
    for (int l = 0; l < scale; ++l, ++k) {
      const double u = draw_unit(splitmix_draw(seed, k));
      const uint32_t bs = u >= tab ? 1u : 0u;                       // c or d
      const uint32_t bd = (u >= ta && u < tab) || u >= tabc ? 1u : 0u;  // b or d
      su = (su << 1) | bs;
      dv = (dv << 1) | bd;
    }
    src[e] = su;
    dst[e] = dv;
  }
}

hipError_t launch_rmat(uint32_t* src, uint32_t* dst, int scale, int64_t nedges, uint64_t seed,
                       double ta, double tab, double tabc, hipStream_t s) {
  if (nedges <= 0) return hipSuccess;
  hipLaunchKernelGGL(rmat_kernel, dim3(ew_grid(nedges, 4)), dim3(EW_BLOCK), 0, s, src, dst, scale,
                     nedges, seed, ta, tab, tabc);
  return hipGetLastError();
}

// ---------------------------------------------------------- probes / misc

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stream_copy_kernel(u32x4* __restrict__ dst,
                                                          const u32x4* __restrict__ src,
                                                          int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if ((bytes & 15u) || ((uintptr_t)dst & 15u) || ((uintptr_t)src & 15u)) return hipErrorInvalidValue;
  const int64_t n16 = (int64_t)(bytes / 16);
  int64_t g = (n16 + 256 * 4 - 1) / (256 * 4);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(stream_copy_kernel, dim3((int)g), dim3(256), 0, s, (u32x4*)dst,
                     (const u32x4*)src, n16);
  return hipGetLastError();
}

__global__ void permute_kernel(const void* __restrict__ in, int type, const int* __restrict__ idx,
                               void* __restrict__ out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    const int64_t j = idx[k];
    switch (type) {
      case T_BOOL: ((uint8_t*)out)[k] = ((const uint8_t*)in)[j]; break;
      case T_INT32: ((int*)out)[k] = ((const int*)in)[j]; break;
      case T_FP32: ((float*)out)[k] = ((const float*)in)[j]; break;
      default: ((double*)out)[k] = ((const double*)in)[j]; break;
    }
  }
}

hipError_t launch_permute(const void* in, int type, const int* idx, void* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(permute_kernel, dim3(ew_grid(n, 4)), dim3(EW_BLOCK), 0, s, in, type, idx, out, n);
  return hipGetLastError();
}

__global__ void row_degree_kernel(const int* rowptr, int64_t n, void* deg, int type) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    store_as<double>(deg, type, i, (double)(rowptr[i + 1] - rowptr[i]));
}

hipError_t launch_row_degree(const int* rowptr, int64_t n, void* deg, int type, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_degree_kernel, dim3(ew_grid(n, 4)), dim3(EW_BLOCK), 0, s, rowptr, n, deg,
                     type);
  return hipGetLastError();
}

__global__ void check_csr_kernel(const int* rowptr, int64_t nrows, const int* col, int64_t nnz,
                                 int64_t ncols, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0 && (rowptr[0] != 0 || (int64_t)rowptr[nrows] != nnz)) atomicOr(flag, 1);
  for (int64_t i = tid; i < nrows; i += stride)
    if (rowptr[i + 1] < rowptr[i]) atomicOr(flag, 1);
  for (int64_t e = tid; e < nnz; e += stride)
    if (col[e] < 0 || (int64_t)col[e] >= ncols) atomicOr(flag, 2);
}

hipError_t launch_check_csr(const int* rowptr, int64_t nrows, const int* col, int64_t nnz,
                            int64_t ncols, int* flag, hipStream_t s) {
  const int64_t work = nrows > nnz ? nrows : nnz;
  hipLaunchKernelGGL(check_csr_kernel, dim3(ew_grid(work + 1, 4)), dim3(EW_BLOCK), 0, s, rowptr,
                     nrows, col, nnz, ncols, flag);
  return hipGetLastError();
}

}  // namespace nbgrb
