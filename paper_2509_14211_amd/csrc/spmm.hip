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

#include "device_util.h"
#include "kernels.h"

namespace nbgrb {

namespace {

constexpr int SB = 1024;   // threads per workgroup
constexpr int SNW = SB / 64;

// Epilogue of row i with its inputs already loaded (xo = x_old row entry,
// dv = d_i).  Seeds are consumed in vertex order: sp is the next unread
// seed, nsv its vertex.  Lane `lane` owns an existing column when `have`,
// one still iterating when `live`.  A frozen column (have, not live) copies
// its value forward, so both buffer sets hold it and every row is stored
// whole: a row store with masked lanes leaves partly written lines in HBM,
// which cost the memory system more than full ones.
template <typename T>
__device__ __forceinline__ void spmm_finish(const SpmmArgs& p, int i, T s, int lane, bool have, bool live, T cfac,
                                            T xo, T dv, int& sp, int& nsv, double& rho, double& dm) {
  T tele = 0;
  while (nsv == i) {
    if (p.seed_c[sp] == lane) tele += (T)p.seed_w[sp] * cfac;
    ++sp;
    nsv = sp < p.nseeds ? p.seed_v[sp] : 0x7fffffff;
  }
  if (!have) return;
  const int64_t at = (int64_t)i * p.k + lane;
  if (p.plain) {
    __builtin_nontemporal_store(s, (T*)p.x_new + at);
    return;
  }
  const T r = live ? s + tele : xo;
  __builtin_nontemporal_store(r, (T*)p.x_new + at);
  ((T*)p.w_new)[at] = r * dv;
  if (live) {
    rho += fabs((double)xo - (double)r);
    if (dv == (T)0) dm += (double)r;
  }
}

template <typename T>
__device__ __forceinline__ T load_xo(const SpmmArgs& p, int i, int lane, bool have) {
  return (have && !p.plain) ? __builtin_nontemporal_load((const T*)p.x_old + (int64_t)i * p.k + lane) : (T)0;
}

template <typename T>
__device__ __forceinline__ T load_dv(const SpmmArgs& p, int i) {
  return p.plain ? (T)0 : ((const T*)p.dvec)[i];
}

// Column c takes part in this pass: it exists and has not converged yet.  A
// converged column is frozen: no lane writes it again, so its iterate of
// the pass it converged in stays in that pass's buffer, and its residual
// and dangling mass stay those of that pass.
__device__ __forceinline__ bool column_live(const SpmmArgs& p, int c) {
  return c < p.k && !(p.hit && p.hit[c] >= 0);
}

// First vertex-sorted seed of tile t (no seeds in a plain product).
__device__ __forceinline__ int first_seed(const SpmmArgs& p, int t) { return p.nseeds > 0 ? p.tile_seed[t] : 0; }

// Hub row h: once every chunk has published its k-wide partial sum, the
// wavefront that finished last adds them in chunk order and runs the
// epilogue; the row's residual and dangling terms go to hub_red[h].
template <typename T>
__device__ void spmm_hub_finish(const SpmmArgs& p, int4 hub, int h, int chunk, int sp0, T acc, int lane, bool have,
                                bool live, T cfac) {
  const bool on = live;  // frozen columns need no sum
  if (on) publish(&p.hub_sum[(int64_t)(hub.z + chunk) * 64 + lane], (double)acc);
  wait_stores();
  int last = 0;
  if (lane == 0)
    last = __hip_atomic_fetch_add(&p.hub_cnt[h], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == hub.y - 1;
  last = __shfl(last, 0, 64);
  if (!last) return;
  T s = 0;
  int q = 0;
  for (; q + 8 <= hub.y; q += 8) {  // eight loads in flight
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = on ? consume(&p.hub_sum[(int64_t)(hub.z + q + u) * 64 + lane]) : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) s += (T)v[u];
  }
  for (; q < hub.y; ++q) s += on ? (T)consume(&p.hub_sum[(int64_t)(hub.z + q) * 64 + lane]) : (T)0;
  int sp = sp0;
  int nsv = sp < p.nseeds ? p.seed_v[sp] : 0x7fffffff;
  double hr = 0.0, hd = 0.0;
  spmm_finish<T>(p, hub.x, s, lane, have, live, cfac, load_xo<T>(p, hub.x, lane, have), load_dv<T>(p, hub.x), sp,
                 nsv, hr, hd);
  publish(&p.hub_red[(int64_t)h * 128 + lane], hr);
  publish(&p.hub_red[(int64_t)h * 128 + 64 + lane], hd);
  if (lane == 0) publish(&p.hub_cnt[h], 0);
}

// Per-column residual and dangling mass of the pass: wavefronts in order,
// then workgroups in order, then hub rows; the last workgroup to arrive
// writes rho_out / d_out of the live columns, marks the ones whose residual
// reached hit_tol, and advances the loop guard on the largest residual of
// the columns that were live in this pass.
__device__ void spmm_reduce(const TilePlanDev& plan, const SpmmArgs& p, double rho, double dm,
                            double (*sr)[64], double (*sd)[64], int* sflag) {
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  sr[wv][lane] = rho;
  sd[wv][lane] = dm;
  __syncthreads();
  if (tid < 64) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < SNW; ++w) {
      a += sr[w][tid];
      b += sd[w][tid];
    }
    publish(&p.wg_part[(int64_t)blockIdx.x * 128 + tid], a);
    publish(&p.wg_part[(int64_t)blockIdx.x * 128 + 64 + tid], b);
  }
  wait_stores();
  __syncthreads();
  if (tid == 0)
    *sflag = __hip_atomic_fetch_add(p.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  __syncthreads();
  if (!*sflag) return;
  {
    // thread (slice, column): slice sl of the workgroup partials and of the
    // hub rows, then the slices of a column in slice order
    const int cc = tid & 63, sl = tid >> 6;
    double a = 0.0, b = 0.0;
    for (int g = sl; g < (int)gridDim.x; g += SNW) {
      a += consume(&p.wg_part[(int64_t)g * 128 + cc]);
      b += consume(&p.wg_part[(int64_t)g * 128 + 64 + cc]);
    }
    for (int h = sl; h < plan.nhubs; h += SNW) {
      a += consume(&p.hub_red[(int64_t)h * 128 + cc]);
      b += consume(&p.hub_red[(int64_t)h * 128 + 64 + cc]);
    }
    sr[sl][cc] = a;
    sd[sl][cc] = b;
  }
  __syncthreads();
  double fa = 0.0, fb = 0.0;
  if (tid < 64) {
    for (int w = 0; w < SNW; ++w) {
      fa += sr[w][tid];
      fb += sd[w][tid];
    }
  }
  __syncthreads();
  if (tid < 64) {
    sr[0][tid] = tid < p.k ? fa : 0.0;
    sd[0][tid] = fb;
  }
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    bool finite = true;
    const int it = p.guard ? p.guard->iters + 1 : 0;
    for (int c = 0; c < p.k; ++c) {
      if (!column_live(p, c)) continue;  // frozen: keeps its values
      p.rho_out[c] = sr[0][c];
      p.d_out[c] = sd[0][c];
      if (sr[0][c] > mx) mx = sr[0][c];
      finite = finite && __builtin_isfinite(sr[0][c]) && __builtin_isfinite(sd[0][c]);
      if (p.hit && p.hit[c] < 0 && p.guard && sr[0][c] <= p.hit_tol) p.hit[c] = it;
    }
    if (p.guard) {
      // a column whose residual or dangling mass is not finite ends the
      // loop and marks the guard bad (reported as an execution error)
      GuardDev* g = p.guard;
      g->rho_prev = g->rho;
      g->rho = finite ? mx : __builtin_nan("");
      g->iters = it;
      if (!finite) g->bad = 1;
      g->active = (finite && mx > g->tol && it < g->itermax) ? 1 : 0;
    }
    publish(p.ticket, 0u);
  }
}

// k-wide rows of the n x k operands, addressed through buffer resources:
// the row's byte offset is a wave-uniform scalar, the lane's column a
// per-lane offset (lanes past k use column 0 and never store).
struct RowBufs {
  __amdgpu_buffer_rsrc_t w, xo, xn, wn;
  int voff;
  unsigned row_bytes;
};
__device__ __forceinline__ int row_off(const RowBufs& b, int i) { return (int)((unsigned)i * b.row_bytes); }

// spmm_finish with buffer-addressed rows.
template <typename T>
__device__ __forceinline__ void spmm_finish_b(const SpmmArgs& p, const RowBufs& b, int i, T s, int lane, bool have,
                                              bool live, T cfac, T xo, T dv, int& sp, int& nsv, double& rho,
                                              double& dm) {
  T tele = 0;
  while (nsv == i) {
    if (wave_uniform(p.seed_c[sp]) == lane) tele += (T)wave_uniform(p.seed_w[sp]) * cfac;
    ++sp;
    nsv = sp < p.nseeds ? wave_uniform(p.seed_v[sp]) : 0x7fffffff;
  }
  if (!have) return;
  const int so = row_off(b, i);
  if (p.plain) {
    buf_store<T, CP_NT>(b.xn, s, b.voff, so);
    return;
  }
  const T r = live ? s + tele : xo;
  buf_store<T, CP_NT>(b.xn, r, b.voff, so);
  buf_store<T, 0>(b.wn, r * dv, b.voff, so);
  if (live) {
    rho += fabs((double)xo - (double)r);
    if (dv == (T)0) dm += (double)r;
  }
}

template <typename T>
struct GatherDepth {
  static constexpr int U = 32;
};
template <>
struct GatherDepth<double> {
  static constexpr int U = 8;
};

// The pass for operands below 4 GiB.  Each wavefront takes one tile at a
// time; the tile's column indices are read 64 at a time into one register
// (lane q holds entry q of the chunk) and broadcast with readlane, so every
// gathered row costs one scalar offset and one vector load, with U rows in
// flight.  The tile's row pointers sit in wave-private LDS.  With
// p.skip_empty, a row with no entries and no seed is not touched: its x and
// w are zero in both buffer sets (the caller keeps them so), and it adds
// nothing to the residual or the dangling mass.
template <typename T>
__global__ __launch_bounds__(SB) __attribute__((amdgpu_waves_per_eu(8))) void spmm_ppr_kernel(
    TilePlanDev plan, SpmmArgs p, const GuardDev* guard) {
  constexpr int TR = WAVE_TILE_ROWS, U = GatherDepth<T>::U;
  static_assert(64 % U == 0, "gather depth divides the chunk");
  if (guard && guard->active == 0) return;
  __shared__ double sr[SNW][64];
  __shared__ double sd[SNW][64];
  __shared__ int srp[SNW][TR + 1];
  __shared__ int sflag;
  const int tid = threadIdx.x, wv = wave_uniform(tid >> 6), lane = tid & 63;
  const bool have = lane < p.k;
  const bool live = column_live(p, lane);
  const bool plain = p.plain != 0;
  const bool skip = p.skip_empty != 0 && !plain;
  RowBufs b;
  b.row_bytes = (unsigned)p.k * (unsigned)sizeof(T);
  b.voff = have ? lane * (int)sizeof(T) : 0;
  b.w = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p.w), (short)0, (int)p.w_bytes, 0x00020000);
  b.xo = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p.x_old), (short)0, (int)p.w_bytes, 0x00020000);
  b.xn = __builtin_amdgcn_make_buffer_rsrc(p.x_new, (short)0, (int)p.w_bytes, 0x00020000);
  b.wn = __builtin_amdgcn_make_buffer_rsrc(p.w_new, (short)0, (int)p.w_bytes, 0x00020000);
  T cfac = (T)0;
  if (live) cfac = (T)(p.c_beta + (p.d_prev ? p.c_alpha * p.d_prev[lane] : 0.0));
  double rho = 0.0, dm = 0.0;
  int* wrp = srp[wv];

  const int nwaves = (int)gridDim.x * SNW;
  for (int t = (int)blockIdx.x * SNW + wv; t < plan.ntiles; t += nwaves) {
    const int4 td = wave_uniform(plan.tiles[t]);
    const int e0 = td.z, ne = td.w;
    if (td.y > 0) {
      const int row0 = td.x, nr = td.y;
      int sp = wave_uniform(first_seed(p, t));
      int nsv = sp < p.nseeds ? wave_uniform(p.seed_v[sp]) : 0x7fffffff;
      if (skip && ne == 0 && nsv >= row0 + nr) continue;  // rows without entries or seeds
      int colv = lane < ne ? p.col[e0 + lane] : 0;
      for (int q = lane; q <= nr; q += 64) wrp[q] = p.rowptr[row0 + q] - e0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      int r = 0;
      int rend = wave_uniform(wrp[1]);
      // row r is left untouched: no entries, no seed
      bool idle = skip && rend == 0 && nsv != row0;
      T acc = 0;
      T xo = (T)0, dv = (T)0;
      if (!idle) {
        xo = plain ? (T)0 : buf_load<T, CP_NT>(b.xo, b.voff, row_off(b, row0));
        dv = wave_uniform(load_dv<T>(p, row0));
      }
      for (int c0 = 0; c0 < ne; c0 += 64) {
        const int cn = c0 + 64 + lane;
        const int coln = cn < ne ? p.col[e0 + cn] : 0;
#pragma unroll
        for (int h = 0; h < 64; h += U) {
          const int base = c0 + h;
          if (base >= ne) break;
          T v[U];
#pragma unroll
          for (int u = 0; u < U; ++u) v[u] = buf_load<T, 0>(b.w, b.voff, row_off(b, __builtin_amdgcn_readlane(colv, h + u)));
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int e = base + u;
            if (e < ne) {
              while (e == rend) {
                if (!idle) spmm_finish_b<T>(p, b, row0 + r, acc, lane, have, live, cfac, xo, dv, sp, nsv, rho, dm);
                acc = 0;
                ++r;
                const int rbeg = rend;
                rend = wave_uniform(wrp[r + 1]);
                idle = skip && rend == rbeg && nsv != row0 + r;
                if (!idle) {
                  xo = plain ? (T)0 : buf_load<T, CP_NT>(b.xo, b.voff, row_off(b, row0 + r));
                  dv = wave_uniform(load_dv<T>(p, row0 + r));
                }
              }
              acc += v[u];
            }
          }
        }
        colv = coln;
      }
      while (r < nr) {  // last row with entries, then empty rows
        if (!idle) spmm_finish_b<T>(p, b, row0 + r, acc, lane, have, live, cfac, xo, dv, sp, nsv, rho, dm);
        acc = 0;
        ++r;
        if (r < nr) {
          // every row from here on has no entries
          idle = skip && nsv != row0 + r;
          if (!idle) {
            xo = plain ? (T)0 : buf_load<T, CP_NT>(b.xo, b.voff, row_off(b, row0 + r));
            dv = wave_uniform(load_dv<T>(p, row0 + r));
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();  // the next tile rewrites wrp
    } else {
      const int h = -td.y - 1;
      int colv = lane < ne ? p.col[e0 + lane] : 0;
      T acc = 0;
      for (int c0 = 0; c0 < ne; c0 += 64) {
        const int cn = c0 + 64 + lane;
        const int coln = cn < ne ? p.col[e0 + cn] : 0;
#pragma unroll
        for (int hh = 0; hh < 64; hh += U) {
          const int base = c0 + hh;
          if (base >= ne) break;
          T v[U];
#pragma unroll
          for (int u = 0; u < U; ++u) v[u] = buf_load<T, 0>(b.w, b.voff, row_off(b, __builtin_amdgcn_readlane(colv, hh + u)));
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (base + u < ne) acc += v[u];
        }
        colv = coln;
      }
      spmm_hub_finish<T>(p, wave_uniform(plan.hubs[h]), h, td.x, wave_uniform(first_seed(p, t)), acc, lane, have,
                         live, cfac);
    }
  }
  if (!plain) spmm_reduce(plan, p, rho, dm, sr, sd, &sflag);
}

// Sum of v over the G = 64 / KP lane groups of a wavefront: every lane ends
// with the sum for its column c = lane % KP.
template <int KP, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = KP; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The buffer-addressed pass for k <= KP columns (KP = 4, 8 or 16): the
// wavefront splits into G = 64 / KP lane groups of KP lanes, lane (g, c)
// owning column c of entry g of each group of G consecutive entries, so
// one vector load gathers G rows of W.  A row's partial sums are added
// across the groups when it ends; group 0 then runs the epilogue, exactly
// as lane c of the one-entry-per-load pass would (same stores, residual,
// seeds and hub handling).  Narrow column counts would otherwise leave
// most lanes of every gathering load idle.
template <typename T, int KP>
__global__ __launch_bounds__(SB) __attribute__((amdgpu_waves_per_eu(8))) void spmm_packed_kernel(
    TilePlanDev plan, SpmmArgs p, const GuardDev* guard) {
  constexpr int TR = WAVE_TILE_ROWS, G = 64 / KP, STEPS = 64 / G;  // STEPS groups of G entries per chunk
  constexpr int UNR = (sizeof(T) == 8 && STEPS > 8) ? 4 : STEPS;     // gathers in flight
  static_assert(KP == 4 || KP == 8 || KP == 16, "lane group width");
  if (guard && guard->active == 0) return;
  __shared__ double sr[SNW][64];
  __shared__ double sd[SNW][64];
  __shared__ int srp[SNW][TR + 1];
  __shared__ int sflag;
  const int tid = threadIdx.x, wv = wave_uniform(tid >> 6), lane = tid & 63;
  const int grp = lane / KP, c = lane % KP;
  const bool gather = c < p.k;                  // lane loads a real column
  const bool have = grp == 0 && c < p.k;        // lane owns column c in the epilogue
  const bool live = grp == 0 && column_live(p, c);
  const bool plain = p.plain != 0;
  const bool skip = p.skip_empty != 0 && !plain;
  RowBufs b;
  b.row_bytes = (unsigned)p.k * (unsigned)sizeof(T);
  b.voff = have ? lane * (int)sizeof(T) : 0;    // lane == c in group 0
  const unsigned coff = gather ? (unsigned)c * (unsigned)sizeof(T) : 0u;
  b.w = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p.w), (short)0, (int)p.w_bytes, 0x00020000);
  b.xo = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p.x_old), (short)0, (int)p.w_bytes, 0x00020000);
  b.xn = __builtin_amdgcn_make_buffer_rsrc(p.x_new, (short)0, (int)p.w_bytes, 0x00020000);
  b.wn = __builtin_amdgcn_make_buffer_rsrc(p.w_new, (short)0, (int)p.w_bytes, 0x00020000);
  T cfac = (T)0;
  if (live) cfac = (T)(p.c_beta + (p.d_prev ? p.c_alpha * p.d_prev[c] : 0.0));
  double rho = 0.0, dm = 0.0;
  int* wrp = srp[wv];

  const int nwaves = (int)gridDim.x * SNW;
  for (int t = (int)blockIdx.x * SNW + wv; t < plan.ntiles; t += nwaves) {
    const int4 td = wave_uniform(plan.tiles[t]);
    const int e0 = td.z, ne = td.w;
    const bool rows = td.y > 0;
    const int row0 = td.x, nr = td.y;
    int sp = wave_uniform(first_seed(p, t));
    int nsv = sp < p.nseeds ? wave_uniform(p.seed_v[sp]) : 0x7fffffff;
    if (rows && skip && ne == 0 && nsv >= row0 + nr) continue;  // rows without entries or seeds
    int colv = lane < ne ? p.col[e0 + lane] : 0;
    int r = 0, rend = 0x7fffffff;
    bool idle = false;
    T xo = (T)0, dv = (T)0;
    if (rows) {
      for (int q = lane; q <= nr; q += 64) wrp[q] = p.rowptr[row0 + q] - e0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      rend = wave_uniform(wrp[1]);
      idle = skip && rend == 0 && nsv != row0;
      if (!idle) {
        xo = plain ? (T)0 : buf_load<T, CP_NT>(b.xo, b.voff, row_off(b, row0));
        dv = wave_uniform(load_dv<T>(p, row0));
      }
    }
    T acc = 0;
    for (int c0 = 0; c0 < ne; c0 += 64) {
      const int cn = c0 + 64 + lane;
      const int coln = cn < ne ? p.col[e0 + cn] : 0;
#pragma unroll
      for (int s0 = 0; s0 < STEPS; s0 += UNR) {
      if (c0 + s0 * G >= ne) break;
      T v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        // entry c0 + s*G + grp, its column index taken from lane s*G + grp
        const int q = (s0 + u) * G + grp;
        const int cj = __builtin_amdgcn_ds_bpermute(q * 4, colv);
        const unsigned off = (c0 + q < ne) ? (unsigned)cj * b.row_bytes + coff : BUF_SKIP;
        v[u] = buf_load<T, 0>(b.w, off);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int eb = c0 + (s0 + u) * G;  // first entry of this group of G
        if (eb >= ne) break;
        T val = v[u];
        // rows that end inside this group, before the tile's last entry
        // (the last row with entries is finished after the loop): their
        // entries are the ones below rend
        const int lim = min(eb + G, ne);
        while (rend < lim) {
          const bool mine = eb + grp < rend;
          acc += mine ? val : (T)0;
          val = mine ? (T)0 : val;
          const int rbeg = wave_uniform(wrp[r]);
          const T tot = rend == rbeg ? (T)0 : group_sum<KP>(acc);
          if (!idle) spmm_finish_b<T>(p, b, row0 + r, tot, lane, have, live, cfac, xo, dv, sp, nsv, rho, dm);
          acc = 0;
          ++r;
          const int nb = rend;
          rend = wave_uniform(wrp[r + 1]);
          idle = skip && rend == nb && nsv != row0 + r;
          if (!idle) {
            xo = plain ? (T)0 : buf_load<T, CP_NT>(b.xo, b.voff, row_off(b, row0 + r));
            dv = wave_uniform(load_dv<T>(p, row0 + r));
          }
        }
        acc += val;
      }
      }
      colv = coln;
    }
    if (rows) {
      while (r < nr) {  // last row with entries, then empty rows
        const T tot = wave_uniform(wrp[r + 1]) == wave_uniform(wrp[r]) ? (T)0 : group_sum<KP>(acc);
        if (!idle) spmm_finish_b<T>(p, b, row0 + r, tot, lane, have, live, cfac, xo, dv, sp, nsv, rho, dm);
        acc = 0;
        ++r;
        if (r < nr) {
          idle = skip && nsv != row0 + r;  // every row from here on has no entries
          if (!idle) {
            xo = plain ? (T)0 : buf_load<T, CP_NT>(b.xo, b.voff, row_off(b, row0 + r));
            dv = wave_uniform(load_dv<T>(p, row0 + r));
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();  // the next tile rewrites wrp
    } else {
      const int h = -td.y - 1;
      acc = group_sum<KP>(acc);
      spmm_hub_finish<T>(p, wave_uniform(plan.hubs[h]), h, td.x, sp, acc, lane, have, live, cfac);
    }
  }
  if (!plain) spmm_reduce(plan, p, rho, dm, sr, sd, &sflag);
}

// The same pass with 64-bit addressing, for operands of 4 GiB or more: the
// tile's column indices are staged in wave-private LDS.  It stores every
// row (p.skip_empty is not used), which leaves the zero rows the
// buffer-addressed pass relies on in place.
template <typename T>
__global__ __launch_bounds__(SB) void spmm_wide_kernel(TilePlanDev plan, SpmmArgs p, const GuardDev* guard) {
  constexpr int TE = WAVE_TILE_ENTRIES, TR = WAVE_TILE_ROWS, U = 16;
  if (guard && guard->active == 0) return;
  __shared__ double sr[SNW][64];
  __shared__ double sd[SNW][64];
  __shared__ __align__(16) int scol[SNW][TE + 16];  // padded: 16-entry reads past ne stay inside
  __shared__ int srp[SNW][TR + 1];
  __shared__ int sflag;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const bool have = lane < p.k;
  const bool live = column_live(p, lane);
  const T* W = (const T*)p.w;
  T cfac = (T)0;
  if (live) cfac = (T)(p.c_beta + (p.d_prev ? p.c_alpha * p.d_prev[lane] : 0.0));
  double rho = 0.0, dm = 0.0;
  int* wcol = scol[wv];
  int* wrp = srp[wv];

  const int nwaves = (int)gridDim.x * SNW;
  for (int t = (int)blockIdx.x * SNW + wv; t < plan.ntiles; t += nwaves) {
    const int4 td = plan.tiles[t];
    const int e0 = td.z, ne = td.w;
    for (int q = lane; q < ne; q += 64) wcol[q] = p.col[e0 + q];
    if (td.y > 0)
      for (int q = lane; q <= td.y; q += 64) wrp[q] = p.rowptr[td.x + q] - e0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    T acc = 0;
    int r = 0, sp = first_seed(p, t);
    int nsv = sp < p.nseeds ? p.seed_v[sp] : 0x7fffffff;
    const int row0 = td.x, nr = td.y;
    int rend = td.y > 0 ? wrp[1] : 0x7fffffff;
    T xo = td.y > 0 ? load_xo<T>(p, row0, lane, have) : (T)0;
    T dv = td.y > 0 ? load_dv<T>(p, row0) : (T)0;
    for (int base = 0; base < ne; base += U) {
      int cj[U];
#pragma unroll
      for (int u = 0; u < U; u += 4) {
        const int4 c4 = *reinterpret_cast<const int4*>(wcol + base + u);
        cj[u] = c4.x;
        cj[u + 1] = c4.y;
        cj[u + 2] = c4.z;
        cj[u + 3] = c4.w;
      }
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = (live && base + u < ne) ? W[(int64_t)cj[u] * p.k + lane] : (T)0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = base + u;
        if (e < ne) {
          while (e == rend) {
            spmm_finish<T>(p, row0 + r, acc, lane, have, live, cfac, xo, dv, sp, nsv, rho, dm);
            acc = 0;
            ++r;
            rend = wrp[r + 1];
            xo = load_xo<T>(p, row0 + r, lane, have);
            dv = load_dv<T>(p, row0 + r);
          }
          acc += v[u];
        }
      }
    }
    if (td.y > 0) {
      while (r < nr) {
        spmm_finish<T>(p, row0 + r, acc, lane, have, live, cfac, xo, dv, sp, nsv, rho, dm);
        acc = 0;
        ++r;
        if (r < nr) {
          xo = load_xo<T>(p, row0 + r, lane, have);
          dv = load_dv<T>(p, row0 + r);
        }
      }
    } else {
      const int h = -td.y - 1;
      spmm_hub_finish<T>(p, plan.hubs[h], h, td.x, sp, acc, lane, have, live, cfac);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // the next tile rewrites wcol / wrp
  }
  if (!p.plain) spmm_reduce(plan, p, rho, dm, sr, sd, &sflag);
}

// First seed (in vertex order) at or after the first row of each tile.
__global__ void spmm_tile_seed_kernel(TilePlanDev plan, const int* __restrict__ seed_v, int nseeds,
                                      int* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= plan.ntiles) return;
  const int4 td = plan.tiles[t];
  const int v = td.y > 0 ? td.x : plan.hubs[-td.y - 1].x;
  int lo = 0, hi = nseeds;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (seed_v[mid] < v) lo = mid + 1; else hi = mid;
  }
  out[t] = lo;
}

// x0 / w0 / D0 of the batch: x0 = V (seed weights), w0 = V .* d,
// D0_c = sum of the seed weights of column c on dangling vertices.
template <typename T>
__global__ void spmm_init_kernel(SpmmArgs p, const int* __restrict__ by_col_ptr,
                                 const int* __restrict__ by_col_v, const double* __restrict__ by_col_w,
                                 uint64_t cols) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= p.k || !((cols >> c) & 1ull)) return;
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

// Clears the selected columns of two n x k row-major blocks: one wavefront
// per row, lane c owns column c (k <= 64), so no lane divides an index.
__global__ void zero_columns_kernel(void* __restrict__ x, void* __restrict__ w, int type, int64_t n, int k,
                                    uint64_t cols) {
  const int lane = threadIdx.x & 63;
  const bool mine = lane < k && ((cols >> lane) & 1ull);
  const int64_t per_step = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; i < n; i += per_step) {
    if (!mine) continue;
    const int64_t q = i * k + lane;
    if (type == T_FP32) {
      ((float*)x)[q] = 0.f;
      ((float*)w)[q] = 0.f;
    } else {
      ((double*)x)[q] = 0.0;
      ((double*)w)[q] = 0.0;
    }
  }
}

// 64 rows per workgroup: the selected columns of the rows go through LDS
// (column c read from in1 when bit c of from1 is set, else from in0), then
// each leaves as 64 values at stride outs.ld.  Each thread issues its 16
// loads before it stores any of them, so a workgroup has its whole tile in
// flight.
template <typename T>
__global__ __launch_bounds__(256) void columns_out_kernel(const T* __restrict__ in0, const T* __restrict__ in1,
                                                          uint64_t from1, const int* __restrict__ idx, int64_t n,
                                                          int k, uint64_t cols, ColumnOutputs outs) {
  __shared__ T tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  T v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int q = (int)threadIdx.x + 256 * j;
    const int r = q >> 6, c = q & 63;  // one row per wavefront and step
    const int64_t i = r0 + r;
    v[j] = (T)0;
    if (i < n && c < k && ((cols >> c) & 1ull)) {
      const T* in = ((from1 >> c) & 1ull) ? in1 : in0;
      v[j] = in[(idx ? (int64_t)idx[i] : i) * k + c];
    }
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int q = (int)threadIdx.x + 256 * j;
    tile[q >> 6][q & 63] = v[j];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 64 * 64; q += 256) {
    const int c = q >> 6, r = q & 63;
    const int64_t i = r0 + r;
    if (i < n && c < k && ((cols >> c) & 1ull)) ((T*)outs.out[c])[i * outs.ld] = tile[r][c];
  }
}

// The reverse of columns_out: vector c < nc (n values) into column
// ins.dst[c] of the n-row array `out` (row stride ins.ld).  64 rows per
// workgroup go through LDS, so each vector is read in whole lines and,
// when nc = ins.ld, each row of `out` is written whole.
template <typename T>
__global__ __launch_bounds__(256) void columns_in_kernel(ColumnInputs ins, int nc, int64_t n, T* __restrict__ out) {
  __shared__ T tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  T v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int q = (int)threadIdx.x + 256 * j;
    const int c = q >> 6, r = q & 63;  // one vector per wavefront and step
    v[j] = (c < nc && r0 + r < n) ? ((const T*)ins.in[c])[r0 + r] : (T)0;
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int q = (int)threadIdx.x + 256 * j;
    tile[q & 63][q >> 6] = v[j];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 64 * 64; q += 256) {
    const int r = q >> 6, c = q & 63;
    if (c < nc && r0 + r < n) out[(r0 + r) * ins.ld + ins.dst[c]] = tile[r][c];
  }
}

// Columns map[j] (j < k2; map[j] < 0: an empty column) of the n x k
// iterate x into the n x k2 arrays x2 and w2 = x2 .* d (the product the
// pass stores, so w2 equals the pre-scaled copy it replaces), with the
// dangling masses; hit of the new columns: -1 for a live one, 0 (frozen)
// for an empty one.  One wavefront per row and four rows in flight, lane j
// owns new column j.
template <typename T>
__global__ __launch_bounds__(256) void compact_columns_kernel(const T* __restrict__ x, const T* __restrict__ dvec,
                                                              const double* __restrict__ d, T* __restrict__ x2,
                                                              T* __restrict__ w2, double* __restrict__ d2,
                                                              int* __restrict__ hit, int64_t n, int k, int k2,
                                                              ColumnMap map) {
  constexpr int R = 4;
  const int lane = threadIdx.x & 63;
  const int src = lane < k2 ? map.c[lane] : -1;
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    if (lane < k2) d2[lane] = src >= 0 ? d[src] : 0.0;
    hit[lane] = (lane < k2 && src >= 0) ? -1 : 0;
  }
  if (lane >= k2) return;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t i0 = ((int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) * R; i0 < n; i0 += waves * R) {
    T v[R], dv[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = i0 + u;
      v[u] = (i < n && src >= 0) ? x[i * k + src] : (T)0;
      dv[u] = i < n ? dvec[i] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t i = i0 + u;
      if (i < n) {
        x2[i * k2 + lane] = v[u];
        w2[i * k2 + lane] = v[u] * dv[u];
      }
    }
  }
}

__global__ void scatter_value_kernel(void* __restrict__ x, int type, const int* __restrict__ idx, int cnt,
                                     double v) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  if (type == T_FP32)
    ((float*)x)[idx[j]] = (float)v;
  else
    ((double*)x)[idx[j]] = v;
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
  if (grid <= 0 || a.k < 1 || a.k > 64 || (a.nseeds > 0 && !a.tile_seed)) return hipErrorInvalidValue;
  if (!a.plain && (!a.x_old || !a.dvec || !a.w_new || !a.rho_out || !a.d_out)) return hipErrorInvalidValue;
  const bool wide = a.w_bytes == 0;  // operand of 4 GiB or more
  if (wide) {
    if (type == T_FP32)
      hipLaunchKernelGGL(spmm_wide_kernel<float>, dim3(grid), dim3(SB), 0, s, plan, a, guard);
    else
      hipLaunchKernelGGL(spmm_wide_kernel<double>, dim3(grid), dim3(SB), 0, s, plan, a, guard);
    return hipGetLastError();
  }
  // k <= 16 columns: several entries per gathering load
  const int kp = a.k <= 4 ? 4 : a.k <= 8 ? 8 : a.k <= 16 ? 16 : 64;
  if (type == T_FP32) {
    if (kp == 4)
      hipLaunchKernelGGL((spmm_packed_kernel<float, 4>), dim3(grid), dim3(SB), 0, s, plan, a, guard);
    else if (kp == 8)
      hipLaunchKernelGGL((spmm_packed_kernel<float, 8>), dim3(grid), dim3(SB), 0, s, plan, a, guard);
    else if (kp == 16)
      hipLaunchKernelGGL((spmm_packed_kernel<float, 16>), dim3(grid), dim3(SB), 0, s, plan, a, guard);
    else
      hipLaunchKernelGGL(spmm_ppr_kernel<float>, dim3(grid), dim3(SB), 0, s, plan, a, guard);
  } else {
    if (kp == 4)
      hipLaunchKernelGGL((spmm_packed_kernel<double, 4>), dim3(grid), dim3(SB), 0, s, plan, a, guard);
    else if (kp == 8)
      hipLaunchKernelGGL((spmm_packed_kernel<double, 8>), dim3(grid), dim3(SB), 0, s, plan, a, guard);
    else if (kp == 16)
      hipLaunchKernelGGL((spmm_packed_kernel<double, 16>), dim3(grid), dim3(SB), 0, s, plan, a, guard);
    else
      hipLaunchKernelGGL(spmm_ppr_kernel<double>, dim3(grid), dim3(SB), 0, s, plan, a, guard);
  }
  return hipGetLastError();
}

hipError_t launch_spmm_tile_seed(const TilePlanDev& plan, const int* seed_v, int nseeds, int* out, hipStream_t s) {
  if (plan.ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(spmm_tile_seed_kernel, dim3((plan.ntiles + 255) / 256), dim3(256), 0, s, plan, seed_v, nseeds,
                     out);
  return hipGetLastError();
}

hipError_t launch_spmm_init(const SpmmArgs& a, int type, const int* by_col_ptr, const int* by_col_v,
                            const double* by_col_w, uint64_t cols, hipStream_t s) {
  if (type == T_FP32)
    hipLaunchKernelGGL(spmm_init_kernel<float>, dim3(1), dim3(64), 0, s, a, by_col_ptr, by_col_v, by_col_w, cols);
  else
    hipLaunchKernelGGL(spmm_init_kernel<double>, dim3(1), dim3(64), 0, s, a, by_col_ptr, by_col_v, by_col_w, cols);
  return hipGetLastError();
}

hipError_t launch_spmm_zero_columns(void* x, void* w, int type, int64_t n, int k, uint64_t cols, hipStream_t s) {
  if (n <= 0 || !cols || k < 1 || k > 64) return n <= 0 || !cols ? hipSuccess : hipErrorInvalidValue;
  int64_t g = (n + 3) / 4;  // four rows per 256-thread workgroup and step
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(zero_columns_kernel, dim3((int)g), dim3(256), 0, s, x, w, type, n, k, cols);
  return hipGetLastError();
}

hipError_t launch_spmm_columns_out(const void* in0, const void* in1, uint64_t from1, int type, const int* idx,
                                   int64_t n, int k, uint64_t cols, const ColumnOutputs& outs, hipStream_t s) {
  if (n <= 0 || !cols) return hipSuccess;
  if (k < 1 || k > 64 || outs.ld < 1) return hipErrorInvalidValue;
  const int g = (int)((n + 63) / 64);
  if (type == T_FP32)
    hipLaunchKernelGGL(columns_out_kernel<float>, dim3(g), dim3(256), 0, s, (const float*)in0, (const float*)in1,
                       from1, idx, n, k, cols, outs);
  else
    hipLaunchKernelGGL(columns_out_kernel<double>, dim3(g), dim3(256), 0, s, (const double*)in0,
                       (const double*)in1, from1, idx, n, k, cols, outs);
  return hipGetLastError();
}

hipError_t launch_columns_in(const ColumnInputs& ins, int nc, int type, int64_t n, void* out, hipStream_t s) {
  if (n <= 0 || nc <= 0) return hipSuccess;
  if (nc > 64 || ins.ld < 1) return hipErrorInvalidValue;
  for (int c = 0; c < nc; ++c)
    if (!ins.in[c] || ins.dst[c] < 0 || ins.dst[c] >= ins.ld) return hipErrorInvalidValue;
  const int g = (int)((n + 63) / 64);
  if (type == T_FP32)
    hipLaunchKernelGGL(columns_in_kernel<float>, dim3(g), dim3(256), 0, s, ins, nc, n, (float*)out);
  else
    hipLaunchKernelGGL(columns_in_kernel<double>, dim3(g), dim3(256), 0, s, ins, nc, n, (double*)out);
  return hipGetLastError();
}

hipError_t launch_spmm_compact(const void* x, const void* dvec, const double* d, void* x2, void* w2, double* d2,
                               int* hit, int type, int64_t n, int k, int k2, const ColumnMap& map, hipStream_t s) {
  if (k < 1 || k > 64 || k2 < 1 || k2 > 64) return hipErrorInvalidValue;
  for (int j = 0; j < k2; ++j)
    if (map.c[j] >= k) return hipErrorInvalidValue;
  int64_t g = (n + 15) / 16;  // four wavefronts of four rows per 256-thread workgroup and step
  if (g > 16384) g = 16384;
  if (g < 1) g = 1;
  if (type == T_FP32)
    hipLaunchKernelGGL(compact_columns_kernel<float>, dim3((int)g), dim3(256), 0, s, (const float*)x,
                       (const float*)dvec, d, (float*)x2, (float*)w2, d2, hit, n, k, k2, map);
  else
    hipLaunchKernelGGL(compact_columns_kernel<double>, dim3((int)g), dim3(256), 0, s, (const double*)x,
                       (const double*)dvec, d, (double*)x2, (double*)w2, d2, hit, n, k, k2, map);
  return hipGetLastError();
}

hipError_t launch_scatter_value(void* x, int type, const int* idx, int cnt, double v, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_value_kernel, dim3((cnt + 255) / 256), dim3(256), 0, s, x, type, idx, cnt, v);
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
