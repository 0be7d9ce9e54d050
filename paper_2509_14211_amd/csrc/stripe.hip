// Stripe-blocked fused PageRank pass (FP32 ranks), the plan kind for graphs
// whose gathered vector is far larger than LDS.
//
// The pass computes the same thing as the other fused kernels (paper,
// Fig. 6: the pre-scaled operand w gathered by the mxv over A^T, the
// teleport/dangling add, the L1 residual and the dangling mass), but it
// reorganises the mxv so that most gathers read LDS instead of memory:
//
//   * Rows of A^T are cut into stripes of at most STRIPE_RMAX rows.  A
//     workgroup keeps the stripe's row sums in LDS.
//   * Columns (sources) are cut into blocks of STRIPE_HB.  Each stripe
//     loads the blocks that hold most of its entries: with vertices
//     renumbered by decreasing out-degree these are the leading blocks (at
//     R-MAT scale 22 the first 8 blocks draw 80% of all gathers); on a
//     graph whose links are mostly local they are the blocks around the
//     stripe's own rows.  For each of its LDS blocks the stripe stores the
//     entries that fall in it as packed words (row in the stripe << 16 |
//     column in the block), sorted by row; the workgroup loads the block of
//     w into LDS once and every such entry reads LDS.
//   * The stripe's remaining entries (columns outside its LDS blocks) are
//     stored as (column, row in the stripe) pairs and gathered from memory
//     while the next block loads.
//   * Row sums are accumulated exactly in 64-bit fixed point with LDS
//     integer atomics: w values are scaled by 2^F, where 2^(62-F) bounds
//     sum |w| -- a row adds distinct entries of w, so no partial sum can
//     overflow -- and integer addition makes the sum independent of the
//     order in which lanes and wavefronts add.  Each lane first adds runs
//     of equal rows among its own entries in registers.  Each term is
//     truncated to the 2^-F grid (at most 2^-62 sum |w| per term; F is
//     capped at 126, so a vector with sum |w| below 2^-64 keeps a grid of
//     2^-126) and the exact sum is rounded once to FP32.
//   * Per row the epilogue is the usual one; it also publishes sum |w'| of
//     the pre-scaled copy it writes (FP64), which the next pass uses for its
//     scale.
//
// The layout is built on the GPU once per matrix and plan: counts of each
// stripe's entries per column block, the choice of the blocks a stripe
// loads (those with the most of its entries, each only when enough of them
// fall in it to pay for reading it), and a stable partition of each
// stripe's entries into its segments (no sort, no temporary arrays).  Stripes are
// assigned to workgroups by longest-processing-time-first on an estimate of
// their cost, so results do not depend on scheduling.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <queue>
#include <vector>

#include "device_util.h"
#include "ops_device.h"
#include "runtime.h"

namespace nbgrb {

namespace {

constexpr int NCLS = STRIPE_NBMAX + 1;  // column classes of a stripe: the LDS blocks, then the rest
constexpr int CHUNK = 64 * STRIPE_K;    // entries one wavefront takes at a time

template <typename V>
__device__ __forceinline__ V wave_sum64(V v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename V, int B>
__device__ __forceinline__ V block_sum_st(V v, V* red) {
  v = wave_sum64(v);
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

// v * 2^F as a two's-complement 64-bit integer, truncated toward zero,
// with fm32 = F - 32.  y = |v| * 2^(F-32) is exact (a power-of-two
// scaling; where y would be subnormal, |v| * 2^F < 1 and the result is 0
// either way), and since |v| * 2^F < 2^62, y < 2^30: the high word is
// floor(y) and the low word floor(frac(y) * 2^32), both exact conversions;
// the sign is applied to the 64-bit pair.  With F <= 126 a subnormal v
// gives 0, as v * 2^F < 1, so this is the exact truncation for every
// float (checked against the bit-level form mant * 2^(E - 150) shifted
// into place, on every exponent, both signs, zeros and subnormals).
__device__ __forceinline__ long long fixed_of(float v, int fm32) {
  const float y = __builtin_amdgcn_ldexpf(__builtin_fabsf(v), fm32);
  const unsigned hi = (unsigned)y;
  const unsigned lo = (unsigned)__builtin_amdgcn_ldexpf(__builtin_amdgcn_fractf(y), 32);
  const unsigned long long q = ((unsigned long long)hi << 32) | lo;
  const unsigned long long sg = (unsigned long long)(long long)((int)__float_as_uint(v) >> 31);
  return (long long)((q ^ sg) - sg);
}

// Adds a lane's entries into the LDS row sums: runs of equal rows are
// summed in registers first.  When the whole wavefront holds one row (a
// long row), one lane adds the wavefront's total.  SORTED: the wavefront's
// rows ascend across lanes (padding rows 0 at the end), so the first and
// the last row decide that; otherwise every row is compared.
template <int K, bool SORTED>
__device__ __forceinline__ void add_runs(unsigned long long* acc, const int (&row)[K], const float (&v)[K],
                                         int fm32) {
  const int first = lane_value(row[0], 0);
  bool one_row;
  if constexpr (SORTED) {
    one_row = first == lane_value(row[K - 1], 63);
  } else {
    bool mine = true;
#pragma unroll
    for (int k = 0; k < K; ++k) mine = mine && row[k] == first;
    one_row = __ballot(mine) == ~0ull;
  }
  if (one_row) {
    long long s = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) s += fixed_of(v[k], fm32);
    s = wave_sum64(s);
    if ((threadIdx.x & 63) == 0) atomicAdd(&acc[first], (unsigned long long)s);
    return;
  }
  int cur = row[0];
  long long s = fixed_of(v[0], fm32);
#pragma unroll
  for (int k = 1; k < K; ++k) {
    if (row[k] != cur) {
      atomicAdd(&acc[cur], (unsigned long long)s);
      cur = row[k];
      s = 0;
    }
    s += fixed_of(v[k], fm32);
  }
  atomicAdd(&acc[cur], (unsigned long long)s);
}

// The workgroup's LDS block after LDS block b of the stripe at list
// position si: the next one of the same stripe, else the first of the next
// stripe in the list that loads any (b = -1: the first of stripe si or
// later), and its column block.  Returns false when there is none.
__device__ __forceinline__ bool next_block(const StripePlanDev& p, int si, int s_end, int b, int& nsi, int& nb_,
                                           int& col_blk) {
  if (si < s_end) {
    const StripeDesc* d = p.desc + wave_uniform(p.wg_list[si]);
    if (b + 1 < wave_uniform(d->nb)) {
      nsi = si;
      nb_ = b + 1;
      col_blk = wave_uniform(d->blk[b + 1]);
      return true;
    }
  }
  for (int k = si + 1; k < s_end; ++k) {
    const StripeDesc* d = p.desc + wave_uniform(p.wg_list[k]);
    if (wave_uniform(d->nb) > 0) {
      nsi = k;
      nb_ = 0;
      col_blk = wave_uniform(d->blk[0]);
      return true;
    }
  }
  return false;
}

// Block b of the gathered vector straight into LDS buffer `buf` (no
// registers): wavefront wv of nw writes the block's 1 KiB pieces wv,
// wv + nw, ..., 16 bytes per lane, with memory-to-LDS loads.  Past the end
// of the vector the loads return zeros.  The writes are complete once the
// wavefront's vector-memory counter reaches zero (wait_block).
__device__ __forceinline__ void dma_block(const float* w, int ncols, int b, float* buf, int wv, int nw, int lane) {
  constexpr int PIECES = STRIPE_HB * 4 / 1024;
  const int b0 = b * STRIPE_HB;
  const int cnt = min(STRIPE_HB, ncols - b0);
  const __amdgpu_buffer_rsrc_t rb = buf_rsrc(w + b0, (unsigned)(cnt > 0 ? cnt : 0) * 4u);
  for (int q = wv; q < PIECES; q += nw)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (__attribute__((address_space(3))) void*)(buf + q * 256), 16,
                                             (unsigned)(q * 1024 + lane * 16), 0, 0, 0);
}

// This wavefront's memory-to-LDS loads (and every other load it issued)
// have completed.
__device__ __forceinline__ void wait_block() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Hot item (phase b, chunk j) of a hot wavefront within a stripe: chunks
// h, h + nh, ... of each LDS block's segment in turn (h = its index among
// the nh hot wavefronts).  Segment starts come from a register holding
// seg[lane] in lane `lane`, read with v_readlane: a scalar memory load here
// would wait for the wavefront's LDS operations too (one counter tracks
// both).
struct HotCursor {
  int b, j;
};

__device__ __forceinline__ int seg_at(int segv, int b) { return __builtin_amdgcn_readlane(segv, b); }

__device__ __forceinline__ void hot_settle(int segv, int nb, int h, HotCursor& c) {
  while (c.b < nb && c.j * CHUNK >= seg_at(segv, c.b + 1) - seg_at(segv, c.b)) {
    ++c.b;
    c.j = h;
  }
}

template <int SP>
__device__ __forceinline__ void hot_words(const unsigned* hot_seg0, int segv, const HotCursor& c, int lane,
                                          uint4& wa, uint4& wb) {
  const int sb0 = seg_at(segv, c.b), sb1 = seg_at(segv, c.b + 1);
  const __amdgpu_buffer_rsrc_t rh = buf_rsrc(hot_seg0 + sb0, (unsigned)(sb1 - sb0) * 4u);
  const unsigned e = (unsigned)(c.j * CHUNK + lane * STRIPE_K);
  wa = buf_load<uint4, SP>(rh, e * 4u);
  wb = buf_load<uint4, SP>(rh, e * 4u + 16u);
}

// Registers of one chunk of gathered entries: column indices, rows in the
// stripe (16 bits each) and the gathered values.
struct ColdRegs {
  uint4 ca, cb, rr;
  float v[STRIPE_K];
};

// Indices of chunk `ch` (past the end the loads return zeros: column 0,
// row slot 0).
template <int SP>
__device__ __forceinline__ void cold_indices(__amdgpu_buffer_rsrc_t rcc, __amdgpu_buffer_rsrc_t rcr, int ch,
                                             int lane, ColdRegs& R) {
  const unsigned e = (unsigned)(ch * CHUNK + lane * STRIPE_K);
  R.ca = buf_load<uint4, SP>(rcc, e * 4u);
  R.cb = buf_load<uint4, SP>(rcc, e * 4u + 16u);
  R.rr = buf_load<uint4, SP>(rcr, e * 2u);
}

__device__ __forceinline__ void cold_gather(__amdgpu_buffer_rsrc_t rw, ColdRegs& R) {
  const unsigned col[STRIPE_K] = {R.ca.x, R.ca.y, R.ca.z, R.ca.w, R.cb.x, R.cb.y, R.cb.z, R.cb.w};
#pragma unroll
  for (int k = 0; k < STRIPE_K; ++k) R.v[k] = buf_load<float>(rw, col[k] * 4u);
}

// PF: the chunk's values were loaded in place of its columns (two-phase
// plan, entries grouped by column block, rows ascending only within a
// group); otherwise they were gathered into R.v.
template <bool PF>
__device__ __forceinline__ void cold_add(unsigned long long* acc, const ColdRegs& R, int fm32) {
  const int row[STRIPE_K] = {(int)(R.rr.x & 0xFFFFu), (int)(R.rr.x >> 16), (int)(R.rr.y & 0xFFFFu),
                             (int)(R.rr.y >> 16),     (int)(R.rr.z & 0xFFFFu), (int)(R.rr.z >> 16),
                             (int)(R.rr.w & 0xFFFFu), (int)(R.rr.w >> 16)};
  if constexpr (PF) {
    const float v[STRIPE_K] = {__uint_as_float(R.ca.x), __uint_as_float(R.ca.y), __uint_as_float(R.ca.z),
                               __uint_as_float(R.ca.w), __uint_as_float(R.cb.x), __uint_as_float(R.cb.y),
                               __uint_as_float(R.cb.z), __uint_as_float(R.cb.w)};
    add_runs<STRIPE_K, false>(acc, row, v, fm32);
  } else {
    add_runs<STRIPE_K, true>(acc, row, R.v, fm32);
  }
}

}  // namespace

// One workgroup per compute unit; workgroup g runs stripes
// wg_list[wg_off[g] .. wg_off[g+1]) one after the other.  Per stripe, all
// wavefronts first gather the entries outside the LDS blocks (software-
// pipelined), then add the entries of each LDS block in turn.  The LDS
// blocks of all the workgroup's stripes form one sequence: while block k
// is read from buffer k mod 2, block k+1 streams from memory straight into
// the other buffer (one workgroup barrier per block).
template <int SP, bool PF>
__global__ __launch_bounds__(STRIPE_BLOCK) void fused_stripe_kernel(StripePlanDev p, FusedArgs<float> a,
                                                                    const double* wsum_in, double* wsum_out,
                                                                    FusedScratch scr, const GuardDev* guard) {
  constexpr int B = STRIPE_BLOCK;
  constexpr int NW = B / 64;
  constexpr int ER = (STRIPE_RMAX + B - 1) / B;  // epilogue rows per thread
  static_assert(STRIPE_HB % 256 == 0, "blocks are loaded in whole 1 KiB pieces");
  if (guard && guard->active == 0) return;

  __shared__ unsigned long long acc[STRIPE_RMAX + 1];  // slot 0 takes the padding entries
  __shared__ __attribute__((aligned(16))) float hot[2][STRIPE_HB];
  __shared__ double sred[NW];
  __shared__ int sflag;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = wave_uniform(tid >> 6);
  const bool pr = a.mode == EPI_PR;
  float c = 0.0f;
  if (pr) c = (float)scalar_value(a.c);

  // fixed-point scale: 2^(62-F) >= sum |w|.  Every partial sum of a row
  // adds distinct entries of w, so its magnitude is at most sum |w|.  F is
  // capped at 126 (a vector whose sum |w| is below 2^-64 keeps a grid of
  // 2^-126, the smallest normal FP32 value).
  const double wsum = *wsum_in;
  const bool finite = __builtin_isfinite(wsum);
  int F = 62;
  if (finite && wsum > 0.0) {
    int k = 0;
    (void)frexp(wsum, &k);  // wsum < 2^k
    F = 62 - k;
  }
  if (F > 126) F = 126;
  const int fm32 = F - 32;
  const double unscale = ldexp(1.0, -F);

  const __amdgpu_buffer_rsrc_t rw = buf_rsrc(a.w, (unsigned)a.ncols * 4u);
  double rho = 0.0, dm = 0.0;
  double wsm = 0.0;  // sum |w'| of this thread's rows

  const int g = blockIdx.x;
  const int s_begin = p.wg_off[g], s_end = p.wg_off[g + 1];

  for (int i = tid; i <= STRIPE_RMAX; i += B) acc[i] = 0ull;
  // LDS block sequence: (bsi, bb) is the last block requested
  int kblk = 0;  // blocks consumed so far: the next one sits in hot[kblk & 1]
  int bsi = s_begin, bb = -1, bcol = 0;
  bool more = s_begin < s_end && next_block(p, bsi, s_end, bb, bsi, bb, bcol);
  if (more) dma_block(a.w, a.ncols, bcol, hot[0], wv, NW, lane);
  wait_block();
  __syncthreads();

  for (int si = s_begin; si < s_end; ++si) {
    const int s = wave_uniform(p.wg_list[si]);
    const StripeDesc* dp = p.desc + s;
    const int r0 = wave_uniform(dp->r0), nrows = wave_uniform(dp->nrows);
    const int nb = wave_uniform(dp->nb), cold_n = wave_uniform(dp->cold_n);
    const long long hot_base = dp->hot_base, cold_base = dp->cold_base;
    const int ncold = (cold_n + CHUNK - 1) / CHUNK;
    // the gathered entries' columns, or in a two-phase plan their values
    const __amdgpu_buffer_rsrc_t rcc =
        PF ? buf_rsrc(p.cold_val + cold_base, (unsigned)cold_n * 4u) : buf_rsrc(p.cold_col + cold_base, (unsigned)cold_n * 4u);
    const __amdgpu_buffer_rsrc_t rcr = buf_rsrc(p.cold_row + cold_base, (unsigned)cold_n * 2u);
    const int segv = lane <= nb ? dp->seg[lane] : 0;
    const unsigned* hot_seg0 = p.hot + hot_base;
    // the first chunk of this wavefront's LDS-block entries is requested
    // now, so its latency overlaps the gathered entries below
    HotCursor cur{0, wv};
    hot_settle(segv, nb, wv, cur);
    uint4 wa = make_uint4(0, 0, 0, 0), wb = make_uint4(0, 0, 0, 0);
    if (cur.b < nb) hot_words<SP>(hot_seg0, segv, cur, lane, wa, wb);

    // Entries outside the LDS blocks, gathered from memory first: this
    // wavefront's chunks wv, wv + 16, ...  Three register sets rotate so the
    // indices of chunk i+2 and the gathers of chunk i+1 are in flight while
    // chunk i is added (unrolled by three: no set is ever copied, which
    // would wait for its loads).
    {
      const int nk = ncold > wv ? (ncold - wv + NW - 1) / NW : 0;
      if (nk > 0) {
        ColdRegs X, Y, Z;
        cold_indices<SP>(rcc, rcr, wv, lane, X);
        cold_indices<SP>(rcc, rcr, wv + NW, lane, Y);
        if constexpr (!PF) cold_gather(rw, X);
        auto step = [&](int i, ColdRegs& P, ColdRegs& G, ColdRegs& F) {
          cold_indices<SP>(rcc, rcr, wv + (i + 2) * NW, lane, F);
          if constexpr (!PF) cold_gather(rw, G);
          cold_add<PF>(acc, P, fm32);
        };
        for (int i = 0;;) {
          step(i, X, Y, Z);
          if (++i >= nk) break;
          step(i, Y, Z, X);
          if (++i >= nk) break;
          step(i, Z, X, Y);
          if (++i >= nk) break;
        }
      }
    }

    // entries in the LDS blocks, one block per phase
    for (int b = 0; b < nb; ++b) {
      // block kblk + 1 of the sequence into the other buffer, whose last
      // readers (phase kblk - 1) passed the barrier that ended their phase
      more = more && next_block(p, bsi, s_end, bb, bsi, bb, bcol);
      if (more) dma_block(a.w, a.ncols, bcol, hot[(kblk + 1) & 1], wv, NW, lane);
      const float* hbuf = hot[kblk & 1];
      while (cur.b == b) {
        const uint4 ca = wa, cb = wb;
        HotCursor nx{cur.b, cur.j + NW};
        hot_settle(segv, nb, wv, nx);
        if (nx.b < nb) hot_words<SP>(hot_seg0, segv, nx, lane, wa, wb);
        const unsigned wd[STRIPE_K] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
        int row[STRIPE_K];
        float v[STRIPE_K];
#pragma unroll
        for (int k = 0; k < STRIPE_K; ++k) {
          row[k] = (int)(wd[k] >> 16);
          v[k] = hbuf[wd[k] & 0xFFFFu];
        }
        add_runs<STRIPE_K, true>(acc, row, v, fm32);
        cur = nx;
      }
      wait_block();  // this wavefront's part of block kblk + 1 is in LDS
      __syncthreads();
      ++kblk;
    }
    if (nb == 0) __syncthreads();  // every gathered entry added

    // epilogue: rows of the stripe (all loads issued first); each slot is
    // cleared for the next stripe
    float xo[ER], dv[ER];
#pragma unroll
    for (int k = 0; k < ER; ++k) {
      const int r = tid + k * B;
      xo[k] = (r < nrows && pr && a.x_old) ? __builtin_nontemporal_load(a.x_old + r0 + r) : 0.0f;
      dv[k] = (r < nrows && pr && a.dvec) ? __builtin_nontemporal_load(a.dvec + r0 + r) : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < ER; ++k) {
      const int r = tid + k * B;
      if (r >= nrows) continue;
      const int i = r0 + r;
      const long long q = (long long)acc[r + 1];
      acc[r + 1] = 0ull;
      const float sv = finite ? (float)((double)q * unscale) : __builtin_nanf("");
      if (!pr) {
        a.s_out[i] = sv;
        continue;
      }
      const float tele = a.tele_vec ? (a.tele_scaled ? a.tele_vec[i] * c : a.tele_vec[i]) : c;
      const float rv = tele + sv;
      if (a.r_out) __builtin_nontemporal_store(rv, a.r_out + i);
      if (a.x_old) rho += fabs((double)xo[k] - (double)rv);
      if (a.w_out) {
        const float wn = a.memo_div ? rv / dv[k] : rv * dv[k];
        a.w_out[i] = wn;
        wsm += fabs((double)wn);
      }
      if (a.do_D) {
        const bool m = a.mask_is_dvec ? (dv[k] != 0.0f) : nonzero_at(a.mask, i);
        if (m != (a.mask_comp != 0)) dm += (double)rv;
      }
    }
    if (tid == 0) acc[0] = 0ull;
    __syncthreads();  // slots are clear before the next stripe adds into them
  }

  const bool reduce = (pr && (a.rho_out.out || a.D_out.out || a.rho_out.guard)) || wsum_out;
  if (!reduce) return;
  const double br = block_sum_st<double, B>(rho, sred);
  const double bd = block_sum_st<double, B>(dm, sred);
  const double bw = block_sum_st<double, B>(wsm, sred);
  if (tid == 0) {
    publish(&scr.wg_part[2 * g], br);
    publish(&scr.wg_part[2 * g + 1], bd);
    publish(&p.wg_sum[g], bw);
    wait_stores();
    sflag = ticket_add(scr.ticket) == gridDim.x - 1;
  }
  __syncthreads();
  if (!sflag) return;
  double pr_ = 0.0, pd = 0.0, pw = 0.0;
  for (int k = tid; k < (int)gridDim.x; k += B) {
    pr_ += consume(&scr.wg_part[2 * k]);
    pd += consume(&scr.wg_part[2 * k + 1]);
    pw += consume(&p.wg_sum[k]);
  }
  const double tr = block_sum_st<double, B>(pr_, sred);
  const double tdm = block_sum_st<double, B>(pd, sred);
  const double tw = block_sum_st<double, B>(pw, sred);
  if (tid == 0) {
    if (pr) {
      if (a.rho_out.out) *a.rho_out.out = tr;
      if (a.D_out.out) *a.D_out.out = tdm;
      if (a.rho_out.guard) guard_advance(a.rho_out.guard, tr, a.do_D ? tdm : 0.0);
    }
    if (wsum_out) *wsum_out = tw;
    publish(scr.ticket, 0u);
  }
}

hipError_t launch_fused_stripe_f32(const StripePlanDev& p, const FusedArgs<float>& a, const double* wsum_in,
                                   double* wsum_out, const FusedScratch& scr, int grid, bool nt_streams,
                                   bool prefilled, const GuardDev* guard, hipStream_t s) {
  if (grid <= 0 || !wsum_in || (prefilled && !p.cold_val) || (!prefilled && !p.cold_col && p.nstripes > 0))
    return hipErrorInvalidValue;
  const dim3 g(grid), b(STRIPE_BLOCK);
  if (prefilled) {
    if (nt_streams)
      hipLaunchKernelGGL((fused_stripe_kernel<CP_NT, true>), g, b, 0, s, p, a, wsum_in, wsum_out, scr, guard);
    else
      hipLaunchKernelGGL((fused_stripe_kernel<0, true>), g, b, 0, s, p, a, wsum_in, wsum_out, scr, guard);
  } else {
    if (nt_streams)
      hipLaunchKernelGGL((fused_stripe_kernel<CP_NT, false>), g, b, 0, s, p, a, wsum_in, wsum_out, scr, guard);
    else
      hipLaunchKernelGGL((fused_stripe_kernel<0, false>), g, b, 0, s, p, a, wsum_in, wsum_out, scr, guard);
  }
  return hipGetLastError();
}

namespace {

// Phase one of a two-phase pass: chunks of the fill list in turn; the
// chunk's column block of w goes to LDS, then each entry's value to its
// slot (the list is ordered by slot within a block, so the writes run
// along each stripe's group of entries from that block).
//
// Consecutive chunks mostly share a column block.  Workgroup g runs on XCD
// g mod 8, so with a grid that is a multiple of 8·FILL_GROUP each round of
// gridDim.x chunks is dealt out in groups of FILL_GROUP consecutive chunks,
// group i to the workgroups of XCD i mod 8: a block then comes from memory
// into one or two XCDs' L2 instead of into most of them.  Any assignment
// gives the same values (each chunk writes only its own slots).
constexpr int FILL_GROUP = 8;

__global__ __launch_bounds__(512) void cold_fill_kernel(ColdFillDev f, const float* __restrict__ w, int ncols,
                                                        const GuardDev* guard) {
  constexpr int NWF = 512 / 64;
  if (guard && guard->active == 0) return;
  __shared__ __attribute__((aligned(16))) float win[STRIPE_HB];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long le = (2ull << lane) - 1ull;  // lanes up to and including this one
  int c0 = blockIdx.x;
  if ((gridDim.x % (8 * FILL_GROUP)) == 0) {
    const int x = blockIdx.x & 7, k = blockIdx.x >> 3;  // XCD, and rank among its workgroups
    c0 = ((k / FILL_GROUP) * 8 + x) * FILL_GROUP + k % FILL_GROUP;
  }
  for (int c = c0; c < f.nchunks; c += gridDim.x) {
    const ColdChunk ch = f.chunk[c];
    const int b0 = ch.blk * STRIPE_HB;
    const int cnt = min(STRIPE_HB, ncols - b0);
    __syncthreads();  // the previous chunk's reads of win are done
    if (cnt == STRIPE_HB && ((uintptr_t)(w + b0) & 15u) == 0) {
      for (int i = threadIdx.x; i < STRIPE_HB / 4; i += blockDim.x)
        ((float4*)win)[i] = ((const float4*)(w + b0))[i];
    } else {
      for (int i = threadIdx.x; i < cnt; i += blockDim.x) win[i] = w[b0 + i];
    }
    __syncthreads();
    // one wavefront per sub-chunk: an entry's run is the last run start at
    // or before it (a ballot over the wavefront, carried between steps)
    const unsigned nsub = (ch.end - ch.start + FILL_SUB - 1) / FILL_SUB;
    for (unsigned j = wv; j < nsub; j += NWF) {
      const unsigned s0 = ch.start + j * FILL_SUB, s1 = min(s0 + FILL_SUB, ch.end);
      unsigned run = f.sub_run[ch.sub0 + j] - 1u;  // s0 starts a run
      unsigned first = s0;
      // U groups of 64 entries at a time: their loads are in flight
      // together, and the next U groups' columns load while these groups'
      // run slots are read and their values stored (two register sets
      // alternate, so neither is copied while its loads are in flight)
      constexpr int U = 8;
      auto load_words = [&](unsigned g0, unsigned (&word)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const unsigned e = g0 + 64u * u + lane;
          word[u] = e < s1 ? (unsigned)f.src[e] : 0u;
        }
      };
      auto place = [&](unsigned g0, const unsigned (&word)[U]) {
        unsigned my_run[U], my_first[U], rp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const unsigned e0 = g0 + 64u * u;
          const unsigned long long bw = __ballot(e0 + lane < s1 && (word[u] & 0x8000u));
          const unsigned long long m = bw & le;
          my_run[u] = run + (unsigned)__popcll(m);
          my_first[u] = m ? e0 + (63u - (unsigned)__clzll(m)) : first;
          run += (unsigned)__popcll(bw);
          if (bw) first = e0 + (63u - (unsigned)__clzll(bw));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) rp[u] = g0 + 64u * u + lane < s1 ? f.run_pos[my_run[u]] : 0u;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const unsigned e = g0 + 64u * u + lane;
          if (e < s1) f.val[rp[u] + (e - my_first[u])] = win[word[u] & 0x3FFFu];
        }
      };
      constexpr unsigned GS = 64u * U;
      unsigned wa[U], wb[U];
      load_words(s0, wa);
      for (unsigned g0 = s0; g0 < s1; g0 += 2 * GS) {
        if (g0 + GS < s1) load_words(g0 + GS, wb);
        place(g0, wa);
        if (g0 + GS >= s1) break;
        if (g0 + 2 * GS < s1) load_words(g0 + 2 * GS, wa);
        place(g0 + GS, wb);
      }
    }
  }
}

}  // namespace

hipError_t launch_cold_fill_f32(const ColdFillDev& f, const float* w, int ncols, const GuardDev* guard,
                                hipStream_t s) {
  if (f.nchunks <= 0) return hipSuccess;
  if (!f.src || !f.run_pos || !f.sub_run || !f.chunk || !f.val || !w) return hipErrorInvalidValue;
  const int grid = std::min(f.nchunks, std::max(1, ctx().cus) * 3);
  hipLaunchKernelGGL(cold_fill_kernel, dim3(grid), dim3(512), 0, s, f, w, ncols, guard);
  return hipGetLastError();
}

// ------------------------------------------------------------ max |x|

// Deterministic two-level FP64 sum of |x| into *out: per-workgroup sums,
// then the last workgroup adds them in workgroup order.
__global__ __launch_bounds__(256) void abssum_kernel(const float* x, int64_t n, double* out, RedScratch scr,
                                                      const GuardDev* guard) {
  if (guard && guard->active == 0) return;
  __shared__ double red[4];
  __shared__ int sflag;
  double a = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) a += fabs((double)x[i]);
  a = block_sum_st<double, 256>(a, red);
  if (threadIdx.x == 0) {
    publish(&scr.partials[blockIdx.x], a);
    wait_stores();
    sflag = ticket_add(scr.ticket) == gridDim.x - 1;
  }
  __syncthreads();
  if (!sflag) return;
  double t = 0.0;
  for (int k = threadIdx.x; k < (int)gridDim.x; k += 256) t += consume(&scr.partials[k]);
  t = block_sum_st<double, 256>(t, red);
  if (threadIdx.x == 0) {
    *out = t;
    publish(scr.ticket, 0u);
  }
}

hipError_t launch_abssum_f32(const float* x, int64_t n, double* out, RedScratch scr, const GuardDev* guard,
                             hipStream_t s) {
  int64_t g = (n + 256 * 8 - 1) / (256 * 8);
  if (g < 1) g = 1;
  if (g > REDUCE_GRID) g = REDUCE_GRID;
  hipLaunchKernelGGL(abssum_kernel, dim3((int)g), dim3(256), 0, s, x, n, out, scr, guard);
  return hipGetLastError();
}

// ------------------------------------------------------------ layout build

namespace {

// The LDS blocks of stripe s: entries per column block counted in an LDS
// histogram (blocks at or past nbins - 1 share the last bin when
// `merged`, and that bin is never chosen), then up to nb_cap rounds pick
// the bin with the most entries (ties: the lower block) while it holds at
// least min_entries.  Writes nbs[s], the chosen blocks ascending in
// blk[s][..] with their entry counts in hcnt[s][..], and cold[s] = the
// stripe's other entries.  One workgroup per stripe.
__global__ __launch_bounds__(1024) void st_select_kernel(const int* rowptr, const int* col, const int* sr0,
                                                         int nbins, int merged, int nb_cap, int min_entries,
                                                         int* nbs, int* blk, int* hcnt, int* cold) {
  __shared__ int h[STRIPE_MAXBLK];
  __shared__ unsigned long long red[16];
  __shared__ unsigned long long pick;
  __shared__ int sb[STRIPE_NBMAX], sc[STRIPE_NBMAX];
  const int s = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int i = t; i < nbins; i += 1024) h[i] = 0;
  __syncthreads();
  const int e0 = rowptr[sr0[s]], e1 = rowptr[sr0[s + 1]];
  for (int e = e0 + t; e < e1; e += 1024) atomicAdd(&h[min(col[e] / STRIPE_HB, nbins - 1)], 1);
  __syncthreads();
  const int choosable = merged ? nbins - 1 : nbins;
  int k = 0;
  for (; k < nb_cap; ++k) {
    // key: count in the high half, ~bin in the low half (larger count, then
    // lower bin, wins)
    unsigned long long best = 0;
    for (int i = t; i < choosable; i += 1024) {
      const int c = h[i];
      if (c > 0) {
        const unsigned long long key = ((unsigned long long)(unsigned)c << 32) | (unsigned)(~(unsigned)i);
        best = key > best ? key : best;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long other = __shfl_xor(best, o, 64);
      best = other > best ? other : best;
    }
    if (lane == 0) red[w] = best;
    __syncthreads();
    if (t == 0) {
      unsigned long long b = 0;
      for (int i = 0; i < 16; ++i) b = red[i] > b ? red[i] : b;
      pick = b;
      const int c = (int)(b >> 32);
      if (c >= min_entries && c > 0) {
        const int bin = (int)~(unsigned)(b & 0xFFFFFFFFull);
        sb[k] = bin;
        sc[k] = c;
        h[bin] = 0;
      }
    }
    __syncthreads();
    const int c = (int)(pick >> 32);
    if (c < min_entries || c == 0) break;
  }
  if (t == 0) {
    // ascending block order (insertion sort of at most STRIPE_NBMAX)
    for (int i = 1; i < k; ++i) {
      const int b = sb[i], c = sc[i];
      int j = i - 1;
      while (j >= 0 && sb[j] > b) {
        sb[j + 1] = sb[j];
        sc[j + 1] = sc[j];
        --j;
      }
      sb[j + 1] = b;
      sc[j + 1] = c;
    }
    int hot = 0;
    for (int i = 0; i < k; ++i) {
      blk[s * STRIPE_NBMAX + i] = sb[i];
      hcnt[s * STRIPE_NBMAX + i] = sc[i];
      hot += sc[i];
    }
    nbs[s] = k;
    cold[s] = (e1 - e0) - hot;
  }
}

// Stable partition of each stripe's entries (in CSR order, so by row) into
// its segments, one workgroup of 256 per stripe.  The class of an entry is
// the position of its column block in the stripe's block list (binary
// search), or nb for the rest.  The entries go in chunks of 256; each
// wavefront ranks its lanes among the lanes of the same class with
// ballots, the four wavefronts' counts are combined in LDS, and the running
// count of each class places the entry in its segment.  Row of an entry:
// binary search over the stripe's row pointers.
__global__ __launch_bounds__(256) void st_partition_kernel(const int* rowptr, const int* col, const int* sr0,
                                                          const int* nbs, const int* blk, const int64_t* obase,
                                                          unsigned* hot, unsigned* ccol, unsigned short* crow) {
  __shared__ int run[NCLS];       // entries of each class placed so far
  __shared__ int wcnt[4][NCLS];   // entries of each class per wavefront in this chunk
  __shared__ int sblk[STRIPE_NBMAX];
  const int s = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int r0 = sr0[s], r1 = sr0[s + 1];
  const int e0 = rowptr[r0], e1 = rowptr[r1];
  const int nb = nbs[s];
  if (t < NCLS) run[t] = 0;
  if (t < nb) sblk[t] = blk[s * STRIPE_NBMAX + t];
  for (int c0 = e0; c0 < e1; c0 += 256) {
    for (int i = t; i < 4 * NCLS; i += 256) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    const int e = c0 + t;
    const bool ok = e < e1;
    int cls = 0, cc = 0, cb = 0;
    if (ok) {
      cc = col[e];
      cb = cc / STRIPE_HB;
      int lo = 0, hi = nb;  // first listed block >= cb
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sblk[mid] < cb) lo = mid + 1; else hi = mid;
      }
      cls = (lo < nb && sblk[lo] == cb) ? lo : nb;
    }
    int rank = 0;
    unsigned long long todo = __ballot(ok);
    while (todo) {
      const int lead = __ffsll((long long)todo) - 1;
      const int k = __shfl(cls, lead, 64);
      const unsigned long long m = __ballot(ok && cls == k);
      if (ok && cls == k) rank = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) wcnt[w][k] = __popcll(m);
      todo &= ~m;
    }
    __syncthreads();
    if (ok) {
      int before = run[cls] + rank;
      for (int v = 0; v < w; ++v) before += wcnt[v][cls];
      int lo = r0, hi = r1;  // row r with rowptr[r] <= e < rowptr[r+1]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rowptr[mid] <= e) lo = mid; else hi = mid;
      }
      const unsigned rl = (unsigned)(lo - r0 + 1);
      const int64_t dst = obase[(int64_t)s * NCLS + cls] + before;
      if (cls < nb) {
        hot[dst] = (rl << 16) | (unsigned)(cc - cb * STRIPE_HB);
      } else {
        ccol[dst] = (unsigned)cc;
        crow[dst] = (unsigned short)rl;
      }
    }
    __syncthreads();
    if (t < NCLS) run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    __syncthreads();  // the counts are read before the next chunk clears them
  }
}

// Exclusive prefix of v over the 1024 threads of the workgroup (ws: 16
// ints of LDS).
__device__ int block_excl_scan_1024(int v, int* ws) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) ws[w] = incl;
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int i = 0; i < 16; ++i) {
      const int x = ws[i];
      ws[i] = run;
      run += x;
    }
  }
  __syncthreads();
  const int r = ws[w] + incl - v;
  __syncthreads();
  return r;
}

// Two-phase plans: each stripe's gathered entries (real ones, not the
// padding) regrouped by column block, into tcol / trow at the same slots;
// the order inside a group is arbitrary (the fixed-point sums do not depend
// on it).  One workgroup of 1024 per stripe; nbins <= STRIPE_MAXBLK.
__global__ __launch_bounds__(1024) void st_group_kernel(const unsigned* ccol, const unsigned short* crow,
                                                        const StripeDesc* desc, const int* ncold, int nbins,
                                                        unsigned* tcol, unsigned short* trow) {
  __shared__ int cnt[STRIPE_MAXBLK];
  __shared__ int ws[16];
  const int s = blockIdx.x, t = threadIdx.x;
  const int64_t base = desc[s].cold_base;
  const int nc = ncold[s];
  for (int i = t; i < nbins; i += 1024) cnt[i] = 0;
  __syncthreads();
  for (int e = t; e < nc; e += 1024) atomicAdd(&cnt[min((int)(ccol[base + e] / STRIPE_HB), nbins - 1)], 1);
  __syncthreads();
  // thread t owns bins [16 t, 16 t + 16)
  int own = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int i = t * 16 + k;
    own += i < nbins ? cnt[i] : 0;
  }
  int run = block_excl_scan_1024(own, ws);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int i = t * 16 + k;
    if (i < nbins) {
      const int c = cnt[i];
      cnt[i] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int e = t; e < nc; e += 1024) {
    const unsigned c = ccol[base + e];
    const int at = atomicAdd(&cnt[min((int)(c / STRIPE_HB), nbins - 1)], 1);
    tcol[base + at] = c;
    trow[base + at] = crow[base + e];
  }
}

// Fill-list keys of the stripes' real gathered entries: (column block << 32
// | slot), the column inside its block as the value; entry e of stripe s
// goes to list position off[s] + e.
__global__ __launch_bounds__(256) void st_fill_keys_kernel(const unsigned* ccol, const StripeDesc* desc,
                                                           const int* ncold, const int64_t* off, uint64_t* keys,
                                                           uint16_t* vals) {
  const int s = blockIdx.x;
  const int64_t base = desc[s].cold_base, o = off[s];
  const int nc = ncold[s];
  for (int e = threadIdx.x; e < nc; e += 256) {
    const unsigned c = ccol[base + e];
    const unsigned b = c / STRIPE_HB;
    keys[o + e] = ((uint64_t)b << 32) | (uint64_t)(base + e);
    vals[o + e] = (uint16_t)(c - b * STRIPE_HB);
  }
}

// Slots from the sorted keys, and the first list position of each column
// block (first[b] stays 0xFFFFFFFF for a block without entries).
// Run starts of the sorted fill list: an entry whose slot does not follow
// its predecessor's (or whose block differs) starts a run.
__global__ void st_run_flags_kernel(const uint64_t* keys, int64_t n, unsigned* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || keys[i] != keys[i - 1] + 1ull) ? 1u : 0u;
}

// Every sub-chunk starts a run.
__global__ void st_sub_flags_kernel(const unsigned* sub_start, int nsub, unsigned* flag) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nsub) flag[sub_start[k]] = 1u;
}

// Run r = rank[i] - 1 of run-start entry i begins at slot pos[i]; the entry
// carries the run-start mark.
__global__ void st_runs_kernel(const unsigned* flag, const unsigned* rank, const uint64_t* keys, int64_t n,
                               unsigned* run_pos, unsigned short* src) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  run_pos[rank[i] - 1u] = (unsigned)(keys[i] & 0xFFFFFFFFull);
  src[i] = (unsigned short)(src[i] | 0x8000u);
}

// Run index at each sub-chunk's first entry.
__global__ void st_sub_runs_kernel(const unsigned* sub_start, int nsub, const unsigned* rank, unsigned* sub_run) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nsub) sub_run[k] = rank[sub_start[k]] - 1u;
}

__global__ void st_fill_finish_kernel(const uint64_t* keys, int64_t n, unsigned* first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = keys[i];
  const unsigned b = (unsigned)(k >> 32);
  if (i == 0 || (unsigned)(keys[i - 1] >> 32) != b) first[b] = (unsigned)i;
}

int64_t pad8(int64_t x) { return (x + 7) & ~(int64_t)7; }

}  // namespace

namespace {

constexpr unsigned FILL_CHUNK = 16384;  // fill-list entries per chunk at most

// The two-phase part of a stripe plan: each stripe's gathered entries
// regrouped by column block, the fill list (entries by column block, then
// by slot) cut into chunks, and the zeroed value array.  The columns are
// not kept: the pass reads values instead.
void build_fill(const MatP& A, Plan& plan, const std::vector<int>& ncold) {
  Ctx& c = ctx();
  const int S = plan.st_nstripes;
  const int64_t ncolblk = (A->ncols + STRIPE_HB - 1) / STRIPE_HB;
  const int nbins = (int)std::max<int64_t>(1, std::min<int64_t>(ncolblk, STRIPE_MAXBLK));
  std::vector<int64_t> off((size_t)S + 1, 0);
  for (int s = 0; s < S; ++s) off[(size_t)s + 1] = off[(size_t)s] + ncold[(size_t)s];
  const int64_t N = off[(size_t)S];
  const size_t slots = (size_t)std::max<int64_t>(plan.st_cold_entries, 8);
  plan.st_cval = dev_alloc(sizeof(float) * slots);
  hip_check(launch_zero(plan.st_cval->p, plan.st_cval->bytes, c.stream), "zero");
  std::vector<ColdChunk> chunks;
  if (N > 0) {
    BufP d_nc = dev_alloc(sizeof(int) * (size_t)S), d_off = dev_alloc(sizeof(int64_t) * (size_t)S);
    hip_check(hipMemcpyAsync(d_nc->p, ncold.data(), sizeof(int) * (size_t)S, hipMemcpyHostToDevice, c.stream),
              "upload");
    hip_check(hipMemcpyAsync(d_off->p, off.data(), sizeof(int64_t) * (size_t)S, hipMemcpyHostToDevice, c.stream),
              "upload");
    // regroup each stripe's entries by column block
    BufP tcol = dev_alloc(plan.st_ccol->bytes), trow = dev_alloc(plan.st_crow->bytes);
    hip_check(launch_zero(tcol->p, tcol->bytes, c.stream), "zero");
    hip_check(launch_zero(trow->p, trow->bytes, c.stream), "zero");
    hipLaunchKernelGGL(st_group_kernel, dim3(S), dim3(1024), 0, c.stream, (const unsigned*)plan.st_ccol->p,
                       (const unsigned short*)plan.st_crow->p, (const StripeDesc*)plan.st_desc->p,
                       (const int*)d_nc->p, nbins, (unsigned*)tcol->p, (unsigned short*)trow->p);
    hip_check(hipGetLastError(), "group gathered entries");
    plan.st_ccol = tcol;
    plan.st_crow = trow;
    // the fill list: (block, slot) keys sorted
    BufP kin = dev_alloc(sizeof(uint64_t) * (size_t)N), kout = dev_alloc(sizeof(uint64_t) * (size_t)N);
    BufP vin = dev_alloc(sizeof(uint16_t) * (size_t)N);
    plan.st_pasrc = dev_alloc(sizeof(uint16_t) * (size_t)N);
    hipLaunchKernelGGL(st_fill_keys_kernel, dim3(S), dim3(256), 0, c.stream, (const unsigned*)plan.st_ccol->p,
                       (const StripeDesc*)plan.st_desc->p, (const int*)d_nc->p, (const int64_t*)d_off->p,
                       (uint64_t*)kin->p, (uint16_t*)vin->p);
    hip_check(hipGetLastError(), "fill keys");
    unsigned end_bit = 32;
    while (end_bit < 64 && ((uint64_t)1 << (end_bit - 32)) < (uint64_t)ncolblk) ++end_bit;
    hip_check(sort_pairs_u64_u16((const uint64_t*)kin->p, (uint64_t*)kout->p, (const uint16_t*)vin->p,
                                 (uint16_t*)plan.st_pasrc->p, N, end_bit, cache_alloc, cache_release, nullptr,
                                 c.stream),
              "sort fill list");
    kin.reset();
    vin.reset();
    BufP first = dev_alloc(sizeof(unsigned) * (size_t)ncolblk);
    hip_check(launch_fill(first->p, T_INT32, ncolblk, -1.0, c.stream), "fill");
    const int64_t g = (N + 255) / 256;
    hipLaunchKernelGGL(st_fill_finish_kernel, dim3((unsigned)g), dim3(256), 0, c.stream, (const uint64_t*)kout->p,
                       N, (unsigned*)first->p);
    hip_check(hipGetLastError(), "fill list");
    std::vector<unsigned> hfirst((size_t)ncolblk);
    hip_check(hipMemcpyAsync(hfirst.data(), first->p, sizeof(unsigned) * (size_t)ncolblk, hipMemcpyDeviceToHost,
                             c.stream),
              "download");
    hip_check(hipStreamSynchronize(c.stream), "sync");
    // chunks of at most FILL_CHUNK entries of one block, cut into
    // sub-chunks of FILL_SUB
    std::vector<unsigned> sub_start;
    int64_t prev_b = -1;
    for (int64_t b = 0; b <= ncolblk; ++b) {
      if (b < ncolblk && hfirst[(size_t)b] == 0xFFFFFFFFu) continue;
      if (prev_b >= 0) {
        const unsigned st = hfirst[(size_t)prev_b];
        const unsigned en = b < ncolblk ? hfirst[(size_t)b] : (unsigned)N;
        if (en < st) fail(GrB_PANIC, "stripe plan: fill list out of order");
        for (unsigned x = st; x < en; x += FILL_CHUNK) {
          const unsigned xe = std::min(en, x + FILL_CHUNK);
          chunks.push_back(ColdChunk{(int)prev_b, x, xe, (unsigned)sub_start.size()});
          for (unsigned y = x; y < xe; y += FILL_SUB) sub_start.push_back(y);
        }
      }
      prev_b = b;
    }
    // runs of consecutive slots: each starts at an entry whose slot does
    // not follow its predecessor's, or at a sub-chunk
    const int nsub = (int)sub_start.size();
    BufP flag = dev_alloc(sizeof(unsigned) * (size_t)N), rank = dev_alloc(sizeof(unsigned) * (size_t)N);
    BufP d_sub = dev_alloc(sizeof(unsigned) * (size_t)std::max(nsub, 1));
    if (nsub > 0)
      hip_check(hipMemcpyAsync(d_sub->p, sub_start.data(), sizeof(unsigned) * (size_t)nsub, hipMemcpyHostToDevice,
                               c.stream),
                "upload");
    hipLaunchKernelGGL(st_run_flags_kernel, dim3((unsigned)g), dim3(256), 0, c.stream, (const uint64_t*)kout->p, N,
                       (unsigned*)flag->p);
    hip_check(hipGetLastError(), "run starts");
    if (nsub > 0) {
      hipLaunchKernelGGL(st_sub_flags_kernel, dim3((nsub + 255) / 256), dim3(256), 0, c.stream,
                         (const unsigned*)d_sub->p, nsub, (unsigned*)flag->p);
      hip_check(hipGetLastError(), "sub-chunk starts");
    }
    hip_check(scan_u32_inclusive((const unsigned*)flag->p, (unsigned*)rank->p, N, cache_alloc, cache_release,
                                 nullptr, c.stream),
              "run ranks");
    unsigned nruns = 0;
    hip_check(hipMemcpyAsync(&nruns, (const unsigned*)rank->p + (N - 1), sizeof(unsigned), hipMemcpyDeviceToHost,
                             c.stream),
              "download");
    hip_check(hipStreamSynchronize(c.stream), "sync");
    plan.st_prun = dev_alloc(sizeof(unsigned) * (size_t)std::max(nruns, 1u));
    plan.st_psub = dev_alloc(sizeof(unsigned) * (size_t)std::max(nsub, 1));
    hipLaunchKernelGGL(st_runs_kernel, dim3((unsigned)g), dim3(256), 0, c.stream, (const unsigned*)flag->p,
                       (const unsigned*)rank->p, (const uint64_t*)kout->p, N, (unsigned*)plan.st_prun->p,
                       (unsigned short*)plan.st_pasrc->p);
    hip_check(hipGetLastError(), "runs");
    if (nsub > 0) {
      hipLaunchKernelGGL(st_sub_runs_kernel, dim3((nsub + 255) / 256), dim3(256), 0, c.stream,
                         (const unsigned*)d_sub->p, nsub, (const unsigned*)rank->p, (unsigned*)plan.st_psub->p);
      hip_check(hipGetLastError(), "sub-chunk runs");
    }
    hip_check(hipStreamSynchronize(c.stream), "sync");
  }
  plan.st_pachunk = dev_alloc(sizeof(ColdChunk) * std::max<size_t>(chunks.size(), 1));
  if (!chunks.empty())
    hip_check(hipMemcpyAsync(plan.st_pachunk->p, chunks.data(), sizeof(ColdChunk) * chunks.size(),
                             hipMemcpyHostToDevice, c.stream),
              "upload");
  hip_check(hipStreamSynchronize(c.stream), "sync");
  plan.st_ccol.reset();  // the pass reads values, not columns
  plan.st_dev.cold_col = nullptr;
  plan.st_dev.cold_row = (const unsigned short*)plan.st_crow->p;
  plan.st_dev.cold_val = (const float*)plan.st_cval->p;
  ColdFillDev& f = plan.st_fill;
  f.src = plan.st_pasrc ? (const unsigned short*)plan.st_pasrc->p : nullptr;
  f.run_pos = plan.st_prun ? (const unsigned*)plan.st_prun->p : nullptr;
  f.sub_run = plan.st_psub ? (const unsigned*)plan.st_psub->p : nullptr;
  f.chunk = (const ColdChunk*)plan.st_pachunk->p;
  f.val = (float*)plan.st_cval->p;
  f.nchunks = (int)chunks.size();
}

}  // namespace

void build_stripe_plan(const MatP& A, Plan& plan, const std::vector<int>& rp) {
  Ctx& c = ctx();
  const PlanConfig& cfg = plan.cfg;
  const int64_t n = A->nrows, m = A->nnz;
  if (A->ncols >= (int64_t)1 << 30) fail(GrB_INVALID_VALUE, "the stripe plan addresses at most 2^30 columns");
  if (m >= (int64_t)1 << 31) fail(GrB_INVALID_VALUE, "the stripe plan holds fewer than 2^31 entries");
  const int G = cfg.grid;
  int maxlen = 0;
  for (int64_t i = 0; i < n; ++i) maxlen = std::max(maxlen, rp[i + 1] - rp[i]);

  // stripes: at most STRIPE_RMAX rows, about m / (2G) entries
  const int64_t emax = std::max<int64_t>(4096, (m + 2 * (int64_t)G - 1) / (2 * (int64_t)G));
  std::vector<int> sr0{0};
  {
    int64_t r0 = 0;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t ecur = rp[i] - rp[r0];
      if (i - r0 >= STRIPE_RMAX || (ecur > 0 && ecur + (rp[i + 1] - rp[i]) > emax)) {
        sr0.push_back((int)i);
        r0 = i;
      }
    }
    if (sr0.back() != (int)n || n == 0) sr0.push_back((int)n);
  }
  const int S = (int)sr0.size() - 1;

  BufP d_sr0 = dev_alloc(sizeof(int) * (size_t)(S + 1));
  hip_check(hipMemcpyAsync(d_sr0->p, sr0.data(), sizeof(int) * (S + 1), hipMemcpyHostToDevice, c.stream), "upload");
  // LDS blocks of each stripe: the blocks with the most entries, each with
  // at least min_entries of them
  const int nb_cap = std::min<int64_t>(STRIPE_NBMAX, cfg.hot > 0 ? std::max(1, cfg.hot / STRIPE_HB) : STRIPE_NBMAX);
  const int64_t ncolblk = (A->ncols + STRIPE_HB - 1) / STRIPE_HB;
  const int nbins = (int)std::max<int64_t>(1, std::min<int64_t>(ncolblk, STRIPE_MAXBLK));
  const int merged = ncolblk > STRIPE_MAXBLK ? 1 : 0;
  const int min_entries = cfg.long_row > 0 ? cfg.long_row : 1024;
  const size_t S1 = (size_t)std::max(S, 1);
  BufP d_nb = dev_alloc(sizeof(int) * S1), d_cold = dev_alloc(sizeof(int) * S1);
  BufP d_blk = dev_alloc(sizeof(int) * S1 * STRIPE_NBMAX), d_hc = dev_alloc(sizeof(int) * S1 * STRIPE_NBMAX);
  const int* rowptr = (const int*)A->rowptr->p;
  const int* col = A->col ? (const int*)A->col->p : nullptr;
  std::vector<int> nbs(S), cold_cnt(S), blk((size_t)S * STRIPE_NBMAX), hcnt((size_t)S * STRIPE_NBMAX);
  if (S > 0 && m > 0) {
    hipLaunchKernelGGL(st_select_kernel, dim3(S), dim3(1024), 0, c.stream, rowptr, col, (const int*)d_sr0->p, nbins,
                       merged, nb_cap, min_entries, (int*)d_nb->p, (int*)d_blk->p, (int*)d_hc->p, (int*)d_cold->p);
    hip_check(hipGetLastError(), "stripe block choice");
    hip_check(hipMemcpyAsync(nbs.data(), d_nb->p, sizeof(int) * S, hipMemcpyDeviceToHost, c.stream), "download");
    hip_check(hipMemcpyAsync(cold_cnt.data(), d_cold->p, sizeof(int) * S, hipMemcpyDeviceToHost, c.stream),
              "download");
    hip_check(hipMemcpyAsync(blk.data(), d_blk->p, sizeof(int) * blk.size(), hipMemcpyDeviceToHost, c.stream),
              "download");
    hip_check(hipMemcpyAsync(hcnt.data(), d_hc->p, sizeof(int) * hcnt.size(), hipMemcpyDeviceToHost, c.stream),
              "download");
  }
  hip_check(hipStreamSynchronize(c.stream), "sync");

  std::vector<StripeDesc> desc(S);
  std::vector<int64_t> obase((size_t)S * NCLS, 0);
  std::vector<double> cost(S);
  int64_t hot_total = 0, cold_total = 0, counted = 0;
  for (int s = 0; s < S; ++s) {
    const int nb = nbs[(size_t)s];
    if (nb < 0 || nb > nb_cap) fail(GrB_PANIC, "stripe plan: bad block count");
    const int* bs = &blk[(size_t)s * STRIPE_NBMAX];
    const int* cs = &hcnt[(size_t)s * STRIPE_NBMAX];
    StripeDesc& d = desc[s];
    std::memset(&d, 0, sizeof(d));
    d.r0 = sr0[s];
    d.nrows = sr0[s + 1] - sr0[s];
    d.nb = nb;
    d.hot_base = hot_total;
    int64_t off = 0, hot_e = 0;
    for (int b = 0; b < nb; ++b) {
      if (bs[b] < 0 || bs[b] >= ncolblk || (b > 0 && bs[b] <= bs[b - 1]))
        fail(GrB_PANIC, "stripe plan: bad block list");
      d.blk[b] = bs[b];
      d.seg[b] = (int)off;
      obase[(size_t)s * NCLS + b] = hot_total + off;
      counted += cs[b];
      off += pad8(cs[b]);
      hot_e += cs[b];
    }
    d.seg[nb] = (int)off;
    hot_total += off;
    const int64_t cold = cold_cnt[(size_t)s];
    obase[(size_t)s * NCLS + nb] = cold_total;
    counted += cold;
    d.cold_base = cold_total;
    d.cold_n = (int)pad8(cold);
    cold_total += pad8(cold);
    // estimated time on one compute unit.  Gathered plan (cycles): entries
    // added from LDS (about 2 per cycle, plus a block load and barrier per
    // LDS block), entries gathered from memory (about 0.3 per cycle), rows
    // of the epilogue.  Two-phase plan (ns, a least-squares fit of measured
    // per-stripe times at R-MAT scale 22, R^2 0.996): 0.16 per LDS-block
    // entry, 0.45 per filled entry, 820 per LDS block, 0.8 per row and
    // 3,300 per stripe.
    if (cfg.kernel == K_STRIPE2)
      cost[s] = 0.163 * (double)hot_e + 0.446 * (double)cold + 823.0 * nb + 0.793 * d.nrows + 3260.0;
    else
      cost[s] = (double)hot_e / 2.0 + nb * 700.0 + (double)cold / 0.3 + d.nrows / 4.0 + 2000.0;
  }
  if (counted != m) fail(GrB_PANIC, "stripe plan: entry counts do not add up");
  if (hot_total >= ((int64_t)1 << 32) || cold_total >= ((int64_t)1 << 32))
    fail(GrB_INVALID_VALUE, "stripe plan too large");

  // packed arrays (padding entries are zero: they add w[0] to the dump slot)
  plan.st_hot = dev_alloc(sizeof(unsigned) * (size_t)std::max<int64_t>(hot_total, 8));
  plan.st_ccol = dev_alloc(sizeof(unsigned) * (size_t)std::max<int64_t>(cold_total, 8));
  plan.st_crow = dev_alloc(sizeof(unsigned short) * (size_t)std::max<int64_t>(cold_total, 8));
  hip_check(launch_zero(plan.st_hot->p, plan.st_hot->bytes, c.stream), "zero");
  hip_check(launch_zero(plan.st_ccol->p, plan.st_ccol->bytes, c.stream), "zero");
  hip_check(launch_zero(plan.st_crow->p, plan.st_crow->bytes, c.stream), "zero");
  if (m > 0 && S > 0) {
    BufP d_ob = dev_alloc(sizeof(int64_t) * obase.size());
    hip_check(hipMemcpyAsync(d_ob->p, obase.data(), sizeof(int64_t) * obase.size(), hipMemcpyHostToDevice,
                             c.stream),
              "upload");
    hipLaunchKernelGGL(st_partition_kernel, dim3(S), dim3(256), 0, c.stream, rowptr, col, (const int*)d_sr0->p,
                       (const int*)d_nb->p, (const int*)d_blk->p, (const int64_t*)d_ob->p,
                       (unsigned*)plan.st_hot->p, (unsigned*)plan.st_ccol->p, (unsigned short*)plan.st_crow->p);
    hip_check(hipGetLastError(), "stripe partition");
    hip_check(hipStreamSynchronize(c.stream), "sync");
  }

  // stripes to workgroups: longest estimated cost first onto the least loaded
  std::vector<int> ord(S);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<std::vector<int>> per(G);
  using Slot = std::pair<double, int>;
  std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> q;
  for (int k = 0; k < G; ++k) q.push({0.0, k});
  for (int s : ord) {
    Slot t = q.top();
    q.pop();
    per[t.second].push_back(s);
    q.push({t.first + cost[s], t.second});
  }
  std::vector<int> wg_off(G + 1, 0), wg_list;
  wg_list.reserve(S);
  for (int k = 0; k < G; ++k) {
    std::sort(per[k].begin(), per[k].end());
    wg_off[k] = (int)wg_list.size();
    wg_list.insert(wg_list.end(), per[k].begin(), per[k].end());
  }
  wg_off[G] = (int)wg_list.size();

  plan.st_desc = dev_alloc(sizeof(StripeDesc) * (size_t)std::max(S, 1));
  plan.st_wgoff = dev_alloc(sizeof(int) * (size_t)(G + 1));
  plan.st_wglist = dev_alloc(sizeof(int) * (size_t)std::max(S, 1));
  plan.st_wgsum = dev_alloc(sizeof(double) * (size_t)G);
  plan.st_mass = dev_alloc(sizeof(double));
  if (S > 0) {
    hip_check(hipMemcpyAsync(plan.st_desc->p, desc.data(), sizeof(StripeDesc) * S, hipMemcpyHostToDevice, c.stream),
              "upload");
    hip_check(hipMemcpyAsync(plan.st_wglist->p, wg_list.data(), sizeof(int) * S, hipMemcpyHostToDevice, c.stream),
              "upload");
  }
  hip_check(hipMemcpyAsync(plan.st_wgoff->p, wg_off.data(), sizeof(int) * (G + 1), hipMemcpyHostToDevice, c.stream),
            "upload");
  hip_check(hipStreamSynchronize(c.stream), "sync");

  plan.st_nstripes = S;
  plan.st_hot_entries = hot_total;
  plan.st_cold_entries = cold_total;
  StripePlanDev& d = plan.st_dev;
  d.desc = (const StripeDesc*)plan.st_desc->p;
  d.hot = (const unsigned*)plan.st_hot->p;
  d.cold_col = (const unsigned*)plan.st_ccol->p;
  d.cold_row = (const unsigned short*)plan.st_crow->p;
  d.wg_off = (const int*)plan.st_wgoff->p;
  d.wg_list = (const int*)plan.st_wglist->p;
  d.wg_sum = (double*)plan.st_wgsum->p;
  d.cold_val = nullptr;
  d.nstripes = S;
  d.maxlen = maxlen;
  if (cfg.kernel == K_STRIPE2) build_fill(A, plan, cold_cnt);
}

}  // namespace nbgrb
