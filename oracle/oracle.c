/*
 * oracle.c -- plain CPU oracle for the PageRank path of "Julia GraphBLAS with
 * Nonblocking Execution" (Costanza, Mattson, Kimmerer, Brock).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  It is used by the test suite, by the smoke check and by
 * the benchmark's CPU-baseline leg, and nowhere else.  It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * Everything is computed the slow, obvious way:
 *   - the graph is built with a plain LSD radix sort of 64-bit (src,dst) keys
 *     followed by a unique pass; the transpose is a stable counting sort;
 *   - PageRank runs in blocking mode (Section II of the paper): every
 *     GraphBLAS operation of the Fig. 6 loop is a separate pass that
 *     materialises its whole output vector, in FP64;
 *   - every floating-point reduction is summed in index order inside fixed
 *     65536-element chunks, and the chunk partials in chunk order, so the
 *     result does not depend on the OpenMP thread count.
 *
 * The only parallelism is an OpenMP "parallel for" over independent rows or
 * chunks; each row sum and each chunk sum is sequential.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_CHUNK 65536

/* ------------------------------------------------------------------------ */
/* Threads                                                                   */
/* ------------------------------------------------------------------------ */

void oracle_set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int oracle_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number      */
/* generators", OOPSLA 2014), used as a counter-based generator: draw k of   */
/* the stream seeded with `seed` is the (k+1)-th output of the generator,    */
/* i.e. the mixing function applied to seed + (k+1)*gamma.                   */
/* ------------------------------------------------------------------------ */

uint64_t oracle_splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* R-MAT edge generator (Chakrabarti, Zhan, Faloutsos, SDM 2004).            */
/*                                                                           */
/* Edge e picks one quadrant per level, most significant bit first.  Level   */
/* l of edge e uses draw k = e*scale + l, turned into u in [0,1) from its    */
/* top 53 bits.  Quadrant a (top-left) sets no bit, b (top-right) sets the   */
/* destination bit, c (bottom-left) the source bit, d both.  The cumulative */
/* thresholds are passed in as given (0.57, 0.76, 0.95 for a=0.57, b=0.19,   */
/* c=0.19, d=0.05).  No noise and no vertex permutation.                     */
/* ------------------------------------------------------------------------ */

void oracle_rmat_edges(int scale, int64_t nedges, uint64_t seed, double t_a,
                       double t_ab, double t_abc, uint32_t *src, uint32_t *dst) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < nedges; ++e) {
    uint32_t s = 0, t = 0;
    for (int l = 0; l < scale; ++l) {
      uint64_t k = (uint64_t)e * (uint64_t)scale + (uint64_t)l;
      double u = (double)(oracle_splitmix64(seed, k) >> 11) * 0x1.0p-53;
      s <<= 1;
      t <<= 1;
      if (u < t_a) {
        /* quadrant a */
      } else if (u < t_ab) {
        t |= 1u; /* quadrant b */
      } else if (u < t_abc) {
        s |= 1u; /* quadrant c */
      } else {
        s |= 1u; /* quadrant d */
        t |= 1u;
      }
    }
    src[e] = s;
    dst[e] = t;
  }
}

/* ------------------------------------------------------------------------ */
/* Web-shaped generator: a synthetic stand-in for the web crawl of the       */
/* paper's evaluation (Section IV: many pages, a high mean degree, strong    */
/* locality).  Every quantity is an unsigned 64-bit integer.                 */
/*                                                                           */
/* model[] = {kmin, kmax, p_zero, p_home, p_local, local_min, hub, perm_a,   */
/* perm_b}; probabilities in units of 2^-16.  The draw with key k is draw k  */
/* of the SplitMix64 stream above.                                           */
/*                                                                           */
/* Heavy-tailed helper: D(c, r) = floor(c * 2^52 / X) with X = (r >> 12)+1  */
/* uniform on 1..2^52, so D >= c and P(D >= x) is about c/x.                 */
/*                                                                           */
/* Vertex u: a page without out-links when the top 16 bits of draw           */
/* (u<<18 | 0x3FFFC) fall below p_zero; otherwise its number of links is    */
/* k_u = min(kmax, D(kmin, draw(u<<18 | 0x3FFFD))).                          */
/*                                                                           */
/* Link j of u, with r = draw(u<<18 | j<<2), q = draw(u<<18 | j<<2 | 1) and  */
/* t = the top 16 bits of r:                                                 */
/*   t < p_home           -> home link: clear the low h = 6 + (r mod 16)     */
/*                           bits of u;                                      */
/*   t < p_home + p_local -> local link at distance                          */
/*                           d = min(n-1, D(max(local_min, k_u), q)),        */
/*                           backwards when bit 4 of r is set, modulo n;     */
/*   otherwise            -> global link to vertex (perm_a*i + perm_b) mod n */
/*                           with i = (D(hub, q) - hub) mod n.               */
/* ------------------------------------------------------------------------ */

static uint64_t web_heavy(uint64_t c, uint64_t r) {
  uint64_t x = (r >> 12) + 1u;        /* 1 .. 2^52 */
  return (c << 52) / x;
}

static uint64_t web_links_of(uint64_t seed, const int64_t *model, uint64_t u) {
  uint64_t kmin = (uint64_t)model[0], kmax = (uint64_t)model[1], p_zero = (uint64_t)model[2];
  uint64_t a = oracle_splitmix64(seed, (u << 18) | 0x3FFFCu);
  if ((a >> 48) < p_zero) return 0;
  uint64_t k = web_heavy(kmin, oracle_splitmix64(seed, (u << 18) | 0x3FFFDu));
  return k < kmax ? k : kmax;
}

static uint64_t web_link(uint64_t n, uint64_t seed, const int64_t *model, uint64_t u,
                         uint64_t j, uint64_t k_u) {
  uint64_t p_home = (uint64_t)model[3], p_local = (uint64_t)model[4];
  uint64_t local_min = (uint64_t)model[5], hub = (uint64_t)model[6];
  uint64_t perm_a = (uint64_t)model[7], perm_b = (uint64_t)model[8];
  uint64_t r = oracle_splitmix64(seed, (u << 18) | (j << 2));
  uint64_t q = oracle_splitmix64(seed, (u << 18) | (j << 2) | 1u);
  uint64_t t = r >> 48;
  if (t < p_home) {
    uint64_t h = 6 + r % 16;
    return (u >> h) << h;
  }
  if (t < p_home + p_local) {
    uint64_t scale = local_min > k_u ? local_min : k_u;
    uint64_t d = web_heavy(scale, q);
    if (d > n - 1) d = n - 1;
    if ((r >> 4) & 1u) return (u + (n - d)) % n; /* u - d modulo n */
    return (u + d) % n;
  }
  uint64_t i = (web_heavy(hub, q) - hub) % n;
  return (perm_a * i + perm_b) % n;
}

/* Number of links of every vertex. */
void oracle_web_degrees(uint64_t n, uint64_t seed, const int64_t *model, int64_t *deg) {
#pragma omp parallel for schedule(static)
  for (int64_t u = 0; u < (int64_t)n; ++u) deg[u] = (int64_t)web_links_of(seed, model, (uint64_t)u);
}

/* All links in order of u then j; off[u] = first link of u (n+1 entries). */
void oracle_web_edges(uint64_t n, uint64_t seed, const int64_t *model, const int64_t *off,
                      uint32_t *src, uint32_t *dst) {
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t u = 0; u < (int64_t)n; ++u) {
    uint64_t k = (uint64_t)(off[u + 1] - off[u]);
    for (uint64_t j = 0; j < k; ++j) {
      src[off[u] + (int64_t)j] = (uint32_t)u;
      dst[off[u] + (int64_t)j] = (uint32_t)web_link(n, seed, model, (uint64_t)u, j, k);
    }
  }
}

/* The links of one vertex (k_u targets in order of j); returns k_u. */
int64_t oracle_web_row(uint64_t n, uint64_t seed, const int64_t *model, uint64_t u, uint32_t *out) {
  uint64_t k = web_links_of(seed, model, u);
  for (uint64_t j = 0; j < k; ++j) out[j] = (uint32_t)web_link(n, seed, model, u, j, k);
  return (int64_t)k;
}

/* Every link (u, v) whose target v has want[v] != 0, in no particular
 * order; returns their number, or -1 when more than cap were found (the
 * arrays then hold the first cap in no particular order). */
int64_t oracle_web_links_into(uint64_t n, uint64_t seed, const int64_t *model, const uint8_t *want,
                              int64_t cap, uint32_t *src, uint32_t *dst) {
  int64_t found = 0;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t u = 0; u < (int64_t)n; ++u) {
    uint64_t k = web_links_of(seed, model, (uint64_t)u);
    for (uint64_t j = 0; j < k; ++j) {
      uint64_t v = web_link(n, seed, model, (uint64_t)u, j, k);
      if (!want[v]) continue;
      int64_t slot;
#pragma omp atomic capture
      slot = found++;
      if (slot < cap) {
        src[slot] = (uint32_t)u;
        dst[slot] = (uint32_t)v;
      }
    }
  }
  return found > cap ? -1 : found;
}

/* ------------------------------------------------------------------------ */
/* Graph construction                                                        */
/* ------------------------------------------------------------------------ */

/* Plain LSD radix sort of unsigned 64-bit keys, 16-bit digits. */
static void radix_sort_u64(uint64_t *keys, int64_t n) {
  uint64_t *tmp = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
  int64_t *count = (int64_t *)malloc(65536 * sizeof(int64_t));
  uint64_t *from = keys, *to = tmp;
  for (int pass = 0; pass < 4; ++pass) {
    int shift = 16 * pass;
    memset(count, 0, 65536 * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) count[(from[i] >> shift) & 0xFFFF]++;
    int64_t run = 0;
    for (int d = 0; d < 65536; ++d) {
      int64_t c = count[d];
      count[d] = run;
      run += c;
    }
    for (int64_t i = 0; i < n; ++i) to[count[(from[i] >> shift) & 0xFFFF]++] = from[i];
    uint64_t *sw = from;
    from = to;
    to = sw;
  }
  /* four passes: the sorted data is back in `keys` */
  free(tmp);
  free(count);
}

/*
 * CSR of the directed graph with vertex set [0,n): row = source, columns =
 * distinct destinations in ascending order.  Self-loops are dropped when
 * drop_self is set, duplicates are always merged (the matrix is a pattern).
 * col must have room for nedges entries.  Returns nnz, or -1 when an
 * endpoint is out of range.
 */
int64_t oracle_build_csr(int64_t n, int64_t nedges, const uint32_t *src,
                         const uint32_t *dst, int drop_self, int32_t *rowptr,
                         int32_t *col) {
  uint64_t *keys = (uint64_t *)malloc((size_t)(nedges > 0 ? nedges : 1) * sizeof(uint64_t));
  int64_t k = 0;
  for (int64_t e = 0; e < nedges; ++e) {
    if ((int64_t)src[e] >= n || (int64_t)dst[e] >= n) {
      free(keys);
      return -1;
    }
    if (drop_self && src[e] == dst[e]) continue;
    keys[k++] = ((uint64_t)src[e] << 32) | (uint64_t)dst[e];
  }
  radix_sort_u64(keys, k);
  for (int64_t i = 0; i <= n; ++i) rowptr[i] = 0;
  int64_t nnz = 0;
  for (int64_t i = 0; i < k; ++i) {
    if (i > 0 && keys[i] == keys[i - 1]) continue;
    uint32_t s = (uint32_t)(keys[i] >> 32);
    col[nnz++] = (int32_t)(uint32_t)(keys[i] & 0xFFFFFFFFu);
    rowptr[s + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) rowptr[i + 1] += rowptr[i];
  free(keys);
  return nnz;
}

/* outdeg[i] = number of entries in row i. */
void oracle_row_counts(int64_t n, const int32_t *rowptr, int32_t *deg) {
  for (int64_t i = 0; i < n; ++i) deg[i] = rowptr[i + 1] - rowptr[i];
}

/*
 * Transpose of a CSR pattern (nrows x ncols) by a stable counting sort: rows
 * of A are visited in ascending order, so each row of the transpose lists
 * its columns in ascending order.
 */
void oracle_transpose(int64_t nrows, int64_t ncols, const int32_t *rowptr,
                      const int32_t *col, int32_t *rowptrT, int32_t *colT) {
  int64_t nnz = rowptr[nrows];
  int64_t *next = (int64_t *)calloc((size_t)ncols + 1, sizeof(int64_t));
  for (int64_t e = 0; e < nnz; ++e) next[col[e] + 1]++;
  for (int64_t j = 0; j < ncols; ++j) next[j + 1] += next[j];
  for (int64_t j = 0; j <= ncols; ++j) rowptrT[j] = (int32_t)next[j];
  for (int64_t i = 0; i < nrows; ++i)
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) colT[next[col[e]]++] = (int32_t)i;
  free(next);
}

/* ------------------------------------------------------------------------ */
/* Reductions: fixed chunks, index order inside a chunk, chunk order after.  */
/* ------------------------------------------------------------------------ */

static double chunked_sum(const double *x, int64_t n) {
  int64_t nchunk = (n + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
  double *part = (double *)malloc((size_t)(nchunk > 0 ? nchunk : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nchunk; ++c) {
    int64_t lo = c * ORACLE_CHUNK, hi = lo + ORACLE_CHUNK < n ? lo + ORACLE_CHUNK : n;
    double s = 0.0;
    for (int64_t i = lo; i < hi; ++i) s += x[i];
    part[c] = s;
  }
  double total = 0.0;
  for (int64_t c = 0; c < nchunk; ++c) total += part[c];
  free(part);
  return total;
}

double oracle_sum(const double *x, int64_t n) { return chunked_sum(x, n); }

/* ------------------------------------------------------------------------ */
/* PageRank, blocking mode, FP64 (Fig. 6 of the paper, one op per pass).     */
/*                                                                           */
/*   w   = ewise_mult:  w_j = damping * x_j / outdeg_j  (0 when outdeg_j=0)  */
/*   s   = mxv(plus, second, AT, w): s_i = sum of w_j over row i of A^T      */
/*   r   = ewise_add(+, teleport, s): r_i = (1-d) v_i [+ d D v_i] + s_i      */
/*   t   = ewise_add(|x-y|, x, r)                                            */
/*   rho = reduce(+, t)                                                      */
/*   D   = sum of r_j over dangling j (outdeg_j = 0), used by the next pass  */
/*                                                                           */
/* mode 0 (DROP) is the paper's variant: the rank held by dangling vertices */
/* is not redistributed.  mode 1 (UNIFORM) hands the dangling mass D back    */
/* through the teleport distribution v, which keeps sum(x) = 1.              */
/* v == NULL means v_i = 1/n (global PageRank); x0 == NULL means x0 = v.     */
/* The loop runs while iters < itermax and rho > tol, with rho = 1 before    */
/* the first pass as in Fig. 6; fixed_iters > 0 runs exactly that many      */
/* passes instead.  Returns the number of passes performed.                  */
/* rho_hist (length >= passes, may be NULL) gets rho_1..rho_k in slots 0..  */
/* k-1; D_hist (length >= passes+1, may be NULL) gets D_0..D_k, the dangling */
/* mass of each iterate, D_0 from x0.                                        */
/* ------------------------------------------------------------------------ */

int oracle_pagerank(int64_t n, const int32_t *rowptrT, const int32_t *colT,
                    const int32_t *outdeg, double damping, double tol,
                    int itermax, int fixed_iters, int mode, const double *v,
                    const double *x0, double *x_out, double *rho_hist,
                    double *D_hist, double *resid_out) {
  double *x = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *w = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *s = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *r = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *t = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *vv = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));

  for (int64_t i = 0; i < n; ++i) vv[i] = v ? v[i] : 1.0 / (double)n;
  for (int64_t i = 0; i < n; ++i) x[i] = x0 ? x0[i] : vv[i];

  /* dangling mass of the start vector */
  for (int64_t i = 0; i < n; ++i) t[i] = outdeg[i] == 0 ? x[i] : 0.0;
  double D = chunked_sum(t, n);
  if (D_hist) D_hist[0] = D;

  double rho = 1.0;
  int iters = 0;
  for (;;) {
    if (fixed_iters > 0) {
      if (iters >= fixed_iters) break;
    } else if (!(iters < itermax && rho > tol)) {
      break;
    }
    /* w = ewise_mult(x, damping / outdeg) */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) w[j] = outdeg[j] > 0 ? damping * x[j] / (double)outdeg[j] : 0.0;
    /* s = A^T (plus, second) w */
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int64_t e = rowptrT[i]; e < rowptrT[i + 1]; ++e) acc += w[colT[e]];
      s[i] = acc;
    }
    /* r = teleport + s */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double tele = (1.0 - damping) * vv[i];
      if (mode == 1) tele += damping * D * vv[i];
      r[i] = tele + s[i];
    }
    /* t = |x - r| ; rho = sum(t) */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) t[i] = fabs(x[i] - r[i]);
    rho = chunked_sum(t, n);
    /* D = sum of r over dangling vertices */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) t[i] = outdeg[i] == 0 ? r[i] : 0.0;
    D = chunked_sum(t, n);
    /* x = r */
    memcpy(x, r, (size_t)n * sizeof(double));
    if (rho_hist) rho_hist[iters] = rho;
    ++iters;
    if (D_hist) D_hist[iters] = D;
  }
  memcpy(x_out, x, (size_t)n * sizeof(double));
  if (resid_out) *resid_out = rho;
  free(x);
  free(w);
  free(s);
  free(r);
  free(t);
  free(vv);
  return iters;
}
