/*
 * Driver for the sanitizer build of the C oracle (tests/test_oracle_asan.py).
 * It is linked with oracle/oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer and calls every exported function on small and
 * degenerate inputs (empty graphs, one vertex, duplicates, self-loops,
 * out-of-range endpoints, every PageRank mode), so that an out-of-bounds
 * access, a leak or undefined arithmetic anywhere in the oracle stops the
 * run.  It also checks a few facts that hold for any correct oracle, so that
 * a silent wrong answer fails too.  Prints "oracle sanitizer run ok" at the
 * end; any failed check exits with status 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_set_threads(int nthreads);
uint64_t oracle_splitmix64(uint64_t seed, uint64_t k);
void oracle_rmat_edges(int scale, int64_t nedges, uint64_t seed, double t_a, double t_ab,
                       double t_abc, uint32_t *src, uint32_t *dst);
void oracle_web_degrees(uint64_t n, uint64_t seed, const int64_t *model, int64_t *deg);
void oracle_web_edges(uint64_t n, uint64_t seed, const int64_t *model, const int64_t *off,
                      uint32_t *src, uint32_t *dst);
int64_t oracle_web_row(uint64_t n, uint64_t seed, const int64_t *model, uint64_t u, uint32_t *out);
int64_t oracle_web_links_into(uint64_t n, uint64_t seed, const int64_t *model, const uint8_t *want,
                              int64_t cap, uint32_t *src, uint32_t *dst);
int64_t oracle_build_csr(int64_t n, int64_t nedges, const uint32_t *src, const uint32_t *dst,
                         int drop_self, int32_t *rowptr, int32_t *col);
void oracle_row_counts(int64_t n, const int32_t *rowptr, int32_t *deg);
void oracle_transpose(int64_t nrows, int64_t ncols, const int32_t *rowptr, const int32_t *col,
                      int32_t *rowptrT, int32_t *colT);
double oracle_sum(const double *x, int64_t n);
int oracle_pagerank(int64_t n, const int32_t *rowptrT, const int32_t *colT, const int32_t *outdeg,
                    double damping, double tol, int itermax, int fixed_iters, int mode,
                    const double *v, const double *x0, double *x_out, double *rho_hist,
                    double *D_hist, double *resid_out);

static int failures = 0;

#define CHECK(cond)                                                           \
  do {                                                                        \
    if (!(cond)) {                                                            \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);      \
      ++failures;                                                             \
    }                                                                         \
  } while (0)

/* exact allocations, so that one entry past the end is a reported error */
static void *xmalloc(size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  if (!p) exit(2);
  return p;
}

typedef struct {
  int64_t n, nnz;
  int32_t *rowptr, *col, *outdeg, *rowptrT, *colT;
} graph;

static graph make_graph(int64_t n, int64_t ne, const uint32_t *src, const uint32_t *dst) {
  graph g;
  g.n = n;
  g.rowptr = (int32_t *)xmalloc((size_t)(n + 1) * sizeof(int32_t));
  int32_t *col = (int32_t *)xmalloc((size_t)ne * sizeof(int32_t));
  g.nnz = oracle_build_csr(n, ne, src, dst, 1, g.rowptr, col);
  CHECK(g.nnz >= 0 && g.nnz <= ne);
  g.col = (int32_t *)xmalloc((size_t)g.nnz * sizeof(int32_t));
  if (g.nnz > 0) memcpy(g.col, col, (size_t)g.nnz * sizeof(int32_t));
  free(col);
  g.outdeg = (int32_t *)xmalloc((size_t)n * sizeof(int32_t));
  oracle_row_counts(n, g.rowptr, g.outdeg);
  g.rowptrT = (int32_t *)xmalloc((size_t)(n + 1) * sizeof(int32_t));
  g.colT = (int32_t *)xmalloc((size_t)g.nnz * sizeof(int32_t));
  oracle_transpose(n, n, g.rowptr, g.col, g.rowptrT, g.colT);
  CHECK(g.rowptrT[n] == g.nnz);
  return g;
}

static void free_graph(graph *g) {
  free(g->rowptr);
  free(g->col);
  free(g->outdeg);
  free(g->rowptrT);
  free(g->colT);
}

/* Runs every PageRank mode on g with exactly sized buffers; returns the
 * number of passes of the free-running uniform solve. */
static int run_pagerank(const graph *g) {
  int64_t n = g->n;
  double *x = (double *)xmalloc((size_t)n * sizeof(double));
  double *v = (double *)xmalloc((size_t)n * sizeof(double));
  double *x0 = (double *)xmalloc((size_t)n * sizeof(double));
  const int itermax = 200;
  double *rho = (double *)xmalloc((size_t)itermax * sizeof(double));
  double *Dh = (double *)xmalloc((size_t)(itermax + 1) * sizeof(double));
  double resid = -1.0;
  for (int64_t i = 0; i < n; ++i) {
    v[i] = (i % 3 == 0) ? 1.0 : 0.0;
    x0[i] = 1.0 / (double)n;
  }
  double vs = oracle_sum(v, n);
  for (int64_t i = 0; i < n; ++i) v[i] = vs > 0 ? v[i] / vs : 1.0 / (double)n;
  int it = 0;
  for (int mode = 0; mode <= 1; ++mode) {
    it = oracle_pagerank(n, g->rowptrT, g->colT, g->outdeg, 0.85, 1e-10, itermax, 0, mode,
                         NULL, NULL, x, rho, Dh, &resid);
    CHECK(it >= 1 && it <= itermax);
    CHECK(resid == rho[it - 1]);
    double s = oracle_sum(x, n);
    if (mode == 1 && n > 0) CHECK(fabs(s - 1.0) < 1e-12);
    if (mode == 0) CHECK(s <= 1.0 + 1e-12);
    for (int64_t i = 0; i < n; ++i) CHECK(x[i] >= 0.0);
    int k = oracle_pagerank(n, g->rowptrT, g->colT, g->outdeg, 0.85, 0.0, 1, 7, mode, v, x0, x,
                            rho, Dh, NULL);
    CHECK(k == 7);
    k = oracle_pagerank(n, g->rowptrT, g->colT, g->outdeg, 0.5, 1e-9, itermax, 0, mode, v, NULL,
                        x, NULL, NULL, NULL);
    CHECK(k >= 1 && k <= itermax);
  }
  free(x);
  free(v);
  free(x0);
  free(rho);
  free(Dh);
  return it;
}


/* Dense solve of M x = b by Gaussian elimination with partial pivoting
 * (M is n x n, row-major, overwritten; b becomes x). */
static void dense_solve(int n, double *M, double *b) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (fabs(M[(size_t)i * n + k]) > fabs(M[(size_t)piv * n + k])) piv = i;
    if (piv != k) {
      for (int j = 0; j < n; ++j) {
        double t = M[(size_t)k * n + j];
        M[(size_t)k * n + j] = M[(size_t)piv * n + j];
        M[(size_t)piv * n + j] = t;
      }
      double t = b[k];
      b[k] = b[piv];
      b[piv] = t;
    }
    for (int i = k + 1; i < n; ++i) {
      double f = M[(size_t)i * n + k] / M[(size_t)k * n + k];
      for (int j = k; j < n; ++j) M[(size_t)i * n + j] -= f * M[(size_t)k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= M[(size_t)i * n + j] * b[j];
    b[i] = s / M[(size_t)i * n + i];
  }
}

/* The PageRank fixed point from the raw edge list, without the oracle's
 * CSR: x = (1-d) v + d P x [+ d (sum of x over dangling j) v], with
 * P[i][j] = 1/outdeg_j for each distinct edge j -> i, j != i.  Returns the
 * L1 distance of the oracle's 400-pass iterate from it, relative to its L1
 * norm. */
static double lu_pin(int n, int64_t ne, const uint32_t *src, const uint32_t *dst, int mode) {
  double *A = (double *)calloc((size_t)n * n, sizeof(double));
  for (int64_t e = 0; e < ne; ++e)
    if (src[e] != dst[e]) A[(size_t)src[e] * n + dst[e]] = 1.0;
  double *outdeg = (double *)calloc((size_t)n, sizeof(double));
  for (int s = 0; s < n; ++s)
    for (int t = 0; t < n; ++t) outdeg[s] += A[(size_t)s * n + t];
  double *M = (double *)xmalloc((size_t)n * n * sizeof(double));
  double *b = (double *)xmalloc((size_t)n * sizeof(double));
  for (int i = 0; i < n; ++i) {
    b[i] = (1.0 - 0.85) / n;
    for (int j = 0; j < n; ++j) {
      double p = outdeg[j] > 0 ? A[(size_t)j * n + i] / outdeg[j] : 0.0;
      if (mode == 1 && outdeg[j] == 0) p = 1.0 / n;
      M[(size_t)i * n + j] = (i == j ? 1.0 : 0.0) - 0.85 * p;
    }
  }
  dense_solve(n, M, b);
  graph g = make_graph(n, ne, src, dst);
  double *x = (double *)xmalloc((size_t)n * sizeof(double));
  int it = oracle_pagerank(n, g.rowptrT, g.colT, g.outdeg, 0.85, 0.0, 1, 400, mode, NULL, NULL, x,
                           NULL, NULL, NULL);
  CHECK(it == 400);
  double err = 0.0, norm = 0.0;
  for (int i = 0; i < n; ++i) {
    err += fabs(x[i] - b[i]);
    norm += fabs(b[i]);
  }
  free_graph(&g);
  free(A);
  free(outdeg);
  free(M);
  free(b);
  free(x);
  return err / norm;
}

int main(void) {
  oracle_set_threads(4);

  /* published first output of SplitMix64 seeded with 1234567 */
  CHECK(oracle_splitmix64(1234567u, 0u) == 6457827717110365317ULL);

  /* R-MAT at scale 10, edge factor 16 */
  {
    const int scale = 10;
    const int64_t n = (int64_t)1 << scale, ne = 16 * n;
    uint32_t *src = (uint32_t *)xmalloc((size_t)ne * sizeof(uint32_t));
    uint32_t *dst = (uint32_t *)xmalloc((size_t)ne * sizeof(uint32_t));
    oracle_rmat_edges(scale, ne, 10u, 0.57, 0.76, 0.95, src, dst);
    for (int64_t e = 0; e < ne; ++e) CHECK(src[e] < (uint32_t)n && dst[e] < (uint32_t)n);
    graph g = make_graph(n, ne, src, dst);
    CHECK(g.nnz > n && g.nnz < ne);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = g.rowptr[i] + 1; e < g.rowptr[i + 1]; ++e) CHECK(g.col[e - 1] < g.col[e]);
    run_pagerank(&g);
    free_graph(&g);
    /* an endpoint out of range is reported, not written */
    dst[ne - 1] = (uint32_t)n;
    int32_t *rp = (int32_t *)xmalloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t *col = (int32_t *)xmalloc((size_t)ne * sizeof(int32_t));
    CHECK(oracle_build_csr(n, ne, src, dst, 1, rp, col) == -1);
    free(rp);
    free(col);
    free(src);
    free(dst);
  }

  /* duplicates and self-loops: 0->1 twice, 1->1, 1->2, 2->0; vertex 3 dangling */
  {
    const uint32_t src[] = {0, 0, 1, 1, 2};
    const uint32_t dst[] = {1, 1, 1, 2, 0};
    graph g = make_graph(4, 5, src, dst);
    CHECK(g.nnz == 3);
    CHECK(g.outdeg[0] == 1 && g.outdeg[1] == 1 && g.outdeg[2] == 1 && g.outdeg[3] == 0);
    run_pagerank(&g);
    free_graph(&g);
    /* the same list with self-loops kept */
    int32_t rp[5], col[5];
    CHECK(oracle_build_csr(4, 5, src, dst, 0, rp, col) == 4);
  }

  /* one vertex; n vertices without edges; a directed cycle (x = 1/n) */
  {
    graph one = make_graph(1, 0, NULL, NULL);
    run_pagerank(&one);
    free_graph(&one);
    graph none = make_graph(9, 0, NULL, NULL);
    run_pagerank(&none);
    free_graph(&none);
    enum { N = 17 };
    uint32_t src[N], dst[N];
    for (uint32_t i = 0; i < N; ++i) {
      src[i] = i;
      dst[i] = (i + 1) % N;
    }
    graph cyc = make_graph(N, N, src, dst);
    double x[N];
    oracle_pagerank(N, cyc.rowptrT, cyc.colT, cyc.outdeg, 0.85, 1e-12, 100, 0, 1, NULL, NULL, x,
                    NULL, NULL, NULL);
    for (int i = 0; i < N; ++i) CHECK(fabs(x[i] - 1.0 / N) < 1e-15);
    free_graph(&cyc);
  }

  /* dense LU pins: R-MAT at scales 3, 5, 7, both dangling modes */
  for (int scale = 3; scale <= 7; scale += 2) {
    const int n = 1 << scale;
    const int64_t ne = 16 * (int64_t)n;
    uint32_t *src = (uint32_t *)xmalloc((size_t)ne * sizeof(uint32_t));
    uint32_t *dst = (uint32_t *)xmalloc((size_t)ne * sizeof(uint32_t));
    oracle_rmat_edges(scale, ne, 100u + (uint64_t)scale, 0.57, 0.76, 0.95, src, dst);
    for (int mode = 0; mode <= 1; ++mode) CHECK(lu_pin(n, ne, src, dst, mode) <= 1e-12);
    free(src);
    free(dst);
  }

  /* closed forms: star inward (m leaves -> centre) and outward (centre ->
   * m leaves), uniform dangling mass */
  {
    enum { M = 40 };
    const double d = 0.85;
    uint32_t a[M], b[M];
    for (uint32_t i = 0; i < M; ++i) {
      a[i] = i + 1;
      b[i] = 0;
    }
    graph in = make_graph(M + 1, M, a, b);
    graph out = make_graph(M + 1, M, b, a);
    double x[M + 1];
    oracle_pagerank(M + 1, in.rowptrT, in.colT, in.outdeg, d, 1e-15, 1000, 0, 1, NULL, NULL, x,
                    NULL, NULL, NULL);
    CHECK(fabs(x[0] - (1 + M * d) / (M + 1 + M * d)) < 1e-14);
    for (int i = 1; i <= M; ++i) CHECK(fabs(x[i] - 1 / (M + 1 + M * d)) < 1e-14);
    oracle_pagerank(M + 1, out.rowptrT, out.colT, out.outdeg, d, 1e-15, 1000, 0, 1, NULL, NULL, x,
                    NULL, NULL, NULL);
    CHECK(fabs(x[0] - 1 / (M + 1 + d)) < 1e-14);
    for (int i = 1; i <= M; ++i) CHECK(fabs(x[i] - (M + d) / (M * (M + 1 + d))) < 1e-14);
    free_graph(&in);
    free_graph(&out);
  }

  /* the empty graph */
  {
    int32_t rp[1], rpT[1];
    CHECK(oracle_build_csr(0, 0, NULL, NULL, 1, rp, NULL) == 0);
    oracle_transpose(0, 0, rp, NULL, rpT, NULL);
    CHECK(rpT[0] == 0);
    CHECK(oracle_sum(NULL, 0) == 0.0);
  }

  /* sums over several chunks of the fixed reduction order */
  {
    const int64_t n = 300001;
    double *x = (double *)xmalloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) x[i] = (double)(i % 7);
    double want = 0.0;
    for (int64_t i = 0; i < n; ++i) want += (double)(i % 7);
    CHECK(oracle_sum(x, n) == want);
    free(x);
  }

  /* the web-shaped generator on a small vertex set */
  {
    const uint64_t n = 5000;
    const int64_t model[9] = {7, 400, 11633, 3277, 39322, 16, 1024, 2654435761LL, 12345};
    int64_t *deg = (int64_t *)xmalloc(n * sizeof(int64_t));
    oracle_web_degrees(n, 3u, model, deg);
    int64_t *off = (int64_t *)xmalloc((n + 1) * sizeof(int64_t));
    off[0] = 0;
    for (uint64_t u = 0; u < n; ++u) {
      CHECK(deg[u] == 0 || (deg[u] >= model[0] && deg[u] <= model[1]));
      off[u + 1] = off[u] + deg[u];
    }
    int64_t m = off[n];
    uint32_t *src = (uint32_t *)xmalloc((size_t)m * sizeof(uint32_t));
    uint32_t *dst = (uint32_t *)xmalloc((size_t)m * sizeof(uint32_t));
    oracle_web_edges(n, 3u, model, off, src, dst);
    for (int64_t e = 0; e < m; ++e) CHECK(src[e] < n && dst[e] < n);
    uint32_t *row = (uint32_t *)xmalloc((size_t)model[1] * sizeof(uint32_t));
    for (uint64_t u = 0; u < n; u += 97) {
      int64_t k = oracle_web_row(n, 3u, model, u, row);
      CHECK(k == deg[u]);
      for (int64_t j = 0; j < k; ++j) CHECK(row[j] == dst[off[u] + j]);
    }
    uint8_t *want = (uint8_t *)xmalloc(n);
    memset(want, 0, n);
    want[1] = want[4999] = 1;
    int64_t into = 0;
    for (int64_t e = 0; e < m; ++e) into += want[dst[e]];
    uint32_t *isrc = (uint32_t *)xmalloc((size_t)(into + 1) * sizeof(uint32_t));
    uint32_t *idst = (uint32_t *)xmalloc((size_t)(into + 1) * sizeof(uint32_t));
    CHECK(oracle_web_links_into(n, 3u, model, want, into, isrc, idst) == into);
    if (into > 0) CHECK(oracle_web_links_into(n, 3u, model, want, into - 1, isrc, idst) == -1);
    graph g = make_graph((int64_t)n, m, src, dst);
    run_pagerank(&g);
    free_graph(&g);
    free(deg);
    free(off);
    free(src);
    free(dst);
    free(row);
    free(want);
    free(isrc);
    free(idst);
  }

  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("oracle sanitizer run ok\n");
  return 0;
}
