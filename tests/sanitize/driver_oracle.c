/* The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer: every
 * entry point on small graphs and point sets, including the degenerate cases
 * the method has (two vertices, coincident points, a star, disconnected
 * pairs in the full stress).  Exits 0 when the calls succeed and their
 * results are finite (a sanitizer report aborts the run). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mm_oracle.h"

static int failures = 0;
#define EXPECT(cond, what)                                   \
  do {                                                       \
    if (!(cond)) { printf("FAILED: %s\n", what); ++failures; } \
  } while (0)

typedef struct { int32_t n; int32_t* rp; int32_t* col; int64_t nnz; } csr;

static csr grid(int a, int b) {
  csr g;
  g.n = a * b;
  g.rp = calloc((size_t)g.n + 1, sizeof(int32_t));
  g.col = malloc(sizeof(int32_t) * 4 * (size_t)g.n);
  int64_t e = 0;
  for (int v = 0; v < g.n; ++v) {
    const int i = v / b, j = v % b;
    int nb[4], m = 0;
    if (i > 0) nb[m++] = v - b;
    if (j > 0) nb[m++] = v - 1;
    if (j + 1 < b) nb[m++] = v + 1;
    if (i + 1 < a) nb[m++] = v + b;
    for (int t = 0; t < m; ++t) g.col[e++] = nb[t];
    g.rp[v + 1] = (int32_t)e;
  }
  g.nnz = e;
  return g;
}

static int finite_all(const double* x, int64_t m) {
  for (int64_t i = 0; i < m; ++i) if (!isfinite(x[i])) return 0;
  return 1;
}

static void run_graph(csr g, int32_t k) {
  const int32_t n = g.n;
  EXPECT(orc_validate(n, g.rp, g.col, NULL, NULL) == 0, "validate");
  int64_t* off = malloc(sizeof(int64_t) * ((size_t)n + 1));
  EXPECT(orc_khop_build(n, g.rp, g.col, k, off, NULL, NULL) == 0, "khop sizes");
  int32_t* hend = malloc(sizeof(int32_t) * (size_t)n * (size_t)k);
  int32_t* nbr = malloc(sizeof(int32_t) * (size_t)(off[n] > 0 ? off[n] : 1));
  EXPECT(orc_khop_build(n, g.rp, g.col, k, off, hend, nbr) == 0, "khop");
  double* x = malloc(sizeof(double) * 2 * (size_t)n);
  double* F = malloc(sizeof(double) * 2 * (size_t)n);
  double* y = malloc(sizeof(double) * 2 * (size_t)n);
  orc_init_layout(n, 7, 0, x);
  for (int32_t i = 0; i < 2 * n; ++i) x[i] *= 5.0;
  if (n > 3) { x[2] = x[0]; x[3] = x[1]; }  /* a coincident pair */
  int64_t st[4];
  uint64_t* codes = malloc(sizeof(uint64_t) * (size_t)n);
  int32_t* order = malloc(sizeof(int32_t) * (size_t)n);
  int64_t* nodes = malloc(sizeof(int64_t) * 5 * 2 * (size_t)n);
  EXPECT(orc_bh(n, x, 0.0, 0.5, F, codes, order, nodes, 2 * (int64_t)n, st) == 0, "barnes-hut");
  EXPECT(finite_all(F, 2 * (int64_t)n), "BH finite");
  orc_farfield_exact(n, x, 1.0, F);
  EXPECT(finite_all(F, 2 * (int64_t)n), "exact finite");
  double d[2];
  int32_t* c = malloc(sizeof(int32_t) * (size_t)n);
  for (int32_t v = 0; v < n; ++v) c[v] = 1 + v % 3;
  EXPECT(orc_sweep(n, 0, k, off, hend, nbr, NULL, 1.0, x, F, 0.3, 0.0, y, d) == 0, "sweep");
  EXPECT(orc_sweep(n, 1, k, off, hend, nbr, c, 1.0, x, F, 0.3, 0.5, y, d) == 0, "coarse sweep");
  EXPECT(orc_sweep_direct(n, 0, k, off, hend, nbr, NULL, 1.0, x, 0.3, 0.0, y, d) == 0, "direct");
  EXPECT(finite_all(y, 2 * (int64_t)n), "sweep finite");
  int32_t rows[3] = {0, n / 2, n - 1};
  double yr[6];
  int64_t sz[3];
  EXPECT(orc_sweep_rows(n, g.rp, g.col, 0, k, NULL, 1.0, x, F, 0.3, 0.0, rows, 3, yr, sz) == 0,
         "sweep rows");
  int32_t* label = malloc(sizeof(int32_t) * (size_t)n);
  int32_t moves[10];
  for (int32_t v = 0; v < n; ++v) label[v] = v;
  const int r = orc_lp(n, g.rp, g.col, c, NULL, 6.0, 10, 3, 1, label, moves);
  EXPECT(r >= 0, "label propagation");
  int32_t* cl = malloc(sizeof(int32_t) * (size_t)n);
  int32_t* crp = malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t* ccol = malloc(sizeof(int32_t) * (size_t)g.nnz);
  int32_t* cc = malloc(sizeof(int32_t) * (size_t)n);
  int32_t* cw = malloc(sizeof(int32_t) * (size_t)g.nnz);
  int64_t cnnz = 0;
  const int32_t nc = orc_contract(n, g.rp, g.col, c, NULL, label, cl, crp, ccol, cc, cw, &cnnz);
  EXPECT(nc >= 1 && nc <= n, "contract");
  double* cx = malloc(sizeof(double) * 2 * (size_t)nc);
  orc_init_layout(nc, 7, 1, cx);
  orc_prolong(n, cl, cc, cx, 7, 0, y);
  EXPECT(finite_all(y, 2 * (int64_t)n), "prolong finite");
  EXPECT(orc_cluster_far(n, x, c, cl, nc, cl, nc, 0.0, F) == 0, "cluster far field");
  double ob[3], fs[3];
  EXPECT(orc_objective(n, 0, k, off, hend, nbr, NULL, 1.0, x, 0.0, ob) == 0, "objective");
  EXPECT(orc_full_stress(n, g.rp, g.col, x, fs) == 0, "full stress");
  EXPECT(finite_all(ob, 3) && finite_all(fs, 3), "objectives finite");
  /* learned far field: random weights */
  double* wts = malloc(sizeof(double) * 4866);
  for (int i = 0; i < 4866; ++i) wts[i] = 0.05 * sin(0.37 * i);
  EXPECT(orc_bh_learned(n, x, 1.0, wts, F) == 0, "learned far field");
  int64_t cnt = 0;
  EXPECT(orc_far_samples(n, x, 1.0, 0, NULL, NULL, NULL, NULL, NULL, &cnt) == 0, "sample count");
  if (cnt > 0) {
    int32_t* su = malloc(sizeof(int32_t) * (size_t)cnt);
    int64_t* sn = malloc(sizeof(int64_t) * (size_t)cnt);
    double* sf = malloc(sizeof(double) * 8 * (size_t)cnt);
    double* stt = malloc(sizeof(double) * 2 * (size_t)cnt);
    double* sc = malloc(sizeof(double) * 2 * (size_t)cnt);
    EXPECT(orc_far_samples(n, x, 1.0, cnt, su, sn, sf, stt, sc, &cnt) == 0, "samples");
    double* h = malloc(sizeof(double) * 2 * (size_t)cnt);
    orc_mlp_forward(wts, cnt, sf, h);
    EXPECT(finite_all(h, 2 * cnt), "mlp finite");
    free(su); free(sn); free(sf); free(stt); free(sc); free(h);
  }
  free(off); free(hend); free(nbr); free(x); free(F); free(y); free(codes); free(order);
  free(nodes); free(c); free(label); free(cl); free(crp); free(ccol); free(cc); free(cw);
  free(cx); free(wts);
}

int main(void) {
  csr g = grid(9, 7);
  run_graph(g, 3);
  run_graph(g, 1);
  free(g.rp); free(g.col);
  csr p = grid(1, 2);  /* two vertices, one edge */
  run_graph(p, 2);
  free(p.rp); free(p.col);
  /* star with 40 leaves */
  csr s;
  s.n = 41;
  s.rp = malloc(sizeof(int32_t) * 42);
  s.col = malloc(sizeof(int32_t) * 80);
  s.rp[0] = 0;
  for (int v = 1; v <= 40; ++v) s.col[v - 1] = v;
  s.rp[1] = 40;
  for (int v = 1; v <= 40; ++v) { s.col[40 + v - 1] = 0; s.rp[v + 1] = 40 + v; }
  s.nnz = 80;
  run_graph(s, 2);
  free(s.rp); free(s.col);
  /* points only: many coincident points in the quadtree */
  const int32_t n = 300;
  double* x = malloc(sizeof(double) * 2 * n);
  double* F = malloc(sizeof(double) * 2 * n);
  for (int32_t i = 0; i < n; ++i) { x[2 * i] = (i % 7) * 0.5; x[2 * i + 1] = (i % 5) * 0.25; }
  int64_t st[4];
  EXPECT(orc_bh(n, x, 0.0, 0.7, F, NULL, NULL, NULL, 0, st) == 0, "coincident BH");
  EXPECT(finite_all(F, 2 * n), "coincident BH finite");
  free(x); free(F);
  printf("oracle entry points: %d failures\n", failures);
  return failures ? 1 : 0;
}
