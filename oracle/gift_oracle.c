/*
 * gift_oracle.c -- plain, slow, FP64 CPU oracle for the GiFt hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the device library; the two meet only through
 * the seeded inputs drawn by the workload generator.
 *
 * What it computes (GiFt, "The Power of Graph Signal Processing for Chip
 * Placement Acceleration", ICCAD'24):
 *
 *   1. netlist -> weighted cell graph with the clique net model (Section 3.2,
 *      the paragraph after Algorithm 1).  A net of M distinct cells adds weight
 *      w(M) to every pair of its cells; w(M) = 1/(M-1) (default) or the
 *      quadratic-wirelength weight 2/M of Section 2.2 (eq. wire_eq).
 *      Optionally a net of more than T cells is expanded as a star around a new
 *      virtual node instead (not in the paper; see build()).
 *   2. adjacency A (weights of parallel edges summed), degrees d_i = sum_j w_ij
 *      (Section 2.1).
 *   3. per self-loop weight sigma: the augmented normalised adjacency
 *      A~_sigma = (D + sigma I)^(-1/2) (A + sigma I) (D + sigma I)^(-1/2)
 *      (Section 3.2.1, eq. A_formulation).
 *   4. g' = sum_t alpha_t A~_{sigma_t}^{k_t} g (eq. proposed_filter), each
 *      power formed by k repeated sparse products (Section 3.2.1, powers of the
 *      augmented adjacency; complexity paragraph of Section 3.2.2).
 *
 * Readings where the paper is silent (each is a stated convention):
 *   - duplicate pins of one net count once; nets with fewer than two distinct
 *     cells add nothing; weights of different nets on one pair are summed;
 *   - the degree excludes the self-loop, which enters only through D + sigma I;
 *   - t_i = d_i + sigma = 0 (isolated cell, sigma = 0) gives s_i = 0, i.e. the
 *     row and column vanish;
 *   - star expansion: edge weight gamma = M * w(M) between the net's virtual
 *     node and every cell of the net (rounded once to FP64: M/(M-1) or
 *     exactly 2); virtual rows carry the self-loop sigma like every row,
 *     start at the mean of their cells' signal and are not returned.  The
 *     virtual nodes are rows N..N+V-1; the paper fixes no labelling of them,
 *     and two are provided (oracle_build_ordered): ascending net id, or
 *     ascending median cell of the net (the distinct cell at index M/2 of the
 *     ascending list), ties by ascending net id.  The two graphs are one
 *     graph under a relabelling of the virtual rows;
 *   - the combine is an FP64 sum in term order.
 * Summation orders are fixed so the structure, weights and degrees have a
 * single correct bit pattern: duplicates are summed in ascending net id,
 * degrees in ascending column, products in ascending column.
 *
 * Build with -ffp-contract=off: no fused multiply-adds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORACLE_OK = 0, ORACLE_EINVAL = 1, ORACLE_ENOMEM = 2 };
enum { ORACLE_W_INV_M1 = 0, ORACLE_W_TWO_OVER_M = 1 };
enum { ORACLE_STARS_BY_NET = 0, ORACLE_STARS_BY_MEDIAN = 1 };

typedef struct {
  int64_t num_cells;   /* N */
  int64_t num_virtual; /* V */
  int64_t num_rows;    /* R = N + V */
  int64_t nnz;         /* off-diagonal entries after merging */
  int64_t *row_ptr;    /* R + 1 */
  int32_t *col;        /* nnz */
  double *w;           /* nnz */
  double *deg;         /* R */
  int64_t num_nets;
  int weight_model;
  int64_t *ucell_ptr;  /* E + 1: sorted distinct cells of every net */
  int32_t *ucell;
  int32_t *virt_net;   /* V: the net each virtual row stands for */
} oracle_graph;

typedef struct {
  int32_t row, col, net;
  double w;
} triple;

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

static int cmp_triple(const void *a, const void *b) {
  const triple *x = (const triple *)a, *y = (const triple *)b;
  if (x->row != y->row) return (x->row > y->row) - (x->row < y->row);
  if (x->col != y->col) return (x->col > y->col) - (x->col < y->col);
  return (x->net > y->net) - (x->net < y->net);
}

/* (median cell, net) of a star net; ordered by median, then net */
typedef struct {
  int64_t median, net;
} star_key;

static int cmp_star_key(const void *a, const void *b) {
  const star_key *x = (const star_key *)a, *y = (const star_key *)b;
  if (x->median != y->median) return (x->median > y->median) - (x->median < y->median);
  return (x->net > y->net) - (x->net < y->net);
}

static double clique_weight(int64_t m, int model) {
  if (model == ORACLE_W_TWO_OVER_M) return 2.0 / (double)m;
  return 1.0 / (double)(m - 1);
}

static double star_weight(int64_t m, int model) {
  if (model == ORACLE_W_TWO_OVER_M) return 2.0;
  return (double)m / (double)(m - 1);
}

void oracle_free(oracle_graph *g) {
  if (!g) return;
  free(g->row_ptr);
  free(g->col);
  free(g->w);
  free(g->deg);
  free(g->ucell_ptr);
  free(g->ucell);
  free(g->virt_net);
  free(g);
}

/* Steps O1-O4: netlist -> canonical CSR of A and degrees, with the virtual
 * rows labelled by star_order (ORACLE_STARS_BY_NET or ORACLE_STARS_BY_MEDIAN,
 * see the header). */
int oracle_build_ordered(int64_t num_cells, int64_t num_nets, int64_t num_pins,
                         const int64_t *net_ptr, const int32_t *pin_cell,
                         int weight_model, int64_t star_threshold, int star_order,
                         oracle_graph **out) {
  *out = NULL;
  if (star_order != ORACLE_STARS_BY_NET && star_order != ORACLE_STARS_BY_MEDIAN)
    return ORACLE_EINVAL;
  if (num_cells < 0 || num_nets < 0 || num_pins < 0) return ORACLE_EINVAL;
  if (weight_model != ORACLE_W_INV_M1 && weight_model != ORACLE_W_TWO_OVER_M)
    return ORACLE_EINVAL;
  if (star_threshold < 0) return ORACLE_EINVAL;
  if (net_ptr[0] != 0 || net_ptr[num_nets] != num_pins) return ORACLE_EINVAL;
  for (int64_t e = 0; e < num_nets; ++e)
    if (net_ptr[e + 1] < net_ptr[e]) return ORACLE_EINVAL;
  for (int64_t p = 0; p < num_pins; ++p)
    if (pin_cell[p] < 0 || pin_cell[p] >= num_cells) return ORACLE_EINVAL;

  oracle_graph *g = (oracle_graph *)calloc(1, sizeof(oracle_graph));
  if (!g) return ORACLE_ENOMEM;
  g->num_cells = num_cells;
  g->num_nets = num_nets;
  g->weight_model = weight_model;
  g->ucell_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(num_nets + 1));
  g->ucell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(num_pins > 0 ? num_pins : 1));
  if (!g->ucell_ptr || !g->ucell) { oracle_free(g); return ORACLE_ENOMEM; }

  /* O1: distinct cells of every net, ascending. */
  int64_t w_at = 0, num_star = 0, z = 0;
  g->ucell_ptr[0] = 0;
  for (int64_t e = 0; e < num_nets; ++e) {
    int64_t a = net_ptr[e], b = net_ptr[e + 1];
    int32_t *dst = g->ucell + w_at;
    memcpy(dst, pin_cell + a, sizeof(int32_t) * (size_t)(b - a));
    qsort(dst, (size_t)(b - a), sizeof(int32_t), cmp_i32);
    int64_t m = 0;
    for (int64_t i = 0; i < b - a; ++i)
      if (m == 0 || dst[i] != dst[m - 1]) dst[m++] = dst[i];
    w_at += m;
    g->ucell_ptr[e + 1] = w_at;
    if (m < 2) continue;
    if (star_threshold > 0 && m > star_threshold) {
      num_star += 1;
      z += 2 * m;
    } else {
      z += m * (m - 1);
    }
  }
  g->num_virtual = num_star;
  g->num_rows = num_cells + num_star;
  g->virt_net = (int32_t *)malloc(sizeof(int32_t) * (size_t)(num_star > 0 ? num_star : 1));
  triple *t = (triple *)malloc(sizeof(triple) * (size_t)(z > 0 ? z : 1));
  if (!g->virt_net || !t) { free(t); oracle_free(g); return ORACLE_ENOMEM; }

  /* The virtual row of every star net: its rank among the star nets in net
   * order, or in (median cell, net) order. */
  int64_t *vrank = (int64_t *)malloc(sizeof(int64_t) * (size_t)(num_nets > 0 ? num_nets : 1));
  star_key *sk = (star_key *)malloc(sizeof(star_key) * (size_t)(num_star > 0 ? num_star : 1));
  if (!vrank || !sk) { free(vrank); free(sk); free(t); oracle_free(g); return ORACLE_ENOMEM; }
  {
    int64_t ns = 0;
    for (int64_t e = 0; e < num_nets; ++e) {
      int64_t a = g->ucell_ptr[e], m = g->ucell_ptr[e + 1] - a;
      if (m < 2 || !(star_threshold > 0 && m > star_threshold)) continue;
      sk[ns].median = star_order == ORACLE_STARS_BY_MEDIAN ? g->ucell[a + m / 2] : 0;
      sk[ns].net = e;
      ++ns;
    }
    if (star_order == ORACLE_STARS_BY_MEDIAN) qsort(sk, (size_t)ns, sizeof(star_key), cmp_star_key);
    for (int64_t r = 0; r < ns; ++r) vrank[sk[r].net] = r;
  }
  free(sk);

  /* O2: expansion into directed (row, col, net, weight) entries. */
  int64_t k = 0;
  for (int64_t e = 0; e < num_nets; ++e) {
    int64_t a = g->ucell_ptr[e], m = g->ucell_ptr[e + 1] - a;
    const int32_t *c = g->ucell + a;
    if (m < 2) continue;
    if (star_threshold > 0 && m > star_threshold) {
      int32_t vid = (int32_t)(num_cells + vrank[e]);
      double gam = star_weight(m, weight_model);
      g->virt_net[vrank[e]] = (int32_t)e;
      for (int64_t i = 0; i < m; ++i) {
        t[k].row = c[i]; t[k].col = vid; t[k].net = (int32_t)e; t[k].w = gam; ++k;
        t[k].row = vid; t[k].col = c[i]; t[k].net = (int32_t)e; t[k].w = gam; ++k;
      }
    } else {
      double wm = clique_weight(m, weight_model);
      for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < m; ++j) {
          if (i == j) continue;
          t[k].row = c[i]; t[k].col = c[j]; t[k].net = (int32_t)e; t[k].w = wm; ++k;
        }
    }
  }

  free(vrank);

  /* O3: sort by (row, col, net); merge equal (row, col) left to right. */
  qsort(t, (size_t)z, sizeof(triple), cmp_triple);
  int64_t nnz = 0;
  for (int64_t i = 0; i < z; ++i)
    if (i == 0 || t[i].row != t[i - 1].row || t[i].col != t[i - 1].col) ++nnz;
  g->nnz = nnz;
  g->row_ptr = (int64_t *)calloc((size_t)(g->num_rows + 1), sizeof(int64_t));
  g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  g->w = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  g->deg = (double *)calloc((size_t)(g->num_rows > 0 ? g->num_rows : 1), sizeof(double));
  if (!g->row_ptr || !g->col || !g->w || !g->deg) { free(t); oracle_free(g); return ORACLE_ENOMEM; }
  int64_t q = -1;
  for (int64_t i = 0; i < z; ++i) {
    if (i == 0 || t[i].row != t[i - 1].row || t[i].col != t[i - 1].col) {
      ++q;
      g->col[q] = t[i].col;
      g->w[q] = t[i].w;
      g->row_ptr[t[i].row + 1] += 1;
    } else {
      g->w[q] = g->w[q] + t[i].w;
    }
  }
  free(t);
  for (int64_t r = 0; r < g->num_rows; ++r) g->row_ptr[r + 1] += g->row_ptr[r];

  /* O4: d_i = sum of row i's weights, ascending column. */
  for (int64_t r = 0; r < g->num_rows; ++r) {
    double d = 0.0;
    for (int64_t p = g->row_ptr[r]; p < g->row_ptr[r + 1]; ++p) d = d + g->w[p];
    g->deg[r] = d;
  }
  *out = g;
  return ORACLE_OK;
}

/* Steps O1-O4 with the virtual rows in ascending net order. */
int oracle_build(int64_t num_cells, int64_t num_nets, int64_t num_pins,
                 const int64_t *net_ptr, const int32_t *pin_cell,
                 int weight_model, int64_t star_threshold, oracle_graph **out) {
  return oracle_build_ordered(num_cells, num_nets, num_pins, net_ptr, pin_cell, weight_model,
                              star_threshold, ORACLE_STARS_BY_NET, out);
}

void oracle_sizes(const oracle_graph *g, int64_t *sizes /* [N, V, R, nnz] */) {
  sizes[0] = g->num_cells;
  sizes[1] = g->num_virtual;
  sizes[2] = g->num_rows;
  sizes[3] = g->nnz;
}

void oracle_export(const oracle_graph *g, int64_t *row_ptr, int32_t *col, double *w,
                   double *deg, int32_t *virt_net) {
  if (row_ptr) memcpy(row_ptr, g->row_ptr, sizeof(int64_t) * (size_t)(g->num_rows + 1));
  if (col) memcpy(col, g->col, sizeof(int32_t) * (size_t)g->nnz);
  if (w) memcpy(w, g->w, sizeof(double) * (size_t)g->nnz);
  if (deg) memcpy(deg, g->deg, sizeof(double) * (size_t)g->num_rows);
  if (virt_net) memcpy(virt_net, g->virt_net, sizeof(int32_t) * (size_t)g->num_virtual);
}

/* Step O5: entries of A~_sigma.  a[p] for the off-diagonal entries of A in CSR
 * order, delta[i] for the diagonal (the self-loop sigma, normalised). */
int oracle_normalise(const oracle_graph *g, double sigma, double *a, double *delta) {
  if (!(sigma >= 0.0)) return ORACLE_EINVAL;
  int64_t rows = g->num_rows;
  double *s = (double *)malloc(sizeof(double) * (size_t)(rows > 0 ? rows : 1));
  if (!s) return ORACLE_ENOMEM;
  for (int64_t i = 0; i < rows; ++i) {
    double ti = g->deg[i] + sigma;
    s[i] = (ti == 0.0) ? 0.0 : 1.0 / sqrt(ti);
  }
  for (int64_t i = 0; i < rows; ++i) {
    for (int64_t p = g->row_ptr[i]; p < g->row_ptr[i + 1]; ++p)
      a[p] = (g->w[p] * s[i]) * s[g->col[p]];
    delta[i] = (sigma * s[i]) * s[i];
  }
  free(s);
  return ORACLE_OK;
}

/* One product y = A~_sigma x over R rows, c columns (row-major, ld = c). */
static void oracle_product(const oracle_graph *g, const double *a, const double *delta,
                           const double *x, double *y, int64_t c) {
  for (int64_t i = 0; i < g->num_rows; ++i) {
    for (int64_t q = 0; q < c; ++q) {
      double acc = 0.0;
      for (int64_t p = g->row_ptr[i]; p < g->row_ptr[i + 1]; ++p)
        acc = acc + a[p] * x[(int64_t)g->col[p] * c + q];
      y[i * c + q] = acc + delta[i] * x[i * c + q];
    }
  }
}

/* Steps O6-O8.  x_in: N x c (ld = c).  Terms (sigma_t, k_t, alpha_t).
 * y_out: N x c.  fixed (nullable): rows with fixed[i] != 0 are copied from
 * x_in after filtering. */
int oracle_filter(const oracle_graph *g, int64_t num_terms, const double *sigma,
                  const int32_t *order, const double *alpha, const double *x_in,
                  int64_t c, const uint8_t *fixed, double *y_out) {
  if (num_terms < 1 || c < 1) return ORACLE_EINVAL;
  for (int64_t t = 0; t < num_terms; ++t)
    if (!(sigma[t] >= 0.0) || order[t] < 1) return ORACLE_EINVAL;
  int64_t rows = g->num_rows, n = g->num_cells;
  size_t rc = (size_t)(rows > 0 ? rows : 1) * (size_t)c;
  double *x0 = (double *)malloc(sizeof(double) * rc);
  double *xa = (double *)malloc(sizeof(double) * rc);
  double *xb = (double *)malloc(sizeof(double) * rc);
  double *saved = (double *)malloc(sizeof(double) * rc * (size_t)num_terms);
  double *a = (double *)malloc(sizeof(double) * (size_t)(g->nnz > 0 ? g->nnz : 1));
  double *delta = (double *)malloc(sizeof(double) * (size_t)(rows > 0 ? rows : 1));
  int *done = (int *)calloc((size_t)num_terms, sizeof(int));
  int status = ORACLE_OK;
  if (!x0 || !xa || !xb || !saved || !a || !delta || !done) { status = ORACLE_ENOMEM; goto out; }

  /* O6: real rows from the input, virtual rows at the mean of their cells. */
  memcpy(x0, x_in, sizeof(double) * (size_t)n * (size_t)c);
  for (int64_t v = 0; v < g->num_virtual; ++v) {
    int64_t e = g->virt_net[v];
    int64_t lo = g->ucell_ptr[e], hi = g->ucell_ptr[e + 1];
    for (int64_t q = 0; q < c; ++q) {
      double sum = 0.0;
      for (int64_t p = lo; p < hi; ++p) sum = sum + x_in[(int64_t)g->ucell[p] * c + q];
      x0[(n + v) * c + q] = sum / (double)(hi - lo);
    }
  }

  /* O7: for every distinct sigma (ascending), repeated products. */
  for (;;) {
    double cur = 0.0;
    int found = 0;
    for (int64_t t = 0; t < num_terms; ++t)
      if (!done[t] && (!found || sigma[t] < cur)) { cur = sigma[t]; found = 1; }
    if (!found) break;
    int32_t kmax = 0;
    for (int64_t t = 0; t < num_terms; ++t)
      if (!done[t] && sigma[t] == cur && order[t] > kmax) kmax = order[t];
    status = oracle_normalise(g, cur, a, delta);
    if (status != ORACLE_OK) goto out;
    memcpy(xa, x0, sizeof(double) * (size_t)rows * (size_t)c);
    for (int32_t k = 1; k <= kmax; ++k) {
      oracle_product(g, a, delta, xa, xb, c);
      double *tmp = xa; xa = xb; xb = tmp;
      for (int64_t t = 0; t < num_terms; ++t)
        if (!done[t] && sigma[t] == cur && order[t] == k)
          memcpy(saved + (size_t)t * rc, xa, sizeof(double) * (size_t)rows * (size_t)c);
    }
    for (int64_t t = 0; t < num_terms; ++t)
      if (sigma[t] == cur) done[t] = 1;
  }

  /* O8: g' = sum_t alpha_t x^{k_t}_{sigma_t}, in term order; real rows only. */
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = 0; q < c; ++q) {
      double acc = 0.0;
      for (int64_t t = 0; t < num_terms; ++t)
        acc = acc + alpha[t] * saved[(size_t)t * rc + (size_t)(i * c + q)];
      y_out[i * c + q] = (fixed && fixed[i]) ? x_in[i * c + q] : acc;
    }
out:
  free(x0); free(xa); free(xb); free(saved); free(a); free(delta); free(done);
  return status;
}

/* Placement metrics of g (N x c, ld = c) on the netlist the graph was built
 * from, per column q, in float64:
 *   S[q]     = sum over nets e with M_e >= 2 distinct cells and over the pairs
 *              c < c' of its cells of w(M_e) (g_c - g_c')^2: the weighted
 *              quadratic wirelength of Section 2.2 (eq. wire_eq) under the
 *              clique net model, i.e. the smoothness g^T L g of eq. smoothness
 *              on the clique-model graph (whatever the star threshold: a star
 *              with its node at the mean of its cells has the same value);
 *   norm2[q] = sum_i g_i^2, so S / norm2 is the Rayleigh quotient of
 *              eq. smoothness_ray;
 *   hpwl[q]  = sum over those nets of max - min of g over the net's cells
 *              (half-perimeter wirelength, the paper's evaluation metric).
 * Sums run in ascending net, then cell, order. */
int oracle_evaluate(const oracle_graph *g, const double *x, int64_t c, double *S,
                    double *norm2, double *hpwl) {
  if (c < 1) return ORACLE_EINVAL;
  for (int64_t q = 0; q < c; ++q) {
    double s = 0.0, h = 0.0, n2 = 0.0;
    for (int64_t e = 0; e < g->num_nets; ++e) {
      int64_t lo = g->ucell_ptr[e], hi = g->ucell_ptr[e + 1];
      int64_t m = hi - lo;
      if (m < 2) continue;
      double w = clique_weight(m, g->weight_model);
      double mn = x[(int64_t)g->ucell[lo] * c + q], mx = mn;
      for (int64_t a = lo; a < hi; ++a) {
        double ga = x[(int64_t)g->ucell[a] * c + q];
        if (ga < mn) mn = ga;
        if (ga > mx) mx = ga;
        for (int64_t b = a + 1; b < hi; ++b) {
          double d = ga - x[(int64_t)g->ucell[b] * c + q];
          s = s + w * (d * d);
        }
      }
      h = h + (mx - mn);
    }
    for (int64_t i = 0; i < g->num_cells; ++i) n2 = n2 + x[i * c + q] * x[i * c + q];
    S[q] = s;
    norm2[q] = n2;
    hpwl[q] = h;
  }
  return ORACLE_OK;
}

/* The exact filter the paper's filter approximates (Section 3.2.2,
 * eq. derivative and eq. spectral): g' = (I + L~_sigma)^-1 g with
 * L~_sigma = I - A~_sigma, i.e. the solution of (2 I - A~_sigma) g' = g on all
 * R rows (virtual rows start from the mean of their cells, as in O6).  The
 * matrix is symmetric positive definite with eigenvalues in [1, 3), so the
 * textbook conjugate-gradient iteration converges quickly; it runs per
 * column in float64 from g' = 0 until ||r|| <= tol ||g|| (or max_iter
 * iterations) and reports the iterations of the slowest column. */
int oracle_filter_exact(const oracle_graph *g, double sigma, const double *x_in, int64_t c,
                        double tol, int64_t max_iter, const uint8_t *fixed, double *y_out,
                        int64_t *iters) {
  if (c < 1 || !(sigma >= 0.0) || !(tol > 0.0) || max_iter < 1) return ORACLE_EINVAL;
  int64_t rows = g->num_rows, n = g->num_cells;
  size_t rr = (size_t)(rows > 0 ? rows : 1);
  double *a = (double *)malloc(sizeof(double) * (size_t)(g->nnz > 0 ? g->nnz : 1));
  double *delta = (double *)malloc(sizeof(double) * rr);
  double *b = (double *)malloc(sizeof(double) * rr);
  double *x = (double *)malloc(sizeof(double) * rr);
  double *r = (double *)malloc(sizeof(double) * rr);
  double *p = (double *)malloc(sizeof(double) * rr);
  double *q = (double *)malloc(sizeof(double) * rr);
  int status = ORACLE_OK;
  if (!a || !delta || !b || !x || !r || !p || !q) { status = ORACLE_ENOMEM; goto out; }
  status = oracle_normalise(g, sigma, a, delta);
  if (status != ORACLE_OK) goto out;
  *iters = 0;
  for (int64_t col = 0; col < c; ++col) {
    /* right-hand side: cells from the input, virtual rows at their mean */
    for (int64_t i = 0; i < n; ++i) b[i] = x_in[i * c + col];
    for (int64_t v = 0; v < g->num_virtual; ++v) {
      int64_t e = g->virt_net[v];
      int64_t lo = g->ucell_ptr[e], hi = g->ucell_ptr[e + 1];
      double sum = 0.0;
      for (int64_t k = lo; k < hi; ++k) sum = sum + x_in[(int64_t)g->ucell[k] * c + col];
      double cells = (double)(hi - lo);
      b[n + v] = sum / cells;
    }
    double bb = 0.0, rho = 0.0;
    for (int64_t i = 0; i < rows; ++i) {
      x[i] = 0.0;
      r[i] = b[i];
      p[i] = b[i];
      bb = bb + b[i] * b[i];
    }
    rho = bb;
    int64_t it = 0;
    while (it < max_iter && rho > tol * tol * bb) {
      /* q = (2 I - A~) p */
      double pq = 0.0;
      for (int64_t i = 0; i < rows; ++i) {
        double acc = 0.0;
        for (int64_t k = g->row_ptr[i]; k < g->row_ptr[i + 1]; ++k)
          acc = acc + a[k] * p[g->col[k]];
        acc = acc + delta[i] * p[i];
        q[i] = 2.0 * p[i] - acc;
        pq = pq + p[i] * q[i];
      }
      double alpha = rho / pq, rho_new = 0.0;
      for (int64_t i = 0; i < rows; ++i) {
        x[i] = x[i] + alpha * p[i];
        r[i] = r[i] - alpha * q[i];
        rho_new = rho_new + r[i] * r[i];
      }
      double beta = rho_new / rho;
      for (int64_t i = 0; i < rows; ++i) p[i] = r[i] + beta * p[i];
      rho = rho_new;
      ++it;
    }
    if (it > *iters) *iters = it;
    for (int64_t i = 0; i < n; ++i)
      y_out[i * c + col] = (fixed && fixed[i]) ? x_in[i * c + col] : x[i];
  }
out:
  free(a); free(delta); free(b); free(x); free(r); free(p); free(q);
  return status;
}

/* Bin density of a placement (Section 2.2, eq. density_eq): the placement
 * region [xl, xh] x [yl, yh] is cut into nbx x nby equal bins and
 *     rho_b = sum_v l_x(v, b) l_y(v, b),
 * the overlap area of bin b with every object v, here the rectangle of width
 * w_v and height h_v centred at the object's position (x_v, y_v).  Objects
 * are the N cells of the graph; x is N x 2 (ld = 2).  density: nby x nbx,
 * row-major (bin (i, j) covers column i and row j).  */
int oracle_bin_density(int64_t n, const double *x, const double *w, const double *h,
                       double xl, double yl, double xh, double yh, int64_t nbx, int64_t nby,
                       double *density) {
  if (nbx < 1 || nby < 1 || !(xh > xl) || !(yh > yl)) return ORACLE_EINVAL;
  double bw = (xh - xl) / (double)nbx, bh = (yh - yl) / (double)nby;
  for (int64_t k = 0; k < nbx * nby; ++k) density[k] = 0.0;
  for (int64_t v = 0; v < n; ++v) {
    double x0 = x[2 * v] - 0.5 * w[v], x1 = x[2 * v] + 0.5 * w[v];
    double y0 = x[2 * v + 1] - 0.5 * h[v], y1 = x[2 * v + 1] + 0.5 * h[v];
    for (int64_t j = 0; j < nby; ++j) {
      double b0 = yl + (double)j * bh, b1 = b0 + bh;
      double ly = (y1 < b1 ? y1 : b1) - (y0 > b0 ? y0 : b0);
      if (ly <= 0.0) continue;
      for (int64_t i = 0; i < nbx; ++i) {
        double a0 = xl + (double)i * bw, a1 = a0 + bw;
        double lx = (x1 < a1 ? x1 : a1) - (x0 > a0 ? x0 : a0);
        if (lx <= 0.0) continue;
        density[j * nbx + i] = density[j * nbx + i] + lx * ly;
      }
    }
  }
  return ORACLE_OK;
}

/* A caller-supplied weighted graph: the undirected weighted graph that
 * Section 2.1 defines (A = {w_ij}, D = diag(sum_j w_ij)) and that Algorithm 1
 * takes as its input.  The CSR must be canonical: row_ptr[0] = 0,
 * non-decreasing, row_ptr[R] = nnz; columns strictly ascending within a row,
 * in [0, R) and never equal to the row (the self-loop is sigma, added in
 * eq. A_formulation); weights finite and >= 0.  Every row is a cell (no
 * virtual rows).  Degrees as in O4: the row's weights summed left to right.
 * Symmetry w_ij = w_ji is the caller's: the definitions above do not need it. */
int oracle_import_csr(int64_t num_rows, int64_t nnz, const int64_t *row_ptr,
                      const int32_t *col, const double *w, oracle_graph **out) {
  *out = NULL;
  if (num_rows < 0 || nnz < 0) return ORACLE_EINVAL;
  if (row_ptr[0] != 0 || row_ptr[num_rows] != nnz) return ORACLE_EINVAL;
  for (int64_t r = 0; r < num_rows; ++r) {
    if (row_ptr[r + 1] < row_ptr[r]) return ORACLE_EINVAL;
    for (int64_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p) {
      if (col[p] < 0 || col[p] >= num_rows || col[p] == r) return ORACLE_EINVAL;
      if (p > row_ptr[r] && col[p] <= col[p - 1]) return ORACLE_EINVAL;
      if (!(w[p] >= 0.0) || !isfinite(w[p])) return ORACLE_EINVAL;
    }
  }
  oracle_graph *g = (oracle_graph *)calloc(1, sizeof(oracle_graph));
  if (!g) return ORACLE_ENOMEM;
  g->num_cells = num_rows;
  g->num_rows = num_rows;
  g->nnz = nnz;
  g->row_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(num_rows + 1));
  g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  g->w = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  g->deg = (double *)malloc(sizeof(double) * (size_t)(num_rows > 0 ? num_rows : 1));
  g->ucell_ptr = (int64_t *)calloc(1, sizeof(int64_t));
  if (!g->row_ptr || !g->col || !g->w || !g->deg || !g->ucell_ptr) {
    oracle_free(g);
    return ORACLE_ENOMEM;
  }
  memcpy(g->row_ptr, row_ptr, sizeof(int64_t) * (size_t)(num_rows + 1));
  if (nnz > 0) {
    memcpy(g->col, col, sizeof(int32_t) * (size_t)nnz);
    memcpy(g->w, w, sizeof(double) * (size_t)nnz);
  }
  for (int64_t r = 0; r < num_rows; ++r) {
    double d = 0.0;
    for (int64_t p = g->row_ptr[r]; p < g->row_ptr[r + 1]; ++p) d = d + g->w[p];
    g->deg[r] = d;
  }
  *out = g;
  return ORACLE_OK;
}

/* Density overflow of a bin-density map (the quantity placers track from the
 * density of Section 2.2, eq. density_eq): the area by which bins exceed
 * `target` times their own area, over the total object area,
 *     sum_b max(0, rho_b - target * A_b) / total_area,
 * A_b = ((xh - xl) / nbx) ((yh - yl) / nby), summed over the bins in row-major
 * order. */
int oracle_density_overflow(const double *density, int64_t nbx, int64_t nby, double xl,
                            double yl, double xh, double yh, double target, double total_area,
                            double *overflow) {
  if (nbx < 1 || nby < 1 || !(xh > xl) || !(yh > yl) || !(total_area > 0.0)) return ORACLE_EINVAL;
  double area = ((xh - xl) / (double)nbx) * ((yh - yl) / (double)nby);
  double s = 0.0;
  for (int64_t k = 0; k < nbx * nby; ++k) {
    double e = density[k] - target * area;
    if (e > 0.0) s = s + e;
  }
  *overflow = s / total_area;
  return ORACLE_OK;
}
