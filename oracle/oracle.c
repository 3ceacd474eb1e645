/*
 * oracle.c -- plain, slow, obviously correct FP64 reference for the CSR
 * SpMV / SpMM path.  TEST INFRASTRUCTURE ONLY: it is called by the test suite,
 * by the smoke check and by the benchmark's CPU-baseline leg, never by the
 * library.  It shares no code, header or helper with the GPU library.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no fast-math, no FMA contraction)
 * so every product is rounded before it is added, in ascending nonzero order.
 *
 * Rows are distributed over OpenMP threads with schedule(dynamic,64), the
 * policy the paper found best for its row-parallel kernel (Sec. 4.1); one
 * thread owns each row, so the result is bit-identical for any thread count.
 *
 * Parity: every function here is pinned by tests against brute force on tiny
 * inputs, invariants or closed forms (no function is "parity unpinned").
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

/* ------------------------------------------------------------------------
 * CRS assembly from triplets (Sec. 3: arrays rptrs, cids, val).
 * Canonical form: rows ascending, columns strictly ascending within a row,
 * rptrs[0] = 0 and rptrs[m] = number of stored nonzeros.  Duplicate (i, j)
 * triplets are merged by summing their values in input order (reading: the
 * paper does not say; summing is the usual assembly convention).
 * Steps: (1) stable bucket sort of triplet indices by row (count, prefix,
 * place in input order); (2) inside each row sort (column, input index);
 * (3) merge equal columns.  Returns 0, or -1 on an out-of-range index.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t col;
  int64_t idx;
} orc_ent;

static int orc_ent_cmp(const void *a, const void *b) {
  const orc_ent *x = (const orc_ent *)a, *y = (const orc_ent *)b;
  if (x->col != y->col) return x->col < y->col ? -1 : 1;
  return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

int orc_csr_from_coo(int32_t m, int32_t n, int64_t nnz_in, const int32_t *r, const int32_t *c,
                     const double *v, int32_t *rowptr, int32_t *colind, double *values,
                     int64_t *nnz_out) {
  for (int64_t t = 0; t < nnz_in; ++t)
    if (r[t] < 0 || r[t] >= m || c[t] < 0 || c[t] >= n) return -1;
  int64_t *start = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
  for (int64_t t = 0; t < nnz_in; ++t) start[r[t] + 1]++;
  for (int32_t i = 0; i < m; ++i) start[i + 1] += start[i];
  orc_ent *ent = (orc_ent *)malloc(sizeof(orc_ent) * (size_t)(nnz_in > 0 ? nnz_in : 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)m + 1));
  memcpy(fill, start, sizeof(int64_t) * ((size_t)m + 1));
  for (int64_t t = 0; t < nnz_in; ++t) {
    int64_t pos = fill[r[t]]++;
    ent[pos].col = c[t];
    ent[pos].idx = t;
  }
  free(fill);
  /* sort each row's entries by (column, input index) */
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < m; ++i)
    qsort(ent + start[i], (size_t)(start[i + 1] - start[i]), sizeof(orc_ent), orc_ent_cmp);
  /* merge duplicates row by row (sequential: output positions depend on all
   * earlier rows) */
  int64_t out = 0;
  rowptr[0] = 0;
  for (int32_t i = 0; i < m; ++i) {
    int64_t p = start[i];
    while (p < start[i + 1]) {
      int32_t col = ent[p].col;
      double s = v[ent[p].idx];
      int64_t q = p + 1;
      while (q < start[i + 1] && ent[q].col == col) {
        s = s + v[ent[q].idx];
        ++q;
      }
      colind[out] = col;
      values[out] = s;
      ++out;
      p = q;
    }
    rowptr[i + 1] = (int32_t)out;
  }
  *nnz_out = out;
  free(ent);
  free(start);
  return 0;
}

/* ------------------------------------------------------------------------
 * Row binning by row length (the GPU analogue of the paper's dynamic row
 * chunks, Sec. 4.1).  Bin b holds the rows whose length L satisfies
 * L <= upper[b] and L > upper[b-1]; the last bin takes every remaining row.
 * row_perm lists bin 0's rows, then bin 1's, ..., ascending inside each bin;
 * bin_off[b] is the position of bin b's first row, bin_off[nbins] = m.
 * ---------------------------------------------------------------------- */
void orc_bin_rows(int32_t m, const int32_t *rowptr, int32_t nbins, const int32_t *upper,
                  int32_t *row_perm, int32_t *bin_off) {
  int32_t *bin = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  for (int32_t i = 0; i < m; ++i) {
    int32_t L = rowptr[i + 1] - rowptr[i];
    int32_t b = 0;
    while (b < nbins - 1 && L > upper[b]) ++b;
    bin[i] = b;
  }
  int32_t pos = 0;
  for (int32_t b = 0; b < nbins; ++b) {
    bin_off[b] = pos;
    for (int32_t i = 0; i < m; ++i)
      if (bin[i] == b) row_perm[pos++] = i;
  }
  bin_off[nbins] = pos;
  free(bin);
}

/* ------------------------------------------------------------------------
 * SpMV, y <- A x (Sec. 3): y_i is the sum over the nonzeros of row i of
 * val[p] * x[cids[p]], taken in ascending p; an empty row gives +0.0; y is
 * overwritten.  nthreads <= 0 uses the OpenMP default.
 * ---------------------------------------------------------------------- */
void orc_spmv(int32_t m, const int32_t *rowptr, const int32_t *colind, const double *values,
              const double *x, double *y, int nthreads) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
  for (int32_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      double prod = values[p] * x[colind[p]];
      s = s + prod;
    }
    y[i] = s;
  }
}

/* ------------------------------------------------------------------------
 * SpMM, Y <- A X (Sec. 5): for row i a temporary of k zeros accumulates
 * val[p] * X[cids[p], :] for each nonzero in ascending p, then is stored into
 * Y[i, :].  X is n x k and Y is m x k, both row-major with leading dimensions
 * ldx and ldy (reading of the paper's X shape: n x k, Sec. 3).
 * ---------------------------------------------------------------------- */
void orc_spmm(int32_t m, int32_t k, const int32_t *rowptr, const int32_t *colind,
              const double *values, const double *X, int64_t ldx, double *Y, int64_t ldy,
              int nthreads) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
  {
    double *temp = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
#pragma omp for schedule(dynamic, 64)
    for (int32_t i = 0; i < m; ++i) {
      for (int32_t j = 0; j < k; ++j) temp[j] = 0.0;
      for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const double *xr = X + (int64_t)colind[p] * ldx;
        for (int32_t j = 0; j < k; ++j) {
          double prod = values[p] * xr[j];
          temp[j] = temp[j] + prod;
        }
      }
      for (int32_t j = 0; j < k; ++j) Y[(int64_t)i * ldy + j] = temp[j];
    }
    free(temp);
  }
}

/* ------------------------------------------------------------------------
 * Transpose product, dX <- A^T dY (the CCS dual of CRS, Sec. 3): for every
 * nonzero p in ascending order, dX[cids[p], :] += val[p] * dY[row(p), :].
 * Columns no nonzero touches get +0.0.  Sequential by construction.
 * ---------------------------------------------------------------------- */
void orc_spmv_t(int32_t m, int32_t n, int32_t k, const int32_t *rowptr, const int32_t *colind,
                const double *values, const double *dY, int64_t lddy, double *dX, int64_t lddx) {
  for (int32_t j = 0; j < n; ++j)
    for (int32_t t = 0; t < k; ++t) dX[(int64_t)j * lddx + t] = 0.0;
  for (int32_t i = 0; i < m; ++i)
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      double *dst = dX + (int64_t)colind[p] * lddx;
      for (int32_t t = 0; t < k; ++t) {
        double prod = values[p] * dY[(int64_t)i * lddy + t];
        dst[t] = dst[t] + prod;
      }
    }
}

/* ------------------------------------------------------------------------
 * Sampled dot (gradient of y = A(values) x with respect to the values):
 * out[p] = sum over t of dY[row(p), t] * X[cids[p], t], ascending t.
 * ---------------------------------------------------------------------- */
void orc_sddmm(int32_t m, int32_t k, const int32_t *rowptr, const int32_t *colind,
               const double *dY, int64_t lddy, const double *X, int64_t ldx, double *out) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < m; ++i)
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      double s = 0.0;
      for (int32_t t = 0; t < k; ++t) {
        double prod = dY[(int64_t)i * lddy + t] * X[(int64_t)colind[p] * ldx + t];
        s = s + prod;
      }
      out[p] = s;
    }
}

/* Per-row magnitude sum_p |val[p] * x[cids[p]]| (the scale in floating-point
 * error bounds of a row's dot product). */
void orc_spmv_abs(int32_t m, const int32_t *rowptr, const int32_t *colind, const double *values,
                  const double *x, double *out) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) s = s + fabs(values[p] * x[colind[p]]);
    out[i] = s;
  }
}

/* ------------------------------------------------------------------------
 * Useful cacheline density (Sec. 4.1): for each nonempty row, the number of
 * nonzeros divided by (line * number of distinct x cachelines the row
 * touches); UCLD is the mean over nonempty rows.  `line` is the number of x
 * elements per cacheline (8 doubles on the paper's machine).  Columns must be
 * sorted within rows.  Returns the mean; *rows_used gets the row count.
 * ---------------------------------------------------------------------- */
double orc_ucld(int32_t m, const int32_t *rowptr, const int32_t *colind, int32_t line,
                int64_t *rows_used) {
  double sum = 0.0;
  int64_t used = 0;
  for (int32_t i = 0; i < m; ++i) {
    int32_t L = rowptr[i + 1] - rowptr[i];
    if (L == 0) continue;
    int64_t lines = 0, last = -1;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      int64_t ln = colind[p] / line;
      if (ln != last) {
        ++lines;
        last = ln;
      }
    }
    sum += (double)L / ((double)line * (double)lines);
    ++used;
  }
  *rows_used = used;
  return used ? sum / (double)used : 0.0;
}

/* ------------------------------------------------------------------------
 * Vector access (Sec. 4.2 and Sec. 4.4): the expected number of times the
 * input vector is moved from memory when rows are dealt to `parts` caches in
 * chunks of `chunk` consecutive rows, round-robin, each cache infinite.  It is
 * the number of distinct (part, x cacheline) pairs touched, divided by the
 * number of x cachelines, ceil(n / line).
 * ---------------------------------------------------------------------- */
double orc_vector_access(int32_t m, int32_t n, const int32_t *rowptr, const int32_t *colind,
                         int32_t line, int32_t parts, int32_t chunk) {
  int64_t nlines = ((int64_t)n + line - 1) / line;
  if (nlines == 0) return 0.0;
  int32_t *seen = (int32_t *)calloc((size_t)nlines, sizeof(int32_t));
  int64_t pairs = 0;
  for (int32_t q = 0; q < parts; ++q) {
    for (int64_t c0 = (int64_t)q * chunk; c0 < m; c0 += (int64_t)parts * chunk) {
      int64_t c1 = c0 + chunk < m ? c0 + chunk : m;
      for (int64_t i = c0; i < c1; ++i) {
        for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
          int64_t ln = colind[p] / line;
          if (seen[ln] != q + 1) {
            seen[ln] = q + 1;
            ++pairs;
          }
        }
      }
    }
  }
  free(seen);
  return (double)pairs / (double)nlines;
}

/* ------------------------------------------------------------------------
 * Distinct x cachelines per row tile (the locality a workgroup sees; the
 * per-tile form of the paper's cacheline counting, Sec. 4.1 and 4.2): rows
 * are cut into tiles of `tile` consecutive rows; the result is the number of
 * distinct (tile, x line) pairs, x line = column / line.  Divided by the
 * number of tiles it is the mean distinct lines a tile gathers; nnz divided
 * by it is the mean number of gathers per fetched line inside a tile.
 * ---------------------------------------------------------------------- */
int64_t orc_tile_lines(int32_t m, int32_t n, const int32_t *rowptr, const int32_t *colind, int32_t line,
                       int32_t tile) {
  int64_t nlines = ((int64_t)n + line - 1) / line;
  if (nlines == 0 || m == 0) return 0;
  int64_t *stamp = (int64_t *)calloc((size_t)nlines, sizeof(int64_t));
  int64_t pairs = 0;
  for (int64_t t = 0; t * tile < m; ++t) {
    int64_t r1 = (t + 1) * tile < m ? (t + 1) * tile : m;
    for (int64_t i = t * tile; i < r1; ++i)
      for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        int64_t ln = colind[p] / line;
        if (stamp[ln] != t + 1) {
          stamp[ln] = t + 1;
          ++pairs;
        }
      }
  }
  free(stamp);
  return pairs;
}

/* ------------------------------------------------------------------------
 * Reverse Cuthill-McKee ordering (Sec. 4.4 applies it to every matrix; the
 * algorithm is Cuthill and McKee's breadth-first numbering, reversed).  The
 * paper used MATLAB's implementation and gives no tie rules, so this reading
 * fixes them:
 *   - the graph is the pattern of A + A^T without the diagonal (n x n);
 *   - components are numbered one after the other; each starts from the
 *     unnumbered vertex of smallest (degree, index), moved to a
 *     pseudo-peripheral vertex by George and Liu's rule: build the level
 *     structure from r, take the vertex of smallest (degree, index) in its
 *     last level, and move there while that deepens the structure;
 *   - breadth-first numbering from the start vertex, the unnumbered
 *     neighbours of each vertex appended in ascending (degree, index);
 *   - the whole numbering is reversed at the end.
 * perm[new] = old.  Returns 0, or -1 if the matrix is not square.
 * ---------------------------------------------------------------------- */
static const int32_t *orc_rcm_deg; /* qsort has no context argument */

static int orc_by_deg(const void *a, const void *b) {
  int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
  if (orc_rcm_deg[u] != orc_rcm_deg[v]) return orc_rcm_deg[u] < orc_rcm_deg[v] ? -1 : 1;
  return (u > v) - (u < v);
}

static int orc_i32_cmp(const void *a, const void *b) {
  int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
  return (u > v) - (u < v);
}

/* Level structure from r over unnumbered vertices: fills `lv` with the
 * vertices in breadth-first order, returns the number of levels and sets
 * [*last0, *last1) to the last level's slice of lv. */
static int32_t orc_levels(int32_t r, const int64_t *xadj, const int32_t *adj, const char *numbered,
                          int32_t *mark, int32_t stamp, int32_t *lv, int32_t *last0, int32_t *last1) {
  int32_t head = 0, tail = 0, nlev = 0;
  lv[tail++] = r;
  mark[r] = stamp;
  while (head < tail) {
    int32_t lo = head, hi = tail;
    ++nlev;
    *last0 = lo;
    *last1 = hi;
    for (int32_t t = lo; t < hi; ++t) {
      int32_t v = lv[t];
      for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e) {
        int32_t w = adj[e];
        if (!numbered[w] && mark[w] != stamp) {
          mark[w] = stamp;
          lv[tail++] = w;
        }
      }
    }
    head = hi;
  }
  return nlev;
}

int orc_rcm(int32_t m, int32_t n, const int32_t *rowptr, const int32_t *colind, int32_t *perm) {
  if (m != n) return -1;
  if (n == 0) return 0;
  /* symmetric adjacency: count both directions, fill, sort, drop repeats */
  int32_t *cnt = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  for (int32_t i = 0; i < n; ++i)
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
      if (colind[p] != i) {
        ++cnt[i];
        ++cnt[colind[p]];
      }
  int64_t *xadj = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  xadj[0] = 0;
  for (int32_t i = 0; i < n; ++i) xadj[i + 1] = xadj[i] + cnt[i];
  int32_t *adj = (int32_t *)malloc((size_t)(xadj[n] > 0 ? xadj[n] : 1) * sizeof(int32_t));
  int64_t *fill = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  for (int32_t i = 0; i < n; ++i) fill[i] = xadj[i];
  for (int32_t i = 0; i < n; ++i)
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      int32_t j = colind[p];
      if (j != i) {
        adj[fill[i]++] = j;
        adj[fill[j]++] = i;
      }
    }
  /* sort each list, remove repeats, compact */
  int64_t out = 0;
  for (int32_t i = 0; i < n; ++i) {
    int64_t b = xadj[i], e = xadj[i + 1];
    qsort(adj + b, (size_t)(e - b), sizeof(int32_t), orc_i32_cmp);
    int64_t start = out;
    for (int64_t t = b; t < e; ++t)
      if (t == b || adj[t] != adj[t - 1]) adj[out++] = adj[t];
    xadj[i] = start;
    cnt[i] = (int32_t)(out - start); /* degree */
  }
  xadj[n] = out;
  for (int32_t i = n - 1; i >= 0; --i) xadj[i + 1] = xadj[i] + cnt[i];
  xadj[0] = 0;
  /* xadj was rebuilt from degrees: lists are contiguous in vertex order */
  orc_rcm_deg = cnt;
  int32_t *bydeg = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  for (int32_t i = 0; i < n; ++i) bydeg[i] = i;
  qsort(bydeg, (size_t)n, sizeof(int32_t), orc_by_deg);
  char *numbered = (char *)calloc((size_t)n, 1);
  int32_t *mark = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  int32_t *lv = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *nb = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t pos = 0, scan = 0, stamp = 0;
  while (pos < n) {
    while (numbered[bydeg[scan]]) ++scan;
    int32_t r = bydeg[scan];
    int32_t l0, l1;
    int32_t depth = orc_levels(r, xadj, adj, numbered, mark, ++stamp, lv, &l0, &l1);
    for (;;) {
      int32_t x = lv[l0];
      for (int32_t t = l0 + 1; t < l1; ++t) {
        int32_t v = lv[t];
        if (cnt[v] < cnt[x] || (cnt[v] == cnt[x] && v < x)) x = v;
      }
      int32_t k0, k1;
      int32_t d2 = orc_levels(x, xadj, adj, numbered, mark, ++stamp, lv, &k0, &k1);
      if (d2 > depth) {
        r = x;
        depth = d2;
        l0 = k0;
        l1 = k1;
      } else {
        break;
      }
    }
    /* breadth-first numbering from r */
    int32_t head = pos;
    order[pos++] = r;
    numbered[r] = 1;
    while (head < pos) {
      int32_t v = order[head++];
      int32_t k = 0;
      for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e)
        if (!numbered[adj[e]]) nb[k++] = adj[e];
      qsort(nb, (size_t)k, sizeof(int32_t), orc_by_deg);
      for (int32_t t = 0; t < k; ++t) {
        numbered[nb[t]] = 1;
        order[pos++] = nb[t];
      }
    }
  }
  for (int32_t i = 0; i < n; ++i) perm[i] = order[n - 1 - i];
  free(cnt);
  free(xadj);
  free(adj);
  free(fill);
  free(bydeg);
  free(numbered);
  free(mark);
  free(lv);
  free(order);
  free(nb);
  return 0;
}

int orc_max_threads(void) { return omp_get_max_threads(); }
