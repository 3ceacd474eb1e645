/*
 * spgen.c -- seeded synthetic sparse-matrix and dense-vector generators.
 *
 * This module only draws inputs: COO triplets (row, col, value) and dense
 * vectors.  It contains none of the arithmetic of the method under test (no
 * CSR assembly, no products, no reductions); both the oracle and the GPU
 * library consume what it produces.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  Every stream is counter
 * addressed so that generation is independent of thread count:
 *   key(seed, tag)      = mix(seed ^ tag)
 *   row stream (key, i) = SplitMix64 state initialised to mix(key ^ ((i+1)*PHI2))
 *   element j of a vector stream = mix(key + (j+1)*GOLDEN), i.e. the j-th
 *   output of a SplitMix64 generator whose state starts at key.
 * Uniform doubles are (z >> 11) * 2^-53 in [0, 1).
 *
 * Row-length law: discrete Zipf-Mandelbrot P(L) proportional to (L+q)^-alpha
 * on L in [1, Lmax], sampled by inverse CDF (binary search on the FP64 CDF).
 * Hot columns: column j gets an integer weight w_j drawn from the same law;
 * each row draws its L_i distinct columns with probability proportional to
 * w_j (rejection of in-row repeats), or, for rows longer than n/4, by
 * Efraimidis-Spirakis keys (log u_j / w_j, largest L_i).
 * Columns are emitted in draw order (not sorted): assembling canonical CSR is
 * the consumer's job.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL
#define PHI2 0xD1B54A32D192ED03ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t next64(uint64_t *s) {
  *s += GOLDEN;
  return mix64(*s);
}
static inline double unit(uint64_t z) { return (double)(z >> 11) * 0x1.0p-53; }

uint64_t spgen_key(uint64_t seed, uint64_t tag) { return mix64(seed ^ tag); }
static inline uint64_t row_state(uint64_t key, int64_t i) {
  return mix64(key ^ ((uint64_t)(i + 1) * PHI2));
}

/* ---- dense vectors ---------------------------------------------------- */

/* out[j] = lo + (hi-lo) * u_j for j in [0, len) */
void spgen_uniform(uint64_t key, int64_t len, double lo, double hi, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < len; ++j)
    out[j] = lo + (hi - lo) * unit(mix64(key + (uint64_t)(j + 1) * GOLDEN));
}

/* Standard normal by Box-Muller on pairs (u1, u2) of the stream. */
void spgen_normal(uint64_t key, int64_t len, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < len; ++j) {
    uint64_t a = mix64(key + (uint64_t)(2 * (j / 2) + 1) * GOLDEN);
    uint64_t b = mix64(key + (uint64_t)(2 * (j / 2) + 2) * GOLDEN);
    double u1 = 1.0 - unit(a); /* (0, 1] */
    double u2 = unit(b);
    double r = sqrt(-2.0 * log(u1));
    out[j] = (j & 1) ? r * sin(2.0 * M_PI * u2) : r * cos(2.0 * M_PI * u2);
  }
}

/* Small integers uniformly in [lo, hi] (exact-arithmetic inputs). */
void spgen_small_ints(uint64_t key, int64_t len, int32_t lo, int32_t hi, double *out) {
  uint64_t span = (uint64_t)(hi - lo + 1);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < len; ++j) {
    uint64_t z = mix64(key + (uint64_t)(j + 1) * GOLDEN);
    out[j] = (double)(lo + (int64_t)(((unsigned __int128)z * span) >> 64));
  }
}

/* ---- Zipf-Mandelbrot law ---------------------------------------------- */

double spgen_zm_mean(double alpha, double q, int32_t lmax) {
  double s = 0.0, sl = 0.0;
  for (int32_t L = lmax; L >= 1; --L) { /* small terms first */
    double p = pow((double)L + q, -alpha);
    s += p;
    sl += p * L;
  }
  return sl / s;
}

/* Shift q such that the mean of ZM(alpha, q) on [1, lmax] equals target.
 * The mean grows with q; bisection on [q_lo, q_hi]. Returns NAN if the target
 * is outside the reachable range. */
double spgen_zm_shift(double alpha, int32_t lmax, double target) {
  double lo = -0.999, hi = 1.0;
  if (spgen_zm_mean(alpha, lo, lmax) > target) return NAN;
  while (spgen_zm_mean(alpha, hi, lmax) < target) {
    hi *= 2.0;
    if (hi > 1e7) return NAN;
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (spgen_zm_mean(alpha, mid, lmax) < target) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

static double *zm_cdf(double alpha, double q, int32_t lmax) {
  double *cdf = (double *)malloc(sizeof(double) * (size_t)lmax);
  double s = 0.0;
  for (int32_t L = 1; L <= lmax; ++L) {
    s += pow((double)L + q, -alpha);
    cdf[L - 1] = s;
  }
  for (int32_t L = 0; L < lmax; ++L) cdf[L] /= s;
  cdf[lmax - 1] = 1.0;
  return cdf;
}

static inline int32_t zm_draw(const double *cdf, int32_t lmax, double u) {
  int32_t lo = 0, hi = lmax - 1; /* first index with cdf > u */
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (cdf[mid] > u) hi = mid; else lo = mid + 1;
  }
  return lo + 1;
}

/* len[i] for i in [0, count): one draw of ZM(alpha, q) on [1, lmax] each. */
void spgen_zm_lengths(uint64_t key, int64_t count, double alpha, double q, int32_t lmax,
                      int32_t *len) {
  double *cdf = zm_cdf(alpha, q, lmax);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i)
    len[i] = zm_draw(cdf, lmax, unit(mix64(key + (uint64_t)(i + 1) * GOLDEN)));
  free(cdf);
}

/* ---- structure generators --------------------------------------------- */

/* Floyd's algorithm (Bentley, "Programming Pearls", CACM 1987): `per_row`
 * distinct uniform columns in [0, n) for each row, in draw order. */
int spgen_uniform_rows(uint64_t key, int32_t m, int32_t n, int32_t per_row, int32_t *r,
                       int32_t *c) {
  if (per_row > n) return -1;
  int ok = 0;
#pragma omp parallel
  {
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t j = 0; j < n; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 256)
    for (int32_t i = 0; i < m; ++i) {
      uint64_t s = row_state(key, i);
      int64_t base = (int64_t)i * per_row;
      int32_t cnt = 0;
      for (int32_t j = n - per_row; j < n; ++j) {
        int32_t t = (int32_t)(((unsigned __int128)next64(&s) * (uint64_t)(j + 1)) >> 64);
        int32_t pick = (mark[t] == i) ? j : t;
        mark[pick] = i;
        r[base + cnt] = i;
        c[base + cnt] = pick;
        ++cnt;
      }
    }
    free(mark);
  }
  return ok;
}

typedef struct {
  double key;
  int32_t col;
} es_item;
static int es_cmp(const void *a, const void *b) {
  const es_item *x = (const es_item *)a, *y = (const es_item *)b;
  if (x->key > y->key) return -1;
  if (x->key < y->key) return 1;
  return (x->col < y->col) ? -1 : (x->col > y->col);
}

/* Distinct weighted columns for each row.  len[i] columns for row i (clamped
 * to n by the caller), written at off[i] (exclusive prefix of len).  wcum is
 * the inclusive prefix sum of the integer column weights (int64, length n).
 * Returns the total number of column draws made (rejections included). */
int64_t spgen_weighted_rows(uint64_t key, int32_t m, int32_t n, const int32_t *len,
                            const int64_t *off, const int64_t *wcum, const int32_t *w,
                            int32_t *r, int32_t *c) {
  int64_t total = wcum[n - 1];
  int64_t draws = 0;
#pragma omp parallel reduction(+ : draws)
  {
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t j = 0; j < n; ++j) mark[j] = -1;
    es_item *es = NULL;
#pragma omp for schedule(dynamic, 64)
    for (int32_t i = 0; i < m; ++i) {
      uint64_t s = row_state(key, i);
      int64_t base = off[i];
      int32_t L = len[i];
      if ((int64_t)L * 4 > n) {
        if (!es) es = (es_item *)malloc(sizeof(es_item) * (size_t)n);
        for (int32_t j = 0; j < n; ++j) {
          double u = 1.0 - unit(next64(&s)); /* (0, 1] */
          es[j].key = log(u) / (double)w[j];
          es[j].col = j;
        }
        draws += n;
        qsort(es, (size_t)n, sizeof(es_item), es_cmp);
        for (int32_t t = 0; t < L; ++t) {
          r[base + t] = i;
          c[base + t] = es[t].col;
        }
        continue;
      }
      int32_t cnt = 0;
      while (cnt < L) {
        int64_t t = (int64_t)(((unsigned __int128)next64(&s) * (uint64_t)total) >> 64);
        int32_t lo = 0, hi = n - 1; /* first j with wcum[j] > t */
        while (lo < hi) {
          int32_t mid = (lo + hi) >> 1;
          if (wcum[mid] > t) hi = mid; else lo = mid + 1;
        }
        ++draws;
        if (mark[lo] == i) continue;
        mark[lo] = i;
        r[base + cnt] = i;
        c[base + cnt] = lo;
        ++cnt;
      }
    }
    free(mark);
    free(es);
  }
  return draws;
}

/* 2D 5-point stencil on an nx-by-ny grid, lexicographic order (x fastest).
 * Row i = x + nx*y couples to (x,y-1), (x-1,y), (x,y), (x+1,y), (x,y+1).
 * Returns the number of triplets written (5*nx*ny - 2*(nx+ny)). */
int64_t spgen_stencil5(int32_t nx, int32_t ny, int32_t *r, int32_t *c) {
  int64_t m = (int64_t)nx * ny;
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ny + 1));
  start[0] = 0;
  for (int32_t y = 0; y < ny; ++y) {
    int64_t per = 0;
    for (int32_t x = 0; x < nx; ++x)
      per += 1 + (y > 0) + (x > 0) + (x < nx - 1) + (y < ny - 1);
    start[y + 1] = start[y] + per;
  }
#pragma omp parallel for schedule(static)
  for (int32_t y = 0; y < ny; ++y) {
    int64_t t = start[y];
    for (int32_t x = 0; x < nx; ++x) {
      int32_t i = x + nx * y;
      if (y > 0) { r[t] = i; c[t++] = i - nx; }
      if (x > 0) { r[t] = i; c[t++] = i - 1; }
      r[t] = i; c[t++] = i;
      if (x < nx - 1) { r[t] = i; c[t++] = i + 1; }
      if (y < ny - 1) { r[t] = i; c[t++] = i + nx; }
    }
  }
  int64_t tot = start[ny];
  free(start);
  (void)m;
  return tot;
}

/* 3D stencil on nx*ny*nz, lexicographic (x fastest).  pts = 7 couples each
 * point to itself and its 6 face neighbours; pts = 27 to the full 3x3x3 cube.
 * Neighbours are emitted in ascending column order. */
int64_t spgen_stencil3d(int32_t nx, int32_t ny, int32_t nz, int32_t pts, int32_t *r, int32_t *c) {
  if (pts != 7 && pts != 27) return -1;
  int64_t plane = (int64_t)nx * ny;
  /* per-z-slab offsets */
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nz + 1));
  start[0] = 0;
  for (int32_t z = 0; z < nz; ++z) {
    int64_t per = 0;
    for (int32_t y = 0; y < ny; ++y)
      for (int32_t x = 0; x < nx; ++x) {
        if (pts == 7) {
          per += 1 + (x > 0) + (x < nx - 1) + (y > 0) + (y < ny - 1) + (z > 0) + (z < nz - 1);
        } else {
          int64_t a = 1 + (x > 0) + (x < nx - 1), b = 1 + (y > 0) + (y < ny - 1),
                  d = 1 + (z > 0) + (z < nz - 1);
          per += a * b * d;
        }
      }
    start[z + 1] = start[z] + per;
  }
#pragma omp parallel for schedule(static)
  for (int32_t z = 0; z < nz; ++z) {
    int64_t t = start[z];
    for (int32_t y = 0; y < ny; ++y)
      for (int32_t x = 0; x < nx; ++x) {
        int32_t i = (int32_t)(x + (int64_t)nx * y + plane * z);
        if (pts == 7) {
          if (z > 0) { r[t] = i; c[t++] = (int32_t)(i - plane); }
          if (y > 0) { r[t] = i; c[t++] = i - nx; }
          if (x > 0) { r[t] = i; c[t++] = i - 1; }
          r[t] = i; c[t++] = i;
          if (x < nx - 1) { r[t] = i; c[t++] = i + 1; }
          if (y < ny - 1) { r[t] = i; c[t++] = i + nx; }
          if (z < nz - 1) { r[t] = i; c[t++] = (int32_t)(i + plane); }
        } else {
          for (int dz = -1; dz <= 1; ++dz) {
            if (z + dz < 0 || z + dz >= nz) continue;
            for (int dy = -1; dy <= 1; ++dy) {
              if (y + dy < 0 || y + dy >= ny) continue;
              for (int dx = -1; dx <= 1; ++dx) {
                if (x + dx < 0 || x + dx >= nx) continue;
                r[t] = i;
                c[t++] = (int32_t)(i + dx + (int64_t)nx * dy + plane * dz);
              }
            }
          }
        }
      }
  }
  int64_t tot = start[nz];
  free(start);
  return tot;
}

/* Values for triplets grouped by row: row i's values come from row stream i
 * in emission order.  kind 0: uniform [-1, 1); 1: small integers in [-8, 8];
 * 2: Laplacian (diag_value on the diagonal, -1 elsewhere). */
void spgen_values_by_row(uint64_t key, int64_t nnz, const int32_t *r, const int32_t *c,
                         int32_t kind, double diag_value, double *v) {
  /* rows are contiguous in the emission order of every structure generator */
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nnz; ++t) {
    if (kind == 2) {
      v[t] = (r[t] == c[t]) ? diag_value : -1.0;
      continue;
    }
    /* position of t inside its row: find the row start by scanning back is
     * O(L); instead derive the value from (row, column) so that it does not
     * depend on emission order within the row. */
    uint64_t z = mix64(row_state(key, r[t]) ^ ((uint64_t)(uint32_t)c[t] * GOLDEN));
    if (kind == 1) {
      v[t] = (double)((int64_t)(((unsigned __int128)z * 17u) >> 64) - 8);
    } else {
      v[t] = 2.0 * unit(z) - 1.0;
    }
  }
}
