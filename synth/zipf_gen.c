/* Power-law CSR generator (input synthesis only; no part of the method).
 *
 * Given row degrees deg[0..m) (already capped at n and summing to nnz) and the
 * cumulative column law cdf[0..n) with cdf[n-1] = 1, each row r draws deg[r]
 * distinct columns with probability proportional to the column weights
 * (weighted sampling without replacement), sorted ascending, and values
 * 1 - U[0,1) rounded to FP32.  Each row has its own splitmix64 stream derived
 * from (seed, r), so the output does not depend on the thread count.
 *   - deg[r] == n          : every column.
 *   - 16 * deg[r] > n      : Efraimidis-Spirakis: key_j = log(-log u_j) -
 *                            log w_j, keep the deg[r] smallest keys.
 *   - otherwise            : draw from the column law by binary search on the
 *                            cdf, reject repeats (open-addressing set).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t sm64(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline double u01(uint64_t *s) { return (double)(sm64(s) >> 11) * 0x1.0p-53; }

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

typedef struct { double key; int32_t idx; } kv;

/* quickselect: move the d smallest keys to the front */
static void select_smallest(kv *a, int64_t n, int64_t d, uint64_t *rng) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    int64_t p = lo + (int64_t)(sm64(rng) % (uint64_t)(hi - lo + 1));
    double pv = a[p].key;
    kv t = a[p]; a[p] = a[hi]; a[hi] = t;
    int64_t st = lo;
    for (int64_t i = lo; i < hi; ++i) {
      if (a[i].key < pv) { t = a[i]; a[i] = a[st]; a[st] = t; ++st; }
    }
    t = a[st]; a[st] = a[hi]; a[hi] = t;
    if (st == d - 1 || st == d) return;
    if (st < d) lo = st + 1; else hi = st - 1;
  }
}

void zipf_fill(int64_t m, int64_t n, const int64_t *row_ptr, const double *cdf,
               const double *logw, uint64_t seed, int32_t *col, float *val) {
#pragma omp parallel
  {
    kv *keys = NULL;
    int32_t *table = NULL;
    int64_t table_cap = 0;
#pragma omp for schedule(dynamic, 256)
    for (int64_t r = 0; r < m; ++r) {
      const int64_t b = row_ptr[r], d = row_ptr[r + 1] - row_ptr[r];
      uint64_t st = seed * 0xD1342543DE82EF95ULL + (uint64_t)r * 0x9E3779B97F4A7C15ULL + 1;
      sm64(&st);
      int32_t *out = col + b;
      if (d == 0) continue;
      if (d >= n) {
        for (int64_t j = 0; j < n; ++j) out[j] = (int32_t)j;
      } else if (16 * d > n) {
        if (!keys) keys = (kv *)malloc(sizeof(kv) * (size_t)n);
        for (int64_t j = 0; j < n; ++j) {
          double u = u01(&st);
          keys[j].key = log(-log(u + 1e-300)) - logw[j];
          keys[j].idx = (int32_t)j;
        }
        select_smallest(keys, n, d, &st);
        for (int64_t j = 0; j < d; ++j) out[j] = keys[j].idx;
      } else {
        int64_t cap = 16;
        while (cap < 2 * d) cap <<= 1;
        if (cap > table_cap) {
          free(table);
          table = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
          table_cap = cap;
        }
        for (int64_t j = 0; j < cap; ++j) table[j] = -1;
        int64_t got = 0;
        while (got < d) {
          double u = u01(&st);
          int64_t lo = 0, hi = n - 1;
          while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (cdf[mid] > u) hi = mid; else lo = mid + 1;
          }
          uint64_t h = ((uint64_t)lo * 0x9E3779B97F4A7C15ULL) >> 7;
          int64_t slot = (int64_t)(h & (uint64_t)(cap - 1));
          int dup = 0;
          while (table[slot] >= 0) {
            if (table[slot] == (int32_t)lo) { dup = 1; break; }
            slot = (slot + 1) & (cap - 1);
          }
          if (dup) continue;
          table[slot] = (int32_t)lo;
          out[got++] = (int32_t)lo;
        }
      }
      qsort(out, (size_t)d, sizeof(int32_t), cmp_i32);
      for (int64_t j = 0; j < d; ++j) val[b + j] = (float)(1.0 - u01(&st));
    }
    free(keys);
    free(table);
  }
}
