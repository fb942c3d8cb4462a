/*
 * Sanitizer driver for the CPU oracle (built with -fsanitize=address,undefined
 * and, separately, -fsanitize=thread by tests/test_sanitizers.py).
 *
 * Seeded random digraphs, each put into the compact CSR with direction bits by
 * a small builder of this file's own; every oracle entry point runs on them and
 * the exact algorithms must agree: the sweep single- and multi-threaded, the
 * partial-task driver, the wedge/triangle decomposition and the brute force
 * (16 classes), and the labelled sweep against its brute force (64 states).
 * Also every labelled digraph on 4 vertices (oracle_exhaustive).
 * Exit status: the number of disagreements (0 = all agree).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_census(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg, uint64_t out[16],
                  uint64_t *hi003);
int oracle_census_mt(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg, int nthreads,
                     uint64_t out[16], uint64_t *hi003);
void oracle_census_tasks_mt(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg,
                            int64_t ntasks, const int64_t *tasks, int nthreads, uint64_t out[16]);
int oracle_wedge_census(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg, int nthreads,
                        uint64_t out[16], uint64_t *hi003);
int oracle_brute(int64_t n, int64_t narcs, const int32_t *src, const int32_t *dst, uint64_t out[16],
                 uint64_t *hi003);
int oracle_labelled_census(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg, uint64_t out[64],
                           uint64_t *hi);
int oracle_brute64(int64_t n, int64_t narcs, const int32_t *src, const int32_t *dst, uint64_t out[64],
                   uint64_t *hi);
int64_t oracle_exhaustive(int n, int64_t mism[2]);
void oracle_choose3(int64_t n, uint64_t *lo, uint64_t *hi);

static uint64_t sm_state;
static uint64_t splitmix64(void) { /* Steele, Lea, Flood: SplitMix64 */
  uint64_t z = (sm_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

typedef struct { int32_t row, col; uint8_t f; } ent;

static int by_row_col(const void *a, const void *b) {
  const ent *x = a, *y = b;
  if (x->row != y->row) return x->row < y->row ? -1 : 1;
  if (x->col != y->col) return x->col < y->col ? -1 : 1;
  return 0;
}

/* CSR of the arcs (no self-loops): both directions of every pair, flags OR-ed. */
static int64_t build(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int64_t **off, int32_t **nbr,
                     uint8_t **flg) {
  ent *e = malloc(sizeof(ent) * (size_t)(2 * m + 1));
  for (int64_t i = 0; i < m; ++i) {
    e[2 * i] = (ent){src[i], dst[i], 1};
    e[2 * i + 1] = (ent){dst[i], src[i], 2};
  }
  qsort(e, (size_t)(2 * m), sizeof(ent), by_row_col);
  int64_t k = 0;
  for (int64_t i = 0; i < 2 * m; ++i) {
    if (k > 0 && e[k - 1].row == e[i].row && e[k - 1].col == e[i].col) e[k - 1].f |= e[i].f;
    else e[k++] = e[i];
  }
  *off = calloc((size_t)n + 1, sizeof(int64_t));
  *nbr = malloc(sizeof(int32_t) * (size_t)(k + 1));
  *flg = calloc((size_t)(k + 3) / 4 + 1, 1);
  for (int64_t i = 0; i < k; ++i) {
    (*off)[e[i].row + 1]++;
    (*nbr)[i] = e[i].col;
    (*flg)[i >> 2] |= (uint8_t)(e[i].f << (2 * (i & 3)));
  }
  for (int64_t x = 0; x < n; ++x) (*off)[x + 1] += (*off)[x];
  free(e);
  return k;
}

static int same(const uint64_t *a, const uint64_t *b, int len, const char *what, int64_t n) {
  if (memcmp(a, b, sizeof(uint64_t) * (size_t)len) == 0) return 0;
  fprintf(stderr, "mismatch: %s (n = %lld)\n", what, (long long)n);
  return 1;
}

int main(void) {
  int bad = 0;
  const int64_t ns[] = {3, 5, 37, 200, 700};
  const double dens[] = {1.0, 0.6, 0.3, 0.05, 0.01};
  sm_state = 12345;
  for (int c = 0; c < 5; ++c) {
    const int64_t n = ns[c];
    const int64_t m = (int64_t)(dens[c] * (double)(n * (n - 1)) / 2) + 1;
    int32_t *src = malloc(sizeof(int32_t) * (size_t)m), *dst = malloc(sizeof(int32_t) * (size_t)m);
    int64_t k = 0;
    for (int64_t i = 0; i < m; ++i) {
      int32_t a = (int32_t)(splitmix64() % (uint64_t)n), b = (int32_t)(splitmix64() % (uint64_t)n);
      if (a == b) continue;
      src[k] = a;
      dst[k] = b;
      ++k;
    }
    int64_t *off;
    int32_t *nbr;
    uint8_t *flg;
    const int64_t nnz = build(n, k, src, dst, &off, &nbr, &flg);
    uint64_t ref[16], x[16], h0 = 0, h1 = 0;
    oracle_brute(n, k, src, dst, ref, &h0);
    oracle_census(n, off, nbr, flg, x, &h1);
    bad += same(ref, x, 16, "sweep vs brute", n);
    oracle_census_mt(n, off, nbr, flg, 4, x, &h1);
    bad += same(ref, x, 16, "threaded sweep vs brute", n);
    oracle_wedge_census(n, off, nbr, flg, 4, x, &h1);
    bad += same(ref, x, 16, "wedge vs brute", n);
    /* every task, split over threads: counts 1..15 equal the full census */
    int64_t *tasks = malloc(sizeof(int64_t) * (size_t)(nnz + 1)), nt = 0;
    for (int64_t r = 0; r < n; ++r)
      for (int64_t j = off[r]; j < off[r + 1]; ++j)
        if (nbr[j] > r) tasks[nt++] = j;
    memset(x, 0, sizeof x);
    oracle_census_tasks_mt(n, off, nbr, flg, nt, tasks, 4, x);
    if (n >= 3) bad += same(ref + 1, x + 1, 15, "task driver vs brute", n);
    uint64_t l64[64], b64[64];
    oracle_labelled_census(n, off, nbr, flg, l64, &h0);
    oracle_brute64(n, k, src, dst, b64, &h1);
    bad += same(b64, l64, 64, "labelled sweep vs brute", n);
    free(tasks);
    free(off);
    free(nbr);
    free(flg);
    free(src);
    free(dst);
  }
  int64_t mism[2];
  if (oracle_exhaustive(4, mism) != 4096 || mism[0] || mism[1]) {
    fprintf(stderr, "exhaustive n = 4: mismatches %lld %lld\n", (long long)mism[0], (long long)mism[1]);
    ++bad;
  }
  uint64_t lo, hi;
  oracle_choose3(4801281, &lo, &hi);
  if (hi != 1) ++bad;
  printf("oracle driver: %d disagreement(s)\n", bad);
  return bad;
}
