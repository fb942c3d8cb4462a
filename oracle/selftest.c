/*
 * CPU ORACLE, part 4: exhaustive self-checks. TEST INFRASTRUCTURE ONLY.
 *
 * Enumerates every labelled simple digraph on n vertices (2^(n(n-1)) of them:
 * 4,096 for n = 4, 1,048,576 for n = 5), builds its symmetric CSR with a tiny
 * builder of its own, and compares the sweep (census_oracle.c) and the
 * wedge/triangle decomposition (wedge.c) with the brute force (brute.c), which
 * reads the arc list directly.
 */
#include <stdint.h>
#include <string.h>

int oracle_census(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg, uint64_t out[16],
                  uint64_t *hi003);
int oracle_brute(int64_t n, int64_t narcs, const int32_t *src, const int32_t *dst, uint64_t out[16],
                 uint64_t *hi003);
int oracle_wedge_census(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg, int nthreads,
                        uint64_t out[16], uint64_t *hi003);

/* mism[0] = sweep vs brute mismatches, mism[1] = wedge vs brute mismatches.
 * Returns the number of graphs checked, or -1 if n is out of range. */
int64_t oracle_exhaustive(int n, int64_t mism[2]) {
  if (n < 1 || n > 5) return -1;
  int pa[20], pb[20], np = 0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      if (a != b) { pa[np] = a; pb[np] = b; ++np; }
  mism[0] = mism[1] = 0;
  const int64_t total = (int64_t)1 << np;
  for (int64_t mask = 0; mask < total; ++mask) {
    int32_t src[20], dst[20];
    int na = 0;
    uint8_t st[5][5];
    memset(st, 0, sizeof st);
    for (int k = 0; k < np; ++k)
      if ((mask >> k) & 1) {
        src[na] = pa[k]; dst[na] = pb[k]; ++na;
        st[pa[k]][pb[k]] |= 1;
        st[pb[k]][pa[k]] |= 2;
      }
    int64_t off[6] = {0};
    int32_t nbr[20];
    uint8_t flg[5];
    memset(flg, 0, sizeof flg);
    int e = 0;
    for (int x = 0; x < n; ++x) {
      for (int y = 0; y < n; ++y)
        if (st[x][y]) {
          nbr[e] = y;
          flg[e >> 2] |= (uint8_t)(st[x][y] << (2 * (e & 3)));
          ++e;
        }
      off[x + 1] = e;
    }
    uint64_t a[16], b[16], c[16], h;
    oracle_census(n, off, nbr, flg, a, &h);
    oracle_brute(n, na, src, dst, b, &h);
    oracle_wedge_census(n, off, nbr, flg, 1, c, &h);
    if (memcmp(a, b, sizeof a)) ++mism[0];
    if (memcmp(c, b, sizeof c)) ++mism[1];
  }
  return total;
}
