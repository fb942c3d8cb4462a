/*
 * CPU ORACLE, part 2: O(n^3) brute-force triad census. TEST INFRASTRUCTURE ONLY.
 *
 * This is the plain definition of the census (Sec. 3 of the paper: count, for
 * every 3-subset of vertices, the isomorphism class of the induced subgraph),
 * evaluated by visiting every triple, the naive algorithm named in Sec. 4.
 * It reads the raw arc list, never the CSR, and classifies each triple by an
 * isomorphism invariant that is independent of the code table used by the
 * sweep: the number of mutual (M) and asymmetric (A) dyads together with the
 * sorted out-degree and in-degree sequences inside the triad. These
 * signatures separate all 16 classes:
 *   021D out (2,0,0)   021U in (2,0,0)   021C otherwise
 *   111D in  (2,1,0)   111U out (2,1,0)
 *   030T out contains a 2                030C otherwise
 *   120D in  (2,2,0)   120U out (2,2,0)   120C otherwise
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum { T003, T012, T102, T021D, T021U, T021C, T111D, T111U, T030T, T030C, T201, T120D, T120U, T120C, T210, T300 };

/* pair state of (a,b): 0 none, 1 a->b only, 2 b->a only, 3 mutual */
static int classify_signature(int sab, int sac, int sbc) {
  int arc[3][3] = {{0}};
  arc[0][1] = sab & 1; arc[1][0] = (sab >> 1) & 1;
  arc[0][2] = sac & 1; arc[2][0] = (sac >> 1) & 1;
  arc[1][2] = sbc & 1; arc[2][1] = (sbc >> 1) & 1;
  int M = (sab == 3) + (sac == 3) + (sbc == 3);
  int A = (sab == 1 || sab == 2) + (sac == 1 || sac == 2) + (sbc == 1 || sbc == 2);
  int od[3] = {0, 0, 0}, id[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (arc[i][j]) { od[i]++; id[j]++; }
  /* sort descending */
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j) {
      if (od[j] > od[i]) { int t = od[i]; od[i] = od[j]; od[j] = t; }
      if (id[j] > id[i]) { int t = id[i]; id[i] = id[j]; id[j] = t; }
    }
  switch (M * 4 + A) {
    case 0: return T003;
    case 1: return T012;
    case 4: return T102;
    case 2:
      if (od[0] == 2 && od[1] == 0) return T021D;
      if (id[0] == 2 && id[1] == 0) return T021U;
      return T021C;
    case 5:
      if (id[0] == 2 && id[1] == 1 && id[2] == 0) return T111D;
      if (od[0] == 2 && od[1] == 1 && od[2] == 0) return T111U;
      return -1;
    case 3: return (od[0] == 2) ? T030T : T030C;
    case 8: return T201;
    case 6:
      if (id[0] == 2 && id[1] == 2 && id[2] == 0) return T120D;
      if (od[0] == 2 && od[1] == 2 && od[2] == 0) return T120U;
      return T120C;
    case 9: return T210;
    case 12: return T300;
  }
  return -1;
}

/* exported for the test suite: the class of a triad given its three pair
 * states (same encoding as above) */
int oracle_brute_classify(int sab, int sac, int sbc) { return classify_signature(sab, sac, sbc); }

/* Census of the digraph with vertices 0..n-1 and the given arcs (duplicates
 * and self-loops ignored). Every triple a<b<c is visited. Returns 1 if the
 * 003 count needs a high word (stored in *hi003). */
int oracle_brute(int64_t n, int64_t narcs, const int32_t *src, const int32_t *dst, uint64_t out[16],
                 uint64_t *hi003) {
  memset(out, 0, 16 * sizeof(uint64_t));
  if (hi003) *hi003 = 0;
  if (n < 3) return 0;
  uint8_t *st = (uint8_t *)calloc((size_t)n * (size_t)n, 1);
  if (!st) return -1;
  for (int64_t i = 0; i < narcs; ++i) {
    int64_t a = src[i], b = dst[i];
    if (a == b) continue;
    st[a * n + b] |= 1; /* a->b seen from a */
    st[b * n + a] |= 2; /* a->b seen from b */
  }
  int8_t memo[64];
  for (int k = 0; k < 64; ++k) memo[k] = (int8_t)classify_signature(k & 3, (k >> 2) & 3, (k >> 4) & 3);
  u128 c003 = 0;
  for (int64_t a = 0; a < n; ++a) {
    const uint8_t *ra = st + a * n;
    for (int64_t b = a + 1; b < n; ++b) {
      const uint8_t *rb = st + b * n;
      int sab = ra[b];
      for (int64_t c = b + 1; c < n; ++c) {
        int t = memo[sab | ra[c] << 2 | rb[c] << 4];
        if (t == T003) ++c003; else out[t]++;
      }
    }
  }
  free(st);
  out[T003] = (uint64_t)c003;
  if (hi003) *hi003 = (uint64_t)(c003 >> 64);
  return (c003 >> 64) != 0;
}

/* The 64-state labelled census by its definition: for every triple a < b < c
 * of vertex ids, the state f_ab | f_ac << 2 | f_bc << 4 of its three pairs
 * (f_xy: bit0 = arc x->y, bit1 = arc y->x, 0 = no arc), counted per state.
 * Sec. 3 of the paper: the 64 states of a labelled triad before they are
 * condensed into 16 isomorphism classes. out[0] (no arc) is returned mod 2^64
 * with its high word in *hi0. */
int oracle_brute64(int64_t n, int64_t narcs, const int32_t *src, const int32_t *dst, uint64_t out[64],
                   uint64_t *hi0) {
  memset(out, 0, 64 * sizeof(uint64_t));
  if (hi0) *hi0 = 0;
  if (n < 3) return 0;
  uint8_t *st = (uint8_t *)calloc((size_t)n * (size_t)n, 1);
  if (!st) return -1;
  for (int64_t i = 0; i < narcs; ++i) {
    int64_t a = src[i], b = dst[i];
    if (a == b) continue;
    st[a * n + b] |= 1;
    st[b * n + a] |= 2;
  }
  u128 c0 = 0;
  for (int64_t a = 0; a < n; ++a) {
    const uint8_t *ra = st + a * n;
    for (int64_t b = a + 1; b < n; ++b) {
      const uint8_t *rb = st + b * n;
      int sab = ra[b];
      for (int64_t c = b + 1; c < n; ++c) {
        int s = sab | ra[c] << 2 | rb[c] << 4;
        if (s == 0) ++c0; else out[s]++;
      }
    }
  }
  free(st);
  out[0] = (uint64_t)c0;
  if (hi0) *hi0 = (uint64_t)(c0 >> 64);
  return (c0 >> 64) != 0;
}
