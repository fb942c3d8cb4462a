/*
 * CPU ORACLE, part 4: the 64-state labelled triad census. TEST
 * INFRASTRUCTURE ONLY (same rules as census_oracle.c: only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it; it shares
 * nothing with the HIP library).
 *
 * What it computes: Sec. 3 of the paper describes a triad by 64 states (the
 * six possible arcs among three vertices) before they are condensed into the
 * 16 isomorphism classes. With the vertices of a triple named by id order,
 * a < b < c, its state is
 *     f_ab | f_ac << 2 | f_bc << 4,
 * f_xy being the direction flag of y in row x (bit0 = x->y, bit1 = y->x, 0
 * for no arc). The labelled census counts the triples in each state; state 0
 * (no arc) is C(n,3) minus the rest, in 128 bits. Condensing the states by
 * the isomorphism class of their code gives the 16-class census.
 *
 * How: the same edge sweep as census_oracle.c (Fig. 5), over every edge
 * {u, v}, u < v, with the two-pointer union walk of Fig. 8, the third vertex
 * w placed by id order:
 *  - v < w: the triple is (u, v, w), state f_uv | f_uw << 2 | f_vw << 4;
 *  - u < w < v and w not adjacent to u: the triple is (u, w, v), state
 *    f_uw | f_uv << 2 | f_wv << 4 with f_uw = 0 and f_wv the mirror of f_vw;
 *  - any other w is owned by another edge (the canonical rule of step 2.1.4).
 * The dyadic triads of step 2.1.3 (only the pair u-v has arcs) are split by
 * where the third vertex lies: below u the triple is (w, u, v) and its state
 * f_uv << 4, between u and v it is (u, w, v) and f_uv << 2, above v it is
 * (u, v, w) and f_uv. Their counts are the ids of each range minus the
 * members of N(u) u N(v) \ {u, v} in it, counted during the walk.
 */
#include <stdint.h>
#include <string.h>

typedef unsigned __int128 u128;

static inline unsigned flag_at(const uint8_t *flg, int64_t j) { return (flg[j >> 2] >> (2 * (j & 3))) & 3u; }
static inline unsigned mirror(unsigned f) { return ((f & 1u) << 1) | (f >> 1); }

static void labelled_task(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg, int64_t u, int64_t j,
                          uint64_t out[64]) {
  const int64_t v = nbr[j];
  const unsigned fuv = flag_at(flg, j);
  int64_t p = off[u], pe = off[u + 1], q = off[v], qe = off[v + 1];
  int64_t below = 0, between = 0, above = 0; /* |N(u) u N(v) \ {u,v}| per range */
  while (p < pe || q < qe) {
    int64_t wu = p < pe ? nbr[p] : INT64_MAX;
    int64_t wv = q < qe ? nbr[q] : INT64_MAX;
    int64_t w;
    unsigned fuw = 0, fvw = 0;
    if (wu < wv) { w = wu; fuw = flag_at(flg, p); ++p; }
    else if (wv < wu) { w = wv; fvw = flag_at(flg, q); ++q; }
    else { w = wu; fuw = flag_at(flg, p); fvw = flag_at(flg, q); ++p; ++q; }
    if (w == u || w == v) continue;
    if (w < u) ++below;
    else if (w < v) ++between;
    else ++above;
    if (v < w) out[fuv | fuw << 2 | fvw << 4] += 1;
    else if (u < w && fuw == 0) out[fuv << 2 | mirror(fvw) << 4] += 1;
  }
  out[fuv << 4] += (uint64_t)(u - below);
  out[fuv << 2] += (uint64_t)(v - u - 1 - between);
  out[fuv] += (uint64_t)(n - 1 - v - above);
}

/* Returns 1 if state 0 needs a high word (stored in *hi0), else 0. */
int oracle_labelled_census(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg, uint64_t out[64],
                           uint64_t *hi0) {
  memset(out, 0, 64 * sizeof(uint64_t));
  if (hi0) *hi0 = 0;
  if (n < 3) return 0;
  for (int64_t u = 0; u < n; ++u)
    for (int64_t j = off[u]; j < off[u + 1]; ++j)
      if (nbr[j] > u) labelled_task(n, off, nbr, flg, u, j, out);
  u128 total = n >= 3 ? (u128)(uint64_t)n * (u128)(uint64_t)(n - 1) * (u128)(uint64_t)(n - 2) / 6 : 0, s = 0;
  for (int k = 1; k < 64; ++k) s += out[k];
  u128 nul = total - s;
  out[0] = (uint64_t)nul;
  if (hi0) *hi0 = (uint64_t)(nul >> 64);
  return (nul >> 64) != 0;
}
