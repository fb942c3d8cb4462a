/*
 * CPU ORACLE, part 3: triad census by wedge/triangle decomposition.
 * TEST INFRASTRUCTURE ONLY. A second exact algorithm, used to cross-check the
 * sweep on graphs too large for the brute force; it shares no step with the
 * sweep's edge-by-edge merge.
 *
 * Every connected triad has either exactly two adjacent vertex pairs (an open
 * wedge, owned by the one vertex adjacent to both others) or three (a
 * triangle). So:
 *  1. At every centre x with o_x out-only, i_x in-only and m_x mutual
 *     neighbours, the wedges of each kind are C(o,2) [021D], C(i,2) [021U],
 *     o*i [021C], m*o [111U], m*i [111D] and C(m,2) [201].
 *  2. Triangles are listed once each (degree-ordered orientation); each is
 *     classified directly and its three closed wedges are removed from the
 *     wedge totals of step 1.
 *  3. 012 and 102 follow from dyad bookkeeping: every asymmetric (mutual)
 *     vertex pair lies in exactly n-2 triads, so
 *     sum_t A_t * count_t = A_tot * (n-2) and sum_t M_t * count_t = M_tot * (n-2),
 *     with A_t, M_t the asymmetric / mutual dyads of class t.
 *  4. 003 = C(n,3) minus the rest (128-bit).
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum { T003, T012, T102, T021D, T021U, T021C, T111D, T111U, T030T, T030C, T201, T120D, T120U, T120C, T210, T300 };

int oracle_brute_classify(int sab, int sac, int sbc); /* brute.c */
void oracle_choose3(int64_t n, uint64_t *lo, uint64_t *hi);

static inline unsigned flag_at(const uint8_t *flg, int64_t j) { return (flg[j >> 2] >> (2 * (j & 3))) & 3u; }
static inline int swap_dir(int s) { return ((s & 1) << 1) | ((s >> 1) & 1); }

/* wedge kind at a centre whose two arms have states s1, s2 (seen from the centre) */
static int wedge_kind(int s1, int s2) {
  if (s1 > s2) { int t = s1; s1 = s2; s2 = t; }
  if (s1 == 1 && s2 == 1) return T021D;
  if (s1 == 2 && s2 == 2) return T021U;
  if (s1 == 1 && s2 == 2) return T021C;
  if (s1 == 1 && s2 == 3) return T111U;
  if (s1 == 2 && s2 == 3) return T111D;
  return T201; /* 3,3 */
}

typedef struct {
  const int64_t *hoff;
  const int32_t *hnb;
  const uint8_t *hst;
  int64_t n;
  atomic_llong next;
  int64_t part[64][16]; /* [T021D..T201] closed wedges; triangle classes */
} tri_ctx;
typedef struct { tri_ctx *c; int t; } tri_arg;

static void *tri_worker(void *p) {
  tri_arg *a = (tri_arg *)p;
  tri_ctx *c = a->c;
  int64_t *part = c->part[a->t];
  for (;;) {
    long long x0 = atomic_fetch_add(&c->next, 64);
    if (x0 >= c->n) break;
    long long x1 = x0 + 64 < c->n ? x0 + 64 : c->n;
    for (int64_t x = x0; x < x1; ++x) {
      for (int64_t k = c->hoff[x]; k < c->hoff[x + 1]; ++k) {
        int64_t y = c->hnb[k];
        int sxy = c->hst[k];
        int64_t p1 = c->hoff[x], e1 = c->hoff[x + 1], p2 = c->hoff[y], e2 = c->hoff[y + 1];
        while (p1 < e1 && p2 < e2) {
          int32_t z1 = c->hnb[p1], z2 = c->hnb[p2];
          if (z1 < z2) ++p1;
          else if (z2 < z1) ++p2;
          else {
            int sxz = c->hst[p1], syz = c->hst[p2];
            int t = oracle_brute_classify(sxy, sxz, syz);
            part[t] += 1; /* triangle class (never a wedge class) */
            /* closed wedges at x, y, z are stored negated in the wedge slots */
            part[wedge_kind(sxy, sxz)] -= 1;
            part[wedge_kind(swap_dir(sxy), syz)] -= 1;
            part[wedge_kind(swap_dir(sxz), swap_dir(syz))] -= 1;
            ++p1; ++p2;
          }
        }
      }
    }
  }
  return NULL;
}

int oracle_wedge_census(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg, int nthreads,
                        uint64_t out[16], uint64_t *hi003) {
  memset(out, 0, 16 * sizeof(uint64_t));
  if (hi003) *hi003 = 0;
  if (n < 3) return 0;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  /* step 1: open + closed wedges by kind, and the dyad totals */
  int64_t W[16] = {0};
  int64_t Mtot2 = 0, Atot2 = 0; /* each pair seen from both ends */
  for (int64_t x = 0; x < n; ++x) {
    int64_t o = 0, i = 0, m = 0;
    for (int64_t j = off[x]; j < off[x + 1]; ++j) {
      unsigned f = flag_at(flg, j);
      if (f == 1) ++o; else if (f == 2) ++i; else ++m;
    }
    W[T021D] += o * (o - 1) / 2;
    W[T021U] += i * (i - 1) / 2;
    W[T021C] += o * i;
    W[T111U] += m * o;
    W[T111D] += m * i;
    W[T201] += m * (m - 1) / 2;
    Mtot2 += m;
    Atot2 += o + i;
  }
  /* step 2: orientation by (degree, id); H(x) = higher-ranked neighbours */
  int64_t *hoff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t x = 0; x < n; ++x) {
    int64_t dx = off[x + 1] - off[x], h = 0;
    for (int64_t j = off[x]; j < off[x + 1]; ++j) {
      int64_t y = nbr[j], dy = off[y + 1] - off[y];
      if (dy > dx || (dy == dx && y > x)) ++h;
    }
    hoff[x + 1] = hoff[x] + h;
  }
  int32_t *hnb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(hoff[n] ? hoff[n] : 1));
  uint8_t *hst = (uint8_t *)malloc((size_t)(hoff[n] ? hoff[n] : 1));
  for (int64_t x = 0; x < n; ++x) {
    int64_t dx = off[x + 1] - off[x], w = hoff[x];
    for (int64_t j = off[x]; j < off[x + 1]; ++j) {
      int64_t y = nbr[j], dy = off[y + 1] - off[y];
      if (dy > dx || (dy == dx && y > x)) { hnb[w] = (int32_t)y; hst[w] = (uint8_t)flag_at(flg, j); ++w; }
    }
  }
  tri_ctx *c = (tri_ctx *)calloc(1, sizeof(tri_ctx));
  c->hoff = hoff; c->hnb = hnb; c->hst = hst; c->n = n;
  atomic_init(&c->next, 0);
  pthread_t th[64];
  tri_arg args[64];
  for (int t = 0; t < nthreads; ++t) { args[t].c = c; args[t].t = t; }
  if (nthreads == 1) {
    tri_worker(&args[0]);
  } else {
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, tri_worker, &args[t]);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  }
  int64_t acc[16] = {0};
  for (int t = 0; t < nthreads; ++t)
    for (int k = 0; k < 16; ++k) acc[k] += c->part[t][k];
  free(c); free(hoff); free(hnb); free(hst);
  /* open wedges = all wedges - closed wedges (acc holds -closed in wedge slots) */
  const int wk[6] = {T021D, T021U, T021C, T111D, T111U, T201};
  for (int k = 0; k < 6; ++k) out[wk[k]] = (uint64_t)(W[wk[k]] + acc[wk[k]]);
  const int tk[7] = {T030T, T030C, T120D, T120U, T120C, T210, T300};
  for (int k = 0; k < 7; ++k) out[tk[k]] = (uint64_t)acc[tk[k]];
  /* step 3: dyad bookkeeping. Per-class (M, A) dyad counts follow from the
   * class definitions. */
  static const int Mt[16] = {0, 0, 1, 0, 0, 0, 1, 1, 0, 0, 2, 1, 1, 1, 2, 3};
  static const int At[16] = {0, 1, 0, 2, 2, 2, 1, 1, 3, 3, 0, 2, 2, 2, 1, 0};
  u128 Aside = (u128)(uint64_t)(Atot2 / 2) * (uint64_t)(n - 2);
  u128 Mside = (u128)(uint64_t)(Mtot2 / 2) * (uint64_t)(n - 2);
  for (int t = 3; t < 16; ++t) {
    Aside -= (u128)At[t] * out[t];
    Mside -= (u128)Mt[t] * out[t];
  }
  out[T012] = (uint64_t)Aside;
  out[T102] = (uint64_t)Mside;
  /* step 4 */
  uint64_t clo, chi;
  oracle_choose3(n, &clo, &chi);
  u128 s = 0;
  for (int t = 1; t < 16; ++t) s += out[t];
  u128 nul = (((u128)chi << 64) | clo) - s;
  out[T003] = (uint64_t)nul;
  if (hi003) *hi003 = (uint64_t)(nul >> 64);
  return (nul >> 64) != 0;
}
