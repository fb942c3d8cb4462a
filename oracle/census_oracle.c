/*
 * CPU ORACLE for the directed triad census. TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. The product path (the HIP census library) never
 * links, loads or calls it, and shares no code, header or table with it.
 *
 * What it computes: the 16-type triad census of a simple digraph, in the
 * standard order 003, 012, 102, 021D, 021U, 021C, 111D, 111U, 030T, 030C,
 * 201, 120D, 120U, 120C, 210, 300 (Sec. 3 of the paper: 64 triad states
 * condensed to 16 isomorphism classes).
 *
 * How: the Batagelj-Mrvar edge sweep of Fig. 5, single-threaded, with the
 * union S = N(u) u N(v) walked by the two-pointer traversal of Sec. 6 /
 * Fig. 8 and the triad code read in situ from the direction bits (Sec. 6).
 *
 * Readings where the paper is silent or garbled (each pinned by tests):
 *  - S excludes u and v, so the dyadic count of step 2.1.3 is
 *    n - |S| - 2 = n - |N(u) u N(v)| (u and v lie in each other's lists).
 *  - uAv means the arc u->v; uÂv means u and v are neighbours (either arc).
 *  - Direction flag of entry y in row x: bit0 = x->y, bit1 = y->x.
 *  - Triad code: bit0 u->v, bit1 v->u, bit2 u->w, bit3 w->u, bit4 v->w,
 *    bit5 w->v, i.e. code = f_uv | f_uw << 2 | f_vw << 4.
 *  - 111D = A<->B<-C (the asymmetric arc points into the mutual dyad),
 *    111U = A<->B->C.
 *  - The null count of step 5 is C(n,3) minus the rest, in 128-bit integers
 *    (C(n,3) exceeds 2^64 from n = 4,801,281).
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum { T003, T012, T102, T021D, T021U, T021C, T111D, T111U, T030T, T030C, T201, T120D, T120U, T120C, T210, T300 };

static inline unsigned flag_at(const uint8_t *flg, int64_t j) { return (flg[j >> 2] >> (2 * (j & 3))) & 3u; }

/* ------------------------------------------------------------------------
 * IsoTricode table (step 2.1.4.1 of Fig. 5), generated from the definition
 * of each isomorphism class by the M/A/N dyad census of the triad plus the
 * role of the distinguished vertex ("MAN" naming of Holland and Leinhardt).
 * Vertices: 0 = u, 1 = v, 2 = w.
 * ---------------------------------------------------------------------- */
static int classify_code(unsigned code) {
  int arc[3][3] = {{0}};
  arc[0][1] = (code >> 0) & 1; arc[1][0] = (code >> 1) & 1;
  arc[0][2] = (code >> 2) & 1; arc[2][0] = (code >> 3) & 1;
  arc[1][2] = (code >> 4) & 1; arc[2][1] = (code >> 5) & 1;
  int M = 0, A = 0;
  int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int k = 0; k < 3; ++k) {
    int x = arc[pa[k]][pb[k]], y = arc[pb[k]][pa[k]];
    if (x && y) ++M; else if (x || y) ++A;
  }
  int outd[3], ind[3];
  for (int i = 0; i < 3; ++i) {
    outd[i] = ind[i] = 0;
    for (int j = 0; j < 3; ++j) if (i != j) { outd[i] += arc[i][j]; ind[i] += arc[j][i]; }
  }
  if (M == 0 && A == 0) return T003;
  if (M == 0 && A == 1) return T012;
  if (M == 1 && A == 0) return T102;
  if (M == 2 && A == 0) return T201;
  if (M == 2 && A == 1) return T210;
  if (M == 3) return T300;
  if (M == 0 && A == 2) {
    /* the vertex incident to both arcs */
    for (int c = 0; c < 3; ++c) {
      int a = (c + 1) % 3, b = (c + 2) % 3;
      int ca = arc[c][a] || arc[a][c], cb = arc[c][b] || arc[b][c];
      if (ca && cb) {
        if (arc[c][a] && arc[c][b]) return T021D; /* centre sends both */
        if (arc[a][c] && arc[b][c]) return T021U; /* centre receives both */
        return T021C;
      }
    }
  }
  if (M == 1 && A == 1) {
    /* find the asymmetric arc x->y; D if y belongs to the mutual dyad */
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y)
        if (x != y && arc[x][y] && !arc[y][x]) {
          int z = 3 - x - y; /* the remaining vertex */
          int y_mut = arc[y][z] && arc[z][y];
          return y_mut ? T111D : T111U;
        }
  }
  if (M == 0 && A == 3) {
    for (int i = 0; i < 3; ++i) if (outd[i] == 2) return T030T;
    return T030C;
  }
  if (M == 1 && A == 2) {
    /* z = the vertex outside the mutual dyad */
    for (int z = 0; z < 3; ++z) {
      int a = (z + 1) % 3, b = (z + 2) % 3;
      if (arc[a][b] && arc[b][a]) {
        if (outd[z] == 2) return T120D;
        if (ind[z] == 2) return T120U;
        return T120C;
      }
    }
  }
  return -1; /* unreachable for a valid code */
}

void oracle_build_lut(uint8_t lut[64]) {
  for (unsigned c = 0; c < 64; ++c) lut[c] = (uint8_t)classify_code(c);
}

/* the table, built once per process */
static uint8_t g_lut[64];
static pthread_once_t g_lut_once = PTHREAD_ONCE_INIT;
static void init_lut(void) { oracle_build_lut(g_lut); }
static const uint8_t *the_lut(void) {
  pthread_once(&g_lut_once, init_lut);
  return g_lut;
}

/* C(n,3) in 128 bits (Sec. 3: a digraph has n(n-1)(n-2)/6 triads). */
void oracle_choose3(int64_t n, uint64_t *lo, uint64_t *hi) {
  u128 r = 0;
  if (n >= 3) r = (u128)(uint64_t)n * (u128)(uint64_t)(n - 1) * (u128)(uint64_t)(n - 2) / 6;
  *lo = (uint64_t)r;
  *hi = (uint64_t)(r >> 64);
}

/* One task of Fig. 5: the edge (u, v = nbr[j]) with u < v. Adds the connected
 * triads it owns (step 2.1.4) and its dyadic count (steps 2.1.2-2.1.3). */
static void sweep_task(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg,
                       const uint8_t lut[64], int64_t u, int64_t j, uint64_t census[16]) {
  const int64_t v = nbr[j];
  const unsigned fuv = flag_at(flg, j);
  int64_t p = off[u], pe = off[u + 1], q = off[v], qe = off[v + 1];
  int64_t S = 0; /* |N(u) u N(v) \ {u, v}| */
  while (p < pe || q < qe) {
    int64_t wu = p < pe ? nbr[p] : INT64_MAX;
    int64_t wv = q < qe ? nbr[q] : INT64_MAX;
    int64_t w;
    unsigned fuw = 0, fvw = 0;
    if (wu < wv) { w = wu; fuw = flag_at(flg, p); ++p; }
    else if (wv < wu) { w = wv; fvw = flag_at(flg, q); ++q; }
    else { w = wu; fuw = flag_at(flg, p); fvw = flag_at(flg, q); ++p; ++q; }
    if (w == u || w == v) continue;
    ++S;
    /* canonical selection: count (u,v,w) unless (u,w,v) owns this triad */
    if (v < w || (u < w && w < v && fuw == 0)) census[lut[fuv | fuw << 2 | fvw << 4]] += 1;
  }
  census[fuv == 3 ? T102 : T012] += (uint64_t)(n - S - 2);
}

/* Tasks whose CSR entry index lies in [j0, j1): partial census, no 003. */
void oracle_census_entries(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg,
                           int64_t j0, int64_t j1, uint64_t out[16]) {
  const uint8_t *lut = the_lut();
  if (j0 >= j1) return;
  /* row of entry j0: last u with off[u] <= j0 */
  int64_t lo = 0, hi = n; /* off[lo] <= j0 < off[hi] */
  while (hi - lo > 1) {
    int64_t mid = lo + (hi - lo) / 2;
    if (off[mid] <= j0) lo = mid; else hi = mid;
  }
  int64_t u = lo;
  for (int64_t j = j0; j < j1; ++j) {
    while (off[u + 1] <= j) ++u;
    if (nbr[j] > u) sweep_task(n, off, nbr, flg, lut, u, j, out);
  }
}

/* Given task list: tasks[k] is a CSR entry index j whose neighbour exceeds
 * its row. Partial census (no 003) over those tasks only. */
void oracle_census_tasks(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg,
                         int64_t ntasks, const int64_t *tasks, uint64_t out[16]) {
  const uint8_t *lut = the_lut();
  for (int64_t k = 0; k < ntasks; ++k) {
    int64_t j = tasks[k];
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
      int64_t mid = lo + (hi - lo) / 2;
      if (off[mid] <= j) lo = mid; else hi = mid;
    }
    if (nbr[j] > lo) sweep_task(n, off, nbr, flg, lut, lo, j, out);
  }
}

/* Steps 3-5: the null count from C(n,3) minus the rest, in 128 bits. */
static int finish_null(int64_t n, uint64_t census[16], uint64_t *hi_out) {
  uint64_t clo, chi;
  oracle_choose3(n, &clo, &chi);
  u128 total = ((u128)chi << 64) | clo, s = 0;
  for (int t = 1; t < 16; ++t) s += census[t];
  u128 nul = total - s;
  census[T003] = (uint64_t)nul;
  if (hi_out) *hi_out = (uint64_t)(nul >> 64);
  return (nul >> 64) != 0;
}

/* Full census, single thread. Returns 1 if 003 >= 2^64 (its high word goes to
 * *hi003), else 0. */
int oracle_census(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg, uint64_t out[16],
                  uint64_t *hi003) {
  memset(out, 0, 16 * sizeof(uint64_t));
  if (n > 0) oracle_census_entries(n, off, nbr, flg, 0, off[n], out);
  if (n < 3) { memset(out, 0, 16 * sizeof(uint64_t)); if (hi003) *hi003 = 0; return 0; }
  return finish_null(n, out, hi003);
}

/* Multi-core driver: the same single-threaded task routine over chunks of CSR
 * entries claimed dynamically by T threads; partial censuses are summed
 * exactly (integer addition commutes). */
typedef struct {
  int64_t n;
  const int64_t *off;
  const int32_t *nbr;
  const uint8_t *flg;
  int64_t nnz, chunk;
  atomic_llong next;
  uint64_t part[64][16];
} mt_ctx;
typedef struct { mt_ctx *c; int t; } mt_arg;

static void *mt_worker(void *p) {
  mt_arg *a = (mt_arg *)p;
  mt_ctx *c = a->c;
  for (;;) {
    long long j0 = atomic_fetch_add(&c->next, c->chunk);
    if (j0 >= c->nnz) break;
    long long j1 = j0 + c->chunk < c->nnz ? j0 + c->chunk : c->nnz;
    oracle_census_entries(c->n, c->off, c->nbr, c->flg, j0, j1, c->part[a->t]);
  }
  return NULL;
}

int oracle_census_mt(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg, int nthreads,
                     uint64_t out[16], uint64_t *hi003) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  memset(out, 0, 16 * sizeof(uint64_t));
  if (n < 3) { if (hi003) *hi003 = 0; return 0; }
  mt_ctx *c = (mt_ctx *)calloc(1, sizeof(mt_ctx));
  c->n = n; c->off = off; c->nbr = nbr; c->flg = flg; c->nnz = off[n]; c->chunk = 256;
  atomic_init(&c->next, 0);
  pthread_t th[64];
  mt_arg args[64];
  for (int t = 0; t < nthreads; ++t) {
    args[t].c = c; args[t].t = t;
    pthread_create(&th[t], NULL, mt_worker, &args[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  for (int t = 0; t < nthreads; ++t)
    for (int k = 1; k < 16; ++k) out[k] += c->part[t][k];
  free(c);
  return finish_null(n, out, hi003);
}

/* Multi-core partial census over a given task list (same semantics as
 * oracle_census_tasks), for timing the oracle on a bounded sample. */
typedef struct {
  int64_t n;
  const int64_t *off;
  const int32_t *nbr;
  const uint8_t *flg;
  const int64_t *tasks;
  int64_t ntasks, chunk;
  atomic_llong next;
  uint64_t part[64][16];
} mtt_ctx;
typedef struct { mtt_ctx *c; int t; } mtt_arg;

static void *mtt_worker(void *p) {
  mtt_arg *a = (mtt_arg *)p;
  mtt_ctx *c = a->c;
  for (;;) {
    long long k0 = atomic_fetch_add(&c->next, c->chunk);
    if (k0 >= c->ntasks) break;
    long long k1 = k0 + c->chunk < c->ntasks ? k0 + c->chunk : c->ntasks;
    oracle_census_tasks(c->n, c->off, c->nbr, c->flg, k1 - k0, c->tasks + k0, c->part[a->t]);
  }
  return NULL;
}

void oracle_census_tasks_mt(int64_t n, const int64_t *off, const int32_t *nbr, const uint8_t *flg,
                            int64_t ntasks, const int64_t *tasks, int nthreads, uint64_t out[16]) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  mtt_ctx *c = (mtt_ctx *)calloc(1, sizeof(mtt_ctx));
  c->n = n; c->off = off; c->nbr = nbr; c->flg = flg; c->tasks = tasks; c->ntasks = ntasks; c->chunk = 64;
  atomic_init(&c->next, 0);
  pthread_t th[64];
  mtt_arg args[64];
  for (int t = 0; t < nthreads; ++t) {
    args[t].c = c; args[t].t = t;
    pthread_create(&th[t], NULL, mtt_worker, &args[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  for (int t = 0; t < nthreads; ++t)
    for (int k = 0; k < 16; ++k) out[k] += c->part[t][k];
  free(c);
}
