// Incremental census of a graph that changes by arc insertions and deletions:
// the census of the graph after a batch of updates, from the census before it
// and a merge of the neighbour lists of each changed pair only (the census at
// fixed time intervals of Sec. 3, Figs. 3-4, without a full sweep per
// interval).
//
// A batch is a sequence of arc operations applied in order (insert x->y, or
// delete it). Only its net effect on each unordered pair {a, b}, a < b,
// matters: the pair's flag f (bit0 = a->b, bit1 = b->a, as in row a of the
// CSR) goes from f0 to f1, each bit being set by the last operation on its arc
// (or kept). Only triads that contain a changed pair change class, and
//     census(after) - census(before)
//       = sum over changed pairs {a, b}, over third vertices w, of
//         [class after] - [class before] of the triad {a, b, w},
// each triad counted by the smallest of its changed pairs (pair order
// a << RB | b). For one changed pair the third vertices are
//   - w in N(a) or N(b), before or after: the triad's code is read from the
//     two rows (and the changed pairs of a and b), before and after;
//   - every other w (n - 2 - |that union| of them): only the pair {a, b} has
//     arcs, so the triad moves from the dyadic class of f0 to that of f1
//     (Fig. 5 steps 2.1.2-2.1.3 for a single edge).
// The classes come from the 64-state table of the census (Fig. 5 step
// 2.1.4.1). The null count stays C(n,3) minus the rest.
//
//   k_upd_keys      one key per operation: pair, arc direction, kind
//   radix sort      by (pair, direction), stable: operations keep their order
//   k_run_heads     first operation of each pair
//   k_pair_state    f0 from the CSR, f1 from the last operation on each arc
//   k_changed_keys  two entries per changed pair (one per row), sorted
//   k_pair_chunks   merged positions of each changed pair cut into work items
//   k_upd_delta     one wavefront per work item: the class changes
//   k_row_marks, k_new_offsets, k_copy_old, k_insert_new, k_pack_bytes
//                   the CSR after the batch
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "device_sort.h"
#include "tile_rows.h"
#include "triad_internal.h"

namespace triad {
namespace {

constexpr int UT = 256;

__device__ __forceinline__ uint32_t mirror2(uint32_t f) { return ((f & 1u) << 1) | (f >> 1); }
__device__ __forceinline__ uint32_t entry_flag(const uint8_t* flg, int64_t j) {
  return (flg[j >> 2] >> (2 * (j & 3))) & 3u;
}

// first position in nbr[b, e) with an id >= y
__device__ __forceinline__ int64_t lower_id(const int32_t* nbr, int64_t b, int64_t e, int32_t y) {
  while (b < e) {
    const int64_t m = (b + e) >> 1;
    if (nbr[m] < y) b = m + 1; else e = m;
  }
  return b;
}

// first position in keys[b, e) whose key is >= k
__device__ __forceinline__ int64_t lower_key(const uint64_t* keys, int64_t b, int64_t e, uint64_t k) {
  while (b < e) {
    const int64_t m = (b + e) >> 1;
    if (keys[m] < k) b = m + 1; else e = m;
  }
  return b;
}

// Operation key: (a << rb | b) << 2 | dir << 1 | insert, a < b the pair, dir =
// 1 for the arc b -> a.
__global__ void k_upd_keys(int64_t n, int64_t k, int rb, const int32_t* __restrict__ src,
                           const int32_t* __restrict__ dst, const uint8_t* __restrict__ ins,
                           uint64_t* __restrict__ keys, uint32_t* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t bits = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride) {
    const int32_t s = src[i], d = dst[i];
    const uint32_t op = ins[i];
    if (s < 0 || d < 0 || s >= n || d >= n || op > 1u) {
      bits |= ERR_RANGE;
      keys[i] = 0;
      continue;
    }
    if (s == d) bits |= ERR_SELFLOOP;
    const uint64_t a = (uint64_t)min(s, d), b = (uint64_t)max(s, d);
    keys[i] = (((a << rb) | b) << 2) | ((uint64_t)(s > d) << 1) | op;
  }
  if (bits) atomicOr(err, bits);
}

__global__ void k_run_heads(const uint64_t* __restrict__ keys, int64_t k, int shift, uint32_t* __restrict__ head) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride)
    head[i] = (i == 0 || (keys[i] >> shift) != (keys[i - 1] >> shift)) ? 1u : 0u;
}

// Per pair (run of operations): f0 from row a of the CSR, f1 = f0 with each
// arc's bit set by the last operation on that arc (runs are sorted by arc
// direction, operations in batch order within it).
__global__ void k_pair_state(const uint64_t* __restrict__ keys, int64_t k, int rb, const uint32_t* __restrict__ head,
                             const uint32_t* __restrict__ hpos, const int64_t* __restrict__ off,
                             const int32_t* __restrict__ nbr, const uint8_t* __restrict__ flg,
                             uint64_t* __restrict__ pkey, uint8_t* __restrict__ pf, uint32_t* __restrict__ chg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t bmask = (1ull << rb) - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride) {
    if (!head[i]) continue;
    const uint64_t pr = keys[i] >> 2;
    const int64_t a = (int64_t)(pr >> rb);
    const int32_t b = (int32_t)(pr & bmask);
    const int64_t e = off[a + 1];
    const int64_t j = lower_id(nbr, off[a], e, b);
    const uint32_t f0 = (j < e && nbr[j] == b) ? entry_flag(flg, j) : 0u;
    uint32_t f1 = f0;
    for (int64_t q = i; q < k && (keys[q] >> 2) == pr; ++q) {
      const uint32_t bit = 1u << ((keys[q] >> 1) & 1u);
      f1 = (keys[q] & 1u) ? (f1 | bit) : (f1 & ~bit);
    }
    const uint32_t r = hpos[i];
    pkey[r] = pr;
    pf[r] = (uint8_t)(f0 | f1 << 2);
    chg[r] = f0 != f1 ? 1u : 0u;
  }
}

// Two entries per changed pair, one in each row: (row << rb | col) << 4 |
// f0 << 2 | f1, flags seen from the row (mirrored in row b).
__global__ void k_changed_keys(const uint64_t* __restrict__ pkey, const uint8_t* __restrict__ pf,
                               const uint32_t* __restrict__ chg, const uint32_t* __restrict__ cpos, int64_t np,
                               int rb, uint64_t* __restrict__ E) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t bmask = (1ull << rb) - 1;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < np; r += stride) {
    if (!chg[r]) continue;
    const uint64_t a = pkey[r] >> rb, b = pkey[r] & bmask;
    const uint32_t f0 = pf[r] & 3u, f1 = pf[r] >> 2;
    const uint32_t c = cpos[r];
    E[2 * (int64_t)c] = (((a << rb) | b) << 4) | (f0 << 2) | f1;
    E[2 * (int64_t)c + 1] = (((b << rb) | a) << 4) | (mirror2(f0) << 2) | mirror2(f1);
  }
}

struct DeltaArgs {
  int64_t n;
  const int64_t* off;
  const int32_t* nbr;
  const uint8_t* flg;
  int rb;
  const uint64_t* E;  // sorted change entries
  int64_t nE;
  uint64_t lut[4];    // class of code c: nibble c & 15 of lut[c >> 4]
  unsigned long long* delta;  // [16], two's complement
  // work items: item it is chunk it - ipre[q] of the pair of entry q (ipre:
  // exclusive prefix of the chunk counts, ipre[nE] = the item count)
  const uint32_t* ipre;
};

// Merged positions of N(a) and N(b) per work item: a longer pair is cut into
// chunks of about UPD_CHUNK positions (at most maxch chunks, which keeps the
// item count below 2^32) that different wavefronts walk, so that a pair on a
// hub row does not hold one wavefront for the whole of its merge.
constexpr int64_t UPD_CHUNK = 8192;

// Chunk count of the pair of each change entry (0 for the entry in the upper
// row: a pair is processed from its lower row).
__global__ void k_pair_chunks(const uint64_t* __restrict__ E, int64_t nE, int rb, const int64_t* __restrict__ off,
                              uint32_t maxch, uint32_t* __restrict__ nch) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t cmask = (1ull << rb) - 1;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nE; q += stride) {
    const uint64_t ent = E[q];
    const int64_t a = (int64_t)(ent >> (4 + rb)), b = (int64_t)((ent >> 4) & cmask);
    const int64_t D = (off[a + 1] - off[a]) + (off[b + 1] - off[b]);
    nch[q] = b < a ? 0u : (uint32_t)min((int64_t)maxch, max((int64_t)1, (D + UPD_CHUNK - 1) / UPD_CHUNK));
  }
}

__device__ __forceinline__ uint32_t class_of(const DeltaArgs& g, uint32_t code) {
  const uint64_t w = code < 16 ? g.lut[0] : code < 32 ? g.lut[1] : code < 48 ? g.lut[2] : g.lut[3];
  return (uint32_t)(w >> (4 * (code & 15u))) & 15u;
}

// Change entry of (x, y) in E[b, e) (the row x range): index or -1.
__device__ __forceinline__ int64_t find_change(const DeltaArgs& g, int64_t b, int64_t e, int64_t x, int32_t y) {
  const uint64_t k = (((uint64_t)x << g.rb) | (uint64_t)y) << 4;
  const int64_t p = lower_key(g.E, b, e, k);
  return (p < e && (g.E[p] >> 4) == (k >> 4)) ? p : -1;
}

// Positions of the merged walk of N(a) and N(b) each lane takes per round.
constexpr int UPD_S = 16;

// Class change of the triad {a, b, w} for the third vertex w with old flags
// g0a (a-w), g0b (b-w) and new ones g1a, g1b (cha, chb: that pair changes),
// counted by the triad's smallest changed pair only.
__device__ __forceinline__ void triad_move(const DeltaArgs& g, int32_t* h, int lane, uint64_t pk, int64_t a, int32_t b,
                                           int32_t w, uint32_t f0, uint32_t f1, uint32_t g0a, uint32_t g1a, bool cha,
                                           uint32_t g0b, uint32_t g1b, bool chb) {
  bool own = true;
  if (cha) own = own && pk < ((((uint64_t)min((int64_t)w, a)) << g.rb) | (uint64_t)max((int64_t)w, a));
  if (chb) own = own && pk < ((((uint64_t)min(w, b)) << g.rb) | (uint64_t)max(w, b));
  if (!own) return;
  const uint32_t oc = class_of(g, f0 | g0a << 2 | g0b << 4), nc = class_of(g, f1 | g1a << 2 | g1b << 4);
  if (oc != nc) {
    h[oc * 64 + lane] -= 1;
    h[nc * 64 + lane] += 1;
  }
}

// One wavefront per work item: a chunk of the merge of a changed pair {a, b}
// (the pairs are the entries of row a in E with a < b). The third vertices are
// the union of four sorted lists: N(a), the changes of a, N(b), the changes of
// b. N(a) and N(b) are walked together, merged in id order (a merge path cut
// into 16 positions per lane and round, a common id consumed once), so each
// vertex of either row comes with both old flags; a vertex adjacent to b only
// whose pair with a changes is left to the pass over the changes of a. The
// pair's first item then takes the changes of a, then of b, each vertex seen
// in an earlier list skipped.
__global__ void __launch_bounds__(UT) k_upd_delta(DeltaArgs g) {
  __shared__ int32_t hist[UT / 64][16][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t* h = &hist[wv][0][0];
  for (int c = 0; c < 16; ++c) h[c * 64 + lane] = 0;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t cmask = (1ull << g.rb) - 1;
  uint32_t steps = 0;
  const int64_t nit = g.ipre[g.nE];
  for (int64_t it = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; it < nit; it += nw) {
    // the item's pair: the last entry q with ipre[q] <= it (one with chunks)
    int64_t q = 0;
    for (int64_t hi = g.nE; hi - q > 1;) {
      const int64_t mid = (q + hi) >> 1;
      if ((int64_t)g.ipre[mid] <= it) q = mid; else hi = mid;
    }
    const int64_t chunk = it - (int64_t)g.ipre[q];
    const uint64_t ent = g.E[q];
    const int64_t a = (int64_t)(ent >> (4 + g.rb));
    const int32_t b = (int32_t)((ent >> 4) & cmask);
    const uint32_t f0 = (ent >> 2) & 3u, f1 = ent & 3u;
    const uint64_t pk = ((uint64_t)a << g.rb) | (uint64_t)b;
    const int64_t oa = g.off[a], ea = g.off[a + 1], ob = g.off[b], eb = g.off[b + 1];
    const int64_t da0 = lower_key(g.E, 0, g.nE, (uint64_t)a << (g.rb + 4));
    const int64_t da1 = lower_key(g.E, da0, g.nE, (uint64_t)(a + 1) << (g.rb + 4));
    const int64_t db0 = lower_key(g.E, 0, g.nE, (uint64_t)b << (g.rb + 4));
    const int64_t db1 = lower_key(g.E, db0, g.nE, (uint64_t)(b + 1) << (g.rb + 4));
    uint32_t ucount = 0;
    // N(a) and N(b) merged
    const int32_t* const A = g.nbr + oa;
    const int32_t* const B = g.nbr + ob;
    const int64_t la = ea - oa, lb = eb - ob, D = la + lb;
    // this item's merged positions [c0, c1) (the pair's nq chunks cover its
    // merge); per lane and round UPD_S of them, or fewer for a short range so
    // that it spreads over the wavefront
    const int64_t nq = (int64_t)g.ipre[q + 1] - (int64_t)g.ipre[q];
    const int64_t csz = (D + nq - 1) / nq;
    const int64_t c0 = min(D, chunk * csz), c1 = min(D, c0 + csz);
    const int64_t S = c1 - c0 < 64 * UPD_S ? max((int64_t)1, (c1 - c0 + 63) >> 6) : (int64_t)UPD_S;
    for (int64_t r0 = c0; r0 < c1; r0 += 64 * S) {
      const int64_t d0 = min(c1, r0 + (int64_t)lane * S), d1 = min(c1, d0 + S);
      // merge-path split of diagonal d0: A elements among the first d0 merged
      int64_t lo = d0 > lb ? d0 - lb : 0, hi = min(d0, la);
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (A[mid] <= B[d0 - mid - 1]) lo = mid + 1; else hi = mid;
      }
      int64_t i = lo, k = d0 - lo;
      // an id shared by A[i-1] and B[k] was taken with A[i-1] by a lane before
      if (i > 0 && k < lb && A[i - 1] == B[k]) ++k;
      if (i + k >= d1) continue;
      // The lane's ids ascend, and so do the change entries of a and of b: one
      // search each for the first change at or after the lane's first id, then
      // cursors that only move forward. (A change list holding only the pair
      // {a, b} itself has no entry for any w walked here.)
      const int32_t wfirst = min(i < la ? A[i] : INT32_MAX, k < lb ? B[k] : INT32_MAX);
      int64_t pa = da1, pb = db1;
      if (da1 - da0 > 1) pa = lower_key(g.E, da0, da1, (((uint64_t)a << g.rb) | (uint64_t)wfirst) << 4);
      if (db1 - db0 > 1) pb = lower_key(g.E, db0, db1, (((uint64_t)b << g.rb) | (uint64_t)wfirst) << 4);
      int64_t ida = pa < da1 ? (int64_t)((g.E[pa] >> 4) & cmask) : INT64_MAX;
      int64_t idb = pb < db1 ? (int64_t)((g.E[pb] >> 4) & cmask) : INT64_MAX;
      while (i + k < d1) {
        const int32_t x = i < la ? A[i] : INT32_MAX, y = k < lb ? B[k] : INT32_MAX;
        const bool inA = x <= y, inB = y <= x;
        const int32_t w = inA ? x : y;
        const uint32_t fa = inA ? entry_flag(g.flg, oa + i) : 0u, fb = inB ? entry_flag(g.flg, ob + k) : 0u;
        i += inA;
        k += inB;
        while (ida < w) {
          ++pa;
          ida = pa < da1 ? (int64_t)((g.E[pa] >> 4) & cmask) : INT64_MAX;
        }
        while (idb < w) {
          ++pb;
          idb = pb < db1 ? (int64_t)((g.E[pb] >> 4) & cmask) : INT64_MAX;
        }
        if (w == a || w == b) continue;
        uint32_t g1a = fa;
        bool cha = false;
        if (ida == w) {
          if (!inA) continue;  // a pair with a that changes: the pass over the changes of a takes w
          cha = true;
          g1a = (uint32_t)(g.E[pa] & 3u);
        }
        const bool chb = idb == w;
        const uint32_t g1b = chb ? (uint32_t)(g.E[pb] & 3u) : fb;
        ++ucount;
        triad_move(g, h, lane, pk, a, b, w, f0, f1, fa, g1a, cha, fb, g1b, chb);
      }
    }
    // the changes of a (vertices not in N(a)), then of b (not in N(b), not
    // seen before): the pair's first item only
    for (int phase = 1; phase < 4 && chunk == 0; phase += 2) {
      const int64_t L0 = phase == 1 ? da0 : db0;
      const int64_t L1 = phase == 1 ? da1 : db1;
      for (int64_t j0 = L0; j0 < L1; j0 += 64) {
        const int64_t j = j0 + lane;
        if (j >= L1) continue;
        int32_t w;
        uint32_t g0a = 0, g1a = 0, g0b = 0, g1b = 0;
        bool cha = false, chb = false, keep = true;
        {
          const uint64_t e = g.E[j];
          w = (int32_t)((e >> 4) & cmask);
          if (w == a || w == b) continue;
          if (phase == 1) {
            g0a = (e >> 2) & 3u;
            g1a = e & 3u;
            cha = true;
            keep = g0a == 0;  // otherwise w is in N(a), seen in the merged walk
            if (keep) {
              const int64_t jb = lower_id(g.nbr, ob, eb, w);
              g0b = (jb < eb && g.nbr[jb] == w) ? entry_flag(g.flg, jb) : 0u;
              const int64_t p = find_change(g, db0, db1, b, w);
              chb = p >= 0;
              g1b = chb ? (uint32_t)(g.E[p] & 3u) : g0b;
            }
          } else {
            g0b = (e >> 2) & 3u;
            g1b = e & 3u;
            chb = true;
            if (g0b != 0) {
              keep = false;  // in N(b), seen in the merged walk
            } else {
              const int64_t ja = lower_id(g.nbr, oa, ea, w);
              keep = !(ja < ea && g.nbr[ja] == w) && find_change(g, da0, da1, a, w) < 0;
            }
          }
        }
        if (!keep) continue;
        ++ucount;
        triad_move(g, h, lane, pk, a, b, w, f0, f1, g0a, g1a, cha, g0b, g1b, chb);
      }
    }
    // every other third vertex: only the pair {a, b} has arcs. Those are the
    // n - 2 others less the vertices the pair's items met; each item takes
    // its own count off (the first adds the n - 2).
    uint32_t u = ucount;
    for (int o = 32; o > 0; o >>= 1) u += __shfl_xor(u, o, 64);
    if (lane == 0) {
      const int64_t rest = (chunk == 0 ? g.n - 2 : 0) - (int64_t)u;
      const uint32_t oc = class_of(g, f0), nc = class_of(g, f1);
      if (rest != 0 && oc != nc) {
        atomicAdd(&g.delta[oc], (unsigned long long)(-rest));
        atomicAdd(&g.delta[nc], (unsigned long long)rest);
      }
    }
    steps += (uint32_t)((c1 - c0 + da1 - da0 + db1 - db0) / 64 + 4);
    if (steps > (1u << 29)) {
      __builtin_amdgcn_wave_barrier();
      for (int c = 0; c < 16; ++c) {
        int64_t x = h[c * 64 + lane];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0 && x) atomicAdd(&g.delta[c], (unsigned long long)x);
        h[c * 64 + lane] = 0;
      }
      steps = 0;
    }
  }
  __builtin_amdgcn_wave_barrier();
  for (int c = 0; c < 16; ++c) {
    int64_t x = h[c * 64 + lane];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0 && x) atomicAdd(&g.delta[c], (unsigned long long)x);
  }
}

// ---------------------------------------------------------- CSR after
// Change entry e is an insertion (f0 = 0), a deletion (f1 = 0) or a new flag.
__global__ void k_change_kinds(const uint64_t* __restrict__ E, int64_t nE, uint32_t* __restrict__ ins,
                               uint32_t* __restrict__ del) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e <= nE; e += stride) {
    const uint32_t f0 = e < nE ? (uint32_t)(E[e] >> 2) & 3u : 1u, f1 = e < nE ? (uint32_t)E[e] & 3u : 1u;
    ins[e] = f0 == 0 ? 1u : 0u;
    del[e] = f1 == 0 ? 1u : 0u;
  }
}

__global__ void k_row_marks(const uint64_t* __restrict__ E, int64_t nE, int rb, uint32_t* __restrict__ mark) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nE; e += stride) {
    const uint64_t x = E[e] >> (4 + rb);
    atomicOr(&mark[x >> 5], 1u << (x & 31));
  }
}

// new_off[x] = off[x] + insertions - deletions in rows below x
__global__ void k_new_offsets(int64_t n, int rb, const int64_t* __restrict__ off, const uint64_t* __restrict__ E,
                              int64_t nE, const uint32_t* __restrict__ I, const uint32_t* __restrict__ D,
                              int64_t* __restrict__ noff) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= n; x += stride) {
    const int64_t e = lower_key(E, 0, nE, (uint64_t)x << (rb + 4));
    noff[x] = off[x] + (int64_t)I[e] - (int64_t)D[e];
  }
}

// Old entries to their new places: rows without changes shift as a whole;
// in a changed row an entry moves by the insertions and deletions before it,
// takes its new flag, or is dropped. The shift of an unchanged row, noff[x] -
// off[x], changes only past a changed row, so a tile of ETILE entries whose
// rows hold at most COPY_MAXCHG changed rows (the usual case) lists those rows
// with their entry ranges, their ranges of change entries and the shift of
// each run of unchanged rows between them: an entry finds its run by comparing
// its index with the few range ends, and an entry of a changed row searches
// only that row's change entries. Other tiles find each entry's row by a
// search of LDS-staged row starts, and its row's change entries by a search of
// all of them.
constexpr int COPY_MAXCHG = 8;
struct CopyTile {
  TileRows T;                        // r[0], r[1]: rows of the tile's first and last entry
  int64_t crow[COPY_MAXCHG];         // the tile's changed rows, ascending
  int64_t cbeg[COPY_MAXCHG], cend[COPY_MAXCHG];  // their entry ranges
  int64_t cex[COPY_MAXCHG], cexe[COPY_MAXCHG];   // their change entries E[cex, cexe)
  int64_t sdelta[COPY_MAXCHG + 1];   // shift of the unchanged rows before changed row s
  int32_t nchg;                      // changed rows; -1: too many (per-entry row search)
};

__global__ void __launch_bounds__(UT) k_copy_old(int64_t n, int64_t nnz, int rb, const int64_t* __restrict__ off,
                                                 const int32_t* __restrict__ nbr, const uint8_t* __restrict__ flg,
                                                 const uint64_t* __restrict__ E, int64_t nE,
                                                 const uint32_t* __restrict__ I, const uint32_t* __restrict__ D,
                                                 const uint32_t* __restrict__ mark, const int64_t* __restrict__ noff,
                                                 int64_t nn, int32_t* __restrict__ nnbr, uint8_t* __restrict__ nfl) {
  __shared__ CopyTile C;
  for (int64_t t0 = (int64_t)blockIdx.x * ETILE; t0 < nnz; t0 += (int64_t)gridDim.x * ETILE) {
    const int64_t t1 = min(t0 + (int64_t)ETILE, nnz);
    __syncthreads();
    if (threadIdx.x < 2) C.T.r[threadIdx.x] = row_search(off, 0, n, threadIdx.x == 0 ? t0 : t1 - 1);
    __syncthreads();
    const int64_t r0 = C.T.r[0], r1 = C.T.r[1];
    // the changed rows among r0..r1 in ascending order, from the row marks:
    // one mark word (32 rows) per lane of the first wavefront
    if (threadIdx.x < 64) {
      const int lane = (int)threadIdx.x;
      const int64_t w0 = r0 >> 5, w1 = r1 >> 5;
      int32_t total = -1;
      if (w1 - w0 < 64) {
        const int64_t w = w0 + lane;
        uint32_t m = 0;
        if (w <= w1) {
          m = mark[w];
          if (w == w0) m &= ~0u << (r0 & 31);
          if (w == w1 && (r1 & 31) != 31) m &= (1u << ((r1 & 31) + 1)) - 1u;
        }
        const uint32_t c = (uint32_t)__popc(m);
        uint32_t pre = c;  // inclusive prefix over the lanes
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t v = __shfl_up(pre, o, 64);
          if (lane >= o) pre += v;
        }
        const uint32_t all = __shfl(pre, 63, 64);
        if (all <= (uint32_t)COPY_MAXCHG) {
          uint32_t q = pre - c;
          while (m) {
            C.crow[q++] = w * 32 + __builtin_ctz(m);
            m &= m - 1u;
          }
          total = (int32_t)all;
        }
      }
      if (lane == 0) C.nchg = total;
    }
    __syncthreads();
    const int32_t nchg = C.nchg;
    if (nchg >= 0) {
      const int q = (int)threadIdx.x;
      if (q <= nchg) {
        const int64_t xs = q == 0 ? r0 : C.crow[q - 1] + 1;  // <= r1 + 1 <= n
        C.sdelta[q] = noff[xs] - off[xs];
        if (q < nchg) {
          const int64_t c = C.crow[q];
          C.cbeg[q] = off[c];
          C.cend[q] = off[c + 1];
          const int64_t ex = lower_key(E, 0, nE, (uint64_t)c << (rb + 4));
          C.cex[q] = ex;
          C.cexe[q] = lower_key(E, ex, nE, (uint64_t)(c + 1) << (rb + 4));
        }
      }
    } else {
      const int64_t nr = r1 - r0 + 1;
      if (nr <= TILE_ROWS)
        for (int64_t x = threadIdx.x; x < nr; x += blockDim.x) {
          const int64_t d = off[r0 + x] - t0;
          C.T.rel[x] = (uint16_t)(d > 0 ? d : 0);
        }
    }
    __syncthreads();
    for (int64_t j = t0 + threadIdx.x; j < t1; j += blockDim.x) {
      const int32_t y = nbr[j];
      uint32_t f = entry_flag(flg, j);
      int64_t x, pos, ex = 0, exe = nE;
      bool changed;
      if (nchg >= 0) {
        int sidx = 0;  // changed rows whose entries all lie before j
        for (int q = 0; q < nchg; ++q) sidx += C.cend[q] <= j ? 1 : 0;
        changed = sidx < nchg && j >= C.cbeg[sidx];
        x = 0;
        pos = j + C.sdelta[sidx];
        if (changed) {
          x = C.crow[sidx];
          pos = noff[x] + (j - C.cbeg[sidx]);
          ex = C.cex[sidx];
          exe = C.cexe[sidx];
        }
      } else {
        x = tile_row(off, C.T, t0, j);
        changed = (mark[x >> 5] >> (x & 31)) & 1u;
        pos = noff[x] + (j - off[x]);
        if (changed) ex = lower_key(E, 0, nE, (uint64_t)x << (rb + 4));
      }
      if (changed) {
        const uint64_t k = (((uint64_t)x << rb) | (uint64_t)y) << 4;
        const int64_t e = lower_key(E, ex, exe, k);
        pos += ((int64_t)I[e] - (int64_t)I[ex]) - ((int64_t)D[e] - (int64_t)D[ex]);
        if (e < nE && (E[e] >> 4) == (k >> 4)) {
          f = (uint32_t)E[e] & 3u;
          if (f == 0) continue;  // deleted
        }
      }
      if (pos >= 0 && pos < nn) {  // always true; keeps a faulty position in bounds
        nnbr[pos] = y;
        nfl[pos] = (uint8_t)f;
      }
    }
  }
}

__global__ void k_insert_new(int rb, const int64_t* __restrict__ off, const int32_t* __restrict__ nbr,
                             const uint64_t* __restrict__ E, int64_t nE, const uint32_t* __restrict__ I,
                             const uint32_t* __restrict__ D, const int64_t* __restrict__ noff, int64_t nn,
                             int32_t* __restrict__ nnbr, uint8_t* __restrict__ nfl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t cmask = (1ull << rb) - 1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nE; e += stride) {
    if (((E[e] >> 2) & 3u) != 0) continue;  // not an insertion
    const int64_t x = (int64_t)(E[e] >> (4 + rb));
    const int32_t y = (int32_t)((E[e] >> 4) & cmask);
    const int64_t ex = lower_key(E, 0, nE, (uint64_t)x << (rb + 4));
    const int64_t below = lower_id(nbr, off[x], off[x + 1], y) - off[x];
    const int64_t pos = noff[x] + below + ((int64_t)I[e] - (int64_t)I[ex]) - ((int64_t)D[e] - (int64_t)D[ex]);
    if (pos >= 0 && pos < nn) {
      nnbr[pos] = y;
      nfl[pos] = (uint8_t)(E[e] & 3u);
    }
  }
}

__global__ void k_pack_bytes(const uint8_t* __restrict__ f, int64_t m, uint8_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, nb = (m + 3) / 4;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += stride) {
    uint32_t v = 0;
    for (int k = 0; k < 4; ++k)
      if (4 * b + k < m) v |= (uint32_t)(f[4 * b + k] & 3u) << (2 * k);
    out[b] = (uint8_t)v;
  }
}

__global__ void k_zero32(uint32_t* p, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) p[i] = 0;
}

__global__ void k_copy_words(const uint32_t* __restrict__ a, uint32_t* __restrict__ b, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) b[i] = a[i];
}
__global__ void k_copy_bytes(const uint8_t* __restrict__ a, uint8_t* __restrict__ b, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) b[i] = a[i];
}
__global__ void k_copy_i64(const int64_t* __restrict__ a, int64_t* __restrict__ b, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) b[i] = a[i];
}

}  // namespace

int census_update(int64_t n, int64_t nnz, const int64_t* off, const int32_t* nbr, const uint8_t* flg, int64_t k,
                  const int32_t* src, const int32_t* dst, const uint8_t* ins, const uint64_t* cin, uint64_t* cout,
                  int64_t* noff, int32_t* nnbr, uint8_t* nflg, int64_t* nnz_new, int64_t* changed_pairs,
                  hipStream_t s) {
  if (n < 0 || n >= ((int64_t)1 << 30)) return fail(TRIAD_EINVAL, "n must be in [0, 2^30)");
  if (nnz < 0 || nnz >= ((int64_t)1 << 32)) return fail(TRIAD_EINVAL, "nnz must be in [0, 2^32)");
  if (k < 0 || k >= ((int64_t)1 << 31)) return fail(TRIAD_EINVAL, "the update count must be in [0, 2^31)");
  if (!off || !cin || !cout || (nnz > 0 && (!nbr || !flg)) || (k > 0 && (!src || !dst || !ins)))
    return fail(TRIAD_EINVAL, "NULL pointer argument");
  const bool new_csr = noff != nullptr;
  if (new_csr && (!nnz_new || !nnbr || !nflg)) return fail(TRIAD_EINVAL, "NULL pointer for the new CSR");
  Scratch scratch(s, 0, true);
  const int rb = std::max(1, 64 - __builtin_clzll((unsigned long long)std::max<int64_t>(n, 1)));
  uint32_t* err = nullptr;
  unsigned long long* delta = nullptr;
  uint32_t* tot = nullptr;
  ALLOC(err, 1);
  ALLOC(delta, 16);
  ALLOC(tot, 4);
  k_zero32<<<1, 64, 0, s>>>(err, 1);
  k_zero32<<<1, 64, 0, s>>>((uint32_t*)delta, 32);
  k_zero32<<<1, 64, 0, s>>>(tot, 4);
  int64_t np = 0, K = 0;
  uint64_t* E = nullptr;
  if (k > 0) {
    uint64_t *ka = nullptr, *kb = nullptr;
    ALLOC(ka, k);
    ALLOC(kb, k);
    k_upd_keys<<<grid_of(k, 256, 65536), 256, 0, s>>>(n, k, rb, src, dst, ins, ka, err);
    uint32_t eh = 0;
    HIPCHK(hipMemcpyAsync(&eh, err, sizeof eh, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (eh) return fail(status_from_bits(eh), eh & ERR_RANGE ? "update endpoint outside [0, n) or kind not 0/1"
                                                             : "update on a self-loop");
    // by (pair, direction); operations keep their batch order within an arc
    if (int st = radix_sort_u64(&ka, &kb, k, 1, 2 + 2 * rb, scratch, s)) return st;
    uint32_t *head = nullptr, *hpos = nullptr;
    ALLOC(head, k);
    ALLOC(hpos, k);
    k_run_heads<<<grid_of(k, 256, 65536), 256, 0, s>>>(ka, k, 2, head);
    if (int st = scan_u32(head, k, hpos, tot, scratch, s)) return st;
    uint32_t h = 0;
    HIPCHK(hipMemcpyAsync(&h, tot, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    np = h;
    uint64_t* pkey = nullptr;
    uint8_t* pf = nullptr;
    uint32_t *chg = nullptr, *cpos = nullptr;
    ALLOC(pkey, np);
    ALLOC(pf, np);
    ALLOC(chg, np);
    ALLOC(cpos, np);
    k_pair_state<<<grid_of(k, 256, 65536), 256, 0, s>>>(ka, k, rb, head, hpos, off, nbr, flg, pkey, pf, chg);
    if (int st = scan_u32(chg, np, cpos, tot + 1, scratch, s)) return st;
    HIPCHK(hipMemcpyAsync(&h, tot + 1, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    K = h;
    if (K > 0) {
      uint64_t* Eb = nullptr;
      ALLOC(E, 2 * K);
      ALLOC(Eb, 2 * K);
      k_changed_keys<<<grid_of(np, 256, 65536), 256, 0, s>>>(pkey, pf, chg, cpos, np, rb, E);
      if (int st = radix_sort_u64(&E, &Eb, 2 * K, 4, 4 + 2 * rb, scratch, s)) return st;
      DeltaArgs g{};
      g.n = n;
      g.off = off;
      g.nbr = nbr;
      g.flg = flg;
      g.rb = rb;
      g.E = E;
      g.nE = 2 * K;
      for (int c = 0; c < 64; ++c) g.lut[c >> 4] |= (uint64_t)classify_code((unsigned)c) << (4 * (c & 15));
      g.delta = delta;
      uint32_t *nch = nullptr, *ipre = nullptr;
      ALLOC(nch, 2 * K);
      ALLOC(ipre, 2 * K + 1);
      const uint32_t maxch = (uint32_t)std::max<int64_t>(1, std::min<int64_t>(4096, 0xFFFFFFFFll / (2 * K)));
      k_pair_chunks<<<grid_of(2 * K, 256, 65536), 256, 0, s>>>(E, 2 * K, rb, off, maxch, nch);
      if (int st = scan_u32(nch, 2 * K, ipre, ipre + 2 * K, scratch, s)) return st;
      g.ipre = ipre;
      k_upd_delta<<<grid_of(2 * K * 64, UT, 8192), UT, 0, s>>>(g);
      HIPCHK(hipGetLastError());
    }
  }
  // the census after the batch
  uint64_t dh[16];
  HIPCHK(hipMemcpyAsync(dh, delta, sizeof dh, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  uint64_t res[17];
  unsigned __int128 sum = 0;
  for (int t = 1; t < 16; ++t) {
    res[t] = cin[t] + dh[t];
    sum += res[t];
  }
  uint64_t clo, chi;
  choose3(n, &clo, &chi);
  const unsigned __int128 nul = (((unsigned __int128)chi << 64) | clo) - sum;
  res[0] = (uint64_t)nul;
  res[16] = (uint64_t)(nul >> 64);
  // the CSR after the batch
  int64_t nn = nnz;
  if (new_csr) {
    if (K == 0) {
      k_copy_i64<<<grid_of(n + 1, 256, 65536), 256, 0, s>>>(off, noff, n + 1);
      if (nnz > 0) {
        k_copy_words<<<grid_of(nnz, 256, 65536), 256, 0, s>>>((const uint32_t*)nbr, (uint32_t*)nnbr, nnz);
        k_copy_bytes<<<grid_of((nnz + 3) / 4, 256, 65536), 256, 0, s>>>(flg, nflg, (nnz + 3) / 4);
      }
    } else {
      const int64_t nE = 2 * K;
      uint32_t *ik = nullptr, *dk = nullptr, *I = nullptr, *D = nullptr, *mark = nullptr;
      uint8_t* nf8 = nullptr;
      ALLOC(ik, nE + 1);
      ALLOC(dk, nE + 1);
      ALLOC(I, nE + 1);
      ALLOC(D, nE + 1);
      ALLOC(mark, (n >> 5) + 1);
      k_change_kinds<<<grid_of(nE + 1, 256, 65536), 256, 0, s>>>(E, nE, ik, dk);
      if (int st = scan_u32(ik, nE + 1, I, tot + 2, scratch, s)) return st;
      if (int st = scan_u32(dk, nE + 1, D, tot + 3, scratch, s)) return st;
      uint32_t idt[2];
      HIPCHK(hipMemcpyAsync(idt, tot + 2, sizeof idt, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      nn = nnz + (int64_t)idt[0] - (int64_t)idt[1];
      ALLOC(nf8, nn);
      k_zero32<<<grid_of((n >> 5) + 1, 256, 4096), 256, 0, s>>>(mark, (n >> 5) + 1);
      k_row_marks<<<grid_of(nE, 256, 65536), 256, 0, s>>>(E, nE, rb, mark);
      k_new_offsets<<<grid_of(n + 1, 256, 65536), 256, 0, s>>>(n, rb, off, E, nE, I, D, noff);
      if (nnz > 0)
        k_copy_old<<<grid_of(nnz, ETILE, 65536), UT, 0, s>>>(n, nnz, rb, off, nbr, flg, E, nE, I, D, mark, noff,
                                                                 nn, nnbr, nf8);
      k_insert_new<<<grid_of(nE, 256, 65536), 256, 0, s>>>(rb, off, nbr, E, nE, I, D, noff, nn, nnbr, nf8);
      k_pack_bytes<<<grid_of((nn + 3) / 4, 256, 65536), 256, 0, s>>>(nf8, nn, nflg);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(s));
    *nnz_new = nn;
  }
  std::memcpy(cout, res, sizeof res);
  if (changed_pairs) *changed_pairs = K;
  return res[16] ? TRIAD_OK_003_WRAPPED : TRIAD_OK;
}

}  // namespace triad

using namespace triad;

extern "C" int triad_census_update(int64_t n, int64_t nnz, const int64_t* d_offsets, const int32_t* d_nbrs,
                                   const uint8_t* d_flags, int64_t nupd, const int32_t* d_src, const int32_t* d_dst,
                                   const uint8_t* d_insert, const uint64_t census_in[17], uint64_t census_out[17],
                                   int64_t* d_offsets_new, int32_t* d_nbrs_new, uint8_t* d_flags_new,
                                   int64_t* nnz_new, int64_t* changed_pairs, void* hip_stream) {
  return census_update(n, nnz, d_offsets, d_nbrs, d_flags, nupd, d_src, d_dst, d_insert, census_in, census_out,
                       d_offsets_new, d_nbrs_new, d_flags_new, nnz_new, changed_pairs, (hipStream_t)hip_stream);
}
