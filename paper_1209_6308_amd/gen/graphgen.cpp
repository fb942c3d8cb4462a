// Seeded synthetic graph generators and the symmetric CSR builder.
//
// This module produces inputs only. It holds none of the census arithmetic:
// no triad codes, no classification, no counting. Both the CPU oracle tests
// and the GPU path consume what it emits.
//
// Input contract produced here (the compact structure of Sec. 6, Fig. 7 of
// the paper, with the direction bits moved out of the id into a packed
// side array):
//   offsets int64[n+1], nbrs int32[nnz] with every row strictly increasing,
//   no self-loops, symmetric (y in N(x) iff x in N(y));
//   flags: 2 bits per entry, entry j at bits 2*(j&3) of byte j>>2;
//   bit0 = arc row->neighbour, bit1 = arc neighbour->row (never 0).
//
// Randomness: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014) used as a counter-based generator:
// draw(seed, stream, i) = mix(mix(seed + stream*G2) + i*G1), so every draw is
// addressed by its counter and results do not depend on thread count.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t G1 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t G2 = 0xD1B54A32D192ED03ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t i) {
  return mix64(mix64(seed + stream * G2 + G1) + i * G1);
}
// uniform double in [0,1) from the top 53 bits
inline double unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

struct Csr {
  int64_t n = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> nbr;
  std::vector<uint8_t> flg;
};

// Arc list -> symmetric CSR with 2-bit direction flags. Drops self-loops and
// duplicate arcs. recip_p > 0 turns each asymmetric pair into a mutual one with
// probability recip_p, decided by a draw keyed on the unordered pair so both
// copies agree.
// Method (no shared counters): every arc yields two entries (row, col << 2 |
// direction bit). Entries are bucketed by row range (P ranges), then each
// range is scattered into its rows, each row is sorted, and the flags of equal
// columns are OR-ed together.
Csr* build_csr(int64_t n, int64_t narcs, const int32_t* src, const int32_t* dst, double recip_p,
               uint64_t recip_seed, int nthreads) {
  Csr* c = new Csr;
  c->n = n;
  const int T = std::max(1, nthreads);
  int shift = 0;
  while ((n >> shift) > 4096) ++shift;  // at most 4097 row ranges
  const int64_t P = (n >> shift) + 1;
  // pass 1: entries per (thread chunk, range)
  std::vector<int64_t> hist((size_t)T * P, 0);
#pragma omp parallel num_threads(T)
  {
    int t = omp_get_thread_num(), nt = omp_get_num_threads();
    int64_t lo = narcs * t / nt, hi = narcs * (t + 1) / nt;
    int64_t* h = &hist[(size_t)t * P];
    for (int64_t i = lo; i < hi; ++i) {
      if (src[i] == dst[i]) continue;
      h[src[i] >> shift]++;
      h[dst[i] >> shift]++;
    }
  }
  std::vector<int64_t> rstart((size_t)P + 1, 0);
  {
    int64_t run = 0;
    for (int64_t r = 0; r < P; ++r) {
      rstart[r] = run;
      for (int t = 0; t < T; ++t) {
        int64_t k = hist[(size_t)t * P + r];
        hist[(size_t)t * P + r] = run;
        run += k;
      }
    }
    rstart[P] = run;
  }
  std::vector<uint64_t> ent((size_t)rstart[P]);
#pragma omp parallel num_threads(T)
  {
    int t = omp_get_thread_num(), nt = omp_get_num_threads();
    int64_t lo = narcs * t / nt, hi = narcs * (t + 1) / nt;
    int64_t* h = &hist[(size_t)t * P];
    for (int64_t i = lo; i < hi; ++i) {
      uint64_t x = (uint32_t)src[i], y = (uint32_t)dst[i];
      if (x == y) continue;
      ent[h[x >> shift]++] = (x << 32) | (y << 2) | 1u;  // row x sees x->y
      ent[h[y >> shift]++] = (y << 32) | (x << 2) | 2u;  // row y sees it incoming
    }
  }
  // pass 2: per range, scatter into rows, sort rows, merge duplicate columns
  std::vector<int64_t> rowlen((size_t)n, 0);
  std::vector<uint32_t> rows((size_t)rstart[P]);
  std::vector<int64_t> rowbeg((size_t)n + 1, 0);
#pragma omp parallel for num_threads(T) schedule(dynamic, 1)
  for (int64_t r = 0; r < P; ++r) {
    int64_t x0 = r << shift, x1 = std::min<int64_t>(n, (r + 1) << shift);
    if (x0 >= x1) continue;
    const int64_t e0 = rstart[r], e1 = rstart[r + 1];
    std::vector<int64_t> cnt((size_t)(x1 - x0) + 1, 0);
    for (int64_t e = e0; e < e1; ++e) cnt[(ent[e] >> 32) - x0 + 1]++;
    for (int64_t k = 0; k < x1 - x0; ++k) cnt[k + 1] += cnt[k];
    for (int64_t x = x0; x < x1; ++x) rowbeg[x] = e0 + cnt[x - x0];
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t e = e0; e < e1; ++e) {
      int64_t x = (int64_t)(ent[e] >> 32);
      rows[e0 + pos[x - x0]++] = (uint32_t)ent[e];
    }
    for (int64_t x = x0; x < x1; ++x) {
      uint32_t* rr = rows.data() + e0 + cnt[x - x0];
      int64_t m = cnt[x - x0 + 1] - cnt[x - x0], w = 0;
      std::sort(rr, rr + m);
      for (int64_t i = 0; i < m;) {
        uint32_t col = rr[i] >> 2, f = 0;
        int64_t j = i;
        while (j < m && (rr[j] >> 2) == col) f |= rr[j++] & 3u;
        if (recip_p > 0 && f != 3) {
          uint64_t lo = std::min<uint64_t>((uint64_t)x, col), hi = std::max<uint64_t>((uint64_t)x, col);
          if (unit(draw(recip_seed, 11, (lo << 32) | hi)) < recip_p) f = 3;
        }
        rr[w++] = (col << 2) | f;
        i = j;
      }
      rowlen[x] = w;
    }
  }
  std::vector<uint64_t>().swap(ent);
  c->off.assign((size_t)n + 1, 0);
  for (int64_t x = 0; x < n; ++x) c->off[x + 1] = c->off[x] + rowlen[x];
  const int64_t nnz = c->off[n];
  c->nbr.resize(nnz);
  c->flg.assign((size_t)((nnz + 3) / 4), 0);
#pragma omp parallel for num_threads(T) schedule(dynamic, 4096)
  for (int64_t x = 0; x < n; ++x) {
    const uint32_t* r = rows.data() + rowbeg[x];
    for (int64_t i = 0; i < rowlen[x]; ++i) c->nbr[c->off[x] + i] = (int32_t)(r[i] >> 2);
  }
  // packed flags: each thread owns whole bytes (4 entries each)
#pragma omp parallel for num_threads(T) schedule(static)
  for (int64_t blk = 0; blk < (n + 4095) / 4096; ++blk) {
    int64_t x0 = blk * 4096, x1 = std::min<int64_t>(n, x0 + 4096);
    for (int64_t x = x0; x < x1; ++x) {
      const uint32_t* r = rows.data() + rowbeg[x];
      for (int64_t i = 0; i < rowlen[x]; ++i) {
        int64_t e = c->off[x] + i;
        __atomic_fetch_or(&c->flg[e >> 2], (uint8_t)((r[i] & 3u) << (2 * (e & 3))), __ATOMIC_RELAXED);
      }
    }
  }
  return c;
}

// Walker alias table for sampling index i with probability w[i]/sum(w).
struct Alias {
  std::vector<double> prob;
  std::vector<int32_t> alias;
  explicit Alias(const std::vector<double>& w) {
    int64_t n = (int64_t)w.size();
    prob.resize(n);
    alias.resize(n);
    double s = 0;
    for (double x : w) s += x;
    std::vector<double> p(n);
    std::vector<int64_t> small, large;
    for (int64_t i = 0; i < n; ++i) {
      p[i] = w[i] * n / s;
      (p[i] < 1.0 ? small : large).push_back(i);
    }
    while (!small.empty() && !large.empty()) {
      int64_t s_ = small.back(); small.pop_back();
      int64_t l_ = large.back(); large.pop_back();
      prob[s_] = p[s_];
      alias[s_] = (int32_t)l_;
      p[l_] = (p[l_] + p[s_]) - 1.0;
      (p[l_] < 1.0 ? small : large).push_back(l_);
    }
    for (int64_t i : large) { prob[i] = 1.0; alias[i] = (int32_t)i; }
    for (int64_t i : small) { prob[i] = 1.0; alias[i] = (int32_t)i; }
  }
  int32_t sample(uint64_t r1, uint64_t r2) const {
    int64_t n = (int64_t)prob.size();
    int64_t i = (int64_t)((unsigned __int128)r1 * (uint64_t)n >> 64);
    return unit(r2) < prob[i] ? (int32_t)i : alias[i];
  }
};

// Chung-Lu weights w_i = w0 * ((i + i0) / i0)^(-1/(gamma-1)), with i0 found by
// bisection so that the mean weight equals mean_deg.
std::vector<double> chung_lu_weights(int64_t n, double gamma, double mean_deg, double w0) {
  const double e = -1.0 / (gamma - 1.0);
  // Sum in fixed blocks added in block order, so the result does not depend
  // on the number of threads.
  const int64_t BS = 65536, nb = (n + BS - 1) / BS;
  std::vector<double> part((size_t)nb);
  auto mean_for = [&](double i0) {
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
      double s = 0;
      int64_t hi = std::min(n, (b + 1) * BS);
      for (int64_t i = b * BS; i < hi; ++i) s += w0 * std::pow((i + i0) / i0, e);
      part[b] = s;
    }
    double s = 0;
    for (int64_t b = 0; b < nb; ++b) s += part[b];
    return s / (double)n;
  };
  double lo = 1e-9, hi = 1e15;
  for (int it = 0; it < 200; ++it) {
    double mid = std::sqrt(lo * hi);
    if (mean_for(mid) < mean_deg) lo = mid; else hi = mid;
    if (hi / lo < 1.0 + 1e-12) break;
  }
  double i0 = std::sqrt(lo * hi);
  std::vector<double> w((size_t)n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) w[i] = w0 * std::pow((i + i0) / i0, e);
  return w;
}

// Random permutation of [0,n) by Fisher-Yates with counter-based draws.
std::vector<int32_t> permutation(int64_t n, uint64_t seed, uint64_t stream) {
  std::vector<int32_t> p((size_t)n);
  for (int64_t i = 0; i < n; ++i) p[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    uint64_t r = draw(seed, stream, (uint64_t)i);
    int64_t j = (int64_t)((unsigned __int128)r * (uint64_t)(i + 1) >> 64);
    std::swap(p[i], p[j]);
  }
  return p;
}

// Open-addressing set of unordered vertex pairs (key = lo<<32|hi, never ~0).
struct PairSet {
  std::vector<uint64_t> slot;
  uint64_t mask;
  static constexpr uint64_t EMPTY = ~0ull;
  explicit PairSet(int64_t cap) {
    uint64_t s = 16;
    while (s < (uint64_t)cap * 2 + 16) s <<= 1;
    slot.assign(s, EMPTY);
    mask = s - 1;
  }
  static uint64_t key(uint32_t a, uint32_t b) {
    uint64_t lo = std::min(a, b), hi = std::max(a, b);
    return (lo << 32) | hi;
  }
  uint64_t h(uint64_t k) const { return mix64(k) & mask; }
  bool has(uint64_t k) const {
    for (uint64_t i = h(k);; i = (i + 1) & mask) {
      if (slot[i] == k) return true;
      if (slot[i] == EMPTY) return false;
    }
  }
  void add(uint64_t k) {
    uint64_t i = h(k);
    while (slot[i] != EMPTY && slot[i] != k) i = (i + 1) & mask;
    slot[i] = k;
  }
  void del(uint64_t k) {  // backward-shift deletion
    uint64_t i = h(k);
    while (slot[i] != k) {
      if (slot[i] == EMPTY) return;
      i = (i + 1) & mask;
    }
    uint64_t j = i;
    for (;;) {
      slot[i] = EMPTY;
      for (;;) {
        j = (j + 1) & mask;
        if (slot[j] == EMPTY) return;
        uint64_t k2 = h(slot[j]);
        // slot[j] may move to i if its home k2 is not cyclically in (i, j]
        bool in_range = (i <= j) ? (i < k2 && k2 <= j) : (i < k2 || k2 <= j);
        if (!in_range) break;
      }
      slot[i] = slot[j];
      i = j;
    }
  }
};

// Distinct arcs (no self-loops) of an arc list, sorted by (src,dst).
void dedup_arcs(std::vector<uint32_t>& s, std::vector<uint32_t>& d) {
  std::vector<uint64_t> k;
  k.reserve(s.size());
  for (size_t i = 0; i < s.size(); ++i)
    if (s[i] != d[i]) k.push_back(((uint64_t)s[i] << 32) | d[i]);
  std::sort(k.begin(), k.end());
  k.erase(std::unique(k.begin(), k.end()), k.end());
  s.resize(k.size());
  d.resize(k.size());
  for (size_t i = 0; i < k.size(); ++i) { s[i] = (uint32_t)(k[i] >> 32); d[i] = (uint32_t)k[i]; }
}

// Degree-preserving double-edge swaps on a simple digraph given as distinct
// arcs. Asymmetric arcs swap with asymmetric arcs (a->b, c->d => a->d, c->b)
// and mutual dyads with mutual dyads ({a,b},{c,d} => {a,d},{c,b}); a swap is
// accepted only if both new vertex pairs are unconnected in either direction.
// In-, out- and mutual degrees are preserved. Returns accepted swaps.
int64_t swap_arcs(std::vector<uint32_t>& s, std::vector<uint32_t>& d, int64_t attempts, uint64_t seed) {
  // split into asymmetric arcs and mutual dyads (a<b)
  PairSet all((int64_t)s.size());
  std::vector<uint64_t> arcset(s.size());
  for (size_t i = 0; i < s.size(); ++i) arcset[i] = ((uint64_t)s[i] << 32) | d[i];
  std::sort(arcset.begin(), arcset.end());
  auto has_arc = [&](uint32_t a, uint32_t b) {
    return std::binary_search(arcset.begin(), arcset.end(), ((uint64_t)a << 32) | b);
  };
  std::vector<uint32_t> as, ad, ma, mb;
  for (size_t i = 0; i < s.size(); ++i) {
    uint32_t a = s[i], b = d[i];
    all.add(PairSet::key(a, b));
    if (has_arc(b, a)) {
      if (a < b) { ma.push_back(a); mb.push_back(b); }
    } else {
      as.push_back(a); ad.push_back(b);
    }
  }
  int64_t acc = 0;
  const int64_t na = (int64_t)as.size(), nm = (int64_t)ma.size();
  const int64_t tot = na + nm;
  if (tot < 2) return 0;
  auto pick = [](uint64_t r, int64_t m) { return (int64_t)((unsigned __int128)r * (uint64_t)m >> 64); };
  for (int64_t t = 0; t < attempts; ++t) {
    uint64_t r0 = draw(seed, 21, (uint64_t)t * 4), r1 = draw(seed, 21, (uint64_t)t * 4 + 1);
    uint64_t r2 = draw(seed, 21, (uint64_t)t * 4 + 2);
    bool mutual = pick(r0, tot) >= na;  // class chosen in proportion to its size
    if (!mutual) {
      if (na < 2) continue;
      int64_t i = pick(r1, na), j = pick(r2, na);
      if (i == j) continue;
      uint32_t a = as[i], b = ad[i], c = as[j], e = ad[j];
      if (a == c || a == e || b == c || b == e) continue;
      uint64_t k1 = PairSet::key(a, e), k2 = PairSet::key(c, b);
      if (k1 == k2 || all.has(k1) || all.has(k2)) continue;
      all.del(PairSet::key(a, b)); all.del(PairSet::key(c, e));
      all.add(k1); all.add(k2);
      ad[i] = e; ad[j] = b;
      ++acc;
    } else {
      if (nm < 2) continue;
      int64_t i = pick(r1, nm), j = pick(r2, nm);
      if (i == j) continue;
      uint32_t a = ma[i], b = mb[i], c = ma[j], e = mb[j];
      if (draw(seed, 22, (uint64_t)t) & 1) std::swap(c, e);  // random orientation of the 2nd dyad
      if (a == c || a == e || b == c || b == e) continue;
      uint64_t k1 = PairSet::key(a, e), k2 = PairSet::key(c, b);
      if (k1 == k2 || all.has(k1) || all.has(k2)) continue;
      all.del(PairSet::key(a, b)); all.del(PairSet::key(c, e));
      all.add(k1); all.add(k2);
      ma[i] = std::min(a, e); mb[i] = std::max(a, e);
      ma[j] = std::min(c, b); mb[j] = std::max(c, b);
      ++acc;
    }
  }
  s.clear(); d.clear();
  for (int64_t i = 0; i < na; ++i) { s.push_back(as[i]); d.push_back(ad[i]); }
  for (int64_t i = 0; i < nm; ++i) {
    s.push_back(ma[i]); d.push_back(mb[i]);
    s.push_back(mb[i]); d.push_back(ma[i]);
  }
  return acc;
}

// One member of the null-model ensemble: parameters and arcs from seed g.
struct BatchMember {
  int64_t n;
  std::vector<uint32_t> s, d;
  double mean, recip, gamma;
  int kind;  // 0 = Erdos-Renyi, 1 = Chung-Lu
};

void make_member(BatchMember& M, uint64_t seed, uint64_t g, int64_t nmin, int64_t nmax, double dmin,
                 double dmax, double rmax, double swap_factor) {
  uint64_t gs = mix64(seed * G2 + g + 1);
  M.kind = (int)(g & 1);
  M.n = nmin + (int64_t)((unsigned __int128)draw(gs, 1, 0) * (uint64_t)(nmax - nmin + 1) >> 64);
  M.mean = dmin + (dmax - dmin) * unit(draw(gs, 1, 1));
  M.recip = rmax * unit(draw(gs, 1, 2));
  M.gamma = 2.1 + 0.9 * unit(draw(gs, 1, 3));
  const int64_t n = M.n;
  const int64_t m = (int64_t)std::llround(M.mean * (double)n);
  M.s.resize(m);
  M.d.resize(m);
  if (M.kind == 0) {
    for (int64_t i = 0; i < m; ++i) {
      uint64_t r1 = draw(gs, 2, 2 * i), r2 = draw(gs, 2, 2 * i + 1);
      M.s[i] = (uint32_t)((unsigned __int128)r1 * (uint64_t)n >> 64);
      M.d[i] = (uint32_t)((unsigned __int128)r2 * (uint64_t)n >> 64);
    }
  } else {
    std::vector<double> w = chung_lu_weights(n, M.gamma, M.mean, std::sqrt((double)n * M.mean));
    Alias al(w);
    std::vector<int32_t> perm = permutation(n, gs, 3);
    for (int64_t i = 0; i < m; ++i) {
      M.s[i] = (uint32_t)al.sample(draw(gs, 4, 4 * i), draw(gs, 4, 4 * i + 1));
      M.d[i] = (uint32_t)perm[al.sample(draw(gs, 4, 4 * i + 2), draw(gs, 4, 4 * i + 3))];
    }
  }
  dedup_arcs(M.s, M.d);
  // reciprocate a fraction of arcs at construction
  {
    std::vector<uint64_t> have(M.s.size());
    for (size_t i = 0; i < M.s.size(); ++i) have[i] = ((uint64_t)M.s[i] << 32) | M.d[i];
    // have is sorted by dedup_arcs
    size_t m0 = M.s.size();
    for (size_t i = 0; i < m0; ++i) {
      uint32_t a = M.s[i], b = M.d[i];
      if (std::binary_search(have.begin(), have.end(), ((uint64_t)b << 32) | a)) continue;
      if (unit(draw(gs, 5, i)) < M.recip) { M.s.push_back(b); M.d.push_back(a); }
    }
    dedup_arcs(M.s, M.d);
  }
  int64_t attempts = (int64_t)std::llround(swap_factor * (double)M.s.size());
  swap_arcs(M.s, M.d, attempts, mix64(gs + 77));
}

}  // namespace

extern "C" {

// R-MAT (Chakrabarti, Zhan, Faloutsos 2004): for arc i, at each of `scale`
// levels (most significant bit first) pick a quadrant with probabilities
// (a, b, c, 1-a-b-c): a=(0,0) b=(0,1) c=(1,0) d=(1,1) for (src bit, dst bit).
// Each 64-bit draw is cut into four 16-bit uniforms, one per level.
// No noise and no vertex permutation. Returns narcs (self-loops and duplicates
// are kept here and removed by the CSR builder).
int64_t tg_rmat(int scale, int64_t narcs, double a, double b, double c, uint64_t seed, int32_t* src,
                int32_t* dst, int nthreads) {
  const uint32_t ta = (uint32_t)std::llround(a * 65536.0);
  const uint32_t tb = (uint32_t)std::llround((a + b) * 65536.0);
  const uint32_t tc = (uint32_t)std::llround((a + b + c) * 65536.0);
#pragma omp parallel for num_threads(std::max(1, nthreads)) schedule(static)
  for (int64_t i = 0; i < narcs; ++i) {
    uint32_t x = 0, y = 0;
    uint64_t r = 0;
    for (int l = 0; l < scale; ++l) {
      if ((l & 3) == 0) r = draw(seed, 1, (uint64_t)i * 16 + (uint64_t)(l >> 2));
      uint32_t q = (uint32_t)(r & 0xFFFF);
      r >>= 16;
      uint32_t bx = (q >= tb) ? 1u : 0u;
      uint32_t by = (q >= ta && q < tb) || (q >= tc) ? 1u : 0u;
      x = (x << 1) | bx;
      y = (y << 1) | by;
    }
    src[i] = (int32_t)x;
    dst[i] = (int32_t)y;
  }
  return narcs;
}

// Chung-Lu directed graph: narcs arcs, source drawn with probability
// proportional to w_i, target proportional to w under an independent random
// permutation of the ids. Weights as in chung_lu_weights (max weight w0).
int64_t tg_chung_lu(int64_t n, double gamma, double mean_deg, double w0, int64_t narcs, uint64_t seed,
                    int32_t* src, int32_t* dst, int nthreads) {
  std::vector<double> w = chung_lu_weights(n, gamma, mean_deg, w0);
  Alias al(w);
  std::vector<int32_t> perm = permutation(n, seed, 3);
#pragma omp parallel for num_threads(std::max(1, nthreads)) schedule(static)
  for (int64_t i = 0; i < narcs; ++i) {
    src[i] = al.sample(draw(seed, 4, 4 * (uint64_t)i), draw(seed, 4, 4 * (uint64_t)i + 1));
    dst[i] = perm[al.sample(draw(seed, 4, 4 * (uint64_t)i + 2), draw(seed, 4, 4 * (uint64_t)i + 3))];
  }
  return narcs;
}

// Uniform random arcs (Erdos-Renyi G(n, M) with replacement; self-loops and
// duplicates are removed by the CSR builder).
int64_t tg_erdos_renyi(int64_t n, int64_t narcs, uint64_t seed, int32_t* src, int32_t* dst) {
  for (int64_t i = 0; i < narcs; ++i) {
    src[i] = (int32_t)((unsigned __int128)draw(seed, 2, 2 * (uint64_t)i) * (uint64_t)n >> 64);
    dst[i] = (int32_t)((unsigned __int128)draw(seed, 2, 2 * (uint64_t)i + 1) * (uint64_t)n >> 64);
  }
  return narcs;
}

// Degree-preserving swaps on an arc list (must be distinct arcs, no
// self-loops). Rewrites src/dst in place (same count); returns accepted swaps.
int64_t tg_swap(int64_t narcs, int32_t* src, int32_t* dst, int64_t attempts, uint64_t seed) {
  std::vector<uint32_t> s(narcs), d(narcs);
  for (int64_t i = 0; i < narcs; ++i) { s[i] = (uint32_t)src[i]; d[i] = (uint32_t)dst[i]; }
  int64_t acc = swap_arcs(s, d, attempts, seed);
  for (int64_t i = 0; i < narcs; ++i) { src[i] = (int32_t)s[i]; dst[i] = (int32_t)d[i]; }
  return acc;
}

// K degree-preserving randomisations of one arc list (copy k from the seed
// stream (seed, k)), copy k written to out_src/out_dst[k * narcs ...].
int64_t tg_swap_ensemble(int64_t narcs, const int32_t* src, const int32_t* dst, int32_t K, int64_t attempts,
                         uint64_t seed, int32_t* out_src, int32_t* out_dst, int nthreads) {
  int64_t acc = 0;
#pragma omp parallel for num_threads(std::max(1, nthreads)) schedule(dynamic, 1) reduction(+ : acc)
  for (int32_t k = 0; k < K; ++k) {
    std::vector<uint32_t> s(narcs), d(narcs);
    for (int64_t i = 0; i < narcs; ++i) { s[i] = (uint32_t)src[i]; d[i] = (uint32_t)dst[i]; }
    acc += swap_arcs(s, d, attempts, mix64(seed * 0x9e3779b97f4a7c15ull + (uint64_t)k + 1));
    for (int64_t i = 0; i < narcs; ++i) {
      out_src[(int64_t)k * narcs + i] = (int32_t)s[i];
      out_dst[(int64_t)k * narcs + i] = (int32_t)d[i];
    }
  }
  return acc;
}

void* tg_csr_build(int64_t n, int64_t narcs, const int32_t* src, const int32_t* dst, double recip_p,
                   uint64_t recip_seed, int nthreads) {
  return build_csr(n, narcs, src, dst, recip_p, recip_seed, nthreads);
}
int64_t tg_csr_nnz(void* h) { return (int64_t)static_cast<Csr*>(h)->nbr.size(); }
void tg_csr_fetch(void* h, int64_t* offsets, int32_t* nbrs, uint8_t* flags) {
  Csr* c = static_cast<Csr*>(h);
  std::memcpy(offsets, c->off.data(), sizeof(int64_t) * c->off.size());
  if (!c->nbr.empty()) std::memcpy(nbrs, c->nbr.data(), sizeof(int32_t) * c->nbr.size());
  if (!c->flg.empty()) std::memcpy(flags, c->flg.data(), c->flg.size());
}
void tg_csr_free(void* h) { delete static_cast<Csr*>(h); }

// Null-model ensemble: G graphs, graph g from seed (seed, g). Half Erdos-Renyi
// (even g), half Chung-Lu (odd g, exponent ~ U[2.1, 3.0], max weight
// sqrt(n*mean)). n ~ U[nmin, nmax], mean out-degree ~ U[dmin, dmax],
// reciprocity ~ U[0, rmax] (fraction of arcs reciprocated at construction),
// then swap_factor * arcs double-edge-swap attempts.
// Output: concatenated CSR; graph g owns rows [vbase[g], vbase[g+1]) and its
// neighbour ids are graph-local; offsets are global entry positions.
struct Batch {
  std::vector<int64_t> vbase, off;
  std::vector<int32_t> nbr;
  std::vector<uint8_t> flg;
  std::vector<double> params;  // per graph: kind, n, mean, recip, gamma, arcs
};
void* tg_batch_build(int32_t G, uint64_t seed, int64_t nmin, int64_t nmax, double dmin, double dmax,
                     double rmax, double swap_factor, int nthreads) {
  std::vector<Csr*> parts(G);
  Batch* B = new Batch;
  B->params.resize((size_t)G * 6);
#pragma omp parallel for num_threads(std::max(1, nthreads)) schedule(dynamic, 1)
  for (int32_t g = 0; g < G; ++g) {
    BatchMember M;
    make_member(M, seed, (uint64_t)g, nmin, nmax, dmin, dmax, rmax, swap_factor);
    std::vector<int32_t> s(M.s.begin(), M.s.end()), d(M.d.begin(), M.d.end());
    parts[g] = build_csr(M.n, (int64_t)s.size(), s.data(), d.data(), 0.0, 0, 1);
    double* p = &B->params[(size_t)g * 6];
    p[0] = M.kind; p[1] = (double)M.n; p[2] = M.mean; p[3] = M.recip; p[4] = M.gamma; p[5] = (double)s.size();
  }
  B->vbase.assign((size_t)G + 1, 0);
  int64_t nnz = 0;
  for (int32_t g = 0; g < G; ++g) {
    B->vbase[g + 1] = B->vbase[g] + parts[g]->n;
    nnz += (int64_t)parts[g]->nbr.size();
  }
  B->off.assign((size_t)B->vbase[G] + 1, 0);
  B->nbr.resize(nnz);
  B->flg.assign((size_t)((nnz + 3) / 4), 0);
  int64_t e0 = 0;
  for (int32_t g = 0; g < G; ++g) {
    Csr* c = parts[g];
    int64_t vb = B->vbase[g];
    for (int64_t x = 0; x <= c->n; ++x) B->off[vb + x] = e0 + c->off[x];
    for (size_t i = 0; i < c->nbr.size(); ++i) {
      int64_t e = e0 + (int64_t)i;
      B->nbr[e] = c->nbr[i];
      uint8_t f = (c->flg[i >> 2] >> (2 * (i & 3))) & 3;
      B->flg[e >> 2] |= (uint8_t)(f << (2 * (e & 3)));
    }
    e0 += (int64_t)c->nbr.size();
    delete c;
  }
  return B;
}
int64_t tg_batch_nv(void* h) { return static_cast<Batch*>(h)->vbase.back(); }
int64_t tg_batch_nnz(void* h) { return (int64_t)static_cast<Batch*>(h)->nbr.size(); }
void tg_batch_fetch(void* h, int64_t* vbase, int64_t* offsets, int32_t* nbrs, uint8_t* flags, double* params) {
  Batch* B = static_cast<Batch*>(h);
  std::memcpy(vbase, B->vbase.data(), sizeof(int64_t) * B->vbase.size());
  std::memcpy(offsets, B->off.data(), sizeof(int64_t) * B->off.size());
  if (!B->nbr.empty()) std::memcpy(nbrs, B->nbr.data(), sizeof(int32_t) * B->nbr.size());
  if (!B->flg.empty()) std::memcpy(flags, B->flg.data(), B->flg.size());
  std::memcpy(params, B->params.data(), sizeof(double) * B->params.size());
}
void tg_batch_free(void* h) { delete static_cast<Batch*>(h); }

// 64-bit content hash of a byte buffer (SplitMix64 over 8-byte words, chained).
uint64_t tg_hash(const void* p, int64_t nbytes, uint64_t h) {
  const uint8_t* b = static_cast<const uint8_t*>(p);
  int64_t i = 0;
  for (; i + 8 <= nbytes; i += 8) {
    uint64_t w;
    std::memcpy(&w, b + i, 8);
    h = mix64(h ^ (w + G1 + (uint64_t)i));
  }
  uint64_t w = 0;
  for (int64_t k = 0; i + k < nbytes; ++k) w |= (uint64_t)b[i + k] << (8 * k);
  return mix64(h ^ (w + G2 + (uint64_t)nbytes));
}

}  // extern "C"
