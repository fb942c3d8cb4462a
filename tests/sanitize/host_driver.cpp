// Sanitizer driver for the library's host code (csrc/host.cpp: contract
// validation, class tables, the 128-bit null count) and the seeded input
// generators (gen/graphgen.cpp), built with -fsanitize=address,undefined by
// tests/test_sanitizers.py. Generated graphs go through the CSR builder and
// host validation; mutated copies must give each documented status; the
// tables must agree with the classifier they are built from.
// Exit status: the number of failed checks (0 = all pass).
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "triad_internal.h"

extern "C" {
int64_t tg_rmat(int scale, int64_t narcs, double a, double b, double c, uint64_t seed, int32_t* src, int32_t* dst,
                int nthreads);
int64_t tg_erdos_renyi(int64_t n, int64_t narcs, uint64_t seed, int32_t* src, int32_t* dst);
int64_t tg_swap_ensemble(int64_t narcs, const int32_t* src, const int32_t* dst, int32_t K, int64_t attempts,
                         uint64_t seed, int32_t* out_src, int32_t* out_dst, int nthreads);
void* tg_csr_build(int64_t n, int64_t narcs, const int32_t* src, const int32_t* dst, double recip_p,
                   uint64_t recip_seed, int nthreads);
int64_t tg_csr_nnz(void* h);
void tg_csr_fetch(void* h, int64_t* offsets, int32_t* nbrs, uint8_t* flags);
void tg_csr_free(void* h);
void* tg_batch_build(int32_t G, uint64_t seed, int64_t nmin, int64_t nmax, double dmin, double dmax, double rmax,
                     double swap_factor, int nthreads);
int64_t tg_batch_nv(void* h);
int64_t tg_batch_nnz(void* h);
void tg_batch_fetch(void* h, int64_t* vbase, int64_t* offsets, int32_t* nbrs, uint8_t* flags, double* params);
void tg_batch_free(void* h);
uint64_t tg_hash(const void* p, int64_t nbytes, uint64_t h);
}

static int bad = 0;
static void check(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "failed: %s\n", what);
    ++bad;
  }
}

struct Graph {
  int64_t n = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> nbr;
  std::vector<uint8_t> flg;
};

static Graph csr(int64_t n, const std::vector<int32_t>& s, const std::vector<int32_t>& d, double recip) {
  void* h = tg_csr_build(n, (int64_t)s.size(), s.data(), d.data(), recip, 7, 4);
  Graph g;
  g.n = n;
  const int64_t nnz = tg_csr_nnz(h);
  g.off.resize(n + 1);
  g.nbr.resize(nnz);
  g.flg.resize((nnz + 3) / 4);
  tg_csr_fetch(h, g.off.data(), g.nbr.data(), g.flg.data());
  tg_csr_free(h);
  return g;
}

static int validate(const Graph& g, int level) {
  return triad_validate_host(g.n, g.off.data(), g.nbr.data(), g.flg.data(), level);
}

int main() {
  // generated graphs pass full validation
  const int scale = 11;
  const int64_t n = 1 << scale, narcs = 8 * n;
  std::vector<int32_t> s(narcs), d(narcs);
  tg_rmat(scale, narcs, 0.57, 0.19, 0.19, 1, s.data(), d.data(), 4);
  Graph g = csr(n, s, d, 0.2);
  check(validate(g, 1) == TRIAD_OK, "R-MAT CSR validates");
  std::vector<int32_t> es(4000), ed(4000);
  tg_erdos_renyi(300, 4000, 3, es.data(), ed.data());
  Graph ge = csr(300, es, ed, 0.0);
  check(validate(ge, 1) == TRIAD_OK, "Erdos-Renyi CSR validates");
  // randomised copies of a simple digraph keep every vertex's in- and out-degree
  std::vector<int32_t> ss, sd;
  {
    std::vector<uint64_t> keys;
    for (size_t i = 0; i < es.size(); ++i)
      if (es[i] != ed[i]) keys.push_back((uint64_t)es[i] << 32 | (uint32_t)ed[i]);
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    for (uint64_t k : keys) ss.push_back((int32_t)(k >> 32)), sd.push_back((int32_t)(k & 0xffffffffu));
  }
  const int K = 3;
  const int64_t m = (int64_t)ss.size();
  std::vector<int32_t> os(K * m), od(K * m);
  check(tg_swap_ensemble(m, ss.data(), sd.data(), K, 10 * m, 5, os.data(), od.data(), 4) > 0, "swaps accepted");
  for (int k = 0; k < K; ++k) {
    std::vector<int64_t> dout(300, 0), din(300, 0);
    for (int64_t i = 0; i < m; ++i) {
      dout[os[k * m + i]]++, din[od[k * m + i]]++;
      dout[ss[i]]--, din[sd[i]]--;
    }
    bool same = true;
    for (int v = 0; v < 300; ++v) same &= dout[v] == 0 && din[v] == 0;
    check(same, "swap ensemble keeps degrees");
  }
  // a batch: every member validates on its own rows
  void* B = tg_batch_build(16, 9, 64, 400, 2.0, 12.0, 0.3, 5.0, 4);
  const int64_t nv = tg_batch_nv(B), bnnz = tg_batch_nnz(B);
  std::vector<int64_t> vb(17), boff(nv + 1);
  std::vector<int32_t> bnb(bnnz);
  std::vector<uint8_t> bfl((bnnz + 3) / 4);
  std::vector<double> params(16 * 6);
  tg_batch_fetch(B, vb.data(), boff.data(), bnb.data(), bfl.data(), params.data());
  tg_batch_free(B);
  for (int m = 0; m < 16; ++m) {
    Graph x;
    x.n = vb[m + 1] - vb[m];
    const int64_t e0 = boff[vb[m]], e1 = boff[vb[m + 1]];
    for (int64_t r = 0; r <= x.n; ++r) x.off.push_back(boff[vb[m] + r] - e0);
    x.nbr.assign(bnb.begin() + e0, bnb.begin() + e1);
    for (int64_t j = e0; j < e1; ++j) {
      if (((j - e0) & 3) == 0) x.flg.push_back(0);
      x.flg.back() |= (uint8_t)(((bfl[j >> 2] >> (2 * (j & 3))) & 3u) << (2 * ((j - e0) & 3)));
    }
    check(validate(x, 1) == TRIAD_OK, "batch member validates");
  }
  check(tg_hash(g.nbr.data(), (int64_t)g.nbr.size() * 4, 1) == tg_hash(g.nbr.data(), (int64_t)g.nbr.size() * 4, 1),
        "hash is deterministic");
  // mutated copies: each documented status
  {
    Graph x = g;
    int64_t r = 0;
    while (x.off[r + 1] - x.off[r] < 2) ++r;
    std::swap(x.nbr[x.off[r]], x.nbr[x.off[r] + 1]);
    check(validate(x, 0) == TRIAD_EUNSORTED, "unsorted row");
  }
  {
    Graph x = g;
    x.nbr[x.nbr.size() / 2] = (int32_t)n;
    check(validate(x, 0) == TRIAD_ERANGE, "id out of range");
  }
  {
    Graph x = g;
    int64_t r = 0;
    while (x.off[r + 1] == x.off[r]) ++r;
    x.flg[x.off[r] >> 2] &= (uint8_t)~(3u << (2 * (x.off[r] & 3)));
    check(validate(x, 0) == TRIAD_ERANGE, "zero flag");
  }
  {
    Graph x = g;
    int64_t r = 0;
    while (x.off[r + 1] == x.off[r] || x.nbr[x.off[r]] < r) ++r;
    x.nbr[x.off[r]] = (int32_t)r;  // the row's smallest id above r becomes r itself
    check(validate(x, 0) == TRIAD_ESELFLOOP, "self-loop");
  }
  {
    Graph x = g;
    const int64_t j = x.off[5];
    const unsigned f = (x.flg[j >> 2] >> (2 * (j & 3))) & 3u;
    if (f != 3u) {
      x.flg[j >> 2] ^= (uint8_t)(3u << (2 * (j & 3)));  // 1 <-> 2: no longer mirrored
      check(validate(x, 0) == TRIAD_OK && validate(x, 1) == TRIAD_EASYM, "flags not mirrored");
    }
  }
  {
    Graph x = g;
    x.off[3] = x.off[4] + 1;
    check(validate(x, 0) == TRIAD_ERANGE, "offsets not monotone");
    check(triad_validate_host(-1, g.off.data(), g.nbr.data(), g.flg.data(), 0) == TRIAD_EINVAL, "negative n");
  }
  // tables against the classifier they come from
  const triad::ClassSlices cs = triad::class_slices();
  for (unsigned f = 1; f < 4; ++f)
    for (unsigned idx = 1; idx < 16; ++idx) {
      const unsigned fa = idx & 3u, fb = idx >> 2;
      check(((cs.s[f] >> (4 * idx)) & 15u) == (unsigned)triad::classify_code(f | fa << 2 | fb << 4),
            "class slice entry");
    }
  int hist[16] = {0};
  for (unsigned c = 0; c < 64; ++c) hist[triad::classify_code(c)]++;
  const int sizes[16] = {1, 6, 3, 3, 3, 6, 6, 6, 6, 2, 3, 3, 3, 6, 6, 1};
  for (int t = 0; t < 16; ++t) check(hist[t] == sizes[t], "class sizes of the 64 states");
  const triad::LabTables lt = triad::lab_tables();
  check(lt.ga_hi[0] != 0 && lt.gb_hi[1] != 0, "labelled tables filled");
  uint64_t lo, hi;
  triad::choose3(4801281, &lo, &hi);
  check(hi == 1, "C(4801281, 3) exceeds 2^64");
  triad::choose3(4801280, &lo, &hi);
  check(hi == 0 && lo == (uint64_t)((unsigned __int128)4801280 * 4801279 * 4801278 / 6), "C(4801280, 3)");
  std::printf("host driver: %d failed check(s)\n", bad);
  return bad;
}
