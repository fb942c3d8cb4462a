// Host-side parts of the census library: error reporting, the 64-state class
// table, the 128-bit null count and host validation of the input contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "triad_internal.h"

namespace triad {

static thread_local std::string g_err;
static std::atomic<int64_t> g_mem_cap{0};
static std::atomic<int32_t> g_inject{0};

int64_t memory_cap() { return g_mem_cap.load(std::memory_order_relaxed); }

bool take_injected_fault() {
  int32_t k = g_inject.load();
  while (k > 0)
    if (g_inject.compare_exchange_weak(k, k - 1)) return true;
  return false;
}

// Held device blocks (see held_take): per device, free blocks by size. The
// table is never destroyed, so that nothing calls into HIP during static
// destruction at process exit (the blocks die with the process).
namespace {
struct HeldBlocks {
  std::mutex mu;
  std::multimap<size_t, void*> free[64];
  size_t bytes[64] = {};
};
HeldBlocks& held_blocks() {
  static HeldBlocks* h = new HeldBlocks;
  return *h;
}
// requests of 1 MiB and more are rounded up to whole MiB, smaller ones to 256 B
size_t block_size(size_t b) {
  const size_t g = b >= ((size_t)1 << 20) ? ((size_t)1 << 20) : 256;
  return (b + g - 1) / g * g;
}
size_t release_device(int dev) {
  HeldBlocks& h = held_blocks();
  std::multimap<size_t, void*> out;
  {
    std::lock_guard<std::mutex> lk(h.mu);
    out.swap(h.free[dev]);
    h.bytes[dev] = 0;
  }
  size_t freed = 0;
  for (const auto& b : out) {
    (void)hipFree(b.second);
    freed += b.first;
  }
  return freed;
}
}  // namespace

hipError_t held_take(void** p, size_t bytes, size_t* got) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  HeldBlocks& h = held_blocks();
  const size_t want = block_size(bytes);
  {
    std::lock_guard<std::mutex> lk(h.mu);
    auto& m = h.free[dev];
    auto it = m.lower_bound(want);
    if (it != m.end() && it->first / 2 <= want) {
      *p = it->second;
      *got = it->first;
      h.bytes[dev] -= it->first;
      m.erase(it);
      return hipSuccess;
    }
  }
  e = hipMalloc(p, want);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    release_device(dev);
    e = hipMalloc(p, want);
  }
  if (e == hipSuccess) *got = want;
  return e;
}

void held_give(void* p, size_t bytes, int dev) {
  if (dev >= 0 && dev < 64) {
    HeldBlocks& h = held_blocks();
    std::lock_guard<std::mutex> lk(h.mu);
    if (h.bytes[dev] + bytes <= HELD_LIMIT) {
      h.free[dev].emplace(bytes, p);
      h.bytes[dev] += bytes;
      return;
    }
  }
  (void)hipFree(p);
}

size_t held_release_all() {
  size_t freed = 0;
  for (int d = 0; d < 64; ++d) freed += release_device(d);
  return freed;
}

size_t held_bytes() {
  HeldBlocks& h = held_blocks();
  std::lock_guard<std::mutex> lk(h.mu);
  size_t t = 0;
  for (int d = 0; d < 64; ++d) t += h.bytes[d];
  return t;
}

void set_error(const std::string& msg) { g_err = msg; }
int fail(int status, const std::string& msg) {
  g_err = msg;
  return status;
}

int status_from_bits(uint32_t bits) {
  if (bits & ERR_RANGE) return TRIAD_ERANGE;
  if (bits & ERR_SELFLOOP) return TRIAD_ESELFLOOP;
  if (bits & ERR_UNSORTED) return TRIAD_EUNSORTED;
  if (bits & ERR_ASYM) return TRIAD_EASYM;
  if (bits & ERR_DEVICE) return TRIAD_EDEVICE;
  return TRIAD_OK;
}

// Class of a 6-bit triad state. Bits: 0 u->v, 1 v->u, 2 u->w, 3 w->u,
// 4 v->w, 5 w->v. The class follows from the number of mutual (M) and
// asymmetric (A) vertex pairs plus the in/out degrees inside the triad
// (Holland-Leinhardt M-A-N naming; Sec. 3 of the paper):
//   021: a vertex sending both arcs = D, receiving both = U, else C
//   111: a vertex receiving two arcs = D (A<->B<-C), else U (A<->B->C)
//   030: a vertex sending two arcs = T, else C (cycle)
//   120: the vertex outside the mutual pair sends both = D, receives both = U, else C
int classify_code(unsigned code) {
  const int src[6] = {0, 1, 0, 2, 1, 2}, dst[6] = {1, 0, 2, 0, 2, 1};
  int out[3] = {0, 0, 0}, in[3] = {0, 0, 0};
  for (int b = 0; b < 6; ++b)
    if ((code >> b) & 1) { out[src[b]]++; in[dst[b]]++; }
  int M = 0, A = 0;
  for (int p = 0; p < 3; ++p) {
    unsigned two = (code >> (2 * p)) & 3u;  // bits (2p, 2p+1) are the two arcs of one pair
    M += two == 3;
    A += two == 1 || two == 2;
  }
  auto any = [&](int o, int i) {
    for (int x = 0; x < 3; ++x)
      if (out[x] == o && in[x] == i) return true;
    return false;
  };
  auto any_out = [&](int o) { return out[0] == o || out[1] == o || out[2] == o; };
  auto any_in = [&](int i) { return in[0] == i || in[1] == i || in[2] == i; };
  switch (M * 4 + A) {
    case 0: return 0;   // 003
    case 1: return 1;   // 012
    case 4: return 2;   // 102
    case 2: return any_out(2) ? 3 : any_in(2) ? 4 : 5;  // 021D / 021U / 021C
    case 5: return any_in(2) ? 6 : 7;                   // 111D / 111U
    case 3: return any_out(2) ? 8 : 9;                  // 030T / 030C
    case 8: return 10;                                  // 201
    case 6: return any(2, 0) ? 11 : any(0, 2) ? 12 : 13;  // 120D / 120U / 120C
    case 9: return 14;                                  // 210
    case 12: return 15;                                 // 300
  }
  return -1;
}

ClassSlices class_slices() {
  ClassSlices cs{};
  for (unsigned f = 0; f < 4; ++f) {
    uint64_t s = 0;
    // idx 0 (w in neither list) never occurs for a counted w: it is the
    // kernel's bin for the w a task does not own, mapped to class 0 (unused)
    for (unsigned idx = 1; idx < 16; ++idx) {
      unsigned fa = idx & 3u, fb = idx >> 2;
      s |= (uint64_t)(classify_code(f | fa << 2 | fb << 4) & 15) << (4 * idx);
    }
    cs.s[f] = s;
    uint32_t ga = 0, gb = 0;
    for (unsigned g = 1; g < 4; ++g) {
      ga |= (uint32_t)((s >> (4 * g)) & 15u) << (4 * g);
      gb |= (uint32_t)((s >> (4 * (g << 2))) & 15u) << (4 * g);
    }
    cs.ga[f] = ga | ga << 16;
    cs.gb[f] = gb | gb << 16;
  }
  return cs;
}

LabTables lab_tables() {
  LabTables t{};
  for (unsigned f = 0; f < 4; ++f) {
    uint32_t ahi = 0, bhi = 0, blo = 0;
    for (unsigned g = 1; g < 4; ++g) {
      const unsigned gm = ((g & 1u) << 1) | (g >> 1);
      ahi |= (f | g << 2) << (8 * g);
      bhi |= (f | g << 4) << (8 * g);
      blo |= (f << 2 | gm << 4) << (8 * g);
    }
    t.ga_hi[f] = ahi;
    t.gb_hi[f] = bhi;
    t.gb_lo[f] = blo;
  }
  return t;
}

void choose3(int64_t n, uint64_t* lo, uint64_t* hi) {
  unsigned __int128 r = 0;
  if (n >= 3) r = (unsigned __int128)(uint64_t)n * (uint64_t)(n - 1) * (uint64_t)(n - 2) / 6;
  *lo = (uint64_t)r;
  *hi = (uint64_t)(r >> 64);
}

int device_info(DeviceInfo* out) {
  static std::mutex mu;
  static DeviceInfo cache[64];
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
    return fail(TRIAD_EDEVICE, "no HIP device available");
  std::lock_guard<std::mutex> lk(mu);
  if (cache[dev].device != dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return fail(TRIAD_EDEVICE, "hipGetDeviceProperties failed");
    cache[dev].device = dev;
    cache[dev].cus = p.multiProcessorCount;
    cache[dev].lds_per_cu = p.maxSharedMemoryPerMultiProcessor;
    cache[dev].name = p.gcnArchName;
  }
  *out = cache[dev];
  return TRIAD_OK;
}

}  // namespace triad

using namespace triad;

extern "C" {

const char* triad_last_error(void) { return g_err.c_str(); }
int triad_version(void) { return TRIAD_ABI_VERSION; }

int triad_set_memory_cap(int64_t bytes) {
  if (bytes < 0) return fail(TRIAD_EINVAL, "memory cap must be >= 0");
  g_mem_cap.store(bytes);
  return TRIAD_OK;
}

int64_t triad_held_memory(void) { return (int64_t)held_bytes(); }

int triad_release_memory(void) {
  (void)held_release_all();
  return TRIAD_OK;
}

int triad_test_inject_device_error(int32_t count) {
  if (count < 0) return fail(TRIAD_EINVAL, "injected fault count must be >= 0");
  g_inject.store(count);
  return TRIAD_OK;
}

int triad_validate_host(int64_t n, const int64_t* off, const int32_t* nbr, const uint8_t* flg, int32_t level) {
  if (n < 0 || n >= ((int64_t)1 << 30)) return fail(TRIAD_EINVAL, "n must be in [0, 2^30)");
  if (!off) return fail(TRIAD_EINVAL, "csr_offsets is NULL");
  if (off[0] != 0) return fail(TRIAD_ERANGE, "csr_offsets[0] != 0");
  const int64_t nnz = off[n];
  if (nnz < 0 || nnz >= ((int64_t)1 << 40)) return fail(TRIAD_ERANGE, "nnz out of range");
  if (nnz > 0 && (!nbr || !flg)) return fail(TRIAD_EINVAL, "csr_nbrs or dir_flags is NULL");
  for (int64_t x = 0; x < n; ++x) {
    if (off[x + 1] < off[x]) return fail(TRIAD_ERANGE, "csr_offsets not monotone at row " + std::to_string(x));
    if (off[x + 1] - off[x] >= ((int64_t)1 << 31)) return fail(TRIAD_EINVAL, "degree >= 2^31");
  }
  uint32_t bits = 0;
  for (int64_t x = 0; x < n && !(bits & ERR_RANGE); ++x) {
    for (int64_t j = off[x]; j < off[x + 1]; ++j) {
      int64_t y = nbr[j];
      unsigned f = (flg[j >> 2] >> (2 * (j & 3))) & 3u;
      if (y < 0 || y >= n || f == 0) { bits |= ERR_RANGE; break; }
      if (y == x) bits |= ERR_SELFLOOP;
      if (j > off[x] && nbr[j - 1] >= y) bits |= ERR_UNSORTED;
    }
  }
  if (!bits && level >= 1) {
    for (int64_t x = 0; x < n && !bits; ++x) {
      for (int64_t j = off[x]; j < off[x + 1]; ++j) {
        int64_t y = nbr[j];
        const int32_t* b = nbr + off[y];
        const int32_t* e = nbr + off[y + 1];
        const int32_t* p = std::lower_bound(b, e, (int32_t)x);
        unsigned f = (flg[j >> 2] >> (2 * (j & 3))) & 3u;
        if (p == e || *p != x) { bits |= ERR_ASYM; break; }
        int64_t k = off[y] + (p - b);
        unsigned g = (flg[k >> 2] >> (2 * (k & 3))) & 3u;
        if (g != (((f & 1u) << 1) | (f >> 1))) { bits |= ERR_ASYM; break; }
      }
    }
  }
  int st = status_from_bits(bits);
  if (st != TRIAD_OK) {
    const char* what = st == TRIAD_ERANGE      ? "neighbour id out of range or zero direction flag"
                       : st == TRIAD_ESELFLOOP ? "self-loop in the CSR"
                       : st == TRIAD_EUNSORTED ? "row not strictly increasing"
                                               : "CSR not symmetric or flags not mirrored";
    return fail(st, what);
  }
  return TRIAD_OK;
}

}  // extern "C"
