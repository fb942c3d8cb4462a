// Construction of the compact CSR with direction bits (Sec. 6, Fig. 7) from
// a list of arcs, on the device.
//
// Every arc (x, y), x != y, yields two entries: row x sees y with bit0 (x->y)
// and row y sees x with bit1 (x->y seen from y). An entry is one 64-bit key
//     row << (RB + 2) | col << 2 | bit,   RB = bit width of n - 1,
// and the keys are sorted on their (row, col) bits only, so the entries come
// in order of row, then column. A self-loop yields two keys whose (row, col)
// bits are all ones, which sort after every real entry (a real pair never has
// row = col) and are dropped. After the sort, a run of equal (row, col) keys
// is one neighbour; its flag is the OR of its keys' bits, recorded by every
// key of the run (one byte per direction and entry, written with the same
// value by each key that has that bit). Duplicate arcs are thereby merged,
// and each pair's two rows get mirrored flags.
//
//   k_arc_keys      two keys per arc, range check, self-loop count
//   radix sort      least-significant-digit first, 8-bit digits, stable:
//                   k_rs_hist (per-tile digit counts), an exclusive scan of
//                   the digit-major counts, k_rs_scatter (per-wave ranks by
//                   ballot matching, per-wave running counts in LDS, the tile
//                   laid out in digit order in LDS and written in runs)
//   k_head_count    per tile, the first keys of (row, col) runs
//   k_emit_csr      ids, the runs' direction bits, row offsets
//   k_pack_flags    2-bit flags, four per byte
#include <hip/hip_runtime.h>

#include <string>

#include "device_sort.h"
#include "triad_internal.h"

namespace triad {
namespace {

constexpr int RS_BITS = 8, RS_BUCKETS = 1 << RS_BITS;
constexpr int RS_THREADS = 256, RS_WAVES = RS_THREADS / 64;
constexpr int RS_ITEMS = 16;                         // keys per thread and tile
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;       // 4,096 keys
constexpr int RS_WAVE_KEYS = RS_TILE / RS_WAVES;     // 1,024 consecutive keys per wavefront
constexpr int RS_ROUNDS = RS_WAVE_KEYS / 64;         // 16 rounds of 64
static_assert(RS_THREADS == RS_BUCKETS, "the scatter gives each digit one thread");

__device__ __forceinline__ int bit_width_u(uint64_t x) { return x ? 64 - __clzll((long long)x) : 0; }

__global__ void k_arc_keys(int64_t n, int64_t narcs, int rb, const int32_t* __restrict__ src,
                           const int32_t* __restrict__ dst, uint64_t* __restrict__ keys,
                           unsigned long long* __restrict__ loops, uint32_t* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t drop = ((1ull << (2 * rb)) - 1) << 2;  // (row, col) all ones: sorts last
  uint32_t bad = 0;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < narcs; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    bool loop = false;
    if (i < narcs) {
      const int32_t x = src[i], y = dst[i];
      if (x < 0 || y < 0 || x >= n || y >= n) {
        bad = 1;
        keys[2 * i] = keys[2 * i + 1] = drop;
      } else if (x == y) {
        loop = true;
        keys[2 * i] = keys[2 * i + 1] = drop;
      } else {
        keys[2 * i] = ((uint64_t)x << (rb + 2)) | ((uint64_t)y << 2) | 1u;
        keys[2 * i + 1] = ((uint64_t)y << (rb + 2)) | ((uint64_t)x << 2) | 2u;
      }
    }
    const uint64_t m = __ballot(loop);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(loops, (unsigned long long)__popcll(m));
  }
  if (bad) atomicOr(err, ERR_RANGE);
}

// Digit counts of one tile: counts[digit * ntiles + tile].
__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint64_t* __restrict__ keys, int64_t N, int shift,
                                                        uint32_t* __restrict__ counts, int64_t ntiles) {
  __shared__ uint32_t h[RS_WAVES][RS_BUCKETS];
  const int w = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < RS_WAVES * RS_BUCKETS; k += RS_THREADS) (&h[0][0])[k] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
  for (int k = 0; k < RS_ITEMS; ++k) {
    const int64_t i = base + (int64_t)k * RS_THREADS + threadIdx.x;
    if (i < N) atomicAdd(&h[w][(uint32_t)(keys[i] >> shift) & (RS_BUCKETS - 1)], 1u);
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int q = 0; q < RS_WAVES; ++q) c += h[q][threadIdx.x];
  counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = c;
}

// Stable scatter of one tile. Wavefront w owns keys [w * 1024, (w+1) * 1024)
// of the tile, 64 per round in order; a key's rank among the equal digits
// before it in its wavefront comes from ballots that match the digit bit by
// bit, and per-wavefront running counts in LDS carry it across rounds. The
// tile is then laid out in LDS in digit order (digit starts from a scan of the
// tile's counts, the wavefronts of one digit in order), and written out from
// there: consecutive threads write consecutive keys, so each digit's keys of
// the tile leave as one contiguous run. Input order within a digit is kept.
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                           int64_t N, int shift, const uint32_t* __restrict__ offs,
                                                           int64_t ntiles) {
  __shared__ uint32_t cnt[RS_WAVES][RS_BUCKETS];
  __shared__ uint32_t lstart[RS_BUCKETS], gstart[RS_BUCKETS], wsum[RS_WAVES + 1];
  __shared__ uint64_t buf[RS_TILE];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < RS_WAVES * RS_BUCKETS; k += RS_THREADS) (&cnt[0][0])[k] = 0;
  __syncthreads();
  const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
  const int64_t base = tbase + (int64_t)w * RS_WAVE_KEYS;
  const uint64_t below = (1ull << lane) - 1;
  uint64_t key[RS_ROUNDS];
  uint32_t pos[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + (int64_t)r * 64 + lane;
    const bool valid = i < N;
    key[r] = valid ? in[i] : 0;
    const uint32_t d = (uint32_t)(key[r] >> shift) & (RS_BUCKETS - 1);
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < RS_BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t mb = __ballot(bit);
      m &= bit ? mb : ~mb;
    }
    // every lane of a digit group reads the running count, then the group's
    // lowest lane advances it (LDS operations of one wavefront run in order)
    const uint32_t c = cnt[w][d];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (valid && (m & below) == 0) cnt[w][d] = c + (uint32_t)__popcll(m);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    pos[r] = c + (uint32_t)__popcll(m & below);
  }
  __syncthreads();
  // per digit (one thread each): the tile's count, its global start, and the
  // wavefronts' starts within the digit
  const int d = threadIdx.x;
  uint32_t tot = 0;
#pragma unroll
  for (int q = 0; q < RS_WAVES; ++q) {
    const uint32_t c = cnt[q][d];
    cnt[q][d] = tot;
    tot += c;
  }
  gstart[d] = offs[(int64_t)d * ntiles + blockIdx.x];
  // exclusive scan of the tile's digit counts across the block
  uint32_t x = tot;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int q = 0; q < RS_WAVES; ++q) {
      const uint32_t t = wsum[q];
      wsum[q] = run;
      run += t;
    }
  }
  __syncthreads();
  lstart[d] = x - tot + wsum[w];
  __syncthreads();
  // the tile in digit order in LDS
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + (int64_t)r * 64 + lane;
    if (i < N) {
      const uint32_t dk = (uint32_t)(key[r] >> shift) & (RS_BUCKETS - 1);
      const uint32_t at = lstart[dk] + cnt[w][dk] + pos[r];
      if (at < (uint32_t)RS_TILE) buf[at] = key[r];  // always true; keeps a faulty rank in bounds
    }
  }
  __syncthreads();
  const int64_t nt = min((int64_t)RS_TILE, N - tbase);
  for (int i = threadIdx.x; i < nt; i += RS_THREADS) {
    const uint64_t k = buf[i];
    const uint32_t dk = (uint32_t)(k >> shift) & (RS_BUCKETS - 1);
    const uint64_t at = (uint64_t)gstart[dk] + (uint32_t)(i - lstart[dk]);
    if (at < (uint64_t)N) out[at] = k;  // always true; keeps a faulty rank in bounds
  }
}

// ---------------------------------------------------------------- u32 scan
// out[0..m) = exclusive prefix of in[0..m) (32-bit; the caller bounds the
// total below 2^32), *total = the sum. Block sums, one block over the block
// sums, block-local scans.
constexpr int SC_T = 256, SC_I = 16, SC_B = SC_T * SC_I;

__device__ uint32_t block_scan_u32(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int k = 0; k < SC_T / 64; ++k) {
      const uint32_t t = sh[k];
      sh[k] = run;
      run += t;
    }
    sh[SC_T / 64] = run;
  }
  __syncthreads();
  const uint32_t r = x - v + sh[w];
  *total = sh[SC_T / 64];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(SC_T) k_sc_sums(const uint32_t* __restrict__ in, int64_t m, uint32_t* __restrict__ bsum) {
  __shared__ uint32_t sh[SC_T / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * SC_B + (int64_t)threadIdx.x * SC_I;
  uint32_t s = 0;
  for (int k = 0; k < SC_I; ++k)
    if (base + k < m) s += in[base + k];
  uint32_t tot;
  block_scan_u32(s, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SC_T) k_sc_top(uint32_t* __restrict__ bsum, int64_t nb, uint32_t* __restrict__ total) {
  __shared__ uint32_t sh[SC_T / 64 + 1];
  uint32_t carry = 0;
  for (int64_t c = 0; c < nb; c += SC_B) {
    const int64_t base = c + (int64_t)threadIdx.x * SC_I;
    uint32_t loc[SC_I], s = 0;
    for (int k = 0; k < SC_I; ++k) {
      loc[k] = base + k < nb ? bsum[base + k] : 0u;
      s += loc[k];
    }
    uint32_t tot;
    uint32_t run = carry + block_scan_u32(s, sh, &tot);
    for (int k = 0; k < SC_I; ++k)
      if (base + k < nb) {
        bsum[base + k] = run;
        run += loc[k];
      }
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void __launch_bounds__(SC_T) k_sc_apply(const uint32_t* __restrict__ in, int64_t m,
                                                   const uint32_t* __restrict__ bsum, uint32_t* __restrict__ out) {
  __shared__ uint32_t sh[SC_T / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * SC_B + (int64_t)threadIdx.x * SC_I;
  uint32_t loc[SC_I], s = 0;
  for (int k = 0; k < SC_I; ++k) {
    loc[k] = base + k < m ? in[base + k] : 0u;
    s += loc[k];
  }
  uint32_t tot;
  uint32_t run = block_scan_u32(s, sh, &tot) + bsum[blockIdx.x];
  for (int k = 0; k < SC_I; ++k)
    if (base + k < m) {
      out[base + k] = run;
      run += loc[k];
    }
}

}  // namespace

int scan_u32(const uint32_t* in, int64_t m, uint32_t* out, uint32_t* total, Scratch& scratch, hipStream_t s) {
  const int64_t nb = (m + SC_B - 1) / SC_B;
  uint32_t* bsum = nullptr;
  ALLOC(bsum, nb + 1);
  if (m > 0) {
    k_sc_sums<<<(unsigned)nb, SC_T, 0, s>>>(in, m, bsum);
    k_sc_top<<<1, SC_T, 0, s>>>(bsum, nb, total);
    k_sc_apply<<<(unsigned)nb, SC_T, 0, s>>>(in, m, bsum, out);
  }
  HIPCHK(hipGetLastError());
  return TRIAD_OK;
}

// Stable LSD radix sort of N 64-bit keys on bits [lo, hi), 8 bits per pass;
// *keys points at the sorted keys on return (one of the two buffers).
int radix_sort_u64(uint64_t** keys, uint64_t** tmp, int64_t N, int lo, int hi, Scratch& scratch, hipStream_t s) {
  if (N >= ((int64_t)1 << 32)) return fail(TRIAD_EINVAL, "radix sort of 2^32 or more keys");
  if (N == 0) return TRIAD_OK;
  const int64_t ntiles = (N + RS_TILE - 1) / RS_TILE;
  uint32_t *counts = nullptr, *offs = nullptr;
  ALLOC(counts, (int64_t)RS_BUCKETS * ntiles);
  ALLOC(offs, (int64_t)RS_BUCKETS * ntiles);
  for (int shift = lo; shift < hi; shift += RS_BITS) {
    k_rs_hist<<<(unsigned)ntiles, RS_THREADS, 0, s>>>(*keys, N, shift, counts, ntiles);
    if (int st = scan_u32(counts, (int64_t)RS_BUCKETS * ntiles, offs, nullptr, scratch, s)) return st;
    k_rs_scatter<<<(unsigned)ntiles, RS_THREADS, 0, s>>>(*keys, *tmp, N, shift, offs, ntiles);
    HIPCHK(hipGetLastError());
    std::swap(*keys, *tmp);
  }
  return TRIAD_OK;
}

namespace {

// ------------------------------------------------------------ runs -> CSR
__device__ __forceinline__ bool run_head(const uint64_t* key, int64_t i) {
  return i == 0 || (key[i] >> 2) != (key[i - 1] >> 2);
}

// Number of run heads among the valid keys of each tile.
__global__ void __launch_bounds__(RS_THREADS) k_head_count(const uint64_t* __restrict__ key, int64_t nvalid,
                                                           uint32_t* __restrict__ tilecnt) {
  __shared__ uint32_t ws[RS_WAVES];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * RS_WAVE_KEYS;
  uint32_t c = 0;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + (int64_t)r * 64 + lane;
    c += (uint32_t)__popcll(__ballot(i < nvalid && run_head(key, i)));
  }
  if (lane == 0) ws[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int q = 0; q < RS_WAVES; ++q) t += ws[q];
    tilecnt[blockIdx.x] = t;
  }
}

// Entry e of the CSR is the e-th run. Its head writes the column; every key of
// the run marks its direction bit (fh[e] = 1 for bit0, ft[e] = 2 for bit1, both
// zeroed before); the head of a row's first run writes the offsets of that row
// and of the empty rows before it, the last valid key those of the rows after
// its own.
__global__ void __launch_bounds__(RS_THREADS) k_emit_csr(const uint64_t* __restrict__ key, int64_t nvalid, int64_t n,
                                                         int rb, const uint32_t* __restrict__ tileoff, uint32_t nnz,
                                                         int64_t* __restrict__ off, int32_t* __restrict__ nbr,
                                                         uint8_t* __restrict__ fh, uint8_t* __restrict__ ft) {
  __shared__ uint32_t ws[RS_WAVES];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * RS_WAVE_KEYS;
  const uint64_t below = (1ull << lane) - 1;
  // heads in this wavefront's part of the tile, for the wavefronts' offsets
  uint32_t c = 0;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + (int64_t)r * 64 + lane;
    c += (uint32_t)__popcll(__ballot(i < nvalid && run_head(key, i)));
  }
  if (lane == 0) ws[w] = c;
  __syncthreads();
  uint32_t run = tileoff[blockIdx.x];
  for (int q = 0; q < w; ++q) run += ws[q];
  const uint64_t colmask = ((1ull << rb) - 1);
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + (int64_t)r * 64 + lane;
    const bool valid = i < nvalid;
    const bool head = valid && run_head(key, i);
    const uint64_t hm = __ballot(head);
    // entry of this key: heads up to and including it, minus one
    const uint32_t e = run + (uint32_t)__popcll(hm & (below | (1ull << lane))) - 1u;
    if (valid && e < nnz) {
      const uint64_t k = key[i];
      const int64_t row = (int64_t)(k >> (rb + 2));
      const uint8_t bitv = (uint8_t)(k & 3u);
      if (head) {
        nbr[e] = (int32_t)((k >> 2) & colmask);
        const int64_t prev = i == 0 ? -1 : (int64_t)(key[i - 1] >> (rb + 2));
        for (int64_t x = prev + 1; x <= row; ++x) off[x] = e;
      }
      if (bitv & 1u) fh[e] = 1;
      if (bitv & 2u) ft[e] = 2;
      const bool last = i + 1 == nvalid;
      if (last)
        for (int64_t x = row + 1; x <= n; ++x) off[x] = nnz;
    }
    run += (uint32_t)__popcll(hm);
  }
}

__global__ void k_pack_flags(const uint8_t* __restrict__ fh, const uint8_t* __restrict__ ft, int64_t nnz,
                             uint8_t* __restrict__ flg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, nbytes = (nnz + 3) / 4;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nbytes; b += stride) {
    uint32_t v = 0;
    for (int k = 0; k < 4; ++k) {
      const int64_t e = 4 * b + k;
      if (e < nnz) v |= (uint32_t)(fh[e] | ft[e]) << (2 * k);
    }
    flg[b] = (uint8_t)v;
  }
}

__global__ void k_fill_off(int64_t* p, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) p[i] = 0;
}
__global__ void k_zero_words(uint32_t* p, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) p[i] = 0;
}

}  // namespace

int grid_of(int64_t work, int threads, int cap) {
  int64_t g = (work + threads - 1) / threads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

int csr_from_arcs(int64_t n, int64_t narcs, const int32_t* src, const int32_t* dst, hipStream_t s, int64_t* off,
                  int32_t* nbr, uint8_t* flg, int64_t* nnz_out, float* ms_out) {
  if (n < 0 || n >= ((int64_t)1 << 30)) return fail(TRIAD_EINVAL, "n must be in [0, 2^30)");
  if (narcs < 0 || narcs >= ((int64_t)1 << 31)) return fail(TRIAD_EINVAL, "narcs must be in [0, 2^31)");
  if (!off || !nnz_out || (narcs > 0 && (!src || !dst || !nbr || !flg)))
    return fail(TRIAD_EINVAL, "NULL pointer argument");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms_out) {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
  }
  auto done = [&](int64_t nnz) -> int {
    if (ms_out) {
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, e0, e1));
      *ms_out = t;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
    *nnz_out = nnz;
    return TRIAD_OK;
  };
  if (narcs == 0) {
    k_fill_off<<<grid_of(n + 1, 256, 4096), 256, 0, s>>>(off, n + 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return done(0);
  }
  Scratch scratch(s, 0, true);
  const int rb = n > 1 ? 64 - __builtin_clzll((unsigned long long)(n - 1)) : 1;  // ids below 2^rb
  const int64_t N = 2 * narcs;
  uint64_t *ka = nullptr, *kb = nullptr;
  uint32_t* err = nullptr;
  unsigned long long* loops = nullptr;
  ALLOC(ka, N);
  ALLOC(kb, N);
  ALLOC(err, 2);
  ALLOC(loops, 1);
  k_zero_words<<<1, 64, 0, s>>>(err, 2);
  k_zero_words<<<1, 64, 0, s>>>((uint32_t*)loops, 2);
  k_arc_keys<<<grid_of(narcs, 256, 65536), 256, 0, s>>>(n, narcs, rb, src, dst, ka, loops, err);
  HIPCHK(hipGetLastError());
  uint32_t errh = 0;
  unsigned long long nloops = 0;
  HIPCHK(hipMemcpyAsync(&errh, err, sizeof errh, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&nloops, loops, sizeof nloops, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (errh) return fail(TRIAD_ERANGE, "arc endpoint outside [0, n)");
  // radix sort over bits [2, 2 + 2 rb): column, row (the direction bits are
  // merged per run, not sorted)
  if (int st = radix_sort_u64(&ka, &kb, N, 2, 2 + 2 * rb, scratch, s)) return st;
  // runs of equal (row, col): one CSR entry each
  const int64_t nvalid = N - 2 * (int64_t)nloops;
  const int64_t vt = std::max<int64_t>(1, (nvalid + RS_TILE - 1) / RS_TILE);
  uint32_t *tilecnt = nullptr, *tileoff = nullptr, *tot = nullptr;
  ALLOC(tilecnt, vt);
  ALLOC(tileoff, vt);
  ALLOC(tot, 1);
  k_zero_words<<<1, 64, 0, s>>>(tot, 1);
  if (nvalid > 0) {
    k_head_count<<<(unsigned)vt, RS_THREADS, 0, s>>>(ka, nvalid, tilecnt);
    if (int st = scan_u32(tilecnt, vt, tileoff, tot, scratch, s)) return st;
  }
  uint32_t nnz = 0;
  HIPCHK(hipMemcpyAsync(&nnz, tot, sizeof nnz, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (nnz == 0) {
    k_fill_off<<<grid_of(n + 1, 256, 4096), 256, 0, s>>>(off, n + 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return done(0);
  }
  uint8_t *fh = nullptr, *ft = nullptr;
  ALLOC(fh, (int64_t)nnz + 4);
  ALLOC(ft, (int64_t)nnz + 4);
  k_zero_words<<<grid_of(((int64_t)nnz + 4) / 4, 256, 65536), 256, 0, s>>>((uint32_t*)fh, ((int64_t)nnz + 4) / 4);
  k_zero_words<<<grid_of(((int64_t)nnz + 4) / 4, 256, 65536), 256, 0, s>>>((uint32_t*)ft, ((int64_t)nnz + 4) / 4);
  k_emit_csr<<<(unsigned)vt, RS_THREADS, 0, s>>>(ka, nvalid, n, rb, tileoff, nnz, off, nbr, fh, ft);
  k_pack_flags<<<grid_of((nnz + 3) / 4, 256, 65536), 256, 0, s>>>(fh, ft, nnz, flg);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return done(nnz);
}

}  // namespace triad

using namespace triad;

extern "C" int triad_csr_from_arcs(int64_t n, int64_t narcs, const int32_t* d_src, const int32_t* d_dst,
                                   void* hip_stream, int64_t* d_offsets, int32_t* d_nbrs, uint8_t* d_flags,
                                   int64_t* nnz_out, float* device_ms) {
  return csr_from_arcs(n, narcs, d_src, d_dst, (hipStream_t)hip_stream, d_offsets, d_nbrs, d_flags, nnz_out,
                       device_ms);
}
