// Rows of CSR entries for kernels that take one thread per entry. Internal;
// not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace triad {

// Last row x in [lo, hi) with off[x] <= j, given off[lo] <= j < off[hi] (an
// empty row is never the answer: the row after it starts at the same offset).
__device__ __forceinline__ int64_t row_search(const int64_t* __restrict__ off, int64_t lo, int64_t hi, int64_t j) {
  while (hi - lo > 1) {
    const int64_t m = (lo + hi) >> 1;
    if (off[m] <= j) lo = m; else hi = m;
  }
  return lo;
}

// Entry kernels take tiles of ETILE entries [t0, t1): two threads find the
// rows of the tile's first and last entry over all offsets (rr), and every
// entry then searches only between those two rows.
constexpr int ETILE = 4096;
__device__ __forceinline__ void tile_rows(const int64_t* __restrict__ off, int64_t n, int64_t t0, int64_t t1,
                                          int64_t* rr) {
  __syncthreads();
  if (threadIdx.x < 2) rr[threadIdx.x] = row_search(off, 0, n, threadIdx.x == 0 ? t0 : t1 - 1);
  __syncthreads();
}

// Staged variant for kernels whose entries each do little else: when the tile
// spans at most TILE_ROWS rows, the starts of rows r0..r1 are staged in LDS as
// 16-bit offsets from t0 (the first clamped to 0; every later one lies in
// (0, ETILE)), and an entry's row is a binary search in LDS instead of one
// over global offsets. (Where each entry also does a long global search, the
// staging costs more than it saves.)
constexpr int TILE_ROWS = 8192;
struct TileRows {
  int64_t r[2];
  uint16_t rel[TILE_ROWS];
};

// Called by every thread of the block (it synchronises the block).
__device__ __forceinline__ void tile_stage(const int64_t* __restrict__ off, int64_t n, int64_t t0, int64_t t1,
                                           TileRows& T) {
  __syncthreads();
  if (threadIdx.x < 2) T.r[threadIdx.x] = row_search(off, 0, n, threadIdx.x == 0 ? t0 : t1 - 1);
  __syncthreads();
  const int64_t r0 = T.r[0], nr = T.r[1] - r0 + 1;
  if (nr <= TILE_ROWS)
    for (int64_t x = threadIdx.x; x < nr; x += blockDim.x) {
      const int64_t d = off[r0 + x] - t0;
      T.rel[x] = (uint16_t)(d > 0 ? d : 0);
    }
  __syncthreads();
}

// Row of entry j of the staged tile starting at t0.
__device__ __forceinline__ int64_t tile_row(const int64_t* __restrict__ off, const TileRows& T, int64_t t0, int64_t j) {
  const int64_t r0 = T.r[0], r1 = T.r[1];
  if (r1 - r0 + 1 > TILE_ROWS) return row_search(off, r0, r1 + 1, j);
  const uint32_t jj = (uint32_t)(j - t0);
  uint32_t lo = 0, hi = (uint32_t)(r1 - r0 + 1);  // rel[lo] <= jj; rows from hi on start past jj
  while (hi - lo > 1) {
    const uint32_t m = (lo + hi) >> 1;
    if (T.rel[m] <= jj) lo = m; else hi = m;
  }
  return r0 + lo;
}

}  // namespace triad
