// Device sort and scan routines shared by the library's graph-building
// sources (CSR construction, incremental updates). Internal; not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "triad_internal.h"

namespace triad {

// Stable least-significant-digit radix sort of N < 2^32 64-bit keys on bits
// [lo, hi) (8 bits per pass; bits outside keep their order within equal
// digits). *keys and *tmp are two device buffers of N keys; on return *keys
// points at the sorted keys.
int radix_sort_u64(uint64_t** keys, uint64_t** tmp, int64_t N, int lo, int hi, Scratch& scratch, hipStream_t s);

// Exclusive prefix of m 32-bit values (the total must stay below 2^32); the
// total goes to *total (device) when total is not NULL.
int scan_u32(const uint32_t* in, int64_t m, uint32_t* out, uint32_t* total, Scratch& scratch, hipStream_t s);

// Grid size for `work` items at `threads` per block, between 1 and cap.
int grid_of(int64_t work, int threads, int cap);

}  // namespace triad
