// Internal declarations shared by the census library's sources (not part of
// the public ABI in include/triad.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "triad.h"

namespace triad {

// Error bits raised by the device-side validation; mapped to a status by
// status_from_bits(). Lower bit = higher priority.
enum : uint32_t {
  ERR_RANGE = 1u,     // neighbour out of range, flag 0, offsets not monotone / not ending at nnz
  ERR_SELFLOOP = 2u,  // a row lists its own vertex
  ERR_UNSORTED = 4u,  // a row not strictly increasing
  ERR_ASYM = 8u,      // missing mirror entry or flag not mirrored
};

int status_from_bits(uint32_t bits);

// thread-local last error message
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);

// 16 nibbles per direction flag f of (u,v): entry idx = fa | fb << 2 gives the
// class of the triad code f | fa << 2 | fb << 4 (fa = flag of w in N(u) or 0,
// fb = flag of w in N(v) or 0).
struct ClassSlices {
  uint64_t s[4];
};
ClassSlices class_slices();
int classify_code(unsigned code);  // 0..15, standard order

// C(n,3) as (lo, hi) 64-bit words.
void choose3(int64_t n, uint64_t* lo, uint64_t* hi);

struct DeviceInfo {
  int device = -1;
  int cus = 0;
  int xcds = 8;
  size_t lds_per_cu = 0;
  std::string name;
};
int device_info(DeviceInfo* out);

}  // namespace triad
