// Internal declarations shared by the census library's sources (not part of
// the public ABI in include/triad.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "triad.h"

namespace triad {

// Error bits raised by the device-side validation; mapped to a status by
// status_from_bits(). Lower bit = higher priority.
enum : uint32_t {
  ERR_RANGE = 1u,     // neighbour out of range, flag 0, offsets not monotone / not ending at nnz
  ERR_SELFLOOP = 2u,  // a row lists its own vertex
  ERR_UNSORTED = 4u,  // a row not strictly increasing
  ERR_ASYM = 8u,      // missing mirror entry or flag not mirrored
  ERR_DEVICE = 16u,   // a fault detected on the device (raised today only by the test hook)
};

int status_from_bits(uint32_t bits);

// thread-local last error message
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);

// 16 nibbles per direction flag f of (u,v): entry idx = fa | fb << 2 gives the
// class of the triad code f | fa << 2 | fb << 4 (fa = flag of w in N(u) or 0,
// fb = flag of w in N(v) or 0).
struct ClassSlices {
  uint64_t s[4];  // [f_uv]: nibble fa | fb << 2 -> class
  // [f_uv]: class of a w found in one list only, by its flag g (nibble g,
  // nibble 0 = 0), the four nibbles repeated at bit 16: ga for N(u) only, gb
  // for N(v) only
  uint32_t ga[4], gb[4];
};
ClassSlices class_slices();

// Labelled census (64 states of a triple a < b < c): per f_uv, the state of a
// third vertex w found in one list only, by its flag g, in 8-bit field g
// (field 0 = 0, not counted): N(u) only above v (f | g << 2), N(v) only above
// v (f | g << 4), N(v) only between u and v (f << 2 | mirror(g) << 4).
struct LabTables {
  uint32_t ga_hi[4], gb_hi[4], gb_lo[4];
};
LabTables lab_tables();
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

#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      return fail(TRIAD_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));     \
  } while (0)

// Process-wide cap on the device memory one call may allocate (0 = none),
// set by triad_set_memory_cap. within_cap(total) says whether a call that has
// allocated `total` bytes so far stays within it.
int64_t memory_cap();
inline bool within_cap(size_t total) {
  const int64_t c = memory_cap();
  return c <= 0 || total <= (size_t)c;
}
// Test hook: true (once per injected fault) when the calling census should
// raise ERR_DEVICE after its census kernel; set by triad_test_inject_device_error.
bool take_injected_fault();

// Device blocks the library keeps between calls, per device. A call that
// drains its stream before it returns can take its scratch from here and give
// it back on return, so that repeated calls of one shape allocate and free
// nothing (freeing gigabytes costs milliseconds of host time per call).
// held_take hands out a held block of at least `bytes` and at most twice that
// (sizes rounded up to 256 B, or to whole MiB from 1 MiB on; its size in
// *got), else allocates one (freeing every held block of the
// device and retrying once if the device is out of memory); held_give keeps a
// block unless the device's held bytes would pass HELD_LIMIT, then frees it.
constexpr size_t HELD_LIMIT = (size_t)64 << 30;
hipError_t held_take(void** p, size_t bytes, size_t* got);
void held_give(void* p, size_t bytes, int device);
size_t held_release_all();  // frees every held block; returns the bytes freed
size_t held_bytes();        // bytes held, all devices

// Scratch memory of one call. By default stream-ordered allocations, released
// (in stream order) on destruction; `total` counts what the call has
// allocated (starting from what it allocated before this object existed) and
// a request that would take it past the memory cap fails. Constructed with
// held = true (for calls that drain their stream before returning), the blocks
// come from the held blocks above and go back to them on destruction, after
// the stream has drained (every use of them is on that stream). Given an
// arena (a caller-owned device range), it hands out 256-byte aligned pieces of
// it instead and allocates nothing; a request past the arena's end fails.
struct Scratch {
  hipStream_t s;
  std::vector<void*> ptrs;
  struct Block {
    void* p;
    size_t bytes;
  };
  std::vector<Block> blocks;  // held = true
  bool held = false;
  int device = -1;
  char* arena = nullptr;
  size_t cap = 0, used = 0, total = 0;
  explicit Scratch(hipStream_t st, size_t allocated_before = 0, bool keep = false)
      : s(st), held(keep), total(allocated_before) {
    // held blocks live on the current device: a stream of another device
    // takes stream-ordered allocations on its own device instead
    hipDevice_t sd = -1;
    if (held && (hipGetDevice(&device) != hipSuccess || hipStreamGetDevice(s, &sd) != hipSuccess || sd != device)) {
      (void)hipGetLastError();
      held = false;
    }
  }
  Scratch(hipStream_t st, void* base, size_t bytes) : s(st), arena(static_cast<char*>(base)), cap(bytes) {}
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFreeAsync(p, s);
    if (blocks.empty()) return;
    if (hipStreamSynchronize(s) == hipSuccess) {
      for (const Block& b : blocks) held_give(b.p, b.bytes, device);
    } else {
      for (const Block& b : blocks) (void)hipFree(b.p);
    }
  }
  template <class T>
  hipError_t get(T** p, int64_t count) {
    size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    if (arena) {
      const size_t at = (used + 255) & ~(size_t)255;
      if (at > cap || bytes > cap - at) return hipErrorOutOfMemory;
      *p = reinterpret_cast<T*>(arena + at);
      used = at + bytes;
      return hipSuccess;
    }
    if (!within_cap(total + bytes)) return hipErrorOutOfMemory;
    if (held) {
      size_t got = 0;
      hipError_t e = held_take((void**)p, bytes, &got);
      if (e == hipSuccess) {
        blocks.push_back({(void*)*p, got});
        total += bytes;
      }
      return e;
    }
    hipError_t e = hipMallocAsync((void**)p, bytes, s);
    if (e == hipSuccess) {
      ptrs.push_back(*p);
      total += bytes;
    }
    return e;
  }
};

#define ALLOC(ptr, count)                                                                        \
  do {                                                                                           \
    hipError_t e_ = scratch.get(&(ptr), (count));                                                \
    if (e_ != hipSuccess) {                                                                      \
      (void)hipGetLastError();                                                                   \
      return fail(TRIAD_ENOMEM, std::string("device allocation of ") + #ptr + " failed");       \
    }                                                                                            \
  } while (0)

// Task (u, k): u in bits 32..61, k (index of v in the row of u) in bits 0..31;
// bit 63 marks a task that is split into chunks (merged from the hub list).
constexpr uint64_t HUB_BIT = 1ull << 63;

// Whole tasks are claimed from the census queue BATCH consecutive tasks at a
// time; a schedule orders these batches.
constexpr int BATCH = 64;

// Schedules: the census claims whole tasks in batches of BATCH consecutive
// queue positions. A schedule keeps the queue in CSR order except for its last
// max(nb / SCHED_TAIL_DIV, SCHED_TAIL_MIN) full batches (all of them if
// fewer), which it puts costliest first by a cost key binned into SCHED_BINS
// bins (stable counting sort: CSR order within a bin). mode 1: d(u)+d(v);
// mode 2: the learned model's predicted log2 cycles (model = device weights).
constexpr int SCHED_BINS = 128;
constexpr int64_t SCHED_TAIL_DIV = 10, SCHED_TAIL_MIN = 4096;
// Reorders the task list (with tskip, each task's count of N(v) ids below u)
// in place, or, if order is not null, leaves both and writes order[queue
// position] = task index for all ntasks positions. The
// reordering happens only when a batch among the last 8,192 is predicted to
// cost more than the mean of the last 32,768 by tail_share / 10,000 (0: the
// default 30; < 0: always) of one wavefront's share of the whole census, the
// census running on nwaves wavefronts; ustart[u] = ids of row u below u.
int schedule_tail(int mode, const float* model, int64_t n, const int64_t* off, const uint32_t* ustart,
                  const uint32_t* packed, uint64_t* tasks, uint32_t* tskip, int64_t ntasks, int64_t* order,
                  int32_t tail_share, int64_t nwaves, Scratch& scratch, hipStream_t s);

}  // namespace triad
