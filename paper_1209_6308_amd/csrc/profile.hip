// Triad significance profile: the census of a graph against the censuses of
// an ensemble of null-model graphs (degree-preserving randomisations, one
// batched census): per type the z-score
//     z_t = (N_t - mean_t) / sd_t
// (ensemble mean and sample standard deviation, divisor G - 1; z_t = 0 when
// the ensemble's counts of the type do not vary), and the profile of the 13
// connected types (021D ... 300), the z-vector scaled to unit length.
//
// One workgroup of 16 wavefronts, one per type. Counts are exact 64-bit
// integers; each type's counts are taken relative to the first graph's (an
// exact integer difference) before they are turned into doubles, so types
// whose counts are large but vary little keep their precision; mean and
// variance are two passes in double precision.
#include <hip/hip_runtime.h>

#include <string>

#include "triad_internal.h"

namespace triad {
namespace {

struct Real16 {
  uint64_t c[16];
};

__device__ __forceinline__ double wave_sum_f64(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__global__ void __launch_bounds__(1024) k_zscores(int32_t G, const uint64_t* __restrict__ ens, Real16 real,
                                                  double* __restrict__ out) {
  __shared__ double z[16];
  const int lane = threadIdx.x & 63, t = threadIdx.x >> 6;
  const uint64_t ref = ens[t];
  double s = 0;
  for (int32_t g = lane; g < G; g += 64) s += (double)(int64_t)(ens[16 * (int64_t)g + t] - ref);
  const double mean = wave_sum_f64(s) / (double)G;
  double q = 0;
  for (int32_t g = lane; g < G; g += 64) {
    const double d = (double)(int64_t)(ens[16 * (int64_t)g + t] - ref) - mean;
    q += d * d;
  }
  const double var = wave_sum_f64(q) / (double)(G - 1);
  if (lane == 0) {
    const double diff = (double)(int64_t)(real.c[t] - ref) - mean;
    z[t] = var > 0 ? diff / sqrt(var) : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double nrm = 0;
    for (int k = 3; k < 16; ++k) nrm += z[k] * z[k];
    nrm = sqrt(nrm);
    for (int k = 0; k < 16; ++k) {
      out[k] = z[k];
      out[16 + k] = (k >= 3 && nrm > 0) ? z[k] / nrm : 0.0;
    }
  }
}

}  // namespace

int significance_profile(int32_t G, const uint64_t* ens, const uint64_t* real, double* z, double* sp, hipStream_t s) {
  if (G < 2) return fail(TRIAD_EINVAL, "the ensemble needs at least two graphs");
  if (!ens || !real || !z || !sp) return fail(TRIAD_EINVAL, "NULL pointer argument");
  Scratch scratch(s);
  double* d_out = nullptr;
  ALLOC(d_out, 32);
  Real16 r;
  for (int k = 0; k < 16; ++k) r.c[k] = real[k];
  k_zscores<<<1, 1024, 0, s>>>(G, ens, r, d_out);
  HIPCHK(hipGetLastError());
  double h[32];
  HIPCHK(hipMemcpyAsync(h, d_out, sizeof h, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int k = 0; k < 16; ++k) {
    z[k] = h[k];
    sp[k] = h[16 + k];
  }
  return TRIAD_OK;
}

}  // namespace triad

using namespace triad;

extern "C" int triad_significance_profile(int32_t G, const uint64_t* d_ensemble, const uint64_t real[16],
                                          double z_out[16], double sp_out[16], void* hip_stream) {
  return significance_profile(G, d_ensemble, real, z_out, sp_out, (hipStream_t)hip_stream);
}
