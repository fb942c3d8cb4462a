// Task scheduling for the census: cost keys (d(u)+d(v), or a learned FP32
// cost model), counting sort of the tasks into cost bins, longest first.
//
// Cost model: multilayer perceptron 6 -> 32 -> 32 -> 1, ReLU hidden layers,
// trained on the GPU by the kernels below (forward, mean-squared-error
// gradient by backpropagation, Adam) on per-task cycle counts recorded by the
// census kernel itself. Parameter layout (TRIAD_MLP_PARAMS floats):
//   W1[32][6] | b1[32] | W2[32][32] | b2[32] | W3[32] | b3
// Features of task (u,v), each log2(1 + x): d(u), d(v), d(u)+d(v),
// min(d(u),d(v)), max(d(u),d(v)), entries of N(u) above v.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "triad_internal.h"

namespace triad {

constexpr int NI = TRIAD_MLP_IN, NH = TRIAD_MLP_HIDDEN, NP = TRIAD_MLP_PARAMS;
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NH;
static_assert(OB3 + 1 == NP, "parameter layout");

// Features of a task (u, v), from the lengths its merge really walks: a = the
// ids of N(u) above u, b = the ids of N(v) from u on, and the ids of N(u)
// above v (the part whose third vertices the task may count).
__device__ __forceinline__ void task_features(uint32_t du, uint32_t dv, uint32_t above, float x[NI]) {
  const uint32_t mn = du < dv ? du : dv, mx = du < dv ? dv : du;
  x[0] = log2f(1.0f + (float)du);
  x[1] = log2f(1.0f + (float)dv);
  x[2] = log2f(1.0f + (float)du + (float)dv);
  x[3] = log2f(1.0f + (float)mn);
  x[4] = log2f(1.0f + (float)mx);
  x[5] = log2f(1.0f + (float)above);
}

// y = W3 . relu(W2 relu(W1 x + b1) + b2) + b3.
__device__ __forceinline__ float mlp_forward(const float* __restrict__ w, const float x[NI]) {
  float h1[NH];
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    float a = w[OB1 + j];
#pragma unroll
    for (int i = 0; i < NI; ++i) a = fmaf(w[OW1 + j * NI + i], x[i], a);
    h1[j] = a > 0.0f ? a : 0.0f;
  }
  float y = w[OB3];
#pragma unroll 1
  for (int j = 0; j < NH; ++j) {
    float a = w[OB2 + j];
#pragma unroll
    for (int k = 0; k < NH; ++k) a = fmaf(w[OW2 + j * NH + k], h1[k], a);
    y = fmaf(w[OW3 + j], a > 0.0f ? a : 0.0f, y);
  }
  return y;
}

__device__ __forceinline__ void load_weights(const float* __restrict__ gw, float* sw) {
  for (int p = threadIdx.x; p < NP; p += blockDim.x) sw[p] = gw[p];
  __syncthreads();
}

// ---------------------------------------------------------------- features

// Features of every task, tasks in CSR order (raw CSR input).
__global__ void k_features_csr(int64_t n, const int64_t* __restrict__ off, const int32_t* __restrict__ nbr,
                               const int64_t* __restrict__ tpre, float* __restrict__ feat) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t u = wave; u < n; u += nwave) {
    const int64_t b = off[u];
    const uint32_t du = (uint32_t)(off[u + 1] - b);
    const int64_t t0 = tpre[u];
    const uint32_t cnt = (uint32_t)(tpre[u + 1] - t0);
    const uint32_t s = du - cnt;  // first entry above u; cnt = d+(u), the ids above u
    for (uint32_t i = lane; i < cnt; i += 64) {
      const uint32_t k = s + i;
      const int32_t v = nbr[b + k];
      // ids of N(v) below u: lower bound of u in the row of v
      int64_t lo = off[v], hi = off[v + 1];
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (nbr[mid] < (int32_t)u) lo = mid + 1; else hi = mid;
      }
      const uint32_t dv = (uint32_t)(off[v + 1] - lo);
      float x[NI];
      task_features(cnt, dv, du - k - 1, x);
      float* o = feat + (t0 + i) * NI;
      for (int q = 0; q < NI; ++q) o[q] = x[q];
    }
  }
}

__global__ void k_task_counts(int64_t n, const int64_t* __restrict__ off, const int32_t* __restrict__ nbr,
                              int64_t* __restrict__ ntask) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    int64_t lo = off[u], hi = off[u + 1];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (nbr[mid] <= (int32_t)u) lo = mid + 1; else hi = mid;
    }
    ntask[u] = off[u + 1] - lo;
  }
}

// ---------------------------------------------------------------- MLP kernels

__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ gw, const float* __restrict__ x, int64_t m,
                              float* __restrict__ y) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < m; s += stride) {
    float xi[NI];
    for (int i = 0; i < NI; ++i) xi[i] = x[s * NI + i];
    y[s] = mlp_forward(gw, xi);
  }
}

// Sample index of position p in a minibatch: identity, or a counter-based
// hash (SplitMix64 finaliser) of (seed, step, p) for sampling with replacement.
__device__ __forceinline__ int64_t sample_index(uint64_t seed, uint64_t step, int64_t p, int64_t m, bool hashed) {
  if (!hashed) return p;
  uint64_t z = seed + step * 0x9E3779B97F4A7C15ull + (uint64_t)p * 0xD1B54A32D192ED03ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (int64_t)((unsigned __int128)z * (uint64_t)m >> 64);
}

// Gradient of L = (1/count) sum_s (model(x_s) - t_s)^2 over `count` samples
// (positions p0 .. p0+count of the sample stream), accumulated into g[NP]
// with one atomic add per parameter per block; loss sum into loss[0].
// Backpropagation: dy = 2(y - t)/count; dW3 = dy h2; dh2 = dy W3 [h2 > 0];
// dW2 = dh2 h1^T; dh1 = W2^T dh2 [h1 > 0]; dW1 = dh1 x^T; biases likewise.
constexpr int GB = 128;  // samples per block
__global__ void __launch_bounds__(GB) k_mlp_grad(const float* __restrict__ gw, const float* __restrict__ x,
                                                 const float* __restrict__ t, int64_t m, int64_t p0, int64_t count,
                                                 uint64_t seed, uint64_t step, int hashed, float* __restrict__ grad,
                                                 float* __restrict__ loss) {
  __shared__ float w[NP];
  __shared__ float H1[GB][NH + 1], H2[GB][NH + 1], D1[GB][NH + 1], D2[GB][NH + 1];
  __shared__ float X[GB][NI], G[GB], LS[GB];
  load_weights(gw, w);
  const int tid = threadIdx.x;
  const int64_t p = (int64_t)blockIdx.x * GB + tid;
  const bool valid = p < count;
  float xi[NI], h1[NH], h2[NH];
  float dy = 0.0f;
  if (valid) {
    const int64_t s = sample_index(seed, step, p0 + p, m, hashed != 0);
    for (int i = 0; i < NI; ++i) xi[i] = x[s * NI + i];
    for (int j = 0; j < NH; ++j) {
      float a = w[OB1 + j];
      for (int i = 0; i < NI; ++i) a = fmaf(w[OW1 + j * NI + i], xi[i], a);
      h1[j] = a > 0.0f ? a : 0.0f;
    }
    float y = w[OB3];
    for (int j = 0; j < NH; ++j) {
      float a = w[OB2 + j];
      for (int k = 0; k < NH; ++k) a = fmaf(w[OW2 + j * NH + k], h1[k], a);
      h2[j] = a > 0.0f ? a : 0.0f;
      y = fmaf(w[OW3 + j], h2[j], y);
    }
    const float e = y - t[s];
    dy = 2.0f * e / (float)count;
    LS[tid] = e * e;
  } else {
    for (int i = 0; i < NI; ++i) xi[i] = 0.0f;
    for (int j = 0; j < NH; ++j) h1[j] = h2[j] = 0.0f;
    LS[tid] = 0.0f;
  }
  float d2[NH];
  for (int j = 0; j < NH; ++j) d2[j] = h2[j] > 0.0f ? dy * w[OW3 + j] : 0.0f;
  for (int k = 0; k < NH; ++k) {
    float a = 0.0f;
    for (int j = 0; j < NH; ++j) a = fmaf(w[OW2 + j * NH + k], d2[j], a);
    D1[tid][k] = h1[k] > 0.0f ? a : 0.0f;
    H1[tid][k] = h1[k];
    H2[tid][k] = h2[k];
    D2[tid][k] = d2[k];
  }
  for (int i = 0; i < NI; ++i) X[tid][i] = xi[i];
  G[tid] = dy;
  __syncthreads();
  // block sums over the samples, one parameter per thread per pass
  for (int q = tid; q < NP; q += GB) {
    float acc = 0.0f;
    if (q < OB1) {
      const int j = q / NI, i = q % NI;
      for (int s = 0; s < GB; ++s) acc = fmaf(D1[s][j], X[s][i], acc);
    } else if (q < OW2) {
      const int j = q - OB1;
      for (int s = 0; s < GB; ++s) acc += D1[s][j];
    } else if (q < OB2) {
      const int j = (q - OW2) / NH, k = (q - OW2) % NH;
      for (int s = 0; s < GB; ++s) acc = fmaf(D2[s][j], H1[s][k], acc);
    } else if (q < OW3) {
      const int j = q - OB2;
      for (int s = 0; s < GB; ++s) acc += D2[s][j];
    } else if (q < OB3) {
      const int j = q - OW3;
      for (int s = 0; s < GB; ++s) acc = fmaf(G[s], H2[s][j], acc);
    } else {
      for (int s = 0; s < GB; ++s) acc += G[s];
    }
    atomicAdd(&grad[q], acc);
  }
  if (tid == 0) {
    float l = 0.0f;
    for (int s = 0; s < GB; ++s) l += LS[s];
    atomicAdd(loss, l);
  }
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m1, float* __restrict__ m2,
                       const float* __restrict__ g, float lr, float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= NP) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gq = g[q];
  const float a = b1 * m1[q] + (1.0f - b1) * gq;
  const float b = b2 * m2[q] + (1.0f - b2) * gq * gq;
  m1[q] = a;
  m2[q] = b;
  w[q] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

__global__ void k_zero_f32(float* p, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) p[i] = 0.0f;
}

// ---------------------------------------------------------------- schedule

// The census claims whole tasks BATCH consecutive CSR tasks at a time; in CSR
// order, neighbouring batches share rows u and keep N(u) in cache. A schedule
// keeps that order for the bulk of the queue and orders only its last batches
// costliest first (longest processing time first), so that no costly batch is
// claimed when the other wavefronts are about to run dry. Batch key: the sum
// over its tasks of the merge length d+(u) + d(v) - s(u, v) + SCHED_TASK_OH
// (heuristic; d+(u) the ids of N(u) above u, s the ids of N(v) below u) or of
// the network's predicted cycles (learned); tasks merged from the hub list add
// nothing. The
// order is a stable counting sort over SCHED_BPO bins per octave of the key,
// the first bin the costliest.
constexpr float SCHED_BPO = 4.0f;
// Per-task cost outside the merge, in merge entries: every task takes at
// least one merge round.
constexpr float SCHED_TASK_OH = 256.0f;
// Batches per chunk of the counting sort: one wavefront each in the scatter.
constexpr int64_t SCHED_CHUNK = 256;
// The reordering pays only when CSR order would leave a batch among the last
// ones claimed (about one per wavefront) costly enough to delay the whole
// census: one of the last SCHED_TAIL_LAST predicted to cost more than the
// mean of the last SCHED_TAIL_SAMPLE by SCHED_TAIL_SHARE / 10,000 of one
// wavefront's share of the census. The share is the total of d+(u)+d(v)+256
// over all tasks, per wavefront, converted to the key's units by the ratio of
// the key sum to the sum of d+(u)+d(v)+256 over the sample. Only the sample is keyed first; the rest of
// the stretch is keyed and the stretch reordered only when the test says so.
// Otherwise the queue keeps its CSR order, and with it the reuse of N(u)
// across batches.
constexpr int64_t SCHED_TAIL_LAST = 8192, SCHED_TAIL_SAMPLE = 32768;
constexpr int SCHED_TAIL_SHARE = 30;

__device__ __forceinline__ int key_bin(float key) {
  if (!(key < 1.0e4f)) return SCHED_BINS - 1;  // also an infinite or NaN key
  const int b = (int)floorf(key * SCHED_BPO);
  return b < 0 ? 0 : (b >= SCHED_BINS ? SCHED_BINS - 1 : b);
}

__device__ __forceinline__ float wave_sum_f32(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
  return x;
}

// Bin of batches from .. nbatch-1 (bin[b - from]), one wavefront per batch
// and one lane per task; with kval given, also the batch's key sum and its
// sum of d+(u)+d(v)+SCHED_TASK_OH (lval). Under the learned key every lane
// evaluates the network; the weights are read at wave-uniform addresses,
// through the scalar cache.
__global__ void __launch_bounds__(256) k_batch_keys(int mode, const float* __restrict__ gw,
                                                    const int64_t* __restrict__ off, const uint32_t* __restrict__ packed,
                                                    const uint64_t* __restrict__ tasks, int64_t ntasks, int64_t from,
                                                    int64_t nbatch, uint8_t* __restrict__ bin,
                                                    float* __restrict__ kval, float* __restrict__ lval,
                                                    const uint32_t* __restrict__ ustart,
                                                    const uint32_t* __restrict__ tskip,
                                                    const uint32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t bt = from + wave; bt < nbatch; bt += nwave) {
    const int64_t t = bt * BATCH + lane;
    uint32_t dp = 0, dv = 0, sv = 0, above = 0;
    bool live = false;
    if (t < ntasks) {
      const uint64_t tk = tasks[t];
      if (!(tk & HUB_BIT)) {
        const uint32_t u = (uint32_t)(tk >> 32) & 0x3FFFFFFFu, k = (uint32_t)tk;
        const int64_t au = off[u];
        const uint32_t du = (uint32_t)(off[u + 1] - au);
        dp = du - ustart[u];
        const uint32_t v = packed[au + k] >> 2;
        dv = (uint32_t)(off[v + 1] - off[v]);
        sv = min(tskip[t], dv);
        above = du - k - 1;
        live = true;
      }
    }
    const float len = (float)dp + (float)dv + SCHED_TASK_OH;
    float c = len - (float)sv;
    if (mode == 2) {
      float x[NI];
      task_features(dp, dv - sv, above, x);
      c = exp2f(mlp_forward(gw, x));
    }
    const float sum = wave_sum_f32(live ? c : 0.0f);
    if (kval) {
      const float lsum = wave_sum_f32(live ? len : 0.0f);
      if (lane == 0) {
        kval[bt - from] = sum;
        lval[bt - from] = lsum;
      }
    }
    if (lane == 0) bin[bt - from] = (uint8_t)(sum > 0.0f ? key_bin(log2f(sum)) : 0);
  }
}

// Each chunk's count per bin, bin-major: cnt[b * nchunks + c].
__global__ void __launch_bounds__(256) k_bin_count(const uint8_t* __restrict__ bin, int64_t m, int64_t chunk,
                                                   int64_t nchunks, unsigned int* __restrict__ cnt,
                                                   const uint32_t* __restrict__ skip) {
  if (skip && *skip) return;  // the bins were not all written
  __shared__ unsigned int h[SCHED_BINS];
  const int64_t c = blockIdx.x;
  for (int b = threadIdx.x; b < SCHED_BINS; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t i1 = min((c + 1) * chunk, m);
  for (int64_t i = c * chunk + threadIdx.x; i < i1; i += blockDim.x) atomicAdd(&h[bin[i]], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < SCHED_BINS; b += blockDim.x) cnt[(int64_t)b * nchunks + c] = h[b];
}

// Per bin (one block each): exclusive prefix of the chunk counts, in place as
// 64-bit offsets within the bin, and the bin's total.
__global__ void __launch_bounds__(256) k_bin_scan(const unsigned int* __restrict__ cnt, int64_t nchunks,
                                                  unsigned long long* __restrict__ pre, unsigned long long* __restrict__ total,
                                                  const uint32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ unsigned long long part[256];
  const int b = blockIdx.x, t = threadIdx.x;
  const int64_t per = (nchunks + 255) / 256, lo = min((int64_t)t * per, nchunks), hi = min(lo + per, nchunks);
  const unsigned int* row = cnt + (int64_t)b * nchunks;
  unsigned long long sum = 0;
  for (int64_t c = lo; c < hi; ++c) sum += row[c];
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    unsigned long long run = 0;
    for (int i = 0; i < 256; ++i) {
      const unsigned long long x = part[i];
      part[i] = run;
      run += x;
    }
    total[b] = run;
  }
  __syncthreads();
  unsigned long long run = part[t];
  unsigned long long* out = pre + (int64_t)b * nchunks;
  for (int64_t c = lo; c < hi; ++c) {
    out[c] = run;
    run += row[c];
  }
}

// Per block of rows: sum over rows u of d+(u)^2 + d(u) d-(u) (d- = ustart,
// d+ = d - d-), i.e. the summed merge length d+(u) + d(v) of all tasks.
__global__ void __launch_bounds__(256) k_list_sums(int64_t n, const int64_t* __restrict__ off,
                                                   const uint32_t* __restrict__ ustart,
                                                   unsigned long long* __restrict__ part) {
  __shared__ unsigned long long red[256];
  unsigned long long acc = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    const unsigned long long d = (unsigned long long)(off[u + 1] - off[u]), dm = ustart[u], dp = d - dm;
    acc += dp * dp + d * dm;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// skip[0] = 1 unless a batch among the last `last` of the sample kval[0, m)
// exceeds the sample mean by share / 10,000 of one wavefront's share of the
// census (share < 0: never skip). One block.
__global__ void __launch_bounds__(256) k_tail_decide(const float* __restrict__ kval, const float* __restrict__ lval,
                                                     int64_t m, int64_t last, const unsigned long long* __restrict__ part,
                                                     int nparts, int64_t ntasks, int64_t nwaves, int share,
                                                     uint32_t* __restrict__ skip) {
  __shared__ double rk[256], rl[256];
  __shared__ float rm[256];
  double sk = 0.0, sl = 0.0;
  float mx = 0.0f;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    sk += kval[i];
    sl += lval[i];
    if (i >= m - last) mx = fmaxf(mx, kval[i]);
  }
  rk[threadIdx.x] = sk;
  rl[threadIdx.x] = sl;
  rm[threadIdx.x] = mx;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int t = 1; t < (int)blockDim.x; ++t) {
    sk += rk[t];
    sl += rl[t];
    mx = fmaxf(mx, rm[t]);
  }
  unsigned long long total_len = 0;
  for (int b = 0; b < nparts; ++b) total_len += part[b];
  const double census = ((double)total_len + (double)SCHED_TASK_OH * (double)ntasks) * (sl > 0.0 ? sk / sl : 1.0);
  const double budget = (double)share * 1e-4 * census / (double)(nwaves > 0 ? nwaves : 1);
  skip[0] = share >= 0 && (double)mx - sk / (double)(m > 0 ? m : 1) <= budget ? 1u : 0u;
}

// Start of each bin in the costliest-first layout.
__global__ void k_bin_starts(unsigned long long* total, const uint32_t* __restrict__ skip) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || (skip && *skip)) return;
  unsigned long long run = 0;
  for (int b = SCHED_BINS - 1; b >= 0; --b) {
    const unsigned long long c = total[b];
    total[b] = run;
    run += c;
  }
}

// Stable scatter, one wavefront per chunk, 64 entries per step: lanes holding
// the same bin are ranked by lane order (their bin equality mask is built
// from one ballot per bin bit), after the chunk's earlier entries of that
// bin. Writes idx[position] = base + entry.
__global__ void __launch_bounds__(64) k_bin_scatter(const uint8_t* __restrict__ bin, int64_t m, int64_t chunk,
                                                    int64_t nchunks, const unsigned long long* __restrict__ pre,
                                                    const unsigned long long* __restrict__ start, int64_t base,
                                                    int64_t* __restrict__ idx, const uint32_t* __restrict__ skip) {
  if (skip && *skip) return;  // the whole block leaves together
  __shared__ unsigned long long next[SCHED_BINS];
  const int lane = threadIdx.x;
  const int64_t c = blockIdx.x;
  for (int b = lane; b < SCHED_BINS; b += 64) next[b] = start[b] + pre[(int64_t)b * nchunks + c];
  __syncthreads();
  const int64_t i0 = c * chunk, i1 = min(i0 + chunk, m);
  const uint64_t below = (1ull << lane) - 1;
  for (int64_t s0 = i0; s0 < i1; s0 += 64) {
    const int64_t i = s0 + lane;
    const bool act = i < i1;
    const uint32_t b = act ? bin[i] : (uint32_t)SCHED_BINS;  // no bin matches an idle lane
    uint64_t eq = ~0ull;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t mk = __ballot((b >> k) & 1u);
      eq &= ((b >> k) & 1u) ? mk : ~mk;
    }
    if (act) idx[next[b] + (unsigned long long)__popcll(eq & below)] = base + i;
    __syncthreads();
    if (act && (eq >> lane) == 1ull) next[b] += (unsigned long long)__popcll(eq);  // last lane of its group
    __syncthreads();
  }
}

static int grid_of(int64_t work, int threads, int cap) {
  int64_t g = (work + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// idx = base + the entries 0..m-1 ordered by bin, highest bin first, stable
// (nothing is written when *skip is set).
static int stable_bin_order(const uint8_t* bin, int64_t m, int64_t chunk, int64_t base, int64_t* idx,
                            const uint32_t* skip, Scratch& scratch, hipStream_t s) {
  const int64_t nchunks = (m + chunk - 1) / chunk;
  unsigned int* cnt = nullptr;
  unsigned long long* pre = nullptr;
  unsigned long long* start = nullptr;
  ALLOC(cnt, nchunks * SCHED_BINS);
  ALLOC(pre, nchunks * SCHED_BINS);
  ALLOC(start, SCHED_BINS);
  hipLaunchKernelGGL(k_bin_count, dim3((unsigned)nchunks), dim3(256), 0, s, bin, m, chunk, nchunks, cnt, skip);
  hipLaunchKernelGGL(k_bin_scan, dim3(SCHED_BINS), dim3(256), 0, s, cnt, nchunks, pre, start, skip);
  hipLaunchKernelGGL(k_bin_starts, dim3(1), dim3(64), 0, s, start, skip);
  hipLaunchKernelGGL(k_bin_scatter, dim3((unsigned)nchunks), dim3(64), 0, s, bin, m, chunk, nchunks, pre, start, base,
                     idx, skip);
  HIPCHK(hipGetLastError());
  return TRIAD_OK;
}

// Queue batch from + i takes task batch border[i]: the task words moved into
// tmp (then copied back), or the task indices written to order.
__global__ void k_apply_batches(const int64_t* __restrict__ border, int64_t from, int64_t tail,
                                const uint64_t* __restrict__ tasks, const uint32_t* __restrict__ tskip,
                                uint64_t* __restrict__ tmp, uint32_t* __restrict__ tmp_skip,
                                int64_t* __restrict__ order, const uint32_t* __restrict__ skip) {
  if (*skip) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, m = tail * BATCH;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
    const int64_t src = border[j / BATCH] * BATCH + (j % BATCH);
    if (order) {
      order[from * BATCH + j] = src;
    } else {
      tmp[j] = tasks[src];
      tmp_skip[j] = tskip[src];
    }
  }
}

__global__ void k_copy_back(const uint64_t* __restrict__ tmp, const uint32_t* __restrict__ tmp_skip, int64_t m,
                            uint64_t* __restrict__ dst, uint32_t* __restrict__ dst_skip,
                            const uint32_t* __restrict__ skip) {
  if (*skip) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
    dst[j] = tmp[j];
    dst_skip[j] = tmp_skip[j];
  }
}

__global__ void k_iota64(int64_t* __restrict__ p, int64_t m) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) p[j] = j;
}

int schedule_tail(int mode, const float* model, int64_t n, const int64_t* off, const uint32_t* ustart,
                  const uint32_t* packed, uint64_t* tasks, uint32_t* tskip, int64_t ntasks, int64_t* order,
                  int32_t tail_share, int64_t nwaves, Scratch& scratch, hipStream_t s) {
  if (mode == 2 && !model) return fail(TRIAD_EINVAL, "learned schedule without a model");
  if (order && ntasks > 0) hipLaunchKernelGGL(k_iota64, dim3(grid_of(ntasks, 256, 65536)), dim3(256), 0, s, order, ntasks);
  // full batches only: a partial last batch stays last
  const int64_t nfull = ntasks / BATCH;
  const int64_t tail = std::min(nfull, std::max(nfull / SCHED_TAIL_DIV, SCHED_TAIL_MIN)), from = nfull - tail;
  if (tail <= 0) return TRIAD_OK;
  uint8_t* bin = nullptr;
  int64_t* border = nullptr;
  uint32_t* skip = nullptr;
  ALLOC(bin, tail);
  ALLOC(border, tail);
  ALLOC(skip, 1);
  // key the last batches, decide, then key the rest of the stretch if needed
  const int64_t ns = std::min(tail, SCHED_TAIL_SAMPLE);
  const int share = tail_share == 0 ? SCHED_TAIL_SHARE : (tail_share < 0 ? -1 : tail_share);
  constexpr int NPARTS = 1024;
  float *kval = nullptr, *lval = nullptr;
  unsigned long long* part = nullptr;
  ALLOC(kval, ns);
  ALLOC(lval, ns);
  ALLOC(part, NPARTS);
  hipLaunchKernelGGL(k_list_sums, dim3(NPARTS), dim3(256), 0, s, n, off, ustart, part);
  hipLaunchKernelGGL(k_batch_keys, dim3(grid_of(ns, 4, 65536)), dim3(256), 0, s, mode, model, off, packed,
                     (const uint64_t*)tasks, ntasks, nfull - ns, nfull, bin + (tail - ns), kval, lval, ustart,
                     (const uint32_t*)tskip, (const uint32_t*)nullptr);
  hipLaunchKernelGGL(k_tail_decide, dim3(1), dim3(256), 0, s, (const float*)kval, (const float*)lval, ns,
                     SCHED_TAIL_LAST, (const unsigned long long*)part, NPARTS, ntasks, nwaves, share, skip);
  if (tail > ns)
    hipLaunchKernelGGL(k_batch_keys, dim3(grid_of(tail - ns, 4, 65536)), dim3(256), 0, s, mode, model, off, packed,
                       (const uint64_t*)tasks, ntasks, from, nfull - ns, bin, (float*)nullptr, (float*)nullptr,
                       ustart, (const uint32_t*)tskip, (const uint32_t*)skip);
  if (int st = stable_bin_order(bin, tail, SCHED_CHUNK, from, border, skip, scratch, s)) return st;
  // the task words move together with their N(v) skip counts
  uint64_t* tmp = nullptr;
  uint32_t* tmp_skip = nullptr;
  if (!order) {
    ALLOC(tmp, tail * BATCH);
    ALLOC(tmp_skip, tail * BATCH);
  }
  hipLaunchKernelGGL(k_apply_batches, dim3(grid_of(tail * BATCH, 256, 65536)), dim3(256), 0, s, (const int64_t*)border,
                     from, tail, (const uint64_t*)tasks, (const uint32_t*)tskip, tmp, tmp_skip, order,
                     (const uint32_t*)skip);
  if (!order)
    hipLaunchKernelGGL(k_copy_back, dim3(grid_of(tail * BATCH, 256, 65536)), dim3(256), 0, s, (const uint64_t*)tmp,
                       (const uint32_t*)tmp_skip, tail * BATCH, tasks + from * BATCH, tskip + from * BATCH,
                       (const uint32_t*)skip);
  HIPCHK(hipGetLastError());
  return TRIAD_OK;
}

}  // namespace triad

using namespace triad;

extern "C" {

int triad_task_features(int64_t n, int64_t nnz, const int64_t* off, const int32_t* nbr, void* stream, float* d_feat,
                        int64_t* ntasks_out) {
  hipStream_t s = (hipStream_t)stream;
  if (n < 0 || n >= ((int64_t)1 << 30) || nnz < 0) return fail(TRIAD_EINVAL, "bad sizes");
  if (!off || (nnz > 0 && !nbr)) return fail(TRIAD_EINVAL, "NULL pointer argument");
  Scratch scratch(s);
  int64_t* ntask = nullptr;
  int64_t* tpre = nullptr;
  ALLOC(ntask, n + 1);
  ALLOC(tpre, n + 1);
  int64_t total = 0;
  if (n > 0) {
    hipLaunchKernelGGL(k_task_counts, dim3(grid_of(n, 256, 65535)), dim3(256), 0, s, n, off, nbr, ntask);
    // exclusive prefix of the per-row task counts (host side: this entry point
    // prepares training data and is not on the census path)
    std::vector<int64_t> h((size_t)n + 1);
    HIPCHK(hipMemcpyAsync(h.data(), ntask, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t run = 0;
    for (int64_t u = 0; u < n; ++u) {
      const int64_t c = h[u];
      h[u] = run;
      run += c;
    }
    h[n] = run;
    total = run;
    HIPCHK(hipMemcpyAsync(tpre, h.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    if (d_feat && total > 0)
      hipLaunchKernelGGL(k_features_csr, dim3(grid_of(n * 64, 256, 32768)), dim3(256), 0, s, n, off, nbr, tpre, d_feat);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  }
  if (ntasks_out) *ntasks_out = total;
  return TRIAD_OK;
}

int triad_mlp_forward(const float* d_w, const float* d_x, int64_t m, float* d_y, void* stream) {
  if (!d_w || (m > 0 && (!d_x || !d_y)) || m < 0) return fail(TRIAD_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  if (m > 0) hipLaunchKernelGGL(k_mlp_forward, dim3(grid_of(m, 256, 65535)), dim3(256), 0, s, d_w, d_x, m, d_y);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return TRIAD_OK;
}

int triad_mlp_loss_grad(const float* d_w, const float* d_x, const float* d_t, int64_t m, float* d_grad, float* d_loss,
                        void* stream) {
  if (!d_w || !d_grad || !d_loss || m <= 0 || !d_x || !d_t) return fail(TRIAD_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_f32, dim3(grid_of(NP, 256, 64)), dim3(256), 0, s, d_grad, (int64_t)NP);
  hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, d_loss, (int64_t)1);
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)((m + GB - 1) / GB)), dim3(GB), 0, s, d_w, d_x, d_t, m, (int64_t)0, m,
                     (uint64_t)0, (uint64_t)0, 0, d_grad, d_loss);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  // the kernel accumulates the squared-error sum; report the mean
  float l = 0;
  HIPCHK(hipMemcpy(&l, d_loss, sizeof(float), hipMemcpyDeviceToHost));
  l /= (float)m;
  HIPCHK(hipMemcpy(d_loss, &l, sizeof(float), hipMemcpyHostToDevice));
  return TRIAD_OK;
}

int triad_mlp_adam(float* d_w, float* d_m, float* d_v, const float* d_grad, int32_t t, float lr, void* stream) {
  if (!d_w || !d_m || !d_v || !d_grad || t < 1) return fail(TRIAD_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, s, d_w, d_m, d_v, d_grad, lr, c1, c2);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return TRIAD_OK;
}

int triad_mlp_train(float* d_w, const float* d_x, const float* d_t, int64_t m, int32_t epochs, int32_t batch, float lr,
                    uint64_t seed, void* stream, float* d_loss_hist) {
  if (!d_w || !d_x || !d_t || m <= 0 || epochs < 1 || batch < 1) return fail(TRIAD_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  Scratch scratch(s);
  float *m1 = nullptr, *m2 = nullptr, *g = nullptr, *loss = nullptr;
  ALLOC(m1, NP);
  ALLOC(m2, NP);
  ALLOC(g, NP);
  ALLOC(loss, epochs);
  hipLaunchKernelGGL(k_zero_f32, dim3(8), dim3(256), 0, s, m1, (int64_t)NP);
  hipLaunchKernelGGL(k_zero_f32, dim3(8), dim3(256), 0, s, m2, (int64_t)NP);
  hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, loss, (int64_t)epochs);
  const int64_t steps = (m + batch - 1) / batch;
  int32_t t = 0;
  for (int e = 0; e < epochs; ++e) {
    for (int64_t st = 0; st < steps; ++st) {
      ++t;
      hipLaunchKernelGGL(k_zero_f32, dim3(8), dim3(256), 0, s, g, (int64_t)NP);
      // minibatch of `batch` samples drawn with replacement by a counter-based hash
      hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)((batch + GB - 1) / GB)), dim3(GB), 0, s, (const float*)d_w, d_x,
                         d_t, m, (int64_t)0, (int64_t)batch, seed, (uint64_t)t, 1, g, loss + e);
      const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
      hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, s, d_w, m1, m2, (const float*)g, lr, c1, c2);
    }
  }
  HIPCHK(hipGetLastError());
  if (d_loss_hist) {
    std::vector<float> h((size_t)epochs);
    HIPCHK(hipMemcpyAsync(h.data(), loss, sizeof(float) * epochs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (auto& x : h) x /= (float)(steps * batch);
    HIPCHK(hipMemcpyAsync(d_loss_hist, h.data(), sizeof(float) * epochs, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  return TRIAD_OK;
}

}  // extern "C"
