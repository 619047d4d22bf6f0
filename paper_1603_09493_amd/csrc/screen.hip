// Screening round of the learned surrogate: candidate designs from Philox4x32-10 uniforms, a score
// per design, and an exact top-k (ties to the lower index) by radix selection.
//
// In the paper (Sec. II.A) the optimizer proposes the next design from a surrogate of the
// objective; here a whole round of candidates is scored at once and only the best are handed
// to the batched solver, which stays the judge.
#include <cmath>

#include "bpm_internal.h"
#include <mutex>

#include "mlp_internal.h"
#include "philox.h"

namespace bpm {

// X[i][f] = 2 u - 1 with u = (x + 1/2) 2^-32 from Philox(key = seed, counter = (i, call)), three
// calls per design give the 12 uniforms in order.
__global__ void sample_kernel(uint64_t seed, long n, float* __restrict__ X) {
  const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    for (uint32_t call = 0; call < 3; ++call) {
      const uint4 r = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)((uint64_t)i >> 32), call, 0u), key);
      const uint32_t w[4] = {r.x, r.y, r.z, r.w};
      for (int q = 0; q < 4; ++q) {
        const double u = ((double)w[q] + 0.5) * (1.0 / 4294967296.0);
        X[i * kMlpIn + 4 * call + q] = (float)(2.0 * u - 1.0);
      }
    }
  }
}

hipError_t sample_designs(uint64_t seed, long n, float* X, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sample_kernel, dim3(2048), dim3(256), 0, s, seed, n, X);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// network inputs of sampled designs, in place: a sample X = 2u - 1 stands for the design
// x = lo + (hi - lo) u (uniform prior); features with lo > 0 become log coordinates
// 2 log(x / lo) / log(hi / lo) - 1, the others stay 2u - 1
// ---------------------------------------------------------------------------------------------
struct Range {
  double lo[12], hi[12];
};

__global__ void features_kernel(float* __restrict__ X, long n, Range R) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    for (int f = 0; f < 12; ++f) {
      if (!(R.lo[f] > 0.0)) continue;
      const double u = 0.5 * ((double)X[i * kMlpIn + f] + 1.0);
      const double x = R.lo[f] + (R.hi[f] - R.lo[f]) * u;
      X[i * kMlpIn + f] = (float)(2.0 * log(x / R.lo[f]) / log(R.hi[f] / R.lo[f]) - 1.0);
    }
  }
}

hipError_t design_features(float* X, long n, const double* lo, const double* hi, hipStream_t s) {
  Range R;
  for (int f = 0; f < 12; ++f) {
    R.lo[f] = lo[f];
    R.hi[f] = hi[f];
  }
  hipLaunchKernelGGL(features_kernel, dim3(2048), dim3(256), 0, s, X, n, R);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// score: predicted logit of switching where the thermal-stability proxy
// (K_s V_s + K_h V_h) / (kB 300 K) reaches min_stability, else -inf
// design features (indices): 0 d, 1 t_soft, 2 t_hard, 5 K_soft, 6 K_hard; a feature with a
// positive lower bound is a log coordinate (x = lo (hi / lo)^u), else linear (x = lo + (hi - lo) u)
// ---------------------------------------------------------------------------------------------

__global__ void score_kernel(const float* __restrict__ X, const float* __restrict__ Y, long n, Range R,
                             double min_stab, float* __restrict__ score) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double p[12];
    for (int f = 0; f < 12; ++f) {
      const double u = 0.5 * ((double)X[i * kMlpIn + f] + 1.0);
      p[f] = R.lo[f] > 0.0 ? R.lo[f] * pow(R.hi[f] / R.lo[f], u) : R.lo[f] + (R.hi[f] - R.lo[f]) * u;
    }
    const double area = kPi * 0.25 * p[0] * p[0];
    const double stab = (p[5] * area * p[1] + p[6] * area * p[2]) / (kBoltzmann * 300.0);
    score[i] = stab >= min_stab ? Y[i * kMlpOut + 2] : -INFINITY;
  }
}

hipError_t screen_score(const float* X, const float* Y, long n, const double* lo, const double* hi, double min_stab,
                        float* score, hipStream_t s) {
  Range R;
  for (int f = 0; f < 12; ++f) {
    R.lo[f] = lo[f];
    R.hi[f] = hi[f];
  }
  hipLaunchKernelGGL(score_kernel, dim3(2048), dim3(256), 0, s, X, Y, n, R, min_stab, score);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// exact top-k: keys order like the scores (NaN lowest); four 8-bit radix passes find the k-th
// largest key T and how many of the keys equal to T are taken; the keys above T and the first
// of the ties by index are gathered and sorted by (key desc, index asc) in one workgroup
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t order_key(float s) {
  if (isnan(s)) return 0u;
  const uint32_t u = __float_as_uint(s);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// state: [0] prefix, [1] mask, [2] k remaining, [3] count of keys above the threshold (gather)
__global__ void radix_hist_kernel(const float* __restrict__ score, long n, int shift, uint32_t* __restrict__ hist,
                                  const uint32_t* __restrict__ state) {
  __shared__ uint32_t h[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const uint32_t prefix = state[0], mask = state[1];
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const uint32_t key = order_key(score[i]);
    if ((key & mask) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ void radix_pick_kernel(int shift, uint32_t* __restrict__ hist, uint32_t* __restrict__ state) {
  if (threadIdx.x == 0) {
    uint32_t krem = state[2], cum = 0;
    int digit = 0;
    for (int d = 255; d >= 0; --d) {
      if (cum + hist[d] >= krem) {
        digit = d;
        break;
      }
      cum += hist[d];
    }
    state[0] |= (uint32_t)digit << shift;
    state[1] |= 255u << shift;
    state[2] = krem - cum;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
}

constexpr int kTieBlock = 1024;

// keys above the threshold go to cand[0 .. k - k_rem) in any order; ties are counted per block
__global__ void gather_above_kernel(const float* __restrict__ score, long n, uint32_t* __restrict__ state,
                                    unsigned long long* __restrict__ cand, uint32_t* __restrict__ blk) {
  const uint32_t T = state[0];
  const long base = (long)blockIdx.x * kTieBlock;
  uint32_t ties = 0;
  for (int j = threadIdx.x; j < kTieBlock; j += blockDim.x) {
    const long i = base + j;
    if (i >= n) break;
    const uint32_t key = order_key(score[i]);
    if (key > T) {
      const uint32_t pos = atomicAdd(&state[3], 1u);
      cand[pos] = ((unsigned long long)key << 32) | (uint32_t)~(uint32_t)i;
    } else if (key == T) {
      ++ties;
    }
  }
  for (int o = 32; o > 0; o >>= 1) ties += __shfl_xor(ties, o, 64);
  __shared__ uint32_t red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ties;
  __syncthreads();
  if (threadIdx.x == 0) blk[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// exclusive scan of the per-block tie counts (one workgroup, sequential chunks)
__global__ void scan_blocks_kernel(uint32_t* __restrict__ blk, long nblk) {
  __shared__ uint32_t carry;
  __shared__ uint32_t buf[256];
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (long b0 = 0; b0 < nblk; b0 += 256) {
    const long b = b0 + threadIdx.x;
    const uint32_t v = b < nblk ? blk[b] : 0u;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0u;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (b < nblk) blk[b] = carry + buf[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 255) carry += buf[255];
    __syncthreads();
  }
}

// ties in index order: the first k_rem of them follow the keys above the threshold
__global__ void gather_ties_kernel(const float* __restrict__ score, long n, long k, const uint32_t* __restrict__ state,
                                   unsigned long long* __restrict__ cand, const uint32_t* __restrict__ blk) {
  const uint32_t T = state[0], krem = state[2];
  const long base = (long)blockIdx.x * kTieBlock;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __shared__ uint32_t wcount[4];
  uint32_t run = blk[blockIdx.x];
  // the block is walked in chunks of 256 consecutive indices, waves in order
  for (int j0 = 0; j0 < kTieBlock; j0 += 256) {
    const long i = base + j0 + threadIdx.x;
    const bool tie = i < n && order_key(score[i]) == T;
    const unsigned long long bal = __ballot(tie);
    const uint32_t before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[wid] = __popcll(bal);
    __syncthreads();
    uint32_t woff = 0;
    for (int w = 0; w < wid; ++w) woff += wcount[w];
    const uint32_t rank = run + woff + before;
    if (tie && rank < krem) cand[(k - krem) + rank] = ((unsigned long long)T << 32) | (uint32_t)~(uint32_t)i;
    run += wcount[0] + wcount[1] + wcount[2] + wcount[3];
    __syncthreads();
  }
}

// bitonic sort of the k candidates (descending composite) and index output
__global__ void sort_out_kernel(long k, const unsigned long long* __restrict__ cand, int64_t* __restrict__ idx) {
  extern __shared__ unsigned long long sk[];
  long P = 1;
  while (P < k) P <<= 1;
  for (long i = threadIdx.x; i < P; i += blockDim.x) sk[i] = i < k ? cand[i] : 0ull;
  __syncthreads();
  for (long size = 2; size <= P; size <<= 1)
    for (long stride = size >> 1; stride > 0; stride >>= 1) {
      for (long i = threadIdx.x; i < P; i += blockDim.x) {
        const long j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;
          const unsigned long long a = sk[i], b = sk[j];
          if (desc ? (a < b) : (a > b)) {
            sk[i] = b;
            sk[j] = a;
          }
        }
      }
      __syncthreads();
    }
  for (long i = threadIdx.x; i < k; i += blockDim.x) idx[i] = (int64_t)(uint32_t)~(uint32_t)(sk[i] & 0xffffffffull);
}

// ---------------------------------------------------------------------------------------------
// Allocation-free top-k: the same kernels on a fixed scratch area in device memory that the library
// holds for the whole process (one copy per GPU), for callers that cannot allocate.
// ---------------------------------------------------------------------------------------------
constexpr long kTopkNoAllocBlk = kTopkNoAllocMaxN / kTieBlock;            // per-block tie counts
constexpr size_t kScratchHist = 0;                                        // uint32 [256]
constexpr size_t kScratchState = kScratchHist + 256 * sizeof(uint32_t);   // uint32 [16]
constexpr size_t kScratchCand = kScratchState + 16 * sizeof(uint32_t);    // uint64 [kTopkMax]
constexpr size_t kScratchBlk = kScratchCand + kTopkMax * sizeof(unsigned long long);   // uint32 [blk]
constexpr size_t kScratchBytes = (kScratchBlk + kTopkNoAllocBlk * sizeof(uint32_t) + 255) / 256 * 256;
static_assert(kScratchBytes == kTopkNoAllocScratchBytes, "scratch size stated in the header");
static_assert(kScratchCand % 8 == 0 && kScratchBlk % 4 == 0, "aligned sub-arrays");

// Host code must not pass this name to a kernel: it is a host-side stand-in.  The device address of
// each GPU's copy comes from hipGetSymbolAddress (scratch_dev below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices] = {};

hipError_t topk_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_dev[device] = p;
  return hipSuccess;
}

// state of a selection: prefix 0, mask 0, k remaining = k, gather count 0; histogram cleared (a
// kernel rather than a memset, so that the sequence can be recorded in a graph)
__global__ void topk_reset_kernel(uint32_t* __restrict__ hist, uint32_t* __restrict__ state, uint32_t k) {
  for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0u;
  if (threadIdx.x < 16) state[threadIdx.x] = threadIdx.x == 2 ? k : 0u;
}

hipError_t topk_select_noalloc(const float* score, long n, long k, int64_t* idx, int device, hipStream_t s) {
  if (n <= 0 || n > kTopkNoAllocMaxN || k <= 0 || k > n || k > kTopkMax) return hipErrorInvalidValue;
  hipError_t e = topk_scratch_init(device);
  if (e != hipSuccess) return e;
  unsigned char* base = static_cast<unsigned char*>(g_scratch_dev[device]);
  uint32_t* hist = reinterpret_cast<uint32_t*>(base + kScratchHist);
  uint32_t* state = reinterpret_cast<uint32_t*>(base + kScratchState);
  unsigned long long* cand = reinterpret_cast<unsigned long long*>(base + kScratchCand);
  uint32_t* blk = reinterpret_cast<uint32_t*>(base + kScratchBlk);
  const long nblk = (n + kTieBlock - 1) / kTieBlock;
  hipLaunchKernelGGL(topk_reset_kernel, dim3(1), dim3(256), 0, s, hist, state, (uint32_t)k);
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    hipLaunchKernelGGL(radix_hist_kernel, dim3(1024), dim3(256), 0, s, score, n, shift, hist, state);
    hipLaunchKernelGGL(radix_pick_kernel, dim3(1), dim3(256), 0, s, shift, hist, state);
  }
  hipLaunchKernelGGL(gather_above_kernel, dim3((unsigned)nblk), dim3(256), 0, s, score, n, state, cand, blk);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(256), 0, s, blk, nblk);
  hipLaunchKernelGGL(gather_ties_kernel, dim3((unsigned)nblk), dim3(256), 0, s, score, n, k, state, cand, blk);
  long P = 1;
  while (P < k) P <<= 1;
  const size_t shm = (size_t)P * sizeof(unsigned long long);
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&sort_out_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(sort_out_kernel, dim3(1), dim3(1024), shm, s, k, cand, idx);
  return hipGetLastError();
}

hipError_t topk_select(const float* score, long n, long k, int64_t* idx, ScreenScratch& sc, hipStream_t s) {
  hipError_t e;
  const long nblk = (n + kTieBlock - 1) / kTieBlock;
  if (!sc.hist) {
    if ((e = hipMalloc(&sc.hist, 256 * sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = hipMalloc(&sc.state, 8 * sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = hipMalloc(&sc.cand, kTopkMax * sizeof(unsigned long long))) != hipSuccess) return e;
  }
  if (sc.blk_cap < nblk) {
    if (sc.blk) hipFree(sc.blk);
    if ((e = hipMalloc(&sc.blk, nblk * sizeof(uint32_t))) != hipSuccess) return e;
    sc.blk_cap = nblk;
  }
  const uint32_t init[8] = {0u, 0u, (uint32_t)k, 0u, 0u, 0u, 0u, 0u};
  if ((e = hipMemcpyAsync(sc.state, init, sizeof(init), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(sc.hist, 0, 256 * sizeof(uint32_t), s)) != hipSuccess) return e;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    hipLaunchKernelGGL(radix_hist_kernel, dim3(1024), dim3(256), 0, s, score, n, shift, sc.hist, sc.state);
    hipLaunchKernelGGL(radix_pick_kernel, dim3(1), dim3(256), 0, s, shift, sc.hist, sc.state);
  }
  hipLaunchKernelGGL(gather_above_kernel, dim3((unsigned)nblk), dim3(256), 0, s, score, n, sc.state, sc.cand, sc.blk);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(256), 0, s, sc.blk, nblk);
  hipLaunchKernelGGL(gather_ties_kernel, dim3((unsigned)nblk), dim3(256), 0, s, score, n, k, sc.state, sc.cand, sc.blk);
  long P = 1;
  while (P < k) P <<= 1;
  const size_t shm = (size_t)P * sizeof(unsigned long long);
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&sort_out_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(sort_out_kernel, dim3(1), dim3(1024), shm, s, k, sc.cand, idx);
  return hipGetLastError();
}

}  // namespace bpm
