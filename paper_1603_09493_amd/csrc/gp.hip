// Expected improvement of the optimiser's kriging model at a large set of candidates (the
// efficient global optimisation of Sec. II.A evaluates the candidate of largest EI).
//
// With R = L L' the training correlation matrix, r the correlations of a candidate with the n
// training points and G the (n + 2) x n matrix [L^-1; alpha'; w'] (alpha = R^-1 (y - 1 mu),
// w = R^-1 1), one product v = G r gives
//   q = |v_0..n-1|^2 = r' R^-1 r,   yhat = mu + v_n,   p = v_{n+1} = 1' R^-1 r,
//   s^2 = sigma^2 (1 - q + (1 - p)^2 / c),  c = 1' R^-1 1,
//   EI = (f_min - yhat) Phi(z) + s phi(z),  z = (f_min - yhat) / s.
// For a block of 64 candidates, L^-1 times their correlations is an n x n by n x 64 matrix
// product, done on the FP64 matrix cores (16 x 16 x 4 steps): each of the four waves owns 16
// candidates and every 16-row tile of a 128-row pass, the correlations are formed while a
// 16-column slice of them is staged in LDS beside the same columns of L^-1, and tiles wholly above
// the diagonal of L^-1 are skipped; alpha' r and w' r are summed while the correlations are formed.
// FP64 throughout (the variance is a difference of nearly equal terms near training points).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "bpm_internal.h"
#include "philox.h"

namespace bpm {

namespace {

constexpr int kGpBS = 256;
constexpr int kGpC = 64;              // candidates per block, 16 per wave
constexpr int kGpK = 16;              // columns of G per LDS stage
constexpr int kGpRT = 8;              // 16-row tiles of L^-1 per pass over the correlations
constexpr int kGpRows = 16 * kGpRT;
static_assert(kGpBS == 4 * kGpC, "four threads form the correlations of each candidate");
static_assert(kGpK % 4 == 0, "a stage is a whole number of 4-deep matrix-core steps");

typedef double gp_d4 __attribute__((ext_vector_type(4)));

// At three or more waves per SIMD the compiler keeps the 32 accumulators of a lane in ordinary
// vector registers (126 in all, four waves per SIMD) instead of 118 + 64 accumulation registers
// (two waves); the extra waves hide the LDS and L2 latency of the staging, 1.4x faster.
__global__ __launch_bounds__(kGpBS) __attribute__((amdgpu_waves_per_eu(3, 8))) void gp_ei_kernel(GpArgs a, long m, double* __restrict__ cand,
                                                      uint64_t seed, double* __restrict__ yhat,
                                                      double* __restrict__ sd, double* __restrict__ ei) {
  __shared__ double xc[kGpC][kMaxGpDim + 1];   // odd row stride: the 64 candidates of a wave
                                               // read one coordinate each from different banks
  __shared__ double Rt[kGpK][kGpC + 1];
  __shared__ double Gt[kGpRows][kGpK + 1];
  __shared__ double th[kMaxGpDim];
  __shared__ double red[2][kGpBS];
  __shared__ double qs[kGpC];
  const int t = threadIdx.x;
  const long c0 = (long)blockIdx.x * kGpC;
  const int d = a.d, n = a.n;
  if (t < d) th[t] = a.theta[t];
  // candidates of this block: generated (Philox, counter (index, dimension / 4)) or read
  for (int e = t; e < kGpC * d; e += kGpBS) {
    const int cc = e / d, l = e - cc * d;
    const long c = c0 + cc;
    double x = 0.0;
    if (c < m) {
      if (seed) {
        const uint4 w = philox4x32_10(make_uint4((uint32_t)c, (uint32_t)((uint64_t)c >> 32), (uint32_t)(l >> 2), 0u),
                                      make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
        x = philox_uniform(ws[l & 3]);
        cand[c * d + l] = x;
      } else {
        x = cand[c * d + l];
      }
    }
    xc[cc][l] = x;
  }
  // matrix-core operands: A = 16 rows x 4 columns of L^-1 (lane: row li, column lk), B = 4
  // columns x 16 candidates of the correlations (lane: column lk, candidate li); the 16 x 16 result
  // leaves rows 4 lk .. 4 lk + 3 of candidate li in each lane
  const int lane = t & 63, wv = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ccr = t & (kGpC - 1);        // the candidate whose correlations this thread forms
  const double* alpha = a.G + (size_t)n * n;
  const double* wv_ = a.G + (size_t)(n + 1) * n;
  double qa = 0.0;                       // |L^-1 r|^2 of candidate 16 wv + li, partial over rows
  double ya = 0.0, pa = 0.0;             // alpha' r and w' r of candidate ccr, partial over its j
  const int np = (n + kGpRows - 1) / kGpRows;   // 128-row passes
  for (int p = 0; p < np; ++p) {
    const int r0 = kGpRows * p;
    const bool last = p == np - 1;
    // rows of L^-1 below r0 + 128 have no entries beyond column r0 + 127; the last pass also
    // forms alpha' r and w' r, so it covers every column
    const int kmax = last ? n : r0 + kGpRows;
    gp_d4 acc[kGpRT];
#pragma unroll
    for (int q = 0; q < kGpRT; ++q) acc[q] = gp_d4{0.0, 0.0, 0.0, 0.0};
    for (int j0 = 0; j0 < kmax; j0 += kGpK) {
      __syncthreads();
      for (int e = t; e < kGpK * kGpC; e += kGpBS) {
        const int jj = e / kGpC, cc = e - jj * kGpC;
        const int j = j0 + jj;
        double r = 0.0;
        if (j < n) {
          double s = 0.0;
          for (int l = 0; l < d; ++l) {
            const double u = xc[cc][l] - a.X[(size_t)j * d + l];
            s += th[l] * u * u;
          }
          r = exp(-s);
          if (last) {
            ya = fma(alpha[j], r, ya);
            pa = fma(wv_[j], r, pa);
          }
        }
        Rt[jj][cc] = r;
      }
      for (int e = t; e < kGpRows * kGpK; e += kGpBS) {
        const int ii = e / kGpK, jj = e - ii * kGpK;
        const int i = r0 + ii, j = j0 + jj;
        Gt[ii][jj] = (i < n && j < n) ? a.G[(size_t)i * n + j] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int s4 = 0; s4 < kGpK / 4; ++s4) {
        const int jk = j0 + 4 * s4;      // first column of this step
        const double bv = Rt[4 * s4 + lk][16 * wv + li];
#pragma unroll
        for (int q = 0; q < kGpRT; ++q) {
          const int rlo = r0 + 16 * q;
          // (wave-uniform) rows past n, or columns wholly above this tile's part of the triangle
          if (rlo >= n || jk > rlo + 15) continue;
          const double av = Gt[16 * q + li][4 * s4 + lk];
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
        }
      }
    }
    // rows at or past n hold zeros (their rows of G were staged as zeros)
#pragma unroll
    for (int q = 0; q < kGpRT; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) qa = fma(acc[q][r], acc[q][r], qa);
  }
  // |L^-1 r|^2: sums over the four lane groups (lk) that hold rows of the same candidate
  qa += __shfl_xor(qa, 16);
  qa += __shfl_xor(qa, 32);
  // alpha' r and w' r: sums over the four threads that formed correlations of one candidate
  red[0][t] = ya;
  red[1][t] = pa;
  if (lk == 0) qs[16 * wv + li] = qa;
  __syncthreads();
  if (t < kGpC) {
    const int cl = t;
    const long c = c0 + cl;
    if (c < m) {
      const double yv = red[0][cl] + red[0][cl + 64] + red[0][cl + 128] + red[0][cl + 192];
      const double pv = red[1][cl] + red[1][cl + 64] + red[1][cl + 128] + red[1][cl + 192];
      const double mu = a.mu + yv;
      const double one_p = 1.0 - pv;
      const double var = a.sigma2 * (1.0 - qs[cl] + one_p * one_p / a.c);
      const double s = var > 0.0 ? sqrt(var) : 0.0;
      const double imp = a.f_min - mu;
      double e;
      if (s > 0.0) {
        const double z = imp / s;
        e = imp * 0.5 * erfc(-z * 0.70710678118654752440) + s * 0.39894228040143267794 * exp(-0.5 * z * z);
      } else {
        e = imp > 0.0 ? imp : 0.0;
      }
      if (yhat) yhat[c] = mu;
      if (sd) sd[c] = s;
      ei[c] = e;
    }
  }
}

// largest value of v [m] and its lowest index: per-block candidates, then one block over them
__global__ __launch_bounds__(kGpBS) void argmax_blocks_kernel(const double* __restrict__ v, long m,
                                                              double* __restrict__ bv, long* __restrict__ bi) {
  __shared__ double sv[kGpBS];
  __shared__ long si[kGpBS];
  double best = -INFINITY;
  long idx = -1;
  for (long q = (long)blockIdx.x * kGpBS + threadIdx.x; q < m; q += (long)gridDim.x * kGpBS) {
    const double x = v[q];
    if (x > best || (x == best && idx < 0)) { best = x; idx = q; }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = idx;
  __syncthreads();
  for (int w = kGpBS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = sv[threadIdx.x], b = sv[threadIdx.x + w];
      const long ia = si[threadIdx.x], ib = si[threadIdx.x + w];
      if (ib >= 0 && (ia < 0 || b > a || (b == a && ib < ia))) { sv[threadIdx.x] = b; si[threadIdx.x] = ib; }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { bv[blockIdx.x] = sv[0]; bi[blockIdx.x] = si[0]; }
}

__global__ __launch_bounds__(kGpBS) void argmax_final_kernel(const double* __restrict__ bv, const long* __restrict__ bi,
                                                             int nb, int64_t* __restrict__ out) {
  __shared__ double sv[kGpBS];
  __shared__ long si[kGpBS];
  double best = -INFINITY;
  long idx = -1;
  for (int q = threadIdx.x; q < nb; q += kGpBS) {
    const long i = bi[q];
    if (i >= 0 && (idx < 0 || bv[q] > best || (bv[q] == best && i < idx))) { best = bv[q]; idx = i; }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = idx;
  __syncthreads();
  for (int w = kGpBS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = sv[threadIdx.x], b = sv[threadIdx.x + w];
      const long ia = si[threadIdx.x], ib = si[threadIdx.x + w];
      if (ib >= 0 && (ia < 0 || b > a || (b == a && ib < ia))) { sv[threadIdx.x] = b; si[threadIdx.x] = ib; }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = si[0];
}

}  // namespace

hipError_t gp_ei_device(const GpArgs& a, long m, double* cand, uint64_t seed, double* yhat, double* sd, double* ei,
                        hipStream_t stream) {
  if (m <= 0) return hipSuccess;
  const long blocks = (m + kGpC - 1) / kGpC;
  hipLaunchKernelGGL(gp_ei_kernel, dim3((unsigned)blocks), dim3(kGpBS), 0, stream, a, m, cand, seed, yhat, sd, ei);
  return hipGetLastError();
}

int argmax_blocks(long m) { return (int)std::min<long>(1024, (m + kGpBS - 1) / kGpBS); }

hipError_t argmax_device(const double* v, long m, double* bv, long* bi, int64_t* out, hipStream_t stream) {
  const int nb = argmax_blocks(m);
  hipLaunchKernelGGL(argmax_blocks_kernel, dim3(nb), dim3(kGpBS), 0, stream, v, m, bv, bi);
  hipLaunchKernelGGL(argmax_final_kernel, dim3(1), dim3(kGpBS), 0, stream, bv, bi, nb, out);
  return hipGetLastError();
}

}  // namespace bpm
