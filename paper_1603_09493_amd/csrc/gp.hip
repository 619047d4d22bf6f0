// Expected improvement of the optimiser's kriging model at a large set of candidates (the
// efficient global optimisation of Sec. II.A evaluates the candidate of largest EI).
//
// With R = L L' the training correlation matrix, r the correlations of a candidate with the n
// training points and G the (n + 2) x n matrix [L^-1; alpha'; w'] (alpha = R^-1 (y - 1 mu),
// w = R^-1 1), one product v = G r gives
//   q = |v_0..n-1|^2 = r' R^-1 r,   yhat = mu + v_n,   p = v_{n+1} = 1' R^-1 r,
//   s^2 = sigma^2 (1 - q + (1 - p)^2 / c),  c = 1' R^-1 1,
//   EI = (f_min - yhat) Phi(z) + s phi(z),  z = (f_min - yhat) / s.
// For a block of 64 candidates that product is a 64 x n by n x (n + 2) matrix product: 256
// threads hold 4 candidates x 4 rows of G each, the correlations are formed while a 16-column
// slice of them is staged in LDS, and only the lower triangle of L^-1 is visited.  FP64
// throughout (the variance is a difference of nearly equal terms near training points).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "bpm_internal.h"
#include "philox.h"

namespace bpm {

namespace {

constexpr int kGpBS = 256;
constexpr int kGpC = 64;      // candidates per block
constexpr int kGpK = 16;      // columns of G per LDS stage

__global__ __launch_bounds__(kGpBS) void gp_ei_kernel(GpArgs a, long m, double* __restrict__ cand,
                                                      uint64_t seed, double* __restrict__ yhat,
                                                      double* __restrict__ sd, double* __restrict__ ei) {
  __shared__ double xc[kGpC][kMaxGpDim];
  __shared__ double Rt[kGpK][kGpC + 1];
  __shared__ double Gt[kGpC][kGpK + 1];
  __shared__ double th[kMaxGpDim];
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
  const int cs = t >> 4, rs = t & 15;    // candidates 4 cs .. 4 cs + 3, rows 4 rs .. 4 rs + 3 of a tile
  double qa[4] = {0, 0, 0, 0}, ya[4] = {0, 0, 0, 0}, pa[4] = {0, 0, 0, 0};
  const int NR = n + 2;
  for (int i0 = 0; i0 < NR; i0 += kGpC) {
    // rows below n are rows of the lower-triangular L^-1: columns beyond the tile's last row are zero
    const int kmax = i0 + kGpC <= n ? i0 + kGpC : n;
    double acc[4][4] = {};
    for (int j0 = 0; j0 < kmax; j0 += kGpK) {
      __syncthreads();
      // correlations of the 64 candidates with training points j0 .. j0 + 15
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
        }
        Rt[jj][cc] = r;
      }
      for (int e = t; e < kGpC * kGpK; e += kGpBS) {
        const int ii = e / kGpK, jj = e - ii * kGpK;
        const int i = i0 + ii, j = j0 + jj;
        Gt[ii][jj] = (i < NR && j < n) ? a.G[(size_t)i * n + j] : 0.0;
      }
      __syncthreads();
#pragma unroll 4
      for (int jj = 0; jj < kGpK; ++jj) {
        double rv[4], gv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) rv[u] = Rt[jj][4 * cs + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) gv[u] = Gt[4 * rs + u][jj];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(rv[u], gv[v], acc[u][v]);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + 4 * rs + v;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (i < n) qa[u] = fma(acc[u][v], acc[u][v], qa[u]);
        else if (i == n) ya[u] += acc[u][v];
        else if (i == n + 1) pa[u] += acc[u][v];
      }
    }
  }
  // sums over the 16 threads (rs) that share a candidate quartet: lanes 16 cs .. 16 cs + 15
#pragma unroll
  for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      qa[u] += __shfl_xor(qa[u], w, 16);
      ya[u] += __shfl_xor(ya[u], w, 16);
      pa[u] += __shfl_xor(pa[u], w, 16);
    }
  if (rs == 0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long c = c0 + 4 * cs + u;
      if (c >= m) continue;
      const double mu = a.mu + ya[u];
      const double one_p = 1.0 - pa[u];
      const double var = a.sigma2 * (1.0 - qa[u] + one_p * one_p / a.c);
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
