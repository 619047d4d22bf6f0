// Redistribution step of the simplified string method (energy barrier of Sec. II.C): a chain of
// images of one island is moved back to equal spacing along its own polyline in the space of
// all node vectors, then every node vector is normalised.
#include <hip/hip_runtime.h>

#include "bpm_internal.h"

namespace bpm {

namespace {

constexpr int kStrBS = 256;

// d[k] = || m^{k+1} - m^k ||_2 over the 3n components (one workgroup per segment k).
template <typename real>
__global__ __launch_bounds__(kStrBS) void string_dist_kernel(StringImages im, long n3, double* __restrict__ d) {
  const int k = blockIdx.x;
  const real* a = static_cast<const real*>(im.p[k]);
  const real* b = static_cast<const real*>(im.p[k + 1]);
  double acc = 0.0;
  for (long q = threadIdx.x; q < n3; q += kStrBS) {
    const double e = (double)b[q] - (double)a[q];
    acc += e * e;
  }
  __shared__ double red[kStrBS];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kStrBS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) d[k] = sqrt(red[0]);
}

// Image j (blockIdx.y) at arc length j L / (P - 1), L the total length: linear interpolation
// between the images that bracket it, node vectors normalised; out is FP64 [P][3][n].
template <typename real>
__global__ __launch_bounds__(kStrBS) void string_interp_kernel(StringImages im, int P, long n,
                                                               const double* __restrict__ d,
                                                               double* __restrict__ out) {
  const int j = blockIdx.y;
  const long i = (long)blockIdx.x * kStrBS + threadIdx.x;
  if (i >= n) return;
  double L = 0.0;
  for (int k = 0; k < P - 1; ++k) L += d[k];
  int k = 0;
  double w = 0.0;
  if (j == P - 1) {
    k = P - 2; w = 1.0;
  } else if (j > 0 && L > 0.0) {
    const double sj = L * (double)j / (double)(P - 1);
    double s = 0.0;
    while (k < P - 2 && s + d[k] < sj) { s += d[k]; ++k; }
    w = d[k] > 0.0 ? fmin(1.0, fmax(0.0, (sj - s) / d[k])) : 0.0;
  }
  const real* a = static_cast<const real*>(im.p[k]);
  const real* b = static_cast<const real*>(im.p[k + 1]);
  double v[3];
  for (int c = 0; c < 3; ++c) v[c] = (1.0 - w) * (double)a[c * n + i] + w * (double)b[c * n + i];
  const double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double* o = out + (size_t)j * 3 * n;
  for (int c = 0; c < 3; ++c) o[c * n + i] = l > 0.0 ? v[c] / l : v[c];
}

}  // namespace

hipError_t string_reparam_device(int precision, long n, int P, const StringImages& im, double* d_dist,
                                 double* d_out, hipStream_t stream) {
  if (P < 3 || P > kStringMaxImages || n <= 0) return hipErrorInvalidValue;
  const dim3 gi((unsigned)((n + kStrBS - 1) / kStrBS), (unsigned)P);
  if (precision == 64) {
    hipLaunchKernelGGL(string_dist_kernel<double>, dim3(P - 1), dim3(kStrBS), 0, stream, im, 3 * n, d_dist);
    hipLaunchKernelGGL(string_interp_kernel<double>, gi, dim3(kStrBS), 0, stream, im, P, n, d_dist, d_out);
  } else {
    hipLaunchKernelGGL(string_dist_kernel<float>, dim3(P - 1), dim3(kStrBS), 0, stream, im, 3 * n, d_dist);
    hipLaunchKernelGGL(string_interp_kernel<float>, gi, dim3(kStrBS), 0, stream, im, P, n, d_dist, d_out);
  }
  return hipGetLastError();
}

}  // namespace bpm
