// GPU assembly of the dense magnetostatic operator S of one island mesh.
//
// The paper's island solver is a hybrid FE/BE method whose magnetostatic part is not specified
// (Sec. II.A).  Here the energy of the nodal charges b_k = integral M . grad phi_k is
// E_d = (mu0/2) b^T S b with S = T^T G T:
//   T_ek = (V_e / 4) / V_k            share of node k's unit charge carried by tetrahedron e
//   G_ef = erf(r / sqrt(2 (s_e^2 + s_f^2))) / (4 pi r),  r = |c_e - c_f|
// i.e. every tet's share sits in a Gaussian blob of standard deviation s_e = beta V_e^(1/3) at
// its centroid c_e, and G_ef is the exact Coulomb interaction of two such blobs (the coincident
// limit is sqrt(2/pi) / (4 pi sqrt(s_e^2 + s_f^2))).  G is a Gram matrix, so S is symmetric
// positive semidefinite.  Two kernels: GT = G T (tet rows, node columns, in chunks of tets) and
// S += T^T GT.
#include <cmath>

#include "bpm_internal.h"

namespace bpm {

__device__ __forceinline__ double blob_pair(double4 a, double4 b) {
  const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double s2 = a.w * a.w + b.w * b.w;
  const double inv4pi = 1.0 / (4.0 * kPi);
  if (r == 0.0) return sqrt(2.0 / kPi) / sqrt(s2) * inv4pi;
  const double x = r / sqrt(2.0 * s2);
  // erf(x) rounds to 1 in double for x > 6
  return (x > 6.0 ? 1.0 : erf(x)) * inv4pi / r;
}

__global__ void demag_gt_kernel(int n, int e0, const double4* __restrict__ tc,
                                const int32_t* __restrict__ n2t_ptr, const int32_t* __restrict__ n2t,
                                const double* __restrict__ wt, double* __restrict__ GT) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = e0 + blockIdx.y;
  if (l >= n) return;
  const double4 ce = tc[e];
  double acc = 0.0;
  for (int q = n2t_ptr[l]; q < n2t_ptr[l + 1]; ++q) acc += blob_pair(ce, tc[n2t[q]]) * wt[q];
  GT[(size_t)blockIdx.y * n + l] = acc;
}

__global__ void demag_s_kernel(int n, int ldS, int e0, int e1, const int32_t* __restrict__ n2t_ptr,
                               const int32_t* __restrict__ n2t, const double* __restrict__ wt,
                               const double* __restrict__ GT, double* __restrict__ S) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (l >= n) return;
  double acc = 0.0;
  for (int q = n2t_ptr[k]; q < n2t_ptr[k + 1]; ++q) {
    const int e = n2t[q];
    if (e < e0 || e >= e1) continue;
    acc += wt[q] * GT[(size_t)(e - e0) * n + l];
  }
  S[(size_t)k * ldS + l] += acc;
}

// S <- (S + S^T) / 2, so that both triangles hold bit-identical values
__global__ void symmetrize_kernel(int n, int ldS, double* __restrict__ S) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (l >= n || l <= k) return;
  const double v = 0.5 * (S[(size_t)k * ldS + l] + S[(size_t)l * ldS + k]);
  S[(size_t)k * ldS + l] = v;
  S[(size_t)l * ldS + k] = v;
}

void symmetrize_device(int n, int ldS, double* S, hipStream_t stream) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3((n + 255) / 256, n), dim3(256), 0, stream, n, ldS, S);
}

__global__ void to_float_kernel(size_t cnt, const double* __restrict__ a, float* __restrict__ b) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < cnt; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

// magnetisation of one instance as FP64 [3][n]: from [R][3][n] (stepping runs, rstride = 1,
// offset = r 3 n) or from [3][n][R] (thermal runs, rstride = R, offset = r)
template <typename real>
__global__ void extract_m_kernel(long n, long rstride, long offset, const real* __restrict__ src,
                                 double* __restrict__ dst) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n) return;
  const long comp = i / n, node = i - comp * n;
  dst[i] = (double)src[offset + (comp * n + node) * rstride];
}

hipError_t extract_m_device(int precision, long n, long rstride, long offset, const void* src, double* dst,
                            hipStream_t stream) {
  const unsigned blocks = (unsigned)((3 * n + 255) / 256);
  if (precision == 64)
    hipLaunchKernelGGL(extract_m_kernel<double>, dim3(blocks), dim3(256), 0, stream, n, rstride, offset,
                       static_cast<const double*>(src), dst);
  else
    hipLaunchKernelGGL(extract_m_kernel<float>, dim3(blocks), dim3(256), 0, stream, n, rstride, offset,
                       static_cast<const float*>(src), dst);
  return hipGetLastError();
}

// FP32 packed upper-triangle tiles of S (layout: bpm_internal.h, kTile); one workgroup per tile
__global__ void pack_tiles_kernel(int n, int ldS, int nb, const double* __restrict__ S, float* __restrict__ T) {
  const long f = blockIdx.x;
  int I = 0;
  long rem = f;
  while (rem >= nb - I) {
    rem -= nb - I;
    ++I;
  }
  const int J = I + (int)rem;
  float* tile = T + f * (long)(kTile * kTile);
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
    const int r = e / kTile, c = e - r * kTile;
    const int row = I * kTile + r, col = J * kTile + c;
    tile[tile_offset(r, c)] = (row < n && col < n) ? (float)S[(size_t)row * ldS + col] : 0.0f;
  }
}

void pack_tiles_device(int n, int ldS, const double* S, float* T, hipStream_t stream) {
  const int nb = (n + kTile - 1) / kTile;
  hipLaunchKernelGGL(pack_tiles_kernel, dim3((unsigned)tile_count(n)), dim3(256), 0, stream, n, ldS, nb, S, T);
}

// max |a| over cnt entries into *out (bit patterns of non-negative floats order like the values)
__global__ void absmax_kernel(size_t cnt, const double* __restrict__ a, unsigned* __restrict__ out) {
  float m = 0.f;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += (size_t)gridDim.x * blockDim.x)
    m = fmaxf(m, (float)fabs(a[q]));
  for (int w = 32; w >= 1; w >>= 1) m = fmaxf(m, __shfl_xor(m, w, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

hipError_t absmax_device(size_t cnt, const double* a, float* out, hipStream_t stream) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(float), stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(absmax_kernel, dim3(512), dim3(256), 0, stream, cnt, a, reinterpret_cast<unsigned*>(out));
  return hipGetLastError();
}

// FP16 packed tiles of S * scale (layout: tile16_offset); one workgroup per tile
__global__ void pack_tiles16_kernel(int n, int ldS, int nb, const double* __restrict__ S, double scale,
                                    _Float16* __restrict__ T) {
  const long f = blockIdx.x;
  int I = 0;
  long rem = f;
  while (rem >= nb - I) {
    rem -= nb - I;
    ++I;
  }
  const int J = I + (int)rem;
  _Float16* tile = T + f * (long)(kTile * kTile);
  for (int e = threadIdx.x; e < kTile * kTile; e += blockDim.x) {
    const int r = e / kTile, c = e - r * kTile;
    const int row = I * kTile + r, col = J * kTile + c;
    tile[tile16_offset(r, c)] = (row < n && col < n) ? (_Float16)(S[(size_t)row * ldS + col] * scale) : (_Float16)0.0f;
  }
}

void pack_tiles16_device(int n, int ldS, const double* S, double scale, uint16_t* T, hipStream_t stream) {
  const int nb = (n + kTile - 1) / kTile;
  hipLaunchKernelGGL(pack_tiles16_kernel, dim3((unsigned)tile_count(n)), dim3(256), 0, stream, n, ldS, nb, S, scale,
                     reinterpret_cast<_Float16*>(T));
}

void to_float_device(size_t cnt, const double* a, float* b, hipStream_t stream) {
  hipLaunchKernelGGL(to_float_kernel, dim3(1024), dim3(256), 0, stream, cnt, a, b);
}

int demag_assemble_device(MeshGroup& g, double beta, hipStream_t stream, std::string& err) {
  const int n = g.n, nt = g.ntet;
  const int ldS = (n + 15) / 16 * 16;
  std::vector<double4> tc(nt);
  for (int e = 0; e < nt; ++e) {
    const int32_t* t = &g.tet[4 * e];
    double cx = 0, cy = 0, cz = 0;
    for (int a = 0; a < 4; ++a) {
      cx += 0.25 * g.x[t[a]];
      cy += 0.25 * g.y[t[a]];
      cz += 0.25 * g.z[t[a]];
    }
    tc[e] = make_double4(cx, cy, cz, beta * std::cbrt(g.tetV[e]));
  }
  std::vector<double> wt(g.n2t.size());
  for (int k = 0; k < n; ++k)
    for (int q = g.n2t_ptr[k]; q < g.n2t_ptr[k + 1]; ++q) wt[q] = 0.25 * g.tetV[g.n2t[q]] / g.V[k];

  double4* dtc = nullptr;
  int32_t *dptr = nullptr, *dn2t = nullptr;
  double *dwt = nullptr, *dGT = nullptr;
  // tets per chunk: keep the GT buffer under ~256 MB
  int chunk = (int)std::min<size_t>((size_t)nt, std::max<size_t>(1, (256u << 20) / (sizeof(double) * (size_t)n)));
  chunk = std::min(chunk, 65535);
  hipError_t e = hipSuccess;
#define CHK(x)                                         \
  do {                                                 \
    e = (x);                                           \
    if (e != hipSuccess) goto fail;                    \
  } while (0)
  CHK(hipMalloc(&dtc, sizeof(double4) * nt));
  CHK(hipMalloc(&dptr, sizeof(int32_t) * (n + 1)));
  CHK(hipMalloc(&dn2t, sizeof(int32_t) * g.n2t.size()));
  CHK(hipMalloc(&dwt, sizeof(double) * wt.size()));
  CHK(hipMalloc(&dGT, sizeof(double) * (size_t)chunk * n));
  if (!g.dS64) CHK(hipMalloc(&g.dS64, sizeof(double) * (size_t)n * ldS));
  CHK(hipMemcpyAsync(dtc, tc.data(), sizeof(double4) * nt, hipMemcpyHostToDevice, stream));
  CHK(hipMemcpyAsync(dptr, g.n2t_ptr.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, stream));
  CHK(hipMemcpyAsync(dn2t, g.n2t.data(), sizeof(int32_t) * g.n2t.size(), hipMemcpyHostToDevice, stream));
  CHK(hipMemcpyAsync(dwt, wt.data(), sizeof(double) * wt.size(), hipMemcpyHostToDevice, stream));
  CHK(hipMemsetAsync(g.dS64, 0, sizeof(double) * (size_t)n * ldS, stream));
  for (int e0 = 0; e0 < nt; e0 += chunk) {
    const int ne = std::min(chunk, nt - e0);
    hipLaunchKernelGGL(demag_gt_kernel, dim3((n + 127) / 128, ne), dim3(128), 0, stream, n, e0, dtc, dptr,
                       dn2t, dwt, dGT);
    CHK(hipGetLastError());
    hipLaunchKernelGGL(demag_s_kernel, dim3((n + 127) / 128, n), dim3(128), 0, stream, n, ldS, e0, e0 + ne,
                       dptr, dn2t, dwt, dGT, g.dS64);
    CHK(hipGetLastError());
  }
  CHK(hipStreamSynchronize(stream));
  (void)hipFree(dtc); (void)hipFree(dptr); (void)hipFree(dn2t); (void)hipFree(dwt); (void)hipFree(dGT);
  return BPM_OK;
fail:
  err = std::string("demag assembly: ") + hipGetErrorString(e);
  (void)hipFree(dtc); (void)hipFree(dptr); (void)hipFree(dn2t); (void)hipFree(dwt); (void)hipFree(dGT);
  return BPM_EHIP;
#undef CHK
}

}  // namespace bpm
