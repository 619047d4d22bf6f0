// Surrogate MLP 12 -> 256 -> 256 -> 256 -> 256 -> 3 (exact-erf GELU) on BF16 MFMA, FP32 accumulate.
//
// The paper's optimizer (Sec. II.A) drives the expensive model evaluation with a Gaussian-process
// surrogate; here a multilayer perceptron trained on solver output screens candidate designs and
// the batched solver stays the judge.  Every operand of a matrix product is rounded to bfloat16
// (round to nearest even); accumulation, bias, GELU, loss and Adam are FP32.
//
// MFMA used: v_mfma_f32_16x16x32_bf16 (gfx950).  Operand lane layout (wave64): lane l holds
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16] for j = 0..7; the accumulator lane l
// holds C[4 (l / 16) + i][l % 16] for i = 0..3.
#include <cmath>

#include "bpm_internal.h"
#include "mlp_internal.h"

namespace bpm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __bf16 to_bf16(float x) {
  // round to nearest even on the bit pattern (NaN kept quiet)
  unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) u |= 0x00400000u;
  else u += 0x7fffu + ((u >> 16) & 1u);
  unsigned short h = (unsigned short)(u >> 16);
  return __builtin_bit_cast(__bf16, h);
}

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ---------------------------------------------------------------------------------------------
// generic GEMM: C[m][n] = sum_k A(m,k) B(k,n) (+ bias[n]);  A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn]; operands rounded to bf16 on load; 64x64 tile per workgroup,
// each of the four waves owns a 32x32 quarter (2x2 MFMA tiles).
// epilogue: EPI_STORE (C = acc + bias), EPI_GELU (also Act = gelu(C))
// ---------------------------------------------------------------------------------------------
enum { EPI_STORE = 0, EPI_GELU = 1 };

template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const float* __restrict__ A, long sam,
                                                        long sak, const float* __restrict__ B, long sbk, long sbn,
                                                        float* __restrict__ C, long ldc,
                                                        const float* __restrict__ bias, float* __restrict__ Act) {
  constexpr int TM = 64, TN = 64, TK = 32, LDK = TK + 8;
  __shared__ __bf16 As[TM * LDK];
  __shared__ __bf16 Bs[TN * LDK];
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = (wid >> 1) * 32, wc = (wid & 1) * 32;
  floatx4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += TK) {
    __syncthreads();
    for (int idx = tid; idx < TM * TK; idx += 256) {
      const int r = idx / TK, kk = idx % TK;
      const int m = m0 + r, k = k0 + kk;
      As[r * LDK + kk] = to_bf16((m < M && k < K) ? A[(long)m * sam + (long)k * sak] : 0.f);
    }
    for (int idx = tid; idx < TN * TK; idx += 256) {
      const int r = idx / TK, kk = idx % TK;
      const int n = n0 + r, k = k0 + kk;
      Bs[r * LDK + kk] = to_bf16((n < N && k < K) ? B[(long)k * sbk + (long)n * sbn] : 0.f);
    }
    __syncthreads();
    bf16x8 af[2], bfr[2];
    for (int t = 0; t < 2; ++t) {
      af[t] = *reinterpret_cast<const bf16x8*>(&As[(wr + 16 * t + (lane & 15)) * LDK + 8 * (lane >> 4)]);
      bfr[t] = *reinterpret_cast<const bf16x8*>(&Bs[(wc + 16 * t + (lane & 15)) * LDK + 8 * (lane >> 4)]);
    }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int i = 0; i < 4; ++i) {
        const int m = m0 + wr + 16 * a + 4 * (lane >> 4) + i;
        const int n = n0 + wc + 16 * b + (lane & 15);
        if (m < M && n < N) {
          float z = acc[a][b][i] + (bias ? bias[n] : 0.f);
          C[(long)m * ldc + n] = z;
          if (EPI == EPI_GELU) Act[(long)m * ldc + n] = gelu_f(z);
        }
      }
}

// ---------------------------------------------------------------------------------------------
// fused inference: 128 samples per workgroup, all five layers, activations (bf16) in LDS
// ---------------------------------------------------------------------------------------------
constexpr int PR = 128;          // rows (samples) per workgroup
constexpr int PLD = 256 + 8;     // LDS row stride of the activation tiles (bf16 elements)

// one hidden layer: out[128][256] = gelu(in[128][K] W^T + b); wave w owns columns 64w..64w+63
template <int K>
__device__ __forceinline__ void fused_layer(const __bf16* __restrict__ in, __bf16* __restrict__ out,
                                            const __bf16* __restrict__ W, const float* __restrict__ b) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int c0 = 64 * wid;
  floatx4 acc[8][4];
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 bfr[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      bfr[c] = *reinterpret_cast<const bf16x8*>(W + (long)(c0 + 16 * c + (lane & 15)) * K + k0 + 8 * (lane >> 4));
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const bf16x8 af = *reinterpret_cast<const bf16x8*>(in + (16 * r + (lane & 15)) * PLD + k0 + 8 * (lane >> 4));
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr[c], acc[r][c], 0, 0, 0);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int col = c0 + 16 * c + (lane & 15);
    const float bb = b[col];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) out[(16 * r + 4 * (lane >> 4) + i) * PLD + col] = to_bf16(gelu_f(acc[r][c][i] + bb));
  }
}

__global__ __launch_bounds__(256) void mlp_predict_kernel(const float* __restrict__ X, float* __restrict__ Y, long n,
                                                          MlpDevParams P) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __bf16* act0 = reinterpret_cast<__bf16*>(smem_raw);
  __bf16* act1 = act0 + PR * PLD;
  const long r0 = (long)blockIdx.x * PR;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // input tile, features padded 12 -> 32 with zeros
  for (int idx = tid; idx < PR * 32; idx += 256) {
    const int r = idx >> 5, k = idx & 31;
    const long row = r0 + r;
    act0[r * PLD + k] = to_bf16((row < n && k < kMlpIn) ? X[row * kMlpIn + k] : 0.f);
  }
  __syncthreads();
  fused_layer<32>(act0, act1, P.w[0], P.b[0]);
  __syncthreads();
  fused_layer<256>(act1, act0, P.w[1], P.b[1]);
  __syncthreads();
  fused_layer<256>(act0, act1, P.w[2], P.b[2]);
  __syncthreads();
  fused_layer<256>(act1, act0, P.w[3], P.b[3]);
  __syncthreads();
  // output layer (3 outputs padded to 16 columns): wave w owns row tiles 2w, 2w+1
  floatx4 acc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
  for (int k0 = 0; k0 < 256; k0 += 32) {
    const bf16x8 bfr = *reinterpret_cast<const bf16x8*>(P.w[4] + (long)(lane & 15) * 256 + k0 + 8 * (lane >> 4));
    for (int t = 0; t < 2; ++t) {
      const bf16x8 af = *reinterpret_cast<const bf16x8*>(act0 + (16 * (2 * wid + t) + (lane & 15)) * PLD + k0 + 8 * (lane >> 4));
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, acc[t], 0, 0, 0);
    }
  }
  const int col = lane & 15;
  if (col < kMlpOut) {
    for (int t = 0; t < 2; ++t)
      for (int i = 0; i < 4; ++i) {
        const long row = r0 + 16 * (2 * wid + t) + 4 * (lane >> 4) + i;
        if (row < n) Y[row * kMlpOut + col] = acc[t][i] + P.b[4][col];
      }
  }
}

// ---------------------------------------------------------------------------------------------
// training helpers
// ---------------------------------------------------------------------------------------------
// dY and the loss (masked MSE on outputs 0,1 + BCE with logits on output 2), mean over batch
__global__ void mlp_loss_kernel(int B, const float* __restrict__ Y, const float* __restrict__ T,
                                const uint8_t* __restrict__ mask, float* __restrict__ dY, double* __restrict__ loss) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (b < B) {
    const float m = mask[b] ? 1.f : 0.f;
    const float d0 = Y[3 * b] - T[3 * b], d1 = Y[3 * b + 1] - T[3 * b + 1];
    const float z = Y[3 * b + 2], t = T[3 * b + 2];
    const float invB = 1.f / (float)B;
    dY[3 * b] = 2.f * m * d0 * invB;
    dY[3 * b + 1] = 2.f * m * d1 * invB;
    dY[3 * b + 2] = (1.f / (1.f + expf(-z)) - t) * invB;
    const double sp = fmax((double)z, 0.0) + log1p(exp(-fabs((double)z)));
    l = ((double)m * ((double)d0 * d0 + (double)d1 * d1) + sp - (double)t * z) / B;
  }
  for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, l);
}

__global__ void gelu_back_kernel(long cnt, const float* __restrict__ dA, const float* __restrict__ Z, float* __restrict__ dZ) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < cnt; i += (long)gridDim.x * blockDim.x)
    dZ[i] = dA[i] * gelu_grad_f(Z[i]);
}

// db[o] = sum_b dZ[b][o]
__global__ void colsum_kernel(int B, int N, const float* __restrict__ dZ, float* __restrict__ db) {
  const int o = blockIdx.x;
  float s = 0.f;
  for (int b = threadIdx.x; b < B; b += blockDim.x) s += dZ[(long)b * N + o];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  __shared__ float red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) db[o] = red[0] + red[1] + red[2] + red[3];
}

__global__ void adam_kernel(long P, float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < P; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

// FP32 master parameters -> padded bf16 weights and FP32 biases for inference
__global__ void pack_weights_kernel(const float* __restrict__ theta, MlpDevParams P) {
  const int layer = blockIdx.y;
  const int ni = mlp_size(layer), no = mlp_size(layer + 1);
  const int kp = layer == 0 ? 32 : 256;      // padded input width
  const int op = layer == 4 ? 16 : 256;      // padded output count
  long off = 0;
  for (int l = 0; l < layer; ++l) off += (long)mlp_size(l) * mlp_size(l + 1) + mlp_size(l + 1);
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < op * kp; idx += gridDim.x * blockDim.x) {
    const int o = idx / kp, i = idx % kp;
    const float w = (o < no && i < ni) ? theta[off + (long)o * ni + i] : 0.f;
    P.w[layer][idx] = to_bf16(w);
  }
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < op; o += gridDim.x * blockDim.x)
    P.b[layer][o] = o < no ? theta[off + (long)no * ni + o] : 0.f;
}

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------
static hipError_t gemm(int epi, int M, int N, int K, const float* A, long sam, long sak, const float* B, long sbk,
                       long sbn, float* C, long ldc, const float* bias, float* Act, hipStream_t s) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  if (epi == EPI_GELU)
    hipLaunchKernelGGL(gemm_bf16_kernel<EPI_GELU>, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, Act);
  else
    hipLaunchKernelGGL(gemm_bf16_kernel<EPI_STORE>, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias, Act);
  return hipGetLastError();
}

hipError_t mlp_pack(Mlp& net, hipStream_t s) {
  hipLaunchKernelGGL(pack_weights_kernel, dim3(64, 5), dim3(256), 0, s, net.theta, net.dev);
  return hipGetLastError();
}

hipError_t mlp_predict(Mlp& net, const float* X, float* Y, long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const size_t shm = 2 * (size_t)PR * PLD * sizeof(__bf16);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mlp_predict_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_predict_kernel, dim3((unsigned)((n + PR - 1) / PR)), dim3(256), shm, s, X, Y, n, net.dev);
  return hipGetLastError();
}

// forward (keeping activations), loss, backward into net.grad; loss accumulated in net.d_loss
hipError_t mlp_forward_backward(Mlp& net, const float* X, const float* T, const uint8_t* mask, int B, hipStream_t s) {
  hipError_t e;
  const float* a = X;
  long off = 0;
  long offs[5];
  for (int l = 0; l < 5; ++l) {
    const int ni = mlp_size(l), no = mlp_size(l + 1);
    offs[l] = off;
    const float* W = net.theta + off;
    const float* bias = W + (long)no * ni;
    float* Z = net.Z[l];
    if (l < 4) e = gemm(EPI_GELU, B, no, ni, a, ni, 1, W, 1, ni, Z, no, bias, net.Aout[l], s);
    else e = gemm(EPI_STORE, B, no, ni, a, ni, 1, W, 1, ni, Z, no, bias, nullptr, s);
    if (e != hipSuccess) return e;
    a = l < 4 ? net.Aout[l] : nullptr;
    off += (long)no * ni + no;
  }
  e = hipMemsetAsync(net.d_loss, 0, sizeof(double), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3((B + 255) / 256), dim3(256), 0, s, B, net.Z[4], T, mask, net.dZ, net.d_loss);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // backward: dz of layer l lives in net.dZ (output layer) or net.dZh; dA in net.dA
  const float* dz = net.dZ;
  for (int l = 4; l >= 0; --l) {
    const int ni = mlp_size(l), no = mlp_size(l + 1);
    const float* aprev = l > 0 ? net.Aout[l - 1] : X;
    float* gW = net.grad + offs[l];
    float* gb = gW + (long)no * ni;
    // dW[o][i] = sum_b dz[b][o] aprev[b][i]
    if ((e = gemm(EPI_STORE, no, ni, B, dz, 1, no, aprev, ni, 1, gW, ni, nullptr, nullptr, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3(no), dim3(256), 0, s, B, no, dz, gb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (l > 0) {
      const float* W = net.theta + offs[l];
      // dA[b][i] = sum_o dz[b][o] W[o][i]
      if ((e = gemm(EPI_STORE, B, ni, no, dz, no, 1, W, ni, 1, net.dA, ni, nullptr, nullptr, s)) != hipSuccess) return e;
      const long cnt = (long)B * ni;
      hipLaunchKernelGGL(gelu_back_kernel, dim3(1024), dim3(256), 0, s, cnt, net.dA, net.Z[l - 1], net.dZh);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      // the next layer down reads dz from dZh; copy so dA/dZh can be reused
      if ((e = hipMemcpyAsync(net.dZh2, net.dZh, sizeof(float) * cnt, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
      dz = net.dZh2;
    }
  }
  return hipSuccess;
}

hipError_t mlp_adam(Mlp& net, float lr, hipStream_t s) {
  net.step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)net.step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)net.step)));
  hipLaunchKernelGGL(adam_kernel, dim3(256), dim3(256), 0, s, (long)kMlpParams, net.theta, net.grad, net.m, net.v, lr,
                     (float)b1, (float)b2, 1e-8f, c1, c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return mlp_pack(net, s);
}

}  // namespace bpm
