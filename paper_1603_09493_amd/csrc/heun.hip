// Stochastic Heun integration of the LLG equation with a Langevin thermal field, for many
// realizations of one island design at once.
//
// The paper's adjacent-track-erasure rate rests on an attempt frequency taken from stochastic-LLG
// simulations (Sec. II.C); here the stochastic LLG itself runs for many realizations in parallel.
// Per step (t_n = n dt) with the same noise xi in both stages:
//   B_th,i = sqrt(2 alpha kB T / (gamma Ms V_i dt)) xi,   xi ~ N(0,1)^3 from Philox4x32-10 with
//            key = the instance seed and counter = (n low, n high, node, 0), Box-Muller on the words
//   k1 = f(m, t_n),  m~ = m + dt k1,  k2 = f(m~, t_n+1),  m <- normalise(m + dt/2 (k1 + k2))
// with f the LLG right-hand side for B_eff + B_th.
//
// Layout: per mesh group the state is [3][N][R] (realization fastest), so the charges of all
// realizations form an N x R matrix B and the demag potentials U = S B are one dense GEMM per
// group, on the matrix cores for FP32 (v_mfma_f32_16x16x4f32) and with FP64 FMA tiles for FP64.
// Three launches per field evaluation (SpMM A, GEMM B, pointwise C); the step counter lives in
// device memory so one step is a replayable HIP graph.
#include <cmath>

#include "bpm_internal.h"
#include "heun_internal.h"

namespace bpm {

__device__ __forceinline__ uint4 philox_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// three standard normals for (key, step, node)
__device__ __forceinline__ void gauss3(uint2 key, unsigned long long step, uint32_t node, double g[3]) {
  const uint4 w = philox_10(make_uint4((uint32_t)step, (uint32_t)(step >> 32), node, 0u), key);
  const double s = 1.0 / 4294967296.0;
  const double u0 = ((double)w.x + 0.5) * s, u1 = ((double)w.y + 0.5) * s;
  const double u2 = ((double)w.z + 0.5) * s, u3 = ((double)w.w + 0.5) * s;
  const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
  double sn, cs;
  sincos(2.0 * kPi * u1, &sn, &cs);
  g[0] = r0 * cs;
  g[1] = r0 * sn;
  g[2] = r1 * cos(2.0 * kPi * u3);
}

__device__ __forceinline__ void applied_field(const InstConst& c, double t, double x, double y, double& bx,
                                              double& by, double& bz) {
  double amp = c.B_peak * ((c.t_rise > 0.0) ? fmin(t / c.t_rise, 1.0) : 1.0);
  if (c.fkind == BPM_FIELD_POLE) {
    const double sx = x - c.x_off[0] - c.v[0] * t;
    const double sy = y - c.x_off[1] - c.v[1] * t;
    amp *= 0.5 * (1.0 - tanh(sx / c.L_grad)) * 0.5 *
           (tanh((sy + 0.5 * c.W_pole) / c.L_grad) - tanh((sy - 0.5 * c.W_pole) / c.L_grad));
  }
  bx = amp * c.dir[0] + c.B_ext[0];
  by = amp * c.dir[1] + c.B_ext[1];
  bz = amp * c.dir[2] + c.B_ext[2];
}

// ---------------------------------------------------------------------------------------------
// phase A: yex = K y, b = D (Ms y) for every (node, realization)
// ---------------------------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(256) void heun_phase_A(const HeunGroup<real>* __restrict__ G,
                                                    const int2* __restrict__ bmap, const InstConst* __restrict__ inst,
                                                    int stage) {
  const int2 bm = bmap[blockIdx.x];
  const HeunGroup<real> g = G[bm.x];
  const long item = (long)bm.y * 256 + threadIdx.x;
  const int R = g.R, n = g.n;
  if (item >= (long)n * R) return;
  const int i = (int)(item / R), r = (int)(item % R);
  const real* y = stage == 0 ? g.m : g.yt;
  const size_t cs = (size_t)n * R;
  const InstConst& ic = inst[g.inst0 + r];
  const real Ms0 = (real)ic.Ms[0], Ms1 = (real)ic.Ms[1];
  real e0 = 0, e1 = 0, e2 = 0, bb = 0;
  for (int q = g.rowptr[i]; q < g.rowptr[i + 1]; ++q) {
    const int j = g.col[q];
    const real yx = y[(size_t)j * R + r], yy = y[cs + (size_t)j * R + r], yz = y[2 * cs + (size_t)j * R + r];
    const real kq = g.K[q];
    e0 += kq * yx;
    e1 += kq * yy;
    e2 += kq * yz;
    bb += (g.layer[j] ? Ms1 : Ms0) * (g.D[3 * q] * yx + g.D[3 * q + 1] * yy + g.D[3 * q + 2] * yz);
  }
  g.yex[(size_t)i * R + r] = e0;
  g.yex[cs + (size_t)i * R + r] = e1;
  g.yex[2 * cs + (size_t)i * R + r] = e2;
  g.b[(size_t)i * R + r] = bb;
}

// ---------------------------------------------------------------------------------------------
// phase B: U[N][R] = S[N][N] B[N][R] on the matrix cores; 64 x 64 output tile per workgroup,
// each wave a 32 x 32 quarter = 2 x 2 tiles of 16 x 16; K staged through LDS 16 at a time
// ---------------------------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));

// FP32: matrix cores.  Lane layout of v_mfma_f32_16x16x4f32 (wave64): lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; the accumulator lane l holds C[4 (l / 16) + i][l % 16].
// FP64: the same tiling with each lane owning a 4 x 4 block of its wave's 32 x 32 quarter (FMA).
template <typename real>
__global__ __launch_bounds__(256) void heun_phase_B(const HeunGroup<real>* __restrict__ G, const int4* __restrict__ tmap) {
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ real As[TK][TM + 4];   // As[k][m]
  __shared__ real Bs[TK][TN + 4];   // Bs[k][n]
  const int4 tm = tmap[blockIdx.x];  // (group, m0, n0, -)
  const HeunGroup<real> g = G[tm.x];
  const int n = g.n, R = g.R, ldS = g.ldS;
  const int m0 = tm.y, n0 = tm.z;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = (wid >> 1) * 32, wc = (wid & 1) * 32;
  floatx4 acc[2][2];
  double accd[4][4];
  if constexpr (sizeof(real) == 4) {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  } else {
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) accd[a][b] = 0.0;
  }
  for (int k0 = 0; k0 < n; k0 += TK) {
    __syncthreads();
    for (int idx = tid; idx < TM * TK; idx += 256) {
      const int mm = idx / TK, kk = idx % TK;           // consecutive threads walk k: rows of S
      const int row = m0 + mm, k = k0 + kk;
      As[kk][mm] = (row < n && k < n) ? g.S[(size_t)row * ldS + k] : (real)0;
    }
    for (int idx = tid; idx < TN * TK; idx += 256) {
      const int kk = idx / TN, nn = idx % TN;           // consecutive threads walk realizations
      const int k = k0 + kk, col = n0 + nn;
      Bs[kk][nn] = (k < n && col < R) ? g.b[(size_t)k * R + col] : (real)0;
    }
    __syncthreads();
    if constexpr (sizeof(real) == 4) {
#pragma unroll
      for (int ks = 0; ks < TK; ks += 4) {
        float af[2], bfr[2];
        for (int t = 0; t < 2; ++t) {
          af[t] = As[ks + (lane >> 4)][wr + 16 * t + (lane & 15)];
          bfr[t] = Bs[ks + (lane >> 4)][wc + 16 * t + (lane & 15)];
        }
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bfr[b], acc[a][b], 0, 0, 0);
      }
    } else {
      const int r4 = wr + 4 * (lane >> 3), c4 = wc + 4 * (lane & 7);
#pragma unroll 4
      for (int kk = 0; kk < TK; ++kk) {
        double av[4], bv[4];
        for (int a = 0; a < 4; ++a) av[a] = (double)As[kk][r4 + a];
        for (int b = 0; b < 4; ++b) bv[b] = (double)Bs[kk][c4 + b];
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) accd[a][b] += av[a] * bv[b];
      }
    }
  }
  if constexpr (sizeof(real) == 4) {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int i = 0; i < 4; ++i) {
          const int row = m0 + wr + 16 * a + 4 * (lane >> 4) + i;
          const int col = n0 + wc + 16 * b + (lane & 15);
          if (row < n && col < R) g.u[(size_t)row * R + col] = acc[a][b][i];
        }
  } else {
    const int r4 = wr + 4 * (lane >> 3), c4 = wc + 4 * (lane & 7);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const int row = m0 + r4 + a, col = n0 + c4 + b;
        if (row < n && col < R) g.u[(size_t)row * R + col] = (real)accd[a][b];
      }
  }
}

// ---------------------------------------------------------------------------------------------
// phase C: effective field + thermal field, LLG, and the Heun stage update
// ---------------------------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(256) void heun_phase_C(const HeunGroup<real>* __restrict__ G,
                                                    const int2* __restrict__ bmap, const InstConst* __restrict__ inst,
                                                    const HeunParams P, int stage) {
  const int2 bm = bmap[blockIdx.x];
  const HeunGroup<real> g = G[bm.x];
  const long item = (long)bm.y * 256 + threadIdx.x;
  const int R = g.R, n = g.n;
  if (item >= (long)n * R) return;
  const int i = (int)(item / R), r = (int)(item % R);
  const size_t cs = (size_t)n * R, at = (size_t)i * R + r;
  const InstConst& ic = inst[g.inst0 + r];
  const unsigned long long step = *P.step;
  const double dt = P.h;
  const double t = (double)step * P.dt + (stage == 0 ? 0.0 : dt);
  const real* y = stage == 0 ? g.m : g.yt;
  const int L = g.layer[i];
  const real Vi = g.V[i];
  const real mx = y[at], my = y[cs + at], mz = y[2 * cs + at];
  const real cex = -(real)ic.cex[L] / Vi;
  real Bx = cex * g.yex[at], By = cex * g.yex[cs + at], Bz = cex * g.yex[2 * cs + at];
  const real ux = (real)ic.axis[L][0], uy = (real)ic.axis[L][1], uz = (real)ic.axis[L][2];
  const real mu = (real)ic.can[L] * (mx * ux + my * uy + mz * uz);
  Bx += mu * ux; By += mu * uy; Bz += mu * uz;
  const int p = g.partner[i];
  if (p >= 0) {
    const real ci = (real)ic.cint[L] * g.aif[i] / Vi;
    const size_t pa = (size_t)p * R + r;
    Bx += ci * y[pa]; By += ci * y[cs + pa]; Bz += ci * y[2 * cs + pa];
  }
  real dx = 0, dy = 0, dz = 0;
  for (int q = g.rowptr[i]; q < g.rowptr[i + 1]; ++q) {
    const real uq = g.u[(size_t)g.col[q] * R + r];
    dx += g.DT[3 * q] * uq;
    dy += g.DT[3 * q + 1] * uq;
    dz += g.DT[3 * q + 2] * uq;
  }
  const real cd = -(real)kMu0 / Vi;
  Bx += cd * dx; By += cd * dy; Bz += cd * dz;
  double zx, zy, zz;
  applied_field(ic, t, g.x[i] + ic.off[0], g.y[i] + ic.off[1], zx, zy, zz);
  // thermal field (same draw in both stages of the step)
  if (P.temperature > 0.0) {
    double gz[3];
    gauss3(make_uint2(ic.key[0], ic.key[1]), step, (uint32_t)i, gz);
    const double w = ic.Ms[L] * (double)Vi;
    const double sig = sqrt(2.0 * ic.alpha * kBoltzmann * P.temperature / (kGammaE * w * dt));
    zx += sig * gz[0]; zy += sig * gz[1]; zz += sig * gz[2];
  }
  Bx += (real)zx; By += (real)zy; Bz += (real)zz;
  const real gp = (real)ic.gp, al = (real)ic.alpha;
  const real cx = my * Bz - mz * By, cy = mz * Bx - mx * Bz, cz = mx * By - my * Bx;
  const real kx = -gp * (cx + al * (my * cz - mz * cy));
  const real ky = -gp * (cy + al * (mz * cx - mx * cz));
  const real kz = -gp * (cz + al * (mx * cy - my * cx));
  const real h = (real)dt;
  if (stage == 0) {
    g.k1[at] = kx; g.k1[cs + at] = ky; g.k1[2 * cs + at] = kz;
    g.yt[at] = mx + h * kx; g.yt[cs + at] = my + h * ky; g.yt[2 * cs + at] = mz + h * kz;
  } else {
    const real hh = (real)(0.5 * dt);
    const real ax = g.m[at] + hh * (g.k1[at] + kx);
    const real ay = g.m[cs + at] + hh * (g.k1[cs + at] + ky);
    const real az = g.m[2 * cs + at] + hh * (g.k1[2 * cs + at] + kz);
    const real inv = (real)1 / sqrt(ax * ax + ay * ay + az * az);
    g.mnext[at] = ax * inv; g.mnext[cs + at] = ay * inv; g.mnext[2 * cs + at] = az * inv;
  }
}

// after a step: m <- mnext (swap handled by copying pointers is not graph friendly, so copy)
template <typename real>
__global__ void heun_commit(const HeunGroup<real>* __restrict__ G, const int2* __restrict__ bmap, HeunParams P) {
  const int2 bm = bmap[blockIdx.x];
  const HeunGroup<real> g = G[bm.x];
  const long item = (long)bm.y * 256 + threadIdx.x;
  const size_t cs = (size_t)g.n * g.R;
  if (item < (long)cs) {
    g.m[item] = g.mnext[item];
    g.m[cs + item] = g.mnext[cs + item];
    g.m[2 * cs + item] = g.mnext[2 * cs + item];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *P.step += 1ull;
}

// final observables per realization: volume-weighted layer means of m_z, |m| deviation
template <typename real>
__global__ void heun_observe(const HeunGroup<real>* __restrict__ G, int ngroups, double* __restrict__ out) {
  const int gi = blockIdx.y;
  if (gi >= ngroups) return;
  const HeunGroup<real> g = G[gi];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= g.R) return;
  const size_t cs = (size_t)g.n * g.R;
  double s = 0, h = 0;
  for (int i = 0; i < g.n; ++i) {
    const double v = (double)g.V[i] * (double)g.m[2 * cs + (size_t)i * g.R + r];
    if (g.layer[i]) h += v; else s += v;
  }
  out[2 * (size_t)(g.inst0 + r)] = g.Vsoft > 0 ? s / g.Vsoft : 0.0;
  out[2 * (size_t)(g.inst0 + r) + 1] = g.Vhard > 0 ? h / g.Vhard : 0.0;
}

// ---------------------------------------------------------------------------------------------
template <typename real>
hipError_t heun_step(const HeunLaunch<real>& L, hipStream_t s) {
  const HeunParams& P = L.params;
  for (int stage = 0; stage < 2; ++stage) {
    hipLaunchKernelGGL(heun_phase_A<real>, dim3(L.nblk), dim3(256), 0, s, L.groups, L.bmap, L.inst, stage);
    hipLaunchKernelGGL(heun_phase_B<real>, dim3(L.ntile), dim3(256), 0, s, L.groups, L.tmap);
    hipLaunchKernelGGL(heun_phase_C<real>, dim3(L.nblk), dim3(256), 0, s, L.groups, L.bmap, L.inst, P, stage);
  }
  hipLaunchKernelGGL(heun_commit<real>, dim3(L.nblk), dim3(256), 0, s, L.groups, L.bmap, P);
  return hipGetLastError();
}

template <typename real>
hipError_t heun_observe_launch(const HeunLaunch<real>& L, int ngroups, int Rmax, double* out, hipStream_t s) {
  hipLaunchKernelGGL(heun_observe<real>, dim3((Rmax + 255) / 256, ngroups), dim3(256), 0, s, L.groups, ngroups, out);
  return hipGetLastError();
}

template hipError_t heun_step<float>(const HeunLaunch<float>&, hipStream_t);
template hipError_t heun_step<double>(const HeunLaunch<double>&, hipStream_t);
template hipError_t heun_observe_launch<float>(const HeunLaunch<float>&, int, int, double*, hipStream_t);
template hipError_t heun_observe_launch<double>(const HeunLaunch<double>&, int, int, double*, hipStream_t);

}  // namespace bpm
