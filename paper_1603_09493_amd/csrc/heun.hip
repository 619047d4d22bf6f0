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
#include "field_eval.h"
#include "philox.h"

namespace bpm {

// three standard normals for (key, step, node)
__device__ __forceinline__ void gauss3(uint2 key, unsigned long long step, uint32_t node, double g[3]) {
  const uint4 w = philox4x32_10(make_uint4((uint32_t)step, (uint32_t)(step >> 32), node, 0u), key);
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

// the same three normals with the transforms in FP32 (FP32 runs; the words are the same)
__device__ __forceinline__ void gauss3(uint2 key, unsigned long long step, uint32_t node, float g[3]) {
  const uint4 w = philox4x32_10(make_uint4((uint32_t)step, (uint32_t)(step >> 32), node, 0u), key);
  const float s = 2.3283064365386963e-10f;   // 2^-32
  const float u0 = ((float)w.x + 0.5f) * s, u1 = ((float)w.y + 0.5f) * s;
  const float u2 = ((float)w.z + 0.5f) * s, u3 = ((float)w.w + 0.5f) * s;
  const float r0 = sqrtf(-2.0f * logf(u0)), r1 = sqrtf(-2.0f * logf(u2));
  float sn, cs;
  sincosf(6.283185307179586f * u1, &sn, &cs);
  g[0] = r0 * cs;
  g[1] = r0 * sn;
  g[2] = r1 * cosf(6.283185307179586f * u3);
}

// ---------------------------------------------------------------------------------------------
// Work items of phases A and C are (node i, realization r) pairs, item = i R + r, 256 per
// workgroup.  Workgroups are spread over the XCDs in contiguous runs (workgroup w takes block
// (w mod 8) * (blocks / 8) + w / 8 of the padded block map), so that each XCD works through a
// contiguous range of nodes and the neighbour rows it gathers stay in its L2.  When R is a
// multiple of 64 every wave holds one node, which the kernels then treat as wave-uniform (CSR
// row, coefficients and per-node data through scalar loads).
// ---------------------------------------------------------------------------------------------
constexpr int kHG = 8;   // CSR gathers issued together
static_assert(kHG <= kCsrPad, "a gather batch may run past the last row by kHG - 1 entries");

// p[r] as base + 32-bit byte offset: with a wave-uniform base (node-uniform rows) this is one
// scalar base and one shared VGPR offset for every gather of the row
template <typename T>
__device__ __forceinline__ T ld_off(const GLB T* base, uint32_t byte_off) {
  return *reinterpret_cast<const GLB T*>(reinterpret_cast<const GLB char*>(base) + byte_off);
}

struct HeunItem {
  int gi, i, r;
  bool ok;
};

template <typename real>
__device__ __forceinline__ HeunItem heun_item(const HeunGroup<real>* __restrict__ G, const int2* __restrict__ bmap) {
  const int nb = gridDim.x, bid = blockIdx.x;
  const int2 bm = bmap[(bid & 7) * (nb >> 3) + (bid >> 3)];
  HeunItem it{bm.x, 0, 0, false};
  if (bm.x < 0) return it;
  const int R = G[bm.x].R, n = G[bm.x].n;
  const long item = (long)bm.y * 256 + threadIdx.x;
  it.ok = item < (long)n * R;
  it.i = (int)(item / R);
  it.r = (int)(item % R);
  return it;
}

// phase A: nodal charges b = D (Ms y) for every (node, realization)
template <typename real, bool kU>
__device__ __forceinline__ void heun_A_item(const HeunGroup<real>& g, const InstConst* __restrict__ inst, int i, int r,
                                            const real* __restrict__ y) {
  const int R = g.R;
  const size_t cs = (size_t)g.n * R;
  const InstConst& ic = inst[g.inst0 + (kU ? 0 : r)];
  const real Ms0 = (real)ic.Ms[0], Ms1 = (real)ic.Ms[1];
  const GLB real* yg = glb(y);
  real bb = 0;
  const uint32_t rb = (uint32_t)r * (uint32_t)sizeof(real);
  const GLB int32_t* rp = glb(g.rowptr);
  const GLB int32_t* cxp = glb(g.colx);
  const GLB real* Dp = glb(g.D);
  const int q0 = rp[i], q1 = rp[i + 1];
  // the row's gathers are issued kHG at a time before any is used (entries past the row's end
  // are the next rows' or the zero padding: valid columns, loaded and not summed), so that a
  // wave keeps many loads in flight
  for (int qb = q0; qb < q1; qb += kHG) {
    real yx[kHG], yy[kHG], yz[kHG], d0[kHG], d1[kHG], d2[kHG];
    int cx[kHG];
#pragma unroll
    for (int t = 0; t < kHG; ++t) {
      const int q = qb + t;
      cx[t] = cxp[q];
      d0[t] = Dp[3 * q];
      d1[t] = Dp[3 * q + 1];
      d2[t] = Dp[3 * q + 2];
      const GLB real* p = yg + (size_t)(cx[t] & 0xFFFF) * R;
      yx[t] = ld_off(p, rb);
      yy[t] = ld_off(p + cs, rb);
      yz[t] = ld_off(p + 2 * cs, rb);
    }
#pragma unroll
    for (int t = 0; t < kHG; ++t)
      if (qb + t < q1) bb += ((cx[t] >> 16) ? Ms1 : Ms0) * (d0[t] * yx[t] + d1[t] * yy[t] + d2[t] * yz[t]);
  }
  glb(g.b)[(size_t)i * g.ldR + r] = bb;
}

// kU: every group's realizations share their constants (read once per group, uniform loads);
// kW: every group's R is a multiple of 64 (one node per wave).  The host picks the variant for
// the whole launch; <false, false> is correct for any batch.
template <typename real, bool kU, bool kW>
__global__ __launch_bounds__(256) void heun_phase_A(const HeunGroup<real>* __restrict__ G,
                                                    const int2* __restrict__ bmap, const InstConst* __restrict__ inst,
                                                    int stage) {
  const HeunItem it = heun_item(G, bmap);
  if (!it.ok) return;
  const HeunGroup<real> g = G[it.gi];
  const real* y = stage == 0 ? g.m : g.yt;
  heun_A_item<real, kU>(g, inst, kW ? __builtin_amdgcn_readfirstlane(it.i) : it.i, it.r, y);
}

// ---------------------------------------------------------------------------------------------
// phase B: U[N][R] = S[N][N] B[N][R]
// ---------------------------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Lane layout of v_mfma_f32_16x16x4f32 (wave64): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
// the accumulator lane l holds C[4 (l / 16) + i][l % 16].
//
// FP32: 128 x 128 output tile per workgroup of four waves, each wave a 64 x 64 quarter = 4 x 4
// matrix-core tiles of 16 x 16; K in slices of 16 through double-buffered LDS (global loads of
// the next slice in flight while the current one is multiplied, one barrier per slice).  S is
// symmetric, so A[m][k] = S[m][k] is read as S[k][m]: both operands are row segments of 128
// values, read with 16-byte loads and stored to LDS unchanged ([k][m] and [k][n]).  The row
// pitch of 144 values puts the four K rows of one fragment read on disjoint banks.  Tiles are
// assigned so that the eight workgroups of a run of consecutive tiles (same mesh, same rows of
// S) share one XCD and its L2: workgroup w runs tile (w mod 8) * (tiles / 8) + w / 8.
constexpr int kHT = 128, kHK = 16, kHP = kHT + 16;

__global__ __launch_bounds__(256) void heun_gemm_f32(const HeunGroup<float>* __restrict__ G,
                                                     const int4* __restrict__ tmap) {
  __shared__ float4 lds4[2 * 2 * kHK * kHP / 4];   // [buffer][operand][k][kHP]
  float* lds = reinterpret_cast<float*>(lds4);
  const int nb = gridDim.x, bid = blockIdx.x;
  const int4 tm = tmap[(bid & 7) * (nb >> 3) + (bid >> 3)];
  if (tm.x < 0) return;
  const HeunGroup<float> g = G[tm.x];
  const int n = g.n, R = g.R, ldS = g.ldS, ldR = g.ldR;
  const int m0 = tm.y, n0 = tm.z;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = (wid >> 1) * 64, wc = (wid & 1) * 64;
  // loader: rows lk and lk + 8 of the slice, columns lc .. lc + 3
  const int lk = tid >> 5, lc = (tid & 31) * 4;
  // every load is in bounds (columns and rows clamped) and out-of-range values are zeroed after
  // the load, so that the loads stay unconditional global loads
  const bool a_in = m0 + lc < ldS, b_in = n0 + lc < ldR;
  const GLB float* Sp = glb(g.S) + (a_in ? m0 + lc : 0);
  const GLB float* Bp = glb(g.b) + (b_in ? n0 + lc : 0);
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  float* const A0 = lds;                        // buffer 0: A slice, then B slice
  float* const A1 = lds + 2 * kHK * kHP;        // buffer 1
  const int lo = lk * kHP + lc, hi = (lk + 8) * kHP + lc;
#define HEUN_GLOAD(k0)                                                              \
  do {                                                                              \
    const int ka = (k0) + lk, kb = ka + 8;                                          \
    const int ca = min(ka, n - 1), cb = min(kb, n - 1);                             \
    ra0 = *reinterpret_cast<const GLB float4*>(Sp + (size_t)ca * ldS);              \
    ra1 = *reinterpret_cast<const GLB float4*>(Sp + (size_t)cb * ldS);              \
    rb0 = *reinterpret_cast<const GLB float4*>(Bp + (size_t)ca * ldR);              \
    rb1 = *reinterpret_cast<const GLB float4*>(Bp + (size_t)cb * ldR);              \
    if (!(ka < n && a_in)) ra0 = z4;                                                \
    if (!(kb < n && a_in)) ra1 = z4;                                                \
    if (!(ka < n && b_in)) rb0 = z4;                                                \
    if (!(kb < n && b_in)) rb1 = z4;                                                \
  } while (0)
#define HEUN_LSTORE(Abuf)                                         \
  do {                                                            \
    *reinterpret_cast<float4*>((Abuf) + lo) = ra0;                \
    *reinterpret_cast<float4*>((Abuf) + hi) = ra1;                \
    *reinterpret_cast<float4*>((Abuf) + kHK * kHP + lo) = rb0;    \
    *reinterpret_cast<float4*>((Abuf) + kHK * kHP + hi) = rb1;    \
  } while (0)
  float4 ra0, ra1, rb0, rb1;
  floatx4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nk = (n + kHK - 1) / kHK;
  HEUN_GLOAD(0);
  HEUN_LSTORE(A0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) HEUN_GLOAD((kt + 1) * kHK);
    const float* A = cur ? A1 : A0;
    const float* B = A + kHK * kHP;
#pragma unroll
    for (int ks = 0; ks < kHK; ks += 4) {
      const int kr = (ks + (lane >> 4)) * kHP + (lane & 15);
      float af[4], bf[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) af[a] = A[kr + wr + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bf[b] = B[kr + wc + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    if (kt + 1 < nk) HEUN_LSTORE(cur ? A0 : A1);
    __syncthreads();
  }
#undef HEUN_GLOAD
#undef HEUN_LSTORE
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int col = n0 + wc + 16 * b + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = m0 + wr + 16 * a + 4 * (lane >> 4) + i;
        if (row < n && col < R) glb(g.u)[(size_t)row * ldR + col] = acc[a][b][i];
      }
    }
}

// FP64 (parity runs): 64 x 64 tiles, each lane owning a 4 x 4 block of its wave's 32 x 32 quarter
// (FMA); the FP32 instantiation of this kernel is the 64 x 64 matrix-core variant.
template <typename real>
__global__ __launch_bounds__(256) void heun_phase_B(const HeunGroup<real>* __restrict__ G, const int4* __restrict__ tmap) {
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ real As[TK][TM + 4];   // As[k][m]
  __shared__ real Bs[TK][TN + 4];   // Bs[k][n]
  const int4 tm = tmap[blockIdx.x];  // (group, m0, n0, -)
  if (tm.x < 0) return;
  const HeunGroup<real> g = G[tm.x];
  const int n = g.n, R = g.R, ldS = g.ldS, ldR = g.ldR;
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
      Bs[kk][nn] = (k < n && col < R) ? g.b[(size_t)k * ldR + col] : (real)0;
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
          if (row < n && col < R) g.u[(size_t)row * ldR + col] = acc[a][b][i];
        }
  } else {
    const int r4 = wr + 4 * (lane >> 3), c4 = wc + 4 * (lane & 7);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const int row = m0 + r4 + a, col = n0 + c4 + b;
        if (row < n && col < R) g.u[(size_t)row * ldR + col] = (real)accd[a][b];
      }
  }
}

// ---------------------------------------------------------------------------------------------
// phase C: effective field + thermal field, LLG, and the Heun stage update
// ---------------------------------------------------------------------------------------------
template <typename real, bool kU>
__device__ __forceinline__ void heun_C_item(const HeunGroup<real>& g, const InstConst* __restrict__ inst,
                                            const HeunParams& P, int stage, int i, int r) {
  const int R = g.R, n = g.n;
  const size_t cs = (size_t)n * R, at = (size_t)i * R + r;
  const InstConst& ic = inst[g.inst0 + (kU ? 0 : r)];
  const unsigned long long step = *P.step;
  const double dt = P.h;
  const double t = (double)step * P.dt + (stage == 0 ? 0.0 : dt);
  const real* y = stage == 0 ? g.m : g.yt;
  const int L = g.layer[i];
  const real Vi = g.V[i];
  const GLB real* yg = glb(y);
  const real mx = yg[at], my = yg[cs + at], mz = yg[2 * cs + at];
  // exchange (K y) and demag (DT u) gathers over the same CSR row
  real ex = 0, ey = 0, ez = 0, dx = 0, dy = 0, dz = 0;
  const GLB real* ug = glb(g.u);
  const uint32_t rb = (uint32_t)r * (uint32_t)sizeof(real);
  const GLB int32_t* rp = glb(g.rowptr);
  const GLB int32_t* cp = glb(g.col);
  const GLB real* Kp = glb(g.K);
  const GLB real* Tp = glb(g.DT);
  const int q0 = rp[i], q1 = rp[i + 1];
  for (int qb = q0; qb < q1; qb += kHG) {   // batched gathers as in phase A
    real yx[kHG], yy[kHG], yz[kHG], uu[kHG], kk[kHG], t0[kHG], t1[kHG], t2[kHG];
#pragma unroll
    for (int t = 0; t < kHG; ++t) {
      const int q = qb + t;
      const int j = cp[q];
      kk[t] = Kp[q];
      t0[t] = Tp[3 * q];
      t1[t] = Tp[3 * q + 1];
      t2[t] = Tp[3 * q + 2];
      const GLB real* p = yg + (size_t)j * R;
      yx[t] = ld_off(p, rb);
      yy[t] = ld_off(p + cs, rb);
      yz[t] = ld_off(p + 2 * cs, rb);
      uu[t] = ld_off(ug + (size_t)j * g.ldR, rb);
    }
#pragma unroll
    for (int t = 0; t < kHG; ++t)
      if (qb + t < q1) {
        ex += kk[t] * yx[t];
        ey += kk[t] * yy[t];
        ez += kk[t] * yz[t];
        dx += t0[t] * uu[t];
        dy += t1[t] * uu[t];
        dz += t2[t] * uu[t];
      }
  }
  const real cex = -(real)ic.cex[L] / Vi;
  real Bx = cex * ex, By = cex * ey, Bz = cex * ez;
  const real ux = (real)ic.axis[L][0], uy = (real)ic.axis[L][1], uz = (real)ic.axis[L][2];
  const real mu = (real)ic.can[L] * (mx * ux + my * uy + mz * uz);
  Bx += mu * ux; By += mu * uy; Bz += mu * uz;
  const int p = g.partner[i];
  if (p >= 0) {
    const real ci = (real)ic.cint[L] * g.aif[i] / Vi;
    const size_t pa = (size_t)p * R + r;
    Bx += ci * yg[pa]; By += ci * yg[cs + pa]; Bz += ci * yg[2 * cs + pa];
  }
  const real cd = -(real)kMu0 / Vi;
  Bx += cd * dx; By += cd * dy; Bz += cd * dz;
  double zx, zy, zz;
  applied_field_at(ic, t, g.x[i] + ic.off[0], g.y[i] + ic.off[1], g.z[i] + ic.off[2], zx, zy, zz);
  Bx += (real)zx; By += (real)zy; Bz += (real)zz;
  // thermal field (same draw in both stages of the step)
  if (P.temperature > 0.0) {
    real gz[3];
    gauss3(g.keys[r], step, (uint32_t)i, gz);
    const double w = ic.Ms[L] * (double)Vi;
    const real sig = (real)sqrt(2.0 * ic.alpha * kBoltzmann * P.temperature / (kGammaE * w * dt));
    Bx += sig * gz[0]; By += sig * gz[1]; Bz += sig * gz[2];
  }
  const real gp = (real)ic.gp, al = (real)ic.alpha;
  const real cx = my * Bz - mz * By, cy = mz * Bx - mx * Bz, cz = mx * By - my * Bx;
  const real kx = -gp * (cx + al * (my * cz - mz * cy));
  const real ky = -gp * (cy + al * (mz * cx - mx * cz));
  const real kz = -gp * (cz + al * (mx * cy - my * cx));
  const real h = (real)dt;
  GLB real* k1 = glb(g.k1);
  if (stage == 0) {
    GLB real* yt = glb(g.yt);
    k1[at] = kx; k1[cs + at] = ky; k1[2 * cs + at] = kz;
    yt[at] = mx + h * kx; yt[cs + at] = my + h * ky; yt[2 * cs + at] = mz + h * kz;
  } else {
    const GLB real* m = glb(g.m);
    GLB real* mn = glb(g.mnext);
    const real hh = (real)(0.5 * dt);
    const real ax = m[at] + hh * (k1[at] + kx);
    const real ay = m[cs + at] + hh * (k1[cs + at] + ky);
    const real az = m[2 * cs + at] + hh * (k1[2 * cs + at] + kz);
    const real inv = (real)1 / sqrt(ax * ax + ay * ay + az * az);
    mn[at] = ax * inv; mn[cs + at] = ay * inv; mn[2 * cs + at] = az * inv;
  }
}

template <typename real, bool kU, bool kW>
__global__ __launch_bounds__(256) void heun_phase_C(const HeunGroup<real>* __restrict__ G,
                                                    const int2* __restrict__ bmap, const InstConst* __restrict__ inst,
                                                    const HeunParams P, int stage) {
  const HeunItem it = heun_item(G, bmap);
  if (!it.ok) return;
  const HeunGroup<real> g = G[it.gi];
  heun_C_item<real, kU>(g, inst, P, stage, kW ? __builtin_amdgcn_readfirstlane(it.i) : it.i, it.r);
}

// advances the device step counter (after both stages of a step)
__global__ void heun_tick(unsigned long long* step) {
  if (threadIdx.x == 0) *step += 1ull;
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
// one step from m into mnext (the caller alternates two group tables whose m and mnext are swapped)
template <typename real, bool kU, bool kW>
static void heun_step_k(const HeunLaunch<real>& L, hipStream_t s) {
  const HeunParams& P = L.params;
  for (int stage = 0; stage < 2; ++stage) {
    hipLaunchKernelGGL((heun_phase_A<real, kU, kW>), dim3(L.nblk), dim3(256), 0, s, L.groups, L.bmap, L.inst, stage);
    if constexpr (sizeof(real) == 4)
      hipLaunchKernelGGL(heun_gemm_f32, dim3(L.ntile), dim3(256), 0, s, L.groups, L.tmap);
    else
      hipLaunchKernelGGL(heun_phase_B<real>, dim3(L.ntile), dim3(256), 0, s, L.groups, L.tmap);
    hipLaunchKernelGGL((heun_phase_C<real, kU, kW>), dim3(L.nblk), dim3(256), 0, s, L.groups, L.bmap, L.inst, P, stage);
  }
  hipLaunchKernelGGL(heun_tick, dim3(1), dim3(64), 0, s, P.step);
}

template <typename real>
hipError_t heun_step(const HeunLaunch<real>& L, hipStream_t s) {
  if (L.all_uniform && L.all_wave) heun_step_k<real, true, true>(L, s);
  else if (L.all_uniform) heun_step_k<real, true, false>(L, s);
  else if (L.all_wave) heun_step_k<real, false, true>(L, s);
  else heun_step_k<real, false, false>(L, s);
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
