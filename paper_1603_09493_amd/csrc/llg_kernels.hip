// Persistent stepping kernels of the batched FE-LLG island solver (gfx950).
//
// The recording simulation of Sec. II.A/II.C of Kovacs et al. (2016): the LLG equation at 0 K
// of an exchange-coupled composite island (Sec. II.B, Fig. 3) in a moving, ramped head field
// plus a global H_ext, integrated here with Dormand-Prince 5(4) (adaptive or fixed step).
//
// One launch integrates every instance to t_end.  A mesh group (shared geometry, K, D, S) is
// owned by G workgroups; G = 1 needs only __syncthreads, G > 1 uses a group barrier in global
// memory (the launch is cooperative, so all workgroups are resident).  Each field evaluation has
// three phases separated by group barriers:
//   A  exchange SpMV  yex = K y   and charges  b = D (Ms y)      (CSR rows of owned nodes)
//   B  potentials     u = S b                                     (dense rows of owned nodes)
//   C  B_eff = exchange + anisotropy + interlayer + demag (-mu0/V D^T u) + Zeeman (+ dipoles),
//      LLG right-hand side, the next stage input, and the reductions of the step control
// The step decision (per system: one instance, or several dipole-coupled instances) is taken
// redundantly by every workgroup of the group from the same reduced values.
#include <cmath>
#include <type_traits>

#include "bpm_internal.h"

namespace bpm {

// Dormand-Prince 5(4) (Dormand & Prince, 1980); the last row of A is the 5th-order solution.
__constant__ double kA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
__constant__ double kC[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
// error weights: 5th-order minus embedded 4th-order weights
__constant__ double kE[7] = {71.0 / 57600, 0, -71.0 / 16695, 71.0 / 1920, -17253.0 / 339200,
                             22.0 / 525, -1.0 / 40};

// ---------------------------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a workgroup of BS threads; the result is valid in every thread.  `red` holds BS/64
// doubles.
template <int BS>
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < BS / 64; ++i) s += red[i];
  return s;
}

// component q of a 16-byte vector (q is a compile-time constant after unrolling)
__device__ __forceinline__ float vcomp(const float4& v, int q) {
  return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}
__device__ __forceinline__ double vcomp(const double2& v, int q) { return q == 0 ? v.x : v.y; }

// instances handled at once in the demag product, and vector loads per lane in flight
template <int BS> struct PhaseBShape { static constexpr int RMAX = 16, U = 8; };
template <> struct PhaseBShape<1024> { static constexpr int RMAX = 8, U = 2; };

struct GroupSync {
  unsigned long long* ctr;
  unsigned long long target;
  int G;
};

// Barrier over the G workgroups of a mesh group.  Writes before the barrier are released at
// agent scope by workgroup thread 0; the wait polls with relaxed agent-scope loads (no cache
// invalidation per poll) and ends with one acquire fence, so every workgroup sees the writes.
__device__ __forceinline__ void group_sync(GroupSync& s) {
  __syncthreads();
  if (s.G > 1) {
    s.target += (unsigned long long)s.G;
    if (threadIdx.x == 0) {
      __hip_atomic_fetch_add(s.ctr, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      while (__hip_atomic_load(s.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < s.target)
        __builtin_amdgcn_s_sleep(1);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
  }
}

__device__ __forceinline__ double rise_of(const InstConst& c, double t) {
  if (!(c.t_rise > 0.0)) return 1.0;
  const double r = t / c.t_rise;
  return r < 1.0 ? r : 1.0;
}

// Applied field (tesla) at world position (x, y) and time t.
__device__ __forceinline__ void applied_B(const InstConst& c, double t, double x, double y,
                                          double& bx, double& by, double& bz) {
  double amp = c.B_peak * rise_of(c, t);
  if (c.fkind == BPM_FIELD_POLE) {
    const double sx = x - c.x_off[0] - c.v[0] * t;
    const double sy = y - c.x_off[1] - c.v[1] * t;
    const double fx = 0.5 * (1.0 - tanh(sx / c.L_grad));
    const double fy = 0.5 * (tanh((sy + 0.5 * c.W_pole) / c.L_grad) - tanh((sy - 0.5 * c.W_pole) / c.L_grad));
    amp *= fx * fy;
  }
  bx = amp * c.dir[0] + c.B_ext[0];
  by = amp * c.dir[1] + c.B_ext[1];
  bz = amp * c.dir[2] + c.B_ext[2];
}

// ---------------------------------------------------------------------------------------------
// control state, replicated per workgroup in LDS
// ---------------------------------------------------------------------------------------------
struct Ctl {
  double t[kMaxSysPerGroup], dt[kMaxSysPerGroup], h[kMaxSysPerGroup], fac[kMaxSysPerGroup];
  double dtmin[kMaxSysPerGroup], dtmax[kMaxSysPerGroup], maxdev[kMaxSysPerGroup];
  double err[kMaxSysPerGroup];
  long long istep[kMaxSysPerGroup], nacc[kMaxSysPerGroup], nrej[kMaxSysPerGroup];
  int status[kMaxSysPerGroup], active[kMaxSysPerGroup], last[kMaxSysPerGroup];
  int accepted[kMaxSysPerGroup], ninst[kMaxSysPerGroup];
  // per instance
  int isys[kMaxInstPerGroup];          // local system of instance r
  int coupled[kMaxInstPerGroup];
  double prev_t[kMaxInstPerGroup], prev_v[kMaxInstPerGroup], tsw[kMaxInstPerGroup];
  double mzs[kMaxInstPerGroup], mzh[kMaxInstPerGroup];
  int crossed[kMaxInstPerGroup];
  long long ntraj[kMaxInstPerGroup];
  double Bdip[kMaxInstPerGroup][3];
  double red[16];
  // per-instance / per-system partial sums of one workgroup (LDS atomics), pushed to global once
  double accL[kMaxInstPerGroup][6];
  double errL[kMaxSysPerGroup];
  int any_active, any_coupled;
};

// CSR rows of the owned nodes [i0, i1): rp[k] .. rp[k+1] index col/K/D/DT for node i0 + k, either
// in global memory (rp = rowptr + i0) or staged once into LDS (rebased to zero).
template <typename real>
struct Csr {
  const int32_t* rp;
  const int32_t* col;
  const real* K;
  const real* D;
  const real* DT;
};

template <typename real>
struct Ptrs {
  real* m;
  real* ys;     // two buffers: [2][R][3][n]
  real* k;      // [R][7][3][n]
  real* yex;
  real* b;
  real* u;
};

// ---------------------------------------------------------------------------------------------
// phase A: yex = K y, b = D (Ms y), dipole moments
// ---------------------------------------------------------------------------------------------
template <typename real, int BS>
__device__ __forceinline__ void phase_A(const GroupView<real>& g, const RunParams& P, Ctl& c, int i0, int i1,
                        const real* __restrict__ ysrc, int ev, const Csr<real>& cs) {
  const int n = g.n, nown = i1 - i0;
  if (c.any_coupled) {
    for (int q = threadIdx.x; q < g.R * 3; q += BS) c.accL[q / 3][q % 3] = 0.0;
    __syncthreads();
  }
  // every (instance, owned node) pair in one pass
  for (int it2 = threadIdx.x; it2 < g.R * nown; it2 += BS) {
    const int r = it2 / nown, i = i0 + (it2 - r * nown);
    if (!c.active[c.isys[r]]) continue;
    const InstConst& ic = P.inst[g.inst0 + r];
    const real Ms0 = (real)ic.Ms[0], Ms1 = (real)ic.Ms[1];
    const real* y = ysrc + (size_t)r * 3 * n;
    real ex0 = 0, ex1 = 0, ex2 = 0, bb = 0;
    const int q1 = cs.rp[i - i0 + 1];
    for (int q = cs.rp[i - i0]; q < q1; ++q) {
      const int j = cs.col[q];
      const real kq = cs.K[q];
      const real yx = y[j], yy = y[n + j], yz = y[2 * n + j];
      ex0 += kq * yx;
      ex1 += kq * yy;
      ex2 += kq * yz;
      const real Msj = g.layer[j] ? Ms1 : Ms0;
      bb += Msj * (cs.D[3 * q] * yx + cs.D[3 * q + 1] * yy + cs.D[3 * q + 2] * yz);
    }
    real* yex = g.yex + (size_t)r * 3 * n;
    yex[i] = ex0;
    yex[n + i] = ex1;
    yex[2 * n + i] = ex2;
    g.b[(size_t)r * n + i] = bb;
    if (c.coupled[r]) {
      const double w = (double)(g.layer[i] ? Ms1 : Ms0) * (double)g.V[i];
      atomicAdd(&c.accL[r][0], w * (double)y[i]);
      atomicAdd(&c.accL[r][1], w * (double)y[n + i]);
      atomicAdd(&c.accL[r][2], w * (double)y[2 * n + i]);
    }
  }
  if (c.any_coupled) {
    __syncthreads();
    for (int q = threadIdx.x; q < g.R * 3; q += BS) {
      const int r = q / 3, d = q % 3;
      if (c.coupled[r] && c.active[c.isys[r]])
        atomicAdd(&P.mom_acc[((size_t)(g.inst0 + r) * 3 + ev % 3) * 3 + d], c.accL[r][d]);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// phase B: u = S b for the owned rows; b of up to RB instances staged in LDS
// ---------------------------------------------------------------------------------------------
template <typename real, int BS>
__device__ __forceinline__ void phase_B(const GroupView<real>& g, Ctl& c, int i0, int i1, real* bL, int RB) {
  const int n = g.n, ldS = g.ldS;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = BS / 64;
  constexpr int VEC = 16 / sizeof(real);
  constexpr int U = PhaseBShape<BS>::U;           // vector loads per lane in flight per row chunk
  constexpr int RMAX = PhaseBShape<BS>::RMAX;
  constexpr int STEP = 64 * VEC;                  // elements one wave covers per load
  using vec_t = typename std::conditional<sizeof(real) == 4, float4, double2>::type;
  RB = min(RB, RMAX);
  for (int rb = 0; rb < g.R; rb += RB) {
    const int rn = min(RB, g.R - rb);
    bool any = false;
    for (int r = rb; r < rb + rn; ++r) any = any || c.active[c.isys[r]];
    if (!any) continue;
    __syncthreads();
    for (int idx = threadIdx.x; idx < rn * ldS; idx += BS) {
      const int r = idx / ldS, l = idx - r * ldS;
      bL[idx] = l < n ? g.b[(size_t)(rb + r) * n + l] : (real)0;
    }
    __syncthreads();
    for (int row = i0 + wid; row < i1; row += nw) {
      const real* Srow = g.S + (size_t)row * ldS;
      real acc[RMAX];
#pragma unroll
      for (int r = 0; r < RMAX; ++r) acc[r] = 0;
      for (int l0 = lane * VEC; l0 < ldS; l0 += STEP * U) {
        vec_t sv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int l = l0 + u * STEP;
          if (l < ldS) sv[u] = *reinterpret_cast<const vec_t*>(Srow + l);
          else sv[u] = vec_t{};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int l = l0 + u * STEP;
          if (l >= ldS) break;
#pragma unroll
          for (int r = 0; r < RMAX; ++r) {
            if (r < rn) {
              const vec_t bv = *reinterpret_cast<const vec_t*>(bL + r * ldS + l);
#pragma unroll
              for (int q = 0; q < VEC; ++q) acc[r] += vcomp(sv[u], q) * vcomp(bv, q);
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        if (r < rn) {
          const real v = wave_sum(acc[r]);
          if (lane == 0) g.u[(size_t)(rb + r) * n + row] = v;
        }
      }
    }
  }
}

// Symmetric variant for a group owned by one workgroup: only the upper triangle of S is read.
// Row k contributes S_kl b_l (l >= k) to u_k through the wave reduction and S_kl b_k (l > k) to u_l
// through LDS atomics; uL (RB x ldS in LDS, after bL) collects u.  The summation order depends on
// the atomics' order, so this variant is used for FP32 runs only.
template <typename real, int BS>
__device__ __forceinline__ void phase_B_sym(const GroupView<real>& g, Ctl& c, real* bL, int RB) {
  const int n = g.n, ldS = g.ldS;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = BS / 64;
  constexpr int VEC = 16 / sizeof(real);
  constexpr int U = 4;
  constexpr int RMAX = PhaseBShape<BS>::RMAX;
  constexpr int STEP = 64 * VEC;
  using vec_t = typename std::conditional<sizeof(real) == 4, float4, double2>::type;
  RB = min(RB, RMAX);
  real* uL = bL + (size_t)RB * ldS;
  for (int rb = 0; rb < g.R; rb += RB) {
    const int rn = min(RB, g.R - rb);
    bool any = false;
    for (int r = rb; r < rb + rn; ++r) any = any || c.active[c.isys[r]];
    if (!any) continue;
    __syncthreads();
    for (int idx = threadIdx.x; idx < rn * ldS; idx += BS) {
      const int r = idx / ldS, l = idx - r * ldS;
      bL[idx] = l < n ? g.b[(size_t)(rb + r) * n + l] : (real)0;
      uL[idx] = (real)0;
    }
    __syncthreads();
    for (int k = wid; k < n; k += nw) {
      const real* Srow = g.S + (size_t)k * ldS;
      real acc[RMAX], bk[RMAX];
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        acc[r] = 0;
        bk[r] = r < rn ? bL[r * ldS + k] : (real)0;
      }
      const int start = k & ~(VEC - 1);
      for (int l0 = start + lane * VEC; l0 < ldS; l0 += STEP * U) {
        vec_t sv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int l = l0 + u * STEP;
          if (l < ldS) sv[u] = *reinterpret_cast<const vec_t*>(Srow + l);
          else sv[u] = vec_t{};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int l = l0 + u * STEP;
          if (l >= ldS) break;
#pragma unroll
          for (int q = 0; q < VEC; ++q) {
            const int col = l + q;
            if (col < k || col >= n) continue;
            const real sq = vcomp(sv[u], q);
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
              if (r < rn) {
                acc[r] += sq * bL[r * ldS + col];
                if (col > k) atomicAdd(&uL[r * ldS + col], sq * bk[r]);
              }
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        if (r < rn) {
          const real v = wave_sum(acc[r]);
          if (lane == 0) atomicAdd(&uL[r * ldS + k], v);
        }
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < rn * n; idx += BS) {
      const int r = idx / n, l = idx - r * n;
      g.u[(size_t)(rb + r) * n + l] = uL[r * ldS + l];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// phase C: effective field, LLG right-hand side, next stage input, reductions
// ---------------------------------------------------------------------------------------------
template <typename real, bool kFixed, int BS>
__device__ __forceinline__ void phase_C(const GroupView<real>& g, const RunParams& P, Ctl& c, int i0, int i1,
                        int s, const real* __restrict__ ysrc, real* __restrict__ ydst, int it, int ev,
                        const Csr<real>& cs) {
  const int n = g.n, nown = i1 - i0;
  const size_t st3 = (size_t)3 * n;
  // dipole fields of coupled instances from the moments of this stage
  if (c.any_coupled) {
    for (int J = threadIdx.x; J < g.R; J += BS) {
      c.Bdip[J][0] = c.Bdip[J][1] = c.Bdip[J][2] = 0.0;
      if (!c.coupled[J]) continue;
      const InstConst& cj = P.inst[g.inst0 + J];
      for (int I = 0; I < g.R; ++I) {
        if (I == J || !c.coupled[I] || c.isys[I] != c.isys[J]) continue;
        const InstConst& ci = P.inst[g.inst0 + I];
        const double* mu = &P.mom_acc[((size_t)(g.inst0 + I) * 3 + ev % 3) * 3];
        const double d0 = cj.off[0] - ci.off[0], d1 = cj.off[1] - ci.off[1], d2 = cj.off[2] - ci.off[2];
        const double rr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double e0 = d0 / rr, e1 = d1 / rr, e2 = d2 / rr;
        const double mr = mu[0] * e0 + mu[1] * e1 + mu[2] * e2;
        const double f = kMu0 / (4.0 * kPi * rr * rr * rr);
        c.Bdip[J][0] += f * (3.0 * mr * e0 - mu[0]);
        c.Bdip[J][1] += f * (3.0 * mr * e1 - mu[1]);
        c.Bdip[J][2] += f * (3.0 * mr * e2 - mu[2]);
      }
    }
  }
  if (s >= 5) {
    for (int q = threadIdx.x; q < g.R * 6; q += BS) c.accL[q / 6][q % 6] = 0.0;
    for (int q = threadIdx.x; q < g.nsys; q += BS) c.errL[q] = 0.0;
  }
  __syncthreads();
  const real rtol = (real)P.rtol, atol = (real)P.atol;
  for (int it2 = threadIdx.x; it2 < g.R * nown; it2 += BS) {
    const int r = it2 / nown, i = i0 + (it2 - r * nown);
    const int sl = c.isys[r];
    if (!c.active[sl]) continue;
    const InstConst& ic = P.inst[g.inst0 + r];
    const double h = c.h[sl];
    const double ts = c.t[sl] + kC[s] * h;
    const real* y = ysrc + (size_t)r * st3;
    const real* yex = g.yex + (size_t)r * st3;
    const real* u = g.u + (size_t)r * n;
    real* kr = g.k + (size_t)r * 7 * st3;
    const real* m = g.m + (size_t)r * st3;
    real* yn = ydst + (size_t)r * st3;
    const real gp = (real)ic.gp, al = (real)ic.alpha;
    const int L = g.layer[i];
    const real Vi = g.V[i];
    const real mx = y[i], my = y[n + i], mz = y[2 * n + i];
    // exchange
    const real cex = -(real)ic.cex[L] / Vi;
    real Bx = cex * yex[i], By = cex * yex[n + i], Bz = cex * yex[2 * n + i];
    // anisotropy
    const real ux = (real)ic.axis[L][0], uy = (real)ic.axis[L][1], uz = (real)ic.axis[L][2];
    const real mu = (real)ic.can[L] * (mx * ux + my * uy + mz * uz);
    Bx += mu * ux; By += mu * uy; Bz += mu * uz;
    // interlayer
    const int p = g.partner[i];
    if (p >= 0) {
      const real ci = (real)ic.cint[L] * g.aif[i] / Vi;
      Bx += ci * y[p]; By += ci * y[n + p]; Bz += ci * y[2 * n + p];
    }
    // demag: -mu0 / V_i (D^T u)_i
    real dx = 0, dy = 0, dz = 0;
    const int q1 = cs.rp[i - i0 + 1];
    for (int q = cs.rp[i - i0]; q < q1; ++q) {
      const real uq = u[cs.col[q]];
      dx += cs.DT[3 * q] * uq;
      dy += cs.DT[3 * q + 1] * uq;
      dz += cs.DT[3 * q + 2] * uq;
    }
    const real cd = -(real)kMu0 / Vi;
    Bx += cd * dx; By += cd * dy; Bz += cd * dz;
    // Zeeman (+ dipoles)
    double zx, zy, zz;
    applied_B(ic, ts, g.x[i] + ic.off[0], g.y[i] + ic.off[1], zx, zy, zz);
    if (c.coupled[r]) { zx += c.Bdip[r][0]; zy += c.Bdip[r][1]; zz += c.Bdip[r][2]; }
    Bx += (real)zx; By += (real)zy; Bz += (real)zz;
    // LLG: dm/dt = -gp [ m x B + alpha m x (m x B) ]
    const real cx = my * Bz - mz * By, cy = mz * Bx - mx * Bz, cz = mx * By - my * Bx;
    const real dx2 = my * cz - mz * cy, dy2 = mz * cx - mx * cz, dz2 = mx * cy - my * cx;
    const real kx = -gp * (cx + al * dx2), ky = -gp * (cy + al * dy2), kz = -gp * (cz + al * dz2);
    real* ks = kr + (size_t)s * st3;
    ks[i] = kx; ks[n + i] = ky; ks[2 * n + i] = kz;
    if (s < 6) {
      // next stage input m + h sum_l a_{s+1,l} k_l (stage 7 input = 5th-order solution)
      real v[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        real acc = 0;
        for (int l = 0; l < s; ++l) acc += (real)(h * kA[s + 1][l]) * kr[(size_t)l * st3 + d * n + i];
        v[d] = m[d * n + i] + acc;
      }
      const real ha = (real)(h * kA[s + 1][s]);
      v[0] += ha * kx; v[1] += ha * ky; v[2] += ha * kz;
      yn[i] = v[0]; yn[n + i] = v[1]; yn[2 * n + i] = v[2];
      if (s == 5) {
        // observables of the normalised candidate
        const double nr = sqrt((double)v[0] * v[0] + (double)v[1] * v[1] + (double)v[2] * v[2]);
        const double Ms = ic.Ms[L], Vd = (double)Vi;
        const double nz = (double)v[2] / nr;
        atomicAdd(&c.accL[r][L ? 1 : 0], Vd * nz);
        atomicAdd(&c.accL[r][2], Ms * Vd * (double)v[0] / nr);
        atomicAdd(&c.accL[r][3], Ms * Vd * (double)v[1] / nr);
        atomicAdd(&c.accL[r][4], Ms * Vd * nz);
        atomicMax(reinterpret_cast<unsigned long long*>(&c.accL[r][5]),
                  (unsigned long long)__double_as_longlong(fabs(1.0 - nr)));
      }
    } else {
      // error estimate h sum_l e_l k_l, scaled per component
      real e[3] = {0, 0, 0};
      for (int l = 0; l < 6; ++l) {
        const real he = (real)(h * kE[l]);
#pragma unroll
        for (int d = 0; d < 3; ++d) e[d] += he * kr[(size_t)l * st3 + d * n + i];
      }
      const real he6 = (real)(h * kE[6]);
      e[0] += he6 * kx; e[1] += he6 * ky; e[2] += he6 * kz;
      const real y0[3] = {m[i], m[n + i], m[2 * n + i]};
      const real y1[3] = {mx, my, mz};
      double es = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const real sc = atol + rtol * fmax(fabs(y0[d]), fabs(y1[d]));
        const real qq = e[d] / sc;
        es += (double)(qq * qq);
      }
      atomicAdd(&c.errL[sl], es);
    }
  }
  if (s >= 5) {
    __syncthreads();
    if (s == 5) {
      for (int q = threadIdx.x; q < g.R * 6; q += BS) {
        const int r = q / 6, d = q % 6;
        if (!c.active[c.isys[r]]) continue;
        double* dst = &P.obs_acc[((size_t)(g.inst0 + r) * 3 + it % 3) * 6 + d];
        if (d < 5) atomicAdd(dst, c.accL[r][d]);
        else atomicMax(reinterpret_cast<unsigned long long*>(dst),
                       reinterpret_cast<const unsigned long long*>(&c.accL[r][0])[5]);
      }
    } else {
      for (int sl = threadIdx.x; sl < g.nsys; sl += BS)
        if (c.active[sl]) atomicAdd(&P.err_acc[(size_t)(g.sys0 + sl) * 3 + it % 3], c.errL[sl]);
    }
  }
}

template <typename real, bool kFixed, int BS>
__device__ __forceinline__ void field_eval(const GroupView<real>& g, const RunParams& P, Ctl& c, GroupSync& gs,
                           int i0, int i1, int s, const real* ysrc, real* ydst, int it, int ev,
                           real* bL, int RB, const Csr<real>& cs) {
  phase_A<real, BS>(g, P, c, i0, i1, ysrc, ev, cs);
  group_sync(gs);
  if (g.G == 1 && (P.flags & BPM_FLAG_SYMMETRIC_DEMAG) && sizeof(real) == 4) phase_B_sym<real, BS>(g, c, bL, RB);
  else phase_B<real, BS>(g, c, i0, i1, bL, RB);
  group_sync(gs);
  phase_C<real, kFixed, BS>(g, P, c, i0, i1, s, ysrc, ydst, it, ev, cs);
  group_sync(gs);
}

// trajectory sample of instance r (called by one thread of the group's first workgroup)
template <typename real, int BS>
__device__ __forceinline__ void save_sample(const GroupView<real>& g, const RunParams& P, Ctl& c, int r, double t,
                            double dt, double err, const double* ob) {
  if (P.traj_cap <= 0 || c.ntraj[r] >= P.traj_cap) return;
  const int gi = g.inst0 + r;
  const InstConst& ic = P.inst[gi];
  double bx, by, bz;
  applied_B(ic, t, g.cen[0] + ic.off[0], g.cen[1] + ic.off[1], bx, by, bz);
  double* smp = P.traj + ((size_t)gi * P.traj_cap + c.ntraj[r]) * kTrajW;
  double wsum = ic.Ms[0] * g.Vsoft + ic.Ms[1] * g.Vhard;
  smp[0] = t;
  smp[1] = ob[2] / wsum;
  smp[2] = ob[3] / wsum;
  smp[3] = ob[4] / wsum;
  smp[4] = g.Vsoft > 0 ? ob[0] / g.Vsoft : 0.0;
  smp[5] = g.Vhard > 0 ? ob[1] / g.Vhard : 0.0;
  smp[6] = sqrt(bx * bx + by * by + bz * bz);
  smp[7] = dt;
  smp[8] = err;
  c.ntraj[r]++;
}

// set the step size of the coming attempt and write the stage-2 input
template <typename real, bool kFixed, int BS>
__device__ __forceinline__ void begin_attempt(const GroupView<real>& g, const RunParams& P, Ctl& c, int i0, int i1,
                              real* ydst, long long nfix) {
  for (int sl = threadIdx.x; sl < g.nsys; sl += BS) {
    if (!c.active[sl]) continue;
    c.last[sl] = 0;
    if (kFixed) {
      const double t0 = (double)c.istep[sl] * P.dt_fixed;
      double t1 = (double)(c.istep[sl] + 1) * P.dt_fixed;
      if (t1 >= P.t_end || c.istep[sl] + 1 >= nfix) { t1 = P.t_end; c.last[sl] = 1; }
      c.t[sl] = t0;
      c.h[sl] = t1 - t0;
    } else {
      double h = c.dt[sl];
      if (c.t[sl] + h >= P.t_end) { h = P.t_end - c.t[sl]; c.last[sl] = 1; }
      c.h[sl] = h;
    }
  }
  __syncthreads();
  const int n = g.n, nown = i1 - i0;
  const size_t st3 = (size_t)3 * n;
  for (int it2 = threadIdx.x; it2 < g.R * nown; it2 += BS) {
    const int r = it2 / nown, i = i0 + (it2 - r * nown);
    const int sl = c.isys[r];
    if (!c.active[sl]) continue;
    const real ha = (real)(c.h[sl] * kA[1][0]);
    const real* m = g.m + (size_t)r * st3;
    const real* k0 = g.k + (size_t)r * 7 * st3;
    real* yn = ydst + (size_t)r * st3;
#pragma unroll
    for (int d = 0; d < 3; ++d) yn[d * n + i] = m[d * n + i] + ha * k0[d * n + i];
  }
}

template <typename real, bool kFixed, int BS>
__global__ __launch_bounds__(BS) void dp5_kernel(const GroupView<real>* __restrict__ groups,
                                                     RunParams P, int RB, int bl_elems, int csr_cap) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  real* bL = reinterpret_cast<real*>(smem_raw);
  __shared__ Ctl c;
  const int2 gm = P.wg_map[blockIdx.x];
  const GroupView<real> g = groups[gm.x];
  const int w = gm.y;
  const int n = g.n;
  const int i0 = (int)((long long)n * w / g.G), i1 = (int)((long long)n * (w + 1) / g.G);
  const size_t st3 = (size_t)3 * n;
  const size_t ybuf = (size_t)g.R * st3;
  GroupSync gs{g.bar, 0ull, g.G};
  const bool lead = (w == 0);
  // CSR rows of the owned nodes: staged in LDS when they fit the budget of this launch
  Csr<real> cs{g.rowptr + i0, g.col, g.K, g.D, g.DT};
  {
    const int q0 = g.rowptr[i0], nq = g.rowptr[i1] - q0;
    if (csr_cap > 0 && nq <= csr_cap && (i1 - i0) < csr_cap) {
      real* KL = bL + bl_elems;                  // [cap]
      real* DL = KL + csr_cap;                   // [cap][3]
      real* DTL = DL + 3 * csr_cap;              // [cap][3]
      int32_t* colL = reinterpret_cast<int32_t*>(DTL + 3 * csr_cap);   // [cap]
      int32_t* rpL = colL + csr_cap;             // [cap + 1]
      for (int q = threadIdx.x; q < nq; q += BS) {
        colL[q] = g.col[q0 + q];
        KL[q] = g.K[q0 + q];
        for (int d = 0; d < 3; ++d) {
          DL[3 * q + d] = g.D[3 * (q0 + q) + d];
          DTL[3 * q + d] = g.DT[3 * (q0 + q) + d];
        }
      }
      for (int k = threadIdx.x; k <= i1 - i0; k += BS) rpL[k] = g.rowptr[i0 + k] - q0;
      cs = Csr<real>{rpL, colL, KL, DL, DTL};
      __syncthreads();
    }
  }
  const long long nfix = kFixed ? (long long)ceil(P.t_end / P.dt_fixed - 1e-9) : 0;

  // ---- init control state
  for (int sl = threadIdx.x; sl < g.nsys; sl += BS) {
    c.t[sl] = 0.0; c.dt[sl] = kFixed ? P.dt_fixed : P.dt0; c.h[sl] = 0.0; c.fac[sl] = 5.0;
    c.dtmin[sl] = INFINITY; c.dtmax[sl] = 0.0; c.maxdev[sl] = 0.0; c.err[sl] = 0.0;
    c.istep[sl] = 0; c.nacc[sl] = 0; c.nrej[sl] = 0;
    c.status[sl] = BPM_OK; c.active[sl] = P.t_end > 0.0 ? 1 : 0; c.last[sl] = 0; c.ninst[sl] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    c.any_coupled = 0;
    for (int r = 0; r < g.R; ++r) {
      const int sl = P.inst[g.inst0 + r].sys - g.sys0;
      c.isys[r] = sl;
      c.ninst[sl] += 1;
      c.coupled[r] = P.sys[g.sys0 + sl].coupled;
      c.any_coupled |= c.coupled[r];
      c.crossed[r] = 0; c.ntraj[r] = 0; c.tsw[r] = NAN;
    }
  }
  __syncthreads();

  // ---- prologue: stage input = m0, observables of m0, first right-hand side
  real* ys0 = g.ys;
  real* ys1 = g.ys + ybuf;
  for (int q = threadIdx.x; q < g.R * 6; q += BS) c.accL[q / 6][q % 6] = 0.0;
  __syncthreads();
  for (int it2 = threadIdx.x; it2 < g.R * (i1 - i0); it2 += BS) {
    const int r = it2 / (i1 - i0), i = i0 + (it2 - r * (i1 - i0));
    const InstConst& ic = P.inst[g.inst0 + r];
    const int L = g.layer[i];
    const double Vd = (double)g.V[i], Ms = ic.Ms[L];
    real v[3];
    for (int d = 0; d < 3; ++d) {
      v[d] = g.m[(size_t)r * st3 + d * n + i];
      ys0[(size_t)r * st3 + d * n + i] = v[d];
    }
    atomicAdd(&c.accL[r][L ? 1 : 0], Vd * (double)v[2]);
    atomicAdd(&c.accL[r][2], Ms * Vd * (double)v[0]);
    atomicAdd(&c.accL[r][3], Ms * Vd * (double)v[1]);
    atomicAdd(&c.accL[r][4], Ms * Vd * (double)v[2]);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < g.R * 5; q += BS)
    atomicAdd(&P.obs_acc[((size_t)(g.inst0 + q / 5) * 3 + 2) * 6 + q % 5], c.accL[q / 5][q % 5]);
  group_sync(gs);
  int ev = 0;
  field_eval<real, kFixed, BS>(g, P, c, gs, i0, i1, 0, ys0, ys1, 2, ev++, bL, RB, cs);
  // initial observables, crossing state, first trajectory sample
  for (int r = threadIdx.x; r < g.R; r += BS) {
    const double* ob = &P.obs_acc[((size_t)(g.inst0 + r) * 3 + 2) * 6];
    const double vh = g.Vhard > 0 ? ob[1] / g.Vhard : 0.0;
    c.prev_t[r] = 0.0; c.prev_v[r] = vh;
    c.mzs[r] = g.Vsoft > 0 ? ob[0] / g.Vsoft : 0.0; c.mzh[r] = vh;
    if (vh <= 0.0) { c.crossed[r] = 1; c.tsw[r] = 0.0; }
    if (lead) save_sample<real, BS>(g, P, c, r, 0.0, 0.0, 0.0, ob);
  }
  __syncthreads();
  begin_attempt<real, kFixed, BS>(g, P, c, i0, i1, ys1, nfix);
  group_sync(gs);

  int it = 0;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int a = 0;
      for (int sl = 0; sl < g.nsys; ++sl) a |= c.active[sl];
      c.any_active = a;
    }
    __syncthreads();
    if (!c.any_active) break;
    // clear the accumulators used two attempts ago (every workgroup has read them)
    if (lead) {
      for (int r = threadIdx.x; r < g.R; r += BS)
        for (int d = 0; d < 6; ++d) P.obs_acc[((size_t)(g.inst0 + r) * 3 + (it + 2) % 3) * 6 + d] = 0.0;
      for (int sl = threadIdx.x; sl < g.nsys; sl += BS) P.err_acc[(size_t)(g.sys0 + sl) * 3 + (it + 2) % 3] = 0.0;
    }
    for (int s = 1; s < 7; ++s) {
      if (lead && c.any_coupled)
        for (int r = threadIdx.x; r < g.R; r += BS)
          for (int d = 0; d < 3; ++d) P.mom_acc[((size_t)(g.inst0 + r) * 3 + (ev + 2) % 3) * 3 + d] = 0.0;
      const real* src = (s & 1) ? ys1 : ys0;
      real* dst = (s & 1) ? ys0 : ys1;
      field_eval<real, kFixed, BS>(g, P, c, gs, i0, i1, s, src, dst, it, ev++, bL, RB, cs);
    }
    // ---- step decision per system (identical in every workgroup)
    for (int sl = threadIdx.x; sl < g.nsys; sl += BS) {
      c.accepted[sl] = 0;
      if (!c.active[sl]) continue;
      const double acc = P.err_acc[(size_t)(g.sys0 + sl) * 3 + it % 3];
      const double err = sqrt(acc / (3.0 * (double)n * (double)c.ninst[sl]));
      const double h = c.h[sl];
      c.err[sl] = err;
      if (!isfinite(err)) {
        c.status[sl] = BPM_ENONFINITE; c.active[sl] = 0;
        continue;
      }
      if (kFixed || err <= 1.0) {
        c.accepted[sl] = 1;
        c.t[sl] = c.last[sl] ? P.t_end : c.t[sl] + h;
        c.nacc[sl] += 1; c.istep[sl] += 1;
        c.dtmin[sl] = fmin(c.dtmin[sl], h); c.dtmax[sl] = fmax(c.dtmax[sl], h);
        if (!kFixed) {
          const double fac = err == 0.0 ? c.fac[sl] : fmin(c.fac[sl], fmax(0.2, 0.9 * pow(err, -0.2)));
          c.dt[sl] = h * fac;
          c.fac[sl] = 5.0;
        }
        if (c.last[sl]) c.active[sl] = 0;
      } else {
        c.nrej[sl] += 1;
        c.dt[sl] = h * fmax(0.2, 0.9 * pow(err, -0.2));
        c.fac[sl] = 1.0;
      }
      if (c.active[sl]) {
        if (!kFixed && c.dt[sl] < P.dt_min) { c.status[sl] = BPM_ESTEPUNDERFLOW; c.active[sl] = 0; }
        else if (P.max_steps > 0 && c.nacc[sl] + c.nrej[sl] >= P.max_steps) { c.status[sl] = BPM_EMAXSTEPS; c.active[sl] = 0; }
      }
    }
    __syncthreads();
    // per-instance observables and crossing of the hard-layer <m_z> through zero
    for (int r = threadIdx.x; r < g.R; r += BS) {
      const int sl = c.isys[r];
      if (!c.accepted[sl]) continue;
      const double* ob = &P.obs_acc[((size_t)(g.inst0 + r) * 3 + it % 3) * 6];
      const double vh = g.Vhard > 0 ? ob[1] / g.Vhard : 0.0;
      const double t = c.t[sl];
      c.mzs[r] = g.Vsoft > 0 ? ob[0] / g.Vsoft : 0.0; c.mzh[r] = vh;
      if (!c.crossed[r] && vh <= 0.0) {
        c.crossed[r] = 1;
        c.tsw[r] = (c.prev_v[r] <= 0.0 || t == c.prev_t[r]) ? t : c.prev_t[r] + (t - c.prev_t[r]) * c.prev_v[r] / (c.prev_v[r] - vh);
      }
      c.prev_t[r] = t; c.prev_v[r] = vh;
      const bool save = (P.save_every > 0 && c.nacc[sl] % P.save_every == 0) || !c.active[sl];
      if (lead && save) save_sample<real, BS>(g, P, c, r, t, c.h[sl], c.err[sl], ob);
    }
    __syncthreads();
    // largest |1 - |y|| before renormalisation, over the instances of each accepted system
    for (int sl = threadIdx.x; sl < g.nsys; sl += BS) {
      if (!c.accepted[sl]) continue;
      for (int r = 0; r < g.R; ++r) {
        if (c.isys[r] != sl) continue;
        const double* ob = &P.obs_acc[((size_t)(g.inst0 + r) * 3 + it % 3) * 6];
        const double dev = __longlong_as_double((long long)reinterpret_cast<const unsigned long long*>(ob)[5]);
        if (dev > c.maxdev[sl]) c.maxdev[sl] = dev;
      }
    }
    // accepted: m <- y / |y| (the stage-7 input), k1 <- k7
    for (int it2 = threadIdx.x; it2 < g.R * (i1 - i0); it2 += BS) {
      const int r = it2 / (i1 - i0), i = i0 + (it2 - r * (i1 - i0));
      const int sl = c.isys[r];
      if (!c.accepted[sl]) continue;
      real* m = g.m + (size_t)r * st3;
      const real* y7 = ys0 + (size_t)r * st3;
      real* k0 = g.k + (size_t)r * 7 * st3;
      const real* k6 = k0 + 6 * st3;
      const real a = y7[i], b = y7[n + i], d = y7[2 * n + i];
      const real inv = (real)1 / sqrt(a * a + b * b + d * d);
      m[i] = a * inv; m[n + i] = b * inv; m[2 * n + i] = d * inv;
      k0[i] = k6[i]; k0[n + i] = k6[n + i]; k0[2 * n + i] = k6[2 * n + i];
    }
    __syncthreads();
    begin_attempt<real, kFixed, BS>(g, P, c, i0, i1, ys1, nfix);
    group_sync(gs);
    ++it;
  }
  // results (every system of the group has finished)
  if (lead) {
    for (int sl = threadIdx.x; sl < g.nsys; sl += BS) {
      SysOut& o = P.sys_out[g.sys0 + sl];
      o.status = c.status[sl]; o.t_reached = c.t[sl]; o.n_accept = c.nacc[sl]; o.n_reject = c.nrej[sl];
      o.dt_min_used = c.nacc[sl] ? c.dtmin[sl] : 0.0; o.dt_max_used = c.dtmax[sl]; o.max_norm_dev = c.maxdev[sl];
    }
    for (int r = threadIdx.x; r < g.R; r += BS) {
      InstOut& o = P.inst_out[g.inst0 + r];
      o.crossed = c.crossed[r]; o.t_sw = c.tsw[r]; o.mz_soft = c.mzs[r]; o.mz_hard = c.mzh[r];
      o.switched = c.mzh[r] < 0.0; o.n_traj = c.ntraj[r];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// energy of each instance at its final state (one workgroup per instance)
// ---------------------------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(256) void energy_kernel(const GroupView<real>* __restrict__ groups,
                                                        const int2* __restrict__ inst_map, RunParams P,
                                                        double* __restrict__ energy) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* bL = reinterpret_cast<double*>(smem_raw);
  __shared__ double red[256 / 64];
  const int2 im = inst_map[blockIdx.x];   // (group, local instance)
  const GroupView<real> g = groups[im.x];
  const int r = im.y, n = g.n;
  const InstConst& ic = P.inst[g.inst0 + r];
  const real* m = g.m + (size_t)r * 3 * n;
  double e_loc = 0.0;
  const double t = P.sys_out[ic.sys].t_reached;
  for (int i = threadIdx.x; i < n; i += 256) {
    const int L = g.layer[i];
    double ex[3] = {0, 0, 0}, bb = 0;
    for (int q = g.rowptr[i]; q < g.rowptr[i + 1]; ++q) {
      const int j = g.col[q];
      const double Msj = ic.Ms[g.layer[j]];
      for (int d = 0; d < 3; ++d) {
        ex[d] += (double)g.K[q] * (double)m[d * n + j];
        bb += Msj * (double)g.D[3 * q + d] * (double)m[d * n + j];
      }
    }
    bL[i] = bb;
    const double mi[3] = {(double)m[i], (double)m[n + i], (double)m[2 * n + i]};
    const double Vi = (double)g.V[i];
    e_loc += ic.A[L] * (mi[0] * ex[0] + mi[1] * ex[1] + mi[2] * ex[2]);
    const double mu = mi[0] * ic.axis[L][0] + mi[1] * ic.axis[L][1] + mi[2] * ic.axis[L][2];
    e_loc += -ic.K[L] * Vi * mu * mu;
    const int p = g.partner[i];
    if (p >= 0 && L == 0)
      e_loc += -ic.Jint * (double)g.aif[i] * (mi[0] * (double)m[p] + mi[1] * (double)m[n + p] + mi[2] * (double)m[2 * n + p]);
    double bx, by, bz;
    applied_B(ic, t, g.x[i] + ic.off[0], g.y[i] + ic.off[1], bx, by, bz);
    e_loc += -ic.Ms[L] * Vi * (mi[0] * bx + mi[1] * by + mi[2] * bz);
  }
  __syncthreads();
  // demag: (mu0/2) b^T S b
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double ed = 0.0;
  for (int k = wid; k < n; k += 256 / 64) {
    double acc = 0.0;
    for (int l = lane; l < n; l += 64) acc += (double)g.S[(size_t)k * g.ldS + l] * bL[l];
    acc = wave_sum(acc);
    if (lane == 0) ed += 0.5 * kMu0 * bL[k] * acc;
  }
  e_loc += ed;
  double tot = block_sum<256>(e_loc, red);
  // point-dipole energy of a coupled island: -1/2 mu_J . B_dip,J (half of each pair energy)
  const SysView sv = P.sys[ic.sys];
  if (sv.coupled && sv.count > 1) {
    double muJ[3] = {0, 0, 0}, Bd[3] = {0, 0, 0};
    for (int I = sv.inst0; I < sv.inst0 + sv.count; ++I) {
      const InstConst& ci = P.inst[I];
      const real* mI = g.m + (size_t)(I - g.inst0) * 3 * n;
      double mu[3];
      for (int d = 0; d < 3; ++d) {
        double a = 0.0;
        for (int i = threadIdx.x; i < n; i += 256) a += ci.Ms[g.layer[i]] * (double)g.V[i] * (double)mI[d * n + i];
        mu[d] = block_sum<256>(a, red);
      }
      if (I == g.inst0 + r) {
        muJ[0] = mu[0]; muJ[1] = mu[1]; muJ[2] = mu[2];
        continue;
      }
      const double d0 = ic.off[0] - ci.off[0], d1 = ic.off[1] - ci.off[1], d2 = ic.off[2] - ci.off[2];
      const double rr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      const double e0 = d0 / rr, e1 = d1 / rr, e2 = d2 / rr;
      const double mr = mu[0] * e0 + mu[1] * e1 + mu[2] * e2;
      const double f = kMu0 / (4.0 * kPi * rr * rr * rr);
      Bd[0] += f * (3.0 * mr * e0 - mu[0]);
      Bd[1] += f * (3.0 * mr * e1 - mu[1]);
      Bd[2] += f * (3.0 * mr * e2 - mu[2]);
    }
    tot += -0.5 * (muJ[0] * Bd[0] + muJ[1] * Bd[1] + muJ[2] * Bd[2]);
  }
  if (threadIdx.x == 0) energy[g.inst0 + r] = tot;
}

// ---------------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------------
template <typename real>
static const void* dp5_fn(bool fixed, int bs) {
  if (bs == 1024)
    return fixed ? reinterpret_cast<const void*>(&dp5_kernel<real, true, 1024>)
                 : reinterpret_cast<const void*>(&dp5_kernel<real, false, 1024>);
  return fixed ? reinterpret_cast<const void*>(&dp5_kernel<real, true, 256>)
               : reinterpret_cast<const void*>(&dp5_kernel<real, false, 256>);
}

// LDS bytes of a CSR staging area of `cap` entries
template <typename real>
size_t csr_stage_bytes(int cap) {
  return cap > 0 ? (size_t)cap * (7 * sizeof(real) + 2 * sizeof(int32_t)) + sizeof(int32_t) : 0;
}

template <typename real>
hipError_t launch_dp5(const GroupView<real>* d_groups, const RunParams& P, int grid, int RB,
                      int ldS_max, bool fixed, bool cooperative, hipStream_t stream, bool sym, int bs,
                      int csr_cap) {
  int bl_elems = (sym ? 2 : 1) * RB * ldS_max;
  const size_t shm = (size_t)bl_elems * sizeof(real) + csr_stage_bytes<real>(csr_cap);
  void* args[] = {(void*)&d_groups, (void*)&P, (void*)&RB, (void*)&bl_elems, (void*)&csr_cap};
  const void* fn = dp5_fn<real>(fixed, bs);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  if (cooperative) return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(bs), args, shm, stream);
  return hipLaunchKernel(fn, dim3(grid), dim3(bs), args, shm, stream);
}

template <typename real>
hipError_t max_coresident(int RB, int ldS_max, bool fixed, int bs, int csr_cap, int* per_cu, int* cus) {
  const size_t shm = (size_t)RB * ldS_max * sizeof(real) + csr_stage_bytes<real>(csr_cap);
  const void* fn = dp5_fn<real>(fixed, bs);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, bs, shm);
  if (e != hipSuccess) return e;
  int dev;
  hipGetDevice(&dev);
  return hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
}

template <typename real>
hipError_t launch_energy(const GroupView<real>* d_groups, const int2* d_inst_map, int ninst,
                         const RunParams& P, double* d_energy, int ldS_max, int nmax, hipStream_t stream) {
  const size_t shm = (size_t)nmax * sizeof(double);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&energy_kernel<real>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  (void)ldS_max;
  hipLaunchKernelGGL(energy_kernel<real>, dim3(ninst), dim3(kBlock), shm, stream, d_groups, d_inst_map,
                     P, d_energy);
  return hipGetLastError();
}

template hipError_t launch_dp5<float>(const GroupView<float>*, const RunParams&, int, int, int, bool, bool, hipStream_t, bool, int, int);
template hipError_t launch_dp5<double>(const GroupView<double>*, const RunParams&, int, int, int, bool, bool, hipStream_t, bool, int, int);
template hipError_t max_coresident<float>(int, int, bool, int, int, int*, int*);
template hipError_t max_coresident<double>(int, int, bool, int, int, int*, int*);
template hipError_t launch_energy<float>(const GroupView<float>*, const int2*, int, const RunParams&, double*, int, int, hipStream_t);
template hipError_t launch_energy<double>(const GroupView<double>*, const int2*, int, const RunParams&, double*, int, int, hipStream_t);

}  // namespace bpm
