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
//
// Memory-level parallelism is the design constraint at these sizes: a field evaluation of a
// 2k-node island is a few MB of traffic spread over up to 256 workgroups, so every phase issues
// its independent loads together (staged right-hand sides in wide vectors, CSR gathers in
// batches, stage combinations with a compile-time stage count) instead of one latency per
// element.  Instance constants, the CSR rows and node data of the owned nodes, and - when they
// fit - the owned rows of S stay in LDS for the whole launch.
#include <cmath>
#include <type_traits>

#include "bpm_internal.h"
#include "field_eval.h"

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

// CSR entries whose gathers are issued together (a whole row in FP32; FP64 halves it to stay in
// registers)
template <typename real, bool kX> struct Gather { static constexpr int W = 24; };
template <bool kX> struct Gather<double, kX> { static constexpr int W = 12; };


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

// Sum over a wave by DPP (pair and quad swaps, half-row and row mirrors, then the row broadcasts
// 15 and 31); the total lands in lane 63.  Every lane of the wave must be active.
template <int CTRL, int RM>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, RM, 0xF, false));
}
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, RM, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, RM, 0xF, false);
  return v + __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// v of the partner lane in halving step M (8, 4, 2, 1) of a butterfly inside each 16-lane row:
// row rotation by 8, half-row mirror, quad permutes [3,2,1,0] and [1,0,3,2].  The partners of
// step M differ in bit log2 M of the lane index and agree in every higher bit, so four steps
// pair every lane of the row with every other exactly once, and a lane can keep the half of
// its values selected by its own bit, as with xor partners; no LDS traffic.
template <int M>
__device__ __forceinline__ float row_step_partner(float v) {
  constexpr int ctrl = M == 8 ? 0x128 : M == 4 ? 0x141 : M == 2 ? 0x1B : 0xB1;
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), ctrl, 0xF, 0xF, false));
}

// h[0..2M) of each lane -> h[0..M): the half picked by the lane's bit M, plus the partner's
template <int M>
__device__ __forceinline__ void row_halve(float* h, bool up) {
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const float keep = up ? h[j + M] : h[j];
    const float send = up ? h[j] : h[j + M];
    h[j] = keep + row_step_partner<M>(send);
  }
}

template <typename T>
__device__ __forceinline__ T wave_sum_to63(T v) {
  v = dpp_add<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xF>(v);   // row_half_mirror
  v = dpp_add<0x140, 0xF>(v);   // row_mirror
  v = dpp_add<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
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

// instances handled at once by the symmetric demag product
template <typename real> struct PhaseBShape { static constexpr int RMAX = 16; };

struct GroupSync {
  unsigned long long* ctr;
  unsigned long long target;
  int G;
};

// Values exchanged between the workgroups of a mesh group within a launch (stage inputs, charges,
// potentials) in a cooperative launch (kX) are written through to the agent coherence point and
// read from it (agent-scope relaxed atomics: sc1 stores and loads), so that the group barrier
// needs neither an L2 writeback nor an L2 invalidate; read-only data (S, the CSR arrays) and the
// data each thread keeps for itself (m, the stage slopes, the exchange sums) stay cached.
template <bool kX, typename T>
__device__ __forceinline__ T xld(const GLB T* p) {
  if constexpr (kX) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
template <bool kX, typename T>
__device__ __forceinline__ void xst(GLB T* p, T v) {
  if constexpr (kX) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}
// the step-control accumulators are updated with device atomics and always read coherently
__device__ __forceinline__ double acc_ld(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void acc_st(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier over the G workgroups of a mesh group.
//  kX: every wave first waits until its own stores and atomics have completed at the coherence
//      point (vmcnt(0); on gfx9 stores count there), then thread 0 arrives on the counter and
//      polls it with relaxed agent-scope loads; the exchanged data are read with coherent loads
//      afterwards, so no cache maintenance is needed.
//  otherwise: thread 0 releases the workgroup's writes at agent scope (L2 writeback), polls, and
//      acquires (L2 invalidate).
template <bool kX>
__device__ __forceinline__ void group_sync(GroupSync& s) {
  if (s.G > 1) {
    if constexpr (kX) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt/lgkmcnt unconstrained
    __syncthreads();
    s.target += (unsigned long long)s.G;
    if (threadIdx.x == 0) {
      if constexpr (kX) {
        __hip_atomic_fetch_add(s.ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (__hip_atomic_load(s.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < s.target)
          __builtin_amdgcn_s_sleep(1);
      } else {
        __hip_atomic_fetch_add(s.ctr, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        while (__hip_atomic_load(s.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < s.target)
          __builtin_amdgcn_s_sleep(1);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
    }
  }
  __syncthreads();
}

// Applied field (tesla) at world position (x, y, z) and time t (field_eval.h).
__device__ __forceinline__ void applied_B(const InstConst& c, double t, double x, double y, double z,
                                          double& bx, double& by, double& bz) {
  applied_field_at(c, t, x, y, z, bx, by, bz);
}

// The same field with the profile evaluated in FP32 (positions and times stay FP64), for FP32
// runs: its rounding (~1e-7) is far below their tolerance.
__device__ __forceinline__ void applied_B_f32(const InstConst& c, double t, double x, double y, double z,
                                              float& bx, float& by, float& bz) {
  if (c.fkind == BPM_FIELD_GRID) {
    double gx, gy, gz;
    applied_field_at(c, t, x, y, z, gx, gy, gz);
    bx = (float)gx; by = (float)gy; bz = (float)gz;
    return;
  }
  float amp = (float)(c.B_peak * field_rise(c, t));
  if (c.fkind == BPM_FIELD_POLE) {
    const float il = (float)(1.0 / c.L_grad);
    const float sx = (float)(x - c.x_off[0] - c.v[0] * t) * il;
    const float sy = (float)(y - c.x_off[1] - c.v[1] * t) * il;
    const float hw = (float)(0.5 * c.W_pole) * il;
    const float fx = 0.5f * (1.0f - tanhf(sx));
    const float fy = 0.5f * (tanhf(sy + hw) - tanhf(sy - hw));
    amp *= fx * fy;
  }
  bx = amp * (float)c.dir[0] + (float)c.B_ext[0];
  by = amp * (float)c.dir[1] + (float)c.B_ext[1];
  bz = amp * (float)c.dir[2] + (float)c.B_ext[2];
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
  double mom[kMaxInstPerGroup][3];
  double red[16];
  // per-instance / per-system partial sums of one workgroup (LDS atomics), pushed to global once
  double accL[kMaxInstPerGroup][6];
  double errL[kMaxSysPerGroup];
  int any_active, any_coupled;
};

// CSR rows and node data of the owned nodes [i0, i1), indexed by k = i - i0 (rp, pt, lay, V,
// aif, x, y) or by the CSR position (col, K, D, DT): staged once into LDS (kL, rp rebased to zero)
// or read from global memory (rp = rowptr + i0, node arrays offset by i0).  col holds the node
// index in its low 16 bits and that node's layer above.
template <typename real, bool kL>
struct Csr {
  template <typename T>
  using ptr = typename std::conditional<kL, const T*, const GLB T*>::type;
  ptr<int32_t> rp, col;
  ptr<real> K, D, DT;
  ptr<int32_t> pt, lay;
  ptr<real> V, aif;
  ptr<double> x, y;
};

// LDS bytes of the staged CSR rows (cap entries) and node data (ocap nodes), 16-byte multiple
template <typename real>
__host__ __device__ inline size_t csr_stage_bytes(int cap, int ocap) {
  if (cap <= 0) return 0;
  const size_t b = (size_t)ocap * 2 * sizeof(double) + (size_t)cap * 7 * sizeof(real) + (size_t)ocap * 2 * sizeof(real) +
                   (size_t)cap * sizeof(int32_t) + (size_t)(ocap + 1) * sizeof(int32_t) + (size_t)ocap * 2 * sizeof(int32_t);
  return (b + 15) / 16 * 16;
}

static_assert(sizeof(InstConst) % 16 == 0, "instance constants are copied to LDS in 16-byte words");
__host__ __device__ inline size_t ic_stage_bytes(int slots) { return (size_t)slots * sizeof(InstConst); }

// pair geometry of dipole-coupled instances: unit vector from I to J and mu0 / (4 pi r^3)
__host__ __device__ inline size_t dip_stage_bytes(int slots) { return (size_t)slots * slots * 4 * sizeof(double); }

template <typename real>
__host__ __device__ inline size_t lds_plan_bytes(const LdsPlan& L) {
  return ic_stage_bytes(L.ic_slots) + dip_stage_bytes(L.dip_slots) + ((size_t)L.bl_elems * sizeof(real) + 15) / 16 * 16 +
         csr_stage_bytes<real>(L.csr_cap, L.own_cap) + (size_t)L.s_rows * L.ldS * sizeof(real);
}

// copy `cnt` 16-byte words from global memory to LDS, UN loads of a thread in flight before its
// stores; kX: the source is exchanged data, read coherently as 8-byte halves.  The copy starts at
// word rot (0 <= rot < cnt) and wraps, so that workgroups copying the same source at the same
// time start on different memory channels.
template <int BS, int UN, bool kX>
__device__ __forceinline__ void copy16(uint4* __restrict__ dst, const GLB uint4* __restrict__ src, int cnt,
                                       int rot = 0) {
  for (int base = threadIdx.x; base < cnt; base += BS * UN) {
    uint4 v[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int q = base + u * BS;
      int qq = q < cnt ? q + rot : cnt - 1;   // in bounds on every lane; stored only where q < cnt
      if (qq >= cnt) qq -= cnt;
      if constexpr (kX) {
        const GLB unsigned long long* h = reinterpret_cast<const GLB unsigned long long*>(src + qq);
        const unsigned long long lo = xld<true>(h), hi = xld<true>(h + 1);
        v[u] = make_uint4((unsigned)lo, (unsigned)(lo >> 32), (unsigned)hi, (unsigned)(hi >> 32));
      } else {
        v[u] = src[qq];
      }
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int q = base + u * BS;
      int qq = q + rot;
      if (qq >= cnt) qq -= cnt;
      if (q < cnt) dst[qq] = v[u];
    }
  }
}

// copy `cnt` 16-byte words from global memory straight into LDS (gfx950 LDS-direct loads: no
// registers, no LDS store instructions).  Each wave fills 64 consecutive words per instruction;
// kX: the loads carry the device-coherence bit, as the exchange loads do.  Returns after this
// thread's loads have landed; a workgroup barrier must follow before other waves read them.
template <int BS, bool kX>
__device__ __forceinline__ void copy16_lds(uint4* __restrict__ dst, const GLB uint4* __restrict__ src, int cnt) {
  for (int q0 = threadIdx.x & ~63; q0 < cnt; q0 += BS) {
    const int q = q0 + (threadIdx.x & 63);
    if (q < cnt)
      __builtin_amdgcn_global_load_lds((const GLB void*)(src + q), (LDSP void*)(dst + q0), 16, 0, kX ? 16 : 0);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the LDS writes of this thread's loads are done
}

// ---------------------------------------------------------------------------------------------
// phase A: yex = K y, b = D (Ms y), dipole moments
// ---------------------------------------------------------------------------------------------
template <typename real, int BS, bool kL, bool kX>
__device__ __forceinline__ void phase_A(const GroupView<real>& g, const RunParams& P, Ctl& c, const InstConst* icL,
                                        int i0, int i1, const real* ysrc_, int ev, const Csr<real, kL>& cs) {
  const int n = g.n, nown = i1 - i0, ldS = g.ldS;
  const GLB real* __restrict__ ysrc = glb(ysrc_);
  GLB real* __restrict__ yexg = glb(g.yex);
  GLB real* __restrict__ bg = glb(g.b);
  // every (instance, owned node) pair in one pass
  for (int it2 = threadIdx.x; it2 < g.R * nown; it2 += BS) {
    const int r = it2 / nown, k = it2 - r * nown, i = i0 + k;
    if (!c.active[c.isys[r]]) continue;
    const real Ms0 = (real)icL[r].Ms[0], Ms1 = (real)icL[r].Ms[1];
    const GLB real* y = ysrc + (size_t)r * 3 * n;
    real ex0 = 0, ex1 = 0, ex2 = 0, bb = 0;
    const int qa = cs.rp[k], qb = cs.rp[k + 1];
    constexpr int kGather = Gather<real, kX>::W;
    for (int q0 = qa; q0 < qb; q0 += kGather) {
      // all gathers of the row in flight at once (masked entries read the node itself)
      int cj[kGather];
      real yx[kGather], yy[kGather], yz[kGather];
#pragma unroll
      for (int u = 0; u < kGather; ++u) cj[u] = q0 + u < qb ? cs.col[q0 + u] : i;
#pragma unroll
      for (int u = 0; u < kGather; ++u) {
        const int j = cj[u] & 0xFFFF;
        yx[u] = xld<kX>(y + j); yy[u] = xld<kX>(y + n + j); yz[u] = xld<kX>(y + 2 * n + j);
      }
#pragma unroll
      for (int u = 0; u < kGather; ++u) {
        const int q = q0 + u;
        if (q < qb) {
          const real kq = cs.K[q];
          ex0 += kq * yx[u];
          ex1 += kq * yy[u];
          ex2 += kq * yz[u];
          const real Msj = (cj[u] >> 16) ? Ms1 : Ms0;
          bb += Msj * (cs.D[3 * q] * yx[u] + cs.D[3 * q + 1] * yy[u] + cs.D[3 * q + 2] * yz[u]);
        }
      }
    }
    GLB real* yex = yexg + (size_t)r * 3 * n;
    yex[i] = ex0;
    yex[n + i] = ex1;
    yex[2 * n + i] = ex2;
    xst<kX>(bg + (size_t)r * ldS + i, bb);
  }
}

// ---------------------------------------------------------------------------------------------
// phase B: u = S b for the owned rows; b of up to RB instances staged in LDS.  kSL: the owned
// rows of S are resident in LDS (SL, row k = node i0 + k), else they stream from global memory.
// A wave takes RWb rows at a time and loads UM 16-byte words of each per lane and round (a round
// covers UM * 64 * VEC columns, the whole row up to 3072 FP32 columns), so about 12 loads per
// lane are in flight;
// then, instance by instance, it reads the staged b words of the same columns, forms the lane
// partial dot products (over the lane's columns, in column order) and sums them over the wave.
// Rows longer than one round add the round sums in a per-wave LDS slot.  The order of every sum
// is the same for either source of S.
// ---------------------------------------------------------------------------------------------
template <typename real, int BS, bool kSL, bool kX, int UM, int RWb>
__device__ __forceinline__ void demag_rows(const GroupView<real>& g, int i0, int nr, const real* bL, const real* SL,
                                           real* part, int rb, int rn) {
  const int ldS = g.ldS;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int nw = BS / 64;
  constexpr int VEC = 16 / sizeof(real);
  constexpr int STEP = 64 * VEC;
  using vec_t = typename std::conditional<sizeof(real) == 4, float4, double2>::type;
  using sptr = typename std::conditional<kSL, const real*, const GLB real*>::type;
  using vptr = typename std::conditional<kSL, const vec_t*, const GLB vec_t*>::type;
  const sptr Sbase = kSL ? (sptr)SL : (sptr)(glb(g.S) + (size_t)i0 * ldS);
  GLB real* __restrict__ ug = glb(g.u);
  real* pw = part + wid * 4 * 16;          // this wave's round sums [RWb <= 4][16]
  const bool multi = ldS > UM * STEP;
  for (int k0 = wid * RWb; k0 < nr; k0 += nw * RWb) {
    sptr Srow[RWb];
#pragma unroll
    for (int w = 0; w < RWb; ++w) Srow[w] = Sbase + (size_t)min(k0 + w, nr - 1) * ldS;
    for (int base = 0; base < ldS; base += UM * STEP) {      // wave-uniform rounds
      vec_t sv[RWb][UM];
#pragma unroll
      for (int u = 0; u < UM; ++u) {
        const int l = base + u * STEP + lane * VEC;
#pragma unroll
        for (int w = 0; w < RWb; ++w) {
          if (l < ldS) sv[w][u] = *reinterpret_cast<vptr>(Srow[w] + l);
          else sv[w][u] = vec_t{};
        }
      }
#pragma unroll 1
      for (int r = 0; r < rn; ++r) {
        vec_t bv[UM];
#pragma unroll
        for (int u = 0; u < UM; ++u) {
          const int l = min(base + u * STEP + lane * VEC, ldS - VEC);   // in bounds; S is zero beyond ldS
          bv[u] = *reinterpret_cast<const vec_t*>(bL + r * ldS + l);
        }
        real a[RWb];
#pragma unroll
        for (int w = 0; w < RWb; ++w) {
          a[w] = 0;
#pragma unroll
          for (int u = 0; u < UM; ++u)
#pragma unroll
            for (int q = 0; q < VEC; ++q) a[w] += vcomp(sv[w][u], q) * vcomp(bv[u], q);
        }
#pragma unroll
        for (int w = 0; w < RWb; ++w) {
          const real t = wave_sum_to63(a[w]);
          if (lane == 63) {
            if (!multi) {
              if (k0 + w < nr) xst<kX>(ug + (size_t)(rb + r) * ldS + i0 + k0 + w, t);
            } else {
              pw[w * 16 + r] = base == 0 ? t : pw[w * 16 + r] + t;
            }
          }
        }
      }
    }
    if (multi && lane == 63)
      for (int w = 0; w < RWb; ++w)
        for (int r = 0; r < rn; ++r)
          if (k0 + w < nr) xst<kX>(ug + (size_t)(rb + r) * ldS + i0 + k0 + w, pw[w * 16 + r]);
  }
}

template <typename real, int BS, bool kSL, bool kX>
__device__ __forceinline__ void phase_B(const GroupView<real>& g, Ctl& c, int i0, int i1, real* bL,
                                        const real* SL, real* part, int RB) {
  const int ldS = g.ldS;
  constexpr int VEC = 16 / sizeof(real);
  constexpr int STEP = 64 * VEC;
  const int nr = i1 - i0;
  const int U = (ldS + STEP - 1) / STEP;   // 16-byte words per lane and row
  RB = min(RB, 16);
  for (int rb = 0; rb < g.R; rb += RB) {
    const int rn = min(RB, g.R - rb);
    bool any = false;
    for (int r = rb; r < rb + rn; ++r) any = any || c.active[c.isys[r]];
    if (!any) continue;
    __syncthreads();
    // b rows are ldS long (zero padded), so the staging is one contiguous 16-byte copy
    copy16_lds<BS, kX>(reinterpret_cast<uint4*>(bL), reinterpret_cast<const GLB uint4*>(glb(g.b) + (size_t)rb * ldS),
                       rn * ldS / VEC);
    __syncthreads();
    if (U <= 3) demag_rows<real, BS, kSL, kX, 3, 4>(g, i0, nr, bL, SL, part, rb, rn);
    else if (U <= 6) demag_rows<real, BS, kSL, kX, 6, 2>(g, i0, nr, bL, SL, part, rb, rn);
    else if (U <= 9) demag_rows<real, BS, kSL, kX, 9, 2>(g, i0, nr, bL, SL, part, rb, rn);
    else demag_rows<real, BS, kSL, kX, 12, 1>(g, i0, nr, bL, SL, part, rb, rn);   // several rounds beyond 12
  }
}

// Symmetric variant for a group owned by one workgroup (FP32): only the 64 x 64 tiles of S on or
// above the diagonal are read, and each is used twice.  Lane (rg, cq) of the wave that takes tile
// (I, J) holds rows 64I + 16rg + t (t < 16) and columns 64J + 4cq .. +3 of it (sixteen 16-byte
// loads in flight per lane) and forms
//   row sums     u_I += S_IJ b_J                   (every tile, the diagonal tile in full), and
//   column sums  u_J += S_IJ^T b_I = S_JI b_I      (tiles above the diagonal).
// Row sums are reduced over the 16 lanes of a row group (a DPP butterfly inside the row, see
// row_halve) and column sums over the four row groups by halving exchanges, so that each lane
// ends with one row (64I + lane) and one column (64J + 4cq + rg), which it adds into u in LDS
// (uL, RB x ldS after bL).  The order of those LDS additions, and with it the rounding of u,
// varies from run to run.  When every instance of the group fits in one block of right-hand
// sides, u stays in LDS for phase C (the pointer returned; nothing is written to global memory),
// else it is copied out block by block.  Tiles go round-robin over the waves of the workgroup.  The tiles come from the packed copy when the group keeps it (each
// load instruction of a wave then reads one contiguous kilobyte), else from the row-major S.
template <typename real, int BS>
__device__ __forceinline__ const real* phase_B_sym(const GroupView<real>& g, Ctl& c, real* bL, int RB) {
  static_assert(sizeof(real) == 4, "the tiled symmetric product is the FP32 path");
  const int n = g.n, ldS = g.ldS;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int nw = BS / 64;
  const int rg = lane >> 4, cq = lane & 15;
  const GLB float* Sg = reinterpret_cast<const GLB float*>(glb(g.S));
  const GLB float* Stg = g.St ? glb(g.St) : nullptr;      // packed tiles, when the group keeps them
  const GLB uint4* St16g = !g.St && g.St16 ? reinterpret_cast<const GLB uint4*>(glb(g.St16)) : nullptr;
  const float sinv = St16g ? g.s16_inv : 1.0f;           // FP16 tiles hold S times a power of two
  GLB float* __restrict__ ug = reinterpret_cast<GLB float*>(glb(g.u));
  const int NB = (n + 63) >> 6;
  const int ntile = NB * (NB + 1) / 2;
  RB = min(RB, PhaseBShape<real>::RMAX);
  float* bLf = reinterpret_cast<float*>(bL);
  float* uL = bLf + (size_t)RB * ldS;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int rb = 0; rb < g.R; rb += RB) {
    const int rn = min(RB, g.R - rb);
    bool any = false;
    for (int r = rb; r < rb + rn; ++r) any = any || c.active[c.isys[r]];
    if (!any) continue;
    __syncthreads();
    copy16<BS, 16, false>(reinterpret_cast<uint4*>(bLf), reinterpret_cast<const GLB uint4*>(glb(g.b) + (size_t)rb * ldS),
                          rn * ldS / 4);
    for (int idx = threadIdx.x; idx < rn * ldS; idx += BS) uL[idx] = 0.f;
    __syncthreads();
    // tile (I, J) of flat upper-triangle index f = wid, wid + nw, ... (row-major over I <= J).
    // With packed tiles the wave loads the first half of its next tile (FP16: all of it) into
    // `pre` while it works on the current one, so that half a tile of loads stays in flight
    // during the arithmetic (a whole FP32 tile there would spill registers).
    int I = 0, J = wid;
    while (J >= NB && I < NB) { J -= NB - I - 1; ++I; }
    constexpr int kPre = 8;
    float4 pre[kPre];
    for (int f = wid; f < ntile; f += nw) {
      const int row0 = 64 * I + 16 * rg;
      const int col0 = 64 * J + 4 * cq;
      const bool cok = col0 < ldS;   // ldS is a multiple of 4: the whole 16-byte word is in the row
      float4 sv[16];
      if (St16g) {
        // FP16 tile: load u of the wave reads the contiguous kilobyte u, two rows per lane; the
        // whole tile was loaded during the previous tile's product
        const GLB uint4* tile = St16g + (size_t)f * (kTile * kTile / 8);
        typedef _Float16 half2v __attribute__((ext_vector_type(2)));
        if (f == wid) {
#pragma unroll
          for (int u = 0; u < 8; ++u) pre[u] = __builtin_bit_cast(float4, tile[(u * 4 + rg) * 16 + cq]);
        }
        uint4 cw[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) cw[u] = __builtin_bit_cast(uint4, pre[u]);
        if (f + nw < ntile) {
          const GLB uint4* nt = tile + (size_t)nw * (kTile * kTile / 8);
#pragma unroll
          for (int u = 0; u < 8; ++u) pre[u] = __builtin_bit_cast(float4, nt[(u * 4 + rg) * 16 + cq]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint4 w = cw[u];
          const half2v a0 = __builtin_bit_cast(half2v, w.x), a1 = __builtin_bit_cast(half2v, w.y);
          const half2v b0 = __builtin_bit_cast(half2v, w.z), b1 = __builtin_bit_cast(half2v, w.w);
          sv[2 * u] = make_float4((float)a0.x, (float)a0.y, (float)a1.x, (float)a1.y);
          sv[2 * u + 1] = make_float4((float)b0.x, (float)b0.y, (float)b1.x, (float)b1.y);
        }
      } else if (Stg) {
        // packed tile: load t of the wave reads the contiguous kilobyte t (zero beyond n); the
        // first half of each tile was loaded during the previous tile's product
        const GLB float4* tile = reinterpret_cast<const GLB float4*>(Stg + (size_t)f * (kTile * kTile));
        if (f == wid) {
#pragma unroll
          for (int t = 0; t < kPre; ++t) pre[t] = tile[(t * 4 + rg) * 16 + cq];
        }
#pragma unroll
        for (int t = kPre; t < 16; ++t) sv[t] = tile[(t * 4 + rg) * 16 + cq];
#pragma unroll
        for (int t = 0; t < kPre; ++t) sv[t] = pre[t];
        if (f + nw < ntile) {
          const GLB float4* nt = tile + (size_t)nw * (kTile * kTile / 4);
#pragma unroll
          for (int t = 0; t < kPre; ++t) pre[t] = nt[(t * 4 + rg) * 16 + cq];
        }
      } else {
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int row = row0 + t;
          sv[t] = (cok && row < n) ? *reinterpret_cast<const GLB float4*>(Sg + (size_t)row * ldS + col0) : z4;
        }
      }
#pragma unroll 1
      for (int r = 0; r < rn; ++r) {
        const float* b = bLf + (size_t)r * ldS;
        const float4 bj = cok ? *reinterpret_cast<const float4*>(b + col0) : z4;
        // row sums over this lane's four columns, then over the 16 lanes of the row group
        float h[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) h[t] = sv[t].x * bj.x + sv[t].y * bj.y + sv[t].z * bj.z + sv[t].w * bj.w;
        row_halve<8>(h, cq & 8);
        row_halve<4>(h, cq & 4);
        row_halve<2>(h, cq & 2);
        row_halve<1>(h, cq & 1);
        if (64 * I + lane < n) atomicAdd(&uL[(size_t)r * ldS + 64 * I + lane], h[0] * sinv);
        if (I < J) {
          // rows 16rg .. 16rg + 15 of b_I (row0 is a multiple of 16, as is ldS)
          float bi[16];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float4 v = row0 < ldS ? *reinterpret_cast<const float4*>(b + row0 + 4 * q) : z4;
            bi[4 * q] = v.x; bi[4 * q + 1] = v.y; bi[4 * q + 2] = v.z; bi[4 * q + 3] = v.w;
          }
          float cp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int t = 0; t < 16; ++t) {
            cp[0] += sv[t].x * bi[t]; cp[1] += sv[t].y * bi[t];
            cp[2] += sv[t].z * bi[t]; cp[3] += sv[t].w * bi[t];
          }
          // over the four row groups (lanes cq + 16 rg): column 4cq + rg stays with lane (rg, cq)
          const bool g1 = rg & 2, g0 = rg & 1;
          const float c0 = (g1 ? cp[2] : cp[0]) + __shfl_xor(g1 ? cp[0] : cp[2], 32, 64);
          const float c1 = (g1 ? cp[3] : cp[1]) + __shfl_xor(g1 ? cp[1] : cp[3], 32, 64);
          const float cs = (g0 ? c1 : c0) + __shfl_xor(g0 ? c0 : c1, 16, 64);
          if (col0 + rg < n) atomicAdd(&uL[(size_t)r * ldS + col0 + rg], cs * sinv);
        }
      }
      // next tile of this wave: nw further along the flat index
      J += nw;
      while (J >= NB && I < NB) { J -= NB - I - 1; ++I; }
    }
    __syncthreads();
    if (g.R <= RB) return reinterpret_cast<const real*>(uL);   // phase C reads u from LDS
    for (int idx = threadIdx.x; idx < rn * n; idx += BS) {
      const int r = idx / n, l = idx - r * n;
      ug[(size_t)(rb + r) * ldS + l] = uL[(size_t)r * ldS + l];
    }
  }
  return nullptr;
}

// Dipole moments of coupled instances, mu_I = sum_i Ms_L(i) V_i y_i of a stage input y: every
// writer of a stage input adds its nodes' share into c.mom (LDS atomics, zeroed by the caller)
// and then into the global slot of the evaluation that reads that input.
__device__ __forceinline__ void mom_add(Ctl& c, const InstConst& ic, int r, int L, double V, double y0,
                                        double y1, double y2) {
  if (!c.coupled[r]) return;
  const double w = ic.Ms[L] * V;
  atomicAdd(&c.mom[r][0], w * y0);
  atomicAdd(&c.mom[r][1], w * y1);
  atomicAdd(&c.mom[r][2], w * y2);
}

// field of the coupled neighbours at each coupled instance from the moments in c.mom
template <int BS>
__device__ __forceinline__ void dipole_fields(Ctl& c, const InstConst* icL, const double* dipL, int R) {
  if (dipL) {
    // one (instance, component) per thread from the pair geometry staged at launch start
    for (int q = threadIdx.x; q < R * 3; q += BS) {
      const int J = q / 3, d = q - 3 * J;
      double B = 0.0;
      if (c.coupled[J]) {
        for (int I = 0; I < R; ++I) {
          if (I == J || !c.coupled[I] || c.isys[I] != c.isys[J]) continue;
          const double* gJI = dipL + ((size_t)J * R + I) * 4;
          const double* mu = c.mom[I];
          const double mr = mu[0] * gJI[0] + mu[1] * gJI[1] + mu[2] * gJI[2];
          B += gJI[3] * (3.0 * mr * gJI[d] - mu[d]);
        }
      }
      c.Bdip[J][d] = B;
    }
  } else {
    for (int J = threadIdx.x; J < R; J += BS) {
      double B0 = 0.0, B1 = 0.0, B2 = 0.0;
      if (c.coupled[J]) {
        const InstConst& cj = icL[J];
        for (int I = 0; I < R; ++I) {
          if (I == J || !c.coupled[I] || c.isys[I] != c.isys[J]) continue;
          const InstConst& ci = icL[I];
          const double* mu = c.mom[I];
          const double d0 = cj.off[0] - ci.off[0], d1 = cj.off[1] - ci.off[1], d2 = cj.off[2] - ci.off[2];
          const double rr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
          const double e0 = d0 / rr, e1 = d1 / rr, e2 = d2 / rr;
          const double mr = mu[0] * e0 + mu[1] * e1 + mu[2] * e2;
          const double f = kMu0 / (4.0 * kPi * rr * rr * rr);
          B0 += f * (3.0 * mr * e0 - mu[0]);
          B1 += f * (3.0 * mr * e1 - mu[1]);
          B2 += f * (3.0 * mr * e2 - mu[2]);
        }
      }
      c.Bdip[J][0] = B0; c.Bdip[J][1] = B1; c.Bdip[J][2] = B2;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// phase C: effective field, LLG right-hand side, next stage input, reductions
// ---------------------------------------------------------------------------------------------

// One (instance r, node i = i0 + k) pair of stage s: every load the pair needs (own and partner
// magnetisation, exchange sums, potentials of the CSR row, m and the earlier stages) is issued
// before the arithmetic that consumes it.  s is uniform over the workgroup, so the loads of the
// stages below s are predicated by scalar branches and stay in flight together.
template <typename real, bool kL, bool kX>
__device__ __forceinline__ void pair_C(const GroupView<real>& g, const RunParams& P, Ctl& c, const InstConst& ic,
                                       int s, int r, int k, int i0, int sl, const GLB real* __restrict__ ysrc,
                                       GLB real* __restrict__ ydst, const Csr<real, kL>& cs, const real* uL) {
  const int nk = s < 6 ? s : 6;     // earlier stages read
  const int n = g.n, ldS = g.ldS, i = i0 + k;
  const size_t st3 = (size_t)3 * n;
  const double h = c.h[sl];
  const double ts = c.t[sl] + kC[s] * h;
  const GLB real* y = ysrc + (size_t)r * st3;
  const GLB real* yex = glb(g.yex) + (size_t)r * st3;
  const GLB real* u = glb(g.u) + (size_t)r * ldS;
  GLB real* kr = glb(g.k) + (size_t)r * 7 * st3;
  const GLB real* m = glb(g.m) + (size_t)r * st3;
  GLB real* yn = ydst + (size_t)r * st3;
  const int L = cs.lay[k];
  const real Vi = cs.V[k];
  const int p = cs.pt[k];
  const int pp = p >= 0 ? p : i;
  // loads
  const real mx = xld<kX>(y + i), my = xld<kX>(y + n + i), mz = xld<kX>(y + 2 * n + i);
  const real ex0 = yex[i], ex1 = yex[n + i], ex2 = yex[2 * n + i];
  const real px = xld<kX>(y + pp), py = xld<kX>(y + n + pp), pz = xld<kX>(y + 2 * n + pp);
  real mm[3], kl[6][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) mm[d] = m[d * n + i];
#pragma unroll
  for (int l = 0; l < 6; ++l)
#pragma unroll
    for (int d = 0; d < 3; ++d) kl[l][d] = l < nk ? kr[(size_t)l * st3 + d * n + i] : (real)0;
  // demag: -mu0 / V_i (D^T u)_i
  real dx = 0, dy = 0, dz = 0;
  const int qa = cs.rp[k], qb = cs.rp[k + 1];
  constexpr int kGather = Gather<real, kX>::W;
  const real* uLr = uL ? uL + (size_t)r * ldS : nullptr;
  for (int q0 = qa; q0 < qb; q0 += kGather) {
    real uq[kGather];
    if (uLr) {
#pragma unroll
      for (int w = 0; w < kGather; ++w) uq[w] = uLr[q0 + w < qb ? (cs.col[q0 + w] & 0xFFFF) : i];
    } else {
#pragma unroll
      for (int w = 0; w < kGather; ++w) uq[w] = xld<kX>(u + (q0 + w < qb ? (cs.col[q0 + w] & 0xFFFF) : i));
    }
#pragma unroll
    for (int w = 0; w < kGather; ++w) {
      const int q = q0 + w;
      if (q < qb) {
        dx += cs.DT[3 * q] * uq[w];
        dy += cs.DT[3 * q + 1] * uq[w];
        dz += cs.DT[3 * q + 2] * uq[w];
      }
    }
  }
  const real gp = (real)ic.gp, al = (real)ic.alpha;
  // exchange
  const real cex = -(real)ic.cex[L] / Vi;
  real Bx = cex * ex0, By = cex * ex1, Bz = cex * ex2;
  // anisotropy
  const real ux = (real)ic.axis[L][0], uy = (real)ic.axis[L][1], uz = (real)ic.axis[L][2];
  const real mu = (real)ic.can[L] * (mx * ux + my * uy + mz * uz);
  Bx += mu * ux; By += mu * uy; Bz += mu * uz;
  // interlayer
  if (p >= 0) {
    const real ci = (real)ic.cint[L] * cs.aif[k] / Vi;
    Bx += ci * px; By += ci * py; Bz += ci * pz;
  }
  const real cd = -(real)kMu0 / Vi;
  Bx += cd * dx; By += cd * dy; Bz += cd * dz;
  // Zeeman (+ dipoles)
  if constexpr (sizeof(real) == 4) {
    float zx, zy, zz;
    const double zi = ic.fkind == BPM_FIELD_GRID ? glb(g.z)[i] + ic.off[2] : 0.0;
    applied_B_f32(ic, ts, cs.x[k] + ic.off[0], cs.y[k] + ic.off[1], zi, zx, zy, zz);
    if (c.coupled[r]) { zx += (float)c.Bdip[r][0]; zy += (float)c.Bdip[r][1]; zz += (float)c.Bdip[r][2]; }
    Bx += zx; By += zy; Bz += zz;
  } else {
    double zx, zy, zz;
    const double zi = ic.fkind == BPM_FIELD_GRID ? glb(g.z)[i] + ic.off[2] : 0.0;
    applied_B(ic, ts, cs.x[k] + ic.off[0], cs.y[k] + ic.off[1], zi, zx, zy, zz);
    if (c.coupled[r]) { zx += c.Bdip[r][0]; zy += c.Bdip[r][1]; zz += c.Bdip[r][2]; }
    Bx += (real)zx; By += (real)zy; Bz += (real)zz;
  }
  // LLG: dm/dt = -gp [ m x B + alpha m x (m x B) ]; relaxation runs drop the precession term and
  // so descend the energy along -m x (m x B)
  const real cx = my * Bz - mz * By, cy = mz * Bx - mx * Bz, cz = mx * By - my * Bx;
  const real dx2 = my * cz - mz * cy, dy2 = mz * cx - mx * cz, dz2 = mx * cy - my * cx;
  const real pr = (P.flags & BPM_FLAG_RELAX) ? (real)0 : (real)1;
  const real kx = -gp * (pr * cx + al * dx2), ky = -gp * (pr * cy + al * dy2), kz = -gp * (pr * cz + al * dz2);
  GLB real* ks = kr + (size_t)s * st3;
  ks[i] = kx; ks[n + i] = ky; ks[2 * n + i] = kz;
  if (s < 6) {
    // next stage input m + h sum_l a_{s+1,l} k_l (stage 7 input = 5th-order solution)
    real v[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      real acc = 0;
#pragma unroll
      for (int l = 0; l < 6; ++l)
        if (l < nk) acc += (real)(h * kA[s + 1][l]) * kl[l][d];
      v[d] = mm[d] + acc;
    }
    const real ha = (real)(h * kA[s + 1][s]);
    v[0] += ha * kx; v[1] += ha * ky; v[2] += ha * kz;
    xst<kX>(yn + i, v[0]); xst<kX>(yn + n + i, v[1]); xst<kX>(yn + 2 * n + i, v[2]);
    if (s >= 1) mom_add(c, ic, r, L, (double)Vi, (double)v[0], (double)v[1], (double)v[2]);
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
    const real rtol = (real)P.rtol, atol = (real)P.atol;
    real e[3] = {0, 0, 0};
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      const real he = (real)(h * kE[l]);
#pragma unroll
      for (int d = 0; d < 3; ++d) e[d] += he * kl[l][d];
    }
    const real he6 = (real)(h * kE[6]);
    e[0] += he6 * kx; e[1] += he6 * ky; e[2] += he6 * kz;
    const real y1[3] = {mx, my, mz};
    double es = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const real sc = atol + rtol * fmax(fabs(mm[d]), fabs(y1[d]));
      const real qq = e[d] / sc;
      es += (double)(qq * qq);
    }
    atomicAdd(&c.errL[sl], es);
  }
}

template <typename real, bool kFixed, int BS, bool kL, bool kX>
__device__ __forceinline__ void phase_C(const GroupView<real>& g, const RunParams& P, Ctl& c, const InstConst* icL,
                                        const double* dipL, int i0, int i1, int s, const real* ysrc_, real* ydst_,
                                        int it, int ev, const Csr<real, kL>& cs, const real* uL) {
  const int nown = i1 - i0;
  const GLB real* ysrc = glb(ysrc_);
  GLB real* ydst = glb(ydst_);
  // moments of the next stage input (written below) of coupled instances
  if (c.any_coupled)
    for (int q = threadIdx.x; q < g.R * 3; q += BS) c.mom[q / 3][q % 3] = 0.0;
  if (s >= 5) {
    for (int q = threadIdx.x; q < g.R * 6; q += BS) c.accL[q / 6][q % 6] = 0.0;
    for (int q = threadIdx.x; q < g.nsys; q += BS) c.errL[q] = 0.0;
  }
  __syncthreads();
  for (int it2 = threadIdx.x; it2 < g.R * nown; it2 += BS) {
    const int r = it2 / nown, k = it2 - r * nown;
    const int sl = c.isys[r];
    if (!c.active[sl]) continue;
    pair_C<real, kL, kX>(g, P, c, icL[r], s, r, k, i0, sl, ysrc, ydst, cs, uL);
  }
  if (c.any_coupled && s >= 1 && s < 6) {
    __syncthreads();
    for (int q = threadIdx.x; q < g.R * 3; q += BS) {
      const int r = q / 3, d = q % 3;
      if (c.coupled[r] && c.active[c.isys[r]])
        atomicAdd(&P.mom_acc[((size_t)(g.inst0 + r) * 3 + (ev + 1) % 3) * 3 + d], c.mom[r][d]);
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

template <typename real, bool kFixed, int BS, bool kL, bool kX>
__device__ __forceinline__ void field_eval(const GroupView<real>& g, const RunParams& P, Ctl& c, const InstConst* icL,
                                           const double* dipL, GroupSync& gs, int i0, int i1, int s, const real* ysrc,
                                           real* ydst, int it, int ev, real* bL, const real* SL, real* part, int RB,
                                           const Csr<real, kL>& cs) {
  phase_A<real, BS, kL, kX>(g, P, c, icL, i0, i1, ysrc, ev, cs);
  group_sync<kX>(gs);
  // dipole moments of this stage input (complete after the barrier): loaded now, consumed after
  // the demag product, so that their latency hides behind it
  const bool mq = c.any_coupled && threadIdx.x < g.R * 3;
  double mv = 0.0;
  if (mq) mv = acc_ld(&P.mom_acc[((size_t)(g.inst0 + threadIdx.x / 3) * 3 + ev % 3) * 3 + threadIdx.x % 3]);
  bool done = false;
  const real* uL = nullptr;
  if constexpr (!kX && sizeof(real) == 4) {
    if (!SL && g.G == 1 && (P.flags & BPM_FLAG_SYMMETRIC_DEMAG)) {
      uL = phase_B_sym<real, BS>(g, c, bL, RB);
      done = true;
    }
  }
  if (!done) {
    if (SL) phase_B<real, BS, true, kX>(g, c, i0, i1, bL, SL, part, RB);
    else phase_B<real, BS, false, kX>(g, c, i0, i1, bL, nullptr, part, RB);
  }
  if (c.any_coupled) {
    if (mq) c.mom[threadIdx.x / 3][threadIdx.x % 3] = mv;
    __syncthreads();
    dipole_fields<BS>(c, icL, dipL, g.R);
  }
  group_sync<kX>(gs);
  phase_C<real, kFixed, BS, kL, kX>(g, P, c, icL, dipL, i0, i1, s, ysrc, ydst, it, ev, cs, uL);
  group_sync<kX>(gs);
}

// trajectory sample of instance r (called by one thread of the group's first workgroup)
template <typename real, int BS>
__device__ __forceinline__ void save_sample(const GroupView<real>& g, const RunParams& P, Ctl& c, const InstConst* icL,
                                            int r, double t, double dt, double err, const double* ob) {
  if (P.traj_cap <= 0 || c.ntraj[r] >= P.traj_cap) return;
  const int gi = g.inst0 + r;
  const InstConst& ic = icL[r];
  double bx, by, bz;
  applied_B(ic, t, g.cen[0] + ic.off[0], g.cen[1] + ic.off[1], g.cen[2] + ic.off[2], bx, by, bz);
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

// step size of the coming attempt of every active system
template <bool kFixed, int BS>
__device__ __forceinline__ void plan_attempt(const RunParams& P, Ctl& c, int nsys, long long nfix) {
  for (int sl = threadIdx.x; sl < nsys; sl += BS) {
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
}

template <typename real, bool kFixed, int BS, bool kL, bool kX>
__device__ __forceinline__ void dp5_body(const GroupView<real>& g, const RunParams& P, Ctl& c, const InstConst* icL,
                                         double* dipL, int w, real* bL, const real* SL, real* part, int RB,
                                         const Csr<real, kL>& cs) {
  const int n = g.n;
  const int i0 = (int)((long long)n * w / g.G), i1 = (int)((long long)n * (w + 1) / g.G);
  const int nown = i1 - i0;
  const size_t st3 = (size_t)3 * n;
  const size_t ybuf = (size_t)g.R * st3;
  GroupSync gs{g.bar, 0ull, g.G};
  const bool lead = (w == 0);
  GLB real* __restrict__ mg = glb(g.m);
  GLB real* __restrict__ kg = glb(g.k);
  const long long nfix = kFixed ? (long long)ceil(P.t_end / P.dt_fixed - 1e-9) : 0;

  // ---- init control state: a fresh run starts at t = 0; a continued run (P.resume) takes the
  // controller state, counters and crossing state the previous launch left in sys_out / inst_out
  for (int sl = threadIdx.x; sl < g.nsys; sl += BS) {
    if (P.resume) {
      const SysOut& so = P.sys_out[g.sys0 + sl];
      c.t[sl] = so.t_reached; c.dt[sl] = so.dt_next; c.fac[sl] = so.fac;
      c.dtmin[sl] = so.n_accept ? so.dt_min_used : INFINITY; c.dtmax[sl] = so.dt_max_used;
      c.maxdev[sl] = so.max_norm_dev; c.istep[sl] = so.istep; c.nacc[sl] = so.n_accept; c.nrej[sl] = so.n_reject;
      c.status[sl] = so.status; c.active[sl] = (so.status == BPM_OK && so.t_reached < P.t_end) ? 1 : 0;
    } else {
      c.t[sl] = 0.0; c.dt[sl] = kFixed ? P.dt_fixed : P.dt0; c.fac[sl] = 5.0;
      c.dtmin[sl] = INFINITY; c.dtmax[sl] = 0.0; c.maxdev[sl] = 0.0;
      c.istep[sl] = 0; c.nacc[sl] = 0; c.nrej[sl] = 0;
      c.status[sl] = BPM_OK; c.active[sl] = P.t_end > 0.0 ? 1 : 0;
    }
    c.h[sl] = 0.0; c.err[sl] = 0.0; c.last[sl] = 0; c.ninst[sl] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    c.any_coupled = 0;
    for (int r = 0; r < g.R; ++r) {
      const int sl = icL[r].sys - g.sys0;
      c.isys[r] = sl;
      c.ninst[sl] += 1;
      c.coupled[r] = P.sys[g.sys0 + sl].coupled;
      c.any_coupled |= c.coupled[r];
      if (P.resume) {
        const InstOut& io = P.inst_out[g.inst0 + r];
        c.crossed[r] = io.crossed; c.ntraj[r] = io.n_traj; c.tsw[r] = io.t_sw;
        c.prev_t[r] = io.prev_t; c.prev_v[r] = io.prev_v; c.mzs[r] = io.mz_soft; c.mzh[r] = io.mz_hard;
      } else {
        c.crossed[r] = 0; c.ntraj[r] = 0; c.tsw[r] = NAN;
      }
    }
  }
  __syncthreads();
  if (dipL) {
    // pair geometry of the coupled instances, the same expressions as the on-the-fly path
    for (int q = threadIdx.x; q < g.R * g.R; q += BS) {
      const int J = q / g.R, I = q - J * g.R;
      double* gJI = dipL + (size_t)q * 4;
      gJI[0] = gJI[1] = gJI[2] = gJI[3] = 0.0;
      if (I == J) continue;
      const double d0 = icL[J].off[0] - icL[I].off[0], d1 = icL[J].off[1] - icL[I].off[1];
      const double d2 = icL[J].off[2] - icL[I].off[2];
      const double rr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      gJI[0] = d0 / rr; gJI[1] = d1 / rr; gJI[2] = d2 / rr;
      gJI[3] = kMu0 / (4.0 * kPi * rr * rr * rr);
    }
    __syncthreads();
  }

  // ---- prologue: stage input = m0, observables of m0, first right-hand side (a continued run
  // keeps m and the first-stage slope k1 of its last accepted step and skips it)
  real* ys0 = g.ys;
  real* ys1 = g.ys + ybuf;
  if (!P.resume) {
  for (int q = threadIdx.x; q < g.R * 6; q += BS) c.accL[q / 6][q % 6] = 0.0;
  __syncthreads();
  for (int it2 = threadIdx.x; it2 < g.R * nown; it2 += BS) {
    const int r = it2 / nown, k = it2 - r * nown, i = i0 + k;
    const InstConst& ic = icL[r];
    const int L = cs.lay[k];
    const double Vd = (double)cs.V[k], Ms = ic.Ms[L];
    real v[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      v[d] = mg[(size_t)r * st3 + d * n + i];
      xst<kX>(glb(ys0) + (size_t)r * st3 + d * n + i, v[d]);
    }
    atomicAdd(&c.accL[r][L ? 1 : 0], Vd * (double)v[2]);
    atomicAdd(&c.accL[r][2], Ms * Vd * (double)v[0]);
    atomicAdd(&c.accL[r][3], Ms * Vd * (double)v[1]);
    atomicAdd(&c.accL[r][4], Ms * Vd * (double)v[2]);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < g.R * 5; q += BS)
    atomicAdd(&P.obs_acc[((size_t)(g.inst0 + q / 5) * 3 + 2) * 6 + q % 5], c.accL[q / 5][q % 5]);
  // dipole moments of m0 (the sums Ms V m of the observables) for the first evaluation
  if (c.any_coupled)
    for (int q = threadIdx.x; q < g.R * 3; q += BS)
      if (c.coupled[q / 3]) atomicAdd(&P.mom_acc[((size_t)(g.inst0 + q / 3) * 3 + 0) * 3 + q % 3], c.accL[q / 3][2 + q % 3]);
  group_sync<kX>(gs);
  }
  // One call site of the field evaluation (its code is large): the evaluation of stage 0 of the
  // prologue is the first pass of the loop, then stages 1..6 of every attempt.  A continued run
  // enters the loop past that evaluation (the moment slot of the next stage input is then 1).
  int ev = P.resume ? 1 : 0, it = 0, s = 0;
  bool skip0 = P.resume != 0;
  for (;;) {
    if (s == 1) {
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
          for (int d = 0; d < 6; ++d) acc_st(&P.obs_acc[((size_t)(g.inst0 + r) * 3 + (it + 2) % 3) * 6 + d], 0.0);
        for (int sl = threadIdx.x; sl < g.nsys; sl += BS) acc_st(&P.err_acc[(size_t)(g.sys0 + sl) * 3 + (it + 2) % 3], 0.0);
      }
    }
    if (!skip0) {
      // the moment slot of the next evaluation, filled by the writers of its stage input
      if (lead && c.any_coupled)
        for (int r = threadIdx.x; r < g.R; r += BS)
          for (int d = 0; d < 3; ++d) acc_st(&P.mom_acc[((size_t)(g.inst0 + r) * 3 + (ev + 1) % 3) * 3 + d], 0.0);
      const real* src = (s & 1) ? ys1 : ys0;
      real* dst = (s & 1) ? ys0 : ys1;
      field_eval<real, kFixed, BS, kL, kX>(g, P, c, icL, dipL, gs, i0, i1, s, src, dst, it, ev++, bL, SL, part, RB, cs);
    }
    if (s == 0) {
      // initial observables, crossing state, first trajectory sample (fresh runs)
      for (int r = threadIdx.x; r < g.R && !skip0; r += BS) {
        double ob[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) ob[d] = acc_ld(&P.obs_acc[((size_t)(g.inst0 + r) * 3 + 2) * 6 + d]);
        const double vh = g.Vhard > 0 ? ob[1] / g.Vhard : 0.0;
        c.prev_t[r] = 0.0; c.prev_v[r] = vh;
        c.mzs[r] = g.Vsoft > 0 ? ob[0] / g.Vsoft : 0.0; c.mzh[r] = vh;
        if (vh <= 0.0) { c.crossed[r] = 1; c.tsw[r] = 0.0; }
        if (lead) save_sample<real, BS>(g, P, c, icL, r, 0.0, 0.0, 0.0, ob);
      }
      skip0 = false;
      for (int q = threadIdx.x; q < g.R * 3; q += BS) c.mom[q / 3][q % 3] = 0.0;
      __syncthreads();
      plan_attempt<kFixed, BS>(P, c, g.nsys, nfix);
      __syncthreads();
      for (int it2 = threadIdx.x; it2 < g.R * nown; it2 += BS) {
        const int r = it2 / nown, k = it2 - r * nown, i = i0 + k;
        const int sl = c.isys[r];
        if (!c.active[sl]) continue;
        const real ha = (real)(c.h[sl] * kA[1][0]);
        const GLB real* m = mg + (size_t)r * st3;
        const GLB real* k0 = kg + (size_t)r * 7 * st3;
        GLB real* yn = glb(ys1) + (size_t)r * st3;
        real v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          v[d] = m[d * n + i] + ha * k0[d * n + i];
          xst<kX>(yn + d * n + i, v[d]);
        }
        mom_add(c, icL[r], r, cs.lay[k], (double)cs.V[k], (double)v[0], (double)v[1], (double)v[2]);
      }
      if (c.any_coupled) {
        __syncthreads();
        for (int q = threadIdx.x; q < g.R * 3; q += BS)
          if (c.coupled[q / 3] && c.active[c.isys[q / 3]])
            atomicAdd(&P.mom_acc[((size_t)(g.inst0 + q / 3) * 3 + ev % 3) * 3 + q % 3], c.mom[q / 3][q % 3]);
      }
      group_sync<kX>(gs);
      s = 1;
      continue;
    }
    if (s < 6) {
      ++s;
      continue;
    }
    s = 1;
    // ---- step decision per system (identical in every workgroup)
    for (int sl = threadIdx.x; sl < g.nsys; sl += BS) {
      c.accepted[sl] = 0;
      if (!c.active[sl]) continue;
      const double acc = acc_ld(&P.err_acc[(size_t)(g.sys0 + sl) * 3 + it % 3]);
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
          // a step shortened to land on t_end hands a continued run the step planned before the
          // shortening when that is longer (c.dt still holds it); a run that ends here is unaffected
          c.dt[sl] = c.last[sl] ? fmax(h * fac, c.dt[sl]) : h * fac;
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
      double ob[6];
#pragma unroll
      for (int d = 0; d < 6; ++d) ob[d] = acc_ld(&P.obs_acc[((size_t)(g.inst0 + r) * 3 + it % 3) * 6 + d]);
      const double vh = g.Vhard > 0 ? ob[1] / g.Vhard : 0.0;
      const double t = c.t[sl];
      c.mzs[r] = g.Vsoft > 0 ? ob[0] / g.Vsoft : 0.0; c.mzh[r] = vh;
      if (!c.crossed[r] && vh <= 0.0) {
        c.crossed[r] = 1;
        c.tsw[r] = (c.prev_v[r] <= 0.0 || t == c.prev_t[r]) ? t : c.prev_t[r] + (t - c.prev_t[r]) * c.prev_v[r] / (c.prev_v[r] - vh);
      }
      c.prev_t[r] = t; c.prev_v[r] = vh;
      const bool save = (P.save_every > 0 && c.nacc[sl] % P.save_every == 0) || !c.active[sl];
      if (lead && save) save_sample<real, BS>(g, P, c, icL, r, t, c.h[sl], c.err[sl], ob);
    }
    __syncthreads();
    // largest |1 - |y|| before renormalisation, over the instances of each accepted system
    for (int sl = threadIdx.x; sl < g.nsys; sl += BS) {
      if (!c.accepted[sl]) continue;
      for (int r = 0; r < g.R; ++r) {
        if (c.isys[r] != sl) continue;
        const double dev = acc_ld(&P.obs_acc[((size_t)(g.inst0 + r) * 3 + it % 3) * 6 + 5]);
        if (dev > c.maxdev[sl]) c.maxdev[sl] = dev;
      }
    }
    for (int q = threadIdx.x; q < g.R * 3; q += BS) c.mom[q / 3][q % 3] = 0.0;
    plan_attempt<kFixed, BS>(P, c, g.nsys, nfix);
    __syncthreads();
    // accepted: m <- y / |y| (the stage-7 input), k1 <- k7; then the stage-2 input of the next
    // attempt of every active system, from the values already in registers
    for (int it2 = threadIdx.x; it2 < g.R * nown; it2 += BS) {
      const int r = it2 / nown, k = it2 - r * nown, i = i0 + k;
      const int sl = c.isys[r];
      const bool acc = c.accepted[sl], act = c.active[sl];
      if (!acc && !act) continue;
      GLB real* m = mg + (size_t)r * st3;
      GLB real* k0 = kg + (size_t)r * 7 * st3;
      real mv[3], kv[3];
      if (acc) {
        const GLB real* y7 = glb(ys0) + (size_t)r * st3;
        const GLB real* k6 = k0 + 6 * st3;
        const real a = xld<kX>(y7 + i), b = xld<kX>(y7 + n + i), d = xld<kX>(y7 + 2 * n + i);
        kv[0] = k6[i]; kv[1] = k6[n + i]; kv[2] = k6[2 * n + i];
        const real inv = (real)1 / sqrt(a * a + b * b + d * d);
        mv[0] = a * inv; mv[1] = b * inv; mv[2] = d * inv;
        m[i] = mv[0]; m[n + i] = mv[1]; m[2 * n + i] = mv[2];
        k0[i] = kv[0]; k0[n + i] = kv[1]; k0[2 * n + i] = kv[2];
      } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) { mv[d] = m[d * n + i]; kv[d] = k0[d * n + i]; }
      }
      if (act) {
        const real ha = (real)(c.h[sl] * kA[1][0]);
        GLB real* yn = glb(ys1) + (size_t)r * st3;
        real v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          v[d] = mv[d] + ha * kv[d];
          xst<kX>(yn + d * n + i, v[d]);
        }
        mom_add(c, icL[r], r, cs.lay[k], (double)cs.V[k], (double)v[0], (double)v[1], (double)v[2]);
      }
    }
    if (c.any_coupled) {
      __syncthreads();
      for (int q = threadIdx.x; q < g.R * 3; q += BS)
        if (c.coupled[q / 3] && c.active[c.isys[q / 3]])
          atomicAdd(&P.mom_acc[((size_t)(g.inst0 + q / 3) * 3 + ev % 3) * 3 + q % 3], c.mom[q / 3][q % 3]);
    }
    group_sync<kX>(gs);
    ++it;
  }
  // results (every system of the group has finished)
  if (lead) {
    for (int sl = threadIdx.x; sl < g.nsys; sl += BS) {
      SysOut& o = P.sys_out[g.sys0 + sl];
      o.status = c.status[sl]; o.t_reached = c.t[sl]; o.n_accept = c.nacc[sl]; o.n_reject = c.nrej[sl];
      o.dt_min_used = c.nacc[sl] ? c.dtmin[sl] : 0.0; o.dt_max_used = c.dtmax[sl]; o.max_norm_dev = c.maxdev[sl];
      o.dt_next = c.dt[sl]; o.fac = c.fac[sl]; o.istep = c.istep[sl];
    }
    for (int r = threadIdx.x; r < g.R; r += BS) {
      InstOut& o = P.inst_out[g.inst0 + r];
      o.crossed = c.crossed[r]; o.t_sw = c.tsw[r]; o.mz_soft = c.mzs[r]; o.mz_hard = c.mzh[r];
      o.switched = c.mzh[r] < 0.0; o.n_traj = c.ntraj[r];
      o.prev_t = c.prev_t[r]; o.prev_v = c.prev_v[r];
    }
  }
}


template <typename real, bool kFixed, int BS, bool kL, bool kX>
__device__ __forceinline__ void dp5_entry(const GroupView<real>* __restrict__ groups, const RunParams& P, int RB,
                                          const LdsPlan& LP, unsigned char* smem_raw, Ctl& c) {
  const int2 gm = P.wg_map[blockIdx.x];
  const GroupView<real> g = groups[gm.x];
  const int w = gm.y;
  const int n = g.n, ldS = g.ldS;
  const int i0 = (int)((long long)n * w / g.G), i1 = (int)((long long)n * (w + 1) / g.G);
  const int nown = i1 - i0;
  // ---- dynamic LDS: instance constants, staged right-hand sides, CSR rows, S rows
  unsigned char* lp = smem_raw;
  InstConst* icL = reinterpret_cast<InstConst*>(lp);
  lp += ic_stage_bytes(LP.ic_slots);
  double* dipL = LP.dip_slots >= g.R ? reinterpret_cast<double*>(lp) : nullptr;
  lp += dip_stage_bytes(LP.dip_slots);
  real* bL = reinterpret_cast<real*>(lp);
  lp += ((size_t)LP.bl_elems * sizeof(real) + 15) / 16 * 16;
  // per-wave round sums of the demag product for rows longer than one round (the launch plan
  // reserves them at the end of the right-hand-side area when such rows can occur)
  real* part = LP.ldS > 12 * (64 * (int)(16 / sizeof(real))) ? bL + LP.bl_elems - (BS / 64) * 4 * 16 : bL;
  unsigned char* csr_lds = lp;
  lp += csr_stage_bytes<real>(LP.csr_cap, LP.own_cap);
  // S rows are resident only when this workgroup's rows fit the planned area
  real* SL = (LP.s_rows > 0 && nown <= LP.s_rows) ? reinterpret_cast<real*>(lp) : nullptr;
  copy16<BS, 4, false>(reinterpret_cast<uint4*>(icL), reinterpret_cast<const GLB uint4*>(glb(P.inst + g.inst0)),
                (int)(g.R * sizeof(InstConst) / 16));
  if (SL) {
    // the owned rows of S, once for the whole launch
    constexpr int VEC = 16 / sizeof(real);
    copy16<BS, 8, false>(reinterpret_cast<uint4*>(SL), reinterpret_cast<const GLB uint4*>(glb(g.S) + (size_t)i0 * ldS),
                  nown * ldS / VEC);
  }
  if constexpr (kL) {
    // CSR rows and node data of the owned nodes, once for the whole launch (the launch plan sizes
    // csr_cap and own_cap for the largest workgroup share; the copies are clamped to them)
    const int cap = LP.csr_cap, ocap = LP.own_cap;
    const int q0 = g.rowptr[i0], nq = min(g.rowptr[i1] - q0, cap), no = min(nown, ocap);
    double* xL = reinterpret_cast<double*>(csr_lds);
    double* yL = xL + ocap;
    real* KL = reinterpret_cast<real*>(yL + ocap);
    real* DL = KL + cap;
    real* DTL = DL + 3 * cap;
    real* VL = DTL + 3 * cap;
    real* aL = VL + ocap;
    int32_t* colL = reinterpret_cast<int32_t*>(aL + ocap);
    int32_t* rpL = colL + cap;
    int32_t* ptL = rpL + ocap + 1;
    int32_t* layL = ptL + ocap;
    const GLB int32_t* colx = glb(g.colx);
    const GLB real* Kg = glb(g.K);
    const GLB real* Dg = glb(g.D);
    const GLB real* DTg = glb(g.DT);
    for (int q = threadIdx.x; q < nq; q += BS) {
      colL[q] = colx[q0 + q];
      KL[q] = Kg[q0 + q];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        DL[3 * q + d] = Dg[3 * (q0 + q) + d];
        DTL[3 * q + d] = DTg[3 * (q0 + q) + d];
      }
    }
    for (int k = threadIdx.x; k <= no; k += BS) rpL[k] = min(g.rowptr[i0 + k] - q0, nq);
    for (int k = threadIdx.x; k < no; k += BS) {
      ptL[k] = g.partner[i0 + k]; layL[k] = g.layer[i0 + k];
      VL[k] = g.V[i0 + k]; aL[k] = g.aif[i0 + k];
      xL[k] = g.x[i0 + k]; yL[k] = g.y[i0 + k];
    }
    const Csr<real, true> cs{rpL, colL, KL, DL, DTL, ptL, layL, VL, aL, xL, yL};
    __syncthreads();
    dp5_body<real, kFixed, BS, true, kX>(g, P, c, icL, dipL, w, bL, SL, part, RB, cs);
  } else {
    const Csr<real, false> cs{glb(g.rowptr) + i0, glb(g.colx), glb(g.K), glb(g.D), glb(g.DT),
                              glb(g.partner) + i0, glb(g.layer) + i0, glb(g.V) + i0, glb(g.aif) + i0,
                              glb(g.x) + i0, glb(g.y) + i0};
    __syncthreads();
    dp5_body<real, kFixed, BS, false, kX>(g, P, c, icL, dipL, w, bL, SL, part, RB, cs);
  }
}

template <typename real, bool kFixed, int BS, bool kL, bool kX>
__global__ __launch_bounds__(BS, 2) void dp5_kernel(const GroupView<real>* __restrict__ groups,
                                                 RunParams P, int RB, LdsPlan LP) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ Ctl c;
  dp5_entry<real, kFixed, BS, kL, kX>(groups, P, RB, LP, smem_raw, c);
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
    applied_B(ic, t, g.x[i] + ic.off[0], g.y[i] + ic.off[1], g.z[i] + ic.off[2], bx, by, bz);
    e_loc += -ic.Ms[L] * Vi * (mi[0] * bx + mi[1] * by + mi[2] * bz);
  }
  __syncthreads();
  // demag: (mu0/2) b^T S b (S entries from the row-major copy, else from the packed tiles)
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nb = (n + kTile - 1) / kTile;
  double ed = 0.0;
  for (int k = wid; k < n; k += 256 / 64) {
    double acc = 0.0;
    for (int l = lane; l < n; l += 64) {
      double skl;
      if (g.S) {
        skl = (double)g.S[(size_t)k * g.ldS + l];
      } else if (!g.St) {
        const int a = min(k, l), b = max(k, l);
        const _Float16 h = reinterpret_cast<const _Float16*>(g.St16)[(size_t)tile_index(nb, a / kTile, b / kTile) * (kTile * kTile) +
                                                                    tile16_offset(a % kTile, b % kTile)];
        skl = (double)h * (double)g.s16_inv;
      } else {
        const int a = min(k, l), b = max(k, l);
        skl = (double)g.St[(size_t)tile_index(nb, a / kTile, b / kTile) * (kTile * kTile) +
                           tile_offset(a % kTile, b % kTile)];
      }
      acc += skl * bL[l];
    }
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
template <typename real, bool kL, bool kX>
static const void* dp5_fn_l(bool fixed, int bs) {
  if (bs == 512)
    return fixed ? reinterpret_cast<const void*>(&dp5_kernel<real, true, 512, kL, kX>)
                 : reinterpret_cast<const void*>(&dp5_kernel<real, false, 512, kL, kX>);
  return fixed ? reinterpret_cast<const void*>(&dp5_kernel<real, true, 256, kL, kX>)
               : reinterpret_cast<const void*>(&dp5_kernel<real, false, 256, kL, kX>);
}

// kernel variant of a launch: cooperative launches (groups spanning several workgroups) use the
// coherent exchange protocol, with the CSR view in LDS when the plan stages it
template <typename real>
static const void* dp5_fn(bool fixed, int bs, const LdsPlan& L, bool coop) {
  if (!coop) return dp5_fn_l<real, false, false>(fixed, bs);
  return L.csr_cap > 0 ? dp5_fn_l<real, true, true>(fixed, bs) : dp5_fn_l<real, false, true>(fixed, bs);
}

template <typename real>
size_t dp5_lds_bytes(const LdsPlan& L) { return lds_plan_bytes<real>(L); }

template <typename real>
hipError_t launch_dp5(const GroupView<real>* d_groups, const RunParams& P, int grid, int RB, const LdsPlan& L,
                      bool fixed, bool cooperative, hipStream_t stream, int bs) {
  const size_t shm = lds_plan_bytes<real>(L);
  LdsPlan Lc = L;
  void* args[] = {(void*)&d_groups, (void*)&P, (void*)&RB, (void*)&Lc};
  const void* fn = dp5_fn<real>(fixed, bs, L, cooperative);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  if (cooperative) return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(bs), args, shm, stream);
  return hipLaunchKernel(fn, dim3(grid), dim3(bs), args, shm, stream);
}

// resident workgroups per CU of the stepping kernel with this LDS plan (0 if it does not fit)
template <typename real>
hipError_t max_coresident(const LdsPlan& L, bool fixed, int bs, bool coop, int* per_cu, int* cus) {
  const size_t shm = lds_plan_bytes<real>(L);
  const void* fn = dp5_fn<real>(fixed, bs, L, coop);
  *per_cu = 0;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    e = hipSuccess;
  } else {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, bs, shm);
    if (e != hipSuccess) return e;
  }
  int dev;
  hipGetDevice(&dev);
  return hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
}

template <typename real>
hipError_t launch_energy(const GroupView<real>* d_groups, const int2* d_inst_map, int ninst,
                         const RunParams& P, double* d_energy, int nmax, hipStream_t stream) {
  const size_t shm = (size_t)nmax * sizeof(double);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&energy_kernel<real>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(energy_kernel<real>, dim3(ninst), dim3(kBlock), shm, stream, d_groups, d_inst_map,
                     P, d_energy);
  return hipGetLastError();
}

template size_t dp5_lds_bytes<float>(const LdsPlan&);
template size_t dp5_lds_bytes<double>(const LdsPlan&);
template hipError_t launch_dp5<float>(const GroupView<float>*, const RunParams&, int, int, const LdsPlan&, bool, bool, hipStream_t, int);
template hipError_t launch_dp5<double>(const GroupView<double>*, const RunParams&, int, int, const LdsPlan&, bool, bool, hipStream_t, int);
template hipError_t max_coresident<float>(const LdsPlan&, bool, int, bool, int*, int*);
template hipError_t max_coresident<double>(const LdsPlan&, bool, int, bool, int*, int*);
template hipError_t launch_energy<float>(const GroupView<float>*, const int2*, int, const RunParams&, double*, int, hipStream_t);
template hipError_t launch_energy<double>(const GroupView<double>*, const int2*, int, const RunParams&, double*, int, hipStream_t);

}  // namespace bpm
