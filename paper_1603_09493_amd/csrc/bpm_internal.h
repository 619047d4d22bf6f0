// Internal data model of the batched FE-LLG island solver (not part of the public ABI).
//
// A *mesh group* holds the geometry shared by its instances: P1 stiffness K and charge operator
// D on one CSR pattern, the transposed charge values DT on the same pattern, lumped node
// volumes, interface partners and areas, and the dense demag operator S.  An *instance* is one
// island simulation on a group (its own material, field schedule, position, seed).  A *system*
// is the unit that shares a clock: one instance, or several dipole-coupled instances.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/bpm_llg.h"

namespace bpm {

// Pointers loaded from memory (group views, launch parameters) are generic to the compiler; the
// hot loops cast them to the global address space so that they compile to global_load/store,
// which (unlike flat accesses) do not make every LDS wait also wait for outstanding HBM loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define GLB __attribute__((address_space(1)))
#define LDSP __attribute__((address_space(3)))
#else
#define GLB
#define LDSP
#endif
template <typename T>
__device__ __forceinline__ GLB T* glb(T* p) { return (GLB T*)p; }
template <typename T>
__device__ __forceinline__ const GLB T* glb(const T* p) { return (const GLB T*)p; }

constexpr int kCsrPad = 8;   // zero CSR entries stored past the last row of every device mesh

// Packed upper-triangle tiles of the FP32 demag operator: the NB (NB + 1) / 2 tiles of 64 x 64
// with I <= J (NB = ceil(n / 64)), in row-major order of (I, J), 4096 floats each, zero beyond n.
// Inside a tile, element (r, c) with r = 16 rg + t and c = 4 cq + q sits at
// ((4 t + rg) * 16 + cq) * 4 + q: the sixteen 16-byte words a lane (rg, cq) of a wave reads are
// one word of each of sixteen contiguous 1 KB blocks, one block per load instruction of the wave.
constexpr int kTile = 64;
__host__ __device__ inline long tile_count(int n) {
  const long nb = (n + kTile - 1) / kTile;
  return nb * (nb + 1) / 2;
}
__host__ __device__ inline long tile_index(int nb, int I, int J) {   // I <= J
  return (long)I * nb - (long)I * (I - 1) / 2 + (J - I);
}
__host__ __device__ inline int tile_offset(int r, int c) {
  return (((r & 15) * 4 + (r >> 4)) * 16 + (c >> 2)) * 4 + (c & 3);
}
// FP16 tiles (same tile order, 4096 halves each): element (r, c) with r = 16 rg + 2 u + v
// (u < 8, v < 2) and c = 4 cq + q sits at (((4 u + rg) * 16 + cq) * 8 + 4 v + q: each 16-byte word
// holds two rows of a lane's four columns, and the eight words of lane (rg, cq) are one word of
// each of eight contiguous 1 KB blocks.
__host__ __device__ inline int tile16_offset(int r, int c) {
  const int t = r & 15;
  return ((((t >> 1) * 4 + (r >> 4)) * 16 + (c >> 2)) * 8) + (t & 1) * 4 + (c & 3);
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4.0e-7 * kPi;          // T m / A
constexpr double kGammaE = 1.76085963023e11;   // rad / (s T)
constexpr double kBoltzmann = 1.380649e-23;    // J / K

constexpr int kMaxSysPerGroup = 64;   // adaptive-control state is replicated in LDS per group
constexpr int kMaxInstPerGroup = 64;
constexpr int kStringMaxImages = 64;   // images of one string (bpm_string_reparam)

// Kriging model of the optimiser, as the expected-improvement kernel reads it (device pointers).
constexpr int kMaxGpDim = 16;
struct GpArgs {
  int32_t n, d;
  double mu, sigma2, c, f_min;
  const double* X;       // [n][d]
  const double* theta;   // [d]
  const double* G;       // [n + 2][n]: L^-1 (zeros above the diagonal), alpha', w'
};

// Device pointers of the images of one string, in chain order (a kernel argument).
struct StringImages {
  const void* p[kStringMaxImages];
};
constexpr int kBlock = 256;           // threads per workgroup of the stepping kernels
constexpr int kTrajW = 9;             // trajectory sample width

// Host-side mesh group (geometry + device copies).
struct MeshGroup {
  int n = 0, ntet = 0, nnz = 0, nif = 0;
  std::vector<double> x, y, z;            // node coordinates
  std::vector<int32_t> tet, layer, iface;
  std::vector<int32_t> rowptr, col;       // CSR pattern: nodes sharing a tetrahedron
  std::vector<double> K, D, DT;           // stiffness, charge operator [nnz][3], transpose [nnz][3]
  std::vector<double> V, tetV;            // lumped node volumes, tet volumes
  std::vector<int32_t> partner;           // interface partner node or -1
  std::vector<double> aif;                // lumped interface area per node (0 off the interface)
  std::vector<int32_t> n2t_ptr, n2t;      // node -> tets
  double centroid[3] = {0, 0, 0};
  double vol_layer[2] = {0, 0};
  // device copies
  double* dS64 = nullptr;                 // [n][n]
  float* dS32 = nullptr;
  float* dS32t = nullptr;                 // FP32 upper-triangle 64x64 tiles, packed (see kTile)
  uint16_t* dS16t = nullptr;              // FP16 tiles of S * s16_scale (see tile16_offset)
  double s16_scale = 1.0;
  bool S_ready = false;
};

// Per-instance constants in the form the kernels use.
struct InstConst {
  double Ms[2];
  double cex[2];      // 2 A / Ms      (B_ex = -cex / V_i (K m)_i)
  double can[2];      // 2 K / Ms      (B_an = can (m.u) u)
  double axis[2][3];
  double cint[2];     // A_int / (delta Ms)   (B_int = cint a_i / V_i m_partner)
  double alpha, gp;   // damping and gamma/(1+alpha^2)
  double A[2], K[2], Jint;   // for energies
  // field
  int32_t fkind, pad_;
  double B_peak, dir[3], t_rise, v[3], x_off[3], L_grad, W_pole, B_ext[3];
  double off[3];      // island position offset
  // gridded field (BPM_FIELD_GRID): [3][nz][ny][nx] tesla, node (i, j, k) at gorig + gh (i, j, k)
  const float* grid;  // device copy (a host copy for host-side evaluation)
  double gorig[3], gh;
  int32_t gn[3], gpad_;
  double gpad2_;
  uint32_t key[2];    // Philox key (seed low, seed high)
  int32_t group, sys, local;   // mesh group, system, index within the group
  int32_t pad2_;
};

struct Instance {
  int32_t mesh = 0;
  InstConst c{};
  std::shared_ptr<const std::vector<float>> grid_host;   // host copy of a gridded field
  std::vector<double> m0;   // [3][n]; empty means every node starts along +z
  int32_t sys = -1;         // -1: own system
  bool coupled = false;
};

// Per-system outputs written by the kernels; a continued run starts from them (time, step size
// and growth cap of the controller, counters).
struct SysOut {
  int32_t status, pad_;
  double t_reached;
  int64_t n_accept, n_reject;
  double dt_min_used, dt_max_used, max_norm_dev;
  double dt_next, fac;        // next step size and its growth cap
  int64_t istep;              // accepted steps (fixed-step time grid index)
};

// Per-instance outputs (and the crossing state a continued run resumes).
struct InstOut {
  int32_t crossed, switched;
  double t_sw, mz_soft, mz_hard;
  int64_t n_traj;
  double prev_t, prev_v;      // last accepted time and hard-layer <m_z>
};

// Kernel view of one mesh group for a run.
template <typename real>
struct GroupView {
  int n, nnz, R, nsys;
  int ldS;                    // row stride of S (n rounded up to a multiple of 16)
  int wg0, G;                 // first workgroup, workgroups per group
  int inst0, sys0;            // first instance / system (contiguous)
  const int32_t* rowptr;
  const int32_t* col;
  const int32_t* colx;        // col | layer(col) << 16 (n <= 65535)
  const real* K;
  const real* D;              // [nnz][3]
  const real* DT;             // [nnz][3]
  const real* S;              // [n][ldS] row-major (may be null when St is given)
  const float* St;            // FP32 packed upper-triangle tiles (null if not kept)
  const uint16_t* St16;       // FP16 packed tiles of S * scale (used when St is null)
  float s16_inv;              // 1 / scale of St16
  const real* V;
  const int32_t* layer;
  const int32_t* partner;
  const real* aif;
  const double* x;            // coordinates in double (field evaluation)
  const double* y;
  const double* z;
  double cen[3];
  double Vsoft, Vhard;
  // state, per instance r at offset r * stride
  real* m;                    // [R][3][n]
  real* ys;                   // [R][3][n] stage input
  real* k;                    // [R][7][3][n]
  real* yex;                  // [R][3][n]
  real* b;                    // [R][ldS], zero beyond n
  real* u;                    // [R][ldS]
  unsigned long long* bar;    // group barrier counter
};

struct SysView {
  int32_t inst0, count, coupled, pad_;
};

struct RunParams {
  int32_t ngroups, ninst, nsys, integrator;
  double t_end, dt0, dt_fixed, rtol, atol, dt_min, temperature;
  int64_t max_steps;
  int32_t save_every, traj_cap;
  int32_t flags, resume;      // resume: continue from sys_out / inst_out and the stored m, k1
  const InstConst* inst;
  const SysView* sys;
  SysOut* sys_out;
  InstOut* inst_out;
  double* traj;               // [ninst][traj_cap][9]
  double* err_acc;            // [nsys][2]
  double* obs_acc;            // [ninst][2][6]: sum V mz soft, sum V mz hard, sum w m (3), max dev
  double* mom_acc;            // [ninst][2][3]
  const int2* wg_map;         // blockIdx -> (group, local wg)
};

// Dynamic LDS of one launch of the stepping kernel, in this order: instance constants
// [ic_slots], demag right-hand sides [bl_elems], CSR rows of the owned nodes (csr_cap entries,
// 0 = read from global memory), and the owned rows of S [s_rows][ldS] (0 = streamed).
struct LdsPlan {
  int32_t ic_slots;   // instance constants (the largest instance count of a group)
  int32_t bl_elems;   // reals of the staged right-hand sides (RB [x2 for the symmetric product] x ldS)
  int32_t csr_cap;    // CSR entries of the owned rows (0: CSR and node data read from global memory)
  int32_t own_cap;    // owned nodes (node data staged beside the CSR rows)
  int32_t s_rows;     // rows of S kept in LDS (0: S streamed from global memory)
  int32_t ldS;        // largest row stride of S in the launch
  int32_t dip_slots;  // instances of the dipole pair-geometry table (0: computed on the fly)
};

std::string hip_err_string(hipError_t e);

// assembly.cpp
int assemble_mesh(MeshGroup& g, std::string& err);
// demag.hip
int demag_assemble_device(MeshGroup& g, double beta, hipStream_t stream, std::string& err);

}  // namespace bpm
