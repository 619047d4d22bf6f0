// Stochastic Heun path: realization-fastest state layout [3][N][R] per mesh group.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bpm_internal.h"

namespace bpm {

template <typename real>
struct HeunGroup {
  int n, R, ldS, inst0;
  int ldR;       // row pitch of b and u (R rounded up to a multiple of 4; padding stays zero)
  int uniform;   // every realization has the same constants (only the Philox key differs)
  const uint2* keys;   // [R] Philox keys of the realizations
  const int32_t* rowptr;
  const int32_t* col;
  const int32_t* colx;   // col | layer(col) << 16
  const real* K;
  const real* D;
  const real* DT;
  const real* S;
  const real* V;
  const int32_t* layer;
  const int32_t* partner;
  const real* aif;
  const double* x;
  const double* y;
  const double* z;
  double Vsoft, Vhard;
  real* m;       // [3][N][R] state at the start of the step
  real* yt;      // predictor
  real* k1;
  real* mnext;   // state at the end of the step (the next step's m)
  real* b;       // [N][ldR]
  real* u;       // [N][ldR]
};

struct HeunParams {
  double dt;            // nominal step (t_n = n dt)
  double h;             // size of this step (dt, or the clipped last step)
  double temperature;
  unsigned long long* step;   // device step counter
};

// output tile edge of the demag product: FP32 matrix-core tiles are 128 x 128, FP64 tiles 64 x 64
template <typename real>
constexpr int heun_tile() { return sizeof(real) == 4 ? 128 : 64; }

template <typename real>
struct HeunLaunch {
  const HeunGroup<real>* groups;
  const int2* bmap;     // A/C blocks -> (group, block within group); padded to a multiple of 8 with group -1
  const int4* tmap;     // GEMM tiles -> (group, m0, n0); padded to a multiple of 8 with group -1
  const InstConst* inst;
  int nblk, ntile;
  HeunParams params;
  bool all_uniform;   // every group has uniform == 1
  bool all_wave;      // every group has R % 64 == 0
};

template <typename real>
hipError_t heun_step(const HeunLaunch<real>& L, hipStream_t s);
template <typename real>
hipError_t heun_observe_launch(const HeunLaunch<real>& L, int ngroups, int Rmax, double* out, hipStream_t s);

}  // namespace bpm
