// Stochastic Heun path: realization-fastest state layout [3][N][R] per mesh group.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bpm_internal.h"

namespace bpm {

template <typename real>
struct HeunGroup {
  int n, R, ldS, inst0;
  const int32_t* rowptr;
  const int32_t* col;
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
  double Vsoft, Vhard;
  real* m;       // [3][N][R]
  real* yt;      // predictor
  real* k1;
  real* mnext;
  real* yex;
  real* b;       // [N][R]
  real* u;       // [N][R]
};

struct HeunParams {
  double dt;            // nominal step (t_n = n dt)
  double h;             // size of this step (dt, or the clipped last step)
  double temperature;
  unsigned long long* step;   // device step counter
};

template <typename real>
struct HeunLaunch {
  const HeunGroup<real>* groups;
  const int2* bmap;     // A/C/commit blocks -> (group, block within group)
  const int4* tmap;     // GEMM tiles -> (group, m0, n0)
  const InstConst* inst;
  int nblk, ntile;
  HeunParams params;
};

template <typename real>
hipError_t heun_step(const HeunLaunch<real>& L, hipStream_t s);
template <typename real>
hipError_t heun_observe_launch(const HeunLaunch<real>& L, int ngroups, int Rmax, double* out, hipStream_t s);

}  // namespace bpm
