// Applied field of an instance, shared by the stepping kernels, the thermal kernels and the host.
//
// The recording simulation moves a precomputed head field down-track over the bit and scales it
// with a 0.1 ns rise, and adds a global field H_ext (Sec. II.A, Sec. II.C):
//   B(x, t) = B_peak r(t) f(x - x_off - v t) + B_ext,  r(t) = min(t / t_rise, 1),
// with f = dir for BPM_FIELD_UNIFORM, dir times a tanh pole profile for BPM_FIELD_POLE, and the
// trilinear interpolation of a field grid (tesla vectors; zero outside the grid) for
// BPM_FIELD_GRID -- the form in which the paper hands the head field to the recording stage.
#pragma once
#include "bpm_internal.h"

namespace bpm {

__host__ __device__ inline double field_rise(const InstConst& c, double t) {
  if (!(c.t_rise > 0.0)) return 1.0;
  const double r = t / c.t_rise;
  return r < 1.0 ? r : 1.0;
}

// Trilinear interpolation of the grid at the field-frame position p (metres); zero outside the
// box spanned by the grid nodes.
__host__ __device__ inline void grid_sample(const InstConst& c, double px, double py, double pz, double& gx,
                                            double& gy, double& gz) {
  gx = gy = gz = 0.0;
  const double u[3] = {(px - c.gorig[0]) / c.gh, (py - c.gorig[1]) / c.gh, (pz - c.gorig[2]) / c.gh};
  int i0[3];
  double w[3];
  for (int d = 0; d < 3; ++d) {
    if (!(u[d] >= 0.0) || u[d] > (double)(c.gn[d] - 1)) return;
    int q = (int)floor(u[d]);
    if (q > c.gn[d] - 2) q = c.gn[d] - 2;       // the last node: the last cell with weight 1
    i0[d] = q;
    w[d] = u[d] - (double)q;
  }
  const long nx = c.gn[0], ny = c.gn[1], nz = c.gn[2];
  const long plane = nx * ny * nz;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const double wt = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) * (dz ? w[2] : 1.0 - w[2]);
        const long idx = ((long)(i0[2] + dz) * ny + (i0[1] + dy)) * nx + (i0[0] + dx);
        gx += wt * (double)c.grid[idx];
        gy += wt * (double)c.grid[plane + idx];
        gz += wt * (double)c.grid[2 * plane + idx];
      }
}

// Applied field (tesla) at world position (x, y, z) and time t.
__host__ __device__ inline void applied_field_at(const InstConst& c, double t, double x, double y, double z,
                                                 double& bx, double& by, double& bz) {
  const double amp = c.B_peak * field_rise(c, t);
  double fx = c.dir[0], fy = c.dir[1], fz = c.dir[2];
  if (c.fkind == BPM_FIELD_POLE) {
    const double sx = x - c.x_off[0] - c.v[0] * t;
    const double sy = y - c.x_off[1] - c.v[1] * t;
    const double prof = 0.5 * (1.0 - tanh(sx / c.L_grad)) * 0.5 *
                        (tanh((sy + 0.5 * c.W_pole) / c.L_grad) - tanh((sy - 0.5 * c.W_pole) / c.L_grad));
    fx *= prof; fy *= prof; fz *= prof;
  } else if (c.fkind == BPM_FIELD_GRID) {
    grid_sample(c, x - c.x_off[0] - c.v[0] * t, y - c.x_off[1] - c.v[1] * t, z - c.x_off[2] - c.v[2] * t, fx, fy, fz);
  }
  bx = amp * fx + c.B_ext[0];
  by = amp * fy + c.B_ext[1];
  bz = amp * fz + c.B_ext[2];
}

}  // namespace bpm
