// Device-side wind evaluation shared by the grid update, its adjoint and
// wind_to_grid: the force property of the wind grid field acting on MPM grid
// nodes (Sec. 3.2) and the drag relation of Sec. 3.4.
#pragma once

#include "dw_internal.h"

namespace dw {

struct WindDev {
  int mode;
  // force grid
  int nwx, nwy, nwz;
  float lox, loy, loz, sx, sy, sz;  // q = (pos - lo) * s, s = (nw - 1) / (hi - lo)
  const float *W;
  int64_t nw3;
  // LBM drag
  int lnx, lny, lnz;
  float lox_l, loy_l, loz_l, inv_ldx;
  const float *u;
  int64_t L;
  float vel_scale, k_drag;
  // precomputed acceleration
  const float *acc;
  int64_t N;
};

int make_wind(const dw_wind *w, const dw_grid *g, WindDev *out);

// Linear-interpolation cell along one axis for coordinate q in [0, n-1].
__device__ __forceinline__ void lin_axis(float q, int n, int &i0, float &t) {
  float fl = floorf(q);
  int i = (int)fl;
  if (i > n - 2) i = n - 2;
  if (i < 0) i = 0;
  i0 = i;
  t = q - (float)i;
}

// Trilinear interpolation of a [3][nx*ny*nz] field at fractional node
// coordinates (qx, qy, qz) already clamped into the box.
__device__ __forceinline__ void trilinear3(const float *__restrict__ f, int nx, int ny, int nz, int64_t L,
                                           float qx, float qy, float qz, float &ax, float &ay, float &az) {
  int ix, iy, iz;
  float tx, ty, tz;
  lin_axis(qx, nx, ix, tx);
  lin_axis(qy, ny, iy, ty);
  lin_axis(qz, nz, iz, tz);
  ax = ay = az = 0.f;
#pragma unroll
  for (int dz = 0; dz < 2; ++dz) {
    float wz = dz ? tz : 1.f - tz;
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      float wy = dy ? ty : 1.f - ty;
#pragma unroll
      for (int dxo = 0; dxo < 2; ++dxo) {
        float wx = dxo ? tx : 1.f - tx;
        float w = wx * wy * wz;
        int64_t idx = (ix + dxo) + (int64_t)nx * ((iy + dy) + (int64_t)ny * (iz + dz));
        ax += w * f[idx];
        ay += w * f[L + idx];
        az += w * f[2 * L + idx];
      }
    }
  }
}

// Interpolated wind velocity U at MPM node (i, j, k) in physical units, for
// the LBM drag modes; false outside the lattice box (no wind there).
__device__ __forceinline__ bool wind_velocity_at_node(const WindDev &w, const GridDev &g, int i, int j, int k,
                                                      float &ux, float &uy, float &uz) {
  float px = g.ox + g.dx * (float)i, py = g.oy + g.dx * (float)j, pz = g.oz + g.dx * (float)k;
  float qx = (px - w.lox_l) * w.inv_ldx, qy = (py - w.loy_l) * w.inv_ldx, qz = (pz - w.loz_l) * w.inv_ldx;
  ux = uy = uz = 0.f;
  if (!(qx >= 0.f && qy >= 0.f && qz >= 0.f && qx <= (float)(w.lnx - 1) && qy <= (float)(w.lny - 1) &&
        qz <= (float)(w.lnz - 1)))
    return false;
  trilinear3(w.u, w.lnx, w.lny, w.lnz, w.L, qx, qy, qz, ux, uy, uz);
  ux *= w.vel_scale;
  uy *= w.vel_scale;
  uz *= w.vel_scale;
  return true;
}

// Wind acceleration at MPM node (i, j, k); (vx, vy, vz) is the node's own
// velocity mv / m, used by the relative drag only.
__device__ __forceinline__ void wind_at_node(const WindDev &w, const GridDev &g, int i, int j, int k,
                                             int64_t node, float vx, float vy, float vz, float &ax, float &ay,
                                             float &az) {
  ax = ay = az = 0.f;
  if (w.mode == DW_WIND_NONE) return;
  if (w.mode == DW_WIND_ACC) {
    ax = w.acc[node];
    ay = w.acc[w.N + node];
    az = w.acc[2 * w.N + node];
    return;
  }
  float px = g.ox + g.dx * (float)i, py = g.oy + g.dx * (float)j, pz = g.oz + g.dx * (float)k;
  if (w.mode == DW_WIND_FORCE_GRID) {
    float qx = fminf(fmaxf((px - w.lox) * w.sx, 0.f), (float)(w.nwx - 1));
    float qy = fminf(fmaxf((py - w.loy) * w.sy, 0.f), (float)(w.nwy - 1));
    float qz = fminf(fmaxf((pz - w.loz) * w.sz, 0.f), (float)(w.nwz - 1));
    trilinear3(w.W, w.nwx, w.nwy, w.nwz, w.nw3, qx, qy, qz, ax, ay, az);
    return;
  }
  // DW_WIND_LBM_DRAG / DW_WIND_LBM_DRAG_REL
  float ux, uy, uz;
  if (!wind_velocity_at_node(w, g, i, j, k, ux, uy, uz)) return;
  if (w.mode == DW_WIND_LBM_DRAG_REL) {
    ux -= vx;
    uy -= vy;
    uz -= vz;
  }
  float s = sqrtf(ux * ux + uy * uy + uz * uz);
  ax = w.k_drag * s * ux;
  ay = w.k_drag * s * uy;
  az = w.k_drag * s * uz;
}

}  // namespace dw
