// Wind force field -> MPM grid nodes (Sec. 3.2) and its transpose.
#include <hip/hip_runtime.h>

#include "dw_internal.h"
#include "dw_kernels.h"

namespace dw {

// launch shape: threads along x, one block row per (y, z) line
constexpr int WIND_BLOCK = 128;
static dim3 node_grid(const GridDev &g) {
  return dim3((unsigned)((g.nx + WIND_BLOCK - 1) / WIND_BLOCK), (unsigned)g.ny, (unsigned)g.nz);
}

__global__ __launch_bounds__(128) void k_wind_to_grid(GridDev g, WindDev w, float *__restrict__ acc, int64_t N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= g.nx) return;
  const int64_t node = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
  float ax, ay, az;
  wind_at_node(w, g, i, j, k, node, 0.f, 0.f, 0.f, ax, ay, az);
  acc[node] = ax;
  acc[N + node] = ay;
  acc[2 * N + node] = az;
}

// Transpose of the trilinear force-grid interpolation.  Every workgroup
// accumulates the whole (small) force-grid adjoint in LDS over a strided
// share of the nodes, then adds its non-zero entries to W_bar.
constexpr int WBAR_LDS_FLOATS = 3 * 4096;  // 48 KiB: force grids up to 16^3 nodes

__global__ __launch_bounds__(256) void k_force_grid_adj_lds(GridDev g, WindDev w, const float *__restrict__ abar,
                                                            int64_t N, float *__restrict__ Wbar) {
  __shared__ float s[WBAR_LDS_FLOATS];
  int64_t M = 3 * w.nw3;
  for (int64_t q = threadIdx.x; q < M; q += blockDim.x) s[q] = 0.f;
  __syncthreads();
  for (int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; node < N;
       node += (int64_t)gridDim.x * blockDim.x) {
    float bx = abar[node], by = abar[N + node], bz = abar[2 * N + node];
    if (bx == 0.f && by == 0.f && bz == 0.f) continue;
    int i = (int)(node % g.nx), j = (int)((node / g.nx) % g.ny), k = (int)(node / ((int64_t)g.nx * g.ny));
    float px = g.ox + g.dx * (float)i, py = g.oy + g.dx * (float)j, pz = g.oz + g.dx * (float)k;
    float qx = fminf(fmaxf((px - w.lox) * w.sx, 0.f), (float)(w.nwx - 1));
    float qy = fminf(fmaxf((py - w.loy) * w.sy, 0.f), (float)(w.nwy - 1));
    float qz = fminf(fmaxf((pz - w.loz) * w.sz, 0.f), (float)(w.nwz - 1));
    int ix, iy, iz;
    float tx, ty, tz;
    lin_axis(qx, w.nwx, ix, tx);
    lin_axis(qy, w.nwy, iy, ty);
    lin_axis(qz, w.nwz, iz, tz);
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dxo = 0; dxo < 2; ++dxo) {
          float wt = (dxo ? tx : 1.f - tx) * (dy ? ty : 1.f - ty) * (dz ? tz : 1.f - tz);
          int64_t idx = (ix + dxo) + (int64_t)w.nwx * ((iy + dy) + (int64_t)w.nwy * (iz + dz));
          atomicAdd(&s[idx], wt * bx);
          atomicAdd(&s[w.nw3 + idx], wt * by);
          atomicAdd(&s[2 * w.nw3 + idx], wt * bz);
        }
  }
  __syncthreads();
  for (int64_t q = threadIdx.x; q < M; q += blockDim.x)
    if (s[q] != 0.f) atomicAdd(&Wbar[q], s[q]);
}

__global__ __launch_bounds__(128) void k_force_grid_adj_global(GridDev g, WindDev w, const float *__restrict__ abar,
                                                               int64_t N, float *__restrict__ Wbar) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= g.nx) return;
  const int64_t node = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
  float bx = abar[node], by = abar[N + node], bz = abar[2 * N + node];
  if (bx == 0.f && by == 0.f && bz == 0.f) return;
  float px = g.ox + g.dx * (float)i, py = g.oy + g.dx * (float)j, pz = g.oz + g.dx * (float)k;
  float qx = fminf(fmaxf((px - w.lox) * w.sx, 0.f), (float)(w.nwx - 1));
  float qy = fminf(fmaxf((py - w.loy) * w.sy, 0.f), (float)(w.nwy - 1));
  float qz = fminf(fmaxf((pz - w.loz) * w.sz, 0.f), (float)(w.nwz - 1));
  int ix, iy, iz;
  float tx, ty, tz;
  lin_axis(qx, w.nwx, ix, tx);
  lin_axis(qy, w.nwy, iy, ty);
  lin_axis(qz, w.nwz, iz, tz);
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dxo = 0; dxo < 2; ++dxo) {
        float wt = (dxo ? tx : 1.f - tx) * (dy ? ty : 1.f - ty) * (dz ? tz : 1.f - tz);
        int64_t idx = (ix + dxo) + (int64_t)w.nwx * ((iy + dy) + (int64_t)w.nwy * (iz + dz));
        atomicAdd(&Wbar[idx], wt * bx);
        atomicAdd(&Wbar[w.nw3 + idx], wt * by);
        atomicAdd(&Wbar[2 * w.nw3 + idx], wt * bz);
      }
}

// Transpose of the drag mode: a = k |U| U, U = s * trilinear(u), so
// dL/dU = k (|U| abar + U (U . abar) / |U|) and u_bar gets s times its
// trilinear transpose.
// JAC = true: transpose of the absolute drag a = k |U| U,
// U = s * trilinear(u): dL/dU = k (|U| abar + U (U . abar) / |U|), then
// u_bar += s trilinear^T(dL/dU).  JAC = false: abar already is dL/dU (the
// relative drag, whose Jacobian the grid-update adjoint applies).
template <bool JAC>
__global__ __launch_bounds__(128) void k_drag_adj(GridDev g, WindDev w, const float *__restrict__ abar, int64_t N,
                                                  float *__restrict__ ubar) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= g.nx) return;
  const int64_t node = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
  float bx = abar[node], by = abar[N + node], bz = abar[2 * N + node];
  if (bx == 0.f && by == 0.f && bz == 0.f) return;
  float px = g.ox + g.dx * (float)i, py = g.oy + g.dx * (float)j, pz = g.oz + g.dx * (float)k;
  float qx = (px - w.lox_l) * w.inv_ldx, qy = (py - w.loy_l) * w.inv_ldx, qz = (pz - w.loz_l) * w.inv_ldx;
  if (!(qx >= 0.f && qy >= 0.f && qz >= 0.f && qx <= (float)(w.lnx - 1) && qy <= (float)(w.lny - 1) &&
        qz <= (float)(w.lnz - 1)))
    return;
  float ux, uy, uz;
  trilinear3(w.u, w.lnx, w.lny, w.lnz, w.L, qx, qy, qz, ux, uy, uz);
  ux *= w.vel_scale;
  uy *= w.vel_scale;
  uz *= w.vel_scale;
  float Ux, Uy, Uz;
  if (JAC) {
    float sp = sqrtf(ux * ux + uy * uy + uz * uz);
    if (!(sp > 0.f)) return;
    float ub = (ux * bx + uy * by + uz * bz) / sp;
    Ux = w.k_drag * (sp * bx + ux * ub) * w.vel_scale;
    Uy = w.k_drag * (sp * by + uy * ub) * w.vel_scale;
    Uz = w.k_drag * (sp * bz + uz * ub) * w.vel_scale;
  } else {
    Ux = bx * w.vel_scale;
    Uy = by * w.vel_scale;
    Uz = bz * w.vel_scale;
  }
  int ix, iy, iz;
  float tx, ty, tz;
  lin_axis(qx, w.lnx, ix, tx);
  lin_axis(qy, w.lny, iy, ty);
  lin_axis(qz, w.lnz, iz, tz);
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dxo = 0; dxo < 2; ++dxo) {
        float wt = (dxo ? tx : 1.f - tx) * (dy ? ty : 1.f - ty) * (dz ? tz : 1.f - tz);
        int64_t idx = (ix + dxo) + (int64_t)w.lnx * ((iy + dy) + (int64_t)w.lny * (iz + dz));
        atomicAdd(&ubar[idx], wt * Ux);
        atomicAdd(&ubar[w.L + idx], wt * Uy);
        atomicAdd(&ubar[2 * w.L + idx], wt * Uz);
      }
}

}  // namespace dw

using namespace dw;

extern "C" int wind_to_grid(const dw_grid *grid, const dw_wind *wind, float *acc, void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  DW_REQUIRE(acc, DW_EINVAL, "wind_to_grid: acc is NULL");
  WindDev wd;
  rc = make_wind(wind, grid, &wd);
  if (rc) return rc;
  DW_REQUIRE(wd.mode != DW_WIND_ACC || wd.acc != acc, DW_EINVAL, "wind_to_grid: acc aliases the input");
  DW_REQUIRE(wd.mode != DW_WIND_LBM_DRAG_REL, DW_EINVAL,
             "wind_to_grid: the relative drag needs the node velocity (mpm_grid_update evaluates it)");
  GridDev g = make_grid(grid);
  int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;
  hipLaunchKernelGGL(k_wind_to_grid, node_grid(g), dim3(WIND_BLOCK), 0, (hipStream_t)stream, g, wd, acc, N);
  return check_launch("wind_to_grid");
}

extern "C" int wind_to_grid_adj(const dw_grid *grid, const dw_wind *wind, const float *acc_bar, float *out_bar,
                                void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  DW_REQUIRE(acc_bar && out_bar, DW_EINVAL, "wind_to_grid_adj: acc_bar / out_bar is NULL");
  WindDev wd;
  rc = make_wind(wind, grid, &wd);
  if (rc) return rc;
  DW_REQUIRE(wd.mode == DW_WIND_FORCE_GRID || wd.mode == DW_WIND_LBM_DRAG || wd.mode == DW_WIND_LBM_DRAG_REL,
             DW_EINVAL, "wind_to_grid_adj: mode must be FORCE_GRID, LBM_DRAG or LBM_DRAG_REL");
  GridDev g = make_grid(grid);
  int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;
  hipStream_t s = (hipStream_t)stream;
  if (wd.mode == DW_WIND_FORCE_GRID) {
    if (3 * wd.nw3 <= WBAR_LDS_FLOATS) {
      unsigned blocks = grid_blocks(N, 256);
      if (blocks > 512) blocks = 512;
      hipLaunchKernelGGL(k_force_grid_adj_lds, dim3(blocks), dim3(256), 0, s, g, wd, acc_bar, N, out_bar);
    } else {
      hipLaunchKernelGGL(k_force_grid_adj_global, node_grid(g), dim3(WIND_BLOCK), 0, s, g, wd, acc_bar, N, out_bar);
    }
  } else if (wd.mode == DW_WIND_LBM_DRAG) {
    hipLaunchKernelGGL(k_drag_adj<true>, node_grid(g), dim3(WIND_BLOCK), 0, s, g, wd, acc_bar, N, out_bar);
  } else {
    hipLaunchKernelGGL(k_drag_adj<false>, node_grid(g), dim3(WIND_BLOCK), 0, s, g, wd, acc_bar, N, out_bar);
  }
  return check_launch("wind_to_grid_adj");
}
