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

// ------------------------------------------------- deterministic transposes
// With dw_wind.deterministic the transposes gather instead of scattering:
// every wind-grid (or lattice) node sums, in a fixed node order, the weighted
// adjoints of the MPM nodes whose interpolation cell has it as a corner, with
// the forward's own weights.  No atomics: the result is bit-reproducible.

// Weight of coarse node jc (along one axis) in the interpolation of
// coordinate q on an axis of n coarse nodes, exactly as lin_axis splits it.
__device__ __forceinline__ float corner_weight(float q, int n, int jc) {
  int i0;
  float t;
  lin_axis(q, n, i0, t);
  return i0 == jc ? 1.f - t : (i0 + 1 == jc ? t : 0.f);
}

// MPM node range [a, b] on one axis whose coordinate q = (o + dx i - lo) s
// can reach coarse node jc, with a margin of one node for rounding; a
// clamped coordinate (outside [0, n - 1]) belongs to the end node.
__device__ __forceinline__ void gather_range(int jc, int n, float o, float dx, float lo, float s, int m, bool clamped,
                                             int &a, int &b) {
  const float x0 = lo + (float)(jc - 1) / s, x1 = lo + (float)(jc + 1) / s;
  a = (int)floorf((x0 - o) / dx) - 1;
  b = (int)ceilf((x1 - o) / dx) + 1;
  if (clamped && jc == 0) a = 0;
  if (clamped && jc == n - 1) b = m - 1;
  a = max(a, 0);
  b = min(b, m - 1);
}

__global__ __launch_bounds__(128) void k_force_grid_adj_gather(GridDev g, WindDev w, const float *__restrict__ abar,
                                                               int64_t N, float *__restrict__ Wbar) {
  const int64_t jn = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (jn >= w.nw3) return;
  const int jx = (int)(jn % w.nwx), jy = (int)((jn / w.nwx) % w.nwy), jz = (int)(jn / ((int64_t)w.nwx * w.nwy));
  int ax, bx, ay, by, az, bz;
  gather_range(jx, w.nwx, g.ox, g.dx, w.lox, w.sx, g.nx, true, ax, bx);
  gather_range(jy, w.nwy, g.oy, g.dx, w.loy, w.sy, g.ny, true, ay, by);
  gather_range(jz, w.nwz, g.oz, g.dx, w.loz, w.sz, g.nz, true, az, bz);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f;
  for (int k = az; k <= bz; ++k) {
    const float pz = g.oz + g.dx * (float)k;
    const float wz = corner_weight(fminf(fmaxf((pz - w.loz) * w.sz, 0.f), (float)(w.nwz - 1)), w.nwz, jz);
    if (wz == 0.f) continue;
    for (int j = ay; j <= by; ++j) {
      const float py = g.oy + g.dx * (float)j;
      const float wy = corner_weight(fminf(fmaxf((py - w.loy) * w.sy, 0.f), (float)(w.nwy - 1)), w.nwy, jy);
      if (wy == 0.f) continue;
      for (int i = ax; i <= bx; ++i) {
        const float px = g.ox + g.dx * (float)i;
        const float wx = corner_weight(fminf(fmaxf((px - w.lox) * w.sx, 0.f), (float)(w.nwx - 1)), w.nwx, jx);
        const float wt = wx * wy * wz;
        const int64_t node = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
        s0 += wt * abar[node];
        s1 += wt * abar[N + node];
        s2 += wt * abar[2 * N + node];
      }
    }
  }
  Wbar[jn] += s0;
  Wbar[w.nw3 + jn] += s1;
  Wbar[2 * w.nw3 + jn] += s2;
}

// drag transpose as a gather over the lattice nodes; the per-MPM-node value
// (dL/dU, JAC as in k_drag_adj) is recomputed by every lattice node it feeds
template <bool JAC>
__global__ __launch_bounds__(128) void k_drag_adj_gather(GridDev g, WindDev w, const float *__restrict__ abar,
                                                         int64_t N, float *__restrict__ ubar) {
  const int64_t ln = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ln >= w.L) return;
  const int jx = (int)(ln % w.lnx), jy = (int)((ln / w.lnx) % w.lny), jz = (int)(ln / ((int64_t)w.lnx * w.lny));
  int ax, bx, ay, by, az, bz;
  const float s = w.inv_ldx;
  gather_range(jx, w.lnx, g.ox, g.dx, w.lox_l, s, g.nx, false, ax, bx);
  gather_range(jy, w.lny, g.oy, g.dx, w.loy_l, s, g.ny, false, ay, by);
  gather_range(jz, w.lnz, g.oz, g.dx, w.loz_l, s, g.nz, false, az, bz);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f;
  for (int k = az; k <= bz; ++k)
    for (int j = ay; j <= by; ++j)
      for (int i = ax; i <= bx; ++i) {
        const int64_t node = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
        const float bxv = abar[node], byv = abar[N + node], bzv = abar[2 * N + node];
        if (bxv == 0.f && byv == 0.f && bzv == 0.f) continue;
        const float px = g.ox + g.dx * (float)i, py = g.oy + g.dx * (float)j, pz = g.oz + g.dx * (float)k;
        const float qx = (px - w.lox_l) * w.inv_ldx, qy = (py - w.loy_l) * w.inv_ldx, qz = (pz - w.loz_l) * w.inv_ldx;
        if (!(qx >= 0.f && qy >= 0.f && qz >= 0.f && qx <= (float)(w.lnx - 1) && qy <= (float)(w.lny - 1) &&
              qz <= (float)(w.lnz - 1)))
          continue;
        const float wt = corner_weight(qx, w.lnx, jx) * corner_weight(qy, w.lny, jy) * corner_weight(qz, w.lnz, jz);
        if (wt == 0.f) continue;
        float Ux, Uy, Uz;
        if (JAC) {
          float ux, uy, uz;
          trilinear3(w.u, w.lnx, w.lny, w.lnz, w.L, qx, qy, qz, ux, uy, uz);
          ux *= w.vel_scale;
          uy *= w.vel_scale;
          uz *= w.vel_scale;
          const float sp = sqrtf(ux * ux + uy * uy + uz * uz);
          if (!(sp > 0.f)) continue;
          const float ub = (ux * bxv + uy * byv + uz * bzv) / sp;
          Ux = w.k_drag * (sp * bxv + ux * ub) * w.vel_scale;
          Uy = w.k_drag * (sp * byv + uy * ub) * w.vel_scale;
          Uz = w.k_drag * (sp * bzv + uz * ub) * w.vel_scale;
        } else {
          Ux = bxv * w.vel_scale;
          Uy = byv * w.vel_scale;
          Uz = bzv * w.vel_scale;
        }
        s0 += wt * Ux;
        s1 += wt * Uy;
        s2 += wt * Uz;
      }
  ubar[ln] += s0;
  ubar[w.L + ln] += s1;
  ubar[2 * w.L + ln] += s2;
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
  if (wind->deterministic) {
    if (wd.mode == DW_WIND_FORCE_GRID)
      hipLaunchKernelGGL(k_force_grid_adj_gather, dim3(grid_blocks(wd.nw3, 128)), dim3(128), 0, s, g, wd, acc_bar, N,
                         out_bar);
    else if (wd.mode == DW_WIND_LBM_DRAG)
      hipLaunchKernelGGL(k_drag_adj_gather<true>, dim3(grid_blocks(wd.L, 128)), dim3(128), 0, s, g, wd, acc_bar, N,
                         out_bar);
    else
      hipLaunchKernelGGL(k_drag_adj_gather<false>, dim3(grid_blocks(wd.L, 128)), dim3(128), 0, s, g, wd, acc_bar, N,
                         out_bar);
  } else if (wd.mode == DW_WIND_FORCE_GRID) {
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
