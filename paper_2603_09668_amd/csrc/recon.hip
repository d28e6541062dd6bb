// Losses and metrics of the wind-force reconstruction (Sec. 3.3 - 3.4 and
// the appendix's evaluation of reconstructed wind force fields):
//  * the physics-informed loss L_phys = sum_i |d_i - (d_i . g_i) g_i|^2
//    with d_i, g_i the unit directions of the reconstructed force and of the
//    LBM velocity guide at wind-grid node i (nodes where either vector is zero
//    contribute nothing), and its gradient with respect to the force field;
//  * the position loss sum_p |x_p - x*_p|^2 that stands in for the
//    photometric loss on synthetic targets, and its gradient;
//  * CosSim and NMSE of unit force directions;
//  * the guide: the lattice velocity sampled at the wind-grid nodes.
// The physics-informed loss runs as one workgroup (the wind grid is small), so
// its sum has a fixed order; the other sums are reduced per block and added
// with one float atomic per block, so their last bits depend on the order the
// blocks finish in.
#include <hip/hip_runtime.h>

#include "dw_internal.h"
#include "dw_kernels.h"

namespace dw {

constexpr int RC_BLOCK = 256;

// block sum of up to three values; thread 0 adds them to out[0..k)
template <int K>
__device__ __forceinline__ void block_add(float (&v)[K], float *out) {
  __shared__ float s_part[RC_BLOCK / 64][K];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    if (lane == 0) s_part[wid][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < K) {
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < RC_BLOCK / 64; ++w) t += s_part[w][threadIdx.x];
    atomicAdd(&out[threadIdx.x], t);
  }
}

// one workgroup: thread t takes nodes t, t + RC_BLOCK, ... (fixed order)
__global__ __launch_bounds__(RC_BLOCK) void k_phys_loss(int n, const float *__restrict__ W,
                                                        const float *__restrict__ G, float weight,
                                                        float *__restrict__ loss, float *__restrict__ Wb) {
  float part[1] = {0.f};
  for (int i = threadIdx.x; i < n; i += RC_BLOCK) {
    const float w[3] = {W[i], W[n + i], W[2 * n + i]};
    const float g[3] = {G[i], G[n + i], G[2 * n + i]};
    const float wn = sqrtf(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    const float gn = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (wn > 0.f && gn > 0.f) {
      const float iw = 1.f / wn, ig = 1.f / gn;
      float d[3], e[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        d[a] = w[a] * iw;
        e[a] = g[a] * ig;
      }
      const float c = d[0] * e[0] + d[1] * e[1] + d[2] * e[2];
      float perp[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) perp[a] = d[a] - c * e[a];
      const float li = perp[0] * perp[0] + perp[1] * perp[1] + perp[2] * perp[2];
      part[0] += weight * li;
      // d L_i / d w = 2 (perp - (perp . d) d) / |w|
      if (Wb) {
        const float pd = perp[0] * d[0] + perp[1] * d[1] + perp[2] * d[2];
#pragma unroll
        for (int a = 0; a < 3; ++a) Wb[(int64_t)a * n + i] += weight * 2.f * (perp[a] - pd * d[a]) * iw;
      }
    }
  }
  if (loss) block_add<1>(part, loss);
}

__global__ __launch_bounds__(RC_BLOCK) void k_position_loss(int n, const float *__restrict__ x,
                                                            const float *__restrict__ xt, float *__restrict__ loss,
                                                            float *__restrict__ xb) {
  const int p = blockIdx.x * RC_BLOCK + threadIdx.x;
  float part[1] = {0.f};
  if (p < n) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float r = x[(int64_t)a * n + p] - xt[(int64_t)a * n + p];
      part[0] += r * r;
      if (xb) xb[(int64_t)a * n + p] = 2.f * r;
    }
  }
  if (loss) block_add<1>(part, loss);
}

__global__ __launch_bounds__(RC_BLOCK) void k_direction_metrics(int n, const float *__restrict__ A,
                                                                const float *__restrict__ B, float *__restrict__ out) {
  const int i = blockIdx.x * RC_BLOCK + threadIdx.x;
  float part[3] = {0.f, 0.f, 0.f};
  if (i < n) {
    const float a[3] = {A[i], A[n + i], A[2 * n + i]};
    const float b[3] = {B[i], B[n + i], B[2 * n + i]};
    const float an = sqrtf(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const float bn = sqrtf(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    if (an > 0.f && bn > 0.f) {
      float c = 0.f, s = 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float ua = a[k] / an, ub = b[k] / bn;
        c += ua * ub;
        s += (ua - ub) * (ua - ub);
      }
      part[0] = c;
      part[1] = s;
      part[2] = 1.f;
    }
  }
  block_add<3>(part, out);
}

__global__ __launch_bounds__(RC_BLOCK) void k_wind_guide(int nwx, int nwy, int nwz, float lox, float loy, float loz,
                                                         float hx, float hy, float hz, WindDev w,
                                                         float *__restrict__ guide) {
  const int64_t n = (int64_t)nwx * nwy * nwz;
  const int64_t i = (int64_t)blockIdx.x * RC_BLOCK + threadIdx.x;
  if (i >= n) return;
  const int ix = (int)(i % nwx), iy = (int)((i / nwx) % nwy), iz = (int)(i / ((int64_t)nwx * nwy));
  const float px = nwx > 1 ? lox + (hx - lox) * (float)ix / (float)(nwx - 1) : lox;
  const float py = nwy > 1 ? loy + (hy - loy) * (float)iy / (float)(nwy - 1) : loy;
  const float pz = nwz > 1 ? loz + (hz - loz) * (float)iz / (float)(nwz - 1) : loz;
  const float qx = (px - w.lox_l) * w.inv_ldx, qy = (py - w.loy_l) * w.inv_ldx, qz = (pz - w.loz_l) * w.inv_ldx;
  float ux = 0.f, uy = 0.f, uz = 0.f;
  if (qx >= 0.f && qy >= 0.f && qz >= 0.f && qx <= (float)(w.lnx - 1) && qy <= (float)(w.lny - 1) &&
      qz <= (float)(w.lnz - 1))
    trilinear3(w.u, w.lnx, w.lny, w.lnz, w.L, qx, qy, qz, ux, uy, uz);
  guide[i] = ux;
  guide[n + i] = uy;
  guide[2 * n + i] = uz;
}

}  // namespace dw

using namespace dw;

extern "C" int phys_loss(int n, const float *W, const float *guide, float weight, float *loss, float *W_bar,
                         void *stream) {
  DW_REQUIRE(n >= 0, DW_EINVAL, "phys_loss: n must be >= 0");
  if (n == 0) return DW_OK;
  DW_REQUIRE(W && guide, DW_EINVAL, "phys_loss: W / guide is NULL");
  DW_REQUIRE(loss || W_bar, DW_EINVAL, "phys_loss: nothing to compute");
  hipLaunchKernelGGL(k_phys_loss, dim3(1), dim3(RC_BLOCK), 0, (hipStream_t)stream, n, W,
                     guide, weight, loss, W_bar);
  return check_launch("phys_loss");
}

extern "C" int position_loss(int n, const float *x, const float *x_target, float *loss, float *x_bar,
                             void *stream) {
  DW_REQUIRE(n >= 0, DW_EINVAL, "position_loss: n must be >= 0");
  if (n == 0) return DW_OK;
  DW_REQUIRE(x && x_target, DW_EINVAL, "position_loss: x / x_target is NULL");
  hipLaunchKernelGGL(k_position_loss, dim3(grid_blocks(n, RC_BLOCK)), dim3(RC_BLOCK), 0, (hipStream_t)stream, n, x,
                     x_target, loss, x_bar);
  return check_launch("position_loss");
}

extern "C" int direction_metrics(int n, const float *F_ref, const float *F, float *out, void *stream) {
  DW_REQUIRE(n >= 0, DW_EINVAL, "direction_metrics: n must be >= 0");
  DW_REQUIRE(out, DW_EINVAL, "direction_metrics: out is NULL");
  if (n == 0) return DW_OK;
  DW_REQUIRE(F_ref && F, DW_EINVAL, "direction_metrics: NULL field");
  hipLaunchKernelGGL(k_direction_metrics, dim3(grid_blocks(n, RC_BLOCK)), dim3(RC_BLOCK), 0, (hipStream_t)stream, n,
                     F_ref, F, out);
  return check_launch("direction_metrics");
}

extern "C" int wind_guide(const dw_lattice *lat, const float *u, const int nw[3], const float lo[3],
                          const float hi[3], float *guide, void *stream) {
  DW_REQUIRE(lat && u && nw && lo && hi && guide, DW_EINVAL, "wind_guide: NULL argument");
  DW_REQUIRE(lat->nx >= 2 && lat->ny >= 2 && lat->nz >= 2 && lat->dx > 0.f, DW_EINVAL,
             "wind_guide: lattice must have >= 2 nodes per axis");
  DW_REQUIRE(nw[0] >= 1 && nw[1] >= 1 && nw[2] >= 1, DW_EINVAL, "wind_guide: nw must be >= 1");
  WindDev w{};
  w.mode = DW_WIND_LBM_DRAG;
  w.lnx = lat->nx;
  w.lny = lat->ny;
  w.lnz = lat->nz;
  w.lox_l = lat->origin[0];
  w.loy_l = lat->origin[1];
  w.loz_l = lat->origin[2];
  w.inv_ldx = 1.f / lat->dx;
  w.u = u;
  w.L = (int64_t)lat->nx * lat->ny * lat->nz;
  const int64_t n = (int64_t)nw[0] * nw[1] * nw[2];
  hipLaunchKernelGGL(k_wind_guide, dim3(grid_blocks(n, RC_BLOCK)), dim3(RC_BLOCK), 0, (hipStream_t)stream, nw[0],
                     nw[1], nw[2], lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], w, guide);
  return check_launch("wind_guide");
}
