// Covariance of each Gaussian kernel after deformation (Sec. 3.2,
// "Interaction Modeling"): every Gaussian is bound to an MPM particle and
// its covariance follows the particle's deformation gradient,
// Sigma_p(t) = F_p(t) Sigma_p F_p(t)^T.  F arrives as H = F - I (the MPM
// storage); with M = Sigma + H Sigma the result is M + M H^T, which keeps
// float32 resolution for F near the identity.  One thread per particle,
// structure-of-arrays loads and stores: an HBM-bound map of 84 bytes per
// particle (H 36, Sigma 24 in; Sigma(t) 24 out).
#include <hip/hip_runtime.h>

#include "dw_internal.h"

namespace dw {

// stored entry e of a symmetric 3x3 matrix: (xx, yy, zz, xy, xz, yz)
__device__ constexpr int S6A[6] = {0, 1, 2, 0, 0, 1};
__device__ constexpr int S6B[6] = {0, 1, 2, 1, 2, 2};
__device__ constexpr int S6IDX[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};

__global__ __launch_bounds__(256) void k_cov(int n, const float *__restrict__ H, const float *__restrict__ s0,
                                             float *__restrict__ s) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  float h[9], S[6];
#pragma unroll
  for (int q = 0; q < 9; ++q) h[q] = H[(int64_t)q * n + p];
#pragma unroll
  for (int e = 0; e < 6; ++e) S[e] = s0[(int64_t)e * n + p];
  // M = Sigma + H Sigma
  float M[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      float v = S[S6IDX[a][b]];
#pragma unroll
      for (int c = 0; c < 3; ++c) v += h[3 * a + c] * S[S6IDX[c][b]];
      M[3 * a + b] = v;
    }
  // Sigma(t)_ab = M_ab + sum_c M_ac H_bc
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int a = S6A[e], b = S6B[e];
    float v = M[3 * a + b];
#pragma unroll
    for (int c = 0; c < 3; ++c) v += M[3 * a + c] * h[3 * b + c];
    s[(int64_t)e * n + p] = v;
  }
}

// Reverse: with G the symmetric matrix of the stored-entry adjoint (G_aa =
// sb_aa, G_ab = G_ba = sb_ab / 2) the loss is tr(G Sigma(t)), so
// H_bar += 2 G F Sigma and Sigma_bar_ab += (F^T G F)_ab (twice for a != b:
// the stored off-diagonal entry stands for two matrix entries).
__global__ __launch_bounds__(256) void k_cov_adj(int n, const float *__restrict__ H, const float *__restrict__ s0,
                                                 const float *__restrict__ sb, float *__restrict__ Hb,
                                                 float *__restrict__ s0b) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  float F[9], S[6], G[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) F[q] = H[(int64_t)q * n + p] + ((q % 4) == 0 ? 1.f : 0.f);
#pragma unroll
  for (int e = 0; e < 6; ++e) S[e] = s0[(int64_t)e * n + p];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const float v = sb[(int64_t)S6IDX[a][b] * n + p];
      G[3 * a + b] = a == b ? v : 0.5f * v;
    }
  // GF = G F
  float GF[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      float v = 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) v += G[3 * a + c] * F[3 * c + b];
      GF[3 * a + b] = v;
    }
  if (Hb) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        float v = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) v += GF[3 * a + c] * S[S6IDX[c][b]];
        Hb[(int64_t)(3 * a + b) * n + p] += 2.f * v;
      }
  }
  if (s0b) {
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int a = S6A[e], b = S6B[e];
      float v = 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) v += F[3 * c + a] * GF[3 * c + b];
      s0b[(int64_t)e * n + p] += a == b ? v : 2.f * v;
    }
  }
}

}  // namespace dw

using namespace dw;

extern "C" int gaussian_covariance(int n, const float *H, const float *sigma0, float *sigma, void *stream) {
  DW_REQUIRE(n >= 0, DW_EINVAL, "gaussian_covariance: n must be >= 0");
  if (n == 0) return DW_OK;
  DW_REQUIRE(H && sigma0 && sigma, DW_EINVAL, "gaussian_covariance: NULL array");
  DW_REQUIRE(sigma != sigma0, DW_EINVAL, "gaussian_covariance: sigma must not alias sigma0");
  hipLaunchKernelGGL(k_cov, dim3(grid_blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, n, H, sigma0, sigma);
  return check_launch("gaussian_covariance");
}

extern "C" int gaussian_covariance_adj(int n, const float *H, const float *sigma0, const float *sigma_bar,
                                       float *H_bar, float *sigma0_bar, void *stream) {
  DW_REQUIRE(n >= 0, DW_EINVAL, "gaussian_covariance_adj: n must be >= 0");
  if (n == 0) return DW_OK;
  DW_REQUIRE(H && sigma0 && sigma_bar, DW_EINVAL, "gaussian_covariance_adj: NULL array");
  hipLaunchKernelGGL(k_cov_adj, dim3(grid_blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, n, H, sigma0,
                     sigma_bar, H_bar, sigma0_bar);
  return check_launch("gaussian_covariance_adj");
}
