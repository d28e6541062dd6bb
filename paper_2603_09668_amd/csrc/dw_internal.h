// Internal helpers shared by the libdiffwind kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/diffwind.h"

namespace dw {

// ------------------------------------------------------------ host errors
int set_error(int code, const char *fmt, ...);
int check_launch(const char *what);

#define DW_REQUIRE(cond, code, ...)                 \
  do {                                              \
    if (!(cond)) return ::dw::set_error(code, __VA_ARGS__); \
  } while (0)

// -------------------------------------------------------------- geometry
constexpr int TILE = 4;  // cell / node tiles are 4x4x4

struct GridDev {
  int nx, ny, nz;
  int tx, ty, tz;  // tiles per axis
  float dx, inv_dx;
  float ox, oy, oz;
};

inline GridDev make_grid(const dw_grid *g) {
  GridDev d;
  d.nx = g->nx; d.ny = g->ny; d.nz = g->nz;
  d.tx = (g->nx + TILE - 1) / TILE;
  d.ty = (g->ny + TILE - 1) / TILE;
  d.tz = (g->nz + TILE - 1) / TILE;
  d.dx = g->dx;
  d.inv_dx = 1.0f / g->dx;
  d.ox = g->origin[0]; d.oy = g->origin[1]; d.oz = g->origin[2];
  return d;
}

// Workspace layout (bytes, all 256-aligned):
//   [0, 256)            header: int32 status, scan totals, P2G tickets
//   tile_count  [T]     int32   particles per cell tile
//   node_flag   [T]     int32   node tile touched by a stencil
//   tile_start  [T+1]   int32
//   cell_tiles  [T]     int32   active cell tiles (tile index)
//   node_tiles  [T]     int32   active node tiles
//   block_sums  [4*NB]  int32   scan partials
//   key, rank, perm, perm_tmp [n] int32
//   item_tile, item_begin [max items], item_first [T], item_part (deterministic)
struct Workspace {
  int32_t *status;
  int32_t *n_cell_tiles;
  int32_t *n_node_tiles;
  int32_t *tile_count;
  int32_t *tile_start;
  int32_t *node_flag;
  int32_t *cell_tiles;
  int32_t *node_tiles;
  int32_t *block_sums;
  int32_t *key;
  int32_t *rank;  // position of each particle inside its tile's range
  int32_t *perm;
  int32_t *perm_tmp;
  int32_t *n_items;     // work items: chunks of <= WORK_CHUNK particles of one cell tile
  int32_t *item_tile;
  int32_t *item_begin;
  int32_t *item_first;  // first work item of each cell tile
  float *item_part;     // deterministic mode: 6^3 x 4 partial node block per work item
  int64_t item_part_floats;
  int64_t n_tiles;
  int64_t n_scan_blocks;
  size_t bytes;
};

constexpr int SCAN_BLOCK = 512;
constexpr int WORK_CHUNK = 512;  // particles per scatter work item

size_t workspace_layout(const dw_grid *g, int n_max, Workspace *ws, void *base, int deterministic = 0);
int check_grid(const dw_grid *g);
int check_particles(const dw_particles *p, bool need_state);
// binds the workspace and checks its size
int bind_workspace(const dw_grid *g, int n, const void *ws, size_t ws_bytes, Workspace *W, int deterministic = 0);

// fill kernels (a kernel rather than hipMemsetAsync, so the calls stay
// capturable in HIP graphs); static: every translation unit launches its own
// k_fill_i32 writes 16 bytes per store over the 16-byte aligned body of the
// range and single words at its ends (launch it for count / 4 + 1 threads)
static __global__ void k_fill_i32(int32_t *p, int64_t count, int32_t value) {
  const int64_t head = min((int64_t)(((16 - ((uintptr_t)p & 15)) & 15) / 4), count);
  const int64_t body = (count - head) / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  int4 *q = reinterpret_cast<int4 *>(p + head);
  for (int64_t i = t; i < body; i += stride) q[i] = make_int4(value, value, value, value);
  const int64_t tail0 = head + body * 4;
  if (t < head) p[t] = value;
  if (t < count - tail0) p[tail0 + t] = value;
}

static __global__ void k_fill_f32(float *p, int64_t count, float value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}
inline unsigned grid_blocks(int64_t work, int block) {
  int64_t b = (work + block - 1) / block;
  return (unsigned)(b < 1 ? 1 : b);
}

// ---------------------------------------------------- device math helpers
__device__ __forceinline__ float det3(const float *m) {
  return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
         m[2] * (m[3] * m[7] - m[4] * m[6]);
}

// inverse-transpose (cofactor / det)
__device__ __forceinline__ void inv_transpose3(const float *m, float det, float *out) {
  float id = 1.0f / det;
  out[0] = (m[4] * m[8] - m[5] * m[7]) * id;
  out[1] = -(m[3] * m[8] - m[5] * m[6]) * id;
  out[2] = (m[3] * m[7] - m[4] * m[6]) * id;
  out[3] = -(m[1] * m[8] - m[2] * m[7]) * id;
  out[4] = (m[0] * m[8] - m[2] * m[6]) * id;
  out[5] = -(m[0] * m[7] - m[1] * m[6]) * id;
  out[6] = (m[1] * m[5] - m[2] * m[4]) * id;
  out[7] = -(m[0] * m[5] - m[2] * m[3]) * id;
  out[8] = (m[0] * m[4] - m[1] * m[3]) * id;
}

__device__ __forceinline__ void matmul3(const float *a, const float *b, float *c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

// c = a * b^T
__device__ __forceinline__ void matmul3_abt(const float *a, const float *b, float *c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[3 * i] * b[3 * j] + a[3 * i + 1] * b[3 * j + 1] + a[3 * i + 2] * b[3 * j + 2];
}

// c = a^T * b
__device__ __forceinline__ void matmul3_atb(const float *a, const float *b, float *c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[i] * b[j] + a[3 + i] * b[3 + j] + a[6 + i] * b[6 + j];
}

__device__ __forceinline__ void lame(float E, float nu, float &mu, float &lam) {
  mu = E / (2.0f * (1.0f + nu));
  lam = E * nu / ((1.0f + nu) * (1.0f - 2.0f * nu));
}

// Sum of the principal 2x2 minors of a 3x3 matrix.
__device__ __forceinline__ float minors2(const float *m) {
  return m[0] * m[4] - m[1] * m[3] + m[0] * m[8] - m[2] * m[6] + m[4] * m[8] - m[5] * m[7];
}

// det(I + H) - 1 = tr H + minors2(H) + det H, free of cancellation for small H.
__device__ __forceinline__ float det_shift(const float *H) {
  return H[0] + H[4] + H[8] + minors2(H) + det3(H);
}

// Rotation factor of the polar decomposition F = R S, F = I + H, returned as
// Y = R - I, with every step written for the deviation Y = X - I so that no
// step subtracts two numbers close to 1 and the strain F - R = H - Y keeps
// float32 relative precision for small strains.  H = 0 gives Y = 0 exactly.
// Stretches near 1 (|F^T F - I|_F < 1/2): Newton-Schulz iteration
//   X <- X (3 I - X^T X) / 2, i.e. S = X^T X - I = Y + Y^T + Y^T Y,
//   Y <- Y - (S + Y S) / 2,
// quadratically convergent there and free of divisions.  Otherwise (or if it
// has not converged in 6 steps) the scaled Newton iteration
// X <- (zeta X + X^{-T} / zeta) / 2 (Higham 1986) continues, with
//   (I + Y)^{-1} - I = (Y^2 - (1 + tr Y) Y - det(Y) I) / det(I + Y)
// (Cayley-Hamilton).  Both stop once a step is below 1e-6 of |Y| + |H|: the
// error left is then of order 1e-12, under float32 round-off.
__device__ __forceinline__ void polar_shift(const float *H, float *Y) {
  float hh = 0.f;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    Y[i] = H[i];
    hh += H[i] * H[i];
  }
  {
    float S[9], s2 = 0.f;
    matmul3_atb(Y, Y, S);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) S[3 * i + j] += Y[3 * i + j] + Y[3 * j + i];
#pragma unroll
    for (int i = 0; i < 9; ++i) s2 += S[i] * S[i];
    if (s2 < 0.25f) {
      for (int it = 0; it < 6; ++it) {
        float YS[9];
        matmul3(Y, S, YS);
        float delta = 0.f, yy = 0.f;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          float e = 0.5f * (S[i] + YS[i]);
          Y[i] -= e;
          delta += e * e;
          yy += Y[i] * Y[i];
        }
        if (delta <= 1e-12f * (yy + hh)) return;
        matmul3_atb(Y, Y, S);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) S[3 * i + j] += Y[3 * i + j] + Y[3 * j + i];
      }
    }
  }
  for (int it = 0; it < 16; ++it) {
    float t = Y[0] + Y[4] + Y[8];
    float Y2[9];
    matmul3(Y, Y, Y2);
    float dY = det3(Y);
    float dA = 1.0f + t + minors2(Y) + dY;  // det(I + Y)
    float id = 1.0f / dA;
    // Z = (I + Y)^{-T} - I
    float Z[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        float v = Y2[3 * j + i] - (1.0f + t) * Y[3 * j + i] - (i == j ? dY : 0.f);
        Z[3 * i + j] = v * id;
      }
    // scaling zeta = sqrt(|X^{-1}|_F / |X|_F), X = I + Y
    float nx = 0.f, ny = 0.f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      float a = Y[i] + ((i % 4) == 0 ? 1.f : 0.f);
      float b = Z[i] + ((i % 4) == 0 ? 1.f : 0.f);
      nx += a * a;
      ny += b * b;
    }
    float zeta = sqrtf(sqrtf(ny / nx));
    float iz = 1.0f / zeta;
    float c = 0.5f * (zeta - 1.0f) * (zeta - 1.0f) * iz;  // (zeta + 1/zeta)/2 - 1
    float delta = 0.f, yy = 0.f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      float yn = 0.5f * (zeta * Y[i] + iz * Z[i]) + ((i % 4) == 0 ? c : 0.f);
      float e = yn - Y[i];
      delta += e * e;
      yy += yn * yn;
      Y[i] = yn;
    }
    if (delta <= 1e-12f * (yy + hh)) break;
  }
}

// Kirchhoff stress tau = P F^T from the shifted deformation gradient H = F - I.
//   fixed-corotated: tau = 2 mu (F - R) F^T + lam (J - 1) J I, F - R = H - (R - I)
//   Neo-Hookean:     tau = mu (F F^T - I) + lam log(J) I, F F^T - I = H + H^T + H H^T
__device__ __forceinline__ void kirchhoff_shift(const float *H, float mu, float lam, int material, float *tau,
                                                int32_t *status) {
  float Jm1 = det_shift(H);
  float J = 1.0f + Jm1;
  if (!(J > 0.f)) {
    if (status) atomicOr(status, DW_STATUS_INVERTED);
  }
  if (material == DW_NEO_HOOKEAN) {
    float HHt[9];
    matmul3_abt(H, H, HHt);
    float l = lam * log1pf(Jm1);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) tau[3 * i + j] = mu * (H[3 * i + j] + H[3 * j + i] + HHt[3 * i + j]);
    tau[0] += l;
    tau[4] += l;
    tau[8] += l;
  } else {
    float Y[9], D[9], F[9];
    polar_shift(H, Y);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      D[i] = H[i] - Y[i];
      F[i] = H[i] + ((i % 4) == 0 ? 1.f : 0.f);
    }
    matmul3_abt(D, F, tau);
    float l = lam * Jm1 * J;
#pragma unroll
    for (int i = 0; i < 9; ++i) tau[i] *= 2.0f * mu;
    tau[0] += l;
    tau[4] += l;
    tau[8] += l;
  }
}

// Kirchhoff stress for the forward P2G.  Fixed-corotated through the left
// stretch: with F = V R, (F - R) F^T = F F^T - V, so
//   tau = 2 mu (B - V) + lam (J - 1) J I,  B = F F^T = I + E,  V = sqrt(B),
// E = H + H^T + H H^T symmetric.  For |E|_F < 0.05 the binomial series
//   B - V = E - (sqrt(I + E) - I) = E/2 + E^2/8 - E^3/16 + 5 E^4/128 - 7 E^5/256 + ...
// (powers of one symmetric matrix commute, so every product stays
// symmetric: six entries) is truncated after E^5; the first dropped term is
// 21/1024 |E|^6, below 2e-8 of E/2 there, under float32 round-off.  Larger
// strains take the polar decomposition of kirchhoff_shift.  Neo-Hookean is
// kirchhoff_shift's closed form.
// symmetric 3x3 as (xx, yy, zz, xy, xz, yz)
__device__ __forceinline__ void sym_mul(const float *a, const float *b, float *c) {
  c[0] = a[0] * b[0] + a[3] * b[3] + a[4] * b[4];
  c[1] = a[3] * b[3] + a[1] * b[1] + a[5] * b[5];
  c[2] = a[4] * b[4] + a[5] * b[5] + a[2] * b[2];
  c[3] = a[0] * b[3] + a[3] * b[1] + a[4] * b[5];
  c[4] = a[0] * b[4] + a[3] * b[5] + a[4] * b[2];
  c[5] = a[3] * b[4] + a[1] * b[5] + a[5] * b[2];
}

__device__ __forceinline__ void kirchhoff_shift_p2g(const float *H, float mu, float lam, int material, float *tau,
                                                    int32_t *status) {
  if (material == DW_FIXED_COROTATED) {
    // E = H + H^T + H H^T
    float E[6];
    E[0] = 2.f * H[0] + H[0] * H[0] + H[1] * H[1] + H[2] * H[2];
    E[1] = 2.f * H[4] + H[3] * H[3] + H[4] * H[4] + H[5] * H[5];
    E[2] = 2.f * H[8] + H[6] * H[6] + H[7] * H[7] + H[8] * H[8];
    E[3] = H[1] + H[3] + H[0] * H[3] + H[1] * H[4] + H[2] * H[5];
    E[4] = H[2] + H[6] + H[0] * H[6] + H[1] * H[7] + H[2] * H[8];
    E[5] = H[5] + H[7] + H[3] * H[6] + H[4] * H[7] + H[5] * H[8];
    const float e2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2] + 2.f * (E[3] * E[3] + E[4] * E[4] + E[5] * E[5]);
    if (e2 < 0.0025f) {
      const float Jm1 = det_shift(H);
      if (!(Jm1 > -1.f) && status) atomicOr(status, DW_STATUS_INVERTED);
      // Horner: T = c1 I + E (c2 I + E (c3 I + E (c4 I + c5 E))), B - V = E T
      float T[6], U[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) T[i] = (-7.f / 256.f) * E[i];
      T[0] += 5.f / 128.f; T[1] += 5.f / 128.f; T[2] += 5.f / 128.f;
      sym_mul(E, T, U);
      U[0] -= 1.f / 16.f; U[1] -= 1.f / 16.f; U[2] -= 1.f / 16.f;
      sym_mul(E, U, T);
      T[0] += 1.f / 8.f; T[1] += 1.f / 8.f; T[2] += 1.f / 8.f;
      sym_mul(E, T, U);
      U[0] += 0.5f; U[1] += 0.5f; U[2] += 0.5f;
      sym_mul(E, U, T);  // T = B - V
      const float l = lam * Jm1 * (1.0f + Jm1);
      const float m2 = 2.0f * mu;
      tau[0] = m2 * T[0] + l;
      tau[4] = m2 * T[1] + l;
      tau[8] = m2 * T[2] + l;
      tau[1] = tau[3] = m2 * T[3];
      tau[2] = tau[6] = m2 * T[4];
      tau[5] = tau[7] = m2 * T[5];
      return;
    }
  }
  kirchhoff_shift(H, mu, lam, material, tau, status);
}

// Element i of an array whose byte offsets fit in 32 bits (i < 2^30): a
// scalar base plus a 32-bit lane offset, which the load / store encodes
// directly (no 64-bit address arithmetic per lane).
__device__ __forceinline__ float ld32(const float *base, uint32_t i) {
  return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + (i << 2));
}
__device__ __forceinline__ void st32(float *base, uint32_t i, float v) {
  *reinterpret_cast<float *>(reinterpret_cast<char *>(base) + (i << 2)) = v;
}

// Grid coordinate X = (x - origin) / dx of a particle and its stencil base
// floor(X - 1/2).  Contraction is disabled so that every kernel rounds the
// same way and a particle lands in the same cell tile in the sort, the
// transfers and the adjoints.
__device__ __forceinline__ float grid_coord(float x, float o, float inv_dx) {
#pragma clang fp contract(off)
  return (x - o) * inv_dx;
}

__device__ __forceinline__ int base_of(float X) {
#pragma clang fp contract(off)
  return (int)floorf(X - 0.5f);
}

// Grid coordinate of a particle on one axis, kept as two parts A + B.
// Absolute positions (no reference array): A = (x - o) / dx, B = 0.
// Positions relative to a per-particle reference xr (the position is
// xr + x): A = (xr - o) / dx and B = x / dx, the displacement scaled on its
// own so that it keeps its float32 resolution.  Each difference and product
// is rounded once (contraction off), the same way in every kernel.  The
// stencil base is base_of(A + B); the fractional position (A - base) + B,
// where A - base is exact.  With B = 0 both reduce to the absolute forms.
struct Coord {
  float A, B;
};

__device__ __forceinline__ Coord make_coord(bool ref, float xr, float x, float o, float inv_dx) {
#pragma clang fp contract(off)
  Coord c;
  if (ref) {
    c.A = (xr - o) * inv_dx;
    c.B = x * inv_dx;
  } else {
    c.A = (x - o) * inv_dx;
    c.B = 0.f;
  }
  return c;
}

// element idx of the position arrays (xr may be NULL: absolute positions)
__device__ __forceinline__ Coord load_coord(const float *xr, const float *x, size_t idx, float o, float inv_dx) {
  return make_coord(xr != nullptr, xr ? xr[idx] : 0.f, x[idx], o, inv_dx);
}

__device__ __forceinline__ float coord_sum(Coord c) {
#pragma clang fp contract(off)
  return c.A + c.B;
}

__device__ __forceinline__ float coord_frac(Coord c, int base) {
#pragma clang fp contract(off)
  return (c.A - (float)base) + c.B;
}

// Quadratic B-spline weights of nodes base + 0, 1, 2 at fractional position
// f = X - base in [1/2, 3/2), and their derivatives d w / d f.
__device__ __forceinline__ void bspline_w(float f, float w[3]) {
  float a = 1.5f - f, b = f - 1.0f, c = f - 0.5f;
  w[0] = 0.5f * a * a;
  w[1] = 0.75f - b * b;
  w[2] = 0.5f * c * c;
}

__device__ __forceinline__ void bspline_dw(float f, float dw[3]) {
  dw[0] = f - 1.5f;
  dw[1] = -2.0f * (f - 1.0f);
  dw[2] = f - 0.5f;
}

__device__ __forceinline__ bool stencil_inside(const GridDev &g, int bx, int by, int bz) {
  return bx >= 0 && by >= 0 && bz >= 0 && bx + 2 < g.nx && by + 2 < g.ny && bz + 2 < g.nz;
}

}  // namespace dw
