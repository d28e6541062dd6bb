// Hand-written adjoints of the MPM substep for gfx950.
//
// Reverse P2G is a gather per particle (each particle reads the grid adjoint
// at its 27 stencil nodes); reverse G2P is a sorted scatter (particles
// grouped by cell tile, the grid adjoint summed on the matrix cores into LDS
// node blocks and added to the global grid with float atomics); reverse grid
// update is pointwise over the active node tiles.  All adjoint outputs
// accumulate (+=).
//
// Forward definitions differentiated here: Eq. P2G with the MLS-MPM stress
// term A = m C - dt V0 (4/dx^2) tau(F), the explicit grid update of
// Eq. continuum_mechanics with the wind acceleration, Eq. G2P with the APIC
// affine matrix and Eq. deformation_update.
#include <hip/hip_runtime.h>

#include <climits>

#include "dw_internal.h"
#include "dw_kernels.h"
#include "dw_scatter.h"

namespace dw {

// skew(y) as a 3x3 matrix
__device__ __forceinline__ void cross_matrix(const float y[3], float Z[9]) {
  Z[0] = 0.f;   Z[1] = -y[2]; Z[2] = y[1];
  Z[3] = y[2];  Z[4] = 0.f;   Z[5] = -y[0];
  Z[6] = -y[1]; Z[7] = y[0];  Z[8] = 0.f;
}

// Vector-Jacobian product of the polar rotation R(F), F = R S:
// dR = R W with W skew solving S W + W S = R^T dF - dF^T R; in vector form
// (tr(S) I - S) w = k.  For a cotangent Rbar this gives
// Fbar += 2 R [y]x with y = (tr(S) I - S)^{-1} g, g the axial vector of
// skew(R^T Rbar).
__device__ __forceinline__ void polar_vjp(const float *F, const float *R, const float *Rbar, float *Fbar) {
  float S[9], G[9];
  matmul3_atb(R, F, S);
  matmul3_atb(R, Rbar, G);
  float g[3] = {0.5f * (G[7] - G[5]), 0.5f * (G[2] - G[6]), 0.5f * (G[3] - G[1])};
  float tr = S[0] + S[4] + S[8];
  float M[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) M[q] = -0.5f * (S[q] + S[(q % 3) * 3 + q / 3]);
  M[0] += tr;
  M[4] += tr;
  M[8] += tr;
  float d = det3(M);
  float MiT[9];
  inv_transpose3(M, d, MiT);  // M symmetric: inverse = inverse-transpose
  float y[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) y[a] = MiT[3 * a] * g[0] + MiT[3 * a + 1] * g[1] + MiT[3 * a + 2] * g[2];
  float Z[9], RZ[9];
  cross_matrix(y, Z);
  matmul3(R, Z, RZ);
#pragma unroll
  for (int q = 0; q < 9; ++q) Fbar[q] += 2.0f * RZ[q];
}

// Vector-Jacobian product of the Kirchhoff stress tau(F; mu, lam), F = I + H.
//   Neo-Hookean: tau = mu (F F^T - I) + lam log J I
//     Fbar += mu (tb + tb^T) F + lam tr(tb) F^{-T}
//   fixed-corotated: tau = 2 mu (F - R) F^T + lam (J - 1) J I
//     Fbar += 2 mu tb F + 2 mu tb^T (F - R) + polar_vjp(Rbar = -2 mu tb F)
//             + lam (2J - 1) J tr(tb) F^{-T}
// Also returns the cotangents of mu and lam.
__device__ __forceinline__ void kirchhoff_vjp(const float *H, float mu, float lam, int material, const float *tb,
                                              float *Fbar, float &mu_bar, float &lam_bar) {
  float F[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) F[q] = H[q] + ((q % 4) == 0 ? 1.f : 0.f);
  float Jm1 = det_shift(H);
  float J = 1.0f + Jm1;
  float FiT[9];
  inv_transpose3(F, J, FiT);
  float trt = tb[0] + tb[4] + tb[8];
  if (material == DW_NEO_HOOKEAN) {
    float S[9], SF[9], HHt[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) S[q] = tb[q] + tb[(q % 3) * 3 + q / 3];
    matmul3(S, F, SF);
#pragma unroll
    for (int q = 0; q < 9; ++q) Fbar[q] += mu * SF[q] + lam * trt * FiT[q];
    matmul3_abt(H, H, HHt);
    float mb = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) mb += tb[3 * i + j] * (H[3 * i + j] + H[3 * j + i] + HHt[3 * i + j]);
    mu_bar = mb;
    lam_bar = trt * log1pf(Jm1);
  } else {
    float Y[9], R[9], D[9], TF[9], TtD[9], Rb[9], DFt[9];
    polar_shift(H, Y);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      D[q] = H[q] - Y[q];
      R[q] = Y[q] + ((q % 4) == 0 ? 1.f : 0.f);
    }
    matmul3(tb, F, TF);
    matmul3_atb(tb, D, TtD);
    float cj = lam * (2.f * J - 1.f) * J * trt;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      Fbar[q] += 2.f * mu * (TF[q] + TtD[q]) + cj * FiT[q];
      Rb[q] = -2.f * mu * TF[q];
    }
    polar_vjp(F, R, Rb, Fbar);
    matmul3_abt(D, F, DFt);
    float mb = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) mb += tb[q] * DFt[q];
    mu_bar = 2.f * mb;
    lam_bar = trt * Jm1 * J;
  }
}

// three consecutive floats (the x-neighbours of a stencil row)
struct AdjRow {
  float v[3];
};

// sum over the 64 lanes of a wave
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct PAdj {
  const float *x, *v, *C, *F, *mass, *vol0, *E, *nu;
  const float *xr;  // position reference or NULL
  const int32_t *region;
  int n, n_regions;
  float *xb, *vb, *Cb, *Fb, *Eb;
  float *Epart;     // deterministic mode: per-wave region sums [waves][n_regions]
};

// ---------------------------------------------------------- reverse P2G
// DET: the E adjoint is not added with atomics; every wave writes its
// per-region sums (fixed-order wave reductions) to P.Epart and
// k_ebar_reduce adds the waves in index order.
template <bool DET>
__global__ __launch_bounds__(256) void k_p2g_adj(GridDev g, PAdj P, float dt, int material,
                                                 const float *__restrict__ mbar, const float *__restrict__ mvbar,
                                                 int64_t N) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  bool live = p < P.n;
  const int n = P.n;
  float Ebar_p = 0.f;
  int r = 0;
  if (live) {
    const Coord cx = load_coord(P.xr, P.x, p, g.ox, g.inv_dx);
    const Coord cy = load_coord(P.xr, P.x, (size_t)n + p, g.oy, g.inv_dx);
    const Coord cz = load_coord(P.xr, P.x, 2 * (size_t)n + p, g.oz, g.inv_dx);
    const float X = coord_sum(cx), Y = coord_sum(cy), Z = coord_sum(cz);
    bool ok = isfinite(X) && isfinite(Y) && isfinite(Z) && fabsf(X) < 1e9f && fabsf(Y) < 1e9f && fabsf(Z) < 1e9f;
    int bx = 0, by = 0, bz = 0;
    if (ok) {
      bx = base_of(X); by = base_of(Y); bz = base_of(Z);
      ok = stencil_inside(g, bx, by, bz);
    }
    if (ok) {
      float f[3] = {coord_frac(cx, bx), coord_frac(cy, by), coord_frac(cz, bz)};
      float w[3][3], dw[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        bspline_w(f[a], w[a]);
        bspline_dw(f[a], dw[a]);
      }
      float F[9], Cm[9], tau[9], A[9];  // F holds H = F - I
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        F[q] = P.F[q * n + p];
        Cm[q] = P.C[q * n + p];
      }
      float m = P.mass[p], V0 = P.vol0[p];
      r = P.region[p];
      float Er = P.E[r], nur = P.nu[r];
      float mu, lam;
      lame(Er, nur, mu, lam);
      kirchhoff_shift(F, mu, lam, material, tau, nullptr);
      float ks = dt * 4.0f * g.inv_dx * g.inv_dx;
#pragma unroll
      for (int q = 0; q < 9; ++q) A[q] = m * Cm[q] - ks * V0 * tau[q];
      float mom[3] = {m * P.v[p], m * P.v[n + p], m * P.v[2 * n + p]};
      const float dx = g.dx;
      // Per node n (offset o, weight w_n, gradient gw_n, d_n = (o - f) dx):
      //   v_bar += m w gb,  A_bar += w gb d^T,
      //   x_bar += gw s - w A^T gb  with s = m mb + gb . (mom + A d).
      // Sums that factor are taken once: G = sum w gb (v_bar = m G, and the
      // A^T term is A^T G), O = sum w gb o^T (A_bar = dx (O - G f^T)), and
      // mom + A d = c0 + dx A o with c0 = mom - dx A f, whose y/z part is
      // constant along a stencil row.
      float c0[3], Ax[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        c0[a] = mom[a] - dx * (A[3 * a] * f[0] + A[3 * a + 1] * f[1] + A[3 * a + 2] * f[2]);
        Ax[a] = dx * A[3 * a];
      }
      float G[3] = {0.f, 0.f, 0.f}, X[3] = {0.f, 0.f, 0.f};
      float O[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      // rows of the stencil one at a time (bounded register use), the three
      // x-neighbours of a row read with one 12-byte load per array
#pragma unroll 1
      for (int r9 = 0; r9 < 9; ++r9) {
        const int oy = r9 % 3, oz = r9 / 3;
        const int64_t row = bx + (int64_t)g.nx * ((by + oy) + (int64_t)g.ny * (bz + oz));
        AdjRow rm, r0, r1, r2;
        __builtin_memcpy(&rm, mbar + row, sizeof(AdjRow));
        __builtin_memcpy(&r0, mvbar + row, sizeof(AdjRow));
        __builtin_memcpy(&r1, mvbar + N + row, sizeof(AdjRow));
        __builtin_memcpy(&r2, mvbar + 2 * N + row, sizeof(AdjRow));
        const float wyz = w[1][oy] * w[2][oz];
        const float gwx = wyz * g.inv_dx, gwy = dw[1][oy] * w[2][oz] * g.inv_dx,
                    gwz = w[1][oy] * dw[2][oz] * g.inv_dx;
        float cy[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) cy[a] = c0[a] + dx * (A[3 * a + 1] * (float)oy + A[3 * a + 2] * (float)oz);
        float RG[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int ox = 0; ox < 3; ++ox) {
          const float wt = w[0][ox] * wyz;
          const float gb[3] = {r0.v[ox], r1.v[ox], r2.v[ox]};
          float s = m * rm.v[ox];
#pragma unroll
          for (int a = 0; a < 3; ++a) s += gb[a] * (cy[a] + Ax[a] * (float)ox);
          X[0] += dw[0][ox] * gwx * s;
          X[1] += w[0][ox] * gwy * s;
          X[2] += w[0][ox] * gwz * s;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const float t = wt * gb[a];
            RG[a] += t;
            O[3 * a] += (float)ox * t;
          }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          G[a] += RG[a];
          O[3 * a + 1] += (float)oy * RG[a];
          O[3 * a + 2] += (float)oz * RG[a];
        }
      }
      float vbar[3], xbar[3], Abar[9];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        vbar[a] = m * G[a];
        // d (A d) / d x = -A   ->   -A^T G
        xbar[a] = X[a] - (A[a] * G[0] + A[3 + a] * G[1] + A[6 + a] * G[2]);
#pragma unroll
        for (int b = 0; b < 3; ++b) Abar[3 * a + b] = dx * (O[3 * a + b] - G[a] * f[b]);
      }
      if (P.vb) {
#pragma unroll
        for (int a = 0; a < 3; ++a) P.vb[a * n + p] += vbar[a];
      }
      if (P.xb) {
#pragma unroll
        for (int a = 0; a < 3; ++a) P.xb[a * n + p] += xbar[a];
      }
      if (P.Cb) {
#pragma unroll
        for (int q = 0; q < 9; ++q) P.Cb[q * n + p] += m * Abar[q];
      }
      if (P.Fb || P.Eb) {
        float tb[9], Fb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 9; ++q) tb[q] = -ks * V0 * Abar[q];
        float mu_b, lam_b;
        kirchhoff_vjp(F, mu, lam, material, tb, Fb, mu_b, lam_b);
        if (P.Fb) {
#pragma unroll
          for (int q = 0; q < 9; ++q) P.Fb[q * n + p] += Fb[q];
        }
        // Eq. young_poisson: d mu / d E = 1 / (2 (1 + nu)), d lam / d E = nu / ((1 + nu)(1 - 2 nu))
        Ebar_p = mu_b / (2.f * (1.f + nur)) + lam_b * nur / ((1.f + nur) * (1.f - 2.f * nur));
      }
    }
  }
  if (P.Eb && DET) {
    // lane l of the wave keeps the sum of region r0 + l; one store per entry
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    for (int r0 = 0; r0 < P.n_regions; r0 += 64) {
      float mine_sum = 0.f;
      unsigned long long pending = __ballot(live && r >= r0 && r < r0 + 64);
      while (pending) {
        const int leader = __ffsll(pending) - 1;
        const int rk = __shfl(r, leader, 64);
        const bool mine = live && r == rk;
        const float sum = wave_sum(mine ? Ebar_p : 0.f);
        if (lane == rk - r0) mine_sum = sum;
        pending &= ~__ballot(mine);
      }
      if (r0 + lane < P.n_regions) P.Epart[wave * P.n_regions + r0 + lane] = mine_sum;
    }
  } else if (P.Eb) {
    // one atomic per (wave, region): a wave holds few regions, while
    // per-lane atomics on a handful of addresses would serialise
    unsigned long long pending = __ballot(live);
    const int lane = threadIdx.x & 63;
    while (pending) {
      const int leader = __ffsll(pending) - 1;
      const int rk = __shfl(r, leader, 64);
      const bool mine = live && r == rk;
      const float sum = wave_sum(mine ? Ebar_p : 0.f);
      if (lane == leader && sum != 0.f) atomicAdd(&P.Eb[rk], sum);
      pending &= ~__ballot(mine);
    }
  }
}

// E adjoint of the deterministic reverse P2G: region r adds the per-wave sums
// in wave order.
__global__ __launch_bounds__(64) void k_ebar_reduce(const float *__restrict__ part, int64_t waves, int R,
                                                    float *__restrict__ Eb) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  float s = 0.f;
  for (int64_t w = 0; w < waves; ++w) s += part[w * R + r];
  Eb[r] += s;
}

// --------------------------------------------------- reverse grid update
__global__ __launch_bounds__(256) void k_grid_update_adj(GridDev g, float dt, float gx, float gy, float gz,
                                                         int bound, const float *__restrict__ gm,
                                                         const float *__restrict__ gmv, WindDev wind,
                                                         const uint8_t *__restrict__ pin,
                                                         const int32_t *__restrict__ node_tiles,
                                                         const int32_t *__restrict__ n_tiles,
                                                         const float *__restrict__ gvb, float *__restrict__ gmb,
                                                         float *__restrict__ gmvb, float *__restrict__ accb,
                                                         int64_t N) {
  int nt = *n_tiles;
  int sub = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int it = blockIdx.x * 4 + sub; it < nt; it += gridDim.x * 4) {
    int t = node_tiles[it];
    int tx = t % g.tx, ty = (t / g.tx) % g.ty, tz = t / (g.tx * g.ty);
    int i = tx * 4 + (l & 3), j = ty * 4 + ((l >> 2) & 3), k = tz * 4 + (l >> 4);
    if (i >= g.nx || j >= g.ny || k >= g.nz) continue;
    int64_t node = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    float m = gm[node];
    if (!(m > 0.f)) continue;
    if (pin && pin[node]) continue;
    float im = 1.0f / m;
    float mv[3] = {gmv[node], gmv[N + node], gmv[2 * N + node]};
    const float vs[3] = {mv[0] * im, mv[1] * im, mv[2] * im};
    float ax, ay, az;
    wind_at_node(wind, g, i, j, k, node, vs[0], vs[1], vs[2], ax, ay, az);
    float v[3] = {vs[0] + dt * (gx + ax), vs[1] + dt * (gy + ay), vs[2] + dt * (gz + az)};
    float vb[3] = {gvb[node], gvb[N + node], gvb[2 * N + node]};
    if ((i < bound && v[0] < 0.f) || (i >= g.nx - bound && v[0] > 0.f)) vb[0] = 0.f;
    if ((j < bound && v[1] < 0.f) || (j >= g.ny - bound && v[1] > 0.f)) vb[1] = 0.f;
    if ((k < bound && v[2] < 0.f) || (k >= g.nz - bound && v[2] > 0.f)) vb[2] = 0.f;
    // adjoint of the acceleration, and of the wind velocity U and of v* for
    // the relative drag a = k |r| r, r = U - v*: with J = k (|r| I + r r^T / |r|)
    // U_bar = J a_bar and v*_bar gets -J a_bar
    float ab[3] = {dt * vb[0], dt * vb[1], dt * vb[2]};
    float vsb[3] = {vb[0], vb[1], vb[2]};
    if (wind.mode == DW_WIND_LBM_DRAG_REL) {
      float U[3];
      float r[3] = {0.f, 0.f, 0.f};
      if (wind_velocity_at_node(wind, g, i, j, k, U[0], U[1], U[2])) {
        r[0] = U[0] - vs[0];
        r[1] = U[1] - vs[1];
        r[2] = U[2] - vs[2];
      }
      const float sp = sqrtf(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      float Jab[3] = {0.f, 0.f, 0.f};
      if (sp > 0.f) {
        const float rb = (r[0] * ab[0] + r[1] * ab[1] + r[2] * ab[2]) / sp;
#pragma unroll
        for (int a = 0; a < 3; ++a) Jab[a] = wind.k_drag * (sp * ab[a] + r[a] * rb);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        vsb[a] -= Jab[a];
        ab[a] = Jab[a];
      }
    }
    if (gmvb) {
      gmvb[node] += vsb[0] * im;
      gmvb[N + node] += vsb[1] * im;
      gmvb[2 * N + node] += vsb[2] * im;
    }
    if (gmb) gmb[node] += -(vsb[0] * mv[0] + vsb[1] * mv[1] + vsb[2] * mv[2]) * im * im;
    if (accb) {
      accb[node] += ab[0];
      accb[N + node] += ab[1];
      accb[2 * N + node] += ab[2];
    }
  }
}

// ---------------------------------------------------------- reverse G2P

// Reverse G2P.  One workgroup per work item (a chunk of at most WORK_CHUNK
// sorted particles of one cell tile), one particle per thread.  Each thread
// redoes the forward gather of its particle (v_p and C_p), applies the
// adjoints of the x, F and C updates and gathers x_bar; the scatter of the
// grid-velocity adjoint, v_bar_i += w_ip (vbt_p + kc Cbt_p (o - f_p)), has
// the P2G form w (q + A o) with q = vbt - kc Cbt f, A = kc Cbt and runs as
// the tile scatter of dw_scatter.h; node owners add the result into the
// global grid adjoint with float atomics.  DET: the particles of a cell take
// their slots in index order and the node owners write the item's 6^3 block
// to item_part instead, which k_det_gather<true> then adds to the grid
// adjoint in a fixed order (bit-reproducible with a deterministic sort).
template <bool DET>
__global__ __launch_bounds__(SC_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_g2p_adj(
    GridDev g, float dt, const float *__restrict__ gv, int64_t N, const float *__restrict__ x,
    const float *__restrict__ xr, const float *__restrict__ F, int n, const float *__restrict__ xob, const float *__restrict__ vob,
    const float *__restrict__ Cob, const float *__restrict__ Fob, float *__restrict__ xb, float *__restrict__ Fb,
    float *__restrict__ gvb, const int32_t *__restrict__ perm, const int32_t *__restrict__ tile_start,
    const int32_t *__restrict__ item_tile, const int32_t *__restrict__ item_begin,
    const int32_t *__restrict__ n_items, float *__restrict__ item_part) {
  __shared__ float s_dat[SC_DAT][SC_PITCH];
  __shared__ unsigned char s_cell[WORK_CHUNK];
  __shared__ float4 s_f[SC_PITCH];                                  // staged f per particle
  __shared__ __attribute__((aligned(16))) float s_node[SC_WAVES][SC_NODES][4];
  __shared__ int s_cnt[64], s_off[64], s_cur[64];
  __shared__ int s_udesc[SC_MAX_UNITS];
  __shared__ int s_nunits;
  __shared__ float s_gv[3][SC_NODES];  // grid velocities of the item's 6^3 node region
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const ScLane L = sc_lane(lane);
  float *s_node_flat = &s_node[0][0][0];
  const int ni = *n_items;
  const float kc = 4.0f * g.inv_dx;
  for (int it = blockIdx.x; it < ni; it += gridDim.x) {
    const int tile = item_tile[it];
    const int b0 = item_begin[it];
    const int nb = min(WORK_CHUNK, tile_start[tile + 1] - b0);
    const int tx = tile % g.tx, ty = (tile / g.tx) % g.ty, tz = tile / (g.tx * g.ty);
    if (tid < 64) s_cnt[tid] = 0;
    for (int q = tid; q < SC_WAVES * SC_NODES; q += SC_THREADS)
      reinterpret_cast<float4 *>(s_node_flat)[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    // every stencil of the item lies in the tile's 6^3 node region: stage its
    // grid velocities once, for both gathers below
    if (tid < SC_NODES) {
      const int gx = 4 * tx + tid % SC_L, gy = 4 * ty + (tid / SC_L) % SC_L, gz = 4 * tz + tid / (SC_L * SC_L);
      float a0 = 0.f, a1 = 0.f, a2 = 0.f;
      if (gx < g.nx && gy < g.ny && gz < g.nz) {
        const int64_t node = gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz);
        a0 = gv[node];
        a1 = gv[N + node];
        a2 = gv[2 * N + node];
      }
      s_gv[0][tid] = a0;
      s_gv[1][tid] = a1;
      s_gv[2][tid] = a2;
    }
    __syncthreads();
    // particle -> cell in the tile
    const bool has = tid < nb;
    const int p = has ? perm[b0 + tid] : 0;
    Coord cx = {0.f, 0.f}, cy = {0.f, 0.f}, cz = {0.f, 0.f};
    int bx = 0, by = 0, bz = 0, c = -1;
    if (has) {
      cx = load_coord(xr, x, p, g.ox, g.inv_dx);
      cy = load_coord(xr, x, (size_t)n + p, g.oy, g.inv_dx);
      cz = load_coord(xr, x, 2 * (size_t)n + p, g.oz, g.inv_dx);
      bx = base_of(coord_sum(cx));
      by = base_of(coord_sum(cy));
      bz = base_of(coord_sum(cz));
      const int lx = bx - 4 * tx, ly = by - 4 * ty, lz = bz - 4 * tz;
      if ((unsigned)lx <= 3u && (unsigned)ly <= 3u && (unsigned)lz <= 3u) {
        c = lx + 4 * (ly + 4 * lz);
        atomicAdd(&s_cnt[c], 1);
      }
    }
    if (DET) s_cell[tid] = (unsigned char)(c >= 0 ? c : 255);
    __syncthreads();
    if (wid == 0) sc_scan_units(lane, s_cnt, s_off, s_cur, s_udesc, &s_nunits);
    __syncthreads();
    if (c >= 0) {
      int slot;
      if (DET) {
        // fixed order: rank among the item's earlier particles of the same cell
        int rank = 0;
        for (int q = 0; q < tid; ++q) rank += s_cell[q] == c;
        slot = s_off[c] + rank;
      } else {
        slot = atomicAdd(&s_cur[c], 1);
      }
      float f[3] = {coord_frac(cx, bx), coord_frac(cy, by), coord_frac(cz, bz)};
      float w[3][3], dw[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        bspline_w(f[a], w[a]);
        bspline_dw(f[a], dw[a]);
      }
      // forward gather: v_p and C_p
      float vp[3] = {0.f, 0.f, 0.f};
      float B[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
      for (int r9 = 0; r9 < 9; ++r9) {
        const int oy = r9 % 3, oz = r9 / 3;
        const int li = (bx - 4 * tx) + SC_L * ((by - 4 * ty + oy) + SC_L * (bz - 4 * tz + oz));
        AdjRow r0, r1, r2;
#pragma unroll
        for (int ox = 0; ox < 3; ++ox) {
          r0.v[ox] = s_gv[0][li + ox];
          r1.v[ox] = s_gv[1][li + ox];
          r2.v[ox] = s_gv[2][li + ox];
        }
#pragma unroll
        for (int ox = 0; ox < 3; ++ox) {
          const float wt = w[0][ox] * w[1][oy] * w[2][oz];
          const float vi[3] = {r0.v[ox], r1.v[ox], r2.v[ox]};
          const float o[3] = {(float)ox - f[0], (float)oy - f[1], (float)oz - f[2]};
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            vp[a] += wt * vi[a];
#pragma unroll
            for (int b = 0; b < 3; ++b) B[3 * a + b] += wt * vi[a] * o[b];
          }
        }
      }
      float Cn[9], Fp[9], Fo[9], Cbt[9], vbt[3];
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        Cn[q] = kc * B[q];
        Fp[q] = F[q * n + p] + ((q % 4) == 0 ? 1.f : 0.f);  // stored as F - I
        Fo[q] = Fob ? Fob[q * n + p] : 0.f;
        Cbt[q] = Cob ? Cob[q * n + p] : 0.f;
      }
      // F' = (I + dt C) F:  Fbar += (I + dt C)^T Fbar',  Cbar += dt Fbar' F^T
      if (Fob) {
        float G[9], GtFo[9], FoFt[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) G[q] = dt * Cn[q];
        G[0] += 1.f;
        G[4] += 1.f;
        G[8] += 1.f;
        matmul3_atb(G, Fo, GtFo);
        matmul3_abt(Fo, Fp, FoFt);
        if (Fb) {
#pragma unroll
          for (int q = 0; q < 9; ++q) Fb[q * n + p] += GtFo[q];
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) Cbt[q] += dt * FoFt[q];
      }
      // x' = x + dt v_p
#pragma unroll
      for (int a = 0; a < 3; ++a) vbt[a] = (vob ? vob[a * n + p] : 0.f) + dt * (xob ? xob[a * n + p] : 0.f);
      // x_bar: gradient of the gather through the weights and the offsets
      float xbar[3] = {xob ? xob[p] : 0.f, xob ? xob[n + p] : 0.f, xob ? xob[2 * n + p] : 0.f};
#pragma unroll 1
      for (int r9 = 0; r9 < 9; ++r9) {
        const int oy = r9 % 3, oz = r9 / 3;
        const int li = (bx - 4 * tx) + SC_L * ((by - 4 * ty + oy) + SC_L * (bz - 4 * tz + oz));
        AdjRow r0, r1, r2;
#pragma unroll
        for (int ox = 0; ox < 3; ++ox) {
          r0.v[ox] = s_gv[0][li + ox];
          r1.v[ox] = s_gv[1][li + ox];
          r2.v[ox] = s_gv[2][li + ox];
        }
#pragma unroll
        for (int ox = 0; ox < 3; ++ox) {
          const float wt = w[0][ox] * w[1][oy] * w[2][oz];
          const float gw[3] = {dw[0][ox] * w[1][oy] * w[2][oz] * g.inv_dx, w[0][ox] * dw[1][oy] * w[2][oz] * g.inv_dx,
                               w[0][ox] * w[1][oy] * dw[2][oz] * g.inv_dx};
          const float o[3] = {(float)ox - f[0], (float)oy - f[1], (float)oz - f[2]};
          const float vi[3] = {r0.v[ox], r1.v[ox], r2.v[ox]};
          float Co[3], CtV[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            Co[a] = Cbt[3 * a] * o[0] + Cbt[3 * a + 1] * o[1] + Cbt[3 * a + 2] * o[2];
            CtV[a] = Cbt[a] * vi[0] + Cbt[3 + a] * vi[1] + Cbt[6 + a] * vi[2];
          }
          const float sdot =
              vi[0] * vbt[0] + vi[1] * vbt[1] + vi[2] * vbt[2] + kc * (vi[0] * Co[0] + vi[1] * Co[1] + vi[2] * Co[2]);
          // d o / d x = -inv_dx I
#pragma unroll
          for (int a = 0; a < 3; ++a) xbar[a] += gw[a] * sdot - wt * kc * g.inv_dx * CtV[a];
        }
      }
      if (xb) {
#pragma unroll
        for (int a = 0; a < 3; ++a) xb[a * n + p] += xbar[a];
      }
      // scatter features: q = vbt - kc Cbt f, A = kc Cbt
      float A[9], qv[3];
#pragma unroll
      for (int q = 0; q < 9; ++q) A[q] = kc * Cbt[q];
#pragma unroll
      for (int a = 0; a < 3; ++a) qv[a] = vbt[a] - (A[3 * a] * f[0] + A[3 * a + 1] * f[1] + A[3 * a + 2] * f[2]);
      sc_stage(s_dat, s_f, slot, f, 0.f, qv, A);
    }
    __syncthreads();
    sc_units_mfma(L, wid, s_dat, s_f, s_udesc, s_nunits, s_node[wid]);
    __syncthreads();
    if (tid < SC_NODES) {
      float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int w = 0; w < SC_WAVES; ++w) {
        s0 += s_node[w][tid][1];
        s1 += s_node[w][tid][2];
        s2 += s_node[w][tid][3];
      }
      if (DET) {
        float *dst = item_part + ((int64_t)it * SC_NODES + tid) * 4;
        dst[0] = 0.f;
        dst[1] = s0;
        dst[2] = s1;
        dst[3] = s2;
      } else if (s0 != 0.f || s1 != 0.f || s2 != 0.f) {
        const int ix = tid % SC_L, iy = (tid / SC_L) % SC_L, iz = tid / (SC_L * SC_L);
        const int64_t node = (4 * tx + ix) + (int64_t)g.nx * ((4 * ty + iy) + (int64_t)g.ny * (4 * tz + iz));
        atomicAdd(&gvb[node], s0);
        atomicAdd(&gvb[N + node], s1);
        atomicAdd(&gvb[2 * N + node], s2);
      }
    }
    __syncthreads();
  }
}

}  // namespace dw

using namespace dw;

extern "C" int mpm_p2g_adj(const dw_grid *grid, const dw_mpm_params *params, const dw_particles *p,
                           const float *grid_m_bar, const float *grid_mv_bar, dw_particles_bar *bar, float *E_bar,
                           void *ws, size_t ws_bytes, void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  DW_REQUIRE(params, DW_EINVAL, "mpm_p2g_adj: params is NULL");
  DW_REQUIRE(params->material == DW_FIXED_COROTATED || params->material == DW_NEO_HOOKEAN, DW_EINVAL,
             "mpm_p2g_adj: unknown material");
  rc = check_particles(p, true);
  if (rc) return rc;
  DW_REQUIRE(grid_m_bar && grid_mv_bar, DW_EINVAL, "mpm_p2g_adj: grid adjoints must be set");
  DW_REQUIRE(bar && bar->n == p->n, DW_EINVAL, "mpm_p2g_adj: bar->n must equal p->n");
  if (p->n == 0) return DW_OK;
  PAdj P;
  P.x = p->x; P.v = p->v; P.C = p->C; P.F = p->F; P.mass = p->mass; P.vol0 = p->vol0;
  P.E = p->E; P.nu = p->nu; P.region = p->region; P.n = p->n; P.xr = p->xref;
  P.xb = bar->x; P.vb = bar->v; P.Cb = bar->C; P.Fb = bar->F; P.Eb = E_bar;
  P.n_regions = p->n_regions;
  P.Epart = nullptr;
  GridDev g = make_grid(grid);
  int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;
  hipStream_t s = (hipStream_t)stream;
  const unsigned blocks = grid_blocks(p->n, 256);
  if (params->deterministic && E_bar) {
    Workspace W;
    rc = bind_workspace(grid, p->n, ws, ws_bytes, &W, 1);
    if (rc) return rc;
    const int64_t waves = (int64_t)blocks * 4;
    DW_REQUIRE(waves * p->n_regions <= W.item_part_floats, DW_EWORKSPACE,
               "mpm_p2g_adj: %d regions need more deterministic scratch than the workspace holds", p->n_regions);
    P.Epart = W.item_part;
    hipLaunchKernelGGL(k_p2g_adj<true>, dim3(blocks), dim3(256), 0, s, g, P, params->dt, params->material,
                       grid_m_bar, grid_mv_bar, N);
    hipLaunchKernelGGL(k_ebar_reduce, dim3(grid_blocks(p->n_regions, 64)), dim3(64), 0, s, W.item_part, waves,
                       p->n_regions, E_bar);
  } else {
    hipLaunchKernelGGL(k_p2g_adj<false>, dim3(blocks), dim3(256), 0, s, g, P, params->dt, params->material,
                       grid_m_bar, grid_mv_bar, N);
  }
  return check_launch("mpm_p2g_adj");
}

extern "C" int mpm_grid_update_adj(const dw_grid *grid, const dw_mpm_params *params, const float *grid_m,
                                   const float *grid_mv, const dw_wind *wind, const uint8_t *pin,
                                   const float *grid_v_bar, float *grid_m_bar, float *grid_mv_bar, float *acc_bar,
                                   const void *ws, size_t ws_bytes, void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  DW_REQUIRE(params && grid_m && grid_mv && grid_v_bar, DW_EINVAL, "mpm_grid_update_adj: missing argument");
  Workspace W;
  rc = bind_workspace(grid, 0, ws, ws_bytes, &W);
  if (rc) return rc;
  WindDev wd;
  rc = make_wind(wind, grid, &wd);
  if (rc) return rc;
  GridDev g = make_grid(grid);
  int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;
  hipLaunchKernelGGL(k_grid_update_adj, dim3(2048), dim3(256), 0, (hipStream_t)stream, g, params->dt,
                     params->gravity[0], params->gravity[1], params->gravity[2], params->bound, grid_m, grid_mv, wd,
                     pin, W.node_tiles, W.n_node_tiles, grid_v_bar, grid_m_bar, grid_mv_bar, acc_bar, N);
  return check_launch("mpm_grid_update_adj");
}

extern "C" int mpm_g2p_adj(const dw_grid *grid, const dw_mpm_params *params, const float *grid_v,
                           const dw_particles *in, const dw_particles_bar *out_bar, dw_particles_bar *in_bar,
                           float *grid_v_bar, const void *ws, size_t ws_bytes, void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  DW_REQUIRE(params && grid_v && in && out_bar && in_bar && grid_v_bar, DW_EINVAL,
             "mpm_g2p_adj: missing argument");
  DW_REQUIRE(in->n >= 0 && out_bar->n == in->n && in_bar->n == in->n, DW_EINVAL, "mpm_g2p_adj: size mismatch");
  if (in->n == 0) return DW_OK;
  DW_REQUIRE(in->x && in->F, DW_EINVAL, "mpm_g2p_adj: in->x / in->F is NULL");
  Workspace W;
  const int det = params->deterministic ? 1 : 0;
  rc = bind_workspace(grid, in->n, ws, ws_bytes, &W, det);
  if (rc) return rc;
  GridDev g = make_grid(grid);
  int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;
  hipStream_t s = (hipStream_t)stream;
  if (det) {
    hipLaunchKernelGGL(k_g2p_adj<true>, dim3(2048), dim3(SC_THREADS), 0, s, g, params->dt, grid_v, N, in->x,
                       in->xref, in->F, in->n, out_bar->x, out_bar->v, out_bar->C, out_bar->F, in_bar->x, in_bar->F,
                       grid_v_bar, W.perm, W.tile_start, W.item_tile, W.item_begin, W.n_items, W.item_part);
    hipLaunchKernelGGL(k_det_gather<true>, dim3(2048), dim3(256), 0, s, g, W.node_tiles, W.n_node_tiles,
                       W.tile_count, W.item_first, W.item_part, (float *)nullptr, grid_v_bar, N);
  } else {
    hipLaunchKernelGGL(k_g2p_adj<false>, dim3(2048), dim3(SC_THREADS), 0, s, g, params->dt, grid_v, N, in->x,
                       in->xref, in->F, in->n, out_bar->x, out_bar->v, out_bar->C, out_bar->F, in_bar->x, in_bar->F,
                       grid_v_bar, W.perm, W.tile_start, W.item_tile, W.item_begin, W.n_items, (float *)nullptr);
  }
  return check_launch("mpm_g2p_adj");
}
