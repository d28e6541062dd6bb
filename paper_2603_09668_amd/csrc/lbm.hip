// D3Q19 lattice Boltzmann for gfx950: fused pull stream-collide with BGK
// collision (Eq. lbe), moments with the half-force shift (Eq. lbm_sum_v2),
// Guo forcing, halfway bounce-back, equilibrium inlet, zero-gradient outlet,
// and the particle-to-voxel solid rule (Eq. point2voxel).  Populations are
// stored as f_i - w_i (structure of arrays [19][L], x fastest), so float32
// keeps its resolution on the deviation from rest.
#include <hip/hip_runtime.h>

#include <mutex>

#include <climits>
#include <utility>

#include "dw_internal.h"

namespace dw {

__device__ constexpr int LC[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                      {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, 0, 1},
                                      {-1, 0, -1}, {0, 1, 1},  {0, -1, -1}, {1, -1, 0}, {-1, 1, 0},
                                      {1, 0, -1}, {-1, 0, 1},  {0, 1, -1}, {0, -1, 1}};
__device__ constexpr int LOPP[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
__device__ constexpr float LW[19] = {1.f / 3,  1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18,
                                     1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36,
                                     1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};

struct LbmDev {
  int nx, ny, nz;
  int64_t L;
  float omega;     // 1 / tau
  float uin[3];
  float F[3];
  int bc[6];
  float gust_amp, gust_inv_period, gust_ky, gust_kz, gust_phase;
  int t;
  const int32_t *t_in;
  int32_t *t_out;
  const int32_t *skip;  // device flag: non-zero makes the launch do nothing
  bool forced;
};

// launch shape: threads along x, one block row per (y, z) line
constexpr int LBM_BLOCK = 128;
constexpr int SOL_W = LBM_BLOCK + 8;  // staged solid bytes per row: x0 - 4 .. x0 + LBM_BLOCK + 3

// Where a pulled population comes from: the source node, this node's
// opposite population (bounce-back), or the inlet ghost.
enum { SRC_NORMAL = 0, SRC_BOUNCE = 1, SRC_INLET = 2 };

// Inflow factor of the gust at inlet-plane (j, k): 1 + a sin(2 pi (t / T +
// ky j / ny + kz k / nz) + phase).  The phase is taken in turns and reduced
// to [0, 1) for the hardware sine of turns (a few instructions instead of a
// library sine; its error is far below float rounding of the inflow).
__device__ __forceinline__ float gust_factor(const LbmDev &P, int j, int k) {
  if (P.gust_amp == 0.f) return 1.0f;
  const int t = P.t_in ? *P.t_in : P.t;
  float rev = (float)t * P.gust_inv_period + P.gust_ky * (float)j / (float)P.ny +
              P.gust_kz * (float)k / (float)P.nz + P.gust_phase * 0.15915494309189535f;
  rev -= floorf(rev);
  return 1.0f + P.gust_amp * __builtin_amdgcn_sinf(rev);
}

// inlet equilibrium population (shifted) in direction q at inlet-plane (j, k)
__device__ __forceinline__ float inlet_feq_shift(const LbmDev &P, int q, int j, int k) {
  const float sfac = gust_factor(P, j, k);
  float ux = P.uin[0] * sfac, uy = P.uin[1] * sfac, uz = P.uin[2] * sfac;
  float cu = LC[q][0] * ux + LC[q][1] * uy + LC[q][2] * uz;
  float uu = ux * ux + uy * uy + uz * uz;
  return LW[q] * (3.f * cu + 4.5f * cu * cu - 1.5f * uu);
}

// Solid flags of the 3 x 3 (y, z) rows around this block's row,
// x0 - 4 .. x0 + LBM_BLOCK + 3, staged in LDS: row r = (dy + 1) + 3 (dz + 1).
// A periodic axis stages the wrapped row / positions, so every source that
// is not a bounce-back or inlet source finds its flag here; rows beyond a
// bounce-back face and positions beyond a non-periodic x face read as fluid.
// Whole 4-byte words are loaded where the row is 4-byte aligned.
constexpr int SOL_WORDS = 9 * (SOL_W / 4);
constexpr int SOL_PER_THREAD = (SOL_WORDS + LBM_BLOCK - 1) / LBM_BLOCK;

__device__ __forceinline__ void load_solid_rows(const LbmDev &P, const uint8_t *__restrict__ solid, int x0, int j,
                                                int k, uint32_t v[SOL_PER_THREAD]) {
  constexpr int WORDS = SOL_W / 4;
  const bool aligned = (P.nx & 3) == 0 && (((uintptr_t)solid) & 3) == 0;
  const bool xper = P.bc[0] == DW_BC_PERIODIC;
#pragma unroll
  for (int u = 0; u < SOL_PER_THREAD; ++u) {
    const int q = threadIdx.x + u * LBM_BLOCK;
    v[u] = 0;
    if (q >= SOL_WORDS) continue;
    const int r = q / WORDS, w = q % WORDS;
    int jj = j + r % 3 - 1, kk = k + r / 3 - 1;
    if ((unsigned)jj >= (unsigned)P.ny) {
      if (P.bc[2] != DW_BC_PERIODIC) continue;
      jj = jj < 0 ? jj + P.ny : jj - P.ny;
    }
    if ((unsigned)kk >= (unsigned)P.nz) {
      if (P.bc[4] != DW_BC_PERIODIC) continue;
      kk = kk < 0 ? kk + P.nz : kk - P.nz;
    }
    const int xs = x0 - 4 + 4 * w;
    const uint32_t row = (uint32_t)P.nx * ((uint32_t)jj + (uint32_t)P.ny * (uint32_t)kk);
    if (aligned && xs >= 0 && xs + 3 < P.nx) {
      v[u] = *reinterpret_cast<const uint32_t *>(solid + row + xs);
    } else if (!xper && (xs + 3 < 0 || xs >= P.nx)) {
      // wholly beyond a non-periodic x face: fluid
    } else {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        int x = xs + b;
        if ((unsigned)x >= (unsigned)P.nx) {
          if (!xper) continue;
          x = ((x % P.nx) + P.nx) % P.nx;
        }
        v[u] |= (uint32_t)solid[row + x] << (8 * b);
      }
    }
  }
}

__device__ __forceinline__ void store_solid_rows(const uint32_t v[SOL_PER_THREAD], uint8_t (*s_sol)[SOL_W]) {
#pragma unroll
  for (int u = 0; u < SOL_PER_THREAD; ++u) {
    const int q = threadIdx.x + u * LBM_BLOCK;
    if (q < SOL_WORDS) reinterpret_cast<uint32_t *>(&s_sol[0][0])[q] = v[u];
  }
}

// ---- forward pull with 32-bit offsets and row-uniform boundary rules
//
// The y and z faces are periodic or bounce-back (inlet and outlet sit on the
// x faces only), so the y/z part of every source is the same for a whole
// block row and is resolved with scalar branches; only the two x-boundary
// lanes of a row take the x rules, by selects.  Node indices are 32-bit
// (a lattice has fewer than 2^29 nodes) and every population plane is a
// scalar base plus a per-lane byte offset.

__device__ __forceinline__ float ld_node(const float *__restrict__ plane, uint32_t node) {
  return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(plane) + (node << 2));
}

__device__ __forceinline__ void st_node(float *__restrict__ plane, uint32_t node, float v) {
  *reinterpret_cast<float *>(reinterpret_cast<char *>(plane) + (node << 2)) = v;
}

// slot of the five directions with c_x = +1 (the ones an x-inlet feeds)
__host__ __device__ constexpr int inlet_slot(int q) {
  return q == 1 ? 0 : q == 7 ? 1 : q == 9 ? 2 : q == 13 ? 3 : q == 15 ? 4 : -1;
}
__device__ constexpr int INLET_Q[5] = {1, 7, 9, 13, 15};

struct PullSrc {
  uint32_t src;  // source node (always inside the lattice)
  int kind;      // SRC_NORMAL / SRC_BOUNCE / SRC_INLET
  int wx;        // x of the source in the staged solid rows (unwrapped; clamped at an outlet)
};

// y/z part of the source row of direction (cy, cz) for row (j, k): wraps a
// periodic face, flags a bounce-back face; *sj, *sk stay inside the lattice.
__device__ __forceinline__ void row_source(const LbmDev &P, int j, int k, int cy, int cz, int *sj, int *sk,
                                           bool *bounce) {
  int a = j - cy, b = k - cz;
  *bounce = false;
  if ((unsigned)a >= (unsigned)P.ny) {
    if (P.bc[2] == DW_BC_PERIODIC) a += cy > 0 ? P.ny : -P.ny;
    else { *bounce = true; a = j; }
  }
  if ((unsigned)b >= (unsigned)P.nz) {
    if (P.bc[4] == DW_BC_PERIODIC) b += cz > 0 ? P.nz : -P.nz;
    else { *bounce = true; b = k; }
  }
  *sj = a;
  *sk = b;
}

template <int Q>
__device__ __forceinline__ PullSrc pull_src(const LbmDev &P, int i, int j, int k) {
  constexpr int CX = LC[Q][0], CY = LC[Q][1], CZ = LC[Q][2];
  int sj = j, sk = k;
  bool bounce = false;
  if (CY != 0 || CZ != 0) row_source(P, j, k, CY, CZ, &sj, &sk, &bounce);
  int si = i - CX, wx = i - CX;
  bool inlet = false;
  if (CX != 0) {
    const bool xout = CX > 0 ? si < 0 : si >= P.nx;
    const int rule = P.bc[CX > 0 ? 0 : 1];
    if (rule == DW_BC_PERIODIC) {
      si = xout ? si + (CX > 0 ? P.nx : -P.nx) : si;
    } else {
      si = xout ? (CX > 0 ? 0 : P.nx - 1) : si;
      wx = xout ? i : wx;
      bounce = bounce || (xout && rule == DW_BC_BOUNCEBACK);
      inlet = CX > 0 && xout && rule == DW_BC_INLET;
    }
  }
  PullSrc s;
  s.src = (uint32_t)si + (uint32_t)P.nx * ((uint32_t)sj + (uint32_t)P.ny * (uint32_t)sk);
  s.kind = bounce ? SRC_BOUNCE : (inlet ? SRC_INLET : SRC_NORMAL);
  s.wx = wx;
  return s;
}

// Does the source of a normal pull hold a solid node?  SOL: 0 = no solid flag
// in the staged rows (so none on any source), 1 = look the flag up there.
template <int Q, int SOL>
__device__ __forceinline__ bool src_solid(const PullSrc &s, const uint8_t (*s_sol)[SOL_W], int x0) {
  constexpr int CY = LC[Q][1], CZ = LC[Q][2];
  if (SOL == 0) return false;
  return s_sol[(1 - CY) + 3 * (1 - CZ)][s.wx - x0 + 4] != 0;
}

// the inlet population of the five c_x = +1 directions for block row (j, k),
// staged by the block that holds x = 0 (threads 0..4)
__device__ __forceinline__ void stage_inlet(const LbmDev &P, int j, int k, float *s_inl) {
  if (threadIdx.x < 5) {
    const int q = INLET_Q[threadIdx.x];
    int sj, sk;
    bool bounce;
    row_source(P, j, k, LC[q][1], LC[q][2], &sj, &sk, &bounce);
    s_inl[threadIdx.x] = inlet_feq_shift(P, q, sj, sk);
  }
}

// Does the population of direction Q bounce back at this node (a bounce-back
// face, or a source on a solid node)?
template <int Q, int SOL>
__device__ __forceinline__ bool pull_bounces(const PullSrc &s, const uint8_t (*s_sol)[SOL_W], int x0) {
  const bool sf = src_solid<Q, SOL>(s, s_sol, x0);
  return s.kind == SRC_BOUNCE || (s.kind == SRC_NORMAL && sf);
}

// The value a population takes comes from plane Q at the source node or, on
// bounce-back, from plane LOPP[Q] at this node.  The two planes are adjacent
// (LOPP pairs q with q +- 1), so one 32-bit offset from the lower of them
// addresses either and the choice is a select: one load per population,
// issued once the bounce flags are known, and no load waits on another.
template <int Q>
__device__ __forceinline__ constexpr int pair_lo() {
  return Q < LOPP[Q] ? Q : LOPP[Q];
}

template <int Q, int SOL>
__device__ __forceinline__ uint32_t pull_offset(const LbmDev &P, const uint8_t (*s_sol)[SOL_W], int i, int j, int k,
                                                int x0, uint32_t node) {
  const PullSrc s = pull_src<Q>(P, i, j, k);
  const bool bb = pull_bounces<Q, SOL>(s, s_sol, x0);
  const uint32_t L = (uint32_t)P.L;
  return bb ? (uint32_t)(LOPP[Q] - pair_lo<Q>()) * L + node : (uint32_t)(Q - pair_lo<Q>()) * L + s.src;
}

// x-inlet lanes (x = 0 of an inlet row) take the staged inlet population
template <int Q>
__device__ __forceinline__ void pull_inlet(const LbmDev &P, const float *s_inl, int i, int j, int k, float &f) {
  if constexpr (inlet_slot(Q) >= 0) {
    if (pull_src<Q>(P, i, j, k).kind == SRC_INLET) f = s_inl[inlet_slot(Q)];
  }
}

template <int SOL, int... Qs>
__device__ __forceinline__ void pull_row(std::integer_sequence<int, Qs...>, const LbmDev &P,
                                         const float *__restrict__ fin, const uint8_t (*s_sol)[SOL_W],
                                         const float *s_inl, bool inlet_wave, int i, int j, int k, int x0,
                                         uint32_t node, float f[19]) {
  uint32_t off[19];
  ((off[Qs] = pull_offset<Qs, SOL>(P, s_sol, i, j, k, x0, node)), ...);
  ((f[Qs] = ld_node(fin + (size_t)pair_lo<Qs>() * P.L, off[Qs])), ...);
  if (inlet_wave) (pull_inlet<Qs>(P, s_inl, i, j, k, f[Qs]), ...);
}

__device__ __forceinline__ void moments(const LbmDev &P, const float f[19], float &rho, float &ux, float &uy,
                                        float &uz) {
  float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    drho += f[q];
    jx += LC[q][0] * f[q];
    jy += LC[q][1] * f[q];
    jz += LC[q][2] * f[q];
  }
  rho = 1.0f + drho;
  float ir = 1.0f / rho;
  ux = (jx + 0.5f * P.F[0]) * ir;
  uy = (jy + 0.5f * P.F[1]) * ir;
  uz = (jz + 0.5f * P.F[2]) * ir;
}

// Workgroups are handed to the 8 XCDs (each with its own L2) in turn, so
// consecutive block indices land on different XCDs.  The pull reads every
// node's populations from the 3 x 3 neighbouring rows; giving each XCD a
// contiguous run of rows (in y, then z) keeps those rows in its L2.
constexpr int N_XCD = 8;

struct RowBlock {
  int x0, j, k;
  bool live;
};

__device__ __forceinline__ RowBlock xcd_row_block(const LbmDev &P) {
  const int nbx = (P.nx + LBM_BLOCK - 1) / LBM_BLOCK;
  const int64_t nblocks = (int64_t)nbx * P.ny * P.nz;
  const int64_t per_xcd = (nblocks + N_XCD - 1) / N_XCD;
  const int64_t b = blockIdx.x;
  const int64_t logical = (b % N_XCD) * per_xcd + b / N_XCD;
  RowBlock r;
  r.live = logical < nblocks;
  const int64_t row = logical / nbx;
  r.x0 = (int)(logical % nbx) * LBM_BLOCK;
  r.j = (int)(row % P.ny);
  r.k = (int)(row / P.ny);
  return r;
}

static dim3 xcd_lbm_grid(const LbmDev &P) {
  const int64_t nbx = (P.nx + LBM_BLOCK - 1) / LBM_BLOCK;
  const int64_t nblocks = nbx * P.ny * P.nz;
  return dim3((unsigned)(((nblocks + N_XCD - 1) / N_XCD) * N_XCD));
}

// Lattices whose two population arrays exceed the 256 MB last-level cache
// (MALL) stream their output with nontemporal stores, which keep the next
// step's reads from being evicted; smaller lattices keep the output cached,
// since the next step reads it back from there.
constexpr double LBM_CACHE_BYTES = 256.0 * 1024 * 1024;

static bool lbm_streams(const LbmDev &P) { return 2.0 * 76.0 * (double)P.L > LBM_CACHE_BYTES; }

template <bool NT>
__device__ __forceinline__ void st_out(float *__restrict__ plane, uint32_t node, float v) {
  float *a = reinterpret_cast<float *>(reinterpret_cast<char *>(plane) + (node << 2));
  if constexpr (NT) __builtin_nontemporal_store(v, a);
  else *a = v;
}

// One row block of the step: LBM_BLOCK nodes along x from x0 in row (j, k).
// BIG: a lattice larger than the last-level cache (lbm_streams): the output
// is stored with nontemporal stores.  Lanes past the lattice's x end return
// after the block's staging barrier.
template <bool SOLID, bool BIG>
__device__ __forceinline__ void lbm_row_block(const LbmDev &P, const float *__restrict__ fin,
                                              float *__restrict__ fout, const uint8_t *__restrict__ solid,
                                              float *__restrict__ rho_out, float *__restrict__ u_out, int x0, int j,
                                              int k, uint8_t (*s_sol)[SOL_W], int *s_any, float *s_inl) {
  const int i = x0 + threadIdx.x;
  if (i == 0 && j == 0 && k == 0 && P.t_out) *P.t_out = (P.t_in ? *P.t_in : P.t) + 1;
  const uint32_t node = (uint32_t)i + (uint32_t)P.nx * ((uint32_t)j + (uint32_t)P.ny * (uint32_t)k);
  float f[19];
  // the row's x = 0 block stages the inlet populations (block-uniform)
  const bool inlet_row = x0 == 0 && P.bc[0] == DW_BC_INLET;
  if (inlet_row) stage_inlet(P, j, k, s_inl);
  // any solid flag in the staged rows?  Most blocks have none and take the
  // plain pull (block-uniform branch).
  bool any = false;
  if (SOLID) {
    uint32_t sv[SOL_PER_THREAD];
    load_solid_rows(P, solid, x0, j, k, sv);
    store_solid_rows(sv, s_sol);
    uint32_t mine = 0;
#pragma unroll
    for (int u = 0; u < SOL_PER_THREAD; ++u) mine |= sv[u];
    const bool wave_any = __ballot(mine != 0) != 0ull;
    if ((threadIdx.x & 63) == 0) s_any[threadIdx.x >> 6] = wave_any;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < LBM_BLOCK / 64; ++w) any = any || s_any[w] != 0;
  } else if (inlet_row) {
    __syncthreads();
  }
  if (i >= P.nx) return;
  // A solid node outputs the rest state (f = w, u = 0, rho = 1).  It runs
  // the pull with its neighbours and only its stores are replaced, so the
  // lanes of a wave write their cache lines together.
  const bool solid_node = any && s_sol[4][i - x0 + 4] != 0;
  // wave-uniform: the first wave of an inlet row's x = 0 block holds the inlet lane
  const bool inlet_wave = inlet_row && threadIdx.x < 64;
  if (any) pull_row<1>(std::make_integer_sequence<int, 19>{}, P, fin, s_sol, s_inl, inlet_wave, i, j, k, x0, node, f);
  else pull_row<0>(std::make_integer_sequence<int, 19>{}, P, fin, s_sol, s_inl, inlet_wave, i, j, k, x0, node, f);
  float rho, ux, uy, uz;
  moments(P, f, rho, ux, uy, uz);
  const float drho = rho - 1.0f;
  const float uu = ux * ux + uy * uy + uz * uz;
  const float om = P.omega;
  // BGK against the shifted equilibrium W (drho + rho (3 cu + 4.5 cu^2 -
  // 1.5 u.u)), a direction and its opposite together: they share the even
  // part W (c0 + 4.5 rho cu^2) and differ in the sign of the odd part
  // 3 W rho cu.
  const float c0 = drho - 1.5f * rho * uu;
  const float r45 = 4.5f * rho, r3 = 3.0f * rho;
  float g[19];
  g[0] = f[0] + om * (LW[0] * c0 - f[0]);
#pragma unroll
  for (int q = 1; q < 19; q += 2) {
    const float cu = LC[q][0] * ux + LC[q][1] * uy + LC[q][2] * uz;
    const float ev = LW[q] * fmaf(r45 * cu, cu, c0);
    const float od = (LW[q] * r3) * cu;
    g[q] = f[q] + om * ((ev + od) - f[q]);
    g[q + 1] = f[q + 1] + om * ((ev - od) - f[q + 1]);
  }
  if (P.forced) {
    const float kf = 1.0f - 0.5f * om;
    const float uF = ux * P.F[0] + uy * P.F[1] + uz * P.F[2];
#pragma unroll
    for (int q = 1; q < 19; ++q) {
      const float cu = LC[q][0] * ux + LC[q][1] * uy + LC[q][2] * uz;
      const float cF = LC[q][0] * P.F[0] + LC[q][1] * P.F[1] + LC[q][2] * P.F[2];
      g[q] += kf * LW[q] * (3.f * (cF - uF) + 9.f * cu * cF);
    }
    g[0] += kf * LW[0] * (-3.f * uF);
  }
#pragma unroll
  for (int q = 0; q < 19; ++q) st_out<BIG>(fout + (size_t)q * P.L, node, solid_node ? 0.f : g[q]);
  if (rho_out) st_out<BIG>(rho_out, node, solid_node ? 1.f : rho);
  if (u_out) {
    st_out<BIG>(u_out, node, solid_node ? 0.f : ux);
    st_out<BIG>(u_out + P.L, node, solid_node ? 0.f : uy);
    st_out<BIG>(u_out + 2 * P.L, node, solid_node ? 0.f : uz);
  }
}

// One workgroup per row block.  Large lattices (BIG): a 3-D grid of row
// blocks; otherwise rows are handed to the XCDs in contiguous runs
// (xcd_row_block) and the output stays cached.  Eight waves per SIMD: the
// plane bases it would otherwise keep in scalar registers limit it to seven
// (some spill to vector-register lanes instead).
template <bool SOLID, bool BIG>
__global__ __launch_bounds__(LBM_BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void k_lbm_step(
    LbmDev P, const float *__restrict__ fin, float *__restrict__ fout, const uint8_t *__restrict__ solid,
    float *__restrict__ rho_out, float *__restrict__ u_out) {
  __shared__ __attribute__((aligned(4))) uint8_t s_sol[9][SOL_W];
  __shared__ int s_any[LBM_BLOCK / 64];
  __shared__ float s_inl[5];
  int x0, j, k;
  if (BIG) {
    x0 = blockIdx.x * LBM_BLOCK;
    j = blockIdx.y;
    k = blockIdx.z;
  } else {
    const RowBlock rb = xcd_row_block(P);
    if (!rb.live) return;  // block-uniform
    x0 = rb.x0;
    j = rb.j;
    k = rb.k;
  }
  lbm_row_block<SOLID, BIG>(P, fin, fout, solid, rho_out, u_out, x0, j, k, s_sol, s_any, s_inl);
}

// The step behind a device switch (dw_lbm_params.skip, e.g. a fallback
// branch of a captured graph): a bounded grid whose workgroups stride over
// the row blocks, so a switched-off step costs a few thousand workgroups
// that return at once instead of one per row block.
constexpr unsigned LBM_GATED_BLOCKS = 2048;

template <bool SOLID, bool BIG>
__global__ __launch_bounds__(LBM_BLOCK) void k_lbm_step_gated(LbmDev P, const float *__restrict__ fin,
                                                              float *__restrict__ fout,
                                                              const uint8_t *__restrict__ solid,
                                                              float *__restrict__ rho_out, float *__restrict__ u_out) {
  __shared__ __attribute__((aligned(4))) uint8_t s_sol[9][SOL_W];
  __shared__ int s_any[LBM_BLOCK / 64];
  __shared__ float s_inl[5];
  if (*P.skip) return;  // grid-uniform
  const int nbx = (P.nx + LBM_BLOCK - 1) / LBM_BLOCK;
  const int64_t nblocks = (int64_t)nbx * P.ny * P.nz;
  for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
    const int64_t row = b / nbx;
    lbm_row_block<SOLID, BIG>(P, fin, fout, solid, rho_out, u_out, (int)(b % nbx) * LBM_BLOCK, (int)(row % P.ny),
                              (int)(row / P.ny), s_sol, s_any, s_inl);
    __syncthreads();  // the next row block restages the shared rows
  }
}

// ------------------------------------------------------------- HOME-LBM
// Moment-encoded step (appendix on HOME-LBM): a node stores its
// post-collision moments, [HM_N][L] = rho - 1, u (3), S (6: xx yy zz xy xz
// yz) with rho S_ab = sum_i (c_a c_b - delta_ab / 3) f_i.  The step pulls,
// for each direction q, the population f_q of the source node rebuilt from
// the source's moments by the third-order Hermite expansion, accumulates the
// moments of the pulled set on the fly (no population is stored), and
// relaxes them in moment space.  40 bytes per node in and out instead of
// the 76 + 76 of the population form.
constexpr int HM_N = 10;

struct Mom {
  float drho, u[3], S[6];  // S: xx yy zz xy xz yz
};

// storage index of S_ab
__host__ __device__ constexpr int sidx(int a, int b) {
  return a == b ? a : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5));
}

// a3_aab = S_aa u_b + 2 S_ab u_a - 2 u_a^2 u_b
template <int A, int B>
__device__ __forceinline__ float home_a3(const Mom &M) {
  return M.S[sidx(A, A)] * M.u[B] + 2.f * M.S[sidx(A, B)] * M.u[A] - 2.f * M.u[A] * M.u[A] * M.u[B];
}

// f_q - w_q of the expansion
//   f_q = w_q rho [1 + 3 c.u + 9/2 H2(c):S + 27/2 sum_(a,a,b) (c_a^2 - 1/3) c_b a3_aab]
// terms with a zero velocity factor are dropped at compile time
// the bracket s of f_q = w_q rho [1 + s]
template <int Q>
__device__ __forceinline__ float home_series(const Mom &M) {
  constexpr int c[3] = {LC[Q][0], LC[Q][1], LC[Q][2]};
  constexpr float h[3] = {c[0] * c[0] - 1.f / 3.f, c[1] * c[1] - 1.f / 3.f, c[2] * c[2] - 1.f / 3.f};
  float s = 4.5f * (h[0] * M.S[0] + h[1] * M.S[1] + h[2] * M.S[2]);
  if constexpr (c[0] != 0) s += 3.f * c[0] * M.u[0];
  if constexpr (c[1] != 0) s += 3.f * c[1] * M.u[1];
  if constexpr (c[2] != 0) s += 3.f * c[2] * M.u[2];
  if constexpr (c[0] * c[1] != 0) s += 9.f * (c[0] * c[1]) * M.S[3];
  if constexpr (c[0] * c[2] != 0) s += 9.f * (c[0] * c[2]) * M.S[4];
  if constexpr (c[1] * c[2] != 0) s += 9.f * (c[1] * c[2]) * M.S[5];
  float t = 0.f;
  if constexpr (c[1] != 0) t += c[1] * (h[0] * home_a3<0, 1>(M) + h[2] * home_a3<2, 1>(M));
  if constexpr (c[0] != 0) t += c[0] * (h[1] * home_a3<1, 0>(M) + h[2] * home_a3<2, 0>(M));
  if constexpr (c[2] != 0) t += c[2] * (h[0] * home_a3<0, 2>(M) + h[1] * home_a3<1, 2>(M));
  s += 13.5f * t;
  return s;
}

template <int Q>
__device__ __forceinline__ float home_pop(const Mom &M) {
  return LW[Q] * (M.drho + (1.f + M.drho) * home_series<Q>(M));
}

// reverse of a3_aab = S_aa u_b + 2 S_ab u_a - 2 u_a^2 u_b, adjoint ab
template <int A, int B>
__device__ __forceinline__ void home_a3_adj(const Mom &M, float ab, Mom &Mb) {
  Mb.S[sidx(A, A)] += ab * M.u[B];
  Mb.S[sidx(A, B)] += 2.f * ab * M.u[A];
  Mb.u[B] += ab * (M.S[sidx(A, A)] - 2.f * M.u[A] * M.u[A]);
  Mb.u[A] += ab * (2.f * M.S[sidx(A, B)] - 4.f * M.u[A] * M.u[B]);
}

// reverse of home_pop<Q>: adds pb * d(f_q - w_q)/dM into Mb
template <int Q>
__device__ __forceinline__ void home_pop_adj(const Mom &M, float pb, Mom &Mb) {
  constexpr int c[3] = {LC[Q][0], LC[Q][1], LC[Q][2]};
  constexpr float h[3] = {c[0] * c[0] - 1.f / 3.f, c[1] * c[1] - 1.f / 3.f, c[2] * c[2] - 1.f / 3.f};
  Mb.drho += pb * LW[Q] * (1.f + home_series<Q>(M));
  const float sb = pb * LW[Q] * (1.f + M.drho);
#pragma unroll
  for (int a = 0; a < 3; ++a) Mb.S[a] += 4.5f * h[a] * sb;
  if constexpr (c[0] != 0) Mb.u[0] += 3.f * c[0] * sb;
  if constexpr (c[1] != 0) Mb.u[1] += 3.f * c[1] * sb;
  if constexpr (c[2] != 0) Mb.u[2] += 3.f * c[2] * sb;
  if constexpr (c[0] * c[1] != 0) Mb.S[3] += 9.f * (c[0] * c[1]) * sb;
  if constexpr (c[0] * c[2] != 0) Mb.S[4] += 9.f * (c[0] * c[2]) * sb;
  if constexpr (c[1] * c[2] != 0) Mb.S[5] += 9.f * (c[1] * c[2]) * sb;
  const float tb = 13.5f * sb;
  if constexpr (c[1] != 0) {
    home_a3_adj<0, 1>(M, tb * c[1] * h[0], Mb);
    home_a3_adj<2, 1>(M, tb * c[1] * h[2], Mb);
  }
  if constexpr (c[0] != 0) {
    home_a3_adj<1, 0>(M, tb * c[0] * h[1], Mb);
    home_a3_adj<2, 0>(M, tb * c[0] * h[2], Mb);
  }
  if constexpr (c[2] != 0) {
    home_a3_adj<0, 2>(M, tb * c[2] * h[0], Mb);
    home_a3_adj<1, 2>(M, tb * c[2] * h[1], Mb);
  }
}

// moments of the pulled set, accumulated direction by direction
struct MomAcc {
  float drho = 0.f, j[3] = {0.f, 0.f, 0.f}, P[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
};

template <int Q>
__device__ __forceinline__ void acc_pop(MomAcc &A, float g) {
  constexpr int c[3] = {LC[Q][0], LC[Q][1], LC[Q][2]};
  A.drho += g;
  if constexpr (c[0] != 0) A.j[0] += c[0] * g;
  if constexpr (c[1] != 0) A.j[1] += c[1] * g;
  if constexpr (c[2] != 0) A.j[2] += c[2] * g;
  // sum H2_ab g (the weights' part sums to zero)
  A.P[0] += (c[0] * c[0] - 1.f / 3.f) * g;
  A.P[1] += (c[1] * c[1] - 1.f / 3.f) * g;
  A.P[2] += (c[2] * c[2] - 1.f / 3.f) * g;
  if constexpr (c[0] * c[1] != 0) A.P[3] += (c[0] * c[1]) * g;
  if constexpr (c[0] * c[2] != 0) A.P[4] += (c[0] * c[2]) * g;
  if constexpr (c[1] * c[2] != 0) A.P[5] += (c[1] * c[2]) * g;
}

// equilibrium moments of an inlet ghost node at inlet-plane (j, k)
__device__ __forceinline__ Mom inlet_mom(const LbmDev &P, int j, int k) {
  const float sfac = gust_factor(P, j, k);
  Mom M;
  M.drho = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) M.u[a] = P.uin[a] * sfac;
#pragma unroll
  for (int a = 0; a < 3; ++a) M.S[a] = M.u[a] * M.u[a];
  M.S[3] = M.u[0] * M.u[1];
  M.S[4] = M.u[0] * M.u[2];
  M.S[5] = M.u[1] * M.u[2];
  return M;
}

// Forward pull of the moment-encoded step with the row-uniform source rules
// and 32-bit offsets of the population step: every bounce decision comes
// from the staged flags first, then each source's ten moments are loaded
// from scalar plane bases (one offset per source) and expanded.
__device__ __forceinline__ Mom load_mom_at(const float *__restrict__ m, size_t L, uint32_t node) {
  Mom M;
  M.drho = ld_node(m, node);
#pragma unroll
  for (int a = 0; a < 3; ++a) M.u[a] = ld_node(m + (1 + a) * L, node);
#pragma unroll
  for (int s = 0; s < 6; ++s) M.S[s] = ld_node(m + (4 + s) * L, node);
  return M;
}

// inlet population of direction INLET_Q[t] for block row (j, k)
__device__ __forceinline__ float home_inlet_pop(const LbmDev &P, int t, int j, int k) {
  const int q = INLET_Q[t];
  int sj, sk;
  bool bounce;
  row_source(P, j, k, LC[q][1], LC[q][2], &sj, &sk, &bounce);
  const Mom M = inlet_mom(P, sj, sk);
  switch (t) {
    case 0: return home_pop<1>(M);
    case 1: return home_pop<7>(M);
    case 2: return home_pop<9>(M);
    case 3: return home_pop<13>(M);
    default: return home_pop<15>(M);
  }
}

template <int SOL, int Q>
__device__ __forceinline__ void home_pull_row(const LbmDev &P, const float *__restrict__ min, const float *s_inl,
                                              bool inlet_wave, int i, int j, int k, const Mom &own, bool bb,
                                              MomAcc &A) {
  float g;
  if constexpr (Q == 0) {
    g = home_pop<0>(own);
  } else {
    const PullSrc s = pull_src<Q>(P, i, j, k);
    g = home_pop<Q>(load_mom_at(min, P.L, s.src));
    if (bb) g = home_pop<LOPP[Q]>(own);
    if constexpr (inlet_slot(Q) >= 0) {
      if (inlet_wave && s.kind == SRC_INLET) g = s_inl[inlet_slot(Q)];
    }
  }
  acc_pop<Q>(A, g);
}

template <int SOL, int... Qs>
__device__ __forceinline__ void home_row_all(std::integer_sequence<int, Qs...>, const LbmDev &P,
                                             const float *__restrict__ min, const uint8_t (*s_sol)[SOL_W],
                                             const float *s_inl, bool inlet_wave, int i, int j, int k, int x0,
                                             const Mom &own, MomAcc &A) {
  bool bb[19];
  ((bb[Qs] = pull_bounces<Qs, SOL>(pull_src<Qs>(P, i, j, k), s_sol, x0)), ...);
  (home_pull_row<SOL, Qs>(P, min, s_inl, inlet_wave, i, j, k, own, bb[Qs], A), ...);
}

template <bool SOLID>
__global__ __launch_bounds__(LBM_BLOCK) void k_home_step(LbmDev P, const float *__restrict__ min,
                                                         float *__restrict__ mout, const uint8_t *__restrict__ solid,
                                                         float *__restrict__ rho_out, float *__restrict__ u_out) {
  __shared__ __attribute__((aligned(4))) uint8_t s_sol[9][SOL_W];
  __shared__ int s_any[LBM_BLOCK / 64];
  __shared__ float s_inl[5];
  const RowBlock rb = xcd_row_block(P);
  if (!rb.live) return;  // block-uniform: padding blocks of the last XCD
  const int x0 = rb.x0;
  const int i = x0 + threadIdx.x, j = rb.j, k = rb.k;
  if (i == 0 && j == 0 && k == 0 && P.t_out) *P.t_out = (P.t_in ? *P.t_in : P.t) + 1;
  const uint32_t node = (uint32_t)i + (uint32_t)P.nx * ((uint32_t)j + (uint32_t)P.ny * (uint32_t)k);
  // the row's x = 0 block stages the inlet populations (block-uniform)
  const bool inlet_row = x0 == 0 && P.bc[0] == DW_BC_INLET;
  if (inlet_row && threadIdx.x < 5) s_inl[threadIdx.x] = home_inlet_pop(P, threadIdx.x, j, k);
  bool any = false;
  if (SOLID) {
    uint32_t sv[SOL_PER_THREAD];
    load_solid_rows(P, solid, x0, j, k, sv);
    store_solid_rows(sv, s_sol);
    uint32_t mine = 0;
#pragma unroll
    for (int u = 0; u < SOL_PER_THREAD; ++u) mine |= sv[u];
    const bool wave_any = __ballot(mine != 0) != 0ull;
    if ((threadIdx.x & 63) == 0) s_any[threadIdx.x >> 6] = wave_any;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < LBM_BLOCK / 64; ++w) any = any || s_any[w] != 0;
  } else if (inlet_row) {
    __syncthreads();
  }
  if (i >= P.nx) return;
  // a solid node outputs the rest state; it runs with its wave and only its
  // stores are replaced, so the lanes of a wave write their lines together
  const bool solid_node = any && s_sol[4][i - x0 + 4] != 0;
  const bool inlet_wave = inlet_row && threadIdx.x < 64;  // wave-uniform
  const Mom own = load_mom_at(min, P.L, node);
  MomAcc A;
  if (any) home_row_all<1>(std::make_integer_sequence<int, 19>{}, P, min, s_sol, s_inl, inlet_wave, i, j, k, x0, own, A);
  else home_row_all<0>(std::make_integer_sequence<int, 19>{}, P, min, s_sol, s_inl, inlet_wave, i, j, k, x0, own, A);
  // moments of the pulled set: u* carries half the force
  const float rho = 1.f + A.drho, ir = 1.f / rho;
  float u[3], Fu = 0.f, uu = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = (A.j[a] + 0.5f * P.F[a]) * ir;
    Fu += P.F[a] * u[a];
    uu += u[a] * u[a];
  }
  float S[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) S[s] = A.P[s] * ir;
  // moment-space collision: deviatoric part relaxes with 1/tau towards
  // dev(u u), the trace is set to |u|^2, Guo's source for the force
  const float om = P.omega, keep = 1.f - om;
  const float tr3 = (S[0] + S[1] + S[2]) * (1.f / 3.f), uu3 = uu * (1.f / 3.f);
  float Sn[6];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    Sn[a] = keep * (S[a] - tr3) + om * (u[a] * u[a] - uu3) + uu3 +
            (P.F[a] * u[a] + keep * (P.F[a] * u[a] - Fu * (1.f / 3.f))) * ir;
  const float kf = (1.f - 0.5f * om) * ir;
  Sn[3] = keep * S[3] + om * u[0] * u[1] + kf * (P.F[0] * u[1] + P.F[1] * u[0]);
  Sn[4] = keep * S[4] + om * u[0] * u[2] + kf * (P.F[0] * u[2] + P.F[2] * u[0]);
  Sn[5] = keep * S[5] + om * u[1] * u[2] + kf * (P.F[1] * u[2] + P.F[2] * u[1]);
  st_node(mout, node, solid_node ? 0.f : A.drho);
#pragma unroll
  for (int a = 0; a < 3; ++a) st_node(mout + (size_t)(1 + a) * P.L, node, solid_node ? 0.f : u[a] + 0.5f * P.F[a] * ir);
#pragma unroll
  for (int s = 0; s < 6; ++s) st_node(mout + (size_t)(4 + s) * P.L, node, solid_node ? 0.f : Sn[s]);
  if (rho_out) st_node(rho_out, node, solid_node ? 1.f : rho);
  if (u_out) {
#pragma unroll
    for (int a = 0; a < 3; ++a) st_node(u_out + (size_t)a * P.L, node, solid_node ? 0.f : u[a]);
  }
}

// equilibrium moments (rho, u, S = u u) from rho [L] and u [3][L] (either
// may be absent: rho = 1, u = the inflow velocity)
__global__ __launch_bounds__(256) void k_home_equilibrium(LbmDev P, const float *__restrict__ rho_in,
                                                          const float *__restrict__ u_in, float *__restrict__ m) {
  int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= P.L) return;
  float u[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = u_in ? u_in[a * P.L + node] : P.uin[a];
  m[node] = rho_in ? rho_in[node] - 1.f : 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    m[(1 + a) * P.L + node] = u[a];
    m[(4 + a) * P.L + node] = u[a] * u[a];
  }
  m[7 * P.L + node] = u[0] * u[1];
  m[8 * P.L + node] = u[0] * u[2];
  m[9 * P.L + node] = u[1] * u[2];
}

// ------------------------------------------------------- HOME-LBM reverse
// Reverse of k_home_step in two passes, neither with atomics.
//  1. k_home_adj_pull, per node: recompute the pulled set's moments, take
//     the adjoints of the stored moments (and of the reported u*) back
//     through the moment collision, and write the adjoint of each of the 19
//     pulled populations to gbar [19][L] (zeros at a solid node: its stored
//     rest state does not depend on the inputs).
//  2. k_adj_gather, per node s: population p rebuilt from the moments
//     of s was pulled either by the node at s + c_p (the transposed
//     streaming, same boundary rules) or, where the pull of opp(p) at s
//     bounced back, by s itself.  T_p gathers gbar_p of the first or
//     gbar_opp(p) of s, and sum_p T_p df_p/dM(s) is added into m_in_bar.
// Every node's m_in_bar is written by one thread, in a fixed order.

struct PopBar {
  float drho, j[3], P[6];  // adjoints of the pulled set's moments
};

// adjoints of the pulled set's moments from those of the stored moments
// (mb) and of the reported u* (ubo), through the collision of k_home_step
__device__ __forceinline__ PopBar home_collision_adj(const LbmDev &P, const MomAcc &A, const float mb[HM_N],
                                                     const float ubo[3]) {
  const float rho = 1.f + A.drho, ir = 1.f / rho;
  float u[3], Fu = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = (A.j[a] + 0.5f * P.F[a]) * ir;
    Fu += P.F[a] * u[a];
  }
  const float om = P.omega, keep = 1.f - om, kf = 1.f - 0.5f * om;
  float Sb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, ub[3] = {0.f, 0.f, 0.f}, irb = 0.f;
  // diagonal S: keep (S_a - tr/3) + om (u_a^2 - |u|^2/3) + |u|^2/3
  //             + (F_a u_a + keep (F_a u_a - F.u/3)) ir
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float sb = mb[4 + a];
    Sb[a] += keep * sb;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      Sb[b] -= keep * sb * (1.f / 3.f);
      ub[b] += sb * keep * 2.f * u[b] * (1.f / 3.f) - sb * keep * P.F[b] * (1.f / 3.f) * ir;
    }
    ub[a] += sb * (2.f * om * u[a] + (1.f + keep) * P.F[a] * ir);
    irb += sb * (P.F[a] * u[a] + keep * (P.F[a] * u[a] - Fu * (1.f / 3.f)));
  }
  // off-diagonal S: keep S_ab + om u_a u_b + kf ir (F_a u_b + F_b u_a)
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int a = pa[e], b = pb[e];
    const float sb = mb[7 + e];
    Sb[3 + e] += keep * sb;
    ub[a] += sb * (om * u[b] + kf * ir * P.F[b]);
    ub[b] += sb * (om * u[a] + kf * ir * P.F[a]);
    irb += sb * kf * (P.F[a] * u[b] + P.F[b] * u[a]);
  }
  // stored u = u* + F / (2 rho), reported u*
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ub[a] += mb[1 + a] + ubo[a];
    irb += mb[1 + a] * 0.5f * P.F[a];
  }
  // S = P ir, u = (j + F/2) ir, ir = 1 / (1 + drho)
  PopBar B;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    B.P[s] = Sb[s] * ir;
    irb += Sb[s] * A.P[s];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    B.j[a] = ub[a] * ir;
    irb += ub[a] * (A.j[a] + 0.5f * P.F[a]);
  }
  B.drho = mb[0] - irb * ir * ir;
  return B;
}

// adjoint of pulled population Q: the pulled set's moments are linear in it
template <int Q>
__device__ __forceinline__ float pop_bar(const PopBar &B) {
  constexpr int c[3] = {LC[Q][0], LC[Q][1], LC[Q][2]};
  float gb = B.drho;
  if constexpr (c[0] != 0) gb += c[0] * B.j[0];
  if constexpr (c[1] != 0) gb += c[1] * B.j[1];
  if constexpr (c[2] != 0) gb += c[2] * B.j[2];
  gb += (c[0] * c[0] - 1.f / 3.f) * B.P[0] + (c[1] * c[1] - 1.f / 3.f) * B.P[1] + (c[2] * c[2] - 1.f / 3.f) * B.P[2];
  if constexpr (c[0] * c[1] != 0) gb += (c[0] * c[1]) * B.P[3];
  if constexpr (c[0] * c[2] != 0) gb += (c[0] * c[2]) * B.P[4];
  if constexpr (c[1] * c[2] != 0) gb += (c[1] * c[2]) * B.P[5];
  return gb;
}

template <int... Qs>
__device__ __forceinline__ void store_pop_bars(std::integer_sequence<int, Qs...>, const LbmDev &P,
                                               float *__restrict__ gbar, uint32_t node, const PopBar &B, bool zero) {
  (st_node(gbar + (size_t)Qs * P.L, node, zero ? 0.f : pop_bar<Qs>(B)), ...);
}

// Solid flags of the 3 x 3 rows around the block's row into LDS; true if any
// is set (block-uniform; has a barrier).
__device__ __forceinline__ bool stage_solid(const LbmDev &P, const uint8_t *__restrict__ solid, int x0, int j, int k,
                                            uint8_t (*s_sol)[SOL_W], int *s_any) {
  uint32_t sv[SOL_PER_THREAD];
  load_solid_rows(P, solid, x0, j, k, sv);
  store_solid_rows(sv, s_sol);
  uint32_t mine = 0;
#pragma unroll
  for (int u = 0; u < SOL_PER_THREAD; ++u) mine |= sv[u];
  const bool wave_any = __ballot(mine != 0) != 0ull;
  if ((threadIdx.x & 63) == 0) s_any[threadIdx.x >> 6] = wave_any;
  __syncthreads();
  bool any = false;
#pragma unroll
  for (int w = 0; w < LBM_BLOCK / 64; ++w) any = any || s_any[w] != 0;
  return any;
}

template <bool SOLID>
__global__ __launch_bounds__(LBM_BLOCK) void k_home_adj_pull(LbmDev P, const float *__restrict__ min,
                                                             const uint8_t *__restrict__ solid,
                                                             const float *__restrict__ mout_bar,
                                                             const float *__restrict__ ubar_out,
                                                             float *__restrict__ gbar) {
  __shared__ __attribute__((aligned(4))) uint8_t s_sol[9][SOL_W];
  __shared__ int s_any[LBM_BLOCK / 64];
  __shared__ float s_inl[5];
  const RowBlock rb = xcd_row_block(P);
  if (!rb.live) return;  // block-uniform
  const int x0 = rb.x0;
  const int i = x0 + threadIdx.x, j = rb.j, k = rb.k;
  const uint32_t node = (uint32_t)i + (uint32_t)P.nx * ((uint32_t)j + (uint32_t)P.ny * (uint32_t)k);
  const bool inlet_row = x0 == 0 && P.bc[0] == DW_BC_INLET;
  if (inlet_row && threadIdx.x < 5) s_inl[threadIdx.x] = home_inlet_pop(P, threadIdx.x, j, k);
  bool any = false;
  if (SOLID) any = stage_solid(P, solid, x0, j, k, s_sol, s_any);
  else if (inlet_row) __syncthreads();
  if (i >= P.nx) return;
  const bool solid_node = any && s_sol[4][i - x0 + 4] != 0;
  const bool inlet_wave = inlet_row && threadIdx.x < 64;  // wave-uniform
  const Mom own = load_mom_at(min, P.L, node);
  MomAcc A;
  if (any) home_row_all<1>(std::make_integer_sequence<int, 19>{}, P, min, s_sol, s_inl, inlet_wave, i, j, k, x0, own, A);
  else home_row_all<0>(std::make_integer_sequence<int, 19>{}, P, min, s_sol, s_inl, inlet_wave, i, j, k, x0, own, A);
  float mb[HM_N], ubo[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < HM_N; ++q) mb[q] = ld_node(mout_bar + (size_t)q * P.L, node);
  if (ubar_out) {
#pragma unroll
    for (int a = 0; a < 3; ++a) ubo[a] = ld_node(ubar_out + (size_t)a * P.L, node);
  }
  store_pop_bars(std::make_integer_sequence<int, 19>{}, P, gbar, node, home_collision_adj(P, A, mb, ubo), solid_node);
}

// Where T_Q of this node comes from: the node at +c_Q pulled population Q
// from here (the source rules of pull_src<opp(Q)> find it), unless the pull
// of opp(Q) here bounced (then gbar_opp(Q) of this node) or came from an
// inlet ghost or an outlet clamp (no node at +c_Q: T_Q = 0).  Planes Q and
// opp(Q) are adjacent, so one offset from the lower addresses either.
template <int Q, int SOL>
__device__ __forceinline__ uint32_t push_offset(const LbmDev &P, const uint8_t (*s_sol)[SOL_W], int i, int j, int k,
                                                int x0, uint32_t node, bool &live) {
  constexpr int R = LOPP[Q];
  const PullSrc s = pull_src<R>(P, i, j, k);
  const bool bb = pull_bounces<R, SOL>(s, s_sol, x0);
  const bool clamped = LC[Q][0] > 0 && i == P.nx - 1 && P.bc[1] == DW_BC_OUTLET;
  live = bb || (s.kind == SRC_NORMAL && !clamped);
  const uint32_t L = (uint32_t)P.L;
  return bb ? (uint32_t)(R - pair_lo<Q>()) * L + node : (uint32_t)(Q - pair_lo<Q>()) * L + s.src;
}

// At the last x of an outlet the pull of each c_x = -1 direction Q by node
// (nx - 1, j + c_Q.y, k + c_Q.z) was clamped onto this node.
template <int Q>
__device__ __forceinline__ void outlet_extra(const LbmDev &P, const float *__restrict__ gbar, int j, int k,
                                             float &T) {
  if constexpr (LC[Q][0] < 0) {
    int sj, sk;
    bool bounce;
    row_source(P, j, k, -LC[Q][1], -LC[Q][2], &sj, &sk, &bounce);
    if (!bounce)
      T += ld_node(gbar + (size_t)Q * P.L,
                   (uint32_t)(P.nx - 1) + (uint32_t)P.nx * ((uint32_t)sj + (uint32_t)P.ny * (uint32_t)sk));
  }
}

template <int SOL, int... Qs>
__device__ __forceinline__ void gather_row(std::integer_sequence<int, Qs...>, const LbmDev &P,
                                           const float *__restrict__ gbar, const uint8_t (*s_sol)[SOL_W], int i,
                                           int j, int k, int x0, uint32_t node, float T[19]) {
  uint32_t off[19];
  bool live[19];
  ((off[Qs] = push_offset<Qs, SOL>(P, s_sol, i, j, k, x0, node, live[Qs])), ...);
  ((T[Qs] = ld_node(gbar + (size_t)pair_lo<Qs>() * P.L, off[Qs])), ...);
  ((T[Qs] = live[Qs] ? T[Qs] : 0.f), ...);
  if (i == P.nx - 1 && P.bc[1] == DW_BC_OUTLET) (outlet_extra<Qs>(P, gbar, j, k, T[Qs]), ...);
}

template <int... Qs>
__device__ __forceinline__ void pops_adj(std::integer_sequence<int, Qs...>, const Mom &M, const float T[19],
                                         Mom &Mb) {
  (home_pop_adj<Qs>(M, T[Qs], Mb), ...);
}

// Pass 2 of both reverse steps, per node: T_p gathered as above, then for
// HOME (bar = m_in_bar [10][L]) sum_p T_p df_p/dM taken through the Hermite
// expansion of this node's moments, for BGK (bar = f_in_bar [19][L]) T_p
// itself.  A solid node's state feeds no population: it adds nothing.
template <bool SOLID, bool HOME>
__global__ __launch_bounds__(LBM_BLOCK) void k_adj_gather(LbmDev P, const float *__restrict__ min,
                                                          const uint8_t *__restrict__ solid,
                                                          const float *__restrict__ gbar, float *__restrict__ bar) {
  __shared__ __attribute__((aligned(4))) uint8_t s_sol[9][SOL_W];
  __shared__ int s_any[LBM_BLOCK / 64];
  const RowBlock rb = xcd_row_block(P);
  if (!rb.live) return;  // block-uniform
  const int x0 = rb.x0;
  const int i = x0 + threadIdx.x, j = rb.j, k = rb.k;
  const uint32_t node = (uint32_t)i + (uint32_t)P.nx * ((uint32_t)j + (uint32_t)P.ny * (uint32_t)k);
  const bool any = SOLID && stage_solid(P, solid, x0, j, k, s_sol, s_any);
  if (i >= P.nx) return;
  const bool solid_node = any && s_sol[4][i - x0 + 4] != 0;
  float T[19];
  if (any) gather_row<1>(std::make_integer_sequence<int, 19>{}, P, gbar, s_sol, i, j, k, x0, node, T);
  else gather_row<0>(std::make_integer_sequence<int, 19>{}, P, gbar, s_sol, i, j, k, x0, node, T);
  if constexpr (HOME) {
    const Mom own = load_mom_at(min, P.L, node);
    Mom Mb{};
    pops_adj(std::make_integer_sequence<int, 19>{}, own, T, Mb);
    const float v[HM_N] = {Mb.drho, Mb.u[0], Mb.u[1], Mb.u[2], Mb.S[0], Mb.S[1], Mb.S[2], Mb.S[3], Mb.S[4], Mb.S[5]};
#pragma unroll
    for (int q = 0; q < HM_N; ++q) {
      float *plane = bar + (size_t)q * P.L;
      st_node(plane, node, ld_node(plane, node) + (solid_node ? 0.f : v[q]));
    }
  } else {
#pragma unroll
    for (int q = 0; q < 19; ++q) {
      float *plane = bar + (size_t)q * P.L;
      st_node(plane, node, ld_node(plane, node) + (solid_node ? 0.f : T[q]));
    }
  }
}

// Reverse of k_lbm_step, pass 1 (pass 2 is k_adj_gather): per node,
// recompute the pulled populations and moments and write the adjoint of each
// pulled population through the BGK collision to fbar [19][L] (zeros at a
// solid node, whose stored rest state does not depend on the inputs).
template <bool SOLID>
__global__ __launch_bounds__(LBM_BLOCK) void k_lbm_adj_pull(LbmDev P, const float *__restrict__ fin,
                                                            const uint8_t *__restrict__ solid,
                                                            const float *__restrict__ gout,
                                                            const float *__restrict__ ubar_out,
                                                            float *__restrict__ fbar) {
  __shared__ __attribute__((aligned(4))) uint8_t s_sol[9][SOL_W];
  __shared__ int s_any[LBM_BLOCK / 64];
  __shared__ float s_inl[5];
  const int x0 = blockIdx.x * LBM_BLOCK;
  const int i = x0 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  const uint32_t node = (uint32_t)i + (uint32_t)P.nx * ((uint32_t)j + (uint32_t)P.ny * (uint32_t)k);
  const bool inlet_row = x0 == 0 && P.bc[0] == DW_BC_INLET;
  if (inlet_row) stage_inlet(P, j, k, s_inl);
  bool any = false;
  if (SOLID) any = stage_solid(P, solid, x0, j, k, s_sol, s_any);
  else if (inlet_row) __syncthreads();
  if (i >= P.nx) return;
  const bool solid_node = any && s_sol[4][i - x0 + 4] != 0;
  const bool inlet_wave = inlet_row && threadIdx.x < 64;  // wave-uniform
  float f[19];
  if (any) pull_row<1>(std::make_integer_sequence<int, 19>{}, P, fin, s_sol, s_inl, inlet_wave, i, j, k, x0, node, f);
  else pull_row<0>(std::make_integer_sequence<int, 19>{}, P, fin, s_sol, s_inl, inlet_wave, i, j, k, x0, node, f);
  float rho, ux, uy, uz;
  moments(P, f, rho, ux, uy, uz);
  const float uu = ux * ux + uy * uy + uz * uz;
  const float om = P.omega, kf = 1.0f - 0.5f * om;
  float g[19];
  float rbar = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    g[q] = ld_node(gout + (size_t)q * P.L, node);
    const float cu = LC[q][0] * ux + LC[q][1] * uy + LC[q][2] * uz;
    // d feq_q / d rho at fixed u = feq_q / rho
    rbar += om * g[q] * LW[q] * (1.f + 3.f * cu + 4.5f * cu * cu - 1.5f * uu);
    // d feq_q / d u = w rho (3 c + 9 (c.u) c - 3 u)
    const float s = om * g[q] * LW[q] * rho;
    bx += s * (3.f * LC[q][0] + 9.f * cu * LC[q][0] - 3.f * ux);
    by += s * (3.f * LC[q][1] + 9.f * cu * LC[q][1] - 3.f * uy);
    bz += s * (3.f * LC[q][2] + 9.f * cu * LC[q][2] - 3.f * uz);
    if (P.forced) {
      const float cF = LC[q][0] * P.F[0] + LC[q][1] * P.F[1] + LC[q][2] * P.F[2];
      const float t = kf * g[q] * LW[q];
      bx += t * (9.f * cF * LC[q][0] - 3.f * P.F[0]);
      by += t * (9.f * cF * LC[q][1] - 3.f * P.F[1]);
      bz += t * (9.f * cF * LC[q][2] - 3.f * P.F[2]);
    }
  }
  if (ubar_out) {
    bx += ld_node(ubar_out, node);
    by += ld_node(ubar_out + P.L, node);
    bz += ld_node(ubar_out + 2 * P.L, node);
  }
  const float ir = 1.0f / rho;
  const float bu = bx * ux + by * uy + bz * uz;
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const float fb = (1.f - om) * g[q] + rbar + (bx * LC[q][0] + by * LC[q][1] + bz * LC[q][2] - bu) * ir;
    st_node(fbar + (size_t)q * P.L, node, solid_node ? 0.f : fb);
  }
}

__global__ __launch_bounds__(256) void k_lbm_equilibrium(LbmDev P, const float *__restrict__ rho_in,
                                                         const float *__restrict__ u_in, float *__restrict__ f) {
  if (P.skip && *P.skip) return;  // grid-uniform
  // grid-stride over the nodes (the grid is bounded, so a switched-off call
  // returns from a few thousand workgroups)
  for (int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; node < P.L;
       node += (int64_t)gridDim.x * blockDim.x) {
    float rho = rho_in ? rho_in[node] : 1.f;
    float ux = u_in ? u_in[node] : P.uin[0];
    float uy = u_in ? u_in[P.L + node] : P.uin[1];
    float uz = u_in ? u_in[2 * P.L + node] : P.uin[2];
    float uu = ux * ux + uy * uy + uz * uz;
    float drho = rho - 1.f;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
      float cu = LC[q][0] * ux + LC[q][1] * uy + LC[q][2] * uz;
      f[(int64_t)q * P.L + node] = LW[q] * (drho + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * uu));
    }
  }
}

// lattice cell coordinate (x - o) / dx, or (xr - o) / dx + x / dx with a
// position reference, each part rounded once
__device__ __forceinline__ float voxel_coord(const float *xr, const float *x, size_t i, float o, float dx) {
#pragma clang fp contract(off)
  if (xr) return (xr[i] - o) / dx + x[i] / dx;
  return (x[i] - o) / dx;
}

__global__ void k_voxelize(int nx, int ny, int nz, float ox, float oy, float oz, float dx,
                           const float *__restrict__ x, const float *__restrict__ xr, int n,
                           uint8_t *__restrict__ solid) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float qx = floorf(voxel_coord(xr, x, p, ox, dx));
  const float qy = floorf(voxel_coord(xr, x, (size_t)n + p, oy, dx));
  const float qz = floorf(voxel_coord(xr, x, 2 * (size_t)n + p, oz, dx));
  // NaN fails every comparison and is dropped here
  if (!(qx >= 0.f && qy >= 0.f && qz >= 0.f && qx < (float)nx && qy < (float)ny && qz < (float)nz)) return;
  int64_t idx = (int64_t)qx + (int64_t)nx * ((int64_t)qy + (int64_t)ny * (int64_t)qz);
  solid[idx] = 1;
}

// zero bytes: 16 per store over the 16-byte aligned body, single bytes at
// the ends (launch it for count / 16 + 16 threads)
__global__ void k_fill_u8(uint8_t *p, int64_t count) {
  const int64_t head = min((int64_t)((16 - ((uintptr_t)p & 15)) & 15), count);
  const int64_t body = (count - head) / 16;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  uint4 *q = reinterpret_cast<uint4 *>(p + head);
  for (int64_t i = t; i < body; i += stride) q[i] = make_uint4(0u, 0u, 0u, 0u);
  const int64_t tail0 = head + body * 16;
  if (t < head) p[t] = 0;
  if (t < count - tail0) p[tail0 + t] = 0;
}

static dim3 lbm_grid(const LbmDev &P) {
  return dim3((unsigned)((P.nx + LBM_BLOCK - 1) / LBM_BLOCK), (unsigned)P.ny, (unsigned)P.nz);
}

static int make_lbm(const dw_lattice *lat, const dw_lbm_params *prm, LbmDev *P) {
  DW_REQUIRE(lat && prm, DW_EINVAL, "lbm: lattice / params is NULL");
  DW_REQUIRE(lat->nx >= 1 && lat->ny >= 1 && lat->nz >= 1, DW_EINVAL, "lbm: lattice dims must be >= 1");
  int64_t L = (int64_t)lat->nx * lat->ny * lat->nz;
  DW_REQUIRE(L < ((int64_t)1 << 29), DW_ERANGE, "lbm: lattice too large (fewer than 2^29 nodes)");
  DW_REQUIRE(lat->ny <= 65535 && lat->nz <= 65535, DW_ERANGE, "lbm: ny, nz must be <= 65535");
  DW_REQUIRE(prm->tau > 0.5f, DW_EINVAL, "lbm: tau must be > 1/2 (got %g)", (double)prm->tau);
  for (int a = 0; a < 3; ++a) {
    int lo = prm->bc[2 * a], hi = prm->bc[2 * a + 1];
    DW_REQUIRE(lo >= 0 && lo <= 3 && hi >= 0 && hi <= 3, DW_EINVAL, "lbm: unknown boundary code");
    DW_REQUIRE((lo == DW_BC_PERIODIC) == (hi == DW_BC_PERIODIC), DW_EINVAL,
               "lbm: periodic faces must pair on axis %d", a);
    DW_REQUIRE(lo != DW_BC_OUTLET && hi != DW_BC_INLET, DW_EINVAL,
               "lbm: inlet only on a low face, outlet only on a high face");
    DW_REQUIRE(a == 0 || (lo != DW_BC_INLET && hi != DW_BC_OUTLET), DW_EINVAL,
               "lbm: inlet / outlet are supported on the x faces only");
  }
  DW_REQUIRE(prm->gust_amp == 0.f || prm->gust_period != 0.f, DW_EINVAL, "lbm: gust period must be non-zero");
  P->nx = lat->nx;
  P->ny = lat->ny;
  P->nz = lat->nz;
  P->L = L;
  P->omega = 1.0f / prm->tau;
  for (int a = 0; a < 3; ++a) {
    P->uin[a] = prm->u_in[a];
    P->F[a] = prm->force[a];
  }
  for (int a = 0; a < 6; ++a) P->bc[a] = prm->bc[a];
  P->gust_amp = prm->gust_amp;
  P->gust_inv_period = prm->gust_amp != 0.f ? 1.0f / prm->gust_period : 0.f;
  P->gust_ky = prm->gust_ky;
  P->gust_kz = prm->gust_kz;
  P->gust_phase = prm->gust_phase;
  P->t = prm->t;
  P->t_in = prm->t_in;
  P->t_out = prm->t_out;
  P->skip = prm->skip;
  DW_REQUIRE(!prm->t_out || (const int32_t *)prm->t_out != prm->t_in, DW_EINVAL, "lbm: t_out must not alias t_in");
  P->forced = prm->force[0] != 0.f || prm->force[1] != 0.f || prm->force[2] != 0.f;
  return DW_OK;
}

}  // namespace dw

using namespace dw;

extern "C" int lbm_step(const dw_lattice *lat, const dw_lbm_params *params, const float *f_in, float *f_out,
                        const uint8_t *solid, float *rho_out, float *u_out, void *stream) {
  LbmDev P;
  int rc = make_lbm(lat, params, &P);
  if (rc) return rc;
  DW_REQUIRE(f_in && f_out, DW_EINVAL, "lbm_step: f_in / f_out is NULL");
  DW_REQUIRE(f_in != f_out, DW_EINVAL, "lbm_step: f_in and f_out must not alias");
  hipStream_t s = (hipStream_t)stream;
  if (P.skip) {
    const int64_t nblocks = (int64_t)((P.nx + LBM_BLOCK - 1) / LBM_BLOCK) * P.ny * P.nz;
    const dim3 grid((unsigned)(nblocks < (int64_t)LBM_GATED_BLOCKS ? nblocks : LBM_GATED_BLOCKS));
    const bool big = lbm_streams(P);
    if (solid && big)
      hipLaunchKernelGGL((k_lbm_step_gated<true, true>), grid, dim3(LBM_BLOCK), 0, s, P, f_in, f_out, solid, rho_out,
                         u_out);
    else if (solid)
      hipLaunchKernelGGL((k_lbm_step_gated<true, false>), grid, dim3(LBM_BLOCK), 0, s, P, f_in, f_out, solid, rho_out,
                         u_out);
    else if (big)
      hipLaunchKernelGGL((k_lbm_step_gated<false, true>), grid, dim3(LBM_BLOCK), 0, s, P, f_in, f_out, solid,
                         rho_out, u_out);
    else
      hipLaunchKernelGGL((k_lbm_step_gated<false, false>), grid, dim3(LBM_BLOCK), 0, s, P, f_in, f_out, solid,
                         rho_out, u_out);
  } else if (lbm_streams(P)) {
    if (solid)
      hipLaunchKernelGGL((k_lbm_step<true, true>), lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, f_out, solid, rho_out,
                         u_out);
    else
      hipLaunchKernelGGL((k_lbm_step<false, true>), lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, f_out, solid,
                         rho_out, u_out);
  } else {
    if (solid)
      hipLaunchKernelGGL((k_lbm_step<true, false>), xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, f_out, solid,
                         rho_out, u_out);
    else
      hipLaunchKernelGGL((k_lbm_step<false, false>), xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, f_out, solid,
                         rho_out, u_out);
  }
  return check_launch("lbm_step");
}

namespace dw {

// The reverse BGK step: pull pass into `work`, then the transposed-streaming
// gather into f_in_bar (shared by lbm_step_adj and lbm_step_adj_static).
static int run_lbm_step_adj(const char *name, const dw_lattice *lat, const dw_lbm_params *params, const float *f_in,
                            const uint8_t *solid, const float *f_out_bar, const float *u_out_bar, float *f_in_bar,
                            float *work, hipStream_t s) {
  LbmDev P;
  int rc = make_lbm(lat, params, &P);
  if (rc) return rc;
  DW_REQUIRE(f_in && f_out_bar && f_in_bar && work, DW_EINVAL, "%s: f_in / f_out_bar / f_in_bar / work is NULL",
             name);
  DW_REQUIRE(f_in_bar != f_in && f_in_bar != f_out_bar, DW_EINVAL, "%s: f_in_bar must not alias", name);
  DW_REQUIRE(work != f_in && work != f_out_bar && work != f_in_bar && work != u_out_bar, DW_EINVAL,
             "%s: work must not alias another argument", name);
  if (solid) {
    hipLaunchKernelGGL(k_lbm_adj_pull<true>, lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, solid, f_out_bar, u_out_bar,
                       work);
    hipLaunchKernelGGL((k_adj_gather<true, false>), xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, solid, work,
                       f_in_bar);
  } else {
    hipLaunchKernelGGL(k_lbm_adj_pull<false>, lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, solid, f_out_bar,
                       u_out_bar, work);
    hipLaunchKernelGGL((k_adj_gather<false, false>), xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, solid, work,
                       f_in_bar);
  }
  return check_launch(name);
}

// Work buffer of lbm_step_adj_static: [19][L] floats for lattices of at most
// DW_STATIC_ADJ_MAX_NODES nodes, a file-scope device array (one copy per
// device, held for the life of the process).  Host code never uses the
// symbol itself as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) float scratch[(size_t)19 * DW_STATIC_ADJ_MAX_NODES];

static std::mutex g_scratch_mu;
static float *g_scratch_ptr[64] = {nullptr};

static int static_scratch(const char *name, float **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  DW_REQUIRE(e == hipSuccess, DW_ELAUNCH, "%s: hipGetDevice failed: %s", name, hipGetErrorString(e));
  DW_REQUIRE(dev >= 0 && dev < 64, DW_ERANGE, "%s: device index %d not supported", name, dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    DW_REQUIRE(e == hipSuccess && ptr, DW_ELAUNCH, "%s: hipGetSymbolAddress(scratch) failed on device %d: %s", name,
               dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<float *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return DW_OK;
}

}  // namespace dw

extern "C" int lbm_step_adj(const dw_lattice *lat, const dw_lbm_params *params, const float *f_in,
                            const uint8_t *solid, const float *f_out_bar, const float *u_out_bar, float *f_in_bar,
                            float *work, void *stream) {
  return run_lbm_step_adj("lbm_step_adj", lat, params, f_in, solid, f_out_bar, u_out_bar, f_in_bar, work,
                          (hipStream_t)stream);
}

extern "C" int lbm_step_adj_static(const dw_lattice *lat, const dw_lbm_params *params, const float *f_in,
                                   const uint8_t *solid, const float *f_out_bar, const float *u_out_bar,
                                   float *f_in_bar, void *stream) {
  DW_REQUIRE(lat, DW_EINVAL, "lbm_step_adj_static: lattice is NULL");
  const int64_t L = (int64_t)lat->nx * lat->ny * lat->nz;
  DW_REQUIRE(L <= DW_STATIC_ADJ_MAX_NODES, DW_ERANGE,
             "lbm_step_adj_static: lattice of %lld nodes exceeds the static work buffer (%d nodes); "
             "use lbm_step_adj with a caller-provided work buffer",
             (long long)L, (int)DW_STATIC_ADJ_MAX_NODES);
  float *work = nullptr;
  int rc = static_scratch("lbm_step_adj_static", &work);
  if (rc) return rc;
  return run_lbm_step_adj("lbm_step_adj_static", lat, params, f_in, solid, f_out_bar, u_out_bar, f_in_bar, work,
                          (hipStream_t)stream);
}

extern "C" int lbm_equilibrium(const dw_lattice *lat, const dw_lbm_params *params, const float *rho,
                               const float *u, float *f, void *stream) {
  LbmDev P;
  dw_lbm_params prm = *params;
  if (prm.tau <= 0.5f) prm.tau = 1.0f;  // tau plays no role here
  int rc = make_lbm(lat, &prm, &P);
  if (rc) return rc;
  DW_REQUIRE(f, DW_EINVAL, "lbm_equilibrium: f is NULL");
  const unsigned eg = grid_blocks(P.L, 256);
  hipLaunchKernelGGL(k_lbm_equilibrium, dim3(eg < 4096u ? eg : 4096u), dim3(256), 0, (hipStream_t)stream, P, rho,
                     u, f);
  return check_launch("lbm_equilibrium");
}

extern "C" int lbm_home_step(const dw_lattice *lat, const dw_lbm_params *params, const float *m_in, float *m_out,
                             const uint8_t *solid, float *rho_out, float *u_out, void *stream) {
  LbmDev P;
  int rc = make_lbm(lat, params, &P);
  if (rc) return rc;
  DW_REQUIRE(m_in && m_out, DW_EINVAL, "lbm_home_step: m_in / m_out is NULL");
  DW_REQUIRE(m_in != m_out, DW_EINVAL, "lbm_home_step: m_in and m_out must not alias");
  if (solid)
    hipLaunchKernelGGL(k_home_step<true>, xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, (hipStream_t)stream, P, m_in, m_out,
                       solid, rho_out, u_out);
  else
    hipLaunchKernelGGL(k_home_step<false>, xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, (hipStream_t)stream, P, m_in, m_out,
                       solid, rho_out, u_out);
  return check_launch("lbm_home_step");
}

extern "C" int lbm_home_equilibrium(const dw_lattice *lat, const dw_lbm_params *params, const float *rho,
                                    const float *u, float *m, void *stream) {
  LbmDev P;
  dw_lbm_params prm = *params;
  if (prm.tau <= 0.5f) prm.tau = 1.0f;  // tau plays no role here
  int rc = make_lbm(lat, &prm, &P);
  if (rc) return rc;
  DW_REQUIRE(m, DW_EINVAL, "lbm_home_equilibrium: m is NULL");
  hipLaunchKernelGGL(k_home_equilibrium, dim3(grid_blocks(P.L, 256)), dim3(256), 0, (hipStream_t)stream, P, rho,
                     u, m);
  return check_launch("lbm_home_equilibrium");
}

extern "C" int lbm_home_step_adj(const dw_lattice *lat, const dw_lbm_params *params, const float *m_in,
                                 const uint8_t *solid, const float *m_out_bar, const float *u_out_bar,
                                 float *m_in_bar, float *work, void *stream) {
  LbmDev P;
  int rc = make_lbm(lat, params, &P);
  if (rc) return rc;
  DW_REQUIRE(m_in && m_out_bar && m_in_bar && work, DW_EINVAL,
             "lbm_home_step_adj: m_in / m_out_bar / m_in_bar / work is NULL");
  DW_REQUIRE(m_in_bar != m_in && m_in_bar != m_out_bar, DW_EINVAL, "lbm_home_step_adj: m_in_bar must not alias");
  DW_REQUIRE(work != m_in && work != m_out_bar && work != m_in_bar && work != u_out_bar, DW_EINVAL,
             "lbm_home_step_adj: work must not alias another argument");
  hipStream_t s = (hipStream_t)stream;
  if (solid) {
    hipLaunchKernelGGL(k_home_adj_pull<true>, xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, m_in, solid, m_out_bar,
                       u_out_bar, work);
    hipLaunchKernelGGL((k_adj_gather<true, true>), xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, m_in, solid, work,
                       m_in_bar);
  } else {
    hipLaunchKernelGGL(k_home_adj_pull<false>, xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, m_in, solid, m_out_bar,
                       u_out_bar, work);
    hipLaunchKernelGGL((k_adj_gather<false, true>), xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, m_in, solid, work,
                       m_in_bar);
  }
  return check_launch("lbm_home_step_adj");
}

extern "C" int lbm_solid_from_particles(const dw_lattice *lat, const float *x, const float *xref, int n,
                                        uint8_t *solid, int accumulate, void *stream) {
  DW_REQUIRE(lat && solid, DW_EINVAL, "lbm_solid_from_particles: lattice / solid is NULL");
  DW_REQUIRE(lat->nx >= 1 && lat->ny >= 1 && lat->nz >= 1 && lat->dx > 0.f, DW_EINVAL,
             "lbm_solid_from_particles: bad lattice");
  DW_REQUIRE(n >= 0 && (n == 0 || x), DW_EINVAL, "lbm_solid_from_particles: bad particles");
  hipStream_t s = (hipStream_t)stream;
  int64_t L = (int64_t)lat->nx * lat->ny * lat->nz;
  if (!accumulate) hipLaunchKernelGGL(k_fill_u8, dim3(grid_blocks(L / 16 + 16, 256)), dim3(256), 0, s, solid, L);
  if (n > 0)
    hipLaunchKernelGGL(k_voxelize, dim3(grid_blocks(n, 256)), dim3(256), 0, s, lat->nx, lat->ny, lat->nz,
                       lat->origin[0], lat->origin[1], lat->origin[2], lat->dx, x, xref, n, solid);
  return check_launch("lbm_solid_from_particles");
}
