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
// the forward step's block width on large lattices whose rows are whole
// multiples of it (one block per row: no x-shifted reads across a block seam)
constexpr int LBM_BLOCK_WIDE = 256;
// row pitch of the staged solid flags: x0 - 4 .. x0 + width + 3 for either width
constexpr int SOL_W = LBM_BLOCK_WIDE + 8;

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
// x0 - 4 .. x0 + BW + 3 (BW: the block width), staged in LDS: row r =
// (dy + 1) + 3 (dz + 1).
// A periodic axis stages the wrapped row / positions, so every source that
// is not a bounce-back or inlet source finds its flag here; rows beyond a
// bounce-back face and positions beyond a non-periodic x face read as fluid.
// Whole 4-byte words are loaded where the row is 4-byte aligned.
template <int BW>
struct SolStage {
  static constexpr int ROW_WORDS = (BW + 8) / 4;              // staged words per row
  static constexpr int WORDS = 9 * ROW_WORDS;
  static constexpr int PER_THREAD = (WORDS + BW - 1) / BW;
};

template <int BW>
__device__ __forceinline__ void load_solid_rows(const LbmDev &P, const uint8_t *__restrict__ solid, int x0, int j,
                                                int k, uint32_t v[SolStage<BW>::PER_THREAD]) {
  using St = SolStage<BW>;
  constexpr int WORDS = St::ROW_WORDS;
  const bool aligned = (P.nx & 3) == 0 && (((uintptr_t)solid) & 3) == 0;
  const bool xper = P.bc[0] == DW_BC_PERIODIC;
#pragma unroll
  for (int u = 0; u < St::PER_THREAD; ++u) {
    const int q = threadIdx.x + u * BW;
    v[u] = 0;
    if (q >= St::WORDS) continue;
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

template <int BW>
__device__ __forceinline__ void store_solid_rows(const uint32_t v[SolStage<BW>::PER_THREAD],
                                                 uint8_t (*s_sol)[SOL_W]) {
  using St = SolStage<BW>;
#pragma unroll
  for (int u = 0; u < St::PER_THREAD; ++u) {
    const int q = threadIdx.x + u * BW;
    if (q < St::WORDS)
      reinterpret_cast<uint32_t *>(&s_sol[0][0])[(q / St::ROW_WORDS) * (SOL_W / 4) + q % St::ROW_WORDS] = v[u];
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
template <bool SOLID, bool BIG, int BW>
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
    uint32_t sv[SolStage<BW>::PER_THREAD];
    load_solid_rows<BW>(P, solid, x0, j, k, sv);
    store_solid_rows<BW>(sv, s_sol);
    uint32_t mine = 0;
#pragma unroll
    for (int u = 0; u < SolStage<BW>::PER_THREAD; ++u) mine |= sv[u];
    const bool wave_any = __ballot(mine != 0) != 0ull;
    if ((threadIdx.x & 63) == 0) s_any[threadIdx.x >> 6] = wave_any;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < BW / 64; ++w) any = any || s_any[w] != 0;
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
// BW: block width (LBM_BLOCK, or LBM_BLOCK_WIDE on a large lattice whose rows
// are whole multiples of it); the XCD row runs are taken with LBM_BLOCK.
template <bool SOLID, bool BIG, int BW = LBM_BLOCK>
__global__ __launch_bounds__(BW) __attribute__((amdgpu_waves_per_eu(8))) void k_lbm_step(
    LbmDev P, const float *__restrict__ fin, float *__restrict__ fout, const uint8_t *__restrict__ solid,
    float *__restrict__ rho_out, float *__restrict__ u_out) {
  static_assert(BIG || BW == LBM_BLOCK, "the XCD row runs are laid out in LBM_BLOCK blocks");
  __shared__ __attribute__((aligned(4))) uint8_t s_sol[9][SOL_W];
  __shared__ int s_any[BW / 64];
  __shared__ float s_inl[5];
  int x0, j, k;
  if (BIG) {
    x0 = blockIdx.x * BW;
    j = blockIdx.y;
    k = blockIdx.z;
  } else {
    const RowBlock rb = xcd_row_block(P);
    if (!rb.live) return;  // block-uniform
    x0 = rb.x0;
    j = rb.j;
    k = rb.k;
  }
  lbm_row_block<SOLID, BIG, BW>(P, fin, fout, solid, rho_out, u_out, x0, j, k, s_sol, s_any, s_inl);
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
    lbm_row_block<SOLID, BIG, LBM_BLOCK>(P, fin, fout, solid, rho_out, u_out, (int)(b % nbx) * LBM_BLOCK,
                                         (int)(row % P.ny), (int)(row / P.ny), s_sol, s_any, s_inl);
    __syncthreads();  // the next row block restages the shared rows
  }
}

// ------------------------------------------------------------- HOME-LBM
// Moment-encoded step (appendix on HOME-LBM): a node stores its
// post-collision moments, [HM_N][L] = rho - 1, u (3), S (6: xx yy zz xy xz
// yz) with rho S_ab = sum_i (c_a c_b - delta_ab / 3) f_i.  The step pulls,
// for each direction q, the population f_q of the source node rebuilt from
// the source's moments by the third-order Hermite expansion, takes the
// moments of the pulled set (no population is stored in memory), and
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

// The expansion of a node's moments into its populations,
//   f_q = w_q rho [1 + 3 c.u + 9/2 H2(c):S + 27/2 sum_(a,a,b) (c_a^2 - 1/3) c_b a3_aab],
// H2(c) = c c - I/3, stored as f_q - w_q.
// Shared terms of f_q - w_q = w_q (drho + (1 + drho) s_q):
//   c = +-e_a:                 s = E_a +- O_a
//   c = sa e_a + sb e_b:       s = K + sa sb C + sa A + sb B   (pair ab, d the third axis)
//   c = 0:                     s = -3/2 tr S
// with a3_AB = u_B (S_AA - 2 u_A^2) + 2 S_AB u_A,
//   E_a = 3 S_aa - 3/2 (S_bb + S_dd),
//   O_a = 3 u_a - 9/2 [u_a (S_bb + S_dd - 2 u_b^2 - 2 u_d^2) + 2 (S_ab u_b + S_ad u_d)],
//   K = 3 (S_aa + S_bb) - 3/2 S_dd,  C = 9 S_ab,
//   A = 3 u_a + 9 a3_ba - 9/2 a3_da,  B = 3 u_b + 9 a3_ab - 9/2 a3_db;
// the pairs keep K + C, K - C, A + B and A - B for their four sign cases.
struct HomeTerms {
  float s0;
  float E[3], O[3];                    // axes x, y, z
  float P1[3], P2[3], ApB[3], AmB[3];  // pairs xy, xz, yz
  float wr[3], wd[3];                  // w (1 + drho), w drho for |c|^2 = 0, 1, 2
};

__device__ __forceinline__ HomeTerms home_terms(const Mom &M) {
  const float *u = M.u, *S = M.S;
  float uu[3], D[3], p[3][3], a3[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    uu[a] = u[a] * u[a];
    D[a] = S[a] - 2.f * uu[a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (a == b) continue;
      p[a][b] = S[sidx(a, b)] * u[a];
      a3[a][b] = fmaf(u[b], D[a], 2.f * p[a][b]);
    }
  HomeTerms H;
  H.s0 = -1.5f * (S[0] + S[1] + S[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, d = (a + 2) % 3;
    const float T = S[b] + S[d];
    const float X = T - 2.f * (uu[b] + uu[d]);
    const float Z = fmaf(u[a], X, 2.f * (p[b][a] + p[d][a]));
    H.E[a] = 3.f * S[a] - 1.5f * T;
    H.O[a] = 3.f * u[a] - 4.5f * Z;
  }
  constexpr int PA[3] = {0, 0, 1}, PB[3] = {1, 2, 2}, PD[3] = {2, 1, 0};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int a = PA[e], b = PB[e], d = PD[e];
    const float K = 3.f * (S[a] + S[b]) - 1.5f * S[d];
    const float C = 9.f * S[sidx(a, b)];
    const float A = 3.f * u[a] + (9.f * a3[b][a] - 4.5f * a3[d][a]);
    const float B = 3.f * u[b] + (9.f * a3[a][b] - 4.5f * a3[d][b]);
    H.P1[e] = K + C;
    H.P2[e] = K - C;
    H.ApB[e] = A + B;
    H.AmB[e] = A - B;
  }
  const float r = 1.f + M.drho;
  constexpr float W[3] = {1.f / 3.f, 1.f / 18.f, 1.f / 36.f};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    H.wr[c] = W[c] * r;
    H.wd[c] = W[c] * M.drho;
  }
  return H;
}

// Direction Q's class: |c|^2 (n), its axis (n = 1) or axis pair (n = 2)
template <int Q>
struct HomeDir {
  static constexpr int c0 = LC[Q][0], c1 = LC[Q][1], c2 = LC[Q][2];
  static constexpr int n = (c0 != 0) + (c1 != 0) + (c2 != 0);
  static constexpr int axis = c0 != 0 ? 0 : (c1 != 0 ? 1 : 2);
  static constexpr int pair = c2 == 0 ? 0 : (c1 == 0 ? 1 : 2);
  static constexpr int pa = pair == 2 ? 1 : 0, pb = pair == 0 ? 1 : 2;
};

// the bracket s_Q of f_Q - w_Q = w_Q (drho + (1 + drho) s_Q)
template <int Q>
__device__ __forceinline__ float home_s_t(const HomeTerms &H) {
  using Dq = HomeDir<Q>;
  if constexpr (Dq::n == 0) {
    return H.s0;
  } else if constexpr (Dq::n == 1) {
    constexpr int a = Dq::axis;
    return LC[Q][a] > 0 ? H.E[a] + H.O[a] : H.E[a] - H.O[a];
  } else {
    constexpr int e = Dq::pair, sa = LC[Q][Dq::pa], sb = LC[Q][Dq::pb];
    if constexpr (sa == sb) return sa > 0 ? H.P1[e] + H.ApB[e] : H.P1[e] - H.ApB[e];
    else return sa > 0 ? H.P2[e] + H.AmB[e] : H.P2[e] - H.AmB[e];
  }
}

// f_Q - w_Q from the shared terms
template <int Q>
__device__ __forceinline__ float home_pop_t(const HomeTerms &H) {
  return fmaf(H.wr[HomeDir<Q>::n], home_s_t<Q>(H), H.wd[HomeDir<Q>::n]);
}

// Reverse of home_pop_t: the adjoint T of f_Q - w_Q added into the adjoints
// of the shared terms (B, zero-initialised by the caller).
template <int Q>
__device__ __forceinline__ void home_pop_t_adj(const HomeTerms &H, float T, HomeTerms &B) {
  using Dq = HomeDir<Q>;
  constexpr int n = Dq::n;
  B.wr[n] += T * home_s_t<Q>(H);
  B.wd[n] += T;
  const float bs = T * H.wr[n];
  if constexpr (n == 0) {
    B.s0 += bs;
  } else if constexpr (n == 1) {
    constexpr int a = Dq::axis;
    B.E[a] += bs;
    B.O[a] += LC[Q][a] > 0 ? bs : -bs;
  } else {
    constexpr int e = Dq::pair, sa = LC[Q][Dq::pa], sb = LC[Q][Dq::pb];
    if constexpr (sa == sb) {
      B.P1[e] += bs;
      B.ApB[e] += sa > 0 ? bs : -bs;
    } else {
      B.P2[e] += bs;
      B.AmB[e] += sa > 0 ? bs : -bs;
    }
  }
}

// Reverse of home_terms: the adjoints of the shared terms (B) taken back to
// those of the moments, every step of home_terms in reverse order.
__device__ __forceinline__ Mom home_terms_adj(const Mom &M, const HomeTerms &B) {
  const float *u = M.u, *S = M.S;
  float uu[3], D[3], p[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    uu[a] = u[a] * u[a];
    D[a] = S[a] - 2.f * uu[a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      if (a != b) p[a][b] = S[sidx(a, b)] * u[a];
  Mom Mb;
  float buu[3] = {0.f, 0.f, 0.f}, bD[3] = {0.f, 0.f, 0.f}, bp[3][3] = {}, ba3[3][3] = {};
  Mb.drho = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) Mb.u[a] = 0.f;
#pragma unroll
  for (int s6 = 0; s6 < 6; ++s6) Mb.S[s6] = 0.f;
  // wr = W (1 + drho), wd = W drho
  constexpr float W[3] = {1.f / 3.f, 1.f / 18.f, 1.f / 36.f};
#pragma unroll
  for (int c = 0; c < 3; ++c) Mb.drho += W[c] * (B.wr[c] + B.wd[c]);
  // pairs: P1 = K + C, P2 = K - C, ApB = A + B, AmB = A - B
  constexpr int PA[3] = {0, 0, 1}, PB[3] = {1, 2, 2}, PD[3] = {2, 1, 0};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const int a = PA[e], b = PB[e], d = PD[e];
    const float bK = B.P1[e] + B.P2[e], bC = B.P1[e] - B.P2[e];
    const float bA = B.ApB[e] + B.AmB[e], bB = B.ApB[e] - B.AmB[e];
    Mb.S[a] += 3.f * bK;
    Mb.S[b] += 3.f * bK;
    Mb.S[d] -= 1.5f * bK;
    Mb.S[sidx(a, b)] += 9.f * bC;
    Mb.u[a] += 3.f * bA;
    ba3[b][a] += 9.f * bA;
    ba3[d][a] -= 4.5f * bA;
    Mb.u[b] += 3.f * bB;
    ba3[a][b] += 9.f * bB;
    ba3[d][b] -= 4.5f * bB;
  }
  // axes: E = 3 S_aa - 3/2 T, O = 3 u_a - 9/2 Z, Z = u_a X + 2 (p_ba + p_da),
  // X = T - 2 (uu_b + uu_d), T = S_bb + S_dd
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, d = (a + 2) % 3;
    const float T = S[b] + S[d];
    const float X = T - 2.f * (uu[b] + uu[d]);
    Mb.S[a] += 3.f * B.E[a];
    Mb.u[a] += 3.f * B.O[a];
    const float bZ = -4.5f * B.O[a];
    Mb.u[a] += X * bZ;
    const float bX = u[a] * bZ;
    bp[b][a] += 2.f * bZ;
    bp[d][a] += 2.f * bZ;
    const float bT = bX - 1.5f * B.E[a];
    buu[b] -= 2.f * bX;
    buu[d] -= 2.f * bX;
    Mb.S[b] += bT;
    Mb.S[d] += bT;
  }
  // s0 = -3/2 tr S
#pragma unroll
  for (int a = 0; a < 3; ++a) Mb.S[a] -= 1.5f * B.s0;
  // a3_ab = u_b D_a + 2 p_ab, p_ab = S_ab u_a
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (a == b) continue;
      Mb.u[b] += D[a] * ba3[a][b];
      bD[a] += u[b] * ba3[a][b];
      bp[a][b] += 2.f * ba3[a][b];
      Mb.S[sidx(a, b)] += u[a] * bp[a][b];
      Mb.u[a] += S[sidx(a, b)] * bp[a][b];
    }
  // D_a = S_aa - 2 uu_a, uu_a = u_a^2
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Mb.S[a] += bD[a];
    buu[a] -= 2.f * bD[a];
    Mb.u[a] += 2.f * u[a] * buu[a];
  }
  return Mb;
}

// moments of the pulled set
struct MomAcc {
  float drho = 0.f, j[3] = {0.f, 0.f, 0.f}, P[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
};

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

// the ten moments of a node (planes of L floats)
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
  const HomeTerms H = home_terms(inlet_mom(P, sj, sk));
  switch (t) {
    case 0: return home_pop_t<1>(H);
    case 1: return home_pop_t<7>(H);
    case 2: return home_pop_t<9>(H);
    case 3: return home_pop_t<13>(H);
    default: return home_pop_t<15>(H);
  }
}

// Collision of the pulled set's moments and the stores of one node (a solid
// node stores the rest state).
__device__ __forceinline__ void home_collide_store(const LbmDev &P, const MomAcc &A, float *__restrict__ mout,
                                                   float *__restrict__ rho_out, float *__restrict__ u_out,
                                                   uint32_t node, bool solid_node) {
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

// ------------------------------------------------------ HOME-LBM tile step
// The moment-encoded step on tiles of HT_X x HT_Y x HT_Z nodes (x fastest),
// one thread per node.  Most terms of the expansion of a node's moments into
// its 19 populations are shared between directions (the third-order
// coefficients a3_aab, the even and odd parts of each axis and of each axis
// pair), so every node evaluates all of its populations at once and pushes
// each into the LDS slot of the node that pulls it; nodes of the one-node
// halo around the tile evaluate only the populations that point into it.
// Every slot has one writer: the source node of the pull, or, where the
// zero-gradient outlet clamps the source, the outlet-face node of the source
// row.  After a barrier each node takes its populations from its slots,
// except where the pull bounces back (its own population of the opposite
// direction, still in registers) or comes from the inlet (staged per row).
constexpr int HT_X = 32, HT_Y = 8, HT_Z = 4, HT_N = HT_X * HT_Y * HT_Z;
constexpr int HT_SX = HT_X + 2, HT_SY = HT_Y + 2, HT_SZ = HT_Z + 2;

struct HomeTile {
  int x0, y0, z0;  // lattice coordinates of the tile's first node
  int wx, wy, wz;  // extents of the tile inside the lattice
  bool live;
};

// Tiles in x, then y, then z; each XCD takes a contiguous run of them, so
// the halo a tile shares with its neighbours stays in one L2.
__device__ __forceinline__ HomeTile home_tile(const LbmDev &P) {
  const int ntx = (P.nx + HT_X - 1) / HT_X, nty = (P.ny + HT_Y - 1) / HT_Y, ntz = (P.nz + HT_Z - 1) / HT_Z;
  const int64_t nt = (int64_t)ntx * nty * ntz;
  const int64_t per_xcd = (nt + N_XCD - 1) / N_XCD;
  const int64_t b = blockIdx.x;
  const int64_t v = (b % N_XCD) * per_xcd + b / N_XCD;
  HomeTile T;
  T.live = v < nt;
  const int64_t r = v / ntx;
  T.x0 = (int)(v % ntx) * HT_X;
  T.y0 = (int)(r % nty) * HT_Y;
  T.z0 = (int)(r / nty) * HT_Z;
  T.wx = min(HT_X, P.nx - T.x0);
  T.wy = min(HT_Y, P.ny - T.y0);
  T.wz = min(HT_Z, P.nz - T.z0);
  return T;
}

static dim3 home_tile_grid(const LbmDev &P) {
  const int64_t nt = (int64_t)((P.nx + HT_X - 1) / HT_X) * ((P.ny + HT_Y - 1) / HT_Y) * ((P.nz + HT_Z - 1) / HT_Z);
  return dim3((unsigned)(((nt + N_XCD - 1) / N_XCD) * N_XCD));
}

// Population Q of a tile node into the slot of the node at +c_Q when that is
// in the tile (ok: the three per-axis tests, taken once per node); an
// outlet-face node (outx) also fills, for c_x < 0, the slot of the
// outlet-face node at +(0, c_y, c_z), whose pull the outlet clamps to here.
template <int Q>
__device__ __forceinline__ void home_push_in(float (*s_pop)[HT_N], int l, const bool okx[3], const bool oky[3],
                                             const bool okz[3], bool outx, float v) {
  constexpr int cx = LC[Q][0], cy = LC[Q][1], cz = LC[Q][2];
  constexpr int off = cx + HT_X * (cy + HT_Y * cz);
  const bool yz = oky[cy + 1] && okz[cz + 1];
  if (yz && okx[cx + 1]) s_pop[Q - 1][l + off] = v;
  if constexpr (cx < 0) {
    if (outx && yz) s_pop[Q - 1][l + off - cx] = v;
  }
}

// The same for a halo node at tile position (sx, sy, sz)
template <int Q>
__device__ __forceinline__ void home_push_halo(float (*s_pop)[HT_N], const HomeTile &T, int sx, int sy, int sz,
                                               bool outx, const HomeTerms &H) {
  constexpr int cx = LC[Q][0], cy = LC[Q][1], cz = LC[Q][2];
  const int dx = sx + cx, dy = sy + cy, dz = sz + cz;
  const bool yz = (unsigned)dy < (unsigned)T.wy && (unsigned)dz < (unsigned)T.wz;
  const int dl = dx + HT_X * (dy + HT_Y * dz);
  const float v = home_pop_t<Q>(H);
  if (yz && (unsigned)dx < (unsigned)T.wx) s_pop[Q - 1][dl] = v;
  if constexpr (cx < 0) {
    if (outx && yz && (unsigned)sx < (unsigned)T.wx) s_pop[Q - 1][dl - cx] = v;
  }
}

template <int... Qs>
__device__ __forceinline__ void home_push_halo_set(float (*s_pop)[HT_N], const HomeTile &T, int sx, int sy, int sz,
                                                   bool outx, const Mom &M) {
  const HomeTerms H = home_terms(M);  // only the terms these directions use survive
  (home_push_halo<Qs>(s_pop, T, sx, sy, sz, outx, H), ...);
}

// Lattice coordinate of tile offset o on an axis of n nodes: wrapped on a
// periodic axis, false where there is no node.
__device__ __forceinline__ bool home_wrap(int &x, int n, bool periodic) {
  if (periodic) x = x < 0 ? x + n : (x >= n ? x - n : x);
  return (unsigned)x < (unsigned)n;
}

// The halo of a tile: the y faces, z faces, x faces, then the yz, xy and xz
// edges (an edge node feeds one population); at most one node per thread.
constexpr int HT_HALO = 2 * (HT_Z * HT_X + HT_Y * HT_X + HT_Z * HT_Y) + 4 * (HT_X + HT_Y + HT_Z);
static_assert(HT_HALO <= HT_N, "the halo is taken in one pass of the workgroup");

struct HaloNode {
  int hx, hy, hz, kind;  // tile position and which populations it feeds
  int x;                 // lattice x (wrapped)
  uint32_t node;
  bool live;             // a node exists there (wrapped on a periodic axis)
};

// The h-th halo node.  FULL: the tile lies wholly inside the lattice, so its
// extents are the constants.
template <bool FULL>
__device__ __forceinline__ HaloNode home_halo_at(const LbmDev &P, const HomeTile &T, int h) {
  const int wx = FULL ? HT_X : T.wx, wy = FULL ? HT_Y : T.wy, wz = FULL ? HT_Z : T.wz;
  const int nA = wz * wx, nB = wy * wx, nC = wz * wy;
  int e = h;
  HaloNode H;
  if (e < 2 * nA) {
    const int side = e >= nA;
    e -= side * nA;
    H.hx = e % wx, H.hz = e / wx, H.hy = side ? wy : -1, H.kind = side;
  } else if ((e -= 2 * nA) < 2 * nB) {
    const int side = e >= nB;
    e -= side * nB;
    H.hx = e % wx, H.hy = e / wx, H.hz = side ? wz : -1, H.kind = 2 + side;
  } else if ((e -= 2 * nB) < 2 * nC) {
    const int side = e >= nC;
    e -= side * nC;
    H.hy = e % wy, H.hz = e / wy, H.hx = side ? wx : -1, H.kind = 4 + side;
  } else if ((e -= 2 * nC) < 4 * wx) {
    const int c = e / wx;
    H.hx = e % wx, H.hy = (c & 1) ? wy : -1, H.hz = (c & 2) ? wz : -1, H.kind = 6 + c;
  } else if ((e -= 4 * wx) < 4 * wz) {
    const int c = e / wz;
    H.hz = e % wz, H.hx = (c & 1) ? wx : -1, H.hy = (c & 2) ? wy : -1, H.kind = 10 + c;
  } else {
    e -= 4 * wz;
    const int c = e / wy;
    H.hy = e % wy, H.hx = (c & 1) ? wx : -1, H.hz = (c & 2) ? wz : -1, H.kind = 14 + c;
  }
  int x = T.x0 + H.hx, y = T.y0 + H.hy, z = T.z0 + H.hz;
  H.live = home_wrap(x, P.nx, P.bc[0] == DW_BC_PERIODIC) && home_wrap(y, P.ny, P.bc[2] == DW_BC_PERIODIC) &&
           home_wrap(z, P.nz, P.bc[4] == DW_BC_PERIODIC);  // else the face rules of the pull decide
  H.x = x;
  H.node = (uint32_t)x + (uint32_t)P.nx * ((uint32_t)y + (uint32_t)P.ny * (uint32_t)z);
  return H;
}

// The populations a live halo node feeds into the tile (none from a solid
// node: pulls from it bounce).
template <bool SOL>
__device__ __forceinline__ void home_halo_push(const LbmDev &P, const HomeTile &T,
                                               const uint8_t (*s_sol)[HT_SY][HT_SX], bool any, float (*s_pop)[HT_N],
                                               const HaloNode &H, const Mom &M) {
  if (SOL && any && s_sol[H.hz + 1][H.hy + 1][H.hx + 1] != 0) return;
  const bool outx = H.x == P.nx - 1 && P.bc[1] == DW_BC_OUTLET;
  const int hx = H.hx, hy = H.hy, hz = H.hz;
  switch (H.kind) {
    case 0: home_push_halo_set<3, 7, 11, 14, 17>(s_pop, T, hx, hy, hz, outx, M); break;   // y- face: c_y = +1
    case 1: home_push_halo_set<4, 8, 12, 13, 18>(s_pop, T, hx, hy, hz, outx, M); break;   // y+ face: c_y = -1
    case 2: home_push_halo_set<5, 9, 11, 16, 18>(s_pop, T, hx, hy, hz, outx, M); break;   // z- face: c_z = +1
    case 3: home_push_halo_set<6, 10, 12, 15, 17>(s_pop, T, hx, hy, hz, outx, M); break;  // z+ face: c_z = -1
    case 4: home_push_halo_set<1, 7, 9, 13, 15>(s_pop, T, hx, hy, hz, outx, M); break;    // x- face: c_x = +1
    case 5: home_push_halo_set<2, 8, 10, 14, 16>(s_pop, T, hx, hy, hz, outx, M); break;   // x+ face: c_x = -1
    case 6: home_push_halo_set<11>(s_pop, T, hx, hy, hz, outx, M); break;                 // yz edges
    case 7: home_push_halo_set<18>(s_pop, T, hx, hy, hz, outx, M); break;
    case 8: home_push_halo_set<17>(s_pop, T, hx, hy, hz, outx, M); break;
    case 9: home_push_halo_set<12>(s_pop, T, hx, hy, hz, outx, M); break;
    case 10: home_push_halo_set<7>(s_pop, T, hx, hy, hz, outx, M); break;                 // xy edges
    case 11: home_push_halo_set<14>(s_pop, T, hx, hy, hz, outx, M); break;
    case 12: home_push_halo_set<13>(s_pop, T, hx, hy, hz, outx, M); break;
    case 13: home_push_halo_set<8>(s_pop, T, hx, hy, hz, outx, M); break;
    case 14: home_push_halo_set<9>(s_pop, T, hx, hy, hz, outx, M); break;                 // xz edges
    case 15: home_push_halo_set<16>(s_pop, T, hx, hy, hz, outx, M); break;
    case 16: home_push_halo_set<15>(s_pop, T, hx, hy, hz, outx, M); break;
    default: home_push_halo_set<10>(s_pop, T, hx, hy, hz, outx, M); break;
  }
}

// Where the pulls of a node leave the lattice: the node sits on a
// non-periodic face (lo: the source is beyond the low face of the axis).
struct HomeFaces {
  bool lo[3], hi[3];
};

// Population Q pulled by the tile node at (tx, ty, tz): from its slot, or its
// own population opp(Q) on bounce-back, or the staged inlet population.  The
// source rules are those of the population step: a y / z face of the node
// that the pull crosses bounces it; an x face bounces it, feeds the inlet,
// or (outlet) clamps its source onto the outlet face of the source row.
// FACES = false: the tile touches no non-periodic face (no face rule applies).
template <int Q, bool SOL, bool FACES>
__device__ __forceinline__ float home_take(const LbmDev &P, const float (*s_pop)[HT_N],
                                           const uint8_t (*s_sol)[HT_SY][HT_SX], const float (*s_inl)[5],
                                           bool inlet_tile, const HomeFaces &F, int l, int tx, int ty, int tz,
                                           const float f[19]) {
  if constexpr (Q == 0) {
    return f[0];
  } else {
    constexpr int R = LOPP[Q], CX = LC[Q][0], CY = LC[Q][1], CZ = LC[Q][2];
    bool yz = false;
    if constexpr (FACES && CY != 0) yz = CY > 0 ? F.lo[1] : F.hi[1];
    if constexpr (FACES && CZ != 0) yz = yz || (CZ > 0 ? F.lo[2] : F.hi[2]);
    bool xo = false;
    if constexpr (FACES && CX != 0) xo = CX > 0 ? F.lo[0] : F.hi[0];
    const int xrule = P.bc[CX > 0 ? 0 : 1];
    float g = s_pop[Q - 1][l];
    // an opaque register value: otherwise the selects below become one load
    // from a selected address, which sends f to private memory
    asm("" : "+v"(g));
    bool bb = yz || (xo && xrule == DW_BC_BOUNCEBACK);
    if constexpr (SOL) {
      const int sx = xo ? tx : tx - CX;  // an outlet clamps the source onto the face
      bb = bb || s_sol[tz + 1 - CZ][ty + 1 - CY][sx + 1] != 0;
    }
    g = bb ? f[R] : g;
    if constexpr (FACES && inlet_slot(Q) >= 0) {
      if (inlet_tile) g = (xo && !yz && xrule == DW_BC_INLET) ? s_inl[ty + HT_Y * tz][inlet_slot(Q)] : g;
    }
    return g;
  }
}

template <bool SOL, bool FACES, int... Qs>
__device__ __forceinline__ void home_take_all(std::integer_sequence<int, Qs...>, const LbmDev &P,
                                              const float (*s_pop)[HT_N], const uint8_t (*s_sol)[HT_SY][HT_SX],
                                              const float (*s_inl)[5], bool inlet_tile, const HomeFaces &F, int l,
                                              int tx, int ty, int tz, const float f[19], float g[19]) {
  ((g[Qs] = home_take<Qs, SOL, FACES>(P, s_pop, s_sol, s_inl, inlet_tile, F, l, tx, ty, tz, f)), ...);
}

// Moments of the pulled set from the sums and differences of opposite
// populations (pairs q, q + 1 for odd q).
__device__ __forceinline__ MomAcc home_pulled_moments(const float g[19]) {
  float sp[19], dp[19];
#pragma unroll
  for (int q = 1; q < 19; q += 2) {
    sp[q] = g[q] + g[q + 1];
    dp[q] = g[q] - g[q + 1];
  }
  MomAcc A;
  A.drho = g[0] + sp[1] + sp[3] + sp[5] + sp[7] + sp[9] + sp[11] + sp[13] + sp[15] + sp[17];
  A.j[0] = dp[1] + dp[7] + dp[9] + dp[13] + dp[15];
  A.j[1] = dp[3] + dp[7] + dp[11] - dp[13] + dp[17];
  A.j[2] = dp[5] + dp[9] + dp[11] - dp[15] - dp[17];
  const float d3 = A.drho * (1.f / 3.f);
  A.P[0] = (sp[1] + sp[7] + sp[9] + sp[13] + sp[15]) - d3;
  A.P[1] = (sp[3] + sp[7] + sp[11] + sp[13] + sp[17]) - d3;
  A.P[2] = (sp[5] + sp[9] + sp[11] + sp[15] + sp[17]) - d3;
  A.P[3] = sp[7] - sp[13];
  A.P[4] = sp[9] - sp[15];
  A.P[5] = sp[11] - sp[17];
  return A;
}

template <int... Qs>
__device__ __forceinline__ void home_push_all(std::integer_sequence<int, Qs...>, float (*s_pop)[HT_N], int l,
                                              const bool okx[3], const bool oky[3], const bool okz[3], bool outx,
                                              const float f[19]) {
  (home_push_in<Qs + 1>(s_pop, l, okx, oky, okz, outx, f[Qs + 1]), ...);
}

template <int... Qs>
__device__ __forceinline__ void home_pops_all(std::integer_sequence<int, Qs...>, const HomeTerms &H, float f[19]) {
  ((f[Qs] = home_pop_t<Qs>(H)), ...);
}

// The pulled set's moments of the tile node of this thread (false for a
// thread outside the lattice, which has nothing more to do); every thread of
// the workgroup calls it (it has barriers).
template <bool SOLID>
__device__ __forceinline__ bool home_tile_pulled(const LbmDev &P, const HomeTile &T, const float *__restrict__ min,
                                                 const uint8_t *__restrict__ solid, float (*s_pop)[HT_N],
                                                 uint8_t (*s_sol)[HT_SY][HT_SX], float (*s_inl)[5], MomAcc &A,
                                                 uint32_t &node, bool &solid_node) {
  const int tid = threadIdx.x;
  const int tx = tid % HT_X, ty = (tid / HT_X) % HT_Y, tz = tid / (HT_X * HT_Y);
  const bool active = tx < T.wx && ty < T.wy && tz < T.wz;
  const int i = T.x0 + tx, j = T.y0 + ty, k = T.z0 + tz;
  node = (uint32_t)i + (uint32_t)P.nx * ((uint32_t)j + (uint32_t)P.ny * (uint32_t)k);
  // this node's and this thread's halo node's moments first: their loads
  // overlap the staging
  Mom M;
  if (active) M = load_mom_at(min, P.L, node);
  const bool full = T.wx == HT_X && T.wy == HT_Y && T.wz == HT_Z;  // block-uniform
  const int nh = 2 * (T.wz * T.wx + T.wy * T.wx + T.wz * T.wy) + 4 * (T.wx + T.wy + T.wz);
  HaloNode H;
  H.live = false;
  if (tid < nh) H = full ? home_halo_at<true>(P, T, tid) : home_halo_at<false>(P, T, tid);
  Mom HM;
  if (H.live) HM = load_mom_at(min, P.L, H.node);
  // the inlet populations of the tile's rows (tiles at x = 0 of an inlet lattice)
  const bool inlet_tile = T.x0 == 0 && P.bc[0] == DW_BC_INLET;
  if (inlet_tile && tid < 5 * HT_Y * HT_Z) {
    const int row = tid / 5, ry = row % HT_Y, rz = row / HT_Y;
    if (ry < T.wy && rz < T.wz) s_inl[row][tid % 5] = home_inlet_pop(P, tid % 5, T.y0 + ry, T.z0 + rz);
  }
  // solid flags of the tile and its halo, one staged row of HT_SX bytes per
  // wave and pass (wrapped; 0 where there is no node)
  bool any = false;
  if (SOLID) {
    const int lane = tid & 63;
    int mine = 0;
    for (int r = __builtin_amdgcn_readfirstlane(tid >> 6); r < HT_SY * HT_SZ; r += HT_N / 64) {
      const int ly = r % HT_SY, lz = r / HT_SY;
      int y = T.y0 + ly - 1, z = T.z0 + lz - 1;
      const bool row_ok = ly <= T.wy + 1 && lz <= T.wz + 1 && home_wrap(y, P.ny, P.bc[2] == DW_BC_PERIODIC) &&
                          home_wrap(z, P.nz, P.bc[4] == DW_BC_PERIODIC);
      if (lane < HT_SX) {
        int x = T.x0 + lane - 1;
        uint8_t v = 0;
        if (row_ok && lane <= T.wx + 1 && home_wrap(x, P.nx, P.bc[0] == DW_BC_PERIODIC))
          v = solid[(uint32_t)x + (uint32_t)P.nx * ((uint32_t)y + (uint32_t)P.ny * (uint32_t)z)];
        s_sol[lz][ly][lane] = v;
        mine |= v;
      }
    }
    any = __syncthreads_or(mine) != 0;
  }
  // halo populations that stream into the tile
  if (H.live) home_halo_push<SOLID>(P, T, s_sol, any, s_pop, H, HM);
  // this node's populations, pushed to the nodes that pull them
  const int l = tid;
  float f[19];
  solid_node = false;
  if (active) {
    home_pops_all(std::make_integer_sequence<int, 19>{}, home_terms(M), f);
    solid_node = SOLID && any && s_sol[tz + 1][ty + 1][tx + 1] != 0;
    if (!solid_node) {
      const bool okx[3] = {tx >= 1, true, tx + 1 < T.wx}, oky[3] = {ty >= 1, true, ty + 1 < T.wy},
                 okz[3] = {tz >= 1, true, tz + 1 < T.wz};
      const bool outx = i == P.nx - 1 && P.bc[1] == DW_BC_OUTLET;
      home_push_all(std::make_integer_sequence<int, 18>{}, s_pop, l, okx, oky, okz, outx, f);
    }
  }
  __syncthreads();
  if (!active) return false;
  HomeFaces F;
  F.lo[0] = i == 0 && P.bc[0] != DW_BC_PERIODIC;
  F.hi[0] = i == P.nx - 1 && P.bc[1] != DW_BC_PERIODIC;
  F.lo[1] = j == 0 && P.bc[2] != DW_BC_PERIODIC;
  F.hi[1] = j == P.ny - 1 && P.bc[3] != DW_BC_PERIODIC;
  F.lo[2] = k == 0 && P.bc[4] != DW_BC_PERIODIC;
  F.hi[2] = k == P.nz - 1 && P.bc[5] != DW_BC_PERIODIC;
  // a tile that touches no non-periodic face takes every pull from its slot
  // or, next to a solid node, bounces it (block-uniform)
  const bool faces = (T.x0 == 0 && P.bc[0] != DW_BC_PERIODIC) || (T.x0 + T.wx == P.nx && P.bc[1] != DW_BC_PERIODIC) ||
                     (T.y0 == 0 && P.bc[2] != DW_BC_PERIODIC) || (T.y0 + T.wy == P.ny && P.bc[3] != DW_BC_PERIODIC) ||
                     (T.z0 == 0 && P.bc[4] != DW_BC_PERIODIC) || (T.z0 + T.wz == P.nz && P.bc[5] != DW_BC_PERIODIC);
  float g[19];
  if (any && faces)
    home_take_all<true, true>(std::make_integer_sequence<int, 19>{}, P, s_pop, s_sol, s_inl, inlet_tile, F, l, tx, ty,
                              tz, f, g);
  else if (any)
    home_take_all<true, false>(std::make_integer_sequence<int, 19>{}, P, s_pop, s_sol, s_inl, inlet_tile, F, l, tx,
                               ty, tz, f, g);
  else if (faces)
    home_take_all<false, true>(std::make_integer_sequence<int, 19>{}, P, s_pop, s_sol, s_inl, inlet_tile, F, l, tx,
                               ty, tz, f, g);
  else
    home_take_all<false, false>(std::make_integer_sequence<int, 19>{}, P, s_pop, s_sol, s_inl, inlet_tile, F, l, tx,
                                ty, tz, f, g);
  A = home_pulled_moments(g);
  return true;
}

// 8 waves per SIMD: two tiles per CU, the 128 x 64 x 64 lattice's 512 tiles
// in one round.
template <bool SOLID>
__global__ __launch_bounds__(HT_N) __attribute__((amdgpu_waves_per_eu(8))) void k_home_tile(
    LbmDev P, const float *__restrict__ min, float *__restrict__ mout, const uint8_t *__restrict__ solid,
    float *__restrict__ rho_out, float *__restrict__ u_out) {
  __shared__ float s_pop[18][HT_N];
  __shared__ uint8_t s_sol[HT_SZ][HT_SY][HT_SX];
  __shared__ float s_inl[HT_Y * HT_Z][5];
  const HomeTile T = home_tile(P);
  if (!T.live) return;  // block-uniform: padding blocks of the last XCD
  if (threadIdx.x == 0 && T.x0 == 0 && T.y0 == 0 && T.z0 == 0 && P.t_out) *P.t_out = (P.t_in ? *P.t_in : P.t) + 1;
  MomAcc A;
  uint32_t node;
  bool solid_node;
  if (!home_tile_pulled<SOLID>(P, T, min, solid, s_pop, s_sol, s_inl, A, node, solid_node)) return;
  home_collide_store(P, A, mout, rho_out, u_out, node, solid_node);
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
// Reverse of k_home_tile in two passes, neither with atomics.
//  1. k_home_tile_adj, per node: recompute the pulled set's moments, take
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
// (mb) and of the reported u* (ubo), through the collision of k_home_tile
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
  uint32_t sv[SolStage<LBM_BLOCK>::PER_THREAD];
  load_solid_rows<LBM_BLOCK>(P, solid, x0, j, k, sv);
  store_solid_rows<LBM_BLOCK>(sv, s_sol);
  uint32_t mine = 0;
#pragma unroll
  for (int u = 0; u < SolStage<LBM_BLOCK>::PER_THREAD; ++u) mine |= sv[u];
  const bool wave_any = __ballot(mine != 0) != 0ull;
  if ((threadIdx.x & 63) == 0) s_any[threadIdx.x >> 6] = wave_any;
  __syncthreads();
  bool any = false;
#pragma unroll
  for (int w = 0; w < LBM_BLOCK / 64; ++w) any = any || s_any[w] != 0;
  return any;
}

template <bool SOLID>
__global__ __launch_bounds__(HT_N) __attribute__((amdgpu_waves_per_eu(8))) void k_home_tile_adj(
    LbmDev P, const float *__restrict__ min, const uint8_t *__restrict__ solid, const float *__restrict__ mout_bar,
    const float *__restrict__ ubar_out, float *__restrict__ gbar) {
  __shared__ float s_pop[18][HT_N];
  __shared__ uint8_t s_sol[HT_SZ][HT_SY][HT_SX];
  __shared__ float s_inl[HT_Y * HT_Z][5];
  const HomeTile T = home_tile(P);
  if (!T.live) return;  // block-uniform: padding blocks of the last XCD
  MomAcc A;
  uint32_t node;
  bool solid_node;
  if (!home_tile_pulled<SOLID>(P, T, min, solid, s_pop, s_sol, s_inl, A, node, solid_node)) return;
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
__device__ __forceinline__ void home_pops_adj(std::integer_sequence<int, Qs...>, const HomeTerms &H, const float T[19],
                                              HomeTerms &B) {
  (home_pop_t_adj<Qs>(H, T[Qs], B), ...);
}

// Pass 2 of both reverse steps, per node: T_p gathered as above, then for
// HOME (bar = m_in_bar [10][L]) sum_p T_p df_p/dM taken through the Hermite
// expansion of this node's moments, for BGK (bar = f_in_bar [19][L]) T_p
// itself.  A solid node's state feeds no population: it adds nothing.
// Occupancy: BGK's pass asks for 8 waves per SIMD (7 % faster than the 7
// its scalar registers allow otherwise); HOME's pass, which also takes the
// expansion's adjoint, is faster at the occupancy its registers give, so it
// asks for none (a minimum of 1).
template <bool SOLID, bool HOME>
__global__ __launch_bounds__(LBM_BLOCK) __attribute__((amdgpu_waves_per_eu(HOME ? 1 : 8))) void k_adj_gather(LbmDev P, const float *__restrict__ min,
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
    HomeTerms B{};
    home_pops_adj(std::make_integer_sequence<int, 19>{}, home_terms(own), T, B);
    const Mom Mb = home_terms_adj(own, B);
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
// XCD: rows handed to the XCDs in contiguous runs (lattices that stay in the
// last-level cache, as in the forward step), else one block per row block.
template <bool SOLID, bool XCD>
__global__ __launch_bounds__(LBM_BLOCK) void k_lbm_adj_pull(LbmDev P, const float *__restrict__ fin,
                                                            const uint8_t *__restrict__ solid,
                                                            const float *__restrict__ gout,
                                                            const float *__restrict__ ubar_out,
                                                            float *__restrict__ fbar) {
  __shared__ __attribute__((aligned(4))) uint8_t s_sol[9][SOL_W];
  __shared__ int s_any[LBM_BLOCK / 64];
  __shared__ float s_inl[5];
  int x0, j, k;
  if (XCD) {
    const RowBlock rb = xcd_row_block(P);
    if (!rb.live) return;  // block-uniform
    x0 = rb.x0;
    j = rb.j;
    k = rb.k;
  } else {
    x0 = blockIdx.x * LBM_BLOCK;
    j = blockIdx.y;
    k = blockIdx.z;
  }
  const int i = x0 + threadIdx.x;
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
#pragma unroll
  for (int q = 0; q < 19; ++q) g[q] = ld_node(gout + (size_t)q * P.L, node);
  // a direction and its opposite together: with S = g_q + g_o, D = g_q - g_o
  // (c_o = -c_q) their terms are om w [S (1 + 9/2 (c.u)^2 - 3/2 u.u) + 3 (c.u) D]
  // for rho and om w rho [c (3 D + 9 (c.u) S) - 3 u S] for u
  const float e0 = 1.f - 1.5f * uu;
  float rbar = LW[0] * g[0] * e0, ws = LW[0] * g[0], bx = 0.f, by = 0.f, bz = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
#pragma unroll
  for (int q = 1; q < 19; q += 2) {
    const float S = g[q] + g[q + 1], D = g[q] - g[q + 1];
    const float cu = LC[q][0] * ux + LC[q][1] * uy + LC[q][2] * uz;
    rbar += LW[q] * (S * (e0 + 4.5f * cu * cu) + 3.f * cu * D);
    ws += LW[q] * S;
    const float T = LW[q] * (3.f * D + 9.f * cu * S);
    if (LC[q][0] != 0) bx += LC[q][0] * T;
    if (LC[q][1] != 0) by += LC[q][1] * T;
    if (LC[q][2] != 0) bz += LC[q][2] * T;
    if (P.forced) {
      const float cF = LC[q][0] * P.F[0] + LC[q][1] * P.F[1] + LC[q][2] * P.F[2];
      const float t = LW[q] * S * 9.f * cF;
      if (LC[q][0] != 0) fx += LC[q][0] * t;
      if (LC[q][1] != 0) fy += LC[q][1] * t;
      if (LC[q][2] != 0) fz += LC[q][2] * t;
    }
  }
  rbar *= om;
  const float orho = om * rho;
  bx = orho * (bx - 3.f * ux * ws);
  by = orho * (by - 3.f * uy * ws);
  bz = orho * (bz - 3.f * uz * ws);
  if (P.forced) {
    // kf w S (9 (c.F) c - 3 F), the rest direction included in the F part
    bx += kf * (fx - 3.f * P.F[0] * ws);
    by += kf * (fy - 3.f * P.F[1] * ws);
    bz += kf * (fz - 3.f * P.F[2] * ws);
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
  } else if (lbm_streams(P) && P.nx % LBM_BLOCK_WIDE == 0) {
    // one block per row
    const dim3 grid((unsigned)(P.nx / LBM_BLOCK_WIDE), (unsigned)P.ny, (unsigned)P.nz);
    if (solid)
      hipLaunchKernelGGL((k_lbm_step<true, true, LBM_BLOCK_WIDE>), grid, dim3(LBM_BLOCK_WIDE), 0, s, P, f_in, f_out,
                         solid, rho_out, u_out);
    else
      hipLaunchKernelGGL((k_lbm_step<false, true, LBM_BLOCK_WIDE>), grid, dim3(LBM_BLOCK_WIDE), 0, s, P, f_in, f_out,
                         solid, rho_out, u_out);
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
  const bool big = lbm_streams(P);
  if (solid) {
    if (big)
      hipLaunchKernelGGL((k_lbm_adj_pull<true, false>), lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, solid, f_out_bar,
                         u_out_bar, work);
    else
      hipLaunchKernelGGL((k_lbm_adj_pull<true, true>), xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, solid,
                         f_out_bar, u_out_bar, work);
    hipLaunchKernelGGL((k_adj_gather<true, false>), xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, solid, work,
                       f_in_bar);
  } else {
    if (big)
      hipLaunchKernelGGL((k_lbm_adj_pull<false, false>), lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, solid,
                         f_out_bar, u_out_bar, work);
    else
      hipLaunchKernelGGL((k_lbm_adj_pull<false, true>), xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, f_in, solid,
                         f_out_bar, u_out_bar, work);
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
    hipLaunchKernelGGL(k_home_tile<true>, home_tile_grid(P), dim3(HT_N), 0, (hipStream_t)stream, P, m_in, m_out,
                       solid, rho_out, u_out);
  else
    hipLaunchKernelGGL(k_home_tile<false>, home_tile_grid(P), dim3(HT_N), 0, (hipStream_t)stream, P, m_in, m_out,
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
    hipLaunchKernelGGL(k_home_tile_adj<true>, home_tile_grid(P), dim3(HT_N), 0, s, P, m_in, solid, m_out_bar,
                       u_out_bar, work);
    hipLaunchKernelGGL((k_adj_gather<true, true>), xcd_lbm_grid(P), dim3(LBM_BLOCK), 0, s, P, m_in, solid, work,
                       m_in_bar);
  } else {
    hipLaunchKernelGGL(k_home_tile_adj<false>, home_tile_grid(P), dim3(HT_N), 0, s, P, m_in, solid, m_out_bar,
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
