// MLS-MPM forward path for gfx950: cell-tile sort, tile-local P2G scatter,
// active-tile grid update with wind coupling, coalesced G2P gather.
//
// Equations: Eq. P2G, Eq. G2P and Eq. deformation_update of the paper's
// appendix ("Material Point Method"), the MLS-MPM stress term
// A_p = m_p C_p - dt V0_p (4/dx^2) tau_p, and the explicit grid update of
// Eq. continuum_mechanics with the wind force field on the MPM grid (Sec. 3.2).
#include <hip/hip_runtime.h>

#include <climits>

#include "dw_internal.h"
#include "dw_kernels.h"
#include "dw_scatter.h"

namespace dw {

// ------------------------------------------------------------------ sort

// Wave-aggregated keyed atomicAdd: lanes holding equal keys share one
// global atomic (particles are spatially coherent, so a wave usually holds one
// or two keys).  Returns base + rank of the lane among the lanes with its key
// (lane order).  The distinct keys are found first with ballots, then their
// leaders issue their atomics together, so a wave waits for one round trip
// however many keys it holds.  Every lane of the wave must call it.
__device__ __forceinline__ int wave_keyed_add(int32_t *counters, int key, bool active) {
  unsigned long long pending = __ballot(active);
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  int my_leader = 0, my_rank = 0, count = 0;
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int k = __shfl(key, leader, 64);
    const bool mine = active && key == k;
    const unsigned long long same = __ballot(mine);
    if (mine) {
      my_leader = leader;
      my_rank = (int)__popcll(same & below);
    }
    if (lane == leader) count = (int)__popcll(same);
    pending &= ~same;
  }
  int base = 0;
  if (count > 0) base = atomicAdd(&counters[key], count);
  base = __shfl(base, my_leader, 64);
  return active ? base + my_rank : 0;
}

// Key of every particle and its rank inside its tile (the tile count's value
// before the particle's wave added to it), so the scatter needs no atomics.
__global__ void k_sort_keys(GridDev g, const float *__restrict__ x, const float *__restrict__ xr, int n,
                            int32_t *__restrict__ key,
                            int32_t *__restrict__ rank, int32_t *__restrict__ tile_count,
                            int32_t *__restrict__ node_flag, int32_t *__restrict__ status) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  bool live = p < n;
  int k = -1;
  int bx = 0, by = 0, bz = 0;
  if (live) {
    const float X = coord_sum(load_coord(xr, x, p, g.ox, g.inv_dx));
    const float Y = coord_sum(load_coord(xr, x, (size_t)n + p, g.oy, g.inv_dx));
    const float Z = coord_sum(load_coord(xr, x, 2 * (size_t)n + p, g.oz, g.inv_dx));
    const float lim = 1.0e9f;  // guard the float -> int conversion
    if (!(isfinite(X) && isfinite(Y) && isfinite(Z))) {
      atomicOr(status, DW_STATUS_NONFINITE);
    } else if (fabsf(X) > lim || fabsf(Y) > lim || fabsf(Z) > lim) {
      atomicOr(status, DW_STATUS_OUT_OF_GRID);
    } else {
      bx = base_of(X); by = base_of(Y); bz = base_of(Z);
      if (stencil_inside(g, bx, by, bz)) k = (bx >> 2) + g.tx * ((by >> 2) + g.ty * (bz >> 2));
      else atomicOr(status, DW_STATUS_OUT_OF_GRID);
    }
  }
  const int r = wave_keyed_add(tile_count, k, k >= 0);
  if (live) {
    key[p] = k;
    rank[p] = r;
  }
  if (k >= 0) {
    int tx = bx >> 2, ty = by >> 2, tz = bz >> 2;
    int ux = (bx + 2) >> 2, uy = (by + 2) >> 2, uz = (bz + 2) >> 2;
    for (int cz = tz; cz <= uz; ++cz)
      for (int cy = ty; cy <= uy; ++cy)
        for (int cx = tx; cx <= ux; ++cx) node_flag[cx + g.tx * (cy + g.ty * cz)] = 1;
  }
}

// wave64 inclusive scan
__device__ __forceinline__ int wave_incl_scan(int v) {
  int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Block-wide exclusive scans of the four tile rows at once (SCAN_BLOCK-thread
// block, two barriers in all): ex[r] = sum of v[r] over the threads before
// this one, tot[r] = the block's total.
constexpr int SCAN_WAVES = SCAN_BLOCK / 64;

__device__ __forceinline__ void block_excl_scan4(const int v[4], int ex[4], int tot[4],
                                                 int (*lds)[4] /* [2 * SCAN_WAVES + 1][4] */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int inc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) inc[r] = wave_incl_scan(v[r]);
  if (lane == 63)
#pragma unroll
    for (int r = 0; r < 4; ++r) lds[wid][r] = inc[r];
  __syncthreads();
  if (wid == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = lane < SCAN_WAVES ? lds[lane][r] : 0;
      const int ti = wave_incl_scan(t);
      if (lane < SCAN_WAVES) lds[SCAN_WAVES + lane][r] = ti - t;
      if (lane == SCAN_WAVES - 1) lds[2 * SCAN_WAVES][r] = ti;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    ex[r] = inc[r] - v[r] + lds[SCAN_WAVES + wid][r];
    tot[r] = lds[2 * SCAN_WAVES][r];
  }
}

// the four rows of tile i: particle count, node-tile flag, occupied, work items
__device__ __forceinline__ void tile_rows(const int32_t *__restrict__ count, const int32_t *__restrict__ flag,
                                          int64_t T, int64_t i, int v[4]) {
  const int c = i < T ? count[i] : 0;
  v[0] = c;
  v[1] = i < T ? (flag[i] != 0) : 0;
  v[2] = c > 0;
  v[3] = (c + WORK_CHUNK - 1) / WORK_CHUNK;
}

// per block: the sums of the four rows (one block-wide reduction)
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const int32_t *__restrict__ count,
                                                            const int32_t *__restrict__ flag, int64_t T,
                                                            int32_t *__restrict__ block_sums, int64_t NB) {
  __shared__ int s_red[SCAN_WAVES][4];
  const int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
  int v[4];
  tile_rows(count, flag, T, i, v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[r] += __shfl_xor(v[r], o, 64);
    if (lane == 0) s_red[wid][r] = v[r];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    int t = 0;
    for (int w = 0; w < SCAN_WAVES; ++w) t += s_red[w][threadIdx.x];
    block_sums[threadIdx.x * NB + blockIdx.x] = t;
  }
}

// Final pass: tile offsets, the compacted active cell / node tile lists and
// the work items (a cell tile cut into chunks of at most WORK_CHUNK sorted
// particles: item = (tile, first particle)).  Each block adds up the block
// sums of the blocks before it itself (there are few: T / SCAN_BLOCK per
// row), and block 0 writes the four totals.
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_final(
    const int32_t *__restrict__ count, const int32_t *__restrict__ flag, int64_t T,
    const int32_t *__restrict__ block_sums, int64_t NB, int32_t *__restrict__ tile_start,
    int32_t *__restrict__ cell_tiles, int32_t *__restrict__ node_tiles, int32_t *__restrict__ item_tile,
    int32_t *__restrict__ item_begin, int32_t *__restrict__ item_first, int32_t *__restrict__ totals /* [4] */) {
  __shared__ int lds[2 * SCAN_WAVES + 1][4];
  __shared__ int s_red[SCAN_WAVES][8];
  __shared__ int s_sum[8];
  // per row: the sum over the blocks before this one (0..3) and over all (4..7),
  // one block-wide reduction of the eight values
  int acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < NB; b += SCAN_BLOCK) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = block_sums[r * NB + b];
      acc[4 + r] += v;
      if (b < (int64_t)blockIdx.x) acc[r] += v;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[r] += __shfl_xor(acc[r], o, 64);
    if (lane == 0) s_red[wid][r] = acc[r];
  }
  // the block's own rows are scanned while the reduction above settles
  const int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
  int v[4], ex[4], tot[4];
  tile_rows(count, flag, T, i, v);
  block_excl_scan4(v, ex, tot, lds);  // its barriers also publish s_red
  if (threadIdx.x < 8) {
    int t = 0;
    for (int w = 0; w < SCAN_WAVES; ++w) t += s_red[w][threadIdx.x];
    s_sum[threadIdx.x] = t;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < 4) totals[threadIdx.x] = s_sum[4 + threadIdx.x];
  if (i < T) {
    const int ec = ex[0] + s_sum[0], ef = ex[1] + s_sum[1], en = ex[2] + s_sum[2], eh = ex[3] + s_sum[3];
    const int c = v[0], ch = v[3];
    tile_start[i] = ec;
    item_first[i] = eh;
    if (v[2]) cell_tiles[en] = (int)i;
    if (v[1]) node_tiles[ef] = (int)i;
    for (int q = 0; q < ch; ++q) {
      item_tile[eh + q] = (int)i;
      item_begin[eh + q] = ec + q * WORK_CHUNK;
    }
    if (i == T - 1) tile_start[T] = ec + c;
  }
}

__global__ void k_sort_scatter(const int32_t *__restrict__ key, const int32_t *__restrict__ rank, int n,
                               const int32_t *__restrict__ tile_start, int32_t *__restrict__ perm) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int k = key[p];
  if (k >= 0) perm[tile_start[k] + rank[p]] = p;
}

// Deterministic mode: sort each tile's segment by particle index (rank by count).
__global__ __launch_bounds__(256) void k_sort_segments(const int32_t *__restrict__ tile_start,
                                                       const int32_t *__restrict__ cell_tiles,
                                                       const int32_t *__restrict__ n_tiles,
                                                       const int32_t *__restrict__ in,
                                                       int32_t *__restrict__ out) {
  __shared__ int32_t chunk[1024];
  int nt = *n_tiles;
  for (int it = blockIdx.x; it < nt; it += gridDim.x) {
    int tile = cell_tiles[it];
    int beg = tile_start[tile], end = tile_start[tile + 1];
    for (int j0 = beg; j0 < end; j0 += blockDim.x) {
      int j = j0 + threadIdx.x;
      int mine = j < end ? in[j] : 0x7fffffff;
      int rank = 0;
      for (int c0 = beg; c0 < end; c0 += 1024) {
        __syncthreads();
        for (int q = threadIdx.x; q < 1024; q += blockDim.x) chunk[q] = (c0 + q < end) ? in[c0 + q] : 0x7fffffff;
        __syncthreads();
        int lim = min(1024, end - c0);
        for (int q = 0; q < lim; ++q) rank += chunk[q] < mine;
      }
      if (j < end) out[beg + rank] = mine;
    }
  }
}

// ------------------------------------------------------------------ P2G

__global__ __launch_bounds__(256) void k_grid_clear(GridDev g, const int32_t *__restrict__ node_tiles,
                                                    const int32_t *__restrict__ n_tiles, float *__restrict__ gm,
                                                    float *__restrict__ gmv, int64_t N) {
  int nt = *n_tiles;
  int sub = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int it = blockIdx.x * 4 + sub; it < nt; it += gridDim.x * 4) {
    int t = node_tiles[it];
    int tx = t % g.tx, ty = (t / g.tx) % g.ty, tz = t / (g.tx * g.ty);
    int i = tx * 4 + (l & 3), j = ty * 4 + ((l >> 2) & 3), k = tz * 4 + (l >> 4);
    if (i < g.nx && j < g.ny && k < g.nz) {
      int64_t node = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
      gm[node] = 0.f;
      gmv[node] = 0.f;
      gmv[N + node] = 0.f;
      gmv[2 * N + node] = 0.f;
    }
  }
}

struct PView {
  const float *x, *v, *C, *F, *mass, *vol0, *E, *nu;
  const float *xr;  // position reference or NULL
  const int32_t *region;
  int n, n_regions;
};

constexpr int P2G_THREADS = SC_THREADS;
constexpr int P2G_PER_CU = 1024 / P2G_THREADS;  // resident workgroups per compute unit

// One workgroup (8 waves) per work item -- a chunk of at most WORK_CHUNK
// sorted particles of one cell tile, so a dense tile is spread over several
// workgroups.  The grid is as many workgroups as fit at once; each draws
// items from a ticket counter until the list is done.  No float atomics in LDS:
// Pass A1: thread j takes the item's particle j, finds its cell in the tile
//   (LDS histogram) and issues the loads of the rest of its state.
// Pass B: exclusive scan of the 64 cell counts; cells cut into units.
// Pass A2: the thread computes the stress (the polar decomposition), the
//   MLS affine matrix A and the momentum and stages, at its particle's slot
//   in cell order, f, m, q = m v - A f dx and A dx.
// Pass C: the units on the matrix cores into per-wave node blocks (the tile
//   scatter of dw_scatter.h).
// Pass D: the thread owning node n of the 6^3 region adds the 8 wave blocks
//   in a fixed order and adds the total into the global grid with a
//   hardware float atomic (nodes that received mass only).
template <bool DET>
__global__ __launch_bounds__(P2G_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_p2g(
    GridDev g, PView P, float dt, int material, const int32_t *__restrict__ perm,
    const int32_t *__restrict__ tile_start, const int32_t *__restrict__ item_tile,
    const int32_t *__restrict__ item_begin, const int32_t *__restrict__ n_items, float *__restrict__ gm,
    float *__restrict__ gmv, int64_t N, int32_t *__restrict__ status, float *__restrict__ item_part) {
  static_assert(WORK_CHUNK == P2G_THREADS, "one staged particle per thread");
  __shared__ float s_dat[SC_DAT][SC_PITCH];                       // staged particles in cell order
  __shared__ float4 s_f[SC_PITCH];                                  // staged f per particle
  __shared__ __attribute__((aligned(16))) float s_node[SC_WAVES][SC_NODES][4];  // per-wave node sums
  __shared__ int s_cnt[64], s_off[64], s_cur[64];
  __shared__ int s_udesc[SC_MAX_UNITS];
  __shared__ int s_nunits, s_next;
  __shared__ unsigned char s_cell[WORK_CHUNK];
  const int n = P.n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const float kstress = dt * 4.0f * g.inv_dx * g.inv_dx;
  const float dx = g.dx;
  const ScLane L = sc_lane(lane);
  float *s_node_flat = &s_node[0][0][0];
  const int ni = *n_items;
  // Workgroup b starts with item b (no stampede on the counter at launch);
  // later items are handed out by a ticket counter (header word 8, cleared
  // by the sort) as items gridDim.x + ticket.
  int32_t *ticket = status + 8;
  for (int it = blockIdx.x; it < ni; it = s_next) {
    const int tile = item_tile[it];
    const int b0 = item_begin[it];
    const int nb = min(WORK_CHUNK, tile_start[tile + 1] - b0);
    const int tx = tile % g.tx, ty = (tile / g.tx) % g.ty, tz = tile / (g.tx * g.ty);
    if (tid < 64) s_cnt[tid] = 0;
    for (int q = tid; q < SC_WAVES * SC_NODES; q += P2G_THREADS)
      reinterpret_cast<float4 *>(s_node_flat)[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    // pass A1: this thread's particle -> cell and histogram; the rest of its
    // state is loaded now and consumed after the scan
    const int j = tid;
    const bool has = j < nb;
    const int p = has ? perm[b0 + j] : 0;
    float fx = 0.f, fy = 0.f, fz = 0.f, H[9], Cm[9], m = 0.f, V0 = 0.f, vx = 0.f, vy = 0.f, vz = 0.f, Er = 0.f,
          nur = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) H[q] = Cm[q] = 0.f;
    unsigned char c = 255;
    if (has) {
      const Coord cx = load_coord(P.xr, P.x, p, g.ox, g.inv_dx);
      const Coord cy = load_coord(P.xr, P.x, (size_t)n + p, g.oy, g.inv_dx);
      const Coord cz = load_coord(P.xr, P.x, 2 * (size_t)n + p, g.oz, g.inv_dx);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        H[q] = P.F[q * n + p];
        Cm[q] = P.C[q * n + p];
      }
      m = P.mass[p];
      V0 = P.vol0[p];
      vx = P.v[p];
      vy = P.v[n + p];
      vz = P.v[2 * n + p];
      const int r = P.region[p];
      Er = P.E[r];
      nur = P.nu[r];
      const int bx = base_of(coord_sum(cx)), by = base_of(coord_sum(cy)), bz = base_of(coord_sum(cz));
      fx = coord_frac(cx, bx);
      fy = coord_frac(cy, by);
      fz = coord_frac(cz, bz);
      const int lx = bx - 4 * tx, ly = by - 4 * ty, lz = bz - 4 * tz;
      if ((unsigned)lx <= 3u && (unsigned)ly <= 3u && (unsigned)lz <= 3u) {
        c = (unsigned char)(lx + 4 * (ly + 4 * lz));
        atomicAdd(&s_cnt[c], 1);
      } else {
        atomicOr(status, DW_STATUS_OUT_OF_GRID);
      }
    }
    s_cell[j] = c;
    __syncthreads();
    // pass B: cell offsets and units
    if (wid == 0) sc_scan_units(lane, s_cnt, s_off, s_cur, s_udesc, &s_nunits);
    __syncthreads();
    // pass A2: stress, APIC matrix and momentum, staged at the particle's
    // slot in cell order
    if (c != 255) {
      int slot;
      if (DET) {
        // fixed order: rank among the item's earlier particles of the same cell
        int rank = 0;
        for (int q = 0; q < j; ++q) rank += s_cell[q] == c;
        slot = s_off[c] + rank;
      } else {
        slot = atomicAdd(&s_cur[c], 1);
      }
      float mu, lam, tau[9];
      lame(Er, nur, mu, lam);
      kirchhoff_shift_p2g(H, mu, lam, material, tau, status);
      const float f[3] = {fx, fy, fz};
      float A[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) A[q] = (m * Cm[q] - kstress * V0 * tau[q]) * dx;
      const float qv[3] = {m * vx - (A[0] * f[0] + A[1] * f[1] + A[2] * f[2]),
                           m * vy - (A[3] * f[0] + A[4] * f[1] + A[5] * f[2]),
                           m * vz - (A[6] * f[0] + A[7] * f[1] + A[8] * f[2])};
      sc_stage(s_dat, s_f, slot, f, m, qv, A);
    }
    __syncthreads();
    // pass C; the next ticket is drawn before it and stored after it, so the
    // atomic's round trip overlaps the matrix work
    int tk = 0;
    if (tid == P2G_THREADS - 1) tk = atomicAdd(ticket, 1);
    sc_units_mfma(L, wid, s_dat, s_f, s_udesc, s_nunits, s_node[wid]);
    if (tid == P2G_THREADS - 1) s_next = (int)gridDim.x + tk;
    __syncthreads();
    // pass D: node owners add the wave blocks in a fixed order
    if (tid < SC_NODES) {
      float sm = 0.f, s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int w = 0; w < SC_WAVES; ++w) {
        sm += s_node[w][tid][0];
        s0 += s_node[w][tid][1];
        s1 += s_node[w][tid][2];
        s2 += s_node[w][tid][3];
      }
      if (DET) {
        float *dst = item_part + ((int64_t)it * SC_NODES + tid) * 4;
        dst[0] = sm;
        dst[1] = s0;
        dst[2] = s1;
        dst[3] = s2;
      } else if (sm != 0.f) {
        const int nx_ = tid % SC_L, ny_ = (tid / SC_L) % SC_L, nz_ = tid / (SC_L * SC_L);
        const int64_t node = (4 * tx + nx_) + (int64_t)g.nx * ((4 * ty + ny_) + (int64_t)g.ny * (4 * tz + nz_));
        atomicAdd(&gm[node], sm);
        atomicAdd(&gmv[node], s0);
        atomicAdd(&gmv[N + node], s1);
        atomicAdd(&gmv[2 * N + node], s2);
      }
    }
    __syncthreads();
  }
  // the last workgroup to finish rewinds the counters for the next call
  if (tid == 0) {
    __threadfence();
    if (atomicAdd(ticket + 1, 1) == (int)gridDim.x - 1) {
      atomicExch(ticket, 0);
      atomicExch(ticket + 1, 0);
    }
  }
}

// ---------------------------------------------------------------- reorder

// out[i] = in[perm[i]] for every per-particle array (SoA, n entries each)
__global__ __launch_bounds__(256) void k_reorder(PView in, float *__restrict__ x, float *__restrict__ xr,
                                                 float *__restrict__ v,
                                                 float *__restrict__ C, float *__restrict__ F,
                                                 float *__restrict__ mass, float *__restrict__ vol0,
                                                 int32_t *__restrict__ region, const int32_t *__restrict__ perm,
                                                 int32_t *__restrict__ perm_out) {
  const int n = in.n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = perm[i];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    x[d * n + i] = in.x[d * n + p];
    v[d * n + i] = in.v[d * n + p];
    if (xr) xr[d * n + i] = in.xr[d * n + p];
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    C[q * n + i] = in.C[q * n + p];
    F[q * n + i] = in.F[q * n + p];
  }
  mass[i] = in.mass[p];
  vol0[i] = in.vol0[p];
  region[i] = in.region[p];
  if (perm_out) perm_out[i] = p;
}

// ------------------------------------------------------------ grid update

__global__ __launch_bounds__(256) void k_grid_update(GridDev g, float dt, float gx, float gy, float gz,
                                                     int bound, const float *__restrict__ gm,
                                                     const float *__restrict__ gmv, WindDev wind,
                                                     const uint8_t *__restrict__ pin,
                                                     const int32_t *__restrict__ node_tiles,
                                                     const int32_t *__restrict__ n_tiles, float *__restrict__ gv,
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
    float vx = 0.f, vy = 0.f, vz = 0.f;
    if (m > 0.f) {
      const float im = 1.0f / m;
      const float sx = gmv[node] * im, sy = gmv[N + node] * im, sz = gmv[2 * N + node] * im;
      float ax = 0.f, ay = 0.f, az = 0.f;
      wind_at_node(wind, g, i, j, k, node, sx, sy, sz, ax, ay, az);
      vx = sx + dt * (gx + ax);
      vy = sy + dt * (gy + ay);
      vz = sz + dt * (gz + az);
      if ((i < bound && vx < 0.f) || (i >= g.nx - bound && vx > 0.f)) vx = 0.f;
      if ((j < bound && vy < 0.f) || (j >= g.ny - bound && vy > 0.f)) vy = 0.f;
      if ((k < bound && vz < 0.f) || (k >= g.nz - bound && vz > 0.f)) vz = 0.f;
      if (pin && pin[node]) vx = vy = vz = 0.f;
    }
    gv[node] = vx;
    gv[N + node] = vy;
    gv[2 * N + node] = vz;
  }
}

// ------------------------------------------------------------------ G2P

// ------------------------------------------------ stencil box staged in LDS
// The 256 particles of a workgroup, stored in tile order, touch few grid
// nodes: the bounding box of their 3 x 3 x 3 stencils.  When it holds at most
// STENCIL_BOX nodes (12^3) a kernel stages the grid arrays it gathers over
// the box in LDS once, and the 27-node gathers read LDS instead of keeping
// the vector memory pipeline busy (they mostly hit L1/L2, but issue 27 loads
// per particle and array).
constexpr int STENCIL_BOX = 1728;

struct StencilBox {
  int lo[3];    // lowest node of the box
  int ex, ey;   // extents in x and y (nodes)
  int nb;       // nodes in the box, 0 if no thread takes part
  bool staged;  // 0 < nb <= STENCIL_BOX
};

// Box of the stencil bases (bx, by, bz) of the threads with `have` set, for a
// 256-thread workgroup; block-uniform.  Two barriers; s_red [4][6] and
// s_box [6] are LDS scratch.
__device__ __forceinline__ StencilBox block_box(bool have, int bx, int by, int bz, int (*s_red)[6], int *s_box) {
  int r[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
  if (have) {
    r[0] = bx; r[1] = by; r[2] = bz;
    r[3] = bx; r[4] = by; r[5] = bz;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r[a] = min(r[a], __shfl_xor(r[a], o, 64));
      r[3 + a] = max(r[3 + a], __shfl_xor(r[3 + a], o, 64));
    }
  }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int a = 0; a < 6; ++a) s_red[threadIdx.x >> 6][a] = r[a];
  __syncthreads();
  if (threadIdx.x < 6) {
    int v = s_red[0][threadIdx.x];
    for (int w = 1; w < 4; ++w) v = threadIdx.x < 3 ? min(v, s_red[w][threadIdx.x]) : max(v, s_red[w][threadIdx.x]);
    s_box[threadIdx.x] = v;
  }
  __syncthreads();
  StencilBox B;
#pragma unroll
  for (int a = 0; a < 3; ++a) B.lo[a] = s_box[a];
  const bool any = s_box[3] >= B.lo[0];
  B.ex = any ? s_box[3] - B.lo[0] + 3 : 0;
  B.ey = any ? s_box[4] - B.lo[1] + 3 : 0;
  B.nb = any ? B.ex * B.ey * (s_box[5] - B.lo[2] + 3) : 0;
  B.staged = any && B.nb <= STENCIL_BOX;
  return B;
}

// LDS index of the box node (i, j, k)
__device__ __forceinline__ int box_index(const StencilBox &B, int i, int j, int k) {
  return (i - B.lo[0]) + B.ex * ((j - B.lo[1]) + B.ey * (k - B.lo[2]));
}

// s[a][q] = src[a][node q of the box] for the NV arrays (grid node indices
// below 2^30): every load first, then the LDS writes, then a barrier.  For a
// staged box, called by the whole workgroup.
template <int NV>
__device__ __forceinline__ void stage_box(const GridDev &g, const StencilBox &B, const float *const (&src)[NV],
                                          float (*s)[STENCIL_BOX]) {
  constexpr int PER = (STENCIL_BOX + 255) / 256;
  float sv[PER][NV];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    if (256 * r < B.nb) {
      const int q = min((int)threadIdx.x + 256 * r, B.nb - 1);
      const int ix = q % B.ex, iy = (q / B.ex) % B.ey, iz = q / (B.ex * B.ey);
      const uint32_t node = (uint32_t)(B.lo[0] + ix) +
                            (uint32_t)g.nx * ((uint32_t)(B.lo[1] + iy) + (uint32_t)g.ny * (uint32_t)(B.lo[2] + iz));
#pragma unroll
      for (int a = 0; a < NV; ++a) sv[r][a] = ld32(src[a], node);
    }
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int q = (int)threadIdx.x + 256 * r;
    if (256 * r < B.nb && q < B.nb) {
#pragma unroll
      for (int a = 0; a < NV; ++a) s[a][q] = sv[r][a];
    }
  }
  __syncthreads();
}


// G2P, one particle per thread, the 27-node gathers from the workgroup's
// stencil box in LDS when it is staged, else from global memory.  One batch
// per workgroup: on this ISA a wave's stores count against the same counter
// as its loads, so a workgroup that went on to a next batch would wait for
// its previous stores at the next staging wait.
struct Float3 {
  float v[3];
};

// v = sum w u and B = sum w u o^T over the stencil, row by row (a row = the
// three x-neighbours at fixed oy, oz): per row r0 = sum_ox wx u and
// r1 = sum_ox wx ox u, the row weight wy wz scaling r0 (v and the y, z
// columns of B) and r1 (the x column).  LDS: the box's node li0 + ox + ex oy
// + exy oz; else the grid row at (bx, by + oy, bz + oz).
template <bool LDS>
__device__ __forceinline__ void g2p_gather(const GridDev &g, const float *__restrict__ gv, int64_t N,
                                           const float (*s_v)[STENCIL_BOX], int li0, int ex, int exy, int bx, int by,
                                           int bz, const float wx[3], const float wy[3], const float wz[3],
                                           float vv[3], float B[9]) {
#pragma unroll
  for (int oz = 0; oz < 3; ++oz)
#pragma unroll
    for (int oy = 0; oy < 3; ++oy) {
      Float3 ra, rb, rc;
      if constexpr (LDS) {
        const int li = li0 + oy * ex + oz * exy;
#pragma unroll
        for (int ox = 0; ox < 3; ++ox) {
          ra.v[ox] = s_v[0][li + ox];
          rb.v[ox] = s_v[1][li + ox];
          rc.v[ox] = s_v[2][li + ox];
        }
      } else {
        // the three x-neighbours are contiguous: one 12-byte load per component
        const int64_t row = bx + (int64_t)g.nx * ((by + oy) + (int64_t)g.ny * (bz + oz));
        __builtin_memcpy(&ra, gv + row, sizeof(Float3));
        __builtin_memcpy(&rb, gv + N + row, sizeof(Float3));
        __builtin_memcpy(&rc, gv + 2 * N + row, sizeof(Float3));
      }
      const float u0[3] = {ra.v[0] * wx[0] + ra.v[1] * wx[1] + ra.v[2] * wx[2],
                           rb.v[0] * wx[0] + rb.v[1] * wx[1] + rb.v[2] * wx[2],
                           rc.v[0] * wx[0] + rc.v[1] * wx[1] + rc.v[2] * wx[2]};
      const float w2 = 2.0f * wx[2];
      const float u1[3] = {ra.v[1] * wx[1] + ra.v[2] * w2, rb.v[1] * wx[1] + rb.v[2] * w2,
                           rc.v[1] * wx[1] + rc.v[2] * w2};
      const float wyz = wy[oy] * wz[oz];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        vv[a] += wyz * u0[a];
        B[3 * a] += wyz * u1[a];
      }
      if (oy > 0) {
        const float wy_ = wyz * (float)oy;
#pragma unroll
        for (int a = 0; a < 3; ++a) B[3 * a + 1] += wy_ * u0[a];
      }
      if (oz > 0) {
        const float wz_ = wyz * (float)oz;
#pragma unroll
        for (int a = 0; a < 3; ++a) B[3 * a + 2] += wz_ * u0[a];
      }
    }
}

// at most 72 VGPRs: 7 workgroups per CU, the count the LDS box allows
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_g2p(GridDev g, float dt, const float *__restrict__ gv, int64_t N,
                                             const float *xin, const float *xref, const float *Fin, float *xout,
                                             float *vout, float *Cout, float *Fout, int n,
                                             int32_t *__restrict__ status) {
  __shared__ float s_v[3][STENCIL_BOX];
  __shared__ int s_red[4][6];
  __shared__ int s_box[6];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = p < n;
  const uint32_t pp = live ? (uint32_t)p : 0u;
  const float px = ld32(xin, pp), py = ld32(xin + n, pp), pz = ld32(xin + 2 * (size_t)n, pp);
  const bool ref = xref != nullptr;
  const Coord cx = make_coord(ref, ref ? ld32(xref, pp) : 0.f, px, g.ox, g.inv_dx);
  const Coord cy = make_coord(ref, ref ? ld32(xref + n, pp) : 0.f, py, g.oy, g.inv_dx);
  const Coord cz = make_coord(ref, ref ? ld32(xref + 2 * (size_t)n, pp) : 0.f, pz, g.oz, g.inv_dx);
  const float X = coord_sum(cx), Y = coord_sum(cy), Z = coord_sum(cz);
  float F[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) F[q] = ld32(Fin + (size_t)q * n, pp);
  bool ok = isfinite(X) && isfinite(Y) && isfinite(Z) && fabsf(X) < 1e9f && fabsf(Y) < 1e9f && fabsf(Z) < 1e9f;
  int bx = 0, by = 0, bz = 0;
  if (ok) {
    bx = base_of(X); by = base_of(Y); bz = base_of(Z);
    ok = stencil_inside(g, bx, by, bz);
  }
  const StencilBox box = block_box(live && ok, bx, by, bz, s_red, s_box);
  if (box.staged) {
    const float *const src[3] = {gv, gv + N, gv + 2 * N};
    stage_box<3>(g, box, src, s_v);
  }
  if (!live) return;
  if (!ok) {
    if (status) atomicOr(status, DW_STATUS_OUT_OF_GRID);
    st32(xout, pp, px); st32(xout + n, pp, py); st32(xout + 2 * (size_t)n, pp, pz);
#pragma unroll
    for (int q = 0; q < 3; ++q) st32(vout + (size_t)q * n, pp, 0.f);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      st32(Cout + (size_t)q * n, pp, 0.f);
      st32(Fout + (size_t)q * n, pp, F[q]);
    }
    return;
  }
  const float fx = coord_frac(cx, bx), fy = coord_frac(cy, by), fz = coord_frac(cz, bz);
  float wx[3], wy[3], wz[3];
  {
    float a = 1.5f - fx, b = fx - 1.0f, c = fx - 0.5f;
    wx[0] = 0.5f * a * a; wx[1] = 0.75f - b * b; wx[2] = 0.5f * c * c;
    a = 1.5f - fy; b = fy - 1.0f; c = fy - 0.5f;
    wy[0] = 0.5f * a * a; wy[1] = 0.75f - b * b; wy[2] = 0.5f * c * c;
    a = 1.5f - fz; b = fz - 1.0f; c = fz - 0.5f;
    wz[0] = 0.5f * a * a; wz[1] = 0.75f - b * b; wz[2] = 0.5f * c * c;
  }
  float vv[3] = {0.f, 0.f, 0.f};
  float B[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (box.staged)
    g2p_gather<true>(g, gv, N, s_v, box_index(box, bx, by, bz), box.ex, box.ex * box.ey, bx, by, bz, wx, wy, wz, vv,
                     B);
  else
    g2p_gather<false>(g, gv, N, s_v, 0, 0, 0, bx, by, bz, wx, wy, wz, vv, B);
  const float ff[3] = {fx, fy, fz};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) B[3 * a + c] -= vv[a] * ff[c];
  // C = (4/dx^2) sum w v d^T with d = (o - f) dx  ->  (4/dx) sum w v (o - f)^T
  const float kc = 4.0f * g.inv_dx;
  float Cn[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) Cn[q] = kc * B[q];
  st32(xout, pp, px + dt * vv[0]);
  st32(xout + n, pp, py + dt * vv[1]);
  st32(xout + 2 * (size_t)n, pp, pz + dt * vv[2]);
  st32(vout, pp, vv[0]);
  st32(vout + n, pp, vv[1]);
  st32(vout + 2 * (size_t)n, pp, vv[2]);
  // F <- (I + dt C) F with F = I + H stored as H:  H <- H + dt C + dt C H
  float G[9], CH[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) G[q] = dt * Cn[q];
  matmul3(G, F, CH);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    st32(Cout + (size_t)q * n, pp, Cn[q]);
    st32(Fout + (size_t)q * n, pp, F[q] + G[q] + CH[q]);
  }
}

}  // namespace dw

// =================================================================== C ABI

namespace dw {

constexpr int PERSISTENT_BLOCKS = 2048;

// compute units of the current device (cached per device)
static int cu_count() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cus[dev] = c;
  }
  return cus[dev];
}

// P2G grid: the workgroups that fit at once (two per compute unit), which
// then draw work items from the ticket counter
static unsigned p2g_blocks() { return (unsigned)(P2G_PER_CU * cu_count()); }

static PView make_pview(const dw_particles *p) {
  PView v;
  v.x = p->x; v.v = p->v; v.C = p->C; v.F = p->F;
  v.mass = p->mass; v.vol0 = p->vol0; v.E = p->E; v.nu = p->nu;
  v.region = p->region;
  v.xr = p->xref;
  v.n = p->n;
  v.n_regions = p->n_regions;
  return v;
}

int run_sort(const dw_grid *grid, int deterministic, const float *x, const float *xref, int n,
             const Workspace &W, hipStream_t s) {
  GridDev g = make_grid(grid);
  int64_t T = W.n_tiles, NB = W.n_scan_blocks;
  // header + tile_count + node_flag are contiguous: clear them
  int64_t clear_words = (int64_t)((char *)W.tile_start - (char *)W.status) / 4;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_blocks(clear_words / 4 + 4, 256)), dim3(256), 0, s, W.status, clear_words, 0);
  if (n > 0)
    hipLaunchKernelGGL(k_sort_keys, dim3(grid_blocks(n, 256)), dim3(256), 0, s, g, x, xref, n, W.key, W.rank,
                       W.tile_count, W.node_flag, W.status);
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)NB), dim3(SCAN_BLOCK), 0, s, W.tile_count, W.node_flag, T,
                     W.block_sums, NB);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)NB), dim3(SCAN_BLOCK), 0, s, W.tile_count, W.node_flag, T,
                     W.block_sums, NB, W.tile_start, W.cell_tiles, W.node_tiles, W.item_tile, W.item_begin,
                     W.item_first, W.status + 3);
  if (n > 0) {
    int32_t *dst = deterministic ? W.perm_tmp : W.perm;
    hipLaunchKernelGGL(k_sort_scatter, dim3(grid_blocks(n, 256)), dim3(256), 0, s, W.key, W.rank, n, W.tile_start,
                       dst);
    if (deterministic)
      hipLaunchKernelGGL(k_sort_segments, dim3(PERSISTENT_BLOCKS), dim3(256), 0, s, W.tile_start, W.cell_tiles,
                         W.n_cell_tiles, W.perm_tmp, W.perm);
  }
  return check_launch("mpm_sort");
}

}  // namespace dw

using namespace dw;

extern "C" int mpm_sort(const dw_grid *grid, const dw_mpm_params *params, const float *x, const float *xref,
                        int n, void *ws, size_t ws_bytes, void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  DW_REQUIRE(n >= 0, DW_EINVAL, "mpm_sort: n must be >= 0");
  DW_REQUIRE(n == 0 || x, DW_EINVAL, "mpm_sort: x is NULL");
  Workspace W;
  rc = bind_workspace(grid, n, ws, ws_bytes, &W);
  if (rc) return rc;
  return run_sort(grid, params ? params->deterministic : 0, x, xref, n, W, (hipStream_t)stream);
}

extern "C" int mpm_reorder(const dw_grid *grid, const dw_particles *in, dw_particles *out, int32_t *perm_out,
                           const void *ws, size_t ws_bytes, void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  rc = check_particles(in, true);
  if (rc) return rc;
  DW_REQUIRE(out && out->n == in->n, DW_EINVAL, "mpm_reorder: out must hold in->n particles");
  DW_REQUIRE(out->x && out->v && out->C && out->F && out->mass && out->vol0 && out->region, DW_EINVAL,
             "mpm_reorder: out arrays must not be NULL");
  DW_REQUIRE(out->x != in->x && out->v != in->v && out->C != in->C && out->F != in->F && out->mass != in->mass &&
                 out->vol0 != in->vol0 && out->region != in->region,
             DW_EINVAL, "mpm_reorder: in and out must not share arrays");
  DW_REQUIRE(!in->xref || (out->xref && out->xref != in->xref), DW_EINVAL,
             "mpm_reorder: with in->xref set, out->xref must be a separate array");
  Workspace W;
  rc = bind_workspace(grid, in->n, ws, ws_bytes, &W, 0);
  if (rc) return rc;
  if (in->n > 0)
    hipLaunchKernelGGL(k_reorder, dim3(grid_blocks(in->n, 256)), dim3(256), 0, (hipStream_t)stream,
                       make_pview(in), out->x, in->xref ? const_cast<float *>(out->xref) : (float *)nullptr,
                       out->v, out->C, out->F, const_cast<float *>(out->mass),
                       const_cast<float *>(out->vol0), const_cast<int32_t *>(out->region), W.perm,
                       perm_out);
  return check_launch("mpm_reorder");
}

extern "C" int mpm_p2g(const dw_grid *grid, const dw_mpm_params *params, const dw_particles *p, float *grid_m,
                       float *grid_mv, void *ws, size_t ws_bytes, void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  DW_REQUIRE(params, DW_EINVAL, "mpm_p2g: params is NULL");
  DW_REQUIRE(params->material == DW_FIXED_COROTATED || params->material == DW_NEO_HOOKEAN, DW_EINVAL,
             "mpm_p2g: unknown material %d", params->material);
  rc = check_particles(p, true);
  if (rc) return rc;
  DW_REQUIRE(grid_m && grid_mv, DW_EINVAL, "mpm_p2g: grid_m / grid_mv is NULL");
  Workspace W;
  rc = bind_workspace(grid, p->n, ws, ws_bytes, &W, params->deterministic);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  GridDev g = make_grid(grid);
  int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;
  if (params->deterministic) {
    DW_REQUIRE(W.item_part, DW_EWORKSPACE, "mpm_p2g: deterministic mode needs a deterministic workspace");
    if (p->n > 0)
      hipLaunchKernelGGL(k_p2g<true>, dim3(p2g_blocks()), dim3(P2G_THREADS), 0, s, g, make_pview(p), params->dt,
                         params->material, W.perm, W.tile_start, W.item_tile, W.item_begin, W.n_items, grid_m,
                         grid_mv, N, W.status, W.item_part);
    hipLaunchKernelGGL(k_det_gather<false>, dim3(PERSISTENT_BLOCKS), dim3(256), 0, s, g, W.node_tiles, W.n_node_tiles,
                       W.tile_count, W.item_first, W.item_part, grid_m, grid_mv, N);
    return check_launch("mpm_p2g");
  }
  hipLaunchKernelGGL(k_grid_clear, dim3(PERSISTENT_BLOCKS), dim3(256), 0, s, g, W.node_tiles, W.n_node_tiles,
                     grid_m, grid_mv, N);
  if (p->n > 0)
    hipLaunchKernelGGL(k_p2g<false>, dim3(p2g_blocks()), dim3(P2G_THREADS), 0, s, g, make_pview(p), params->dt,
                       params->material, W.perm, W.tile_start, W.item_tile, W.item_begin, W.n_items, grid_m,
                       grid_mv, N, W.status, (float *)nullptr);
  return check_launch("mpm_p2g");
}

extern "C" int mpm_grid_update(const dw_grid *grid, const dw_mpm_params *params, const float *grid_m,
                               const float *grid_mv, const dw_wind *wind, const uint8_t *pin, float *grid_v,
                               const void *ws, size_t ws_bytes, void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  DW_REQUIRE(params, DW_EINVAL, "mpm_grid_update: params is NULL");
  DW_REQUIRE(grid_m && grid_mv && grid_v, DW_EINVAL, "mpm_grid_update: grid arrays must be set");
  DW_REQUIRE(params->bound >= 0, DW_EINVAL, "mpm_grid_update: bound must be >= 0");
  Workspace W;
  rc = bind_workspace(grid, 0, ws, ws_bytes, &W);
  if (rc) return rc;
  WindDev wd;
  rc = make_wind(wind, grid, &wd);
  if (rc) return rc;
  GridDev g = make_grid(grid);
  int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;
  hipLaunchKernelGGL(k_grid_update, dim3(PERSISTENT_BLOCKS), dim3(256), 0, (hipStream_t)stream, g, params->dt,
                     params->gravity[0], params->gravity[1], params->gravity[2], params->bound, grid_m, grid_mv,
                     wd, pin, W.node_tiles, W.n_node_tiles, grid_v, N);
  return check_launch("mpm_grid_update");
}

extern "C" int mpm_g2p(const dw_grid *grid, const dw_mpm_params *params, const float *grid_v,
                       const dw_particles *in, dw_particles *out, void *stream) {
  int rc = check_grid(grid);
  if (rc) return rc;
  DW_REQUIRE(params && grid_v, DW_EINVAL, "mpm_g2p: params / grid_v is NULL");
  DW_REQUIRE(in && out && in->n == out->n && in->n >= 0, DW_EINVAL, "mpm_g2p: in / out mismatch");
  if (in->n == 0) return DW_OK;
  DW_REQUIRE(in->x && in->F && out->x && out->v && out->C && out->F, DW_EINVAL,
             "mpm_g2p: in->x, in->F, out->x, v, C, F must be set");
  DW_REQUIRE((int64_t)in->n * 9 < (int64_t)INT_MAX, DW_ERANGE, "mpm_g2p: too many particles");
  GridDev g = make_grid(grid);
  int64_t N = (int64_t)grid->nx * grid->ny * grid->nz;
  hipLaunchKernelGGL(k_g2p, dim3(grid_blocks(in->n, 256)), dim3(256), 0, (hipStream_t)stream, g, params->dt,
                     grid_v, N, in->x, in->xref, in->F, out->x, out->v, out->C, out->F, in->n,
                     (int32_t *)nullptr);
  return check_launch("mpm_g2p");
}
