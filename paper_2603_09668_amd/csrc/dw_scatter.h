// Tile scatter on the matrix cores, shared by P2G and the reverse of G2P.
//
// Both add, for every particle p of a cell tile and every stencil offset
// o = (ox, oy, oz) in {0,1,2}^3, the value w_o(f_p) (q_p + A_p o) into node
// base_p + o of the tile's 6^3 node region, with f_p the particle's position
// in its base cell (in cells), w_o the quadratic B-spline weight, q_p a
// 3-vector and A_p a 3x3 matrix (P2G also adds w_o m_p as a fourth value).
// A workgroup stages its particles in LDS in cell order (f as one 16-byte
// record per particle, read with one instruction; m, q, A row-major as 13
// feature rows), cuts each cell into units of at most SC_UNIT
// particles, and per unit forms Feat (13 x n) W (n x 27) with fp32 MFMA
// 16x16x4 (four particles per step, offsets in two 16-column tiles), the
// rows ordered so that the four result rows a lane holds give one node
// value: (1, ox, oy, oz) . rows.  Every wave adds its units' 27 x 4 values
// into its own 6^3 node block in LDS (a unit's 27 offsets reach 27 distinct
// nodes: plain adds); the node owners then add the wave blocks.
#pragma once

#include "dw_internal.h"

namespace dw {

constexpr int SC_L = 6;           // local node extent of a cell tile's stencils
constexpr int SC_NODES = 216;     // 6^3
constexpr int SC_DAT = 13;        // staged feature rows per particle: m, q(3), A(9)
constexpr int SC_UNIT = 16;       // particles per unit (4 MFMA steps): a dense cell spreads over waves
constexpr int SC_MAX_UNITS = 64 + WORK_CHUNK / SC_UNIT;  // bounds the sum over cells of ceil(count / unit)
constexpr int SC_THREADS = WORK_CHUNK;
constexpr int SC_WAVES = SC_THREADS / 64;
constexpr int SC_PITCH = WORK_CHUNK + 4;  // staged rows padded: the 13 feature rows of one operand hit distinct banks

typedef float floatx4_t __attribute__((ext_vector_type(4)));

// Stencil weight polynomial of offset component oo: w = a + b f + c f^2,
// w0 = (3/2 - f)^2 / 2, w1 = 3/4 - (f - 1)^2, w2 = (f - 1/2)^2 / 2.
__device__ __forceinline__ void sc_coef(int oo, float &a, float &b, float &c) {
  if (oo == 0) { a = 1.125f; b = -1.5f; c = 0.5f; }
  else if (oo == 1) { a = -0.25f; b = 2.0f; c = -1.0f; }
  else { a = 0.125f; b = -0.5f; c = 0.5f; }
}

// Per-lane constants of the MFMA 16x16x4 roles: r16 = row of the feature
// operand / column (offset within a 16-wide tile) of the weight operand,
// kq = particle slot of the step.
struct ScLane {
  int kq, feat;
  int oo[2], onode[2];
  float cfa[2][3], cfb[2][3], cfc[2][3], fo[2][3];
};

__device__ __forceinline__ ScLane sc_lane(int lane) {
  ScLane L;
  const int r16 = lane & 15;
  L.kq = lane >> 4;
  // staged feature of operand row r16, grouped so that result rows 4 kq ..
  // 4 kq + 3 (held by lane group kq) all feed node value kq:
  //   rows 0-3: m, -, -, -;  rows 4 + 4d .. 7 + 4d: q_d, A_d0, A_d1, A_d2
  L.feat = r16 == 0 ? 0 : (r16 < 4 ? -1 : ((r16 & 3) == 0 ? (r16 >> 2) : 4 + 3 * ((r16 >> 2) - 1) + (r16 & 3) - 1));
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int o = t * 16 + r16;
    L.oo[t] = o;
    const int oc = o < 27 ? o : 0;
    const int ox = oc % 3, oy = (oc / 3) % 3, oz = oc / 9;
    L.onode[t] = ox + SC_L * (oy + SC_L * oz);
    sc_coef(ox, L.cfa[t][0], L.cfb[t][0], L.cfc[t][0]);
    sc_coef(oy, L.cfa[t][1], L.cfb[t][1], L.cfc[t][1]);
    sc_coef(oz, L.cfa[t][2], L.cfb[t][2], L.cfc[t][2]);
    L.fo[t][0] = (float)ox;
    L.fo[t][1] = (float)oy;
    L.fo[t][2] = (float)oz;
  }
  return L;
}

// DPP source v shifted by CTRL within the enabled rows (ROWS mask), zero
// where the source lane lies outside the row or the row is not enabled
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int sc_dpp(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}

// Inclusive scan over the 64 lanes of a fully active wave without LDS round
// trips: Hillis-Steele inside each 16-lane row (row shifts by 1, 2, 4, 8),
// then row 0's total broadcast into row 1 and row 2's into row 3 (row
// broadcast of lane 15), then the total of rows 0-1 into rows 2 and 3 (row
// broadcast of lane 31).
__device__ __forceinline__ int sc_wave_scan(int v) {
  v += sc_dpp<0x111>(v);
  v += sc_dpp<0x112>(v);
  v += sc_dpp<0x114>(v);
  v += sc_dpp<0x118>(v);
  v += sc_dpp<0x142, 0xA>(v);
  v += sc_dpp<0x143, 0xC>(v);
  return v;
}

// Wave 0: exclusive scan of the 64 cell counts into s_off / s_cur and the
// unit descriptors (first slot | count << 10 | node base << 17).  The units
// are listed whole ones first, then the partial ones (each cell's last) by
// decreasing length, so that the two units a wave takes at a time have
// nearly the same length and the matrix core idles less on the shorter.
// The order depends only on the counts.
__device__ __forceinline__ void sc_scan_units(int lane, const int *s_cnt, int *s_off, int *s_cur, int *s_udesc,
                                              int *s_nunits) {
  const int v = s_cnt[lane];
  const int inc = sc_wave_scan(v);
  s_off[lane] = inc - v;
  s_cur[lane] = inc - v;
  const int nbase = (lane & 3) + SC_L * (((lane >> 2) & 3) + SC_L * (lane >> 4));
  const int nf = v / SC_UNIT, pl = v % SC_UNIT;  // whole units, length of the partial one
  const int finc = sc_wave_scan(nf);
  const int nfull = __shfl(finc, 63, 64);
  for (int q = 0; q < nf; ++q) s_udesc[finc - nf + q] = (inc - v + q * SC_UNIT) | (SC_UNIT << 10) | (nbase << 17);
  const uint64_t below = (1ull << lane) - 1ull;
  int pos = nfull;
  for (int len = SC_UNIT - 1; len > 0; --len) {
    const uint64_t m = __ballot(pl == len);
    if (pl == len) s_udesc[pos + __popcll(m & below)] = (inc - v + nf * SC_UNIT) | (len << 10) | (nbase << 17);
    pos += __popcll(m);
  }
  if (lane == 63) *s_nunits = pos;
}

// Stage one particle at `slot`: f, then m, q, A (A row-major).
__device__ __forceinline__ void sc_stage(float (*s_dat)[SC_PITCH], float4 *s_f, int slot, const float f[3], float m,
                                         const float q[3], const float A[9]) {
  s_f[slot] = make_float4(f[0], f[1], f[2], 0.f);
  s_dat[0][slot] = m;
  s_dat[1][slot] = q[0];
  s_dat[2][slot] = q[1];
  s_dat[3][slot] = q[2];
#pragma unroll
  for (int k = 0; k < 9; ++k) s_dat[4 + k][slot] = A[k];
}

// Pass over the units on the matrix cores; wave `wid` adds into wnode.
// Two adjacent units of the list (nearly equal lengths) per wave at a time.
__device__ __forceinline__ void sc_units_mfma(const ScLane &L, int wid, const float (*s_dat)[SC_PITCH],
                                              const float4 *s_f, const int *s_udesc, int nunits, float (*wnode)[4]) {
  for (int u = 2 * wid; u < nunits; u += 2 * SC_WAVES) {
    int k0[2], kn[2], cb[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int ue = u + e;
      const int d = ue < nunits ? s_udesc[ue] : 0;
      k0[e] = d & 1023;
      kn[e] = (d >> 10) & 127;
      cb[e] = d >> 17;
    }
    floatx4_t acc[2][2];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[e][t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    const int len = max(kn[0], kn[1]);
    for (int kk = 0; kk < len; kk += 4) {
      // LDS reads of both units' next four particles first
      float f3[2][3], av[2];
      bool live[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int r = kk + L.kq;
        live[e] = r < kn[e];
        const int jj = k0[e] + (live[e] ? r : 0);
        const float4 fv = s_f[jj];
        f3[e][0] = fv.x;
        f3[e][1] = fv.y;
        f3[e][2] = fv.z;
        av[e] = (live[e] && L.feat >= 0) ? s_dat[L.feat < 0 ? 0 : L.feat][jj] : 0.f;
      }
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          // no mask on w: a padding particle's feature operand is zero, a
          // padding column (offset >= 27) is dropped below, and w is finite
          // for both (f of a staged particle, the coefficients of offset 0)
          float w = 1.f;
#pragma unroll
          for (int d = 0; d < 3; ++d) w *= L.cfa[t][d] + f3[e][d] * (L.cfb[t][d] + L.cfc[t][d] * f3[e][d]);
          acc[e][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[e], w, acc[e][t], 0, 0, 0);
        }
    }
    // lane (kq, r16) holds rows 4 kq + i of column r16 (offset o) of each
    // tile: node value kq of node cell + o is row 4 kq + (1, ox, oy, oz).
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (kn[e] == 0) continue;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const floatx4_t a4 = acc[e][t];
        const float v = a4[0] + L.fo[t][0] * a4[1] + L.fo[t][1] * a4[2] + L.fo[t][2] * a4[3];
        if (L.oo[t] < 27) wnode[cb[e] + L.onode[t]][L.kq] += v;
      }
    }
  }
}

// Deterministic mode, second pass of the tile scatter: every node of an
// active node tile sums, in a fixed order (cell tile z, y, x, then work
// item), the partial node blocks (item_part, 6^3 x 4 values per work item)
// of the work items whose 6^3 region covers it.  ADJ = false (P2G):
// overwrites gm with value 0 and gmv with values 1-3.  ADJ = true (reverse
// G2P): adds values 1-3 into gmv, the grid-velocity adjoint.
// Bit-reproducible given a deterministic particle order.
template <bool ADJ>
static __global__ __launch_bounds__(256) void k_det_gather(GridDev g, const int32_t *__restrict__ node_tiles,
                                                        const int32_t *__restrict__ n_tiles,
                                                        const int32_t *__restrict__ tile_count,
                                                        const int32_t *__restrict__ item_first,
                                                        const float *__restrict__ item_part, float *__restrict__ gm,
                                                        float *__restrict__ gmv, int64_t N) {
  int nt = *n_tiles;
  int sub = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int it = blockIdx.x * 4 + sub; it < nt; it += gridDim.x * 4) {
    int t = node_tiles[it];
    int tx = t % g.tx, ty = (t / g.tx) % g.ty, tz = t / (g.tx * g.ty);
    int lx = l & 3, ly = (l >> 2) & 3, lz = l >> 4;
    int i = tx * 4 + lx, j = ty * 4 + ly, k = tz * 4 + lz;
    if (i >= g.nx || j >= g.ny || k >= g.nz) continue;
    float sm = 0.f, s0 = 0.f, s1 = 0.f, s2 = 0.f;
    for (int dz = 1; dz >= 0; --dz) {
      int cz = tz - dz, oz = lz + 4 * dz;
      if (cz < 0 || oz > 5) continue;
      for (int dy = 1; dy >= 0; --dy) {
        int cy = ty - dy, oy = ly + 4 * dy;
        if (cy < 0 || oy > 5) continue;
        for (int dxx = 1; dxx >= 0; --dxx) {
          int cx = tx - dxx, ox = lx + 4 * dxx;
          if (cx < 0 || ox > 5) continue;
          int ct = cx + g.tx * (cy + g.ty * cz);
          int nitem = (tile_count[ct] + WORK_CHUNK - 1) / WORK_CHUNK;
          int li = ox + SC_L * (oy + SC_L * oz);
          for (int q = 0; q < nitem; ++q) {
            const float *src = item_part + ((int64_t)(item_first[ct] + q) * SC_NODES + li) * 4;
            sm += src[0];
            s0 += src[1];
            s1 += src[2];
            s2 += src[3];
          }
        }
      }
    }
    int64_t node = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
    if (ADJ) {
      gmv[node] += s0;
      gmv[N + node] += s1;
      gmv[2 * N + node] += s2;
    } else {
      gm[node] = sm;
      gmv[node] = s0;
      gmv[N + node] = s1;
      gmv[2 * N + node] = s2;
    }
  }
}

}  // namespace dw
