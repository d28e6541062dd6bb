// BF16 MFMA 3x3x3 convolutions of the wind surrogate (gfx950), FP32 accumulation.
//
// The surrogate advances a wind velocity field k LBM steps at once:
//   u_{t+k} = u_t + g s net(u_t / s),  net = conv(32->3) o silu o conv(32->32)
//   o silu o conv(32->32) o silu o conv(3->32),  3x3x3 kernels, zero padding,
// s the per-field inflow speed, g a fixed output gain (the caller's scale of
// the output layer's residual).  Its error is measured against the lattice
// Boltzmann step of Eq. lbe.
//
// Implicit GEMM per layer: M = output channels (tiles of 16), N = a row of 16
// voxels along x, K = (tap, input channel).  Activations are channels-last
// BF16 [B][nz][ny][nx][C] with C padded to 8 (3-channel fields) or 32.  One
// v_mfma_f32_16x16x32_bf16 consumes K = 32: one tap of 32 channels, or four
// taps of 8 (padded) channels.  A workgroup (4 waves) stages zero-padded
// input patches of its output tiles in LDS; for 32-channel inputs a wave's
// m-tile weight fragments stay in registers for the life of the persistent
// workgroup.  Lane layout of the 16x16x32 MFMA: lane l holds
// A[l % 16][8 (l / 16) .. +8], B[8 (l / 16) .. +8][l % 16] and
// D[4 (l / 16) .. +4][l % 16].
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <climits>

#include "dw_internal.h"

namespace dw {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// float -> bf16, round to nearest even (one v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
// two floats -> packed bf16 pair (a in the low half), one instruction
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(float2v{a, b}, bf16x2));
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// logistic function with the hardware exponential and reciprocal (about
// 1 ulp each, far below the bf16 rounding of every value it feeds)
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float silu_grad(float z) {
  const float sg = sigmoid(z);
  return sg * (1.0f + z * (1.0f - sg));
}

constexpr int CT_X = 16, CT_Y = 4, CT_Z = 4;              // output voxels per workgroup tile
constexpr int PX = CT_X + 2, PY = CT_Y + 2, PZ = CT_Z + 2;  // staged input patch

struct ConvGeom {
  int B, nx, ny, nz;
  int64_t L;  // voxels per field
  int tiles_x, tiles_y, tiles_z;
  int64_t n_tiles;
};

// ----------------------------------------------------------------- forward
//
// Forward / data-gradient layer.  A workgroup (4 waves, 2 resident per CU)
// copies zero-padded input patches into LDS with buffer_load ... lds
// (channels-last, 16-byte chunks of 8 channels), then:
//  * 32-channel inputs: tiles of FX x FY x CZ = 16 x 4 x 4 outputs; a
//    workgroup walks a column of tiles along z, the patch planes in a ring
//    of RING slots, and copies the next tile's CZ new planes into the slots
//    the current tile does not read while its MFMAs run.  Wave w computes a
//    4 (y) x RZ (z) block of output rows for one 16-channel m-tile, holding
//    that m-tile's 27 weight fragments in registers for the life of the
//    kernel.  For each x-shift it walks the (RZ+2) x 6 input rows; every
//    fragment read from LDS feeds up to 3 RZ MFMAs (all (dz, dy) taps that
//    map it onto an output row).
//  * 8-channel inputs (3 channels padded): tiles of FX x FY x FZ = 16 x 4 x 8
//    outputs, one patch per tile; K = 32 spans 4 taps; each wave computes 8
//    whole rows, all m-tiles, two rows at a time.
// The 4 chunks of a voxel's 32 channels are stored permuted by swz(x) so the
// 16 lanes of a fragment read (16 consecutive x) spread over the LDS banks.

constexpr int FX = 16, FY = 4, FZ = 8;                 // output tile
constexpr int QX = FX + 2, QY = FY + 2, QZ = FZ + 2;   // input patch
constexpr int QVOX = QX * QY * QZ;

// 32-channel inputs: tiles of FX x FY x CZ outputs, walked along z; the
// patch planes live in a ring of RING slots of CPLANE elements in LDS
constexpr int CZ = 4, CQZ = CZ + 2, RING = QZ;
constexpr int CPLANE = QX * QY * 32;
static_assert(RING >= CQZ + CZ, "the next tile's new planes need slots of their own");

struct FwdTiles {
  int tx, ty, tz, n;  // tiles per axis, total over the batch
  // 32-channel inputs: work items are (column, z segment) pairs; a column is
  // the tzc tiles (CZ planes each) of one (x, y) tile position of one field
  int tzc, ncol, zlen, nitems;
};

struct TileOrigin {
  int b, x0, y0, z0;
};
__device__ __forceinline__ TileOrigin fwd_tile(const FwdTiles &T, int t) {
  TileOrigin o;
  o.x0 = (t % T.tx) * FX;
  int r = t / T.tx;
  o.y0 = (r % T.ty) * FY;
  r /= T.ty;
  o.z0 = (r % T.tz) * FZ;
  o.b = r / T.tz;
  return o;
}

// chunk c of a patch voxel with x index xx is stored at position c ^ swz(xx).
// A 16-byte LDS read is served 16 lanes (256 bytes) at a time; the 16 lanes
// of a fragment read take 16 consecutive x, whose voxels lie 64 bytes apart,
// so x and x + 4, x + 8, x + 12 would share banks without the permutation.
__device__ __forceinline__ int swz(int xx) { return (xx >> 2) & 3; }

typedef __attribute__((address_space(3))) void *lds_ptr_t;

// Copy the zero-padded input patch of a tile into LDS.  Chunk q of the patch
// lands at s_in + 16 q (each wave fills 64 consecutive chunks per
// instruction); voxels outside the field, and chunks past the patch up to the
// wave's 64, get an offset beyond the buffer's size, which the hardware
// returns as zeros: s_in must hold the patch rounded up to 64 chunks.
template <int CINP>
__device__ __forceinline__ void stage_patch(const ConvGeom &G, const uint16_t *__restrict__ x,
                                            const TileOrigin &o, uint16_t *s_in) {
  constexpr int VEC = CINP / 8;
  constexpr int NV = QVOX * VEC;
  constexpr int ITER = (NV + 255) / 256;
  // each iteration moves a lane 256 chunks = D voxels on through the patch:
  // its coordinates and field index advance by constant steps with carries
  // (no divisions or 32-bit multiplies per chunk)
  constexpr int D = 256 / VEC;
  constexpr int DX = D % QX, DY = (D / QX) % QY, DZ = D / (QX * QY);
  static_assert(256 % VEC == 0, "a lane keeps its channel chunk across iterations");
  const uint16_t *field = x + (int64_t)o.b * G.L * CINP;
  __amdgpu_buffer_rsrc_t rsrc =
      __builtin_amdgcn_make_buffer_rsrc((void *)field, (short)0, (int)(G.L * CINP * 2), 0x00020000);
  const int wid = threadIdx.x >> 6;
  int lane = threadIdx.x & 63;
  // recompute the per-lane patch coordinates for every tile rather than
  // keeping them live across the tile loop
  asm volatile("" : "+v"(lane));
  const int ql = wid * 64 + lane;  // this lane's chunk in iteration 0
  const int p = ql % VEC;
  const int v = ql / VEC;
  int xx = v % QX, yy = (v / QX) % QY;
  int gx = o.x0 + xx - 1, gy = o.y0 + yy - 1, gz = o.z0 + v / (QX * QY) - 1;
  const int sy = G.nx, sz = G.nx * G.ny;
  int lin = gx + sy * gy + sz * gz;
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int q0 = it * 256 + wid * 64;  // first chunk of this wave (uniform)
    if (q0 >= NV) break;
    const int q = q0 + lane;
    const int c = VEC == 4 ? (p ^ swz(xx)) : p;  // channel chunk stored at position p
    const bool in = q < NV && (unsigned)gx < (unsigned)G.nx && (unsigned)gy < (unsigned)G.ny &&
                    (unsigned)gz < (unsigned)G.nz;
    const unsigned off = in ? (unsigned)((lin * CINP + c * 8) * 2) : 0x80000000u;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_ptr_t)(s_in + q0 * 8), 16, off, 0, 0, 0);
    xx += DX; gx += DX; lin += DX;
    if (xx >= QX) { xx -= QX; gx -= QX; yy += 1; gy += 1; lin += sy - QX; }
    yy += DY; gy += DY; lin += DY * sy;
    if (yy >= QY) { yy -= QY; gy -= QY; gz += 1; lin += sz - QY * sy; }
    gz += DZ; lin += DZ * sz;
  }
}

// Copy planes zi0 .. zi0 + np - 1 of the zero-padded input patch of tile o
// (patch-relative z) into LDS at dst (np consecutive plane slots of
// QX * QY voxels).  Lanes past the range issue no copy, so the slots after
// the range are left as they are.
template <int CINP>
__device__ __forceinline__ void stage_planes(const ConvGeom &G, const uint16_t *__restrict__ x, const TileOrigin &o,
                                             uint16_t *dst, int zi0, int np) {
  constexpr int VEC = CINP / 8;
  constexpr int D = 256 / VEC;
  constexpr int DX = D % QX, DY = (D / QX) % QY, DZ = D / (QX * QY);
  static_assert(256 % VEC == 0, "a lane keeps its channel chunk across iterations");
  const int nch = np * QX * QY * VEC;
  const uint16_t *field = x + (int64_t)o.b * G.L * CINP;
  __amdgpu_buffer_rsrc_t rsrc =
      __builtin_amdgcn_make_buffer_rsrc((void *)field, (short)0, (int)(G.L * CINP * 2), 0x00020000);
  const int wid = threadIdx.x >> 6;
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  const int ql = wid * 64 + lane;
  const int p = ql % VEC;
  const int v = ql / VEC;
  int xx = v % QX, yy = (v / QX) % QY;
  int gx = o.x0 + xx - 1, gy = o.y0 + yy - 1, gz = o.z0 + zi0 + v / (QX * QY) - 1;
  const int sy = G.nx, sz = G.nx * G.ny;
  int lin = gx + sy * gy + sz * gz;
  for (int q0 = wid * 64; q0 < nch; q0 += 256) {
    const int q = q0 + lane;
    const int c = VEC == 4 ? (p ^ swz(xx)) : p;
    const bool in = (unsigned)gx < (unsigned)G.nx && (unsigned)gy < (unsigned)G.ny && (unsigned)gz < (unsigned)G.nz;
    const unsigned off = in ? (unsigned)((lin * CINP + c * 8) * 2) : 0x80000000u;
    if (q < nch) __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_ptr_t)(dst + q0 * 8), 16, off, 0, 0, 0);
    xx += DX; gx += DX; lin += DX;
    if (xx >= QX) { xx -= QX; gx -= QX; yy += 1; gy += 1; lin += sy - QX; }
    yy += DY; gy += DY; lin += DY * sy;
    if (yy >= QY) { yy -= QY; gy -= QY; gz += 1; lin += sz - QY * sy; }
    gz += DZ; lin += DZ * sz;
  }
}

// Work item v of the column plan: column v % ncol, z segment v / ncol.
struct ColItem {
  int b, x0, y0, zt0, zt1;  // field, tile origin in x and y, z tiles [zt0, zt1)
};
__device__ __forceinline__ ColItem col_item(const FwdTiles &T, int v) {
  ColItem c;
  const int col = v % T.ncol, seg = v / T.ncol;
  c.x0 = (col % T.tx) * FX;
  const int r = col / T.tx;
  c.y0 = (r % T.ty) * FY;
  c.b = r / T.ty;
  c.zt0 = seg * T.zlen;
  c.zt1 = min(T.tzc, c.zt0 + T.zlen);
  return c;
}

// Epilogue of one output row: lane holds channels co0 .. co0 + 3 of voxel
// vi of field o.b (acc = those 4 sums); live = the voxel is inside the field
// (ragged edge tiles).  Per-field bases plus 32-bit element offsets.
template <int COUTP, int EPI>
__device__ __forceinline__ void conv_epilogue(const ConvGeom &G, const TileOrigin &o, bool live, uint32_t vi,
                                              int co0, floatx4 acc, const float *s_bias, int cout,
                                              uint16_t *__restrict__ y, uint16_t *__restrict__ zpre,
                                              const uint16_t *__restrict__ zgate, const float *__restrict__ u,
                                              float sb, float *__restrict__ u_out) {
  if (!live) return;
  const uint32_t ei = vi * COUTP + co0;  // element offset in the field's activations
  const size_t fb = (size_t)o.b * G.L * COUTP;
  if (EPI == DW_CONV_HIDDEN) {
    float zv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) zv[j] = acc[j] + s_bias[co0 + j];
    *reinterpret_cast<uint2 *>(y + fb + ei) = make_uint2(f2bf2(silu(zv[0]), silu(zv[1])), f2bf2(silu(zv[2]), silu(zv[3])));
    if (zpre) *reinterpret_cast<uint2 *>(zpre + fb + ei) = make_uint2(f2bf2(zv[0], zv[1]), f2bf2(zv[2], zv[3]));
  } else if (EPI == DW_CONV_OUTPUT) {
    const size_t ub = (size_t)o.b * cout * G.L;
    const uint32_t L = (uint32_t)G.L;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int co = co0 + j;
      if (co < cout) {
        const uint32_t ui = (uint32_t)co * L + vi;
        u_out[ub + ui] = u[ub + ui] + sb * (acc[j] + s_bias[co]);
      }
    }
  } else {  // DW_CONV_DGRAD: gradient through the previous layer's silu
    const uint2 zg = *reinterpret_cast<const uint2 *>(zgate + fb + ei);
    const float zf[4] = {bf2f((uint16_t)(zg.x & 0xffff)), bf2f((uint16_t)(zg.x >> 16)), bf2f((uint16_t)(zg.y & 0xffff)),
                         bf2f((uint16_t)(zg.y >> 16))};
    float ob[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) ob[j] = acc[j] * silu_grad(zf[j]);
    *reinterpret_cast<uint2 *>(y + fb + ei) = make_uint2(f2bf2(ob[0], ob[1]), f2bf2(ob[2], ob[3]));
  }
}

// Packed weights: [chunk][COUTP][32] bf16, see conv_pack_weights.
template <int CINP, int COUTP, int EPI>
__global__ __launch_bounds__(256, 2) void k_conv(ConvGeom G, FwdTiles T, const uint16_t *__restrict__ x,
                                                 const uint16_t *__restrict__ wk, const float *__restrict__ bias,
                                                 int cout, uint16_t *__restrict__ y, uint16_t *__restrict__ zpre,
                                                 const uint16_t *__restrict__ zgate, const float *__restrict__ u,
                                                 const float *__restrict__ scale, float *__restrict__ u_out) {
  constexpr int MT = COUTP / 16;
  constexpr int PATCH = (QVOX * CINP / 8 + 63) / 64 * 64 * 8;  // bf16 elements, whole waves of chunks
  __shared__ __attribute__((aligned(16))) uint16_t s_in[PATCH];
  __shared__ float s_bias[32];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  if (threadIdx.x < 32) s_bias[threadIdx.x] = (bias && (int)threadIdx.x < cout) ? bias[threadIdx.x] : 0.f;

  if constexpr (CINP == 32) {
    // wave -> (m-tile, z rows of the 16 x 4 x 4 tile)
    constexpr int RZ = MT == 2 ? 2 : 1;
    const int mt = MT == 2 ? (wid & 1) : 0;
    const int zb = MT == 2 ? (wid >> 1) * 2 : wid;
    bf16x8 wf[27];
#pragma unroll
    for (int tap = 0; tap < 27; ++tap)
      wf[tap] = *reinterpret_cast<const bf16x8 *>(wk + ((tap * COUTP + mt * 16 + r16) * 32 + g * 8));
    // Work items in an order that gives the workgroups of one XCD (dispatch
    // is round-robin over the 8 XCDs) neighbouring columns, so the x and y
    // halos of concurrent tiles meet in one L2.  A column is walked along z
    // with its patch planes in a ring of RING slots: a tile reads CQZ slots,
    // and the CZ new planes of the column's next tile are copied into the
    // other CZ slots while this tile's MFMAs run.
    const int nb = (int)gridDim.x;
    int v = (nb & 7) ? (int)blockIdx.x : ((int)blockIdx.x & 7) * (nb >> 3) + ((int)blockIdx.x >> 3);
    ColItem ci{};
    int zt = 0, rot = 0;
    bool fresh = true;
    if (v < T.nitems) {
      ci = col_item(T, v);
      zt = ci.zt0;
    }
    floatx4 acc[RZ][FY];
    float uin[RZ][FY][3];
    TileOrigin op{};
    bool have_prev = false;
    auto epilogue = [&](const TileOrigin &oe) {
      const int gx = oe.x0 + r16;
      const uint32_t sy = (uint32_t)G.nx, sz = (uint32_t)G.nx * (uint32_t)G.ny;
      const uint32_t v00 = (uint32_t)gx + sy * (uint32_t)oe.y0 + sz * (uint32_t)(oe.z0 + zb);
      const float sb = EPI == DW_CONV_OUTPUT ? scale[oe.b] : 0.f;
#pragma unroll
      for (int zo = 0; zo < RZ; ++zo)
#pragma unroll
        for (int yo = 0; yo < FY; ++yo) {
          const bool live = gx < G.nx && oe.y0 + yo < G.ny && oe.z0 + zb + zo < G.nz;
          if constexpr (EPI == DW_CONV_OUTPUT) {
            // u_{t+k} = u_t + s (acc + bias), channels 0 .. cout-1 held by the lanes of group 0
            if (live && g == 0) {
              const size_t ub = (size_t)oe.b * cout * G.L;
              const uint32_t L = (uint32_t)G.L;
#pragma unroll
              for (int j = 0; j < 3; ++j)
                if (j < cout)
                  u_out[ub + (uint32_t)j * L + v00 + yo * sy + zo * sz] = uin[zo][yo][j] + sb * (acc[zo][yo][j] + s_bias[j]);
            }
          } else {
            conv_epilogue<COUTP, EPI>(G, oe, live, v00 + yo * sy + zo * sz, mt * 16 + 4 * g, acc[zo][yo], s_bias,
                                      cout, y, zpre, zgate, u, sb, u_out);
          }
        }
    };
    while (v < T.nitems) {
      const TileOrigin o{ci.b, ci.x0, ci.y0, zt * CZ};
      if (fresh) {
        __syncthreads();  // every wave is done with the previous tile's planes
        stage_planes<CINP>(G, x, o, s_in, 0, CQZ);
        rot = 0;
        fresh = false;
      }
      __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's copies have landed
      __syncthreads();  // every wave's have, and every wave is done with the previous tile
      const bool more = zt + 1 < ci.zt1;
      if (more) {
        // planes 2 .. CQZ-1 of the next tile into slots rot + CQZ .. rot + RING - 1
        const TileOrigin on{ci.b, ci.x0, ci.y0, (zt + 1) * CZ};
        const int s0 = rot + CQZ >= RING ? rot + CQZ - RING : rot + CQZ;
        const int n1 = RING - s0 < CZ ? RING - s0 : CZ;
        stage_planes<CINP>(G, x, on, s_in + s0 * CPLANE, 2, n1);
        if (n1 < CZ) stage_planes<CINP>(G, x, on, s_in, 2 + n1, CZ - n1);
      }
      // epilogue of the previous tile: its stores are issued before this
      // tile's MFMAs and complete while they run, so the next barrier does
      // not wait for them
      if (have_prev) epilogue(op);
      // output layer: the input field's values at this wave's outputs are
      // requested now and arrive during the MFMAs
      if constexpr (EPI == DW_CONV_OUTPUT) {
        const int gx = o.x0 + r16;
        const uint32_t sy = (uint32_t)G.nx, sz = (uint32_t)G.nx * (uint32_t)G.ny;
        const uint32_t v00 = (uint32_t)gx + sy * (uint32_t)o.y0 + sz * (uint32_t)(o.z0 + zb);
        const size_t ub = (size_t)o.b * cout * G.L;
        const uint32_t L = (uint32_t)G.L;
#pragma unroll
        for (int zo = 0; zo < RZ; ++zo)
#pragma unroll
          for (int yo = 0; yo < FY; ++yo) {
            const bool live = g == 0 && gx < G.nx && o.y0 + yo < G.ny && o.z0 + zb + zo < G.nz;
#pragma unroll
            for (int j = 0; j < 3; ++j)
              uin[zo][yo][j] = (live && j < cout) ? u[ub + (uint32_t)j * L + v00 + yo * sy + zo * sz] : 0.f;
          }
      }
#pragma unroll
      for (int zo = 0; zo < RZ; ++zo)
#pragma unroll
        for (int yo = 0; yo < FY; ++yo) acc[zo][yo] = floatx4{0.f, 0.f, 0.f, 0.f};
      // lane's fragment offset per x-shift; every read below adds a constant.
      // The empty asm keeps the compiler from hoisting 108 precomputed
      // addresses out of the tile loop (which costs 108 registers).
      int base[3];
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) base[dx] = (r16 + dx) * 32 + (g ^ swz(r16 + dx)) * 8;
      asm volatile("" : "+v"(base[0]), "+v"(base[1]), "+v"(base[2]));
      // LDS offset of the slot that holds patch plane zb + zi
      int poff[RZ + 2];
#pragma unroll
      for (int zi = 0; zi < RZ + 2; ++zi) {
        const int sl = rot + zb + zi;
        poff[zi] = (sl >= RING ? sl - RING : sl) * CPLANE;
      }
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
        for (int zi = 0; zi < RZ + 2; ++zi) {
          // the row's six fragments are read together, so their LDS latency
          // overlaps instead of stalling the matrix core per fragment
          bf16x8 bfr[QY];
#pragma unroll
          for (int yi = 0; yi < QY; ++yi)
            bfr[yi] = *reinterpret_cast<const bf16x8 *>(s_in + base[dx] + poff[zi] + QX * yi * 32);
          __builtin_amdgcn_sched_barrier(0);  // keep the six reads ahead of the MFMAs
#pragma unroll
          for (int yi = 0; yi < QY; ++yi) {
#pragma unroll
            for (int dz = 0; dz < 3; ++dz) {
              const int zo = zi - dz;
              if (zo < 0 || zo >= RZ) continue;
#pragma unroll
              for (int dy = 0; dy < 3; ++dy) {
                const int yo = yi - dy;
                if (yo < 0 || yo >= FY) continue;
                acc[zo][yo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[9 * dz + 3 * dy + dx], bfr[yi],
                                                                      acc[zo][yo], 0, 0, 0);
              }
            }
          }
        }
      }
      op = o;
      have_prev = true;
      if (more) {
        ++zt;
        rot = rot + CZ >= RING ? rot + CZ - RING : rot + CZ;
      } else {
        v += nb;
        if (v < T.nitems) {
          ci = col_item(T, v);
          zt = ci.zt0;
          fresh = true;
        }
      }
    }
    if (have_prev) epilogue(op);
  } else {
    // 8-channel input: chunk c covers taps 4c .. 4c + 3 (lane group g: tap 4c + g)
    bf16x8 wf[7][MT];
#pragma unroll
    for (int c = 0; c < 7; ++c)
#pragma unroll
      for (int m = 0; m < MT; ++m)
        wf[c][m] = *reinterpret_cast<const bf16x8 *>(wk + ((c * COUTP + m * 16 + r16) * 32 + g * 8));
    for (int t = blockIdx.x; t < T.n; t += gridDim.x) {
      const TileOrigin o = fwd_tile(T, t);
      __syncthreads();
      stage_patch<CINP>(G, x, o, s_in);
      __builtin_amdgcn_s_waitcnt(0x0f70);
      __syncthreads();
      const float sb = EPI == DW_CONV_OUTPUT ? scale[o.b] : 0.f;
#pragma unroll
      for (int pr = 0; pr < 4; ++pr) {
        floatx4 acc[2][MT];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int m = 0; m < MT; ++m) acc[i][m] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 7; ++c) {
          const int tap = 4 * c + g;
          const bool live = tap < 27;
          const int tt = live ? tap : 0;
          const int dz = tt / 9, dy = (tt / 3) % 3, dxx = tt % 3;
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const int row = wid * 8 + pr * 2 + i;  // row = yo + FY * zo
            const int yo = row % FY, zo = row / FY;
            int v = (r16 + dxx) + QX * ((yo + dy) + QY * (zo + dz));
            bf16x8 bfr = *reinterpret_cast<const bf16x8 *>(s_in + v * 8);
            if (!live) bfr = bf16x8{};
#pragma unroll
            for (int m = 0; m < MT; ++m)
              acc[i][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[c][m], bfr, acc[i][m], 0, 0, 0);
          }
        }
        const int gx = o.x0 + r16;
        const uint32_t sy = (uint32_t)G.nx, sz = (uint32_t)G.nx * (uint32_t)G.ny;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int row = wid * 8 + pr * 2 + i;
          const int gy = o.y0 + row % FY, gz = o.z0 + row / FY;
          const bool live = gx < G.nx && gy < G.ny && gz < G.nz;
          const uint32_t vi = (uint32_t)gx + sy * (uint32_t)gy + sz * (uint32_t)gz;
#pragma unroll
          for (int m = 0; m < MT; ++m)
            conv_epilogue<COUTP, EPI>(G, o, live, vi, m * 16 + 4 * g, acc[i][m], s_bias, cout, y, zpre, zgate, u, sb,
                                      u_out);
        }
      }
    }
  }
}

// u [B][3][L] float -> BF16 channels-last [B][L][8], scaled by 1/scale[b], padded with zeros
__global__ void k_conv_prep_input(ConvGeom G, const float *__restrict__ u, const float *__restrict__ scale,
                                  uint16_t *__restrict__ x0) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)G.B * G.L) return;
  int b = (int)(q / G.L);
  int64_t v = q - (int64_t)b * G.L;
  float is = 1.0f / scale[b];
  uint16_t h[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) h[c] = c < 3 ? f2bf(u[((int64_t)b * 3 + c) * G.L + v] * is) : (uint16_t)0;
  uint4 val = make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16),
                         h[4] | ((uint32_t)h[5] << 16), h[6] | ((uint32_t)h[7] << 16));
  *reinterpret_cast<uint4 *>(x0 + q * 8) = val;
}

// Pack FP32 weights w[cout][cin][27] (torch layout, tap = 9 dz + 3 dy + dx)
// into [chunk][COUTP][32] BF16 fragments.  flip != 0 packs the weights of
// the transposed convolution instead (data gradient): taps mirrored
// (26 - tap) and the roles of cin and cout exchanged.
__global__ void k_conv_pack(const float *__restrict__ w, int cin, int cout, int flip, int cinp, int coutp,
                            uint16_t *__restrict__ wk) {
  int nchunk = cinp == 32 ? 27 : 7;
  int64_t total = (int64_t)nchunk * coutp * 32;
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= total) return;
  int k = (int)(q % 32);
  int m = (int)((q / 32) % coutp);
  int c = (int)(q / (32 * coutp));
  int tap, ci;
  if (cinp == 32) {
    tap = c;
    ci = k;
  } else {
    tap = 4 * c + k / 8;
    ci = k % 8;
  }
  // the packed layer maps `cin_l` input channels to `cout_l` outputs
  int cin_l = flip ? cout : cin, cout_l = flip ? cin : cout;
  float val = 0.f;
  if (tap < 27 && ci < cin_l && m < cout_l) {
    if (flip) val = w[((int64_t)ci * cin + m) * 27 + (26 - tap)];  // w[co = ci][ci = m][mirrored tap]
    else val = w[((int64_t)m * cin + ci) * 27 + tap];
  }
  wk[q] = f2bf(val);
}

// Weight gradient of one layer on MFMA:
//   dW[tap][co][ci] = sum over voxels v of dz[v][co] * x[v + off(tap)][ci]
// (x zero-padded), M = co, K = 32 voxels per MFMA (two rows of 16), N =
// (dz, dy, ci) of one x-shift dx.  Per tile the output gradient is staged
// transposed as [co][256 voxels] and, once per dx, the input patch transposed
// and shifted as [ci][z][y][16 x], so every fragment is one aligned 16-byte
// LDS read.  Each wave owns a fixed quarter of the (dx, n-tile, m-tile)
// combinations and accumulates it over all its tiles; the workgroup's partial
// sums go to part[block][27][COUTP][CINP] and conv_wgrad_reduce adds the
// blocks in a fixed order.
template <int CINP, int COUTP>
__global__ __launch_bounds__(256) void k_conv_wgrad(ConvGeom G, const uint16_t *__restrict__ x,
                                                    const uint16_t *__restrict__ dz, int zs, int cout,
                                                    float *__restrict__ part) {
  constexpr int MT = COUTP / 16;
  constexpr int NPASS = 9 * CINP;                // n extent per dx pass
  constexpr int NT = (NPASS + 15) / 16;          // n tiles per pass
  constexpr int QP = NT * MT;                    // combinations per pass
  constexpr int NQ = (3 * QP + 3) / 4;           // accumulators per wave
  __shared__ __attribute__((aligned(16))) uint16_t s_dz[COUTP * 256];
  __shared__ __attribute__((aligned(16))) uint16_t s_x[CINP * PZ * PY * 16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  floatx4 acc[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) acc[a] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int64_t t = blockIdx.x; t < G.n_tiles; t += gridDim.x) {
    int tx = (int)(t % G.tiles_x);
    int ty = (int)((t / G.tiles_x) % G.tiles_y);
    int64_t r = t / ((int64_t)G.tiles_x * G.tiles_y);
    int tz = (int)(r % G.tiles_z);
    int b = (int)(r / G.tiles_z);
    int x0 = tx * CT_X, y0 = ty * CT_Y, z0 = tz * CT_Z;
    __syncthreads();
    for (int q = threadIdx.x; q < COUTP * 256; q += blockDim.x) {
      int v = q % 256, co = q / 256;
      int row = v / 16, xx = v % 16;
      int gx = x0 + xx, gy = y0 + row % CT_Y, gz = z0 + row / CT_Y;
      bool in = co < cout && gx < G.nx && gy < G.ny && gz < G.nz;
      int64_t gv = (int64_t)b * G.L + gx + (int64_t)G.nx * (gy + (int64_t)G.ny * gz);
      s_dz[q] = in ? dz[gv * zs + co] : (uint16_t)0;
    }
#pragma unroll 1
    for (int dx = 0; dx < 3; ++dx) {
      __syncthreads();
      for (int q = threadIdx.x; q < CINP * PZ * PY * 16; q += blockDim.x) {
        int xx = q % 16, yy = (q / 16) % PY, zz = (q / (16 * PY)) % PZ, ci = q / (16 * PY * PZ);
        int gx = x0 - 1 + dx + xx, gy = y0 - 1 + yy, gz = z0 - 1 + zz;
        uint16_t val = 0;
        if (gx >= 0 && gy >= 0 && gz >= 0 && gx < G.nx && gy < G.ny && gz < G.nz)
          val = x[((int64_t)b * G.L + gx + (int64_t)G.nx * (gy + (int64_t)G.ny * gz)) * CINP + ci];
        s_x[q] = val;
      }
      __syncthreads();
#pragma unroll
      for (int a = 0; a < NQ; ++a) {
        int qg = a * 4 + wid;
        if (qg >= 3 * QP || qg / QP != dx) continue;
        int qq = qg % QP;
        int mt = qq % MT, nt = qq / MT;
        int n = nt * 16 + r16;
        bool nlive = n < NPASS;
        int dzdy = nlive ? n / CINP : 0, ci = nlive ? n % CINP : 0;
        int ddz = dzdy / 3, ddy = dzdy % 3;
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
          int row = 2 * ks + (g >> 1), xo = 8 * (g & 1);
          bf16x8 af = *reinterpret_cast<const bf16x8 *>(s_dz + (mt * 16 + r16) * 256 + row * 16 + xo);
          int rz = row / CT_Y, ry = row % CT_Y;
          bf16x8 bfr = *reinterpret_cast<const bf16x8 *>(s_x + ((ci * PZ + rz + ddz) * PY + ry + ddy) * 16 + xo);
          if (!nlive) bfr = bf16x8{};
          acc[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, acc[a], 0, 0, 0);
        }
      }
    }
  }
  // lane holds D[co = mt*16 + 4g + j][n = nt*16 + r16]
#pragma unroll
  for (int a = 0; a < NQ; ++a) {
    int qg = a * 4 + wid;
    if (qg >= 3 * QP) continue;
    int dx = qg / QP, qq = qg % QP;
    int mt = qq % MT, nt = qq / MT;
    int n = nt * 16 + r16;
    if (n >= NPASS) continue;
    int dzdy = n / CINP, ci = n % CINP;
    int tap = (dzdy / 3) * 9 + (dzdy % 3) * 3 + dx;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int co = mt * 16 + 4 * g + j;
      part[(((int64_t)blockIdx.x * 27 + tap) * COUTP + co) * CINP + ci] = acc[a][j];
    }
  }
}

// dW[co][ci][tap] (+)= sum over blocks of part[block][tap][co][ci], fixed order
__global__ void k_conv_wgrad_reduce(const float *__restrict__ part, int nblocks, int cinp, int coutp, int cin,
                                    int cout, float *__restrict__ dw, int accumulate) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= cout * cin * 27) return;
  int tap = q % 27, ci = (q / 27) % cin, co = q / (27 * cin);
  float s = 0.f;
  for (int k = 0; k < nblocks; ++k) s += part[(((int64_t)k * 27 + tap) * coutp + co) * cinp + ci];
  dw[q] = accumulate ? dw[q] + s : s;
}

// bias gradient: db[c] = sum over voxels of dz[v][c], per-block partials
__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t *__restrict__ dz, int64_t nvox, int zs, int c,
                                                   float *__restrict__ part) {
  __shared__ float red[256];
  int ch = threadIdx.x % 32, ph = threadIdx.x / 32;
  float s = 0.f;
  if (ch < c)
    for (int64_t v = (int64_t)blockIdx.x * 8 + ph; v < nvox; v += (int64_t)gridDim.x * 8) s += bf2f(dz[v * zs + ch]);
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < 32) {
    float t = 0.f;
    for (int k = 0; k < 8; ++k) t += red[k * 32 + threadIdx.x];
    part[blockIdx.x * 32 + threadIdx.x] = t;
  }
}

__global__ void k_bias_grad_reduce(const float *__restrict__ part, int nblocks, int c, float *__restrict__ db,
                                   int accumulate) {
  int q = threadIdx.x;
  if (q >= c) return;
  float s = 0.f;
  for (int k = 0; k < nblocks; ++k) s += part[k * 32 + q];
  db[q] = accumulate ? db[q] + s : s;
}

// Loss L = mean over b, c, v of ((u_out - u_tgt) / s_b)^2 and its gradient
// with respect to the net output y (u_out = u + s y): dL/dy = 2 (u_out -
// u_tgt) / (s_b count), written as BF16 [B][L][8]; per-block loss partials.
__global__ __launch_bounds__(256) void k_mse_grad(ConvGeom G, const float *__restrict__ u_out,
                                                  const float *__restrict__ u_tgt, const float *__restrict__ scale,
                                                  uint16_t *__restrict__ dy, float *__restrict__ loss_part) {
  __shared__ float red[256];
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  double cnt = 3.0 * (double)G.B * (double)G.L;
  if (q < (int64_t)G.B * G.L) {
    int b = (int)(q / G.L);
    int64_t v = q - (int64_t)b * G.L;
    float is = 1.0f / scale[b];
    uint16_t h[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) h[c] = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      int64_t ui = ((int64_t)b * 3 + c) * G.L + v;
      float d = (u_out[ui] - u_tgt[ui]) * is;
      l += d * d;
      h[c] = f2bf((float)(2.0 * d / cnt));
    }
    uint4 val = make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16), 0, 0);
    *reinterpret_cast<uint4 *>(dy + q * 8) = val;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = (float)(red[0] / cnt);
}

// Adam (Kingma & Ba 2015) on FP32 parameters.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Per-field checks of a velocity field u [B][3][L] (solid [B][L] nullable,
// one mask per field): the sum of the squared central-difference divergence
// over interior fluid nodes, their count, and the kinetic energy 1/2 |u|^2
// summed over fluid nodes.  Pass 1: a workgroup takes rpi = 256 / nx rows
// of x per iteration (one row when nx >= 256), strides over the (y, z) rows
// of its field, and writes its three sums to part [B][nblk][3]; no node
// coordinate needs a 64-bit division and no two workgroups add to one
// address.  Pass 2 (k_field_stats_reduce) sums a field's partials in a
// fixed order in double, so the result does not depend on scheduling.
constexpr int FS_MAX_BLOCKS = 2048;

__host__ __device__ inline int fs_lanes_per_row(int nx) { return nx >= 256 ? 256 : nx; }

inline int fs_blocks(int nx, int ny, int nz) {
  const int64_t rpi = 256 / fs_lanes_per_row(nx);
  const int64_t need = ((int64_t)ny * nz + rpi - 1) / rpi;
  return (int)(need < FS_MAX_BLOCKS ? need : FS_MAX_BLOCKS);
}

__global__ __launch_bounds__(256) void k_field_stats(ConvGeom G, const float *__restrict__ u,
                                                     const uint8_t *__restrict__ solid, float *__restrict__ part) {
  __shared__ float r0[256 / 64], r1[256 / 64], r2[256 / 64];
  const int b = blockIdx.y;
  float dsum = 0.f, dcnt = 0.f, ke = 0.f;
  const float *ux = u + (int64_t)b * 3 * G.L, *uy = ux + G.L, *uz = uy + G.L;
  const uint8_t *sb = solid ? solid + (int64_t)b * G.L : nullptr;
  const int64_t sy = G.nx, sz = (int64_t)G.nx * G.ny;
  const int rows = G.ny * G.nz;
  const int lpr = fs_lanes_per_row(G.nx), rpi = 256 / lpr;
  const int sub = threadIdx.x / lpr, i0 = threadIdx.x - sub * lpr;
  if (sub < rpi) {
    for (int r = blockIdx.x * rpi + sub; r < rows; r += gridDim.x * rpi) {
      const int j = r % G.ny, k = r / G.ny;
      const bool inner_row = j > 0 && k > 0 && j < G.ny - 1 && k < G.nz - 1;
      const int64_t row0 = (int64_t)r * G.nx;
      for (int i = i0; i < G.nx; i += lpr) {
        const int64_t v = row0 + i;
        if (sb && sb[v]) continue;
        ke += 0.5f * (ux[v] * ux[v] + uy[v] * uy[v] + uz[v] * uz[v]);
        if (inner_row && i > 0 && i < G.nx - 1) {
          const float d = 0.5f * (ux[v + 1] - ux[v - 1] + uy[v + sy] - uy[v - sy] + uz[v + sz] - uz[v - sz]);
          dsum += d * d;
          dcnt += 1.f;
        }
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    dsum += __shfl_xor(dsum, o, 64);
    dcnt += __shfl_xor(dcnt, o, 64);
    ke += __shfl_xor(ke, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    r0[threadIdx.x >> 6] = dsum;
    r1[threadIdx.x >> 6] = dcnt;
    r2[threadIdx.x >> 6] = ke;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const float *rr = threadIdx.x == 0 ? r0 : threadIdx.x == 1 ? r1 : r2;
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < 256 / 64; ++w) t += rr[w];
    part[((int64_t)b * gridDim.x + blockIdx.x) * 3 + threadIdx.x] = t;
  }
}

// out[b][c] = sum over the nblk partials of field b (one workgroup per
// field; fixed summation order, double accumulation).
__global__ __launch_bounds__(256) void k_field_stats_reduce(int nblk, const float *__restrict__ part,
                                                            float *__restrict__ out) {
  __shared__ double s[3][256];
  const int b = blockIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int q = threadIdx.x; q < nblk; q += 256) {
    const float *pq = part + ((int64_t)b * nblk + q) * 3;
    a0 += pq[0];
    a1 += pq[1];
    a2 += pq[2];
  }
  s[0][threadIdx.x] = a0;
  s[1][threadIdx.x] = a1;
  s[2][threadIdx.x] = a2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      s[0][threadIdx.x] += s[0][threadIdx.x + h];
      s[1][threadIdx.x] += s[1][threadIdx.x + h];
      s[2][threadIdx.x] += s[2][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) out[b * 3 + threadIdx.x] = (float)s[threadIdx.x][0];
}

// Acceptance of surrogate fields on the device (no host synchronisation):
// from field_stats of the input fields (prev) and of the predictions (new),
// accept[b] = 1 iff the prediction's RMS divergence is at most div_factor
// times the input's and its kinetic energy is within [ke_lo, ke_hi] times
// the input's; a non-finite prediction makes its sums non-finite and fails
// both comparisons.  reject[b] = 1 - accept[b] (the skip flag of the
// fallback branch is the acceptance, its run flag the rejection).
__global__ void k_field_accept(int B, const float *__restrict__ prev, const float *__restrict__ pred,
                               float div_factor, float ke_lo, float ke_hi, int32_t *__restrict__ accept,
                               int32_t *__restrict__ reject) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float rms0 = sqrtf(prev[3 * b] / fmaxf(prev[3 * b + 1], 1.f));
  const float rms1 = sqrtf(pred[3 * b] / fmaxf(pred[3 * b + 1], 1.f));
  const float ratio = pred[3 * b + 2] / fmaxf(prev[3 * b + 2], 1e-30f);
  const bool ok = (rms1 <= div_factor * rms0 + 1e-12f) && (ratio >= ke_lo) && (ratio <= ke_hi);
  accept[b] = ok ? 1 : 0;
  if (reject) reject[b] = ok ? 0 : 1;
}

// u_out[b] = accept[b] ? u_pred[b] with zero velocity on solid nodes : u_alt[b]
__global__ void k_field_select(int B, int64_t L, const int32_t *__restrict__ accept, const float *__restrict__ u_pred,
                               const float *__restrict__ u_alt, const uint8_t *__restrict__ solid,
                               float *__restrict__ u_out) {
  const int b = blockIdx.y;
  const bool ok = accept[b] != 0;
  const float *src = (ok ? u_pred : u_alt) + (int64_t)b * 3 * L;
  const uint8_t *sb = solid ? solid + (int64_t)b * L : nullptr;
  float *dst = u_out + (int64_t)b * 3 * L;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < L; v += (int64_t)gridDim.x * blockDim.x) {
    const bool zero = ok && sb && sb[v];
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[c * L + v] = zero ? 0.f : src[c * L + v];
  }
}

static int make_geom(int B, int nx, int ny, int nz, ConvGeom *G) {
  DW_REQUIRE(B >= 1 && nx >= 1 && ny >= 1 && nz >= 1, DW_EINVAL, "conv: bad field size");
  DW_REQUIRE(nx <= (1 << 20) && ny <= (1 << 20) && nz <= (1 << 20), DW_ERANGE, "conv: field too large");
  G->B = B;
  G->nx = nx;
  G->ny = ny;
  G->nz = nz;
  G->L = (int64_t)nx * ny * nz;
  // byte offsets within one field's 32-channel activations fit 31 bits
  DW_REQUIRE(G->L * 64 < ((int64_t)1 << 31), DW_ERANGE, "conv: field too large (at most 2^25 voxels)");
  DW_REQUIRE(G->L * B < ((int64_t)1 << 31), DW_ERANGE, "conv: batch too large (at most 2^31 voxels)");
  G->tiles_x = (nx + CT_X - 1) / CT_X;  // edge tiles may be partial
  G->tiles_y = (ny + CT_Y - 1) / CT_Y;
  G->tiles_z = (nz + CT_Z - 1) / CT_Z;
  G->n_tiles = (int64_t)G->tiles_x * G->tiles_y * G->tiles_z * B;
  return DW_OK;
}

static FwdTiles fwd_tiles(const ConvGeom &G) {
  FwdTiles T;
  T.tx = (G.nx + FX - 1) / FX;
  T.ty = (G.ny + FY - 1) / FY;
  T.tz = (G.nz + FZ - 1) / FZ;
  T.n = T.tx * T.ty * T.tz * G.B;
  // columns, split into z segments when there are fewer columns than the
  // 512 resident workgroups
  T.tzc = (G.nz + CZ - 1) / CZ;
  T.ncol = T.tx * T.ty * G.B;
  int segs = T.ncol >= 512 ? 1 : (512 + T.ncol - 1) / T.ncol;
  segs = segs < T.tzc ? segs : T.tzc;
  T.zlen = (T.tzc + segs - 1) / segs;
  T.nitems = T.ncol * ((T.tzc + T.zlen - 1) / T.zlen);
  return T;
}

// persistent grid: two workgroups per CU
static unsigned fwd_blocks(const FwdTiles &T) { return (unsigned)(T.n < 512 ? T.n : 512); }
static unsigned col_blocks(const FwdTiles &T) { return (unsigned)(T.nitems < 512 ? T.nitems : 512); }

}  // namespace dw

using namespace dw;

extern "C" int conv_pack_weights(const float *w, int cin, int cout, int flip, uint16_t *wk, void *stream) {
  DW_REQUIRE(w && wk, DW_EINVAL, "conv_pack_weights: NULL pointer");
  DW_REQUIRE((cin == 3 || cin == 32) && (cout == 3 || cout == 32), DW_EINVAL,
             "conv_pack_weights: channels must be 3 or 32");
  int cin_l = flip ? cout : cin, cout_l = flip ? cin : cout;
  int cinp = cin_l == 3 ? 8 : 32, coutp = cout_l == 3 ? 16 : 32;
  int nchunk = cinp == 32 ? 27 : 7;
  int64_t total = (int64_t)nchunk * coutp * 32;
  hipLaunchKernelGGL(k_conv_pack, dim3(grid_blocks(total, 256)), dim3(256), 0, (hipStream_t)stream, w, cin, cout,
                     flip, cinp, coutp, wk);
  return check_launch("conv_pack_weights");
}

extern "C" size_t conv_packed_weight_elems(int cin, int cout) {
  int cinp = cin == 3 ? 8 : 32, coutp = cout == 3 ? 16 : 32;
  return (size_t)(cinp == 32 ? 27 : 7) * coutp * 32;
}

extern "C" int conv_prep_input(int B, int nx, int ny, int nz, const float *u, const float *scale, uint16_t *x0,
                               void *stream) {
  ConvGeom G;
  int rc = make_geom(B, nx, ny, nz, &G);
  if (rc) return rc;
  DW_REQUIRE(u && scale && x0, DW_EINVAL, "conv_prep_input: NULL pointer");
  hipLaunchKernelGGL(k_conv_prep_input, dim3(grid_blocks((int64_t)B * G.L, 256)), dim3(256), 0,
                     (hipStream_t)stream, G, u, scale, x0);
  return check_launch("conv_prep_input");
}

extern "C" int conv3d_bf16(int B, int nx, int ny, int nz, int cin, int cout, int epilogue, const uint16_t *x,
                           const uint16_t *wk, const float *bias, uint16_t *y, uint16_t *zpre, const uint16_t *zgate,
                           const float *u, const float *scale, float *u_out, void *stream) {
  ConvGeom G;
  int rc = make_geom(B, nx, ny, nz, &G);
  if (rc) return rc;
  DW_REQUIRE(x && wk, DW_EINVAL, "conv3d_bf16: x / weights NULL");
  DW_REQUIRE((cin == 3 || cin == 32) && (cout == 3 || cout == 32), DW_EINVAL, "conv3d_bf16: channels 3 or 32");
  hipStream_t s = (hipStream_t)stream;
  const FwdTiles T = fwd_tiles(G);
  const unsigned nb = fwd_blocks(T), nb32 = col_blocks(T);
  if (epilogue == DW_CONV_HIDDEN) {
    DW_REQUIRE(cout == 32 && bias && y, DW_EINVAL, "conv3d_bf16: hidden layer needs cout 32, bias, y");
    if (cin == 3)
      hipLaunchKernelGGL((k_conv<8, 32, DW_CONV_HIDDEN>), dim3(nb), dim3(256), 0, s, G, T, x, wk, bias, cout, y, zpre,
                         nullptr, nullptr, nullptr, nullptr);
    else
      hipLaunchKernelGGL((k_conv<32, 32, DW_CONV_HIDDEN>), dim3(nb32), dim3(256), 0, s, G, T, x, wk, bias, cout, y,
                         zpre, nullptr, nullptr, nullptr, nullptr);
  } else if (epilogue == DW_CONV_OUTPUT) {
    DW_REQUIRE(cin == 32 && cout == 3 && bias && u && scale && u_out, DW_EINVAL,
               "conv3d_bf16: output layer needs 32 -> 3, bias, u, scale, u_out");
    hipLaunchKernelGGL((k_conv<32, 16, DW_CONV_OUTPUT>), dim3(nb32), dim3(256), 0, s, G, T, x, wk, bias, cout, nullptr,
                       nullptr, nullptr, u, scale, u_out);
  } else if (epilogue == DW_CONV_DGRAD) {
    // transposed convolution of the gradient: input channels = the layer's cout
    DW_REQUIRE(cin == 32 && y && zgate, DW_EINVAL, "conv3d_bf16: data gradient needs cin 32 (the layer input), y, zgate");
    if (cout == 3)
      hipLaunchKernelGGL((k_conv<8, 32, DW_CONV_DGRAD>), dim3(nb), dim3(256), 0, s, G, T, x, wk, nullptr, 32, y,
                         nullptr, zgate, nullptr, nullptr, nullptr);
    else
      hipLaunchKernelGGL((k_conv<32, 32, DW_CONV_DGRAD>), dim3(nb32), dim3(256), 0, s, G, T, x, wk, nullptr, 32, y,
                         nullptr, zgate, nullptr, nullptr, nullptr);
  } else {
    return set_error(DW_EINVAL, "conv3d_bf16: unknown epilogue %d", epilogue);
  }
  return check_launch("conv3d_bf16");
}

constexpr int WGRAD_BLOCKS = 512;
constexpr int BGRAD_BLOCKS = 256;

extern "C" size_t conv_wgrad_scratch_floats(void) {
  return (size_t)WGRAD_BLOCKS * 27 * 32 * 32 + (size_t)BGRAD_BLOCKS * 32;
}

extern "C" int conv3d_bf16_wgrad(int B, int nx, int ny, int nz, int cin, int cout, const uint16_t *x,
                                 const uint16_t *dz, float *dw, float *db, int accumulate, float *scratch,
                                 void *stream) {
  ConvGeom G;
  int rc = make_geom(B, nx, ny, nz, &G);
  if (rc) return rc;
  DW_REQUIRE(x && dz && dw && scratch, DW_EINVAL, "conv3d_bf16_wgrad: NULL pointer");
  DW_REQUIRE((cin == 3 || cin == 32) && (cout == 3 || cout == 32), DW_EINVAL, "conv3d_bf16_wgrad: channels");
  hipStream_t s = (hipStream_t)stream;
  int cinp = cin == 3 ? 8 : 32, coutp = cout == 3 ? 16 : 32, zs = cout == 3 ? 8 : 32;
  unsigned nb = (unsigned)(G.n_tiles < WGRAD_BLOCKS ? G.n_tiles : WGRAD_BLOCKS);
  if (cinp == 8 && coutp == 32)
    hipLaunchKernelGGL((k_conv_wgrad<8, 32>), dim3(nb), dim3(256), 0, s, G, x, dz, zs, cout, scratch);
  else if (cinp == 32 && coutp == 32)
    hipLaunchKernelGGL((k_conv_wgrad<32, 32>), dim3(nb), dim3(256), 0, s, G, x, dz, zs, cout, scratch);
  else if (cinp == 32 && coutp == 16)
    hipLaunchKernelGGL((k_conv_wgrad<32, 16>), dim3(nb), dim3(256), 0, s, G, x, dz, zs, cout, scratch);
  else
    return set_error(DW_EINVAL, "conv3d_bf16_wgrad: unsupported layer %d -> %d", cin, cout);
  hipLaunchKernelGGL(k_conv_wgrad_reduce, dim3(grid_blocks((int64_t)cout * cin * 27, 256)), dim3(256), 0, s,
                     scratch, (int)nb, cinp, coutp, cin, cout, dw, accumulate);
  if (db) {
    float *bpart = scratch + (size_t)WGRAD_BLOCKS * 27 * 32 * 32;
    hipLaunchKernelGGL(k_bias_grad, dim3(BGRAD_BLOCKS), dim3(256), 0, s, dz, (int64_t)B * G.L, zs, cout, bpart);
    hipLaunchKernelGGL(k_bias_grad_reduce, dim3(1), dim3(32), 0, s, bpart, BGRAD_BLOCKS, cout, db, accumulate);
  }
  return check_launch("conv3d_bf16_wgrad");
}

extern "C" int conv_mse_grad(int B, int nx, int ny, int nz, const float *u_out, const float *u_tgt,
                             const float *scale, uint16_t *dy, float *loss_part, void *stream) {
  ConvGeom G;
  int rc = make_geom(B, nx, ny, nz, &G);
  if (rc) return rc;
  DW_REQUIRE(u_out && u_tgt && scale && dy && loss_part, DW_EINVAL, "conv_mse_grad: NULL pointer");
  hipLaunchKernelGGL(k_mse_grad, dim3(grid_blocks((int64_t)B * G.L, 256)), dim3(256), 0, (hipStream_t)stream, G,
                     u_out, u_tgt, scale, dy, loss_part);
  return check_launch("conv_mse_grad");
}

extern "C" int adam_step(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                         float eps, int step, void *stream) {
  DW_REQUIRE(p && g && m && v && n >= 0 && step >= 1, DW_EINVAL, "adam_step: bad arguments");
  float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, p, g, m, v, n, lr, b1, b2,
                     eps, bc1, bc2);
  return check_launch("adam_step");
}

extern "C" size_t field_stats_workspace_bytes(int B, int nx, int ny, int nz) {
  if (B < 1 || B > 65535 || nx < 1 || ny < 1 || nz < 1 || (int64_t)ny * nz >= (1LL << 31)) return 0;
  return (size_t)B * fs_blocks(nx, ny, nz) * 3 * sizeof(float);
}

extern "C" int field_stats(int B, int nx, int ny, int nz, const float *u, const uint8_t *solid, float *out, void *ws,
                           size_t ws_bytes, void *stream) {
  DW_REQUIRE(B >= 1 && nx >= 1 && ny >= 1 && nz >= 1 && B <= 65535, DW_EINVAL, "field_stats: bad size");
  DW_REQUIRE(u && out && ws, DW_EINVAL, "field_stats: NULL pointer");
  DW_REQUIRE((int64_t)ny * nz < (1LL << 31), DW_ERANGE, "field_stats: too many rows");
  const int nblk = fs_blocks(nx, ny, nz);
  DW_REQUIRE(ws_bytes >= (size_t)B * nblk * 3 * sizeof(float), DW_EWORKSPACE, "field_stats: workspace too small");
  ConvGeom G{};
  G.B = B;
  G.nx = nx;
  G.ny = ny;
  G.nz = nz;
  G.L = (int64_t)nx * ny * nz;
  float *part = static_cast<float *>(ws);
  hipLaunchKernelGGL(k_field_stats, dim3(nblk, B), dim3(256), 0, (hipStream_t)stream, G, u, solid, part);
  int rc = check_launch("field_stats");
  if (rc) return rc;
  hipLaunchKernelGGL(k_field_stats_reduce, dim3(B), dim3(256), 0, (hipStream_t)stream, nblk, part, out);
  return check_launch("field_stats_reduce");
}

extern "C" int field_accept(int B, const float *stats_prev, const float *stats_pred, float div_factor, float ke_lo,
                            float ke_hi, int32_t *accept, int32_t *reject, void *stream) {
  DW_REQUIRE(B >= 1 && stats_prev && stats_pred && accept, DW_EINVAL, "field_accept: bad arguments");
  DW_REQUIRE(reject != accept, DW_EINVAL, "field_accept: reject must not alias accept");
  hipLaunchKernelGGL(k_field_accept, dim3(grid_blocks(B, 64)), dim3(64), 0, (hipStream_t)stream, B, stats_prev,
                     stats_pred, div_factor, ke_lo, ke_hi, accept, reject);
  return check_launch("field_accept");
}

extern "C" int field_select(int B, int nx, int ny, int nz, const int32_t *accept, const float *u_pred,
                            const float *u_alt, const uint8_t *solid, float *u_out, void *stream) {
  DW_REQUIRE(B >= 1 && B <= 65535 && nx >= 1 && ny >= 1 && nz >= 1, DW_EINVAL, "field_select: bad size");
  DW_REQUIRE(accept && u_pred && u_alt && u_out, DW_EINVAL, "field_select: NULL pointer");
  const int64_t L = (int64_t)nx * ny * nz;
  unsigned bx = grid_blocks(L, 256);
  if (bx > 2048) bx = 2048;
  hipLaunchKernelGGL(k_field_select, dim3(bx, B), dim3(256), 0, (hipStream_t)stream, B, L, accept, u_pred, u_alt,
                     solid, u_out);
  return check_launch("field_select");
}
