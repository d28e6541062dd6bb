// Differentiable rendering of the 3D Gaussian kernels and the photometric
// loss L_render (Sec. 3.3, Eq. rendering and L_render; appendix "3D Gaussian
// Representation").
//
// Forward (gs_render), every stage a kernel of this file:
//   1. k_gs_project: per kernel, camera point p = R mu + t, projected centre,
//      2-D covariance J R Sigma R^T J^T and its inverse (the conic), the
//      pixel box where alpha can reach alpha_min, and the 16 x 16 pixel
//      tiles that box covers.  Kernels behind the near plane, with a
//      degenerate 2-D covariance or with no pixel in reach are not drawn.
//   2. stable LSD radix sort of (depth bits, kernel) -- 4 passes of 8 bits;
//      kernels that are not drawn carry the largest key and no tiles.
//   3. exclusive scan of the tile counts in depth order; every drawn kernel
//      writes one (tile, kernel) pair per covered tile, in depth order.
//   4. stable radix sort of the pairs by tile (depth order kept inside a
//      tile), then each tile's range in the sorted list.
//   5. k_gs_raster: one 256-thread workgroup per tile, one pixel per thread;
//      batches of 256 kernels staged in LDS, alpha blended front to back.
//      A pixel stops once its transmittance falls below t_min; its count of
//      blended list entries is kept for the reverse pass.
// Reverse (gs_render_adj): the same traversal per pixel, front to back,
// recomputing alpha and T; dC/dalpha_i = T_i c_i - (C - A_i) / (1 - alpha_i)
// with A_i the colour blended up to and including i (C includes the
// background term).  The reverse pass runs one wave per tile with four
// pixels per lane: per-kernel adjoints of the centre, conic, opacity and
// colour are summed over the lane's pixels, then over the wave with DPP
// row operations, and added to global memory with one atomic per value;
// k_gs_project_adj then takes the centre and conic adjoints back to mu and
// Sigma through the projection.
// Loss (render_loss): L1 and SSIM with an 11 x 11 Gaussian window
// (sigma 1.5, zero padding) per channel; the five window sums are separable
// convolutions staged in LDS; the gradient of the SSIM mean is the window
// correlation of the per-pixel partial derivatives (the window is
// symmetric).  Loss partial sums are reduced in a fixed order.
#include <hip/hip_runtime.h>

#include "dw_internal.h"

namespace dw {

constexpr int GS_TILE = 16;
constexpr int GS_THREADS = GS_TILE * GS_TILE;
constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_CHUNK = RS_THREADS * RS_ROUNDS;  // keys per radix-sort block
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER = 8;
constexpr int SCAN_CHUNK = SCAN_THREADS * SCAN_PER;
constexpr int SCAN_TOP_THREADS = 1024;
constexpr int SCAN_TOP_MAX = SCAN_TOP_THREADS * 16;  // block sums the top level scans

// workspace header: [0] status, [1] pair count, [GS_CNT0 ...] 64 partial
// 64-bit pair totals (one per block residue, to spread the atomics)
constexpr int GS_HDR_INTS = 256;
constexpr int GS_CNT0 = 64;
constexpr int GS_NCNT = 64;

struct CamDev {
  int W, H, tw, th;
  float fx, fy, cx, cy;
  float R[9], t[3];
  float near_, amin, tmin;
  float bg[3];
};

// Workspace of gs_render / gs_render_adj (all sections 256-aligned):
//   header [256] int32: status, pair count, 64 partial pair totals (u64)
//   rec [n] 3 float4: (mx, my, A, B), (C, o, c0, c1), (c2, -, -, -)
//   rect [n] int4 tile box (tx0, tx1, ty0, ty1); cnt [n] int32
//   key_a, key_b [n] u32, id_a, id_b [n] int32   (depth sort)
//   off [n + 1] int32 (tile-count scan in depth order)
//   pk_a, pk_b [P] u32, pv_a, pv_b [P] int32      (pair sort)
//   hist [256 * nblk(max(n, P))] int32, bsum [SCAN_TOP_MAX] int32
//   range [T] int2, last [W * H] int32
//   gbar [5][n] float (centre and conic adjoints, reverse pass)
struct GsWs {
  int32_t *hdr;
  float4 *rec;
  int4 *rect;
  int32_t *cnt;
  uint32_t *key_a, *key_b;
  int32_t *id_a, *id_b;
  int32_t *off;
  uint32_t *pk_a, *pk_b;
  int32_t *pv_a, *pv_b;
  int32_t *hist, *bsum;
  int2 *range;
  int32_t *last;
  float *gbar;
  size_t bytes;
};

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

static int64_t rs_blocks(int64_t m) { return (m + RS_CHUNK - 1) / RS_CHUNK; }

static GsWs gs_layout(char *base, int64_t n, int64_t P, int W, int H) {
  GsWs w;
  const int64_t T = (int64_t)((W + GS_TILE - 1) / GS_TILE) * ((H + GS_TILE - 1) / GS_TILE);
  const int64_t nb = rs_blocks(n > P ? n : P);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + o : nullptr;
    o += al256(bytes);
    return p;
  };
  w.hdr = (int32_t *)take(GS_HDR_INTS * 4);
  w.rec = (float4 *)take((size_t)n * 3 * sizeof(float4));
  w.rect = (int4 *)take((size_t)n * sizeof(int4));
  w.cnt = (int32_t *)take((size_t)n * 4);
  w.key_a = (uint32_t *)take((size_t)n * 4);
  w.key_b = (uint32_t *)take((size_t)n * 4);
  w.id_a = (int32_t *)take((size_t)n * 4);
  w.id_b = (int32_t *)take((size_t)n * 4);
  w.off = (int32_t *)take((size_t)(n + 1) * 4);
  w.pk_a = (uint32_t *)take((size_t)P * 4);
  w.pk_b = (uint32_t *)take((size_t)P * 4);
  w.pv_a = (int32_t *)take((size_t)P * 4);
  w.pv_b = (int32_t *)take((size_t)P * 4);
  w.hist = (int32_t *)take((size_t)256 * nb * 4);
  w.bsum = (int32_t *)take((size_t)SCAN_TOP_MAX * 4);
  w.range = (int2 *)take((size_t)T * sizeof(int2));
  w.last = (int32_t *)take((size_t)W * H * 4);
  w.gbar = (float *)take((size_t)5 * n * 4);
  w.bytes = o;
  return w;
}

// ------------------------------------------------------------- projection

// Everything of one kernel that the raster and its reverse need.
struct Proj {
  bool drawn;
  float px, py, pz;      // camera point
  float mx, my;          // projected centre (pixels)
  float a, b, c;         // 2-D covariance [[a, b], [b, c]]
  float A, B, C;         // its inverse
  float T0[3], T1[3];    // rows of J R
  int tx0, tx1, ty0, ty1;
};

__device__ __forceinline__ Proj gs_proj(const CamDev &K, float mux, float muy, float muz, const float S[6],
                                        float o) {
  Proj r;
  r.drawn = false;
  r.tx0 = r.ty0 = 0;
  r.tx1 = r.ty1 = -1;
  r.px = K.R[0] * mux + K.R[1] * muy + K.R[2] * muz + K.t[0];
  r.py = K.R[3] * mux + K.R[4] * muy + K.R[5] * muz + K.t[1];
  r.pz = K.R[6] * mux + K.R[7] * muy + K.R[8] * muz + K.t[2];
  if (!(r.pz > K.near_)) return r;
  const float iz = 1.0f / r.pz;
  r.mx = K.fx * r.px * iz + K.cx;
  r.my = K.fy * r.py * iz + K.cy;
  // J = [[fx/z, 0, -fx px/z^2], [0, fy/z, -fy py/z^2]]; T = J R
  const float j00 = K.fx * iz, j02 = -K.fx * r.px * iz * iz;
  const float j11 = K.fy * iz, j12 = -K.fy * r.py * iz * iz;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    r.T0[c] = j00 * K.R[c] + j02 * K.R[6 + c];
    r.T1[c] = j11 * K.R[3 + c] + j12 * K.R[6 + c];
  }
  // Sigma T^T columns
  const float Sm[9] = {S[0], S[3], S[4], S[3], S[1], S[5], S[4], S[5], S[2]};
  float u0[3], u1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u0[a] = Sm[3 * a] * r.T0[0] + Sm[3 * a + 1] * r.T0[1] + Sm[3 * a + 2] * r.T0[2];
    u1[a] = Sm[3 * a] * r.T1[0] + Sm[3 * a + 1] * r.T1[1] + Sm[3 * a + 2] * r.T1[2];
  }
  r.a = r.T0[0] * u0[0] + r.T0[1] * u0[1] + r.T0[2] * u0[2];
  r.b = r.T0[0] * u1[0] + r.T0[1] * u1[1] + r.T0[2] * u1[2];
  r.c = r.T1[0] * u1[0] + r.T1[1] * u1[1] + r.T1[2] * u1[2];
  const float det = r.a * r.c - r.b * r.b;
  if (!(det > 0.f) || !(r.a > 0.f)) return r;
  const float id = 1.0f / det;
  r.A = r.c * id;
  r.B = -r.b * id;
  r.C = r.a * id;
  // pixel box: alpha = o exp(-q/2) >= amin  <=>  q <= Q = 2 ln(o / amin);
  // the ellipse q <= Q reaches sqrt(Q a) in x and sqrt(Q c) in y (padded by a
  // relative 1e-4 and 1e-3 pixel against rounding at the rim)
  int i0 = 0, i1 = K.W - 1, j0 = 0, j1 = K.H - 1;
  if (K.amin > 0.f) {
    if (!(o >= K.amin)) return r;
    const float Q = 2.0f * logf(o / K.amin);
    const float ex = sqrtf(Q * r.a) * 1.0001f + 1e-3f, ey = sqrtf(Q * r.c) * 1.0001f + 1e-3f;
    const float fx0 = ceilf(r.mx - ex - 0.5f), fx1 = floorf(r.mx + ex - 0.5f);
    const float fy0 = ceilf(r.my - ey - 0.5f), fy1 = floorf(r.my + ey - 0.5f);
    if (!(fx1 >= 0.f && fx0 <= (float)(K.W - 1) && fy1 >= 0.f && fy0 <= (float)(K.H - 1))) return r;
    i0 = (int)fmaxf(fx0, 0.f);
    i1 = (int)fminf(fx1, (float)(K.W - 1));
    j0 = (int)fmaxf(fy0, 0.f);
    j1 = (int)fminf(fy1, (float)(K.H - 1));
    if (i0 > i1 || j0 > j1) return r;
  }
  r.tx0 = i0 / GS_TILE;
  r.tx1 = i1 / GS_TILE;
  r.ty0 = j0 / GS_TILE;
  r.ty1 = j1 / GS_TILE;
  r.drawn = true;
  return r;
}

__global__ __launch_bounds__(256) void k_gs_project(CamDev K, int n, const float *__restrict__ mu,
                                                    const float *__restrict__ sigma, const float *__restrict__ col,
                                                    const float *__restrict__ op, GsWs w) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const bool has = g < n;
  float S[6] = {1.f, 1.f, 1.f, 0.f, 0.f, 0.f};
  float o = 0.f, m0 = 0.f, m1 = 0.f, m2 = 0.f;
  if (has) {
#pragma unroll
    for (int e = 0; e < 6; ++e) S[e] = sigma[(int64_t)e * n + g];
    o = op[g];
    m0 = mu[g];
    m1 = mu[(int64_t)n + g];
    m2 = mu[2 * (int64_t)n + g];
  }
  Proj r = gs_proj(K, m0, m1, m2, S, o);
  r.drawn = r.drawn && has;
  int c = 0;
  uint32_t key = 0xffffffffu;
  if (r.drawn) {
    c = (r.tx1 - r.tx0 + 1) * (r.ty1 - r.ty0 + 1);
    key = __float_as_uint(r.pz);  // pz > near >= 0: the bits order like the values
    w.rec[3 * (int64_t)g] = make_float4(r.mx, r.my, r.A, r.B);
    w.rec[3 * (int64_t)g + 1] = make_float4(r.C, o, col[g], col[(int64_t)n + g]);
    w.rec[3 * (int64_t)g + 2] = make_float4(col[2 * (int64_t)n + g], 0.f, 0.f, 0.f);
  }
  if (has) {
    w.rect[g] = make_int4(r.tx0, r.tx1, r.ty0, r.ty1);
    w.cnt[g] = c;
    w.key_a[g] = key;
    w.id_a[g] = g;
  }
  // 64-bit pair total (the int32 scan below is only trusted when it fits):
  // a block sum added to one of 64 partial counters
  __shared__ unsigned long long s_c[256 / 64];
  unsigned long long sw = (unsigned long long)c;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) sw += __shfl_xor(sw, m, 64);
  if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = sw;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long b = s_c[0] + s_c[1] + s_c[2] + s_c[3];
    if (b) atomicAdd(reinterpret_cast<unsigned long long *>(w.hdr + GS_CNT0) + (blockIdx.x % GS_NCNT), b);
  }
}

// ------------------------------------------------------------ scan (int32)

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int sh = 1; sh < 64; sh <<= 1) {
    const int t = __shfl_up(v, sh, 64);
    if (lane >= sh) v += t;
  }
  return v;
}

// exclusive scan of the per-thread values of a 256-thread block; returns the
// thread's offset, *total the block sum
__device__ __forceinline__ int block_excl_scan(int v, int *s_w, int *total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int inc = wave_incl_scan(v, lane);
  if (lane == 63) s_w[wid] = inc;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < SCAN_THREADS / 64; ++q) {
    base += q < wid ? s_w[q] : 0;
    tot += s_w[q];
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

// Length m may live on the device (m_dev, not NULL) with m_cap as bound.
__device__ __forceinline__ int64_t dev_len(const int32_t *m_dev, int64_t m_cap) {
  if (!m_dev) return m_cap;
  const int64_t m = *m_dev;
  return m <= m_cap ? m : 0;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(const int32_t *__restrict__ in, int64_t m_cap,
                                                            const int32_t *m_dev, int32_t *__restrict__ bsum) {
  __shared__ int s_w[SCAN_THREADS / 64];
  const int64_t m = dev_len(m_dev, m_cap);
  const int64_t b0 = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
  int v = 0;
#pragma unroll
  for (int q = 0; q < SCAN_PER; ++q) v += b0 + q < m ? in[b0 + q] : 0;
  int tot;
  block_excl_scan(v, s_w, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// one 1024-thread block: exclusive scan of nb <= SCAN_TOP_MAX block sums in
// place, the grand total to *total
__global__ __launch_bounds__(SCAN_TOP_THREADS) void k_scan_top(int32_t *__restrict__ bsum, int nb,
                                                               int32_t *__restrict__ total) {
  __shared__ int s_w[SCAN_TOP_THREADS / 64];
  constexpr int PER = SCAN_TOP_MAX / SCAN_TOP_THREADS;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int b0 = threadIdx.x * PER;
  int v[PER], s = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    v[q] = b0 + q < nb ? bsum[b0 + q] : 0;
    s += v[q];
  }
  const int inc = wave_incl_scan(s, lane);
  if (lane == 63) s_w[wid] = inc;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < SCAN_TOP_THREADS / 64; ++q) {
    base += q < wid ? s_w[q] : 0;
    tot += s_w[q];
  }
  int run = base + inc - s;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (b0 + q < nb) bsum[b0 + q] = run;
    run += v[q];
  }
  if (threadIdx.x == 0 && total) *total = tot;
}

// out[i] = bsum[block] + exclusive scan of in inside the block; out may alias in
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(const int32_t *in, int64_t m_cap, const int32_t *m_dev,
                                                             const int32_t *__restrict__ bsum, int32_t *out) {
  __shared__ int s_w[SCAN_THREADS / 64];
  const int64_t m = dev_len(m_dev, m_cap);
  const int64_t b0 = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
  int v[SCAN_PER], s = 0;
#pragma unroll
  for (int q = 0; q < SCAN_PER; ++q) {
    v[q] = b0 + q < m ? in[b0 + q] : 0;
    s += v[q];
  }
  int tot;
  int run = bsum[blockIdx.x] + block_excl_scan(s, s_w, &tot);
#pragma unroll
  for (int q = 0; q < SCAN_PER; ++q) {
    if (b0 + q < m) out[b0 + q] = run;
    run += v[q];
  }
}

// Exclusive scan of in[0, m) into out (may alias), m = min(*m_dev, m_cap)
// when m_dev is set; *total (optional) receives the sum.
static void scan_excl(const int32_t *in, int32_t *out, int64_t m_cap, const int32_t *m_dev, int32_t *bsum,
                      int32_t *total, hipStream_t s) {
  const int64_t nb = (m_cap + SCAN_CHUNK - 1) / SCAN_CHUNK;
  const unsigned g = (unsigned)(nb < 1 ? 1 : nb);
  hipLaunchKernelGGL(k_scan_sums, dim3(g), dim3(SCAN_THREADS), 0, s, in, m_cap, m_dev, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_TOP_THREADS), 0, s, bsum, (int)g, total);
  hipLaunchKernelGGL(k_scan_apply, dim3(g), dim3(SCAN_THREADS), 0, s, in, m_cap, m_dev, bsum, out);
}

// -------------------------------------------------- stable LSD radix sort
//
// One pass sorts by the 8-bit digit at `shift`: per block of RS_CHUNK keys a
// digit histogram (hist[digit][block]), an exclusive scan of the histogram
// in that order, then each block places its keys in 16 rounds of 256: a
// key's slot is its digit's running base in the block plus the same-digit
// keys before it in the round (earlier waves from LDS counts, earlier lanes
// of its wave from a 64-bit peer mask built with eight ballots).  Keys of
// equal digit keep their input order, so the passes compose to a stable sort.

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint32_t *__restrict__ key, int64_t m_cap,
                                                        const int32_t *m_dev, int shift, int32_t *__restrict__ hist,
                                                        int nblk) {
  __shared__ int s_h[256];
  const int64_t m = dev_len(m_dev, m_cap);
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * RS_CHUNK;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = b0 + r * RS_THREADS + threadIdx.x;
    if (i < m) atomicAdd(&s_h[(key[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = s_h[threadIdx.x];
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint32_t *__restrict__ kin,
                                                           const int32_t *__restrict__ vin, int64_t m_cap,
                                                           const int32_t *m_dev, int shift,
                                                           const int32_t *__restrict__ hist, int nblk,
                                                           uint32_t *__restrict__ kout, int32_t *__restrict__ vout) {
  __shared__ int s_base[256];
  __shared__ int s_wc[RS_THREADS / 64][256];
  const int64_t m = dev_len(m_dev, m_cap);
  const int64_t b0 = (int64_t)blockIdx.x * RS_CHUNK;
  if (b0 >= m) return;  // block-uniform
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  s_base[threadIdx.x] = hist[(int64_t)threadIdx.x * nblk + blockIdx.x];
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int r = 0; r < RS_ROUNDS; ++r) {
#pragma unroll
    for (int w = 0; w < RS_THREADS / 64; ++w) s_wc[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = b0 + r * RS_THREADS + threadIdx.x;
    const bool valid = i < m;
    uint32_t k = 0;
    int32_t v = 0;
    if (valid) {
      k = kin[i];
      v = vin[i];
    }
    const uint32_t d = (k >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t bal = __ballot(valid && ((d >> bit) & 1u));
      peers &= ((d >> bit) & 1u) ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt);
    if (valid && (peers >> lane) == 1ull) s_wc[wid][d] = __popcll(peers);  // the highest lane of its digit
    __syncthreads();
    if (valid) {
      int pos = s_base[d] + rank;
      for (int w = 0; w < wid; ++w) pos += s_wc[w][d];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int w = 0; w < RS_THREADS / 64; ++w) add += s_wc[w][threadIdx.x];
    s_base[threadIdx.x] += add;
    // the next round's clear is ordered after these reads by its barrier
    __syncthreads();
  }
}

// Sorts (key, value) pairs by key bits [0, bits) stably; the result ends in
// *ka / *va (the pointers are swapped when it lands in the second buffer).
static void radix_sort(uint32_t **ka, int32_t **va, uint32_t **kb, int32_t **vb, int64_t m_cap, const int32_t *m_dev,
                       int bits, int32_t *hist, int32_t *bsum, hipStream_t s) {
  const int64_t nb = rs_blocks(m_cap);
  const unsigned g = (unsigned)(nb < 1 ? 1 : nb);
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(g), dim3(RS_THREADS), 0, s, *ka, m_cap, m_dev, shift, hist, (int)g);
    scan_excl(hist, hist, (int64_t)256 * g, nullptr, bsum, nullptr, s);
    hipLaunchKernelGGL(k_rs_scatter, dim3(g), dim3(RS_THREADS), 0, s, *ka, *va, m_cap, m_dev, shift, hist, (int)g, *kb,
                       *vb);
    uint32_t *tk = *ka;
    *ka = *kb;
    *kb = tk;
    int32_t *tv = *va;
    *va = *vb;
    *vb = tv;
  }
}

// ---------------------------------------------------------- tile binning

__global__ __launch_bounds__(256) void k_gs_cnt_by_rank(int n, const int32_t *__restrict__ id,
                                                        const int32_t *__restrict__ cnt, int32_t *__restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[r] = cnt[id[r]];
}

// A pair total (64-bit, hdr[2..3]) above the capacity sets status bit
// DW_STATUS_RENDER_OVERFLOW and the pair count hdr[1] to 0: nothing is
// emitted, sorted or drawn.
__global__ void k_gs_check(int64_t cap, int32_t *hdr) {
  if (threadIdx.x != 0) return;
  unsigned long long t = 0;
  for (int q = 0; q < GS_NCNT; ++q) t += reinterpret_cast<const unsigned long long *>(hdr + GS_CNT0)[q];
  if (t > (unsigned long long)cap) {
    hdr[0] |= DW_STATUS_RENDER_OVERFLOW;
    hdr[1] = 0;
  }
}

__global__ void k_gs_status(const int32_t *hdr, int32_t *out) {
  if (threadIdx.x < 2) out[threadIdx.x] = hdr[threadIdx.x];
}

__device__ __forceinline__ bool gs_failed(const int32_t *hdr) { return (hdr[0] & DW_STATUS_RENDER_OVERFLOW) != 0; }

// Pairs in depth order.  Block b writes pairs [b E, (b + 1) E) of the list
// (E = GS_EMIT): two threads find by binary search the depth ranks that own
// its first and last pair (off is the exclusive scan of the tile counts in
// depth order; every drawn kernel owns at least one pair and the kernels
// that are not drawn sort last, so at most E ranks are involved); their
// offsets and ids are staged in LDS; thread t fills pairs t*16 .. t*16 + 15
// into an LDS copy of the block's slice, walking its kernels' tile boxes
// incrementally from one binary search; the slice is then stored with
// contiguous writes.  The work per block is fixed whatever the kernels'
// sizes, so a kernel covering thousands of tiles does not hold up a wave.
constexpr int GS_EMIT = 4096;
constexpr int GS_EMIT_PER = GS_EMIT / 256;

__global__ __launch_bounds__(256) void k_gs_emit(int n, CamDev K, const int32_t *__restrict__ id,
                                                 const int32_t *__restrict__ off, const int4 *__restrict__ rect,
                                                 const int32_t *hdr, uint32_t *__restrict__ pk,
                                                 int32_t *__restrict__ pv) {
  __shared__ int s_off[GS_EMIT], s_g[GS_EMIT];
  __shared__ uint32_t s_pk[GS_EMIT];
  __shared__ int32_t s_pv[GS_EMIT];
  __shared__ int s_r[2];
  if (gs_failed(hdr)) return;  // grid-uniform
  const int64_t total = hdr[1];
  const int64_t P0 = (int64_t)blockIdx.x * GS_EMIT;
  if (P0 >= total) return;  // block-uniform
  const int m_pairs = (int)min((int64_t)GS_EMIT, total - P0);
  if (threadIdx.x < 2) {
    // last rank whose first pair is at or before the target pair
    const int64_t tgt = threadIdx.x == 0 ? P0 : P0 + m_pairs - 1;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= tgt) lo = mid;
      else hi = mid - 1;
    }
    s_r[threadIdx.x] = lo;
  }
  __syncthreads();
  const int r_lo = s_r[0], m_ranks = s_r[1] - s_r[0] + 1;  // <= GS_EMIT
  for (int k = threadIdx.x; k < m_ranks; k += 256) {
    s_off[k] = (int)(off[r_lo + k] - P0);
    s_g[k] = id[r_lo + k];
  }
  __syncthreads();
  const int j0 = threadIdx.x * GS_EMIT_PER;
  if (j0 < m_pairs) {
    int lo = 0, hi = m_ranks - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= j0) lo = mid;
      else hi = mid - 1;
    }
    int k = lo;
    int g = s_g[k];
    int4 b = rect[g];
    int w = b.y - b.x + 1;
    const int q0 = j0 - s_off[k];
    int tx = q0 % w, ty = q0 / w;
    int rows = b.w - b.z + 1;
    const int j1 = min(j0 + GS_EMIT_PER, m_pairs);
    for (int j = j0; j < j1; ++j) {
      if (ty == rows) {  // next kernel (at least one pair each)
        ++k;
        g = s_g[k];
        b = rect[g];
        w = b.y - b.x + 1;
        rows = b.w - b.z + 1;
        tx = 0;
        ty = 0;
      }
      s_pk[j] = (uint32_t)(b.x + tx + K.tw * (b.z + ty));
      s_pv[j] = g;
      if (++tx == w) {
        tx = 0;
        ++ty;
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < m_pairs; j += 256) {
    pk[P0 + j] = s_pk[j];
    pv[P0 + j] = s_pv[j];
  }
}

// grid-stride over the pairs actually present (the grid is sized for a
// typical count, not for the capacity)
__global__ __launch_bounds__(256) void k_gs_ranges(const uint32_t *__restrict__ pk, const int32_t *__restrict__ hdr,
                                                   int2 *__restrict__ range) {
  const int64_t m = hdr[1];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t t = pk[i];
    if (i == 0 || pk[i - 1] != t) range[t].x = (int)i;
    if (i == m - 1 || pk[i + 1] != t) range[t].y = (int)(i + 1);
  }
}

// ------------------------------------------------------------- raster

struct GsRec {
  float mx, my, A, B, C, o, c0, c1, c2;
};

__device__ __forceinline__ GsRec load_rec(const float4 *rec, int g) {
  const float4 a = rec[3 * (int64_t)g], b = rec[3 * (int64_t)g + 1], c = rec[3 * (int64_t)g + 2];
  return GsRec{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x};
}

// alpha of kernel r at pixel centre (x, y); the same expression in the
// forward and reverse passes, so both take the same alpha_min decisions
__device__ __forceinline__ float gs_alpha(const GsRec &r, float x, float y, float &dx, float &dy, float &e) {
  dx = x - r.mx;
  dy = y - r.my;
  const float q = r.A * dx * dx + 2.0f * r.B * dx * dy + r.C * dy * dy;
  e = __expf(-0.5f * q);
  return r.o * e;
}

__global__ __launch_bounds__(GS_THREADS) void k_gs_raster(CamDev K, const int32_t *__restrict__ hdr,
                                                         const int2 *__restrict__ range,
                                                         const int32_t *__restrict__ pv, const float4 *__restrict__ rec,
                                                         float *__restrict__ image, int32_t *__restrict__ last) {
  __shared__ GsRec s_r[GS_THREADS];
  if (gs_failed(hdr)) return;  // over capacity: the image is not written
  const int tile = blockIdx.x;
  const int tx = tile % K.tw, ty = tile / K.tw;
  const int i = tx * GS_TILE + (threadIdx.x % GS_TILE), j = ty * GS_TILE + (threadIdx.x / GS_TILE);
  const bool inside = i < K.W && j < K.H;
  const float x = i + 0.5f, y = j + 0.5f;
  const int2 rg = range[tile];
  float T = 1.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
  int used = 0;
  bool done = !inside;
  for (int b = rg.x; b < rg.y; b += GS_THREADS) {
    if (__syncthreads_count(!done) == 0) break;
    const int nbatch = min(GS_THREADS, rg.y - b);
    if ((int)threadIdx.x < nbatch) s_r[threadIdx.x] = load_rec(rec, pv[b + threadIdx.x]);
    __syncthreads();
    if (!done) {
      for (int q = 0; q < nbatch; ++q) {
        const GsRec r = s_r[q];
        float dx, dy, e;
        const float al = gs_alpha(r, x, y, dx, dy, e);
        if (al >= K.amin) {
          const float wgt = T * al;
          c0 += wgt * r.c0;
          c1 += wgt * r.c1;
          c2 += wgt * r.c2;
          T *= 1.0f - al;
        }
        if (T < K.tmin) {
          used = b - rg.x + q + 1;
          done = true;
          break;
        }
      }
      if (!done) used = b - rg.x + nbatch;
    }
  }
  if (!inside) return;
  const int64_t pix = i + (int64_t)K.W * j, HW = (int64_t)K.W * K.H;
  image[pix] = c0 + T * K.bg[0];
  image[HW + pix] = c1 + T * K.bg[1];
  image[2 * HW + pix] = c2 + T * K.bg[2];
  last[pix] = used;
}

// ------------------------------------------------------- raster reverse

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Sum over the 64 lanes of a wave whose lanes are all active: four DPP
// steps give every lane its 16-lane row total (quad_perm [1,0,3,2] and
// [2,3,0,1], then row rotations by 4 and 8), four lane reads add the rows.
// The result is wave-uniform.
template <int CTRL>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_total(float v) {
  v = dpp_add<0xB1>(v);
  v = dpp_add<0x4E>(v);
  v = dpp_add<0x124>(v);
  v = dpp_add<0x128>(v);
  const int b = __float_as_int(v);
  return (__int_as_float(__builtin_amdgcn_readlane(b, 0)) + __int_as_float(__builtin_amdgcn_readlane(b, 16))) +
         (__int_as_float(__builtin_amdgcn_readlane(b, 32)) + __int_as_float(__builtin_amdgcn_readlane(b, 48)));
}

// per-kernel adjoints in LDS for one batch: centre (2), conic (3), opacity,
// colour (3)
constexpr int GS_NB = 9;

// One wave per tile, four pixels per lane (lane l: column l % 16, rows
// 4 (l / 16) .. 4 (l / 16) + 3), so each list entry's per-kernel adjoints
// are summed over the lane's pixels in registers and then over the wave
// once (DPP), and lane 0 adds them to global memory.
constexpr int GS_ADJ_PX = 4;

__global__ __launch_bounds__(64) void k_gs_raster_adj(
    CamDev K, const int32_t *__restrict__ hdr, const int2 *__restrict__ range,
    const int32_t *__restrict__ pv, const float4 *__restrict__ rec, const int32_t *__restrict__ last,
    const float *__restrict__ image, const float *__restrict__ image_bar, int n, float *__restrict__ gbar,
    float *__restrict__ color_bar, float *__restrict__ opacity_bar) {
  __shared__ GsRec s_r[64];
  __shared__ int s_g[64];
  if (gs_failed(hdr)) return;
  const int tile = blockIdx.x;
  const int tx = tile % K.tw, ty = tile / K.tw;
  const int lane = threadIdx.x;
  const int i = tx * GS_TILE + (lane % GS_TILE);
  const int jb = ty * GS_TILE + GS_ADJ_PX * (lane / GS_TILE);
  const int2 rg = range[tile];
  const int64_t HW = (int64_t)K.W * K.H;
  const float x = i + 0.5f;
  float G[GS_ADJ_PX][3], Ct[GS_ADJ_PX][3], T[GS_ADJ_PX], Acc[GS_ADJ_PX][3];
  int used[GS_ADJ_PX];
  int maxused = 0;
#pragma unroll
  for (int k = 0; k < GS_ADJ_PX; ++k) {
    const int j = jb + k;
    const bool inside = i < K.W && j < K.H;
    const int64_t pix = i + (int64_t)K.W * j;
    used[k] = inside ? last[pix] : 0;
    T[k] = 1.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      G[k][c] = inside ? image_bar[c * HW + pix] : 0.f;
      Ct[k][c] = inside ? image[c * HW + pix] : 0.f;
      Acc[k][c] = 0.f;
    }
    maxused = max(maxused, used[k]);
  }
  // the tile's furthest pixel bounds the traversal (wave maximum)
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) maxused = max(maxused, __shfl_xor(maxused, m, 64));
  for (int b = 0; b < maxused; b += 64) {
    const int nbatch = min(64, maxused - b);
    __syncthreads();
    if (lane < nbatch) {
      const int g = pv[rg.x + b + lane];
      s_g[lane] = g;
      s_r[lane] = load_rec(rec, g);
    }
    __syncthreads();
    for (int q = 0; q < nbatch; ++q) {
      const GsRec r = s_r[q];
      const float cc[3] = {r.c0, r.c1, r.c2};
      float d[GS_NB];
#pragma unroll
      for (int v = 0; v < GS_NB; ++v) d[v] = 0.f;
      bool any = false;
#pragma unroll
      for (int k = 0; k < GS_ADJ_PX; ++k) {
        float dx, dy, e;
        const float al = gs_alpha(r, x, (float)(jb + k) + 0.5f, dx, dy, e);
        if ((b + q < used[k]) && al >= K.amin) {
          any = true;
          const float wgt = T[k] * al;
          float dal = 0.f;
          const float inv1m = 1.0f / (1.0f - al);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            Acc[k][c] += wgt * cc[c];
            d[6 + c] += wgt * G[k][c];                                 // colour
            dal += G[k][c] * (T[k] * cc[c] - (Ct[k][c] - Acc[k][c]) * inv1m);
          }
          T[k] *= 1.0f - al;
          d[5] += dal * e;                                             // opacity
          const float dq = -0.5f * al * dal;                           // alpha = o exp(-q/2)
          d[0] += -2.0f * dq * (r.A * dx + r.B * dy);                  // centre x
          d[1] += -2.0f * dq * (r.B * dx + r.C * dy);                  // centre y
          d[2] += dq * dx * dx;                                        // conic A
          d[3] += dq * 2.0f * dx * dy;                                 // conic B (q has 2 B dx dy)
          d[4] += dq * dy * dy;                                        // conic C
        }
      }
      if (__ballot(any) == 0ull) continue;  // wave-uniform
#pragma unroll
      for (int v = 0; v < GS_NB; ++v) d[v] = wave_total(d[v]);
      if (lane == 0) {
        const int g = s_g[q];
        if (d[0] != 0.f) atomicAdd(&gbar[g], d[0]);
        if (d[1] != 0.f) atomicAdd(&gbar[(int64_t)n + g], d[1]);
        if (d[2] != 0.f) atomicAdd(&gbar[2 * (int64_t)n + g], d[2]);
        if (d[3] != 0.f) atomicAdd(&gbar[3 * (int64_t)n + g], d[3]);
        if (d[4] != 0.f) atomicAdd(&gbar[4 * (int64_t)n + g], d[4]);
        if (opacity_bar && d[5] != 0.f) atomicAdd(&opacity_bar[g], d[5]);
        if (color_bar) {
#pragma unroll
          for (int c = 0; c < 3; ++c)
            if (d[6 + c] != 0.f) atomicAdd(&color_bar[c * (int64_t)n + g], d[6 + c]);
        }
      }
    }
  }
}

// Centre and conic adjoints back to mu and Sigma through the projection.
// conic K = Sigma2^-1: Sigma2_bar = -K Kbar K (Kbar the symmetric matrix of
// the conic adjoint, off-diagonal B_bar / 2); Sigma2 = T Sigma T^T with T = J R:
// Sigma_bar = T^T Sigma2_bar T, T_bar = 2 Sigma2_bar T Sigma; J_bar = T_bar R^T
// and the centre adjoint go to the camera point p, and mu_bar = R^T p_bar.
__global__ __launch_bounds__(256) void k_gs_project_adj(CamDev K, int n, const float *__restrict__ mu,
                                                        const float *__restrict__ sigma, const float *__restrict__ op,
                                                        const float *__restrict__ gbar, float *__restrict__ mu_bar,
                                                        float *__restrict__ sigma_bar) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  float S[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) S[e] = sigma[(int64_t)e * n + g];
  const Proj r = gs_proj(K, mu[g], mu[(int64_t)n + g], mu[2 * (int64_t)n + g], S, op[g]);
  if (!r.drawn) return;
  const float mxb = gbar[g], myb = gbar[(int64_t)n + g];
  const float Ab = gbar[2 * (int64_t)n + g], Bb = gbar[3 * (int64_t)n + g], Cb = gbar[4 * (int64_t)n + g];
  if (mxb == 0.f && myb == 0.f && Ab == 0.f && Bb == 0.f && Cb == 0.f) return;
  // Sigma2_bar = -K Kbar K, K = [[A, B], [B, C]], Kbar = [[Ab, Bb/2], [Bb/2, Cb]]
  const float kb01 = 0.5f * Bb;
  const float m00 = r.A * Ab + r.B * kb01, m01 = r.A * kb01 + r.B * Cb;  // K Kbar
  const float m10 = r.B * Ab + r.C * kb01, m11 = r.B * kb01 + r.C * Cb;
  const float s00 = -(m00 * r.A + m01 * r.B), s01 = -(m00 * r.B + m01 * r.C);
  const float s11 = -(m10 * r.B + m11 * r.C);
  // Sigma_bar = T^T Sigma2_bar T (symmetric); stored off-diagonals count twice
  float Sb[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      Sb[3 * a + c] = r.T0[a] * (s00 * r.T0[c] + s01 * r.T1[c]) + r.T1[a] * (s01 * r.T0[c] + s11 * r.T1[c]);
  if (sigma_bar) {
    sigma_bar[g] += Sb[0];
    sigma_bar[(int64_t)n + g] += Sb[4];
    sigma_bar[2 * (int64_t)n + g] += Sb[8];
    sigma_bar[3 * (int64_t)n + g] += Sb[1] + Sb[3];
    sigma_bar[4 * (int64_t)n + g] += Sb[2] + Sb[6];
    sigma_bar[5 * (int64_t)n + g] += Sb[5] + Sb[7];
  }
  if (!mu_bar) return;
  // T_bar = 2 Sigma2_bar T Sigma (rows 0, 1)
  const float Sm[9] = {S[0], S[3], S[4], S[3], S[1], S[5], S[4], S[5], S[2]};
  float TS0[3], TS1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    TS0[c] = r.T0[0] * Sm[c] + r.T0[1] * Sm[3 + c] + r.T0[2] * Sm[6 + c];
    TS1[c] = r.T1[0] * Sm[c] + r.T1[1] * Sm[3 + c] + r.T1[2] * Sm[6 + c];
  }
  float Tb0[3], Tb1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    Tb0[c] = 2.0f * (s00 * TS0[c] + s01 * TS1[c]);
    Tb1[c] = 2.0f * (s01 * TS0[c] + s11 * TS1[c]);
  }
  // J_bar = T_bar R^T; only J00, J02, J11, J12 are non-zero functions of p
  const float jb00 = Tb0[0] * K.R[0] + Tb0[1] * K.R[1] + Tb0[2] * K.R[2];
  const float jb02 = Tb0[0] * K.R[6] + Tb0[1] * K.R[7] + Tb0[2] * K.R[8];
  const float jb11 = Tb1[0] * K.R[3] + Tb1[1] * K.R[4] + Tb1[2] * K.R[5];
  const float jb12 = Tb1[0] * K.R[6] + Tb1[1] * K.R[7] + Tb1[2] * K.R[8];
  const float iz = 1.0f / r.pz, iz2 = iz * iz, iz3 = iz2 * iz;
  // J00 = fx/z, J02 = -fx px/z^2, J11 = fy/z, J12 = -fy py/z^2;
  // mx = fx px/z + cx, my = fy py/z + cy
  const float pxb = -K.fx * iz2 * jb02 + K.fx * iz * mxb;
  const float pyb = -K.fy * iz2 * jb12 + K.fy * iz * myb;
  const float pzb = -K.fx * iz2 * jb00 + 2.0f * K.fx * r.px * iz3 * jb02 - K.fy * iz2 * jb11 +
                    2.0f * K.fy * r.py * iz3 * jb12 - K.fx * r.px * iz2 * mxb - K.fy * r.py * iz2 * myb;
  // mu_bar = R^T p_bar
#pragma unroll
  for (int a = 0; a < 3; ++a)
    mu_bar[(int64_t)a * n + g] += K.R[a] * pxb + K.R[3 + a] * pyb + K.R[6 + a] * pzb;
}

// ------------------------------------------------------------- loss

constexpr int SS_T = 16;               // output tile of the SSIM kernels
constexpr int SS_R = 5;                // window radius (11 x 11)
constexpr int SS_E = SS_T + 2 * SS_R;  // staged extent
constexpr float SS_C1 = 0.01f * 0.01f, SS_C2 = 0.03f * 0.03f;

__device__ __forceinline__ float ss_w(int k) {
  // normalised 1-D Gaussian, sigma 1.5, taps -5..5 (computed once per use;
  // the 2-D window is its outer product)
  float s = 0.f;
#pragma unroll
  for (int q = -SS_R; q <= SS_R; ++q) s += expf(-(float)(q * q) / 4.5f);
  return expf(-(float)(k * k) / 4.5f) / s;
}

// Pass 1: per channel and 16 x 16 tile: the five window sums of a and b
// (zero outside the image), the SSIM map value m and its partial
// derivatives with respect to mu_a, E[a^2] and E[ab] (written to d3 [3][C][HW]
// for pass 2); per block: sum of m and of |a - b| (fixed order).
__global__ __launch_bounds__(SS_T *SS_T) void k_ssim_fwd(int C, int H, int W, const float *__restrict__ a,
                                                          const float *__restrict__ b, float *__restrict__ d3,
                                                          float *__restrict__ part) {
  __shared__ float s_a[SS_E][SS_E], s_b[SS_E][SS_E];
  __shared__ float s_h[5][SS_E][SS_T];
  __shared__ float s_red[2][SS_T * SS_T / 64];
  __shared__ float s_wt[2 * SS_R + 1];
  const int tw = (W + SS_T - 1) / SS_T;
  const int tile = blockIdx.x, ch = blockIdx.y;
  const int X0 = (tile % tw) * SS_T - SS_R, Y0 = (tile / tw) * SS_T - SS_R;
  const int64_t HW = (int64_t)H * W;
  const float *A = a + ch * HW, *B = b + ch * HW;
  if (threadIdx.x < 2 * SS_R + 1) s_wt[threadIdx.x] = ss_w((int)threadIdx.x - SS_R);
  for (int q = threadIdx.x; q < SS_E * SS_E; q += SS_T * SS_T) {
    const int yy = Y0 + q / SS_E, xx = X0 + q % SS_E;
    const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
    s_a[q / SS_E][q % SS_E] = in ? A[(int64_t)yy * W + xx] : 0.f;
    s_b[q / SS_E][q % SS_E] = in ? B[(int64_t)yy * W + xx] : 0.f;
  }
  __syncthreads();
  // horizontal pass over the staged rows
  for (int q = threadIdx.x; q < SS_E * SS_T; q += SS_T * SS_T) {
    const int row = q / SS_T, col = q % SS_T;
    float h0 = 0.f, h1 = 0.f, h2 = 0.f, h3 = 0.f, h4 = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * SS_R; ++k) {
      const float wk = s_wt[k], va = s_a[row][col + k], vb = s_b[row][col + k];
      h0 += wk * va;
      h1 += wk * vb;
      h2 += wk * va * va;
      h3 += wk * vb * vb;
      h4 += wk * va * vb;
    }
    s_h[0][row][col] = h0;
    s_h[1][row][col] = h1;
    s_h[2][row][col] = h2;
    s_h[3][row][col] = h3;
    s_h[4][row][col] = h4;
  }
  __syncthreads();
  const int tx = threadIdx.x % SS_T, ty = threadIdx.x / SS_T;
  const int x = X0 + SS_R + tx, y = Y0 + SS_R + ty;
  float m = 0.f, l1 = 0.f;
  if (x < W && y < H) {
    float S[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k <= 2 * SS_R; ++k) {
      const float wk = s_wt[k];
#pragma unroll
      for (int v = 0; v < 5; ++v) S[v] += wk * s_h[v][ty + k][tx];
    }
    const float mu_a = S[0], mu_b = S[1];
    const float va = S[2] - mu_a * mu_a, vb = S[3] - mu_b * mu_b, cab = S[4] - mu_a * mu_b;
    const float n1 = 2.f * mu_a * mu_b + SS_C1, n2 = 2.f * cab + SS_C2;
    const float e1 = mu_a * mu_a + mu_b * mu_b + SS_C1, e2 = va + vb + SS_C2;
    const float den = e1 * e2;
    m = n1 * n2 / den;
    // m as a function of (mu_a, E[a^2], E[ab]) with mu_b, E[b^2] fixed:
    // dn1/dmu_a = 2 mu_b; dn2/dmu_a = -2 mu_b, dn2/dE[ab] = 2;
    // de1/dmu_a = 2 mu_a; de2/dmu_a = -2 mu_a, de2/dE[a^2] = 1
    const float dmu = (2.f * mu_b * n2 - 2.f * mu_b * n1) / den - m * (2.f * mu_a * e2 - 2.f * mu_a * e1) / den;
    const float dEaa = -m / e2;
    const float dEab = 2.f * n1 / den;
    const int64_t pix = (int64_t)y * W + x;
    d3[(int64_t)ch * HW + pix] = dmu;
    d3[((int64_t)C + ch) * HW + pix] = dEaa;
    d3[(2 * (int64_t)C + ch) * HW + pix] = dEab;
    l1 = fabsf(s_a[ty + SS_R][tx + SS_R] - s_b[ty + SS_R][tx + SS_R]);
  }
  // block sums, fixed order
  const float sm = wave_sum(m), sl = wave_sum(l1);
  if ((threadIdx.x & 63) == 0) {
    s_red[0][threadIdx.x >> 6] = sm;
    s_red[1][threadIdx.x >> 6] = sl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float t0 = 0.f, t1 = 0.f;
#pragma unroll
    for (int w = 0; w < SS_T * SS_T / 64; ++w) {
      t0 += s_red[0][w];
      t1 += s_red[1][w];
    }
    const int64_t blk = (int64_t)ch * gridDim.x + tile;
    part[2 * blk] = t0;
    part[2 * blk + 1] = t1;
  }
}

// one block: loss = (1 - lam) mean|a - b| + lam (1 - mean SSIM), added to
// *loss in a fixed order over the block partials
__global__ __launch_bounds__(256) void k_loss_final(int nblk, int64_t count, float lam,
                                                    const float *__restrict__ part, float *__restrict__ loss) {
  __shared__ float s_m[256], s_l[256];
  float m = 0.f, l = 0.f;
  for (int q = threadIdx.x; q < nblk; q += 256) {
    m += part[2 * q];
    l += part[2 * q + 1];
  }
  s_m[threadIdx.x] = m;
  s_l[threadIdx.x] = l;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s_m[threadIdx.x] += s_m[threadIdx.x + h];
      s_l[threadIdx.x] += s_l[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float inv = 1.0f / (float)count;
    *loss += (1.0f - lam) * s_l[0] * inv + lam * (1.0f - s_m[0] * inv);
  }
}

// Pass 2: dL/da = (1 - lam)/N sign(a - b) - lam/N (w * dmu + 2 a (w * dEaa)
// + b (w * dEab)), the window correlations over the staged partials (zero
// outside the image); ADDS to a_bar.
__global__ __launch_bounds__(SS_T *SS_T) void k_ssim_bwd(int C, int H, int W, float lam, const float *__restrict__ a,
                                                          const float *__restrict__ b, const float *__restrict__ d3,
                                                          float *__restrict__ a_bar) {
  __shared__ float s_d[3][SS_E][SS_E];
  __shared__ float s_h[3][SS_E][SS_T];
  __shared__ float s_wt[2 * SS_R + 1];
  const int tw = (W + SS_T - 1) / SS_T;
  const int tile = blockIdx.x, ch = blockIdx.y;
  const int X0 = (tile % tw) * SS_T - SS_R, Y0 = (tile / tw) * SS_T - SS_R;
  const int64_t HW = (int64_t)H * W;
  if (threadIdx.x < 2 * SS_R + 1) s_wt[threadIdx.x] = ss_w((int)threadIdx.x - SS_R);
  for (int q = threadIdx.x; q < SS_E * SS_E; q += SS_T * SS_T) {
    const int yy = Y0 + q / SS_E, xx = X0 + q % SS_E;
    const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
    const int64_t pix = (int64_t)yy * W + xx;
#pragma unroll
    for (int v = 0; v < 3; ++v) s_d[v][q / SS_E][q % SS_E] = in ? d3[((int64_t)v * C + ch) * HW + pix] : 0.f;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < SS_E * SS_T; q += SS_T * SS_T) {
    const int row = q / SS_T, col = q % SS_T;
    float h[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k <= 2 * SS_R; ++k)
#pragma unroll
      for (int v = 0; v < 3; ++v) h[v] += s_wt[k] * s_d[v][row][col + k];
#pragma unroll
    for (int v = 0; v < 3; ++v) s_h[v][row][col] = h[v];
  }
  __syncthreads();
  const int tx = threadIdx.x % SS_T, ty = threadIdx.x / SS_T;
  const int x = X0 + SS_R + tx, y = Y0 + SS_R + ty;
  if (x >= W || y >= H) return;
  float S[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k <= 2 * SS_R; ++k)
#pragma unroll
    for (int v = 0; v < 3; ++v) S[v] += s_wt[k] * s_h[v][ty + k][tx];
  const int64_t pix = (int64_t)ch * HW + (int64_t)y * W + x;
  const float va = a[pix], vb = b[pix];
  const float inv = 1.0f / (float)(C * HW);
  const float sg = va > vb ? 1.f : (va < vb ? -1.f : 0.f);
  a_bar[pix] += (1.0f - lam) * inv * sg - lam * inv * (S[0] + 2.f * va * S[1] + vb * S[2]);
}

static int make_cam(const dw_camera *c, CamDev *K) {
  DW_REQUIRE(c, DW_EINVAL, "render: camera is NULL");
  DW_REQUIRE(c->width >= 1 && c->height >= 1 && c->width <= 16384 && c->height <= 16384, DW_ERANGE,
             "render: image size must be 1..16384 per axis");
  DW_REQUIRE(c->near_plane >= 0.f, DW_EINVAL, "render: near plane must be >= 0");
  DW_REQUIRE(c->alpha_min >= 0.f && c->alpha_min < 1.f, DW_EINVAL, "render: alpha_min must be in [0, 1)");
  DW_REQUIRE(c->t_min >= 0.f && c->t_min < 1.f, DW_EINVAL, "render: t_min must be in [0, 1)");
  K->W = c->width;
  K->H = c->height;
  K->tw = (c->width + GS_TILE - 1) / GS_TILE;
  K->th = (c->height + GS_TILE - 1) / GS_TILE;
  K->fx = c->fx;
  K->fy = c->fy;
  K->cx = c->cx;
  K->cy = c->cy;
  for (int q = 0; q < 9; ++q) K->R[q] = c->R[q];
  for (int q = 0; q < 3; ++q) {
    K->t[q] = c->t[q];
    K->bg[q] = c->bg[q];
  }
  K->near_ = c->near_plane;
  K->amin = c->alpha_min;
  K->tmin = c->t_min;
  return DW_OK;
}

static int bits_for(int64_t v) {
  int b = 0;
  while (((int64_t)1 << b) < v) ++b;
  return b;
}

// passes of the pair sort by tile; an odd count leaves the pairs in buffer b
static int pair_bits(int64_t T) { return bits_for(T) < 1 ? 1 : bits_for(T); }
static bool pairs_in_b(int64_t T) { return ((pair_bits(T) + 7) / 8) % 2 == 1; }

}  // namespace dw

using namespace dw;

extern "C" size_t gs_render_workspace_bytes(int n, const dw_camera *cam, int64_t max_pairs) {
  if (n < 0 || !cam || cam->width < 1 || cam->height < 1 || max_pairs < 0) return 0;
  return gs_layout(nullptr, n, max_pairs, cam->width, cam->height).bytes;
}

static int gs_common(const char *who, const dw_camera *cam, int n, const float *mu, const float *sigma,
                     const float *color, const float *opacity, int64_t max_pairs, void *ws, size_t ws_bytes,
                     CamDev *K, GsWs *w) {
  int rc = make_cam(cam, K);
  if (rc) return rc;
  DW_REQUIRE(n >= 0, DW_EINVAL, "%s: n must be >= 0", who);
  DW_REQUIRE(max_pairs >= 0 && max_pairs < ((int64_t)1 << 31), DW_ERANGE, "%s: max_pairs must be in [0, 2^31)", who);
  DW_REQUIRE(ws, DW_EINVAL, "%s: workspace is NULL", who);
  DW_REQUIRE(n == 0 || (mu && sigma && color && opacity), DW_EINVAL, "%s: kernel arrays are NULL", who);
  *w = gs_layout((char *)ws, n, max_pairs, cam->width, cam->height);
  DW_REQUIRE(ws_bytes >= w->bytes, DW_EWORKSPACE, "%s: workspace too small (%zu < %zu bytes)", who, ws_bytes,
             w->bytes);
  DW_REQUIRE(rs_blocks(n > max_pairs ? n : max_pairs) * 256 <= (int64_t)SCAN_CHUNK * SCAN_TOP_MAX &&
                 (n + (int64_t)SCAN_CHUNK - 1) / SCAN_CHUNK <= SCAN_TOP_MAX,
             DW_ERANGE, "%s: too many kernels or pairs for the scan", who);
  return DW_OK;
}

extern "C" int gs_render(const dw_camera *cam, int n, const float *mu, const float *sigma, const float *color,
                         const float *opacity, float *image, int64_t max_pairs, void *ws, size_t ws_bytes,
                         void *stream) {
  CamDev K;
  GsWs w;
  int rc = gs_common("gs_render", cam, n, mu, sigma, color, opacity, max_pairs, ws, ws_bytes, &K, &w);
  if (rc) return rc;
  DW_REQUIRE(image, DW_EINVAL, "gs_render: image is NULL");
  hipStream_t s = (hipStream_t)stream;
  const int64_t T = (int64_t)K.tw * K.th;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, w.hdr, (int64_t)GS_HDR_INTS, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_blocks(2 * T, 256 * 4)), dim3(256), 0, s, (int32_t *)w.range, 2 * T, 0);
  if (n > 0) {
    hipLaunchKernelGGL(k_gs_project, dim3(grid_blocks(n, 256)), dim3(256), 0, s, K, n, mu, sigma, color, opacity, w);
    uint32_t *ka = w.key_a, *kb = w.key_b;
    int32_t *va = w.id_a, *vb = w.id_b;
    radix_sort(&ka, &va, &kb, &vb, n, nullptr, 32, w.hist, w.bsum, s);  // 4 passes: back in buffer a
    hipLaunchKernelGGL(k_gs_cnt_by_rank, dim3(grid_blocks(n, 256)), dim3(256), 0, s, n, va, w.cnt, w.off);
    scan_excl(w.off, w.off, n, nullptr, w.bsum, w.hdr + 1, s);
    hipLaunchKernelGGL(k_gs_check, dim3(1), dim3(64), 0, s, max_pairs, w.hdr);
    if (max_pairs > 0) {
      hipLaunchKernelGGL(k_gs_emit, dim3(grid_blocks(max_pairs, GS_EMIT)), dim3(256), 0, s, n, K, va, w.off, w.rect,
                         w.hdr, w.pk_a, w.pv_a);
      uint32_t *pa = w.pk_a, *pb = w.pk_b;
      int32_t *qa = w.pv_a, *qb = w.pv_b;
      radix_sort(&pa, &qa, &pb, &qb, max_pairs, w.hdr + 1, pair_bits(T), w.hist, w.bsum, s);
      hipLaunchKernelGGL(k_gs_ranges, dim3(grid_blocks(max_pairs < 8 * (int64_t)n ? max_pairs : 8 * (int64_t)n, 256)),
                         dim3(256), 0, s, pa, w.hdr, w.range);
    }
  }
  const int32_t *ids = pairs_in_b(T) ? w.pv_b : w.pv_a;
  hipLaunchKernelGGL(k_gs_raster, dim3((unsigned)T), dim3(GS_THREADS), 0, s, K, w.hdr, w.range, ids, w.rec, image,
                     w.last);
  return check_launch("gs_render");
}

extern "C" int gs_render_adj(const dw_camera *cam, int n, const float *mu, const float *sigma, const float *color,
                             const float *opacity, const float *image, const float *image_bar, float *mu_bar,
                             float *sigma_bar, float *color_bar, float *opacity_bar, int64_t max_pairs, void *ws,
                             size_t ws_bytes, void *stream) {
  CamDev K;
  GsWs w;
  int rc = gs_common("gs_render_adj", cam, n, mu, sigma, color, opacity, max_pairs, ws, ws_bytes, &K, &w);
  if (rc) return rc;
  DW_REQUIRE(image && image_bar, DW_EINVAL, "gs_render_adj: image / image_bar is NULL");
  if (n == 0) return DW_OK;
  hipStream_t s = (hipStream_t)stream;
  const int64_t T = (int64_t)K.tw * K.th;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_blocks(5 * (int64_t)n, 256 * 8)), dim3(256), 0, s, w.gbar, 5 * (int64_t)n,
                     0.f);
  const int32_t *ids = pairs_in_b(T) ? w.pv_b : w.pv_a;
  hipLaunchKernelGGL(k_gs_raster_adj, dim3((unsigned)T), dim3(64), 0, s, K, w.hdr, w.range, ids, w.rec,
                     w.last, image, image_bar, n, w.gbar, color_bar, opacity_bar);
  hipLaunchKernelGGL(k_gs_project_adj, dim3(grid_blocks(n, 256)), dim3(256), 0, s, K, n, mu, sigma, opacity, w.gbar,
                     mu_bar, sigma_bar);
  return check_launch("gs_render_adj");
}

extern "C" int gs_render_status(const void *ws, int32_t *status_out, void *stream) {
  DW_REQUIRE(ws && status_out, DW_EINVAL, "gs_render_status: NULL argument");
  hipLaunchKernelGGL(k_gs_status, dim3(1), dim3(64), 0, (hipStream_t)stream, (const int32_t *)ws, status_out);
  return check_launch("gs_render_status");
}

static size_t loss_layout(int C, int H, int W, float **d3, float **part, char *base) {
  const int64_t HW = (int64_t)H * W;
  const int64_t nblk = (int64_t)C * ((W + SS_T - 1) / SS_T) * ((H + SS_T - 1) / SS_T);
  size_t o = 0;
  if (d3) *d3 = base ? (float *)(base + o) : nullptr;
  o += al256((size_t)3 * C * HW * 4);
  if (part) *part = base ? (float *)(base + o) : nullptr;
  o += al256((size_t)2 * nblk * 4);
  return o;
}

extern "C" size_t render_loss_workspace_bytes(int C, int H, int W) {
  if (C < 1 || H < 1 || W < 1) return 0;
  return loss_layout(C, H, W, nullptr, nullptr, nullptr);
}

extern "C" int render_loss(int C, int H, int W, const float *image, const float *target, float lambda, float *loss,
                           float *image_bar, void *ws, size_t ws_bytes, void *stream) {
  DW_REQUIRE(C >= 1 && H >= 1 && W >= 1, DW_EINVAL, "render_loss: sizes must be >= 1");
  DW_REQUIRE(image && target && ws, DW_EINVAL, "render_loss: image / target / workspace is NULL");
  DW_REQUIRE(lambda >= 0.f && lambda <= 1.f, DW_EINVAL, "render_loss: lambda must be in [0, 1]");
  DW_REQUIRE(C <= 65535, DW_ERANGE, "render_loss: too many channels");
  float *d3, *part;
  const size_t need = loss_layout(C, H, W, &d3, &part, (char *)ws);
  DW_REQUIRE(ws_bytes >= need, DW_EWORKSPACE, "render_loss: workspace too small (%zu < %zu bytes)", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  const unsigned tiles = (unsigned)(((W + SS_T - 1) / SS_T) * ((H + SS_T - 1) / SS_T));
  hipLaunchKernelGGL(k_ssim_fwd, dim3(tiles, (unsigned)C), dim3(SS_T * SS_T), 0, s, C, H, W, image, target, d3, part);
  if (loss)
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, (int)(tiles * C), (int64_t)C * H * W, lambda, part,
                       loss);
  if (image_bar)
    hipLaunchKernelGGL(k_ssim_bwd, dim3(tiles, (unsigned)C), dim3(SS_T * SS_T), 0, s, C, H, W, lambda, image, target,
                       d3, image_bar);
  return check_launch("render_loss");
}
