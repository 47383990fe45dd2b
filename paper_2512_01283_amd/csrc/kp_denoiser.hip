// kp_denoiser.hip -- kernels of the learned Stokes-map denoiser on gfx950.
//
// The network is a small U-Net (3x3 convolutions at widths c1/c2/c3, 2x2 mean
// pooling, 2x nearest upsampling, skip concatenation, a 1x1 head that adds a
// correction to the input's Q and U).  It is not part of the radiative
// transfer method: it post-processes the step-2 Stokes maps.
//
// Tensors are NHWC BF16 (stored as uint16_t) with a per-pixel stride, so a
// concatenation is two producers writing disjoint channel ranges of one
// buffer.  Pixel p = (n H + h) W + w.  Every channel count is a multiple of 8,
// so 8 consecutive channels are one 16-byte load.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (FP32
// accumulation).  The GEMM K index is k = kk * cin + c with kk = 3 dy + dx
// the tap and c the input channel; K = 9 cin is zero-padded to a multiple of
// 32 in the packed weights.  A lane's 8 consecutive K elements never straddle
// a tap because cin % 8 == 0.
//
// MFMA 16x16x32 BF16 operand layout (wave64, lane l, i = l % 16, g = l / 16):
// A[i][8g + j] and B[8g + j][i] for j = 0..7 come from lane l; the result
// D[4g + j][i], j = 0..3, lands in lane l.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "kp_dn_internal.hpp"

namespace kp {
namespace dn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (inputs are finite)
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ bool bf_pos(uint16_t b) { return !(b & 0x8000u) && b != 0; }

__device__ __forceinline__ u32x4 ld16(const uint16_t* p) { return *(const u32x4*)p; }
__device__ __forceinline__ void st16(uint16_t* p, u32x4 v) { *(u32x4*)p = v; }

// unpack / pack 8 BF16 held in a 16-byte vector
__device__ __forceinline__ void unpack8(u32x4 v, float* f) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    f[2 * j] = __uint_as_float(v[j] << 16);
    f[2 * j + 1] = __uint_as_float(v[j] & 0xFFFF0000u);
  }
}
__device__ __forceinline__ u32x4 pack8(const float* f) {
  u32x4 v;
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = (uint32_t)f2bf(f[2 * j]) | ((uint32_t)f2bf(f[2 * j + 1]) << 16);
  return v;
}

__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

// ---------------------------------------------------------------------------
// 3x3 convolution as an implicit GEMM:
//   y[p][n] = epi( sum_{kk, c} x[p + off(kk)][c] * w[n][kk * cin + c] )
// off(kk) = (kk / 3 - 1, kk % 3 - 1), zero outside the image.  The forward
// pass uses the layer's weights; the input gradient of a layer uses the same
// kernel with the flipped, transposed weights wd[ci][kk * cout + co] =
// w[co][8 - kk][ci], because off(8 - kk) = -off(kk).
// One wave computes 32 pixels x 64 output channels (2 x 4 MFMA tiles).
// ---------------------------------------------------------------------------
// MODE: CONV_RELU (bias, relu), CONV_LINEAR (bias), CONV_MASK (no bias; zero where mask <= 0 if mask)
template <int MODE>
__global__ void __launch_bounds__(256) k_conv3(ConvArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int P = a.B * a.H * a.W;
  const int ngroups = (a.nout + 63) >> 6;
  const int ptile = wave / ngroups, ng = wave - ptile * ngroups;
  if (ptile * 32 >= P) return;
  const int i = lane & 15, g = lane >> 4;
  int ph[2], pw[2], pn[2];
  bool pv[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int p = ptile * 32 + 16 * r + i;
    pv[r] = p < P;
    const int q = pv[r] ? p : 0;
    pw[r] = q % a.W;
    ph[r] = (q / a.W) % a.H;
    pn[r] = q / (a.W * a.H);
  }
  const int n0 = ng * 64;
  const int ntile = min(4, (a.nout - n0) >> 4);
  f32x4 acc[2][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[r][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* wrow[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) wrow[t] = a.w + (size_t)(n0 + 16 * min(t, ntile - 1) + i) * a.kp + 8 * g;
  const int K = 9 * a.cin;
  int kk = 0, c = 8 * g;
  while (c >= a.cin) {
    c -= a.cin;
    ++kk;
  }
  const u32x4 zero = {0u, 0u, 0u, 0u};
  for (int k0 = 0; k0 < K; k0 += 32) {
    const int dy = kk / 3 - 1, dx = kk % 3 - 1;
    u32x4 av[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int hh = ph[r] + dy, ww = pw[r] + dx;
      const bool ok = pv[r] && kk < 9 && hh >= 0 && hh < a.H && ww >= 0 && ww < a.W;
      av[r] = ok ? ld16(a.x + ((size_t)(pn[r] * a.H + hh) * a.W + ww) * a.xs + c) : zero;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < ntile) {
        const u32x4 bv = ld16(wrow[t] + k0);
        acc[0][t] = mfma(av[0], bv, acc[0][t]);
        acc[1][t] = mfma(av[1], bv, acc[1][t]);
      }
    }
    c += 32;
    while (c >= a.cin) {
      c -= a.cin;
      ++kk;
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t >= ntile) continue;
    const int n = n0 + 16 * t + i;
    const float bn = MODE == CONV_MASK ? 0.f : a.bias[n];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = ptile * 32 + 16 * r + 4 * g + j;
        if (p >= P) continue;
        float v = acc[r][t][j] + bn;
        if (MODE == CONV_RELU) v = fmaxf(v, 0.f);
        if (MODE == CONV_MASK && a.mask && !bf_pos(a.mask[(size_t)p * a.ms + n])) v = 0.f;
        a.y[(size_t)p * a.ys + n] = f2bf(v);
      }
  }
}

// LDS access rule of gfx950 used by the layouts below (measured with the
// SQ_LDS_BANK_CONFLICT counter on access patterns of known shape): 64 banks
// of 4 bytes; a 16-byte access is served in four passes of 16 lanes, the
// pass of lane L being (bit 5 of L, parity of bits 2, 3 and 4 of L); an
// 8-byte access in two passes of 32 consecutive lanes.  A pass without two
// lanes on one bank (at different addresses) takes one cycle.
//
// The same convolution with the input tile staged in LDS: a workgroup owns a
// 16 x 16 block of output pixels of one image x 16 NT output channels; each
// wave computes 4 rows of it (64 pixels) x 16 NT channels (4 x NT MFMA tiles).
// NT (1..4) divides cout / 16, so no tile is partial and no MFMA is wasted.  The K
// loop runs over blocks of 32 input channels: per block the 18 x 18 input
// halo (zero outside the image and past cin) and the weights of all 9 taps
// for these channels go to LDS once, and the 9 taps then read their operands
// from it, so each input value is fetched from memory once instead of once
// per tap.  LDS rows (a pixel's or an output channel's 32 channels) are
// padded to 80 bytes and a row's four 16-byte chunks stored in the order
// 0, 2, 1, 3; MFMA row i of an operand tile is pixel (or channel) ch_row(i)
// of the 16, a permutation found by exhaustive search under the rule above
// for which every 16-byte operand read is conflict-free at any row offset;
// every operand address is a per-lane base plus an immediate.  The
// next block's loads are in flight in registers during the current block's
// 144 MFMAs per wave.
constexpr int CH_E = 18;                  // halo edge (16 + 2)
constexpr int CH_ROWB = 80;               // LDS bytes per row: 64 data + 16 pad
constexpr int CH_HALO_B = CH_E * CH_E * CH_ROWB;
constexpr int CH_LDS_B = CH_HALO_B + 9 * 64 * CH_ROWB;
constexpr int CH_NH = (CH_E * CH_E * 4 + 255) / 256;  // halo chunks per thread (6)

// LDS slot of 16-byte chunk c of a row, and the tile row held by MFMA row i
__device__ __forceinline__ int ch_slot(int c) { return ((c & 1) << 1) | (c >> 1); }
// ch_row: 0 2 4 6 1 3 5 7 9 11 13 15 8 10 12 14
__device__ __forceinline__ int ch_row(int i) { return (((i & 3) << 1) | ((i >> 2) & 1) | (i & 8)) ^ (i >> 3); }

template <int MODE, int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_conv3_halo(ConvArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[CH_LDS_B];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int ngroups = a.nout / (16 * NT);
  const int txn = (a.W + 15) >> 4, tyn = (a.H + 15) >> 4;
  int bid = blockIdx.x;
  const int ng = bid % ngroups;
  bid /= ngroups;
  const int tx = bid % txn;
  bid /= txn;
  const int ty = bid % tyn;
  const int img = bid / tyn;
  const int n0 = ng * 16 * NT;
  const int y0 = ty * 16, x0 = tx * 16;
  // loader slots: 16-byte chunk c = tid & 3 (channels 8c..8c+7 of the block)
  // of halo pixels (tid >> 2) + 64 u and of weight rows (tap u, channel tid >> 2)
  const int c8 = (tid & 3) * 8;
  int hpix[CH_NH];  // input pixel of each halo slot, -1 outside the image or the halo
#pragma unroll
  for (int u = 0; u < CH_NH; ++u) {
    const int hp = (tid >> 2) + 64 * u;
    const int hy = hp / CH_E, hx = hp - hy * CH_E;
    const int yy = y0 + hy - 1, xx = x0 + hx - 1;
    const bool ok = hp < CH_E * CH_E && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
    hpix[u] = ok ? (img * a.H + yy) * a.W + xx : -1;
  }
  const int hdst = (tid >> 2) * CH_ROWB + ch_slot(tid & 3) * 16;  // + 64 u rows
  const int wco = tid >> 2;
  const uint16_t* wsrc = wco < 16 * NT ? a.w + (size_t)(n0 + wco) * a.kp + c8 : nullptr;
  const int wdst = CH_HALO_B + wco * CH_ROWB + ch_slot(tid & 3) * 16;  // + 64 u rows
  const u32x4 zero = {0u, 0u, 0u, 0u};
  u32x4 hv[CH_NH], wvv[9];
  auto load = [&](int cb) {
    const int ch = cb * 32 + c8;
    const bool cok = ch < a.cin;
#pragma unroll
    for (int u = 0; u < CH_NH; ++u)
      hv[u] = (cok && hpix[u] >= 0) ? ld16(a.x + (size_t)hpix[u] * a.xs + ch) : zero;
#pragma unroll
    for (int u = 0; u < 9; ++u) wvv[u] = (cok && wsrc) ? ld16(wsrc + u * a.cin + cb * 32) : zero;
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < CH_NH; ++u)
      if ((tid >> 2) + 64 * u < CH_E * CH_E) *(u32x4*)(lds + hdst + u * 64 * CH_ROWB) = hv[u];
    if (wsrc)
#pragma unroll
      for (int u = 0; u < 9; ++u) *(u32x4*)(lds + wdst + u * 64 * CH_ROWB) = wvv[u];
  };
  f32x4 acc[4][NT];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[r][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  // operand bases: MFMA row i reads tile pixel (4 wv, ch_row(i)) at halo pixel
  // (4 wv + 1, ch_row(i) + 1) (the taps add -1..1) and output channel ch_row(i)
  const unsigned char* abase = lds + (4 * wv * CH_E + ch_row(i)) * CH_ROWB + 16 * ch_slot(g);
  const unsigned char* bbase = lds + CH_HALO_B + ch_row(i) * CH_ROWB + 16 * ch_slot(g);
  const int nb = (a.cin + 31) >> 5;
  load(0);
  for (int cb = 0; cb < nb; ++cb) {
    if (cb > 0) __syncthreads();
    store();
    __syncthreads();
    if (cb + 1 < nb) load(cb + 1);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap % 3;  // halo offsets 0..2
      u32x4 av[4], bv[NT];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = *(const u32x4*)(abase + ((r + dy) * CH_E + dx) * CH_ROWB);
#pragma unroll
      for (int t = 0; t < NT; ++t) bv[t] = *(const u32x4*)(bbase + (tap * 64 + 16 * t) * CH_ROWB);
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r][t] = mfma(av[r], bv[t], acc[r][t]);
      // keep the scheduler from hoisting later taps' operand reads (registers)
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int n = n0 + 16 * t + ch_row(i);
    const float bn_v = MODE == CONV_MASK ? 0.f : a.bias[n];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int yy = y0 + 4 * wv + r;
      if (yy >= a.H) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int xx = x0 + ch_row(4 * g + j);
        if (xx >= a.W) continue;
        const size_t p = (size_t)(img * a.H + yy) * a.W + xx;
        float v = acc[r][t][j] + bn_v;
        if (MODE == CONV_RELU) v = fmaxf(v, 0.f);
        if (MODE == CONV_MASK && a.mask && !bf_pos(a.mask[p * a.ms + n])) v = 0.f;
        a.y[p * a.ys + n] = f2bf(v);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient:  gw[co][kk][c] += sum_p gz[p][co] * x[p + off(kk)][c]
// GEMM M = co, N = k = kk * cin + c, reduction over pixels.  A workgroup owns
// a 64 x 64 (co, k) tile and a chunk of pixels, taken in slabs of 128 pixels.
// A thread loads 4 consecutive pixels x 8 channels of gz and of the im2col
// matrix (16-byte buffer loads, 8 lanes cover one pixel's 64 channels) and
// writes them transposed to LDS, one 8-byte store per channel (4 pixels).
// Buffer loads give 0 outside the resource's byte range, so the zero padding
// of the im2col matrix, the channels past cout and the pixels past the chunk
// cost no branches: an invalid lane takes an offset past the range.  LDS rows
// are a channel's 128 pixels; the 16-byte chunk c of row r sits at chunk
// position c ^ 2 ((r ^ (r >> 3)) & 7), which keeps both the transposing
// 8-byte stores and the MFMA operand reads (8 consecutive pixels, one 16-byte
// read) free of bank conflicts under the LDS access rule stated below.  Each wave runs 16 MFMAs per slab; the next slab's global
// loads are in flight meanwhile (double-buffered LDS, one barrier per slab).
// Partial tiles are added to the FP32 gradient with atomics; the workgroups
// of the first K tile also add the bias gradient sum_p gz[p][co].  About 1024
// workgroups per launch (two passes of two per CU) keep the atomics few.
// ---------------------------------------------------------------------------
constexpr int WG_PPT = 4;                 // pixels per thread per slab
constexpr int BUF_DWORD3 = 0x00020000;    // buffer resource word 3: raw 32-bit data
constexpr int BUF_OUT = 0x7FFFFFF0;       // an offset past every resource's range

__device__ __forceinline__ int wg_swz(int r, int c) { return c ^ (2 * ((r ^ (r >> 3)) & 7)); }

// q = p / d, r = p - q d for 0 <= p < 2^24, d >= 1, with rd = 1 / d
__device__ __forceinline__ void wg_divmod(int p, int d, float rd, int& q, int& r) {
  q = (int)((float)p * rd);
  r = p - q * d;
  if (r < 0) {
    --q;
    r += d;
  } else if (r >= d) {
    ++q;
    r -= d;
  }
}

// (low half of x, low half of y) and (high half of x, high half of y) as one
// word each: v_perm_b32 picks bytes of {S0 = y, S1 = x}, 0..3 from x, 4..7 from y
__device__ __forceinline__ uint32_t lo16x2(uint32_t x, uint32_t y) { return __builtin_amdgcn_perm(y, x, 0x05040100u); }
__device__ __forceinline__ uint32_t hi16x2(uint32_t x, uint32_t y) { return __builtin_amdgcn_perm(y, x, 0x07060302u); }

__device__ __forceinline__ u32x4 bload16(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
}

__global__ void __launch_bounds__(256) k_wgrad(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][64 * WG_SLAB];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][64 * WG_SLAB];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int P = a.B * a.H * a.W;
  // Workgroups are handed to the 8 XCDs round-robin by launch index; regroup
  // them so that one XCD runs all tiles of consecutive pixel chunks and its L2
  // serves their shared gz and x rows (the last N % 8 keep their own index).
  const int tiles = a.mtiles * a.ktiles, nwg = tiles * a.nch;
  int wg = blockIdx.x;
  if (wg < nwg - nwg % 8) wg = (wg & 7) * (nwg / 8) + (wg >> 3);
  const int chn = wg / tiles, tile = wg - chn * tiles;
  const int mt = tile / a.ktiles, kt = tile - mt * a.ktiles;
  const int m0 = mt * 64, kb = kt * 64;
  const int p_begin = chn * a.chunk;
  const int p_end = min(P, p_begin + a.chunk);
  // this thread's load slots: pixels 4 sp .. 4 sp + 3 of the slab, 8-column group s8
  const int sp = tid >> 3, s8 = (tid & 7) * 8;
  const bool a_ok = m0 + s8 < a.cout;
  const int kx = kb + s8;
  const int lkk = kx / a.cin, lc = kx - lkk * a.cin;
  const bool b_ok = lkk < 9;
  const int ldy = lkk / 3 - 1, ldx = lkk % 3 - 1;
  const int rel = ldy * a.W + ldx;  // pixel offset of the tap
  const float rW = 1.f / (float)a.W, rH = 1.f / (float)a.H;
  // LDS element offsets: the transposing stores of columns s8 + j ...
  int st_off[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) st_off[j] = (s8 + j) * WG_SLAB + 8 * wg_swz(s8 + j, sp >> 1) + (sp & 1) * 4;
  // ... and the MFMA operand reads: chunk 4 m + g of row 16 wv + i (A), 16 t + i (B)
  int ra_off[4], rb_off[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int ra = 16 * wv + i;
    ra_off[m] = ra * WG_SLAB + 8 * wg_swz(ra, 4 * m + g);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int rb = 16 * t + i;
      rb_off[t][m] = rb * WG_SLAB + 8 * wg_swz(rb, 4 * m + g);
    }
  }
  // the first K tile's workgroups also sum gz over their pixels: the bias gradient
  const bool do_bias = kt == 0 && a_ok;
  float bsum[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) bsum[j] = 0.f;
  // global loads of this thread's 4 pixels of the slab at s0 into registers
  auto load = [&](int s0, u32x4* va, u32x4* vb) {
    // gz rows s0 .. min(s0 + 128, p_end) - 1, channels from m0
    const int nv = min(WG_SLAB, p_end - s0);
    const __amdgpu_buffer_rsrc_t ra =
        __builtin_amdgcn_make_buffer_rsrc((void*)(a.gz + (size_t)s0 * a.gzs + m0), (short)0,
                                          (nv * a.gzs - m0) * 2, BUF_DWORD3);
    // x rows the slab's taps can reach
    const int bp = max(0, s0 - a.W - 1), ep = min(P, s0 + WG_SLAB + a.W + 1);
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(a.x + (size_t)bp * a.xs), (short)0, (ep - bp) * a.xs * 2, BUF_DWORD3);
    const int p0 = s0 + WG_PPT * sp;
    int hw, w, n, h;
    wg_divmod(min(p0, P - 1), a.W, rW, hw, w);
    wg_divmod(hw, a.H, rH, n, h);
#pragma unroll
    for (int q = 0; q < WG_PPT; ++q) {
      va[q] = bload16(ra, a_ok ? ((WG_PPT * sp + q) * a.gzs + s8) * 2 : BUF_OUT);
      const int hh = h + ldy, ww = w + ldx;
      const bool ok = b_ok && (unsigned)hh < (unsigned)a.H && (unsigned)ww < (unsigned)a.W;
      vb[q] = bload16(rx, ok ? ((p0 + q + rel - bp) * a.xs + lc) * 2 : BUF_OUT);
      if (++w == a.W) {
        w = 0;
        if (++h == a.H) h = 0;
      }
    }
  };
  // transposed store of the 4 pixels into LDS buffer `buf` (+ bias partial sums)
  auto stage = [&](int buf, const u32x4* va, const u32x4* vb) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      *(uint2*)&As[buf][st_off[2 * j]] = uint2{lo16x2(va[0][j], va[1][j]), lo16x2(va[2][j], va[3][j])};
      *(uint2*)&As[buf][st_off[2 * j + 1]] = uint2{hi16x2(va[0][j], va[1][j]), hi16x2(va[2][j], va[3][j])};
      *(uint2*)&Bs[buf][st_off[2 * j]] = uint2{lo16x2(vb[0][j], vb[1][j]), lo16x2(vb[2][j], vb[3][j])};
      *(uint2*)&Bs[buf][st_off[2 * j + 1]] = uint2{hi16x2(vb[0][j], vb[1][j]), hi16x2(vb[2][j], vb[3][j])};
    }
    if (do_bias) {
#pragma unroll
      for (int q = 0; q < WG_PPT; ++q) {
        float f[8];
        unpack8(va[q], f);
#pragma unroll
        for (int j = 0; j < 8; ++j) bsum[j] += f[j];
      }
    }
  };
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  u32x4 va[WG_PPT], vb[WG_PPT];
  // one slab from LDS buffer `cur` (a literal at each use), the next slab's
  // loads in flight and staged into the other buffer; false after the last
  auto slab = [&](int s0, int cur) {
    const bool more = s0 + WG_SLAB < p_end;
    if (more) load(s0 + WG_SLAB, va, vb);
#pragma unroll
    for (int m = 0; m < WG_SLAB / 32; ++m) {
      const u32x4 av = *(const u32x4*)(&As[cur][ra_off[m]]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const u32x4 bv = *(const u32x4*)(&Bs[cur][rb_off[t][m]]);
        acc[t] = mfma(av, bv, acc[t]);
      }
    }
    if (more) stage(cur ^ 1, va, vb);
    __syncthreads();
    return more;
  };
  load(p_begin, va, vb);
  stage(0, va, vb);
  __syncthreads();
  for (int s0 = p_begin;; s0 += 2 * WG_SLAB) {
    if (!slab(s0, 0)) break;
    if (!slab(s0 + WG_SLAB, 1)) break;
  }
  if (kt == 0) {
    // lanes with equal (lane & 7) hold the same 8 channels: reduce them, then
    // over the 4 waves through LDS (free after the loop's last barrier)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      for (int off = 8; off < 64; off <<= 1) bsum[j] += __shfl_xor(bsum[j], off);
    float* red = (float*)&As[0][0];
    if (lane < 8)
#pragma unroll
      for (int j = 0; j < 8; ++j) red[wv * 64 + s8 + j] = bsum[j];
    __syncthreads();
    if (tid < 64 && m0 + tid < a.cout)
      atomicAdd(a.gb + m0 + tid, red[tid] + red[64 + tid] + red[128 + tid] + red[192 + tid]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = kb + 16 * t + i;
    const int kk = k / a.cin, c = k - kk * a.cin;
    if (kk >= 9 || c >= a.cin_true) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int co = m0 + 16 * wv + 4 * g + j;
      if (co < a.cout) atomicAdd(a.gw + ((size_t)co * 9 + kk) * a.cin_true + c, acc[t][j]);
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient with the input staged once for all nine taps (cin >= 48):
// a workgroup owns 64 output channels (co) x 64 input channels (c) x the 9
// taps, i.e. a 64 x 576 block of the gradient, and a chunk of pixel tiles of
// 8 rows x 16 columns of one image.  Per tile the 128 pixels of gz (as a
// channel-major gz^T, the layout and swizzle of k_wgrad's slab) and the
// 10 x 18 halo of x (zero outside the image) go to LDS once; each tap then
// reads its operand at its (dy, dx) offset inside the halo, so x is fetched
// 1.4 times per tile instead of once per tap, and gz once per 576 gradient
// columns instead of once per 64 -- k_wgrad is bound by those re-fetches.
// x^T rows: channel c, halo row hr, 32 columns (64 bytes, 18 used), channel
// stride 672 bytes, the 16-byte chunk k of a row at slot k ^ ((c >> 3) & 3).
// Under the measured gfx950 rule (a 16-byte read in four passes of 16 lanes
// grouped by bit 5 and the parity of bits 2-4 of the lane) the operand reads
// are 2-way conflicted and the transposing 8-byte stores about 2-way; the
// unswizzled layout makes the reads conflict-free but the stores 8-way, and
// a search of per-channel XOR tables found nothing better than a 4 % saving
// of LDS cycles over both.  A tap's operand is columns
// col..col+7 of a halo row with col = 8 (g & 1) + dx: two aligned 16-byte
// reads per (row, dy) give the three dx shifts (dx = 1 by byte alignment, dx
// = 2 by a dword shift).  Eight waves: waves 0-3 load and stage gz, waves
// 4-7 the x halo; wave w computes output channels 32 (w >> 2)..+31 x input
// channels 16 (w & 3)..+15 of every tap (2 x 9 MFMA tiles, 18 MFMAs per 32
// pixels against 8 operand reads).  The next tile's loads are in flight in
// registers during the current tile's MFMAs (double-buffered LDS, one
// barrier per tile, one workgroup per CU).  Each workgroup writes its
// partial 64 x 576 block to a scratch area with plain stores and
// k_wgrad_sum adds the chunks into the gradient: the blocks of all resident
// workgroups land at the end of the launch, and as FP32 atomics (1.2e6
// 64-byte requests per launch at two 4-wave workgroups per CU) they took
// as long as the MFMAs.  The workgroups of the first channel tile add the
// bias gradient with atomics (64 each).
// ---------------------------------------------------------------------------
constexpr int WH_TH = 8, WH_TW = 16;          // pixel tile (128 pixels)
constexpr int WH_HR = WH_TH + 2;              // halo rows
constexpr int WH_NQ = 5;                      // 4-pixel quads per halo row (20 >= 18 columns)
constexpr int WH_NU = WH_HR * WH_NQ;          // quads per halo (50)
constexpr int WH_ROWB = 64;                   // LDS bytes per halo row of one channel
constexpr int WH_CHB = WH_HR * WH_ROWB + 32;  // LDS bytes per channel (672)
constexpr int WH_GZB = 64 * 128 * 2;          // gz^T: 64 channels x 128 pixels
constexpr int WH_BUF = WH_GZB + 64 * WH_CHB;  // one tile's operands (59392 bytes)
constexpr int WH_TARGET = 256;                // workgroups per launch (one per CU)
constexpr int WH_MIN_CIN = 48;                // narrower inputs keep k_wgrad

__global__ void __launch_bounds__(512) k_wgrad_halo(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[2 * WH_BUF];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int tyn = (a.H + WH_TH - 1) / WH_TH, txn = (a.W + WH_TW - 1) / WH_TW;
  const int ntile = a.B * tyn * txn;
  // the 8 XCDs take workgroups round-robin: regroup so that one XCD runs all
  // channel blocks of consecutive chunks (they share gz and x rows in its L2)
  const int tiles = a.mtiles * a.ktiles, nwg = tiles * a.nch;
  int wg = blockIdx.x;
  if (wg < nwg - nwg % 8) wg = (wg & 7) * (nwg / 8) + (wg >> 3);
  const int chn = wg / tiles, tile = wg - chn * tiles;
  const int mt = tile / a.ktiles, ct = tile - mt * a.ktiles;
  const int m0 = mt * 64, c0 = ct * 64;
  const int t_begin = chn * a.chunk, t_end = min(ntile, t_begin + a.chunk);
  // loaders: waves 0-3 stage gz (pixels 4 sp .. 4 sp + 3 of the tile: row
  // sp >> 2, columns 4 (sp & 3) ..; channels m0 + s8 ..), waves 4-7 the x
  // halo (quads u0 and u0 + 32: halo row u % 10, columns 4 (u / 10) ..;
  // channels c0 + s8 ..); both hold their loads in the same registers
  const bool gz_role = wv < 4;
  const int lt = tid & 255;
  const int sp = lt >> 3, a8 = lt & 7, s8 = 8 * a8;
  const bool a_ok = m0 + s8 < a.cout, x_ok = c0 + s8 < a.cin;
  const int u0 = lt >> 3;
  const bool u1_ok = u0 + 32 < WH_NU;
  int xst[2];  // byte offset of channel s8's row slot for each quad; + j * WH_CHB per channel
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const int u = u0 + 32 * v, hr = u % WH_HR, q = u / WH_HR;
    xst[v] = WH_GZB + s8 * WH_CHB + hr * WH_ROWB + 16 * ((q >> 1) ^ (a8 & 3)) + 8 * (q & 1);
  }
  // wave w computes output channels 32 (w >> 2) .. + 31 (two MFMA rows of
  // 16) x input channels 16 (w & 3) .. + 15 of all nine taps.  A row 16 mb +
  // i: chunk 4 kc + g sits at slot (4 kc + g) ^ ra_sw[m]; B channel cx, halo
  // row 2 kc + (g >> 1) + dy, chunks (g & 1) and (g & 1) + 1
  const int mh = wv >> 2;
  int ra_sw[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) ra_sw[m] = wg_swz(16 * (2 * mh + m) + i, 0);
  const int cx = 16 * (wv & 3) + i, xsw = (cx >> 3) & 3;
  const int bx = WH_GZB + cx * WH_CHB + (g >> 1) * WH_ROWB;
  const int bs0 = 16 * ((g & 1) ^ xsw), bs1 = 16 * (((g & 1) + 1) ^ xsw);
  const bool do_bias = ct == 0 && gz_role && a_ok;
  float bsum[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) bsum[j] = 0.f;
  const u32x4 zero = {0u, 0u, 0u, 0u};
  u32x4 pre[8];  // gz role: pixels 0..3; x role: quad u0 (0..3) and u0 + 32 (4..7)
  auto load = [&](int t) {
    const int img = t / (tyn * txn), rt = t - img * tyn * txn;
    const int y0 = (rt / txn) * WH_TH, x0 = (rt % txn) * WH_TW;
    if (gz_role) {
      const int yy = y0 + (sp >> 2), xb = x0 + 4 * (sp & 3);
      const size_t prow = (size_t)(img * a.H + yy) * a.W;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool ok = a_ok && yy < a.H && xb + q < a.W;
        pre[q] = ok ? ld16(a.gz + (prow + xb + q) * a.gzs + m0 + s8) : zero;
      }
    } else {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int u = u0 + 32 * v, hr = u % WH_HR, q = u / WH_HR;
        const int yy = y0 + hr - 1, xb = x0 + 4 * q - 1;
        const bool rok = x_ok && (v == 0 || u1_ok) && yy >= 0 && yy < a.H;
        const size_t prow = (size_t)(img * a.H + yy) * a.W;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int xx = xb + e;
          const bool ok = rok && 4 * q + e < WH_TW + 2 && xx >= 0 && xx < a.W;
          pre[4 * v + e] = ok ? ld16(a.x + (prow + xx) * a.xs + c0 + s8) : zero;
        }
      }
    }
  };
  // transposed stores of the loaded tile into LDS buffer `buf`
  auto stage = [&](int buf) {
    unsigned char* b = lds + buf * WH_BUF;
    if (gz_role) {
      uint16_t* gzT = (uint16_t*)b;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r0 = s8 + 2 * j, r1 = r0 + 1;
        *(uint2*)&gzT[r0 * 128 + 8 * wg_swz(r0, sp >> 1) + (sp & 1) * 4] =
            uint2{lo16x2(pre[0][j], pre[1][j]), lo16x2(pre[2][j], pre[3][j])};
        *(uint2*)&gzT[r1 * 128 + 8 * wg_swz(r1, sp >> 1) + (sp & 1) * 4] =
            uint2{hi16x2(pre[0][j], pre[1][j]), hi16x2(pre[2][j], pre[3][j])};
      }
      if (do_bias) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float f[8];
          unpack8(pre[q], f);
#pragma unroll
          for (int j = 0; j < 8; ++j) bsum[j] += f[j];
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        if (v == 1 && !u1_ok) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          *(uint2*)(b + xst[v] + (2 * j) * WH_CHB) =
              uint2{lo16x2(pre[4 * v][j], pre[4 * v + 1][j]), lo16x2(pre[4 * v + 2][j], pre[4 * v + 3][j])};
          *(uint2*)(b + xst[v] + (2 * j + 1) * WH_CHB) =
              uint2{hi16x2(pre[4 * v][j], pre[4 * v + 1][j]), hi16x2(pre[4 * v + 2][j], pre[4 * v + 3][j])};
        }
      }
    }
  };
  f32x4 acc[2][9];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) acc[m][tap] = f32x4{0.f, 0.f, 0.f, 0.f};
  // one tile from LDS buffer `cur` (a literal at each use), the next tile's
  // loads in flight and staged into the other buffer; false after the last
  auto step = [&](int t, int cur) {
    const bool more = t + 1 < t_end;
    if (more) load(t + 1);
    const unsigned char* b = lds + cur * WH_BUF;
    const uint16_t* gzT = (const uint16_t*)b;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      u32x4 av[2];
#pragma unroll
      for (int m = 0; m < 2; ++m)
        av[m] = *(const u32x4*)&gzT[(16 * (2 * mh + m) + i) * 128 + 8 * ((4 * kc + g) ^ ra_sw[m])];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const unsigned char* row = b + bx + (2 * kc + dy) * WH_ROWB;
        const u32x4 w0 = *(const u32x4*)(row + bs0), w1 = *(const u32x4*)(row + bs1);
        const u32x4 b1 = {__builtin_amdgcn_alignbyte(w0[1], w0[0], 2), __builtin_amdgcn_alignbyte(w0[2], w0[1], 2),
                          __builtin_amdgcn_alignbyte(w0[3], w0[2], 2), __builtin_amdgcn_alignbyte(w1[0], w0[3], 2)};
        const u32x4 b2 = {w0[1], w0[2], w0[3], w1[0]};
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          acc[m][3 * dy] = mfma(av[m], w0, acc[m][3 * dy]);
          acc[m][3 * dy + 1] = mfma(av[m], b1, acc[m][3 * dy + 1]);
          acc[m][3 * dy + 2] = mfma(av[m], b2, acc[m][3 * dy + 2]);
        }
      }
    }
    if (more) stage(cur ^ 1);
    __syncthreads();
    return more;
  };
  if (t_begin < t_end) {
    load(t_begin);
    stage(0);
    __syncthreads();
    for (int t = t_begin;; t += 2) {
      if (!step(t, 0)) break;
      if (!step(t + 1, 1)) break;
    }
  }
  if (ct == 0) {
    // gz lanes with equal (lane & 7) hold the same 8 channels: reduce them,
    // then over the 4 gz waves through LDS (free after the loop's last barrier)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      for (int off = 8; off < 64; off <<= 1) bsum[j] += __shfl_xor(bsum[j], off);
    float* red = (float*)lds;
    if (gz_role && lane < 8)
#pragma unroll
      for (int j = 0; j < 8; ++j) red[wv * 64 + s8 + j] = bsum[j];
    __syncthreads();
    if (tid < 64 && m0 + tid < a.cout)
      atomicAdd(a.gb + m0 + tid, red[tid] + red[64 + tid] + red[128 + tid] + red[192 + tid]);
  }
  // partial block [co 64][tap 9][c 64] of this chunk and channel tile
  float* pb = a.part + ((size_t)chn * tiles + tile) * (64 * 576);
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int tap = 0; tap < 9; ++tap)
        pb[((16 * (2 * mh + m) + 4 * g + j) * 9 + tap) * 64 + cx] = acc[m][tap][j];
}

// gw[co][tap][c] += sum over the nch chunks of the partial blocks of
// k_wgrad_halo.  A 256-thread block takes 16 consecutive elements of the
// (tiles x 64 x 576) blocks; its 16 groups of 16 lanes sum every 16th chunk
// (coalesced 64-byte reads) and meet in LDS.
__global__ void __launch_bounds__(256) k_wgrad_sum(const float* __restrict__ part, int tiles, int nch, int ktiles,
                                                   int cout, int cin_true, float* __restrict__ gw) {
  __shared__ float red[16][16];
  const size_t blk = (size_t)64 * 576;
  const size_t e = (size_t)blockIdx.x * 16 + (threadIdx.x & 15);
  const int grp = threadIdx.x >> 4;
  float s = 0.f;
  if (e < (size_t)tiles * blk) {
    const int tile = (int)(e / blk);
    const size_t r = e % blk;
    for (int k = grp; k < nch; k += 16) s += part[((size_t)k * tiles + tile) * blk + r];
  }
  red[grp][threadIdx.x & 15] = s;
  __syncthreads();
  if (threadIdx.x < 16 && e < (size_t)tiles * blk) {
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) t += red[k][threadIdx.x];
    const int tile = (int)(e / blk), r = (int)(e % blk);
    const int co = (tile / ktiles) * 64 + r / 576, tap = (r % 576) / 64, c = (tile % ktiles) * 64 + r % 64;
    if (co < cout && c < cin_true) gw[((size_t)co * 9 + tap) * cin_true + c] += t;
  }
}

// ---------------------------------------------------------------------------
// resampling, 8 channels per thread.  Sizes: fine grid H x W, coarse H/2 x W/2.
// ---------------------------------------------------------------------------
// y (coarse) = mean of each 2x2 block of x (fine)
__global__ void k_pool(const uint16_t* __restrict__ x, int xs, uint16_t* __restrict__ y, int ys, int B, int H, int W,
                       int C) {
  const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
  const size_t n = (size_t)B * Ho * Wo * C8;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(k % C8) * 8;
    const size_t q = k / C8;
    const int w = (int)(q % Wo), h = (int)((q / Wo) % Ho), b = (int)(q / ((size_t)Wo * Ho));
    const size_t f = (size_t)(b * H + 2 * h) * W + 2 * w;
    float s[8], t[8];
    unpack8(ld16(x + f * xs + c), s);
    const size_t nb[3] = {f + 1, f + W, f + W + 1};
    for (int m = 0; m < 3; ++m) {
      unpack8(ld16(x + nb[m] * xs + c), t);
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += t[j];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] *= 0.25f;
    st16(y + q * ys + c, pack8(s));
  }
}

// y (fine) = x (coarse) repeated over each 2x2 block
__global__ void k_up(const uint16_t* __restrict__ x, int xs, uint16_t* __restrict__ y, int ys, int B, int H, int W,
                     int C) {
  const int C8 = C / 8, Wc = W / 2, Hc = H / 2;
  const size_t n = (size_t)B * H * W * C8;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(k % C8) * 8;
    const size_t p = k / C8;
    const int w = (int)(p % W), h = (int)((p / W) % H), b = (int)(p / ((size_t)W * H));
    const size_t q = (size_t)(b * Hc + h / 2) * Wc + w / 2;
    st16(y + p * ys + c, ld16(x + q * xs + c));
  }
}

// gx (coarse) = (sum of each 2x2 block of gy (fine)) where mask (coarse) > 0, else 0
__global__ void k_up_bwd(const uint16_t* __restrict__ gy, int gys, uint16_t* __restrict__ gx, int gxs,
                         const uint16_t* __restrict__ mask, int ms, int B, int H, int W, int C) {
  const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
  const size_t n = (size_t)B * Ho * Wo * C8;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(k % C8) * 8;
    const size_t q = k / C8;
    const int w = (int)(q % Wo), h = (int)((q / Wo) % Ho), b = (int)(q / ((size_t)Wo * Ho));
    const size_t f = (size_t)(b * H + 2 * h) * W + 2 * w;
    float s[8], t[8];
    unpack8(ld16(gy + f * gys + c), s);
    const size_t nb[3] = {f + 1, f + W, f + W + 1};
    for (int m = 0; m < 3; ++m) {
      unpack8(ld16(gy + nb[m] * gys + c), t);
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += t[j];
    }
    const u32x4 mv = ld16(mask + q * ms + c);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint16_t mb = (uint16_t)((mv[j / 2] >> (16 * (j & 1))) & 0xFFFFu);
      if (!bf_pos(mb)) s[j] = 0.f;
    }
    st16(gx + q * gxs + c, pack8(s));
  }
}

// dst (fine) = (a (fine) + g (coarse parent) / 4) where mask (fine) > 0, else 0
__global__ void k_pool_bwd_add(const uint16_t* __restrict__ a, int as, const uint16_t* __restrict__ g, int gs,
                               const uint16_t* __restrict__ mask, int ms, uint16_t* __restrict__ dst, int ds, int B,
                               int H, int W, int C) {
  const int C8 = C / 8, Wc = W / 2, Hc = H / 2;
  const size_t n = (size_t)B * H * W * C8;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(k % C8) * 8;
    const size_t p = k / C8;
    const int w = (int)(p % W), h = (int)((p / W) % H), b = (int)(p / ((size_t)W * H));
    const size_t q = (size_t)(b * Hc + h / 2) * Wc + w / 2;
    float s[8], t[8];
    unpack8(ld16(a + p * as + c), s);
    unpack8(ld16(g + q * gs + c), t);
    const u32x4 mv = ld16(mask + p * ms + c);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint16_t mb = (uint16_t)((mv[j / 2] >> (16 * (j & 1))) & 0xFFFFu);
      s[j] = bf_pos(mb) ? s[j] + 0.25f * t[j] : 0.f;
    }
    st16(dst + p * ds + c, pack8(s));
  }
}

// ---------------------------------------------------------------------------
// input normalisation, head, loss, output, optimiser
// ---------------------------------------------------------------------------
// sums[2b] += sum of I, sums[2b+1] += sum of I^2 over image b of maps [B][4][H*W]
// (256-thread blocks; one pair of atomics per block)
__global__ void k_sums(const double* __restrict__ maps, int HW, int runs, double* __restrict__ sums) {
  __shared__ double red[2][4];
  const int b = blockIdx.y;
  double a1 = 0.0, a2 = 0.0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < HW; p += gridDim.x * blockDim.x) {
    const double* m = maps + (size_t)b * 4 * runs * HW + p;
    const double I = runs == 2 ? 0.5 * (m[0] + m[4 * (size_t)HW]) : m[0];
    a1 += I;
    a2 += I * I;
  }
  for (int off = 32; off > 0; off >>= 1) {
    a1 += __shfl_xor(a1, off);
    a2 += __shfl_xor(a2, off);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a1;
    red[1][threadIdx.x >> 6] = a2;
  }
  __syncthreads();
  if (threadIdx.x < 2)
    atomicAdd(sums + 2 * b + threadIdx.x,
              red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3]);
}

// Input features of pixel p of image b (s = the image's mean I, Ihat = I/s):
//   x[p][0..7] = ln max(Ihat, 1e-6), Q/I, U/I, V/I (0 where I <= 0), 0, 0, 0, 0 (BF16)
//   xq[p] = (Q/I, U/I) and ihat[p] = Ihat in FP32; tgt[p] = (Q, U) of the
//   target maps / s (FP32).
// With runs == 2 an input image is two independent runs A and B ([8][H][W]:
// A's I, Q, U, V, then B's); (I, Q, U, V) above are then their mean, and
// x[p][4..7] = |S_A - S_B| / (2 I) for S = I, Q, U, V (clamped to 1, 0 where
// I <= 0): a one-sample estimate of the mean's per-pixel noise, unchanged by
// swapping the runs and by the dihedral transforms' signs.
// With aug, image b is first transformed by the dihedral element aug[b] =
// r + 4 f: mirror the width axis if f, then r quarter turns (numpy's rot90;
// dihedral_source gives the pixel read); Stokes (Q, U, V) ->
// ((-1)^r Q, (-1)^(r+f) U, (-1)^f V).  Odd r requires H == W.
// Pixel (h, w) of the image T = rot^r(mirror^f(m)) of an H x W image m
// (code = r + 4 f; rot = numpy's rot90 on (H, W), T is W x H for odd r): on
// return (h, w) is the pixel of m it reads and (sq, su, sv) the signs of its
// Q, U, V.  Source in mirror^f(m): r = 1: (w, W-1-h); r = 2: (H-1-h,
// W-1-w); r = 3: (H-1-w, h); then the mirror flips the column.
__device__ __forceinline__ void dihedral_source(int code, int H, int W, int& h, int& w, double& sq, double& su,
                                                double& sv) {
  const int r = code & 3, f = code >> 2;
  const int h0 = h, w0 = w;
  if (r == 1) {
    h = w0;
    w = W - 1 - h0;
  } else if (r == 2) {
    h = H - 1 - h0;
    w = W - 1 - w0;
  } else if (r == 3) {
    h = H - 1 - w0;
    w = h0;
  }
  if (f) w = W - 1 - w;
  sq = (r & 1) ? -1.0 : 1.0;
  su = ((r + f) & 1) ? -1.0 : 1.0;
  sv = f ? -1.0 : 1.0;
}

// code_all >= 0 (with aug == nullptr) applies that one element to every image.
__global__ void k_prep(const double* __restrict__ maps, const double* __restrict__ target,
                       const double* __restrict__ sums, const int32_t* __restrict__ aug, int code_all, int B, int H,
                       int W, int runs, uint16_t* __restrict__ x, float* __restrict__ xq, float* __restrict__ ihat,
                       float* __restrict__ tgt) {
  const int HW = H * W;
  const size_t n = (size_t)B * HW;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const size_t b = k / HW;
    int h = (int)(k % HW) / W, w = (int)(k % HW) % W;
    double sq = 1.0, su = 1.0, sv = 1.0;
    if (aug) dihedral_source(aug[b], H, W, h, w, sq, su, sv);
    else if (code_all >= 0) dihedral_source(code_all, H, W, h, w, sq, su, sv);
    const size_t p = (size_t)h * W + w;
    const double mean = sums[2 * b] / HW;
    const double* m = maps + b * 4 * runs * HW + p;
    const size_t rb = 4 * (size_t)HW;  // run B's maps (runs == 2)
    auto stokes = [&](int c) { return runs == 2 ? 0.5 * (m[c * (size_t)HW] + m[rb + c * (size_t)HW]) : m[c * (size_t)HW]; };
    const double I = stokes(0);
    const double Ih = mean > 0.0 ? I / mean : 0.0;
    // ratios by division (in the wings of a thick disk I can be subnormal,
    // where 1 / I overflows), clamped to [-1, 1], the range of a physical
    // Stokes vector (I >= |(Q, U, V)|)
    const bool pos = I > 0.0;
    auto frac = [&](double x) { return pos ? (float)fmin(1.0, fmax(-1.0, x / I)) : 0.f; };
    float f8[8];
    f8[0] = (float)log(fmax(Ih, 1e-6));
    f8[1] = (float)sq * frac(stokes(1));
    f8[2] = (float)su * frac(stokes(2));
    f8[3] = (float)sv * frac(stokes(3));
#pragma unroll
    for (int c = 0; c < 4; ++c)
      f8[4 + c] = runs == 2 ? frac(0.5 * fabs(m[c * (size_t)HW] - m[rb + c * (size_t)HW])) : 0.f;
    st16(x + k * 8, pack8(f8));
    xq[2 * k] = f8[1];
    xq[2 * k + 1] = f8[2];
    ihat[k] = (float)Ih;
    if (target) {
      const double* r = target + b * 4 * HW + p;
      const double is = mean > 0.0 ? 1.0 / mean : 0.0;
      tgt[2 * k] = (float)(sq * r[HW] * is);
      tgt[2 * k + 1] = (float)(su * r[2 * (size_t)HW] * is);
    }
  }
}

// out[p][o] = xq[p][o] + hb[o] + sum_c d[p][c] hw[o][c]   (C % 8 == 0)
// Eight lanes per pixel: lane g of a group reads channels 8g + 64i (16 bytes
// each), so a group's loads of one pixel are contiguous and each load
// instruction of a wave reads eight whole pixels (with one lane per pixel
// every instruction touched 64 lines for 16 bytes of each: 3.5x slower).
// The partial sums meet by lane shuffles inside the group; all eight lanes
// of a group take the same p, so a shuffle never reads an inactive lane.
__global__ void k_head(const uint16_t* __restrict__ d, int C, const float* __restrict__ hw,
                       const float* __restrict__ hb, const float* __restrict__ xq, float* __restrict__ out, size_t P) {
  const int g = threadIdx.x & 7;
  const size_t stride = ((size_t)gridDim.x * blockDim.x) >> 3;
  for (size_t p = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3; p < P; p += stride) {
    float a0 = 0.f, a1 = 0.f;
    for (int c = 8 * g; c < C; c += 64) {
      float v[8];
      unpack8(ld16(d + p * C + c), v);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        a0 += v[j] * hw[c + j];
        a1 += v[j] * hw[C + c + j];
      }
    }
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
      a0 += __shfl_xor(a0, off);
      a1 += __shfl_xor(a1, off);
    }
    if (g == 0) {
      out[2 * p] = xq[2 * p] + hb[0] + a0;
      out[2 * p + 1] = xq[2 * p + 1] + hb[1] + a1;
    }
  }
}

// Relative-error loss: with e = out * Ihat - tgt (both channels) and
// W_b = sum_p Ihat^2 = (sum I^2) / s^2 of image b,
//   loss += sum_p |e|^2 / (B W_b)   (FP64),   go = 2 e Ihat / (B W_b).
// Grid (blocks, B) of 256-thread blocks: image b = blockIdx.y, so the scale
// is formed once per thread; one atomic per block.
__global__ void k_loss(const float* __restrict__ out, const float* __restrict__ tgt,
                       const float* __restrict__ ihat, const double* __restrict__ sums, int B, int HW,
                       float* __restrict__ go, double* __restrict__ loss) {
  __shared__ double red[4];
  const int b = blockIdx.y;
  const double mean = sums[2 * b] / HW;
  const double wb = mean > 0.0 ? sums[2 * b + 1] / (mean * mean) : 0.0;
  const double scale = wb > 0.0 ? 1.0 / (B * wb) : 0.0;
  const float s2 = (float)(2.0 * scale);
  double acc = 0.0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < HW; p += gridDim.x * blockDim.x) {
    const size_t k = (size_t)b * HW + p;
    const float ih = ihat[k];
    const float2 o = *(const float2*)(out + 2 * k), t = *(const float2*)(tgt + 2 * k);
    const float e0 = o.x * ih - t.x, e1 = o.y * ih - t.y;
    *(float2*)(go + 2 * k) = float2{s2 * e0 * ih, s2 * e1 * ih};
    acc += (double)e0 * e0 + (double)e1 * e1;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, (red[0] + red[1] + red[2] + red[3]) * scale);
}

// Head backward over a chunk of pixels (256-thread blocks): thread t owns
// channels 8 (t % C8) .. +7 (C8 = C / 8) of pixels t / C8, + 256 / C8, ...:
// ghw[o][c] += sum_p go[p][o] d[p][c]; ghb[o] += sum_p go[p][o];
// gd[p][c] = (sum_o go[p][o] hw[o][c]) where d[p][c] > 0, else 0.
// Per-thread sums are combined in LDS, then one atomic per weight per block.
constexpr int HB_CHUNK = 1024;  // pixels per block
__global__ void k_head_bwd(const float* __restrict__ go, const uint16_t* __restrict__ d, int C,
                           const float* __restrict__ hw, float* __restrict__ ghw, float* __restrict__ ghb,
                           uint16_t* __restrict__ gd, size_t P) {
  __shared__ float red[2 * 512 + 2];
  const int tid = threadIdx.x;
  const int C8 = C >> 3, pp = 256 / C8;
  for (int k = tid; k < 2 * C + 2; k += 256) red[k] = 0.f;
  __syncthreads();
  const int g = tid % C8, pl = tid / C8;
  if (pl < pp) {
    float h0[8], h1[8], a0[8], a1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      h0[j] = hw[8 * g + j];
      h1[j] = hw[C + 8 * g + j];
      a0[j] = a1[j] = 0.f;
    }
    float sb0 = 0.f, sb1 = 0.f;
    const size_t p0 = (size_t)blockIdx.x * HB_CHUNK;
    const size_t pe = P - p0 < (size_t)HB_CHUNK ? P : p0 + HB_CHUNK;
    for (size_t p = p0 + pl; p < pe; p += pp) {
      const float2 o = *(const float2*)(go + 2 * p);
      float v[8], r[8];
      unpack8(ld16(d + p * C + 8 * g), v);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        a0[j] += o.x * v[j];
        a1[j] += o.y * v[j];
        r[j] = v[j] > 0.f ? o.x * h0[j] + o.y * h1[j] : 0.f;
      }
      st16(gd + p * C + 8 * g, pack8(r));
      sb0 += o.x;
      sb1 += o.y;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      atomicAdd(&red[8 * g + j], a0[j]);
      atomicAdd(&red[C + 8 * g + j], a1[j]);
    }
    if (g == 0) {
      atomicAdd(&red[2 * C], sb0);
      atomicAdd(&red[2 * C + 1], sb1);
    }
  }
  __syncthreads();
  for (int k = tid; k < 2 * C; k += 256) atomicAdd(ghw + k, red[k]);
  if (tid < 2) atomicAdd(ghb + tid, red[2 * C + tid]);
}

// Test-time averaging: out holds the network's fractions (q', u') of the
// images transformed by `code`; each is moved back to its source pixel with
// the inverse Stokes signs (the signs are their own inverses) and added to
// acc ([B][HW][2] in the original pixel order), or stored there if first.
// The transform is a bijection of each image's pixels: no two threads write
// the same element.
__global__ void k_tta_acc(const float* __restrict__ out, int B, int H, int W, int code, int first,
                          float* __restrict__ acc) {
  const int HW = H * W;
  const size_t n = (size_t)B * HW;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const size_t b = k / HW;
    int h = (int)(k % HW) / W, w = (int)(k % HW) % W;
    double sq, su, sv;
    dihedral_source(code, H, W, h, w, sq, su, sv);
    const size_t src = b * HW + (size_t)h * W + w;
    const float q = (float)sq * out[2 * k], u = (float)su * out[2 * k + 1];
    acc[2 * src] = first ? q : acc[2 * src] + q;
    acc[2 * src + 1] = first ? u : acc[2 * src + 1] + u;
  }
}

// denoised maps: I and V from the input (the two runs' mean if runs == 2),
// Q = scale q' I and U = scale u' I
__global__ void k_output(const double* __restrict__ maps, const float* __restrict__ out, int B, int HW, int runs,
                         double scale, double* __restrict__ dst) {
  const size_t n = (size_t)B * HW;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const size_t b = k / HW, p = k % HW;
    const double* m = maps + b * 4 * runs * HW + p;
    double* o = dst + b * 4 * HW + p;
    const size_t rb = 4 * (size_t)HW;
    const double I = runs == 2 ? 0.5 * (m[0] + m[rb]) : m[0];
    o[0] = I;
    o[HW] = (double)out[2 * k] * scale * I;
    o[2 * (size_t)HW] = (double)out[2 * k + 1] * scale * I;
    o[3 * (size_t)HW] = runs == 2 ? 0.5 * (m[3 * (size_t)HW] + m[rb + 3 * (size_t)HW]) : m[3 * (size_t)HW];
  }
}

// (1 - beta) is passed from the host, formed in FP64: 0.999 is not an FP32
// number and 1 - fl(0.999) would be off by 1.3e-5 relative.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float omb1, float omb2,
                       float eps, float c1, float c2) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const float gk = g[k];
    const float mk = b1 * m[k] + omb1 * gk;
    const float vk = b2 * v[k] + omb2 * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  }
}

// FP32 master weights [cout][9][cin_true] -> BF16 GEMM weights
//   w[co][kk * cin + c] (zero for c >= cin_true and for k >= 9 cin, up to kp)
//   wd[ci][kk * cout + co] = w[co][8 - kk][ci] (zero-padded to kpd), if wd != null
__global__ void k_pack(const float* __restrict__ wf, int cout, int cin, int cin_true, int kp, int kpd,
                       uint16_t* __restrict__ w, uint16_t* __restrict__ wd) {
  const size_t n = (size_t)cout * kp;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const int co = (int)(k / kp), kx = (int)(k % kp);
    const int kk = kx / cin, c = kx % cin;
    const float v = (kk < 9 && c < cin_true) ? wf[((size_t)co * 9 + kk) * cin_true + c] : 0.f;
    w[k] = f2bf(v);
  }
  if (!wd) return;
  const size_t nd = (size_t)cin_true * kpd;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nd; k += (size_t)gridDim.x * blockDim.x) {
    const int ci = (int)(k / kpd), kx = (int)(k % kpd);
    const int kk = kx / cout, co = kx % cout;
    const float v = kk < 9 ? wf[((size_t)co * 9 + (8 - kk)) * cin_true + ci] : 0.f;
    wd[k] = f2bf(v);
  }
}

__global__ void k_zero32(uint32_t* __restrict__ p, size_t n) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = 0u;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned grid_for(size_t n, size_t cap = 65536) {
  size_t g = (n + 255) / 256;
  if (g > cap) g = cap;
  return (unsigned)(g ? g : 1);
}

void conv3(const ConvArgs& a, int mode, hipStream_t s) {
  const size_t P = (size_t)a.B * a.H * a.W;
  const unsigned ngroups = (unsigned)((a.nout + 63) / 64);
  if (P >= CONV_TILED_MIN_PIXELS) {
    // widest channel group (16 NT, NT <= 4) that divides cout
    const int t16 = a.nout / 16;
    const int nt = t16 % 4 == 0 ? 4 : t16 % 3 == 0 ? 3 : t16 % 2 == 0 ? 2 : 1;
    const dim3 grid((unsigned)(a.B * ((a.H + 15) / 16) * ((a.W + 15) / 16) * (t16 / nt)));
    switch (mode * 4 + nt - 1) {
#define KP_HALO_CASE(M, N) \
  case M * 4 + N - 1: hipLaunchKernelGGL((k_conv3_halo<M, N>), grid, dim3(256), 0, s, a); break;
      KP_HALO_CASE(CONV_RELU, 1) KP_HALO_CASE(CONV_RELU, 2) KP_HALO_CASE(CONV_RELU, 3) KP_HALO_CASE(CONV_RELU, 4)
      KP_HALO_CASE(CONV_LINEAR, 1) KP_HALO_CASE(CONV_LINEAR, 2) KP_HALO_CASE(CONV_LINEAR, 3)
      KP_HALO_CASE(CONV_LINEAR, 4) KP_HALO_CASE(CONV_MASK, 1) KP_HALO_CASE(CONV_MASK, 2)
      KP_HALO_CASE(CONV_MASK, 3) KP_HALO_CASE(CONV_MASK, 4)
#undef KP_HALO_CASE
    }
    return;
  }
  const size_t waves = ((P + 31) / 32) * ngroups;
  const dim3 grid((unsigned)((waves + 3) / 4));
  if (mode == CONV_RELU) hipLaunchKernelGGL(k_conv3<CONV_RELU>, grid, dim3(256), 0, s, a);
  else if (mode == CONV_LINEAR) hipLaunchKernelGGL(k_conv3<CONV_LINEAR>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_conv3<CONV_MASK>, grid, dim3(256), 0, s, a);
}

WgradPlan wgrad_plan(int cout, int cin, size_t P) {
  WgradPlan w;
  w.ktiles = (9 * cin + 63) / 64;
  w.mtiles = (cout + 63) / 64;
  const size_t tiles = (size_t)w.mtiles * w.ktiles;
  // about WG_TARGET workgroups in all, each chunk at least WG_MIN_CHUNK
  // pixels and a whole number of slabs: few partial tiles to add atomically
  size_t nch = (WG_TARGET + tiles - 1) / tiles;
  const size_t most = (P + WG_MIN_CHUNK - 1) / WG_MIN_CHUNK;
  if (nch > most) nch = most;
  if (nch < 1) nch = 1;
  size_t chunk = (P + nch - 1) / nch;
  chunk = (chunk + WG_SLAB - 1) / WG_SLAB * WG_SLAB;
  w.chunk = (int)chunk;
  w.nch = (int)((P + chunk - 1) / chunk);
  return w;
}

WgradPlan wgrad_halo_plan(int cout, int cin, int B, int H, int W) {
  WgradPlan w;
  w.mtiles = (cout + 63) / 64;
  w.ktiles = (cin + 63) / 64;  // input-channel tiles
  const long ntile = (long)B * ((H + WH_TH - 1) / WH_TH) * ((W + WH_TW - 1) / WH_TW);
  const long tiles = (long)w.mtiles * w.ktiles;
  long nch = (WH_TARGET + tiles / 2) / tiles;
  if (nch > ntile) nch = ntile;
  if (nch < 1) nch = 1;
  const long chunk = (ntile + nch - 1) / nch;
  w.chunk = (int)chunk;
  w.nch = (int)((ntile + chunk - 1) / chunk);
  return w;
}

size_t wgrad_part_floats(int cout, int cin) {
  if (cin < WH_MIN_CIN) return 0;
  // nch * tiles <= max(WH_TARGET + tiles / 2, tiles) for every image size
  const size_t tiles = (size_t)((cout + 63) / 64) * ((cin + 63) / 64);
  return std::max((size_t)WH_TARGET + tiles / 2, tiles) * (64 * 576);
}

void wgrad(WgradArgs a, hipStream_t s) {
  if (a.cin >= WH_MIN_CIN) {
    const WgradPlan w = wgrad_halo_plan(a.cout, a.cin, a.B, a.H, a.W);
    a.ktiles = w.ktiles;
    a.mtiles = w.mtiles;
    a.nch = w.nch;
    a.chunk = w.chunk;
    hipLaunchKernelGGL(k_wgrad_halo, dim3((unsigned)(w.mtiles * w.ktiles * w.nch)), dim3(512), 0, s, a);
    const int tiles = w.mtiles * w.ktiles;
    hipLaunchKernelGGL(k_wgrad_sum, dim3((unsigned)((size_t)tiles * 64 * 576 / 16)), dim3(256), 0, s, a.part, tiles,
                       w.nch, w.ktiles, a.cout, a.cin_true, a.gw);
    return;
  }
  const WgradPlan w = wgrad_plan(a.cout, a.cin, (size_t)a.B * a.H * a.W);
  a.ktiles = w.ktiles;
  a.mtiles = w.mtiles;
  a.nch = w.nch;
  a.chunk = w.chunk;
  hipLaunchKernelGGL(k_wgrad, dim3((unsigned)(w.mtiles * w.ktiles * w.nch)), dim3(256), 0, s, a);
}

void pool(const uint16_t* x, int xs, uint16_t* y, int ys, int B, int H, int W, int C, hipStream_t s) {
  hipLaunchKernelGGL(k_pool, dim3(grid_for((size_t)B * H * W * C / 32)), dim3(256), 0, s, x, xs, y, ys, B, H, W, C);
}
void up(const uint16_t* x, int xs, uint16_t* y, int ys, int B, int H, int W, int C, hipStream_t s) {
  hipLaunchKernelGGL(k_up, dim3(grid_for((size_t)B * H * W * C / 8)), dim3(256), 0, s, x, xs, y, ys, B, H, W, C);
}
void up_bwd(const uint16_t* gy, int gys, uint16_t* gx, int gxs, const uint16_t* mask, int ms, int B, int H, int W,
            int C, hipStream_t s) {
  hipLaunchKernelGGL(k_up_bwd, dim3(grid_for((size_t)B * H * W * C / 32)), dim3(256), 0, s, gy, gys, gx, gxs, mask,
                     ms, B, H, W, C);
}
void pool_bwd_add(const uint16_t* a, int as, const uint16_t* g, int gs, const uint16_t* mask, int ms, uint16_t* dst,
                  int ds, int B, int H, int W, int C, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_bwd_add, dim3(grid_for((size_t)B * H * W * C / 8)), dim3(256), 0, s, a, as, g, gs, mask,
                     ms, dst, ds, B, H, W, C);
}
void sums(const double* maps, int B, int HW, int runs, double* sum, hipStream_t s) {
  hipLaunchKernelGGL(k_sums, dim3(grid_for(HW, 32), B), dim3(256), 0, s, maps, HW, runs, sum);
}
void prep(const double* maps, const double* target, const double* sum, const int32_t* aug, int code_all, int B,
          int H, int W, int runs, uint16_t* x, float* xq, float* ihat, float* tgt, hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3(grid_for((size_t)B * H * W)), dim3(256), 0, s, maps, target, sum, aug, code_all,
                     B, H, W, runs, x, xq, ihat, tgt);
}
void head(const uint16_t* d, int C, const float* hw, const float* hb, const float* xq, float* out, size_t P,
          hipStream_t s) {
  hipLaunchKernelGGL(k_head, dim3(grid_for(P * 8)), dim3(256), 0, s, d, C, hw, hb, xq, out, P);
}
void loss(const float* out, const float* tgt, const float* ihat, const double* sum, int B, int HW, float* go,
          double* l, hipStream_t s) {
  // few blocks per image: the per-block results meet in one FP64 atomic
  hipLaunchKernelGGL(k_loss, dim3(grid_for(HW, 32), B), dim3(256), 0, s, out, tgt, ihat, sum, B, HW, go, l);
}
void head_bwd(const float* go, const uint16_t* d, int C, const float* hw, float* ghw, float* ghb, uint16_t* gd,
              size_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_head_bwd, dim3((unsigned)((P + HB_CHUNK - 1) / HB_CHUNK)), dim3(256), 0, s, go, d, C, hw, ghw,
                     ghb, gd, P);
}
void tta_acc(const float* out, int B, int H, int W, int code, bool first, float* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_tta_acc, dim3(grid_for((size_t)B * H * W)), dim3(256), 0, s, out, B, H, W, code, (int)first,
                     acc);
}
void output(const double* maps, const float* out, int B, int HW, int runs, double scale, double* dst,
            hipStream_t s) {
  hipLaunchKernelGGL(k_output, dim3(grid_for((size_t)B * HW)), dim3(256), 0, s, maps, out, B, HW, runs, scale, dst);
}
void adam(float* p, const float* g, float* m, float* v, size_t n, float lr, int t, hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, t)), c2 = (float)(1.0 - std::pow(b2, t));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, (float)b1, (float)b2,
                     (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2);
}
void pack(const float* wf, int cout, int cin, int cin_true, int kp, int kpd, uint16_t* w, uint16_t* wd,
          hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(grid_for((size_t)cout * kp)), dim3(256), 0, s, wf, cout, cin, cin_true, kp, kpd, w,
                     wd);
}
void zero(void* p, size_t bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_zero32, dim3(grid_for(bytes / 4)), dim3(256), 0, s, (uint32_t*)p, bytes / 4);
}

}  // namespace dn
}  // namespace kp
