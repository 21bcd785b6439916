// Learned RFI flagger kernels for gfx950: a four-layer convolutional network
// over per-baseline dynamic spectra, with its training step.
//
// Layers (stride 1, zero 'same' padding, cross-correlation):
//   L1 3x3 1->32 ReLU, L2 5x5 32->32 ReLU, L3 5x5 dilation 2 32->32 ReLU,
//   L4 1x1 32->1 logit.
// Activations are float32 [image][channel][row][col]; images are one
// baseline's (time x channel) plane.  Weights arrive as W[out][in][ky][kx]
// and are repacked per call to [in][ky][kx][out], so the out-channel
// weights of one tap are contiguous and uniform across a workgroup (they are
// read through scalar loads and broadcast to every lane).
//
// Backward data of a stride-1 'same' layer is the same correlation with the
// kernel flipped and in/out swapped, so it reuses the forward kernel.
// Weight gradients accumulate per workgroup in registers over pixel tiles
// and are reduced across workgroups in a fixed order (no float atomics:
// every result is deterministic).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "qc_kernels.h"

namespace qc {

namespace {

constexpr int CT_H = 8;   // output tile rows
constexpr int CT_W = 32;  // output tile columns; 256 threads, one pixel each
constexpr int CNT = CT_H * CT_W;

typedef float mf32x16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int64_t img_off(int64_t n, int c, int C, int H, int W) {
  return ((n * C + c) * (int64_t)H) * W;
}

// The output layer fused into the last convolution's epilogue: logits
// and/or the flag mask in the [time][baseline][chan] layout.
struct HeadArgs {
  const float* w4;  // 32 weights, then the bias
  float* logits;    // [n_img][H][W] or null
  float thr;
  int64_t img0, n_base;
  uint8_t* mask;    // or null
};

// Repack W[o][i][ky][kx] -> P[i][ky][kx][o]; with flip, the backward-data
// kernel P[o][K-1-ky][K-1-kx][i] (inputs and outputs exchanged).
__global__ void cnn_pack_kernel(const float* __restrict__ w, int CI, int CO, int K, int flip,
                                float* __restrict__ p) {
  const int n = CI * CO * K * K;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int kx = e % K, ky = (e / K) % K, i = (e / (K * K)) % CI, o = e / (K * K * CI);
  const float v = w[e];
  if (!flip)
    p[((i * K + ky) * K + kx) * CO + o] = v;
  else
    p[((o * K + (K - 1 - ky)) * K + (K - 1 - kx)) * CI + i] = v;
}

// MODE 0: out = relu(acc + b); MODE 1: out = acc * (gate > 0) (backward data
// through the ReLU of the layer below); MODE 2: out = acc + b.
template <int CI, int CO, int K, int D, int MODE>
__global__ void __launch_bounds__(CNT)
cnn_conv_kernel(const float* __restrict__ in, const float* __restrict__ wp, const float* __restrict__ bias,
                const float* __restrict__ gate, int H, int W, int tiles_x, int tiles_per_img,
                float* __restrict__ out) {
  constexpr int R = D * (K - 1) / 2;
  constexpr int LH = CT_H + 2 * R, LW = CT_W + 2 * R;
  constexpr int CIC = CI < 8 ? CI : 8;  // input channels staged per pass
  constexpr int CS = LH * LW + 1;       // odd channel stride
  __shared__ float tile[CIC * CS];
  const int64_t n = blockIdx.x / tiles_per_img;
  const int tt = blockIdx.x % tiles_per_img;
  const int y0 = (tt / tiles_x) * CT_H, x0 = (tt % tiles_x) * CT_W;
  const int t = threadIdx.x, ty = t / CT_W, tx = t % CT_W;
  float acc[CO];
#pragma unroll
  for (int o = 0; o < CO; ++o) acc[o] = 0.f;
  for (int c0 = 0; c0 < CI; c0 += CIC) {
    for (int e = t; e < CIC * LH * LW; e += CNT) {
      const int c = e / (LH * LW), r = (e / LW) % LH, q = e % LW;
      const int y = y0 + r - R, x = x0 + q - R;
      float v = 0.f;
      if (y >= 0 && y < H && x >= 0 && x < W) v = in[img_off(n, c0 + c, CI, H, W) + (int64_t)y * W + x];
      tile[c * CS + r * LW + q] = v;
    }
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < CIC; ++c) {
#pragma unroll
      for (int ky = 0; ky < K; ++ky) {
#pragma unroll
        for (int kx = 0; kx < K; ++kx) {
          const float v = tile[c * CS + (ty + ky * D) * LW + tx + kx * D];
          const float* wk = wp + (((c0 + c) * K + ky) * K + kx) * CO;
#pragma unroll
          for (int o = 0; o < CO; ++o) acc[o] = fmaf(wk[o], v, acc[o]);
        }
      }
    }
    __syncthreads();
  }
  const int y = y0 + ty, x = x0 + tx;
  if (y < H && x < W) {
#pragma unroll
    for (int o = 0; o < CO; ++o) {
      const int64_t oi = img_off(n, o, CO, H, W) + (int64_t)y * W + x;
      float v = acc[o];
      if constexpr (MODE == 0) v = fmaxf(v + bias[o], 0.f);
      if constexpr (MODE == 1) v = gate[oi] > 0.f ? v : 0.f;
      if constexpr (MODE == 2) v = v + bias[o];
      out[oi] = v;
    }
  }
}

// Float32 5x5 32 -> 32 convolution on the matrix cores, an implicit GEMM:
// out[co][p] = sum over (tap, ci) of P[ci][tap][co] in[ci][p + tap offset],
// one v_mfma_f32_32x32x2_f32 per tap and pair of input channels.  P is the
// [in][tap][out] packing cnn_pack writes for both directions.  A tile is
// 8 x 32 pixels (wave w: row w), reduced in two halves of 16 input channels
// h; within a half, product (q, j) pairs channels 16h + 4q + j and
// 16h + 8 + 4q + j (lane l: output channel = pixel slot l % 32, the pair's
// member l / 32), so each lane's operands of four products are 16
// contiguous bytes in LDS: the weights [tap][h][q][lane][4] (copied once
// per workgroup, 100 KB) and the staged half-tile channel-fastest,
// [pixel][16 channels] with an 80-byte pixel stride (conflict-free 16-byte
// reads).  The next half-tile's values travel in registers while this one
// is reduced; four accumulators take the four j.  MODE as for
// cnn_conv_kernel, and 3: forward with ReLU followed by the output layer,
// writing logits and/or flags instead of the activations.
constexpr int CM_NTH = 512, CM_HC = 16, CM_PS = 20;

constexpr int cm_pl(int D) { return (CT_H + 4 * D) * (CT_W + 4 * D); }
constexpr size_t cm_lds(int D) { return sizeof(float) * (25 * 16 * 64 + cm_pl(D) * CM_PS); }

template <int D, int MODE>
__global__ void __launch_bounds__(CM_NTH)
cnn_conv32_mfma_kernel(const float* __restrict__ in, const float* __restrict__ wp, const float* __restrict__ bias,
                       const float* __restrict__ gate, int H, int W, int tiles_x, int tiles_per_img,
                       int64_t n_tiles, float* __restrict__ out, HeadArgs hd) {
  constexpr int C = 32, NT = 25, R = 2 * D;
  constexpr int LH = CT_H + 2 * R, LW = CT_W + 2 * R, PL = LH * LW;
  constexpr int IH = (CM_HC * PL + CM_NTH - 1) / CM_NTH;
  static_assert(cm_lds(D) <= 160 * 1024, "LDS");
  static_assert(CM_NTH / 64 == CT_H && CT_W == 32, "one tile row per wave, one MFMA column block");
  extern __shared__ float4 sm4[];
  float4* sw = sm4;                                              // [tap][h][q][lane]
  float* st = reinterpret_cast<float*>(sm4 + NT * 2 * 2 * 64);  // [pixel][CM_PS]
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int px = lane & 31, kh = lane >> 5;
  for (int e = t; e < NT * 2 * 2 * 64; e += CM_NTH) {
    const int l = e & 63, q = (e >> 6) & 1, h = (e >> 7) & 1, tap = e >> 8;
    const int c0 = 16 * h + 8 * (l >> 5) + 4 * q, co = l & 31;
    sw[e] = make_float4(wp[((c0 + 0) * NT + tap) * C + co], wp[((c0 + 1) * NT + tap) * C + co],
                        wp[((c0 + 2) * NT + tap) * C + co], wp[((c0 + 3) * NT + tap) * C + co]);
  }
  float bco[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) bco[r] = MODE != 1 ? bias[8 * (r >> 2) + 4 * kh + (r & 3)] : 0.f;
  const int HW = H * W;             // C * H * W < 2^31: 32-bit offsets in an image
  float pre[IH];
  // half h of tile tl: input channels 16 h .. 16 h + 15 with the halo,
  // element f = [channel][row][col] (coalesced global reads)
  auto load_half = [&](int64_t tl, int h) {
    const int64_t n = tl / tiles_per_img;
    const int tt = (int)(tl % tiles_per_img);
    const int y0 = (tt / tiles_x) * CT_H, x0 = (tt % tiles_x) * CT_W;
    const float* ip = in + img_off(n, CM_HC * h, C, H, W);
    int tv = t;
    asm volatile("" : "+v"(tv));    // offsets are recomputed per stage, not held live
#pragma unroll
    for (int i = 0; i < IH; ++i) {
      const int f = tv + CM_NTH * i;
      const int c = f / PL, r = (f / LW) % LH, q = f % LW;
      const int y = y0 + r - R, x = x0 + q - R;
      const bool ok = (IH * CM_NTH == CM_HC * PL || f < CM_HC * PL) && y >= 0 && y < H && x >= 0 && x < W;
      const float v = ip[ok ? c * HW + y * W + x : 0];
      pre[i] = ok ? v : 0.f;
    }
  };
  if ((int64_t)blockIdx.x < n_tiles) load_half(blockIdx.x, 0);
  for (int64_t tl = blockIdx.x; tl < n_tiles; tl += gridDim.x) {
    mf32x16_t acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      __syncthreads();  // the previous stage's reads are done (and the weights stored)
      {
        int tv = t;
        asm volatile("" : "+v"(tv));
#pragma unroll
        for (int i = 0; i < IH; ++i) {
          const int f = tv + CM_NTH * i;
          if (IH * CM_NTH == CM_HC * PL || f < CM_HC * PL) st[(f % PL) * CM_PS + f / PL] = pre[i];
        }
      }
      __syncthreads();
      if (h == 0)
        load_half(tl, 1);
      else if (tl + gridDim.x < n_tiles)
        load_half(tl + gridDim.x, 0);
      const float4* ab = sw + h * 2 * 64 + lane;
      const float* bb = st + (wave * LW + px) * CM_PS + 8 * kh;
      // operands of tap + 1 are read while tap's products run
      float4 a0 = ab[0], a1 = ab[64];
      float4 b0 = *reinterpret_cast<const float4*>(bb), b1 = *reinterpret_cast<const float4*>(bb + 4);
#pragma unroll 5
      for (int tap = 0; tap < NT; ++tap) {
        const int tn = tap + 1 < NT ? tap + 1 : tap;
        const float4* a = ab + tn * 4 * 64;
        const float* b = bb + ((tn / 5) * D * LW + (tn % 5) * D) * CM_PS;
        const float4 an0 = a[0], an1 = a[64];
        const float4 bn0 = *reinterpret_cast<const float4*>(b), bn1 = *reinterpret_cast<const float4*>(b + 4);
        __builtin_amdgcn_sched_barrier(0);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.x, b0.x, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.y, b0.y, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.z, b0.z, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.w, b0.w, acc[3], 0, 0, 0);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.x, b1.x, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.y, b1.y, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.z, b1.z, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.w, b1.w, acc[3], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        a0 = an0;
        a1 = an1;
        b0 = bn0;
        b1 = bn1;
      }
    }
    const int64_t n = tl / tiles_per_img;
    const int tt = (int)(tl % tiles_per_img);
    const int y = (tt / tiles_x) * CT_H + wave, x = (tt % tiles_x) * CT_W + px;
    if constexpr (MODE == 3) {
      // the output layer on this pixel's 32 activations: the partner lane
      // (l ^ 32) passes its 16 channels over, lane l < 32 sums all 32 in
      // channel order from the bias (as the separate output-layer kernel)
      float v[16], o[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = fmaxf((acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]) + bco[r], 0.f);
#pragma unroll
      for (int r = 0; r < 16; ++r) o[r] = __shfl_xor(v[r], 32);
      if (kh == 0 && y < H && x < W) {
        float z = hd.w4[32];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
#pragma unroll
          for (int i = 0; i < 4; ++i) z = fmaf(hd.w4[8 * g + i], v[4 * g + i], z);
#pragma unroll
          for (int i = 0; i < 4; ++i) z = fmaf(hd.w4[8 * g + 4 + i], o[4 * g + i], z);
        }
        if (hd.logits) hd.logits[(n * H + y) * (int64_t)W + x] = z;
        if (hd.mask) hd.mask[((int64_t)y * hd.n_base + (hd.img0 + n)) * W + x] = z > hd.thr ? 1 : 0;
      }
    } else if (y < H && x < W) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int o = 8 * (r >> 2) + 4 * kh + (r & 3);   // accumulator row: output channel
        const int64_t oi = img_off(n, o, C, H, W) + (int64_t)y * W + x;
        float v = (acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]);
        if constexpr (MODE == 0) v = fmaxf(v + bco[r], 0.f);
        if constexpr (MODE == 1) v = gate[oi] > 0.f ? v : 0.f;
        if constexpr (MODE == 2) v = v + bco[r];
        out[oi] = v;
      }
    }
  }
}

// Weight gradient of a 32->32 layer: dW[o][i][ky][kx] = sum over pixels of
// g[o](p) * a[i](p + tap offset), db[o] = sum g[o](p).  Input channels are
// staged 8 at a time; a lane owns 4 outputs x 1 staged input, a wave owns a
// group of taps (so tap offsets are uniform).  Workgroups stride over pixel
// tiles; each writes its partial sums to part[block][...].
template <int K, int D>
__global__ void __launch_bounds__(256)
cnn_wgrad32_kernel(const float* __restrict__ a, const float* __restrict__ g, int H, int W, int tiles_x,
                   int tiles_per_img, int64_t n_tiles, float* __restrict__ part) {
  constexpr int C = 32;
  constexpr int R = D * (K - 1) / 2;
  constexpr int LH = CT_H + 2 * R, LW = CT_W + 2 * R;
  constexpr int AS = LH * LW + 1;   // odd strides: the rows a wave reads at one
  constexpr int GS = CNT + 1;       // pixel fall in distinct banks
  constexpr int NT = K * K;
  constexpr int TG = (NT + 3) / 4;  // taps per wave
  constexpr int CIC = 8;
  extern __shared__ float sm[];
  float* sg = sm;                   // [32][GS]
  float* sa = sm + C * GS;          // [CIC][AS]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int ib = lane & 7, ob = lane >> 3;
  const int tap0 = wave * TG;
  float* out = part + (int64_t)blockIdx.x * (C * C * NT + C);
  for (int c0 = 0; c0 < C; c0 += CIC) {
    float acc[4][TG];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < TG; ++q) acc[j][q] = 0.f;
    for (int64_t tl = blockIdx.x; tl < n_tiles; tl += gridDim.x) {
      const int64_t n = tl / tiles_per_img;
      const int tt = (int)(tl % tiles_per_img);
      const int y0 = (tt / tiles_x) * CT_H, x0 = (tt % tiles_x) * CT_W;
      for (int e = t; e < C * CNT; e += 256) {
        const int o = e / CNT, p = e % CNT;
        const int y = y0 + p / CT_W, x = x0 + p % CT_W;
        sg[o * GS + p] = (y < H && x < W) ? g[img_off(n, o, C, H, W) + (int64_t)y * W + x] : 0.f;
      }
      for (int e = t; e < CIC * LH * LW; e += 256) {
        const int c = e / (LH * LW), r = (e / LW) % LH, q = e % LW;
        const int y = y0 + r - R, x = x0 + q - R;
        float v = 0.f;
        if (y >= 0 && y < H && x >= 0 && x < W) v = a[img_off(n, c0 + c, C, H, W) + (int64_t)y * W + x];
        sa[c * AS + r * LW + q] = v;
      }
      __syncthreads();
#pragma unroll 1
      for (int p = 0; p < CNT; ++p) {
        const int py = p / CT_W, px = p % CT_W;
        float gv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) gv[j] = sg[(4 * ob + j) * GS + p];
#pragma unroll
        for (int q = 0; q < TG; ++q) {
          const int tap = tap0 + q;
          if (tap < NT) {
            const int ky = tap / K, kx = tap % K;
            const float av = sa[ib * AS + (py + ky * D) * LW + px + kx * D];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j][q] = fmaf(gv[j], av, acc[j][q]);
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < TG; ++q) {
        const int tap = tap0 + q;
        if (tap < NT) out[((4 * ob + j) * C + (c0 + ib)) * NT + tap] = acc[j][q];
      }
  }
  // bias: one lane per output channel sums its gradient over the same tiles
  if (t < C) {
    float sb = 0.f;
    for (int64_t tl = blockIdx.x; tl < n_tiles; tl += gridDim.x) {
      const int64_t n = tl / tiles_per_img;
      const int tt = (int)(tl % tiles_per_img);
      const int y0 = (tt / tiles_x) * CT_H, x0 = (tt % tiles_x) * CT_W;
      for (int p = 0; p < CNT; ++p) {
        const int y = y0 + p / CT_W, x = x0 + p % CT_W;
        if (y < H && x < W) sb += g[img_off(n, t, C, H, W) + (int64_t)y * W + x];
      }
    }
    out[C * C * NT + t] = sb;
  }
}

// One staged pixel tile's products for a wave's NQ taps: rows of 32 pixels,
// each two pixels per step (lanes 32..63 the odd one), every tap's operand at
// the tap's offset from the same pixel.  g points at channel cl's gradient
// row plus the lane's pixel slot, a at channel cl's input tile likewise.
template <int NQ, int TG, int LW>
__device__ __forceinline__ void wgrad_tile_products(const float* __restrict__ g, const float* __restrict__ a,
                                                    const int (&toff)[TG], mf32x16_t (&acc)[TG]) {
  // operands of step px + 2 are read before step px's products are issued
#pragma unroll 1
  for (int py = 0; py < CT_H; ++py) {
    const float* gr = g + py * CT_W;
    const float* ar[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) ar[q] = a + py * LW + toff[q];
    float gv = gr[0], av[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) av[q] = ar[q][0];
#pragma unroll
    for (int px = 0; px < CT_W; px += 2) {
      float gn = 0.f, an[NQ];
      if (px + 2 < CT_W) {
        gn = gr[px + 2];
#pragma unroll
        for (int q = 0; q < NQ; ++q) an[q] = ar[q][px + 2];
      }
      __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the products
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(gv, av[q], acc[q], 0, 0, 0);
      gv = gn;
#pragma unroll
      for (int q = 0; q < NQ; ++q) av[q] = an[q];
    }
  }
}

// The same weight gradient on the matrix cores: per tap t, dW_t = G A_t^T
// with G = g [32 outputs x pixels] and A_t = a shifted by the tap's offset
// [32 inputs x pixels], a 32 x 32 product reduced over pixels two at a time
// by v_mfma_f32_32x32x2_f32 (lane l: channel l % 32, pixel slot l / 32 of
// both operands).  All 32 input channels of a pixel tile are staged at once,
// the next tile's values travelling in registers while this one is reduced.
// Wave w owns taps w, w + 8, w + 16, w + 24, so that the two waves sharing a
// SIMD hold 6 or 7 of the 25 taps.  The bias gradient is summed from the
// staged tile, 16 lanes per output channel.  Workgroups stride over pixel
// tiles and write their partial sums to part[block][...] in the layout of
// the vector-ALU kernel.
template <int K, int D>
__global__ void __launch_bounds__(512)
cnn_wgrad32_mfma_kernel(const float* __restrict__ a, const float* __restrict__ g, int H, int W,
                        int tiles_x, int tiles_per_img, int64_t n_tiles, float* __restrict__ part) {
  constexpr int C = 32, NTH = 512, NW = NTH / 64;
  constexpr int R = D * (K - 1) / 2;
  constexpr int LH = CT_H + 2 * R, LW = CT_W + 2 * R;
  constexpr int AS = LH * LW + 1;   // odd channel strides: the 32 channels a
  constexpr int GS = CNT + 1;       // wave reads at one pixel hit distinct banks
  constexpr int NT = K * K;
  constexpr int TG = (NT + NW - 1) / NW;
  constexpr int IG = C * CNT / NTH, IA = C * LH * LW / NTH, ITER = IG + IA;
  static_assert(IG * NTH == C * CNT && IA * NTH == C * LH * LW && NTH % CNT == 0, "whole staging rounds");
  static_assert(CNT % 2 == 0 && CNT == 16 * 16, "pixel pairs; 16 lanes x 16 pixels per bias sum");
  extern __shared__ float sm[];
  float* sg = sm;                   // [32][GS]
  float* sa = sm + C * GS;          // [32][AS]
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int cl = lane & 31, kh = lane >> 5;
  mf32x16_t acc[TG];
#pragma unroll
  for (int q = 0; q < TG; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.f;
  float sb = 0.f;                   // bias partial: channel t / 16, pixels t % 16 + 16 j
  int toff[TG];                     // LDS offsets of the wave's taps (uniform)
#pragma unroll
  for (int q = 0; q < TG; ++q) {
    const int tap = wave + NW * q;
    toff[q] = tap < NT ? (tap / K) * D * LW + (tap % K) * D : 0;
  }
  const int nq = wave + NW * (TG - 1) < NT ? TG : TG - 1;
  static_assert(NW * (TG - 1) < NT, "every wave holds at least TG - 1 taps");
  float pre[ITER];
  const int HW = H * W;             // C * H * W < 2^31: 32-bit offsets in an image
  // Staging: the gradient tile as 16 rounds of 2 channels (thread t: channel
  // t / 256 + 2 i, pixel t % 256), the input tile with halo as IA rounds over
  // [channel][row][col].  Padding reads a valid element and discards it, so
  // the loads are straight-line code.
  auto load_tile = [&](int64_t tl) {
    const int64_t n = tl / tiles_per_img;
    const int tt = (int)(tl % tiles_per_img);
    const int y0 = (tt / tiles_x) * CT_H, x0 = (tt % tiles_x) * CT_W;
    const float* gi = g + img_off(n, 0, C, H, W);
    const float* ai = a + img_off(n, 0, C, H, W);
    int tv = t, hw = HW;
    asm volatile("" : "+v"(tv), "+s"(hw));   // offsets are recomputed per tile, not held live
    {
      const int p = tv % CNT, y = y0 + p / CT_W, x = x0 + p % CT_W;
      const bool in = y < H && x < W;
      int o = in ? (tv / CNT) * hw + y * W + x : 0;
      const int step = in ? (NTH / CNT) * hw : 0;
#pragma unroll
      for (int i = 0; i < IG; ++i, o += step) {
        const float v = gi[o];
        pre[i] = in ? v : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int f = tv + NTH * i;
      const int c = f / (LH * LW), r = (f / LW) % LH, q = f % LW;
      const int y = y0 + r - R, x = x0 + q - R;
      const bool in = y >= 0 && y < H && x >= 0 && x < W;
      const float v = ai[in ? c * HW + y * W + x : 0];
      pre[IG + i] = in ? v : 0.f;
    }
  };
  if (blockIdx.x < n_tiles) load_tile(blockIdx.x);
  for (int64_t tl = blockIdx.x; tl < n_tiles; tl += gridDim.x) {
    __syncthreads();  // the previous tile's reads are done
    int tv = t;
    asm volatile("" : "+v"(tv));
#pragma unroll
    for (int i = 0; i < IG; ++i) sg[((NTH / CNT) * i + tv / CNT) * GS + tv % CNT] = pre[i];
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int f = tv + NTH * i;
      sa[f + f / (LH * LW)] = pre[IG + i];   // channel stride LH * LW + 1
    }
    __syncthreads();
    if (tl + gridDim.x < n_tiles) load_tile(tl + gridDim.x);
#pragma unroll
    for (int j = 0; j < 16; ++j) sb += sg[(t >> 4) * GS + (t & 15) + 16 * j];
    if (nq == TG)
      wgrad_tile_products<TG, TG, LW>(sg + cl * GS + kh, sa + cl * AS + kh, toff, acc);
    else
      wgrad_tile_products<TG - 1, TG, LW>(sg + cl * GS + kh, sa + cl * AS + kh, toff, acc);
  }
  float* out = part + (int64_t)blockIdx.x * (C * C * NT + C);
#pragma unroll
  for (int q = 0; q < TG; ++q) {
    const int tap = wave + NW * q;
    if (tap < NT) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int o = 8 * (r >> 2) + 4 * kh + (r & 3);   // accumulator row
        out[(o * C + cl) * NT + tap] = acc[q][r];
      }
    }
  }
#pragma unroll
  for (int m = 8; m >= 1; m >>= 1) sb += __shfl_xor(sb, m, 16);
  if ((t & 15) == 0) out[C * C * NT + (t >> 4)] = sb;
}

// L1's weight gradient (3 x 3, 1 -> 32) on the matrix cores: per pair of
// pixels one v_mfma_f32_32x32x2_f32 forms dW[o][tap] for all 32 outputs
// (rows, A = the output gradient) and the 9 taps (columns, B = the input at
// the tap's offset), with column 9 holding 1 so that the bias gradient is
// the same sum; columns 10..31 are zero.  Wave w takes tile rows 2w, 2w+1;
// the four waves' sums are added in wave order at the end and written to
// part[block][...] in the layout of the vector-ALU kernel.
constexpr int L1M_NT = 256;

__global__ void __launch_bounds__(L1M_NT)
cnn_wgrad_l1_mfma_kernel(const float* __restrict__ a, const float* __restrict__ g, int H, int W, int tiles_x,
                         int tiles_per_img, int64_t n_tiles, float* __restrict__ part) {
  constexpr int C = 32, NTAP = 9, LH = CT_H + 2, LW = CT_W + 2, GS = CNT + 1, NWV = L1M_NT / 64;
  static_assert(CT_H == 2 * NWV, "two tile rows per wave");
  __shared__ float sg[C * GS];
  __shared__ float sa[LH * LW];
  __shared__ float red[NWV][16][64];
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int j = lane & 31, kh = lane >> 5;        // column (tap) and pixel slot
  const int ky = j / 3, kx = j % 3;
  mf32x16_t acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int64_t tl = blockIdx.x; tl < n_tiles; tl += gridDim.x) {
    const int64_t n = tl / tiles_per_img;
    const int tt = (int)(tl % tiles_per_img);
    const int y0 = (tt / tiles_x) * CT_H, x0 = (tt % tiles_x) * CT_W;
    static_assert(L1M_NT == CNT, "thread t stages pixel t of every channel");
    // all 32 channels of this thread's pixel: independent loads, in flight together
    float gv[C];
    {
      const int y = y0 + t / CT_W, x = x0 + t % CT_W;
      const bool in = y < H && x < W;
      const float* gp = g + img_off(n, 0, C, H, W) + (in ? (int64_t)y * W + x : 0);
#pragma unroll
      for (int o = 0; o < C; ++o) {
        const float v = gp[(int64_t)o * H * W];
        gv[o] = in ? v : 0.f;
      }
    }
    __syncthreads();  // the previous tile's reads are done
#pragma unroll
    for (int o = 0; o < C; ++o) sg[o * GS + t] = gv[o];
    for (int e = t; e < LH * LW; e += L1M_NT) {
      const int y = y0 + e / LW - 1, x = x0 + e % LW - 1;
      sa[e] = (y >= 0 && y < H && x >= 0 && x < W) ? a[img_off(n, 0, 1, H, W) + (int64_t)y * W + x] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      const int py = 2 * wave + rr;
#pragma unroll 4
      for (int px = 0; px < CT_W; px += 2) {
        const float av = sg[j * GS + py * CT_W + px + kh];   // A: row = output channel j
        float bv = 0.f;
        if (j < NTAP) bv = sa[(py + ky) * LW + px + kh + kx];
        else if (j == NTAP) bv = 1.f;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) red[wave][r][lane] = acc[r];
  __syncthreads();
  float* out = part + (int64_t)blockIdx.x * (C * NTAP + C);
  for (int e = t; e < C * (NTAP + 1); e += L1M_NT) {
    const int o = e / (NTAP + 1), col = e % (NTAP + 1);
    // accumulator row o lives in register 4 (o / 8) + o % 4 of lanes with kh = (o / 4) % 2
    const int r = 4 * (o >> 3) + (o & 3), ln = col + 32 * ((o >> 2) & 1);
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < NWV; ++w) sum += red[w][r][ln];
    if (col < NTAP) out[o * NTAP + col] = sum;
    else out[C * NTAP + o] = sum;
  }
}

// Weight gradient of a layer with few weights (L1: 1 input channel): one
// lane per weight, pixel tiles staged in LDS.
template <int CI, int CO, int K, int D>
__global__ void __launch_bounds__(256)
cnn_wgrad_small_kernel(const float* __restrict__ a, const float* __restrict__ g, int H, int W, int tiles_x,
                       int tiles_per_img, int64_t n_tiles, float* __restrict__ part) {
  constexpr int R = D * (K - 1) / 2;
  constexpr int LH = CT_H + 2 * R, LW = CT_W + 2 * R;
  constexpr int NW = CO * CI * K * K + CO;
  constexpr int PER = (NW + 255) / 256;
  constexpr int GS = CNT + 1;
  __shared__ float sg[CO * GS];
  __shared__ float sa[CI * LH * LW];
  const int t = threadIdx.x;
  float s[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) s[j] = 0.f;
  for (int64_t tl = blockIdx.x; tl < n_tiles; tl += gridDim.x) {
    const int64_t n = tl / tiles_per_img;
    const int tt = (int)(tl % tiles_per_img);
    const int y0 = (tt / tiles_x) * CT_H, x0 = (tt % tiles_x) * CT_W;
    for (int e = t; e < CO * CNT; e += 256) {
      const int o = e / CNT, p = e % CNT;
      const int y = y0 + p / CT_W, x = x0 + p % CT_W;
      sg[o * GS + p] = (y < H && x < W) ? g[img_off(n, o, CO, H, W) + (int64_t)y * W + x] : 0.f;
    }
    for (int e = t; e < CI * LH * LW; e += 256) {
      const int c = e / (LH * LW), r = (e / LW) % LH, q = e % LW;
      const int y = y0 + r - R, x = x0 + q - R;
      float v = 0.f;
      if (y >= 0 && y < H && x >= 0 && x < W) v = a[img_off(n, c, CI, H, W) + (int64_t)y * W + x];
      sa[e] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int wi = t + j * 256;
      if (wi < NW) {
        float acc = s[j];
        if (wi < CO * CI * K * K) {
          const int kx = wi % K, ky = (wi / K) % K, c = (wi / (K * K)) % CI, o = wi / (K * K * CI);
          for (int p = 0; p < CNT; ++p)
            acc = fmaf(sg[o * GS + p], sa[c * LH * LW + (p / CT_W + ky * D) * LW + p % CT_W + kx * D], acc);
        } else {
          const int o = wi - CO * CI * K * K;
          for (int p = 0; p < CNT; ++p) acc += sg[o * GS + p];
        }
        s[j] = acc;
      }
    }
    __syncthreads();
  }
  float* out = part + (int64_t)blockIdx.x * NW;
#pragma unroll
  for (int j = 0; j < PER; ++j)
    if (t + j * 256 < NW) out[t + j * 256] = s[j];
}

// sum_b part[b][e] for the workgroup's 64 elements e = 64 blockIdx.x + lane,
// in a fixed order: wave w sums parts w, w + SP_WAVES, ... and wave 0 adds
// the waves' sums in wave order.  Valid in wave 0 (e < n); all threads call.
constexpr int SP_WAVES = 16;

__device__ __forceinline__ float sum_parts_block(const float* __restrict__ part, int n_parts, int n) {
  __shared__ float red[SP_WAVES][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (e < n) {
#pragma unroll 8
    for (int b = w; b < n_parts; b += SP_WAVES) s += part[(int64_t)b * n + e];
  }
  red[w][lane] = s;
  __syncthreads();
  float t = 0.f;
  if (w == 0) {
#pragma unroll
    for (int k = 0; k < SP_WAVES; ++k) t += red[k][lane];
  }
  return t;
}

// dst[e] = sum_b part[b][e]
__global__ void __launch_bounds__(64 * SP_WAVES)
cnn_sum_parts_kernel(const float* __restrict__ part, int n_parts, int n, float* __restrict__ dst) {
  const float s = sum_parts_block(part, n_parts, n);
  const int e = blockIdx.x * 64 + (threadIdx.x & 63);
  if (threadIdx.x < 64 && e < n) dst[e] = s;
}

// L4 forward: logit = b + sum_c w[c] a[c]; optionally the flag decision
// written in the [time][baseline][chan] layout of the visibilities.
__global__ void cnn_head_kernel(const float* __restrict__ a, const float* __restrict__ w4, int H, int W,
                                int64_t n_img, float* __restrict__ logits, float thr, int64_t img0,
                                int64_t n_base, uint8_t* __restrict__ mask) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t hw = (int64_t)H * W;
  if (e >= n_img * hw) return;
  const int64_t n = e / hw, p = e % hw;
  float z = w4[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) z = fmaf(w4[c], a[(n * 32 + c) * hw + p], z);
  if (logits) logits[e] = z;
  if (mask) {
    const int64_t tt = p / W, f = p % W;
    mask[(tt * n_base + (img0 + n)) * W + f] = z > thr ? 1 : 0;
  }
}

// grad4[0..31] = sum_b part[b][0..31] (dW4), grad4[32] = sum_b part[b][33]
// (db4), loss = inv_count * sum_b part[b][32] (the mean); one workgroup.
__global__ void __launch_bounds__(64 * SP_WAVES)
cnn_head_finish_kernel(const float* __restrict__ part, int n_parts, float inv_count, float* __restrict__ grad4,
                       float* __restrict__ loss) {
  const float s = sum_parts_block(part, n_parts, 34);
  const int t = threadIdx.x;
  if (t < 32) grad4[t] = s;
  else if (t == 32) *loss = s * inv_count;
  else if (t == 33) grad4[32] = s;
}

__device__ __forceinline__ float softplus_f(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }

// Loss and the start of backpropagation: dz = d(mean BCE)/dlogit, then
// g3[c] = w4[c] dz (a3[c] > 0).  Per-workgroup partials of the loss, of
// dW4[c] = sum dz a3[c] and of db4 = sum dz (34 values).
__global__ void __launch_bounds__(256)
cnn_bce_head_bwd_kernel(const float* __restrict__ logits, const uint8_t* __restrict__ labels,
                        const float* __restrict__ a3, const float* __restrict__ w4, int64_t n_pix_img,
                        int64_t n_total, float pos_weight, float inv_count, float* __restrict__ g3,
                        float* __restrict__ part) {
  __shared__ float red[34][257];
  const int t = threadIdx.x;
  float sv[34];
#pragma unroll
  for (int j = 0; j < 34; ++j) sv[j] = 0.f;
  for (int64_t e = (int64_t)blockIdx.x * 256 + t; e < n_total; e += (int64_t)gridDim.x * 256) {
    const float z = logits[e];
    const float y = labels[e] ? 1.f : 0.f;
    const float sg = 1.f / (1.f + expf(-z));
    sv[32] += pos_weight * y * softplus_f(-z) + (1.f - y) * softplus_f(z);
    const float dz = (-pos_weight * y * (1.f - sg) + (1.f - y) * sg) * inv_count;
    sv[33] += dz;
    const int64_t n = e / n_pix_img, p = e % n_pix_img;
#pragma unroll
    for (int c = 0; c < 32; ++c) {
      const int64_t ai = (n * 32 + c) * n_pix_img + p;
      const float av = a3[ai];
      sv[c] = fmaf(dz, av, sv[c]);
      g3[ai] = av > 0.f ? w4[c] * dz : 0.f;
    }
  }
#pragma unroll
  for (int j = 0; j < 34; ++j) red[j][t] = sv[j];
  __syncthreads();
  if (t < 34) {
    float s = 0.f;
    for (int i = 0; i < 256; ++i) s += red[t][i];
    part[(int64_t)blockIdx.x * 34 + t] = s;
  }
}

// Adam with bias correction (Kingma & Ba), float32 state.
__global__ void cnn_adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                                float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  w[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Network input of one baseline plane: A = |V| (float64, rounded to
// float32), r = (A - med)/(1.4826 MAD), x = sign(r) log1p|r|.
__global__ void cnn_normalize_kernel(const float2* __restrict__ vis, const double* __restrict__ stats,
                                     int64_t n_time, int64_t n_base, int n_chan, int64_t b0, int64_t nb,
                                     float* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = n_time * n_chan;
  if (e >= nb * per) return;
  const int64_t bl = e / per, p = e % per;
  const int64_t b = b0 + bl, tt = p / n_chan, f = p % n_chan;
  const float2 v = vis[(tt * n_base + b) * n_chan + f];
  const double re = (double)v.x, im = (double)v.y;
  const float A = (float)sqrt(re * re + im * im);
  const double med = stats[2 * b], mad = stats[2 * b + 1];
  double scale = 1.4826 * mad;
  if (scale == 0.0) scale = 1.0;
  const double r = ((double)A - med) / scale;
  const double xv = r < 0.0 ? -log1p(-r) : log1p(r);
  x[e] = (float)xv;
}

// ---------------------------------------------------------------------------
// FP16-activation inference path (FP32 accumulation), activations NHWC:
// [image][row][col][32] half.  L2 and L3 run on the matrix cores as an
// implicit GEMM: C[co][pixel] += sum over (tap, ci) of W[co][ci][tap] *
// in[pixel + tap offset][ci], one v_mfma_f32_32x32x16_f16 per 16 input
// channels of a tap.  Operand layout: lane l holds row/column l % 32 and
// reduction slots 8*(l/32)..+7 (A: weights of output channel l%32; B: the
// 8 input channels of pixel l%32, 16 contiguous bytes in NHWC).
// ---------------------------------------------------------------------------
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float16_t __attribute__((ext_vector_type(16)));

// tile rows: 8 waves x mt_u(D) rows, as many as fit the LDS beside the
// packed weights (each weight operand read from LDS feeds MT_U products)
constexpr int mt_u(int D) { return D == 1 ? 4 : 3; }
constexpr int mt_h(int D) { return 8 * mt_u(D); }
constexpr int MT_W = 32;     // tile columns (one MFMA column block)
constexpr int MT_NT = 512;
constexpr int MT_PS = 40;    // LDS pixel stride in halves (80 B: conflict-free 16-byte reads)
constexpr int MT_SLICES = 50;  // 25 taps x 2 halves of the input channels

// Weights of a 5x5 32->32 layer in A-operand order: [slice][lane][8 halves],
// slice = tap*2 + h, lane l: output channel l%32, input channels
// 16h + 8(l/32) .. +7.
__global__ void cnn_pack_mfma_kernel(const float* __restrict__ w, _Float16* __restrict__ p) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // over 50*64*8
  if (e >= MT_SLICES * 64 * 8) return;
  const int j = e % 8, lane = (e / 8) % 64, sl = e / 512;
  const int tap = sl / 2, h = sl % 2;
  const int co = lane % 32, ci = 16 * h + 8 * (lane / 32) + j;
  p[e] = (_Float16)w[(co * 32 + ci) * 25 + tap];
}


// HEAD: instead of storing the activations, apply L4 to them: the partner
// lane (l ^ 32) passes its 16 channels of the pixel over, and lane l < 32
// sums all 32 in channel order from the bias, each activation rounded to
// half first, which is exactly what the separate output-layer kernel
// computes from stored half activations.
template <int D, bool HEAD>
__global__ void __launch_bounds__(MT_NT)
cnn_mfma_conv_kernel(const _Float16* __restrict__ in, const _Float16* __restrict__ wp,
                     const float* __restrict__ bias, int H, int W, int tiles_x, int tiles_per_img,
                     int64_t n_tiles, _Float16* __restrict__ out, HeadArgs hd) {
  constexpr int R = 2 * D;  // D*(5-1)/2
  constexpr int U = mt_u(D), MT_H = mt_h(D);
  constexpr int LH = MT_H + 2 * R, LW = MT_W + 2 * R;
  extern __shared__ uint4 smem[];
  uint4* sw = smem;                                       // [50][64] 16-byte operands
  _Float16* st = reinterpret_cast<_Float16*>(smem + MT_SLICES * 64);  // [LH][LW][MT_PS]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int i = t; i < MT_SLICES * 64; i += MT_NT) sw[i] = reinterpret_cast<const uint4*>(wp)[i];
  const int px = lane & 31, kh = lane >> 5;
  float bco[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) bco[r] = bias[8 * (r >> 2) + 4 * kh + (r & 3)];
  // The input tile with its halo (4 16-byte chunks per pixel) is loaded
  // into registers one tile ahead: the loads of the next tile are in
  // flight while the matrix cores work on this one.
  constexpr int CHUNKS = LH * LW * 4;
  constexpr int NPRE = (CHUNKS + MT_NT - 1) / MT_NT;
  uint4 pre[NPRE];
  auto load_tile = [&](int64_t tl) {
    const int64_t n = tl / tiles_per_img;
    const int tt = (int)(tl % tiles_per_img);
    const int y0 = (tt / tiles_x) * MT_H, x0 = (tt % tiles_x) * MT_W;
#pragma unroll
    for (int i = 0; i < NPRE; ++i) {
      const int e = t + i * MT_NT;
      const int c4 = e & 3, pix = e >> 2;
      const int r = pix / LW, q = pix % LW;
      const int y = y0 + r - R, x = x0 + q - R;
      pre[i] = make_uint4(0u, 0u, 0u, 0u);
      if (e < CHUNKS && y >= 0 && y < H && x >= 0 && x < W)
        pre[i] = reinterpret_cast<const uint4*>(in + (((n * H + y) * (int64_t)W + x) * 32))[c4];
    }
  };
  if ((int64_t)blockIdx.x < n_tiles) load_tile(blockIdx.x);
  for (int64_t tl = blockIdx.x; tl < n_tiles; tl += gridDim.x) {
    const int64_t n = tl / tiles_per_img;
    const int tt = (int)(tl % tiles_per_img);
    const int y0 = (tt / tiles_x) * MT_H, x0 = (tt % tiles_x) * MT_W;
    __syncthreads();  // previous tile's reads done (and weights stored)
#pragma unroll
    for (int i = 0; i < NPRE; ++i) {
      const int e = t + i * MT_NT;
      if (e < CHUNKS) {
        const int c4 = e & 3, pix = e >> 2;
        *reinterpret_cast<uint4*>(st + pix * MT_PS + 8 * c4) = pre[i];
      }
    }
    __syncthreads();
    if (tl + gridDim.x < n_tiles) load_tile(tl + gridDim.x);
    float16_t acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[u][r] = 0.f;
    // operands of slice sl + 1 are read while slice sl's products run
    auto opa = [&](int sl) { return __builtin_bit_cast(half8_t, sw[sl * 64 + lane]); };
    auto opb = [&](int sl, int u) {
      const int tap = sl >> 1, h = sl & 1;
      const int row = U * wave + u + (tap / 5) * D;
      return __builtin_bit_cast(
          half8_t, *reinterpret_cast<const uint4*>(st + (row * LW + px + (tap % 5) * D) * MT_PS + 16 * h + 8 * kh));
    };
    half8_t a = opa(0), b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) b[u] = opb(0, u);
#pragma unroll 10
    for (int sl = 0; sl < MT_SLICES; ++sl) {
      const int sn = sl + 1 < MT_SLICES ? sl + 1 : sl;
      const half8_t an = opa(sn);
      half8_t bn[U];
#pragma unroll
      for (int u = 0; u < U; ++u) bn[u] = opb(sn, u);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u) acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b[u], acc[u], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      a = an;
#pragma unroll
      for (int u = 0; u < U; ++u) b[u] = bn[u];
    }
    // epilogue: bias, ReLU, half; lane holds output channels
    // {8g + 4kh + i} of pixel px for g, i < 4
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int y = y0 + U * wave + u, x = x0 + px;
      if constexpr (HEAD) {
        float v[16], o[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = (float)(_Float16)fmaxf(acc[u][r] + bco[r], 0.f);
#pragma unroll
        for (int r = 0; r < 16; ++r) o[r] = __shfl_xor(v[r], 32);
        if (kh == 0 && y < H && x < W) {
          float z = hd.w4[32];
#pragma unroll
          for (int g = 0; g < 4; ++g) {
#pragma unroll
            for (int i = 0; i < 4; ++i) z = fmaf(hd.w4[8 * g + i], v[4 * g + i], z);
#pragma unroll
            for (int i = 0; i < 4; ++i) z = fmaf(hd.w4[8 * g + 4 + i], o[4 * g + i], z);
          }
          if (hd.logits) hd.logits[(n * H + y) * (int64_t)W + x] = z;
          if (hd.mask) hd.mask[((int64_t)y * hd.n_base + (hd.img0 + n)) * W + x] = z > hd.thr ? 1 : 0;
        }
      } else if (y < H && x < W) {
        _Float16* o = out + ((n * H + y) * (int64_t)W + x) * 32;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
          half4_t v;
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = (_Float16)fmaxf(acc[u][4 * g + i] + bco[4 * g + i], 0.f);
          *reinterpret_cast<half4_t*>(o + 8 * g + 4 * kh) = v;
        }
      }
    }
  }
}

// L1 (3x3, 1 -> 32, ReLU) from the float32 image to NHWC half.
__global__ void __launch_bounds__(256)
cnn_l1_nhwc_kernel(const float* __restrict__ x, const float* __restrict__ w1, const float* __restrict__ b1,
                   int H, int W, int64_t n_pix, _Float16* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_pix) return;
  const int64_t hw = (int64_t)H * W;
  const int64_t n = e / hw;
  const int y = (int)((e % hw) / W), xx = (int)(e % W);
  float v[9];
#pragma unroll
  for (int ky = 0; ky < 3; ++ky)
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) {
      const int yy = y + ky - 1, xc = xx + kx - 1;
      v[ky * 3 + kx] = (yy >= 0 && yy < H && xc >= 0 && xc < W) ? x[n * hw + (int64_t)yy * W + xc] : 0.f;
    }
  typedef _Float16 half8v __attribute__((ext_vector_type(8)));
#pragma unroll
  for (int c8 = 0; c8 < 4; ++c8) {
    half8v o;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int co = 8 * c8 + i;
      float a = b1[co];
#pragma unroll
      for (int k = 0; k < 9; ++k) a = fmaf(w1[co * 9 + k], v[k], a);
      o[i] = (_Float16)fmaxf(a, 0.f);
    }
    *reinterpret_cast<half8v*>(out + e * 32 + 8 * c8) = o;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

hipError_t cnn_pack(const float* w, int CI, int CO, int K, int flip, float* p, hipStream_t s) {
  const int n = CI * CO * K * K;
  hipLaunchKernelGGL(cnn_pack_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, w, CI, CO, K, flip, p);
  return hipGetLastError();
}

// Float32 kernels of the flagger: matrix cores (default) or vector ALU.
static bool g_cnn_mfma = true;

void set_cnn_mfma(bool on) { g_cnn_mfma = on; }
bool get_cnn_mfma() { return g_cnn_mfma; }

template <int CI, int CO, int K, int D, int MODE>
static hipError_t conv_t(const float* in, const float* wp, const float* b, const float* gate, int64_t n_img,
                         int H, int W, float* out, hipStream_t s) {
  const int tx = ceil_div(W, CT_W), ty = ceil_div(H, CT_H);
  const int64_t blocks = n_img * tx * ty;
  if (blocks <= 0) return hipSuccess;
  if constexpr (CI == 32 && CO == 32 && K == 5) {
    // the matrix-core kernel addresses an image's 32 channels with 32-bit offsets
    if (g_cnn_mfma && 32LL * H * W < (1LL << 31)) {
      const size_t lds = cm_lds(D);
      const void* k = reinterpret_cast<const void*>(cnn_conv32_mfma_kernel<D, MODE>);
      hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      const int64_t grid = blocks < 256 ? blocks : 256;   // one workgroup per CU, striding over tiles
      hipLaunchKernelGGL((cnn_conv32_mfma_kernel<D, MODE>), dim3((unsigned)grid), dim3(CM_NTH), lds, s, in, wp, b,
                         gate, H, W, tx, tx * ty, blocks, out, HeadArgs{});
      return hipGetLastError();
    }
  }
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((cnn_conv_kernel<CI, CO, K, D, MODE>), dim3((unsigned)blocks), dim3(CNT), 0, s, in, wp, b,
                     gate, H, W, tx, tx * ty, out);
  return hipGetLastError();
}

hipError_t cnn_conv(int layer, int dir, const float* in, const float* wp, const float* b, const float* gate,
                    int64_t n_img, int H, int W, float* out, hipStream_t s) {
  // dir 0: forward (ReLU for L1..L3); dir 1: backward data of layer `layer`
  // (gated by the activation of the layer below)
  if (dir == 0) {
    if (layer == 1) return conv_t<1, 32, 3, 1, 0>(in, wp, b, nullptr, n_img, H, W, out, s);
    if (layer == 2) return conv_t<32, 32, 5, 1, 0>(in, wp, b, nullptr, n_img, H, W, out, s);
    if (layer == 3) return conv_t<32, 32, 5, 2, 0>(in, wp, b, nullptr, n_img, H, W, out, s);
  } else {
    if (layer == 2) return conv_t<32, 32, 5, 1, 1>(in, wp, nullptr, gate, n_img, H, W, out, s);
    if (layer == 3) return conv_t<32, 32, 5, 2, 1>(in, wp, nullptr, gate, n_img, H, W, out, s);
  }
  return hipErrorInvalidValue;
}


int64_t cnn_wgrad_blocks(int64_t n_img, int H, int W) {
  const int64_t tiles = n_img * ceil_div(W, CT_W) * ceil_div(H, CT_H);
  return tiles < 512 ? tiles : 512;
}

// blocks: in, the partial-sum slots available; out, the slots written.
template <int K, int D>
static hipError_t wgrad32_t(const float* a, const float* g, int64_t n_img, int H, int W, float* part,
                            int64_t& blocks, hipStream_t s) {
  constexpr int R = D * (K - 1) / 2;
  constexpr int LH = CT_H + 2 * R, LW = CT_W + 2 * R;
  const int tx = ceil_div(W, CT_W), ty = ceil_div(H, CT_H);
  // the matrix-core kernel addresses an image's 32 channels with 32-bit offsets
  if (g_cnn_mfma && 32LL * H * W < (1LL << 31)) {
    // one 512-thread workgroup fills a CU's LDS: one per CU
    if (blocks > 256) blocks = 256;
    const size_t lds = sizeof(float) * (32 * (CNT + 1) + 32 * (LH * LW + 1));
    const void* k = reinterpret_cast<const void*>(cnn_wgrad32_mfma_kernel<K, D>);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((cnn_wgrad32_mfma_kernel<K, D>), dim3((unsigned)blocks), dim3(512), lds, s, a, g, H, W,
                       tx, tx * ty, n_img * tx * ty, part);
    return hipGetLastError();
  }
  const size_t lds = sizeof(float) * (32 * (CNT + 1) + 8 * (LH * LW + 1));
  hipLaunchKernelGGL((cnn_wgrad32_kernel<K, D>), dim3((unsigned)blocks), dim3(256), lds, s, a, g, H, W, tx,
                     tx * ty, n_img * tx * ty, part);
  return hipGetLastError();
}

// Gradient of layer `layer`'s weights and bias (flat, W then b) into dst.
hipError_t cnn_wgrad(int layer, const float* a, const float* g, int64_t n_img, int H, int W, float* part,
                     float* dst, hipStream_t s) {
  int64_t blocks = cnn_wgrad_blocks(n_img, H, W);
  if (blocks <= 0) return hipSuccess;
  int nw = 0;
  hipError_t e = hipSuccess;
  const int tx = ceil_div(W, CT_W), ty = ceil_div(H, CT_H);
  if (layer == 1) {
    nw = 32 * 9 + 32;
    if (g_cnn_mfma)
      hipLaunchKernelGGL(cnn_wgrad_l1_mfma_kernel, dim3((unsigned)blocks), dim3(L1M_NT), 0, s, a, g, H, W, tx,
                         tx * ty, n_img * tx * ty, part);
    else
      hipLaunchKernelGGL((cnn_wgrad_small_kernel<1, 32, 3, 1>), dim3((unsigned)blocks), dim3(256), 0, s, a, g, H,
                         W, tx, tx * ty, n_img * tx * ty, part);
    e = hipGetLastError();
  } else if (layer == 2) {
    nw = 32 * 32 * 25 + 32;
    e = wgrad32_t<5, 1>(a, g, n_img, H, W, part, blocks, s);
  } else if (layer == 3) {
    nw = 32 * 32 * 25 + 32;
    e = wgrad32_t<5, 2>(a, g, n_img, H, W, part, blocks, s);
  } else {
    return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cnn_sum_parts_kernel, dim3(ceil_div(nw, 64)), dim3(64 * SP_WAVES), 0, s, part, (int)blocks, nw,
                     dst);
  return hipGetLastError();
}

hipError_t cnn_conv3_head(const float* a2, const float* w3p, const float* b3, const float* w4, int64_t n_img,
                          int H, int W, float* a3, float* logits, float thr, int64_t img0, int64_t n_base,
                          uint8_t* mask, hipStream_t s) {
  const int tx = ceil_div(W, CT_W), ty = ceil_div(H, CT_H);
  const int64_t blocks = n_img * tx * ty;
  if (blocks <= 0) return hipSuccess;
  if (g_cnn_mfma && 32LL * H * W < (1LL << 31)) {
    const size_t lds = cm_lds(2);
    const void* k = reinterpret_cast<const void*>(cnn_conv32_mfma_kernel<2, 3>);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int64_t grid = blocks < 256 ? blocks : 256;
    hipLaunchKernelGGL((cnn_conv32_mfma_kernel<2, 3>), dim3((unsigned)grid), dim3(CM_NTH), lds, s, a2, w3p, b3,
                       nullptr, H, W, tx, tx * ty, blocks, nullptr, HeadArgs{w4, logits, thr, img0, n_base, mask});
    return hipGetLastError();
  }
  hipError_t e = cnn_conv(3, 0, a2, w3p, b3, nullptr, n_img, H, W, a3, s);
  if (e != hipSuccess) return e;
  return cnn_head(a3, w4, n_img, H, W, logits, thr, img0, n_base, mask, s);
}

hipError_t cnn_head(const float* a3, const float* w4, int64_t n_img, int H, int W, float* logits, float thr,
                    int64_t img0, int64_t n_base, uint8_t* mask, hipStream_t s) {
  const int64_t n = n_img * H * W;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cnn_head_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, a3, w4, H, W, n_img,
                     logits, thr, img0, n_base, mask);
  return hipGetLastError();
}

int64_t cnn_head_bwd_blocks(int64_t n_total) {
  const int64_t b = (n_total + 255) / 256;
  return b < 1024 ? b : 1024;
}

// grad4: dW4[0..31], db4 at [32]; loss: one float.
hipError_t cnn_head_bwd(const float* logits, const uint8_t* labels, const float* a3, const float* w4,
                        int64_t n_img, int H, int W, float pos_weight, float* g3, float* part, float* grad4,
                        float* loss, hipStream_t s) {
  const int64_t n_total = n_img * H * W;
  const int64_t blocks = cnn_head_bwd_blocks(n_total);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(cnn_bce_head_bwd_kernel, dim3((unsigned)blocks), dim3(256), 0, s, logits, labels, a3, w4,
                     (int64_t)H * W, n_total, pos_weight, (float)(1.0 / (double)n_total), g3, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cnn_head_finish_kernel, dim3(1), dim3(64 * SP_WAVES), 0, s, part, (int)blocks,
                     (float)(1.0 / (double)n_total), grad4, loss);
  return hipGetLastError();
}

hipError_t cnn_adam(float* w, const float* g, float* m, float* v, int n, int64_t step, float lr, float b1,
                    float b2, float eps, hipStream_t s) {
  const double c1 = 1.0 - std::pow((double)b1, (double)step);
  const double c2 = 1.0 - std::pow((double)b2, (double)step);
  hipLaunchKernelGGL(cnn_adam_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps,
                     (float)c1, (float)c2);
  return hipGetLastError();
}

hipError_t cnn_pack_mfma(const float* w, _Float16* p, hipStream_t s) {
  hipLaunchKernelGGL(cnn_pack_mfma_kernel, dim3(ceil_div(MT_SLICES * 64 * 8, 256)), dim3(256), 0, s, w, p);
  return hipGetLastError();
}

size_t cnn_mfma_lds_bytes(int D) {
  const int R = 2 * D;
  return sizeof(uint4) * MT_SLICES * 64 + sizeof(_Float16) * (mt_h(D) + 2 * R) * (MT_W + 2 * R) * MT_PS;
}

// Inference forward with half activations: x [n][H][W] float32 ->
// logits / mask.  A and B hold n*H*W*32 halves each.
hipError_t cnn_forward_f16(const float* params, const _Float16* w2p, const _Float16* w3p, const float* x,
                           int64_t n_img, int H, int W, _Float16* A, _Float16* B, float* logits, float thr,
                           int64_t img0, int64_t n_base, uint8_t* mask, hipStream_t s) {
  const int64_t n_pix = n_img * H * W;
  if (n_pix <= 0) return hipSuccess;
  hipLaunchKernelGGL(cnn_l1_nhwc_kernel, dim3((unsigned)ceil_div(n_pix, 256)), dim3(256), 0, s, x,
                     params + CNN_OFF_L1, params + CNN_OFF_L1 + 288, H, W, n_pix, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int tx = ceil_div(W, MT_W), ty2 = ceil_div(H, mt_h(1)), ty3 = ceil_div(H, mt_h(2));
  const int64_t n_tiles2 = n_img * tx * ty2, n_tiles3 = n_img * tx * ty3;
  const unsigned grid2 = (unsigned)(n_tiles2 < 1024 ? n_tiles2 : 1024);
  const unsigned grid3 = (unsigned)(n_tiles3 < 1024 ? n_tiles3 : 1024);
  const size_t l2 = cnn_mfma_lds_bytes(1), l3 = cnn_mfma_lds_bytes(2);
  static_assert(sizeof(uint4) * MT_SLICES * 64 + sizeof(_Float16) * (mt_h(2) + 8) * (MT_W + 8) * MT_PS <=
                    160 * 1024 && sizeof(uint4) * MT_SLICES * 64 + sizeof(_Float16) * (mt_h(1) + 4) * (MT_W + 4) * MT_PS <= 160 * 1024,
                "half convolution tiles: LDS");
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(cnn_mfma_conv_kernel<1, false>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)l2);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(cnn_mfma_conv_kernel<2, true>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)l3);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((cnn_mfma_conv_kernel<1, false>), dim3(grid2), dim3(MT_NT), l2, s, A, w2p,
                     params + CNN_OFF_L2 + 25600, H, W, tx, tx * ty2, n_tiles2, B, HeadArgs{});
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // L3 with the output layer in its epilogue (its activations are not stored)
  const HeadArgs hd{params + CNN_OFF_L4, logits, thr, img0, n_base, mask};
  hipLaunchKernelGGL((cnn_mfma_conv_kernel<2, true>), dim3(grid3), dim3(MT_NT), l3, s, B, w3p,
                     params + CNN_OFF_L3 + 25600, H, W, tx, tx * ty3, n_tiles3, nullptr, hd);
  return hipGetLastError();
}

hipError_t cnn_normalize(const float2* vis, const double* stats, int64_t n_time, int64_t n_base, int n_chan,
                         int64_t b0, int64_t nb, float* x, hipStream_t s) {
  const int64_t n = nb * n_time * n_chan;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cnn_normalize_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, vis, stats, n_time,
                     n_base, n_chan, b0, nb, x);
  return hipGetLastError();
}

}  // namespace qc
