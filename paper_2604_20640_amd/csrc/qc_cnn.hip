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

__device__ __forceinline__ int64_t img_off(int64_t n, int c, int C, int H, int W) {
  return ((n * C + c) * (int64_t)H) * W;
}

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

// dst[e] = sum_b part[b][e], in block order.
__global__ void cnn_sum_parts_kernel(const float* __restrict__ part, int n_parts, int n, float* __restrict__ dst) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float s = 0.f;
  for (int b = 0; b < n_parts; ++b) s += part[(int64_t)b * n + e];
  dst[e] = s;
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
// (db4), loss = inv_count * sum_b part[b][32] (the mean); in block order.
__global__ void cnn_head_finish_kernel(const float* __restrict__ part, int n_parts, float inv_count,
                                       float* __restrict__ grad4, float* __restrict__ loss) {
  const int t = threadIdx.x;
  if (t >= 34) return;
  float s = 0.f;
  for (int b = 0; b < n_parts; ++b) s += part[(int64_t)b * 34 + t];
  if (t < 32) grad4[t] = s;
  else if (t == 32) *loss = s * inv_count;
  else grad4[32] = s;
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

template <int CI, int CO, int K, int D, int MODE>
static hipError_t conv_t(const float* in, const float* wp, const float* b, const float* gate, int64_t n_img,
                         int H, int W, float* out, hipStream_t s) {
  const int tx = ceil_div(W, CT_W), ty = ceil_div(H, CT_H);
  const int64_t blocks = n_img * tx * ty;
  if (blocks <= 0) return hipSuccess;
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

template <int K, int D>
static hipError_t wgrad32_t(const float* a, const float* g, int64_t n_img, int H, int W, float* part,
                            int64_t blocks, hipStream_t s) {
  constexpr int R = D * (K - 1) / 2;
  constexpr int LH = CT_H + 2 * R, LW = CT_W + 2 * R;
  const size_t lds = sizeof(float) * (32 * (CNT + 1) + 8 * (LH * LW + 1));
  const int tx = ceil_div(W, CT_W), ty = ceil_div(H, CT_H);
  hipLaunchKernelGGL((cnn_wgrad32_kernel<K, D>), dim3((unsigned)blocks), dim3(256), lds, s, a, g, H, W, tx,
                     tx * ty, n_img * tx * ty, part);
  return hipGetLastError();
}

// Gradient of layer `layer`'s weights and bias (flat, W then b) into dst.
hipError_t cnn_wgrad(int layer, const float* a, const float* g, int64_t n_img, int H, int W, float* part,
                     float* dst, hipStream_t s) {
  const int64_t blocks = cnn_wgrad_blocks(n_img, H, W);
  if (blocks <= 0) return hipSuccess;
  int nw = 0;
  hipError_t e = hipSuccess;
  const int tx = ceil_div(W, CT_W), ty = ceil_div(H, CT_H);
  if (layer == 1) {
    nw = 32 * 9 + 32;
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
  hipLaunchKernelGGL(cnn_sum_parts_kernel, dim3(ceil_div(nw, 256)), dim3(256), 0, s, part, (int)blocks, nw, dst);
  return hipGetLastError();
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
  hipLaunchKernelGGL(cnn_head_finish_kernel, dim3(1), dim3(64), 0, s, part, (int)blocks,
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

hipError_t cnn_normalize(const float2* vis, const double* stats, int64_t n_time, int64_t n_base, int n_chan,
                         int64_t b0, int64_t nb, float* x, hipStream_t s) {
  const int64_t n = nb * n_time * n_chan;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cnn_normalize_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, vis, stats, n_time,
                     n_base, n_chan, b0, nb, x);
  return hipGetLastError();
}

}  // namespace qc
