// F-engine over every input word of the paper's acquisition chain (Sec. 3.3
// quantisation modes; Sec. 4.2 "F-engine": raw samples are unpacked and
// converted into complex voltage streams):
//   ST 0: real int8   (8-bit truncated mode)
//   ST 1: real int16  (default 16-bit padded mode: the 14-bit ADC value
//                      stored in 16 bits, taken as the integer it is)
//   ST 2: complex int8  (I, Q interleaved)
//   ST 3: complex int16 (I, Q interleaved)
//
// FIR: y_m[n] = sum_p h[pN+n] x[(m-P+1+p)N + n] with the real prototype h
// applied to I and Q alike.  DFT: forward exp(-2 pi i k n / N), unnormalised.
// Real words: two antennas share one complex transform (z = y_a + i y_b;
// Y_a[k] = (Z[k] + conj Z[N-k]) / 2, Y_b[k] = (Z[k] - conj Z[N-k]) / 2i) and
// channels k = 0 .. N/2-1 are kept.  Complex words: one antenna per
// transform, all N channels k = 0 .. N-1 in natural order.
//
// Per-antenna power-of-two scales for requantised output come from the exact
// integer power sum of |x|^2 (I^2 + Q^2 for complex words) over the first
// n_use samples, as for int8.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "qc_fft.h"
#include "qc_kernels.h"

namespace qc {

namespace {

template <int ST>
struct Word {
  static constexpr bool CPLX = ST >= 2;
  static constexpr int BYTES = (ST == 0) ? 1 : (ST == 3) ? 4 : 2;  // bytes per sample
};

// Four consecutive samples n0..n0+3 of one row (16-byte aligned for complex
// int16, 8-byte for int16 and complex int8, 4-byte for int8).
// Real words fill re[0..3]; complex words fill re (I) and im (Q).
template <int ST>
__device__ __forceinline__ void load4(const unsigned char* __restrict__ row, int64_t n0, float re[4],
                                      float im[4]) {
  if constexpr (ST == 0) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(row + n0);
#pragma unroll
    for (int i = 0; i < 4; ++i) re[i] = (float)(int8_t)((w >> (8 * i)) & 0xffu);
  } else if constexpr (ST == 1) {
    const uint2 w = *reinterpret_cast<const uint2*>(row + 2 * n0);
    re[0] = (float)(int16_t)(w.x & 0xffffu);
    re[1] = (float)(int16_t)(w.x >> 16);
    re[2] = (float)(int16_t)(w.y & 0xffffu);
    re[3] = (float)(int16_t)(w.y >> 16);
  } else if constexpr (ST == 2) {
    const uint2 w = *reinterpret_cast<const uint2*>(row + 2 * n0);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      re[i] = (float)(int8_t)((w.x >> (16 * i)) & 0xffu);
      im[i] = (float)(int8_t)((w.x >> (16 * i + 8)) & 0xffu);
      re[2 + i] = (float)(int8_t)((w.y >> (16 * i)) & 0xffu);
      im[2 + i] = (float)(int8_t)((w.y >> (16 * i + 8)) & 0xffu);
    }
  } else {
    const uint4 w = *reinterpret_cast<const uint4*>(row + 4 * n0);
    const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      re[i] = (float)(int16_t)(v[i] & 0xffffu);
      im[i] = (float)(int16_t)(v[i] >> 16);
    }
  }
}

// Row `r` of the input (antenna r), stream block blk (blk < 0: history or
// zeros), samples n0..n0+3.
template <int ST>
__device__ __forceinline__ void load_block4(const unsigned char* __restrict__ x, int64_t ld_bytes,
                                            const unsigned char* __restrict__ hist, int r, int64_t blk,
                                            int n0, int N, int P, float re[4], float im[4]) {
  if (blk >= 0) {
    load4<ST>(x + (int64_t)r * ld_bytes, blk * N + n0, re, im);
  } else if (hist) {
    const int64_t keep = (int64_t)(P - 1) * N;
    load4<ST>(hist + (int64_t)r * keep * Word<ST>::BYTES, (blk + P - 1) * N + n0, re, im);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) re[i] = im[i] = 0.f;
  }
}

template <int N>
struct XCfg {
  static constexpr int S = N >= 4096 ? 1 : 4096 / N;  // transforms in flight per block
  static constexpr int NT = S * N / 16;
  static constexpr int LDS = lds_padded_size(S * N);
};

__device__ __forceinline__ uint32_t enc16(float v, int prec) {
  if (prec == 1) {
    v = fminf(fmaxf(v, -65504.f), 65504.f);
    return __half_as_ushort(__float2half_rn(v));
  }
  uint32_t u = __float_as_uint(v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// Store one channelised value (already scaled) in the output's format.
template <int PREC>
__device__ __forceinline__ void store_val(void* __restrict__ out, int64_t i, float re, float im) {
  if constexpr (PREC == 0) {
    reinterpret_cast<float2*>(out)[i] = make_float2(re, im);
  } else if constexpr (PREC == 1 || PREC == 2) {
    reinterpret_cast<uint32_t*>(out)[i] = enc16(re, PREC) | (enc16(im, PREC) << 16);
  } else {
    const float a = fminf(fmaxf(re, -448.f), 448.f);
    const float b = fminf(fmaxf(im, -448.f), 448.f);
    reinterpret_cast<uint16_t*>(out)[i] = (uint16_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  }
}

}  // namespace

// Grid (spectrum blocks, rows): a row is an antenna pair for real words and
// one antenna for complex words.  S transforms of N points in flight.
template <int N, int ST, int PREC>
__global__ void __launch_bounds__(XCfg<N>::NT)
chanx_kernel(const unsigned char* __restrict__ x, int64_t ld_bytes, int n_ant, int64_t n_spec,
             const unsigned char* __restrict__ hist, const float* __restrict__ taps, int P,
             const float2* __restrict__ tw, int64_t spec_per_blk, const float* __restrict__ scale,
             void* __restrict__ out) {
  using C = XCfg<N>;
  constexpr bool CPLX = Word<ST>::CPLX;
  constexpr int NCH = CPLX ? N : N / 2;
  extern __shared__ float2 buf[];
  const int tid = threadIdx.x;
  const int row = blockIdx.y;
  const int a0 = CPLX ? row : 2 * row;
  const int a1 = CPLX ? -1 : ((2 * row + 1 < n_ant) ? 2 * row + 1 : -1);
  const int64_t m_lo = (int64_t)blockIdx.x * spec_per_blk;
  int64_t m_hi = m_lo + spec_per_blk;
  if (m_hi > n_spec) m_hi = n_spec;
  float sa = 1.f, sb = 1.f;
  if (PREC != 0) {
    sa = scale[a0];
    sb = a1 >= 0 ? scale[a1] : 1.f;
  }
  for (int64_t m0 = m_lo; m0 < m_hi; m0 += C::S) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int c4 = tid + g * C::NT;
      const int s = c4 / (N / 4);
      const int n0 = 4 * (c4 % (N / 4));
      float y0[4] = {0.f, 0.f, 0.f, 0.f}, y1[4] = {0.f, 0.f, 0.f, 0.f};
      if (m0 + s < m_hi) {
        const int64_t blk0 = m0 + s - P + 1;
        for (int q = 0; q < P; ++q) {
          const float4 h = *reinterpret_cast<const float4*>(taps + (int64_t)q * N + n0);
          const float hv[4] = {h.x, h.y, h.z, h.w};
          float re[4], im[4];
          load_block4<ST>(x, ld_bytes, hist, a0, blk0 + q, n0, N, P, re, im);
          if constexpr (CPLX) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              y0[i] += hv[i] * re[i];
              y1[i] += hv[i] * im[i];
            }
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) y0[i] += hv[i] * re[i];
            if (a1 >= 0) {
              load_block4<ST>(x, ld_bytes, hist, a1, blk0 + q, n0, N, P, re, im);
#pragma unroll
              for (int i = 0; i < 4; ++i) y1[i] += hv[i] * re[i];
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) buf[lds_pad(s * N + n0 + i)] = make_float2(y0[i], y1[i]);
    }
    __syncthreads();
    fft_lds<N, C::NT>(buf, tw, tid);
    constexpr int PER = C::S * NCH / C::NT;  // outputs per thread (8 real, 16 complex)
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * C::NT;
      const int s = e / NCH, k = e % NCH;
      const int64_t m = m0 + s;
      if (m < m_hi) {
        const float2 zk = buf[lds_pad(s * N + k)];
        if constexpr (CPLX) {
          store_val<PREC>(out, ((int64_t)a0 * n_spec + m) * NCH + k, zk.x * sa, zk.y * sa);
        } else {
          const float2 zn = buf[lds_pad(s * N + ((N - k) & (N - 1)))];
          // (Z[k] + conj Z[N-k]) / 2 and (Z[k] - conj Z[N-k]) / 2i
          const float ha = 0.5f * sa, hb = 0.5f * sb;
          store_val<PREC>(out, ((int64_t)a0 * n_spec + m) * NCH + k, (zk.x + zn.x) * ha, (zk.y - zn.y) * ha);
          if (a1 >= 0)
            store_val<PREC>(out, ((int64_t)a1 * n_spec + m) * NCH + k, (zk.y + zn.y) * hb,
                            (zn.x - zk.x) * hb);
        }
      }
    }
    __syncthreads();
  }
}

template <int N, int ST>
static hipError_t launch_chanx_n(const ChanxArgs& a, int prec, void* out, const float* scale,
                                 hipStream_t s) {
  using C = XCfg<N>;
  const int64_t n_spec = a.n_samp / N;
  const int rows = Word<ST>::CPLX ? a.n_ant : (a.n_ant + 1) / 2;
  int64_t per = (n_spec * rows + 2047) / 2048;  // ~2048 blocks in total
  per = ((per + C::S - 1) / C::S) * C::S;
  if (per < C::S) per = C::S;
  const int64_t nbx = (n_spec + per - 1) / per;
  const size_t lds = sizeof(float2) * C::LDS;
  const void* k = nullptr;
  switch (prec) {
    case 0: k = reinterpret_cast<const void*>(chanx_kernel<N, ST, 0>); break;
    case 1: k = reinterpret_cast<const void*>(chanx_kernel<N, ST, 1>); break;
    case 2: k = reinterpret_cast<const void*>(chanx_kernel<N, ST, 2>); break;
    default: k = reinterpret_cast<const void*>(chanx_kernel<N, ST, 3>); break;
  }
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)nbx, (unsigned)rows);
  const int64_t ldb = a.ld_x * Word<ST>::BYTES;
  const unsigned char* xb = static_cast<const unsigned char*>(a.x);
  const unsigned char* hb = static_cast<const unsigned char*>(a.hist);
#define QC_CHANX(PR)                                                                                   \
  return launch(chanx_kernel<N, ST, PR>, grid, dim3(C::NT), lds, s, xb, ldb, a.n_ant, n_spec, hb, a.taps, \
                a.n_taps, a.tw, per, scale, out)
  switch (prec) {
    case 0: QC_CHANX(0);
    case 1: QC_CHANX(1);
    case 2: QC_CHANX(2);
    default: QC_CHANX(3);
  }
#undef QC_CHANX
}

template <int ST>
static hipError_t launch_chanx_st(const ChanxArgs& a, int prec, void* out, const float* scale,
                                  hipStream_t s) {
  switch (a.n_fft) {
    case 4: return launch_chanx_n<4, ST>(a, prec, out, scale, s);
    case 8: return launch_chanx_n<8, ST>(a, prec, out, scale, s);
    case 16: return launch_chanx_n<16, ST>(a, prec, out, scale, s);
    case 32: return launch_chanx_n<32, ST>(a, prec, out, scale, s);
    case 64: return launch_chanx_n<64, ST>(a, prec, out, scale, s);
    case 128: return launch_chanx_n<128, ST>(a, prec, out, scale, s);
    case 256: return launch_chanx_n<256, ST>(a, prec, out, scale, s);
    case 512: return launch_chanx_n<512, ST>(a, prec, out, scale, s);
    case 1024: return launch_chanx_n<1024, ST>(a, prec, out, scale, s);
    case 2048: return launch_chanx_n<2048, ST>(a, prec, out, scale, s);
    case 4096: return launch_chanx_n<4096, ST>(a, prec, out, scale, s);
    case 8192: return launch_chanx_n<8192, ST>(a, prec, out, scale, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_channelize_any(const ChanxArgs& a, int sample, int prec, void* out, const float* scale,
                                 hipStream_t s) {
  const hipError_t r = launch_channelize_ring_any(a, sample, prec, out, scale, s);
  if (r != hipErrorNotSupported) return r;
  switch (sample) {
    case 0: return launch_chanx_st<0>(a, prec, out, scale, s);
    case 1: return launch_chanx_st<1>(a, prec, out, scale, s);
    case 2: return launch_chanx_st<2>(a, prec, out, scale, s);
    case 3: return launch_chanx_st<3>(a, prec, out, scale, s);
  }
  return hipErrorInvalidValue;
}

// ---- per-antenna scales: exact integer sum of |x|^2 over the first n_use samples
template <int ST>
__global__ void __launch_bounds__(256)
scalesx_partial_kernel(const unsigned char* __restrict__ x, int64_t ld_bytes, int64_t n_use,
                       unsigned long long* __restrict__ part) {
  __shared__ unsigned long long red[4];
  const int a = blockIdx.y;
  const unsigned char* xa = x + (int64_t)a * ld_bytes;
  const int64_t n0 = n_use * blockIdx.x / SC_BLOCKS, n1 = n_use * (blockIdx.x + 1) / SC_BLOCKS;
  unsigned long long acc = 0;
  for (int64_t n = n0 + threadIdx.x; n < n1; n += 256) {
    long long v;
    if constexpr (ST == 0) {
      const long long r = (int8_t)xa[n];
      v = r * r;
    } else if constexpr (ST == 1) {
      const long long r = reinterpret_cast<const int16_t*>(xa)[n];
      v = r * r;
    } else if constexpr (ST == 2) {
      const long long r = (int8_t)xa[2 * n], i = (int8_t)xa[2 * n + 1];
      v = r * r + i * i;
    } else {
      const long long r = reinterpret_cast<const int16_t*>(xa)[2 * n];
      const long long i = reinterpret_cast<const int16_t*>(xa)[2 * n + 1];
      v = r * r + i * i;
    }
    acc += (unsigned long long)v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)a * SC_BLOCKS + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void scalesx_finish_kernel(const unsigned long long* __restrict__ part, int n_ant, int64_t n_use,
                                      double sum_h2, double target, float* __restrict__ scale_out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_ant) return;
  unsigned long long tot = 0;
  for (int b = 0; b < SC_BLOCKS; ++b) tot += part[(int64_t)a * SC_BLOCKS + b];
  const double rms = sqrt((double)tot / (double)n_use * sum_h2);
  float sc = 1.f;
  if (rms > 0.0) sc = (float)ldexp(1.0, (int)rint(log2(target / rms)));
  scale_out[a] = sc;
}

hipError_t launch_scales_any(const void* x, int sample, int64_t ld_x, int n_ant, int64_t n_use, double sum_h2,
                             double target, unsigned long long* part, float* scale_out, hipStream_t s) {
  const unsigned char* xb = static_cast<const unsigned char*>(x);
  const int bytes = sample == 0 ? 1 : sample == 3 ? 4 : 2;
  const dim3 grid(SC_BLOCKS, n_ant);
  hipError_t e;
  switch (sample) {
    case 0: e = launch(scalesx_partial_kernel<0>, grid, dim3(256), 0, s, xb, ld_x * bytes, n_use, part); break;
    case 1: e = launch(scalesx_partial_kernel<1>, grid, dim3(256), 0, s, xb, ld_x * bytes, n_use, part); break;
    case 2: e = launch(scalesx_partial_kernel<2>, grid, dim3(256), 0, s, xb, ld_x * bytes, n_use, part); break;
    case 3: e = launch(scalesx_partial_kernel<3>, grid, dim3(256), 0, s, xb, ld_x * bytes, n_use, part); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return launch(scalesx_finish_kernel, dim3((n_ant + 255) / 256), dim3(256), 0, s, part, n_ant, n_use, sum_h2,
                target, scale_out);
}

}  // namespace qc
