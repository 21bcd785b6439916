// X-engine on the gfx950 matrix cores for requantised channelised voltages.
//
// The X-engine of arXiv 2604.20640 (Sec. 4.1 eq. 1; Sec. 4.2) forms
// V_ij[k] = sum_m X_i,m[k] conj(X_j,m[k]).  Per channel this is a complex
// Gram matrix G = X X^H of the (antenna x spectrum) matrix X = A + iB:
//   Re G = A A^T + B B^T,   Im G = B A^T - A B^T.
// With antennas as rows and spectra as the reduction dimension, each term
// is a real 32x32xK product; A (or B) serves as both the left and the right
// MFMA operand because the gfx950 32x32x16 operand layouts coincide
// (lane l holds row/column l%32, reduction slots 8*(l/32)..+7).  The
// subtraction uses a sign-flipped A.  Inputs are FP16, BF16 or OCP E4M3
// (power-of-two per-antenna scales s_a); products accumulate in FP32 and the
// result is divided exactly by s_i s_j.
//
// Tiling: a workgroup of 8 waves owns 32 channels and a run of spectra; per
// step of 16 spectra it stages the [32 ant][16 spec][32 chan] tile through
// LDS, transposed to [chan][ant][spec] so each lane reads its 8 spectra as
// one contiguous run; each wave then issues 4 MFMAs for each of its 4
// channels.  n_ant <= 32 and n_chan % 32 == 0.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qc_kernels.h"

namespace qc {

namespace {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float16_t __attribute__((ext_vector_type(16)));

constexpr int XM_NT = 512;     // 8 waves
constexpr int XM_CB = 32;      // channels per workgroup
constexpr int XM_KS = 16;      // spectra per step
constexpr int XM_NA = 32;      // antenna rows of the tile

// LDS row (one channel) in 32-bit words for 16-bit pairs: 32 ant x 16 spec + pad
constexpr int XM_CSTR16 = XM_NA * XM_KS + 4;
// LDS row in 16-bit units for fp8 pairs
constexpr int XM_CSTR8 = XM_NA * XM_KS + 8;

template <int PREC>
struct Op;

template <>
struct Op<1> {  // FP16
  static __device__ __forceinline__ float16_t mfma(uint4 a, uint4 b, float16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8_t, a),
                                                  __builtin_bit_cast(half8_t, b), c, 0, 0, 0);
  }
};
template <>
struct Op<2> {  // BF16
  static __device__ __forceinline__ float16_t mfma(uint4 a, uint4 b, float16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                   __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
  }
};
template <>
struct Op<3> {  // FP8 E4M3
  static __device__ __forceinline__ float16_t mfma(uint2 a, uint2 b, float16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(__builtin_bit_cast(long, a),
                                                      __builtin_bit_cast(long, b), c, 0, 0, 0);
  }
};

}  // namespace

template <int PREC>
__global__ void __launch_bounds__(XM_NT)
xeng_mfma_kernel(const void* __restrict__ vin, const float* __restrict__ scale, int n_ant,
                 int64_t n_spec, int n_chan, int64_t spec_per_dump, int64_t ksplit, int n_cb,
                 float2* __restrict__ part) {
  constexpr bool F8 = (PREC == 3);
  // 16-bit formats: 4 bytes per complex; fp8: 2 bytes
  constexpr int CB_BYTES = F8 ? 2 : 4;
  constexpr int CHUNKS_PER_ROW = XM_CB * CB_BYTES / 16;       // 16-byte chunks per (ant, spec)
  constexpr int CHUNKS = XM_NA * XM_KS * CHUNKS_PER_ROW;      // per tile
  constexpr int CPT = CHUNKS / XM_NT;                         // per thread
  constexpr int CH_PER_CHUNK = 16 / CB_BYTES;                 // channels per chunk
  extern __shared__ uint32_t lds[];  // xm_lds_bytes(PREC)

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int cb = (int)(blockIdx.x % n_cb);
  const int64_t dz = blockIdx.x / n_cb;
  const int64_t d = dz / ksplit, ks = dz % ksplit;
  const int64_t m_lo = d * spec_per_dump + (ks * spec_per_dump) / ksplit;
  const int64_t m_hi = d * spec_per_dump + ((ks + 1) * spec_per_dump) / ksplit;
  const uint8_t* vb = reinterpret_cast<const uint8_t*>(vin);

  float16_t accR[4], accI[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      accR[c][r] = 0.f;
      accI[c][r] = 0.f;
    }

  uint4 pre[CPT];
  auto gload = [&](int64_t m0) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int q = tid + i * XM_NT;
      const int ch = q % CHUNKS_PER_ROW;
      const int m = (q / CHUNKS_PER_ROW) % XM_KS;
      const int a = q / (CHUNKS_PER_ROW * XM_KS);
      const int64_t mm = m0 + m;
      if (a < n_ant && mm < m_hi) {
        const int64_t off = (((int64_t)a * n_spec + mm) * n_chan + (int64_t)cb * XM_CB) * CB_BYTES + ch * 16;
        pre[i] = *reinterpret_cast<const uint4*>(vb + off);
      } else {
        pre[i] = make_uint4(0u, 0u, 0u, 0u);
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int q = tid + i * XM_NT;
      const int ch = q % CHUNKS_PER_ROW;
      const int m = (q / CHUNKS_PER_ROW) % XM_KS;
      const int a = q / (CHUNKS_PER_ROW * XM_KS);
      const uint32_t w[4] = {pre[i].x, pre[i].y, pre[i].z, pre[i].w};
      if constexpr (!F8) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = ch * CH_PER_CHUNK + e;
          lds[c * XM_CSTR16 + a * XM_KS + m] = w[e];
        }
      } else {
        uint16_t* l16 = reinterpret_cast<uint16_t*>(lds);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int c = ch * CH_PER_CHUNK + e;
          l16[c * XM_CSTR8 + a * XM_KS + m] = (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
        }
      }
    }
  };

  const int ra = lane & 31, rh = lane >> 5;
  int64_t m0 = m_lo;
  if (m0 < m_hi) gload(m0);
  for (; m0 < m_hi; m0 += XM_KS) {
    __syncthreads();
    lstore();
    __syncthreads();
    if (m0 + XM_KS < m_hi) gload(m0 + XM_KS);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int ch = wave * 4 + c;
      if constexpr (!F8) {
        const uint4* p = reinterpret_cast<const uint4*>(&lds[ch * XM_CSTR16 + ra * XM_KS + 8 * rh]);
        const uint4 u0 = p[0], u1 = p[1];
        const uint32_t w[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
        uint4 re, im;
        re.x = __builtin_amdgcn_perm(w[1], w[0], 0x05040100u);
        re.y = __builtin_amdgcn_perm(w[3], w[2], 0x05040100u);
        re.z = __builtin_amdgcn_perm(w[5], w[4], 0x05040100u);
        re.w = __builtin_amdgcn_perm(w[7], w[6], 0x05040100u);
        im.x = __builtin_amdgcn_perm(w[1], w[0], 0x07060302u);
        im.y = __builtin_amdgcn_perm(w[3], w[2], 0x07060302u);
        im.z = __builtin_amdgcn_perm(w[5], w[4], 0x07060302u);
        im.w = __builtin_amdgcn_perm(w[7], w[6], 0x07060302u);
        const uint4 nre = make_uint4(re.x ^ 0x80008000u, re.y ^ 0x80008000u, re.z ^ 0x80008000u,
                                     re.w ^ 0x80008000u);
        accR[c] = Op<PREC>::mfma(re, re, accR[c]);
        accR[c] = Op<PREC>::mfma(im, im, accR[c]);
        accI[c] = Op<PREC>::mfma(im, re, accI[c]);
        accI[c] = Op<PREC>::mfma(nre, im, accI[c]);
      } else {
        const uint16_t* l16 = reinterpret_cast<const uint16_t*>(lds);
        const uint4 u = *reinterpret_cast<const uint4*>(&l16[ch * XM_CSTR8 + ra * XM_KS + 8 * rh]);
        uint2 re, im;
        re.x = __builtin_amdgcn_perm(u.y, u.x, 0x06040200u);
        re.y = __builtin_amdgcn_perm(u.w, u.z, 0x06040200u);
        im.x = __builtin_amdgcn_perm(u.y, u.x, 0x07050301u);
        im.y = __builtin_amdgcn_perm(u.w, u.z, 0x07050301u);
        const uint2 nre = make_uint2(re.x ^ 0x80808080u, re.y ^ 0x80808080u);
        accR[c] = Op<PREC>::mfma(re, re, accR[c]);
        accR[c] = Op<PREC>::mfma(im, im, accR[c]);
        accI[c] = Op<PREC>::mfma(im, re, accI[c]);
        accI[c] = Op<PREC>::mfma(nre, im, accI[c]);
      }
    }
  }
  // write the upper triangle, unscaled by 1/(s_i s_j)
  const int nb = n_ant * (n_ant + 1) / 2;
  float2* out = part + dz * (int64_t)nb * n_chan;
  const int j = lane & 31;
  const float inv_j = j < n_ant ? 1.0f / scale[j] : 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int k = cb * XM_CB + wave * 4 + c;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (i <= j && j < n_ant) {
        const float inv = (1.0f / scale[i]) * inv_j;
        const int b = i * n_ant - i * (i - 1) / 2 + (j - i);
        out[(int64_t)b * n_chan + k] = make_float2(accR[c][r] * inv, i == j ? 0.f : accI[c][r] * inv);
      }
    }
  }
}

int64_t xeng_mfma_ksplit(int n_ant, int64_t spd, int n_chan, int64_t n_dump) {
  if (n_ant > XM_NA || n_chan % XM_CB != 0) return 0;
  const int64_t blocks = (int64_t)(n_chan / XM_CB) * n_dump;
  int64_t ks = (1024 + blocks - 1) / blocks;
  const int64_t maxk = spd / 64 > 0 ? spd / 64 : 1;
  if (ks > maxk) ks = maxk;
  return ks < 1 ? 1 : ks;
}

static constexpr size_t xm_lds_bytes(int prec) {
  return prec == 3 ? (size_t)XM_CB * XM_CSTR8 * 2 : (size_t)XM_CB * XM_CSTR16 * 4;
}

template <int PREC>
static hipError_t launch_xm_t(dim3 grid, const void* v, const float* scale, int n_ant, int64_t n_spec,
                              int n_chan, int64_t spd, int64_t ksplit, int n_cb, float2* part,
                              hipStream_t s) {
  const size_t lds = xm_lds_bytes(PREC);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(xeng_mfma_kernel<PREC>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(xeng_mfma_kernel<PREC>, grid, dim3(XM_NT), lds, s, v, scale, n_ant, n_spec,
                     n_chan, spd, ksplit, n_cb, part);
  return hipGetLastError();
}

hipError_t launch_xeng_mfma(const void* v, int prec, const float* scale, int n_ant, int64_t n_spec,
                            int n_chan, int64_t spd, int64_t n_dump, int64_t ksplit, float2* part,
                            hipStream_t s) {
  const int n_cb = n_chan / XM_CB;
  dim3 grid((unsigned)(n_cb * n_dump * ksplit));
  switch (prec) {
    case 1: return launch_xm_t<1>(grid, v, scale, n_ant, n_spec, n_chan, spd, ksplit, n_cb, part, s);
    case 2: return launch_xm_t<2>(grid, v, scale, n_ant, n_spec, n_chan, spd, ksplit, n_cb, part, s);
    case 3: return launch_xm_t<3>(grid, v, scale, n_ant, n_spec, n_chan, spd, ksplit, n_cb, part, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace qc
