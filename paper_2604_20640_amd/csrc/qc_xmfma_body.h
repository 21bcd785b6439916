// Matrix-core X-engine body (see qc_xmfma.hip for the method): the
// operand helpers, the staging layout and the per-block body, shared by the
// X-engine kernel and the batched plans' persistent kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "qc_kernels.h"

namespace qc {

namespace {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float16_t __attribute__((ext_vector_type(16)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void_t;

constexpr int XM_NT = 512;              // 8 waves
constexpr int XM_NA = 32;               // antenna rows of the tile
constexpr int XM_CHUNK = 1024 + 16;     // LDS bytes per chunk (64 lanes x 16 B + pad)
constexpr int XM_NCHUNK = 64;           // chunks per stage (64 KiB of data)
// Output staging reuses the stage buffers: up to 528 baselines (32
// antennas) as two halves of XM_HALF rows, each row CB channels plus an
// 8-byte pad; float32 keeps its P tiles ([8 waves][32][33] floats) in
// front of its rows.
constexpr int XM_HALF = 264;
constexpr int XM_PT = 32 * 33;
constexpr int XM_PTILES = 8 * XM_PT * 4;
constexpr int xm_max(int a, int b) { return a > b ? a : b; }
constexpr int XM_STAGE = xm_max(xm_max(XM_NCHUNK * XM_CHUNK, XM_HALF * (32 * 8 + 8)),
                                XM_PTILES + XM_HALF * (16 * 8 + 8));
constexpr int XM_CPW = XM_NCHUNK / (XM_NT / 64);  // chunks each wave loads per stage

// Kernel codes: 0 float32 on 32 x 32 tiles, 1 FP16, 2 BF16, 3 E4M3, 4
// float32 on 16 x 16 tiles (v_mfma_f32_16x16x4_f32, up to 16 antennas).
// Per code: antennas of the tile, channels per workgroup, bytes per complex
// sample, spectra per stage, accumulator floats per lane.
template <int PREC>
struct XmCfg {
  static constexpr bool F32 = PREC == 0 || PREC == 4;
  static constexpr int TA = PREC == 4 ? 16 : 32;
  static constexpr int CB = F32 ? 16 : 32;
  static constexpr int EB = F32 ? 8 : PREC == 3 ? 2 : 4;
  static constexpr int KS = (PREC == 3 || PREC == 4) ? 32 : 16;
  static constexpr int ACC = TA == 32 ? 16 : 4;
  static constexpr int RB = CB * EB;        // bytes of one (antenna, spectrum) row
  static constexpr int GPR = RB / 16;       // 16-byte granules per row
  static_assert(TA * KS * RB == XM_NCHUNK * 1024, "stage = 64 chunks of 1 KiB");
};

// Row r of chunk j holds antenna j % TA at spectrum offset row_spec(j, r):
//   float32, 32 x 32: chunk half h = j/32 holds spectra 2r + h  (k-slot h of k-step r)
//   float32, 16 x 16: chunk quarter h = j/16 holds spectra 4r + h
//   FP16/BF16:        chunk half h holds spectra 8h + r          (lane half h's 8 slots)
//   E4M3:             chunk half g holds spectra 16g + r         (k-group g of the stage)
template <int PREC>
__device__ __forceinline__ int row_spec(int j, int r) {
  if constexpr (PREC == 4) return 4 * r + (j >> 4);
  const int h = j >> 5;
  if constexpr (PREC == 0) return 2 * r + h;
  else if constexpr (PREC == 3) return 16 * h + r;
  else return 8 * h + r;
}

// Gram row of accumulator slot r in lane l (its column is l % TA).
template <int TA>
__device__ __forceinline__ int acc_row(int l, int r) {
  if constexpr (TA == 32) return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
  else return 4 * (l >> 4) + r;
}

__device__ __forceinline__ void wait_vmem_all() {
  // s_waitcnt vmcnt(0), expcnt and lgkmcnt left at their maxima
  __builtin_amdgcn_s_waitcnt(0x0F70);
}

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

// Four products of one channel from eight 16-bit complex samples per lane
// (w[p] = re | im << 16 of spectrum 8h + p).
template <int PREC>
__device__ __forceinline__ void gram16(const uint32_t (&w)[8], float16_t& accR, float16_t& accI) {
  uint4 re, im;
  re.x = __builtin_amdgcn_perm(w[1], w[0], 0x05040100u);
  re.y = __builtin_amdgcn_perm(w[3], w[2], 0x05040100u);
  re.z = __builtin_amdgcn_perm(w[5], w[4], 0x05040100u);
  re.w = __builtin_amdgcn_perm(w[7], w[6], 0x05040100u);
  im.x = __builtin_amdgcn_perm(w[1], w[0], 0x07060302u);
  im.y = __builtin_amdgcn_perm(w[3], w[2], 0x07060302u);
  im.z = __builtin_amdgcn_perm(w[5], w[4], 0x07060302u);
  im.w = __builtin_amdgcn_perm(w[7], w[6], 0x07060302u);
  const uint4 nre = make_uint4(re.x ^ 0x80008000u, re.y ^ 0x80008000u, re.z ^ 0x80008000u, re.w ^ 0x80008000u);
  accR = Op<PREC>::mfma(re, re, accR);
  accR = Op<PREC>::mfma(im, im, accR);
  accI = Op<PREC>::mfma(im, re, accI);
  accI = Op<PREC>::mfma(nre, im, accI);
}

// The same for E4M3 pairs: raw[p] holds four channels' (re, im) byte pairs
// of spectrum 8h + p; channel e's pair is 16-bit half (e & 1) of word e >> 1.
__device__ __forceinline__ void gram8(const uint2 (&raw)[8], int e, float16_t& accR, float16_t& accI) {
  const uint32_t s = 2u * (uint32_t)(e & 1);
  // bytes (re_p, re_p+1, im_p, im_p+1) from words of spectra p (low) and p+1 (high)
  const uint32_t sel = s | ((4u + s) << 8) | ((s + 1u) << 16) | ((5u + s) << 24);
  uint32_t t[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t lo = (e >> 1) ? raw[2 * q].y : raw[2 * q].x;
    const uint32_t hi = (e >> 1) ? raw[2 * q + 1].y : raw[2 * q + 1].x;
    t[q] = __builtin_amdgcn_perm(hi, lo, sel);
  }
  uint2 re, im;
  re.x = __builtin_amdgcn_perm(t[1], t[0], 0x05040100u);
  re.y = __builtin_amdgcn_perm(t[3], t[2], 0x05040100u);
  im.x = __builtin_amdgcn_perm(t[1], t[0], 0x07060302u);
  im.y = __builtin_amdgcn_perm(t[3], t[2], 0x07060302u);
  const uint2 nre = make_uint2(re.x ^ 0x80808080u, re.y ^ 0x80808080u);
  accR = Op<3>::mfma(re, re, accR);
  accR = Op<3>::mfma(im, im, accR);
  accI = Op<3>::mfma(im, re, accI);
  accI = Op<3>::mfma(nre, im, accI);
}

// Stages [s_lo, s_hi) of dump d for split ks: stage boundaries are
// multiples of KS spectra, so only a dump's last stage can be ragged.
template <int KS>
__device__ __forceinline__ void split_range(int64_t spd, int64_t ksplit, int64_t dz, int64_t& m_lo,
                                            int64_t& m_hi) {
  const int64_t d = dz / ksplit, ks = dz % ksplit;
  const int64_t nst = (spd + KS - 1) / KS;
  const int64_t s_lo = ks * nst / ksplit, s_hi = (ks + 1) * nst / ksplit;
  m_lo = d * spd + s_lo * KS;
  const int64_t e = s_hi * KS < spd ? s_hi * KS : spd;
  m_hi = d * spd + e;
}

// Body of the matrix-core X-engine for channel block cb (CB channels) and
// run dz = dump * ksplit + split, by all XM_NT threads of a block, with two
// LDS stage buffers of XM_STAGE bytes each (16-byte aligned).
template <int PREC, bool WT = false>
__device__ __forceinline__ void xeng_mfma_body(const void* __restrict__ vin, const float* __restrict__ scale,
                                               int n_ant, int64_t n_spec, int n_chan, int64_t spec_per_dump,
                                               int64_t ksplit, int cb, int64_t dz, float2* __restrict__ part,
                                               uint8_t* st0, uint8_t* st1) {
  using C = XmCfg<PREC>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int64_t m_lo, m_hi;
  split_range<C::KS>(spec_per_dump, ksplit, dz, m_lo, m_hi);
  const int64_t n_st = (m_hi - m_lo + C::KS - 1) / C::KS;
  const uint8_t* vb = reinterpret_cast<const uint8_t*>(vin) + (int64_t)cb * C::RB;
  const int64_t row_pitch = (int64_t)n_chan * C::EB;

  // float32: per wave two channels, Re and P; otherwise four channels, Re and Im
  constexpr int NCW = C::F32 ? 2 : 4;
  using Acc = typename std::conditional<C::TA == 32, float16_t, float4_t>::type;
  Acc accR[NCW], accI[NCW];
#pragma unroll
  for (int c = 0; c < NCW; ++c)
#pragma unroll
    for (int r = 0; r < C::ACC; ++r) {
      accR[c][r] = 0.f;
      accI[c][r] = 0.f;
    }

  // One stage of loads: chunk j = wave*CPW + u, lane -> (row, granule).
  // Rows of antennas >= n_ant are not loaded (their products only reach
  // discarded outputs); rows past m_hi load row m_hi-1 and are zeroed later.
  // The source address is a wave-uniform base (antenna, stage) plus a
  // 32-bit lane offset (row, granule).
  auto issue = [&](uint8_t* dst, int64_t m0) {
    const int r = lane / C::GPR, g = lane % C::GPR;
    const int64_t left = m_hi - 1 - m0;
    const int lim = left < C::KS ? (int)left : C::KS;
#pragma unroll
    for (int u = 0; u < XM_CPW; ++u) {
      const int j = wave * XM_CPW + u;
      const int a = j & (C::TA - 1);
      if (a < n_ant) {
        int rs = row_spec<PREC>(j, r);
        rs = rs < lim ? rs : lim;
        const uint8_t* base = vb + ((int64_t)a * n_spec + m0) * row_pitch;
        const uint32_t off = (uint32_t)rs * (uint32_t)row_pitch + (uint32_t)(g * 16);
        __builtin_amdgcn_global_load_lds(base + off, (lds_void_t*)(dst + j * XM_CHUNK), 16, 0, 0);
      }
    }
  };
  auto zero_tail = [&](uint8_t* cur, int64_t m0) {
    for (int q = tid; q < XM_NCHUNK * 64; q += XM_NT) {
      const int j = q >> 6, i = q & 63;
      if (m0 + row_spec<PREC>(j, i / C::GPR) >= m_hi)
        *reinterpret_cast<uint4*>(cur + j * XM_CHUNK + i * 16) = make_uint4(0u, 0u, 0u, 0u);
    }
  };
  const int ra = lane & 31, rh = lane >> 5;
  auto compute = [&](const uint8_t* cur) {
    if constexpr (PREC == 4) {
      // lane (antenna l % 16, k-slot l / 16); k-step t covers spectra 4t..4t+3
      const uint8_t* p = cur + ((lane >> 4) * 16 + (lane & 15)) * XM_CHUNK + wave * 16;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float4 q = *reinterpret_cast<const float4*>(p + t * 128);
        accR[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(q.x, q.x, accR[0], 0, 0, 0);
        accR[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(q.y, q.y, accR[0], 0, 0, 0);
        accI[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(q.y, q.x, accI[0], 0, 0, 0);
        accR[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(q.z, q.z, accR[1], 0, 0, 0);
        accR[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(q.w, q.w, accR[1], 0, 0, 0);
        accI[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(q.w, q.z, accI[1], 0, 0, 0);
      }
    } else if constexpr (PREC == 0) {
      const uint8_t* p = cur + (rh * 32 + ra) * XM_CHUNK + wave * 16;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float4 q = *reinterpret_cast<const float4*>(p + t * 128);
        // channel 2*wave: (q.x, q.y); channel 2*wave+1: (q.z, q.w)
        accR[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(q.x, q.x, accR[0], 0, 0, 0);
        accR[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(q.y, q.y, accR[0], 0, 0, 0);
        accI[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(q.y, q.x, accI[0], 0, 0, 0);
        accR[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(q.z, q.z, accR[1], 0, 0, 0);
        accR[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(q.w, q.w, accR[1], 0, 0, 0);
        accI[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(q.w, q.z, accI[1], 0, 0, 0);
      }
    } else if constexpr (PREC == 3) {
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const uint8_t* p = cur + (g * 32 + ra) * XM_CHUNK + (8 * rh) * 64 + wave * 8;
        uint2 raw[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) raw[q] = *reinterpret_cast<const uint2*>(p + q * 64);
#pragma unroll
        for (int e = 0; e < 4; ++e) gram8(raw, e, accR[e], accI[e]);
      }
    } else {
      const uint8_t* p = cur + (rh * 32 + ra) * XM_CHUNK + wave * 16;
      uint4 raw[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) raw[q] = *reinterpret_cast<const uint4*>(p + q * 128);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        uint32_t w[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) w[q] = e == 0 ? raw[q].x : e == 1 ? raw[q].y : e == 2 ? raw[q].z : raw[q].w;
        gram16<PREC>(w, accR[e], accI[e]);
      }
    }
  };
  // wait for the current stage, release the other buffer, refill it, compute
  auto step = [&](uint8_t* cur, uint8_t* nxt, int64_t s) {
    wait_vmem_all();
    __syncthreads();
    const int64_t m0 = m_lo + s * C::KS;
    if (m0 + C::KS > m_hi) {
      zero_tail(cur, m0);
      __syncthreads();
    }
    if (s + 1 < n_st) issue(nxt, m0 + C::KS);
    compute(cur);
  };

  if (n_st > 0) issue(st0, m_lo);
  int64_t s = 0;
  for (; s + 1 < n_st; s += 2) {
    step(st0, st1, s);
    step(st1, st0, s + 1);
  }
  if (s < n_st) step(st0, st1, s);  // odd count: the last stage sits in st0

  // Output: the block's [baseline][CB channels] tile is assembled in LDS
  // (rows of baselines < XM_HALF in st0, the rest in st1; each row padded
  // by 8 bytes so that the lanes of one Gram row, which hold consecutive
  // baselines, write different banks) and leaves as one contiguous run:
  // partials are tile-major, [dz][n_chan / CB][nb][CB].
  const int nb = n_ant * (n_ant + 1) / 2;
  float2* out = part + dz * (int64_t)nb * n_chan + (int64_t)cb * nb * C::CB;
  const int j = lane & (C::TA - 1);
  constexpr int PITCH = C::CB * 8 + 8;                  // bytes per staged row
  constexpr int TOFF = C::F32 ? XM_PTILES : 0;          // float32: P tiles first
  auto trow = [&](int b) -> float2* {
    uint8_t* base = b < XM_HALF ? st0 : st1;
    return reinterpret_cast<float2*>(base + TOFF + (b < XM_HALF ? b : b - XM_HALF) * PITCH);
  };
  __syncthreads();  // all waves are done reading the stages
  if constexpr (C::F32) {
    // Im = P - P^T: every wave puts its P tiles in LDS (channel 0 in st0,
    // channel 1 in st1; [wave][i][j] with a padded row of TA + 1 floats)
    constexpr int PP = C::TA + 1;
    float* pt0 = reinterpret_cast<float*>(st0) + wave * XM_PT;
    float* pt1 = reinterpret_cast<float*>(st1) + wave * XM_PT;
#pragma unroll
    for (int r = 0; r < C::ACC; ++r) {
      const int i = acc_row<C::TA>(lane, r);
      pt0[i * PP + j] = accI[0][r];
      pt1[i * PP + j] = accI[1][r];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const float* pt = c ? pt1 : pt0;
#pragma unroll
      for (int r = 0; r < C::ACC; ++r) {
        const int i = acc_row<C::TA>(lane, r);
        if (i <= j && j < n_ant) {
          const int b = i * n_ant - i * (i - 1) / 2 + (j - i);
          const float im = i == j ? 0.f : accI[c][r] - pt[j * PP + i];
          trow(b)[2 * wave + c] = make_float2(accR[c][r], im);
        }
      }
    }
  } else {
    // unscaled by 1/(s_i s_j)
    const float inv_j = j < n_ant ? 1.0f / scale[j] : 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int r = 0; r < C::ACC; ++r) {
        const int i = acc_row<C::TA>(lane, r);
        if (i <= j && j < n_ant) {
          const float inv = (1.0f / scale[i]) * inv_j;
          const int b = i * n_ant - i * (i - 1) / 2 + (j - i);
          trow(b)[4 * wave + c] = make_float2(accR[c][r] * inv, i == j ? 0.f : accI[c][r] * inv);
        }
      }
    }
  }
  __syncthreads();
  for (int q = tid; q < nb * C::CB; q += XM_NT) st_f2<WT>(&out[q], trow(q / C::CB)[q % C::CB]);
}

}  // namespace

}  // namespace qc
