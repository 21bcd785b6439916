// X-engine on the gfx950 matrix cores.
//
// The X-engine of arXiv 2604.20640 (Sec. 4.1 eq. 1; Sec. 4.2) forms
// V_ij[k] = sum_m X_i,m[k] conj(X_j,m[k]).  Per channel this is a complex
// Gram matrix G = X X^H of the (antenna x spectrum) matrix X = A + iB:
//   Re G = A A^T + B B^T,   Im G = B A^T - A B^T.
// With antennas as rows and spectra as the reduction dimension, each term
// is a real 32x32xK product; A (or B) serves as both the left and the right
// MFMA operand because the gfx950 32x32 operand layouts coincide (lane l
// holds row/column l%32 and a run of reduction slots chosen by l/32).
//
// Precisions:
//   * float32 (complex64 input): v_mfma_f32_32x32x2_f32, three products per
//     pair of spectra: A A^T + B B^T into Re, P = B A^T into P; at the end
//     Im = P - P^T (AB^T = (BA^T)^T), the transpose taken through LDS.  Up
//     to 16 antennas the same on 16 x 16 tiles with v_mfma_f32_16x16x4_f32
//     (a quarter of the matrix work);
//   * FP16 / BF16 / OCP E4M3 (power-of-two per-antenna scales s_a):
//     v_mfma_f32_32x32x16_{f16,bf16,fp8_fp8}, four products per 16 spectra
//     (the subtraction uses a sign-flipped A), FP32 accumulation; the result
//     is divided exactly by s_i s_j.
//
// Staging: a workgroup of 8 waves owns CB channels (16 for float32, 32
// otherwise) and a run of spectra.  The input is read as (antenna, spectrum)
// rows of CB channels (128 bytes; 64 for E4M3) by direct global -> LDS
// loads (global_load_lds_dwordx4: no registers hold data in flight), in
// stages of 64 KiB, double-buffered: the loads of stage s+1 are in flight
// while the matrix cores consume stage s.  Each 1 KiB group of 64 lanes'
// loads lands as one LDS chunk; which rows go into which chunk is chosen so
// that a lane's operand reads are contiguous runs, and chunks are padded by
// 16 bytes so that consecutive antennas' operand reads fall in different
// banks.  The two stage buffers are distinct LDS objects and the loop is
// unrolled by two, so the compiler can tell that operand reads of one stage
// never alias the loads in flight into the other, and waits only where the
// code says so.  At the end each block's partial visibilities are assembled
// in the freed stage buffers as [baseline][CB channels] rows and written as
// whole rows.  n_ant <= 32, n_chan % CB == 0, v 16-byte aligned.
#include "qc_xmfma_body.h"

namespace qc {

template <int PREC>
__global__ void __launch_bounds__(XM_NT)
xeng_mfma_kernel(const void* __restrict__ vin, const float* __restrict__ scale, int n_ant,
                 int64_t n_spec, int n_chan, int64_t spec_per_dump, int64_t ksplit, int n_cb,
                 float2* __restrict__ part) {
  // two distinct LDS objects: the compiler can tell the operand reads of
  // one stage from the loads in flight into the other
  __shared__ __attribute__((aligned(16))) uint8_t st0[XM_STAGE];
  __shared__ __attribute__((aligned(16))) uint8_t st1[XM_STAGE];
  xeng_mfma_body<PREC>(vin, scale, n_ant, n_spec, n_chan, spec_per_dump, ksplit, (int)(blockIdx.x % n_cb),
                       (int64_t)(blockIdx.x / n_cb), part, st0, st1);
}

namespace {

constexpr int xm_cb(int prec) { return prec == 0 || prec == 4 ? 16 : 32; }
constexpr int xm_ks(int prec) { return prec == 3 || prec == 4 ? 32 : 16; }
constexpr int xm_ta(int prec) { return prec == 4 ? 16 : XM_NA; }

// Splits of each dump's stages so that the grid holds about one workgroup
// per CU (one is resident at a time: 136 KiB of LDS) with at least four
// stages each; fewer splits also mean fewer partials to reduce.
int64_t xm_ksplit(int prec, int n_ant, int64_t spd, int n_chan, int64_t n_dump) {
  if (n_ant < 1 || n_ant > xm_ta(prec) || n_chan % xm_cb(prec) != 0) return 0;
  const int64_t blocks = (int64_t)(n_chan / xm_cb(prec)) * n_dump;
  int64_t ks = (256 + blocks - 1) / blocks;
  const int64_t nst = (spd + xm_ks(prec) - 1) / xm_ks(prec);
  const int64_t maxk = nst / 4 > 0 ? nst / 4 : 1;
  if (ks > maxk) ks = maxk;
  return ks < 1 ? 1 : ks;
}

template <int PREC>
hipError_t launch_xm_t(const void* v, const float* scale, int n_ant, int64_t n_spec, int n_chan,
                       int64_t spd, int64_t n_dump, int64_t ksplit, float2* part, hipStream_t s) {
  const int n_cb = n_chan / XmCfg<PREC>::CB;
  const int64_t blocks = (int64_t)n_cb * n_dump * ksplit;
  if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  return launch(xeng_mfma_kernel<PREC>, dim3((unsigned)blocks), dim3(XM_NT), 0, s, v, scale, n_ant, n_spec,
                n_chan, spd, ksplit, n_cb, part);
}

}  // namespace

int64_t xeng_mfma_ksplit(int prec, int n_ant, int64_t spd, int n_chan, int64_t n_dump) {
  return prec >= 1 && prec <= 3 ? xm_ksplit(prec, n_ant, spd, n_chan, n_dump) : 0;
}

hipError_t launch_xeng_mfma(const void* v, int prec, const float* scale, int n_ant, int64_t n_spec,
                            int n_chan, int64_t spd, int64_t n_dump, int64_t ksplit, float2* part,
                            hipStream_t s) {
  if (n_ant < 1 || n_ant > XM_NA || n_chan % 32 != 0 || (reinterpret_cast<uintptr_t>(v) & 15u))
    return hipErrorInvalidValue;
  switch (prec) {
    case 1: return launch_xm_t<1>(v, scale, n_ant, n_spec, n_chan, spd, n_dump, ksplit, part, s);
    case 2: return launch_xm_t<2>(v, scale, n_ant, n_spec, n_chan, spd, n_dump, ksplit, part, s);
    case 3: return launch_xm_t<3>(v, scale, n_ant, n_spec, n_chan, spd, n_dump, ksplit, part, s);
  }
  return hipErrorInvalidValue;
}

bool xeng_f32_mfma_supported(int n_ant, int n_chan, const void* v) {
  return n_ant >= 1 && n_ant <= XM_NA && n_chan % 16 == 0 && (reinterpret_cast<uintptr_t>(v) & 15u) == 0;
}

// float32: 16 x 16 tiles (a quarter of the matrix work) up to 16 antennas
static int xm_f32_code(int n_ant) { return n_ant <= 16 ? 4 : 0; }

int64_t xeng_f32_mfma_ksplit(int n_ant, int64_t spd, int n_chan, int64_t n_dump) {
  return xm_ksplit(xm_f32_code(n_ant), n_ant, spd, n_chan, n_dump);
}

hipError_t launch_xeng_f32_mfma(const float2* v, int n_ant, int64_t n_spec, int n_chan, int64_t spd,
                                int64_t n_dump, int64_t ksplit, float2* part, hipStream_t s) {
  if (!xeng_f32_mfma_supported(n_ant, n_chan, v)) return hipErrorInvalidValue;
  if (xm_f32_code(n_ant) == 4)
    return launch_xm_t<4>(v, nullptr, n_ant, n_spec, n_chan, spd, n_dump, ksplit, part, s);
  return launch_xm_t<0>(v, nullptr, n_ant, n_spec, n_chan, spd, n_dump, ksplit, part, s);
}

}  // namespace qc
