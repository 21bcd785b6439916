// F-engine and X-engine kernels for gfx950.
//
// Method (arXiv 2604.20640): Sec. 4.1 steps 1 and 3 with eq. (1); Sec. 4.2
// "F-engine (PFB and FFT)" and "X-engine and integration"; Alg. 1 F-Engine,
// X-Engine and Integration steps.
//
// F-engine: y_m[n] = sum_p h[pN+n] x[(m-P+1+p)N + n] (polyphase FIR), then an
// N-point real DFT.  Two antennas a, b share one complex transform:
// z = y_a + i y_b, Z = FFT(z), and
//   Y_a[k] = (Z[k] + conj Z[N-k]) / 2,  Y_b[k] = (Z[k] - conj Z[N-k]) / (2i).
// The factor 1/2 is applied as an exact power-of-two scale at the end.
//
// X-engine: V_ij[k] += Y_i[k] conj(Y_j[k]) for i <= j; autos keep an exactly
// zero imaginary part.  Integration is a plain sum over a dump's spectra.
// Each workgroup accumulates a contiguous run of spectra in registers and
// writes one partial; partials are summed in a fixed order (deterministic,
// no floating-point atomics).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <atomic>
#include <type_traits>

#include "qc_fft.h"
#include "qc_kernels.h"
#include "qc_xmfma_body.h"

namespace qc {

// ==== fused F+X kernels ====================================================

// ---------------------------------------------------------------------------
// int8 block loads (4 consecutive samples as one dword)
// ---------------------------------------------------------------------------
// Stream block `blk` of antenna `a`, samples n0..n0+3.  Blocks before the
// stream come from `hist` ((P-1) blocks per antenna) or are zero.
__device__ __forceinline__ uint32_t load_x4(const int8_t* __restrict__ x, int64_t ld_x,
                                            const int8_t* __restrict__ hist, int a, int64_t blk,
                                            int n0, int N, int P) {
  if (blk >= 0) {
    return *reinterpret_cast<const uint32_t*>(x + (int64_t)a * ld_x + blk * N + n0);
  }
  if (hist == nullptr) return 0u;
  const int64_t hb = blk + (P - 1);  // 0 .. P-2
  return *reinterpret_cast<const uint32_t*>(hist + ((int64_t)a * (P - 1) + hb) * N + n0);
}

__device__ __forceinline__ float sbyte(uint32_t w, int i) {
  return (float)(int8_t)((w >> (8 * i)) & 0xffu);
}

// An empty asm that reads and writes the K 32-bit words: loads into them
// complete here.  Used on a register ring before its loop, so that the loop holds
// no wait for loads issued before it (the compiler otherwise places such a
// wait inside the loop, where it also waits for the loop's own memory
// operations).
template <int K, typename T>
__device__ __forceinline__ void settle_words(T* w) {
#pragma unroll
  for (int i = 0; i < K; ++i) asm volatile("" : "+v"(w[i]));
}

// Ring words: four consecutive samples of one input row as loaded (Sec. 3.3
// quantisation modes).  Real words (int8, int16) fill two antennas per
// packed transform; complex words (I, Q interleaved int8 or int16) fill
// one antenna per transform, I as the real and Q as the imaginary part.
template <int ST> struct RingWord;
template <> struct RingWord<0> { using T = uint32_t; static constexpr int BYTES = 1; static constexpr bool CPLX = false; };
template <> struct RingWord<1> { using T = uint2; static constexpr int BYTES = 2; static constexpr bool CPLX = false; };
template <> struct RingWord<2> { using T = uint2; static constexpr int BYTES = 2; static constexpr bool CPLX = true; };
template <> struct RingWord<3> { using T = uint4; static constexpr int BYTES = 4; static constexpr bool CPLX = true; };

__device__ __forceinline__ float s16(uint32_t w, int hi) {
  return (float)(int16_t)(hi ? (w >> 16) : (w & 0xffffu));
}
// Sample i of a ring word: the real value (real words) or I (complex).
template <int ST, class T>
__device__ __forceinline__ float word_re(const T& w, int i) {
  if constexpr (ST == 0) return sbyte(w, i);
  else if constexpr (ST == 1) return s16(i < 2 ? w.x : w.y, i & 1);
  else if constexpr (ST == 2) return sbyte(i < 2 ? w.x : w.y, 2 * (i & 1));
  else return s16(i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w, 0);
}
// Q of sample i of a complex ring word.
template <int ST, class T>
__device__ __forceinline__ float word_im(const T& w, int i) {
  if constexpr (ST == 2) return sbyte(i < 2 ? w.x : w.y, 2 * (i & 1) + 1);
  else return s16(i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w, 1);
}
// An empty asm reading and writing a ring word (keeps its update in place).
__device__ __forceinline__ void pin_word(uint32_t& w) { asm volatile("" : "+v"(w)); }
__device__ __forceinline__ void pin_word(uint2& w) { asm volatile("" : "+v"(w.x), "+v"(w.y)); }
__device__ __forceinline__ void pin_word(uint4& w) {
  asm volatile("" : "+v"(w.x), "+v"(w.y), "+v"(w.z), "+v"(w.w));
}

// FIR for 4 consecutive samples n0..n0+3 of spectrum m, antennas a0 (real
// part) and a1 (imaginary part; a1 < 0 means none).
__device__ __forceinline__ void fir4(const int8_t* __restrict__ x, int64_t ld_x,
                                     const int8_t* __restrict__ hist,
                                     const float* __restrict__ taps, int a0, int a1, int64_t m,
                                     int n0, int N, int P, float2 out[4]) {
  float y0[4] = {0.f, 0.f, 0.f, 0.f}, y1[4] = {0.f, 0.f, 0.f, 0.f};
  for (int q = 0; q < P; ++q) {
    const int64_t blk = m - P + 1 + q;
    const float4 h = *reinterpret_cast<const float4*>(taps + (int64_t)q * N + n0);
    const uint32_t w0 = load_x4(x, ld_x, hist, a0, blk, n0, N, P);
    y0[0] += h.x * sbyte(w0, 0);
    y0[1] += h.y * sbyte(w0, 1);
    y0[2] += h.z * sbyte(w0, 2);
    y0[3] += h.w * sbyte(w0, 3);
    if (a1 >= 0) {
      const uint32_t w1 = load_x4(x, ld_x, hist, a1, blk, n0, N, P);
      y1[0] += h.x * sbyte(w1, 0);
      y1[1] += h.y * sbyte(w1, 1);
      y1[2] += h.z * sbyte(w1, 2);
      y1[3] += h.w * sbyte(w1, 3);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) out[i] = make_float2(y0[i], y1[i]);
}

// Separate one packed transform into its two real-input spectra (times 2).
__device__ __forceinline__ void separate(float2 zk, float2 zn, float2& ya, float2& yb) {
  ya = make_float2(zk.x + zn.x, zk.y - zn.y);
  yb = make_float2(zk.y + zn.y, zn.x - zk.x);
}

// ---------------------------------------------------------------------------
// Fused F+X: NA antennas (NP = ceil(NA/2) packed transforms), S spectra in
// flight, V complex values per thread per FFT pass (NT = NP*S*N/V threads),
// optional ping-pong LDS buffers (PP) and a compile-time tap count (P > 0;
// P = 0 reads it at run time).  Grid: n_dump * chunks_per_dump blocks.
// ---------------------------------------------------------------------------
template <int N, int NA, int S, int V, bool PP, int OCC = 0>
struct FusedCfg {
  static constexpr int NP = (NA + 1) / 2;
  static constexpr int NFFT = NP * S;
  static constexpr int NT = NFFT * N / V;
  static constexpr int NCH = N / 2;
  static constexpr int NB = NA * (NA + 1) / 2;
  static constexpr int CPT = (NCH + NT - 1) / NT;
  static constexpr int BUF = lds_padded_size(NFFT * N);
  static constexpr int LDS = (PP ? 2 : 1) * BUF;
  static constexpr int CHUNKS = V / 4;  // FIR chunks of 4 samples per thread
  // hide loop-invariant address/twiddle work from hoisting when the
  // register budget is 128 per lane or less
  static constexpr bool LN = NT >= 1024 || OCC >= 4;
};

// FIR for 4 consecutive samples of antennas a0 (real part) and a1 (imaginary
// part; none when a1 < 0), stream block blk0 = m - P + 1 of spectrum m.
template <int PT>
__device__ __forceinline__ void fir4_t(const int8_t* __restrict__ xa0, const int8_t* __restrict__ xa1,
                                       const int8_t* __restrict__ ha0, const int8_t* __restrict__ ha1,
                                       const float* __restrict__ taps, int P_rt, int64_t blk0, int n0,
                                       int N, float2 out[4]) {
  const int P = PT > 0 ? PT : P_rt;
  float y0[4] = {0.f, 0.f, 0.f, 0.f}, y1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < (PT > 0 ? PT : 16); ++q) {
    if (PT == 0 && q >= P) break;
    const int64_t blk = blk0 + q;
    const float4 h = *reinterpret_cast<const float4*>(taps + q * N + n0);
    uint32_t w0, w1 = 0u;
    if (blk >= 0) {
      const int off = (int)blk * N + n0;
      w0 = *reinterpret_cast<const uint32_t*>(xa0 + off);
      if (xa1) w1 = *reinterpret_cast<const uint32_t*>(xa1 + off);
    } else if (ha0) {
      const int off = (int)(blk + (P - 1)) * N + n0;
      w0 = *reinterpret_cast<const uint32_t*>(ha0 + off);
      if (ha1) w1 = *reinterpret_cast<const uint32_t*>(ha1 + off);
    } else {
      w0 = 0u;
    }
    y0[0] += h.x * sbyte(w0, 0);
    y0[1] += h.y * sbyte(w0, 1);
    y0[2] += h.z * sbyte(w0, 2);
    y0[3] += h.w * sbyte(w0, 3);
    y1[0] += h.x * sbyte(w1, 0);
    y1[1] += h.y * sbyte(w1, 1);
    y1[2] += h.z * sbyte(w1, 2);
    y1[3] += h.w * sbyte(w1, 3);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) out[i] = make_float2(y0[i], y1[i]);
}

// Body of the fused kernel for work unit w (chunk w % cpd of dump w / cpd),
// run by all C::NT threads of a block on the LDS region buf.
template <int N, int NA, int S, int V, bool PP, int OCC, int PT, bool WT = false>
__device__ __forceinline__ void fused_body(const int8_t* __restrict__ x, int64_t ld_x,
                                           const int8_t* __restrict__ hist,
                                           const float* __restrict__ taps, int P_rt,
                                           const float2* __restrict__ tw, int64_t spec_per_dump,
                                           int64_t cpd, float2* __restrict__ part, int64_t w,
                                           float2* buf) {
  using C = FusedCfg<N, NA, S, V, PP, OCC>;
  using F = Fft<N, C::NT, V, PP, C::LN>;
  float2* b0 = buf;
  float2* b1 = buf + (PP ? C::BUF : 0);
  const float2* bout = F::OUT ? b1 : b0;
  const int P = PT > 0 ? PT : P_rt;
  const int64_t d = w / cpd, c = w % cpd;
  const int64_t m_lo = d * spec_per_dump + (c * spec_per_dump) / cpd;
  const int64_t m_hi = d * spec_per_dump + ((c + 1) * spec_per_dump) / cpd;

  float2 acc[C::CPT][C::NB];
#pragma unroll
  for (int cc = 0; cc < C::CPT; ++cc)
#pragma unroll
    for (int b = 0; b < C::NB; ++b) acc[cc][b] = make_float2(0.f, 0.f);

  for (int64_t m0 = m_lo; m0 < m_hi; m0 += S) {
    int tid = threadIdx.x;  // per iteration: see the note in stockham_pass
    if constexpr (C::LN) asm volatile("" : "+v"(tid));
    // polyphase FIR into the packed transform inputs (buffer 0); one chunk
    // at a time keeps the tap and sample registers of only one chunk live
#pragma unroll 1
    for (int g = 0; g < C::CHUNKS; ++g) {
      const int c4 = tid + g * C::NT;
      const int f = c4 / (N / 4);
      const int n0 = 4 * (c4 % (N / 4));
      const int s = f / C::NP, p = f % C::NP;
      const int64_t m = m0 + s;
      const int a0 = 2 * p, a1 = (2 * p + 1 < NA) ? 2 * p + 1 : -1;
      float2 y[4];
      if (m < m_hi) {
        const int8_t* xa0 = x + (int64_t)a0 * ld_x;
        const int8_t* xa1 = a1 >= 0 ? x + (int64_t)a1 * ld_x : nullptr;
        const int8_t* ha0 = hist ? hist + (int64_t)a0 * (P - 1) * N : nullptr;
        const int8_t* ha1 = (hist && a1 >= 0) ? hist + (int64_t)a1 * (P - 1) * N : nullptr;
        fir4_t<PT>(xa0, xa1, ha0, ha1, taps, P, m - P + 1, n0, N, y);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] = make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) b0[lds_pad(f * N + n0 + i)] = y[i];
    }
    __syncthreads();
    F::run(b0, b1, tw, tid);
    // separate and cross-multiply
#pragma unroll
    for (int cc = 0; cc < C::CPT; ++cc) {
      const int k = tid + cc * C::NT;
      if (C::NCH % C::NT == 0 || k < C::NCH) {
        const int kn = (N - k) & (N - 1);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          if (m0 + s < m_hi) {
            float2 X[2 * C::NP];
#pragma unroll
            for (int p = 0; p < C::NP; ++p) {
              const float2 zk = bout[lds_pad((s * C::NP + p) * N + k)];
              const float2 zn = bout[lds_pad((s * C::NP + p) * N + kn)];
              separate(zk, zn, X[2 * p], X[2 * p + 1]);
            }
            int b = 0;
#pragma unroll
            for (int i = 0; i < NA; ++i) {
              acc[cc][b].x += X[i].x * X[i].x + X[i].y * X[i].y;
              ++b;
#pragma unroll
              for (int j = i + 1; j < NA; ++j) {
                acc[cc][b].x += X[i].x * X[j].x + X[i].y * X[j].y;
                acc[cc][b].y += X[i].y * X[j].x - X[i].x * X[j].y;
                ++b;
              }
            }
          }
        }
      }
    }
    // with an in-place transform (or an output in buffer 0) the next FIR
    // overwrites what was just read; with the output in buffer 1 the next
    // FIR writes buffer 0, last read before the final pass's barrier
    if constexpr (F::OUT == 0) __syncthreads();
  }
  float2* out = part + w * (int64_t)C::NB * C::NCH;
#pragma unroll
  for (int cc = 0; cc < C::CPT; ++cc) {
    const int k = (int)threadIdx.x + cc * C::NT;
    if (C::NCH % C::NT == 0 || k < C::NCH) {
#pragma unroll
      for (int b = 0; b < C::NB; ++b) st_f2<WT>(&out[(int64_t)b * C::NCH + k], acc[cc][b]);
    }
  }
}

template <int N, int NA, int S, int V, bool PP, int OCC, int PT>
__global__ void __launch_bounds__((FusedCfg<N, NA, S, V, PP, OCC>::NT), (OCC > 0 ? OCC : 1))
fx_fused_kernel(const int8_t* __restrict__ x, int64_t ld_x, const int8_t* __restrict__ hist,
                const float* __restrict__ taps, int P_rt, const float2* __restrict__ tw,
                int64_t spec_per_dump, int64_t cpd, float2* __restrict__ part) {
  extern __shared__ float2 buf[];
  fused_body<N, NA, S, V, PP, OCC, PT>(x, ld_x, hist, taps, P_rt, tw, spec_per_dump, cpd, part,
                                        (int64_t)blockIdx.x, buf);
}

// Ring variant of the fused kernel (one spectrum in flight, compile-time P):
// each thread keeps its samples of the last P blocks in a register ring and
// prefetches the next block at the start of every spectrum, so the newest
// block's memory latency is hidden behind the FFT and X steps; the taps are
// read from LDS (loaded once per workgroup).  Sums are the same as the plain
// variant's.
template <int N, int NA, int V, int P>
struct RingCfg {
  using C = FusedCfg<N, NA, 1, V, false, 0>;
  static constexpr int TAPS = P * N / 2;  // floats: half of a symmetric prototype
  static constexpr size_t LDS_BYTES =
      sizeof(float2) * (C::LDS + N) + sizeof(float) * TAPS;  // FFT, twiddles, taps
};

// ST selects the input word (real int8 or real int16, Sec. 3.3).  With
// int16 words the ring is twice as wide, so the taps are read from LDS at
// each use instead of being held in registers.
template <int N, int NA, int V, int P, int ST = 0>
__global__ void __launch_bounds__((FusedCfg<N, NA, 1, V, false, 0>::NT))
fx_fused_ring_kernel(const int8_t* __restrict__ x, int64_t ld_x, const int8_t* __restrict__ hist,
                     const float* __restrict__ taps, const float2* __restrict__ tw,
                     int64_t spec_per_dump, int64_t cpd, float2* __restrict__ part) {
  using C = FusedCfg<N, NA, 1, V, false, 0>;
  using F = Fft<N, C::NT, V, false, false, true>;
  using W = RingWord<ST>;
  using T = typename W::T;
  static_assert(!W::CPLX, "real words: two antennas per packed transform");
  constexpr bool TAPS_IN_REGS = ST == 0;
  constexpr int G = C::CHUNKS;
  constexpr int L = P * N;
  extern __shared__ float2 buf[];
  float2* b0 = buf;
  float2* twl = buf + C::LDS;                             // per-pass twiddles, N-1
  float4* tl = reinterpret_cast<float4*>(twl + N);        // taps h[0 .. L/2)
  const int tid = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int64_t d = w / cpd, c = w % cpd;
  const int64_t m_lo = d * spec_per_dump + (c * spec_per_dump) / cpd;
  const int64_t m_hi = d * spec_per_dump + ((c + 1) * spec_per_dump) / cpd;

  // the prototype is symmetric, h[q] = h[L-1-q]: keep its first half
  for (int i = tid; i < L / 8; i += C::NT) tl[i] = reinterpret_cast<const float4*>(taps)[i];
  build_pass_twiddles<N, V>(twl, tw, tid, C::NT);

  // this thread's FIR chunks: chunk g belongs to packed pair g / GP (a
  // compile-time constant), so the antenna rows are wave-uniform and only
  // the sample offset n0 varies per lane
  constexpr int GP = G / C::NP;
  static_assert(GP * C::NP == G && GP * C::NT * 4 == N, "ring chunk mapping");
  int cn0[G];
#pragma unroll
  for (int g = 0; g < G; ++g) cn0[g] = 4 * (tid + (g % GP) * C::NT);
  auto row = [&](int a) -> const int8_t* { return x + (int64_t)a * ld_x * W::BYTES; };
  auto hrow = [&](int a) -> const int8_t* {
    return hist ? hist + (int64_t)a * (P - 1) * N * W::BYTES : nullptr;
  };
  auto load_blk = [&](int g, int which, int64_t blk) -> T {
    const int a = 2 * (g / GP) + which;
    if (a >= NA) return T{};
    if (blk >= 0) return *reinterpret_cast<const T*>(row(a) + ((int)blk * N + cn0[g]) * W::BYTES);
    const int8_t* h = hrow(a);
    if (!h) return T{};
    return *reinterpret_cast<const T*>(h + ((int)(blk + P - 1) * N + cn0[g]) * W::BYTES);
  };
  // Prefetch of stream block nb >= 0 for the next spectrum (block m again
  // on the last one, its value then unused).  The load is unconditional so
  // the loop body stays one basic block and the wait for it falls at the
  // end of the iteration, not inside the FIR.
  auto load_next = [&](int g, int which, int nb) -> T {
    const int a = 2 * (g / GP) + which;
    return a < NA ? *reinterpret_cast<const T*>(row(a) + (nb * N + cn0[g]) * W::BYTES) : T{};
  };
  T ring[P][G][2];
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t blk = m_lo - P + 1 + q;
      ring[q][g][0] = load_blk(g, 0, blk);
      ring[q][g][1] = load_blk(g, 1, blk);
    }

  float2 acc[C::CPT][C::NB];
#pragma unroll
  for (int cc = 0; cc < C::CPT; ++cc)
#pragma unroll
    for (int b = 0; b < C::NB; ++b) acc[cc][b] = make_float2(0.f, 0.f);
  __syncthreads();  // taps in LDS
  // tap q at the thread's chunk position gp (chunks g and g + GP share one)
  auto tap = [&](int gp, int q) -> float4 {
    if (2 * q < P) return tl[(q * N + cn0[gp]) / 4];
    const float4 r = tl[(L - q * N - cn0[gp] - 4) / 4];
    return make_float4(r.w, r.z, r.y, r.x);
  };
  // with int8 words the taps stay in registers for the whole run
  float4 hr[TAPS_IN_REGS ? GP : 1][P];
  if constexpr (TAPS_IN_REGS) {
#pragma unroll
    for (int g = 0; g < GP; ++g)
#pragma unroll
      for (int q = 0; q < P; ++q) hr[g][q] = tap(g, q);
  }

  settle_words<P * G * 2 * (int)(sizeof(T) / 4)>(reinterpret_cast<uint32_t*>(&ring[0][0][0]));
  for (int64_t m = m_lo; m < m_hi; ++m) {
    // prefetch block m+1 (consumed at the end of this iteration); int16
    // words issue it after the FIR, whose registers it would otherwise
    // share with the wider ring
    T nxt[G][2];
    const int nb = (int)(m + 1 < m_hi ? m + 1 : m);
    auto prefetch = [&]() {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        nxt[g][0] = load_next(g, 0, nb);
        nxt[g][1] = load_next(g, 1, nb);
      }
    };
    if constexpr (ST == 0) prefetch();
    // polyphase FIR from the ring
#pragma unroll
    for (int g = 0; g < G; ++g) {
      float y0[4] = {0.f, 0.f, 0.f, 0.f}, y1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < P; ++q) {
        float4 h;
        if constexpr (TAPS_IN_REGS) h = hr[g % GP][q];
        else h = tap(g % GP, q);
        const float hv[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          y0[i] += hv[i] * word_re<ST>(ring[q][g][0], i);
          y1[i] += hv[i] * word_re<ST>(ring[q][g][1], i);
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) b0[lds_pad((g / GP) * N + cn0[g] + i)] = make_float2(y0[i], y1[i]);
    }
    if constexpr (ST != 0) prefetch();
    __syncthreads();
    F::run(b0, b0, twl, tid);
    static_assert(C::NCH % C::NT == 0, "every thread has CPT channels");
    // all of the thread's transform outputs are read before any is used
    float2 zk[C::CPT][C::NP], zn[C::CPT][C::NP];
#pragma unroll
    for (int cc = 0; cc < C::CPT; ++cc) {
      const int k = tid + cc * C::NT;
      const int kn = (N - k) & (N - 1);
#pragma unroll
      for (int p = 0; p < C::NP; ++p) {
        zk[cc][p] = b0[lds_pad(p * N + k)];
        zn[cc][p] = b0[lds_pad(p * N + kn)];
      }
    }
#pragma unroll
    for (int cc = 0; cc < C::CPT; ++cc) {
      float2 X[2 * C::NP];
#pragma unroll
      for (int p = 0; p < C::NP; ++p) separate(zk[cc][p], zn[cc][p], X[2 * p], X[2 * p + 1]);
      int b = 0;
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        acc[cc][b].x += X[i].x * X[i].x + X[i].y * X[i].y;
        ++b;
#pragma unroll
        for (int j = i + 1; j < NA; ++j) {
          acc[cc][b].x += X[i].x * X[j].x + X[i].y * X[j].y;
          acc[cc][b].y += X[i].y * X[j].x - X[i].x * X[j].y;
          ++b;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q + 1 < P; ++q)
#pragma unroll
      for (int g = 0; g < G; ++g) {
        ring[q][g][0] = ring[q + 1][g][0];
        ring[q][g][1] = ring[q + 1][g][1];
      }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      ring[P - 1][g][0] = nxt[g][0];
      ring[P - 1][g][1] = nxt[g][1];
    }
  }
  float2* out = part + w * (int64_t)C::NB * C::NCH;
#pragma unroll
  for (int cc = 0; cc < C::CPT; ++cc) {
    const int k = tid + cc * C::NT;
#pragma unroll
    for (int b = 0; b < C::NB; ++b) out[(int64_t)b * C::NCH + k] = acc[cc][b];
  }
}

// Ping-pong ring variant.  Same sums as the ring variant; the transform
// passes alternate between two LDS buffers, so each pass ends with one
// barrier instead of two: four per spectrum (after the FIR and after each of
// the three passes; the next spectrum's FIR writes the buffer the last pass
// read, and its first pass writes the buffer the X step read, each behind a
// barrier).  Beside the two buffers, LDS holds the per-pass twiddle table up
// to the last pass's r = 8 (a prefix of the per-pass layout); the last
// pass forms W^{jm (8+q)} = W^{jm q} W^{8 jm} for q = 1..7 (seven complex
// products per spectrum, which keeps the whole working set within 160 KiB).
// The taps of a thread's chunk positions are read from global memory into
// registers once (any P = 4 prototype).
template <int N, int V>
struct PpTw {
  static constexpr int PASSES = fft_pass_count(N, V);
  static constexpr int last_ns() {
    int ns = 1;
    while (N / ns > fft_radix(N / ns, V)) ns *= fft_radix(N / ns, V);
    return ns;
  }
  static constexpr int NSL = last_ns();
  static constexpr int RLAST = N / NSL;
  static_assert(RLAST == 16, "the last pass has radix 16");
  // per-pass entries before the last pass, then the last pass's r = 1..8
  static constexpr int EARLY = (N - 1) - (RLAST - 1) * NSL;
  static constexpr int LDS_TW = EARLY + 8 * NSL;
};

// Last pass (stride NS, radix 16, one butterfly per thread) with the
// twiddles of r = 1..8 from the LDS table and r = 9..15 from products.
template <int N, int NS, int NT>
__device__ __forceinline__ void stockham_last_pass_half(const float2* src, float2* dst, const float2* twl,
                                                        int tid) {
  constexpr int R = 16;
  constexpr int NB = N / R;
  const int f = tid / NB, j = tid % NB;
  const int jm = j % NS;
  float2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = src[lds_pad(f * N + j + r * NB)];
  float2 w[R];
#pragma unroll
  for (int r = 1; r <= 8; ++r) w[r] = twl[(NS - 1) + (r - 1) * NS + jm];
#pragma unroll
  for (int q = 1; q < 8; ++q) w[8 + q] = cmul(w[q], w[8]);
#pragma unroll
  for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
  dft_r<R>(v);
  const int k = (j / NS) * NS * R + jm;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[lds_pad(f * N + k + r * NS)] = v[r];
  __syncthreads();
}

// TWG: table twiddles read in groups of TWG, 0 for one wait per read (see
// stockham_pass).
template <int N, int NS, int NT, int V, int PASS, int TWG = 4>
__device__ __forceinline__ void fft_pp_passes(float2* b0, float2* b1, const float2* twl, int tid) {
  constexpr int REM = N / NS;
  if constexpr (REM > 1) {
    constexpr int R = fft_radix(REM, V);
    float2* src = (PASS % 2 == 0) ? b0 : b1;
    float2* dst = (PASS % 2 == 0) ? b1 : b0;
    if constexpr (NS * R == N)
      stockham_last_pass_half<N, NS, NT>(src, dst, twl, tid);
    else
      stockham_pass<N, R, NS, NT, V, false, false, true, TWG>(src, dst, twl, tid);
    fft_pp_passes<N, NS * R, NT, V, PASS + 1, TWG>(b0, b1, twl, tid);
  }
}

template <int N, int NA, int V, int P>
struct RingPpCfg {
  using C = FusedCfg<N, NA, 1, V, false, 0>;
  static constexpr int BUF = C::BUF;  // padded buffer
  static constexpr size_t LDS_BYTES = sizeof(float2) * (2 * (size_t)BUF + PpTw<N, V>::LDS_TW);
};

template <int N, int NA, int V, int P>
__global__ void __launch_bounds__((FusedCfg<N, NA, 1, V, false, 0>::NT))
fx_fused_ring_pp_kernel(const int8_t* __restrict__ x, int64_t ld_x, const int8_t* __restrict__ hist,
                        const float* __restrict__ taps, const float2* __restrict__ twp,
                        int64_t spec_per_dump, int64_t cpd, float2* __restrict__ part) {
  using C = FusedCfg<N, NA, 1, V, false, 0>;
  using RC = RingPpCfg<N, NA, V, P>;
  static_assert(fft_pass_count(N, V) % 2 == 1, "odd pass count: the output lands in the second buffer");
  constexpr int G = C::CHUNKS;
  extern __shared__ float2 buf[];
  float2* b0 = buf;
  float2* b1 = buf + RC::BUF;
  float2* twl = buf + 2 * RC::BUF;  // per-pass twiddles up to the last pass's r = 8
  const int tid = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int64_t d = w / cpd, c = w % cpd;
  const int64_t m_lo = d * spec_per_dump + (c * spec_per_dump) / cpd;
  const int64_t m_hi = d * spec_per_dump + ((c + 1) * spec_per_dump) / cpd;

  for (int i = tid; i < PpTw<N, V>::LDS_TW; i += C::NT) twl[i] = twp[i];

  constexpr int GP = G / C::NP;
  static_assert(GP * C::NP == G && GP * C::NT * 4 == N, "ring chunk mapping");
  int cn0[G];
#pragma unroll
  for (int g = 0; g < G; ++g) cn0[g] = 4 * (tid + (g % GP) * C::NT);
  auto row = [&](int a) -> const int8_t* { return x + (int64_t)a * ld_x; };
  auto hrow = [&](int a) -> const int8_t* {
    return hist ? hist + (int64_t)a * (P - 1) * N : nullptr;
  };
  auto load_blk = [&](int g, int which, int64_t blk) -> uint32_t {
    const int a = 2 * (g / GP) + which;
    if (a >= NA) return 0u;
    if (blk >= 0) return *reinterpret_cast<const uint32_t*>(row(a) + (int)blk * N + cn0[g]);
    const int8_t* h = hrow(a);
    if (!h) return 0u;
    return *reinterpret_cast<const uint32_t*>(h + (int)(blk + P - 1) * N + cn0[g]);
  };
  // Prefetch of stream block nb >= 0 for the next spectrum (block m again
  // on the last one, its value then unused).  The load is unconditional so
  // the loop body stays one basic block and the wait for it falls at the
  // end of the iteration, not inside the FIR.
  auto load_next = [&](int g, int which, int nb) -> uint32_t {
    const int a = 2 * (g / GP) + which;
    return a < NA ? *reinterpret_cast<const uint32_t*>(row(a) + nb * N + cn0[g]) : 0u;
  };
  uint32_t ring[P][G][2];
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t blk = m_lo - P + 1 + q;
      ring[q][g][0] = load_blk(g, 0, blk);
      ring[q][g][1] = load_blk(g, 1, blk);
    }
  float4 hr[GP][P];
#pragma unroll
  for (int g = 0; g < GP; ++g)
#pragma unroll
    for (int q = 0; q < P; ++q) hr[g][q] = *reinterpret_cast<const float4*>(taps + q * N + cn0[g]);

  float2 acc[C::CPT][C::NB];
#pragma unroll
  for (int cc = 0; cc < C::CPT; ++cc)
#pragma unroll
    for (int b = 0; b < C::NB; ++b) acc[cc][b] = make_float2(0.f, 0.f);
  __syncthreads();  // twiddles in LDS

  settle_words<P * G * 2>(&ring[0][0][0]);
  settle_words<GP * P * 4>(&hr[0][0].x);
  for (int64_t m = m_lo; m < m_hi; ++m) {
    // prefetch block m+1 (consumed at the end of this iteration)
    uint32_t nxt[G][2];
    const int nb = (int)(m + 1 < m_hi ? m + 1 : m);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      nxt[g][0] = load_next(g, 0, nb);
      nxt[g][1] = load_next(g, 1, nb);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      float y0[4] = {0.f, 0.f, 0.f, 0.f}, y1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const float4 h = hr[g % GP][q];
        const uint32_t w0 = ring[q][g][0], w1 = ring[q][g][1];
        y0[0] += h.x * sbyte(w0, 0);
        y0[1] += h.y * sbyte(w0, 1);
        y0[2] += h.z * sbyte(w0, 2);
        y0[3] += h.w * sbyte(w0, 3);
        y1[0] += h.x * sbyte(w1, 0);
        y1[1] += h.y * sbyte(w1, 1);
        y1[2] += h.z * sbyte(w1, 2);
        y1[3] += h.w * sbyte(w1, 3);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) b0[lds_pad((g / GP) * N + cn0[g] + i)] = make_float2(y0[i], y1[i]);
    }
    __syncthreads();
    fft_pp_passes<N, 1, C::NT, V, 0>(b0, b1, twl, tid);
    static_assert(C::NCH % C::NT == 0, "every thread has CPT channels");
    // all of the thread's transform outputs are read before any is used, so
    // the reads overlap instead of each waiting for the one before
    float2 zk[C::CPT][C::NP], zn[C::CPT][C::NP];
#pragma unroll
    for (int cc = 0; cc < C::CPT; ++cc) {
      const int k = tid + cc * C::NT;
      const int kn = (N - k) & (N - 1);
#pragma unroll
      for (int p = 0; p < C::NP; ++p) {
        zk[cc][p] = b1[lds_pad(p * N + k)];
        zn[cc][p] = b1[lds_pad(p * N + kn)];
      }
    }
#pragma unroll
    for (int cc = 0; cc < C::CPT; ++cc) {
      {
        float2 X[2 * C::NP];
#pragma unroll
        for (int p = 0; p < C::NP; ++p) separate(zk[cc][p], zn[cc][p], X[2 * p], X[2 * p + 1]);
        int b = 0;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
          acc[cc][b].x += X[i].x * X[i].x + X[i].y * X[i].y;
          ++b;
#pragma unroll
          for (int j = i + 1; j < NA; ++j) {
            acc[cc][b].x += X[i].x * X[j].x + X[i].y * X[j].y;
            acc[cc][b].y += X[i].y * X[j].x - X[i].x * X[j].y;
            ++b;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q + 1 < P; ++q)
#pragma unroll
      for (int g = 0; g < G; ++g) {
        ring[q][g][0] = ring[q + 1][g][0];
        ring[q][g][1] = ring[q + 1][g][1];
      }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      ring[P - 1][g][0] = nxt[g][0];
      ring[P - 1][g][1] = nxt[g][1];
    }
  }
  float2* out = part + w * (int64_t)C::NB * C::NCH;
#pragma unroll
  for (int cc = 0; cc < C::CPT; ++cc) {
    const int k = tid + cc * C::NT;
    if (C::NCH % C::NT == 0 || k < C::NCH) {
#pragma unroll
      for (int b = 0; b < C::NB; ++b) out[(int64_t)b * C::NCH + k] = acc[cc][b];
    }
  }
}

template <int N, int NA, int V>
static hipError_t launch_fused_ring_pp(const FxArgs& a, int64_t n_dump, int64_t spd, int64_t cpd,
                                       float2* part, hipStream_t s) {
  using RC = RingPpCfg<N, NA, V, 4>;
  static_assert(RC::LDS_BYTES <= 160 * 1024, "ping-pong ring tile: LDS");
  if (a.n_taps != 4) return hipErrorInvalidValue;
  auto kern = fx_fused_ring_pp_kernel<N, NA, V, 4>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)RC::LDS_BYTES);
  if (e != hipSuccess) return e;
  if (!a.twp) return hipErrorInvalidValue;
  return launch(kern, dim3((unsigned)(n_dump * cpd)), dim3(RC::C::NT), RC::LDS_BYTES, s, a.x, a.ld_x, a.hist,
                a.taps, a.twp, spd, cpd, part);
}

template <int N, int NA, int V, int ST = 0>
static hipError_t launch_fused_ring(const FxArgs& a, int64_t n_dump, int64_t spd, int64_t cpd,
                                    float2* part, hipStream_t s) {
  using RC = RingCfg<N, NA, V, 4>;
  static_assert(RC::LDS_BYTES <= 160 * 1024, "ring tile: LDS");
  if (a.n_taps != 4) return hipErrorInvalidValue;
  auto kern = fx_fused_ring_kernel<N, NA, V, 4, ST>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)RC::LDS_BYTES);
  if (e != hipSuccess) return e;
  return launch(kern, dim3((unsigned)(n_dump * cpd)), dim3(RC::C::NT), RC::LDS_BYTES, s, a.x, a.ld_x, a.hist,
                a.taps, a.tw, spd, cpd, part);
}

template <int N, int NA, int S, int V, bool PP, int OCC, int PT>
static hipError_t launch_fused_t(const FxArgs& a, int64_t n_dump, int64_t spd, int64_t cpd,
                                 float2* part, hipStream_t s) {
  using C = FusedCfg<N, NA, S, V, PP, OCC>;
  const size_t lds = sizeof(float2) * C::LDS;
  auto kern = fx_fused_kernel<N, NA, S, V, PP, OCC, PT>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return launch(kern, dim3((unsigned)(n_dump * cpd)), dim3(C::NT), lds, s, a.x, a.ld_x, a.hist, a.taps,
                a.n_taps, a.tw, spd, cpd, part);
}

template <int N, int NA, int S, int V, bool PP, int OCC>
static hipError_t launch_fused_p(const FxArgs& a, int64_t n_dump, int64_t spd, int64_t cpd,
                                 float2* part, hipStream_t s) {
  using C = FusedCfg<N, NA, S, V, PP, OCC>;
  static_assert(C::NT >= 64 && C::NT <= 1024, "fused tile: threads per block");
  static_assert(C::LDS * sizeof(float2) <= 160 * 1024, "fused tile: LDS");
  if (a.n_taps == 4) return launch_fused_t<N, NA, S, V, PP, OCC, 4>(a, n_dump, spd, cpd, part, s);
  return launch_fused_t<N, NA, S, V, PP, OCC, 0>(a, n_dump, spd, cpd, part, s);
}

// Tile shapes of the fused kernel per (n_fft, n_ant): spectra in flight S,
// values per thread per FFT pass V, ping-pong LDS buffers PP.  Entry 0 is
// the default; the others are the candidates an autotuner may time.
struct FusedTile {
  int S, V;  // S = 0: ring variant (one spectrum in flight, register ring)
  bool PP;
  int OCC;  // minimum waves per SIMD requested from the compiler (0: none)
};

template <int N, int NA>
struct TileList {
  static constexpr int count = 0;
  static constexpr FusedTile tiles[1] = {{1, 16, false, 0}};
};
#define QC_TILES(NN, NAA, ...)                                                  \
  template <>                                                                   \
  struct TileList<NN, NAA> {                                                    \
    static constexpr FusedTile tiles[] = {__VA_ARGS__};                         \
    static constexpr int count = (int)(sizeof(tiles) / sizeof(tiles[0]));       \
  };
QC_TILES(4096, 4, {0, 16, false, 0}, {1, 16, false, 0}, {1, 16, true, 0}, {2, 16, false, 0},
         {1, 8, true, 0}, {1, 16, false, 4}, {0, 16, true, 0})
QC_TILES(1024, 4, {2, 16, true, 0}, {2, 16, false, 0}, {4, 16, false, 0}, {2, 8, true, 0},
         {1, 16, true, 4}, {2, 16, false, 4}, {0, 16, false, 0})
QC_TILES(2048, 4, {0, 16, false, 0}, {1, 16, true, 0}, {1, 16, false, 0}, {1, 16, false, 4},
         {1, 8, true, 0})
QC_TILES(512, 4, {4, 16, true, 0}, {4, 16, false, 0}, {2, 16, true, 4})
QC_TILES(1024, 8, {1, 16, true, 0}, {1, 8, true, 0})
QC_TILES(2048, 8, {1, 8, true, 0}, {1, 8, false, 0})
QC_TILES(1024, 2, {4, 16, true, 0}, {4, 16, false, 0}, {2, 16, true, 4})
QC_TILES(4096, 2, {0, 16, false, 0}, {1, 16, true, 0}, {1, 16, false, 0}, {1, 16, false, 4}, {0, 16, true, 0})
#undef QC_TILES

template <int N, int NA, int I>
static hipError_t dispatch_tile(int tile, const FxArgs& a, int64_t n_dump, int64_t spd, int64_t cpd,
                                float2* part, hipStream_t s) {
  if constexpr (I >= TileList<N, NA>::count) {
    return hipErrorInvalidValue;
  } else {
    if (tile == I) {
      constexpr FusedTile t = TileList<N, NA>::tiles[I];
      if constexpr (t.S == 0 && t.PP) {
        // ping-pong ring variant (one spectrum in flight): needs P = 4, any taps
        if (a.n_taps == 4) return launch_fused_ring_pp<N, NA, t.V>(a, n_dump, spd, cpd, part, s);
        return launch_fused_p<N, NA, 1, t.V, false, 0>(a, n_dump, spd, cpd, part, s);
      } else if constexpr (t.S == 0) {
        // ring variant (one spectrum in flight): needs P = 4 and the built-in
        // (symmetric) prototype
        if (a.n_taps == 4 && a.taps_symmetric)
          return launch_fused_ring<N, NA, t.V>(a, n_dump, spd, cpd, part, s);
        return launch_fused_p<N, NA, 1, t.V, false, 0>(a, n_dump, spd, cpd, part, s);
      } else {
        return launch_fused_p<N, NA, t.S, t.V, t.PP, t.OCC>(a, n_dump, spd, cpd, part, s);
      }
    }
    return dispatch_tile<N, NA, I + 1>(tile, a, n_dump, spd, cpd, part, s);
  }
}

template <int N, int NA>
static int tile_count() {
  return TileList<N, NA>::count;
}

int fused_tile_count(int n_fft, int n_ant) {
#define QC_CASE(NN, NAA) \
  if (n_fft == NN && n_ant == NAA) return tile_count<NN, NAA>();
  QC_CASE(4096, 4) QC_CASE(1024, 4) QC_CASE(2048, 4) QC_CASE(512, 4)
  QC_CASE(1024, 8) QC_CASE(2048, 8) QC_CASE(1024, 2) QC_CASE(4096, 2)
#undef QC_CASE
  return 0;
}

bool fused_supported(int n_fft, int n_ant) { return fused_tile_count(n_fft, n_ant) > 0; }

int device_cu_count() {
  static std::atomic<int> cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
  if (dev < 64) {
    const int c = cached[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) return 256;
  if (dev < 64) cached[dev].store(n, std::memory_order_relaxed);
  return n;
}

int64_t fused_chunks_per_dump(int n_fft, int n_ant, int64_t n_dump, int64_t spd, int64_t workgroups) {
  // the default of 512 is two rounds of workgroups over 256 CUs
  if (workgroups < 1) workgroups = 512;
  int64_t want = (workgroups + n_dump - 1) / n_dump;
  int64_t maxc = spd / 8 > 0 ? spd / 8 : 1;
  int64_t c = want < maxc ? want : maxc;
  return c < 1 ? 1 : c;
}

// Fused F+X of real int16 words (the 16-bit padded mode): the in-place ring
// tile, for the shapes that have one, with P = 4 and the built-in prototype.
bool fused_words_supported(int sample, int n_fft, int n_ant, int n_taps, bool taps_symmetric) {
  if (sample != 1 || n_taps != 4 || !taps_symmetric) return false;
  return (n_ant == 4 && (n_fft == 1024 || n_fft == 2048 || n_fft == 4096)) || (n_ant == 2 && n_fft == 4096);
}

hipError_t launch_fused_words(const FxArgs& a, int sample, int64_t n_dump, int64_t spd, int64_t cpd,
                              float2* part, hipStream_t s) {
  if (!fused_words_supported(sample, a.n_fft, a.n_ant, a.n_taps, a.taps_symmetric)) return hipErrorNotSupported;
  if (a.n_ant == 2) return launch_fused_ring<4096, 2, 16, 1>(a, n_dump, spd, cpd, part, s);
  switch (a.n_fft) {
    case 1024: return launch_fused_ring<1024, 4, 16, 1>(a, n_dump, spd, cpd, part, s);
    case 2048: return launch_fused_ring<2048, 4, 16, 1>(a, n_dump, spd, cpd, part, s);
    default: return launch_fused_ring<4096, 4, 16, 1>(a, n_dump, spd, cpd, part, s);
  }
}

hipError_t launch_fused(const FxArgs& a, int64_t n_dump, int64_t spd, int64_t cpd, float2* part,
                        hipStream_t s, int tile) {
#define QC_CASE(NN, NAA)                 \
  if (a.n_fft == NN && a.n_ant == NAA) \
    return dispatch_tile<NN, NAA, 0>(tile, a, n_dump, spd, cpd, part, s);
  QC_CASE(4096, 4) QC_CASE(1024, 4) QC_CASE(2048, 4) QC_CASE(512, 4)
  QC_CASE(1024, 8) QC_CASE(2048, 8) QC_CASE(1024, 2) QC_CASE(4096, 2)
#undef QC_CASE
  return hipErrorInvalidValue;
}

// ==== end of fused F+X kernels =============================================

// ---------------------------------------------------------------------------
// Fixed-order reduction of partials.
// ---------------------------------------------------------------------------
// Sum of the cpd partials of each dump.  Partials are [dump*cpd][elems];
// with tile > 0 each partial is tile-major, [n_chan/tile][nb][tile] (one
// X-engine workgroup's output per tile), and the sum lands in the
// [nb][n_chan] layout of the visibilities.
__global__ void reduce_partials_kernel(const float2* __restrict__ part, int64_t cpd, int64_t elems,
                                       int64_t bx_per_dump, float scale, int accumulate, int tile,
                                       int64_t nb, int64_t n_chan, float2* __restrict__ vis) {
  const int64_t d = blockIdx.x / bx_per_dump;
  const int64_t bx = blockIdx.x % bx_per_dump;
  for (int64_t e = bx * blockDim.x + threadIdx.x; e < elems; e += bx_per_dump * blockDim.x) {
    float2 sacc = make_float2(0.f, 0.f);
    const float2* p = part + d * cpd * elems + e;
    for (int64_t c = 0; c < cpd; ++c) {
      const float2 v = p[c * elems];
      sacc.x += v.x;
      sacc.y += v.y;
    }
    sacc.x *= scale;
    sacc.y *= scale;
    int64_t oe = e;
    if (tile > 0) {
      const int64_t t = e / tile, col = e - t * tile;
      const int64_t cb = t / nb, b = t - cb * nb;
      oe = b * n_chan + cb * tile + col;
    }
    float2* o = vis + d * elems + oe;
    if (accumulate) {
      const float2 old = *o;
      sacc.x += old.x;
      sacc.y += old.y;
    }
    *o = sacc;
  }
}

hipError_t launch_reduce(const float2* part, int64_t n_dump, int64_t cpd, int64_t elems,
                         float scale, int accumulate, float2* vis, hipStream_t s, int tile, int64_t nb) {
  if (n_dump <= 0 || elems <= 0) return hipSuccess;
  if (tile > 0 && (nb <= 0 || elems % (nb * tile) != 0)) return hipErrorInvalidValue;
  int64_t bx = (elems + 255) / 256;
  if (bx > 4096) bx = 4096;
  const int64_t n_chan = tile > 0 ? elems / nb : 0;
  return launch(reduce_partials_kernel, dim3((unsigned)(bx * n_dump)), dim3(256), 0, s, part, cpd, elems, bx,
                scale, accumulate, tile, nb, n_chan, vis);
}

// ---------------------------------------------------------------------------
// Requantisation helpers (round to nearest even, saturating).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t enc_f16(float v) {
  v = fminf(fmaxf(v, -65504.f), 65504.f);
  return __half_as_ushort(__float2half_rn(v));
}

__device__ __forceinline__ uint16_t enc_bf16(float v) {
  uint32_t u = __float_as_uint(v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// OCP E4M3 ("fn"): bias 7, 3 mantissa bits, max 448, subnormal step 2^-9.
// Two values to OCP E4M3 (re in the low byte, im in the high byte): the
// hardware conversion rounds to nearest even; values are clamped to the
// largest finite magnitude, 448, first (saturating, never NaN).
__device__ __forceinline__ uint16_t enc_e4m3x2(float re, float im) {
  const float a = fminf(fmaxf(re, -448.f), 448.f);
  const float b = fminf(fmaxf(im, -448.f), 448.f);
  return (uint16_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
}

// ---------------------------------------------------------------------------
// Standalone F-engine: one antenna pair per block, S spectra in flight.
// ---------------------------------------------------------------------------
template <int N, int SS = (N >= 4096 ? 1 : 4096 / N)>
struct ChanCfg {
  static constexpr int S = SS;
  static constexpr int NT = S * N / 16;
  static constexpr int NCH = N / 2;
  static constexpr int LDS = lds_padded_size(S * N);
};

// Body of the F-engine for antenna pair p and spectra block bx (spec_per_blk
// spectra), run by all NT threads of a block on the LDS region buf.
template <int N, int SS, int PREC, bool WT = false>
__device__ __forceinline__ void chan_body(const int8_t* __restrict__ x, int64_t ld_x, int n_ant,
                                          int64_t n_spec, const int8_t* __restrict__ hist,
                                          const float* __restrict__ taps, int P,
                                          const float2* __restrict__ tw, int64_t spec_per_blk,
                                          const float* __restrict__ scale, void* __restrict__ out,
                                          int64_t bx, int p, float2* buf) {
  using C = ChanCfg<N, SS>;
  const int tid = threadIdx.x;
  const int a0 = 2 * p, a1 = (2 * p + 1 < n_ant) ? 2 * p + 1 : -1;
  const int64_t m_lo = bx * spec_per_blk;
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
      float2 y[4];
      if (m0 + s < m_hi) {
        fir4(x, ld_x, hist, taps, a0, a1, m0 + s, n0, N, P, y);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) y[i] = make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) buf[lds_pad(s * N + n0 + i)] = y[i];
    }
    __syncthreads();
    fft_lds<N, C::NT>(buf, tw, tid);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = tid + i * C::NT;  // over S * NCH
      const int s = e / C::NCH, k = e % C::NCH;
      const int64_t m = m0 + s;
      if (m < m_hi) {
        const float2 zk = buf[lds_pad(s * N + k)];
        const float2 zn = buf[lds_pad(s * N + ((N - k) & (N - 1)))];
        float2 ya, yb;
        separate(zk, zn, ya, yb);
        const float ha = 0.5f * sa, hb = 0.5f * sb;
        const int64_t ia = ((int64_t)a0 * n_spec + m) * C::NCH + k;
        const int64_t ib = ((int64_t)a1 * n_spec + m) * C::NCH + k;
        if constexpr (PREC == 0) {
          float2* o = reinterpret_cast<float2*>(out);
          st_f2<WT>(&o[ia], make_float2(ya.x * 0.5f, ya.y * 0.5f));
          if (a1 >= 0) st_f2<WT>(&o[ib], make_float2(yb.x * 0.5f, yb.y * 0.5f));
        } else if constexpr (PREC == 1 || PREC == 2) {
          uint32_t* o = reinterpret_cast<uint32_t*>(out);
          auto enc = [](float v) -> uint32_t {
            if constexpr (PREC == 1) return enc_f16(v);
            else return enc_bf16(v);
          };
          o[ia] = enc(ya.x * ha) | (enc(ya.y * ha) << 16);
          if (a1 >= 0) o[ib] = enc(yb.x * hb) | (enc(yb.y * hb) << 16);
        } else {
          uint16_t* o = reinterpret_cast<uint16_t*>(out);
          o[ia] = enc_e4m3x2(ya.x * ha, ya.y * ha);
          if (a1 >= 0) o[ib] = enc_e4m3x2(yb.x * hb, yb.y * hb);
        }
      }
    }
    __syncthreads();
  }
}

template <int N, int PREC>
__global__ void __launch_bounds__(ChanCfg<N>::NT)
channelize_kernel(const int8_t* __restrict__ x, int64_t ld_x, int n_ant, int64_t n_spec,
                  const int8_t* __restrict__ hist, const float* __restrict__ taps, int P,
                  const float2* __restrict__ tw, int64_t spec_per_blk, const float* __restrict__ scale,
                  void* __restrict__ out) {
  extern __shared__ float2 buf[];
  chan_body<N, ChanCfg<N>::S, PREC>(x, ld_x, n_ant, n_spec, hist, taps, P, tw, spec_per_blk, scale,
                                     out, (int64_t)blockIdx.x, (int)blockIdx.y, buf);
}

// Ring variant of the F-engine: the fused ring tile's FIR and transform
// (register ring of the last P blocks, next block prefetched, taps in
// registers, per-pass twiddles in LDS) for a group of NA antennas (NA/2
// packed transforms: four antennas up to N = 4096, two at N = 8192),
// writing the separated spectra out instead of correlating them.
// Block = (antenna group, run of spectra).  The half of the symmetric
// prototype the threads pick their taps from is staged once through the
// transform buffer, so LDS holds only the buffer(s) and the twiddles.
// With PP the transform ping-pongs between two buffers as in the fused
// ping-pong tile (one barrier per radix pass, none after the stores);
// without it the transform runs in place.
template <int N, int NA, int V, int P, bool PP = false>
struct ChanRingCfg {
  using C = FusedCfg<N, NA, 1, V, false, 0>;
  static constexpr int TAPS = P * N / 2;  // floats: half of a symmetric prototype
  static_assert(sizeof(float) * TAPS <= sizeof(float2) * C::LDS, "taps staged in the transform buffer");
  static constexpr size_t lds_bytes() {
    if constexpr (PP) return RingPpCfg<N, NA, V, P>::LDS_BYTES;
    else return sizeof(float2) * (C::LDS + N);  // transform, twiddles
  }
  static constexpr size_t LDS_BYTES = lds_bytes();
};

// 8-bit ring words as halves: four real samples -> two half2, four complex
// samples (I, Q) -> four half2; other words unchanged.
__device__ __forceinline__ uint32_t half2_of(uint32_t w, int lo_byte) {
  const __half a = __short2half_rn((short)(int8_t)((w >> (8 * lo_byte)) & 0xffu));
  const __half b = __short2half_rn((short)(int8_t)((w >> (8 * lo_byte + 8)) & 0xffu));
  const __half2 p = __halves2half2(a, b);
  return *reinterpret_cast<const uint32_t*>(&p);
}
template <int ST, bool HALF, class T>
__device__ __forceinline__ auto ring_word(const T& w) {
  if constexpr (!HALF) {
    return w;
  } else if constexpr (ST == 0) {
    return make_uint2(half2_of(w, 0), half2_of(w, 2));
  } else {
    return make_uint4(half2_of(w.x, 0), half2_of(w.x, 2), half2_of(w.y, 0), half2_of(w.y, 2));
  }
}
// Half number j (0-based, low half first) of a ring word of halves, as float.
__device__ __forceinline__ float half_at(const uint2& w, int j) {
  const uint32_t u = j < 2 ? w.x : w.y;
  const __half2 p = *reinterpret_cast<const __half2*>(&u);
  return (j & 1) ? __high2float(p) : __low2float(p);
}
__device__ __forceinline__ float half_at(const uint4& w, int j) {
  const uint32_t u = j < 2 ? w.x : j < 4 ? w.y : j < 6 ? w.z : w.w;
  const __half2 p = *reinterpret_cast<const __half2*>(&u);
  return (j & 1) ? __high2float(p) : __low2float(p);
}

// Body of the ring F-engine for antenna group grp and run chk of spb
// spectra, by all threads of a block, on an LDS region of
// ChanRingCfg<N, NAF, V, P, PP>::LDS_BYTES (NAF = NA for real words, 2 NA
// for complex ones: the same number of transforms).  x and hist are byte
// pointers to rows of ST words (ld_x in samples).  twp: the per-pass
// twiddle table (read with PP only).  Output [antenna][spectrum][channel]:
// N/2 channels for real words (separated, times 1/2), N for complex words.
template <int N, int NA, int V, int P, int PREC, bool PP = false, int ST = 0, bool WT = false>
__device__ __forceinline__ void chan_ring_body(const int8_t* __restrict__ x, int64_t ld_x, int n_ant,
                                               const int8_t* __restrict__ hist, const float* __restrict__ taps,
                                               const float2* __restrict__ tw, int64_t n_spec, int64_t spb,
                                               int grp, int64_t chk, const float* __restrict__ scale,
                                               void* __restrict__ out, float2* buf,
                                               const float2* __restrict__ twp = nullptr) {
  using W = RingWord<ST>;
  using T = typename W::T;
  constexpr bool CPLX = W::CPLX;
  // 8-bit words enter the ring as halves (exact): the FIR then takes each
  // sample straight from its half in the FMA (v_fma_mix_f32), one
  // conversion per sample instead of one per tap
  // (up to N = 4096: at 8192 a thread holds four tap positions and the
  // wider ring would spill; and for requantised output only: with float32
  // output the wider ring measured 3 % slower, with FP16 3 % faster)
  constexpr bool HALF = (ST == 0 || ST == 2) && N <= 4096 && PREC != 0;
  using RT = typename std::conditional<HALF, typename std::conditional<CPLX, uint4, uint2>::type, T>::type;
  constexpr int SL = CPLX ? 1 : 2;               // ring slots per chunk
  constexpr int NAF = CPLX ? 2 * NA : NA;
  using C = FusedCfg<N, NAF, 1, V, false, 0>;
  using F = Fft<N, C::NT, V, false, false, true>;
  constexpr int G = C::CHUNKS;
  constexpr int L = P * N;
  constexpr int NCH = CPLX ? N : N / 2;          // channels out per transform
  constexpr int CPT = NCH / C::NT;               // per thread per transform
  static_assert(NCH % C::NT == 0, "every thread has CPT channels");
  static_assert(!PP || fft_pass_count(N, V) % 2 == 1, "odd pass count: the output lands in the second buffer");
  float2* b0 = buf;
  float2* b1 = PP ? buf + C::BUF : buf;      // where the transform's output lands
  float2* twl = PP ? buf + 2 * C::BUF : buf + C::LDS;
  float4* tl = reinterpret_cast<float4*>(b0);  // taps, until they are in registers
  const int tid = threadIdx.x;
  const int a_base = NA * grp;
  const int64_t m_lo = chk * spb;
  const int64_t m_hi = m_lo + spb < n_spec ? m_lo + spb : n_spec;

  for (int i = tid; i < L / 8; i += C::NT) tl[i] = reinterpret_cast<const float4*>(taps)[i];
  if constexpr (PP) {
    for (int i = tid; i < PpTw<N, V>::LDS_TW; i += C::NT) twl[i] = twp[i];
  } else {
    build_pass_twiddles<N, V>(twl, tw, tid, C::NT);
  }

  constexpr int GP = G / C::NP;
  static_assert(GP * C::NP == G && GP * C::NT * 4 == N, "ring chunk mapping");
  int cn0[G];
#pragma unroll
  for (int g = 0; g < G; ++g) cn0[g] = 4 * (tid + (g % GP) * C::NT);
  // antenna of chunk g, slot `which`
  auto ant = [&](int g, int which) -> int { return a_base + (CPLX ? g / GP : 2 * (g / GP) + which); };
  auto load_blk = [&](int g, int which, int64_t blk) -> T {
    const int a = ant(g, which);
    if (a >= n_ant) return T{};
    if (blk >= 0)
      return *reinterpret_cast<const T*>(x + ((int64_t)a * ld_x + (int)blk * N + cn0[g]) * W::BYTES);
    if (!hist) return T{};
    return *reinterpret_cast<const T*>(hist + ((int64_t)a * (P - 1) * N + (int)(blk + P - 1) * N + cn0[g]) *
                                                  W::BYTES);
  };
  // Prefetch of stream block nb >= 0 (see the fused ring tile): one
  // unconditional load per chunk, from the last antenna for a slot past it
  // (zeroed when it enters the ring).
  auto load_next = [&](int g, int which, int nb) -> T {
    int a = ant(g, which);
    a = a < n_ant ? a : n_ant - 1;
    return *reinterpret_cast<const T*>(x + ((int64_t)a * ld_x + nb * N + cn0[g]) * W::BYTES);
  };
  RT ring[P][G][SL];
#pragma unroll
  for (int q = 0; q < P; ++q)
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int w = 0; w < SL; ++w) ring[q][g][w] = ring_word<ST, HALF>(load_blk(g, w, m_lo - P + 1 + q));
  // output scale per antenna: with the 1/2 of the separation for real words
  float hs[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int a = a_base + i;
    hs[i] = (CPLX ? 1.f : 0.5f) * ((PREC != 0 && a < n_ant) ? scale[a] : 1.f);
  }
  __syncthreads();  // taps and twiddles in LDS
  float4 hr[GP][P];   // taps of the thread's distinct chunk positions
#pragma unroll
  for (int g = 0; g < GP; ++g)
#pragma unroll
    for (int q = 0; q < P; ++q) {
      if (2 * q < P) {
        hr[g][q] = tl[(q * N + cn0[g]) / 4];
      } else {
        const float4 r = tl[(L - q * N - cn0[g] - 4) / 4];
        hr[g][q] = make_float4(r.w, r.z, r.y, r.x);
      }
    }
  __syncthreads();  // the transform buffer is free for the FIR output

  settle_words<P * G * SL * (int)(sizeof(RT) / 4)>(reinterpret_cast<uint32_t*>(&ring[0][0][0]));
  for (int64_t m = m_lo; m < m_hi; ++m) {
    T nxt[G][SL];
    const int nb = (int)(m + 1 < m_hi ? m + 1 : m);
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int w = 0; w < SL; ++w) nxt[g][w] = load_next(g, w, nb);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      float y0[4] = {0.f, 0.f, 0.f, 0.f}, y1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const float4 h = hr[g % GP][q];
        const float hv[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if constexpr (HALF && CPLX) {
            y0[i] = fmaf(hv[i], half_at(ring[q][g][0], 2 * i), y0[i]);
            y1[i] = fmaf(hv[i], half_at(ring[q][g][0], 2 * i + 1), y1[i]);
          } else if constexpr (HALF) {
            y0[i] = fmaf(hv[i], half_at(ring[q][g][0], i), y0[i]);
            y1[i] = fmaf(hv[i], half_at(ring[q][g][SL - 1], i), y1[i]);
          } else if constexpr (CPLX) {
            y0[i] += hv[i] * word_re<ST>(ring[q][g][0], i);
            y1[i] += hv[i] * word_im<ST>(ring[q][g][0], i);
          } else {
            y0[i] += hv[i] * word_re<ST>(ring[q][g][0], i);
            y1[i] += hv[i] * word_re<ST>(ring[q][g][SL - 1], i);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) b0[lds_pad((g / GP) * N + cn0[g] + i)] = make_float2(y0[i], y1[i]);
    }
    __syncthreads();
    if constexpr (PP) fft_pp_passes<N, 1, C::NT, V, 0, 0>(b0, b1, twl, tid);
    else F::run(b0, b0, twl, tid);
    // The FIR of spectrum m is done: shift the ring here, before the
    // stores, so the wait for the prefetch does not also wait for them.
#pragma unroll
    for (int q = 0; q + 1 < P; ++q)
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int w = 0; w < SL; ++w) ring[q][g][w] = ring[q + 1][g][w];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int w = 0; w < SL; ++w) {
        ring[P - 1][g][w] = ring_word<ST, HALF>(ant(g, w) < n_ant ? nxt[g][w] : T{});
        // pin the update here (it would otherwise sink past the stores)
        pin_word(ring[P - 1][g][w]);
      }
    // the thread's transform outputs, all read before any is used
    float2 zk[CPT][C::NP], zn[CPT][C::NP];
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
      const int k = tid + cc * C::NT;
      const int kn = (N - k) & (N - 1);
#pragma unroll
      for (int p = 0; p < C::NP; ++p) {
        zk[cc][p] = b1[lds_pad(p * N + k)];
        if constexpr (!CPLX) zn[cc][p] = b1[lds_pad(p * N + kn)];
      }
    }
    auto put = [&](int a, int k, float2 y, float hh) {
      const int64_t idx = ((int64_t)a * n_spec + m) * NCH + k;
      if constexpr (PREC == 0) {
        st_f2<WT>(&reinterpret_cast<float2*>(out)[idx], make_float2(y.x * hh, y.y * hh));
      } else if constexpr (PREC == 1) {
        reinterpret_cast<uint32_t*>(out)[idx] = enc_f16(y.x * hh) | (enc_f16(y.y * hh) << 16);
      } else if constexpr (PREC == 2) {
        reinterpret_cast<uint32_t*>(out)[idx] = enc_bf16(y.x * hh) | (enc_bf16(y.y * hh) << 16);
      } else {
        reinterpret_cast<uint16_t*>(out)[idx] = enc_e4m3x2(y.x * hh, y.y * hh);
      }
    };
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
      const int k = tid + cc * C::NT;
#pragma unroll
      for (int p = 0; p < C::NP; ++p) {
        if constexpr (CPLX) {
          const int a = a_base + p;
          if (a < n_ant) put(a, k, zk[cc][p], hs[p]);
        } else {
          float2 ya, yb;
          separate(zk[cc][p], zn[cc][p], ya, yb);
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int a = a_base + 2 * p + u;
            if (a < n_ant) put(a, k, u ? yb : ya, hs[2 * p + u]);
          }
        }
      }
    }
    // the next FIR overwrites b0: without PP every thread must be done
    // reading it; with PP the transform output was read from b1, which the
    // next FIR's barrier protects
    if constexpr (!PP) __syncthreads();
  }
}


template <int N, int NA, int V, int P, int PREC, bool PP, int ST>
__global__ void __launch_bounds__((FusedCfg<N, (ST >= 2 ? 2 * NA : NA), 1, V, false, 0>::NT))
chan_ring_kernel(const int8_t* __restrict__ x, int64_t ld_x, int n_ant, const int8_t* __restrict__ hist,
                 const float* __restrict__ taps, const float2* __restrict__ tw, const float2* __restrict__ twp,
                 int64_t n_spec, int64_t spb, int64_t chunks, const float* __restrict__ scale,
                 void* __restrict__ out) {
  extern __shared__ float2 buf[];
  chan_ring_body<N, NA, V, P, PREC, PP, ST>(x, ld_x, n_ant, hist, taps, tw, n_spec, spb,
                                            (int)(blockIdx.x / chunks), (int64_t)(blockIdx.x % chunks), scale,
                                            out, buf, twp);
}

// The ring F-engine over n_ant rows of ST words.  Four real antennas (two
// packed transforms) per workgroup up to N = 4096 and two at N = 8192;
// complex words take half as many antennas, one transform each.  Ping-pong
// transform buffers at N = 4096 (154 KiB of LDS).
template <int N, int PREC, int ST>
static hipError_t launch_chan_ring_w(const int8_t* x, int64_t ld_x, int n_ant, int64_t n_samp,
                                     const int8_t* hist, const float* taps, const float2* tw,
                                     const float2* twp, void* out, const float* scale, hipStream_t s) {
  constexpr int V = 16;
  constexpr bool PP = N == 4096;
  constexpr int NAR = N >= 8192 ? 2 : 4;
  constexpr int NA = ST >= 2 ? NAR / 2 : NAR;
  using RC = ChanRingCfg<N, NAR, V, 4, PP>;
  using C = FusedCfg<N, NAR, 1, V, false, 0>;
  static_assert(RC::LDS_BYTES <= 160 * 1024, "channelize ring: LDS");
  if (PP && !twp) return hipErrorInvalidValue;
  const int64_t n_spec = n_samp / N;
  const int groups = (n_ant + NA - 1) / NA;
  // runs of at least 16 spectra (the ring reloads P-1 blocks per run and
  // each workgroup rebuilds its twiddle tables).  Workgroups of 512 threads
  // (N >= 4096) are resident one per CU: one workgroup per CU in total, a
  // single round (1-4 % faster than two rounds at 32 antennas, N = 4096);
  // smaller ones keep 512 in total
  const int64_t wg = C::NT >= 512 ? device_cu_count() : 512;
  int64_t spb = (n_spec * groups + wg - 1) / wg;
  if (spb < 16) spb = 16;
  const int64_t chunks = (n_spec + spb - 1) / spb;
  if ((int64_t)groups * chunks > 0x7fffffffLL) return hipErrorInvalidValue;
  const void* k = reinterpret_cast<const void*>(chan_ring_kernel<N, NA, V, 4, PREC, PP, ST>);
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)RC::LDS_BYTES);
  if (e != hipSuccess) return e;
  return launch(chan_ring_kernel<N, NA, V, 4, PREC, PP, ST>, dim3((unsigned)(groups * chunks)), dim3(C::NT),
                RC::LDS_BYTES, s, x, ld_x, n_ant, hist, taps, tw, twp, n_spec, spb, chunks, scale, out);
}

template <int N, int ST>
static hipError_t launch_chan_ring_st(const int8_t* x, int64_t ld_x, int n_ant, int64_t n_samp,
                                      const int8_t* hist, const float* taps, const float2* tw,
                                      const float2* twp, int prec, void* out, const float* scale,
                                      hipStream_t s) {
  switch (prec) {
    case 0: return launch_chan_ring_w<N, 0, ST>(x, ld_x, n_ant, n_samp, hist, taps, tw, twp, out, scale, s);
    case 1: return launch_chan_ring_w<N, 1, ST>(x, ld_x, n_ant, n_samp, hist, taps, tw, twp, out, scale, s);
    case 2: return launch_chan_ring_w<N, 2, ST>(x, ld_x, n_ant, n_samp, hist, taps, tw, twp, out, scale, s);
    default: return launch_chan_ring_w<N, 3, ST>(x, ld_x, n_ant, n_samp, hist, taps, tw, twp, out, scale, s);
  }
}

template <int N>
static hipError_t launch_chan_ring(const FxArgs& a, int prec, void* out, const float* scale, hipStream_t s) {
  return launch_chan_ring_st<N, 0>(a.x, a.ld_x, a.n_ant, a.n_samp, a.hist, a.taps, a.tw, a.twp, prec, out,
                                   scale, s);
}

template <int N>
static hipError_t launch_chan_t(const FxArgs& a, int prec, void* out, const float* scale,
                                hipStream_t s) {
  using C = ChanCfg<N>;
  const int64_t n_spec = a.n_samp / N;
  const int n_pair = (a.n_ant + 1) / 2;
  // spectra per block: a multiple of S giving ~2048 blocks in total
  int64_t per = (n_spec * n_pair + 2047) / 2048;
  per = ((per + C::S - 1) / C::S) * C::S;
  if (per < C::S) per = C::S;
  const int64_t nbx = (n_spec + per - 1) / per;
  const size_t lds = sizeof(float2) * C::LDS;
  const void* k = nullptr;
  switch (prec) {
    case 0: k = reinterpret_cast<const void*>(channelize_kernel<N, 0>); break;
    case 1: k = reinterpret_cast<const void*>(channelize_kernel<N, 1>); break;
    case 2: k = reinterpret_cast<const void*>(channelize_kernel<N, 2>); break;
    default: k = reinterpret_cast<const void*>(channelize_kernel<N, 3>); break;
  }
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)nbx, (unsigned)n_pair);
#define QC_CHAN_LAUNCH(PR)                                                                              \
  return launch(channelize_kernel<N, PR>, grid, dim3(C::NT), lds, s, a.x, a.ld_x, a.n_ant, n_spec, a.hist, \
                a.taps, a.n_taps, a.tw, per, scale, out)
  switch (prec) {
    case 0: QC_CHAN_LAUNCH(0);
    case 1: QC_CHAN_LAUNCH(1);
    case 2: QC_CHAN_LAUNCH(2);
    default: QC_CHAN_LAUNCH(3);
  }
#undef QC_CHAN_LAUNCH
}

static int g_chan_variant = 0;  // 0: ring variant where it applies, 1: always the plain kernel

void set_channelize_variant(int v) { g_chan_variant = v; }
int get_channelize_variant() { return g_chan_variant; }

template <int N>
static hipError_t launch_chan_ring_any_n(const ChanxArgs& a, int sample, int prec, void* out,
                                         const float* scale, hipStream_t s) {
  const int8_t* x = static_cast<const int8_t*>(a.x);
  const int8_t* h = static_cast<const int8_t*>(a.hist);
  switch (sample) {
    case 0: return launch_chan_ring_st<N, 0>(x, a.ld_x, a.n_ant, a.n_samp, h, a.taps, a.tw, a.twp, prec, out, scale, s);
    case 1: return launch_chan_ring_st<N, 1>(x, a.ld_x, a.n_ant, a.n_samp, h, a.taps, a.tw, a.twp, prec, out, scale, s);
    case 2: return launch_chan_ring_st<N, 2>(x, a.ld_x, a.n_ant, a.n_samp, h, a.taps, a.tw, a.twp, prec, out, scale, s);
    case 3: return launch_chan_ring_st<N, 3>(x, a.ld_x, a.n_ant, a.n_samp, h, a.taps, a.tw, a.twp, prec, out, scale, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_channelize_ring_any(const ChanxArgs& a, int sample, int prec, void* out, const float* scale,
                                      hipStream_t s) {
  if (g_chan_variant != 0 || a.n_taps != 4 || !a.taps_symmetric) return hipErrorNotSupported;
  // 16-bit words at N = 8192 (four distinct tap positions per thread and a
  // ring twice as wide) would spill inside the loop: the plain kernel
  if (a.n_fft == 8192 && (sample == 1 || sample == 3)) return hipErrorNotSupported;
  switch (a.n_fft) {
    case 1024: return launch_chan_ring_any_n<1024>(a, sample, prec, out, scale, s);
    case 2048: return launch_chan_ring_any_n<2048>(a, sample, prec, out, scale, s);
    case 4096: return launch_chan_ring_any_n<4096>(a, sample, prec, out, scale, s);
    case 8192: return launch_chan_ring_any_n<8192>(a, sample, prec, out, scale, s);
  }
  return hipErrorNotSupported;
}

hipError_t launch_channelize(const FxArgs& a, int prec, void* out, const float* scale,
                             hipStream_t s) {
  if (g_chan_variant == 0 && a.n_taps == 4 && a.taps_symmetric) {
    switch (a.n_fft) {
      case 1024: return launch_chan_ring<1024>(a, prec, out, scale, s);
      case 2048: return launch_chan_ring<2048>(a, prec, out, scale, s);
      case 4096: return launch_chan_ring<4096>(a, prec, out, scale, s);
      case 8192: return launch_chan_ring<8192>(a, prec, out, scale, s);
      default: break;
    }
  }
  switch (a.n_fft) {
    case 4: return launch_chan_t<4>(a, prec, out, scale, s);
    case 8: return launch_chan_t<8>(a, prec, out, scale, s);
    case 16: return launch_chan_t<16>(a, prec, out, scale, s);
    case 32: return launch_chan_t<32>(a, prec, out, scale, s);
    case 64: return launch_chan_t<64>(a, prec, out, scale, s);
    case 128: return launch_chan_t<128>(a, prec, out, scale, s);
    case 256: return launch_chan_t<256>(a, prec, out, scale, s);
    case 512: return launch_chan_t<512>(a, prec, out, scale, s);
    case 1024: return launch_chan_t<1024>(a, prec, out, scale, s);
    case 2048: return launch_chan_t<2048>(a, prec, out, scale, s);
    case 4096: return launch_chan_t<4096>(a, prec, out, scale, s);
    case 8192: return launch_chan_t<8192>(a, prec, out, scale, s);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Per-antenna power-of-two scale from the input power: the sum of squares of
// the first n_use samples, split over SC_BLOCKS workgroups per antenna
// (exact 64-bit integer partials, so the split does not change the sum),
// then one thread per antenna turns the total into the scale.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
scales_partial_kernel(const int8_t* __restrict__ x, int64_t ld_x, int64_t n_use,
                      unsigned long long* __restrict__ part) {
  __shared__ unsigned long long red[4];
  const int a = blockIdx.y;
  const int8_t* xa = x + (int64_t)a * ld_x;
  const uint32_t* xw = reinterpret_cast<const uint32_t*>(xa);
  const int64_t nw = n_use / 4;
  const int64_t w0 = nw * blockIdx.x / SC_BLOCKS, w1 = nw * (blockIdx.x + 1) / SC_BLOCKS;
  // squares of the four samples of a word: at most 4 * 128^2, exact in 32 bits
  auto sq4 = [](uint32_t v) -> unsigned {
    unsigned t = 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = (int)(int8_t)((v >> (8 * i)) & 0xffu);
      t += (unsigned)(b * b);
    }
    return t;
  };
  unsigned long long acc = 0;
  int64_t wt = w0;
  if ((reinterpret_cast<uintptr_t>(xw + w0) & 15u) == 0) {
    // 16-byte loads, four in flight per thread before any is used
    constexpr int U = 4;
    const uint4* x4 = reinterpret_cast<const uint4*>(xw + w0);
    const int64_t n4 = (w1 - w0) / 4;
    for (int64_t j0 = threadIdx.x; j0 < n4; j0 += (int64_t)U * 256) {
      uint4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = j0 + (int64_t)u * 256;
        v[u] = j < n4 ? x4[j] : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc += (unsigned long long)(sq4(v[u].x) + sq4(v[u].y) + sq4(v[u].z) + sq4(v[u].w));
    }
    wt = w0 + 4 * n4;
  }
  for (int64_t w = wt + threadIdx.x; w < w1; w += 256) acc += (unsigned long long)sq4(xw[w]);
  if (blockIdx.x == SC_BLOCKS - 1 && threadIdx.x == 0)
    for (int64_t n = nw * 4; n < n_use; ++n) acc += (unsigned long long)((int)xa[n] * (int)xa[n]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)a * SC_BLOCKS + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void scales_finish_kernel(const unsigned long long* __restrict__ part, int n_ant, int64_t n_use,
                                     double sum_h2, double target, float* __restrict__ scale_out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_ant) return;
  unsigned long long tot = 0;
  for (int b = 0; b < SC_BLOCKS; ++b) tot += part[(int64_t)a * SC_BLOCKS + b];
  const double pw = (double)tot / (double)n_use;
  const double rms = sqrt(pw * sum_h2);
  float sc = 1.f;
  if (rms > 0.0) {
    const double e = rint(log2(target / rms));
    sc = (float)ldexp(1.0, (int)e);
  }
  scale_out[a] = sc;
}

hipError_t launch_scales(const int8_t* x, int64_t ld_x, int n_ant, int64_t n_use, double sum_h2,
                         double target, unsigned long long* part, float* scale_out, hipStream_t s) {
  hipError_t e = launch(scales_partial_kernel, dim3(SC_BLOCKS, n_ant), dim3(256), 0, s, x, ld_x, n_use, part);
  if (e != hipSuccess) return e;
  return launch(scales_finish_kernel, dim3((n_ant + 255) / 256), dim3(256), 0, s, part, n_ant, n_use, sum_h2,
                target, scale_out);
}

// ---------------------------------------------------------------------------
// History for the next chunk: last `keep` samples of (hist ++ x).
// ---------------------------------------------------------------------------
__global__ void hist_copy_kernel(const int8_t* __restrict__ x, int64_t ld_x, int64_t n_samp,
                                 const int8_t* __restrict__ hist, int64_t keep,
                                 int8_t* __restrict__ hist_out) {
  const int a = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < keep;
       i += (int64_t)gridDim.x * blockDim.x) {
    // position in (hist ++ x) coordinates: n = n_samp - keep + i (may be < 0)
    const int64_t n = n_samp - keep + i;
    int8_t v;
    if (n >= 0) v = x[(int64_t)a * ld_x + n];
    else v = hist ? hist[(int64_t)a * keep + (keep + n)] : (int8_t)0;
    hist_out[(int64_t)a * keep + i] = v;
  }
}

hipError_t launch_hist_copy(const int8_t* x, int64_t ld_x, int n_ant, int64_t n_samp,
                            const int8_t* hist, int64_t keep, int8_t* hist_out, hipStream_t s) {
  if (keep <= 0) return hipSuccess;
  int64_t bx = (keep + 255) / 256;
  if (bx > 1024) bx = 1024;
  return launch(hist_copy_kernel, dim3((unsigned)bx, n_ant), dim3(256), 0, s, x, ld_x, n_samp, hist, keep,
                hist_out);
}

// ---------------------------------------------------------------------------
// X-engine on the vector ALUs (float32), any n_ant.  Thread = one channel and
// one 4x4 antenna block pair (I <= J); spectra split into `ksplit` runs.
// ---------------------------------------------------------------------------
// Body of the X-engine for channel group cg (NTX channels), antenna block
// pair bp and run dz (= dump * ksplit + split).
template <int NTX, bool WT = false>
__device__ __forceinline__ void xeng_f32_body(const float2* __restrict__ v, int n_ant, int64_t n_spec,
                                              int n_chan, int64_t spec_per_dump, int64_t ksplit,
                                              int cg, int bp_in, int64_t dz, float2* __restrict__ part) {
  const int nblk = (n_ant + 3) / 4;
  // block pair index -> (I, J), I <= J
  int bp = bp_in, I = 0;
  while (bp >= nblk - I) { bp -= nblk - I; ++I; }
  const int J = I + bp;
  const int k = cg * NTX + (int)threadIdx.x;
  const int64_t d = dz / ksplit, ks = dz % ksplit;
  const int64_t m_lo = d * spec_per_dump + (ks * spec_per_dump) / ksplit;
  const int64_t m_hi = d * spec_per_dump + ((ks + 1) * spec_per_dump) / ksplit;
  if (k >= n_chan) return;
  float2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_float2(0.f, 0.f);
  int ai[4], aj[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ai[i] = 4 * I + i < n_ant ? 4 * I + i : n_ant - 1;
    aj[i] = 4 * J + i < n_ant ? 4 * J + i : n_ant - 1;
  }
  for (int64_t m = m_lo; m < m_hi; ++m) {
    float2 xi[4], xj[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      xi[i] = v[((int64_t)ai[i] * n_spec + m) * n_chan + k];
      xj[i] = v[((int64_t)aj[i] * n_spec + m) * n_chan + k];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j].x += xi[i].x * xj[j].x + xi[i].y * xj[j].y;
        acc[i][j].y += xi[i].y * xj[j].x - xi[i].x * xj[j].y;
      }
  }
  const int nb = n_ant * (n_ant + 1) / 2;
  float2* out = part + dz * (int64_t)nb * n_chan;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gi = 4 * I + i, gj = 4 * J + j;
      if (gi < n_ant && gj < n_ant && gi <= gj) {
        const int b = gi * n_ant - gi * (gi - 1) / 2 + (gj - gi);
        float2 r = acc[i][j];
        if (gi == gj) r.y = 0.f;
        st_f2<WT>(&out[(int64_t)b * n_chan + k], r);
      }
    }
}

__global__ void __launch_bounds__(256)
xeng_f32_kernel(const float2* __restrict__ v, int n_ant, int64_t n_spec, int n_chan,
                int64_t spec_per_dump, int64_t ksplit, int n_cgrp, float2* __restrict__ part) {
  xeng_f32_body<256>(v, n_ant, n_spec, n_chan, spec_per_dump, ksplit, (int)(blockIdx.x % n_cgrp),
                     (int)blockIdx.y, (int64_t)(blockIdx.x / n_cgrp), part);
}

static int g_xef_variant = 0;

void set_xeng_f32_variant(int v) { g_xef_variant = v; }
int get_xeng_f32_variant() { return g_xef_variant; }

bool xeng_f32_use_mfma(int n_ant, int n_chan, const void* v) {
  if (g_xef_variant == 1 || !xeng_f32_mfma_supported(n_ant, n_chan, v)) return false;
  return g_xef_variant == 2 || n_ant >= XEF_MFMA_MIN_ANT;
}

static int64_t xeng_f32_valu_ksplit(int n_ant, int64_t spd, int n_chan, int64_t n_dump) {
  const int nblk = (n_ant + 3) / 4;
  const int64_t waves = (int64_t)nblk * (nblk + 1) / 2 * ((n_chan + 63) / 64) * n_dump;
  int64_t ks = (8192 + waves - 1) / waves;
  const int64_t maxk = spd / 64 > 0 ? spd / 64 : 1;
  if (ks > maxk) ks = maxk;
  return ks < 1 ? 1 : ks;
}

int xeng_f32_tile(int n_ant, int n_chan, const void* v) {
  return xeng_f32_use_mfma(n_ant, n_chan, v) ? 16 : 0;
}

int64_t xeng_f32_ksplit(int n_ant, int64_t spd, int n_chan, int64_t n_dump) {
  // any 16-byte aligned address stands for the buffer the caller will pass
  if (xeng_f32_use_mfma(n_ant, n_chan, reinterpret_cast<const void*>(uintptr_t(256))))
    return xeng_f32_mfma_ksplit(n_ant, spd, n_chan, n_dump);
  return xeng_f32_valu_ksplit(n_ant, spd, n_chan, n_dump);
}

hipError_t launch_xeng_f32(const float2* v, int n_ant, int64_t n_spec, int n_chan, int64_t spd,
                           int64_t n_dump, int64_t ksplit, float2* part, hipStream_t s) {
  if (xeng_f32_use_mfma(n_ant, n_chan, v))
    return launch_xeng_f32_mfma(v, n_ant, n_spec, n_chan, spd, n_dump, ksplit, part, s);
  const int nblk = (n_ant + 3) / 4;
  const int n_cgrp = (n_chan + 255) / 256;
  dim3 grid((unsigned)(n_cgrp * n_dump * ksplit), (unsigned)(nblk * (nblk + 1) / 2));
  return launch(xeng_f32_kernel, grid, dim3(256), 0, s, v, n_ant, n_spec, n_chan, spd, ksplit, n_cgrp, part);
}

// ---------------------------------------------------------------------------
// Batched plans: every array's work in one persistent launch.  Blocks of
// PL_NT threads claim items from a queue in order (one atomic per item);
// items that depend on others (X-engine on F-engine output, reductions on
// partials) come later in the queue than everything they depend on, so a
// block only ever waits for items already claimed by running blocks.  Each
// wait is bounded in time; on expiry the error flag is set, the item is
// skipped and still counted, and every later wait gives up at once, so
// every block reaches the queue's end and exits.
// ---------------------------------------------------------------------------
// Fused items for 4 antennas.  At 8 antennas the fused body's accumulators
// (36 baselines per channel) do not fit the 248 registers an item function
// gets inside the persistent kernel and spill; those arrays take the
// two-pass items (F-engine, then the matrix-core X-engine).
bool plan_fused_supported(int n_fft, int n_ant) {
  return n_ant == 4 && (n_fft == 1024 || n_fft == 2048 || n_fft == 4096);
}

bool plan_chan_supported(int n_fft) { return n_fft >= 16 && n_fft <= 8192; }

// LDS frame of the persistent kernel: its largest item body, the
// matrix-core X-engine's two stages (or the ring F-engine at N = 8192:
// transform buffer and twiddles); the plain bodies' buffer fits inside.
constexpr size_t PLAN_LDS = ChanRingCfg<8192, 2, 16, 4>::LDS_BYTES > (size_t)(2 * XM_STAGE)
                                ? ChanRingCfg<8192, 2, 16, 4>::LDS_BYTES
                                : (size_t)(2 * XM_STAGE);
static_assert(PLAN_LDS >= sizeof(float2) * lds_padded_size(8192), "plain bodies' buffer");

__global__ void plan_reset_kernel(unsigned* ctr, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) ctr[i] = 0u;
}

// The item functions below are not inlined, so their arguments reach them in
// vector registers and the compiler takes every value derived from them for
// a per-lane one: loops whose bounds come from the descriptor would be
// compiled as lane-divergent loops around the bodies' barriers.  All of them
// are in fact the same for the whole block; readfirstlane says so, and the
// loops become scalar.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uni(T* p) {
  return reinterpret_cast<T*>(uni((int64_t)reinterpret_cast<uintptr_t>(p)));
}
// uni() for a pointer known to address global memory (a plan's arrays):
// the value passes through a global-address-space pointer, so accesses
// through it compile to global rather than flat instructions (flat ones
// also count against the LDS counter, so every LDS wait waits for them).
template <class T>
__device__ __forceinline__ T* uni_global(T* p) {
  const uint64_t v = (uint64_t)uni((int64_t)reinterpret_cast<uintptr_t>(p));
  return (T*)(__attribute__((address_space(1))) T*)v;
}
__device__ __forceinline__ float uni(float v) { return __int_as_float(uni((int32_t)__float_as_int(v))); }

static_assert(sizeof(PlArray) == 160, "load_uniform copies every field of PlArray");
__device__ __forceinline__ PlArray load_uniform(const PlArray* Ap) {
  const PlArray* p = uni(Ap);
  PlArray A;
  A.x = uni_global(p->x);
  A.vis = uni_global(p->vis);
  A.part = uni_global(p->part);
  A.chan = uni_global(p->chan);
  A.taps = uni_global(p->taps);
  A.tw = uni_global(p->tw);
  A.n_samp = uni(p->n_samp);
  A.spd = uni(p->spd);
  A.n_dump = uni(p->n_dump);
  A.n_split = uni(p->n_split);
  A.spec_per_item = uni(p->spec_per_item);
  A.n_ant = uni(p->n_ant);
  A.n_fft = uni(p->n_fft);
  A.n_taps = uni(p->n_taps);
  A.mode = uni(p->mode);
  A.n_chan_items = uni(p->n_chan_items);
  A.n_part_items = uni(p->n_part_items);
  A.n_cgrp = uni(p->n_cgrp);
  A.n_bp = uni(p->n_bp);
  A.n_red_blocks = uni(p->n_red_blocks);
  A.scale = uni(p->scale);
  A.spb = uni(p->spb);
  A.n_chunks = uni(p->n_chunks);
  A.x_kind = uni(p->x_kind);
  A.n_cb = uni(p->n_cb);
  A.tile = uni(p->tile);
  A.red_block = uni(p->red_block);
  A.pad1 = 0;
  return A;
}

__device__ __noinline__ void reduce_item(const PlArray* __restrict__ Ap, int64_t index_in) {
  const PlArray A = load_uniform(Ap);
  const int64_t index = uni(index_in);
  const int64_t nb = (int64_t)A.n_ant * (A.n_ant + 1) / 2;
  const int64_t elems = nb * (A.n_fft / 2);
  const int64_t d = index / A.n_red_blocks, eb = index % A.n_red_blocks;
  const int64_t e_end = min(elems, (eb + 1) * (int64_t)A.red_block);
  for (int64_t e = eb * A.red_block + threadIdx.x; e < e_end; e += PL_NT) {
    float2 acc = make_float2(0.f, 0.f);
    const float2* p = A.part + d * A.n_split * elems + e;
    // partials added in order; unrolled so that several loads are in flight
#pragma unroll 8
    for (int64_t c = 0; c < A.n_split; ++c) {
      const float2 v = p[c * elems];
      acc.x += v.x;
      acc.y += v.y;
    }
    int64_t oe = e;
    if (A.tile > 0) {  // tile-major partials of the matrix-core X-engine
      const int64_t t = e / A.tile, col = e - t * A.tile;
      const int64_t cb = t / nb, b = t - cb * nb;
      oe = b * (A.n_fft / 2) + cb * A.tile + col;
    }
    A.vis[d * elems + oe] = make_float2(acc.x * A.scale, acc.y * A.scale);
  }
}

template <int N, int NA>
__device__ __noinline__ void plan_fused(const PlArray* __restrict__ Ap, int64_t w_in, float2* buf_in) {
  const PlArray A = load_uniform(Ap);
  const int64_t w = uni(w_in);
  float2* buf = uni(buf_in);
  constexpr int S = 8192 / (((NA + 1) / 2) * N);
  static_assert(FusedCfg<N, NA, S, 16, false, 0>::NT == PL_NT, "plan fused tile");
  if (A.n_taps == 4)
    fused_body<N, NA, S, 16, false, 0, 4, true>(A.x, A.n_samp, nullptr, A.taps, 4, A.tw, A.spd, A.n_split,
                                          A.part, w, buf);
  else
    fused_body<N, NA, S, 16, false, 0, 0, true>(A.x, A.n_samp, nullptr, A.taps, A.n_taps, A.tw, A.spd,
                                          A.n_split, A.part, w, buf);
}

template <int N>
__device__ __noinline__ void plan_chan(const PlArray* __restrict__ Ap, int64_t index_in, float2* buf_in) {
  const PlArray A = load_uniform(Ap);
  const int64_t index = uni(index_in);
  float2* buf = uni(buf_in);
  constexpr int S = 8192 / N;
  static_assert(ChanCfg<N, S>::NT == PL_NT, "plan F-engine tile");
  const int n_pair = (A.n_ant + 1) / 2;
  const int p = (int)(index % n_pair);
  const int64_t bx = index / n_pair;
  const int64_t n_spec = A.n_dump * A.spd;
  chan_body<N, S, 0, true>(A.x, A.n_samp, A.n_ant, n_spec, nullptr, A.taps, A.n_taps, A.tw,
                     A.spec_per_item, nullptr, A.chan, bx, p, buf);
}

__device__ __noinline__ void xeng_item(const PlArray* __restrict__ Ap, int64_t index_in) {
  const PlArray A = load_uniform(Ap);
  const int64_t index = uni(index_in);
  // index -> (run dz, block pair bp, channel group cg)
  const int64_t per_dz = (int64_t)A.n_bp * A.n_cgrp;
  const int64_t dz = index / per_dz;
  const int rem = (int)(index % per_dz);
  xeng_f32_body<PL_NT, true>(A.chan, A.n_ant, A.n_dump * A.spd, A.n_fft / 2, A.spd, A.n_split,
                       rem % A.n_cgrp, rem / A.n_cgrp, dz, A.part);
}

template <int N, int NA>
__device__ __noinline__ void plan_chan_ring(const PlArray* __restrict__ Ap, int64_t index_in, float2* buf_in) {
  const PlArray A = load_uniform(Ap);
  const int64_t index = uni(index_in);
  float2* buf = uni(buf_in);
  static_assert(FusedCfg<N, NA, 1, 16, false, 0>::NT == PL_NT, "plan ring F-engine tile");
  static_assert(ChanRingCfg<N, NA, 16, 4>::LDS_BYTES <= PLAN_LDS, "plan ring F-engine LDS");
  chan_ring_body<N, NA, 16, 4, 0, false, 0, true>(A.x, A.n_samp, A.n_ant, nullptr, A.taps, A.tw, A.n_dump * A.spd, A.spb,
                                  (int)(index / A.n_chunks), index % A.n_chunks, nullptr, A.chan, buf);
}

__device__ __noinline__ void plan_xmfma(const PlArray* __restrict__ Ap, int64_t index_in, float2* buf_in) {
  const PlArray A = load_uniform(Ap);
  const int64_t index = uni(index_in);
  uint8_t* st0 = reinterpret_cast<uint8_t*>(uni(buf_in));
  uint8_t* st1 = st0 + XM_STAGE;
  static_assert(XM_NT == PL_NT && 2 * XM_STAGE <= PLAN_LDS, "plan matrix-core X-engine frame");
  const int cb = (int)(index % A.n_cb);
  const int64_t dz = index / A.n_cb;
  const int64_t n_spec = A.n_dump * A.spd;
  if (A.x_kind == 1)
    xeng_mfma_body<0, true>(A.chan, nullptr, A.n_ant, n_spec, A.n_fft / 2, A.spd, A.n_split, cb, dz, A.part, st0, st1);
  else
    xeng_mfma_body<4, true>(A.chan, nullptr, A.n_ant, n_spec, A.n_fft / 2, A.spd, A.n_split, cb, dz, A.part, st0, st1);
}

// Every branch of the persistent loop below is wave-uniform.  The claim, the
// polls and the publish are done by all 64 lanes of wave 0, selected by a
// readfirstlane'd wave index (a scalar branch), never by a `threadIdx.x == 0`
// test: a lane-divergent branch at the loop's head or latch lets the
// optimizer thread the two `thread 0` tests into a shortcut for the other
// lanes, and the structurizer then nests the loop so that lane 0 leaves an
// inner loop after publishing while its wave's other lanes (and the other
// waves) go round through the barriers again, read the stale item index and
// redo the same item for ever.  With only scalar branches every lane of a
// wave takes the same path, so each wave meets the barriers in program
// order.

// Value of one lane-0-only atomic add done by the whole wave: lane 0 adds
// `v`, the other lanes add 0, and lane 0's old value (the count before the
// add, whatever order the lanes' adds take) is returned to every lane.
__device__ __forceinline__ unsigned wave_fetch_add(unsigned* p, unsigned v) {
  const unsigned mine = (threadIdx.x & 63u) == 0u ? v : 0u;
  return (unsigned)__builtin_amdgcn_readfirstlane((int)atomicAdd(p, mine));
}

__device__ __forceinline__ unsigned wave_load(const unsigned* p) {
  return (unsigned)__builtin_amdgcn_readfirstlane(
      (int)__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Bounded dependency wait, run by the whole block.  Wave 0 polls the
// counter with relaxed agent-scope loads (a coherent read, no cache
// maintenance per poll) until it reaches `target`, the time limit (in ticks
// of the constant-rate wall clock) passes, or another block has already
// given up (error flag set).  After the barrier every wave issues one
// agent-scope acquire fence, so the producers' results are read fresh.
__device__ __forceinline__ bool plan_wait(const unsigned* ctr, unsigned target, unsigned* err,
                                          int64_t limit_ticks, int wave, int* sflag) {
  if (wave == 0) {
    int ok = 1;
    if (wave_load(ctr) < target) {
      const int64_t t0 = wall_clock64();
      while (wave_load(ctr) < target) {
        if (wave_load(err) != 0u || wall_clock64() - t0 > limit_ticks) {
          ok = 0;
          (void)wave_fetch_add(err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(16);
      }
    }
    *sflag = ok;  // the same value from every lane
  }
  __syncthreads();
  const bool ok = __builtin_amdgcn_readfirstlane(*sflag) != 0;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
  return ok;
}

__global__ void __launch_bounds__(PL_NT) plan_kernel(PlArgs a) {
  extern __shared__ float2 buf[];
  __shared__ int s_item, s_flag;
  unsigned* err = a.ctr + 1;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for (;;) {
    if (wave == 0) s_item = (int)wave_fetch_add(a.ctr, 1u);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= a.n_items) break;
    const PlItem item = a.items[it];
    const PlArray* Ap = a.arr + item.array;
    unsigned* done_part = a.ctr + 2 + 2 * item.array;
    unsigned* done_chan = a.ctr + 3 + 2 * item.array;
    bool ok = true;
    if (item.kind == PL_XENG || item.kind == PL_XMFMA)
      ok = plan_wait(done_chan, (unsigned)(Ap->n_chan_items + a.wait_bias), err, a.wait_ticks, wave,
                     &s_flag);
    else if (item.kind == PL_REDUCE)
      ok = plan_wait(done_part, (unsigned)(Ap->n_part_items + a.wait_bias), err, a.wait_ticks, wave,
                     &s_flag);
    if (ok) {
      const int N = Ap->n_fft, NA = Ap->n_ant;
      if (item.kind == PL_FUSED) {
        if (N == 1024) plan_fused<1024, 4>(Ap, item.index, buf);
        else if (N == 2048) plan_fused<2048, 4>(Ap, item.index, buf);
        else plan_fused<4096, 4>(Ap, item.index, buf);
      } else if (item.kind == PL_CHAN) {
        switch (N) {
          case 16: plan_chan<16>(Ap, item.index, buf); break;
          case 32: plan_chan<32>(Ap, item.index, buf); break;
          case 64: plan_chan<64>(Ap, item.index, buf); break;
          case 128: plan_chan<128>(Ap, item.index, buf); break;
          case 256: plan_chan<256>(Ap, item.index, buf); break;
          case 512: plan_chan<512>(Ap, item.index, buf); break;
          case 1024: plan_chan<1024>(Ap, item.index, buf); break;
          case 2048: plan_chan<2048>(Ap, item.index, buf); break;
          case 4096: plan_chan<4096>(Ap, item.index, buf); break;
          case 8192: plan_chan<8192>(Ap, item.index, buf); break;
        }
      } else if (item.kind == PL_CHAN_RING) {
        if (N == 2048) plan_chan_ring<2048, 8>(Ap, item.index, buf);
        else if (N == 4096) plan_chan_ring<4096, 4>(Ap, item.index, buf);
        else plan_chan_ring<8192, 2>(Ap, item.index, buf);
      } else if (item.kind == PL_XENG) {
        xeng_item(Ap, item.index);
      } else if (item.kind == PL_XMFMA) {
        plan_xmfma(Ap, item.index, buf);
      } else {
        reduce_item(Ap, item.index);
      }
    }
    if (item.kind != PL_REDUCE) {
      // publish.  What an item hands on (spectra, partials) was written
      // with agent-scope stores (st_f2<true>), which write through the L2;
      // every wave waits until its stores are complete, the barrier joins
      // the waves, and one increment counts the item done (skipped items
      // count too).  The consumers' acquire (plan_wait) invalidates their
      // L2.  An agent-scope release here would also write back the whole
      // L2 of this XCD, about 20 us per item.
      __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
      __syncthreads();
      if (wave == 0)
        __hip_atomic_fetch_add((item.kind == PL_CHAN || item.kind == PL_CHAN_RING) ? done_chan : done_part,
                               (threadIdx.x & 63u) == 0u ? 1u : 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __syncthreads();  // LDS and s_item reuse
    }
  }
}


hipError_t prepare_plan() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(plan_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)PLAN_LDS);
}

hipError_t launch_plan(const PlArgs& a, int grid, hipStream_t s) {
  const int nctr = 2 + 2 * PL_MAX_ARRAYS;
  hipError_t e = launch(plan_reset_kernel, dim3(1), dim3(64), 0, s, a.ctr, nctr);
  if (e != hipSuccess) return e;
  return launch(plan_kernel, dim3(grid), dim3(PL_NT), PLAN_LDS, s, a);
}

}  // namespace qc
