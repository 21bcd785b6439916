// Device building blocks of the F-engine: complex helpers, register DFTs of
// size 2..16 and an LDS-resident Stockham FFT for N = 2^n, 4 <= N <= 8192.
//
// Transform convention: forward kernel exp(-2 pi i k n / N), unnormalised
// (the DFT of the F-engine, Sec. 4.1 step 1 / Sec. 4.2).  The FFT is
// Cooley-Tukey (1965) in Stockham's self-sorting form: pass s combines
// sub-transforms of length Ns into length Ns*R with twiddles
// W_{Ns R}^{(j mod Ns) r}, reading at stride N/R and writing in natural
// order, so no bit-reversal pass is needed.  Radix 16 is used while it
// divides what is left, then one pass of the remaining radix.
//
// Work split: every thread holds exactly 16 complex values per pass (one
// radix-16 butterfly, two radix-8, four radix-4 or eight radix-2), so a
// group of NFFT transforms of length N needs NFFT*N/16 threads.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qc {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * (-i)
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }

// W_8^1 = (1 - i)/sqrt(2), W_8^3 = (-1 - i)/sqrt(2)
__device__ __forceinline__ float2 cmul_w8_1(float2 a) {
  const float s = 0.70710678118654752f;
  return make_float2((a.x + a.y) * s, (a.y - a.x) * s);
}
__device__ __forceinline__ float2 cmul_w8_3(float2 a) {
  const float s = 0.70710678118654752f;
  return make_float2((a.y - a.x) * s, -(a.x + a.y) * s);
}

// In-place forward DFTs, natural order in and out.
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

__device__ __forceinline__ void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  float2 a = cadd(x0, x2), b = csub(x0, x2);
  float2 c = cadd(x1, x3), d = cmul_mi(csub(x1, x3));
  x0 = cadd(a, c);
  x2 = csub(a, c);
  x1 = cadd(b, d);
  x3 = csub(b, d);
}

// 8 = 2 x 4: even/odd 4-point transforms, then W_8^k combination.
__device__ __forceinline__ void dft8(float2* v) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  o1 = cmul_w8_1(o1);
  o2 = cmul_mi(o2);
  o3 = cmul_w8_3(o3);
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.
//   A_{n2}[k1] = DFT4_{n1}(x[4 n1 + n2]);  A_{n2}[k1] *= W16^{n2 k1};
//   X[k1 + 4 k2] = DFT4_{n2}(A_{n2}[k1]).
__device__ __forceinline__ void dft16(float2* v) {
  const float c1 = 0.92387953251128676f;  // cos(pi/8)
  const float s1 = 0.38268343236508977f;  // sin(pi/8)
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // after this, A_{n2}[k1] lives in v[4*k1 + n2]
  // n2 = 1: W16^{k1} for k1 = 1, 2, 3
  v[5] = make_float2(v[5].x * c1 + v[5].y * s1, v[5].y * c1 - v[5].x * s1);   // W16^1
  v[9] = cmul_w8_1(v[9]);                                                        // W16^2
  v[13] = make_float2(v[13].x * s1 + v[13].y * c1, v[13].y * s1 - v[13].x * c1); // W16^3
  // n2 = 2: W16^{2 k1}
  v[6] = cmul_w8_1(v[6]);   // W16^2
  v[10] = cmul_mi(v[10]);   // W16^4
  v[14] = cmul_w8_3(v[14]); // W16^6
  // n2 = 3: W16^{3 k1}
  v[7] = make_float2(v[7].x * s1 + v[7].y * c1, v[7].y * s1 - v[7].x * c1);      // W16^3
  v[11] = cmul_w8_3(v[11]);                                                       // W16^6
  v[15] = make_float2(-v[15].x * c1 - v[15].y * s1, -v[15].y * c1 + v[15].x * s1); // W16^9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  // X[k1 + 4 k2] now in v[4*k1 + k2]: transpose 4x4 to natural order
  float2 t;
  t = v[1]; v[1] = v[4]; v[4] = t;
  t = v[2]; v[2] = v[8]; v[8] = t;
  t = v[3]; v[3] = v[12]; v[12] = t;
  t = v[6]; v[6] = v[9]; v[9] = t;
  t = v[7]; v[7] = v[13]; v[13] = t;
  t = v[11]; v[11] = v[14]; v[14] = t;
}

template <int R>
__device__ __forceinline__ void dft_r(float2* v) {
  if constexpr (R == 2) dft2(v[0], v[1]);
  else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8(v);
  else if constexpr (R == 16) dft16(v);
  else static_assert(R == 2 || R == 4 || R == 8 || R == 16, "radix");
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// LDS index with one pad slot per 16 complex values (breaks the power-of-two
// strides of the Stockham reads and writes across banks).
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_padded_size(int n) { return n + (n >> 4) + 1; }

// One Stockham pass of radix R over NFFT transforms of length N stored back
// to back (padded).  NT threads each hold V complex values (V/R butterflies).
// With INPLACE the pass reads and writes the same buffer, so a barrier
// separates all loads from all stores; otherwise src and dst differ.
// Twiddle layouts.  TWL = false: tw[e] = W_N^e, e = 0..N-1 (read at
// e = jm*r*N/(NS*R)).  TWL = true: per-pass tables, the pass with stride NS
// holding T[(NS-1) + (r-1)*NS + jm] = W_{NS R}^{jm r}; for a fixed r the
// lanes of a wave then read consecutive entries (no LDS bank conflicts).
// Over all passes the per-pass tables take exactly N-1 entries.
template <int N, int V>
__device__ __forceinline__ void build_pass_twiddles(float2* dst, const float2* __restrict__ tw, int tid,
                                                    int nt) {
  for (int i = tid; i < N - 1; i += nt) {
    // find the pass: offsets NS-1 for NS = 1, R1, R1*R2, ...
    int ns = 1, off = 0;
    while (true) {
      const int R = (N / ns) >= V ? V : (N / ns);
      const int size = (R - 1) * ns;
      if (i < off + size || ns * R >= N) {
        const int q = i - off;
        const int r = 1 + q / ns, jm = q % ns;
        dst[i] = tw[jm * r * (N / (ns * R))];
        break;
      }
      off += size;
      ns *= R;
    }
  }
}

// TWG > 0 (with TWL): the table twiddles are read in groups of TWG, each
// group issued together so it waits once instead of once per read (for
// kernels with the registers to hold a group).
template <int N, int R, int NS, int NT, int V, bool INPLACE, bool LN, bool TWL = false, int TWG = 0>
__device__ __forceinline__ void stockham_pass(const float2* src, float2* dst,
                                              const float2* __restrict__ tw, int tid) {
  // Twiddles and LDS addresses depend only on the thread index, so the
  // compiler would hoist every pass's twiddle loads and address arithmetic
  // out of the caller's spectrum loop and keep them live in registers.
  // Hiding the values here (LN) keeps that work inside the pass, for blocks
  // whose register budget cannot afford to keep them.
  if constexpr (LN) {
    asm volatile("" : "+s"(tw));
    asm volatile("" : "+v"(tid));
  }
  constexpr int Q = V / R;   // butterflies per thread
  constexpr int NB = N / R;  // butterflies per transform
  static_assert(Q >= 1, "radix larger than the values a thread holds");
  float2 v[Q][R];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int q = tid + i * NT;
    const int f = q / NB, j = q % NB;
#pragma unroll
    for (int r = 0; r < R; ++r) v[i][r] = src[lds_pad(f * N + j + r * NB)];
  }
  if constexpr (INPLACE) __syncthreads();
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int q = tid + i * NT;
    const int f = q / NB, j = q % NB;
    const int jm = j % NS;
    if constexpr (NS > 1 && TWL && TWG > 0) {
#pragma unroll
      for (int r0 = 1; r0 < R; r0 += TWG) {
        float2 wt[TWG];
#pragma unroll
        for (int u = 0; u < TWG; ++u)
          if (r0 + u < R) wt[u] = tw[(NS - 1) + (r0 + u - 1) * NS + jm];
#pragma unroll
        for (int u = 0; u < TWG; ++u)
          if (r0 + u < R) v[i][r0 + u] = cmul(v[i][r0 + u], wt[u]);
      }
    } else if constexpr (NS > 1) {
      constexpr int STEP = N / (NS * R);
#pragma unroll
      for (int r = 1; r < R; ++r)
        v[i][r] = cmul(v[i][r], TWL ? tw[(NS - 1) + (r - 1) * NS + jm] : tw[jm * r * STEP]);
    }
    dft_r<R>(v[i]);
    const int k = (j / NS) * NS * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[lds_pad(f * N + k + r * NS)] = v[i][r];
  }
  __syncthreads();
}

constexpr int fft_radix(int rem, int V) { return rem >= V ? V : rem; }

constexpr int fft_pass_count(int N, int V) {
  int c = 0;
  for (int ns = 1; N / ns > 1; ns *= fft_radix(N / ns, V)) ++c;
  return c;
}

// Passes NS.. of a Stockham FFT.  PP selects ping-pong buffers: pass p reads
// buffer p%2 and writes buffer (p+1)%2 (one barrier per pass); without PP
// every pass works in place in buffer 0 (two barriers per pass).
template <int N, int NS, int NT, int V, bool PP, bool LN, int PASS, bool TWL = false>
__device__ __forceinline__ void fft_passes(float2* b0, float2* b1, const float2* __restrict__ tw,
                                           int tid) {
  constexpr int REM = N / NS;
  if constexpr (REM > 1) {
    constexpr int R = fft_radix(REM, V);
    if constexpr (PP) {
      float2* src = (PASS % 2 == 0) ? b0 : b1;
      float2* dst = (PASS % 2 == 0) ? b1 : b0;
      stockham_pass<N, R, NS, NT, V, false, LN, TWL>(src, dst, tw, tid);
    } else {
      stockham_pass<N, R, NS, NT, V, true, LN, TWL>(b0, b0, tw, tid);
    }
    fft_passes<N, NS * R, NT, V, PP, LN, PASS + 1, TWL>(b0, b1, tw, tid);
  }
}

// NFFT forward transforms of length N, natural order in and out, each
// thread holding V values per pass (NT = NFFT*N/V threads).  The input is
// read from b0; the output is in b0, or in b(fft_pass_count % 2) with
// ping-pong.  Must be called by all NT threads of the block; begins with
// the block synchronised and ends with a barrier.
template <int N, int NT, int V, bool PP, bool LN = false, bool TWL = false>
struct Fft {
  static constexpr int PASSES = fft_pass_count(N, V);
  static constexpr int OUT = PP ? (PASSES % 2) : 0;
  static __device__ __forceinline__ void run(float2* b0, float2* b1, const float2* __restrict__ tw,
                                             int tid) {
    fft_passes<N, 1, NT, V, PP, LN, 0, TWL>(b0, b1, tw, tid);
  }
};

// In-place, 16 values per thread (NT = NFFT*N/16).
template <int N, int NT>
__device__ __forceinline__ void fft_lds(float2* buf, const float2* __restrict__ tw, int tid) {
  Fft<N, NT, 16, false, (NT >= 1024)>::run(buf, buf, tw, tid);
}

}  // namespace qc
