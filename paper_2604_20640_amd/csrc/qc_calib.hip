// MAD flagging and delay/phase application for gfx950.
//
// MAD (arXiv 2604.20640 Sec. 7, eq. 2): T = median(A) + sigma*1.4826*MAD(A)
// on the visibility amplitude A; flag A > T.  Medians are exact order
// statistics found by radix selection (most significant digit first) over
// the bit patterns of non-negative floats, whose unsigned order equals their
// numeric order: float32 amplitudes and float64 deviations |A - median|.
// Even counts average the two middle order statistics; the upper one comes
// from the lower by one counting pass.  One workgroup
// handles one population; its amplitudes are cached in LDS when they fit
// (1024 threads and 11-bit digits for large populations, one wave and 8-bit
// digits for small ones).
//
// Delay/phase application (Sec. 4.1 step 2 and eq. 1; Sec. 7 delay and phase
// corrections): V_ij[k] *= exp(+i [2 pi f_k (tau_i - tau_j) + phi_i - phi_j]).
// The rotation is formed in float64: cycles = f_k (tau_i - tau_j) +
// (phi_i - phi_j)/(2 pi), reduced modulo 1, then sincospi.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qc_kernels.h"

namespace qc {

namespace {

// Every float64 step of the threshold is a separately rounded IEEE operation
// (no contraction into fused multiply-adds), so the decisions match a plain
// float64 evaluation of the same expressions bit for bit.
#pragma clang fp contract(off)

struct Pop {
  int64_t base, count, inner_n, s_inner, s_outer;
  __device__ __forceinline__ int64_t off(int64_t i) const {
    return base + (i / inner_n) * s_outer + (i % inner_n) * s_inner;
  }
};

__device__ __forceinline__ float amp_f32(float2 v) {
  const double re = (double)v.x, im = (double)v.y;
  return (float)sqrt(re * re + im * im);
}

// Amplitudes of a population: from an LDS cache when it fits, else from a
// materialised amplitude array, else recomputed from vis.
struct AmpSrc {
  const float2* vis;
  Pop pop;
  const float* cache;  // LDS copy, or the population's slice of the materialised array; may be null
  __device__ __forceinline__ float operator()(int64_t i) const {
    return cache ? cache[i] : amp_f32(vis[pop.off(i)]);
  }
};

// Block-wide search of the digit that holds rank kk in hist[0..NBINS):
// returns (digit, rank within the digit) through sh[].
template <int NT, int NBINS>
__device__ __forceinline__ void find_digit(const unsigned* hist, int64_t kk, unsigned* wsum,
                                           unsigned long long* sh) {
  constexpr int PER = NBINS / NT;  // bins per thread (>= 1)
  constexpr int NW = NT / 64;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  unsigned loc = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) loc += hist[t * PER + i];
  unsigned v = loc;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned n = __shfl_up(v, d);
    if (lane >= d) v += n;
  }
  if (NW > 1) {
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    if (t == 0) {
      unsigned acc = 0;
      for (int w = 0; w < NW; ++w) {
        acc += wsum[w];
        wsum[w] = acc;
      }
    }
    __syncthreads();
  }
  const int64_t incl = (int64_t)v + ((NW > 1 && wave > 0) ? wsum[wave - 1] : 0u);
  const int64_t excl = incl - loc;
  if (excl <= kk && kk < incl) {
    int64_t c = excl;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const unsigned h = hist[t * PER + i];
      if (kk < c + (int64_t)h) {
        sh[0] = (unsigned long long)(t * PER + i);
        sh[1] = (unsigned long long)(kk - c);
        break;
      }
      c += h;
    }
  }
  __syncthreads();
}

// k-th smallest (0-based) key of the population, most significant digit
// first.  KEY(i) returns the unsigned key of element i; W is the key width.
template <int NT, int DB, typename K, typename KeyFn>
__device__ K radix_select(int64_t count, int64_t k, KeyFn key, unsigned* hist, unsigned* wsum,
                          unsigned long long* sh, unsigned long long* red) {
  constexpr int W = (int)sizeof(K) * 8;
  constexpr int NBINS = 1 << DB;
  // the leading bits that every key shares need no histogram pass (and
  // would send every count of the first pass to one bin): start below them
  K kmin = ~(K)0, kmax = 0;
  for (int64_t i = threadIdx.x; i < count; i += NT) {
    const K kv = key(i);
    kmin = kv < kmin ? kv : kmin;
    kmax = kv > kmax ? kv : kmax;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const K a = (K)__shfl_down((unsigned long long)kmin, d);
    const K b = (K)__shfl_down((unsigned long long)kmax, d);
    kmin = a < kmin ? a : kmin;
    kmax = b > kmax ? b : kmax;
  }
  if ((threadIdx.x & 63) == 0) {
    red[2 * (threadIdx.x >> 6)] = (unsigned long long)kmin;
    red[2 * (threadIdx.x >> 6) + 1] = (unsigned long long)kmax;
  }
  __syncthreads();
  kmin = ~(K)0;
  kmax = 0;
  for (int w = 0; w < NT / 64; ++w) {
    const K a = (K)red[2 * w], b = (K)red[2 * w + 1];
    kmin = a < kmin ? a : kmin;
    kmax = b > kmax ? b : kmax;
  }
  __syncthreads();
  const K diff = kmin ^ kmax;
  if (diff == 0) return kmin;
  int top = W - 1;  // highest differing bit
  while (!((diff >> top) & (K)1)) --top;
  const K low = (top + 1 >= W) ? ~(K)0 : (((K)1 << (top + 1)) - 1);
  K prefix = kmin & ~low, mask = ~low;
  int64_t kk = k;
  for (int hi = top + 1; hi > 0; hi -= DB) {
    const int width = hi >= DB ? DB : hi;
    const int shift = hi - width;
    const K dmask = (K)((1u << width) - 1u);
    for (int i = threadIdx.x; i < NBINS; i += NT) hist[i] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < count; i += NT) {
      const K kv = key(i);
      if ((kv & mask) == prefix) atomicAdd(&hist[(unsigned)((kv >> shift) & dmask)], 1u);
    }
    __syncthreads();
    find_digit<NT, NBINS>(hist, kk, wsum, sh);
    prefix |= (K)sh[0] << shift;
    mask |= dmask << shift;
    kk = (int64_t)sh[1];
    __syncthreads();
  }
  return prefix;
}

// The order statistic of rank k+1 given the one of rank k (key kk): kk
// itself if more than k+1 keys are <= kk, else the smallest key above kk.
// One pass: a count and a minimum, reduced over the block.
template <int NT, typename K, typename KeyFn>
__device__ K next_rank(int64_t count, int64_t k, K kk, KeyFn key, unsigned long long* red) {
  constexpr int NW = NT / 64;
  unsigned long long le = 0;
  K mn = ~(K)0;
  for (int64_t i = threadIdx.x; i < count; i += NT) {
    const K kv = key(i);
    if (kv <= kk) ++le;
    else if (kv < mn) mn = kv;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    le += __shfl_down(le, d);
    const K o = (K)__shfl_down((unsigned long long)mn, d);
    mn = o < mn ? o : mn;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[2 * wave] = le;
    red[2 * wave + 1] = (unsigned long long)mn;
  }
  __syncthreads();
  unsigned long long tle = 0;
  K tmn = ~(K)0;
  for (int w = 0; w < NW; ++w) {
    tle += red[2 * w];
    const K o = (K)red[2 * w + 1];
    tmn = o < tmn ? o : tmn;
  }
  __syncthreads();
  return (int64_t)tle > k + 1 ? kk : tmn;
}

__device__ __forceinline__ Pop make_pop(int64_t id, int64_t n_time, int64_t n_base, int n_chan,
                                        int population) {
  const int64_t plane = n_base * (int64_t)n_chan;
  if (population == 0) return Pop{id * n_chan, n_time * n_chan, n_chan, 1, plane};
  if (population == 1) {
    const int64_t b = id / n_chan, k = id % n_chan;
    return Pop{b * n_chan + k, n_time, 1, 0, plane};
  }
  const int64_t t = id / n_base, b = id % n_base;
  return Pop{t * plane + b * n_chan, n_chan, n_chan, 1, 0};
}

}  // namespace

// One block per population.  Amplitudes are cached in dynamic LDS when the
// population has at most `cap` members.
// Amplitudes of every population, each population contiguous:
// amp[id * count + i] = |V| of its element i (as amp_f32).
__global__ void mad_amp_kernel(const float2* __restrict__ vis, int64_t n_time, int64_t n_base, int n_chan,
                               int population, int64_t count, int64_t total, float* __restrict__ amp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t id = e / count, i = e % count;
  amp[e] = amp_f32(vis[make_pop(id, n_time, n_base, n_chan, population).off(i)]);
}

template <int NT, int DB>
__global__ void __launch_bounds__(NT)
mad_kernel(const float2* __restrict__ vis, int64_t n_time, int64_t n_base, int n_chan, float sigma,
           int population, int64_t cap, const float* __restrict__ gamp, uint8_t* __restrict__ mask,
           double* __restrict__ thresh, double* __restrict__ stats) {
  __shared__ unsigned hist[1 << DB];
  __shared__ unsigned wsum[NT / 64];
  __shared__ unsigned long long sh[2];
  __shared__ unsigned long long red[2 * (NT / 64)];
  extern __shared__ float acache[];
  const int64_t id = blockIdx.x;
  const Pop pop = make_pop(id, n_time, n_base, n_chan, population);
  const int64_t n = pop.count;
  const bool cached = n <= cap;
  if (cached) {
    for (int64_t i = threadIdx.x; i < n; i += NT)
      acache[i] = gamp ? gamp[id * n + i] : amp_f32(vis[pop.off(i)]);
    __syncthreads();
  }
  const AmpSrc amp{vis, pop, cached ? acache : (gamp ? gamp + id * n : nullptr)};
  const int64_t k1 = (n - 1) / 2, k2 = n / 2;
  auto akey = [&](int64_t i) -> uint32_t { return __float_as_uint(amp(i)); };
  const uint32_t a1 = radix_select<NT, DB, uint32_t>(n, k1, akey, hist, wsum, sh, red);
  const uint32_t a2 = (k2 == k1) ? a1 : next_rank<NT, uint32_t>(n, k1, a1, akey, red);
  const double med = ((double)__uint_as_float(a1) + (double)__uint_as_float(a2)) / 2.0;
  auto dkey = [&](int64_t i) -> uint64_t {
    return (uint64_t)__double_as_longlong(fabs((double)amp(i) - med));
  };
  const uint64_t d1 = radix_select<NT, DB, uint64_t>(n, k1, dkey, hist, wsum, sh, red);
  const uint64_t d2 = (k2 == k1) ? d1 : next_rank<NT, uint64_t>(n, k1, d1, dkey, red);
  const double madv =
      (__longlong_as_double((long long)d1) + __longlong_as_double((long long)d2)) / 2.0;
  const double c = (double)sigma * 1.4826;
  const double T = med + c * madv;
  if (mask)
    for (int64_t i = threadIdx.x; i < n; i += NT) mask[pop.off(i)] = (double)amp(i) > T ? 1 : 0;
  if (threadIdx.x == 0) {
    if (thresh) thresh[id] = T;
    if (stats) {
      stats[2 * id] = med;
      stats[2 * id + 1] = madv;
    }
  }
}

#pragma clang fp contract(on)

constexpr int64_t MAD_CAP_BIG = 36864;   // floats cached in LDS (144 KiB)
constexpr int64_t MAD_CAP_SMALL = 2048;

int64_t mad_scratch_floats(int64_t n_time, int64_t n_base, int n_chan, int population) {
  const int64_t npop = population == 0 ? n_base : population == 1 ? n_base * n_chan : n_time * n_base;
  const int64_t count = population == 0 ? n_time * n_chan : population == 1 ? n_time : n_chan;
  return count > MAD_CAP_BIG ? npop * count : 0;
}

hipError_t launch_mad(const float2* vis, int64_t n_time, int64_t n_base, int n_chan, float sigma,
                      int population, uint8_t* mask, double* thresh, double* stats, float* amp_scratch,
                      hipStream_t s) {
  const int64_t npop = population == 0 ? n_base : population == 1 ? n_base * n_chan : n_time * n_base;
  const int64_t count = population == 0 ? n_time * n_chan : population == 1 ? n_time : n_chan;
  if (npop <= 0) return hipSuccess;
  if (count <= MAD_CAP_SMALL) {
    const size_t lds = (size_t)count * sizeof(float);
    hipLaunchKernelGGL((mad_kernel<64, 8>), dim3((unsigned)npop), dim3(64), lds, s, vis, n_time,
                       n_base, n_chan, sigma, population, MAD_CAP_SMALL, nullptr, mask, thresh, stats);
  } else {
    const int64_t cap = count <= MAD_CAP_BIG ? count : 0;
    const float* gamp = nullptr;
    if (cap == 0 && amp_scratch) {
      // populations beyond the LDS cache: their amplitudes are formed once
      // and every selection pass reads 4 bytes instead of 8 and a square root
      const int64_t total = npop * count;
      hipLaunchKernelGGL(mad_amp_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, vis, n_time,
                         n_base, n_chan, population, count, total, amp_scratch);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      gamp = amp_scratch;
    }
    const size_t lds = (size_t)cap * sizeof(float);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(mad_kernel<1024, 11>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((mad_kernel<1024, 11>), dim3((unsigned)npop), dim3(1024), lds, s, vis, n_time,
                       n_base, n_chan, sigma, population, cap, gamp, mask, thresh, stats);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Delay/phase application.
// ---------------------------------------------------------------------------
constexpr int APPLY_MAX_ANT = 64;
struct AntTable {
  double tau[APPLY_MAX_ANT];
  double phi[APPLY_MAX_ANT];
};

__global__ void __launch_bounds__(256)
apply_kernel(float2* __restrict__ vis, int n_ant, int n_chan, double f0, double df, AntTable t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_chan) return;
  int b = blockIdx.y, i = 0;
  while (b >= n_ant - i) { b -= n_ant - i; ++i; }
  const int j = i + b;
  if (i == j) return;  // zero rotation: autos unchanged
  const double inv2pi = 0.15915494309189533577;
  const double fk = f0 + (double)k * df;
  double cyc = fk * (t.tau[i] - t.tau[j]) + (t.phi[i] - t.phi[j]) * inv2pi;
  cyc -= rint(cyc);
  double sn, cs;
  sincospi(2.0 * cyc, &sn, &cs);
  const int64_t nb = (int64_t)n_ant * (n_ant + 1) / 2;
  float2* p = vis + ((int64_t)blockIdx.z * nb + blockIdx.y) * n_chan + k;
  const float2 v = *p;
  const double re = (double)v.x * cs - (double)v.y * sn;
  const double im = (double)v.x * sn + (double)v.y * cs;
  *p = make_float2((float)re, (float)im);
}

hipError_t launch_apply(float2* vis, int64_t n_time, int n_ant, int n_chan, double f0, double df,
                        const double* tau, const double* phi, hipStream_t s) {
  if (n_ant > APPLY_MAX_ANT) return hipErrorInvalidValue;
  AntTable t{};
  for (int a = 0; a < n_ant; ++a) {
    t.tau[a] = tau[a];
    t.phi[a] = phi[a];
  }
  const int nb = n_ant * (n_ant + 1) / 2;
  if (n_time <= 0 || nb <= 0 || n_chan <= 0) return hipSuccess;
  dim3 grid((unsigned)((n_chan + 255) / 256), (unsigned)nb, (unsigned)n_time);
  hipLaunchKernelGGL(apply_kernel, grid, dim3(256), 0, s, vis, n_ant, n_chan, f0, df, t);
  return hipGetLastError();
}

}  // namespace qc
