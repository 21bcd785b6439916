// MAD flagging and delay/phase application for gfx950.
//
// MAD (arXiv 2604.20640 Sec. 7, eq. 2): T = median(A) + sigma*1.4826*MAD(A)
// on the visibility amplitude A; flag A > T.  Medians are exact order
// statistics found by radix selection (most significant digit first) over
// the bit patterns of non-negative floats, whose unsigned order equals their
// numeric order: float32 amplitudes and float64 deviations |A - median|.
// The key range comes for free (amplitudes: a min/max taken while they are
// loaded; deviations: [0, the larger deviation of the extreme amplitudes]),
// so bits shared by the whole range need no pass.  Once the digit holding
// the wanted rank contains at most SEL_CAND keys, one pass gathers them and
// one wave ranks them.  Even counts average the two middle order
// statistics; the upper one is read off the same candidates when it lies
// among them (else one counting pass finds it).  Once the digit holding the
// wanted rank has few enough keys for the LDS left over, their values are
// compacted into LDS and the remaining passes scan only them.  One workgroup handles one
// population (1024 threads and 11-bit digits for large populations, one
// wave and 8-bit digits for small ones); large populations get their
// amplitudes formed once by a whole-GPU pass and cached in LDS when they
// fit.
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
    // 32-bit division when the index and the inner extent fit (every
    // population but the very largest): a fraction of the 64-bit sequence
    if (i <= 0x7fffffffLL && inner_n <= 0x7fffffffLL) {
      const uint32_t q = (uint32_t)i / (uint32_t)inner_n;
      const uint32_t r = (uint32_t)i - q * (uint32_t)inner_n;
      return base + (int64_t)q * s_outer + (int64_t)r * s_inner;
    }
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

// A block-uniform 64-bit value read back from LDS, made wave-uniform for
// the compiler (branches on it hold barriers).
__device__ __forceinline__ int64_t rfl64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

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
  // each thread adds the totals of the waves before its own (independent
  // broadcast reads instead of one thread's serial prefix and a barrier)
  unsigned before = 0u;
  if (NW > 1) {
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NW; ++w) before += w < wave ? wsum[w] : 0u;
  }
  const int64_t incl = (int64_t)v + before;
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

// Keys of a selection that are still candidates once few remain: they are
// gathered and ranked by one wave instead of further histogram passes.
constexpr int SEL_CAND = 64;

// fn(i, key(i)) for this thread's elements i = threadIdx.x + NT j.  The
// large-population kernel forms its keys in batches of 8 so that as many
// loads are in flight per thread (populations read from global memory are
// latency-bound otherwise); the one-wave kernel reads LDS and keeps one.
template <int NT, typename K, typename KeyFn, typename Fn>
__device__ __forceinline__ void for_keys(int64_t count, KeyFn key, Fn fn) {
  constexpr int B = NT >= 256 ? 8 : 1;
  int64_t i = threadIdx.x;
  if constexpr (B > 1) {
    for (; i + (int64_t)(B - 1) * NT < count; i += (int64_t)B * NT) {
      K kv[B];
#pragma unroll
      for (int u = 0; u < B; ++u) kv[u] = key(i + (int64_t)u * NT);
#pragma unroll
      for (int u = 0; u < B; ++u) fn(i + (int64_t)u * NT, kv[u]);
    }
  }
  for (; i < count; i += NT) fn(i, key(i));
}

struct SelScratch {
  unsigned* hist;            // 2^DB bins
  unsigned* wsum;            // NT / 64
  unsigned long long* sh;    // 4
  unsigned long long* red;   // 2 * NT / 64
  unsigned long long* cand;  // SEL_CAND
  unsigned* ncand;           // 1
  float* comp;               // compacted values still in play (LDS), comp_cap of them
  int64_t comp_cap;          // 0: no compaction
};

// Appends v to sc.comp where hit, one LDS atomic per wave: the lanes that
// hit take consecutive slots after the count so far.
__device__ __forceinline__ void append_wave(const SelScratch& sc, bool hit, float v) {
  const unsigned long long bal = __ballot(hit);
  if (bal == 0ull) return;
  const int lane = (int)(threadIdx.x & 63u);
  const int leader = __ffsll((long long)bal) - 1;
  unsigned base = 0u;
  if (lane == leader) base = atomicAdd(sc.ncand, (unsigned)__popcll(bal));
  base = __shfl(base, leader);
  if (hit) sc.comp[base + (unsigned)__popcll(bal & ((1ull << lane) - 1ull))] = v;
}

// k-th smallest (0-based) key of the population, most significant digit
// first, for keys known to lie in [kmin, kmax].  Element i has the value
// VAL(i) and the unsigned key KEYOF(value).  Bits that every key in the
// range shares need no pass.  Once the digit that holds rank k has at most
// comp_cap keys, one pass copies their values into sc.comp and every later
// pass scans only those.  When it has at most SEL_CAND keys, one pass
// gathers them and one wave ranks them.  With want2, the key of rank k+1 is
// also returned (has2) when it lies among the same candidates.
template <int NT, int DB, typename K, typename ValFn, typename KeyOf>
__device__ __forceinline__ K radix_select(int64_t count, int64_t k, K kmin, K kmax, ValFn val, KeyOf keyof,
                          const SelScratch& sc, bool want2, K& v2, bool& has2) {
  constexpr int W = (int)sizeof(K) * 8;
  constexpr int NBINS = 1 << DB;
  has2 = false;
  // the range and counts are block-uniform; say so to the compiler, so the
  // pass loop below (barriers inside) is a scalar loop
  if constexpr (sizeof(K) == 8) {
    kmin = (K)rfl64((int64_t)kmin);
    kmax = (K)rfl64((int64_t)kmax);
  } else {
    kmin = (K)__builtin_amdgcn_readfirstlane((int)kmin);
    kmax = (K)__builtin_amdgcn_readfirstlane((int)kmax);
  }
  count = rfl64(count);
  k = rfl64(k);
  const K diff = kmin ^ kmax;
  if (diff == 0) {  // every key equals kmin
    v2 = kmin;
    has2 = true;
    return kmin;
  }
  int top = W - 1;  // highest differing bit
  while (!((diff >> top) & (K)1)) --top;
  top = __builtin_amdgcn_readfirstlane(top);
  const K low = (top + 1 >= W) ? ~(K)0 : (((K)1 << (top + 1)) - 1);
  K prefix = kmin & ~low, mask = ~low;
  int64_t kk = k;
  // keys scanned per pass: the whole population, or its compacted part
  bool compact = false;
  int64_t n_in = count;
  auto key = [&](int64_t i) -> K { return compact ? keyof(sc.comp[i]) : keyof(val(i)); };
  for (int hi = top + 1; hi > 0; hi -= DB) {
    const int width = hi >= DB ? DB : hi;
    const int shift = hi - width;
    const K dmask = (K)((1u << width) - 1u);
    for (int i = threadIdx.x; i < NBINS; i += NT) sc.hist[i] = 0;
    __syncthreads();
    for_keys<NT, K>(n_in, key, [&](int64_t, K kv) {
      if ((kv & mask) == prefix) atomicAdd(&sc.hist[(unsigned)((kv >> shift) & dmask)], 1u);
    });
    __syncthreads();
    find_digit<NT, NBINS>(sc.hist, kk, sc.wsum, sc.sh);
    // block-uniform values read back from LDS: made wave-uniform, so that
    // the branches and loop exits that depend on them are scalar
    const unsigned digit = (unsigned)__builtin_amdgcn_readfirstlane((int)sc.sh[0]);
    int64_t c = (int64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)sc.hist[digit]);  // keys sharing the extended prefix
    prefix |= (K)digit << shift;
    mask |= dmask << shift;
    kk = rfl64((int64_t)sc.sh[1]);
    __syncthreads();
    if (shift == 0) {  // all bits resolved: the key is the prefix, repeated c times
      if (want2 && kk + 1 < c) {
        v2 = prefix;
        has2 = true;
      }
      return prefix;
    }
    if (c <= SEL_CAND) {
      // With rank k the largest key of its digit, rank k+1 is the smallest
      // key of the next non-empty digit of this pass: gather that digit
      // too when both fit.
      K prefix2 = prefix;
      int64_t c2 = 0;
      if (want2 && kk + 1 == c) {
        if (threadIdx.x == 0) *sc.ncand = NBINS;
        __syncthreads();
        for (int b = (int)digit + 1 + threadIdx.x; b < NBINS; b += NT)
          if (sc.hist[b] != 0u) atomicMin(sc.ncand, (unsigned)b);
        __syncthreads();
        const unsigned d2 = (unsigned)__builtin_amdgcn_readfirstlane((int)*sc.ncand);
        if (d2 < (unsigned)NBINS && c + (int64_t)sc.hist[d2] <= SEL_CAND) {
          prefix2 = (prefix & ~(dmask << shift)) | ((K)d2 << shift);
          c2 = sc.hist[d2];
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) *sc.ncand = 0;
      __syncthreads();
      for_keys<NT, K>(n_in, key, [&](int64_t, K kv) {
        const K km = kv & mask;
        if (km == prefix || (c2 > 0 && km == prefix2))
          sc.cand[atomicAdd(sc.ncand, 1u)] = (unsigned long long)kv;
      });
      c += c2;
      __syncthreads();
      if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const K mine = lane < c ? (K)sc.cand[lane] : ~(K)0;
        int64_t less = 0, same = 0;
        for (int t = 0; t < (int)c; ++t) {
          const K o = (K)sc.cand[t];
          less += o < mine;
          same += o == mine;
        }
        // a lane whose key covers rank kk (ties write the same value)
        if (lane < c && less <= kk && kk < less + same) sc.sh[2] = (unsigned long long)mine;
        if (lane < c && less <= kk + 1 && kk + 1 < less + same) sc.sh[3] = (unsigned long long)mine;
      }
      __syncthreads();
      const K v1 = (K)sc.sh[2];
      if (want2 && kk + 1 < c) {
        v2 = (K)sc.sh[3];
        has2 = true;
      }
      __syncthreads();
      return v1;
    }
    if (!compact && c <= sc.comp_cap) {
      // the c keys sharing the prefix: their values into sc.comp (in any
      // order; only counts and values matter from here on)
      if (threadIdx.x == 0) *sc.ncand = 0;
      __syncthreads();
      for_keys<NT, float>(n_in, val, [&](int64_t, float v) {
        append_wave(sc, (keyof(v) & mask) == prefix, v);
      });
      __syncthreads();
      compact = true;
      n_in = c;
    }
  }
  return prefix;  // not reached: the last pass has shift == 0
}

// Ascending bitonic sort of one key per lane across a wave (64 keys), by
// cross-lane exchanges: no LDS, no block barrier.
template <typename K>
__device__ __forceinline__ K wave_sort64(K v) {
  const int lane = (int)(threadIdx.x & 63u);
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      K o;
      if constexpr (sizeof(K) == 8) {
        o = (K)__shfl_xor((unsigned long long)v, j);
      } else {
        o = (K)__shfl_xor((unsigned)v, j);
      }
      const bool lower = (lane & j) == 0;        // keeps the smaller of the pair
      const bool up = (lane & k) == 0;           // ascending run
      const K mn = o < v ? o : v, mx = o < v ? v : o;
      v = (lower == up) ? mn : mx;
    }
  }
  return v;
}

// Exact k-th smallest key (and the (k+1)-th when it sits in the same or
// the next non-empty bin, has2) with bins fitted to the data.  The range
// [kmin, kmax] that the radix passes split is set by the extreme keys, and
// when a few outliers stretch it, the first digit puts the bulk of the keys
// into a handful of bins, whose LDS atomics then serialise.  Here wave 0
// sorts a 64-key sample (odd stride) in registers and takes the window
// [lo, hi] between its ranks 8 and 56; one pass histograms every key into
// NBINS - 2 equal bins of 2^s keys across the window plus an underflow and
// an overflow bin, and when the bin holding rank k has at most SEL_CAND
// keys, one pass gathers them and one wave ranks them.  Returns false with
// nothing selected when rank k falls outside the window or its bin holds
// more keys (the caller then runs the radix selection).
template <int NT, int NBINS, typename K, typename ValFn, typename KeyOf>
__device__ __forceinline__ bool window_select(int64_t n, int64_t k, bool want2, ValFn val, KeyOf keyof,
                                              const SelScratch& sc, K& v1, K& v2, bool& has2) {
  const int lane = (int)(threadIdx.x & 63u);
  auto key = [&](int64_t i) -> K { return keyof(val(i)); };
  has2 = false;
  if (threadIdx.x < 64) {
    int64_t stride = n / 64;
    if (stride % 2 == 0) --stride;
    const K srt = wave_sort64<K>(key((int64_t)lane * stride));
    K lo, hi;
    if constexpr (sizeof(K) == 8) {
      lo = (K)__shfl((unsigned long long)srt, 8);
      hi = (K)__shfl((unsigned long long)srt, 56);
    } else {
      lo = (K)__shfl((unsigned)srt, 8);
      hi = (K)__shfl((unsigned)srt, 56);
    }
    int sh = 0;
    while (sh < (int)(8 * sizeof(K)) - 1 && ((hi - lo) >> sh) >= (K)(NBINS - 2)) ++sh;
    if (lane == 0) {
      sc.sh[0] = (unsigned long long)lo;
      sc.sh[1] = (unsigned long long)sh;
    }
  }
  for (int i = threadIdx.x; i < NBINS; i += NT) sc.hist[i] = 0;
  __syncthreads();
  const K lo = (K)rfl64((int64_t)sc.sh[0]);
  const int sh = __builtin_amdgcn_readfirstlane((int)sc.sh[1]);
  auto bin = [&](K kv) -> unsigned {
    if (kv < lo) return 0u;
    const K q = (kv - lo) >> sh;
    return q >= (K)(NBINS - 2) ? (unsigned)(NBINS - 1) : (unsigned)q + 1u;
  };
  __syncthreads();  // lo and sh read before sh[] is reused
  // keys outside the window all land in the two end bins: counted in
  // registers and added once per wave instead of by same-address atomics
  // (32-bit keys; with 64-bit keys the extra tests cost more VALU time
  // than the atomics they save)
  if constexpr (sizeof(K) == 4) {
    unsigned under = 0u, over = 0u;
    for_keys<NT, K>(n, key, [&](int64_t, K kv) {
      const unsigned q = bin(kv);
      if (q == 0u) ++under;
      else if (q == (unsigned)(NBINS - 1)) ++over;
      else atomicAdd(&sc.hist[q], 1u);
    });
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      under += __shfl_xor(under, d);
      over += __shfl_xor(over, d);
    }
    if (lane == 0) {
      if (under) atomicAdd(&sc.hist[0], under);
      if (over) atomicAdd(&sc.hist[NBINS - 1], over);
    }
  } else {
    for_keys<NT, K>(n, key, [&](int64_t, K kv) { atomicAdd(&sc.hist[bin(kv)], 1u); });
  }
  __syncthreads();
  find_digit<NT, NBINS>(sc.hist, k, sc.wsum, sc.sh);
  const unsigned b = (unsigned)__builtin_amdgcn_readfirstlane((int)sc.sh[0]);
  const int64_t kk = rfl64((int64_t)sc.sh[1]);
  int64_t c = (int64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)sc.hist[b]);
  __syncthreads();
  if (b == 0u || b == (unsigned)(NBINS - 1) || (c > SEL_CAND && c > sc.comp_cap)) return false;
  if (c > SEL_CAND) {
    // a fuller bin: its values into the compaction buffer, then the radix
    // selection among them, within the bin's key range
    if (threadIdx.x == 0) *sc.ncand = 0;
    __syncthreads();
    for_keys<NT, float>(n, val, [&](int64_t, float v) { append_wave(sc, bin(keyof(v)) == b, v); });
    __syncthreads();
    const K base = (K)(b - 1u) << sh;
    const K kmin = lo + base;
    const K span = (K)1 << sh;
    const K kmax = kmin + (span - 1) < kmin ? ~(K)0 : kmin + (span - 1);
    SelScratch in = sc;
    in.comp_cap = 0;
    const float* cv = sc.comp;
    auto cval = [&](int64_t i) -> float { return cv[i]; };
    v1 = radix_select<NT, NBINS == 2048 ? 11 : 8, K>(c, kk, kmin, kmax, cval, keyof, in, want2, v2, has2);
    return true;
  }
  // with rank k the last key of its bin, rank k+1 is the smallest key of the
  // next non-empty bin: gather that bin too when it is an interior one and fits
  unsigned b2 = (unsigned)NBINS;
  if (want2 && kk + 1 == c) {
    if (threadIdx.x == 0) *sc.ncand = (unsigned)NBINS;
    __syncthreads();
    for (int q = (int)b + 1 + threadIdx.x; q < NBINS; q += NT)
      if (sc.hist[q] != 0u) atomicMin(sc.ncand, (unsigned)q);
    __syncthreads();
    const unsigned d2 = (unsigned)__builtin_amdgcn_readfirstlane((int)*sc.ncand);
    if (d2 < (unsigned)(NBINS - 1) && c + (int64_t)sc.hist[d2] <= SEL_CAND) b2 = d2;
    __syncthreads();
  }
  const int64_t c2 = b2 < (unsigned)NBINS ? (int64_t)sc.hist[b2] : 0;
  if (threadIdx.x == 0) *sc.ncand = 0;
  __syncthreads();
  for_keys<NT, K>(n, key, [&](int64_t, K kv) {
    const unsigned q = bin(kv);
    if (q == b || q == b2) sc.cand[atomicAdd(sc.ncand, 1u)] = (unsigned long long)kv;
  });
  c += c2;
  __syncthreads();
  if (threadIdx.x < 64) {
    // rank every candidate against the others, held one per lane
    const K mine = lane < c ? (K)sc.cand[lane] : ~(K)0;
    int64_t less = 0, same = 0;
    for (int t = 0; t < (int)c; ++t) {
      K o;
      if constexpr (sizeof(K) == 8) {
        const uint32_t olo = __builtin_amdgcn_readlane((uint32_t)mine, t);
        const uint32_t ohi = __builtin_amdgcn_readlane((uint32_t)(mine >> 32), t);
        o = (K)(((uint64_t)ohi << 32) | olo);
      } else {
        o = (K)__builtin_amdgcn_readlane((uint32_t)mine, t);
      }
      less += o < mine;
      same += o == mine;
    }
    if (lane < c && less <= kk && kk < less + same) sc.sh[2] = (unsigned long long)mine;
    if (lane < c && less <= kk + 1 && kk + 1 < less + same) sc.sh[3] = (unsigned long long)mine;
  }
  __syncthreads();
  v1 = (K)sc.sh[2];
  if (want2 && kk + 1 < c) {
    v2 = (K)sc.sh[3];
    has2 = true;
  }
  __syncthreads();
  return true;
}

// The order statistic of rank k+1 given the one of rank k (key kk): kk
// itself if more than k+1 keys are <= kk, else the smallest key above kk.
// One pass: a count and a minimum, reduced over the block.
template <int NT, typename K, typename KeyFn>
__device__ __forceinline__ K next_rank(int64_t count, int64_t k, K kk, KeyFn key, unsigned long long* red) {
  constexpr int NW = NT / 64;
  unsigned long long le = 0;
  K mn = ~(K)0;
  for_keys<NT, K>(count, key, [&](int64_t, K kv) {
    if (kv <= kk) ++le;
    else if (kv < mn) mn = kv;
  });
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
  int64_t id, i;
  if (total <= 0x7fffffffLL) {  // 32-bit division
    const uint32_t q = (uint32_t)e / (uint32_t)count;
    id = q;
    i = (uint32_t)e - q * (uint32_t)count;
  } else {
    id = e / count;
    i = e % count;
  }
  amp[e] = amp_f32(vis[make_pop(id, n_time, n_base, n_chan, population).off(i)]);
}

// The same for per-baseline populations (contiguous runs of n_chan, a
// multiple of 4) of a 32-byte aligned plane: four amplitudes per thread from
// two 16-byte loads, written with one 16-byte store.
__global__ void mad_amp4_kernel(const float4* __restrict__ vis, int64_t n_base, int n_chan, int64_t count,
                                int64_t total4, float4* __restrict__ amp) {
  const int64_t e4 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e4 >= total4) return;
  const int64_t e = 4 * e4;
  int64_t id, t, k;  // baseline, integration, channel (k % 4 == 0)
  if (4 * total4 <= 0x7fffffffLL) {  // 32-bit division
    const uint32_t q = (uint32_t)e / (uint32_t)count, i = (uint32_t)e - q * (uint32_t)count;
    const uint32_t tq = i / (uint32_t)n_chan;
    id = q;
    t = tq;
    k = i - tq * (uint32_t)n_chan;
  } else {
    const int64_t i = e % count;
    id = e / count;
    t = i / n_chan;
    k = i % n_chan;
  }
  const int64_t v = ((t * n_base + id) * n_chan + k) / 2;  // float4 = two visibilities
  const float4 a = vis[v], b = vis[v + 1];
  amp[e4] = make_float4(amp_f32(make_float2(a.x, a.y)), amp_f32(make_float2(a.z, a.w)),
                        amp_f32(make_float2(b.x, b.y)), amp_f32(make_float2(b.z, b.w)));
}

template <int NT, int DB>
__global__ void __launch_bounds__(NT)
mad_kernel(const float2* __restrict__ vis, int64_t n_time, int64_t n_base, int n_chan, float sigma,
           int population, int64_t cap, int64_t comp_cap, const float* __restrict__ gamp,
           uint8_t* __restrict__ mask, double* __restrict__ thresh, double* __restrict__ stats) {
  __shared__ unsigned hist[1 << DB];
  __shared__ unsigned wsum[NT / 64];
  __shared__ unsigned long long sh[4];
  __shared__ unsigned long long red[2 * (NT / 64)];
  __shared__ unsigned long long cand[SEL_CAND];
  __shared__ unsigned ncand;
  extern __shared__ __align__(16) float acache[];  // [cap] amplitude cache, then [comp_cap] compaction buffer
  const int64_t id = blockIdx.x;
  const Pop pop = make_pop(id, n_time, n_base, n_chan, population);
  const int64_t n = pop.count;
  const bool cached = n <= cap;
  const SelScratch sc{hist, wsum, sh, red, cand, &ncand, acache + (cached ? n : 0), comp_cap};
  const AmpSrc amp{vis, pop, cached ? acache : (gamp ? gamp + id * n : nullptr)};
  // one pass: the amplitudes into the LDS cache (when they fit) and the
  // range of their keys
  uint32_t amin = ~0u, amax = 0u;
  const bool vec4 = gamp && cached && n % 4 == 0 && (reinterpret_cast<uintptr_t>(gamp + id * n) & 15u) == 0;
  if (vec4) {
    // four amplitudes per 16-byte load, eight loads in flight per thread
    constexpr int U = 8;
    const float4* g4 = reinterpret_cast<const float4*>(gamp + id * n);
    float4* c4 = reinterpret_cast<float4*>(acache);
    const int64_t n4 = n / 4;
    for (int64_t j0 = threadIdx.x; j0 < n4; j0 += (int64_t)U * NT) {
      float4 a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = j0 + (int64_t)u * NT;
        a[u] = j < n4 ? g4[j] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = j0 + (int64_t)u * NT;
        if (j < n4) {
          c4[j] = a[u];
          const uint32_t k4[4] = {__float_as_uint(a[u].x), __float_as_uint(a[u].y), __float_as_uint(a[u].z),
                                  __float_as_uint(a[u].w)};
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            amin = k4[v] < amin ? k4[v] : amin;
            amax = k4[v] > amax ? k4[v] : amax;
          }
        }
      }
    }
  } else {
    // eight loads in flight per thread before their amplitudes are formed
    constexpr int U = 8;
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += (int64_t)U * NT) {
      float a[U];
      if (gamp) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t i = i0 + (int64_t)u * NT;
          a[u] = i < n ? gamp[id * n + i] : 0.f;
        }
      } else {
        float2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t i = i0 + (int64_t)u * NT;
          v[u] = i < n ? vis[pop.off(i)] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = amp_f32(v[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + (int64_t)u * NT;
        if (i < n) {
          if (cached) acache[i] = a[u];
          const uint32_t kv = __float_as_uint(a[u]);
          amin = kv < amin ? kv : amin;
          amax = kv > amax ? kv : amax;
        }
      }
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint32_t a = __shfl_down(amin, d), b = __shfl_down(amax, d);
    amin = a < amin ? a : amin;
    amax = b > amax ? b : amax;
  }
  if ((threadIdx.x & 63) == 0) {
    red[2 * (threadIdx.x >> 6)] = amin;
    red[2 * (threadIdx.x >> 6) + 1] = amax;
  }
  __syncthreads();
  amin = ~0u;
  amax = 0u;
  for (int w = 0; w < NT / 64; ++w) {
    amin = (uint32_t)red[2 * w] < amin ? (uint32_t)red[2 * w] : amin;
    amax = (uint32_t)red[2 * w + 1] > amax ? (uint32_t)red[2 * w + 1] : amax;
  }
  // block-uniform values from LDS, and every value derived from them below
  // (the medians, the key ranges): wave-uniform for the compiler, so the
  // selection loops that depend on them are scalar loops
  amin = (uint32_t)__builtin_amdgcn_readfirstlane((int)amin);
  amax = (uint32_t)__builtin_amdgcn_readfirstlane((int)amax);
  __syncthreads();
  const int64_t k1 = (n - 1) / 2, k2 = n / 2;
  auto akeyof = [](float a) -> uint32_t { return __float_as_uint(a); };
  auto akey = [&](int64_t i) -> uint32_t { return akeyof(amp(i)); };
  uint32_t a2;
  bool has2;
  // windowed first pass for the large populations, radix passes otherwise
  // (or when the window misses)
  constexpr bool WIN = NT >= 1024;
  uint32_t a1 = 0u;
  if (!(WIN && window_select<NT, (1 << DB), uint32_t>(n, k1, k2 != k1, amp, akeyof, sc, a1, a2, has2)))
    a1 = radix_select<NT, DB, uint32_t>(n, k1, amin, amax, amp, akeyof, sc, k2 != k1, a2, has2);
  if (k2 == k1) a2 = a1;
  else if (!has2) a2 = next_rank<NT, uint32_t>(n, k1, a1, akey, red);
  a1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)a1);
  a2 = (uint32_t)__builtin_amdgcn_readfirstlane((int)a2);
  const double med = ((double)__uint_as_float(a1) + (double)__uint_as_float(a2)) / 2.0;
  auto dkeyof = [&](float a) -> uint64_t { return (uint64_t)__double_as_longlong(fabs((double)a - med)); };
  auto dkey = [&](int64_t i) -> uint64_t { return dkeyof(amp(i)); };
  // deviations lie in [0, the larger deviation of the two extreme amplitudes]
  const double dlo = fabs((double)__uint_as_float(amin) - med);
  const double dhi = fabs((double)__uint_as_float(amax) - med);
  const uint64_t dmax = (uint64_t)__double_as_longlong(dlo > dhi ? dlo : dhi);
  uint64_t d2;
  uint64_t d1 = 0ull;
  if (!(WIN && window_select<NT, (1 << DB), uint64_t>(n, k1, k2 != k1, amp, dkeyof, sc, d1, d2, has2)))
    d1 = radix_select<NT, DB, uint64_t>(n, k1, 0ull, dmax, amp, dkeyof, sc, k2 != k1, d2, has2);
  if (k2 == k1) d2 = d1;
  else if (!has2) d2 = next_rank<NT, uint64_t>(n, k1, d1, dkey, red);
  d1 = (uint64_t)rfl64((int64_t)d1);
  d2 = (uint64_t)rfl64((int64_t)d2);
  const double madv =
      (__longlong_as_double((long long)d1) + __longlong_as_double((long long)d2)) / 2.0;
  const double c = (double)sigma * 1.4826;
  const double T = med + c * madv;
  if (mask) {
    if (cached && pop.s_inner == 1 && pop.inner_n % 4 == 0 && pop.base % 4 == 0 && pop.s_outer % 4 == 0 &&
        (reinterpret_cast<uintptr_t>(mask) & 3u) == 0 && n % 4 == 0) {
      // four consecutive elements (one row, contiguous flags) per thread:
      // one 16-byte LDS read and one 4-byte store; element 4j = q * inner_n + r
      const float4* c4 = reinterpret_cast<const float4*>(acache);
      const int64_t n4 = n / 4;
      int64_t q = 0, r = 4 * (int64_t)threadIdx.x;
      while (r >= pop.inner_n) {
        r -= pop.inner_n;
        ++q;
      }
      for (int64_t j = threadIdx.x; j < n4; j += NT) {
        const float4 a = c4[j];
        const uint32_t f = ((double)a.x > T ? 1u : 0u) | ((double)a.y > T ? 1u << 8 : 0u) |
                           ((double)a.z > T ? 1u << 16 : 0u) | ((double)a.w > T ? 1u << 24 : 0u);
        *reinterpret_cast<uint32_t*>(mask + pop.base + q * pop.s_outer + r) = f;
        r += 4 * NT;
        while (r >= pop.inner_n) {
          r -= pop.inner_n;
          ++q;
        }
      }
    } else if (cached && pop.inner_n >= NT) {
      // element i = q * inner_n + r; a step of NT carries into q at most once
      int64_t q = 0, r = threadIdx.x;
      for (int64_t i = threadIdx.x; i < n; i += NT) {
        mask[pop.base + q * pop.s_outer + r * pop.s_inner] = (double)amp(i) > T ? 1 : 0;
        r += NT;
        if (r >= pop.inner_n) {
          r -= pop.inner_n;
          ++q;
        }
      }
    } else {
      for_keys<NT, float>(n, amp, [&](int64_t i, float a) { mask[pop.off(i)] = (double)a > T ? 1 : 0; });
    }
  }
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
constexpr int64_t MAD_LDS_FLOATS = 38400;  // dynamic LDS of the 1024-thread kernel: cache + compaction
constexpr int64_t MAD_COMP_MAX = 32768;

int64_t mad_scratch_floats(int64_t n_time, int64_t n_base, int n_chan, int population) {
  const int64_t npop = population == 0 ? n_base : population == 1 ? n_base * n_chan : n_time * n_base;
  const int64_t count = population == 0 ? n_time * n_chan : population == 1 ? n_time : n_chan;
  return count > MAD_CAP_SMALL ? npop * count : 0;
}

hipError_t launch_mad(const float2* vis, int64_t n_time, int64_t n_base, int n_chan, float sigma,
                      int population, uint8_t* mask, double* thresh, double* stats, float* amp_scratch,
                      hipStream_t s) {
  const int64_t npop = population == 0 ? n_base : population == 1 ? n_base * n_chan : n_time * n_base;
  const int64_t count = population == 0 ? n_time * n_chan : population == 1 ? n_time : n_chan;
  if (npop <= 0) return hipSuccess;
  if (count <= MAD_CAP_SMALL) {
    const size_t lds = (size_t)count * sizeof(float);
    return launch(mad_kernel<64, 8>, dim3((unsigned)npop), dim3(64), lds, s, vis, n_time, n_base, n_chan, sigma,
                  population, MAD_CAP_SMALL, (int64_t)0, nullptr, mask, thresh, stats);
  } else {
    const int64_t cap = count <= MAD_CAP_BIG ? count : 0;
    const float* gamp = nullptr;
    if (amp_scratch) {
      // the amplitudes are formed once, by the whole GPU: the selection
      // workgroups (one per population) then load 4 contiguous bytes per
      // element instead of forming a float64 square root each, and
      // populations beyond the LDS cache read 4 bytes per pass
      const int64_t total = npop * count;
      hipError_t e;
      if (population == 0 && n_chan % 4 == 0 && (reinterpret_cast<uintptr_t>(vis) & 31u) == 0 &&
          (reinterpret_cast<uintptr_t>(amp_scratch) & 15u) == 0) {
        const int64_t total4 = total / 4;
        e = launch(mad_amp4_kernel, dim3((unsigned)((total4 + 255) / 256)), dim3(256), 0, s,
                   reinterpret_cast<const float4*>(vis), n_base, n_chan, count, total4,
                   reinterpret_cast<float4*>(amp_scratch));
      } else {
        e = launch(mad_amp_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, vis, n_time, n_base,
                   n_chan, population, count, total, amp_scratch);
      }
      if (e != hipSuccess) return e;
      gamp = amp_scratch;
    }
    // what LDS the cache leaves holds the compaction buffer
    int64_t comp_cap = MAD_LDS_FLOATS - cap;
    comp_cap = comp_cap < MAD_COMP_MAX ? comp_cap : MAD_COMP_MAX;
    if (comp_cap < 256) comp_cap = 0;
    const size_t lds = (size_t)(cap + comp_cap) * sizeof(float);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(mad_kernel<1024, 11>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return launch(mad_kernel<1024, 11>, dim3((unsigned)npop), dim3(1024), lds, s, vis, n_time, n_base, n_chan,
                  sigma, population, cap, comp_cap, gamp, mask, thresh, stats);
  }
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
  return launch(apply_kernel, grid, dim3(256), 0, s, vis, n_ant, n_chan, f0, df, t);
}

}  // namespace qc
