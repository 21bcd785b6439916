// MAD flagging and delay/phase application for gfx950.
//
// MAD (arXiv 2604.20640 Sec. 7, eq. 2): T = median(A) + sigma*1.4826*MAD(A)
// on the visibility amplitude A; flag A > T.  Medians are exact order
// statistics found by radix selection (8-bit digits, most significant
// first) over the bit patterns of non-negative floats, whose unsigned order
// equals their numeric order: float32 amplitudes (4 passes), float64
// deviations |A - median| (8 passes).  Even counts average the two middle
// order statistics.  One workgroup handles one population.
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

constexpr int MAD_NT = 256;

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

// k-th smallest (0-based) amplitude bit pattern in the population.
__device__ uint32_t select_amp(const float2* __restrict__ vis, const Pop& pop, int64_t k,
                               unsigned* hist, unsigned long long* sh) {
  uint32_t prefix = 0, mask = 0;
  int64_t kk = k;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += MAD_NT) hist[i] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < pop.count; i += MAD_NT) {
      const uint32_t key = __float_as_uint(amp_f32(vis[pop.off(i)]));
      if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t cum = 0;
      int dsel = 255;
      for (int dgt = 0; dgt < 256; ++dgt) {
        if (cum + hist[dgt] > kk) { dsel = dgt; break; }
        cum += hist[dgt];
      }
      sh[0] = (unsigned long long)dsel;
      sh[1] = (unsigned long long)(kk - cum);
    }
    __syncthreads();
    prefix |= (uint32_t)sh[0] << shift;
    mask |= 255u << shift;
    kk = (int64_t)sh[1];
    __syncthreads();
  }
  return prefix;
}

// k-th smallest deviation |A - med| (float64 bit pattern).
__device__ uint64_t select_dev(const float2* __restrict__ vis, const Pop& pop, int64_t k, double med,
                               unsigned* hist, unsigned long long* sh) {
  uint64_t prefix = 0, mask = 0;
  int64_t kk = k;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += MAD_NT) hist[i] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < pop.count; i += MAD_NT) {
      const double dev = fabs((double)amp_f32(vis[pop.off(i)]) - med);
      const uint64_t key = (uint64_t)__double_as_longlong(dev);
      if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t cum = 0;
      int dsel = 255;
      for (int dgt = 0; dgt < 256; ++dgt) {
        if (cum + hist[dgt] > kk) { dsel = dgt; break; }
        cum += hist[dgt];
      }
      sh[0] = (unsigned long long)dsel;
      sh[1] = (unsigned long long)(kk - cum);
    }
    __syncthreads();
    prefix |= (uint64_t)sh[0] << shift;
    mask |= (uint64_t)255u << shift;
    kk = (int64_t)sh[1];
    __syncthreads();
  }
  return prefix;
}

}  // namespace

__global__ void __launch_bounds__(MAD_NT)
mad_kernel(const float2* __restrict__ vis, int64_t n_time, int64_t n_base, int n_chan, float sigma,
           int population, uint8_t* __restrict__ mask, double* __restrict__ thresh) {
  __shared__ unsigned hist[256];
  __shared__ unsigned long long sh[2];
  const int64_t id = blockIdx.x;
  Pop pop;
  const int64_t plane = n_base * (int64_t)n_chan;
  if (population == 0) {
    pop = Pop{id * n_chan, n_time * n_chan, n_chan, 1, plane};
  } else if (population == 1) {
    const int64_t b = id / n_chan, k = id % n_chan;
    pop = Pop{b * n_chan + k, n_time, 1, 0, plane};
  } else {
    const int64_t t = id / n_base, b = id % n_base;
    pop = Pop{t * plane + b * n_chan, n_chan, n_chan, 1, 0};
  }
  const int64_t n = pop.count;
  const int64_t k1 = (n - 1) / 2, k2 = n / 2;
  const uint32_t a1 = select_amp(vis, pop, k1, hist, sh);
  const uint32_t a2 = (k2 == k1) ? a1 : select_amp(vis, pop, k2, hist, sh);
  const double med = ((double)__uint_as_float(a1) + (double)__uint_as_float(a2)) / 2.0;
  const uint64_t d1 = select_dev(vis, pop, k1, med, hist, sh);
  const uint64_t d2 = (k2 == k1) ? d1 : select_dev(vis, pop, k2, med, hist, sh);
  const double madv = (__longlong_as_double((long long)d1) + __longlong_as_double((long long)d2)) / 2.0;
  const double T = med + ((double)sigma * 1.4826) * madv;
  for (int64_t i = threadIdx.x; i < n; i += MAD_NT) {
    const int64_t o = pop.off(i);
    mask[o] = (double)amp_f32(vis[o]) > T ? 1 : 0;
  }
  if (thresh && threadIdx.x == 0) thresh[id] = T;
}

hipError_t launch_mad(const float2* vis, int64_t n_time, int64_t n_base, int n_chan, float sigma,
                      int population, uint8_t* mask, double* thresh, hipStream_t s) {
  int64_t npop = population == 0 ? n_base : population == 1 ? n_base * n_chan : n_time * n_base;
  if (npop <= 0) return hipSuccess;
  hipLaunchKernelGGL(mad_kernel, dim3((unsigned)npop), dim3(MAD_NT), 0, s, vis, n_time, n_base,
                     n_chan, sigma, population, mask, thresh);
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
