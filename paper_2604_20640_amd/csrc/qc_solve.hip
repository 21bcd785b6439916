// Delay and phase calibration solve for gfx950 (arXiv 2604.20640 Sec. 7,
// three serial steps, eq. 3).
//
// Per cross baseline (one workgroup each):
//   * integrate the flag-zeroed visibilities over time (float64 sums);
//   * coarse delay: peak of the delay spectrum D[l] = sum_k V[k] e^{+2 pi i k l / L},
//     evaluated as conj(FFT(conj V)) with the LDS Stockham FFT on L lags
//     (float32), argmax with ties to the smallest lag;
//   * fine delay: the phase of V e^{+2 pi i f_k tau_c} over the clean band
//     (float32 atan2), unwrapped by integer jumps (a step above pi in
//     magnitude gets a 2 pi correction of the opposite sign), then the
//     weighted least-squares slope with float64 normal-equation sums,
//     tau = tau_c - slope / 2 pi;
//   * residual phase: phi = -arg of the band's mean vector of
//     V e^{+2 pi i f_k tau} (float64 sum).
// Per antenna: float64 least squares of tau_i - tau_j = tau_b over the cross
// baselines with the reference antenna at zero (closed form, one thread per
// antenna); phases start from the reference-antenna baselines and are
// refined by least squares on the wrapped residuals.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qc_fft.h"
#include "qc_kernels.h"

namespace qc {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Sums K doubles over the block; every thread gets the totals.
template <int NT, int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < K; ++q) red[q * NT + t] = v[q];
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if (t < st) {
#pragma unroll
      for (int q = 0; q < K; ++q) red[q * NT + t] += red[q * NT + t + st];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < K; ++q) v[q] = red[q * NT];
  __syncthreads();
}

__device__ __forceinline__ double wrap_pi(double a) {
  double r = fmod(a + kPi, 2.0 * kPi);
  if (r < 0.0) r += 2.0 * kPi;
  return r - kPi;
}

}  // namespace

template <int NLAG>
__global__ void __launch_bounds__(NLAG / 16)
solve_baseline_kernel(const float2* __restrict__ vis, const uint8_t* __restrict__ mask, int64_t n_time,
                      int n_ant, int n_chan, double f0, double df, int chan_lo, int chan_hi,
                      const float2* __restrict__ tw, double* __restrict__ tau_b,
                      double* __restrict__ phi_b) {
  constexpr int NT = NLAG / 16;
  extern __shared__ double smem[];
  double* red = smem;                                          // 6 * NT doubles
  float2* buf = reinterpret_cast<float2*>(red + 6 * NT);       // padded NLAG
  float2* vi = buf + lds_padded_size(NLAG);                    // n_chan
  float* psi = reinterpret_cast<float*>(vi + n_chan);          // band
  int* cnt = reinterpret_cast<int*>(psi + (chan_hi - chan_lo)); // NT
  const int tid = threadIdx.x;

  // cross baseline index -> (i, j), i < j, and its row in vis
  int c = blockIdx.x, i = 0;
  while (c >= n_ant - 1 - i) { c -= n_ant - 1 - i; ++i; }
  const int j = i + 1 + c;
  const int64_t b = (int64_t)i * n_ant - (int64_t)i * (i - 1) / 2 + (j - i);
  const int64_t nb = (int64_t)n_ant * (n_ant + 1) / 2;

  // 1. time integration with flags zeroed
  for (int k = tid; k < n_chan; k += NT) {
    double sx = 0.0, sy = 0.0;
    for (int64_t t = 0; t < n_time; ++t) {
      const int64_t o = (t * nb + b) * n_chan + k;
      if (mask == nullptr || mask[o] == 0) {
        const float2 v = vis[o];
        sx += (double)v.x;
        sy += (double)v.y;
      }
    }
    vi[k] = make_float2((float)sx, (float)sy);
  }
  __syncthreads();
  for (int l = tid; l < NLAG; l += NT) {
    const float2 v = l < n_chan ? vi[l] : make_float2(0.f, 0.f);
    buf[lds_pad(l)] = make_float2(v.x, -v.y);
  }
  __syncthreads();
  // 2. coarse delay: |D[l]| = |FFT(conj V)[l]|
  fft_lds<NLAG, NT>(buf, tw, tid);
  float best = -1.f;
  int best_l = 0;
  for (int l = tid; l < NLAG; l += NT) {
    const float2 z = buf[lds_pad(l)];
    const float m = z.x * z.x + z.y * z.y;
    if (m > best) {
      best = m;
      best_l = l;
    }
  }
  red[tid] = (double)best;
  cnt[tid] = best_l;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if (tid < st) {
      const double o = red[tid + st];
      const int ol = cnt[tid + st];
      if (o > red[tid] || (o == red[tid] && ol < cnt[tid])) {
        red[tid] = o;
        cnt[tid] = ol;
      }
    }
    __syncthreads();
  }
  const int lstar = cnt[0];
  __syncthreads();
  const int ls = lstar < NLAG / 2 ? lstar : lstar - NLAG;
  const double tau_c = (double)ls / ((double)NLAG * df);

  // 3. fine delay over the band [chan_lo, chan_hi)
  const int nbnd = chan_hi - chan_lo;
  for (int q = tid; q < nbnd; q += NT) {
    const int k = chan_lo + q;
    const double fk = f0 + (double)k * df;
    double cyc = fk * tau_c;
    cyc -= rint(cyc);
    double sn, cs;
    sincospi(2.0 * cyc, &sn, &cs);
    const float2 v = vi[k];
    const float wx = (float)((double)v.x * cs - (double)v.y * sn);
    const float wy = (float)((double)v.x * sn + (double)v.y * cs);
    psi[q] = atan2f(wy, wx);
  }
  __syncthreads();
  // unwrap: integer jump counts, prefix-summed over contiguous segments
  const int seg = (nbnd + NT - 1) / NT;
  const int q0 = tid * seg, q1 = min(nbnd, q0 + seg);
  int local = 0;
  for (int q = q0; q < q1; ++q) {
    if (q == 0) continue;
    const float dd = psi[q] - psi[q - 1];
    local += dd > (float)kPi ? -1 : (dd < -(float)kPi ? 1 : 0);
  }
  cnt[tid] = local;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int t = 0; t < NT; ++t) {
      const int v = cnt[t];
      cnt[t] = acc;
      acc += v;
    }
  }
  __syncthreads();
  double sums[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int cj = cnt[tid];
  for (int q = q0; q < q1; ++q) {
    if (q > 0) {
      const float dd = psi[q] - psi[q - 1];
      cj += dd > (float)kPi ? -1 : (dd < -(float)kPi ? 1 : 0);
    }
    const int k = chan_lo + q;
    const double fk = f0 + (double)k * df;
    const double pu = (double)psi[q] + 2.0 * kPi * (double)cj;
    const float2 v = vi[k];
    const double w = sqrt((double)v.x * v.x + (double)v.y * v.y);
    sums[0] += w;
    sums[1] += w * fk;
    sums[2] += w * fk * fk;
    sums[3] += w * pu;
    sums[4] += w * fk * pu;
  }
  block_sum<NT, 5>(sums, red);
  const double det = sums[0] * sums[2] - sums[1] * sums[1];
  const double slope = (sums[0] * sums[4] - sums[1] * sums[3]) / det;
  const double tau = tau_c - slope / (2.0 * kPi);

  // 4. residual phase from the mean vector
  double u[2] = {0.0, 0.0};
  for (int q = tid; q < nbnd; q += NT) {
    const int k = chan_lo + q;
    const double fk = f0 + (double)k * df;
    double cyc = fk * tau;
    cyc -= rint(cyc);
    double sn, cs;
    sincospi(2.0 * cyc, &sn, &cs);
    const float2 v = vi[k];
    u[0] += (double)v.x * cs - (double)v.y * sn;
    u[1] += (double)v.x * sn + (double)v.y * cs;
  }
  block_sum<NT, 2>(u, red);
  if (tid == 0) {
    tau_b[blockIdx.x] = tau;
    phi_b[blockIdx.x] = -atan2(u[1], u[0]);
  }
}

// Per-antenna least squares over the cross baselines, the reference antenna
// fixed at zero.  With unit weights on every cross baseline the normal
// matrix of the F = n - 1 free antennas is N = n I - 1 1^T (an antenna is
// on n - 1 baselines; two free antennas share one), and
// (n I - 1 1^T)(I + 1 1^T) = n I + (n - 1 - F) 1 1^T = n I, so the
// solution of N x = r is x = (r + sum(r) 1) / n.  One thread per antenna
// forms its right-hand side r = G^T b (baselines in row-major order).
__global__ void solve_antenna_kernel(const double* __restrict__ tau_b, const double* __restrict__ phi_b,
                                     int n_ant, int ref, double* __restrict__ tau_out,
                                     double* __restrict__ phi_out) {
  extern __shared__ double sm[];
  double* phi0 = sm;            // n_ant: first phases, from the reference baselines
  double* rt = phi0 + n_ant;    // n_ant: right-hand sides (delay)
  double* rp = rt + n_ant;      // n_ant: right-hand sides (phase residual)
  __shared__ double tot[2];
  const int n = n_ant;
  // index of cross baseline (i, j), i < j, in row-major order
  auto cb = [&](int i, int j) { return i * n - i * (i + 1) / 2 + (j - i - 1); };
  for (int a = threadIdx.x; a < n; a += blockDim.x)
    phi0[a] = a == ref ? 0.0 : a < ref ? phi_b[cb(a, ref)] : -phi_b[cb(ref, a)];
  __syncthreads();
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    double st = 0.0, sp = 0.0;
    if (a != ref) {
      for (int b = 0; b < n; ++b) {
        if (b == a) continue;
        const int i = a < b ? a : b, j = a < b ? b : a;
        const int r = cb(i, j);
        const double res = wrap_pi(phi_b[r] - (phi0[i] - phi0[j]));
        if (a == i) {
          st += tau_b[r];
          sp += res;
        } else {
          st -= tau_b[r];
          sp -= res;
        }
      }
    }
    rt[a] = st;
    rp[a] = sp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0, q = 0.0;
    for (int a = 0; a < n; ++a)
      if (a != ref) {
        t += rt[a];
        q += rp[a];
      }
    tot[0] = t;
    tot[1] = q;
  }
  __syncthreads();
  for (int a = threadIdx.x; a < n; a += blockDim.x) {
    tau_out[a] = a == ref ? 0.0 : (rt[a] + tot[0]) / (double)n;
    phi_out[a] = a == ref ? wrap_pi(phi0[a]) : wrap_pi(phi0[a] + (rp[a] + tot[1]) / (double)n);
  }
}

size_t solve_lds_bytes(int n_lag, int n_chan, int band) {
  const int nt = n_lag / 16;
  return 6 * nt * sizeof(double) + sizeof(float2) * (lds_padded_size(n_lag) + n_chan) +
         sizeof(float) * band + sizeof(int) * nt;
}

template <int NLAG>
static hipError_t launch_solve_t(const float2* vis, const uint8_t* mask, int64_t n_time, int n_ant,
                                 int n_chan, double f0, double df, int lo, int hi, const float2* tw,
                                 double* tau_b, double* phi_b, hipStream_t s) {
  const size_t lds = solve_lds_bytes(NLAG, n_chan, hi - lo);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(solve_baseline_kernel<NLAG>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int n_cross = n_ant * (n_ant - 1) / 2;
  hipLaunchKernelGGL(solve_baseline_kernel<NLAG>, dim3(n_cross), dim3(NLAG / 16), lds, s, vis, mask,
                     n_time, n_ant, n_chan, f0, df, lo, hi, tw, tau_b, phi_b);
  return hipGetLastError();
}

hipError_t launch_solve(const float2* vis, const uint8_t* mask, int64_t n_time, int n_ant, int n_chan,
                        double f0, double df, int ref, int lo, int hi, int n_lag, const float2* tw,
                        double* tau_b, double* phi_b, double* tau, double* phi, hipStream_t s) {
  hipError_t e = hipErrorInvalidValue;
  switch (n_lag) {
    case 16: e = launch_solve_t<16>(vis, mask, n_time, n_ant, n_chan, f0, df, lo, hi, tw, tau_b, phi_b, s); break;
    case 32: e = launch_solve_t<32>(vis, mask, n_time, n_ant, n_chan, f0, df, lo, hi, tw, tau_b, phi_b, s); break;
    case 64: e = launch_solve_t<64>(vis, mask, n_time, n_ant, n_chan, f0, df, lo, hi, tw, tau_b, phi_b, s); break;
    case 128: e = launch_solve_t<128>(vis, mask, n_time, n_ant, n_chan, f0, df, lo, hi, tw, tau_b, phi_b, s); break;
    case 256: e = launch_solve_t<256>(vis, mask, n_time, n_ant, n_chan, f0, df, lo, hi, tw, tau_b, phi_b, s); break;
    case 512: e = launch_solve_t<512>(vis, mask, n_time, n_ant, n_chan, f0, df, lo, hi, tw, tau_b, phi_b, s); break;
    case 1024: e = launch_solve_t<1024>(vis, mask, n_time, n_ant, n_chan, f0, df, lo, hi, tw, tau_b, phi_b, s); break;
    case 2048: e = launch_solve_t<2048>(vis, mask, n_time, n_ant, n_chan, f0, df, lo, hi, tw, tau_b, phi_b, s); break;
    case 4096: e = launch_solve_t<4096>(vis, mask, n_time, n_ant, n_chan, f0, df, lo, hi, tw, tau_b, phi_b, s); break;
    case 8192: e = launch_solve_t<8192>(vis, mask, n_time, n_ant, n_chan, f0, df, lo, hi, tw, tau_b, phi_b, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const size_t lds = sizeof(double) * 3 * n_ant;
  hipLaunchKernelGGL(solve_antenna_kernel, dim3(1), dim3(64), lds, s, tau_b, phi_b, n_ant, ref, tau, phi);
  return hipGetLastError();
}

}  // namespace qc
