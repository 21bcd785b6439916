// Synthesis imaging of calibrated visibilities for gfx950 (arXiv 2604.20640
// Sec. 8.1: gridding, Fourier inversion to a dirty image and synthesized
// beam, Hogbom CLEAN deconvolution).
//
// Conventions (n a power of two; cell = image pixel in radians;
// du = 1 / (n cell) wavelengths):
//   * gridding: nearest cell, iu = floor(u/du + 1/2) + n/2 (likewise v),
//     the product u * (n cell) formed in float64; the conjugate visibility
//     goes to the mirrored cell (n - iu, n - iv); a sample is dropped unless
//     both cells lie in [0, n).  The grid is indexed [iu][iv]; W, the total
//     gridded weight (both copies), is accumulated in float64.
//   * inversion: I[il][im] = Re sum G[iu][iv] e^{+2 pi i ((iu-n/2)(il-n/2) +
//     (iv-n/2)(im-n/2)) / n} / W.  With X = (-1)^(iu+iv) G, the sum is
//     (-1)^(il+im) conj(FFT2(conj X)) (forward FFTs of the LDS Stockham
//     engine), so I = (-1)^(il+im) Re FFT2(conj X) / W.  The 2-D transform
//     is rows, a tiled transpose, rows again; the final step reads the
//     transposed result back.
//   * Hogbom CLEAN on one workgroup, float32: each iteration subtracts the
//     previous component's beam g * psf[(p - peak + (n/2, n/2)) mod n]
//     (product and difference rounded separately: no contraction) and,
//     in the same sweep, finds the next peak: largest |residual|, ties to
//     the smallest flat index il * n + im.  g = gain * peak (rounded).
//     Stops when |peak| < threshold or after max_iter components.  Every
//     thread owns the same pixels in every sweep, so the only cross-thread
//     step is the block reduction of the peak.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qc.h"
#include "qc_fft.h"
#include "qc_internal.h"

namespace qc {

namespace {

__global__ void image_grid_kernel(const float* __restrict__ u, const float* __restrict__ v,
                                  const float2* __restrict__ vis, const float* __restrict__ weight,
                                  int64_t n_vis, int n, double inv_du, float2* __restrict__ grid,
                                  double* __restrict__ wsum) {
  __shared__ double red[4];
  double wacc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_vis;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t iu = (int64_t)floor((double)u[k] * inv_du + 0.5) + n / 2;
    const int64_t iv = (int64_t)floor((double)v[k] * inv_du + 0.5) + n / 2;
    const int64_t ju = n - iu, jv = n - iv;
    if (iu < 0 || iu >= n || iv < 0 || iv >= n || ju < 0 || ju >= n || jv < 0 || jv >= n) continue;
    const float w = weight ? weight[k] : 1.f;
    const float2 z = vis[k];
    float* a = reinterpret_cast<float*>(grid + iu * n + iv);
    float* b = reinterpret_cast<float*>(grid + ju * n + jv);
    atomicAdd(a, w * z.x);
    atomicAdd(a + 1, w * z.y);
    atomicAdd(b, w * z.x);
    atomicAdd(b + 1, -w * z.y);
    wacc += 2.0 * (double)w;
  }
  for (int d = 32; d >= 1; d >>= 1) wacc += __shfl_down(wacc, d);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = wacc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(wsum, red[0] + red[1] + red[2] + red[3]);
}

__global__ void image_zero_kernel(float2* __restrict__ grid, int64_t npix, double* __restrict__ wsum) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < npix) grid[e] = make_float2(0.f, 0.f);
  if (e == 0) *wsum = 0.0;
}

// X = conj((-1)^(iu+iv) G), into a work buffer.
__global__ void image_prep_kernel(const float2* __restrict__ g, int n, float2* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int iu = (int)(e / n), iv = (int)(e % n);
  const float s = ((iu + iv) & 1) ? -1.f : 1.f;
  const float2 z = g[e];
  x[e] = make_float2(s * z.x, -s * z.y);
}

// In-place forward FFT of `rows` contiguous rows of length N, S rows per
// workgroup (S N = 4096 values in LDS, one row for N >= 4096).
template <int N>
struct RowCfg {
  static constexpr int S = N >= 4096 ? 1 : 4096 / N;
  static constexpr int NT = S * N / 16;
  static constexpr int LDS = lds_padded_size(S * N);
};

template <int N>
__global__ void __launch_bounds__(RowCfg<N>::NT)
image_rows_fft_kernel(float2* __restrict__ x, int rows, const float2* __restrict__ tw) {
  using C = RowCfg<N>;
  extern __shared__ float2 buf[];
  const int r0 = blockIdx.x * C::S;
  for (int i = threadIdx.x; i < C::S * N; i += C::NT) {
    const int r = r0 + i / N;
    buf[lds_pad(i)] = r < rows ? x[(int64_t)r * N + (i % N)] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_lds<N, C::NT>(buf, tw, threadIdx.x);
  for (int i = threadIdx.x; i < C::S * N; i += C::NT) {
    const int r = r0 + i / N;
    if (r < rows) x[(int64_t)r * N + (i % N)] = buf[lds_pad(i)];
  }
}

// y[c][r] = x[r][c] for an n x n complex matrix, 32 x 32 tiles through LDS.
__global__ void __launch_bounds__(256) image_transpose_kernel(const float2* __restrict__ x, int n,
                                                              float2* __restrict__ y) {
  __shared__ float2 t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int j = ty; j < 32; j += 8) t[j][tx] = x[(int64_t)(by + j) * n + bx + tx];
  __syncthreads();
  for (int j = ty; j < 32; j += 8) y[(int64_t)(bx + j) * n + by + tx] = t[tx][j];
}

// image[il][im] = (-1)^(il+im) Re(Y[il][im]) / W with Y held transposed:
// yt[im][il] = Y[il][im].
__global__ void image_final_kernel(const float2* __restrict__ yt, int n, const double* __restrict__ wsum,
                                   float* __restrict__ image) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int il = (int)(e / n), im = (int)(e % n);
  const double W = *wsum;
  const float s = ((il + im) & 1) ? -1.f : 1.f;
  const float re = yt[(int64_t)im * n + il].x;
  image[e] = W > 0.0 ? (float)((double)(s * re) / W) : 0.f;
}

template <int N>
hipError_t launch_rows(float2* x, int rows, const float2* tw, hipStream_t s) {
  using C = RowCfg<N>;
  const size_t lds = sizeof(float2) * C::LDS;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(image_rows_fft_kernel<N>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(image_rows_fft_kernel<N>, dim3((unsigned)((rows + C::S - 1) / C::S)), dim3(C::NT), lds, s,
                     x, rows, tw);
  return hipGetLastError();
}

hipError_t rows_fft(float2* x, int n, const float2* tw, hipStream_t s) {
  switch (n) {
    case 64: return launch_rows<64>(x, n, tw, s);
    case 128: return launch_rows<128>(x, n, tw, s);
    case 256: return launch_rows<256>(x, n, tw, s);
    case 512: return launch_rows<512>(x, n, tw, s);
    case 1024: return launch_rows<1024>(x, n, tw, s);
    case 2048: return launch_rows<2048>(x, n, tw, s);
    case 4096: return launch_rows<4096>(x, n, tw, s);
  }
  return hipErrorInvalidValue;
}

constexpr int CLEAN_NT = 1024;

// The beam subtraction rounds the product and the difference separately: no
// contraction into a fused multiply-add in this kernel (the pragma covers
// expressions written here, not inlined library helpers, so the arithmetic
// is spelled out).
#pragma clang fp contract(off)

__global__ void __launch_bounds__(CLEAN_NT)
image_clean_kernel(float* __restrict__ r, const float* __restrict__ psf, int n, float gain, float thr,
                   int max_iter, int* __restrict__ comp_pix, float* __restrict__ comp_flux,
                   int* __restrict__ n_comp) {
  __shared__ float bval[CLEAN_NT / 64];
  __shared__ float bsig[CLEAN_NT / 64];
  __shared__ int bidx[CLEAN_NT / 64];
  __shared__ float peak_s;
  __shared__ int pidx_s;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t npix = (int64_t)n * n;
  const int mask = n - 1, h = n / 2;
  float g = 0.f;   // flux of the component whose beam is still to subtract
  int pl = 0, pm = 0;
  int it = 0;
  for (;; ++it) {
    // subtract the previous component's beam (none before the first peak)
    // and find the next peak in the same sweep
    float best = -1.f, bv = 0.f;  // largest |residual| and its signed value
    int bi = 0x7fffffff;
    for (int64_t p = t; p < npix; p += CLEAN_NT) {
      float v = r[p];
      if (it > 0) {
        const int il = (int)(p / n), im = (int)(p % n);
        const int qi = (il - pl + h) & mask, qm = (im - pm + h) & mask;
        const float prod = g * psf[(int64_t)qi * n + qm];  // rounded product
        v = v - prod;                                       // rounded difference
        r[p] = v;
      }
      const float a = fabsf(v);
      if (a > best) {  // p increases along the thread's sweep: ties keep the first
        best = a;
        bv = v;
        bi = (int)p;
      }
    }
    for (int d = 32; d >= 1; d >>= 1) {
      const float ob = __shfl_down(best, d);
      const float ov = __shfl_down(bv, d);
      const int oi = __shfl_down(bi, d);
      if (lane + d < 64 && (ob > best || (ob == best && oi < bi))) {
        best = ob;
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      bval[wave] = best;
      bsig[wave] = bv;
      bidx[wave] = bi;
    }
    __syncthreads();
    if (t == 0) {
      float b = bval[0], sv = bsig[0];
      int i = bidx[0];
      for (int w = 1; w < CLEAN_NT / 64; ++w)
        if (bval[w] > b || (bval[w] == b && bidx[w] < i)) {
          b = bval[w];
          sv = bsig[w];
          i = bidx[w];
        }
      pidx_s = i;
      peak_s = sv;
    }
    __syncthreads();
    const float peak = peak_s;
    const int pi = pidx_s;
    __syncthreads();  // the shared values are read before the next reduction writes them
    if (it >= max_iter || !(fabsf(peak) >= thr)) break;
    g = gain * peak;
    pl = pi / n;
    pm = pi % n;
    if (t == 0) {
      comp_pix[it] = pi;
      comp_flux[it] = g;
    }
  }
  if (t == 0) *n_comp = it;
}

#pragma clang fp contract(on)

}  // namespace

}  // namespace qc

namespace {

bool img_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

extern "C" qc_status qc_image_grid(const float* u, const float* v, const float* vis, const float* weight,
                                   int64_t n_vis, int32_t n, double cell_rad, float* grid, double* wsum,
                                   void* stream) {
  qc::api_clear_error();
  if (!img_pow2(n) || n < 64 || n > 4096)
    return qc::api_fail(QC_EINVAL, "n must be a power of two in [64, 4096] (got %d)", n);
  if (!(cell_rad > 0.0)) return qc::api_fail(QC_EINVAL, "cell_rad must be positive");
  if (n_vis < 0) return qc::api_fail(QC_EINVAL, "n_vis must be >= 0");
  if (n_vis > 0 && (!u || !v || !vis)) return qc::api_fail(QC_EINVAL, "u, v and vis must be non-null");
  if (!grid || !wsum) return qc::api_fail(QC_EINVAL, "grid and wsum must be non-null");
  if ((reinterpret_cast<uintptr_t>(vis) | reinterpret_cast<uintptr_t>(grid)) & 7u)
    return qc::api_fail(QC_EINVAL, "vis and grid must be 8-byte aligned");
  if (reinterpret_cast<uintptr_t>(wsum) & 7u) return qc::api_fail(QC_EINVAL, "wsum must be 8-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t npix = (int64_t)n * n;
  hipLaunchKernelGGL(qc::image_zero_kernel, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<float2*>(grid), npix, wsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return qc::api_fail(QC_EHIP, "zero kernel: %s", hipGetErrorString(e));
  if (n_vis > 0) {
    const int64_t blocks = (n_vis + 255) / 256 < 4096 ? (n_vis + 255) / 256 : 4096;
    hipLaunchKernelGGL(qc::image_grid_kernel, dim3((unsigned)blocks), dim3(256), 0, s, u, v,
                       reinterpret_cast<const float2*>(vis), weight, n_vis, (int)n, (double)n * cell_rad,
                       reinterpret_cast<float2*>(grid), wsum);
    e = hipGetLastError();
    if (e != hipSuccess) return qc::api_fail(QC_EHIP, "grid kernel: %s", hipGetErrorString(e));
  }
  return QC_OK;
}

extern "C" qc_status qc_image_invert(const float* grid, const double* wsum, int32_t n, float* work,
                                     float* image, void* stream) {
  qc::api_clear_error();
  if (!img_pow2(n) || n < 64 || n > 4096)
    return qc::api_fail(QC_EINVAL, "n must be a power of two in [64, 4096] (got %d)", n);
  if (!grid || !wsum || !work || !image) return qc::api_fail(QC_EINVAL, "null buffer");
  if ((reinterpret_cast<uintptr_t>(grid) | reinterpret_cast<uintptr_t>(work)) & 7u)
    return qc::api_fail(QC_EINVAL, "grid and work must be 8-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float2* tw = nullptr;
  qc_status st = qc::api_twiddles(n, &tw);
  if (st != QC_OK) return st;
  const int64_t npix = (int64_t)n * n;
  float2* x = reinterpret_cast<float2*>(work);
  float2* y = x + npix;
  const unsigned blocks = (unsigned)((npix + 255) / 256);
  hipLaunchKernelGGL(qc::image_prep_kernel, dim3(blocks), dim3(256), 0, s,
                     reinterpret_cast<const float2*>(grid), (int)n, x);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = qc::rows_fft(x, n, tw, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(qc::image_transpose_kernel, dim3(n / 32, n / 32), dim3(256), 0, s, x, (int)n, y);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = qc::rows_fft(y, n, tw, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(qc::image_final_kernel, dim3(blocks), dim3(256), 0, s, y, (int)n, wsum, image);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return qc::api_fail(QC_EHIP, "inversion kernels: %s", hipGetErrorString(e));
  return QC_OK;
}

extern "C" qc_status qc_image_clean(float* residual, const float* psf, int32_t n, float gain, float threshold,
                                    int32_t max_iter, int32_t* comp_pix, float* comp_flux, int32_t* n_comp,
                                    void* stream) {
  qc::api_clear_error();
  if (!img_pow2(n) || n < 2 || n > 8192)
    return qc::api_fail(QC_EINVAL, "n must be a power of two in [2, 8192] (got %d)", n);
  if (!(gain > 0.f && gain <= 1.f)) return qc::api_fail(QC_EINVAL, "gain must be in (0, 1]");
  if (!(threshold >= 0.f)) return qc::api_fail(QC_EINVAL, "threshold must be >= 0");
  if (max_iter < 0) return qc::api_fail(QC_EINVAL, "max_iter must be >= 0");
  if (!residual || !psf || !n_comp || (max_iter > 0 && (!comp_pix || !comp_flux)))
    return qc::api_fail(QC_EINVAL, "null buffer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(qc::image_clean_kernel, dim3(1), dim3(qc::CLEAN_NT), 0, s, residual, psf, (int)n, gain,
                     threshold, (int)max_iter, reinterpret_cast<int*>(comp_pix), comp_flux,
                     reinterpret_cast<int*>(n_comp));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return qc::api_fail(QC_EHIP, "clean kernel: %s", hipGetErrorString(e));
  return QC_OK;
}
