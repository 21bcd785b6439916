// Fused float32 F+X that allocates no device memory: qc_xcorrelate_noalloc.
//
// For callers that cannot allocate (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  The work memory that
// qc_xcorrelate takes from the stream-ordered pool (FFT twiddles, the
// built-in prototype's taps, per-workgroup partial visibilities) lives here
// in one fixed device array, `scratch`, of QC_NOALLOC_SCRATCH_BYTES per GPU.
// The array stays resident on every GPU the library runs on until the
// process ends.  Its device address is looked up once per device with
// hipGetSymbolAddress (in host code the array's name is not a device
// address); every later use goes through that pointer.
//
// The kernels are the fused F+X kernels and the fixed-order reduction of
// qc_xcorrelate.  Dumps are processed in batches whose partial sums fit the
// array; a batch that starts inside the stream takes the (P-1) N samples
// before it as its filter history (copied into the array by the history
// kernel), so results equal one pass over all dumps up to the order of the
// partial sums.
//
// Every call on a GPU uses that GPU's one array and leaves its contents
// behind: calls that overlap on one GPU (other streams, other threads) race.
#include <hip/hip_runtime.h>

#include <math.h>
#include <mutex>

#include "qc.h"
#include "qc_internal.h"
#include "qc_kernels.h"

namespace {

constexpr int64_t kScratchBytes = QC_NOALLOC_SCRATCH_BYTES;
constexpr int64_t kTwBytes = 8192 * 8;        // float2 [n_fft], n_fft <= 8192
constexpr int64_t kTapsBytes = 16 * 8192 * 4; // float [P * n_fft], P <= 16
constexpr int64_t kHistBytes = 1 << 20;       // int8 [n_ant][(P-1) n_fft]
constexpr int64_t kTwpBytes = 8192 * 8;       // float2 [n_fft - 1], per-pass twiddles
constexpr int64_t kPartOff = kTwBytes + kTapsBytes + kHistBytes + kTwpBytes;
static_assert(kPartOff % 256 == 0, "scratch regions stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this GPU's array (looked up once per device).
qc_status scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return qc::api_fail(QC_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return qc::api_fail(QC_EUNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return qc::api_fail(QC_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return QC_OK;
}

// twp: the per-pass twiddles of the radix-16 Stockham FFT (pass of stride NS
// and radix R: W_{NS R}^{jm r} at (NS-1) + (r-1) NS + jm), entry i < N-1;
// tw[e] = exp(-2 pi i e / N) from the exact integer e (float64, rounded once);
// h[q] = Hann-windowed sinc of L = P N taps, centre (L-1)/2, sinc zeros every
// N, unnormalised (the built-in prototype).  Same definitions as the cached
// host-built tables of qc_xcorrelate.
__global__ void noalloc_tables_kernel(int N, int P, int build_taps, float2* __restrict__ tw,
                                      float* __restrict__ taps, float2* __restrict__ twp) {
  const int L = N * P;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N + L; i += gridDim.x * blockDim.x) {
    if (i < N - 1) {
      int ns = 1, off = 0;
      while (true) {
        const int R = (N / ns) >= 16 ? 16 : N / ns;
        if (i < off + (R - 1) * ns) {
          const int q = i - off, r = 1 + q / ns, jm = q % ns;
          double sv, cv;
          sincospi(-2.0 * (double)((jm * r) % (ns * R)) / (double)(ns * R), &sv, &cv);
          twp[i] = make_float2((float)cv, (float)sv);
          break;
        }
        off += (R - 1) * ns;
        ns *= R;
      }
    }
    if (i < N) {
      double sv, cv;
      sincospi(-2.0 * (double)i / (double)N, &sv, &cv);
      tw[i] = make_float2((float)cv, (float)sv);
    } else if (build_taps) {
      const int q = i - N;
      const double w = 0.5 - 0.5 * cospi(2.0 * (double)q / (double)(L - 1));
      const double u = ((double)q - (L - 1) / 2.0) / (double)N;
      const double s = (u == 0.0) ? 1.0 : sinpi(u) / (3.14159265358979323846 * u);
      taps[q] = (float)(w * s);
    }
  }
}

}  // namespace

extern "C" qc_status qc_xcorrelate_noalloc(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                                           const qc_pfb_params* p, const int8_t* hist, int8_t* hist_out,
                                           int64_t spec_per_dump, float* vis, int32_t accumulate,
                                           int64_t* n_dumps_out, void* stream) {
  qc::api_clear_error();
  qc_status st = qc::api_check_stream_args(x, ld_x, n_ant, n_samp, p, hist, hist_out);
  if (st != QC_OK) return st;
  if (spec_per_dump < 1) return qc::api_fail(QC_EINVAL, "spec_per_dump must be >= 1");
  const int N = p->n_fft, P = p->n_taps;
  if (!qc::fused_supported(N, n_ant))
    return qc::api_fail(QC_EUNSUPPORTED,
                        "no fused F+X kernel for n_fft %d with %d antennas (qc_xcorrelate_noalloc "
                        "covers the fused shapes only)", N, n_ant);
  const int64_t n_dump = (n_samp / N) / spec_per_dump;
  if (n_dump > 0 && !vis) return qc::api_fail(QC_EINVAL, "vis is NULL");
  if (reinterpret_cast<uintptr_t>(vis) & 7u) return qc::api_fail(QC_EINVAL, "vis must be 8-byte aligned");
  const int nch = N / 2;
  const int64_t nb = (int64_t)n_ant * (n_ant + 1) / 2;
  const int64_t keep = (int64_t)(P - 1) * N;
  const int64_t part_bytes = (int64_t)nb * nch * (int64_t)sizeof(float2);  // one workgroup's partial
  const int64_t cap = (kScratchBytes - kPartOff) / part_bytes;             // partials that fit
  if (cap < 1 || (int64_t)n_ant * keep > kHistBytes)
    return qc::api_fail(QC_EUNSUPPORTED,
                        "qc_xcorrelate_noalloc: one dump of %d antennas x %d channels needs more than "
                        "its %lld-byte work array", n_ant, nch, (long long)kScratchBytes);
  if (n_dumps_out) *n_dumps_out = n_dump;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (n_dump > 0) {
    void* base = nullptr;
    st = scratch_ptr(&base);
    if (st != QC_OK) return st;
    unsigned char* b = static_cast<unsigned char*>(base);
    float2* tw = reinterpret_cast<float2*>(b);
    float* taps_dev = reinterpret_cast<float*>(b + kTwBytes);
    int8_t* bhist = reinterpret_cast<int8_t*>(b + kTwBytes + kTapsBytes);
    float2* twp = reinterpret_cast<float2*>(b + kTwBytes + kTapsBytes + kHistBytes);
    float2* part = reinterpret_cast<float2*>(b + kPartOff);
    const int build_taps = p->taps == nullptr;
    const int n_tab = N + (build_taps ? N * P : 0);
    hipLaunchKernelGGL(noalloc_tables_kernel, dim3((unsigned)((n_tab + 255) / 256)), dim3(256), 0, s, N, P,
                       build_taps, tw, taps_dev, twp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return qc::api_fail(QC_EHIP, "tables kernel: %s", hipGetErrorString(e));
    qc::FxArgs a{x, ld_x, n_ant, 0, N, P, build_taps ? taps_dev : p->taps, tw, hist, build_taps != 0, twp};
    const int tile = qc_fx_get_tile(N, n_ant);
    const int64_t nd_max = cap < n_dump ? cap : n_dump;
    for (int64_t d0 = 0; d0 < n_dump; d0 += nd_max) {
      const int64_t nd = (n_dump - d0) < nd_max ? (n_dump - d0) : nd_max;
      int64_t cpd = qc::fused_chunks_per_dump(N, n_ant, nd, spec_per_dump);
      if (cpd > cap / nd) cpd = cap / nd;
      const int64_t s0 = d0 * spec_per_dump * N;  // first sample of the batch
      qc::FxArgs ab = a;
      ab.x = x + s0;
      ab.n_samp = nd * spec_per_dump * N;
      if (d0 > 0) {
        if (keep > 0) {
          e = qc::launch_hist_copy(x, ld_x, n_ant, s0, hist, keep, bhist, s);
          if (e != hipSuccess) return qc::api_fail(QC_EHIP, "history copy: %s", hipGetErrorString(e));
        }
        ab.hist = keep > 0 ? bhist : nullptr;
      }
      e = qc::launch_fused(ab, nd, spec_per_dump, cpd, part, s, tile);
      if (e != hipSuccess) return qc::api_fail(QC_EHIP, "fused F+X kernel: %s", hipGetErrorString(e));
      e = qc::launch_reduce(part, nd, cpd, nb * nch, 0.25f, accumulate,
                            reinterpret_cast<float2*>(vis) + d0 * nb * nch, s);
      if (e != hipSuccess) return qc::api_fail(QC_EHIP, "reduce kernel: %s", hipGetErrorString(e));
    }
  }
  if (hist_out && P > 1) {
    hipError_t e = qc::launch_hist_copy(x, ld_x, n_ant, n_samp, hist, keep, hist_out, s);
    if (e != hipSuccess) return qc::api_fail(QC_EHIP, "history copy: %s", hipGetErrorString(e));
  }
  return QC_OK;
}
