// C-ABI entry points of libqc: host-side argument validation, per-device
// caches of filter taps and FFT twiddles, workspace management and kernel
// selection.  See include/qc.h for the contract of each call.
#include "qc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <fstream>
#include <sstream>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "qc_internal.h"
#include "qc_kernels.h"

#include <new>

namespace {

thread_local std::string g_err;

qc_status fail(qc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

qc_status hip_fail(hipError_t e, const char* what) {
  return fail(QC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define QC_HIP(call, what)                        \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// ---- built-in prototype filter and twiddles (float64 on the host) ----------

// Hann-windowed sinc, L = P*N taps, centre (L-1)/2, sinc zeros every N.
std::vector<double> hann_sinc(int N, int P) {
  const int L = N * P;
  std::vector<double> h(L);
  const double pi = 3.14159265358979323846;
  for (int q = 0; q < L; ++q) {
    const double w = L > 1 ? 0.5 - 0.5 * std::cos(2.0 * pi * q / (L - 1)) : 1.0;
    const double u = (q - (L - 1) / 2.0) / N;
    const double s = (u == 0.0) ? 1.0 : std::sin(pi * u) / (pi * u);
    h[q] = w * s;
  }
  return h;
}

// Modified Bessel function of the first kind, order 0, by its power series
// sum_k ((x/2)^k / k!)^2 (all terms positive; stops once a term no longer
// changes the float64 sum).
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= q / ((double)k * (double)k);
    const double next = sum + term;
    if (next == sum) break;
    sum = next;
  }
  return sum;
}

// Prototype filters for qc_pfb_design_taps, float64: window 0 Hann-sinc
// (the built-in prototype), 1 Kaiser(beta)-sinc, 2 all ones (no filter).
std::vector<double> design_taps(int N, int P, int window, double beta) {
  if (window == 0) return hann_sinc(N, P);
  const int L = N * P;
  std::vector<double> h(L, 1.0);
  if (window == 2) return h;
  const double pi = 3.14159265358979323846;
  const double i0b = bessel_i0(beta);
  for (int q = 0; q < L; ++q) {
    double w = 1.0;
    if (L > 1) {
      const double r = 2.0 * q / (L - 1) - 1.0;
      const double t = 1.0 - r * r;
      w = bessel_i0(beta * std::sqrt(t > 0.0 ? t : 0.0)) / i0b;
    }
    const double u = (q - (L - 1) / 2.0) / N;
    const double sn = (u == 0.0) ? 1.0 : std::sin(pi * u) / (pi * u);
    h[q] = w * sn;
  }
  return h;
}

int sample_bytes(int sample) { return sample == 0 ? 1 : sample == 3 ? 4 : 2; }
bool sample_complex(int sample) { return sample >= 2; }

struct TapsEntry {
  float* dev = nullptr;
  double sum_h2 = 0.0;
};

std::mutex g_mu;
std::map<std::tuple<int, int, int>, TapsEntry> g_taps;  // (device, N, P)
std::map<std::pair<int, int>, float2*> g_tw;            // (device, N)

qc_status get_taps(int N, int P, TapsEntry* out) {
  int dev = 0;
  QC_HIP(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(dev, N, P);
  auto it = g_taps.find(key);
  if (it != g_taps.end()) {
    *out = it->second;
    return QC_OK;
  }
  std::vector<double> h = hann_sinc(N, P);
  std::vector<float> hf(h.size());
  double s2 = 0.0;
  for (size_t i = 0; i < h.size(); ++i) {
    hf[i] = (float)h[i];
    s2 += h[i] * h[i];
  }
  TapsEntry e;
  QC_HIP(hipMalloc(&e.dev, hf.size() * sizeof(float)), "hipMalloc(taps)");
  QC_HIP(hipMemcpy(e.dev, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice),
         "hipMemcpy(taps)");
  e.sum_h2 = s2;
  g_taps[key] = e;
  *out = e;
  return QC_OK;
}

// Once per device: keep freed stream-ordered allocations in the device's
// default pool instead of returning them at every synchronisation, so the
// per-call scratch buffers are reused rather than re-mapped.
std::map<int, bool> g_pool_ready;

qc_status device_init_locked(int dev) {
  if (g_pool_ready.count(dev)) return QC_OK;
  hipMemPool_t pool = nullptr;
  QC_HIP(hipDeviceGetDefaultMemPool(&pool, dev), "hipDeviceGetDefaultMemPool");
  uint64_t thr = UINT64_MAX;
  QC_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr), "hipMemPoolSetAttribute");
  g_pool_ready[dev] = true;
  return QC_OK;
}

qc_status ensure_device() {
  int dev = 0;
  QC_HIP(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  return device_init_locked(dev);
}

qc_status get_twiddles(int N, float2** out) {
  int dev = 0;
  QC_HIP(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  qc_status st = device_init_locked(dev);
  if (st != QC_OK) return st;
  auto key = std::make_pair(dev, N);
  auto it = g_tw.find(key);
  if (it != g_tw.end()) {
    *out = it->second;
    return QC_OK;
  }
  // exp(-2 pi i e / N): angle from the exact integer e, evaluated in float64,
  // rounded once to float32.
  std::vector<float2> tw(N);
  const double pi = 3.14159265358979323846;
  for (int e = 0; e < N; ++e) {
    const double a = -2.0 * pi * (double)e / (double)N;
    tw[e] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  float2* d = nullptr;
  QC_HIP(hipMalloc(&d, N * sizeof(float2)), "hipMalloc(twiddles)");
  QC_HIP(hipMemcpy(d, tw.data(), N * sizeof(float2), hipMemcpyHostToDevice), "hipMemcpy(twiddles)");
  g_tw[key] = d;
  *out = d;
  return QC_OK;
}

std::map<std::pair<int, int>, float2*> g_twp;  // (device, N): per-pass radix-16 twiddles

// Per-pass twiddles of the radix-16 Stockham FFT (radix 16 while it divides
// what is left, then the remainder): the pass of stride NS and radix R holds
// W_{NS R}^{jm r} = exp(-2 pi i jm r / (NS R)) at (NS-1) + (r-1) NS + jm,
// r = 1..R-1, jm = 0..NS-1; N-1 entries over all passes.  The angle comes
// from the exact integers, in float64, rounded once to float32.
qc_status get_pass_twiddles(int N, float2** out) {
  int dev = 0;
  QC_HIP(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, N);
  auto it = g_twp.find(key);
  if (it != g_twp.end()) {
    *out = it->second;
    return QC_OK;
  }
  std::vector<float2> t(N > 1 ? N - 1 : 1, make_float2(0.f, 0.f));
  const double pi = 3.14159265358979323846;
  int ns = 1, off = 0;
  while (N / ns > 1) {
    const int R = (N / ns) >= 16 ? 16 : N / ns;
    for (int r = 1; r < R; ++r)
      for (int jm = 0; jm < ns; ++jm) {
        const long long e = (long long)jm * r;  // exponent of W_{ns R}
        const double a = -2.0 * pi * (double)(e % (ns * R)) / (double)(ns * R);
        t[off + (r - 1) * ns + jm] = make_float2((float)std::cos(a), (float)std::sin(a));
      }
    off += (R - 1) * ns;
    ns *= R;
  }
  float2* d = nullptr;
  QC_HIP(hipMalloc(&d, t.size() * sizeof(float2)), "hipMalloc(pass twiddles)");
  QC_HIP(hipMemcpy(d, t.data(), t.size() * sizeof(float2), hipMemcpyHostToDevice), "hipMemcpy(pass twiddles)");
  g_twp[key] = d;
  *out = d;
  return QC_OK;
}

qc_status check_pfb(const qc_pfb_params* p) {
  if (!p) return fail(QC_EINVAL, "pfb params is NULL");
  if (!is_pow2(p->n_fft) || p->n_fft < 4 || p->n_fft > 8192)
    return fail(QC_EINVAL, "n_fft must be a power of two in [4, 8192] (got %d)", p->n_fft);
  if (p->n_taps < 1 || p->n_taps > 16)
    return fail(QC_EINVAL, "n_taps must be in [1, 16] (got %d)", p->n_taps);
  if (p->keep_nyquist != 0) return fail(QC_EUNSUPPORTED, "keep_nyquist must be 0");
  if (p->taps && (reinterpret_cast<uintptr_t>(p->taps) & 15u))
    return fail(QC_EINVAL, "taps must be 16-byte aligned");
  return QC_OK;
}

qc_status check_stream_args(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                            const qc_pfb_params* p, const int8_t* hist, const int8_t* hist_out) {
  qc_status st = check_pfb(p);
  if (st != QC_OK) return st;
  if (n_ant < 1 || n_ant > 4096) return fail(QC_EINVAL, "n_ant must be in [1, 4096] (got %d)", n_ant);
  if (n_samp < 0 || n_samp % p->n_fft)
    return fail(QC_EINVAL, "n_samp (%lld) must be a non-negative multiple of n_fft (%d)",
                (long long)n_samp, p->n_fft);
  if (n_samp > 0x7fffffffLL) return fail(QC_EINVAL, "n_samp must be below 2^31 per antenna");
  if (n_samp > 0 && !x) return fail(QC_EINVAL, "x is NULL");
  if (ld_x < n_samp || (ld_x & 3)) return fail(QC_EINVAL, "ld_x must be >= n_samp and a multiple of 4");
  if (reinterpret_cast<uintptr_t>(x) & 3u) return fail(QC_EINVAL, "x must be 4-byte aligned");
  if (hist && (reinterpret_cast<uintptr_t>(hist) & 3u)) return fail(QC_EINVAL, "hist must be 4-byte aligned");
  if (hist && hist == hist_out) return fail(QC_EINVAL, "hist_out may not alias hist");
  return QC_OK;
}

struct Resolved {
  qc::FxArgs args;
  double sum_h2;
};

qc_status resolve(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                  const qc_pfb_params* p, const int8_t* hist, Resolved* r) {
  float2* tw = nullptr;
  qc_status st = get_twiddles(p->n_fft, &tw);
  if (st != QC_OK) return st;
  const float* taps = p->taps;
  double s2 = 0.0;
  if (!taps) {
    TapsEntry e;
    st = get_taps(p->n_fft, p->n_taps, &e);
    if (st != QC_OK) return st;
    taps = e.dev;
    s2 = e.sum_h2;
  }
  float2* twp = nullptr;
  st = get_pass_twiddles(p->n_fft, &twp);
  if (st != QC_OK) return st;
  r->args = qc::FxArgs{x, ld_x, n_ant, n_samp, p->n_fft, p->n_taps, taps, tw, hist, p->taps == nullptr, twp};
  r->sum_h2 = s2;
  return QC_OK;
}

// sum of squares of user taps (float64), read back from the device
qc_status user_sum_h2(const float* taps, int L, double* out) {
  std::vector<float> h(L);
  QC_HIP(hipMemcpy(h.data(), taps, L * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy(user taps)");
  double s = 0.0;
  for (float v : h) s += (double)v * (double)v;
  *out = s;
  return QC_OK;
}

double prec_target(int prec) {
  return prec == QC_F16 ? 256.0 : prec == QC_BF16 ? 1.0 : 32.0;
}

size_t prec_pair_bytes(int prec) {
  return prec == QC_F32 ? 8 : prec == QC_FP8_E4M3 ? 2 : 4;
}

// Stream-ordered scratch allocation released at scope end (also stream-ordered).
struct AsyncBuf {
  void* p = nullptr;
  hipStream_t s = nullptr;
  ~AsyncBuf() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

qc_status alloc_async(AsyncBuf& b, size_t bytes, hipStream_t s) {
  b.s = s;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMallocAsync(&b.p, bytes, s);
  if (e != hipSuccess) return fail(QC_ENOMEM, "hipMallocAsync(%zu): %s", bytes, hipGetErrorString(e));
  return QC_OK;
}

// ---- kernel timing ----------------------------------------------------------
// Mode 1 brackets each timed call with two events recorded on its stream.
// Mode 2 records no packet of its own: every kernel the library launches
// carries a stop event (timing_stop_event), and a timed call runs from the
// stop event of the library's previous launch on the same stream (an event
// recorded just before it when there is none) to the stop event of its own
// last launch.
struct TimingRec {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[QC_KERNEL_COUNT];
  std::vector<hipEvent_t> owned;             // every event created while timing
  std::map<hipStream_t, hipEvent_t> tail;    // mode 2: last stop event per stream
};
std::mutex g_tmu;
std::atomic<int> g_timing{0};  // written under g_tmu; read without it on the launch path
TimingRec g_trec;

void timing_clear_locked() {
  for (hipEvent_t e : g_trec.owned) (void)hipEventDestroy(e);
  g_trec.owned.clear();
  for (auto& v : g_trec.ev) v.clear();
  g_trec.tail.clear();
}

// Timing-only events: no system-scope fence when they complete, so binding
// one to a launch adds no cache writeback after it.
hipEvent_t timing_new_event_locked() {
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  g_trec.owned.push_back(e);
  return e;
}

struct KTimer;
thread_local KTimer* t_ktimer = nullptr;

// Brackets one timed call on its stream while timing is enabled.
struct KTimer {
  int k;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  KTimer* outer = nullptr;
  KTimer(int kernel, hipStream_t st) : k(kernel), s(st) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (g_timing == 2) {
      outer = t_ktimer;
      t_ktimer = this;
      return;
    }
    if (g_timing != 1) return;
    a = timing_new_event_locked();
    b = timing_new_event_locked();
    if (!a || !b) { a = b = nullptr; return; }
    (void)hipEventRecord(a, s);
  }
  ~KTimer() {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (t_ktimer == this) t_ktimer = outer;
    if (!a || !b) return;
    if (g_timing == 1) (void)hipEventRecord(b, s);
    g_trec.ev[k].emplace_back(a, b);
  }
};

}  // namespace

namespace qc {
hipEvent_t timing_stop_event(hipStream_t s) {
  if (g_timing.load(std::memory_order_relaxed) != 2) return nullptr;
  // launches being captured into a graph carry no events
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  std::lock_guard<std::mutex> lk(g_tmu);
  if (g_timing.load(std::memory_order_relaxed) != 2) return nullptr;
  hipEvent_t e = timing_new_event_locked();
  if (!e) return nullptr;
  KTimer* t = t_ktimer;
  if (t && t->s == s) {
    if (!t->a) {
      auto it = g_trec.tail.find(s);
      if (it != g_trec.tail.end()) {
        t->a = it->second;
      } else if ((t->a = timing_new_event_locked()) != nullptr) {
        (void)hipEventRecord(t->a, s);
      }
    }
    t->b = e;
  }
  g_trec.tail[s] = e;
  return e;
}
}  // namespace qc

namespace {

// ---- fused-kernel tile selection (default 0; set by the autotuner) ---------
std::mutex g_tile_mu;
std::map<std::pair<int, int>, int> g_tile;  // (n_fft, n_ant) -> tile index
// (n_fft, n_ant) -> workgroups per fused launch (absent: the default policy)
std::map<std::pair<int, int>, int64_t> g_width;

int fused_tile_for(int n_fft, int n_ant) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  auto it = g_tile.find({n_fft, n_ant});
  return it == g_tile.end() ? 0 : it->second;
}

int64_t fused_width_for(int n_fft, int n_ant) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  auto it = g_width.find({n_fft, n_ant});
  return it == g_width.end() ? 0 : it->second;
}

qc_status channelize_impl(const Resolved& r, qc_prec out_prec, void* out, float* scale_out,
                          hipStream_t s) {
  const qc::FxArgs& a = r.args;
  if (out_prec != QC_F32) {
    double s2 = r.sum_h2;
    if (a.taps != nullptr && s2 == 0.0) {
      qc_status st = user_sum_h2(a.taps, a.n_fft * a.n_taps, &s2);
      if (st != QC_OK) return st;
    }
    const int64_t n_use = a.n_samp < (1 << 20) ? a.n_samp : (1 << 20);
    if (n_use > 0) {
      AsyncBuf sp;
      qc_status st = alloc_async(sp, (size_t)a.n_ant * qc::SC_BLOCKS * sizeof(unsigned long long), s);
      if (st != QC_OK) return st;
      QC_HIP(qc::launch_scales(a.x, a.ld_x, a.n_ant, n_use, s2, prec_target(out_prec),
                               (unsigned long long*)sp.p, scale_out, s),
             "scales kernel");
    }
  }
  if (a.n_samp > 0) {
    KTimer t(QC_KERNEL_CHANNELIZE, s);
    QC_HIP(qc::launch_channelize(a, (int)out_prec, out, scale_out, s), "channelize kernel");
  }
  return QC_OK;
}

qc_status check_any_args(const void* x, int32_t sample, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                         const qc_pfb_params* p, const void* hist, const void* hist_out) {
  qc_status st = check_pfb(p);
  if (st != QC_OK) return st;
  if (sample < QC_SAMPLE_I8 || sample > QC_SAMPLE_CI16) return fail(QC_EINVAL, "bad sample word %d", sample);
  if (n_ant < 1 || n_ant > 4096) return fail(QC_EINVAL, "n_ant must be in [1, 4096] (got %d)", n_ant);
  if (n_samp < 0 || n_samp % p->n_fft)
    return fail(QC_EINVAL, "n_samp (%lld) must be a non-negative multiple of n_fft (%d)",
                (long long)n_samp, p->n_fft);
  if (n_samp > 0x7fffffffLL) return fail(QC_EINVAL, "n_samp must be below 2^31 per antenna");
  if (n_samp > 0 && !x) return fail(QC_EINVAL, "x is NULL");
  if (ld_x < n_samp || (ld_x & 3)) return fail(QC_EINVAL, "ld_x must be >= n_samp and a multiple of 4");
  const uintptr_t al = 4u * (uintptr_t)sample_bytes(sample) - 1u;
  if (reinterpret_cast<uintptr_t>(x) & al)
    return fail(QC_EINVAL, "x must be aligned to 4 samples (%d bytes)", (int)(al + 1));
  if (hist && (reinterpret_cast<uintptr_t>(hist) & al))
    return fail(QC_EINVAL, "hist must be aligned to 4 samples (%d bytes)", (int)(al + 1));
  if (hist && hist == hist_out) return fail(QC_EINVAL, "hist_out may not alias hist");
  return QC_OK;
}

// The F-engine of any word into `out` (n_samp samples, caller-validated).
qc_status channelize_any_impl(const void* x, int32_t sample, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                              const qc_pfb_params* p, const void* hist, qc_prec out_prec, void* out,
                              float* scale_out, hipStream_t s) {
  Resolved r;
  qc_status st = resolve(nullptr, ld_x, n_ant, n_samp, p, nullptr, &r);
  if (st != QC_OK) return st;
  const qc::ChanxArgs a{x, ld_x, n_ant, n_samp, p->n_fft, p->n_taps, r.args.taps, r.args.tw, hist,
                       r.args.taps_symmetric, r.args.twp};
  if (out_prec != QC_F32) {
    double s2 = r.sum_h2;
    if (p->taps != nullptr) {
      st = user_sum_h2(p->taps, p->n_fft * p->n_taps, &s2);
      if (st != QC_OK) return st;
    }
    const int64_t n_use = n_samp < (1 << 20) ? n_samp : (1 << 20);
    if (n_use > 0) {
      AsyncBuf sp;
      st = alloc_async(sp, (size_t)n_ant * qc::SC_BLOCKS * sizeof(unsigned long long), s);
      if (st != QC_OK) return st;
      QC_HIP(qc::launch_scales_any(x, sample, ld_x, n_ant, n_use, s2, prec_target(out_prec),
                                   (unsigned long long*)sp.p, scale_out, s),
             "scales kernel");
    }
  }
  if (n_samp > 0) {
    KTimer t(QC_KERNEL_CHANNELIZE, s);
    QC_HIP(qc::launch_channelize_any(a, sample, (int)out_prec, out, scale_out, s), "channelize kernel");
  }
  return QC_OK;
}

qc_status hist_copy_any(const void* x, int32_t sample, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                        const qc_pfb_params* p, const void* hist, void* hist_out, hipStream_t s) {
  if (!hist_out || p->n_taps <= 1) return QC_OK;
  const int b = sample_bytes(sample);
  const int64_t keep = (int64_t)(p->n_taps - 1) * p->n_fft;
  // byte-wise copy of the last keep samples of (hist ++ x)
  QC_HIP(qc::launch_hist_copy(static_cast<const int8_t*>(x), ld_x * b, n_ant, n_samp * b,
                              static_cast<const int8_t*>(hist), keep * b, static_cast<int8_t*>(hist_out), s),
         "history copy");
  return QC_OK;
}

}  // namespace

namespace qc {

void api_clear_error() { g_err.clear(); }

qc_status api_fail(qc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

qc_status api_check_stream_args(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                                const qc_pfb_params* p, const int8_t* hist, const int8_t* hist_out) {
  return check_stream_args(x, ld_x, n_ant, n_samp, p, hist, hist_out);
}

qc_status api_twiddles(int n, float2** out) { return get_twiddles(n, out); }

}  // namespace qc

extern "C" {

const char* qc_status_string(qc_status s) {
  switch (s) {
    case QC_OK: return "QC_OK";
    case QC_EINVAL: return "QC_EINVAL";
    case QC_EUNSUPPORTED: return "QC_EUNSUPPORTED";
    case QC_EHIP: return "QC_EHIP";
    case QC_ENOMEM: return "QC_ENOMEM";
    case QC_ESTATE: return "QC_ESTATE";
  }
  return "QC_UNKNOWN";
}

const char* qc_last_error(void) { return g_err.c_str(); }

const char* qc_version(void) { return "qc 0.1.0 (gfx950)"; }

qc_status qc_pfb_channelize(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                            const qc_pfb_params* p, const int8_t* hist, int8_t* hist_out,
                            qc_prec out_prec, void* out, float* scale_out, void* stream) {
  g_err.clear();
  qc_status st = check_stream_args(x, ld_x, n_ant, n_samp, p, hist, hist_out);
  if (st != QC_OK) return st;
  if (out_prec < QC_F32 || out_prec > QC_FP8_E4M3) return fail(QC_EINVAL, "bad out_prec %d", (int)out_prec);
  if (n_samp > 0 && !out) return fail(QC_EINVAL, "out is NULL");
  if (out_prec != QC_F32 && !scale_out) return fail(QC_EINVAL, "scale_out is NULL for reduced precision");
  if (reinterpret_cast<uintptr_t>(out) % prec_pair_bytes(out_prec))
    return fail(QC_EINVAL, "out is misaligned for its precision");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Resolved r;
  st = resolve(x, ld_x, n_ant, n_samp, p, hist, &r);
  if (st != QC_OK) return st;
  st = channelize_impl(r, out_prec, out, scale_out, s);
  if (st != QC_OK) return st;
  if (hist_out && p->n_taps > 1)
    QC_HIP(qc::launch_hist_copy(x, ld_x, n_ant, n_samp, hist, (int64_t)(p->n_taps - 1) * p->n_fft,
                                hist_out, s),
           "history copy");
  return QC_OK;
}

qc_status qc_xcorrelate(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                        const qc_pfb_params* p, const int8_t* hist, int8_t* hist_out,
                        int64_t spec_per_dump, qc_prec x_prec, float* vis, int32_t accumulate,
                        int64_t* n_dumps_out, void* stream) {
  g_err.clear();
  qc_status st = check_stream_args(x, ld_x, n_ant, n_samp, p, hist, hist_out);
  if (st != QC_OK) return st;
  if (spec_per_dump < 1) return fail(QC_EINVAL, "spec_per_dump must be >= 1");
  if (x_prec < QC_F32 || x_prec > QC_FP8_E4M3) return fail(QC_EINVAL, "bad x_prec %d", (int)x_prec);
  const int N = p->n_fft;
  const int64_t n_spec = n_samp / N;
  const int64_t n_dump = n_spec / spec_per_dump;
  if (n_dump > 0 && !vis) return fail(QC_EINVAL, "vis is NULL");
  if (reinterpret_cast<uintptr_t>(vis) & 7u) return fail(QC_EINVAL, "vis must be 8-byte aligned");
  if (n_dumps_out) *n_dumps_out = n_dump;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int nch = N / 2;
  const int64_t nb = (int64_t)n_ant * (n_ant + 1) / 2;
  if (n_dump > 0) {
    Resolved r;
    st = resolve(x, ld_x, n_ant, n_samp, p, hist, &r);
    if (st != QC_OK) return st;
    // only the spectra of full dumps are transformed
    r.args.n_samp = n_dump * spec_per_dump * N;
    if (x_prec == QC_F32 && qc::fused_supported(N, n_ant)) {
      const int64_t cpd = qc::fused_chunks_per_dump(N, n_ant, n_dump, spec_per_dump, fused_width_for(N, n_ant));
      AsyncBuf part;
      st = alloc_async(part, (size_t)(n_dump * cpd) * nb * nch * sizeof(float2), s);
      if (st != QC_OK) return st;
      {
        KTimer t(QC_KERNEL_FX_FUSED, s);
        QC_HIP(qc::launch_fused(r.args, n_dump, spec_per_dump, cpd, (float2*)part.p, s,
                                fused_tile_for(N, n_ant)),
               "fused F+X kernel");
      }
      KTimer t(QC_KERNEL_REDUCE, s);
      QC_HIP(qc::launch_reduce((const float2*)part.p, n_dump, cpd, nb * nch, 0.25f, accumulate,
                               reinterpret_cast<float2*>(vis), s),
             "reduce kernel");
    } else {
      // two passes: F-engine to HBM, then the X-engine
      const int64_t ns = n_dump * spec_per_dump;
      AsyncBuf v, scale;
      st = alloc_async(v, (size_t)n_ant * ns * nch * prec_pair_bytes(x_prec), s);
      if (st != QC_OK) return st;
      st = alloc_async(scale, (size_t)n_ant * sizeof(float), s);
      if (st != QC_OK) return st;
      st = channelize_impl(r, x_prec, v.p, (float*)scale.p, s);
      if (st != QC_OK) return st;
      st = qc_xcorrelate_chan(v.p, x_prec, (const float*)scale.p, n_ant, ns, nch, spec_per_dump,
                              vis, accumulate, stream);
      if (st != QC_OK) return st;
    }
  }
  if (hist_out && p->n_taps > 1)
    QC_HIP(qc::launch_hist_copy(x, ld_x, n_ant, n_samp, hist, (int64_t)(p->n_taps - 1) * N, hist_out, s),
           "history copy");
  return QC_OK;
}

qc_status qc_pfb_design_taps(int32_t n_fft, int32_t n_taps, int32_t window, double beta, float* taps,
                             void* stream) {
  g_err.clear();
  if (!is_pow2(n_fft) || n_fft < 4 || n_fft > 8192)
    return fail(QC_EINVAL, "n_fft must be a power of two in [4, 8192] (got %d)", n_fft);
  if (n_taps < 1 || n_taps > 16) return fail(QC_EINVAL, "n_taps must be in [1, 16] (got %d)", n_taps);
  if (window < QC_WINDOW_HANN || window > QC_WINDOW_RECT) return fail(QC_EINVAL, "bad window %d", window);
  if (window == QC_WINDOW_KAISER && !(beta >= 0.0 && beta <= 100.0))
    return fail(QC_EINVAL, "Kaiser beta must be in [0, 100]");
  if (!taps) return fail(QC_EINVAL, "taps is NULL");
  if (reinterpret_cast<uintptr_t>(taps) & 15u) return fail(QC_EINVAL, "taps must be 16-byte aligned");
  const std::vector<double> h = design_taps(n_fft, n_taps, window, beta);
  std::vector<float> hf(h.begin(), h.end());
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  QC_HIP(hipMemcpyAsync(taps, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice, s),
         "hipMemcpyAsync(taps)");
  QC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  return QC_OK;
}

qc_status qc_pfb_channelize_ex(const void* x, int32_t sample, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                               const qc_pfb_params* p, const void* hist, void* hist_out, qc_prec out_prec,
                               void* out, float* scale_out, void* stream) {
  g_err.clear();
  qc_status st = check_any_args(x, sample, ld_x, n_ant, n_samp, p, hist, hist_out);
  if (st != QC_OK) return st;
  if (out_prec < QC_F32 || out_prec > QC_FP8_E4M3) return fail(QC_EINVAL, "bad out_prec %d", (int)out_prec);
  if (n_samp > 0 && !out) return fail(QC_EINVAL, "out is NULL");
  if (out_prec != QC_F32 && !scale_out) return fail(QC_EINVAL, "scale_out is NULL for reduced precision");
  if (reinterpret_cast<uintptr_t>(out) % prec_pair_bytes(out_prec))
    return fail(QC_EINVAL, "out is misaligned for its precision");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  st = channelize_any_impl(x, sample, ld_x, n_ant, n_samp, p, hist, out_prec, out, scale_out, s);
  if (st != QC_OK) return st;
  return hist_copy_any(x, sample, ld_x, n_ant, n_samp, p, hist, hist_out, s);
}

qc_status qc_xcorrelate_ex(const void* x, int32_t sample, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                           const qc_pfb_params* p, const void* hist, void* hist_out, int64_t spec_per_dump,
                           qc_prec x_prec, float* vis, int32_t accumulate, int64_t* n_dumps_out,
                           void* stream) {
  g_err.clear();
  qc_status st = check_any_args(x, sample, ld_x, n_ant, n_samp, p, hist, hist_out);
  if (st != QC_OK) return st;
  if (sample == QC_SAMPLE_I8)
    return qc_xcorrelate(static_cast<const int8_t*>(x), ld_x, n_ant, n_samp, p,
                         static_cast<const int8_t*>(hist), static_cast<int8_t*>(hist_out), spec_per_dump,
                         x_prec, vis, accumulate, n_dumps_out, stream);
  if (spec_per_dump < 1) return fail(QC_EINVAL, "spec_per_dump must be >= 1");
  if (x_prec < QC_F32 || x_prec > QC_FP8_E4M3) return fail(QC_EINVAL, "bad x_prec %d", (int)x_prec);
  const int N = p->n_fft;
  const int n_chan = sample_complex(sample) ? N : N / 2;
  const int64_t n_dump = (n_samp / N) / spec_per_dump;
  if (n_dump > 0 && !vis) return fail(QC_EINVAL, "vis is NULL");
  if (reinterpret_cast<uintptr_t>(vis) & 7u) return fail(QC_EINVAL, "vis must be 8-byte aligned");
  if (x_prec != QC_F32 && (n_ant > 32 || n_chan % 32))
    return fail(QC_EUNSUPPORTED, "matrix-core X-engine needs n_ant <= 32 and n_chan %% 32 == 0");
  if (n_dumps_out) *n_dumps_out = n_dump;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (n_dump > 0 && x_prec == QC_F32 &&
      qc::fused_words_supported(sample, N, n_ant, p->n_taps, p->taps == nullptr)) {
    // real int16 words at a fused ring shape: F+X in one pass, as for int8
    Resolved r;
    st = resolve(static_cast<const int8_t*>(x), ld_x, n_ant, n_samp, p, static_cast<const int8_t*>(hist), &r);
    if (st != QC_OK) return st;
    r.args.n_samp = n_dump * spec_per_dump * N;
    const int64_t nb = (int64_t)n_ant * (n_ant + 1) / 2;
    // the 4-antenna int16 tile at N = 4096 is resident one workgroup per
    // CU: a single round of them (12-15 % faster than two rounds); the
    // default otherwise
    const int64_t width = (N == 4096 && n_ant == 4) ? qc::device_cu_count() : 0;
    const int64_t cpd = qc::fused_chunks_per_dump(N, n_ant, n_dump, spec_per_dump, width);
    AsyncBuf part;
    st = alloc_async(part, (size_t)(n_dump * cpd) * nb * n_chan * sizeof(float2), s);
    if (st != QC_OK) return st;
    {
      KTimer t(QC_KERNEL_FX_FUSED, s);
      QC_HIP(qc::launch_fused_words(r.args, sample, n_dump, spec_per_dump, cpd, (float2*)part.p, s),
             "fused F+X kernel");
    }
    KTimer t(QC_KERNEL_REDUCE, s);
    QC_HIP(qc::launch_reduce((const float2*)part.p, n_dump, cpd, nb * n_chan, 0.25f, accumulate,
                             reinterpret_cast<float2*>(vis), s),
           "reduce kernel");
  } else if (n_dump > 0) {
    // two passes: the F-engine of the full dumps' spectra to HBM, then the X-engine
    const int64_t ns = n_dump * spec_per_dump;
    AsyncBuf v, scale;
    st = alloc_async(v, (size_t)n_ant * ns * n_chan * prec_pair_bytes(x_prec), s);
    if (st != QC_OK) return st;
    st = alloc_async(scale, (size_t)n_ant * sizeof(float), s);
    if (st != QC_OK) return st;
    st = channelize_any_impl(x, sample, ld_x, n_ant, ns * N, p, hist, x_prec, v.p, (float*)scale.p, s);
    if (st != QC_OK) return st;
    st = qc_xcorrelate_chan(v.p, x_prec, (const float*)scale.p, n_ant, ns, n_chan, spec_per_dump, vis,
                            accumulate, stream);
    if (st != QC_OK) return st;
  }
  return hist_copy_any(x, sample, ld_x, n_ant, n_samp, p, hist, hist_out, s);
}

qc_status qc_xcorrelate_chan(const void* v, qc_prec prec, const float* scale, int32_t n_ant,
                             int64_t n_spec, int32_t n_chan, int64_t spec_per_dump, float* vis,
                             int32_t accumulate, void* stream) {
  g_err.clear();
  if (prec < QC_F32 || prec > QC_FP8_E4M3) return fail(QC_EINVAL, "bad prec %d", (int)prec);
  if (n_ant < 1 || n_ant > 4096) return fail(QC_EINVAL, "n_ant must be in [1, 4096]");
  if (n_chan < 1 || n_spec < 0 || spec_per_dump < 1) return fail(QC_EINVAL, "bad sizes");
  const int64_t n_dump = n_spec / spec_per_dump;
  if (n_dump == 0) return QC_OK;
  if (!v || !vis) return fail(QC_EINVAL, "v or vis is NULL");
  if (prec != QC_F32 && !scale) return fail(QC_EINVAL, "scale is NULL for reduced precision");
  if (reinterpret_cast<uintptr_t>(v) % prec_pair_bytes(prec)) return fail(QC_EINVAL, "v misaligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t nb = (int64_t)n_ant * (n_ant + 1) / 2;
  if (prec == QC_F32) {
    const int64_t ks = qc::xeng_f32_ksplit(n_ant, spec_per_dump, n_chan, n_dump);
    AsyncBuf part;
    qc_status st = alloc_async(part, (size_t)(n_dump * ks) * nb * n_chan * sizeof(float2), s);
    if (st != QC_OK) return st;
    {
      KTimer t(QC_KERNEL_XENG_F32, s);
      QC_HIP(qc::launch_xeng_f32((const float2*)v, n_ant, n_spec, n_chan, spec_per_dump, n_dump, ks,
                                 (float2*)part.p, s),
             "X-engine f32 kernel");
    }
    KTimer t(QC_KERNEL_REDUCE, s);
    QC_HIP(qc::launch_reduce((const float2*)part.p, n_dump, ks, nb * n_chan, 1.0f, accumulate,
                             reinterpret_cast<float2*>(vis), s, qc::xeng_f32_tile(n_ant, n_chan, v), nb),
           "reduce kernel");
    return QC_OK;
  }
  const int64_t ks = qc::xeng_mfma_ksplit((int)prec, n_ant, spec_per_dump, n_chan, n_dump);
  if (ks <= 0)
    return fail(QC_EUNSUPPORTED, "matrix-core X-engine needs n_ant <= 32 and n_chan %% 32 == 0");
  if (reinterpret_cast<uintptr_t>(v) & 15u) return fail(QC_EINVAL, "v must be 16-byte aligned");
  AsyncBuf part;
  qc_status st = alloc_async(part, (size_t)(n_dump * ks) * nb * n_chan * sizeof(float2), s);
  if (st != QC_OK) return st;
  {
    KTimer t(QC_KERNEL_XENG_MFMA, s);
    QC_HIP(qc::launch_xeng_mfma(v, (int)prec, scale, n_ant, n_spec, n_chan, spec_per_dump, n_dump, ks,
                                (float2*)part.p, s),
           "X-engine matrix-core kernel");
  }
  KTimer t(QC_KERNEL_REDUCE, s);
  QC_HIP(qc::launch_reduce((const float2*)part.p, n_dump, ks, nb * n_chan, 1.0f, accumulate,
                           reinterpret_cast<float2*>(vis), s, qc::XM_TILE, nb),
         "reduce kernel");
  return QC_OK;
}

qc_status qc_mad_flag(const float* vis, int64_t n_time, int64_t n_base, int32_t n_chan, float sigma,
                      int32_t population, uint8_t* mask, double* thresh_out, void* stream) {
  g_err.clear();
  if (population < 0 || population > 2) return fail(QC_EINVAL, "population must be 0, 1 or 2");
  if (n_time < 1 || n_base < 1 || n_chan < 1) return fail(QC_EINVAL, "sizes must be >= 1");
  if (!(sigma >= 0.0f) || !std::isfinite(sigma)) return fail(QC_EINVAL, "sigma must be finite and >= 0");
  if (!vis || !mask) return fail(QC_EINVAL, "vis or mask is NULL");
  if (reinterpret_cast<uintptr_t>(vis) & 7u) return fail(QC_EINVAL, "vis must be 8-byte aligned");
  const int64_t npop = population == 0 ? n_base : population == 1 ? n_base * n_chan : n_time * n_base;
  if (npop > 0x7fffffffLL) return fail(QC_EINVAL, "too many populations");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  AsyncBuf amp;
  const int64_t na = qc::mad_scratch_floats(n_time, n_base, n_chan, population);
  if (na > 0) {
    qc_status st = ensure_device();
    if (st != QC_OK) return st;
    if ((st = alloc_async(amp, sizeof(float) * (size_t)na, s)) != QC_OK) return st;
  }
  KTimer t(QC_KERNEL_MAD, s);
  QC_HIP(qc::launch_mad(reinterpret_cast<const float2*>(vis), n_time, n_base, n_chan, sigma, population,
                        mask, thresh_out, nullptr, (float*)amp.p, s),
         "MAD kernel");
  return QC_OK;
}

qc_status qc_apply_delay_phase(float* vis, int64_t n_time, int32_t n_ant, int32_t n_chan, double f0_hz,
                               double df_hz, const double* tau_s, const double* phi_rad, void* stream) {
  g_err.clear();
  if (n_ant < 1 || n_ant > 64) return fail(QC_EINVAL, "n_ant must be in [1, 64]");
  if (n_time < 0 || n_time > 65535 || n_chan < 1) return fail(QC_EINVAL, "bad n_time/n_chan");
  if (!tau_s || !phi_rad) return fail(QC_EINVAL, "tau_s or phi_rad is NULL");
  if (!std::isfinite(f0_hz) || !std::isfinite(df_hz)) return fail(QC_EINVAL, "f0/df must be finite");
  for (int a = 0; a < n_ant; ++a)
    if (!std::isfinite(tau_s[a]) || !std::isfinite(phi_rad[a]))
      return fail(QC_EINVAL, "tau/phi must be finite");
  if (n_time == 0) return QC_OK;
  if (!vis) return fail(QC_EINVAL, "vis is NULL");
  if (reinterpret_cast<uintptr_t>(vis) & 7u) return fail(QC_EINVAL, "vis must be 8-byte aligned");
  KTimer t(QC_KERNEL_APPLY, reinterpret_cast<hipStream_t>(stream));
  QC_HIP(qc::launch_apply(reinterpret_cast<float2*>(vis), n_time, n_ant, n_chan, f0_hz, df_hz, tau_s,
                          phi_rad, reinterpret_cast<hipStream_t>(stream)),
         "apply kernel");
  return QC_OK;
}

qc_status qc_solve_delay_phase(const float* vis, const uint8_t* mask, int64_t n_time, int32_t n_ant,
                               int32_t n_chan, double f0_hz, double df_hz, int32_t ref_ant,
                               int32_t chan_lo, int32_t chan_hi, int32_t lag_pad, double* tau_s,
                               double* phi_rad, void* stream) {
  g_err.clear();
  if (n_ant < 2 || n_ant > 64) return fail(QC_EINVAL, "n_ant must be in [2, 64]");
  if (n_chan < 4 || n_chan > 4096) return fail(QC_EINVAL, "n_chan must be in [4, 4096]");
  if (n_time < 1) return fail(QC_EINVAL, "n_time must be >= 1");
  if (chan_lo < 0 || chan_hi > n_chan || chan_hi - chan_lo < 2)
    return fail(QC_EINVAL, "need 0 <= chan_lo, chan_hi <= n_chan and at least two band channels");
  if (ref_ant < 0 || ref_ant >= n_ant) return fail(QC_EINVAL, "ref_ant out of range");
  if (lag_pad < 1 || lag_pad > 64) return fail(QC_EINVAL, "lag_pad must be in [1, 64]");
  if (!std::isfinite(f0_hz) || !std::isfinite(df_hz) || !(df_hz > 0.0))
    return fail(QC_EINVAL, "f0 must be finite and df positive");
  if (!vis || !tau_s || !phi_rad) return fail(QC_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(vis) & 7u) return fail(QC_EINVAL, "vis must be 8-byte aligned");
  // lag grid: smallest power of two >= lag_pad * n_chan, at most 8192, at least n_chan
  int n_lag = 1;
  while (n_lag < lag_pad * n_chan) n_lag *= 2;
  if (n_lag > 8192) n_lag = 8192;
  while (n_lag < n_chan) n_lag *= 2;
  if (n_lag < 16) n_lag = 16;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float2* tw = nullptr;
  qc_status st = get_twiddles(n_lag, &tw);
  if (st != QC_OK) return st;
  const int n_cross = n_ant * (n_ant - 1) / 2;
  AsyncBuf scratch;
  st = alloc_async(scratch, sizeof(double) * (2 * n_cross + 2 * n_ant), s);
  if (st != QC_OK) return st;
  double* tb = (double*)scratch.p;
  double* pb = tb + n_cross;
  double* ta = pb + n_cross;
  double* pa = ta + n_ant;
  QC_HIP(qc::launch_solve(reinterpret_cast<const float2*>(vis), mask, n_time, n_ant, n_chan, f0_hz, df_hz,
                          ref_ant, chan_lo, chan_hi, n_lag, tw, tb, pb, ta, pa, s),
         "solve kernels");
  QC_HIP(hipMemcpyAsync(tau_s, ta, sizeof(double) * n_ant, hipMemcpyDeviceToHost, s), "copy tau");
  QC_HIP(hipMemcpyAsync(phi_rad, pa, sizeof(double) * n_ant, hipMemcpyDeviceToHost, s), "copy phi");
  QC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  return QC_OK;
}

int32_t qc_fx_tile_count(int32_t n_fft, int32_t n_ant) { return qc::fused_tile_count(n_fft, n_ant); }

qc_status qc_fx_set_tile(int32_t n_fft, int32_t n_ant, int32_t tile) {
  g_err.clear();
  const int n = qc::fused_tile_count(n_fft, n_ant);
  if (n == 0) return fail(QC_EUNSUPPORTED, "no fused kernel for n_fft=%d n_ant=%d", n_fft, n_ant);
  if (tile < 0 || tile >= n) return fail(QC_EINVAL, "tile %d out of range [0, %d)", tile, n);
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tile[{n_fft, n_ant}] = tile;
  return QC_OK;
}

int32_t qc_fx_get_tile(int32_t n_fft, int32_t n_ant) { return fused_tile_for(n_fft, n_ant); }

qc_status qc_fx_set_width(int32_t n_fft, int32_t n_ant, int64_t workgroups) {
  g_err.clear();
  if (qc::fused_tile_count(n_fft, n_ant) == 0)
    return fail(QC_EUNSUPPORTED, "no fused kernel for n_fft=%d n_ant=%d", n_fft, n_ant);
  if (workgroups < 0 || workgroups > (1 << 20)) return fail(QC_EINVAL, "workgroups must be in [0, 2^20]");
  std::lock_guard<std::mutex> lk(g_tile_mu);
  if (workgroups == 0)
    g_width.erase({n_fft, n_ant});
  else
    g_width[{n_fft, n_ant}] = workgroups;
  return QC_OK;
}

int64_t qc_fx_get_width(int32_t n_fft, int32_t n_ant) { return fused_width_for(n_fft, n_ant); }

qc_status qc_fx_autotune(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                         const qc_pfb_params* p, int64_t spec_per_dump, int32_t reps, float* vis,
                         double* ms_per_tile, int32_t cap, int32_t* best_out, void* stream) {
  g_err.clear();
  qc_status st = check_stream_args(x, ld_x, n_ant, n_samp, p, nullptr, nullptr);
  if (st != QC_OK) return st;
  const int n = qc::fused_tile_count(p->n_fft, n_ant);
  if (n == 0) return fail(QC_EUNSUPPORTED, "no fused kernel for n_fft=%d n_ant=%d", p->n_fft, n_ant);
  if (reps < 1 || spec_per_dump < 1 || n_samp / p->n_fft < spec_per_dump)
    return fail(QC_EINVAL, "need reps >= 1 and at least one full dump");
  if (!vis) return fail(QC_EINVAL, "vis is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int dev = 0, n_cu = 0;
  QC_HIP(hipGetDevice(&dev), "hipGetDevice");
  QC_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
  if (n_cu < 1) n_cu = 256;
  hipEvent_t a = nullptr, b = nullptr;
  QC_HIP(hipEventCreate(&a), "hipEventCreate");
  QC_HIP(hipEventCreate(&b), "hipEventCreate");
  const std::pair<int, int> key{p->n_fft, n_ant};
  const int prev = fused_tile_for(p->n_fft, n_ant);
  const int64_t prev_w = fused_width_for(p->n_fft, n_ant);
  // one untimed call (first-use set-up), then reps timed calls
  auto time_calls = [&](double* per) -> qc_status {
    qc_status q = qc_xcorrelate(x, ld_x, n_ant, n_samp, p, nullptr, nullptr, spec_per_dump, QC_F32, vis, 0,
                                nullptr, stream);
    if (q != QC_OK) return q;
    QC_HIP(hipEventRecord(a, s), "hipEventRecord");
    for (int r = 0; r < reps; ++r) {
      q = qc_xcorrelate(x, ld_x, n_ant, n_samp, p, nullptr, nullptr, spec_per_dump, QC_F32, vis, 0, nullptr,
                        stream);
      if (q != QC_OK) return q;
    }
    QC_HIP(hipEventRecord(b, s), "hipEventRecord");
    QC_HIP(hipEventSynchronize(b), "hipEventSynchronize");
    float ms = 0.f;
    QC_HIP(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
    *per = (double)ms / reps;
    return QC_OK;
  };
  auto set_choice = [&](int t, int64_t w) {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_tile[key] = t;
    if (w > 0)
      g_width[key] = w;
    else
      g_width.erase(key);
  };
  // tiles at the default width (512 workgroups), then the best tile at one
  // and at four workgroups per CU (a tile that holds one workgroup per CU
  // fills the chip in a single round at the first)
  double best = 1e300;
  int best_t = 0;
  int64_t best_w = 0;
  for (int t = 0; t < n && st == QC_OK; ++t) {
    set_choice(t, 0);
    double per = 0.0;
    st = time_calls(&per);
    if (st != QC_OK) break;
    if (ms_per_tile && t < cap) ms_per_tile[t] = per;
    if (per < best) {
      best = per;
      best_t = t;
    }
  }
  for (int64_t w : {(int64_t)n_cu, 4 * (int64_t)n_cu}) {
    if (st != QC_OK) break;
    set_choice(best_t, w);
    double per = 0.0;
    st = time_calls(&per);
    if (st == QC_OK && per < best) {
      best = per;
      best_w = w;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != QC_OK) {
    set_choice(prev, prev_w);
    return st;
  }
  set_choice(best_t, best_w);
  if (best_out) *best_out = best_t;
  return QC_OK;
}

qc_status qc_timing_enable(int32_t on) {
  g_err.clear();
  if (on < 0 || on > 2) return fail(QC_EINVAL, "timing mode %d (0 off, 1 event pairs, 2 chained)", on);
  std::lock_guard<std::mutex> lk(g_tmu);
  if (on) timing_clear_locked();
  g_timing = on;
  return QC_OK;
}

qc_status qc_timing_read(int32_t kernel, double* total_ms, int64_t* launches) {
  g_err.clear();
  if (kernel < 0 || kernel >= QC_KERNEL_COUNT) return fail(QC_EINVAL, "bad kernel id %d", kernel);
  if (!total_ms || !launches) return fail(QC_EINVAL, "NULL output");
  std::lock_guard<std::mutex> lk(g_tmu);
  double tot = 0.0;
  for (auto& p : g_trec.ev[kernel]) {
    QC_HIP(hipEventSynchronize(p.second), "hipEventSynchronize");
    float ms = 0.f;
    QC_HIP(hipEventElapsedTime(&ms, p.first, p.second), "hipEventElapsedTime");
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)g_trec.ev[kernel].size();
  return QC_OK;
}

}  // extern "C"

// ---- batched plans ------------------------------------------------------------
// Two implementations of one contract.  The default (QC_PLAN_GRAPH) records,
// per array, the same kernels qc_xcorrelate launches (fused F+X and reduction,
// or F-engine, FP32 X-engine and reduction) into plan-owned buffers, each
// array on a stream of its own between a fork and a join event, so that one
// captured graph holds every array as an independent branch.  The second
// (QC_PLAN_PERSISTENT: one persistent launch claiming work items from a
// queue, with bounded waits between dependent items) does every array's
// work in one launch.
namespace {
constexpr int PLAN_SLOTS = 16;  // descriptor slots for executions in flight (+1 for a graph)

struct PlanArr {
  bool fused = false;
  int tile = 0;           // fused kernel tile (index into the (n_fft, n_ant) tile list)
  int64_t split = 1;      // fused: chunks per dump; two-pass: X-engine k-split
  int64_t split_max = 1;  // capacity of the partial buffer, splits per dump
  int64_t n_dump = 0;
  const float* taps = nullptr;
  float2* tw = nullptr;
  float2* twp = nullptr;  // per-pass twiddles (ping-pong tiles)
  float2* part = nullptr;
  float2* chan = nullptr;
};
}  // namespace

struct qc_plan {
  int device = 0;
  int n = 0;
  int mode = QC_PLAN_GRAPH;
  qc_array_desc desc[qc::PL_MAX_ARRAYS];
  // graph mode
  PlanArr ga[qc::PL_MAX_ARRAYS];
  int concurrent = 1;  // arrays on streams of their own (1) or in order on the caller's stream (0)
  hipStream_t st[qc::PL_MAX_ARRAYS] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[qc::PL_MAX_ARRAYS] = {};
  std::vector<void*> gbufs;
  // persistent mode
  qc::PlArray arr[qc::PL_MAX_ARRAYS];
  int64_t fused_items = 128;  // target fused items per array (each at least 32 spectra)
  int64_t chan_mult = 4;      // F-engine item = spectra-in-flight * chan_mult spectra
  int64_t x_split = 2;        // X-engine k-split
  int grid = 256;             // persistent blocks
  int64_t wait_us = 2000000;  // time limit of one dependency wait
  int64_t clock_khz = 0;      // device wall-clock rate
  int wait_bias = 0;
  std::vector<qc::PlItem> items;
  qc::PlItem* d_items = nullptr;
  unsigned* d_ctr = nullptr;
  qc::PlArray* d_slots = nullptr;  // (PLAN_SLOTS + 1) * PL_MAX_ARRAYS
  qc::PlArray* h_slots = nullptr;  // pinned staging, same shape
  hipEvent_t slot_ev[PLAN_SLOTS] = {};
  bool slot_used[PLAN_SLOTS] = {};
  int next_slot = 0;
  std::vector<void*> bufs;
  // the captured graph (either mode)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

namespace {

void persist_free(qc_plan* P) {
  if (!P->bufs.empty() || P->d_items) (void)hipDeviceSynchronize();
  for (void* b : P->bufs) (void)hipFree(b);
  P->bufs.clear();
  if (P->d_items) (void)hipFree(P->d_items);
  P->d_items = nullptr;
}

void plan_drop_graph(qc_plan* P) {
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  P->gexec = nullptr;
  P->graph = nullptr;
}

qc_status persist_build(qc_plan* P) {
  // a captured graph refers to the buffers and items rebuilt here
  plan_drop_graph(P);
  persist_free(P);
  std::vector<qc::PlItem> first, xeng, red;
  for (int i = 0; i < P->n; ++i) {
    const qc_array_desc& D = P->desc[i];
    qc::PlArray& A = P->arr[i];
    A = qc::PlArray{};
    const int N = D.n_fft, NA = D.n_ant, NCH = N / 2;
    const int64_t NB = (int64_t)NA * (NA + 1) / 2;
    A.n_samp = D.n_samp;
    A.spd = D.spec_per_dump;
    A.n_dump = (D.n_samp / N) / D.spec_per_dump;
    A.n_ant = NA;
    A.n_fft = N;
    A.n_taps = D.n_taps;
    TapsEntry te;
    qc_status st = get_taps(N, D.n_taps, &te);
    if (st != QC_OK) return st;
    float2* tw = nullptr;
    st = get_twiddles(N, &tw);
    if (st != QC_OK) return st;
    A.taps = te.dev;
    A.tw = tw;
    const int64_t elems = NB * NCH;
    void* part = nullptr;
    if (qc::plan_fused_supported(N, NA)) {
      A.mode = 0;
      const int S = 8192 / (((NA + 1) / 2) * N);
      // items of at least 32 spectra: each writes a whole partial tile
      // (baselines x channels), which must stay small beside its input
      int64_t cpd = (P->fused_items + A.n_dump - 1) / A.n_dump;
      const int64_t per = std::max<int64_t>(S, 32);
      cpd = std::max<int64_t>(1, std::min<int64_t>(cpd, A.spd / per > 0 ? A.spd / per : 1));
      A.n_split = cpd;
      A.n_part_items = (int32_t)(A.n_dump * cpd);
      A.scale = 0.25f;
      for (int64_t w = 0; w < A.n_dump * cpd; ++w) first.push_back({qc::PL_FUSED, (uint16_t)i, (uint32_t)w});
    } else {
      A.mode = 1;
      const int64_t ns = A.n_dump * A.spd;
      // F-engine items: the ring body (groups of 8 antennas at N = 2048, 4
      // at 4096, 2 at 8192: 512 threads each; the built-in P = 4 prototype)
      // or the plain body
      const bool ring = (N == 2048 || N == 4096 || N == 8192) && D.n_taps == 4;
      if (ring) {
        const int na_g = N == 8192 ? 2 : N == 4096 ? 4 : 8;
        const int64_t groups = (NA + na_g - 1) / na_g;
        int64_t spb = (ns * groups + 511) / 512;  // about 512 items, runs of >= 16 spectra
        spb = std::max<int64_t>(16, spb);
        A.spb = spb;
        A.n_chunks = (int32_t)((ns + spb - 1) / spb);
        A.n_chan_items = (int32_t)(groups * A.n_chunks);
      } else {
        const int S = 8192 / N;
        A.spec_per_item = std::min<int64_t>(ns, (int64_t)S * P->chan_mult);
        const int64_t nbx = (ns + A.spec_per_item - 1) / A.spec_per_item;
        A.n_chan_items = (int32_t)(nbx * ((NA + 1) / 2));
      }
      // X-engine items: matrix cores for 5..32 antennas (16 x 16 tiles up to
      // 16), the vector ALU otherwise
      if (NA >= 5 && NA <= 32 && NCH % 16 == 0) {
        A.x_kind = NA <= 16 ? 2 : 1;
        A.n_cb = NCH / 16;
        A.tile = 16;
        A.n_split = std::max<int64_t>(1, qc::xeng_f32_mfma_ksplit(NA, A.spd, NCH, A.n_dump));
        A.n_part_items = (int32_t)(A.n_dump * A.n_split * A.n_cb);
      } else {
        const int64_t ks = std::max<int64_t>(1, std::min<int64_t>(P->x_split, A.spd / 16 > 0 ? A.spd / 16 : 1));
        A.n_split = ks;
        A.n_cgrp = (NCH + qc::PL_NT - 1) / qc::PL_NT;
        const int nblk = (NA + 3) / 4;
        A.n_bp = nblk * (nblk + 1) / 2;
        A.n_part_items = (int32_t)(A.n_dump * ks * A.n_bp * A.n_cgrp);
      }
      A.scale = 1.0f;
      void* chan = nullptr;
      hipError_t e = hipMalloc(&chan, sizeof(float2) * (size_t)NA * ns * NCH);
      if (e != hipSuccess) return fail(QC_ENOMEM, "plan spectra buffer: %s", hipGetErrorString(e));
      P->bufs.push_back(chan);
      A.chan = (float2*)chan;
      const uint16_t fk = A.n_chunks > 0 ? qc::PL_CHAN_RING : qc::PL_CHAN;
      const uint16_t xk = A.x_kind > 0 ? qc::PL_XMFMA : qc::PL_XENG;
      for (int64_t q = 0; q < A.n_chan_items; ++q) first.push_back({fk, (uint16_t)i, (uint32_t)q});
      for (int64_t q = 0; q < A.n_part_items; ++q) xeng.push_back({xk, (uint16_t)i, (uint32_t)q});
    }
    hipError_t e = hipMalloc(&part, sizeof(float2) * (size_t)A.n_dump * A.n_split * elems);
    if (e != hipSuccess) return fail(QC_ENOMEM, "plan partial buffer: %s", hipGetErrorString(e));
    P->bufs.push_back(part);
    A.part = (float2*)part;
    // reduction items of about PL_RED_LOADS partial loads each: many
    // visibilities where there are few partials, few where there are many
    int64_t rb = qc::PL_RED_LOADS / std::max<int64_t>(1, A.n_split);
    rb = std::max<int64_t>(qc::PL_NT, std::min<int64_t>(rb, 64 * qc::PL_NT));
    rb = (rb / qc::PL_NT) * qc::PL_NT;
    A.red_block = (int32_t)rb;
    A.n_red_blocks = (int32_t)((elems + rb - 1) / rb);
    for (int64_t q = 0; q < A.n_dump * A.n_red_blocks; ++q) red.push_back({qc::PL_REDUCE, (uint16_t)i, (uint32_t)q});
  }
  // spectra items of the two-pass arrays first (they feed the longest
  // chains), the largest arrays' first, then the X-engine items array by
  // array in the same order (the longest items first, the shortest at the
  // end); an array's reduction items follow the next array's X items (by
  // then its partials are normally done, so they neither wait nor pile up
  // at the end)
  auto size_of = [&](int i) { return (int64_t)P->desc[i].n_ant * P->desc[i].n_samp; };
  std::stable_sort(first.begin(), first.end(), [&](const qc::PlItem& a, const qc::PlItem& b) {
    if (a.kind != b.kind) return a.kind > b.kind;
    return size_of(a.array) > size_of(b.array);
  });
  std::stable_sort(xeng.begin(), xeng.end(), [&](const qc::PlItem& a, const qc::PlItem& b) {
    return size_of(a.array) > size_of(b.array);
  });
  P->items = first;
  std::vector<int> x_order;  // arrays with X items, in queue order
  for (const qc::PlItem& it : xeng)
    if (x_order.empty() || x_order.back() != it.array) x_order.push_back(it.array);
  auto put_red = [&](int arr) {
    for (const qc::PlItem& it : red)
      if (it.array == arr) P->items.push_back(it);
  };
  std::vector<bool> red_done(P->n, false);
  for (size_t j = 0; j < x_order.size(); ++j) {
    for (const qc::PlItem& it : xeng)
      if (it.array == x_order[j]) P->items.push_back(it);
    if (j == 0) {
      // the fused arrays' partials come from the first items of the queue
      for (int i = 0; i < P->n; ++i)
        if (P->arr[i].mode == 0) {
          put_red(i);
          red_done[i] = true;
        }
    } else {
      put_red(x_order[j - 1]);
      red_done[x_order[j - 1]] = true;
    }
  }
  for (int i = 0; i < P->n; ++i)
    if (!red_done[i]) put_red(i);
  if (P->items.size() >= 0x7fffffffu) return fail(QC_EUNSUPPORTED, "too many plan items");
  // the persistent kernel relies on these: per array, the counted items
  // match the wait targets, and every item precedes the items that wait on it
  for (int i = 0; i < P->n; ++i) {
    int64_t n_chan = 0, n_part = 0, last_chan = -1, last_part = -1;
    int64_t first_x = INT64_MAX, first_red = INT64_MAX;
    for (size_t q = 0; q < P->items.size(); ++q) {
      const qc::PlItem& it = P->items[q];
      if (it.array != i) continue;
      const int64_t pos = (int64_t)q;
      const bool chan = it.kind == qc::PL_CHAN || it.kind == qc::PL_CHAN_RING;
      const bool xk = it.kind == qc::PL_XENG || it.kind == qc::PL_XMFMA;
      if (chan) { ++n_chan; last_chan = pos; }
      if (it.kind == qc::PL_FUSED || xk) { ++n_part; last_part = pos; }
      if (xk) first_x = std::min(first_x, pos);
      if (it.kind == qc::PL_REDUCE) first_red = std::min(first_red, pos);
    }
    const qc::PlArray& A = P->arr[i];
    if (n_chan != A.n_chan_items || n_part != A.n_part_items || last_chan >= first_x ||
        last_part >= first_red)
      return fail(QC_ESTATE, "internal: plan item order for array %d", i);
  }
  hipError_t e = hipMalloc(&P->d_items, sizeof(qc::PlItem) * P->items.size());
  if (e != hipSuccess) return fail(QC_ENOMEM, "plan items: %s", hipGetErrorString(e));
  e = hipMemcpy(P->d_items, P->items.data(), sizeof(qc::PlItem) * P->items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "plan items upload");
  return QC_OK;
}

qc_status persist_enqueue(qc_plan* P, const int8_t* const* x, float* const* vis, hipStream_t s, int slot) {
  qc::PlArray* h = P->h_slots + (size_t)slot * qc::PL_MAX_ARRAYS;
  qc::PlArray* d = P->d_slots + (size_t)slot * qc::PL_MAX_ARRAYS;
  for (int i = 0; i < P->n; ++i) {
    h[i] = P->arr[i];
    h[i].x = x[i];
    h[i].vis = reinterpret_cast<float2*>(vis[i]);
  }
  QC_HIP(hipMemcpyAsync(d, h, sizeof(qc::PlArray) * P->n, hipMemcpyHostToDevice, s), "plan descriptors");
  qc::PlArgs a{};
  a.arr = d;
  a.items = P->d_items;
  a.n_items = (int32_t)P->items.size();
  a.wait_ticks = P->wait_us * P->clock_khz / 1000;
  a.wait_bias = P->wait_bias;
  a.ctr = P->d_ctr;
  QC_HIP(qc::launch_plan(a, P->grid, s), "plan kernel");
  return QC_OK;
}

qc_status persist_setup(qc_plan* P) {
  hipError_t e = hipSuccess;
  int khz = 0;
  e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, P->device);
  P->clock_khz = khz > 0 ? khz : 100000;
  if (e == hipSuccess) e = hipMalloc(&P->d_ctr, sizeof(unsigned) * (2 + 2 * qc::PL_MAX_ARRAYS));
  if (e == hipSuccess)
    e = hipMalloc(&P->d_slots, sizeof(qc::PlArray) * (PLAN_SLOTS + 1) * qc::PL_MAX_ARRAYS);
  if (e == hipSuccess)
    e = hipHostMalloc(&P->h_slots, sizeof(qc::PlArray) * (PLAN_SLOTS + 1) * qc::PL_MAX_ARRAYS, 0);
  for (int i = 0; e == hipSuccess && i < PLAN_SLOTS; ++i)
    e = hipEventCreateWithFlags(&P->slot_ev[i], hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "plan allocation");
  return persist_build(P);
}

qc_status persist_execute(qc_plan* P, const int8_t* const* x, float* const* vis, hipStream_t s) {
  const int slot = P->next_slot;
  P->next_slot = (P->next_slot + 1) % PLAN_SLOTS;
  // the slot's staging may still be read by an earlier execution's copy
  if (P->slot_used[slot]) QC_HIP(hipEventSynchronize(P->slot_ev[slot]), "plan slot wait");
  QC_HIP(qc::prepare_plan(), "plan kernel attributes");
  qc_status st = persist_enqueue(P, x, vis, s, slot);
  if (st != QC_OK) return st;
  QC_HIP(hipEventRecord(P->slot_ev[slot], s), "plan slot event");
  P->slot_used[slot] = true;
  return QC_OK;
}

// ---- graph mode ----

void graph_free(qc_plan* P) {
  if (!P->gbufs.empty()) (void)hipDeviceSynchronize();
  for (void* b : P->gbufs) (void)hipFree(b);
  P->gbufs.clear();
}

qc_status graph_setup(qc_plan* P) {
  for (int i = 0; i < P->n; ++i) {
    const qc_array_desc& D = P->desc[i];
    PlanArr& G = P->ga[i];
    const int N = D.n_fft, NA = D.n_ant, nch = N / 2;
    const int64_t nb = (int64_t)NA * (NA + 1) / 2, elems = nb * nch;
    G.n_dump = (D.n_samp / N) / D.spec_per_dump;
    TapsEntry te;
    qc_status st = get_taps(N, D.n_taps, &te);
    if (st != QC_OK) return st;
    G.taps = te.dev;
    st = get_twiddles(N, &G.tw);
    if (st != QC_OK) return st;
    st = get_pass_twiddles(N, &G.twp);
    if (st != QC_OK) return st;
    G.fused = qc::fused_supported(N, NA);
    if (G.fused) {
      G.tile = 0;
      G.split = qc::fused_chunks_per_dump(N, NA, G.n_dump, D.spec_per_dump);
      G.split_max = std::min<int64_t>(D.spec_per_dump, 2 * G.split);
    } else {
      G.split = qc::xeng_f32_ksplit(NA, D.spec_per_dump, nch, G.n_dump);
      G.split_max = std::min<int64_t>(D.spec_per_dump, std::max<int64_t>(16, G.split));
      void* chan = nullptr;
      const size_t bytes = sizeof(float2) * (size_t)NA * G.n_dump * D.spec_per_dump * nch;
      hipError_t e = hipMalloc(&chan, bytes);
      if (e != hipSuccess) return fail(QC_ENOMEM, "plan spectra buffer: %s", hipGetErrorString(e));
      P->gbufs.push_back(chan);
      G.chan = (float2*)chan;
    }
    void* part = nullptr;
    hipError_t e = hipMalloc(&part, sizeof(float2) * (size_t)(G.n_dump * G.split_max) * elems);
    if (e != hipSuccess) return fail(QC_ENOMEM, "plan partial buffer: %s", hipGetErrorString(e));
    P->gbufs.push_back(part);
    G.part = (float2*)part;
    QC_HIP(hipStreamCreateWithFlags(&P->st[i], hipStreamNonBlocking), "hipStreamCreateWithFlags");
    QC_HIP(hipEventCreateWithFlags(&P->join_ev[i], hipEventDisableTiming), "hipEventCreate");
  }
  QC_HIP(hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming), "hipEventCreate");
  return QC_OK;
}

// one array's kernels on stream s
qc_status graph_array(qc_plan* P, int i, const int8_t* x, float* vis, hipStream_t s) {
  const qc_array_desc& D = P->desc[i];
  const PlanArr& G = P->ga[i];
  const int N = D.n_fft, NA = D.n_ant, nch = N / 2;
  const int64_t nb = (int64_t)NA * (NA + 1) / 2, elems = nb * nch;
  const int64_t ns = G.n_dump * D.spec_per_dump;
  const qc::FxArgs a{x, D.n_samp, NA, ns * N, N, D.n_taps, G.taps, G.tw, nullptr, true, G.twp};
  float2* v = reinterpret_cast<float2*>(vis);
  if (G.fused) {
    QC_HIP(qc::launch_fused(a, G.n_dump, D.spec_per_dump, G.split, G.part, s, G.tile), "fused F+X kernel");
    QC_HIP(qc::launch_reduce(G.part, G.n_dump, G.split, elems, 0.25f, 0, v, s), "reduce kernel");
  } else {
    QC_HIP(qc::launch_channelize(a, 0, G.chan, nullptr, s), "channelize kernel");
    QC_HIP(qc::launch_xeng_f32(G.chan, NA, ns, nch, D.spec_per_dump, G.n_dump, G.split, G.part, s),
           "X-engine f32 kernel");
    QC_HIP(qc::launch_reduce(G.part, G.n_dump, G.split, elems, 1.0f, 0, v, s,
                             qc::xeng_f32_tile(NA, nch, G.chan), nb),
           "reduce kernel");
  }
  return QC_OK;
}

qc_status graph_execute(qc_plan* P, const int8_t* const* x, float* const* vis, hipStream_t s) {
  const bool fork = P->concurrent && P->n > 1;
  if (fork) QC_HIP(hipEventRecord(P->fork_ev, s), "hipEventRecord(fork)");
  for (int i = 0; i < P->n; ++i) {
    hipStream_t si = fork ? P->st[i] : s;
    if (fork) QC_HIP(hipStreamWaitEvent(si, P->fork_ev, 0), "hipStreamWaitEvent(fork)");
    qc_status st = graph_array(P, i, x[i], vis[i], si);
    if (st != QC_OK) return st;
    if (fork) {
      QC_HIP(hipEventRecord(P->join_ev[i], si), "hipEventRecord(join)");
      QC_HIP(hipStreamWaitEvent(s, P->join_ev[i], 0), "hipStreamWaitEvent(join)");
    }
  }
  return QC_OK;
}

int graph_launches(const qc_plan* P) {
  int k = 0;
  for (int i = 0; i < P->n; ++i) k += P->ga[i].fused ? 2 : 3;
  return k;
}

qc_status plan_check_args(qc_plan* P, const int8_t* const* x, float* const* vis) {
  if (!P || !x || !vis) return fail(QC_EINVAL, "NULL argument");
  for (int i = 0; i < P->n; ++i) {
    if (!x[i] || !vis[i]) return fail(QC_EINVAL, "array %d: NULL x or vis", i);
    if ((reinterpret_cast<uintptr_t>(x[i]) & 3u) || (reinterpret_cast<uintptr_t>(vis[i]) & 7u))
      return fail(QC_EINVAL, "array %d: misaligned x or vis", i);
  }
  return QC_OK;
}

qc_status plan_run(qc_plan* P, const int8_t* const* x, float* const* vis, hipStream_t s) {
  return P->mode == QC_PLAN_GRAPH ? graph_execute(P, x, vis, s) : persist_execute(P, x, vis, s);
}

std::string plan_signature(const qc_plan* P) {
  std::ostringstream o;
  for (int i = 0; i < P->n; ++i)
    o << P->desc[i].n_ant << "x" << P->desc[i].n_samp << "x" << P->desc[i].n_fft << "x"
      << P->desc[i].n_taps << "x" << P->desc[i].spec_per_dump << (i + 1 < P->n ? "," : "");
  return o.str();
}

// timed executions (eager, on s) with the plan's current knobs
qc_status plan_time(qc_plan* P, const int8_t* const* x, float* const* vis, int reps, hipStream_t s,
                    hipEvent_t a, hipEvent_t b, double* ms_out) {
  qc_status q = plan_run(P, x, vis, s);  // untimed
  if (q != QC_OK) return q;
  QC_HIP(hipEventRecord(a, s), "hipEventRecord");
  for (int r = 0; r < reps && q == QC_OK; ++r) q = plan_run(P, x, vis, s);
  if (q != QC_OK) return q;
  QC_HIP(hipEventRecord(b, s), "hipEventRecord");
  QC_HIP(hipEventSynchronize(b), "hipEventSynchronize");
  float ms = 0.f;
  QC_HIP(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
  *ms_out = ms / reps;
  return QC_OK;
}

// Coordinate descent over the graph-mode knobs: concurrency, then per
// array the fused tile and the split (chunks per dump, or X-engine k-split).
qc_status graph_tune(qc_plan* P, const int8_t* const* x, float* const* vis, int reps, hipStream_t s,
                     hipEvent_t a, hipEvent_t b) {
  double best = 0.0;
  qc_status st = plan_time(P, x, vis, reps, s, a, b, &best);
  auto try_value = [&](auto set, auto get, const std::vector<int64_t>& cand) -> qc_status {
    const int64_t keep = get();
    int64_t bestv = keep;
    for (int64_t v : cand) {
      if (v == keep) continue;
      set(v);
      double ms = 0.0;
      qc_status q = plan_time(P, x, vis, reps, s, a, b, &ms);
      if (q != QC_OK) {
        set(keep);
        return q;
      }
      if (ms < best) {
        best = ms;
        bestv = v;
      }
    }
    set(bestv);
    return QC_OK;
  };
  for (int pass = 0; st == QC_OK && pass < 2; ++pass) {
    st = try_value([&](int64_t v) { P->concurrent = (int)v; }, [&] { return (int64_t)P->concurrent; },
                   {0, 1});
    for (int i = 0; st == QC_OK && i < P->n; ++i) {
      PlanArr& G = P->ga[i];
      const qc_array_desc& D = P->desc[i];
      if (G.fused) {
        std::vector<int64_t> tiles;
        for (int t = 0; t < qc::fused_tile_count(D.n_fft, D.n_ant); ++t) tiles.push_back(t);
        st = try_value([&](int64_t v) { G.tile = (int)v; }, [&] { return (int64_t)G.tile; }, tiles);
        if (st != QC_OK) break;
      }
      std::vector<int64_t> splits;
      for (int64_t v : {1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024})
        if (v <= G.split_max) splits.push_back(v);
      st = try_value([&](int64_t v) { G.split = v; }, [&] { return G.split; }, splits);
    }
  }
  return st;
}

std::string graph_knobs(const qc_plan* P) {
  std::ostringstream o;
  o << P->concurrent;
  for (int i = 0; i < P->n; ++i) o << " " << (P->ga[i].fused ? P->ga[i].tile : -1) << " " << P->ga[i].split;
  return o.str();
}

bool graph_knobs_parse(qc_plan* P, std::istringstream& ls) {
  int conc = 0;
  if (!(ls >> conc) || (conc != 0 && conc != 1)) return false;
  int tile[qc::PL_MAX_ARRAYS];
  int64_t split[qc::PL_MAX_ARRAYS];
  for (int i = 0; i < P->n; ++i) {
    if (!(ls >> tile[i] >> split[i])) return false;
    const PlanArr& G = P->ga[i];
    const qc_array_desc& D = P->desc[i];
    if (split[i] < 1 || split[i] > G.split_max) return false;
    if (G.fused && (tile[i] < 0 || tile[i] >= qc::fused_tile_count(D.n_fft, D.n_ant))) return false;
  }
  P->concurrent = conc;
  for (int i = 0; i < P->n; ++i) {
    if (P->ga[i].fused) P->ga[i].tile = tile[i];
    P->ga[i].split = split[i];
  }
  return true;
}

}  // namespace

extern "C" {

qc_status qc_plan_create(const qc_array_desc* arrays, int32_t n_arrays, qc_plan** out) {
  g_err.clear();
  if (!arrays || !out) return fail(QC_EINVAL, "NULL argument");
  *out = nullptr;
  if (n_arrays < 1 || n_arrays > qc::PL_MAX_ARRAYS)
    return fail(QC_EINVAL, "n_arrays must be in [1, %d]", qc::PL_MAX_ARRAYS);
  for (int i = 0; i < n_arrays; ++i) {
    const qc_array_desc& D = arrays[i];
    if (D.n_ant < 1 || D.n_ant > 64) return fail(QC_EINVAL, "array %d: n_ant must be in [1, 64]", i);
    if (!is_pow2(D.n_fft) || D.n_fft < 16 || D.n_fft > 8192)
      return fail(QC_EINVAL, "array %d: n_fft must be a power of two in [16, 8192]", i);
    if (D.n_taps < 1 || D.n_taps > 16) return fail(QC_EINVAL, "array %d: n_taps must be in [1, 16]", i);
    if (D.n_samp <= 0 || D.n_samp % D.n_fft || D.n_samp > 0x7fffffffLL)
      return fail(QC_EINVAL, "array %d: n_samp must be a positive multiple of n_fft below 2^31", i);
    if (D.spec_per_dump < 1 || (D.n_samp / D.n_fft) < D.spec_per_dump)
      return fail(QC_EINVAL, "array %d: need at least one full dump", i);
  }
  qc_plan* P = new (std::nothrow) qc_plan();
  if (!P) return fail(QC_ENOMEM, "host allocation");
  P->n = n_arrays;
  for (int i = 0; i < n_arrays; ++i) P->desc[i] = arrays[i];
  hipError_t e = hipGetDevice(&P->device);
  if (e != hipSuccess) {
    delete P;
    return hip_fail(e, "hipGetDevice");
  }
  qc_status st = graph_setup(P);
  if (st != QC_OK) {
    qc_plan_destroy(P);
    return st;
  }
  *out = P;
  return QC_OK;
}

qc_status qc_plan_set_mode(qc_plan* P, int32_t mode) {
  g_err.clear();
  if (!P) return fail(QC_EINVAL, "NULL plan");
  if (mode == QC_PLAN_GRAPH) {
    if (P->mode != mode) plan_drop_graph(P);
    P->mode = mode;
    return QC_OK;
  }
  if (mode != QC_PLAN_PERSISTENT) return fail(QC_EINVAL, "unknown plan mode %d", mode);
  if (P->mode != mode) {
    plan_drop_graph(P);
    qc_status st = P->d_ctr ? persist_build(P) : persist_setup(P);
    if (st != QC_OK) return st;
  }
  P->mode = mode;
  return QC_OK;
}

qc_status qc_plan_execute(qc_plan* P, const int8_t* const* x, float* const* vis, void* stream) {
  g_err.clear();
  qc_status st = plan_check_args(P, x, vis);
  if (st != QC_OK) return st;
  return plan_run(P, x, vis, reinterpret_cast<hipStream_t>(stream));
}

qc_status qc_plan_check(qc_plan* P, void* stream) {
  g_err.clear();
  if (!P) return fail(QC_EINVAL, "NULL plan");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  QC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (P->mode != QC_PLAN_PERSISTENT) return QC_OK;
  unsigned flag = 0;
  QC_HIP(hipMemcpy(&flag, P->d_ctr + 1, sizeof(unsigned), hipMemcpyDeviceToHost), "plan flag");
  if (flag) return fail(QC_ESTATE, "a bounded dependency wait expired in the last plan execution");
  return QC_OK;
}

qc_status qc_plan_set_wait_timeout(qc_plan* P, int64_t microseconds) {
  g_err.clear();
  if (!P || microseconds < 1 || microseconds > 600000000LL) return fail(QC_EINVAL, "bad plan or timeout");
  P->wait_us = microseconds;
  return QC_OK;
}

qc_status qc_plan_set_wait_bias(qc_plan* P, int32_t bias) {
  g_err.clear();
  if (!P || bias < 0) return fail(QC_EINVAL, "bad plan or bias");
  P->wait_bias = bias;
  return QC_OK;
}

qc_status qc_plan_info(const qc_plan* P, int32_t* n_launches, int32_t* concurrent, int32_t* tiles,
                       int64_t* splits) {
  g_err.clear();
  if (!P) return fail(QC_EINVAL, "NULL plan");
  if (n_launches) *n_launches = P->mode == QC_PLAN_GRAPH ? graph_launches(P) : 2;
  if (concurrent) *concurrent = P->concurrent;
  for (int i = 0; i < P->n; ++i) {
    if (tiles) tiles[i] = P->ga[i].fused ? P->ga[i].tile : -1;
    if (splits) splits[i] = P->ga[i].split;
  }
  return QC_OK;
}

qc_status qc_plan_execute_separate(qc_plan* P, const int8_t* const* x, float* const* vis, void* stream) {
  g_err.clear();
  qc_status st = plan_check_args(P, x, vis);
  if (st != QC_OK) return st;
  for (int i = 0; i < P->n; ++i) {
    const qc_array_desc& D = P->desc[i];
    qc_pfb_params pp{D.n_fft, D.n_taps, nullptr, 0};
    st = qc_xcorrelate(x[i], D.n_samp, D.n_ant, D.n_samp, &pp, nullptr, nullptr, D.spec_per_dump, QC_F32,
                       vis[i], 0, nullptr, stream);
    if (st != QC_OK) return st;
  }
  return QC_OK;
}

qc_status qc_plan_capture_graph(qc_plan* P, const int8_t* const* x, float* const* vis, void* stream) {
  g_err.clear();
  qc_status st = plan_check_args(P, x, vis);
  if (st != QC_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (s == nullptr) return fail(QC_EINVAL, "graph capture needs a non-default stream");
  plan_drop_graph(P);
  QC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (P->mode == QC_PLAN_PERSISTENT) QC_HIP(qc::prepare_plan(), "plan kernel attributes");
  QC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  st = P->mode == QC_PLAN_GRAPH ? graph_execute(P, x, vis, s)
                                : persist_enqueue(P, x, vis, s, PLAN_SLOTS);  // the graph's own slot
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (st != QC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  P->graph = g;
  QC_HIP(hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
  return QC_OK;
}

qc_status qc_plan_replay(qc_plan* P, void* stream) {
  g_err.clear();
  if (!P || !P->gexec) return fail(QC_ESTATE, "no captured graph");
  // created streams only: a multi-branch graph replayed on the legacy default
  // stream (which synchronises implicitly with every blocking stream) once
  // left a later device-wide synchronisation waiting
  if (stream == nullptr) return fail(QC_EINVAL, "graph replay needs a non-default stream");
  QC_HIP(hipGraphLaunch(P->gexec, reinterpret_cast<hipStream_t>(stream)), "hipGraphLaunch");
  return QC_OK;
}

qc_status qc_plan_autotune(qc_plan* P, const int8_t* const* x, float* const* vis, int32_t reps,
                           const char* cache_path, int32_t* from_cache, void* stream) {
  g_err.clear();
  qc_status st = plan_check_args(P, x, vis);
  if (st != QC_OK) return st;
  if (reps < 1) return fail(QC_EINVAL, "reps must be >= 1");
  if (P->mode != QC_PLAN_GRAPH) return fail(QC_EUNSUPPORTED, "autotuning covers the graph mode only");
  if (from_cache) *from_cache = 0;
  const std::string sig = plan_signature(P);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      if (ls >> k && k == sig && graph_knobs_parse(P, ls)) {
        plan_drop_graph(P);
        if (from_cache) *from_cache = 1;
        return QC_OK;
      }
    }
  }
  plan_drop_graph(P);  // knobs change the recorded launches
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  QC_HIP(hipEventCreate(&a), "hipEventCreate");
  hipError_t e = hipEventCreate(&b);
  if (e != hipSuccess) {
    (void)hipEventDestroy(a);
    return hip_fail(e, "hipEventCreate");
  }
  st = graph_tune(P, x, vis, reps, s, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != QC_OK) return st;
  if (cache_path) {
    std::ofstream o(cache_path, std::ios::app);
    o << sig << " " << graph_knobs(P) << "\n";
  }
  return QC_OK;
}

void qc_plan_destroy(qc_plan* P) {
  if (!P) return;
  (void)hipDeviceSynchronize();
  plan_drop_graph(P);
  graph_free(P);
  for (int i = 0; i < qc::PL_MAX_ARRAYS; ++i) {
    if (P->st[i]) (void)hipStreamDestroy(P->st[i]);
    if (P->join_ev[i]) (void)hipEventDestroy(P->join_ev[i]);
  }
  if (P->fork_ev) (void)hipEventDestroy(P->fork_ev);
  persist_free(P);
  for (auto& ev : P->slot_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (P->d_ctr) (void)hipFree(P->d_ctr);
  if (P->d_slots) (void)hipFree(P->d_slots);
  if (P->h_slots) (void)hipHostFree(P->h_slots);
  delete P;
}

}  // extern "C"

// ---- learned RFI flagger ------------------------------------------------------
namespace {

qc_status cnn_check_img(const void* params, const float* x, int32_t n_img, int32_t H, int32_t W) {
  if (!params || !x) return fail(QC_EINVAL, "params or x is NULL");
  if (n_img < 1 || H < 1 || W < 1) return fail(QC_EINVAL, "n_img, height and width must be >= 1");
  if ((int64_t)n_img * H * W > 0x7fffffffLL) return fail(QC_EINVAL, "n_img * height * width must be < 2^31");
  if ((reinterpret_cast<uintptr_t>(params) | reinterpret_cast<uintptr_t>(x)) & 3u)
    return fail(QC_EINVAL, "params and x must be 4-byte aligned");
  return QC_OK;
}

// Packed weights of L1..L3 (forward) and, with bwd, of L2 and L3 (backward data).
struct CnnPacked {
  AsyncBuf buf;
  float *w1 = nullptr, *w2 = nullptr, *w3 = nullptr, *w2b = nullptr, *w3b = nullptr;
};

qc_status cnn_pack_all(const float* p, bool bwd, CnnPacked& pk, hipStream_t s) {
  const size_t n1 = 9 * 32, n2 = 25 * 32 * 32;
  qc_status st = alloc_async(pk.buf, sizeof(float) * (n1 + (bwd ? 4 : 2) * n2), s);
  if (st != QC_OK) return st;
  float* b = (float*)pk.buf.p;
  pk.w1 = b;
  pk.w2 = b + n1;
  pk.w3 = pk.w2 + n2;
  QC_HIP(qc::cnn_pack(p + qc::CNN_OFF_L1, 1, 32, 3, 0, pk.w1, s), "pack L1");
  QC_HIP(qc::cnn_pack(p + qc::CNN_OFF_L2, 32, 32, 5, 0, pk.w2, s), "pack L2");
  QC_HIP(qc::cnn_pack(p + qc::CNN_OFF_L3, 32, 32, 5, 0, pk.w3, s), "pack L3");
  if (bwd) {
    pk.w2b = pk.w3 + n2;
    pk.w3b = pk.w2b + n2;
    QC_HIP(qc::cnn_pack(p + qc::CNN_OFF_L2, 32, 32, 5, 1, pk.w2b, s), "pack L2 (backward)");
    QC_HIP(qc::cnn_pack(p + qc::CNN_OFF_L3, 32, 32, 5, 1, pk.w3b, s), "pack L3 (backward)");
  }
  return QC_OK;
}

// Forward of images [n][H][W]: a1 and a2/a3 ping-pong in A and B.
qc_status cnn_forward_chunk(const float* p, const CnnPacked& pk, const float* x, int64_t n, int H, int W,
                            float* A, float* B, float* logits, float thr, int64_t img0, int64_t n_base,
                            uint8_t* mask, hipStream_t s) {
  QC_HIP(qc::cnn_conv(1, 0, x, pk.w1, p + qc::CNN_OFF_L1 + 288, nullptr, n, H, W, A, s), "conv L1");
  QC_HIP(qc::cnn_conv(2, 0, A, pk.w2, p + qc::CNN_OFF_L2 + 25600, nullptr, n, H, W, B, s), "conv L2");
  QC_HIP(qc::cnn_conv3_head(B, pk.w3, p + qc::CNN_OFF_L3 + 25600, p + qc::CNN_OFF_L4, n, H, W, A, logits, thr,
                            img0, n_base, mask, s),
         "conv L3 + head");
  return QC_OK;
}

constexpr int64_t CNN_CHUNK_BYTES = (int64_t)1 << 30;  // per activation buffer

int64_t cnn_chunk_images(int64_t H, int64_t W, int64_t bytes_per = sizeof(float)) {
  const int64_t per = 32 * H * W * bytes_per;
  const int64_t c = CNN_CHUNK_BYTES / per;
  return c < 1 ? 1 : c;
}

// Workspace of the half-activation path: matrix-core weights of L2 and L3
// and two NHWC half activation buffers for `chunk` images.
struct CnnHalf {
  AsyncBuf w, a, b;
  int64_t chunk = 1;
  _Float16* w2() const { return (_Float16*)w.p; }
  _Float16* w3() const { return (_Float16*)w.p + 50 * 64 * 8; }
  _Float16* A() const { return (_Float16*)a.p; }
  _Float16* B() const { return (_Float16*)b.p; }
};

qc_status cnn_half_setup(const float* params, int64_t n_img, int H, int W, CnnHalf& hf, hipStream_t s) {
  hf.chunk = std::min<int64_t>(n_img, cnn_chunk_images(H, W, 2));
  const size_t ab = sizeof(_Float16) * 32 * (size_t)hf.chunk * H * W;
  qc_status st;
  if ((st = alloc_async(hf.w, sizeof(_Float16) * 2 * 50 * 64 * 8, s)) != QC_OK ||
      (st = alloc_async(hf.a, ab, s)) != QC_OK || (st = alloc_async(hf.b, ab, s)) != QC_OK)
    return st;
  QC_HIP(qc::cnn_pack_mfma(params + qc::CNN_OFF_L2, hf.w2(), s), "pack L2 (matrix cores)");
  QC_HIP(qc::cnn_pack_mfma(params + qc::CNN_OFF_L3, hf.w3(), s), "pack L3 (matrix cores)");
  return QC_OK;
}

}  // namespace

extern "C" {

int32_t qc_cnn_param_count(void) { return qc::CNN_PARAMS; }

qc_status qc_channelize_set_variant(int32_t variant) {
  g_err.clear();
  if (variant < 0 || variant > 1) return fail(QC_EINVAL, "variant must be 0 or 1");
  qc::set_channelize_variant(variant);
  return QC_OK;
}

int32_t qc_channelize_get_variant(void) { return qc::get_channelize_variant(); }

qc_status qc_xengine_set_variant(int32_t variant) {
  g_err.clear();
  if (variant < 0 || variant > 2) return fail(QC_EINVAL, "variant must be 0, 1 or 2");
  qc::set_xeng_f32_variant(variant);
  return QC_OK;
}

int32_t qc_xengine_get_variant(void) { return qc::get_xeng_f32_variant(); }

qc_status qc_measure_peak(int32_t kind, void* scratch, int64_t bytes, int32_t reps, double* rate,
                          void* stream) {
  g_err.clear();
  if (kind < QC_PEAK_HBM_READ || kind > QC_PEAK_MFMA_F16) return fail(QC_EINVAL, "unknown kind %d", kind);
  if (!scratch || !rate) return fail(QC_EINVAL, "scratch and rate must be non-null");
  if (reps < 1) return fail(QC_EINVAL, "reps must be >= 1");
  if (reinterpret_cast<uintptr_t>(scratch) & 15u) return fail(QC_EINVAL, "scratch must be 16-byte aligned");
  const int64_t need = kind <= QC_PEAK_HBM_COPY ? (int64_t)64 << 20 : (int64_t)64 << 10;
  if (bytes < need) return fail(QC_EINVAL, "scratch of %lld bytes is below the %lld this kind needs",
                                (long long)bytes, (long long)need);
  QC_HIP(qc::measure_peak(kind, scratch, bytes, reps, rate, (hipStream_t)stream), "measure_peak");
  return QC_OK;
}

qc_status qc_cnn_set_variant(int32_t variant) {
  g_err.clear();
  if (variant < 0 || variant > 1) return fail(QC_EINVAL, "variant must be 0 or 1");
  qc::set_cnn_mfma(variant == 0);
  return QC_OK;
}

int32_t qc_cnn_get_variant(void) { return qc::get_cnn_mfma() ? 0 : 1; }

qc_status qc_cnn_normalize(const float* vis, int64_t n_time, int64_t n_base, int32_t n_chan, float* x,
                           void* stream) {
  g_err.clear();
  if (!vis || !x) return fail(QC_EINVAL, "vis or x is NULL");
  if (n_time < 1 || n_base < 1 || n_chan < 1) return fail(QC_EINVAL, "sizes must be >= 1");
  if (n_base > 0x7fffffffLL) return fail(QC_EINVAL, "too many baselines");
  if (reinterpret_cast<uintptr_t>(vis) & 7u) return fail(QC_EINVAL, "vis must be 8-byte aligned");
  qc_status st = ensure_device();
  if (st != QC_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  AsyncBuf stats;
  st = alloc_async(stats, sizeof(double) * 2 * n_base, s);
  if (st != QC_OK) return st;
  const float2* v = reinterpret_cast<const float2*>(vis);
  AsyncBuf amp;
  const int64_t na = qc::mad_scratch_floats(n_time, n_base, n_chan, 0);
  if (na > 0 && (st = alloc_async(amp, sizeof(float) * (size_t)na, s)) != QC_OK) return st;
  QC_HIP(qc::launch_mad(v, n_time, n_base, n_chan, 0.f, 0, nullptr, nullptr, (double*)stats.p, (float*)amp.p, s),
         "MAD stats");
  QC_HIP(qc::cnn_normalize(v, (const double*)stats.p, n_time, n_base, n_chan, 0, n_base, x, s), "normalise");
  return QC_OK;
}

qc_status qc_cnn_forward(const float* params, const float* x, int32_t n_img, int32_t H, int32_t W,
                         int32_t act_prec, float* logits, void* stream) {
  g_err.clear();
  qc_status st = cnn_check_img(params, x, n_img, H, W);
  if (st != QC_OK) return st;
  if (!logits) return fail(QC_EINVAL, "logits is NULL");
  if (act_prec != 0 && act_prec != 1) return fail(QC_EINVAL, "act_prec must be 0 (float32) or 1 (half)");
  st = ensure_device();
  if (st != QC_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (act_prec == 1) {
    CnnHalf hf;
    if ((st = cnn_half_setup(params, n_img, H, W, hf, s)) != QC_OK) return st;
    const int64_t hw = (int64_t)H * W;
    for (int64_t i0 = 0; i0 < n_img; i0 += hf.chunk) {
      const int64_t n = std::min<int64_t>(hf.chunk, n_img - i0);
      QC_HIP(qc::cnn_forward_f16(params, hf.w2(), hf.w3(), x + i0 * hw, n, H, W, hf.A(), hf.B(), logits + i0 * hw,
                                 0.f, 0, 0, nullptr, s),
             "half forward");
    }
    return QC_OK;
  }
  CnnPacked pk;
  st = cnn_pack_all(params, false, pk, s);
  if (st != QC_OK) return st;
  const int64_t chunk = std::min<int64_t>(n_img, cnn_chunk_images(H, W));
  const size_t abytes = sizeof(float) * 32 * (size_t)chunk * H * W;
  AsyncBuf A, B;
  if ((st = alloc_async(A, abytes, s)) != QC_OK || (st = alloc_async(B, abytes, s)) != QC_OK) return st;
  const int64_t hw = (int64_t)H * W;
  for (int64_t i0 = 0; i0 < n_img; i0 += chunk) {
    const int64_t n = std::min<int64_t>(chunk, n_img - i0);
    st = cnn_forward_chunk(params, pk, x + i0 * hw, n, H, W, (float*)A.p, (float*)B.p, logits + i0 * hw, 0.f, 0,
                           0, nullptr, s);
    if (st != QC_OK) return st;
  }
  return QC_OK;
}

qc_status qc_cnn_grad(const float* params, const float* x, const uint8_t* labels, int32_t n_img, int32_t H,
                      int32_t W, float pos_weight, float* grad, float* loss, void* stream) {
  g_err.clear();
  qc_status st = cnn_check_img(params, x, n_img, H, W);
  if (st != QC_OK) return st;
  if (!labels || !grad || !loss) return fail(QC_EINVAL, "labels, grad or loss is NULL");
  if (!(pos_weight > 0.f) || !std::isfinite(pos_weight)) return fail(QC_EINVAL, "pos_weight must be > 0");
  const int64_t act = 32 * (int64_t)n_img * H * W;
  if (act * (int64_t)sizeof(float) > ((int64_t)8 << 30))
    return fail(QC_EINVAL, "batch too large: one activation would exceed 8 GiB");
  st = ensure_device();
  if (st != QC_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  CnnPacked pk;
  st = cnn_pack_all(params, true, pk, s);
  if (st != QC_OK) return st;
  const int64_t hw = (int64_t)H * W;
  const int64_t wblocks = qc::cnn_wgrad_blocks(n_img, H, W);
  const int64_t hblocks = qc::cnn_head_bwd_blocks((int64_t)n_img * hw);
  const size_t part_floats = std::max<size_t>((size_t)wblocks * 25632, (size_t)hblocks * 34);
  AsyncBuf a1, a2, a3, z, gA, gB, part;
  const size_t ab = sizeof(float) * (size_t)act;
  if ((st = alloc_async(a1, ab, s)) != QC_OK || (st = alloc_async(a2, ab, s)) != QC_OK ||
      (st = alloc_async(a3, ab, s)) != QC_OK || (st = alloc_async(gA, ab, s)) != QC_OK ||
      (st = alloc_async(gB, ab, s)) != QC_OK || (st = alloc_async(z, sizeof(float) * n_img * hw, s)) != QC_OK ||
      (st = alloc_async(part, sizeof(float) * part_floats, s)) != QC_OK)
    return st;
  float *A1 = (float*)a1.p, *A2 = (float*)a2.p, *A3 = (float*)a3.p, *Z = (float*)z.p;
  float *GA = (float*)gA.p, *GB = (float*)gB.p, *PT = (float*)part.p;
  const float* p = params;
  QC_HIP(qc::cnn_conv(1, 0, x, pk.w1, p + qc::CNN_OFF_L1 + 288, nullptr, n_img, H, W, A1, s), "conv L1");
  QC_HIP(qc::cnn_conv(2, 0, A1, pk.w2, p + qc::CNN_OFF_L2 + 25600, nullptr, n_img, H, W, A2, s), "conv L2");
  QC_HIP(qc::cnn_conv(3, 0, A2, pk.w3, p + qc::CNN_OFF_L3 + 25600, nullptr, n_img, H, W, A3, s), "conv L3");
  QC_HIP(qc::cnn_head(A3, p + qc::CNN_OFF_L4, n_img, H, W, Z, 0.f, 0, 0, nullptr, s), "head");
  QC_HIP(qc::cnn_head_bwd(Z, labels, A3, p + qc::CNN_OFF_L4, n_img, H, W, pos_weight, GA, PT,
                          grad + qc::CNN_OFF_L4, loss, s),
         "loss and head backward");
  QC_HIP(qc::cnn_wgrad(3, A2, GA, n_img, H, W, PT, grad + qc::CNN_OFF_L3, s), "L3 weight gradient");
  QC_HIP(qc::cnn_conv(3, 1, GA, pk.w3b, nullptr, A2, n_img, H, W, GB, s), "L3 backward data");
  QC_HIP(qc::cnn_wgrad(2, A1, GB, n_img, H, W, PT, grad + qc::CNN_OFF_L2, s), "L2 weight gradient");
  QC_HIP(qc::cnn_conv(2, 1, GB, pk.w2b, nullptr, A1, n_img, H, W, GA, s), "L2 backward data");
  QC_HIP(qc::cnn_wgrad(1, x, GA, n_img, H, W, PT, grad + qc::CNN_OFF_L1, s), "L1 weight gradient");
  return QC_OK;
}

qc_status qc_cnn_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr, float beta1,
                      float beta2, float eps, void* stream) {
  g_err.clear();
  if (!params || !grad || !m || !v) return fail(QC_EINVAL, "NULL argument");
  if (step < 1) return fail(QC_EINVAL, "step must be >= 1");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(QC_EINVAL, "bad Adam hyper-parameters");
  QC_HIP(qc::cnn_adam(params, grad, m, v, qc::CNN_PARAMS, step, lr, beta1, beta2, eps,
                      reinterpret_cast<hipStream_t>(stream)),
         "Adam kernel");
  return QC_OK;
}

qc_status qc_cnn_train_step(float* params, float* m, float* v, int64_t step, const float* x,
                            const uint8_t* labels, int32_t n_img, int32_t H, int32_t W, float pos_weight,
                            float lr, float* loss, void* stream) {
  g_err.clear();
  if (!m || !v) return fail(QC_EINVAL, "m or v is NULL");
  if (step < 1) return fail(QC_EINVAL, "step must be >= 1");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  AsyncBuf g;
  qc_status st = alloc_async(g, sizeof(float) * qc::CNN_PARAMS, s);
  if (st != QC_OK) return st;
  st = qc_cnn_grad(params, x, labels, n_img, H, W, pos_weight, (float*)g.p, loss, stream);
  if (st != QC_OK) return st;
  return qc_cnn_adam(params, (const float*)g.p, m, v, step, lr, 0.9f, 0.999f, 1e-8f, stream);
}

qc_status qc_cnn_flag(const float* params, const float* vis, int64_t n_time, int64_t n_base, int32_t n_chan,
                      float logit_threshold, int32_t act_prec, uint8_t* mask, void* stream) {
  g_err.clear();
  if (!params || !vis || !mask) return fail(QC_EINVAL, "params, vis or mask is NULL");
  if (act_prec != 0 && act_prec != 1) return fail(QC_EINVAL, "act_prec must be 0 (float32) or 1 (half)");
  if (n_time < 1 || n_base < 1 || n_chan < 1) return fail(QC_EINVAL, "sizes must be >= 1");
  if (n_time * n_chan > 0x7fffffffLL || n_base > 0x7fffffffLL) return fail(QC_EINVAL, "plane too large");
  if (reinterpret_cast<uintptr_t>(vis) & 7u) return fail(QC_EINVAL, "vis must be 8-byte aligned");
  if (!std::isfinite(logit_threshold)) return fail(QC_EINVAL, "threshold must be finite");
  qc_status st = ensure_device();
  if (st != QC_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int H = (int)n_time, W = n_chan;
  const int64_t hw = (int64_t)H * W;
  AsyncBuf stats;
  if ((st = alloc_async(stats, sizeof(double) * 2 * n_base, s)) != QC_OK) return st;
  const float2* v = reinterpret_cast<const float2*>(vis);
  {
    AsyncBuf amp;
    const int64_t na = qc::mad_scratch_floats(n_time, n_base, n_chan, 0);
    if (na > 0 && (st = alloc_async(amp, sizeof(float) * (size_t)na, s)) != QC_OK) return st;
    QC_HIP(qc::launch_mad(v, n_time, n_base, n_chan, 0.f, 0, nullptr, nullptr, (double*)stats.p, (float*)amp.p,
                          s),
           "MAD stats");
  }
  if (act_prec == 1) {
    CnnHalf hf;
    if ((st = cnn_half_setup(params, n_base, H, W, hf, s)) != QC_OK) return st;
    AsyncBuf X;
    if ((st = alloc_async(X, sizeof(float) * (size_t)hf.chunk * hw, s)) != QC_OK) return st;
    for (int64_t b0 = 0; b0 < n_base; b0 += hf.chunk) {
      const int64_t n = std::min<int64_t>(hf.chunk, n_base - b0);
      QC_HIP(qc::cnn_normalize(v, (const double*)stats.p, n_time, n_base, n_chan, b0, n, (float*)X.p, s),
             "normalise");
      QC_HIP(qc::cnn_forward_f16(params, hf.w2(), hf.w3(), (const float*)X.p, n, H, W, hf.A(), hf.B(), nullptr,
                                 logit_threshold, b0, n_base, mask, s),
             "half forward");
    }
    return QC_OK;
  }
  CnnPacked pk;
  if ((st = cnn_pack_all(params, false, pk, s)) != QC_OK) return st;
  const int64_t chunk = std::min<int64_t>(n_base, cnn_chunk_images(H, W));
  AsyncBuf X, A, B;
  if ((st = alloc_async(X, sizeof(float) * (size_t)chunk * hw, s)) != QC_OK ||
      (st = alloc_async(A, sizeof(float) * 32 * (size_t)chunk * hw, s)) != QC_OK ||
      (st = alloc_async(B, sizeof(float) * 32 * (size_t)chunk * hw, s)) != QC_OK)
    return st;
  for (int64_t b0 = 0; b0 < n_base; b0 += chunk) {
    const int64_t n = std::min<int64_t>(chunk, n_base - b0);
    QC_HIP(qc::cnn_normalize(v, (const double*)stats.p, n_time, n_base, n_chan, b0, n, (float*)X.p, s),
           "normalise");
    st = cnn_forward_chunk(params, pk, (const float*)X.p, n, H, W, (float*)A.p, (float*)B.p, nullptr,
                           logit_threshold, b0, n_base, mask, s);
    if (st != QC_OK) return st;
  }
  return QC_OK;
}

}  // extern "C"
