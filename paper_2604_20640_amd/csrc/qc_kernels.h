// Launchers shared between the C-ABI layer and the kernel translation units.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <tuple>
#include <type_traits>
#include <utility>

namespace qc {

struct FxArgs {
  const int8_t* x;
  int64_t ld_x;
  int32_t n_ant;
  int64_t n_samp;
  int32_t n_fft;
  int32_t n_taps;
  const float* taps;   // device [P*N]
  const float2* tw;    // device [N], exp(-2 pi i e/N)
  const int8_t* hist;  // device [n_ant][(P-1)N] or null
  bool taps_symmetric; // h[q] == h[P*N-1-q] (the built-in prototype)
  // device [N-1]: per-pass twiddles of the radix-16 Stockham FFT, the pass
  // of stride NS holding W_{NS R}^{jm r} at (NS-1) + (r-1) NS + jm
  const float2* twp = nullptr;
};

// Fused F+X for small arrays.  Returns false if no fused kernel exists for
// (n_fft, n_ant); part must hold fused_part_elems() float2.
bool fused_supported(int n_fft, int n_ant);
int fused_tile_count(int n_fft, int n_ant);
// Compute units of the current device (cached per device; 256 if the query
// fails).
int device_cu_count();

// Chunks per dump of a fused launch: about `workgroups` workgroups in all
// (at least 8 spectra per chunk).
int64_t fused_chunks_per_dump(int n_fft, int n_ant, int64_t n_dump, int64_t spec_per_dump,
                              int64_t workgroups = 512);
// tile: index into the (n_fft, n_ant) tile list; 0 is the default shape.
hipError_t launch_fused(const FxArgs& a, int64_t n_dump, int64_t spec_per_dump,
                        int64_t chunks_per_dump, float2* part, hipStream_t s, int tile);

// Deterministic reduction of per-chunk partials:
// vis[d][e] = (accumulate ? vis[d][e] : 0) + scale * sum_c part[d*cpd + c][e].
// tile > 0: each partial is tile-major, [n_chan/tile][nb][tile], and e is
// mapped to the [nb][n_chan] position of the visibilities.
hipError_t launch_reduce(const float2* part, int64_t n_dump, int64_t cpd, int64_t elems,
                         float scale, int accumulate, float2* vis, hipStream_t s, int tile = 0,
                         int64_t nb = 0);

// Standalone F-engine.  out layout [n_ant][n_spec][n_chan]; prec 0..3 as qc_prec.
// Variant 0 uses the ring kernel where it applies (P = 4, built-in taps,
// N = 1024..4096), 1 always the plain kernel.
void set_channelize_variant(int v);
int get_channelize_variant();
hipError_t launch_channelize(const FxArgs& a, int prec, void* out, const float* scale,
                             hipStream_t s);

// F-engine over any input word (sample: 0 real int8, 1 real int16, 2 complex
// int8, 3 complex int16; I and Q interleaved).  ld_x and n_samp count
// samples; hist holds (P-1)N samples per antenna of the same word.  Output
// [n_ant][n_spec][n_chan] with n_chan = N/2 (real words) or N (complex).
struct ChanxArgs {
  const void* x;
  int64_t ld_x;
  int32_t n_ant;
  int64_t n_samp;
  int32_t n_fft;
  int32_t n_taps;
  const float* taps;  // device [P*N]
  const float2* tw;   // device [N], exp(-2 pi i e/N)
  const void* hist;   // device [n_ant][(P-1)N] samples or null
  bool taps_symmetric = false;  // h[q] == h[P*N-1-q] (the built-in prototype)
  const float2* twp = nullptr;  // per-pass twiddles, as in FxArgs
};
// Fused F+X of real int16 words where a ring tile applies (n_ant 4 at
// N = 1024, 2048, 4096, or 2 at 4096; P = 4, the built-in prototype); the
// partials as launch_fused's.
bool fused_words_supported(int sample, int n_fft, int n_ant, int n_taps, bool taps_symmetric);
hipError_t launch_fused_words(const FxArgs& a, int sample, int64_t n_dump, int64_t spd, int64_t cpd,
                              float2* part, hipStream_t s);
// The ring F-engine for any word where it applies (P = 4, symmetric taps,
// N = 1024..8192, ring variant selected); hipErrorNotSupported otherwise.
hipError_t launch_channelize_ring_any(const ChanxArgs& a, int sample, int prec, void* out, const float* scale,
                                      hipStream_t s);
hipError_t launch_channelize_any(const ChanxArgs& a, int sample, int prec, void* out, const float* scale,
                                 hipStream_t s);
// Scales as launch_scales, from |x|^2 of any input word.
hipError_t launch_scales_any(const void* x, int sample, int64_t ld_x, int n_ant, int64_t n_use,
                             double sum_h2, double target, unsigned long long* part, float* scale_out,
                             hipStream_t s);

// Per-antenna power-of-two scales for requantised output from the first
// n_use samples; part holds n_ant * SC_BLOCKS partial sums (scratch).
constexpr int SC_BLOCKS = 64;
hipError_t launch_scales(const int8_t* x, int64_t ld_x, int n_ant, int64_t n_use, double sum_h2,
                         double target, unsigned long long* part, float* scale_out, hipStream_t s);

// Copy the last (P-1)N samples of (hist ++ x) to hist_out.
hipError_t launch_hist_copy(const int8_t* x, int64_t ld_x, int n_ant, int64_t n_samp,
                            const int8_t* hist, int64_t keep, int8_t* hist_out, hipStream_t s);

// X-engine (float32) over v[n_ant][n_spec][n_chan] cfloat, on the matrix
// cores (16x16 tiles up to 16 antennas, 32x32 above; n_ant <= 32,
// n_chan % 16 == 0, v 16-byte aligned) or
// the vector ALU.  Variant: 0 = matrix cores for XEF_MFMA_MIN_ANT..32
// antennas, 1 = always the vector ALU, 2 = matrix cores wherever supported.
// xeng_f32_ksplit sizes the partial buffer for the kernel that
// launch_xeng_f32 picks for a 16-byte aligned v.
constexpr int XEF_MFMA_MIN_ANT = 5;
void set_xeng_f32_variant(int v);
int get_xeng_f32_variant();
bool xeng_f32_use_mfma(int n_ant, int n_chan, const void* v);
// Partial layout launch_xeng_f32 writes for v: 0 = [nb][n_chan], else the
// tile width of the tile-major layout (see launch_reduce).
int xeng_f32_tile(int n_ant, int n_chan, const void* v);
int64_t xeng_f32_ksplit(int n_ant, int64_t spec_per_dump, int n_chan, int64_t n_dump);
hipError_t launch_xeng_f32(const float2* v, int n_ant, int64_t n_spec, int n_chan,
                           int64_t spec_per_dump, int64_t n_dump, int64_t ksplit, float2* part,
                           hipStream_t s);
bool xeng_f32_mfma_supported(int n_ant, int n_chan, const void* v);
int64_t xeng_f32_mfma_ksplit(int n_ant, int64_t spec_per_dump, int n_chan, int64_t n_dump);
hipError_t launch_xeng_f32_mfma(const float2* v, int n_ant, int64_t n_spec, int n_chan,
                                int64_t spec_per_dump, int64_t n_dump, int64_t ksplit, float2* part,
                                hipStream_t s);

// X-engine on matrix cores over requantised v (prec 1..3); partials are
// tile-major with tile XM_TILE.
constexpr int XM_TILE = 32;
hipError_t launch_xeng_mfma(const void* v, int prec, const float* scale, int n_ant,
                            int64_t n_spec, int n_chan, int64_t spec_per_dump, int64_t n_dump,
                            int64_t ksplit, float2* part, hipStream_t s);
int64_t xeng_mfma_ksplit(int prec, int n_ant, int64_t spec_per_dump, int n_chan, int64_t n_dump);

// MAD flagging.  mask, thresh and stats ([pop][2]: median, MAD) may be null.
// Populations above the single-wave size take their amplitudes from
// amp_scratch (mad_scratch_floats() floats), formed there first by one
// whole-GPU pass; null: each workgroup forms them from vis.
int64_t mad_scratch_floats(int64_t n_time, int64_t n_base, int n_chan, int population);
hipError_t launch_mad(const float2* vis, int64_t n_time, int64_t n_base, int n_chan, float sigma,
                      int population, uint8_t* mask, double* thresh, double* stats, float* amp_scratch,
                      hipStream_t s);

// Delay/phase application; tau/phi host arrays of n_ant doubles (n_ant <= 64).
hipError_t launch_apply(float2* vis, int64_t n_time, int n_ant, int n_chan, double f0, double df,
                        const double* tau, const double* phi, hipStream_t s);

// Delay/phase solve: per-cross-baseline fits, then the per-antenna solution.
// tau_b, phi_b: device scratch double[n_ant(n_ant-1)/2]; tau, phi: device double[n_ant].
hipError_t launch_solve(const float2* vis, const uint8_t* mask, int64_t n_time, int n_ant, int n_chan,
                        double f0, double df, int ref, int lo, int hi, int n_lag, const float2* tw,
                        double* tau_b, double* phi_b, double* tau, double* phi, hipStream_t s);

// ---- batched plans: one persistent launch over heterogeneous work items ----
constexpr int PL_NT = 512;          // threads per block of the persistent kernel
constexpr int PL_MAX_ARRAYS = 8;
constexpr int PL_RED_LOADS = 1 << 14;  // partial loads per reduction item (sizing target)

// Work-item kinds: fused F+X; F-engine (plain body, or the ring body at
// N = 4096 / 8192); X-engine (vector ALU, or matrix cores for 5..32
// antennas); reduction of partials.
enum { PL_FUSED = 0, PL_CHAN = 1, PL_XENG = 2, PL_REDUCE = 3, PL_CHAN_RING = 4, PL_XMFMA = 5 };

struct PlArray {
  const int8_t* x;       // [n_ant][n_samp] (set per execution)
  float2* vis;           // [n_dump][n_base][n_chan] (set per execution)
  float2* part;          // partial visibilities [n_dump * n_split][n_base][n_chan]
  float2* chan;          // two-pass only: float32 spectra [n_ant][n_spec][n_chan]
  const float* taps;
  const float2* tw;
  int64_t n_samp, spd, n_dump, n_split;  // n_split: fused chunks per dump / X-engine k-split
  int64_t spec_per_item;                 // two-pass: spectra per F-engine item
  int32_t n_ant, n_fft, n_taps, mode;    // mode 0 fused, 1 two-pass
  int32_t n_chan_items, n_part_items, n_cgrp, n_bp, n_red_blocks;
  float scale;                           // reduction scale (1/4 for two-for-one spectra)
  int64_t spb;                           // ring F-engine items: spectra per item
  int32_t n_chunks;                      // ring F-engine items: runs of spb per antenna group
  int32_t x_kind;                        // 0 vector ALU, 1 matrix cores 32 x 32, 2 matrix cores 16 x 16
  int32_t n_cb;                          // matrix-core X items: channel blocks of 16
  int32_t tile;                          // partials: 0 [baseline][chan], else tile-major of this width
  int32_t red_block;                     // reduction items: visibilities per item (a multiple of PL_NT)
  int32_t pad1;
};

// A float2 store for data that workgroups of the persistent plan kernel
// hand to one another.  WT = true: an agent-scope relaxed atomic store,
// which writes through the XCD's L2 to the device's coherence point, so
// that publishing needs no writeback of the L2 (see plan_kernel).  The
// separate kernels use plain stores (WT = false).
template <bool WT>
__device__ __forceinline__ void st_f2(float2* p, float2 v) {
  if constexpr (WT) {
    const uint64_t b = ((uint64_t)__float_as_uint(v.y) << 32) | __float_as_uint(v.x);
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    *p = v;
  }
}

struct PlItem {
  uint16_t kind, array;
  uint32_t index;
};

struct PlArgs {
  const PlArray* arr;  // device [n_arrays]
  const PlItem* items;
  int32_t n_items;
  int32_t wait_bias;   // added to every wait target (failure injection; 0 in use)
  int64_t wait_ticks;  // time limit of one dependency wait, wall-clock ticks
  unsigned* ctr;  // [0] queue head, [1] error flag, [2+2a] partials done, [3+2a] spectra done
};

bool plan_fused_supported(int n_fft, int n_ant);
bool plan_chan_supported(int n_fft);
// Sets the persistent kernel's LDS limit on the current device; call before
// launch_plan and outside stream capture.
hipError_t prepare_plan();
hipError_t launch_plan(const PlArgs& a, int grid, hipStream_t s);

// ---- learned RFI flagger ----
constexpr int CNN_PARAMS = 51617;
constexpr int CNN_OFF_L1 = 0, CNN_OFF_L2 = 320, CNN_OFF_L3 = 25952, CNN_OFF_L4 = 51584;
// Repack W[o][i][ky][kx] for the convolution kernel (flip: backward data).
hipError_t cnn_pack(const float* w, int CI, int CO, int K, int flip, float* p, hipStream_t s);
// dir 0: layer 1..3 forward with bias and ReLU; dir 1: backward data of
// layer 2 or 3, gated by gate > 0 (the activation of the layer below).
hipError_t cnn_conv(int layer, int dir, const float* in, const float* wp, const float* b, const float* gate,
                    int64_t n_img, int H, int W, float* out, hipStream_t s);
int64_t cnn_wgrad_blocks(int64_t n_img, int H, int W);
// Float32 convolutions and weight gradients of the 32 -> 32 layers on the
// matrix cores (default) or the vector ALU (process-wide).
void set_cnn_mfma(bool on);
bool get_cnn_mfma();
// Weight and bias gradient of layer 1..3 into dst (flat W then b); part
// holds cnn_wgrad_blocks() * (weights + biases) floats.
hipError_t cnn_wgrad(int layer, const float* a, const float* g, int64_t n_img, int H, int W, float* part,
                     float* dst, hipStream_t s);
// Output layer: logits and/or a flag mask in [time][baseline][chan] layout.
hipError_t cnn_head(const float* a3, const float* w4, int64_t n_img, int H, int W, float* logits, float thr,
                    int64_t img0, int64_t n_base, uint8_t* mask, hipStream_t s);
// L3 forward followed by the output layer (inference): on the matrix cores
// the logits/flags come from L3's epilogue and a3 is not written; otherwise
// L3 into a3, then cnn_head.
hipError_t cnn_conv3_head(const float* a2, const float* w3p, const float* b3, const float* w4, int64_t n_img,
                          int H, int W, float* a3, float* logits, float thr, int64_t img0, int64_t n_base,
                          uint8_t* mask, hipStream_t s);
int64_t cnn_head_bwd_blocks(int64_t n_total);
// Loss, dW4/db4 (grad4[33]) and g3; part holds cnn_head_bwd_blocks() * 34 floats.
hipError_t cnn_head_bwd(const float* logits, const uint8_t* labels, const float* a3, const float* w4,
                        int64_t n_img, int H, int W, float pos_weight, float* g3, float* part, float* grad4,
                        float* loss, hipStream_t s);
hipError_t cnn_adam(float* w, const float* g, float* m, float* v, int n, int64_t step, float lr, float b1,
                    float b2, float eps, hipStream_t s);
hipError_t cnn_normalize(const float2* vis, const double* stats, int64_t n_time, int64_t n_base, int n_chan,
                         int64_t b0, int64_t nb, float* x, hipStream_t s);
// Half-activation inference: weights of L2/L3 packed by cnn_pack_mfma
// (50*64*8 halves each); A, B: n_img*H*W*32 halves.
hipError_t cnn_pack_mfma(const float* w, _Float16* p, hipStream_t s);
hipError_t cnn_forward_f16(const float* params, const _Float16* w2p, const _Float16* w3p, const float* x,
                           int64_t n_img, int H, int W, _Float16* A, _Float16* B, float* logits, float thr,
                           int64_t img0, int64_t n_base, uint8_t* mask, hipStream_t s);

// Rate one measurement kernel of the given kind sustains (see qc_measure_peak).
hipError_t measure_peak(int kind, void* scratch, int64_t bytes, int reps, double* rate, hipStream_t s);

// Stop event to bind to a kernel launch on stream s, or null.  Non-null only
// while chained kernel timing is enabled (qc_timing_enable(2)): the event
// then records the end of that launch itself, with no packet of its own.
hipEvent_t timing_stop_event(hipStream_t s);

template <typename T>
using launch_arg_t = std::remove_cv_t<std::remove_reference_t<T>>;

template <typename Tup, size_t... I>
inline void launch_arg_ptrs(Tup& t, void** p, std::index_sequence<I...>) {
  ((p[I] = static_cast<void*>(&std::get<I>(t))), ...);
}

// Launches kernel k with its arguments converted to the kernel's own
// parameter types.  With chained timing on, the launch carries the stop
// event timing_stop_event() hands out.  Returns the launch's status.
template <typename... P, typename... A>
inline hipError_t launch(void (*k)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t s, A&&... a) {
  static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
  std::tuple<launch_arg_t<P>...> t{static_cast<launch_arg_t<P>>(std::forward<A>(a))...};
  void* ptrs[sizeof...(P) + 1];
  launch_arg_ptrs(t, ptrs, std::index_sequence_for<P...>{});
  hipEvent_t stop = timing_stop_event(s);
  hipError_t e = stop ? hipExtLaunchKernel(reinterpret_cast<const void*>(k), grid, block, ptrs, lds, s,
                                           nullptr, stop, 0)
                      : hipLaunchKernel(reinterpret_cast<const void*>(k), grid, block, ptrs, lds, s);
  hipError_t last = hipGetLastError();
  return e != hipSuccess ? e : last;
}

}  // namespace qc
