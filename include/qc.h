/*
 * qc.h -- C ABI of libqc, an FX-correlator hot path for AMD gfx950 (MI355X).
 *
 * The method is that of arXiv 2604.20640 (QUEST Python/CuPy correlator):
 *   F-engine  : polyphase-filter-bank weighting, then a real FFT of each
 *               antenna's int8 voltage stream (Sec. 4.1 step 1; Sec. 4.2
 *               "F-engine (PFB and FFT)"; Alg. 1 "Apply PFB weighting -> FFT").
 *   X-engine  : V_ij(k) = sum_m X_i,m(k) conj(X_j,m(k)) for all baselines,
 *               autos included, integrated over a dump (Sec. 4.1 eq. 1;
 *               Sec. 4.2 "X-engine and integration"; Alg. 1).
 *   MAD flags : T = median(A) + sigma * 1.4826 * MAD(A), flag A > T (Sec. 7 eq. 2).
 *   Delay/phase application: V_ij *= exp(+i[2 pi f (tau_i - tau_j) + phi_i - phi_j])
 *               (Sec. 4.1 step 2 and eq. 1; Sec. 7 delay and phase steps).
 *   Beside it: streaming ingest (Alg. 1), a matrix-core X-engine in reduced
 *   precision, the float64 delay/phase solve (Sec. 7), batched plans for
 *   several arrays and a learned RFI flagger judged by MAD.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers   : "device" pointers are HIP device memory owned by the caller; the
 *              library never frees or retains them after the call returns.
 *              "host" pointers are read (or written) before the call returns.
 * Streams    : every call is asynchronous on `stream` (a hipStream_t passed as
 *              void*; NULL = the default stream) unless its comment says it
 *              synchronises.
 * Errors     : arguments are validated on the host before anything is
 *              launched; a bad argument returns QC_EINVAL (or QC_EUNSUPPORTED
 *              for a valid but unimplemented combination) and launches nothing.
 *              A HIP failure returns QC_EHIP.  qc_last_error() gives a
 *              thread-local description of the last failure.
 * Complex    : interleaved (re, im) float32 pairs ("cfloat" below).
 * Antennas   : int8 input is antenna-major: x[a * ld_x + n], n = 0..n_samp-1.
 * Baselines  : b(i, j) = i*n_ant - i*(i-1)/2 + (j - i) for 0 <= i <= j < n_ant
 *              (upper triangle, row-major, autos included);
 *              n_base = n_ant*(n_ant+1)/2.
 * Channels   : n_chan = n_fft/2; channel k is DFT bin k of an n_fft-point real
 *              transform with kernel exp(-2 pi i k n / n_fft), no normalisation;
 *              the Nyquist bin is dropped.
 * Spectra    : spectrum m uses stream blocks m-P+1 .. m (block = n_fft samples);
 *              samples before the stream are `hist` if given, else zero, so a
 *              stream of n_samp samples gives n_samp / n_fft spectra.
 */
#ifndef QC_H
#define QC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qc_status;
enum {
  QC_OK = 0,
  QC_EINVAL = -1,       /* bad argument: nothing launched */
  QC_EUNSUPPORTED = -2, /* valid but not implemented: nothing launched */
  QC_EHIP = -3,         /* a HIP runtime call failed */
  QC_ENOMEM = -4,       /* device or host allocation failed */
  QC_ESTATE = -5        /* object used in the wrong state */
};

typedef enum { QC_F32 = 0, QC_F16 = 1, QC_BF16 = 2, QC_FP8_E4M3 = 3 } qc_prec;

/* Polyphase filter bank parameters (Sec. 4.3: FFT length and number of PFB
 * taps are runtime parameters).
 *   n_fft : N, a power of two, 4 <= N <= 8192.
 *   n_taps: P, 1 <= P <= 16.
 *   taps  : device float[P*N] prototype h[q], or NULL for the built-in
 *           Hann-windowed sinc h[q] = w[q] sinc((q-(L-1)/2)/N), L = P*N,
 *           w[q] = 0.5 - 0.5 cos(2 pi q/(L-1)), unnormalised.  The filter
 *           applied is y_m[n] = sum_p h[p*N+n] x[(m-P+1+p)*N + n].
 *   keep_nyquist: must be 0 (reserved). */
typedef struct {
  int32_t n_fft;
  int32_t n_taps;
  const float* taps;
  int32_t keep_nyquist;
} qc_pfb_params;

/* F-engine alone (Sec. 4.2 "F-engine", Alg. 1 F-Engine step).
 *   x       : device int8, antenna stride ld_x bytes (ld_x >= n_samp, ld_x % 4 == 0,
 *             x 4-byte aligned).
 *   n_samp  : samples per antenna, a multiple of n_fft, below 2^31.
 *   hist    : device int8 [n_ant][(P-1)*N] samples preceding x, or NULL (zeros).
 *   hist_out: device int8 [n_ant][(P-1)*N] receives the last (P-1)*N samples of
 *             (hist ++ x) for the next call, or NULL.  May not alias hist.
 *   out_prec: QC_F32 -> out is cfloat [n_ant][n_spec][n_chan];
 *             QC_F16 / QC_BF16 -> out is pairs of 16-bit (re, im) in the same
 *             layout; QC_FP8_E4M3 -> pairs of E4M3 bytes.  For reduced
 *             precision each antenna's values are multiplied by the power of
 *             two scale_out[a] before rounding (round to nearest even,
 *             saturating at the format's largest finite value).
 *   scale_out: device float[n_ant], written when out_prec != QC_F32 (may be NULL
 *             for QC_F32).  s_a = 2^round(log2(target/rms_a)), rms_a =
 *             sqrt(mean(x_a^2) * sum h^2) over the first min(n_samp, 2^20)
 *             samples; target 256 (F16), 1 (BF16), 32 (E4M3). */
qc_status qc_pfb_channelize(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                            const qc_pfb_params* p, const int8_t* hist, int8_t* hist_out,
                            qc_prec out_prec, void* out, float* scale_out, void* stream);

/* Fused F+X from int8 (the hot path; Sec. 4.2, Alg. 1 F-Engine, X-Engine and
 * Integration steps).
 *   spec_per_dump: spectra integrated per dump (>= 1).
 *   x_prec  : QC_F32: the fused F+X kernel where a fused tile exists (2, 4 or
 *             8 antennas for the tabulated n_fft), else the F-engine then the
 *             FP32 X-engine.  QC_F16 / QC_BF16 / QC_FP8_E4M3: the F-engine
 *             writes requantised spectra (as qc_pfb_channelize), then the
 *             matrix-core X-engine (as qc_xcorrelate_chan); needs n_ant <= 32
 *             and n_chan % 32 == 0.  Work buffers come from the device's
 *             stream-ordered memory pool.
 *   vis     : device cfloat [n_dump][n_base][n_chan], n_dump = n_spec / spec_per_dump;
 *             a trailing partial dump is not integrated.
 *   accumulate: nonzero adds into vis, zero overwrites it.
 *   n_dumps_out: host int64* (or NULL) receives n_dump.
 * Deterministic: per-workgroup partial sums are reduced in a fixed order. */
qc_status qc_xcorrelate(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                        const qc_pfb_params* p, const int8_t* hist, int8_t* hist_out,
                        int64_t spec_per_dump, qc_prec x_prec, float* vis, int32_t accumulate,
                        int64_t* n_dumps_out, void* stream);

/* Input words of the acquisition chain (Sec. 3.3 quantisation modes; Sec.
 * 4.2: raw samples are unpacked into complex voltage streams).
 *   QC_SAMPLE_I8  : real int8 (the 8-bit truncated mode).
 *   QC_SAMPLE_I16 : real int16 (the default 16-bit padded mode: the 14-bit
 *                   ADC value stored in 16 bits, used as the integer it is).
 *   QC_SAMPLE_CI8 : complex int8, I and Q interleaved (2 bytes per sample).
 *   QC_SAMPLE_CI16: complex int16, I and Q interleaved (4 bytes per sample).
 * Real words give n_chan = N/2 channels k = 0..N/2-1; complex words an
 * N-point complex DFT with all n_chan = N channels k = 0..N-1 in natural
 * order (k >= N/2 are the negative frequencies).  The same real prototype
 * filters I and Q. */
typedef enum { QC_SAMPLE_I8 = 0, QC_SAMPLE_I16 = 1, QC_SAMPLE_CI8 = 2, QC_SAMPLE_CI16 = 3 } qc_sample;

/* F-engine of any input word (Sec. 4.2 "F-engine"; Sec. 3.3).  As
 * qc_pfb_channelize, except:
 *   x, hist, hist_out: device buffers of the word `sample`; ld_x and n_samp
 *     count samples (an I/Q pair is one sample); x and hist aligned to 4
 *     samples; hist / hist_out hold (P-1)*N samples per antenna.
 *   out: [n_ant][n_spec][n_chan] with n_chan as above.  Scales for reduced
 *     precision use mean |x|^2 (I^2 + Q^2 for complex words).
 *   QC_SAMPLE_I8 gives exactly qc_pfb_channelize's result. */
qc_status qc_pfb_channelize_ex(const void* x, int32_t sample, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                               const qc_pfb_params* p, const void* hist, void* hist_out, qc_prec out_prec,
                               void* out, float* scale_out, void* stream);

/* F+X of any input word (Sec. 4.1 eq. 1; Sec. 4.2; Sec. 3.3).  As
 * qc_xcorrelate with the word conventions of qc_pfb_channelize_ex; vis is
 * [n_dump][n_base][n_chan].  QC_SAMPLE_I8 calls qc_xcorrelate; other words
 * run the F-engine of the full dumps' spectra into a stream-ordered pool
 * buffer, then qc_xcorrelate_chan.  Reduced x_prec needs n_ant <= 32 and
 * n_chan % 32 == 0 (else QC_EUNSUPPORTED). */
qc_status qc_xcorrelate_ex(const void* x, int32_t sample, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                           const qc_pfb_params* p, const void* hist, void* hist_out, int64_t spec_per_dump,
                           qc_prec x_prec, float* vis, int32_t accumulate, int64_t* n_dumps_out,
                           void* stream);

/* File ingest (Alg. 1 with its reader threads, pinned buffers and bounded
 * DataQueue; Sec. 4.2 "Asynchronous I/O"; the batch-packets / queue-max
 * operating point of Sec. 6).
 *   paths: n_ant files, each the raw samples of one antenna (words of type
 *     `sample`, as qc_pfb_channelize_ex; no header).
 *   packet_samp: samples per antenna per packet; batch_packets: packets per
 *     GPU batch; queue_max: page-locked batch buffers the readers may fill
 *     ahead of the GPU (the bounded queue); n_readers: reader threads
 *     (antennas split round-robin); depth: device batch slots (1..16).
 *   A batch (packet_samp * batch_packets samples per antenna, a multiple of
 *   n_fft) either holds whole dumps or a whole number of batches make one
 *   dump.  Reader threads fill buffers in batch order; the calling thread
 *   copies each complete batch to the device on a copy stream and
 *   correlates it (F-engine, X-engine, integration, the filter history
 *   carried across batches) on a compute stream, overlapping reads, copies
 *   and compute.  vis: device cfloat [max_dumps][n_base][n_chan] receives
 *   the whole dumps found in every file (at most max_dumps; max_dumps < 0:
 *   no limit, then vis must hold every dump); n_chan as qc_pfb_channelize_ex.
 *   Synchronous: returns when the last dump is on the device.  Allocates its
 *   pinned buffers, device slots and streams per call (default priority). */
typedef struct {
  int32_t n_ant;
  int32_t sample;          /* qc_sample */
  int64_t packet_samp;
  int32_t batch_packets;
  int32_t queue_max;
  int32_t n_readers;
  int32_t depth;
  qc_pfb_params pfb;
  int64_t spec_per_dump;
} qc_ingest_config;
typedef struct {
  int64_t bytes;       /* input bytes correlated */
  int64_t batches;
  int64_t dumps;
  double wall_s;       /* first read to the end of the last computation */
  double read_s;       /* reader threads' time inside file reads (summed) */
  double h2d_s;        /* host-to-device copies (HIP events, summed) */
  double compute_s;    /* F+X per batch (HIP events, summed) */
  double wait_s;       /* consumer waiting for a complete buffer */
} qc_ingest_stats;
qc_status qc_ingest_run(const char* const* paths, const qc_ingest_config* cfg, float* vis, int64_t max_dumps,
                        qc_ingest_stats* stats);

/* Synthesis imaging of calibrated visibilities (Sec. 8.1: gridding,
 * Fourier inversion to the dirty image and synthesized beam, CLEAN).
 * n: image and grid size, a power of two; cell_rad: image pixel (radians);
 * the uv cell is du = 1 / (n cell_rad) wavelengths; grid cell (iu, iv) is
 * at u = (iu - n/2) du, v = (iv - n/2) du, image pixel (il, im) at
 * l = (il - n/2) cell, m = (im - n/2) cell.  All calls are asynchronous on
 * `stream` and allocate nothing.
 *
 * qc_image_grid: nearest-cell gridding.  u, v: device float [n_vis]
 *   (wavelengths); vis: device cfloat [n_vis]; weight: device float
 *   [n_vis] or NULL (1).  Cell iu = floor(u * n cell_rad + 1/2) + n/2
 *   (float64), likewise iv; the weighted visibility is added at (iu, iv)
 *   and its conjugate at (n - iu, n - iv); samples with a cell outside
 *   [0, n) are dropped.  grid: device cfloat [n][n] (indexed [iu][iv]),
 *   overwritten; wsum: device double[1] receives the total gridded weight
 *   (both copies).  64 <= n <= 4096.  Float32 atomic sums: the grid's
 *   rounding depends on the order of arrival.
 * qc_image_invert: image[il][im] = Re sum_{iu,iv} grid[iu][iv]
 *   exp(+2 pi i ((iu-n/2)(il-n/2) + (iv-n/2)(im-n/2)) / n) / wsum, so a unit
 *   point source at the phase centre peaks at 1 (with unit visibilities the
 *   result is the synthesized beam, peak at (n/2, n/2)).  work: device
 *   cfloat [2 n n] scratch; image: device float [n][n].  64 <= n <= 4096.
 * qc_image_clean: Hogbom CLEAN in place on residual (device float [n][n],
 *   the dirty image on entry) with the beam psf (device float [n][n], peak
 *   at (n/2, n/2)).  Each iteration takes the pixel of largest |residual|
 *   (ties: smallest flat index il*n + im), stops if that magnitude is below
 *   threshold or max_iter components are found, records flux
 *   g = gain * peak and the flat index in comp_flux / comp_pix (device
 *   [max_iter]), and subtracts g * psf[((p - peak + (n/2, n/2)) mod n] from
 *   every pixel p (the dirty image of gridded data is periodic over the
 *   field), product and difference each rounded to float32.  n_comp:
 *   device int32[1] receives the number of components.  One workgroup;
 *   2 <= n <= 8192, 0 < gain <= 1. */
qc_status qc_image_grid(const float* u, const float* v, const float* vis, const float* weight, int64_t n_vis,
                        int32_t n, double cell_rad, float* grid, double* wsum, void* stream);
qc_status qc_image_invert(const float* grid, const double* wsum, int32_t n, float* work, float* image,
                          void* stream);
qc_status qc_image_clean(float* residual, const float* psf, int32_t n, float gain, float threshold,
                         int32_t max_iter, int32_t* comp_pix, float* comp_flux, int32_t* n_comp, void* stream);

/* Prototype filters (Fig. pfb_fft compares an 8-tap Kaiser PFB, beta = 8,
 * with a plain rectangular-window FFT).  Writes P*N float taps, designed in
 * float64 and rounded once, to device memory `taps` (16-byte aligned) for
 * use as qc_pfb_params.taps; synchronises `stream`.
 *   QC_WINDOW_HANN  : the built-in Hann-windowed sinc (beta ignored).
 *   QC_WINDOW_KAISER: w[q] = I0(beta sqrt(1 - (2q/(L-1) - 1)^2)) / I0(beta),
 *                     h[q] = w[q] sinc((q - (L-1)/2)/N), unnormalised;
 *                     beta in [0, 100].
 *   QC_WINDOW_RECT  : h[q] = 1 (with P = 1, the plain FFT). */
typedef enum { QC_WINDOW_HANN = 0, QC_WINDOW_KAISER = 1, QC_WINDOW_RECT = 2 } qc_window;
qc_status qc_pfb_design_taps(int32_t n_fft, int32_t n_taps, int32_t window, double beta, float* taps,
                             void* stream);

/* qc_xcorrelate without device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Arguments, layouts, accumulate, n_dumps_out and
 * results as qc_xcorrelate with x_prec = QC_F32 (within the ordering of the
 * float32 partial sums), restricted to the shapes with a fused F+X kernel:
 * n_fft 512, 1024, 2048 or 4096 with 4 antennas, 1024 or 2048 with 8,
 * 1024 or 4096 with 2 (else QC_EUNSUPPORTED; nothing is launched).
 * Work memory is one device array of QC_NOALLOC_SCRATCH_BYTES inside the
 * library, per GPU, held until the process ends: FFT twiddles and the
 * built-in taps are rebuilt in it at every call, and dumps are correlated in
 * batches whose partial sums fit it (a batch inside the stream takes its
 * filter history from the stream).  No call allocates or frees device or
 * host memory.  Calls that overlap on one GPU (other streams or threads)
 * share that array and race: serialise them.  Sizes whose single dump does
 * not fit the array are rejected with QC_EUNSUPPORTED (none of the shapes
 * above reaches it). */
#define QC_NOALLOC_SCRATCH_BYTES (64ll << 20)
qc_status qc_xcorrelate_noalloc(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                                const qc_pfb_params* p, const int8_t* hist, int8_t* hist_out,
                                int64_t spec_per_dump, float* vis, int32_t accumulate,
                                int64_t* n_dumps_out, void* stream);

/* X-engine alone from channelised voltages as written by qc_pfb_channelize
 * (Sec. 4.1 eq. 1; Sec. 4.2 X-engine and integration).
 *   v      : device [n_ant][n_spec][n_chan] (re, im) pairs of type prec.
 *   scale  : device float[n_ant] per-antenna scales for reduced precision
 *            (visibilities are divided by scale_i*scale_j), NULL for QC_F32.
 *   QC_F32 runs on the vector ALUs; QC_F16 / QC_BF16 / QC_FP8_E4M3 run on the
 *   matrix cores with float32 accumulation.
 *   vis    : device cfloat [n_spec/spec_per_dump][n_base][n_chan]. */
qc_status qc_xcorrelate_chan(const void* v, qc_prec prec, const float* scale, int32_t n_ant,
                             int64_t n_spec, int32_t n_chan, int64_t spec_per_dump,
                             float* vis, int32_t accumulate, void* stream);

/* MAD flagging (Sec. 7 eq. 2).
 *   vis        : device cfloat [n_time][n_base][n_chan].
 *   sigma      : threshold in units of 1.4826*MAD (the paper uses 5).
 *   population : 0 = per baseline over its (time x channel) plane;
 *                1 = per (baseline, channel) over time;
 *                2 = per (baseline, time) over channel.
 *   mask       : device uint8, same shape as vis; 1 = flagged (A > T).
 *   thresh_out : device double [n_base] (population 0), [n_base][n_chan] (1) or
 *                [n_time][n_base] (2), or NULL.
 * Amplitudes are |V| formed in float64 and rounded once to float32; medians,
 * the MAD and T = med + (sigma*1.4826)*MAD are float64, the even-count median
 * is the mean of the two middle values, and MAD = 0 gives T = median.
 * Populations of more than 36864 values take a work buffer of 4 bytes per
 * visibility from the stream-ordered memory pool. */
qc_status qc_mad_flag(const float* vis, int64_t n_time, int64_t n_base, int32_t n_chan,
                      float sigma, int32_t population, uint8_t* mask, double* thresh_out,
                      void* stream);

/* In-place per-antenna delay and phase correction (Sec. 4.1 step 2, eq. 1;
 * Sec. 7 delay/phase correction).  For b = (i, j) and channel k:
 *   V[t][b][k] *= exp(+i [2 pi f_k (tau_i - tau_j) + (phi_i - phi_j)]),
 *   f_k = f0_hz + k * df_hz.
 *   tau_s, phi_rad: HOST double[n_ant], copied before the call returns.
 * The phase is formed in float64 (cycles reduced modulo 1 before sin/cos). */
qc_status qc_apply_delay_phase(float* vis, int64_t n_time, int32_t n_ant, int32_t n_chan,
                               double f0_hz, double df_hz, const double* tau_s,
                               const double* phi_rad, void* stream);

/* Delay and phase calibration solve (Sec. 7, the three serial steps: coarse
 * group delay from the delay-spectrum peak, fine delay from a weighted fit
 * of unwrapped phase against frequency in a clean band (eq. 3), residual
 * phase from the band's mean complex vector).  Per baseline the visibilities
 * are summed over time with flagged cells (mask != 0) left out; the delay
 * spectrum has n_lag lags, the smallest power of two >= lag_pad*n_chan, at
 * most 8192 (and at least n_chan).  Phases and the delay spectrum are
 * float32; the least-squares sums and solves are float64.  The per-antenna
 * solution is the float64 least-squares fit of tau_i - tau_j over the cross
 * baselines with tau_ref = phi_ref = 0, in the sign convention of
 * qc_apply_delay_phase (applying the result flattens the phases).
 *   vis   : device cfloat [n_time][n_ant(n_ant+1)/2][n_chan]; mask: device
 *           uint8 of the same shape, or NULL.
 *   band  : channels [chan_lo, chan_hi), at least two.
 *   tau_s, phi_rad: HOST double[n_ant] outputs.  Synchronises `stream`.
 *   2 <= n_ant <= 64, 4 <= n_chan <= 4096. */
qc_status qc_solve_delay_phase(const float* vis, const uint8_t* mask, int64_t n_time, int32_t n_ant,
                               int32_t n_chan, double f0_hz, double df_hz, int32_t ref_ant,
                               int32_t chan_lo, int32_t chan_hi, int32_t lag_pad, double* tau_s,
                               double* phi_rad, void* stream);

/* Batched plans: several arrays (antenna counts, channel counts, dumps of
 * their own) correlated together, with the same float32 sums as
 * qc_xcorrelate (built-in Hann-sinc taps).  Alg. 1 runs the same
 * F-X-integrate steps per array; the plan's tuned knobs play the role of the
 * paper's batch-packets / queue-max operating point (Sec. 6).
 *
 * Modes (qc_plan_set_mode):
 *   QC_PLAN_GRAPH (default): per array, the fused F+X kernel and its
 *     fixed-order reduction (arrays of 2, 4 or 8 antennas with a fused tile
 *     for their n_fft), or F-engine, FP32 X-engine and reduction, into
 *     plan-owned buffers.  With `concurrent` set, every array runs on a
 *     stream of its own between a fork and a join event on the caller's
 *     stream, so a captured graph holds the arrays as independent branches.
 *   QC_PLAN_PERSISTENT: every array's work in one persistent launch (256
 *     workgroups of 512 threads) that claims work items from one ordered
 *     queue: fused F+X items (2, 4 or 8 antennas at their fused sizes),
 *     F-engine items (the ring F-engine at n_fft 4096 / 8192 with 4 taps,
 *     else the plain one), FP32 X-engine items (matrix cores for 5..32
 *     antennas, else the vector ALU) and reductions.  An item that needs others (X-engine after its array's
 *     F-engine, reduction after its partials) waits for their done counter,
 *     bounded in time (qc_plan_set_wait_timeout); on expiry the item is
 *     skipped, an error flag is set that qc_plan_check reports, and every
 *     later wait gives up at once, so the launch always drains.  Reductions
 *     scale like qc_xcorrelate's, so both modes give the same float32 sums
 *     up to the grouping of partial sums.
 *
 *   qc_plan_create: n_arrays in [1, 8]; each array 1..64 antennas, n_fft a
 *     power of two in [16, 8192], n_samp a multiple of n_fft (< 2^31), at
 *     least one full dump.  Allocates device buffers, streams and events
 *     (default priority); synchronises.
 *   qc_plan_execute: x[i]: device int8 [n_ant][n_samp] (contiguous); vis[i]:
 *     device cfloat [n_dump][n_base][n_chan], overwritten.  Asynchronous with
 *     respect to the host; ordered on `stream` (work forked to the plan's
 *     streams is joined back to it).  Executions of one plan share its
 *     buffers: issue them on one stream.
 *   qc_plan_check: synchronises `stream`; in the persistent mode QC_ESTATE
 *     if a bounded dependency wait expired in the last execution.
 *   qc_plan_set_wait_timeout / qc_plan_set_wait_bias: persistent mode only
 *     (time limit of one dependency wait in microseconds, default 2 s; test
 *     hook that makes every wait target unreachable).
 *   qc_plan_capture_graph: captures one execution (fixed x / vis pointers)
 *     on a non-default stream into a hipGraph; qc_plan_replay launches it,
 *     also on a non-default stream (QC_EINVAL on the legacy default stream).
 *     Changing the mode or re-tuning drops the graph.
 *   qc_plan_autotune: graph mode; times executions over the knobs
 *     (concurrency; per array the fused tile and the split: chunks per dump
 *     of the fused kernel or k-split of the X-engine) by coordinate descent
 *     and keeps the fastest.  With cache_path (or NULL) a previous result for
 *     the same arrays is reused (*from_cache = 1) and new results appended.
 *     Synchronises.
 *   qc_plan_execute_separate: the same work as separate qc_xcorrelate calls
 *     (for comparison).
 *   qc_plan_info: launches per execution, the concurrency flag, and per
 *     array the fused tile (-1 for the two-pass path) and the split; any
 *     output may be NULL (tiles and splits hold n_arrays entries). */
typedef struct qc_plan qc_plan;
typedef struct {
  int32_t n_ant;
  int64_t n_samp;
  int32_t n_fft;
  int32_t n_taps;
  int64_t spec_per_dump;
} qc_array_desc;
enum { QC_PLAN_GRAPH = 0, QC_PLAN_PERSISTENT = 1 };
qc_status qc_plan_create(const qc_array_desc* arrays, int32_t n_arrays, qc_plan** out);
qc_status qc_plan_set_mode(qc_plan* plan, int32_t mode);
qc_status qc_plan_execute(qc_plan* plan, const int8_t* const* x, float* const* vis, void* stream);
qc_status qc_plan_check(qc_plan* plan, void* stream);
qc_status qc_plan_set_wait_timeout(qc_plan* plan, int64_t microseconds);
qc_status qc_plan_set_wait_bias(qc_plan* plan, int32_t bias);
qc_status qc_plan_capture_graph(qc_plan* plan, const int8_t* const* x, float* const* vis, void* stream);
qc_status qc_plan_replay(qc_plan* plan, void* stream);
qc_status qc_plan_autotune(qc_plan* plan, const int8_t* const* x, float* const* vis, int32_t reps,
                           const char* cache_path, int32_t* from_cache, void* stream);
qc_status qc_plan_execute_separate(qc_plan* plan, const int8_t* const* x, float* const* vis,
                                   void* stream);
qc_status qc_plan_info(const qc_plan* plan, int32_t* n_launches, int32_t* concurrent, int32_t* tiles,
                       int64_t* splits);
void qc_plan_destroy(qc_plan* plan);

/* Streaming ingest (Alg. 1: pinned host buffers, asynchronous host-to-device
 * copies on a stream, then F-engine, X-engine and integration; Sec. 4.2
 * "Asynchronous I/O").  The library owns a ring of `depth` device slots, a
 * copy stream and a compute stream, and carries the PFB history between
 * chunks, so a chunked stream gives the spectra of one long stream.
 *   qc_stream_create: chunk_samp samples per antenna per chunk (a multiple of
 *     n_fft holding a whole number of dumps).  Synchronises once.
 *   qc_stream_push: host_chunk is int8 [n_ant][chunk_samp] in page-locked host
 *     memory; it must stay unchanged until qc_stream_wait_copied(st, seq) or
 *     qc_stream_sync returns.  seq must increase; a gap (seq != previous + 1)
 *     marks dropped chunks and restarts the filter history from zeros.
 *     host_chunk NULL pushes chunk seq as dropped: its samples count as
 *     zeros, vis_out is zero-filled and the next chunk starts from a zero
 *     history.  vis_out: device cfloat [chunk dumps][n_base][n_chan],
 *     written on the compute stream.  n_dumps_out: host, or NULL.
 *     Asynchronous.
 *   qc_stream_valid_spectra: host int64 n_valid[n] receives, per dump of the
 *     last pushed chunk, the spectra whose whole FIR window (their block and
 *     the P-1 before it) holds received samples: spec_per_dump, less the
 *     first P-1 spectra after a zero-filled history (stream start, a gap, a
 *     dropped chunk), and 0 for a dropped chunk.  A weight for averaging
 *     dumps; the visibilities themselves are not rescaled.
 *   qc_stream_wait_copied: blocks until chunk seq has reached the device.
 *   qc_stream_sync: blocks until all pushed work is done.
 *   qc_stream_compute_stream: the hipStream_t (as void*) results are written on.
 *   qc_stream_last_error: thread-local detail of the last streaming failure. */
typedef struct qc_stream qc_stream;
qc_status qc_stream_create(int32_t n_ant, int64_t chunk_samp, const qc_pfb_params* p,
                           int64_t spec_per_dump, int32_t depth, qc_stream** out);
qc_status qc_stream_push(qc_stream* st, const int8_t* host_chunk, int64_t seq, float* vis_out,
                         int64_t* n_dumps_out);
qc_status qc_stream_valid_spectra(const qc_stream* st, int64_t* n_valid, int64_t n);
qc_status qc_stream_wait_copied(qc_stream* st, int64_t seq);
qc_status qc_stream_sync(qc_stream* st);
void* qc_stream_compute_stream(qc_stream* st);
void qc_stream_destroy(qc_stream* st);
const char* qc_stream_last_error(void);

/* Tile shape of the fused F+X kernel for one (n_fft, n_ant): an index into a
 * fixed list of shapes (spectra in flight, values per thread per FFT pass,
 * ping-pong LDS buffers).  Every shape computes the same sums; shapes differ
 * in speed only.  Index 0 is the default.  qc_fx_tile_count returns 0 when
 * no fused kernel exists for the pair.  The choice is process-wide and is
 * what the autotuner sets. */
int32_t qc_fx_tile_count(int32_t n_fft, int32_t n_ant);
qc_status qc_fx_set_tile(int32_t n_fft, int32_t n_ant, int32_t tile);
int32_t qc_fx_get_tile(int32_t n_fft, int32_t n_ant);
/* Launch width of qc_xcorrelate's fused F+X kernel for one (n_fft, n_ant):
 * the number of workgroups a launch aims at, by splitting each dump into
 * chunks of spectra whose partial visibilities the fixed-order reduction
 * sums (each chunk keeps at least 8 spectra).  0 restores the default of
 * 512; otherwise 1..2^20 (QC_EINVAL beyond; QC_EUNSUPPORTED when no fused
 * kernel exists for the pair).  Sums are equal up to float32 rounding order
 * whatever the width.  Process-wide; set by the autotuner. */
qc_status qc_fx_set_width(int32_t n_fft, int32_t n_ant, int64_t workgroups);
int64_t qc_fx_get_width(int32_t n_fft, int32_t n_ant);
/* Autotuner for the fused kernel: times every tile shape of (n_fft, n_ant) on
 * the caller's input (reps calls of qc_xcorrelate each, after one untimed
 * call) with HIP events on `stream` at the default width, then the fastest
 * tile at one and at four workgroups per compute unit of the current device;
 * keeps the fastest pair via qc_fx_set_tile and qc_fx_set_width and returns
 * the tile's index in *best_out (host).  vis: device scratch sized for the
 * output of qc_xcorrelate on this input.  ms_per_tile: host double[cap] for
 * the per-tile average times at the default width, or NULL.  Synchronises. */
qc_status qc_fx_autotune(const int8_t* x, int64_t ld_x, int32_t n_ant, int64_t n_samp,
                         const qc_pfb_params* p, int64_t spec_per_dump, int32_t reps, float* vis,
                         double* ms_per_tile, int32_t cap, int32_t* best_out, void* stream);

/* Kernel timing for measurement harnesses.  qc_timing_enable(mode) starts a
 * fresh record, qc_timing_enable(0) stops recording; qc_timing_read
 * synchronises on the recorded events and returns the summed duration in
 * milliseconds and the launch count of the calls timed under each id below.
 * Mode 1: each timed call is bracketed by two HIP events recorded on the
 *   stream it runs on (the figure is the call's own duration; each event is a
 *   packet of its own, which adds a few microseconds between launches).
 * Mode 2 (chained): every kernel the library launches carries a stop event
 *   bound to the launch itself (no extra packet, so the launches run as they
 *   would untimed).  A timed call runs from the end of the library's previous
 *   kernel on the same stream (or from an event recorded just before it when
 *   there is none since timing was enabled) to the end of its own last
 *   kernel.  Work the caller enqueues on that stream between library calls,
 *   and time the stream sits idle waiting for the host, are therefore counted
 *   in the next call's figure: use it where the stream runs library calls
 *   only and the host enqueues ahead of the GPU.  The events carry no
 *   system-scope fence (they serve timing only).  Launches made while the
 *   stream is being captured into a graph are not timed.
 * Every recorded event is kept (for qc_timing_read) until timing is next
 * enabled: enable it for bounded measurement windows.
 * Any other mode is QC_EINVAL.  Not thread-safe with respect to concurrent
 * enable/read. */
enum {
  QC_KERNEL_FX_FUSED = 0,   /* fused F+X (int8 -> per-chunk partial visibilities) */
  QC_KERNEL_CHANNELIZE = 1, /* standalone F-engine */
  QC_KERNEL_XENG_F32 = 2,   /* X-engine, vector ALUs */
  QC_KERNEL_XENG_MFMA = 3,  /* X-engine, matrix cores */
  QC_KERNEL_REDUCE = 4,     /* fixed-order partial reduction */
  QC_KERNEL_MAD = 5,        /* MAD flagging */
  QC_KERNEL_APPLY = 6,      /* delay/phase application */
  QC_KERNEL_COUNT = 7
};
qc_status qc_timing_enable(int32_t on);
qc_status qc_timing_read(int32_t kernel, double* total_ms, int64_t* launches);

/* F-engine kernel choice (process-wide; not thread-safe against concurrent
 * calls): 0 (default) uses the register-ring kernel where it applies (P = 4,
 * built-in taps, n_fft 1024..4096: the fused ring tile's FIR and transform,
 * writing spectra out), 1 always the plain kernel.  Both compute the same
 * sums (Sec. 4.2 F-engine); the choice only affects speed.  Used by
 * qc_pfb_channelize and the two-pass paths of qc_xcorrelate. */
qc_status qc_channelize_set_variant(int32_t variant);
int32_t qc_channelize_get_variant(void);

/* Float32 X-engine kernel choice (process-wide; not thread-safe against
 * concurrent calls).  The matrix-core kernel forms each channel's Gram
 * matrix on 16 x 16 tiles with v_mfma_f32_16x16x4_f32 up to 16 antennas
 * and on 32 x 32 tiles with v_mfma_f32_32x32x2_f32 above (needs
 * n_ant <= 32, n_chan % 16 == 0 and v 16-byte aligned); the vector-ALU
 * kernel takes 4 x 4 antenna blocks per thread and serves every shape.
 * 0 (default): matrix cores for 5..32 antennas, where the fixed tile cost
 * beats the block pairs; 1: always the vector ALU; 2: matrix cores
 * wherever supported.  Both sum the same products in float32 (Sec. 4.1 eq. 1); the
 * choice affects rounding order and speed only.  Used by
 * qc_xcorrelate_chan (QC_F32), the two-pass path of qc_xcorrelate and
 * batched plans. */
qc_status qc_xengine_set_variant(int32_t variant);
int32_t qc_xengine_get_variant(void);

/* Learned RFI flagger beside MAD.  MAD thresholds visibility amplitude
 * (Sec. 7, eq. 2); RFI is structured in time and frequency (Sec. 5: lines,
 * bursts).  A four-layer convolutional network over one baseline's
 * (time x channel) amplitude plane learns that structure:
 *   L1 3x3 1->32 ReLU, L2 5x5 32->32 ReLU, L3 5x5 dilation 2 32->32 ReLU,
 *   L4 1x1 32->1 logit; stride 1, zero 'same' padding, cross-correlation.
 * Parameters: device float32[qc_cnn_param_count()] = W1[32][1][3][3], b1[32],
 * W2[32][32][5][5], b2[32], W3[32][32][5][5], b3[32], W4[1][32][1][1], b4[1].
 * Activations are float32, accumulation float32.
 *   qc_cnn_normalize: vis [n_time][n_base][n_chan] cfloat -> x, device float
 *     [n_base][n_time][n_chan]: A = |V| (float32), r = (A - med)/(1.4826 MAD)
 *     over the baseline's plane (exact order statistics, scale 1 if MAD = 0),
 *     x = sign(r) log1p|r|.
 *   qc_cnn_forward: x [n_img][H][W] -> logits [n_img][H][W].  act_prec 0:
 *     float32 activations on the vector ALUs; 1: half activations with
 *     float32 accumulation, L2 and L3 on the matrix cores (inference only).
 *   qc_cnn_grad: mean over cells of the binary cross-entropy of the logits
 *     against labels (uint8 [n_img][H][W], nonzero = RFI), positives weighted
 *     by pos_weight; writes the gradient (float[param_count]) and the loss
 *     (one float), both device memory.  Deterministic.
 *   qc_cnn_adam: Adam with bias correction, step >= 1; m, v: device float
 *     [param_count], zero before step 1.
 *   qc_cnn_train_step: qc_cnn_grad then qc_cnn_adam (beta 0.9/0.999, eps 1e-8).
 *   qc_cnn_flag: normalise, forward (act_prec as for qc_cnn_forward) and
 *     flag (logit > logit_threshold) every baseline; mask: device uint8
 *     [n_time][n_base][n_chan] like qc_mad_flag.
 * All asynchronous on `stream`; n_img*H*W and n_time*n_chan below 2^31. */
int32_t qc_cnn_param_count(void);
qc_status qc_cnn_normalize(const float* vis, int64_t n_time, int64_t n_base, int32_t n_chan, float* x,
                           void* stream);
qc_status qc_cnn_forward(const float* params, const float* x, int32_t n_img, int32_t height,
                         int32_t width, int32_t act_prec, float* logits, void* stream);
qc_status qc_cnn_grad(const float* params, const float* x, const uint8_t* labels, int32_t n_img,
                      int32_t height, int32_t width, float pos_weight, float* grad, float* loss,
                      void* stream);
qc_status qc_cnn_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr,
                      float beta1, float beta2, float eps, void* stream);
qc_status qc_cnn_train_step(float* params, float* m, float* v, int64_t step, const float* x,
                            const uint8_t* labels, int32_t n_img, int32_t height, int32_t width,
                            float pos_weight, float lr, float* loss, void* stream);
qc_status qc_cnn_flag(const float* params, const float* vis, int64_t n_time, int64_t n_base,
                      int32_t n_chan, float logit_threshold, int32_t act_prec, uint8_t* mask,
                      void* stream);

/* Kernel choice for the flagger's float32 work (the two 32 -> 32 layers'
 * convolutions forward and backward-data, and the weight gradients of L1,
 * L2 and L3), used by
 * qc_cnn_forward (act_prec 0), qc_cnn_grad, qc_cnn_train_step and qc_cnn_flag
 * (act_prec 0); process-wide, not thread-safe against concurrent calls.
 * 0 (default): the matrix cores, v_mfma_f32_32x32x2_f32 (convolution: per
 * tap, a 32 x 32 weight block times the shifted input; weight gradient: per
 * tap, the output gradient times the shifted input over the pixels, for L1
 * all 9 taps and the bias in one product);
 * 1: the vector ALU.  Both are float32 throughout and deterministic; the
 * choice affects rounding order and speed only. */
qc_status qc_cnn_set_variant(int32_t variant);
int32_t qc_cnn_get_variant(void);

/* Measurement helper, not part of the method: the rate that one kernel of
 * the given kind sustains on this GPU, so that the library's kernels can be
 * read against what the hardware delivers as well as against its published
 * peaks.  One warm-up launch, then `reps` back-to-back launches timed with
 * HIP events on `stream`; synchronous.
 *   QC_PEAK_HBM_READ: streaming read of `bytes` of scratch, GB/s;
 *   QC_PEAK_HBM_COPY: copy of the first half of scratch into the second,
 *     GB/s of bytes read plus written;
 *   QC_PEAK_VALU_F32: independent float32 FMAs, scalar instructions (the
 *     library is built without packed FP32), TFLOP/s;
 *   QC_PEAK_MFMA_F32: v_mfma_f32_32x32x2_f32, TFLOP/s;
 *   QC_PEAK_MFMA_F16: v_mfma_f32_32x32x16_f16, TFLOP/s.
 * scratch: device memory, 16-byte aligned, `bytes` long: at least 64 MiB
 * for the two memory kinds (larger reads the steady state better), at
 * least 64 KiB for the others (written only in a case that cannot occur,
 * which keeps the results live).  QC_EINVAL on a bad kind, pointer, size or
 * reps, before any GPU work. */
enum {
  QC_PEAK_HBM_READ = 0,
  QC_PEAK_HBM_COPY = 1,
  QC_PEAK_VALU_F32 = 2,
  QC_PEAK_MFMA_F32 = 3,
  QC_PEAK_MFMA_F16 = 4
};
qc_status qc_measure_peak(int32_t kind, void* scratch, int64_t bytes, int32_t reps, double* rate,
                          void* stream);

/* Human-readable name of a status code (static storage). */
const char* qc_status_string(qc_status s);
/* Thread-local detail of the last failure in this thread ("" if none). */
const char* qc_last_error(void);
/* Library version string (static storage). */
const char* qc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QC_H */
