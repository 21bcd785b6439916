// Streaming ingest (arXiv 2604.20640 Alg. 1 and Sec. 4.2 "Asynchronous I/O"):
// chunks of every antenna's stream arrive in page-locked host memory, are
// copied to the device on a copy stream, and are correlated on a compute
// stream while the next copy proceeds.  The PFB history ((P-1)*N samples per
// antenna) is carried from chunk to chunk on the device, so a chunked
// stream gives the same spectra as one long stream.
//
// Ordering: a ring of `depth` device slots.  The copy into slot s waits for
// the compute that last read slot s; the compute on slot s waits for its
// copy.  Both streams are created by the library with default priority.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "qc.h"

struct qc_stream {
  int32_t n_ant = 0;
  int64_t chunk_samp = 0;
  qc_pfb_params pfb{};
  int64_t spec_per_dump = 0;
  int32_t depth = 0;
  int device = 0;
  hipStream_t copy = nullptr, compute = nullptr;
  std::vector<int8_t*> slot;
  std::vector<hipEvent_t> copied, computed;
  int8_t* hist[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t pushed = 0;
  int64_t last_seq = -1;
  std::vector<int64_t> slot_seq;
  // the next chunk's filter history is zero-filled (stream start, a gap in
  // the sequence, or a dropped chunk before it)
  bool fresh = true;
  std::vector<int64_t> valid;  // valid spectra per dump of the last chunk
};

namespace {
thread_local std::string g_serr;

qc_status sfail(qc_status s, const char* msg, hipError_t e = hipSuccess) {
  g_serr = msg;
  if (e != hipSuccess) {
    g_serr += ": ";
    g_serr += hipGetErrorString(e);
  }
  return s;
}

void release(qc_stream* st) {
  if (!st) return;
  for (auto p : st->slot)
    if (p) (void)hipFree(p);
  for (auto e : st->copied)
    if (e) (void)hipEventDestroy(e);
  for (auto e : st->computed)
    if (e) (void)hipEventDestroy(e);
  for (auto h : st->hist)
    if (h) (void)hipFree(h);
  if (st->copy) (void)hipStreamDestroy(st->copy);
  if (st->compute) (void)hipStreamDestroy(st->compute);
  delete st;
}
}  // namespace

namespace {
// Valid spectra per dump: a spectrum counts when its whole FIR window (its
// block and the P-1 before it) holds received samples.  After a zero-filled
// history the chunk's first P-1 spectra do not.
void count_valid(qc_stream* st, bool fresh, bool dropped) {
  const int64_t spd = st->spec_per_dump;
  const int64_t n_dump = (st->chunk_samp / st->pfb.n_fft) / spd;
  st->valid.assign((size_t)n_dump, dropped ? 0 : spd);
  if (dropped || !fresh) return;
  int64_t bad = st->pfb.n_taps - 1;
  for (int64_t d = 0; d < n_dump && bad > 0; ++d) {
    const int64_t k = bad < spd ? bad : spd;
    st->valid[(size_t)d] -= k;
    bad -= k;
  }
}

// A dropped chunk: its samples count as zeros.  Its dumps are written as
// zero visibilities with no valid spectrum, and the history the next chunk
// starts from is zeros.
qc_status push_dropped(qc_stream* st, int64_t seq, float* vis_out, int64_t* n_dumps_out) {
  const int64_t N = st->pfb.n_fft, spd = st->spec_per_dump;
  const int64_t n_dump = (st->chunk_samp / N) / spd;
  const size_t vbytes = sizeof(float) * 2 * (size_t)n_dump * ((size_t)st->n_ant * (st->n_ant + 1) / 2) *
                        (size_t)(N / 2);
  const size_t hbytes = (size_t)st->n_ant * (size_t)(st->pfb.n_taps - 1) * N;
  hipError_t e = hipMemsetAsync(vis_out, 0, vbytes, st->compute);
  if (e == hipSuccess && hbytes) e = hipMemsetAsync(st->hist[st->cur], 0, hbytes, st->compute);
  if (e != hipSuccess) return sfail(QC_EHIP, "zero fill", e);
  count_valid(st, true, true);
  if (n_dumps_out) *n_dumps_out = n_dump;
  st->fresh = true;
  st->last_seq = seq;
  return QC_OK;
}
}  // namespace

extern "C" {

const char* qc_stream_last_error(void) { return g_serr.c_str(); }

qc_status qc_stream_create(int32_t n_ant, int64_t chunk_samp, const qc_pfb_params* p,
                           int64_t spec_per_dump, int32_t depth, qc_stream** out) {
  g_serr.clear();
  if (!out || !p) return sfail(QC_EINVAL, "NULL argument");
  *out = nullptr;
  if (n_ant < 1 || n_ant > 4096) return sfail(QC_EINVAL, "n_ant must be in [1, 4096]");
  if (depth < 1 || depth > 64) return sfail(QC_EINVAL, "depth must be in [1, 64]");
  if (p->n_fft < 4 || p->n_fft > 8192 || (p->n_fft & (p->n_fft - 1)))
    return sfail(QC_EINVAL, "n_fft must be a power of two in [4, 8192]");
  if (p->n_taps < 1 || p->n_taps > 16) return sfail(QC_EINVAL, "n_taps must be in [1, 16]");
  if (chunk_samp <= 0 || chunk_samp % p->n_fft) return sfail(QC_EINVAL, "chunk_samp must be a positive multiple of n_fft");
  if (spec_per_dump < 1 || (chunk_samp / p->n_fft) % spec_per_dump)
    return sfail(QC_EINVAL, "a chunk must hold a whole number of dumps");
  qc_stream* st = new (std::nothrow) qc_stream();
  if (!st) return sfail(QC_ENOMEM, "host allocation");
  st->n_ant = n_ant;
  st->chunk_samp = chunk_samp;
  st->pfb = *p;
  st->spec_per_dump = spec_per_dump;
  st->depth = depth;
  hipError_t e = hipGetDevice(&st->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&st->copy, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&st->compute, hipStreamNonBlocking);
  if (e != hipSuccess) {
    release(st);
    return sfail(QC_EHIP, "stream creation", e);
  }
  st->slot.assign(depth, nullptr);
  st->copied.assign(depth, nullptr);
  st->computed.assign(depth, nullptr);
  st->slot_seq.assign(depth, -1);
  const size_t slot_bytes = (size_t)n_ant * (size_t)chunk_samp;
  for (int i = 0; i < depth; ++i) {
    e = hipMalloc(&st->slot[i], slot_bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st->copied[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st->computed[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      release(st);
      return sfail(e == hipErrorOutOfMemory ? QC_ENOMEM : QC_EHIP, "slot allocation", e);
    }
  }
  const size_t hbytes = (size_t)n_ant * (size_t)(p->n_taps - 1) * p->n_fft;
  for (int i = 0; i < 2; ++i) {
    e = hipMalloc(&st->hist[i], hbytes ? hbytes : 4);
    if (e == hipSuccess && hbytes) e = hipMemsetAsync(st->hist[i], 0, hbytes, st->compute);
    if (e != hipSuccess) {
      release(st);
      return sfail(QC_EHIP, "history allocation", e);
    }
  }
  e = hipStreamSynchronize(st->compute);
  if (e != hipSuccess) {
    release(st);
    return sfail(QC_EHIP, "stream synchronise", e);
  }
  *out = st;
  return QC_OK;
}


qc_status qc_stream_push(qc_stream* st, const int8_t* host_chunk, int64_t seq, float* vis_out,
                         int64_t* n_dumps_out) {
  g_serr.clear();
  if (!st || !vis_out) return sfail(QC_EINVAL, "NULL argument");
  if (seq <= st->last_seq) return sfail(QC_ESTATE, "sequence numbers must increase");
  if (!host_chunk) return push_dropped(st, seq, vis_out, n_dumps_out);
  const int s = (int)(st->pushed % st->depth);
  const size_t bytes = (size_t)st->n_ant * (size_t)st->chunk_samp;
  const size_t hbytes = (size_t)st->n_ant * (size_t)(st->pfb.n_taps - 1) * st->pfb.n_fft;
  const bool gap = st->last_seq >= 0 && seq != st->last_seq + 1;
  hipError_t e;
  // the copy into slot s may start once the compute that last read it is done
  if (st->slot_seq[s] >= 0) {
    e = hipStreamWaitEvent(st->copy, st->computed[s], 0);
    if (e != hipSuccess) return sfail(QC_EHIP, "wait", e);
  }
  e = hipMemcpyAsync(st->slot[s], host_chunk, bytes, hipMemcpyHostToDevice, st->copy);
  if (e != hipSuccess) return sfail(QC_EHIP, "host-to-device copy", e);
  e = hipEventRecord(st->copied[s], st->copy);
  if (e != hipSuccess) return sfail(QC_EHIP, "event", e);
  e = hipStreamWaitEvent(st->compute, st->copied[s], 0);
  if (e != hipSuccess) return sfail(QC_EHIP, "wait", e);
  // a gap in the sequence: the samples before this chunk are unknown, so the
  // filter history restarts from zero (as at the start of a stream)
  if (gap && hbytes) {
    e = hipMemsetAsync(st->hist[st->cur], 0, hbytes, st->compute);
    if (e != hipSuccess) return sfail(QC_EHIP, "history reset", e);
  }
  const int nxt = 1 - st->cur;
  qc_status q = qc_xcorrelate(st->slot[s], st->chunk_samp, st->n_ant, st->chunk_samp, &st->pfb,
                              hbytes ? st->hist[st->cur] : nullptr, hbytes ? st->hist[nxt] : nullptr,
                              st->spec_per_dump, QC_F32, vis_out, 0, n_dumps_out, st->compute);
  if (q != QC_OK) return sfail(q, qc_last_error());
  e = hipEventRecord(st->computed[s], st->compute);
  if (e != hipSuccess) return sfail(QC_EHIP, "event", e);
  count_valid(st, st->fresh || gap, false);
  st->fresh = false;
  st->cur = nxt;
  st->slot_seq[s] = seq;
  st->last_seq = seq;
  ++st->pushed;
  return QC_OK;
}

qc_status qc_stream_valid_spectra(const qc_stream* st, int64_t* n_valid, int64_t n) {
  g_serr.clear();
  if (!st || !n_valid || n < 0) return sfail(QC_EINVAL, "NULL argument or negative count");
  if (st->last_seq < 0) return sfail(QC_ESTATE, "no chunk pushed yet");
  for (int64_t d = 0; d < n && d < (int64_t)st->valid.size(); ++d) n_valid[d] = st->valid[(size_t)d];
  return QC_OK;
}

qc_status qc_stream_wait_copied(qc_stream* st, int64_t seq) {
  g_serr.clear();
  if (!st) return sfail(QC_EINVAL, "NULL stream");
  for (int s = 0; s < st->depth; ++s) {
    if (st->slot_seq[s] == seq) {
      hipError_t e = hipEventSynchronize(st->copied[s]);
      return e == hipSuccess ? QC_OK : sfail(QC_EHIP, "event synchronise", e);
    }
  }
  return QC_OK;  // long since copied (its slot was reused)
}

qc_status qc_stream_sync(qc_stream* st) {
  g_serr.clear();
  if (!st) return sfail(QC_EINVAL, "NULL stream");
  hipError_t e = hipStreamSynchronize(st->copy);
  if (e == hipSuccess) e = hipStreamSynchronize(st->compute);
  return e == hipSuccess ? QC_OK : sfail(QC_EHIP, "stream synchronise", e);
}

void* qc_stream_compute_stream(qc_stream* st) { return st ? (void*)st->compute : nullptr; }

void qc_stream_destroy(qc_stream* st) {
  if (!st) return;
  (void)hipStreamSynchronize(st->copy);
  (void)hipStreamSynchronize(st->compute);
  release(st);
}

}  // extern "C"
