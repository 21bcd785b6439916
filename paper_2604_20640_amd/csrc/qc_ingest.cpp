// File ingest (arXiv 2604.20640 Alg. 1 and Sec. 4.2 "Asynchronous I/O";
// the batch-packets / queue-max operating point of Sec. 6).
//
// Producer side: reader threads copy each antenna's raw samples, one batch
// of `batch_packets` packets at a time, into page-locked host buffers
// ("PinnedBuffer_i" of Alg. 1).  There are `queue_max` buffers, used as a
// ring: batch b fills buffer b mod queue_max once the consumer has released
// batch b - queue_max, so at most queue_max batches are read ahead (the
// bounded DataQueue).  A buffer is complete when every antenna's row is in.
//
// Consumer side (the calling thread): batches are taken in order; each is
// copied to a device slot on a copy stream and correlated (F-engine,
// X-engine, integration) on a compute stream, with the filter history
// carried across batches on the device.  The copy into a device slot waits
// for the compute that last read it; the compute waits for its copy.  Once
// a batch's copy is done its host buffer is released to the readers.  A
// batch holds either a whole number of dumps, or a whole number of batches
// make one dump (the dump is then accumulated batch by batch).
//
// Times: read_s sums the readers' time inside file reads; h2d_s and
// compute_s sum HIP event intervals per batch; wait_s is the consumer's time
// waiting for a complete buffer; wall_s runs from the first read to the end
// of the last computation.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "qc.h"
#include "qc_internal.h"

namespace {

struct HostBuf {
  unsigned char* p = nullptr;
  int64_t batch = -1;     // batch currently held (or being filled)
  int rows_done = 0;      // antenna rows read for `batch`
  bool failed = false;
};

struct Shared {
  std::mutex mu;
  std::condition_variable cv;
  std::vector<HostBuf> buf;
  int64_t released = 0;   // batches [0, released) have left their host buffer
  bool stop = false;
  std::string err;
};

int word_bytes(int sample) { return sample == 0 ? 1 : sample == 3 ? 4 : 2; }

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Reader thread: antennas ant0, ant0 + stride, ... for every batch in order.
void reader(Shared* sh, const std::vector<std::string>* paths, int ant0, int stride, int n_ant,
            int64_t n_batches, int64_t batch_bytes, int queue_max, std::atomic<double>* read_s) {
  std::vector<FILE*> f;
  for (int a = ant0; a < n_ant; a += stride) {
    FILE* fp = std::fopen((*paths)[a].c_str(), "rb");
    if (!fp) {
      std::lock_guard<std::mutex> lk(sh->mu);
      sh->err = "cannot open " + (*paths)[a];
      sh->stop = true;
      sh->cv.notify_all();
      for (FILE* g : f) std::fclose(g);
      return;
    }
    f.push_back(fp);
  }
  double spent = 0.0;
  for (int64_t b = 0; b < n_batches; ++b) {
    HostBuf* hb = &sh->buf[b % queue_max];
    {
      std::unique_lock<std::mutex> lk(sh->mu);
      // the buffer is free once batch b - queue_max has been released
      sh->cv.wait(lk, [&] { return sh->stop || sh->released >= b - queue_max + 1; });
      if (sh->stop) break;
      if (hb->batch != b) {  // the first reader to get here claims the buffer
        hb->batch = b;
        hb->rows_done = 0;
        hb->failed = false;
      }
    }
    bool ok = true;
    int k = 0;
    for (int a = ant0; a < n_ant; a += stride, ++k) {
      const double t0 = now_s();
      const size_t got = std::fread(hb->p + (size_t)a * (size_t)batch_bytes, 1, (size_t)batch_bytes, f[k]);
      spent += now_s() - t0;
      if (got != (size_t)batch_bytes) ok = false;
    }
    std::lock_guard<std::mutex> lk(sh->mu);
    if (!ok) {
      sh->err = "short read";
      sh->stop = true;
    }
    hb->rows_done += k;
    sh->cv.notify_all();
    if (sh->stop) break;
  }
  for (FILE* g : f) std::fclose(g);
  double cur = read_s->load();
  while (!read_s->compare_exchange_weak(cur, cur + spent)) {
  }
}

}  // namespace

extern "C" qc_status qc_ingest_run(const char* const* paths, const qc_ingest_config* cfg, float* vis,
                                   int64_t max_dumps, qc_ingest_stats* stats) {
  qc::api_clear_error();
  if (!paths || !cfg || !stats) return qc::api_fail(QC_EINVAL, "NULL argument");
  const qc_ingest_config c = *cfg;
  if (c.n_ant < 1 || c.n_ant > 4096) return qc::api_fail(QC_EINVAL, "n_ant must be in [1, 4096]");
  if (c.sample < QC_SAMPLE_I8 || c.sample > QC_SAMPLE_CI16) return qc::api_fail(QC_EINVAL, "bad sample word");
  if (c.packet_samp < 1 || c.batch_packets < 1 || c.queue_max < 1 || c.queue_max > 1024 || c.n_readers < 1 ||
      c.depth < 1 || c.depth > 16)
    return qc::api_fail(QC_EINVAL, "packet_samp, batch_packets, n_readers >= 1; queue_max in [1, 1024]; "
                                   "depth in [1, 16]");
  const int N = c.pfb.n_fft;
  if (N < 4 || N > 8192 || (N & (N - 1))) return qc::api_fail(QC_EINVAL, "n_fft must be a power of two in [4, 8192]");
  if (c.pfb.n_taps < 1 || c.pfb.n_taps > 16) return qc::api_fail(QC_EINVAL, "n_taps must be in [1, 16]");
  const int64_t batch_samp = c.packet_samp * c.batch_packets;
  if (batch_samp % N) return qc::api_fail(QC_EINVAL, "a batch must hold a whole number of spectra");
  const int64_t bspec = batch_samp / N, spd = c.spec_per_dump;
  if (spd < 1 || (bspec % spd != 0 && spd % bspec != 0))
    return qc::api_fail(QC_EINVAL, "batch spectra (%lld) and spec_per_dump (%lld) must divide one another",
                        (long long)bspec, (long long)spd);
  if (batch_samp > 0x7fffffffLL) return qc::api_fail(QC_EINVAL, "a batch must be below 2^31 samples");
  const int wb = word_bytes(c.sample);
  const int64_t batch_bytes = batch_samp * wb;
  // batches available: whole batches present in every file
  int64_t n_batches = -1;
  std::vector<std::string> pv(c.n_ant);
  for (int a = 0; a < c.n_ant; ++a) {
    if (!paths[a]) return qc::api_fail(QC_EINVAL, "path %d is NULL", a);
    pv[a] = paths[a];
    FILE* fp = std::fopen(paths[a], "rb");
    if (!fp) return qc::api_fail(QC_EINVAL, "cannot open %s", paths[a]);
    std::fseek(fp, 0, SEEK_END);
    const long long sz = std::ftell(fp);
    std::fclose(fp);
    const int64_t nb = sz / batch_bytes;
    n_batches = (n_batches < 0 || nb < n_batches) ? nb : n_batches;
  }
  // whole dumps only
  const int64_t per_dump = spd >= bspec ? spd / bspec : 1;    // batches per dump
  const int64_t dumps_per_batch = spd >= bspec ? 1 : bspec / spd;
  int64_t n_dumps = spd >= bspec ? n_batches / per_dump : n_batches * dumps_per_batch;
  if (max_dumps >= 0 && n_dumps > max_dumps) n_dumps = max_dumps;
  // whole batches whose dumps all fit: never more dumps than vis holds
  n_batches = spd >= bspec ? n_dumps * per_dump : n_dumps / dumps_per_batch;
  n_dumps = spd >= bspec ? n_dumps : n_batches * dumps_per_batch;
  *stats = qc_ingest_stats{};
  if (n_batches == 0) return QC_OK;
  if (!vis) return qc::api_fail(QC_EINVAL, "vis is NULL");
  const int64_t n_chan = c.sample >= QC_SAMPLE_CI8 ? N : N / 2;
  const int64_t nb = (int64_t)c.n_ant * (c.n_ant + 1) / 2;

  // device resources
  Shared sh;
  sh.buf.resize(c.queue_max);
  std::vector<unsigned char*> dslot(c.depth, nullptr);
  std::vector<hipEvent_t> ev_copy0(c.depth, nullptr), ev_copied(c.depth, nullptr), ev_computed(c.depth, nullptr),
      ev_comp0(c.depth, nullptr);
  void* hist[2] = {nullptr, nullptr};
  hipStream_t scopy = nullptr, scomp = nullptr;
  qc_status st = QC_OK;
  const int64_t hbytes = (int64_t)c.n_ant * (c.pfb.n_taps - 1) * N * wb;
  auto cleanup = [&]() {
    if (scopy) (void)hipStreamSynchronize(scopy);
    if (scomp) (void)hipStreamSynchronize(scomp);
    for (auto& h : sh.buf)
      if (h.p) (void)hipHostFree(h.p);
    for (auto p : dslot)
      if (p) (void)hipFree(p);
    for (auto* v : {&ev_copy0, &ev_copied, &ev_computed, &ev_comp0})
      for (auto e : *v)
        if (e) (void)hipEventDestroy(e);
    for (auto h : hist)
      if (h) (void)hipFree(h);
    if (scopy) (void)hipStreamDestroy(scopy);
    if (scomp) (void)hipStreamDestroy(scomp);
  };
  hipError_t e = hipStreamCreateWithFlags(&scopy, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&scomp, hipStreamNonBlocking);
  for (int i = 0; i < c.queue_max && e == hipSuccess; ++i)
    e = hipHostMalloc(reinterpret_cast<void**>(&sh.buf[i].p), (size_t)c.n_ant * (size_t)batch_bytes, 0);
  for (int i = 0; i < c.depth && e == hipSuccess; ++i) {
    e = hipMalloc(reinterpret_cast<void**>(&dslot[i]), (size_t)c.n_ant * (size_t)batch_bytes);
    if (e == hipSuccess) e = hipEventCreate(&ev_copy0[i]);
    if (e == hipSuccess) e = hipEventCreate(&ev_copied[i]);
    if (e == hipSuccess) e = hipEventCreate(&ev_comp0[i]);
    if (e == hipSuccess) e = hipEventCreate(&ev_computed[i]);
  }
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipMalloc(&hist[i], hbytes ? (size_t)hbytes : 4);
    if (e == hipSuccess && hbytes) e = hipMemsetAsync(hist[i], 0, (size_t)hbytes, scomp);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(scomp);
  if (e != hipSuccess) {
    cleanup();
    return qc::api_fail(e == hipErrorOutOfMemory ? QC_ENOMEM : QC_EHIP, "ingest set-up: %s", hipGetErrorString(e));
  }

  const int n_readers = c.n_readers < c.n_ant ? c.n_readers : c.n_ant;
  std::atomic<double> read_s{0.0};
  const double t_start = now_s();
  std::vector<std::thread> th;
  for (int r = 0; r < n_readers; ++r)
    th.emplace_back(reader, &sh, &pv, r, n_readers, c.n_ant, n_batches, batch_bytes, c.queue_max, &read_s);

  double wait_s = 0.0, h2d_s = 0.0, comp_s = 0.0;
  int cur = 0;
  for (int64_t b = 0; b < n_batches && st == QC_OK; ++b) {
    HostBuf* hb = &sh.buf[b % c.queue_max];
    {
      const double t0 = now_s();
      std::unique_lock<std::mutex> lk(sh.mu);
      sh.cv.wait(lk, [&] { return sh.stop || (hb->batch == b && hb->rows_done == c.n_ant); });
      wait_s += now_s() - t0;
      if (sh.stop) {
        st = qc::api_fail(QC_EHIP, "reader failed: %s", sh.err.c_str());
        break;
      }
    }
    const int s = (int)(b % c.depth);
    if (b >= c.depth) {
      // the slot's previous batch: collect its event times, then reuse the slot
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev_copy0[s], ev_copied[s]) == hipSuccess) h2d_s += ms * 1e-3;
      if (hipEventElapsedTime(&ms, ev_comp0[s], ev_computed[s]) == hipSuccess) comp_s += ms * 1e-3;
      e = hipStreamWaitEvent(scopy, ev_computed[s], 0);
    }
    if (e == hipSuccess) e = hipEventRecord(ev_copy0[s], scopy);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dslot[s], hb->p, (size_t)c.n_ant * (size_t)batch_bytes, hipMemcpyHostToDevice, scopy);
    if (e == hipSuccess) e = hipEventRecord(ev_copied[s], scopy);
    if (e == hipSuccess) e = hipStreamWaitEvent(scomp, ev_copied[s], 0);
    if (e == hipSuccess) e = hipEventRecord(ev_comp0[s], scomp);
    if (e != hipSuccess) {
      st = qc::api_fail(QC_EHIP, "enqueue: %s", hipGetErrorString(e));
      break;
    }
    // correlate this batch
    const int nxt = 1 - cur;
    int64_t call_spd, dump0;
    int acc = 0;
    if (spd >= bspec) {  // per_dump batches make one dump
      call_spd = bspec;
      dump0 = b / per_dump;
      acc = (b % per_dump) != 0;
    } else {
      call_spd = spd;
      dump0 = b * dumps_per_batch;
    }
    st = qc_xcorrelate_ex(dslot[s], c.sample, batch_samp, c.n_ant, batch_samp, &c.pfb, hbytes ? hist[cur] : nullptr,
                          hbytes ? hist[nxt] : nullptr, call_spd, QC_F32, vis + 2 * dump0 * nb * n_chan, acc,
                          nullptr, scomp);
    if (st != QC_OK) break;
    cur = nxt;
    e = hipEventRecord(ev_computed[s], scomp);
    // release the host buffer once its copy is done
    if (e == hipSuccess) e = hipEventSynchronize(ev_copied[s]);
    if (e != hipSuccess) {
      st = qc::api_fail(QC_EHIP, "copy: %s", hipGetErrorString(e));
      break;
    }
    {
      std::lock_guard<std::mutex> lk(sh.mu);
      sh.released = b + 1;
      sh.cv.notify_all();
    }
  }
  {
    std::lock_guard<std::mutex> lk(sh.mu);
    if (st != QC_OK) sh.stop = true;
    sh.released = n_batches + c.queue_max;  // no reader waits on a buffer any more
    sh.cv.notify_all();
  }
  for (auto& t : th) t.join();
  e = hipStreamSynchronize(scomp);
  const double t_end = now_s();
  if (st == QC_OK && e != hipSuccess) st = qc::api_fail(QC_EHIP, "compute: %s", hipGetErrorString(e));
  if (st == QC_OK) {
    // event times of the batches still in the slots
    const int64_t first = n_batches > c.depth ? n_batches - c.depth : 0;
    for (int64_t b = first; b < n_batches; ++b) {
      const int s = (int)(b % c.depth);
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev_copy0[s], ev_copied[s]) == hipSuccess) h2d_s += ms * 1e-3;
      if (hipEventElapsedTime(&ms, ev_comp0[s], ev_computed[s]) == hipSuccess) comp_s += ms * 1e-3;
    }
    stats->bytes = n_batches * (int64_t)c.n_ant * batch_bytes;
    stats->batches = n_batches;
    stats->dumps = n_dumps;
    stats->wall_s = t_end - t_start;
    stats->read_s = read_s.load();
    stats->h2d_s = h2d_s;
    stats->compute_s = comp_s;
    stats->wait_s = wait_s;
  }
  cleanup();
  return st;
}
