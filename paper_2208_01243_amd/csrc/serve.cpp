// Serving form: a request server that batches alignment requests of
// different sizes and algorithms as they arrive and runs them on the GPU.
//
// Paper: Overall Workflow -- the host gathers pairs, dispatches them to the
// processing units, and retrieves score and operations; here that loop runs
// continuously.  Requests are admitted by their device-memory footprint
// against a budget (FIFO, never dropped, never bypassed), admitted requests
// with the same (algorithm, penalties, threshold) are merged into one device
// batch by whichever of the N stream workers is free, and the batches of
// different workers overlap on the device.  Everything below uses the public
// C ABI (aim.h); each worker owns a context, a stream, device buffers and
// pinned staging, all grown on demand and kept across batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "aim.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Key {
  int32_t alg, x, o, e, max_score, want_cigar, enc;
  bool operator==(const Key &k) const {
    return alg == k.alg && x == k.x && o == k.o && e == k.e && max_score == k.max_score &&
           want_cigar == k.want_cigar && enc == k.enc;
  }
};

struct Req {
  int64_t id = 0;
  Key key{};
  aim_penalties pen{};
  int64_t n = 0;
  int32_t max_len = 0;
  std::vector<uint8_t> pat, txt;
  std::vector<int64_t> pat_off, txt_off;
  std::vector<int32_t> pat_len, txt_len;
  int64_t footprint = 0;
  Clock::time_point t_submit;
  // results
  bool done = false;
  aim_status err = AIM_OK;
  std::vector<int32_t> score;
  std::vector<int8_t> status;
  std::vector<uint32_t> cigar;
  std::vector<int64_t> cigar_off;
  double latency_us = 0;
};

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Grows a staging buffer.  Device buffers are freed and allocated in stream
// order on the worker's stream (idle here: every batch ends with a stream
// synchronisation), so a growing worker does not synchronise the device and
// stall the others; pinned host buffers double, so they rarely grow.
bool grow(DevBuf &b, size_t bytes, bool pinned, hipStream_t s) {
  if (b.bytes >= bytes) return true;
  if (b.p) {
    if (pinned) (void)hipHostFree(b.p);
    else (void)hipFreeAsync(b.p, s);
  }
  b.p = nullptr;
  b.bytes = 0;
  size_t want = pinned ? 2 * bytes + 4096 : bytes + bytes / 4 + 4096;
  hipError_t e = pinned ? hipHostMalloc(&b.p, want, hipHostMallocDefault) : hipMallocAsync(&b.p, want, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return false;
  }
  b.bytes = want;
  return true;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct aim_server {
  int32_t device = 0;
  aim_server_options opt{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req *> pending;  // submitted, waiting for budget (FIFO)
  std::deque<Req *> ready;    // admitted, waiting for a worker
  std::unordered_map<int64_t, Req *> reqs;
  int64_t next_id = 1;
  int64_t used = 0, peak = 0;
  int64_t submitted = 0, completed = 0, pairs_done = 0, batches = 0;
  std::vector<double> lat;
  Clock::time_point t_first;
  bool any = false;
  bool stop = false;
  std::vector<std::thread> workers;
  std::string init_error;
  int32_t init_failed = 0;
};

namespace {

thread_local std::string s_err;

aim_status sfail(aim_status code, const std::string &m) {
  s_err = m;
  return code;
}

// device bytes a request occupies while it is in flight: sequences, CSR
// arrays, outputs with a worst-case CIGAR, and the library's per-pair scratch
int64_t footprint_of(const Req &r) {
  const int64_t bases = (int64_t)r.pat.size() + (int64_t)r.txt.size();
  return bases                      // sequence bytes
         + r.n * (8 + 8 + 4 + 4)     // offsets and lengths
         + r.n * (4 + 1 + 8) + 8     // score, status, cigar_off
         + 4 * (bases + r.n)         // worst-case CIGAR runs
         + r.n * 1024 + bases * 8;   // per-pair slots, lists and wavefront/band scratch
}

void admit_locked(aim_server *s) {
  while (!s->pending.empty() && s->used + s->pending.front()->footprint <= s->opt.budget_bytes) {
    Req *r = s->pending.front();
    s->pending.pop_front();
    s->used += r->footprint;
    s->peak = std::max(s->peak, s->used);
    s->ready.push_back(r);
  }
  s->cv_work.notify_all();
}

struct Worker {
  aim_server *s;
  aim_context *ctx = nullptr;
  hipStream_t stream = nullptr;
  DevBuf din, dout, hin, hout;
};

// Runs one batch of requests sharing a key; fills their results.
aim_status run_batch(Worker &w, std::vector<Req *> &batch) {
  const Key k = batch[0]->key;
  int64_t n = 0, pb = 0, tb = 0;
  int32_t L = 0;
  for (Req *r : batch) {
    n += r->n;
    pb += (int64_t)r->pat.size();
    tb += (int64_t)r->txt.size();
    L = std::max(L, r->max_len);
  }
  // input block layout (host pinned and device alike)
  const size_t o_pat = 0, o_txt = align256(o_pat + pb), o_poff = align256(o_txt + tb),
               o_toff = align256(o_poff + 8 * n), o_plen = align256(o_toff + 8 * n),
               o_tlen = align256(o_plen + 4 * n), in_bytes = align256(o_tlen + 4 * n);
  const int64_t cig_cap = k.want_cigar ? pb + tb + n : 0;
  const size_t q_score = 0, q_status = align256(4 * n), q_coff = align256(q_status + n),
               q_cig = align256(q_coff + 8 * (n + 1)), out_bytes = align256(q_cig + 4 * cig_cap);
  if (!grow(w.hin, in_bytes, true, w.stream) || !grow(w.din, in_bytes, false, w.stream) ||
      !grow(w.hout, out_bytes, true, w.stream) || !grow(w.dout, out_bytes, false, w.stream))
    return sfail(AIM_ERR_OOM, "serving buffers");
  char *h = (char *)w.hin.p;
  int64_t ip = 0, it = 0, q = 0;
  for (Req *r : batch) {
    memcpy(h + o_pat + ip, r->pat.data(), r->pat.size());
    memcpy(h + o_txt + it, r->txt.data(), r->txt.size());
    for (int64_t i = 0; i < r->n; ++i) {
      ((int64_t *)(h + o_poff))[q + i] = ip + r->pat_off[i];
      ((int64_t *)(h + o_toff))[q + i] = it + r->txt_off[i];
    }
    memcpy(h + o_plen + 4 * q, r->pat_len.data(), 4 * r->n);
    memcpy(h + o_tlen + 4 * q, r->txt_len.data(), 4 * r->n);
    ip += (int64_t)r->pat.size();
    it += (int64_t)r->txt.size();
    q += r->n;
  }
  char *d = (char *)w.din.p;
  char *dout = (char *)w.dout.p;
  if (hipMemcpyAsync(d, h, in_bytes, hipMemcpyHostToDevice, w.stream) != hipSuccess)
    return sfail(AIM_ERR_HIP, "H2D copy failed");
  aim_batch B{n, k.enc, L, d + o_pat, (const int64_t *)(d + o_poff), (const int32_t *)(d + o_plen),
              d + o_txt, (const int64_t *)(d + o_toff), (const int32_t *)(d + o_tlen)};
  aim_results R{(int32_t *)(dout + q_score), (int8_t *)(dout + q_status),
                k.want_cigar ? (uint32_t *)(dout + q_cig) : nullptr, (int64_t *)(dout + q_coff), cig_cap,
                k.want_cigar};
  aim_status st = aim_align_batch(w.ctx, &B, k.alg, batch[0]->pen, k.max_score, &R, w.stream);
  if (st != AIM_OK) return sfail(st, aim_last_error());
  char *ho = (char *)w.hout.p;
  if (hipMemcpyAsync(ho, dout, q_cig, hipMemcpyDeviceToHost, w.stream) != hipSuccess ||
      hipStreamSynchronize(w.stream) != hipSuccess)
    return sfail(AIM_ERR_HIP, "D2H copy failed");
  const int64_t *coff = (const int64_t *)(ho + q_coff);
  const int64_t ncig = k.want_cigar ? coff[n] : 0;
  if (ncig > 0) {
    if (hipMemcpyAsync(ho + q_cig, dout + q_cig, 4 * ncig, hipMemcpyDeviceToHost, w.stream) != hipSuccess ||
        hipStreamSynchronize(w.stream) != hipSuccess)
      return sfail(AIM_ERR_HIP, "D2H copy failed");
  }
  q = 0;
  for (Req *r : batch) {
    r->score.assign((int32_t *)(ho + q_score) + q, (int32_t *)(ho + q_score) + q + r->n);
    r->status.assign((int8_t *)(ho + q_status) + q, (int8_t *)(ho + q_status) + q + r->n);
    r->cigar_off.resize(r->n + 1);
    const int64_t c0 = coff[q];
    for (int64_t i = 0; i <= r->n; ++i) r->cigar_off[i] = coff[q + i] - c0;
    const uint32_t *cg = (const uint32_t *)(ho + q_cig);
    r->cigar.assign(cg + c0, cg + coff[q + r->n]);
    q += r->n;
  }
  return AIM_OK;
}

void worker_main(aim_server *s, int idx) {
  Worker w;
  w.s = s;
  (void)hipSetDevice(s->device);
  aim_options o{AIM_KERNEL_AUTO, 0, std::max<int64_t>((int64_t)1 << 30, s->opt.budget_bytes / std::max(1, s->opt.n_streams))};
  bool ok = aim_create(&w.ctx, s->device, &o) == AIM_OK &&
            hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) == hipSuccess;
  // staging for batches of up to 64 MiB in and out from the start
  ok = ok && grow(w.hin, (size_t)64 << 20, true, w.stream) && grow(w.din, (size_t)64 << 20, false, w.stream) &&
       grow(w.hout, (size_t)64 << 20, true, w.stream) && grow(w.dout, (size_t)64 << 20, false, w.stream) &&
       hipStreamSynchronize(w.stream) == hipSuccess;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (!ok) {
      s->init_failed += 1;
      s->init_error = "worker init failed";
    }
  }
  for (;;) {
    std::vector<Req *> batch;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->ready.empty(); });
      if (s->ready.empty()) break;  // stop requested and nothing left
      // the oldest admitted request decides the key; merge every admitted
      // request with the same key up to the pair cap
      const Key k = s->ready.front()->key;
      int64_t pairs = 0;
      for (auto it = s->ready.begin(); it != s->ready.end();) {
        if ((*it)->key == k && (batch.empty() || pairs + (*it)->n <= s->opt.max_batch_pairs)) {
          pairs += (*it)->n;
          batch.push_back(*it);
          it = s->ready.erase(it);
        } else {
          ++it;
        }
      }
    }
    aim_status st = ok ? run_batch(w, batch) : AIM_ERR_HIP;
    const auto now = Clock::now();
    std::lock_guard<std::mutex> g(s->mu);
    for (Req *r : batch) {
      r->err = st;
      r->done = true;
      r->latency_us = std::chrono::duration<double, std::micro>(now - r->t_submit).count();
      s->used -= r->footprint;
      s->completed += 1;
      s->pairs_done += r->n;
      s->lat.push_back(r->latency_us);
    }
    s->batches += 1;
    admit_locked(s);
    s->cv_done.notify_all();
  }
  if (w.stream) {
    if (w.din.p) (void)hipFreeAsync(w.din.p, w.stream);
    if (w.dout.p) (void)hipFreeAsync(w.dout.p, w.stream);
    (void)hipStreamSynchronize(w.stream);
    (void)hipStreamDestroy(w.stream);
  }
  if (w.ctx) aim_destroy(w.ctx);
  if (w.hin.p) (void)hipHostFree(w.hin.p);
  if (w.hout.p) (void)hipHostFree(w.hout.p);
  (void)idx;
}

void fill_result(const Req *r, aim_request_result *res) {
  res->n_pairs = r->n;
  res->score = r->score.data();
  res->status = r->status.data();
  res->cigar = r->cigar.data();
  res->cigar_off = r->cigar_off.data();
  res->latency_us = r->latency_us;
}

}  // namespace

extern "C" {

aim_status aim_server_create(int32_t device, const aim_server_options *opt, aim_server **out) {
  s_err.clear();
  if (!out) return sfail(AIM_ERR_INVALID_ARG, "srv is NULL");
  *out = nullptr;
  aim_server_options o{4, 0, (int64_t)64 << 30, (int64_t)1 << 16};
  if (opt) {
    o = *opt;
    if (o.n_streams == 0) o.n_streams = 4;
    if (o.budget_bytes == 0) o.budget_bytes = (int64_t)64 << 30;
    // 65,536: batches stay large enough to fill the GPU at the serving load,
    // and a merged batch no longer holds its requests for a million pairs
    if (o.max_batch_pairs == 0) o.max_batch_pairs = (int64_t)1 << 16;
  }
  if (o.n_streams < 1 || o.n_streams > 16) return sfail(AIM_ERR_INVALID_ARG, "n_streams must be in [1, 16]");
  if (o.budget_bytes < ((int64_t)1 << 20)) return sfail(AIM_ERR_INVALID_ARG, "budget_bytes below 1 MiB");
  if (o.max_batch_pairs < 1) return sfail(AIM_ERR_INVALID_ARG, "max_batch_pairs < 1");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return sfail(AIM_ERR_INVALID_ARG, "bad device");
  auto *s = new aim_server();
  s->device = device;
  s->opt = o;
  for (int i = 0; i < o.n_streams; ++i) s->workers.emplace_back(worker_main, s, i);
  *out = s;
  return AIM_OK;
}

aim_status aim_server_submit(aim_server *s, const aim_request *q, int64_t *id) {
  s_err.clear();
  if (!s || !q || !id) return sfail(AIM_ERR_INVALID_ARG, "NULL argument");
  if (q->enc != AIM_ENC_ASCII && q->enc != AIM_ENC_CODE) return sfail(AIM_ERR_INVALID_ARG, "enc must be ASCII or CODE");
  if (q->alg < AIM_NW_LINEAR || q->alg > AIM_WFA_AFFINE) return sfail(AIM_ERR_INVALID_ARG, "unknown algorithm");
  if (q->n_pairs < 0) return sfail(AIM_ERR_INVALID_ARG, "n_pairs < 0");
  if (q->n_pairs > 0 && (!q->pat || !q->pat_off || !q->pat_len || !q->txt || !q->txt_off || !q->txt_len))
    return sfail(AIM_ERR_INVALID_ARG, "NULL sequence array");
  auto *r = new Req();
  r->key = {q->alg, q->pen.mismatch, q->pen.gap_open, q->pen.gap_extend, q->max_score, q->want_cigar ? 1 : 0, q->enc};
  r->pen = q->pen;
  r->n = q->n_pairs;
  r->pat_off.resize(r->n);
  r->txt_off.resize(r->n);
  r->pat_len.assign(q->pat_len, q->pat_len + r->n);
  r->txt_len.assign(q->txt_len, q->txt_len + r->n);
  int64_t pb = 0, tb = 0;
  for (int64_t i = 0; i < r->n; ++i) {
    if (r->pat_len[i] < 0 || r->txt_len[i] < 0 || r->pat_len[i] > (1 << 20) || r->txt_len[i] > (1 << 20)) {
      delete r;
      return sfail(AIM_ERR_INVALID_ARG, "sequence length out of range");
    }
    r->pat_off[i] = pb;
    r->txt_off[i] = tb;
    pb += r->pat_len[i];
    tb += r->txt_len[i];
    r->max_len = std::max(r->max_len, std::max(r->pat_len[i], r->txt_len[i]));
  }
  r->pat.resize(pb);
  r->txt.resize(tb);
  for (int64_t i = 0; i < r->n; ++i) {
    memcpy(r->pat.data() + r->pat_off[i], q->pat + q->pat_off[i], r->pat_len[i]);
    memcpy(r->txt.data() + r->txt_off[i], q->txt + q->txt_off[i], r->txt_len[i]);
  }
  r->footprint = footprint_of(*r);
  if (r->footprint > s->opt.budget_bytes) {
    delete r;
    return sfail(AIM_ERR_INVALID_ARG, "request larger than the server's memory budget");
  }
  std::lock_guard<std::mutex> g(s->mu);
  r->id = s->next_id++;
  r->t_submit = Clock::now();
  if (!s->any) {
    s->any = true;
    s->t_first = r->t_submit;
  }
  s->reqs[r->id] = r;
  s->pending.push_back(r);
  s->submitted += 1;
  admit_locked(s);
  *id = r->id;
  return AIM_OK;
}

aim_status aim_server_poll(aim_server *s, int64_t id, aim_request_result *res) {
  s_err.clear();
  if (!s) return sfail(AIM_ERR_INVALID_ARG, "srv is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return sfail(AIM_ERR_NOT_FOUND, "unknown request id");
  if (!it->second->done) return sfail(AIM_ERR_BUSY, "request still running");
  if (it->second->err != AIM_OK) return sfail(it->second->err, "request failed on the device");
  if (res) fill_result(it->second, res);
  return AIM_OK;
}

aim_status aim_server_wait(aim_server *s, int64_t id, int32_t timeout_ms, aim_request_result *res) {
  s_err.clear();
  if (!s) return sfail(AIM_ERR_INVALID_ARG, "srv is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return sfail(AIM_ERR_NOT_FOUND, "unknown request id");
  Req *r = it->second;
  auto pred = [&] { return r->done; };
  if (timeout_ms < 0) s->cv_done.wait(lk, pred);
  else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
    return sfail(AIM_ERR_BUSY, "timed out");
  if (r->err != AIM_OK) return sfail(r->err, "request failed on the device");
  if (res) fill_result(r, res);
  return AIM_OK;
}

aim_status aim_server_release(aim_server *s, int64_t id) {
  s_err.clear();
  if (!s) return sfail(AIM_ERR_INVALID_ARG, "srv is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return sfail(AIM_ERR_NOT_FOUND, "unknown request id");
  if (!it->second->done) return sfail(AIM_ERR_BUSY, "request still running");
  delete it->second;
  s->reqs.erase(it);
  return AIM_OK;
}

aim_status aim_server_stats_get(aim_server *s, aim_server_stats *st) {
  s_err.clear();
  if (!s || !st) return sfail(AIM_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  memset(st, 0, sizeof *st);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->pairs_completed = s->pairs_done;
  st->batches = s->batches;
  st->bytes_in_use = s->used;
  st->peak_bytes = s->peak;
  st->budget_bytes = s->opt.budget_bytes;
  st->queued = (int64_t)s->pending.size() + (int64_t)s->ready.size();
  if (!s->lat.empty()) {
    std::vector<double> v = s->lat;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) { return v[std::min(v.size() - 1, (size_t)(p * (v.size() - 1) + 0.5))]; };
    st->p50_us = pct(0.50);
    st->p99_us = pct(0.99);
    st->max_us = v.back();
    double sum = 0;
    for (double x : v) sum += x;
    st->mean_us = sum / v.size();
  }
  if (s->any) st->elapsed_s = std::chrono::duration<double>(Clock::now() - s->t_first).count();
  return AIM_OK;
}

aim_status aim_server_reset_stats(aim_server *s) {
  s_err.clear();
  if (!s) return sfail(AIM_ERR_INVALID_ARG, "srv is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  s->lat.clear();
  s->completed = s->submitted = s->pairs_done = s->batches = 0;
  s->peak = s->used;
  s->any = false;
  return AIM_OK;
}

const char *aim_server_last_error(void) { return s_err.c_str(); }

void aim_server_destroy(aim_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto &t : s->workers) t.join();
  // every submitted request is in the map (pending ones were drained by the
  // workers before they stopped)
  for (auto &kv : s->reqs) delete kv.second;
  delete s;
}

}  // extern "C"
