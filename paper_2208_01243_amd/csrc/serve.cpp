// Serving form: a request server that batches alignment requests of
// different sizes and algorithms as they arrive and runs them on the GPU.
//
// Paper: Overall Workflow -- the host gathers pairs, dispatches them to the
// processing units, and retrieves score and operations; here that loop runs
// continuously.  The queue, merging and splitting rules are in
// serve_sched.h; this file holds the workers.  Each of the N workers owns a
// context, a stream, device staging and pinned host staging, and a fixed
// share of the device-memory budget: its staging is capped, and its context
// is created with a hard scratch limit, so the device memory the server
// holds stays within the budget.  Batches of different workers overlap on
// the device.  Everything below uses the public C ABI (aim.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "aim.h"
#include "serve_sched.h"

namespace {

using Clock = std::chrono::steady_clock;
using aim_serve::Job;

struct Req : Job {
  aim_penalties pen{};
  int64_t n = 0;
  int32_t max_len = 0;
  std::vector<uint8_t> pat, txt;
  std::vector<int64_t> pat_off, txt_off;
  std::vector<int32_t> pat_len, txt_len;
  Clock::time_point t_submit;
  // results
  bool done = false;
  aim_status err = AIM_OK;
  std::string err_msg;
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

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Staging layout of a batch (host pinned and device alike): input block of
// sequences, offsets and lengths; output block of score, status, CIGAR
// offsets and runs.
struct Layout {
  size_t o_pat, o_txt, o_poff, o_toff, o_plen, o_tlen, in_bytes;
  size_t q_score, q_status, q_coff, q_cig, out_bytes;
  int64_t cig_cap;
};

Layout layout_of(int64_t n, int64_t pb, int64_t tb, bool want_cigar) {
  Layout l;
  l.o_pat = 0;
  l.o_txt = align256(l.o_pat + pb);
  l.o_poff = align256(l.o_txt + tb);
  l.o_toff = align256(l.o_poff + 8 * n);
  l.o_plen = align256(l.o_toff + 8 * n);
  l.o_tlen = align256(l.o_plen + 4 * n);
  l.in_bytes = align256(l.o_tlen + 4 * n);
  l.cig_cap = want_cigar ? pb + tb + n : 0;
  l.q_score = 0;
  l.q_status = align256(4 * n);
  l.q_coff = align256(l.q_status + n);
  l.q_cig = align256(l.q_coff + 8 * (n + 1));
  l.out_bytes = align256(l.q_cig + 4 * l.cig_cap);
  return l;
}

// A worker's device buffer, grown on demand up to `cap` bytes, freed and
// allocated in stream order on the worker's stream (idle here: every batch
// ends with a stream synchronisation), so a growing worker does not
// synchronise the device; pinned host buffers (cap 0: none) double.
bool grow(DevBuf &b, size_t bytes, bool pinned, size_t cap, hipStream_t s) {
  if (b.bytes >= bytes) return true;
  if (b.p) {
    if (pinned) (void)hipHostFree(b.p);
    else (void)hipFreeAsync(b.p, s);
  }
  b.p = nullptr;
  b.bytes = 0;
  size_t want = pinned ? 2 * bytes + 4096 : bytes + bytes / 4 + 4096;
  if (cap) want = std::max(bytes, std::min(want, cap));
  hipError_t e = pinned ? hipHostMalloc(&b.p, want, hipHostMallocDefault) : hipMallocAsync(&b.p, want, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return false;
  }
  b.bytes = want;
  return true;
}

}  // namespace

struct aim_server {
  int32_t device = 0;
  aim_server_options opt{};
  // per worker: staging caps (input, output) and the context's scratch cap
  int64_t in_cap = 0, out_cap = 0, scratch_cap = 0;
  aim_serve::Scheduler *sched = nullptr;
  std::mutex mu;  // everything below
  std::condition_variable cv_done;
  std::unordered_map<int64_t, Req *> reqs;
  int64_t next_id = 1;
  int64_t submitted = 0, completed = 0, pairs_done = 0, batches = 0;
  std::vector<int64_t> wbytes, wpeak;  // per worker: device bytes held now, and at most
  int64_t peak = 0;                    // most device bytes held by all workers together
  std::vector<double> lat;
  Clock::time_point t_first;
  bool any = false;
  std::vector<std::thread> workers;
  std::string init_error;
  int32_t init_failed = 0;
};

namespace {

thread_local std::string s_err;

constexpr int64_t MIN_SHARE = (int64_t)64 << 20;  // device bytes per worker at least

aim_status sfail(aim_status code, const std::string &m) {
  s_err = m;
  return code;
}

struct Worker {
  aim_server *s;
  int idx = 0;
  aim_context *ctx = nullptr;
  hipStream_t stream = nullptr;
  DevBuf din, dout, hin, hout;
};

// device bytes the worker holds (staging plus its context's scratch), now
// and at most; recorded under the server lock
void record_memory(Worker &w) {
  int64_t cur = 0, pk = 0;
  if (w.ctx) (void)aim_scratch_usage(w.ctx, &cur, &pk);
  const int64_t st = (int64_t)w.din.bytes + (int64_t)w.dout.bytes;
  std::lock_guard<std::mutex> g(w.s->mu);
  w.s->wbytes[w.idx] = cur + st;
  w.s->wpeak[w.idx] = pk + st;
  int64_t sum = 0;
  for (int64_t v : w.s->wpeak) sum += v;
  w.s->peak = std::max(w.s->peak, sum);
}

// Runs one batch of requests sharing a key; fills their results.
aim_status run_batch(Worker &w, const std::vector<Job *> &jobs) {
  const Req *r0 = static_cast<const Req *>(jobs[0]);
  const aim_serve::Key k = r0->key;
  int64_t n = 0, pb = 0, tb = 0;
  int32_t L = 0;
  for (Job *j : jobs) {
    const Req *r = static_cast<const Req *>(j);
    n += r->n;
    pb += (int64_t)r->pat.size();
    tb += (int64_t)r->txt.size();
    L = std::max(L, r->max_len);
  }
  const Layout l = layout_of(n, pb, tb, k.want_cigar != 0);
  if (!grow(w.hin, l.in_bytes, true, 0, w.stream) || !grow(w.din, l.in_bytes, false, w.s->in_cap, w.stream) ||
      !grow(w.hout, l.out_bytes, true, 0, w.stream) || !grow(w.dout, l.out_bytes, false, w.s->out_cap, w.stream))
    return sfail(AIM_ERR_OOM, "serving buffers");
  char *h = (char *)w.hin.p;
  int64_t ip = 0, it = 0, q = 0;
  for (Job *j : jobs) {
    const Req *r = static_cast<const Req *>(j);
    memcpy(h + l.o_pat + ip, r->pat.data(), r->pat.size());
    memcpy(h + l.o_txt + it, r->txt.data(), r->txt.size());
    for (int64_t i = 0; i < r->n; ++i) {
      ((int64_t *)(h + l.o_poff))[q + i] = ip + r->pat_off[i];
      ((int64_t *)(h + l.o_toff))[q + i] = it + r->txt_off[i];
    }
    memcpy(h + l.o_plen + 4 * q, r->pat_len.data(), 4 * r->n);
    memcpy(h + l.o_tlen + 4 * q, r->txt_len.data(), 4 * r->n);
    ip += (int64_t)r->pat.size();
    it += (int64_t)r->txt.size();
    q += r->n;
  }
  char *d = (char *)w.din.p;
  char *dout = (char *)w.dout.p;
  if (hipMemcpyAsync(d, h, l.in_bytes, hipMemcpyHostToDevice, w.stream) != hipSuccess)
    return sfail(AIM_ERR_HIP, "H2D copy failed");
  aim_batch B{n, k.enc, L, d + l.o_pat, (const int64_t *)(d + l.o_poff), (const int32_t *)(d + l.o_plen),
              d + l.o_txt, (const int64_t *)(d + l.o_toff), (const int32_t *)(d + l.o_tlen)};
  aim_results R{(int32_t *)(dout + l.q_score), (int8_t *)(dout + l.q_status),
                k.want_cigar ? (uint32_t *)(dout + l.q_cig) : nullptr, (int64_t *)(dout + l.q_coff), l.cig_cap,
                k.want_cigar};
  aim_status st = aim_align_batch(w.ctx, &B, k.alg, r0->pen, k.max_score, &R, w.stream);
  if (st != AIM_OK) {
    const std::string msg = aim_last_error();
    (void)hipStreamSynchronize(w.stream);  // whatever was enqueued before the error
    return sfail(st, msg);
  }
  char *ho = (char *)w.hout.p;
  if (hipMemcpyAsync(ho, dout, l.q_cig, hipMemcpyDeviceToHost, w.stream) != hipSuccess ||
      hipStreamSynchronize(w.stream) != hipSuccess)
    return sfail(AIM_ERR_HIP, "D2H copy failed");
  const int64_t *coff = (const int64_t *)(ho + l.q_coff);
  const int64_t ncig = k.want_cigar ? coff[n] : 0;
  if (ncig > 0) {
    if (hipMemcpyAsync(ho + l.q_cig, dout + l.q_cig, 4 * ncig, hipMemcpyDeviceToHost, w.stream) != hipSuccess ||
        hipStreamSynchronize(w.stream) != hipSuccess)
      return sfail(AIM_ERR_HIP, "D2H copy failed");
  }
  q = 0;
  for (Job *j : jobs) {
    Req *r = static_cast<Req *>(j);
    r->score.assign((int32_t *)(ho + l.q_score) + q, (int32_t *)(ho + l.q_score) + q + r->n);
    r->status.assign((int8_t *)(ho + l.q_status) + q, (int8_t *)(ho + l.q_status) + q + r->n);
    r->cigar_off.resize(r->n + 1);
    const int64_t c0 = coff[q];
    for (int64_t i = 0; i <= r->n; ++i) r->cigar_off[i] = coff[q + i] - c0;
    const uint32_t *cg = (const uint32_t *)(ho + l.q_cig);
    r->cigar.assign(cg + c0, cg + coff[q + r->n]);
    q += r->n;
  }
  return AIM_OK;
}

void worker_main(aim_server *s, int idx) {
  Worker w;
  w.s = s;
  w.idx = idx;
  (void)hipSetDevice(s->device);
  aim_options o{AIM_KERNEL_AUTO, AIM_FLAG_HARD_LIMIT, s->scratch_cap};
  bool ok = aim_create(&w.ctx, s->device, &o) == AIM_OK &&
            hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) == hipSuccess;
  // staging for batches of up to 64 MiB in and out from the start
  const size_t init = (size_t)64 << 20;
  ok = ok && grow(w.hin, std::min<size_t>(init, s->in_cap), true, 0, w.stream) &&
       grow(w.din, std::min<size_t>(init, s->in_cap), false, s->in_cap, w.stream) &&
       grow(w.hout, std::min<size_t>(init, s->out_cap), true, 0, w.stream) &&
       grow(w.dout, std::min<size_t>(init, s->out_cap), false, s->out_cap, w.stream) &&
       hipStreamSynchronize(w.stream) == hipSuccess;
  if (!ok) {
    std::lock_guard<std::mutex> g(s->mu);
    s->init_failed += 1;
    s->init_error = "worker init failed";
  }
  record_memory(w);
  auto exec = [&](const std::vector<Job *> &jobs) -> int32_t {
    const aim_status st = ok ? run_batch(w, jobs) : AIM_ERR_HIP;
    record_memory(w);
    return st;
  };
  auto done = [&](const std::vector<Job *> &jobs, int32_t st) {
    const auto now = Clock::now();
    std::lock_guard<std::mutex> g(s->mu);
    for (Job *j : jobs) {
      Req *r = static_cast<Req *>(j);
      r->err = st;
      if (st != AIM_OK) r->err_msg = s_err;  // this worker thread's last failure
      r->done = true;
      r->latency_us = std::chrono::duration<double, std::micro>(now - r->t_submit).count();
      s->completed += 1;
      s->pairs_done += r->n;
      s->lat.push_back(r->latency_us);
    }
    s->batches += 1;
    s->cv_done.notify_all();
  };
  aim_serve::worker_loop(*s->sched, exec, done, AIM_ERR_OOM);
  if (w.stream) {
    if (w.din.p) (void)hipFreeAsync(w.din.p, w.stream);
    if (w.dout.p) (void)hipFreeAsync(w.dout.p, w.stream);
    (void)hipStreamSynchronize(w.stream);
    (void)hipStreamDestroy(w.stream);
  }
  if (w.ctx) aim_destroy(w.ctx);
  if (w.hin.p) (void)hipHostFree(w.hin.p);
  if (w.hout.p) (void)hipHostFree(w.hout.p);
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
  if (o.budget_bytes / o.n_streams < MIN_SHARE)
    return sfail(AIM_ERR_INVALID_ARG, "budget_bytes must give each stream at least 64 MiB");
  if (o.max_batch_pairs < 1) return sfail(AIM_ERR_INVALID_ARG, "max_batch_pairs < 1");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return sfail(AIM_ERR_INVALID_ARG, "bad device");
  auto *s = new aim_server();
  s->device = device;
  s->opt = o;
  // each worker's share: an eighth each way for staging (at most 1 GiB,
  // far more than a batch of the merge cap needs), the rest for its
  // context's scratch (a hard limit)
  const int64_t share = o.budget_bytes / o.n_streams;
  s->in_cap = s->out_cap = std::min<int64_t>(share / 8, (int64_t)1 << 30);
  s->scratch_cap = share - s->in_cap - s->out_cap;
  s->sched = new aim_serve::Scheduler(aim_serve::Limits{o.max_batch_pairs, s->in_cap, s->out_cap});
  s->wbytes.assign(o.n_streams, 0);
  s->wpeak.assign(o.n_streams, 0);
  for (int i = 0; i < o.n_streams; ++i) s->workers.emplace_back(worker_main, s, i);
  *out = s;
  return AIM_OK;
}

aim_status aim_server_submit(aim_server *s, const aim_request *q, int64_t *id) {
  s_err.clear();
  if (!s || !q || !id) return sfail(AIM_ERR_INVALID_ARG, "NULL argument");
  if (q->enc != AIM_ENC_ASCII && q->enc != AIM_ENC_CODE) return sfail(AIM_ERR_INVALID_ARG, "enc must be ASCII or CODE");
  if (q->alg < AIM_NW_LINEAR || q->alg > AIM_GENASM) return sfail(AIM_ERR_INVALID_ARG, "unknown algorithm");
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
  // staging of the request alone, plus the alignment padding a merged
  // layout may add, so that a batch's staging is at most its requests' sum
  const Layout l = layout_of(r->n, pb, tb, q->want_cigar != 0);
  r->id = 0;
  r->pairs = r->n;
  r->in_bytes = (int64_t)l.in_bytes + 6 * 256;
  r->out_bytes = (int64_t)l.out_bytes + 4 * 256;
  if (!s->sched->fits(*r)) {
    delete r;
    return sfail(AIM_ERR_INVALID_ARG, "request larger than a stream's share of the budget");
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    r->id = s->next_id++;
    r->t_submit = Clock::now();
    if (!s->any) {
      s->any = true;
      s->t_first = r->t_submit;
    }
    s->reqs[r->id] = r;
    s->submitted += 1;
    *id = r->id;
  }
  s->sched->submit(r);
  return AIM_OK;
}

aim_status aim_server_poll(aim_server *s, int64_t id, aim_request_result *res) {
  s_err.clear();
  if (!s) return sfail(AIM_ERR_INVALID_ARG, "srv is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return sfail(AIM_ERR_NOT_FOUND, "unknown request id");
  if (!it->second->done) return sfail(AIM_ERR_BUSY, "request still running");
  if (it->second->err != AIM_OK) return sfail(it->second->err, "request failed: " + it->second->err_msg);
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
  if (r->err != AIM_OK) return sfail(r->err, "request failed: " + r->err_msg);
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
  for (int64_t v : s->wbytes) st->bytes_in_use += v;
  st->peak_bytes = s->peak;
  st->budget_bytes = s->opt.budget_bytes;
  st->queued = s->sched->queued();
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
  s->peak = 0;
  for (int64_t v : s->wpeak) s->peak += v;
  s->any = false;
  return AIM_OK;
}

const char *aim_server_last_error(void) { return s_err.c_str(); }

void aim_server_destroy(aim_server *s) {
  if (!s) return;
  s->sched->stop();
  for (auto &t : s->workers) t.join();
  delete s->sched;
  // every submitted request is in the map (queued ones were drained by the
  // workers before they stopped)
  for (auto &kv : s->reqs) delete kv.second;
  delete s;
}

}  // extern "C"
