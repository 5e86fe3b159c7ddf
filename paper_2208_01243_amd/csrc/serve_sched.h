// Request scheduling of the serving form, free of device code, so that it
// builds and is tested on the host alone (with a fake executor, under a
// thread sanitizer).  serve.cpp runs it with one HIP worker per stream.
//
// Paper: Overall Workflow -- the host gathers pairs and dispatches them to
// the processing units; run continuously, that is a queue of requests and a
// set of workers.  The rules:
//   - requests wait in one FIFO queue, never dropped; requests of one key
//     (algorithm, penalties, threshold, outputs, encoding) start in queue
//     order;
//   - a free worker takes the oldest request and the queued requests with
//     the same key after it, in queue order, up to the first that would pass
//     the per-worker limits (pairs, input and output staging bytes); the
//     oldest request always fits, because a request larger than the staging
//     limits is refused at submit, and runs alone if it has more pairs than
//     a batch may merge;
//   - a batch the executor refuses for lack of device memory is split in two
//     by request and each half run again; a single request refused so fails.
// Every worker owns a fixed share of the device-memory budget (staging plus a
// hard-capped library context), so the device memory in use never passes the
// budget whatever the queue holds: a request is admitted to the device when
// a worker, and with it that share of memory, frees up.
#pragma once

#include <stdint.h>

#include <condition_variable>
#include <deque>
#include <mutex>
#include <vector>

namespace aim_serve {

struct Key {
  int32_t alg = 0, x = 0, o = 0, e = 0, max_score = 0, want_cigar = 0, enc = 0;
  bool operator==(const Key &k) const {
    return alg == k.alg && x == k.x && o == k.o && e == k.e && max_score == k.max_score &&
           want_cigar == k.want_cigar && enc == k.enc;
  }
};

// What the scheduler knows of a request.  in_bytes / out_bytes: the staging
// the request needs when batched alone; a merged batch needs at most the sum.
struct Job {
  int64_t id = 0;
  int64_t seq = 0;  // queue position, set by submit
  Key key{};
  int64_t pairs = 0;
  int64_t in_bytes = 0, out_bytes = 0;
};

struct Limits {
  int64_t max_pairs = 1;  // pairs per merged batch (a larger single request runs alone)
  int64_t in_cap = 0;     // input staging bytes per worker
  int64_t out_cap = 0;    // output staging bytes per worker
};

class Scheduler {
 public:
  explicit Scheduler(const Limits &l) : lim_(l) {}

  const Limits &limits() const { return lim_; }

  // whether a request can ever be run (else submit must refuse it)
  bool fits(const Job &j) const { return j.in_bytes <= lim_.in_cap && j.out_bytes <= lim_.out_cap; }

  void submit(Job *j) {
    {
      std::lock_guard<std::mutex> g(mu_);
      j->seq = next_seq_++;
      queue_.push_back(j);
    }
    cv_.notify_one();
  }

  // Blocks until a batch is formed (true) or the scheduler stops with an
  // empty queue (false).  `batch` receives the requests in queue order;
  // `order`, if given, the batch's rank among all batches taken.
  bool take(std::vector<Job *> &batch, int64_t *order = nullptr) {
    batch.clear();
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return stop_ || !queue_.empty(); });
    if (queue_.empty()) return false;
    const Key k = queue_.front()->key;
    int64_t pairs = 0, in = 0, out = 0;
    for (auto it = queue_.begin(); it != queue_.end();) {
      Job *j = *it;
      if (!(j->key == k)) {
        ++it;
        continue;
      }
      const bool fit = batch.empty() || (pairs + j->pairs <= lim_.max_pairs && in + j->in_bytes <= lim_.in_cap &&
                                         out + j->out_bytes <= lim_.out_cap);
      if (!fit) break;  // later requests of this key wait behind it
      pairs += j->pairs;
      in += j->in_bytes;
      out += j->out_bytes;
      batch.push_back(j);
      it = queue_.erase(it);
    }
    if (order) *order = taken_;
    taken_ += 1;
    return true;
  }

  int64_t queued() {
    std::lock_guard<std::mutex> g(mu_);
    return (int64_t)queue_.size();
  }

  // after this, take() drains the queue and then returns false
  void stop() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
    }
    cv_.notify_all();
  }

 private:
  Limits lim_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Job *> queue_;
  int64_t next_seq_ = 0, taken_ = 0;
  bool stop_ = false;
};

// Runs `batch` with exec(batch) -> status; on `oom` with more than one
// request, splits it in two by request (queue order kept) and runs each half
// the same way.  done(batch, status) is called once for every part run.
template <class Exec, class Done>
void run_split(std::vector<Job *> &batch, Exec &exec, Done &done, int32_t oom) {
  const int32_t st = exec(batch);
  if (st == oom && batch.size() > 1) {
    const size_t h = batch.size() / 2;
    std::vector<Job *> a(batch.begin(), batch.begin() + h), b(batch.begin() + h, batch.end());
    run_split(a, exec, done, oom);
    run_split(b, exec, done, oom);
    return;
  }
  done(batch, st);
}

// One worker: takes batches until the scheduler stops.
template <class Exec, class Done>
void worker_loop(Scheduler &s, Exec &exec, Done &done, int32_t oom) {
  std::vector<Job *> batch;
  while (s.take(batch)) run_split(batch, exec, done, oom);
}

}  // namespace aim_serve
