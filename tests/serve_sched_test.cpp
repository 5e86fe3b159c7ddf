// Host-only test of the serving scheduler (serve_sched.h): producers submit
// jobs of several keys and sizes from several threads while workers take,
// "run" (a fake executor that refuses large batches as out of memory) and
// complete them.  Checks: every job completes exactly once; a batch holds
// one key, in queue order, within the merge limits unless it is one job;
// jobs of one key start in queue order; refused batches are split and only
// single jobs that are still too large fail; merging happens.  Built and run
// by tests/test_serve_sched.py, also under a thread sanitizer.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "serve_sched.h"

using aim_serve::Job;

namespace {

constexpr int32_t OK = 0, OOM = -3;
constexpr int64_t MAX_PAIRS = 100, CAP = 1000;
constexpr int64_t EXEC_PAIRS = 60;    // the fake device holds merged batches of at most this many pairs
constexpr int64_t SINGLE_FAIL = 140;  // a single job above this fails even alone

int g_fail = 0;
std::mutex g_mu;

void check(bool ok, const char *what) {
  if (!ok) {
    std::lock_guard<std::mutex> g(g_mu);
    if (g_fail++ < 10) std::fprintf(stderr, "FAIL: %s\n", what);
  }
}

struct Rec {
  int64_t order;
  std::vector<Job *> jobs;
};

}  // namespace

int main() {
  const int producers = 3, workers = 4, per_producer = 1500;
  aim_serve::Scheduler s(aim_serve::Limits{MAX_PAIRS, CAP, CAP});
  std::vector<Job> jobs((size_t)producers * per_producer);
  std::vector<std::atomic<int>> done_count(jobs.size());
  std::vector<int32_t> status(jobs.size(), 1);
  std::mutex rec_mu;
  std::vector<Rec> taken;
  std::atomic<int64_t> merged{0}, splits{0};

  auto worker = [&]() {
    auto exec = [&](const std::vector<Job *> &b) -> int32_t {
      int64_t pairs = 0;
      for (Job *j : b) pairs += j->pairs;
      std::this_thread::sleep_for(std::chrono::microseconds(20 + pairs % 50));
      if (b.size() > 1 && pairs > EXEC_PAIRS) {
        splits += 1;
        return OOM;
      }
      if (b.size() == 1 && pairs > SINGLE_FAIL) return OOM;
      return OK;
    };
    auto done = [&](const std::vector<Job *> &b, int32_t st) {
      for (Job *j : b) {
        done_count[(size_t)j->id] += 1;
        status[(size_t)j->id] = st;  // each id is written by one worker only
      }
    };
    // the worker loop of serve_sched.h, with the batch rank recorded
    std::vector<Job *> b;
    int64_t order = 0;
    while (s.take(b, &order)) {
      {
        std::lock_guard<std::mutex> g(rec_mu);
        taken.push_back({order, b});
      }
      if (b.size() > 1) merged += 1;
      aim_serve::run_split(b, exec, done, OOM);
    }
  };

  std::vector<std::thread> ws;
  for (int w = 0; w < workers; ++w) ws.emplace_back(worker);
  std::vector<std::thread> ps;
  for (int p = 0; p < producers; ++p) {
    ps.emplace_back([&, p]() {
      std::mt19937_64 rng(1234 + p);
      for (int i = 0; i < per_producer; ++i) {
        Job &j = jobs[(size_t)p * per_producer + i];
        j.id = (int64_t)p * per_producer + i;
        j.key.alg = (int32_t)(rng() % 3);
        j.key.max_score = (int32_t)(rng() % 2);
        j.pairs = 1 + (int64_t)(rng() % 160);
        j.in_bytes = 1 + (int64_t)(rng() % CAP);
        j.out_bytes = 1 + (int64_t)(rng() % CAP);
        check(s.fits(j), "generated job fits");
        s.submit(&j);
        if (rng() % 8 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
      }
    });
  }
  for (auto &t : ps) t.join();
  s.stop();
  for (auto &t : ws) t.join();

  for (size_t i = 0; i < jobs.size(); ++i) {
    check(done_count[i].load() == 1, "every job completes exactly once");
    const bool should_fail = jobs[i].pairs > SINGLE_FAIL;
    check(status[i] == (should_fail ? OOM : OK), "only single jobs too large for the device fail");
  }
  check(s.queued() == 0, "queue drained");
  std::sort(taken.begin(), taken.end(), [](const Rec &a, const Rec &b) { return a.order < b.order; });
  std::map<int64_t, int64_t> last_seq;  // key hash -> seq of the last job started
  for (const Rec &r : taken) {
    check(!r.jobs.empty(), "no empty batch");
    int64_t pairs = 0, in = 0, out = 0;
    for (size_t k = 0; k < r.jobs.size(); ++k) {
      const Job *j = r.jobs[k];
      check(j->key == r.jobs[0]->key, "one key per batch");
      if (k) check(j->seq > r.jobs[k - 1]->seq, "queue order inside a batch");
      pairs += j->pairs;
      in += j->in_bytes;
      out += j->out_bytes;
      const int64_t kh = (int64_t)j->key.alg * 2 + j->key.max_score;
      auto it = last_seq.find(kh);
      check(it == last_seq.end() || j->seq > it->second, "jobs of one key start in queue order");
      last_seq[kh] = j->seq;
    }
    if (r.jobs.size() > 1) check(pairs <= MAX_PAIRS && in <= CAP && out <= CAP, "merge limits");
  }
  check(merged.load() > 0, "some batches merge several jobs");
  check(splits.load() > 0, "some batches are split");
  std::printf("jobs %zu batches %zu merged %lld splits %lld failures %d\n", jobs.size(), taken.size(),
              (long long)merged.load(), (long long)splits.load(), g_fail);
  if (g_fail) return 1;
  std::printf("OK\n");
  return 0;
}
