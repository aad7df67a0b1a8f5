// Serving loop: requests (graph, query, seed, trials) against resident graphs.
//
// Admission is by device footprint: a request starts when a worker slot is
// free and its footprint fits what the budget has left (a request that would
// never fit is run alone).  Requests start in arrival order, except that while
// the oldest waiting request does not fit, a later one that fits may start
// ahead of it, at most kMaxBypass times per waiting request; after that the
// oldest one is next, so no request waits behind an unbounded stream of
// smaller ones.  Each worker
// owns a HIP stream, so admitted requests run concurrently on the device and a
// request that arrives while others run starts as soon as a slot and memory
// free up.  The arithmetic is exactly cc_count's, so a result does not depend
// on what else is running.
#include <chrono>
#include <cmath>
#include <algorithm>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

#include "cc_internal.h"


namespace {

using Clock = std::chrono::steady_clock;

// how many later requests may start ahead of a waiting request that does not fit
constexpr int kMaxBypass = 8;

struct Request {
  uint64_t ticket;
  int graph;
  const cc::Plan *plan;
  uint64_t seed;
  int trials;
  uint64_t bytes;
  int bypassed = 0;  // later requests started ahead of this one
  Clock::time_point t_submit;
  // results
  bool done = false;
  cc_status st = CC_OK;
  std::vector<uint64_t> counts;
  std::vector<uint8_t> ovf;
  double estimate = NAN;
  double latency = 0;
};

}  // namespace

struct cc_server_s {
  uint64_t budget;
  int max_inflight;
  std::vector<const cc::DevGraph *> graphs;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<uint64_t> queue;
  std::map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  uint64_t in_use = 0;
  int running = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  int device = 0;

  void worker() {
    (void)hipSetDevice(device);
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
    for (;;) {
      uint64_t tk = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (stop && queue.empty()) {
            (void)hipStreamDestroy(st);
            return;
          }
          if (!queue.empty()) {
            Request &h = reqs[queue.front()];
            auto it = queue.end();
            if (in_use + h.bytes <= budget || running == 0) {
              it = queue.begin();
            } else if (h.bypassed < kMaxBypass) {
              // the oldest request waits for memory: start the first later one that fits
              for (auto j = queue.begin() + 1; j != queue.end(); ++j)
                if (in_use + reqs[*j].bytes <= budget) {
                  it = j;
                  h.bypassed++;
                  break;
                }
            }
            if (it != queue.end()) {
              tk = *it;
              queue.erase(it);
              in_use += reqs[tk].bytes;
              running++;
              break;
            }
          }
          cv.wait(lk);
        }
      }
      Request *r;
      {
        std::lock_guard<std::mutex> lk(mu);
        r = &reqs[tk];
      }
      cc_status stt = CC_OK;
      std::vector<uint64_t> counts(r->trials);
      std::vector<uint8_t> ovf(r->trials);
      double est = NAN;
      try {
        cc::ColourSource cs;
        cs.seed = r->seed;
        cc::ExecOptions o;
        o.mem_budget = r->bytes;
        auto res = cc::run_count(*graphs[r->graph], *r->plan, r->trials, cs, o, st, nullptr);
        for (int t = 0; t < r->trials; t++) {
          bool of = res.overflow[t] || (res.exact[t] >> 64) != 0;
          counts[t] = of ? UINT64_MAX : (uint64_t)res.exact[t];
          ovf[t] = of;
        }
        est = cc::estimate_from(*r->plan, res.exact, res.overflow);
      } catch (const cc::Error &e) {
        stt = e.st;
      } catch (...) {
        stt = CC_E_DEVICE;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        r->st = stt;
        r->counts = std::move(counts);
        r->ovf = std::move(ovf);
        r->estimate = est;
        r->latency = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
        r->done = true;
        in_use -= r->bytes;
        running--;
      }
      cv.notify_all();
      cv_done.notify_all();
    }
  }
};

extern "C" {

cc_status cc_server_create(uint64_t hbm_budget_bytes, int32_t max_inflight, cc_server *out) {
  if (!out || max_inflight < 1 || max_inflight > 64) return CC_E_ARG;
  try {
    auto s = new cc_server_s;
    size_t fr = 0, tot = 0;
    (void)hipGetDevice(&s->device);
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 0;
    s->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(fr * 0.8);
    s->max_inflight = max_inflight;
    for (int i = 0; i < max_inflight; i++) s->workers.emplace_back([s] { s->worker(); });
    *out = s;
    return CC_OK;
  } catch (...) {
    return CC_E_DEVICE;
  }
}

cc_status cc_server_add_graph(cc_server s, cc_graph g, int32_t *graph_id) {
  if (!s || !g || !graph_id) return CC_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  s->graphs.push_back(g->g.get());
  *graph_id = (int32_t)s->graphs.size() - 1;
  return CC_OK;
}

cc_status cc_server_submit(cc_server s, int32_t graph_id, cc_query q, uint64_t seed, int32_t trials,
                           uint64_t *ticket) {
  if (!s || !q || !ticket || trials < 1) return CC_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (graph_id < 0 || graph_id >= (int)s->graphs.size()) return CC_E_ARG;
  if (s->reqs.size() >= 1u << 16) return CC_E_BUSY;
  Request r;
  r.ticket = s->next_ticket++;
  r.graph = graph_id;
  r.plan = &q->plan;
  r.seed = seed;
  r.trials = trials;
  cc::ExecOptions o;
  // a request never claims more than the whole budget: one larger than it
  // runs alone, with its trial groups and source groups sized to the budget
  r.bytes = std::min<uint64_t>(cc::footprint(*s->graphs[graph_id], q->plan, trials, o), s->budget);
  r.t_submit = Clock::now();
  s->reqs[r.ticket] = std::move(r);
  s->queue.push_back(s->next_ticket - 1);
  *ticket = s->next_ticket - 1;
  s->cv.notify_all();
  return CC_OK;
}

cc_status cc_server_poll(cc_server s, uint64_t ticket, int32_t *done, uint64_t *counts, uint8_t *overflow,
                         double *estimate, double *latency_s) {
  if (!s || !done) return CC_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return CC_E_ARG;
  Request &r = it->second;
  if (!r.done) {
    *done = 0;
    return CC_OK;
  }
  *done = 1;
  cc_status st = r.st;
  if (st == CC_OK) {
    if (counts) std::copy(r.counts.begin(), r.counts.end(), counts);
    if (overflow) std::copy(r.ovf.begin(), r.ovf.end(), overflow);
    if (estimate) *estimate = r.estimate;
  }
  if (latency_s) *latency_s = r.latency;
  s->reqs.erase(it);
  return st;
}

cc_status cc_server_drain(cc_server s) {
  if (!s) return CC_E_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] {
    if (!s->queue.empty() || s->running) return false;
    return true;
  });
  return CC_OK;
}

cc_status cc_server_destroy(cc_server s) {
  if (!s) return CC_E_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto &t : s->workers) t.join();
  delete s;
  return CC_OK;
}

}  // extern "C"
