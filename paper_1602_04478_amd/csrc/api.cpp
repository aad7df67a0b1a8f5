// The C ABI (include/cc.h): argument checking, handles, and translation of
// internal errors into status codes.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <atomic>
#include <thread>

#include "cc_internal.h"

namespace cc {

static thread_local std::string g_last_error;

void fail(cc_status st, const std::string &msg) { throw Error{st, msg}; }
void set_last_error(const std::string &msg) { g_last_error = msg; }

}  // namespace cc


namespace {

template <typename F>
cc_status guard(F f) {
  try {
    cc::set_last_error("");
    f();
    return CC_OK;
  } catch (const cc::Error &e) {
    cc::set_last_error(e.msg);
    return e.st;
  } catch (const std::bad_alloc &) {
    cc::set_last_error("host allocation failed");
    return CC_E_NOMEM;
  } catch (const std::exception &e) {
    cc::set_last_error(e.what());
    return CC_E_ARG;
  }
}

void write_results(const cc::Plan &plan, const cc::CountResult &r, int trials, uint64_t *counts, uint8_t *overflow,
                   cc_u128 *exact, double *estimate) {
  for (int t = 0; t < trials; t++) {
    bool of = r.overflow[t] || (r.exact[t] >> 64) != 0;
    counts[t] = of ? UINT64_MAX : (uint64_t)r.exact[t];
    overflow[t] = of ? 1 : 0;
    if (exact) {
      if (r.overflow[t]) {
        exact[t].lo = exact[t].hi = UINT64_MAX;
      } else {
        exact[t].lo = (uint64_t)r.exact[t];
        exact[t].hi = (uint64_t)(r.exact[t] >> 64);
      }
    }
  }
  if (estimate) *estimate = cc::estimate_from(plan, r.exact, r.overflow);
}

cc::ExecOptions opts_from(const cc_tuning *t) {
  cc::ExecOptions o;
  if (t) {
    o.group_sources = t->group_sources;
    o.trial_group = t->trial_group;
    o.light_max_keys = t->light_max_keys;
    o.use_graphs = t->use_graphs;
    o.dense_sources = t->dense_sources;
  }
  return o;
}

}  // namespace

extern "C" {

const char *cc_status_str(cc_status st) {
  switch (st) {
    case CC_OK: return "ok";
    case CC_E_ARG: return "invalid argument";
    case CC_E_GRAPH: return "malformed graph";
    case CC_E_QUERY_TW: return "query treewidth exceeds 2";
    case CC_E_QUERY_DISCONNECTED: return "query is disconnected";
    case CC_E_K_RANGE: return "k out of range";
    case CC_E_UNSUPPORTED: return "unsupported query decomposition";
    case CC_E_NOMEM: return "out of device memory budget";
    case CC_E_DEVICE: return "device error";
    case CC_E_BUSY: return "busy";
  }
  return "unknown status";
}

const char *cc_last_error(void) { return cc::g_last_error.c_str(); }

cc_status cc_graph_create(int64_t n, const int64_t *row_ptr, const int32_t *col, uint32_t flags, void *stream,
                          cc_graph *out) {
  return guard([&] {
    if (!out) cc::fail(CC_E_ARG, "null output handle");
    auto g = cc::make_graph(n, row_ptr, col, flags, (hipStream_t)stream);
    *out = new cc_graph_s{std::move(g)};
  });
}

cc_status cc_graph_destroy(cc_graph g) {
  return guard([&] {
    if (!g) cc::fail(CC_E_ARG, "null graph");
    delete g;
  });
}

cc_status cc_graph_info(cc_graph g, int64_t *n, int64_t *m, int64_t *max_degree) {
  return guard([&] {
    if (!g) cc::fail(CC_E_ARG, "null graph");
    if (n) *n = g->g->n;
    if (m) *m = g->g->m2 / 2;
    if (max_degree) *max_degree = g->g->max_degree;
  });
}

cc_status cc_query_create(int32_t k, int32_t num_edges, const int32_t *edges, cc_query *out) {
  return cc_query_create_ex(k, num_edges, edges, 0u, -1, out);
}

cc_status cc_query_create_ex(int32_t k, int32_t num_edges, const int32_t *edges, uint32_t flags, int32_t tree,
                             cc_query *out) {
  return guard([&] {
    if (!out) cc::fail(CC_E_ARG, "null output handle");
    if (num_edges < 0 || (num_edges > 0 && !edges)) cc::fail(CC_E_ARG, "bad edge list");
    if (flags & ~(uint32_t)CC_QUERY_PATH_SPLITTING) cc::fail(CC_E_ARG, "unknown query flag");
    std::vector<std::pair<int, int>> e;
    for (int i = 0; i < num_edges; i++) e.push_back({edges[2 * i], edges[2 * i + 1]});
    auto q = new cc_query_s;
    try {
      q->plan = cc::make_plan(k, e, (flags & CC_QUERY_PATH_SPLITTING) ? cc::PLAN_PS : cc::PLAN_DB, tree);
      if (const char *vb = getenv("CC_VERBOSE"); vb && *vb == '1') cc::dump_programs(q->plan);
    } catch (...) {
      delete q;
      throw;
    }
    *out = q;
  });
}

cc_status cc_query_tree_info(cc_query q, int32_t *tree, int32_t *num_trees, int32_t *pair_keyed_blocks) {
  return guard([&] {
    if (!q) cc::fail(CC_E_ARG, "null query");
    if (tree) *tree = q->plan.tree;
    if (num_trees) *num_trees = q->plan.num_trees;
    if (pair_keyed_blocks) {
      int c = 0;
      for (auto &B : q->plan.blocks) c += B.pair_keyed ? 1 : 0;
      *pair_keyed_blocks = c;
    }
  });
}

cc_status cc_query_destroy(cc_query q) {
  return guard([&] {
    if (!q) cc::fail(CC_E_ARG, "null query");
    delete q;
  });
}

cc_status cc_query_info(cc_query q, uint64_t *aut, int32_t *num_blocks, int32_t *longest_cycle) {
  return guard([&] {
    if (!q) cc::fail(CC_E_ARG, "null query");
    if (aut) *aut = q->plan.aut;
    if (num_blocks) *num_blocks = (int32_t)q->plan.blocks.size();
    if (longest_cycle) *longest_cycle = q->plan.longest_cycle;
  });
}

cc_status cc_query_plan(cc_query q, int32_t *out, int32_t cap, int32_t *len) {
  return guard([&] {
    if (!q || !len) cc::fail(CC_E_ARG, "null argument");
    auto v = cc::describe_plan(q->plan);
    *len = (int32_t)v.size();
    if (out && cap >= (int32_t)v.size()) std::memcpy(out, v.data(), sizeof(int32_t) * v.size());
  });
}

cc_status cc_footprint(cc_graph g, cc_query q, int32_t trials, uint64_t *bytes) {
  return guard([&] {
    if (!g || !q || !bytes || trials < 1) cc::fail(CC_E_ARG, "bad argument");
    *bytes = cc::footprint(*g->g, q->plan, trials, cc::ExecOptions());
  });
}

cc_status cc_colors(cc_graph g, int32_t k, uint64_t seed, int32_t trial, uint8_t *out) {
  return guard([&] {
    if (!g || !out || trial < 0) cc::fail(CC_E_ARG, "bad argument");
    if (k < 2 || k > 12) cc::fail(CC_E_K_RANGE, "k must be in [2, 12]");
    cc::colours_to_host(*g->g, k, seed, trial, out, nullptr);
  });
}

cc_status cc_count(cc_graph g, cc_query q, uint64_t seed, int32_t trials, uint64_t *counts, uint8_t *overflow,
                   cc_u128 *exact, double *estimate, void *stream) {
  return guard([&] {
    if (!g || !q || !counts || !overflow || trials < 1) cc::fail(CC_E_ARG, "bad argument");
    cc::ColourSource cs;
    cs.from_seed = true;
    cs.seed = seed;
    auto r = cc::run_count(*g->g, q->plan, trials, cs, cc::ExecOptions(), (hipStream_t)stream, nullptr);
    write_results(q->plan, r, trials, counts, overflow, exact, estimate);
  });
}

cc_status cc_count_static(cc_graph g, cc_query q, uint64_t seed, int32_t trials, uint64_t *counts,
                          uint8_t *overflow, cc_u128 *exact, double *estimate, void *stream) {
  return guard([&] {
    if (!g || !q || !counts || !overflow || trials < 1) cc::fail(CC_E_ARG, "bad argument");
    const int dev = g->g->device;
    HIP_CHECK(hipSetDevice(dev));
    // one solve at a time per device: they share its scratch
    std::lock_guard<std::mutex> lk(cc::static_scratch_lock(dev));
    cc::ExecOptions o;
    o.arena = cc::static_scratch(dev);
    o.arena_bytes = cc::kStaticScratchBytes;
    cc::ColourSource cs;
    cs.from_seed = true;
    cs.seed = seed;
    auto r = cc::run_count(*g->g, q->plan, trials, cs, o, (hipStream_t)stream, nullptr);
    write_results(q->plan, r, trials, counts, overflow, exact, estimate);
  });
}

cc_status cc_count_colors(cc_graph g, cc_query q, int32_t trials, const uint8_t *colors, uint64_t *counts,
                          uint8_t *overflow, cc_u128 *exact, cc_u128 *per_source, void *stream) {
  return guard([&] {
    if (!g || !q || !colors || !counts || !overflow || trials < 1) cc::fail(CC_E_ARG, "bad argument");
    int64_t n = g->g->n;
    for (int64_t i = 0; i < n * trials; i++)
      if (colors[i] >= q->plan.k) cc::fail(CC_E_ARG, "colour out of range");
    cc::ColourSource cs;
    cs.from_seed = false;
    cs.host = colors;
    std::vector<cc::u128> per;
    auto r = cc::run_count(*g->g, q->plan, trials, cs, cc::ExecOptions(), (hipStream_t)stream,
                           per_source ? &per : nullptr);
    write_results(q->plan, r, trials, counts, overflow, exact, nullptr);
    if (per_source)
      for (size_t i = 0; i < per.size(); i++) {
        per_source[i].lo = (uint64_t)per[i];
        per_source[i].hi = (uint64_t)(per[i] >> 64);
      }
  });
}

cc_status cc_count_batch(cc_graph g, int32_t nq, const cc_query *qs, const uint64_t *seeds, const int32_t *trials,
                         uint64_t *counts, uint8_t *overflow, double *estimates, const cc_tuning *tuning,
                         void *stream) {
  return guard([&] {
    if (!g || nq < 0 || (nq > 0 && (!qs || !seeds || !trials || !counts || !overflow)))
      cc::fail(CC_E_ARG, "bad argument");
    cc::ExecOptions o = opts_from(tuning);
    for (int i = 0; i < nq; i++)
      if (!qs[i] || trials[i] < 1) cc::fail(CC_E_ARG, "bad query or trial count");
    std::vector<size_t> off(nq + 1, 0);
    for (int i = 0; i < nq; i++) off[i + 1] = off[i] + (size_t)trials[i];
    // Several queries run side by side: up to four workers, each with a
    // stream of its own and a share of the device memory, take the queries
    // in order (the small launches of one overlap the others').  The call
    // first waits for `stream`, and returns when every query is done.
    int workers = std::min(nq, 4);
    if (const char *ev = getenv("CC_BATCH_STREAMS")) workers = std::max(1, std::min(workers, atoi(ev)));
    if (workers <= 1) {
      for (int i = 0; i < nq; i++) {
        auto r = cc::run_batched(*g->g, qs[i]->plan, trials[i], seeds[i], tuning ? &o : nullptr, (hipStream_t)stream);
        write_results(qs[i]->plan, r, trials[i], counts + off[i], overflow + off[i], nullptr,
                      estimates ? estimates + i : nullptr);
      }
      return;
    }
    HIP_CHECK(hipSetDevice(g->g->device));
    if (stream) HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
    size_t fr = 0, tot = 0;
    HIP_CHECK(hipMemGetInfo(&fr, &tot));
    const uint64_t share = (uint64_t)(fr * 0.85) / (uint64_t)workers;
    std::atomic<int> next{0};
    std::mutex emu;
    cc_status est = CC_OK;
    std::string emsg;
    cc::TuneReport last{};
    int last_i = -1;
    auto work = [&]() {
      hipStream_t st = nullptr;
      try {
        HIP_CHECK(hipSetDevice(g->g->device));
        HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        for (;;) {
          const int i = next.fetch_add(1);
          if (i >= nq) break;
          {
            std::lock_guard<std::mutex> lk(emu);
            if (est != CC_OK) break;
          }
          cc::ExecOptions oi = o;
          if (!oi.mem_budget) oi.mem_budget = share;
          auto r = cc::run_batched(*g->g, qs[i]->plan, trials[i], seeds[i], tuning ? &oi : nullptr, st, share);
          write_results(qs[i]->plan, r, trials[i], counts + off[i], overflow + off[i], nullptr,
                        estimates ? estimates + i : nullptr);
          std::lock_guard<std::mutex> lk(emu);
          if (i > last_i) {
            last_i = i;
            last = cc::last_tune();
          }
        }
      } catch (const cc::Error &e) {
        std::lock_guard<std::mutex> lk(emu);
        if (est == CC_OK) {
          est = e.st;
          emsg = e.msg;
        }
      } catch (const std::exception &e) {
        std::lock_guard<std::mutex> lk(emu);
        if (est == CC_OK) {
          est = CC_E_DEVICE;
          emsg = e.what();
        }
      }
      if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
      }
    };
    std::vector<std::thread> pool;
    for (int w = 0; w < workers; w++) pool.emplace_back(work);
    for (auto &t : pool) t.join();
    if (est != CC_OK) cc::fail(est, emsg);
    cc::set_last_tune(last);
  });
}

cc_status cc_last_tune_report(cc_tune_report *out) {
  return guard([&] {
    if (!out) cc::fail(CC_E_ARG, "null output");
    cc::TuneReport r = cc::last_tune();
    out->trial_group = r.trial_group;
    out->candidates = r.candidates;
    for (int i = 0; i < 8; i++) {
      out->tried_trial_group[i] = r.tried_T[i];
      out->tried_seconds_per_colouring[i] = r.tried_sec_per_colouring[i];
    }
    out->graph_replays = r.replays;
    out->dense_sources = r.dense_sources;
    for (int i = 0; i < 8; i++) out->tried_dense_sources[i] = r.tried_dense[i];
    out->tree = r.tree;
    out->trees_tried = r.trees_tried;
    for (int i = 0; i < 8; i++) {
      out->tried_tree[i] = r.tried_tree[i];
      out->tried_tree_seconds[i] = r.tried_tree_seconds[i];
    }
  });
}

cc_status cc_last_solve_stats(cc_solve_stats *out) {
  return guard([&] {
    if (!out) cc::fail(CC_E_ARG, "null output");
    cc::SolveStats s = cc::last_solve_stats();
    out->sources = s.sources;
    out->dense_sources = s.dense;
    out->light_sources = s.light;
    out->handed_back = s.handed_back;
    out->trial_group = s.trial_group;
    out->group_sources = s.group_sources;
  });
}

cc_status cc_probe_copy(uint64_t bytes, int32_t reps, double *gbps) {
  return guard([&] {
    if (!gbps || reps < 1 || bytes < 16 || bytes % 16) cc::fail(CC_E_ARG, "bad argument");
    *gbps = cc::probe_copy(bytes, reps);
  });
}

cc_status cc_profile_enable(int32_t on) {
  return guard([&] { cc::profile_enable(on); });
}

cc_status cc_profile_read(cc_kernel_stat *out, int32_t cap, int32_t *len) {
  return guard([&] {
    if (!len) cc::fail(CC_E_ARG, "null length");
    auto v = cc::profile_read();
    *len = (int32_t)v.size();
    for (int32_t i = 0; out && i < cap && i < (int32_t)v.size(); i++) {
      std::memset(out[i].name, 0, sizeof(out[i].name));
      std::strncpy(out[i].name, v[i].name.c_str(), sizeof(out[i].name) - 1);
      out[i].launches = v[i].launches;
      out[i].seconds = v[i].seconds;
      out[i].bytes = v[i].bytes;
      for (int j = 0; j < 3; j++) out[i].work[j] = v[i].work[j];
    }
  });
}

}  // extern "C"
