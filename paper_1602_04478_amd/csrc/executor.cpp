// Executor: runs a plan over a resident graph for a batch of colourings.
//
// Blocks are solved bottom-up (the overall algorithm of Section 4.2): a leaf
// block by one per-vertex kernel, a cycle block by running its frontier
// program (see planner.cpp) for every group of sources, the root by a final
// reduction.  Colourings are the batch dimension of every launch.
//
// Sources of a cycle block are the vertices with at least two lower
// neighbours (both cycle neighbours of the highest vertex are lower).  They
// are taken in decreasing rank, so a group's frontier vertices all lie below
// the rank of its first source.  The highest-reaching sources (by their
// two-step reach) run in dense groups, where every (vertex, source) pair is a
// potential entry and the EdgeJoin pulls over all vertices; the rest run in
// sparse groups, whose registers keep lists of their live entries.
#include <algorithm>
#include <array>
#include <functional>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "cc_internal.h"
#include "kernels.h"

namespace cc {

namespace {

struct DevMem {
  void *p = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  explicit DevMem(size_t b) { alloc(b); }
  void alloc(size_t b) {
    release();
    if (b == 0) b = 8;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      fail(CC_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
    }
    bytes = b;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  ~DevMem() { release(); }
  DevMem(const DevMem &) = delete;
  DevMem &operator=(const DevMem &) = delete;
  template <typename T>
  T *as() const {
    return (T *)p;
  }
};

struct RegBuf {
  DevMem val, mask;
};
struct LevelBuf {
  DevMem m, base, list, cnt, bcnt;
};

int table_C(const Plan &p, int blk) {
  const PBlock &B = p.blocks[blk];
  if (B.boundary.size() == 2) return (int)slots_pair(p.k, B.size);
  return (int)slots_unary(p.k, B.size);
}

bool is_edge_table(const Plan &p, int blk) { return p.blocks[blk].boundary.size() == 2; }

struct Sizing {
  int T;             // trials per group
  int B_dense;       // sources per dense group
  int B_sparse;      // sources per sparse group
  int64_t dense_cut; // number of leading sources run dense
};

uint64_t program_bytes_per_vb(const Plan &p, int T) {
  // bytes per (vertex, source) pair over all registers of all programs (max)
  uint64_t best = 0;
  for (size_t i = 0; i < p.blocks.size(); i++) {
    const Program &P = p.programs[i];
    uint64_t b = 0;
    for (int s : P.reg_s) b += (uint64_t)slots_pair(p.k, s) * T * 8 + 1 + 8;
    best = std::max(best, b);
  }
  return best;
}

uint64_t table_bytes(const DevGraph &g, const Plan &p, int T) {
  uint64_t b = 0;
  for (size_t i = 0; i < p.blocks.size(); i++) {
    const PBlock &B = p.blocks[i];
    if (B.kind == BK_ROOT_CYCLE || B.kind == BK_ROOT_SINGLE) continue;
    uint64_t keys = is_edge_table(p, (int)i) ? (uint64_t)g.m2 : (uint64_t)g.n;
    b += keys * (uint64_t)T * table_C(p, (int)i) * 8;
  }
  return b;
}

uint64_t free_bytes() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return 0;
  return (uint64_t)fr;
}

Sizing choose(const DevGraph &g, const Plan &p, int trials, const ExecOptions &opt, uint64_t budget) {
  Sizing z{};
  z.T = opt.trial_group > 0 ? std::min(opt.trial_group, 64) : std::min(trials, 64);
  if (z.T < 1) z.T = 1;
  for (;;) {
    uint64_t tabs = table_bytes(g, p, z.T);
    uint64_t per_vb = program_bytes_per_vb(p, z.T);
    uint64_t n = (uint64_t)std::max<int64_t>(1, g.n);
    uint64_t left = budget > tabs ? budget - tabs : 0;
    int64_t B = per_vb ? (int64_t)(left / (per_vb * n)) : 64;
    if (B >= 1 || z.T == 1) {
      B = std::max<int64_t>(1, std::min<int64_t>(B, 64));
      if (opt.group_sources > 0) B = std::min<int64_t>(B, opt.group_sources);
      // one workgroup covers every (source, trial, slot) of a vertex
      int cmax = 1;
      for (auto &P : p.programs)
        for (int s : P.reg_s) cmax = std::max(cmax, (int)slots_pair(p.k, s));
      for (auto &B2 : p.blocks)
        if (B2.kind == BK_CYCLE) cmax = std::max(cmax, (int)binom(p.k - 1, B2.size - 1));
      if ((int64_t)z.T * cmax > max_row_slots()) {
        if (z.T > 1) {
          z.T = std::max(1, z.T / 2);
          continue;
        }
        fail(CC_E_UNSUPPORTED, "signature tables too wide for one workgroup");
      }
      z.B_dense = (int)B;
      z.B_sparse = (int)B;
      if (tabs + per_vb * n * B > budget) fail(CC_E_NOMEM, "plan does not fit the device memory budget");
      return z;
    }
    z.T = std::max(1, z.T / 2);
  }
}

// ------------------------------------------------------------------ profiling
struct ProfStat {
  uint64_t launches = 0;
  double seconds = 0, bytes = 0;
  uint64_t work[3] = {0, 0, 0};
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, ProfStat> g_prof;

// Records of the launches of one call (events are resolved at its end).
// events for per-launch timing, reused across solves
std::mutex g_ev_mu;
std::vector<hipEvent_t> g_ev_pool;
hipEvent_t take_event() {
  {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    if (!g_ev_pool.empty()) {
      hipEvent_t e = g_ev_pool.back();
      g_ev_pool.pop_back();
      return e;
    }
  }
  hipEvent_t e;
  HIP_CHECK(hipEventCreate(&e));
  return e;
}
void give_event(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(g_ev_mu);
  g_ev_pool.push_back(e);
}

struct Profiler {
  bool on = false;
  hipStream_t st;
  struct Rec {
    std::string name;
    hipEvent_t a, b;
    int ctr;            // counter triple index, or -1
    double per_scan, per_active, per_entry;
  };
  std::vector<Rec> recs;
  std::vector<uint64_t *> ctrs;
  int nctr = 0;
  DevMem ctrmem;
  explicit Profiler(hipStream_t s) : st(s) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    on = g_prof_on;
    if (on) ctrmem.alloc(sizeof(uint64_t) * 3 * 65536);
  }
  // returns a zeroed counter triple for an EdgeJoin launch (or null)
  uint64_t *begin(const char *name, bool counters, double per_scan, double per_active, double per_entry) {
    if (!on) return nullptr;
    Rec r;
    r.name = name;
    r.ctr = -1;
    uint64_t *c = nullptr;
    if (counters && nctr < 65536) {
      r.ctr = nctr++;
      c = ctrmem.as<uint64_t>() + 3 * r.ctr;
      launch_fill_u64(c, 3, st);
    }
    r.a = take_event();
    r.b = take_event();
    HIP_CHECK(hipEventRecord(r.a, st));
    r.per_scan = per_scan;
    r.per_active = per_active;
    r.per_entry = per_entry;
    recs.push_back(r);
    return c;
  }
  void end() {
    if (!on) return;
    HIP_CHECK(hipEventRecord(recs.back().b, st));
  }
  void finish() {
    if (!on) return;
    HIP_CHECK(hipStreamSynchronize(st));
    std::vector<uint64_t> h(3 * (size_t)std::max(1, nctr));
    if (nctr) HIP_CHECK(hipMemcpy(h.data(), ctrmem.p, sizeof(uint64_t) * 3 * nctr, hipMemcpyDeviceToHost));
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : recs) {
      float ms = 0;
      HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
      ProfStat &p = g_prof[r.name];
      p.launches++;
      p.seconds += ms * 1e-3;
      if (r.ctr >= 0) {
        p.bytes += h[3 * r.ctr] * r.per_scan + h[3 * r.ctr + 1] * r.per_active + h[3 * r.ctr + 2] * r.per_entry;
        for (int i = 0; i < 3; i++) p.work[i] += h[3 * r.ctr + i];
      }
      give_event(r.a);
      give_event(r.b);
    }
    recs.clear();
  }
};

}  // namespace

void profile_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on;
}

std::vector<KernelProfile> profile_read() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::vector<KernelProfile> v;
  for (auto &kv : g_prof) {
    const ProfStat &p = kv.second;
    v.push_back({kv.first, p.launches, p.seconds, p.bytes, {p.work[0], p.work[1], p.work[2]}});
  }
  g_prof.clear();
  return v;
}

uint64_t footprint(const DevGraph &g, const Plan &p, int trials, const ExecOptions &opt) {
  int T = std::min(std::max(trials, 1), 64);
  if (opt.trial_group > 0) T = std::min(T, opt.trial_group);
  uint64_t tabs = table_bytes(g, p, T);
  uint64_t per_vb = program_bytes_per_vb(p, T);
  int B = opt.group_sources > 0 ? std::min(opt.group_sources, 64) : 64;
  return tabs + per_vb * (uint64_t)g.n * B + (uint64_t)g.n * T;
}

void colours_to_host(const DevGraph &g, int k, uint64_t seed, int trial, uint8_t *out, hipStream_t st) {
  DevMem d(g.n);
  launch_colour(g.orig, g.n, k, seed, trial, 1, d.as<uint8_t>(), st);
  HIP_CHECK(hipGetLastError());
  std::vector<uint8_t> h(g.n);
  HIP_CHECK(hipMemcpyAsync(h.data(), d.p, g.n, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  for (int64_t r = 0; r < g.n; r++) out[g.h_orig[r]] = h[r];
}

double estimate_from(const Plan &p, const std::vector<u128> &exact, const std::vector<uint8_t> &ovf) {
  if (exact.empty()) return NAN;
  for (auto o : ovf)
    if (o) return NAN;
  u128 sum = 0;
  for (auto x : exact) sum += x;
  // (sum * k^k) / (T * k! * aut), exact numerator and denominator in 128 bits
  // when they fit, else in long double.
  long double num = (long double)sum, den = (long double)exact.size() * (long double)p.aut;
  for (int i = 1; i <= p.k; i++) {
    num *= p.k;
    den *= i;
  }
  u128 kk = 1, kf = 1;
  bool fits = true;
  for (int i = 1; i <= p.k; i++) {
    kk *= (u128)p.k;
    kf *= (u128)i;
  }
  u128 d128 = kf * (u128)exact.size() * (u128)p.aut;
  if (sum != 0 && kk > (~(u128)0) / sum) fits = false;
  if (fits) {
    u128 n128 = sum * kk;
    u128 q = n128 / d128, r = n128 % d128;
    return (double)((long double)q + (long double)r / (long double)d128);
  }
  return (double)(num / den);
}

// ------------------------------------------------------------------ main
CountResult run_count(const DevGraph &g, const Plan &p, int trials, const ColourSource &cs, const ExecOptions &opt,
                      hipStream_t st, std::vector<u128> *per_source) {
  if (trials < 1) fail(CC_E_ARG, "trials must be >= 1");
  HIP_CHECK(hipSetDevice(g.device));
  const int k = p.k;
  uint64_t budget = opt.mem_budget ? opt.mem_budget : (uint64_t)(free_bytes() * 0.85);
  Sizing z = choose(g, p, trials, opt, budget);
  const int T = z.T;

  CountResult res;
  res.exact.assign(trials, 0);
  res.overflow.assign(trials, 0);
  if (per_source) per_source->assign((size_t)trials * g.n, 0);

  GraphDev gd{g.rp, g.col, g.rev, g.n, g.m2};

  // sources: lowcnt >= 2, descending rank
  std::vector<int32_t> sources;
  for (int64_t r = g.n - 1; r >= 0; r--)
    if (g.h_lowcnt[r] >= 2) sources.push_back((int32_t)r);
  // dense cut: sources whose two-step reach covers a good part of their prefix
  int64_t ndense = 0;
  for (size_t i = 0; i < sources.size(); i++) {
    int64_t u = sources[i];
    if (g.h_r2[u] * 16 >= u && u > 4096) ndense = (int64_t)i + 1;
    else break;
  }
  // CC_DENSE=all / none overrides the choice (used to exercise both paths)
  bool force_sparse = false;
  if (const char *ev = getenv("CC_DENSE")) {
    if (!strcmp(ev, "all")) ndense = (int64_t)sources.size();
    if (!strcmp(ev, "none")) {
      ndense = 0;
      force_sparse = true;
    }
  }
  bool use_light = true;
  if (const char *ev = getenv("CC_LIGHT"))
    if (!strcmp(ev, "0")) use_light = false;
  int64_t light_scratch = 2 << 20;
  if (const char *ev = getenv("CC_LIGHT_SCRATCH")) light_scratch = std::max<int64_t>(4096, atoll(ev));
  int Bmax = std::max(z.B_dense, z.B_sparse);
  int64_t nlim_max = sources.empty() ? 1 : sources[0];
  if (nlim_max < 1) nlim_max = 1;

  DevMem d_src(sizeof(int32_t) * std::max<size_t>(1, sources.size()));
  if (!sources.empty())
    HIP_CHECK(hipMemcpyAsync(d_src.p, sources.data(), sizeof(int32_t) * sources.size(), hipMemcpyHostToDevice, st));
  DevMem d_col((size_t)g.n * T);
  DevMem d_sum(sizeof(uint64_t) * 2 * 64), d_ovf(sizeof(uint32_t) * 64);
  DevMem d_per(per_source ? sizeof(uint64_t) * 2 * (size_t)g.n * T : 8);
  DevMem d_hcol;
  if (!cs.from_seed) d_hcol.alloc((size_t)g.n * T);

  // child tables
  std::vector<DevMem> tabs(p.blocks.size());
  for (size_t i = 0; i < p.blocks.size(); i++) {
    const PBlock &B = p.blocks[i];
    if (B.kind == BK_ROOT_CYCLE || B.kind == BK_ROOT_SINGLE) continue;
    int64_t keys = is_edge_table(p, (int)i) ? g.m2 : g.n;
    tabs[i].alloc(sizeof(uint64_t) * (size_t)std::max<int64_t>(1, keys) * T * table_C(p, (int)i));
  }
  auto tabdev = [&](int blk) {
    TabDev t{nullptr, 0, 0};
    if (blk >= 0) {
      t.val = tabs[blk].as<uint64_t>();
      t.C = table_C(p, blk);
      t.s = p.blocks[blk].size;
    }
    return t;
  };

  // registers and levels: pools sized for the largest program
  size_t nregs = 0;
  int dmax = 1;
  for (auto &P : p.programs) {
    nregs = std::max(nregs, P.reg_s.size());
    dmax = std::max(dmax, P.max_depth);
  }
  std::vector<RegBuf> regs(nregs);
  auto ensure_reg = [&](int r, int s) {
    RegBuf &R = regs[r];
    int C = (int)slots_pair(k, s);
    size_t vb = sizeof(uint64_t) * (size_t)nlim_max * Bmax * T * C;
    if (R.val.bytes < vb) R.val.alloc(vb);
    if (R.mask.bytes < sizeof(uint64_t) * (size_t)nlim_max) R.mask.alloc(sizeof(uint64_t) * (size_t)nlim_max);
  };
  std::vector<LevelBuf> levels(dmax + 2);
  const size_t nf_max = (size_t)nlim_max * Bmax;
  auto ensure_level = [&](int d) {
    LevelBuf &L = levels[d];
    if (L.m.bytes >= sizeof(uint64_t) * (size_t)nlim_max) return;
    L.m.alloc(sizeof(uint64_t) * (size_t)nlim_max);
    launch_fill_u64(L.m.as<uint64_t>(), nlim_max, st);
    L.base.alloc(sizeof(uint32_t) * (size_t)nlim_max);
    L.list.alloc(sizeof(int64_t) * nf_max);
    L.cnt.alloc(sizeof(uint32_t));
    L.bcnt.alloc(sizeof(uint32_t) * (size_t)level_chunks(nlim_max));
  };
  auto leveldev = [&](int d) {
    LevelDev L;
    L.m = levels[d].m.as<uint64_t>();
    L.base = levels[d].base.as<uint32_t>();
    L.list = levels[d].list.as<int64_t>();
    L.cnt = levels[d].cnt.as<uint32_t>();
    L.bcnt = levels[d].bcnt.as<uint32_t>();
    return L;
  };

  const int32_t *lowcnt_d = g.lowcnt;
  Profiler prof(st);
  DevMem light_scratch_buf;
  int64_t light_handled = 0;

  for (int t0 = 0; t0 < trials; t0 += T) {
    int Tg = std::min(T, trials - t0);
    // colours of this trial group, rank order
    if (cs.from_seed) {
      launch_colour(g.orig, g.n, k, cs.seed, t0, Tg, d_col.as<uint8_t>(), st);
    } else {
      HIP_CHECK(hipMemcpyAsync(d_hcol.p, cs.host + (size_t)t0 * g.n, (size_t)g.n * Tg, hipMemcpyHostToDevice, st));
      launch_permute_colours(d_hcol.as<uint8_t>(), g.orig, g.n, Tg, d_col.as<uint8_t>(), st);
    }
    const uint8_t *colr = d_col.as<uint8_t>();
    HIP_CHECK(hipMemsetAsync(d_sum.p, 0, d_sum.bytes, st));
    HIP_CHECK(hipMemsetAsync(d_ovf.p, 0, d_ovf.bytes, st));
    if (per_source) HIP_CHECK(hipMemsetAsync(d_per.p, 0, d_per.bytes, st));
    AccDev acc{d_sum.as<uint64_t>(), d_ovf.as<uint32_t>(), per_source ? d_per.as<uint64_t>() : nullptr};
    uint32_t *ovf = d_ovf.as<uint32_t>();

    for (size_t bi = 0; bi < p.blocks.size(); bi++) {
      const PBlock &B = p.blocks[bi];
      if (B.kind == BK_LEAF) {
        int a = B.nodes[0];
        (void)a;
        int ec = B.edge_child[0];
        launch_leaf(gd, Tg, k, colr, tabdev(B.node_child[0]), tabdev(ec), ec >= 0 ? B.edge_first_lo[0] : 0,
                    tabdev(B.node_child[1]), tabs[bi].as<uint64_t>(), B.size, table_C(p, (int)bi), ovf, st);
        HIP_CHECK(hipGetLastError());
        continue;
      }
      if (B.kind == BK_ROOT_SINGLE) {
        TabDev u = tabdev(B.single_child);
        launch_root_single(g.n, Tg, u, acc, st);
        HIP_CHECK(hipGetLastError());
        continue;
      }
      // cycle block
      const Program &P = p.programs[bi];
      uint64_t *out = nullptr;
      int C_out = 0;
      if (B.kind == BK_CYCLE) {
        out = tabs[bi].as<uint64_t>();
        C_out = table_C(p, (int)bi);
        int64_t keys = is_edge_table(p, (int)bi) ? g.m2 : g.n;
        launch_fill_u64(out, keys * Tg * C_out, st);
      }
      for (size_t r = 0; r < P.reg_s.size(); r++) ensure_reg((int)r, P.reg_s[r]);
      for (int d = 1; d <= P.max_depth; d++) ensure_level(d);
      // NodeJoin outputs keep their input's activity mask
      std::vector<int> mown(P.reg_s.size());
      for (size_t r = 0; r < mown.size(); r++) mown[r] = (int)r;
      for (auto &op : P.ops)
        if (op.kind == OP_NJ) mown[op.dst] = mown[op.a];
      auto regdev = [&](int r) {
        RegDev d;
        d.val = regs[r].val.as<uint64_t>();
        d.mask = regs[mown[r]].mask.as<uint64_t>();
        d.C = (int)slots_pair(k, P.reg_s[r]);
        d.s = P.reg_s[r];
        return d;
      };
      auto lv = [&](int r) { return leveldev(P.reg_depth[r]); };
      struct Grp {
        const int32_t *dsrc;          // device sources of the group
        const int32_t *hsrc;          // host copy
        int64_t B;
        bool dense;
      };
      auto run_group = [&](const Grp &G) {
        GroupDev grp;
        grp.src = G.dsrc;
        grp.B = (int)G.B;
        grp.T = Tg;
        grp.k = k;
        grp.n_lim = G.hsrc[0];
        grp.dense = G.dense ? 1 : 0;
        grp.prof = nullptr;
        int max_low = 0;
        for (int64_t i = 0; i < G.B; i++) max_low = std::max(max_low, g.h_lowcnt[G.hsrc[i]]);
        std::vector<char> built(P.max_depth + 2, 0);
        std::function<void(int)> build = [&](int d) {  // sparse groups: entries of depth d
          if (G.dense || built[d]) return;
          prof.begin("level_build_sparse", false, 0, 0, 0);
          if (d == 1) {
            launch_level_init(gd, grp, lowcnt_d, max_low, leveldev(1), st);
            launch_level_compact(grp, leveldev(1), st);
          } else {
            build(d - 1);
            launch_level_next(gd, grp, leveldev(d - 1), leveldev(d), st);
          }
          HIP_CHECK(hipGetLastError());
          prof.end();
          built[d] = 1;
        };
        for (size_t oi = 0; oi < P.ops.size(); oi++) {
          const Op &op = P.ops[oi];
          static const char *names[] = {"init", "nodejoin", "edgejoin", "axpy", "merge_root",
                                        "merge_u", "merge_v", "merge_edge", "merge_edge_t"};
          std::string nm = std::string(names[op.kind]) + (G.dense ? "_dense" : "_sparse");
          if (op.kind == OP_INIT) build(1);
          if (op.kind == OP_EJ) build(P.reg_depth[op.dst]);
          if (op.kind == OP_EJ) {
            // algorithmic bytes: a 4-byte neighbour id per scanned pair, an
            // input row (plus the annotated edge's table row) per relaxation,
            // an output row per entry
            const double Cin = (double)slots_pair(k, P.reg_s[op.a]), Cout = (double)slots_pair(k, P.reg_s[op.dst]);
            const double Ce = op.tab >= 0 ? (double)table_C(p, op.tab) : 0.0;
            grp.prof = prof.begin(nm.c_str(), true, 4.0, 8.0 * (Cin + Ce), 8.0 * Tg * Cout);
          } else {
            grp.prof = nullptr;
            prof.begin(nm.c_str(), false, 0, 0, 0);
          }
          switch (op.kind) {
            case OP_INIT: {
              RegDev d = regdev(op.dst);
              if (G.dense) {
                launch_fill_u64(d.val, grp.n_lim * grp.B * (int64_t)Tg * d.C, st);
                launch_fill_u64(d.mask, grp.n_lim, st);
              }
              launch_init(gd, grp, lowcnt_d, max_low, colr, lv(op.dst), d, tabdev(op.tab), op.tab_src_first,
                          tabdev(op.ntab), ovf, st);
              break;
            }
            case OP_NJ:
              launch_nj(gd, grp, colr, lv(op.a), regdev(op.a), regdev(op.dst), tabdev(op.tab), ovf, st);
              break;
            case OP_EJ:
              launch_ej(gd, grp, colr, lv(op.a), lv(op.dst), regdev(op.a), regdev(op.dst), tabdev(op.tab),
                        op.tab_src_first, ovf, st);
              break;
            case OP_AXPY:
              launch_axpy(grp, lv(op.a), regdev(op.a), regdev(op.dst), op.w, op.first, ovf, st);
              break;
            case OP_MROOT:
              launch_mroot(grp, g.n, colr, lv(op.a), lv(op.b), regdev(op.a), regdev(op.b), op.w, acc, st);
              break;
            case OP_MU:
            case OP_MV:
              launch_munary(grp, g.n, colr, lv(op.a), lv(op.b), regdev(op.a), regdev(op.b), op.w,
                            op.kind == OP_MU, out, op.s, C_out, ovf, st);
              break;
            case OP_MEDGE:
              launch_medge(gd, grp, colr, lv(op.a), lv(op.b), regdev(op.a), regdev(op.b), tabdev(op.tab),
                           op.tab_src_first, op.first, op.w, out, op.s, C_out, ovf, st);
              break;
            case OP_MEDGE_T:
              launch_medge_t(gd, grp, colr, lowcnt_d, max_low, tabdev(op.ntab), lv(op.b), regdev(op.b),
                             tabdev(op.tab), op.tab_src_first, op.first, op.w, out, op.s, C_out, ovf, st);
              break;
          }
          HIP_CHECK(hipGetLastError());
          prof.end();
        }
        for (int d = 1; d <= P.max_depth; d++)
          if (built[d]) launch_level_reset(grp, leveldev(d), st);
      };
      // 1. dense groups: the sources with the widest reach
      for (int64_t i = 0; i < ndense; i += z.B_dense)
        run_group({d_src.as<int32_t>() + i, sources.data() + i, std::min<int64_t>(z.B_dense, ndense - i), true});
      // 2. one workgroup per source for the rest; 3. grouped sparse path for what does not fit
      std::vector<int32_t> rest(sources.begin() + ndense, sources.end());
      const int64_t nrest = (int64_t)rest.size();
      bool light_ok = use_light && nrest > 0 && P.max_depth <= light_max_depth() &&
                      (int)P.reg_s.size() <= light_max_regs();
      if (light_ok) {
        std::vector<LOp> lops;
        for (auto &o : P.ops)
          lops.push_back({(int)o.kind, o.dst, o.a, o.b, o.tab, o.tab_src_first, o.ntab, o.s, o.first, o.swapped,
                          o.w});
        std::vector<int32_t> rd(P.reg_s.size()), rC(P.reg_s.size()), rs(P.reg_s.size());
        for (size_t r = 0; r < P.reg_s.size(); r++) {
          rd[r] = P.reg_depth[r];
          rC[r] = (int32_t)slots_pair(k, P.reg_s[r]);
          rs[r] = P.reg_s[r];
        }
        std::vector<TabDev> tv(p.blocks.size());
        for (size_t b2 = 0; b2 < p.blocks.size(); b2++) tv[b2] = tabdev(tabs[b2].p ? (int)b2 : -1);
        DevMem d_ops(sizeof(LOp) * lops.size()), d_rd(4 * rd.size()), d_rC(4 * rC.size()), d_rs(4 * rs.size());
        DevMem d_tv(sizeof(TabDev) * tv.size()), d_ctr(8), d_fail(4 * nrest);
        HIP_CHECK(hipMemcpyAsync(d_ops.p, lops.data(), sizeof(LOp) * lops.size(), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipMemcpyAsync(d_rd.p, rd.data(), 4 * rd.size(), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipMemcpyAsync(d_rC.p, rC.data(), 4 * rC.size(), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipMemcpyAsync(d_rs.p, rs.data(), 4 * rs.size(), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipMemcpyAsync(d_tv.p, tv.data(), sizeof(TabDev) * tv.size(), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipMemsetAsync(d_ctr.p, 0, 8, st));
        int ncu = 0;
        HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, g.device));
        int grid = std::max(1, ncu) * 3;
        if (light_scratch_buf.bytes < (size_t)light_scratch * grid) light_scratch_buf.alloc((size_t)light_scratch * grid);
        DevMem d_rest(4 * nrest);
        HIP_CHECK(hipMemcpyAsync(d_rest.p, rest.data(), 4 * nrest, hipMemcpyHostToDevice, st));
        LightArgs la;
        la.g = gd;
        la.lowcnt = lowcnt_d;
        la.colr = colr;
        la.T = Tg;
        la.k = k;
        la.src = d_rest.as<int32_t>();
        la.nsrc = (int)nrest;
        la.next = d_ctr.as<uint32_t>();
        la.fail = d_fail.as<int32_t>();
        la.nfail = d_ctr.as<uint32_t>() + 1;
        la.ops = d_ops.as<LOp>();
        la.nops = (int)lops.size();
        la.reg_depth = d_rd.as<int32_t>();
        la.reg_C = d_rC.as<int32_t>();
        la.reg_s = d_rs.as<int32_t>();
        la.nregs = (int)rd.size();
        la.D = P.max_depth;
        la.tabs = d_tv.as<TabDev>();
        la.out = out;
        la.s_out = B.size;
        la.C_out = C_out;
        la.acc = acc;
        la.scratch = light_scratch_buf.as<uint8_t>();
        la.scratch_per_wg = light_scratch;
        la.lut = lut_device(g.device);
        prof.begin("light", false, 0, 0, 0);
        launch_light(la, grid, st);
        HIP_CHECK(hipGetLastError());
        prof.end();
        uint32_t hc[2];
        HIP_CHECK(hipMemcpyAsync(hc, d_ctr.p, 8, hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        rest.resize(hc[1]);
        if (hc[1]) HIP_CHECK(hipMemcpy(rest.data(), d_fail.p, 4 * (size_t)hc[1], hipMemcpyDeviceToHost));
        std::sort(rest.begin(), rest.end(), std::greater<int32_t>());
        light_handled += nrest - (int64_t)hc[1];
      }
      if (!rest.empty()) {
        DevMem d_f(4 * rest.size());
        HIP_CHECK(hipMemcpyAsync(d_f.p, rest.data(), 4 * rest.size(), hipMemcpyHostToDevice, st));
        // what the one-workgroup path handed back has wide reach: dense groups,
        // unless every path is forced sparse
        bool fdense = false;
        if (const char *ev = getenv("CC_FALLBACK"))
          if (!strcmp(ev, "dense")) fdense = true;
        for (int64_t i = 0; i < (int64_t)rest.size(); i += z.B_sparse)
          run_group({d_f.as<int32_t>() + i, rest.data() + i, std::min<int64_t>(z.B_sparse, (int64_t)rest.size() - i),
                     fdense});
        HIP_CHECK(hipStreamSynchronize(st));
      }
    }
    // results of this trial group
    std::vector<uint64_t> hs(2 * 64);
    std::vector<uint32_t> ho(64);
    HIP_CHECK(hipMemcpyAsync(hs.data(), d_sum.p, sizeof(uint64_t) * 2 * 64, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(ho.data(), d_ovf.p, sizeof(uint32_t) * 64, hipMemcpyDeviceToHost, st));
    std::vector<uint64_t> hp;
    if (per_source) {
      hp.resize(2 * (size_t)g.n * Tg);
      HIP_CHECK(hipMemcpyAsync(hp.data(), d_per.p, sizeof(uint64_t) * hp.size(), hipMemcpyDeviceToHost, st));
    }
    HIP_CHECK(hipStreamSynchronize(st));
    prof.finish();
    for (int t = 0; t < Tg; t++) {
      res.exact[t0 + t] = (u128)hs[2 * t] | ((u128)hs[2 * t + 1] << 64);
      res.overflow[t0 + t] = ho[t] ? 1 : 0;
    }
    if (per_source)
      for (int64_t r = 0; r < g.n; r++)
        for (int t = 0; t < Tg; t++) {
          size_t i = 2 * ((size_t)r * Tg + t);
          (*per_source)[(size_t)(t0 + t) * g.n + g.h_orig[r]] = (u128)hp[i] | ((u128)hp[i + 1] << 64);
        }
  }
  return res;
}

}  // namespace cc
