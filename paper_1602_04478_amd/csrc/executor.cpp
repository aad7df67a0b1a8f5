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
#include <chrono>
#include <memory>
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

// Device memory of the solves is recycled: a released block goes to a
// per-device cache and is handed out again for a request of similar size, so
// solves do not pay hipMalloc / hipFree (whose implicit device-wide
// synchronisation would also serialise solves running side by side).  Blocks
// are released only after the owning solve has synchronised its stream.
struct BlockCache {
  std::mutex mu;
  std::map<int, std::multimap<size_t, void *>> free;  // device -> size -> block
  std::map<int, size_t> cached;
};
BlockCache &block_cache() {
  static BlockCache *c = new BlockCache;  // outlives every solve
  return *c;
}
size_t round_block(size_t b) {
  if (b < ((size_t)1 << 20)) return (b + 255) & ~(size_t)255;
  size_t q = ((size_t)1 << (63 - __builtin_clzll(b))) / 8;  // 8 size classes per power of two
  return (b + q - 1) / q * q;
}
int cur_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}
void *cache_take(int dev, size_t b, size_t &got) {
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto &fl = c.free[dev];
  auto it = fl.lower_bound(b);
  if (it == fl.end() || it->first > b + b / 4) return nullptr;
  void *p = it->second;
  got = it->first;
  c.cached[dev] -= got;
  fl.erase(it);
  return p;
}
void cache_give(int dev, void *p, size_t b) {
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.free[dev].insert({b, p});
  c.cached[dev] += b;
}
void cache_trim(int dev) {
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto &kv : c.free[dev]) (void)hipFree(kv.second);
  c.free[dev].clear();
  c.cached[dev] = 0;
}
size_t cache_bytes(int dev) {
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  return c.cached[dev];
}

// An allocation-free solve carves its device buffers from a caller-given
// region instead (see ExecOptions::arena): blocks are never returned to it,
// the whole region is reused by the next such solve.
struct Arena {
  uint8_t *base = nullptr;
  size_t size = 0, used = 0;
};
thread_local Arena *g_arena = nullptr;

struct DevMem {
  void *p = nullptr;
  size_t bytes = 0;
  int dev = 0;
  bool carved = false;  // from the arena (not the block cache)
  DevMem() = default;
  explicit DevMem(size_t b) { alloc(b); }
  void alloc(size_t b) {
    release();
    if (b == 0) b = 8;
    if (g_arena) {
      const size_t a = (b + 255) & ~(size_t)255;
      if (g_arena->used + a > g_arena->size)
        fail(CC_E_NOMEM, "the solve needs more than the static scratch of " + std::to_string(g_arena->size) +
                             " bytes");
      p = g_arena->base + g_arena->used;
      g_arena->used += a;
      bytes = a;
      carved = true;
      return;
    }
    b = round_block(b);
    dev = cur_device();
    size_t got = 0;
    if ((p = cache_take(dev, b, got))) {
      bytes = got;
      return;
    }
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {  // give the cached blocks back to the device and retry once
      (void)hipGetLastError();
      cache_trim(dev);
      e = hipMalloc(&p, b);
    }
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      fail(CC_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
    }
    bytes = b;
  }
  void release() {
    if (p && !carved) cache_give(dev, p, bytes);
    p = nullptr;
    bytes = 0;
    carved = false;
  }
  ~DevMem() { release(); }
  DevMem(const DevMem &) = delete;
  DevMem &operator=(const DevMem &) = delete;
  DevMem(DevMem &&o) noexcept : p(o.p), bytes(o.bytes), dev(o.dev), carved(o.carved) {
    o.p = nullptr;
    o.bytes = 0;
    o.carved = false;
  }
  DevMem &operator=(DevMem &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      dev = o.dev;
      carved = o.carved;
      o.p = nullptr;
      o.bytes = 0;
      o.carved = false;
    }
    return *this;
  }
  template <typename T>
  T *as() const {
    return (T *)p;
  }
};

struct RegBuf {
  DevMem val, mask;
};
struct LevelBuf {
  DevMem mb, list, cnt, bcnt, vlist;
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

uint64_t table_bytes(const DevGraph &g, const Plan &p, int T) {
  uint64_t b = 0;
  for (size_t i = 0; i < p.blocks.size(); i++) {
    const PBlock &B = p.blocks[i];
    if (B.kind == BK_ROOT_CYCLE || B.kind == BK_ROOT_SINGLE || B.pair_keyed) continue;
    uint64_t keys = is_edge_table(p, (int)i) ? (uint64_t)g.m2 : (uint64_t)g.n;
    b += keys * (uint64_t)T * table_C(p, (int)i) * 8;
  }
  return b;
}

uint64_t free_bytes() {  // free on the device, counting the recycled blocks as free
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return 0;
  return (uint64_t)fr + cache_bytes(cur_device());
}

// scratch of the one-workgroup tier per workgroup: enough for the frontiers a
// graph of this size can have, within 2 MiB (larger frontiers are handed back)
int64_t light_scratch_bytes(const DevGraph &g, int T) {
  int64_t b = (int64_t)g.n * T * 128;
  if (const char *ev = getenv("CC_LIGHT_SCRATCH")) return std::max<int64_t>(4096, atoll(ev));
  return std::max<int64_t>(64 << 10, std::min<int64_t>(b, 2 << 20));
}
bool large_light_on() {
  const char *ev = getenv("CC_LIGHT_LARGE");
  return ev && *ev == '1';
}
int light_grid(int device) {
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) ncu = 256;
  return std::max(1, ncu) * 3;
}

// Device bytes of a solve with trial groups of T: a part that does not
// depend on the sources per group B and a part per source of B.
struct Bytes {
  uint64_t fixed, per_B;
};
Bytes solver_bytes(const DevGraph &g, const Plan &p, int T, bool noalloc = false) {
  const uint64_t n = (uint64_t)std::max<int64_t>(1, g.n);
  // registers are pooled by index across the programs: register r holds the
  // widest row any program puts there
  std::vector<uint64_t> rmax;
  int dmax = 1;
  for (auto &P : p.programs) {
    if (rmax.size() < P.reg_s.size()) rmax.resize(P.reg_s.size(), 0);
    for (size_t r = 0; r < P.reg_s.size(); r++) rmax[r] = std::max<uint64_t>(rmax[r], slots_pair(p.k, P.reg_s[r]));
    dmax = std::max(dmax, P.max_depth);
  }
  uint64_t slots = 0;
  for (auto c : rmax) slots += c;
  const uint64_t nregs = rmax.size();
  Bytes b;
  b.fixed = table_bytes(g, p, T) + 2 * n * T                   // tables, colours (+ host-colour staging)
            + nregs * 8 * n                                    // activity masks
            + (uint64_t)dmax * (16 * n + 4 * (n / 4096 + 2))   // level marks and bases
            + (noalloc ? (uint64_t)(1 << 20)  // no one-workgroup tier; alignment of the carved buffers
                       : (uint64_t)light_scratch_bytes(g, T) * light_grid(g.device) + (64 << 20) +
                             (large_light_on() ? (uint64_t)(32 << 20) * (light_grid(g.device) / 3) : 0));
  b.per_B = 8 * n * T * slots + (uint64_t)dmax * 8 * n;        // registers, level lists
  return b;
}

Sizing choose(const DevGraph &g, const Plan &p, int trials, const ExecOptions &opt, uint64_t budget) {
  Sizing z{};
  z.T = opt.trial_group > 0 ? std::min(opt.trial_group, 64) : std::min(trials, 64);
  if (z.T < 1) z.T = 1;
  // one workgroup covers every (source, trial, slot) of a vertex
  int cmax = 1;
  for (auto &P : p.programs)
    for (int s : P.reg_s) cmax = std::max(cmax, (int)slots_pair(p.k, s));
  for (auto &B2 : p.blocks)
    if (B2.kind == BK_CYCLE) cmax = std::max(cmax, (int)binom(p.k - 1, B2.size - 1));
  if (cmax > max_row_slots()) fail(CC_E_UNSUPPORTED, "signature tables too wide for one workgroup");
  while ((int64_t)z.T * cmax > max_row_slots()) z.T = std::max(1, z.T / 2);
  for (;;) {
    Bytes b = solver_bytes(g, p, z.T, opt.arena != nullptr);
    int64_t B = budget > b.fixed && b.per_B ? (int64_t)((budget - b.fixed) / b.per_B) : 0;
    if (B >= 1 || z.T == 1) {
      if (B < 1) fail(CC_E_NOMEM, "plan does not fit the device memory budget");
      B = std::min<int64_t>(B, 64);
      if (opt.group_sources > 0) B = std::min<int64_t>(B, opt.group_sources);
      z.B_dense = (int)B;
      z.B_sparse = (int)B;
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
int g_prof_on = 0;  // 1: per-launch event timing; 2: also the kernels' work counters; 3: events around EdgeJoins only
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

// CC_PROFILE_BY_OP=1: one profile record per operation of a program
static bool by_op() {
  static const bool on = [] {
    const char *ev = getenv("CC_PROFILE_BY_OP");
    return ev && *ev == '1';
  }();
  return on;
}

struct Profiler {
  bool on = false, counting = false, ej_only = false;
  bool skipped = false;  // the current launch is not timed (level 3, not an EdgeJoin)
  hipStream_t st;
  struct Rec {
    std::string name;
    hipEvent_t a, b;
    int ctr;            // counter triple index, or -1
    double per_scan, per_active, per_entry;  // bytes per unit of each counter
    double fixed;       // algorithmic bytes known on the host (no counters)
  };
  std::vector<Rec> recs;
  std::vector<uint64_t *> ctrs;
  static constexpr int kMaxCtr = 65536;  // records with counters per solve (larger graphs have more groups)
  int nctr = 0;
  DevMem ctrmem;
  explicit Profiler(hipStream_t s, bool allowed = true) : st(s) {
    if (!allowed) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    on = g_prof_on >= 1;
    counting = g_prof_on == 2;
    ej_only = g_prof_on == 3;
    if (counting) ctrmem.alloc(sizeof(uint64_t) * 3 * PROF_LANES * kMaxCtr);
  }
  // returns a zeroed counter triple for an EdgeJoin launch (or null)
  uint64_t *begin(const char *name, bool counters, double per_scan, double per_active, double per_entry) {
    if (!on) return nullptr;
    skipped = ej_only && strncmp(name, "edgejoin", 8) != 0;
    if (skipped) return nullptr;
    Rec r;
    r.name = name;
    r.ctr = -1;
    uint64_t *c = nullptr;
    if (counters && counting && nctr < kMaxCtr) {
      r.ctr = nctr++;
      c = ctrmem.as<uint64_t>() + (size_t)3 * PROF_LANES * r.ctr;
      launch_fill_u64(c, 3 * PROF_LANES, st);
    }
    r.a = take_event();
    r.b = take_event();
    HIP_CHECK(hipEventRecord(r.a, st));
    r.per_scan = per_scan;
    r.per_active = per_active;
    r.per_entry = per_entry;
    r.fixed = 0;
    recs.push_back(r);
    return c;
  }
  // forget the current record (nothing was launched for it)
  void drop() {
    if (skipped) {
      skipped = false;
      return;
    }
    if (!on || recs.empty()) return;
    give_event(recs.back().a);
    give_event(recs.back().b);
    if (recs.back().ctr == nctr - 1 && nctr > 0) nctr--;
    recs.pop_back();
  }
  // the current record's operation name (a launch that turned out to be another kind)
  void rename(const std::string &nm) {
    if (on && !skipped && !recs.empty()) recs.back().name = nm;
  }
  // algorithmic bytes of the current record computed on the host
  void add_fixed(double bytes) {
    if (on && !skipped && !recs.empty()) recs.back().fixed += bytes;
  }
  void end() {
    if (!on) return;
    if (skipped) {
      skipped = false;
      return;
    }
    HIP_CHECK(hipEventRecord(recs.back().b, st));
  }
  void finish() {
    if (!on) return;
    HIP_CHECK(hipStreamSynchronize(st));
    std::vector<uint64_t> hl((size_t)3 * PROF_LANES * std::max(1, nctr)), h(3 * (size_t)std::max(1, nctr), 0);
    if (nctr)
      HIP_CHECK(hipMemcpyAsync(hl.data(), ctrmem.p, sizeof(uint64_t) * 3 * PROF_LANES * nctr, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    for (int r = 0; r < nctr; r++)
      for (int l = 0; l < PROF_LANES; l++)
        for (int i = 0; i < 3; i++) h[3 * r + i] += hl[((size_t)r * PROF_LANES + l) * 3 + i];
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : recs) {
      float ms = 0;
      HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
      ProfStat &p = g_prof[r.name];
      p.launches++;
      p.seconds += ms * 1e-3;
      p.bytes += r.fixed;
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

void profile_enable(int level) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = level < 0 ? 0 : level > 3 ? 3 : level;
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

double probe_copy(uint64_t bytes, int reps) {
  DevMem a(bytes), b(bytes);
  hipStream_t st;
  HIP_CHECK(hipStreamCreate(&st));
  launch_fill_u64(a.as<uint64_t>(), (int64_t)(bytes / 8), st);
  launch_copy16(a.p, b.p, (int64_t)(bytes / 16), st);  // warm
  hipEvent_t e0 = take_event(), e1 = take_event();
  HIP_CHECK(hipEventRecord(e0, st));
  for (int i = 0; i < reps; i++) launch_copy16(a.p, b.p, (int64_t)(bytes / 16), st);
  HIP_CHECK(hipEventRecord(e1, st));
  HIP_CHECK(hipStreamSynchronize(st));
  float ms = 0;
  HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
  give_event(e0);
  give_event(e1);
  (void)hipStreamDestroy(st);
  return 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
}


uint64_t footprint(const DevGraph &g, const Plan &p, int trials, const ExecOptions &opt) {
  int T = std::min(std::max(trials, 1), 64);
  if (opt.trial_group > 0) T = std::min(T, opt.trial_group);
  int B = opt.group_sources > 0 ? std::min(opt.group_sources, 64) : 64;
  Bytes b = solver_bytes(g, p, T);
  return b.fixed + b.per_B * (uint64_t)B;
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

// ------------------------------------------------------------------ fused schedule
//
// For the grouped path, a cycle program is regrouped into steps: a plain op,
// or an EdgeJoin followed by the row-local ops (NodeJoin, AXPY, root merge)
// that can run on its output vertex while the EdgeJoin row is in LDS.  A
// register computed in such an epilogue is written to memory only if an op
// after the step reads it.  An AXPY chain d = sum_k w_k x_k is rebuilt so that
// a local term that dies there lends d its LDS block (scaled in place).
struct EpiPlan {
  std::vector<int> ops;      // NJ/MROOT op indices, or -1 - k for the k-th rebuilt AXPY
  struct Axpy {
    int dst, a;
    uint64_t w;
    int first;
  };
  std::vector<Axpy> axpy;
  std::vector<int> regs;     // epilogue register -> program register (0: the EdgeJoin's output)
  std::vector<int> col;      // LDS column of each epilogue register, -1: global
  std::vector<int> write;
  int ncols = 0;
};
struct Step {
  int op;                    // the op (an EdgeJoin when fused)
  bool fused = false;
  EpiPlan epi;
};

static std::vector<Step> schedule(const Program &P, int k) {
  const int n = (int)P.ops.size();
  auto reads = [&](const Op &o, int r) {
    if (o.a == r || (o.kind == OP_MROOT || o.kind == OP_MU || o.kind == OP_MV || o.kind == OP_MEDGE ||
                     o.kind == OP_MEDGE_T || o.kind == OP_MPAIR) && o.b == r)
      return true;
    return o.kind == OP_AXPY && !o.first && o.dst == r;
  };
  auto used_from = [&](int r, int j) {
    for (int q = j; q < n; q++)
      if (reads(P.ops[q], r)) return true;
    return false;
  };
  std::vector<char> mat(P.reg_s.size(), 0);  // in memory after the steps so far
  std::vector<Step> out;
  int i = 0;
  while (i < n) {
    const Op &op = P.ops[i];
    if (op.kind != OP_EJ) {
      out.push_back({i, false, {}});
      if (op.dst >= 0) mat[op.dst] = 1;
      i++;
      continue;
    }
    const int depth = P.reg_depth[op.dst];
    std::vector<char> loc(P.reg_s.size(), 0);
    loc[op.dst] = 1;
    int j = i + 1;
    for (; j < n; j++) {
      const Op &o = P.ops[j];
      if (o.kind != OP_NJ && o.kind != OP_AXPY && o.kind != OP_MROOT) break;
      auto avail = [&](int r) { return r >= 0 && (loc[r] || mat[r]); };
      bool ok = avail(o.a);
      if (o.kind == OP_MROOT) ok = ok && avail(o.b) && (loc[o.a] || loc[o.b]);
      if (o.kind != OP_MROOT) ok = ok && P.reg_depth[o.dst] == depth && !mat[o.dst];
      if (o.kind == OP_NJ) ok = ok && o.tab >= 0;
      if (o.kind == OP_AXPY && !o.first) ok = ok && loc[o.dst];
      if (ok && o.kind == OP_AXPY && o.first) {
        // the chain is rebuilt here: every term must be ready now, and no op
        // before its last link may read the partial sum
        int last = j;
        for (int q2 = j; q2 < n; q2++) {
          const Op &o2 = P.ops[q2];
          if (o2.kind != OP_NJ && o2.kind != OP_AXPY && o2.kind != OP_MROOT) break;
          if (o2.kind == OP_AXPY && o2.dst == o.dst) last = q2;
        }
        for (int q2 = j; q2 <= last && ok; q2++) {
          const Op &o2 = P.ops[q2];
          if (o2.kind == OP_AXPY && o2.dst == o.dst) ok = avail(o2.a) && !(q2 > j && o2.first);
          else ok = !reads(o2, o.dst);
        }
      }
      if (!ok) break;
      if (o.kind != OP_MROOT) loc[o.dst] = 1;
    }
    Step stp{i, j > i + 1, {}};
    if (!stp.fused) {
      out.push_back(stp);
      mat[op.dst] = 1;
      i++;
      continue;
    }
    EpiPlan &E = stp.epi;
    auto reg_of = [&](int r) {
      for (size_t q = 0; q < E.regs.size(); q++)
        if (E.regs[q] == r) return (int)q;
      E.regs.push_back(r);
      E.col.push_back(-1);
      E.write.push_back(0);
      return (int)E.regs.size() - 1;
    };
    auto new_block = [&](int e) {
      E.col[e] = E.ncols;
      E.ncols += (int)slots_pair(k, P.reg_s[E.regs[e]]);
    };
    new_block(reg_of(op.dst));
    // registers that leave the step
    auto leaves = [&](int r) { return used_from(r, j); };
    for (int q = i + 1; q < j; q++) {
      const Op &o = P.ops[q];
      if (o.kind == OP_NJ || o.kind == OP_MROOT) {
        if (o.kind == OP_NJ) new_block(reg_of(o.dst));
        reg_of(o.a);
        if (o.kind == OP_MROOT) reg_of(o.b);
        E.ops.push_back(q);
        continue;
      }
      // AXPY: a chain building o.dst from here
      if (!o.first) {  // a later link of a chain already rebuilt
        continue;
      }
      std::vector<std::pair<int, uint64_t>> terms;  // (register, weight)
      int last = q;
      for (int q2 = q; q2 < j; q2++) {
        const Op &o2 = P.ops[q2];
        if (o2.kind == OP_AXPY && o2.dst == o.dst) {
          terms.push_back({o2.a, o2.w});
          last = q2;
        }
      }
      // a local term that dies here lends its block
      int lend = -1;
      for (size_t t = 0; t < terms.size() && lend < 0; t++) {
        const int r = terms[t].first;
        if (!loc[r] || leaves(r)) continue;
        bool later = false;
        for (int q3 = last + 1; q3 < j; q3++) later |= reads(P.ops[q3], r);
        for (size_t t2 = 0; t2 < terms.size(); t2++) later |= t2 != t && terms[t2].first == r;
        if (!later) lend = (int)t;
      }
      const int d = reg_of(o.dst);
      if (lend >= 0) {
        const int x = reg_of(terms[lend].first);
        E.col[d] = E.col[x];
        E.axpy.push_back({d, x, terms[lend].second, 1});
      } else {
        new_block(d);
        E.axpy.push_back({d, reg_of(terms[0].first), terms[0].second, 1});
      }
      E.ops.push_back(-1 - (int)(E.axpy.size() - 1));
      for (size_t t = 0; t < terms.size(); t++) {
        if ((int)t == (lend >= 0 ? lend : 0)) continue;
        E.axpy.push_back({d, reg_of(terms[t].first), terms[t].second, 0});
        E.ops.push_back(-1 - (int)(E.axpy.size() - 1));
      }
    }
    for (size_t e = 0; e < E.regs.size(); e++) {
      const int r = E.regs[e];
      if (E.col[e] >= 0 && leaves(r)) {
        E.write[e] = 1;
        mat[r] = 1;
      }
    }
    out.push_back(stp);
    i = j;
  }
  return out;
}

// ------------------------------------------------------------------ solver
//
// A Solver holds everything one (graph, plan, trial-group size) needs on the
// device: colours, child tables, frontier registers, levels, the one-workgroup
// tier's program and its scratch.  After the first trial group -- which learns
// which sources the one-workgroup tier hands back (that depends only on the
// graph and the program) -- the launch sequence of a trial group is fixed:
// no allocation, no host synchronisation, every clear a kernel.  It can then
// be captured once in a hipGraph and replayed per trial group, the seed and
// first trial read from device memory.
class Solver {
 public:
  Solver(const DevGraph &g, const Plan &p, int trials, const ExecOptions &opt, hipStream_t st);
  ~Solver();
  // trials [t0, t0 + Tg) into res (and per_source, indexed [t][orig id])
  void run_group_of_trials(int t0, int Tg, const ColourSource &cs, CountResult &res, std::vector<u128> *per_source);
  int T() const { return z_.T; }
  int64_t ndense() const { return ndense_; }
  SolveStats stats() const {
    SolveStats s;
    s.sources = (int64_t)sources_.size();
    s.dense = ndense_;
    s.trial_group = z_.T;
    s.group_sources = z_.B_dense;
    for (size_t bi = 0; bi < p_.blocks.size(); bi++) {
      if (p_.blocks[bi].kind != BK_CYCLE && p_.blocks[bi].kind != BK_ROOT_CYCLE) continue;
      s.sources = (int64_t)bx_[bi].src.size();
      s.dense = bx_[bi].ndense;
      const Light &L = light2_[bi].large ? light2_[bi] : light_[bi];
      s.light = (int64_t)(light_[bi].src.size() + (light2_[bi].large ? light2_[bi].src.size() : 0));
      s.handed_back = (int64_t)L.fails.size();
    }
    return s;
  }
  uint64_t graph_replays = 0;

 private:
  struct Grp {
    const int32_t *dsrc;  // device sources of the group
    const int32_t *hsrc;  // host copy
    int64_t B;
    bool dense;
  };
  struct Light {  // one stage of a cycle block's one-workgroup tier
    bool probed = false;
    bool large = false;          // the big-LDS kernel (takes what the small one hands back)
    std::vector<int32_t> src;    // sources it runs
    std::vector<int32_t> fails;  // sources it hands back (descending)
    DevMem d_ops, d_rd, d_rC, d_rs, d_tv, d_ctr, d_fail, d_src, d_fails;
    LightArgs la{};
    int grid = 0;
  };
  // How a cycle block runs its sources.  Degree-based blocks share the
  // library's sources (at least two lower neighbours) and dense cut.  A
  // path-splitting block (filter off) takes every vertex with a neighbour as
  // a source.  A block that reads a pair-keyed table (an edge of its cycle is
  // annotated by a block whose two boundary nodes are not adjacent) walks
  // that table's graph and runs every vertex in dense groups, as does the
  // pair-keyed block itself.
  struct BlockExec {
    bool nofilter = false, all_dense = false;
    std::vector<int32_t> src;  // descending rank
    int64_t ndense = 0;
    DevMem d_src;
  };
  // A pair-keyed table: its entries (u, v) are listed by the merges, then
  // laid out as a graph H of its own (symmetric CSR over the pairs, rows
  // sorted, reverse slots) whose slots the table's rows are aligned to, as
  // edge tables are aligned to the data graph's slots.  Rebuilt per trial
  // group (the nonzero pairs depend on the colourings).
  struct PairTab {
    int64_t m2 = 0;
    std::vector<int32_t> h_lowcnt, h_deg;
    DevMem rp, col, rev, lowcnt, deg, idx;
    DevMem keys, vals, cnt, stage_val, stage_mask;
    uint64_t cap = 0;
  };
  void run_light(Light &L, bool probe, int Tg, Profiler *prof);
  void enqueue(int Tg, bool seed_dev, bool probe, Profiler *prof);
  void enqueue_block(size_t bi, int Tg, bool probe, Profiler *prof);
  void run_group(size_t bi, const Program &P, const Grp &G, int Tg, uint64_t *out, int C_out, Profiler *prof);
  void finish_pairs(size_t bi, int Tg);
  bool pair_tab(int tab) const { return tab >= 0 && p_.blocks[tab].pair_keyed; }
  // the graph whose slots a child table is aligned to (the data graph, or a pair table's)
  GraphDev graph_of(int tab) const {
    if (!pair_tab(tab)) return gd_;
    const PairTab &P = pt_[tab];
    return GraphDev{P.rp.as<int64_t>(), P.col.as<int32_t>(), P.rev.as<int64_t>(), g_.n, P.m2};
  }
  // per vertex: the neighbours a walk may take first over that graph (lower
  // ones, or all with the filter off), on the device and its maximum over a group
  const int32_t *cnt_of(int tab, bool nofilter) const {
    if (!pair_tab(tab)) return nofilter ? g_.deg : g_.lowcnt;
    return nofilter ? pt_[tab].deg.as<int32_t>() : pt_[tab].lowcnt.as<int32_t>();
  }
  int max_cnt(int tab, bool nofilter, const Grp &G) const {
    const std::vector<int32_t> &c =
        !pair_tab(tab) ? (nofilter ? g_.h_deg : g_.h_lowcnt) : (nofilter ? pt_[tab].h_deg : pt_[tab].h_lowcnt);
    int m = 0;
    for (int64_t i = 0; i < G.B; i++) m = std::max(m, c[G.hsrc[i]]);
    return m;
  }
  TabDev tabdev(int blk) const {
    TabDev t{nullptr, 0, 0};
    if (blk >= 0) {
      t.val = tabs_[blk].as<uint64_t>();
      t.C = table_C(p_, blk);
      t.s = p_.blocks[blk].size;
    }
    return t;
  }
  LevelDev leveldev(int d) {
    LevelDev L;
    L.mb = levels_[d].mb.as<uint64_t>();
    L.list = levels_[d].list.as<int64_t>();
    L.cnt = levels_[d].cnt.as<uint32_t>();
    L.bcnt = levels_[d].bcnt.as<uint32_t>();
    L.vlist = levels_[d].vlist.as<int32_t>();
    return L;
  }

  const DevGraph &g_;
  const Plan &p_;
  ExecOptions opt_;
  hipStream_t st_;
  Sizing z_{};
  GraphDev gd_{};
  std::vector<int32_t> sources_;
  int64_t ndense_ = 0;
  std::vector<BlockExec> bx_;
  std::vector<PairTab> pt_;
  bool has_pairs_ = false;
  bool use_light_ = true, fallback_dense_ = false;
  int64_t light_scratch_ = 2 << 20;
  int64_t nlim_max_ = 1;
  DevMem d_src_, d_col_, d_sum_, d_ovf_, d_per_, d_hcol_, d_param_;
  bool per_alloc_ = false;
  std::vector<DevMem> tabs_;
  std::vector<RegBuf> regs_;
  std::vector<LevelBuf> levels_;
  std::vector<Light> light_;   // small stage per block
  std::vector<Light> light2_;  // large stage per block (used when use_large_)
  bool use_large_ = false;
  int64_t light_scratch_large_ = 32 << 20;
  DevMem light_scratch_buf_, light_scratch_large_buf_;
  AccDev acc_{};
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
  int exec_T_ = 0;
  hipStream_t own_st_ = nullptr;
};

Solver::Solver(const DevGraph &g, const Plan &p, int trials, const ExecOptions &opt, hipStream_t st)
    : g_(g), p_(p), opt_(opt), st_(st) {
  if (trials < 1) fail(CC_E_ARG, "trials must be >= 1");
  HIP_CHECK(hipSetDevice(g.device));
  if (!st_ && !opt.arena) {  // the null stream cannot be captured: work on a stream of our own
    HIP_CHECK(hipStreamCreateWithFlags(&own_st_, hipStreamNonBlocking));
    st_ = own_st_;
    st = st_;
  }
  const int k = p.k;
  if (!ejmaps_prepare(k)) fail(CC_E_DEVICE, "EdgeJoin slot maps: device allocation failed");
  uint64_t budget = opt.arena ? opt.arena_bytes : opt.mem_budget ? opt.mem_budget : (uint64_t)(free_bytes() * 0.85);
  z_ = choose(g, p, trials, opt, budget);
  const int T = z_.T;
  gd_ = GraphDev{g.rp, g.col, g.rev, g.n, g.m2};

  // sources: lowcnt >= 2, descending rank
  for (int64_t r = g.n - 1; r >= 0; r--)
    if (g.h_lowcnt[r] >= 2) sources_.push_back((int32_t)r);
  // dense cut.  A dense group scans every edge below its top source once per
  // level (cost ~ rp[u], the directed edges of the vertices below u); a
  // source in a sparse group costs about its two-step high-start reach r2(u).
  // A source goes dense while 64 sources like it would cost the grouped
  // sparse path more than one dense group: r2(u) * 64 * kappa >= rp[u], with
  // kappa = 13 measured on the 1e6-vertex power-law workload (dense cuts of
  // 0 .. 24576 sources: best near 3072).
  for (size_t i = 0; i < sources_.size(); i++) {
    const int64_t u = sources_[i];
    if (g.h_r2[u] * 64 * 13 >= g.h_rp[u] && u > 4096) ndense_ = (int64_t)i + 1;
    else break;
  }
  if (opt.dense_sources >= 0) ndense_ = std::min<int64_t>(opt.dense_sources, (int64_t)sources_.size());
  // CC_DENSE=all / none overrides the choice (used to exercise both paths)
  if (const char *ev = getenv("CC_DENSE")) {
    if (!strcmp(ev, "all")) ndense_ = (int64_t)sources_.size();
    else if (!strcmp(ev, "none")) ndense_ = 0;
    else if (*ev >= '0' && *ev <= '9') ndense_ = std::min<int64_t>(atoll(ev), (int64_t)sources_.size());
  }
  if (const char *ev = getenv("CC_LIGHT"))
    if (!strcmp(ev, "0")) use_light_ = false;
  if (opt.arena) use_light_ = false;  // its per-workgroup scratch would not fit
  light_scratch_ = light_scratch_bytes(g, T);
  if (const char *ev = getenv("CC_FALLBACK"))
    if (!strcmp(ev, "dense")) fallback_dense_ = true;
  const int Bmax = std::max(z_.B_dense, z_.B_sparse);
  nlim_max_ = sources_.empty() ? 1 : std::max<int64_t>(1, sources_[0]);

  d_src_.alloc(sizeof(int32_t) * std::max<size_t>(1, sources_.size()));
  if (!sources_.empty())
    HIP_CHECK(hipMemcpyAsync(d_src_.p, sources_.data(), sizeof(int32_t) * sources_.size(), hipMemcpyHostToDevice, st));
  // per cycle block: which sources, which tiers, filter on or off
  bx_.resize(p.blocks.size());
  pt_.resize(p.blocks.size());
  std::vector<int32_t> all_v, ps_src, ps_dense_order;
  for (size_t bi = 0; bi < p.blocks.size(); bi++) {
    const PBlock &B = p.blocks[bi];
    BlockExec &X = bx_[bi];
    if (B.kind != BK_CYCLE && B.kind != BK_ROOT_CYCLE) continue;
    bool reads_pairs = false;
    for (int c : B.edge_child) reads_pairs |= pair_tab(c);
    X.nofilter = B.ps;
    X.all_dense = reads_pairs || B.pair_keyed;
    has_pairs_ |= B.pair_keyed;
    if (X.all_dense) {
      if (all_v.empty())
        for (int64_t r = g.n - 1; r >= 0; r--) all_v.push_back((int32_t)r);
      X.src = all_v;
      X.ndense = (int64_t)X.src.size();
    } else if (X.nofilter) {
      // path splitting: every vertex with a neighbour may start the paths;
      // dense groups for the sources whose unfiltered two-step reach would
      // cost the sparse path more than one dense group (the degree-based
      // cut with every edge of the graph below every source)
      if (ps_src.empty()) {
        std::vector<std::pair<int64_t, int32_t>> r2;
        for (int64_t r = g.n - 1; r >= 0; r--) {
          if (g.h_deg[r] < 1) continue;
          int64_t reach = 0;
          for (int64_t e = g.h_rp[r]; e < g.h_rp[r + 1]; e++) reach += g.h_deg[g.h_col[e]];
          r2.push_back({reach, (int32_t)r});
        }
        std::stable_sort(r2.begin(), r2.end(), [](auto &a, auto &b2) { return a.first > b2.first; });
        for (auto &x : r2) ps_src.push_back(x.second);
        int64_t nd = 0;
        for (size_t i = 0; i < r2.size(); i++) {
          if (r2[i].first * 64 * 13 >= g.m2 && g.n > 4096) nd = (int64_t)i + 1;
          else break;
        }
        if (const char *ev = getenv("CC_DENSE")) {
          if (!strcmp(ev, "all")) nd = (int64_t)r2.size();
          else if (!strcmp(ev, "none")) nd = 0;
        }
        ps_dense_order.assign(1, (int32_t)nd);
      }
      X.src = ps_src;
      X.ndense = ps_dense_order[0];
    } else {
      X.src = sources_;
      X.ndense = ndense_;
    }
    if (X.nofilter || X.all_dense) nlim_max_ = std::max<int64_t>(nlim_max_, g.n);
    X.d_src.alloc(sizeof(int32_t) * std::max<size_t>(1, X.src.size()));
    if (!X.src.empty())
      HIP_CHECK(hipMemcpyAsync(X.d_src.p, X.src.data(), sizeof(int32_t) * X.src.size(), hipMemcpyHostToDevice, st));
  }
  d_col_.alloc((size_t)g.n * T);
  d_sum_.alloc(sizeof(uint64_t) * 2 * 64);
  d_ovf_.alloc(sizeof(uint32_t) * 64);
  d_per_.alloc(8);
  d_param_.alloc(sizeof(uint64_t) * 2);
  acc_ = AccDev{d_sum_.as<uint64_t>(), d_ovf_.as<uint32_t>(), nullptr};

  // child tables
  tabs_.resize(p.blocks.size());
  for (size_t i = 0; i < p.blocks.size(); i++) {
    const PBlock &B = p.blocks[i];
    if (B.kind == BK_ROOT_CYCLE || B.kind == BK_ROOT_SINGLE || B.pair_keyed) continue;
    int64_t keys = is_edge_table(p, (int)i) ? g.m2 : g.n;
    tabs_[i].alloc(sizeof(uint64_t) * (size_t)std::max<int64_t>(1, keys) * T * table_C(p, (int)i));
  }
  // registers and levels: pools sized for the largest program
  size_t nregs = 0;
  int dmax = 1;
  std::vector<int> reg_smax;
  for (auto &P : p.programs) {
    nregs = std::max(nregs, P.reg_s.size());
    dmax = std::max(dmax, P.max_depth);
    if (reg_smax.size() < P.reg_s.size()) reg_smax.resize(P.reg_s.size(), 0);
    for (size_t r = 0; r < P.reg_s.size(); r++) reg_smax[r] = std::max(reg_smax[r], (int)slots_pair(k, P.reg_s[r]));
  }
  regs_.resize(nregs);
  for (size_t r = 0; r < nregs; r++) {
    regs_[r].val.alloc(sizeof(uint64_t) * (size_t)nlim_max_ * Bmax * T * reg_smax[r]);
    regs_[r].mask.alloc(sizeof(uint64_t) * (size_t)nlim_max_);
  }
  levels_.resize(dmax + 2);
  const size_t nf_max = (size_t)nlim_max_ * Bmax;
  for (int d = 1; d <= dmax; d++) {
    LevelBuf &L = levels_[d];
    L.mb.alloc(2 * sizeof(uint64_t) * (size_t)nlim_max_);
    launch_fill_u64(L.mb.as<uint64_t>(), 2 * nlim_max_, st);
    L.list.alloc(sizeof(int64_t) * nf_max);
    L.cnt.alloc(2 * sizeof(uint32_t));
    L.bcnt.alloc(2 * sizeof(uint32_t) * (size_t)level_chunks(nlim_max_));
    L.vlist.alloc(sizeof(int32_t) * (size_t)nlim_max_);
  }
  // pair-keyed blocks: the staging register of their merges and the entry
  // list, whose capacity is what the memory left holds (with room for the
  // table of twice as many slots that is laid out from it)
  for (size_t bi = 0; bi < p.blocks.size(); bi++) {
    if (!p.blocks[bi].pair_keyed) continue;
    PairTab &Q = pt_[bi];
    const int C = table_C(p, (int)bi);
    Q.stage_val.alloc(sizeof(uint64_t) * (size_t)nlim_max_ * Bmax * T * C);
    Q.stage_mask.alloc(sizeof(uint64_t) * (size_t)nlim_max_);
    Q.cnt.alloc(sizeof(uint64_t));
    const uint64_t row = 8 + 8 * (uint64_t)T * C;
    const uint64_t left = opt.arena ? (uint64_t)(g_arena ? g_arena->size - g_arena->used : 0) / 2
                                    : (uint64_t)(free_bytes() * 0.4);
    Q.cap = std::min<uint64_t>(std::min<uint64_t>((uint64_t)g.n * (uint64_t)g.n, (uint64_t)1 << 26), left / (3 * row));
    if (Q.cap < 1) fail(CC_E_NOMEM, "no memory left for the pair-keyed table");
    Q.keys.alloc(sizeof(int32_t) * 2 * Q.cap);
    Q.vals.alloc(sizeof(uint64_t) * (size_t)Q.cap * T * C);
  }
  // one-workgroup tier per cycle block
  light_.resize(p.blocks.size());
  const int lgrid = light_grid(g.device);
  for (size_t bi = 0; bi < p.blocks.size(); bi++) {
    const PBlock &B = p.blocks[bi];
    Light &L = light_[bi];
    if (B.kind != BK_CYCLE && B.kind != BK_ROOT_CYCLE) {
      L.probed = true;
      continue;
    }
    const BlockExec &X = bx_[bi];
    std::vector<int32_t> rest(X.src.begin() + X.ndense, X.src.end());
    const Program &P = p.programs[bi];
    const bool ok = use_light_ && !rest.empty() && !X.all_dense && P.max_depth <= light_max_depth() &&
                    (int)P.reg_s.size() <= light_max_regs();
    if (!ok) {
      L.probed = true;
      L.fails = rest;  // copies are made from members, which outlive them
      if (!L.fails.empty()) {
        L.d_fails.alloc(4 * L.fails.size());
        HIP_CHECK(hipMemcpyAsync(L.d_fails.p, L.fails.data(), 4 * L.fails.size(), hipMemcpyHostToDevice, st));
      }
      continue;
    }
    L.src = rest;
    std::vector<LOp> lops;
    for (auto &o : P.ops)
      lops.push_back({(int)o.kind, o.dst, o.a, o.b, o.tab, o.tab_src_first, o.ntab, o.s, o.first, o.swapped, o.w});
    std::vector<int32_t> rd(P.reg_s.size()), rC(P.reg_s.size()), rs(P.reg_s.size());
    for (size_t r = 0; r < P.reg_s.size(); r++) {
      rd[r] = P.reg_depth[r];
      rC[r] = (int32_t)slots_pair(k, P.reg_s[r]);
      rs[r] = P.reg_s[r];
    }
    std::vector<TabDev> tv(p.blocks.size());
    for (size_t b2 = 0; b2 < p.blocks.size(); b2++) tv[b2] = tabdev(tabs_[b2].p ? (int)b2 : -1);
    L.d_ops.alloc(sizeof(LOp) * lops.size());
    L.d_rd.alloc(4 * rd.size());
    L.d_rC.alloc(4 * rC.size());
    L.d_rs.alloc(4 * rs.size());
    L.d_tv.alloc(sizeof(TabDev) * tv.size());
    L.d_ctr.alloc(sizeof(uint64_t));
    L.d_fail.alloc(4 * rest.size());
    L.d_src.alloc(4 * rest.size());
    L.d_fails.alloc(4 * rest.size());
    HIP_CHECK(hipMemcpyAsync(L.d_ops.p, lops.data(), sizeof(LOp) * lops.size(), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipMemcpyAsync(L.d_rd.p, rd.data(), 4 * rd.size(), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipMemcpyAsync(L.d_rC.p, rC.data(), 4 * rC.size(), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipMemcpyAsync(L.d_rs.p, rs.data(), 4 * rs.size(), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipMemcpyAsync(L.d_tv.p, tv.data(), sizeof(TabDev) * tv.size(), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipMemcpyAsync(L.d_src.p, L.src.data(), 4 * L.src.size(), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipStreamSynchronize(st));  // lops, rd, rC, rs and tv are local to this iteration
    L.grid = lgrid;
    LightArgs &la = L.la;
    la.g = gd_;
    la.nofilter = X.nofilter ? 1 : 0;
    la.lowcnt = X.nofilter ? g.deg : g.lowcnt;
    la.colr = d_col_.as<uint8_t>();
    la.k = k;
    la.src = L.d_src.as<int32_t>();
    la.nsrc = (int)rest.size();
    la.next = L.d_ctr.as<uint32_t>();
    la.fail = L.d_fail.as<int32_t>();
    la.nfail = L.d_ctr.as<uint32_t>() + 1;
    la.ops = L.d_ops.as<LOp>();
    la.nops = (int)lops.size();
    la.reg_depth = L.d_rd.as<int32_t>();
    la.reg_C = L.d_rC.as<int32_t>();
    la.reg_s = L.d_rs.as<int32_t>();
    la.nregs = (int)rd.size();
    la.D = P.max_depth;
    la.tabs = L.d_tv.as<TabDev>();
    la.out = B.kind == BK_CYCLE ? tabs_[bi].as<uint64_t>() : nullptr;
    la.s_out = B.size;
    la.C_out = B.kind == BK_CYCLE ? table_C(p, (int)bi) : 0;
    la.scratch_per_wg = light_scratch_;
    la.lut = lut_device(g.device);
    if (light_scratch_buf_.bytes < (size_t)light_scratch_ * L.grid)
      light_scratch_buf_.alloc((size_t)light_scratch_ * L.grid);
  }
  for (auto &L : light_) L.la.scratch = light_scratch_buf_.as<uint8_t>();
  // the large stage (CC_LIGHT_LARGE=1): one workgroup per compute unit.  Off by
  // default: on the 1e6-vertex workload it takes 9.7k of the 23k hand-backs
  // in 0.26 s but saves the grouped path only about as much.
  use_large_ = large_light_on() && !opt.arena;
  if (const char *ev = getenv("CC_LIGHT_SCRATCH_LARGE")) light_scratch_large_ = std::max<int64_t>(4096, atoll(ev));
  light2_.resize(p.blocks.size());
  if (use_large_) {
    const int lgrid2 = lgrid / 3;
    bool any = false;
    for (size_t bi = 0; bi < p.blocks.size(); bi++) {
      Light &L = light_[bi], &L2 = light2_[bi];
      L2.probed = true;
      if (L.src.empty()) continue;
      const size_t ns = L.src.size();
      L2.probed = false;
      L2.large = true;
      L2.grid = std::max(1, lgrid2);
      L2.d_ctr.alloc(sizeof(uint64_t));
      L2.d_fail.alloc(4 * ns);
      L2.d_src.alloc(4 * ns);
      L2.d_fails.alloc(4 * ns);
      L2.la = L.la;  // same program, tables and outputs
      L2.la.src = L2.d_src.as<int32_t>();
      L2.la.nsrc = 0;
      L2.la.next = L2.d_ctr.as<uint32_t>();
      L2.la.fail = L2.d_fail.as<int32_t>();
      L2.la.nfail = L2.d_ctr.as<uint32_t>() + 1;
      L2.la.scratch_per_wg = light_scratch_large_;
      any = true;
    }
    if (any) {
      light_scratch_large_buf_.alloc((size_t)light_scratch_large_ * std::max(1, lgrid / 3));
      for (auto &L2 : light2_) L2.la.scratch = light_scratch_large_buf_.as<uint8_t>();
    }
  } else {
    for (auto &L2 : light2_) L2.probed = true;
  }
  (void)lut_device(g.device);  // built before any capture
  HIP_CHECK(hipStreamSynchronize(st));
}

Solver::~Solver() {
  if (exec_) (void)hipGraphExecDestroy(exec_);
  if (graph_) (void)hipGraphDestroy(graph_);
  if (own_st_) {
    (void)hipStreamSynchronize(own_st_);
    (void)hipStreamDestroy(own_st_);
  }
}

void Solver::run_group(size_t bi, const Program &P, const Grp &G, int Tg, uint64_t *out, int C_out, Profiler *prof) {
  const int k = p_.k;
  const BlockExec &X = bx_[bi];
  hipStream_t st = st_;
  const uint8_t *colr = d_col_.as<uint8_t>();
  uint32_t *ovf = d_ovf_.as<uint32_t>();
  // the steps: with CC_FUSE=1, EdgeJoins with their row-local followers fused
  // where the epilogue fits.  Off by default: the fused epilogue runs one lane
  // per row through every slot, and on the 1e6-vertex workload that costs more
  // (5.2 s per colouring) than the separate flat passes it replaces (3.5 s).
  const char *fuse_env = getenv("CC_FUSE");
  const bool fuse_on = fuse_env && *fuse_env == '1';
  std::vector<Step> steps;
  if (fuse_on) {
    steps = schedule(P, k);
  } else {
    for (size_t i = 0; i < P.ops.size(); i++) steps.push_back({(int)i, false, {}});
  }
  std::vector<Step> flat;
  for (auto &stp : steps) {
    const Op &op = P.ops[stp.op];
    const int ce = op.tab >= 0 ? table_C(p_, op.tab) : 0;
    if (stp.fused && !epi_fits(stp.epi.ncols, Tg, ce)) {
      // run the step's ops one by one: every op from the EdgeJoin up to the next step
      const size_t nx = (size_t)(&stp - steps.data()) + 1;
      const int end = nx < steps.size() ? steps[nx].op : (int)P.ops.size();
      for (int q = stp.op; q < end; q++) flat.push_back({q, false, {}});
    } else {
      flat.push_back(stp);
    }
  }
  steps.swap(flat);
  // NodeJoin outputs of unfused NodeJoins keep their input's activity mask
  std::vector<int> mown(P.reg_s.size());
  for (size_t r = 0; r < mown.size(); r++) mown[r] = (int)r;
  for (auto &stp : steps)
    if (!stp.fused && P.ops[stp.op].kind == OP_NJ) mown[P.ops[stp.op].dst] = mown[P.ops[stp.op].a];
  auto regdev = [&](int r) {
    RegDev d;
    d.val = regs_[r].val.as<uint64_t>();
    d.mask = regs_[mown[r]].mask.as<uint64_t>();
    d.C = (int)slots_pair(k, P.reg_s[r]);
    d.s = P.reg_s[r];
    return d;
  };
  auto lv = [&](int r) { return leveldev(P.reg_depth[r]); };
  GroupDev grp;
  grp.src = G.dsrc;
  grp.B = (int)G.B;
  grp.T = Tg;
  grp.k = k;
  grp.n_lim = G.hsrc[0];
  for (int64_t i = 1; i < G.B; i++) grp.n_lim = std::max<int64_t>(grp.n_lim, G.hsrc[i]);
  grp.nofilter = X.nofilter ? 1 : 0;
  if (X.nofilter) grp.n_lim = g_.n;  // paths may reach any vertex
  grp.dense = G.dense ? 1 : 0;
  grp.prof = nullptr;
  grp.hitems = nullptr;
  grp.nh = 0;
  grp.split_chunk = g_.split_chunk;
  grp.split_lo = g_.split_lo;
  if (G.dense) g_.split_range(grp.n_lim, &grp.hitems, &grp.nh);
  if (!grp.hitems) grp.nh = 0;
  const int max_low = max_cnt(-1, X.nofilter, G);
  const int32_t *lowcnt_d = cnt_of(-1, X.nofilter);
  // an EdgeJoin over a pair table's graph has no hub schedule (that is the data graph's)
  auto grp_for = [&](int tab) {
    GroupDev g2 = grp;
    if (pair_tab(tab)) {
      g2.nh = 0;
      g2.hitems = nullptr;
    }
    return g2;
  };
  std::vector<char> built(P.max_depth + 2, 0);
  std::function<void(int)> build = [&](int d) {  // sparse groups: entries of depth d
    if (G.dense || built[d]) return;
    // the level kernels count bytes read and written
    if (prof) grp.prof = prof->begin("level_build_sparse", true, 1.0, 1.0, 0.0);
    if (d == 1) {
      launch_level_init(gd_, grp, lowcnt_d, max_low, leveldev(1), st);
      launch_level_compact(grp, leveldev(1), st);
    } else {
      build(d - 1);
      launch_level_next(gd_, grp, leveldev(d - 1), leveldev(d), st);
    }
    HIP_CHECK(hipGetLastError());
    if (prof) prof->end();
    grp.prof = nullptr;
    built[d] = 1;
  };
  size_t skip_until = 0;  // steps folded into an earlier launch
  // A plain NodeJoin whose output is read only as a term of the AXPY chain
  // right after it is not run on its own: the chain's pass computes its slots
  // (deferred[r] = the NodeJoin producing r, or -1).
  std::vector<int> deferred(P.reg_s.size(), -1);
  auto chain_term_only = [&](size_t si) {
    const Op &nj = P.ops[steps[si].op];
    if (si + 1 >= steps.size() || steps[si + 1].fused) return false;
    const Op &first = P.ops[steps[si + 1].op];
    if (first.kind != OP_AXPY || !first.first) return false;
    size_t sj = si + 1;
    int uses = 0;
    for (; sj < steps.size() && sj < si + 5 && !steps[sj].fused; sj++) {
      const Op &o2 = P.ops[steps[sj].op];
      if (o2.kind != OP_AXPY || o2.dst != first.dst || (sj > si + 1 && o2.first) || o2.a == first.dst) break;
      uses += o2.a == nj.dst;
    }
    int reads = 0;
    for (auto &o : P.ops)
      reads += o.a == nj.dst || o.b == nj.dst || (o.kind == OP_AXPY && !o.first && o.dst == nj.dst);
    return uses >= 1 && uses == reads;
  };
  for (const Step &stp : steps) {
    if ((size_t)(&stp - steps.data()) < skip_until) continue;
    const Op &op = P.ops[stp.op];
    if (!stp.fused && op.kind == OP_NJ && chain_term_only((size_t)(&stp - steps.data()))) {
      deferred[op.dst] = stp.op;
      continue;
    }
    static const char *names[] = {"init", "nodejoin", "edgejoin", "axpy", "merge_root",
                                  "merge_u", "merge_v", "merge_edge", "merge_edge_t", "merge_pair"};
    if (op.kind == OP_INIT) build(1);
    if (op.kind == OP_EJ) build(P.reg_depth[op.dst]);
    grp.prof = nullptr;
    if (stp.fused) {
      const EpiPlan &E = stp.epi;
      Epilogue epi{};
      epi.nregs = (int)E.regs.size();
      epi.ncols = E.ncols;
      double out_slots = 0;  // per entry and trial: rows written and global rows read
      for (size_t e = 0; e < E.regs.size(); e++) {
        RegDev d = regdev(E.regs[e]);
        if (E.col[e] >= 0) d.mask = regs_[E.regs[e]].mask.as<uint64_t>();
        epi.regs[e] = EpiReg{d, lv(E.regs[e]), E.col[e], E.write[e]};
        if (E.write[e] || E.col[e] < 0) out_slots += d.C;
      }
      auto idx = [&](int r) {
        for (size_t e = 0; e < E.regs.size(); e++)
          if (E.regs[e] == r) return (int)e;
        fail(CC_E_DEVICE, "fused step refers to a register it does not hold");
        return 0;
      };
      for (int q : E.ops) {
        EpiOp eo{};
        if (q < 0) {
          const EpiPlan::Axpy &x = E.axpy[-1 - q];
          eo = EpiOp{EPI_AXPY, x.dst, x.a, -1, TabDev{nullptr, 0, 0}, x.w, x.first};
        } else {
          const Op &o = P.ops[q];
          if (o.kind == OP_NJ) {
            eo = EpiOp{EPI_NJ, idx(o.dst), idx(o.a), -1, tabdev(o.tab), 1, 0};
            out_slots += table_C(p_, o.tab);
          } else {
            eo = EpiOp{EPI_MROOT, -1, idx(o.a), idx(o.b), TabDev{nullptr, 0, 0}, o.w, 0};
          }
        }
        epi.ops[epi.nops++] = eo;
      }
      if (prof) {
        std::string nm = std::string("edgejoin") + (G.dense ? "_dense" : "_sparse");
        const double Cin = (double)slots_pair(k, P.reg_s[op.a]);
        const double Ce = op.tab >= 0 ? (double)table_C(p_, op.tab) : 0.0;
        grp.prof = prof->begin(nm.c_str(), true, 4.0, 8.0 * (Cin + Ce), 8.0 * Tg * out_slots);
      }
      launch_ej_epi(gd_, grp, colr, lv(op.a), regdev(op.a), epi, tabdev(op.tab), op.tab_src_first, ovf, acc_, st);
      HIP_CHECK(hipGetLastError());
      if (prof) prof->end();
      continue;
    }
    // two data-edge EdgeJoins in a row from the same level (the second not
    // reading the first's output): one launch over one neighbour scan
    if (op.kind == OP_EJ && op.tab < 0) {
      const size_t si = (size_t)(&stp - steps.data());
      if (si + 1 < steps.size() && !steps[si + 1].fused) {
        const Op &o2 = P.ops[steps[si + 1].op];
        if (o2.kind == OP_EJ && o2.tab < 0 && o2.a != op.dst && o2.dst != op.a && o2.dst != op.dst &&
            P.reg_depth[o2.a] == P.reg_depth[op.a]) {
          if (prof) {
            std::string nm = std::string("edgejoin2") + (G.dense ? "_dense" : "_sparse");
            if (by_op()) nm += "_op" + std::to_string(stp.op) + "+" + std::to_string(steps[si + 1].op);
            // counted in slots: 8 B per input slot relaxed, 8 B per slot written
            grp.prof = prof->begin(nm.c_str(), true, 4.0, 8.0, 8.0 * Tg);
          }
          if (launch_ej_dual(gd_, grp, colr, lv(op.a), lv(op.dst), regdev(op.a), regdev(op.dst), regdev(o2.a),
                             regdev(o2.dst), ovf, st)) {
            HIP_CHECK(hipGetLastError());
            if (prof) prof->end();
            skip_until = si + 2;
            continue;
          }
          if (prof) prof->drop();
          grp.prof = nullptr;
        }
      }
    }
    if (prof) {
      std::string nm = std::string(names[op.kind]) + (G.dense ? "_dense" : "_sparse");
      if (by_op()) nm += "_op" + std::to_string(stp.op);  // one record per operation of the program
      if (op.kind == OP_EJ) {
        // algorithmic bytes: a 4-byte neighbour id per scanned pair, an
        // input row (plus the annotated edge's table row) per relaxation,
        // an output row per entry
        const double Cin = (double)slots_pair(k, P.reg_s[op.a]), Cout = (double)slots_pair(k, P.reg_s[op.dst]);
        const double Ce = op.tab >= 0 ? (double)table_C(p_, op.tab) : 0.0;
        grp.prof = prof->begin(nm.c_str(), true, 4.0, 8.0 * (Cin + Ce), 8.0 * Tg * Cout);
      } else {
        // the other kernels count their bytes read and written themselves
        grp.prof = prof->begin(nm.c_str(), true, 1.0, 1.0, 0.0);
      }
    }
    switch (op.kind) {
      case OP_INIT: {
        RegDev d = regdev(op.dst);
        // dense: only the activity words are cleared; k_init writes every slot
        // of the rows it marks, and every reader of a dense register reads a
        // row only when its activity bit is set
        if (G.dense) launch_fill_u64(d.mask, grp.n_lim, st);
        launch_init(graph_of(op.tab), grp, cnt_of(op.tab, X.nofilter), max_cnt(op.tab, X.nofilter, G), colr,
                    lv(op.dst), d, tabdev(op.tab), op.tab_src_first, tabdev(op.ntab), ovf, st);
        break;
      }
      case OP_NJ:
        launch_nj(gd_, grp, colr, lv(op.a), regdev(op.a), regdev(op.dst), tabdev(op.tab), ovf, st);
        break;
      case OP_EJ:
        launch_ej(graph_of(op.tab), grp_for(op.tab), colr, lv(op.a), lv(op.dst), regdev(op.a), regdev(op.dst),
                  tabdev(op.tab), op.tab_src_first, ovf, st);
        break;
      case OP_AXPY: {
        // a chain dst = w1 a1 + w2 a2 + ... in the next steps runs as one pass
        size_t si = (size_t)(&stp - steps.data());
        if (op.first) {
          std::vector<RegDev> ta;
          std::vector<TabDev> tn;
          std::vector<uint64_t> tw;
          bool any_nj = false;
          auto term = [&](int r, uint64_t w2) {
            if (deferred[r] >= 0) {  // NodeJoin(x, table) computed in the pass
              const Op &nj = P.ops[deferred[r]];
              ta.push_back(regdev(nj.a));
              tn.push_back(tabdev(nj.tab));
              any_nj = true;
            } else {
              ta.push_back(regdev(r));
              tn.push_back(TabDev{nullptr, 0, 0});
            }
            tw.push_back(w2);
          };
          term(op.a, op.w);
          size_t sj = si + 1;
          while (sj < steps.size() && ta.size() < 4 && !steps[sj].fused) {
            const Op &o2 = P.ops[steps[sj].op];
            if (o2.kind != OP_AXPY || o2.first || o2.dst != op.dst || o2.a == op.dst) break;
            term(o2.a, o2.w);
            sj++;
          }
          if (ta.size() > 1 || any_nj) {
            // a chain read only by the root merge right after it is summed
            // inside that merge's pass (linearity), never stored
            if (sj < steps.size() && !steps[sj].fused) {
              const Op &mr = P.ops[steps[sj].op];
              int reads = 0;
              for (auto &o : P.ops) reads += (o.a == op.dst) + (o.b == op.dst);
              if (mr.kind == OP_MROOT && (mr.a == op.dst) != (mr.b == op.dst) && reads == 1) {
                const int other = mr.a == op.dst ? mr.b : mr.a;
                if (launch_mroot_terms(grp, g_.n, colr, lv(op.dst), lv(other), ta.data(), tn.data(), tw.data(),
                                       (int)ta.size(), (int)slots_pair(k, P.reg_s[op.dst]), P.reg_s[op.dst],
                                       regdev(other), mr.w, acc_, st)) {
                  if (prof) prof->rename(std::string("merge_root_terms") + (G.dense ? "_dense" : "_sparse"));
                  skip_until = sj + 1;
                  break;
                }
              }
            }
            launch_axpyn(grp, g_.n, colr, lv(op.a), ta.data(), tn.data(), tw.data(), (int)ta.size(), regdev(op.dst),
                         ovf, st);
            skip_until = sj;
            break;
          }
        }
        launch_axpy(grp, lv(op.a), regdev(op.a), regdev(op.dst), op.w, op.first, ovf, st);
        break;
      }
      case OP_MROOT:
        launch_mroot(grp, g_.n, colr, lv(op.a), lv(op.b), regdev(op.a), regdev(op.b), op.w, acc_, st);
        break;
      case OP_MU:
      case OP_MV:
        launch_munary(grp, g_.n, colr, lv(op.a), lv(op.b), regdev(op.a), regdev(op.b), op.w, op.kind == OP_MU, out,
                      op.s, C_out, ovf, st);
        break;
      case OP_MEDGE:
        launch_medge(graph_of(op.tab), grp, colr, lv(op.a), lv(op.b), regdev(op.a), regdev(op.b), tabdev(op.tab),
                     op.tab_src_first, op.first, op.w, out, op.s, C_out, ovf, st);
        break;
      case OP_MEDGE_T:
        launch_medge_t(graph_of(op.tab), grp, colr, cnt_of(op.tab, X.nofilter), max_cnt(op.tab, X.nofilter, G),
                       tabdev(op.ntab), lv(op.b), regdev(op.b), tabdev(op.tab), op.tab_src_first, op.first, op.w,
                       out, op.s, C_out, ovf, st);
        break;
      case OP_MPAIR: {
        if (!G.dense) fail(CC_E_DEVICE, "a pair-keyed merge runs in dense groups only");
        PairTab &Q = pt_[bi];
        RegDev stg{Q.stage_val.as<uint64_t>(), Q.stage_mask.as<uint64_t>(), (int)table_C(p_, (int)bi),
                   p_.blocks[bi].size};
        launch_mpair(grp, g_.n, colr, regdev(op.a), regdev(op.b), op.w, stg, Q.keys.as<int32_t>(),
                     Q.vals.as<uint64_t>(), Q.cap, (unsigned long long *)Q.cnt.p, ovf, st);
        break;
      }
    }
    HIP_CHECK(hipGetLastError());
    if (prof) prof->end();
  }
  for (int d = 1; d <= P.max_depth; d++)
    if (built[d]) launch_level_reset(grp, leveldev(d), st);
}

void Solver::enqueue_block(size_t bi, int Tg, bool probe, Profiler *prof) {
  const PBlock &B = p_.blocks[bi];
  const int k = p_.k;
  hipStream_t st = st_;
  const uint8_t *colr = d_col_.as<uint8_t>();
  uint32_t *ovf = d_ovf_.as<uint32_t>();
  if (B.kind == BK_LEAF) {
    int ec = B.edge_child[0];
    if (prof) {
      // algorithmic bytes of the leaf join: the CSR and colours, per (x, y)
      // the annotation rows of the edge and of y, per x its own annotation
      // row and its output row
      prof->begin("leaf", false, 0, 0, 0);
      const double n = (double)g_.n, M = (double)g_.m2;
      auto tc = [&](int blk) { return blk >= 0 ? (double)table_C(p_, blk) : 0.0; };
      prof->add_fixed(8.0 * (n + 1) + 4.0 * M + (double)Tg * n +
                      8.0 * Tg * (n * tc(B.node_child[0]) + M * (tc(ec) + tc(B.node_child[1])) +
                                  n * table_C(p_, (int)bi)));
    }
    launch_leaf(graph_of(ec), Tg, k, colr, tabdev(B.node_child[0]), tabdev(ec), ec >= 0 ? B.edge_first_lo[0] : 0,
                tabdev(B.node_child[1]), tabs_[bi].as<uint64_t>(), B.size, table_C(p_, (int)bi), ovf, st);
    HIP_CHECK(hipGetLastError());
    if (prof) prof->end();
    return;
  }
  if (B.kind == BK_ROOT_SINGLE) {
    launch_root_single(g_.n, Tg, tabdev(B.single_child), acc_, st);
    HIP_CHECK(hipGetLastError());
    return;
  }
  // cycle block
  const Program &P = p_.programs[bi];
  uint64_t *out = nullptr;
  int C_out = 0;
  const BlockExec &X = bx_[bi];
  if (B.kind == BK_CYCLE && !B.pair_keyed) {
    out = tabs_[bi].as<uint64_t>();
    C_out = table_C(p_, (int)bi);
    int64_t keys = is_edge_table(p_, (int)bi) ? g_.m2 : g_.n;
    launch_fill_u64(out, keys * Tg * C_out, st);
  }
  if (B.pair_keyed) launch_fill_u64(pt_[bi].cnt.as<uint64_t>(), 1, st);
  static const bool progress = [] {
    const char *v = getenv("CC_VERBOSE");
    return v && atoi(v) >= 2;
  }();
  // 1. dense groups: the sources with the widest reach
  for (int64_t i = 0; i < X.ndense; i += z_.B_dense) {
    run_group(bi, P,
              {X.d_src.as<int32_t>() + i, X.src.data() + i, std::min<int64_t>(z_.B_dense, X.ndense - i), true}, Tg,
              out, C_out, prof);
    if (progress) fprintf(stderr, "[cc] block %zu: dense group at source %lld enqueued\n", bi, (long long)i), fflush(stderr);
  }
  // 2. one workgroup per source for the rest: the small stage, then the
  // large stage on what the small one hands back
  Light &L = light_[bi], &L2 = light2_[bi];
  run_light(L, probe, Tg, prof);
  const bool two = use_large_ && L2.large;
  if (two) {
    if (probe && !L2.probed && L2.src.empty() && L.probed && !L.fails.empty()) {
      L2.src = L.fails;
      L2.la.nsrc = (int)L2.src.size();
      HIP_CHECK(hipMemcpyAsync(L2.d_src.p, L2.src.data(), 4 * L2.src.size(), hipMemcpyHostToDevice, st));
    }
    run_light(L2, probe, Tg, prof);
    if (L.probed && L.fails.empty()) L2.probed = true;
  }
  Light &LF = two ? L2 : L;  // whose hand-backs run as groups
  // 3. grouped path for what the one-workgroup tier does not take
  if (!LF.fails.empty()) {
    for (int64_t i = 0; i < (int64_t)LF.fails.size(); i += z_.B_sparse) {
      run_group(bi, P,
                {LF.d_fails.as<int32_t>() + i, LF.fails.data() + i,
                 std::min<int64_t>(z_.B_sparse, (int64_t)LF.fails.size() - i), fallback_dense_},
                Tg, out, C_out, prof);
      if (progress && (i / z_.B_sparse) % 32 == 0)
        fprintf(stderr, "[cc] block %zu: sparse group at source %lld of %zu enqueued\n", bi, (long long)i,
                LF.fails.size()), fflush(stderr);
    }
  }
  if (B.pair_keyed) finish_pairs(bi, Tg);
}

// Lay out a pair-keyed block's entries as the graph H of its table (host:
// sort the pairs of both orientations into rows, find each slot's entry and
// reverse slot), then gather the entries' rows into slot order.  Needs the
// entries on the host, so a solve with pair-keyed blocks synchronises here
// (and is not captured in a graph).
void Solver::finish_pairs(size_t bi, int Tg) {
  PairTab &Q = pt_[bi];
  hipStream_t st = st_;
  const int C = table_C(p_, (int)bi);
  const int64_t n = g_.n;
  uint64_t cnt = 0;
  HIP_CHECK(hipMemcpyAsync(&cnt, Q.cnt.p, sizeof(cnt), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  if (cnt > Q.cap)
    fail(CC_E_NOMEM, "pair-keyed table of " + std::to_string(cnt) + " entries; memory for " + std::to_string(Q.cap));
  std::vector<int32_t> keys(2 * cnt);
  if (cnt) HIP_CHECK(hipMemcpyAsync(keys.data(), Q.keys.p, sizeof(int32_t) * 2 * cnt, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  // entries sorted by (u, v), for the slot -> entry lookup
  std::vector<int64_t> ent(cnt);
  for (uint64_t i = 0; i < cnt; i++) ent[i] = (int64_t)i;
  auto key = [&](int64_t i) { return ((int64_t)keys[2 * i] << 32) | (uint32_t)keys[2 * i + 1]; };
  std::sort(ent.begin(), ent.end(), [&](int64_t a, int64_t b) { return key(a) < key(b); });
  // arcs of both orientations, sorted and unique: the rows of H
  std::vector<int64_t> arcs;
  arcs.reserve(2 * cnt);
  for (uint64_t i = 0; i < cnt; i++) {
    const int64_t u = keys[2 * i], v = keys[2 * i + 1];
    arcs.push_back((u << 32) | v);
    arcs.push_back((v << 32) | u);
  }
  std::sort(arcs.begin(), arcs.end());
  arcs.erase(std::unique(arcs.begin(), arcs.end()), arcs.end());
  const int64_t m2 = (int64_t)arcs.size();
  std::vector<int64_t> rp(n + 1, 0), rev(m2), idx(m2);
  std::vector<int32_t> col(m2);
  for (int64_t e = 0; e < m2; e++) {
    rp[(arcs[e] >> 32) + 1]++;
    col[e] = (int32_t)(arcs[e] & 0xffffffff);
  }
  for (int64_t x = 0; x < n; x++) rp[x + 1] += rp[x];
  Q.h_lowcnt.assign(n, 0);
  Q.h_deg.assign(n, 0);
  for (int64_t x = 0; x < n; x++) {
    const int32_t *r0 = col.data() + rp[x], *r1 = col.data() + rp[x + 1];
    Q.h_deg[x] = (int32_t)(r1 - r0);
    Q.h_lowcnt[x] = (int32_t)(std::lower_bound(r0, r1, (int32_t)x) - r0);
  }
  for (int64_t e = 0; e < m2; e++) {
    const int64_t x = arcs[e] >> 32, y = col[e];
    const int32_t *ry = col.data() + rp[y], *ry1 = col.data() + rp[y + 1];
    rev[e] = rp[y] + (std::lower_bound(ry, ry1, (int32_t)x) - ry);
    const int64_t want = (x << 32) | (uint32_t)y;
    auto it = std::lower_bound(ent.begin(), ent.end(), want, [&](int64_t i, int64_t w) { return key(i) < w; });
    idx[e] = (it != ent.end() && key(*it) == want) ? *it : -1;
  }
  Q.m2 = m2;
  auto put = [&](DevMem &d, const void *h, size_t bytes) {
    if (d.bytes < std::max<size_t>(bytes, 8)) d.alloc(std::max<size_t>(bytes, 8));
    if (bytes) HIP_CHECK(hipMemcpyAsync(d.p, h, bytes, hipMemcpyHostToDevice, st));
  };
  put(Q.rp, rp.data(), sizeof(int64_t) * (n + 1));
  put(Q.col, col.data(), sizeof(int32_t) * m2);
  put(Q.rev, rev.data(), sizeof(int64_t) * m2);
  put(Q.idx, idx.data(), sizeof(int64_t) * m2);
  put(Q.lowcnt, Q.h_lowcnt.data(), sizeof(int32_t) * n);
  put(Q.deg, Q.h_deg.data(), sizeof(int32_t) * n);
  const size_t tb = sizeof(uint64_t) * (size_t)std::max<int64_t>(1, m2) * Tg * C;
  if (tabs_[bi].bytes < tb) tabs_[bi].alloc(tb);
  launch_pair_gather(Q.idx.as<int64_t>(), m2, Q.vals.as<uint64_t>(), (int64_t)Tg * C, tabs_[bi].as<uint64_t>(), st);
  HIP_CHECK(hipGetLastError());
  // the host vectors above are read by the copies: wait for them
  HIP_CHECK(hipStreamSynchronize(st));
}

void Solver::run_light(Light &L, bool probe, int Tg, Profiler *prof) {
  hipStream_t st = st_;
  if (L.src.empty()) return;
  L.la.T = Tg;
  L.la.acc = acc_;
  launch_fill_u64((uint64_t *)L.d_ctr.p, 1, st);
  // the kernel counts its bytes read and written itself (level 2)
  L.la.prof = prof ? prof->begin(L.large ? "light_large" : "light", true, 1.0, 1.0, 0.0) : nullptr;
  launch_light(L.la, L.grid, L.large, st);
  HIP_CHECK(hipGetLastError());
  if (prof) prof->end();
  if (probe && !L.probed) {
    // learn what it hands back: from now on those sources go to the next stage
    uint32_t hc[2];
    HIP_CHECK(hipMemcpyAsync(hc, L.d_ctr.p, 8, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    std::vector<int32_t> f(hc[1]);
    if (hc[1]) HIP_CHECK(hipMemcpyAsync(f.data(), L.d_fail.p, 4 * (size_t)hc[1], hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    std::sort(f.begin(), f.end(), std::greater<int32_t>());
    std::vector<int32_t> keep;
    {
      std::vector<int32_t> fs = f;
      std::sort(fs.begin(), fs.end());
      for (int32_t s2 : L.src)
        if (!std::binary_search(fs.begin(), fs.end(), s2)) keep.push_back(s2);
    }
    L.src = keep;
    L.fails = f;
    L.la.nsrc = (int)L.src.size();
    if (!L.src.empty())
      HIP_CHECK(hipMemcpyAsync(L.d_src.p, L.src.data(), 4 * L.src.size(), hipMemcpyHostToDevice, st));
    if (!L.fails.empty())
      HIP_CHECK(hipMemcpyAsync(L.d_fails.p, L.fails.data(), 4 * L.fails.size(), hipMemcpyHostToDevice, st));
    L.probed = true;
  }
}

void Solver::enqueue(int Tg, bool seed_dev, bool probe, Profiler *prof) {
  if (seed_dev) launch_colour_dev(g_.orig, g_.n, p_.k, d_param_.as<uint64_t>(), Tg, d_col_.as<uint8_t>(), st_);
  launch_fill_u64(d_sum_.as<uint64_t>(), 2 * 64, st_);
  launch_fill_u64((uint64_t *)d_ovf_.p, 32, st_);
  if (acc_.per_src) launch_fill_u64(acc_.per_src, 2 * g_.n * (int64_t)Tg, st_);
  for (size_t bi = 0; bi < p_.blocks.size(); bi++) enqueue_block(bi, Tg, probe, prof);
}

void Solver::run_group_of_trials(int t0, int Tg, const ColourSource &cs, CountResult &res,
                                 std::vector<u128> *per_source) {
  HIP_CHECK(hipSetDevice(g_.device));
  hipStream_t st = st_;
  if (per_source && !per_alloc_) {
    d_per_.alloc(sizeof(uint64_t) * 2 * (size_t)g_.n * z_.T);
    per_alloc_ = true;
  }
  acc_.per_src = per_source ? d_per_.as<uint64_t>() : nullptr;
  bool probed = true;
  std::vector<char> was_probed(2 * light_.size());
  for (size_t bi = 0; bi < light_.size(); bi++) {
    was_probed[2 * bi] = light_[bi].probed;
    was_probed[2 * bi + 1] = light2_[bi].probed;
    probed &= light_[bi].probed && light2_[bi].probed;
  }
  if (cs.from_seed) {
    uint64_t prm[2] = {cs.seed, (uint64_t)t0};
    HIP_CHECK(hipMemcpyAsync(d_param_.p, prm, sizeof(prm), hipMemcpyHostToDevice, st));
  } else {
    if (!d_hcol_.p) d_hcol_.alloc((size_t)g_.n * z_.T);
    HIP_CHECK(hipMemcpyAsync(d_hcol_.p, cs.host + (size_t)t0 * g_.n, (size_t)g_.n * Tg, hipMemcpyHostToDevice, st));
    launch_permute_colours(d_hcol_.as<uint8_t>(), g_.orig, g_.n, Tg, d_col_.as<uint8_t>(), st);
  }
  Profiler prof(st, !opt_.arena);
  const bool graphs = opt_.use_graphs && probed && cs.from_seed && !per_source && !prof.on && !has_pairs_;
  if (graphs) {
    if (!exec_ || exec_T_ != Tg) {
      if (exec_) (void)hipGraphExecDestroy(exec_);
      if (graph_) (void)hipGraphDestroy(graph_);
      exec_ = nullptr;
      graph_ = nullptr;
      HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        enqueue(Tg, true, false, nullptr);
      } catch (...) {
        hipGraph_t gtmp = nullptr;
        (void)hipStreamEndCapture(st, &gtmp);
        if (gtmp) (void)hipGraphDestroy(gtmp);
        throw;
      }
      HIP_CHECK(hipStreamEndCapture(st, &graph_));
      HIP_CHECK(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
      exec_T_ = Tg;
    }
    HIP_CHECK(hipGraphLaunch(exec_, st));
    graph_replays++;
  } else {
    enqueue(Tg, cs.from_seed, true, prof.on ? &prof : nullptr);
  }
  // results of this trial group
  std::vector<uint64_t> hs(2 * 64);
  std::vector<uint32_t> ho(64);
  HIP_CHECK(hipMemcpyAsync(hs.data(), d_sum_.p, sizeof(uint64_t) * 2 * 64, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipMemcpyAsync(ho.data(), d_ovf_.p, sizeof(uint32_t) * 64, hipMemcpyDeviceToHost, st));
  std::vector<uint32_t> lf(4 * light_.size(), 0);
  for (size_t bi = 0; bi < light_.size(); bi++) {
    if (!light_[bi].src.empty()) HIP_CHECK(hipMemcpyAsync(&lf[4 * bi], light_[bi].d_ctr.p, 8, hipMemcpyDeviceToHost, st));
    if (!light2_[bi].src.empty())
      HIP_CHECK(hipMemcpyAsync(&lf[4 * bi + 2], light2_[bi].d_ctr.p, 8, hipMemcpyDeviceToHost, st));
  }
  std::vector<uint64_t> hp;
  if (per_source) {
    hp.resize(2 * (size_t)g_.n * Tg);
    HIP_CHECK(hipMemcpyAsync(hp.data(), d_per_.p, sizeof(uint64_t) * hp.size(), hipMemcpyDeviceToHost, st));
  }
  HIP_CHECK(hipStreamSynchronize(st));
  prof.finish();
  for (size_t bi = 0; bi < light_.size(); bi++)
    if ((was_probed[2 * bi] && lf[4 * bi + 1] != 0) || (was_probed[2 * bi + 1] && lf[4 * bi + 3] != 0))
      fail(CC_E_DEVICE, "the one-workgroup tier handed back a source it completed before");
  for (int t = 0; t < Tg; t++) {
    res.exact[t0 + t] = (u128)hs[2 * t] | ((u128)hs[2 * t + 1] << 64);
    res.overflow[t0 + t] = ho[t] ? 1 : 0;
  }
  if (per_source)
    for (int64_t r = 0; r < g_.n; r++)
      for (int t = 0; t < Tg; t++) {
        size_t i = 2 * ((size_t)r * Tg + t);
        (*per_source)[(size_t)(t0 + t) * g_.n + g_.h_orig[r]] = (u128)hp[i] | ((u128)hp[i + 1] << 64);
      }
}

// ------------------------------------------------------------------ main
namespace {
thread_local SolveStats g_last_stats;
}
SolveStats last_solve_stats() { return g_last_stats; }

CountResult run_count(const DevGraph &g, const Plan &p, int trials, const ColourSource &cs, const ExecOptions &opt,
                      hipStream_t st, std::vector<u128> *per_source) {
  if (trials < 1) fail(CC_E_ARG, "trials must be >= 1");
  // allocation-free: every DevMem of this solve (all made on this thread) is
  // carved from the given region
  Arena arena{opt.arena, (size_t)opt.arena_bytes, 0};
  struct ArenaScope {
    Arena *prev;
    explicit ArenaScope(Arena *a) : prev(g_arena) { g_arena = a; }
    ~ArenaScope() { g_arena = prev; }
  } scope(opt.arena ? &arena : g_arena);
  Solver S(g, p, trials, opt, st);
  CountResult res;
  res.exact.assign(trials, 0);
  res.overflow.assign(trials, 0);
  if (per_source) per_source->assign((size_t)trials * g.n, 0);
  for (int t0 = 0; t0 < trials; t0 += S.T()) S.run_group_of_trials(t0, std::min(S.T(), trials - t0), cs, res, per_source);
  g_last_stats = S.stats();
  return res;
}

// ------------------------------------------------------------------ batched
//
// All trials of one query through one Solver whose trial groups replay a
// captured hipGraph.  Without a given tuning the trial-group size is tuned
// online: candidates 1, 2, 4, ... each run one group to learn the one-
// workgroup tier's hand-backs and one timed group as a graph replay (both on
// real trials, whose results are kept), until the time per colouring stops
// improving; the remaining trials run with the best.
namespace {
thread_local TuneReport g_last_tune;
}

TuneReport last_tune() { return g_last_tune; }
void set_last_tune(const TuneReport &r) { g_last_tune = r; }

CountResult run_batched(const DevGraph &g, const Plan &p, int trials, uint64_t seed, const ExecOptions *given,
                        hipStream_t st, uint64_t mem_budget) {
  if (trials < 1) fail(CC_E_ARG, "trials must be >= 1");
  CountResult res;
  res.exact.assign(trials, 0);
  res.overflow.assign(trials, 0);
  ColourSource cs;
  cs.from_seed = true;
  cs.seed = seed;
  TuneReport rep;
  int t0 = 0;
  if (given) {
    ExecOptions o = *given;
    Solver S(g, p, trials, o, st);
    for (; t0 < trials; t0 += S.T()) S.run_group_of_trials(t0, std::min(S.T(), trials - t0), cs, res, nullptr);
    rep.trial_group = S.T();
    rep.candidates = 0;
    rep.replays = S.graph_replays;
    g_last_stats = S.stats();
    g_last_tune = rep;
    return res;
  }
  std::vector<std::unique_ptr<Plan>> plans;  // other trees' plans (they outlive the solvers)
  std::unique_ptr<Solver> best;
  double best_per = 0;
  int best_T = 1, best_dense = -1;
  // 0. the decomposition tree (Section 8: trees of one query can differ
  // several-fold in time): when the query has more than one and there are
  // colourings to spare, up to four trees -- the heuristic's first -- each
  // solve colourings like the candidates below, and the fastest is kept.
  // Every tree gives the same counts, so those colourings are results.
  const Plan *pl = &p;
  rep.tree = p.tree;
  // one candidate: a solver for (trial group, dense cut), a first group that
  // learns the hand-backs, a timed replayed group; false when too few trials
  // are left to time it
  auto trial = [&](int cand_T, int dense) -> bool {
    ExecOptions o;
    o.use_graphs = 1;
    o.trial_group = cand_T;
    o.dense_sources = dense;
    o.mem_budget = mem_budget;
    auto S = std::make_unique<Solver>(g, *pl, std::min(cand_T, trials), o, st);
    const int T = S->T();
    S->run_group_of_trials(t0, std::min(T, trials - t0), cs, res, nullptr);
    t0 += std::min(T, trials - t0);
    if (t0 + T > trials) {
      if (!best) best = std::move(S);
      return false;
    }
    auto a = std::chrono::steady_clock::now();
    S->run_group_of_trials(t0, T, cs, res, nullptr);
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
    t0 += T;
    const int c = std::min(rep.candidates, 7);
    rep.candidates++;
    rep.tried_T[c] = T;
    rep.tried_dense[c] = (int)S->ndense();
    rep.tried_sec_per_colouring[c] = dt / T;
    if (!best || dt / T < best_per) {
      best_per = dt / T;
      best_T = T;
      best_dense = (int)S->ndense();
      best = std::move(S);
    }
    return true;
  };
  if (p.num_trees > 1 && p.tree >= 0 && trials >= 32) {
    std::vector<int> cands{p.tree};
    for (int t = 0; t < p.num_trees && cands.size() < 4; t++)
      if (t != p.tree) cands.push_back(t);
    double tbest = 0;
    const Plan *pbest = &p;
    for (size_t ci = 0; ci < cands.size() && t0 + 2 <= trials; ci++) {
      const Plan *cand = &p;
      if (ci > 0) {
        plans.push_back(std::make_unique<Plan>(make_plan(p.k, p.edges, p.mode, cands[ci])));
        cand = plans.back().get();
      }
      pl = cand;
      best.reset();
      best_per = 0;
      const int before = rep.candidates;
      if (!trial(1, -1)) break;
      const double per = rep.tried_sec_per_colouring[std::min(before, 7)];
      if (ci < 8) {
        rep.tried_tree[ci] = cands[ci];
        rep.tried_tree_seconds[ci] = per;
      }
      rep.trees_tried = (int)ci + 1;
      if (ci == 0 || per < tbest) {
        tbest = per;
        pbest = cand;
      }
    }
    pl = pbest;
    rep.tree = pl->tree;
    best.reset();  // the dense cut and trial group are tuned on the chosen tree
    best_per = 0;
  }
  // 1. the dense cut, one colouring per group: the cost model's, half, double
  if (t0 < trials && trial(1, -1)) {
    const int d0 = best_dense;
    for (int d : {d0 / 2, d0 * 2}) {
      if (d == d0 || t0 >= trials) continue;
      if (!trial(1, d)) break;
    }
  }
  // 2. the trial-group size at that cut: 2, 4, ... while it keeps improving.
  // Skipped when one colouring already takes long (kTrialGroupMaxSec): its
  // work then outweighs its launch sequence, and groups of one colouring keep
  // the packed EdgeJoin (one trial only).
  constexpr double kTrialGroupMaxSec = 0.25;
  for (int cand = 2; cand <= 64 && t0 + 2 * cand <= trials && best_per < kTrialGroupMaxSec; cand *= 2) {
    const double before = best_per;
    if (!trial(cand, best_dense)) break;
    if (best_per >= before) break;
  }
  if (best) {
    for (; t0 < trials; t0 += best->T()) best->run_group_of_trials(t0, std::min(best->T(), trials - t0), cs, res, nullptr);
    rep.trial_group = best->T();
    rep.dense_sources = (int)best->ndense();
    rep.replays = best->graph_replays;
    g_last_stats = best->stats();
  }
  g_last_tune = rep;
  return res;
}

void dump_programs(const Plan &p) {
    static const char *kn[] = {"INIT", "NJ", "EJ", "AXPY", "MROOT", "MU", "MV", "MEDGE", "MEDGE_T", "MPAIR"};
    for (size_t bi = 0; bi < p.programs.size(); bi++) {
      const Program &P = p.programs[bi];
      if (P.ops.empty()) continue;
      fprintf(stderr, "[cc] block %zu program: %zu ops, %zu registers, depth %d\n", bi, P.ops.size(), P.reg_s.size(),
              P.max_depth);
      for (auto &o : P.ops)
        fprintf(stderr, "[cc]   %-7s dst=%d(s%d,d%d) a=%d b=%d tab=%d ntab=%d w=%llu first=%d\n", kn[o.kind], o.dst,
                o.dst >= 0 ? P.reg_s[o.dst] : -1, o.dst >= 0 ? P.reg_depth[o.dst] : -1, o.a, o.b, o.tab, o.ntab,
                (unsigned long long)o.w, o.first);
    }
  for (size_t bi = 0; bi < p.programs.size(); bi++) {
    const Program &P = p.programs[bi];
    if (P.ops.empty()) continue;
    for (auto &stp : schedule(P, p.k)) {
      if (!stp.fused) {
        fprintf(stderr, "[cc] step op %d\n", stp.op);
        continue;
      }
      fprintf(stderr, "[cc] step op %d fused: %zu epilogue ops, %d LDS columns; regs", stp.op, stp.epi.ops.size(),
              stp.epi.ncols);
      for (size_t e = 0; e < stp.epi.regs.size(); e++)
        fprintf(stderr, " r%d(col %d%s)", stp.epi.regs[e], stp.epi.col[e], stp.epi.write[e] ? ",w" : "");
      fprintf(stderr, "\n");
      for (int q : stp.epi.ops) {
        if (q < 0) {
          auto &x = stp.epi.axpy[-1 - q];
          fprintf(stderr, "[cc]     AXPY e%d %s= %llu * e%d\n", x.dst, x.first ? "" : "+", (unsigned long long)x.w, x.a);
        } else {
          fprintf(stderr, "[cc]     op %d\n", q);
        }
      }
    }
  }
}

}  // namespace cc
