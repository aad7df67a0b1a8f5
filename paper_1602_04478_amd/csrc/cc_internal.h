// Internal declarations shared by the host parts of the library (planner,
// graph residency, executor, API, server).  Device code lives in kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cc.h"
#include "kernels.h"

namespace cc {

typedef unsigned __int128 u128;

// ------------------------------------------------------------------ errors
struct Error {
  cc_status st;
  std::string msg;
};
[[noreturn]] void fail(cc_status st, const std::string &msg);
void set_last_error(const std::string &msg);
#define HIP_CHECK(x)                                                                   \
  do {                                                                                 \
    hipError_t _e = (x);                                                               \
    if (_e != hipSuccess)                                                              \
      ::cc::fail(CC_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(_e));          \
  } while (0)

// ------------------------------------------------------------------ planner
enum BlockKind { BK_LEAF = 0, BK_CYCLE = 1, BK_ROOT_CYCLE = 2, BK_ROOT_SINGLE = 3 };

// A block of the decomposition tree (Section 4.1).  For a cycle, nodes are
// a_0..a_{L-1} in cycle order; edge i joins nodes[i] and nodes[i+1 mod L].
// For a leaf, nodes = {a, b} with b the removed leaf and a the boundary.
struct PBlock {
  BlockKind kind;
  std::vector<int> nodes;
  std::vector<int> node_child;      // per node: child block annotating it, or -1
  std::vector<int> edge_child;      // per edge: child block annotating it, or -1 (a data edge)
  std::vector<char> edge_first_lo;  // per annotated edge: the child's first boundary is nodes[i]
  std::vector<int> boundary;        // ordered boundary nodes (first, second)
  int size = 0;                     // |SQ(B)|: number of query nodes in the subquery
  int single_child = -1;            // BK_ROOT_SINGLE: the block annotating the last node
  // Path splitting (Section 5.1, the baseline procedure): the cycle is split
  // at its boundary nodes (the root at a_0 and the node opposite), the paths
  // run from the image of the first boundary node with no degree-order
  // filter, and every match is counted once.  Used for every block of a
  // path-splitting plan, and in degree-based plans for the blocks whose two
  // boundary nodes are not adjacent (their table is keyed by vertex pairs).
  bool ps = false;
  // the table is keyed by pairs of vertices that need not be adjacent: two
  // boundary nodes not adjacent on the cycle
  bool pair_keyed = false;
};

struct Op {
  OpKind kind;
  int dst = -1, a = -1, b = -1;  // frontier registers
  int tab = -1;                  // child block of the joined edge (INIT/EJ/MEDGE*), node (NJ), -1 = none
  int tab_src_first = 0;         // edge tables: the traversal's source end is the child's first boundary
  int ntab = -1;                 // INIT / MEDGE_T: node table joined at u (a_h's block), or -1
  uint64_t w = 1;                // weight / multiplicity
  int s = 0;                     // signature size of dst (merges: of the output)
  int first = 0;                 // AXPY: dst is fresh (overwrite); MEDGE*: x-end is the table's first boundary
  int swapped = 0;               // MEDGE_T: u is the image of the second boundary
};

struct Program {
  std::vector<Op> ops;
  std::vector<int> reg_s;        // signature size per register
  std::vector<int> reg_depth;    // path length (edges from u) of each register's key vertex
  std::vector<int> last_use;     // op index of each register's last use
  int max_depth = 0;
};

// Plan modes: the degree-based program (Section 5.1, DB) or the path-splitting
// baseline for every block.
enum PlanMode { PLAN_DB = 0, PLAN_PS = 1 };

struct Plan {
  int k = 0;
  int mode = PLAN_DB;
  int tree = -1;                 // index of the chosen tree among the enumerated ones
  int num_trees = 0;             // distinct decomposition trees enumerated
  std::vector<std::pair<int, int>> edges;
  std::vector<PBlock> blocks;    // children before parents; the root is last
  std::vector<Program> programs; // per block (cycles only)
  uint64_t aut = 1;
  int longest_cycle = 0;
  int sum_boundary = 0;
  int num_annotations = 0;
};

// Build the plan; throws Error (via fail) on invalid queries.  tree < 0:
// the tree the heuristic of Section 6 picks; else the tree of that index in
// the planner's enumeration order (CC_E_ARG when there is no such tree).
Plan make_plan(int k, const std::vector<std::pair<int, int>> &edges, int mode = PLAN_DB, int tree = -1);
// Flatten the tree for cc_query_plan.
std::vector<int32_t> describe_plan(const Plan &p);

// binomial coefficient
inline int64_t binom(int n, int r) {
  if (r < 0 || r > n || n < 0) return 0;
  int64_t c = 1;
  for (int i = 1; i <= r; i++) c = c * (n - r + i) / i;
  return c;
}
// Slots of a table: unary (one key vertex) or binary (two key vertices / path key).
inline int64_t slots_unary(int k, int s) { return binom(k - 1, s - 1); }
inline int64_t slots_pair(int k, int s) { return binom(k - 2, s - 2); }

// ------------------------------------------------------------------ graph
struct DevGraph {
  int64_t n = 0, m2 = 0;      // vertices, directed slots (2m)
  int64_t max_degree = 0;
  uint32_t flags = 0;
  // host copies (rank order)
  std::vector<int64_t> h_rp;
  std::vector<int32_t> h_col;
  std::vector<int32_t> h_orig;      // rank -> original id
  std::vector<int32_t> h_rank;      // original id -> rank
  std::vector<int32_t> h_lowcnt;    // number of lower neighbours
  std::vector<int32_t> h_deg;       // degree
  std::vector<int64_t> h_r2;        // two-step high-start reach estimate per source
  // hub schedule of the dense EdgeJoin: the vertices of degree > 2 * split_chunk
  // (ranks >= split_lo) as (vertex, neighbour offset) chunks, vertex descending
  int split_chunk = 0;
  int64_t split_lo = 0;
  std::vector<int32_t> h_split_w;   // vertex of each chunk item
  int32_t *split_items = nullptr;   // device: (vertex, offset) per item
  // device copies
  int64_t *rp = nullptr;
  int32_t *col = nullptr;
  int64_t *rev = nullptr;
  int32_t *orig = nullptr;
  int32_t *lowcnt = nullptr;
  int32_t *deg = nullptr;
  int device = 0;
  // items of the hub schedule usable below n_lim: a suffix of the list
  void split_range(int64_t n_lim, const int32_t **items, int *count) const;
  ~DevGraph();
};

std::unique_ptr<DevGraph> make_graph(int64_t n, const int64_t *row_ptr, const int32_t *col, uint32_t flags,
                                     hipStream_t stream);

// ------------------------------------------------------------------ executor
struct CountResult {
  std::vector<u128> exact;        // per trial
  std::vector<uint8_t> overflow;  // per trial
};

struct ExecOptions {
  int group_sources = 0;
  int trial_group = 0;
  int light_max_keys = 0;
  int use_graphs = 0;
  int dense_sources = -1;         // sources run as dense groups (-1: the cost model's cut)
  uint64_t mem_budget = 0;        // bytes; 0 = from the device's free memory
  // Allocation-free solve: every device buffer is carved from [arena,
  // arena + arena_bytes) (no hipMalloc, no stream or event creation, no
  // one-workgroup tier, no profiling).  Null: the block cache.
  uint8_t *arena = nullptr;
  uint64_t arena_bytes = 0;
};

// Colours in rank order for `trials` trials: either from (seed) by the
// contract, or from host colours indexed by original id.
struct ColourSource {
  bool from_seed = true;
  uint64_t seed = 0;
  const uint8_t *host = nullptr;  // trials * n, original ids
};

CountResult run_count(const DevGraph &g, const Plan &p, int trials, const ColourSource &cs,
                      const ExecOptions &opt, hipStream_t stream, std::vector<u128> *per_source);

uint64_t footprint(const DevGraph &g, const Plan &p, int trials, const ExecOptions &opt);

// All trials of one query with captured launch sequences replayed per trial
// group; `tuning` null = tune the trial-group size online.
struct TuneReport {
  int trial_group = 0;     // chosen
  int candidates = 0;      // trial-group sizes timed
  int tried_T[8] = {0};
  int tried_dense[8] = {0};  // dense-group sources of each candidate
  int dense_sources = 0;     // chosen
  double tried_sec_per_colouring[8] = {0};
  uint64_t replays = 0;    // graph replays by the chosen solver
  int tree = -1;           // chosen decomposition tree
  int trees_tried = 0;
  int tried_tree[8] = {0};
  double tried_tree_seconds[8] = {0};
};
// mem_budget: device bytes the tuned solvers may use (0: from the free memory)
CountResult run_batched(const DevGraph &g, const Plan &p, int trials, uint64_t seed, const ExecOptions *tuning,
                        hipStream_t stream, uint64_t mem_budget = 0);
TuneReport last_tune();  // of the calling thread's last run_batched
void set_last_tune(const TuneReport &r);

// How the calling thread's last solve (any counting call) split its sources
// over the tiers, for the root block (the last cycle block of the plan).
struct SolveStats {
  int64_t sources = 0, dense = 0, light = 0, handed_back = 0;
  int trial_group = 0, group_sources = 0;
};
SolveStats last_solve_stats();

// Device colouring (rank order) for one trial, copied to host by original id.
void colours_to_host(const DevGraph &g, int k, uint64_t seed, int trial, uint8_t *out, hipStream_t stream);

void profile_enable(int level);  // 0 off, 1 event timing, 2 timing and work counters
struct KernelProfile {
  std::string name;
  uint64_t launches;
  double seconds, bytes;
  uint64_t work[3];
};
std::vector<KernelProfile> profile_read();
void dump_programs(const Plan &p);  // the cycle programs, to stderr
double probe_copy(uint64_t bytes, int reps);  // GB/s of a plain device copy (read + write)

double estimate_from(const Plan &p, const std::vector<u128> &exact, const std::vector<uint8_t> &ovf);

// ------------------------------------------------------------------ static device memory (static_mem.hip)
// Size of `scratch`, the per-device work memory of cc_count_static.
constexpr size_t kStaticScratchBytes = (size_t)256 << 20;
// Device address of this device's scratch (looked up once per device; the
// device must be current).  Throws CC_E_DEVICE when the lookup fails.
uint8_t *static_scratch(int dev);
// Serialises the calls that use one device's scratch.
std::mutex &static_scratch_lock(int dev);

}  // namespace cc

// opaque handle types of the C ABI
struct cc_graph_s {
  std::unique_ptr<cc::DevGraph> g;
};
struct cc_query_s {
  cc::Plan plan;
};
