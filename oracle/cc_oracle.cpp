// Colourful subgraph counting oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow CPU implementation used to check the device library.  Only
// the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
// It shares no code, header or table with the device library.
//
// Exact unsigned 128-bit counts throughout.
//
//   o1_*   brute-force enumeration of matches (the problem definition,
//          Preliminaries: injective, edge-preserving maps; colourful = all k
//          colours used).
//   o3_*   the degree-based (DB) dynamic program over the decomposition tree
//          (Sections 4.1-5.2), written from the paper's description:
//            - decomposition by contracting leaf edges and contractible
//              cycles (Cases 1-3 of Section 4.1);
//            - cycles solved by partitioning the colourful matches by their
//              highest node (Eq. (1)), building high-starting path tables
//              P+ and P- from the node opposite d = h + floor(L/2), with
//              NodeJoin/EdgeJoin (Fig. "DB Procedure for General Cycle
//              Blocks"), boundary images recorded in extra fields when a
//              boundary node lies strictly inside a path (configurations
//              (A)/(B), Section 5.1), and merged with a1 n a2 = {chi(u),chi(v)};
//            - leaf blocks by joining the annotations of a, (a,b) and b;
//            - the root by counting (cycle) or summing the table (singleton).
//   Colouring contract: chi_t(v) = ((mix(mix(seed + t) ^ v) >> 32) * k) >> 32
//   where mix is the splitmix64 output function (Vigna, public domain).
//
// Readings of points the paper leaves open (listed in the design notes):
//   * colours are 0..k-1; the degree order ties are broken by vertex id, in
//     either direction (the oracle defaults to the reverse of the library's);
//   * in the general-cycle procedure the EdgeJoins run for j = h+1 .. d-1
//     and NodeJoin(a_d) runs once, at the end of P+; the block on a_h is
//     joined in P-, on the start vertex, together with the first edge;
//   * "highest" ranges over the cycle's own nodes only; vertices matched
//     inside annotating blocks are unconstrained.
//
// Build: g++ -O2 -std=c++17 -fopenmp -shared -fPIC -o liboracle.so cc_oracle.cpp

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;
typedef uint64_t u64;

namespace {

// ---------------------------------------------------------------- graph
struct G {
  int64_t n;
  const int64_t *rp;
  const int32_t *col;
  int64_t deg(int64_t v) const { return rp[v + 1] - rp[v]; }
  bool adj(int64_t a, int64_t b) const {
    const int32_t *s = col + rp[a], *e = col + rp[a + 1];
    return std::binary_search(s, e, (int32_t)b);
  }
};

// ---------------------------------------------------------------- colours
static inline u64 mix64(u64 x) {
  u64 z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline int colour_of(u64 seed, int trial, int k, u64 v) {
  u64 key = mix64(seed + (u64)trial);
  u64 h = mix64(key ^ v);
  return (int)(((h >> 32) * (u64)k) >> 32);
}

static inline int popc(unsigned x) { return __builtin_popcount(x); }

// ---------------------------------------------------------------- query
struct Query {
  int k;
  std::vector<std::vector<int>> adj;  // sorted
  bool has(int a, int b) const {
    return std::binary_search(adj[a].begin(), adj[a].end(), b);
  }
};

static Query make_query(int k, int ne, const int32_t *e) {
  Query q;
  q.k = k;
  q.adj.assign(k, {});
  for (int i = 0; i < ne; i++) {
    int a = e[2 * i], b = e[2 * i + 1];
    if (a < 0 || b < 0 || a >= k || b >= k || a == b) throw std::runtime_error("bad query edge");
    q.adj[a].push_back(b);
    q.adj[b].push_back(a);
  }
  for (auto &l : q.adj) {
    std::sort(l.begin(), l.end());
    if (std::adjacent_find(l.begin(), l.end()) != l.end()) throw std::runtime_error("duplicate query edge");
  }
  return q;
}

// ---------------------------------------------------------------- O1
// Brute force over maps that are edge-preserving.  `colourful` asks that the
// k images carry k distinct colours (which forces injectivity); otherwise
// injectivity is checked directly (plain matches, for the estimator).
struct Brute {
  const G &g;
  const Query &q;
  const uint8_t *colour;  // may be null when !colourful
  bool colourful;
  std::vector<int> order, anchor;
  std::vector<int64_t> img;
  u128 total = 0;

  Brute(const G &g_, const Query &q_, const uint8_t *c, bool cf) : g(g_), q(q_), colour(c), colourful(cf) {
    // BFS order from node 0; the anchor of a node is an earlier neighbour.
    int k = q.k;
    std::vector<int> seen(k, 0);
    order.push_back(0);
    seen[0] = 1;
    anchor.assign(k, -1);
    for (size_t i = 0; i < order.size(); i++)
      for (int b : q.adj[order[i]])
        if (!seen[b]) {
          seen[b] = 1;
          anchor[b] = order[i];
          order.push_back(b);
        }
    if ((int)order.size() != k) throw std::runtime_error("query not connected");
    img.assign(k, -1);
  }

  bool ok(int a, int64_t x, unsigned used) {
    if (colourful) {
      if (used >> colour[x] & 1u) return false;
    } else {
      for (int b = 0; b < q.k; b++)
        if (img[b] == x) return false;
    }
    for (int b : q.adj[a])
      if (img[b] >= 0 && !g.adj(img[b], x)) return false;
    return true;
  }

  u128 rec(int i, unsigned used) {
    if (i == q.k) return 1;
    int a = order[i];
    int64_t p = img[anchor[a]];
    u128 s = 0;
    for (int64_t e = g.rp[p]; e < g.rp[p + 1]; e++) {
      int64_t x = g.col[e];
      if (!ok(a, x, used)) continue;
      img[a] = x;
      s += rec(i + 1, colourful ? (used | (1u << colour[x])) : used);
      img[a] = -1;
    }
    return s;
  }

  u128 run_from(int64_t x0) {
    unsigned used = colourful ? (1u << colour[x0]) : 0u;
    img[order[0]] = x0;
    u128 s = (q.k == 1) ? 1 : rec(1, used);
    img[order[0]] = -1;
    return s;
  }
};

// ---------------------------------------------------------------- decomposition
// Block kinds.  Node annotations and edge annotations refer to child blocks.
enum Kind { LEAF = 0, CYCLE = 1 };

struct Block {
  Kind kind;
  std::vector<int> nodes;        // LEAF: {a, b} (b is the removed leaf); CYCLE: a_0..a_{L-1}
  std::vector<int> node_ann;     // per node: child block or -1
  std::vector<int> edge_ann;     // per edge (nodes[i], nodes[i+1 mod L]); LEAF: one entry
  std::vector<int> edge_first;   // per annotated edge: query node that is the child's first boundary
  std::vector<int> boundary;     // query nodes, ordered (first, second)
  int size = 0;                  // number of query nodes in SQ(B)
  bool root = false;
};

struct Plan {
  std::vector<Block> blocks;  // in contraction order (children before parents)
  int root_block = -1;        // a root CYCLE, or -1 when the root is a singleton
  int root_single_child = -1; // block annotating the final single node
};

struct WorkQ {
  int k;
  std::vector<std::set<int>> adj;
  std::vector<int> alive;
  std::vector<int> nann;                               // node annotation
  std::map<std::pair<int, int>, std::pair<int, int>> eann;  // (min,max) -> (block, first node)
  std::vector<int> sq;                                 // size of the subquery hanging on a node/edge
};

static std::pair<int, int> ekey(int a, int b) { return {std::min(a, b), std::max(a, b)}; }

// All simple cycles (as node sequences) of the live query, each once.
static void cycles_of(const WorkQ &w, std::vector<std::vector<int>> &out) {
  int k = w.k;
  std::vector<int> path, on(k, 0);
  for (int s = 0; s < k; s++) {
    if (!w.alive[s]) continue;
    path.assign(1, s);
    on.assign(k, 0);
    on[s] = 1;
    // depth-first over nodes greater than s
    std::vector<std::vector<int>> stack_nb;
    std::function<void(int)> dfs = [&](int x) {
      for (int y : w.adj[x]) {
        if (y == s && path.size() >= 3 && path[1] < path.back()) out.push_back(path);
        if (y <= s || on[y]) continue;
        on[y] = 1;
        path.push_back(y);
        dfs(y);
        path.pop_back();
        on[y] = 0;
      }
    };
    dfs(s);
  }
}

// `forced`, when non-empty, lists the node sets to contract, in order; each
// must be a block (leaf edge or contractible cycle) when its turn comes.
static Plan decompose(const Query &q, const std::vector<std::vector<int>> &forced = {}) {
  size_t fi = 0;
  WorkQ w;
  w.k = q.k;
  w.adj.assign(q.k, {});
  for (int a = 0; a < q.k; a++)
    for (int b : q.adj[a]) w.adj[a].insert(b);
  w.alive.assign(q.k, 1);
  w.nann.assign(q.k, -1);
  Plan plan;
  auto nlive = [&]() { int c = 0; for (int x : w.alive) c += x; return c; };
  // size of a subquery: nodes of the block plus nodes hidden in annotations
  std::vector<int> hidden_node(q.k, 0);  // extra nodes hanging on a node annotation
  std::map<std::pair<int, int>, int> hidden_edge;

  while (nlive() > 1) {
    bool done = false;
    std::set<int> want;
    if (fi < forced.size()) want = std::set<int>(forced[fi].begin(), forced[fi].end());
    bool want_leaf = false;
    if (!want.empty()) {
      if (want.size() == 2) {
        int x = *want.begin(), y = *want.rbegin();
        want_leaf = w.adj[x].count(y) && (w.adj[x].size() == 1 || w.adj[y].size() == 1);
      }
      fi++;
    }
    // Case 3: a leaf edge (a, b), b of degree one; lowest b first.
    for (int b = 0; b < q.k && !done; b++) {
      if (!w.alive[b] || w.adj[b].size() != 1) continue;
      int a = *w.adj[b].begin();
      if (!want.empty() && !(want_leaf && want.count(a) && want.count(b))) continue;
      Block B;
      B.kind = LEAF;
      B.nodes = {a, b};
      B.node_ann = {w.nann[a], w.nann[b]};
      auto it = w.eann.find(ekey(a, b));
      int ea = -1, ef = -1;
      if (it != w.eann.end()) { ea = it->second.first; ef = it->second.second; w.eann.erase(it); }
      B.edge_ann = {ea};
      B.edge_first = {ef};
      B.boundary = {a};
      B.size = 2 + hidden_node[a] + hidden_node[b] + hidden_edge[ekey(a, b)];
      w.adj[a].erase(b);
      w.adj[b].erase(a);
      w.alive[b] = 0;
      int id = (int)plan.blocks.size();
      plan.blocks.push_back(B);
      w.nann[a] = id;
      hidden_node[a] = B.size - 1;
      w.nann[b] = -1;
      done = true;
    }
    if (done) continue;
    // Contractible cycles: induced, at most two boundary nodes.  Pick the
    // one whose sorted node list is lexicographically smallest.
    std::vector<std::vector<int>> cyc;
    cycles_of(w, cyc);
    std::vector<int> best;
    std::vector<int> bestsorted;
    std::vector<int> bestbd;
    for (auto &c : cyc) {
      std::set<int> cs(c.begin(), c.end());
      int L = (int)c.size();
      // induced: every edge between cycle nodes is a cycle edge
      int inner = 0;
      for (int x : c)
        for (int y : w.adj[x])
          if (cs.count(y)) inner++;
      if (inner != 2 * L) continue;
      std::vector<int> bd;
      for (int x : c) {
        bool out = false;
        for (int y : w.adj[x])
          if (!cs.count(y)) out = true;
        if (out) bd.push_back(x);
      }
      if (bd.size() > 2) continue;
      if (bd.empty() && nlive() != L) continue;
      if (!want.empty() && cs != want) continue;
      std::vector<int> srt(c.begin(), c.end());
      std::sort(srt.begin(), srt.end());
      if (best.empty() || srt < bestsorted) { best = c; bestsorted = srt; bestbd = bd; }
    }
    if (best.empty()) throw std::runtime_error("query has treewidth > 2 (no block found)");
    Block B;
    B.kind = CYCLE;
    B.nodes = best;
    int L = (int)best.size();
    B.size = L;
    for (int i = 0; i < L; i++) {
      int a = best[i], b = best[(i + 1) % L];
      B.node_ann.push_back(w.nann[a]);
      B.size += hidden_node[a];
      auto it = w.eann.find(ekey(a, b));
      if (it != w.eann.end()) {
        B.edge_ann.push_back(it->second.first);
        B.edge_first.push_back(it->second.second);
      } else {
        B.edge_ann.push_back(-1);
        B.edge_first.push_back(-1);
      }
      B.size += hidden_edge[ekey(a, b)];
    }
    B.boundary = bestbd;
    int id = (int)plan.blocks.size();
    // remove the cycle's edges and its non-boundary nodes
    for (int i = 0; i < L; i++) {
      int a = best[i], b = best[(i + 1) % L];
      w.adj[a].erase(b);
      w.adj[b].erase(a);
      w.eann.erase(ekey(a, b));
      hidden_edge.erase(ekey(a, b));
    }
    std::set<int> bds(bestbd.begin(), bestbd.end());
    for (int x : best)
      if (!bds.count(x)) { w.alive[x] = 0; w.nann[x] = -1; hidden_node[x] = 0; }
    if (bestbd.empty()) {
      B.root = true;
      plan.blocks.push_back(B);
      plan.root_block = id;
      for (int x : best) w.alive[x] = 0;
      return plan;
    }
    plan.blocks.push_back(B);
    if (bestbd.size() == 1) {           // Case 1
      w.nann[bestbd[0]] = id;
      hidden_node[bestbd[0]] = B.size - 1;
    } else {                            // Case 2
      int a = bestbd[0], b = bestbd[1];
      w.adj[a].insert(b);
      w.adj[b].insert(a);
      w.eann[ekey(a, b)] = {id, a};
      hidden_edge[ekey(a, b)] = B.size - 2;
      w.nann[a] = w.nann[b] = -1;
      hidden_node[a] = hidden_node[b] = 0;
    }
  }
  // single node left
  for (int x = 0; x < q.k; x++)
    if (w.alive[x]) plan.root_single_child = w.nann[x];
  return plan;
}

// ---------------------------------------------------------------- tables
// Unary table: per vertex, signature -> count.
// Binary table: per ordered vertex pair, signature -> count.
typedef std::unordered_map<unsigned, u128> SigMap;
typedef std::vector<SigMap> Unary;
struct PairHash {
  size_t operator()(const std::pair<int64_t, int64_t> &p) const {
    return std::hash<int64_t>()(p.first * 1000003LL + p.second);
  }
};
typedef std::unordered_map<std::pair<int64_t, int64_t>, SigMap, PairHash> Binary;
// Binary tables are also indexed by first vertex for joins.
struct BinIndex {
  std::unordered_map<int64_t, std::vector<std::pair<int64_t, const SigMap *>>> by_first;
};

struct Ctx {
  G g;
  int k;
  const uint8_t *chi;          // colours by vertex id
  std::vector<int64_t> rank;   // position in the degree order
  std::vector<Unary> unary;    // per block (valid for 1-boundary blocks)
  std::vector<Binary> binary;  // per block (valid for 2-boundary blocks)
  std::vector<BinIndex> bidx;  // by first boundary image
  std::vector<BinIndex> bidx_rev;  // by second boundary image
  Plan plan;
};

static inline unsigned cbit(const Ctx &c, int64_t v) { return 1u << c.chi[v]; }

// u succeeds w in the degree order
static inline bool higher(const Ctx &c, int64_t u, int64_t w) { return c.rank[u] > c.rank[w]; }

// The table of a node annotation at vertex x, or the identity {chi(x)} -> 1.
static SigMap node_table(const Ctx &c, int blk, int64_t x) {
  if (blk < 0) return SigMap{{cbit(c, x), (u128)1}};
  return c.unary[blk][x];
}

// Edge (a_i, a_j) of a block read between data vertices x = pi(a_i), y = pi(a_j).
// `first_is_i` tells whether a_i is the child's first boundary node.
static void edge_entries(const Ctx &c, int blk, bool first_is_i, int64_t x,
                         std::vector<std::pair<int64_t, SigMap>> &out) {
  out.clear();
  if (blk < 0) {
    for (int64_t e = c.g.rp[x]; e < c.g.rp[x + 1]; e++) {
      int64_t y = c.g.col[e];
      if (c.chi[x] == c.chi[y]) continue;
      out.push_back({y, SigMap{{cbit(c, x) | cbit(c, y), (u128)1}}});
    }
    return;
  }
  const BinIndex &bi = first_is_i ? c.bidx[blk] : c.bidx_rev[blk];
  auto it = bi.by_first.find(x);
  if (it == bi.by_first.end()) return;
  for (auto &pr : it->second) out.push_back({pr.first, *pr.second});
}

// Product of two signature maps that must meet exactly in `shared`.
static void join_into(SigMap &dst, const SigMap &a, const SigMap &b, unsigned shared, u128 scale = 1) {
  for (auto &x : a)
    for (auto &y : b)
      if ((x.first & y.first) == shared) dst[x.first | y.first] += x.second * y.second * scale;
}

// ---------------------------------------------------------------- leaf block
// U(x, alpha) = sum over y in N(x) of A_a(x) * E(x,y) * A_b(y), the three
// pieces meeting in chi(x) and chi(y) respectively and disjoint otherwise.
static void solve_leaf(Ctx &c, int bi) {
  const Block &B = c.plan.blocks[bi];
  int a = B.nodes[0];
  Unary U(c.g.n);
  int ea = B.edge_ann[0];
  bool first_is_a = (ea >= 0) && (B.edge_first[0] == a);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t x = 0; x < c.g.n; x++) {
    std::vector<std::pair<int64_t, SigMap>> ent;
    edge_entries(c, ea, first_is_a, x, ent);
    SigMap ax = node_table(c, B.node_ann[0], x);
    SigMap acc;
    for (auto &pr : ent) {
      int64_t y = pr.first;
      SigMap ay = node_table(c, B.node_ann[1], y);
      SigMap t;
      join_into(t, ax, pr.second, cbit(c, x));
      SigMap t2;
      join_into(t2, t, ay, cbit(c, y));
      for (auto &z : t2) acc[z.first] += z.second;
    }
    U[x] = std::move(acc);
  }
  c.unary[bi] = std::move(U);
}

// ---------------------------------------------------------------- cycle block
// Path-table key: end vertex v plus the recorded images of boundary nodes
// lying strictly inside the path (up to two extra fields).
struct PKey {
  int64_t v, x1, x2;
  unsigned sig;
  bool operator==(const PKey &o) const { return v == o.v && x1 == o.x1 && x2 == o.x2 && sig == o.sig; }
};
struct PKeyHash {
  size_t operator()(const PKey &p) const {
    u64 h = mix64((u64)p.v ^ mix64((u64)p.x1 + 7 * (u64)p.x2) ^ ((u64)p.sig << 40));
    return (size_t)h;
  }
};
typedef std::unordered_map<PKey, u128, PKeyHash> PTable;

// Position of a query node among a block's boundary nodes, or -1.
static int bpos(const Block &B, int node) {
  for (size_t i = 0; i < B.boundary.size(); i++)
    if (B.boundary[i] == node) return (int)i;
  return -1;
}

// Build cnt*(u, ., . | P) for the path that starts at cycle position h and
// walks `dir` (+1 or -1) for `len` edges.  `join_start` joins a_h's block on
// u; `join_end` joins a_d's block at the end.  Boundary nodes met strictly
// inside the path have their image recorded in x1 (first boundary) or x2.
static PTable build_path(const Ctx &c, const Block &B, int h, int dir, int len, int64_t u,
                         bool join_start, bool join_end) {
  int L = (int)B.nodes.size();
  auto pos = [&](int s) { return ((h + dir * s) % L + L) % L; };
  // edge index between positions p and p+dir, and whether a_p is the child's first boundary
  auto edge_of = [&](int p) {
    int e = dir > 0 ? p : ((p - 1) % L + L) % L;
    return e;
  };
  PTable cur;
  // init: edge (a_h, a_{h+dir}), optionally joined with a_h's block at u
  {
    int p0 = pos(0), p1 = pos(1);
    int e = edge_of(p0);
    int blk = B.edge_ann[e];
    bool first_is_p0 = blk >= 0 && B.edge_first[e] == B.nodes[p0];
    std::vector<std::pair<int64_t, SigMap>> ent;
    edge_entries(c, blk, first_is_p0, u, ent);
    SigMap au = join_start ? node_table(c, B.node_ann[p0], u) : SigMap{{cbit(c, u), (u128)1}};
    int bp = (len > 1) ? bpos(B, B.nodes[p1]) : -1;
    for (auto &pr : ent) {
      int64_t v = pr.first;
      if (!higher(c, u, v)) continue;
      SigMap t;
      join_into(t, au, pr.second, cbit(c, u));
      for (auto &z : t) {
        PKey key{v, -1, -1, z.first};
        if (bp == 0) key.x1 = v;
        if (bp == 1) key.x2 = v;
        cur[key] += z.second;
      }
    }
  }
  // steps j = 1 .. len-1: NodeJoin(a_j) then EdgeJoin over (a_j, a_{j+dir})
  for (int s = 1; s < len; s++) {
    int pj = pos(s), pn = pos(s + 1);
    int nblk = B.node_ann[pj];
    if (nblk >= 0) {
      PTable nxt;
      for (auto &kv : cur) {
        const SigMap &U = c.unary[nblk][kv.first.v];
        for (auto &z : U)
          if ((z.first & kv.first.sig) == cbit(c, kv.first.v)) {
            PKey key = kv.first;
            key.sig |= z.first;
            nxt[key] += kv.second * z.second;
          }
      }
      cur.swap(nxt);
    }
    int e = edge_of(pj);
    int eblk = B.edge_ann[e];
    bool first_is_pj = eblk >= 0 && B.edge_first[e] == B.nodes[pj];
    int bp = (s + 1 < len) ? bpos(B, B.nodes[pn]) : -1;
    PTable nxt;
    std::vector<std::pair<int64_t, SigMap>> ent;
    for (auto &kv : cur) {
      int64_t v = kv.first.v;
      edge_entries(c, eblk, first_is_pj, v, ent);
      for (auto &pr : ent) {
        int64_t w = pr.first;
        if (!higher(c, u, w)) continue;
        for (auto &z : pr.second) {
          if ((z.first & kv.first.sig) != cbit(c, v)) continue;
          PKey key = kv.first;
          key.v = w;
          key.sig |= z.first;
          if (bp == 0) key.x1 = w;
          if (bp == 1) key.x2 = w;
          nxt[key] += kv.second * z.second;
        }
      }
    }
    cur.swap(nxt);
  }
  if (join_end) {
    int pd = pos(len);
    int nblk = B.node_ann[pd];
    if (nblk >= 0) {
      PTable nxt;
      for (auto &kv : cur) {
        const SigMap &U = c.unary[nblk][kv.first.v];
        for (auto &z : U)
          if ((z.first & kv.first.sig) == cbit(c, kv.first.v)) {
            PKey key = kv.first;
            key.sig |= z.first;
            nxt[key] += kv.second * z.second;
          }
      }
      cur.swap(nxt);
    }
  }
  return cur;
}

struct CycleOut {
  u128 scalar = 0;
  Unary unary;
  Binary binary;
};

// Solve a cycle block: sum over h of the high-starting merges (Eq. (1)).
// For the root, `per_source` (if given) receives the count of the colourful
// matches whose highest cycle vertex is each source u.
static void solve_cycle(Ctx &c, int bi, const std::vector<int64_t> &sources, u128 *per_source,
                        u128 *total) {
  const Block &B = c.plan.blocks[bi];
  int L = (int)B.nodes.size();
  int nb = (int)B.boundary.size();
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  std::vector<u128> tsum(nthreads, 0);
  std::vector<Unary> tun(nb == 1 ? nthreads : 0);
  std::vector<Binary> tbin(nb == 2 ? nthreads : 0);
  for (auto &x : tun) x.assign(c.g.n, SigMap());

#pragma omp parallel for schedule(dynamic, 1)
  for (size_t si = 0; si < sources.size(); si++) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    int64_t u = sources[si];
    u128 mine = 0;
    for (int h = 0; h < L; h++) {
      int half = L / 2;
      int d = (h + half) % L;
      // P+ walks +1 for floor(L/2) edges and joins a_d; P- walks -1 for the
      // rest and joins a_h on u.
      PTable pp = build_path(c, B, h, +1, half, u, false, true);
      if (pp.empty()) continue;
      PTable pm = build_path(c, B, h, -1, L - half, u, true, false);
      if (pm.empty()) continue;
      // group P- by end vertex
      std::unordered_map<int64_t, std::vector<std::pair<const PKey *, u128>>> byv;
      for (auto &kv : pm) byv[kv.first.v].push_back({&kv.first, kv.second});
      unsigned cu = cbit(c, u);
      for (auto &kv : pp) {
        auto it = byv.find(kv.first.v);
        if (it == byv.end()) continue;
        int64_t v = kv.first.v;
        unsigned both = cu | cbit(c, v);
        for (auto &o : it->second) {
          if ((kv.first.sig & o.first->sig) != both) continue;
          u128 val = kv.second * o.second;
          unsigned sig = kv.first.sig | o.first->sig;
          // image of each boundary node
          int64_t img[2] = {-1, -1};
          for (int b = 0; b < nb; b++) {
            int node = B.boundary[b];
            if (node == B.nodes[h]) img[b] = u;
            else if (node == B.nodes[d]) img[b] = v;
            else {
              int64_t f1 = b == 0 ? kv.first.x1 : kv.first.x2;
              int64_t f2 = b == 0 ? o.first->x1 : o.first->x2;
              img[b] = f1 >= 0 ? f1 : f2;
            }
          }
          if (nb == 0) {
            mine += val;
          } else if (nb == 1) {
            tun[tid][img[0]][sig] += val;
          } else {
            tbin[tid][{img[0], img[1]}][sig] += val;
          }
        }
      }
    }
    if (nb == 0) {
      tsum[tid] += mine;
      if (per_source) per_source[si] = mine;
    }
  }
  if (nb == 0) {
    u128 s = 0;
    for (auto x : tsum) s += x;
    *total = s;
  } else if (nb == 1) {
    Unary U(c.g.n);
    for (auto &t : tun)
      for (int64_t x = 0; x < c.g.n; x++)
        for (auto &z : t[x]) U[x][z.first] += z.second;
    c.unary[bi] = std::move(U);
  } else {
    Binary T;
    for (auto &t : tbin)
      for (auto &kv : t)
        for (auto &z : kv.second) T[kv.first][z.first] += z.second;
    c.binary[bi] = std::move(T);
    BinIndex f, r;
    for (auto &kv : c.binary[bi]) {
      f.by_first[kv.first.first].push_back({kv.first.second, &kv.second});
      r.by_first[kv.first.second].push_back({kv.first.first, &kv.second});
    }
    c.bidx[bi] = std::move(f);
    c.bidx_rev[bi] = std::move(r);
  }
}

static void setup(Ctx &c, int64_t n, const int64_t *rp, const int32_t *col, const uint8_t *chi, int k,
                  const Query &q, int reverse_ties) {
  c.g = G{n, rp, col};
  c.k = k;
  c.chi = chi;
  // degree order: ascending degree, ties by id (ascending, or descending when
  // reverse_ties); rank = position in that order
  std::vector<int64_t> ord(n);
  for (int64_t i = 0; i < n; i++) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    int64_t da = c.g.deg(a), db = c.g.deg(b);
    if (da != db) return da < db;
    return reverse_ties ? a > b : a < b;
  });
  c.rank.assign(n, 0);
  for (int64_t i = 0; i < n; i++) c.rank[ord[i]] = i;
  c.plan = decompose(q);
  size_t nbk = c.plan.blocks.size();
  c.unary.assign(nbk, Unary());
  c.binary.assign(nbk, Binary());
  c.bidx.assign(nbk, BinIndex());
  c.bidx_rev.assign(nbk, BinIndex());
}

static void solve_non_root(Ctx &c) {
  std::vector<int64_t> all(c.g.n);
  for (int64_t i = 0; i < c.g.n; i++) all[i] = i;
  for (size_t bi = 0; bi < c.plan.blocks.size(); bi++) {
    const Block &B = c.plan.blocks[bi];
    if (B.root) continue;
    if (B.kind == LEAF) solve_leaf(c, (int)bi);
    else solve_cycle(c, (int)bi, all, nullptr, nullptr);
  }
}

static u128 root_count(Ctx &c, const std::vector<int64_t> &sources, u128 *per_source) {
  if (c.plan.root_block >= 0) {
    u128 t = 0;
    solve_cycle(c, c.plan.root_block, sources, per_source, &t);
    return t;
  }
  // singleton root: sum of the child table over all vertices (full colour set)
  unsigned K = (c.k >= 32) ? 0xffffffffu : ((1u << c.k) - 1u);
  u128 s = 0;
  int ch = c.plan.root_single_child;
  for (size_t i = 0; i < sources.size(); i++) {
    int64_t x = sources[i];
    u128 v = 0;
    if (ch >= 0) {
      auto it = c.unary[ch][x].find(K);
      if (it != c.unary[ch][x].end()) v = it->second;
    }
    if (per_source) per_source[i] = v;
    s += v;
  }
  return s;
}

static void put128(u128 v, u64 *out) {
  out[0] = (u64)v;
  out[1] = (u64)(v >> 64);
}

}  // namespace

// ================================================================ C ABI
extern "C" {

// splitmix64 output function and the colouring contract.
u64 orc_mix64(u64 x) { return mix64(x); }

void orc_colours(int64_t n, int k, u64 seed, int trial, uint8_t *out) {
  for (int64_t v = 0; v < n; v++) out[v] = (uint8_t)colour_of(seed, trial, k, (u64)v);
}

// O1: number of colourful matches (colours != null) or of all matches
// (colours == null).  Result in out[0] (low) and out[1] (high).
int orc_brute(int64_t n, const int64_t *rp, const int32_t *col, const uint8_t *colours, int k, int ne,
              const int32_t *qe, u64 *out) {
  try {
    G g{n, rp, col};
    Query q = make_query(k, ne, qe);
    u128 total = 0;
#pragma omp parallel reduction(+ : total)
    {
      Brute br(g, q, colours, colours != nullptr);
#pragma omp for schedule(dynamic, 16)
      for (int64_t x = 0; x < n; x++) total += br.run_from(x);
    }
    put128(total, out);
    return 0;
  } catch (...) {
    return -1;
  }
}

// Describe the oracle's own decomposition: for each block, kind, size,
// boundary count, its nodes, and its children.  Format (ints):
//   [nblocks, root_block, root_single_child,
//    per block: kind, root, size, L, nodes[L], nbd, bd[nbd], nchild, child[nchild]]
// `order` (may be null) is a flat list of node sets to contract in sequence,
// each given as a count followed by that many nodes; `norder` ints in total.
int orc_plan(int k, int ne, const int32_t *qe, const int32_t *order, int norder, int32_t *out, int cap) {
  try {
    Query q = make_query(k, ne, qe);
    std::vector<std::vector<int>> forced;
    for (int i = 0; order && i < norder;) {
      int c = order[i++];
      forced.push_back(std::vector<int>(order + i, order + i + c));
      i += c;
    }
    Plan p = decompose(q, forced);
    std::vector<int32_t> v;
    v.push_back((int32_t)p.blocks.size());
    v.push_back(p.root_block);
    v.push_back(p.root_single_child);
    for (auto &B : p.blocks) {
      v.push_back(B.kind);
      v.push_back(B.root ? 1 : 0);
      v.push_back(B.size);
      v.push_back((int32_t)B.nodes.size());
      for (int x : B.nodes) v.push_back(x);
      v.push_back((int32_t)B.boundary.size());
      for (int x : B.boundary) v.push_back(x);
      std::vector<int> ch;
      for (int x : B.node_ann) if (x >= 0) ch.push_back(x);
      for (int x : B.edge_ann) if (x >= 0) ch.push_back(x);
      v.push_back((int32_t)ch.size());
      for (int x : ch) v.push_back(x);
    }
    if ((int)v.size() > cap) return -2;
    std::copy(v.begin(), v.end(), out);
    return (int)v.size();
  } catch (std::exception &) {
    return -1;
  }
}

// O3: the DB dynamic program.  Writes the exact colourful count (u128 as two
// u64).  When `sources`/`nsrc` are given, only those root sources are
// counted and `per_source` (2*nsrc u64) receives each one's share; the
// non-root tables are always built in full.
int orc_db(int64_t n, const int64_t *rp, const int32_t *col, const uint8_t *colours, int k, int ne,
           const int32_t *qe, int reverse_ties, const int64_t *sources, int64_t nsrc, u64 *per_source,
           u64 *out) {
  try {
    Query q = make_query(k, ne, qe);
    Ctx c;
    setup(c, n, rp, col, colours, k, q, reverse_ties);
    solve_non_root(c);
    std::vector<int64_t> src;
    if (sources) src.assign(sources, sources + nsrc);
    else { src.resize(n); for (int64_t i = 0; i < n; i++) src[i] = i; }
    std::vector<u128> ps(src.size(), 0);
    u128 t = root_count(c, src, ps.data());
    put128(t, out);
    if (per_source)
      for (size_t i = 0; i < src.size(); i++) put128(ps[i], per_source + 2 * i);
    return 0;
  } catch (std::exception &) {
    return -1;
  }
}

// O3 with the width check of 64-bit tables (the paper fixes no counter
// width; the reading used here: table entries are 64-bit and overflow is
// flagged, never wrapped).  out[0..1] = the exact count (u128), out[2] = 1
// when some entry of a child block's table -- a count of colourful matches
// of the block's subquery keyed by its boundary images (Section 4.3) -- does
// not fit in 64 bits.  The oracle's path tables and partial sums are not
// checked: they depend on its own tie-break and decomposition.
int orc_db_flagged(int64_t n, const int64_t *rp, const int32_t *col, const uint8_t *colours, int k, int ne,
                   const int32_t *qe, int reverse_ties, u64 *out) {
  try {
    Query q = make_query(k, ne, qe);
    Ctx c;
    setup(c, n, rp, col, colours, k, q, reverse_ties);
    solve_non_root(c);
    const u128 lim = (u128)1 << 64;
    bool wide = false;
    for (size_t bi = 0; bi < c.plan.blocks.size(); bi++) {
      for (auto &row : c.unary[bi])
        for (auto &z : row) wide |= z.second >= lim;
      for (auto &kv : c.binary[bi])
        for (auto &z : kv.second) wide |= z.second >= lim;
    }
    std::vector<int64_t> src(n);
    for (int64_t i = 0; i < n; i++) src[i] = i;
    std::vector<u128> ps(src.size(), 0);
    put128(root_count(c, src, ps.data()), out);
    out[2] = wide ? 1 : 0;
    return 0;
  } catch (std::exception &) {
    return -1;
  }
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
