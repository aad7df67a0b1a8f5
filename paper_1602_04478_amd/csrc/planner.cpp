// Host planner: decomposition trees (Section 4.1), the tree-choice heuristic
// (Section 6), aut(Q) (Preliminaries) and, per cycle block, the frontier
// program that the device executor runs for each group of sources.
//
// Cycle programs.  For a cycle block, the colourful matches are partitioned
// by the cycle node a_h whose image u is highest in the degree order (Eq. (1));
// for each h the matches are assembled from high-starting paths out of u
// (every other cycle vertex lower than u).  Which split is used depends on
// where the block's boundary nodes sit:
//   * no boundary (root): split at d = h + floor(L/2) (P+ gets floor(L/2)
//     edges and a_d's block, P- the rest and a_h's block) and count;
//   * one boundary a_p, h = p: same split, counts summed over the meeting
//     vertex into the table row of u;
//   * one boundary a_p, h != p: split at p instead of d -- the two paths meet
//     at p's image, which keys the output directly, so no extra field is
//     needed to carry it;
//   * two adjacent boundaries a_i, a_{i+1}: the two paths run from u to a_i
//     and to a_{i+1} and are closed through the edge (a_i, a_{i+1}); when
//     a_h is itself one of the two, one side is just u.
// Each path is a chain of frontier operations (INIT over the first edge,
// NodeJoin, EdgeJoin).  Identical chain prefixes are computed once, and
// merges sharing one side are combined by linearity (sum of the other sides,
// factored from the end of the chains), which is where the h-cases of a
// cycle with few annotations collapse into a handful of chains.
#include <algorithm>
#include <functional>
#include <map>
#include <set>
#include <sstream>
#include <tuple>

#include "cc_internal.h"

namespace cc {

namespace {

// ------------------------------------------------------------------ working query
struct Ann {
  std::string desc;   // canonical description of the annotating block
  int id = -1;        // block index in the tree being built
};

struct WQ {
  int k;
  std::vector<char> alive;
  std::vector<std::set<int>> adj;
  std::vector<int> node_ann;                        // block index or -1
  std::map<std::pair<int, int>, std::pair<int, int>> edge_ann;  // (lo,hi) -> (block, first node)
};

static std::pair<int, int> ek(int a, int b) { return {std::min(a, b), std::max(a, b)}; }

struct Tree {
  std::vector<PBlock> blocks;
  std::vector<std::string> desc;  // canonical text per block
};

// canonical text of a block: kind, sorted node set, boundary, child descs
static std::string block_desc(const PBlock &B, const std::vector<std::string> &descs) {
  std::ostringstream os;
  os << (B.kind == BK_LEAF ? "L" : "C") << "[";
  std::vector<int> ns = B.nodes;
  std::sort(ns.begin(), ns.end());
  for (int x : ns) os << x << ",";
  os << "|";
  std::vector<int> bd = B.boundary;
  std::sort(bd.begin(), bd.end());
  for (int x : bd) os << x << ",";
  os << "|";
  std::vector<std::string> ch;
  for (int c : B.node_child)
    if (c >= 0) ch.push_back(descs[c]);
  for (int c : B.edge_child)
    if (c >= 0) ch.push_back(descs[c]);
  std::sort(ch.begin(), ch.end());
  for (auto &c : ch) os << c << ";";
  os << "]";
  return os.str();
}

static std::string state_key(const WQ &w, const Tree &t) {
  std::ostringstream os;
  for (int x = 0; x < w.k; x++)
    if (w.alive[x]) {
      os << x << ":" << (w.node_ann[x] >= 0 ? t.desc[w.node_ann[x]] : "-") << "{";
      for (int y : w.adj[x])
        if (y > x) {
          auto it = w.edge_ann.find(ek(x, y));
          os << y;
          if (it != w.edge_ann.end()) os << "=" << t.desc[it->second.first] << "@" << it->second.second;
          os << ",";
        }
      os << "}";
    }
  return os.str();
}

static int nalive(const WQ &w) {
  int c = 0;
  for (char a : w.alive) c += a;
  return c;
}

// all simple cycles of the live query, each once (as a node sequence)
static void all_cycles(const WQ &w, std::vector<std::vector<int>> &out) {
  std::vector<int> path;
  std::vector<char> on(w.k, 0);
  for (int s = 0; s < w.k; s++) {
    if (!w.alive[s]) continue;
    path.assign(1, s);
    std::fill(on.begin(), on.end(), 0);
    on[s] = 1;
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

// contractible cycles: induced, <= 2 boundary nodes (0 only if it is all of Q)
struct CycleCand {
  std::vector<int> nodes;
  std::vector<int> bd;
};
static std::vector<CycleCand> contractible(const WQ &w) {
  std::vector<std::vector<int>> cyc;
  all_cycles(w, cyc);
  std::vector<CycleCand> out;
  int live = nalive(w);
  for (auto &c : cyc) {
    std::set<int> cs(c.begin(), c.end());
    int L = (int)c.size(), inner = 0;
    for (int x : c)
      for (int y : w.adj[x])
        if (cs.count(y)) inner++;
    if (inner != 2 * L) continue;
    std::vector<int> bd;
    for (int x : c) {
      bool outside = false;
      for (int y : w.adj[x])
        if (!cs.count(y)) outside = true;
      if (outside) bd.push_back(x);
    }
    if (bd.size() > 2) continue;
    if (bd.empty() && live != L) continue;
    out.push_back({c, bd});
  }
  return out;
}

static int new_block(WQ &w, Tree &t, PBlock B) {
  int id = (int)t.blocks.size();
  t.desc.push_back(block_desc(B, t.desc));
  t.blocks.push_back(std::move(B));
  return id;
}

// Case 3: contract leaf edge (a, b), b of degree one.
static void contract_leaf(WQ &w, Tree &t, int a, int b) {
  PBlock B;
  B.kind = BK_LEAF;
  B.nodes = {a, b};
  B.node_child = {w.node_ann[a], w.node_ann[b]};
  auto it = w.edge_ann.find(ek(a, b));
  if (it != w.edge_ann.end()) {
    B.edge_child = {it->second.first};
    B.edge_first_lo = {(char)(it->second.second == a)};
    w.edge_ann.erase(it);
  } else {
    B.edge_child = {-1};
    B.edge_first_lo = {0};
  }
  B.boundary = {a};
  B.size = 2;
  for (int c : B.node_child)
    if (c >= 0) B.size += t.blocks[c].size - 1;
  if (B.edge_child[0] >= 0) B.size += t.blocks[B.edge_child[0]].size - 2;
  w.adj[a].erase(b);
  w.adj[b].erase(a);
  w.alive[b] = 0;
  w.node_ann[b] = -1;
  int id = new_block(w, t, std::move(B));
  w.node_ann[a] = id;
}

// Cases 1 and 2 (and the root cycle when it has no boundary).
static void contract_cycle(WQ &w, Tree &t, const CycleCand &cc) {
  PBlock B;
  int L = (int)cc.nodes.size();
  B.kind = cc.bd.empty() ? BK_ROOT_CYCLE : BK_CYCLE;
  B.nodes = cc.nodes;
  B.boundary = cc.bd;
  B.size = L;
  for (int i = 0; i < L; i++) {
    int a = cc.nodes[i], b = cc.nodes[(i + 1) % L];
    B.node_child.push_back(w.node_ann[a]);
    if (w.node_ann[a] >= 0) B.size += t.blocks[w.node_ann[a]].size - 1;
    auto it = w.edge_ann.find(ek(a, b));
    if (it != w.edge_ann.end()) {
      B.edge_child.push_back(it->second.first);
      B.edge_first_lo.push_back((char)(it->second.second == a));
      B.size += t.blocks[it->second.first].size - 2;
      w.edge_ann.erase(it);
    } else {
      B.edge_child.push_back(-1);
      B.edge_first_lo.push_back(0);
    }
    w.adj[a].erase(b);
    w.adj[b].erase(a);
  }
  std::set<int> bds(cc.bd.begin(), cc.bd.end());
  for (int x : cc.nodes) {
    w.node_ann[x] = -1;
    if (!bds.count(x)) w.alive[x] = 0;
  }
  int id = new_block(w, t, std::move(B));
  if (cc.bd.empty()) {
    for (int x : cc.nodes) w.alive[x] = 0;
  } else if (cc.bd.size() == 1) {
    w.node_ann[cc.bd[0]] = id;
  } else {
    int a = cc.bd[0], b = cc.bd[1];
    w.adj[a].insert(b);
    w.adj[b].insert(a);
    w.edge_ann[ek(a, b)] = {id, a};
  }
}

static bool adjacent_in_cycle(const std::vector<int> &c, int a, int b) {
  int L = (int)c.size();
  for (int i = 0; i < L; i++)
    if ((c[i] == a && c[(i + 1) % L] == b) || (c[i] == b && c[(i + 1) % L] == a)) return true;
  return false;
}

struct TreeScore {
  int no_pairs;      // 1 if every two-boundary block has adjacent boundary nodes (no pair-keyed table)
  int root_is_cycle; // prefer a cycle root (no table for it)
  int longest, sumbd, nann;
};

static TreeScore score(const Tree &t) {
  TreeScore s{1, 0, 0, 0, 0};
  for (auto &B : t.blocks) {
    if (B.kind == BK_CYCLE || B.kind == BK_ROOT_CYCLE) s.longest = std::max(s.longest, (int)B.nodes.size());
    s.sumbd += (int)B.boundary.size();
    for (int c : B.node_child) s.nann += c >= 0;
    for (int c : B.edge_child) s.nann += c >= 0;
    if (B.boundary.size() == 2 && !adjacent_in_cycle(B.nodes, B.boundary[0], B.boundary[1])) s.no_pairs = 0;
  }
  s.root_is_cycle = !t.blocks.empty() && t.blocks.back().kind == BK_ROOT_CYCLE;
  return s;
}

static bool better(const TreeScore &a, const TreeScore &b) {
  // trees without pair-keyed tables first (those tables can be quadratic in
  // the data graph); then the heuristic of Section 6; then a cycle root
  if (a.no_pairs != b.no_pairs) return a.no_pairs > b.no_pairs;
  if (a.longest != b.longest) return a.longest < b.longest;
  if (a.sumbd != b.sumbd) return a.sumbd < b.sumbd;
  if (a.nann != b.nann) return a.nann < b.nann;
  return a.root_is_cycle > b.root_is_cycle;
}

// Enumerate trees: leaf edges are contracted greedily (lowest leaf first);
// every choice among contractible cycles is a branch.  States reached twice
// (independent contractions commute) are explored once.
struct Search {
  std::set<std::string> seen;
  std::set<std::string> seen_trees;
  bool have = false;
  Tree best;
  TreeScore best_score{};
  int best_index = -1;
  int states = 0;
  bool found_any = false;
  // every distinct tree, in the order found (kept up to kMaxTrees)
  static constexpr size_t kMaxTrees = 4096;
  std::vector<Tree> trees;
  std::vector<TreeScore> scores;

  void finish(WQ &w, Tree &t) {
    // the last live node, if any, becomes a singleton root
    Tree tt = t;
    int last = -1;
    for (int x = 0; x < w.k; x++)
      if (w.alive[x]) last = x;
    if (last >= 0) {
      PBlock R;
      R.kind = BK_ROOT_SINGLE;
      R.nodes = {last};
      R.node_child = {w.node_ann[last]};
      R.single_child = w.node_ann[last];
      R.size = w.node_ann[last] >= 0 ? tt.blocks[w.node_ann[last]].size : 1;
      tt.desc.push_back("R");
      tt.blocks.push_back(R);
    }
    std::string key;
    for (auto &d : tt.desc) key += d + "#";
    found_any = true;
    if (!seen_trees.insert(key).second) return;
    TreeScore s = score(tt);
    if (trees.size() < kMaxTrees) {
      trees.push_back(tt);
      scores.push_back(s);
    }
    if (!have || better(s, best_score)) {
      have = true;
      best = tt;
      best_score = s;
      best_index = trees.size() <= kMaxTrees ? (int)trees.size() - 1 : -1;
    }
  }

  void rec(WQ w, Tree t) {
    // greedy leaves
    for (;;) {
      if (nalive(w) <= 1) {
        finish(w, t);
        return;
      }
      int leaf = -1;
      for (int b = 0; b < w.k; b++)
        if (w.alive[b] && w.adj[b].size() == 1) {
          leaf = b;
          break;
        }
      if (leaf < 0) break;
      contract_leaf(w, t, *w.adj[leaf].begin(), leaf);
    }
    if (!seen.insert(state_key(w, t)).second) return;
    if (++states > 20000) return;
    auto cands = contractible(w);
    for (auto &c : cands) {
      WQ w2 = w;
      Tree t2 = t;
      contract_cycle(w2, t2, c);
      if (c.bd.empty()) {
        finish(w2, t2);
      } else {
        rec(w2, t2);
      }
    }
  }
};

static uint64_t count_aut(int k, const std::vector<std::set<int>> &adj) {
  std::vector<int> img(k, -1), used(k, 0);
  uint64_t cnt = 0;
  std::function<void(int)> rec = [&](int i) {
    if (i == k) {
      cnt++;
      return;
    }
    for (int j = 0; j < k; j++) {
      if (used[j] || adj[j].size() != adj[i].size()) continue;
      bool ok = true;
      for (int p = 0; p < i && ok; p++) ok = (adj[i].count(p) > 0) == (adj[j].count(img[p]) > 0);
      if (!ok) continue;
      used[j] = 1;
      img[i] = j;
      rec(i + 1);
      used[j] = 0;
      img[i] = -1;
    }
  };
  rec(0);
  return cnt;
}

// ------------------------------------------------------------------ cycle programs
struct Tok {
  int kind;  // 0 INIT, 1 NJ, 2 EJ
  int tab;
  int src_first;
  int ntab;
  bool operator<(const Tok &o) const {
    return std::tie(kind, tab, src_first, ntab) < std::tie(o.kind, o.tab, o.src_first, o.ntab);
  }
  bool operator==(const Tok &o) const {
    return kind == o.kind && tab == o.tab && src_first == o.src_first && ntab == o.ntab;
  }
};
typedef std::vector<Tok> Chain;

struct ProgBuilder {
  const Plan &plan;
  const PBlock &B;
  Program prog;
  std::map<std::pair<int, Tok>, int> memo;  // (input register or -1, token) -> register

  ProgBuilder(const Plan &p, const PBlock &b) : plan(p), B(b) {}

  int child_size(int c, int dflt) const { return c >= 0 ? plan.blocks[c].size : dflt; }

  int new_reg(int s) {
    prog.reg_s.push_back(s);
    return (int)prog.reg_s.size() - 1;
  }

  int apply(int in, const Tok &t) {
    auto key = std::make_pair(in, t);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    Op op;
    int s;
    if (t.kind == 0) {
      op.kind = OP_INIT;
      s = child_size(t.ntab, 1) + child_size(t.tab, 2) - 1;
      op.tab = t.tab;
      op.tab_src_first = t.src_first;
      op.ntab = t.ntab;
    } else if (t.kind == 1) {
      op.kind = OP_NJ;
      op.a = in;
      s = prog.reg_s[in] + child_size(t.tab, 1) - 1;
      op.tab = t.tab;
    } else {
      op.kind = OP_EJ;
      op.a = in;
      s = prog.reg_s[in] + child_size(t.tab, 2) - 1;
      op.tab = t.tab;
      op.tab_src_first = t.src_first;
    }
    op.s = s;
    op.dst = new_reg(s);
    prog.ops.push_back(op);
    memo[key] = op.dst;
    return op.dst;
  }

  int chain(const Chain &c) {
    int r = -1;
    for (auto &t : c) r = apply(r, t);
    return r;
  }

  // sum_i w_i * chain_i, factoring equal trailing operations (linearity of
  // NodeJoin and EdgeJoin).  Returns (register, scalar multiplier).
  std::pair<int, uint64_t> sum(const std::vector<std::pair<uint64_t, Chain>> &items) {
    if (items.size() == 1) return {chain(items[0].second), items[0].first};
    std::map<Tok, std::vector<std::pair<uint64_t, Chain>>> groups;
    std::vector<Tok> order;
    for (auto &it : items) {
      const Tok &last = it.second.back();
      if (!groups.count(last)) order.push_back(last);
      groups[last].push_back(it);
    }
    std::vector<std::pair<int, uint64_t>> terms;
    for (auto &last : order) {
      auto &g = groups[last];
      if (last.kind == 0) {  // chains that are just INIT
        uint64_t wsum = 0;
        for (auto &x : g) wsum += x.first;
        terms.push_back({chain(g[0].second), wsum});
        continue;
      }
      std::vector<std::pair<uint64_t, Chain>> inner;
      for (auto &x : g) inner.push_back({x.first, Chain(x.second.begin(), x.second.end() - 1)});
      auto r = sum(inner);
      terms.push_back({apply(r.first, last), r.second});
    }
    if (terms.size() == 1) return terms[0];
    int s = prog.reg_s[terms[0].first];
    int dst = new_reg(s);
    for (size_t i = 0; i < terms.size(); i++) {
      Op op;
      op.kind = OP_AXPY;
      op.dst = dst;
      op.a = terms[i].first;
      op.w = terms[i].second;
      op.s = s;
      op.first = (i == 0);
      prog.ops.push_back(op);
    }
    return {dst, 1};
  }

  // Chain of a path from cycle position h walking `dir` for `len` edges;
  // `join_start` joins a_h's block on u with the first edge, `join_end`
  // joins the last node's block at the end.
  Chain path(int h, int dir, int len, bool join_start, bool join_end) const {
    int L = (int)B.nodes.size();
    auto pos = [&](int s) { return ((h + dir * s) % L + L) % L; };
    auto edge_tok = [&](int p, int kind, int ntab) {
      int e = dir > 0 ? p : (p - 1 + L) % L;
      Tok t{kind, B.edge_child[e], 0, ntab};
      if (t.tab >= 0) t.src_first = (p == e) ? B.edge_first_lo[e] : !B.edge_first_lo[e];
      return t;
    };
    Chain c;
    c.push_back(edge_tok(pos(0), 0, join_start ? B.node_child[pos(0)] : -1));
    for (int s = 1; s < len; s++) {
      int nc = B.node_child[pos(s)];
      if (nc >= 0) c.push_back(Tok{1, nc, 0, -1});
      c.push_back(edge_tok(pos(s), 2, -1));
    }
    if (join_end) {
      int nc = B.node_child[pos(len)];
      if (nc >= 0) c.push_back(Tok{1, nc, 0, -1});
    }
    return c;
  }
};

struct MergeReq {
  OpKind kind;
  Chain x, y;
  uint64_t w;
};

static Program build_program(const Plan &plan, int bi) {
  const PBlock &B = plan.blocks[bi];
  ProgBuilder pb(plan, B);
  int L = (int)B.nodes.size();
  int half = L / 2;
  std::vector<MergeReq> reqs;
  auto posof = [&](int node) {
    for (int i = 0; i < L; i++)
      if (B.nodes[i] == node) return i;
    return -1;
  };
  int nb = (int)B.boundary.size();
  int edge_i = -1, first_is_lo = 0;
  if (nb == 2 && !B.pair_keyed) {
    int pf = posof(B.boundary[0]), ps = posof(B.boundary[1]);
    if (ps == (pf + 1) % L) {
      edge_i = pf;
      first_is_lo = 1;
    } else {
      edge_i = ps;
      first_is_lo = 0;
    }
  }
  // path splitting: one h only -- the first boundary node (a_0 at the root);
  // a pair-keyed block splits at its two boundary nodes
  const int h_ps = nb == 0 ? 0 : posof(B.boundary[0]);
  for (int h = 0; h < L; h++) {
    if (B.ps && h != h_ps) continue;
    if (B.pair_keyed) {
      const int d = posof(B.boundary[1]);
      const int lx = ((d - h) % L + L) % L;
      Chain x = pb.path(h, +1, lx, false, true);
      Chain y = pb.path(h, -1, L - lx, true, false);
      reqs.push_back({OP_MPAIR, x, y, 1});
      continue;
    }
    if (nb == 0 || (nb == 1 && posof(B.boundary[0]) == h)) {
      Chain pp = pb.path(h, +1, half, false, true);
      Chain pm = pb.path(h, -1, L - half, true, false);
      reqs.push_back({nb == 0 ? OP_MROOT : OP_MU, pp, pm, 1});
    } else if (nb == 1) {
      int p = posof(B.boundary[0]);
      int lx = ((p - h) % L + L) % L;
      Chain x = pb.path(h, +1, lx, false, true);
      Chain y = pb.path(h, -1, L - lx, true, false);
      reqs.push_back({OP_MV, x, y, 1});
    } else {
      int i = edge_i, j = (edge_i + 1) % L;
      if (h != i && h != j) {
        int lx = ((i - h) % L + L) % L;
        Chain x = pb.path(h, +1, lx, false, true);
        Chain y = pb.path(h, -1, L - 1 - lx, true, true);
        reqs.push_back({OP_MEDGE, x, y, 1});
      } else {
        // one side is u itself; the other runs the long way round
        MergeReq r;
        r.kind = OP_MEDGE_T;
        r.w = 1;
        if (h == i) r.y = pb.path(h, -1, L - 1, false, true);
        else r.x = pb.path(h, +1, L - 1, false, true);
        reqs.push_back(r);
      }
    }
  }
  // Symmetric merges (root, MU, MV, pair): put the more frequent side second.
  auto symmetric = [](int kind) {
    return kind == OP_MROOT || kind == OP_MU || kind == OP_MV || kind == OP_MPAIR;
  };
  std::map<Chain, int> freq;
  for (auto &r : reqs)
    if (symmetric(r.kind)) {
      freq[r.x]++;
      freq[r.y]++;
    }
  for (auto &r : reqs)
    if (symmetric(r.kind)) {
      int fx = freq[r.x], fy = freq[r.y];
      if (fx > fy || (fx == fy && r.y < r.x)) std::swap(r.x, r.y);
    }
  // Edge merges: group on whichever side has fewer distinct chains.
  std::set<Chain> dx, dy;
  for (auto &r : reqs)
    if (r.kind == OP_MEDGE) {
      dx.insert(r.x);
      dy.insert(r.y);
    }
  bool group_on_x = dx.size() < dy.size();
  // group: (kind, fixed side) -> list of (w, other side)
  std::map<std::pair<int, Chain>, std::vector<std::pair<uint64_t, Chain>>> groups;
  std::vector<std::pair<int, Chain>> gorder;
  std::vector<MergeReq> trivial;
  for (auto &r : reqs) {
    if (r.kind == OP_MEDGE_T) {
      trivial.push_back(r);
      continue;
    }
    bool fixx = (r.kind == OP_MEDGE) && group_on_x;
    auto key = std::make_pair((int)r.kind * 2 + (fixx ? 1 : 0), fixx ? r.x : r.y);
    if (!groups.count(key)) gorder.push_back(key);
    groups[key].push_back({r.w, fixx ? r.y : r.x});
  }
  for (auto &key : gorder) {
    OpKind kind = (OpKind)(key.first / 2);
    bool fixx = key.first % 2;
    auto other = pb.sum(groups[key]);
    int fixed = pb.chain(key.second);
    Op op;
    op.kind = kind;
    op.a = fixx ? fixed : other.first;
    op.b = fixx ? other.first : fixed;
    op.w = other.second;
    if (kind == OP_MEDGE) {
      op.tab = B.edge_child[edge_i];
      op.tab_src_first = op.tab >= 0 ? B.edge_first_lo[edge_i] : 0;
      op.first = first_is_lo;
    }
    op.s = B.size;
    pb.prog.ops.push_back(op);
  }
  for (auto &r : trivial) {
    Op op;
    op.kind = OP_MEDGE_T;
    op.w = r.w;
    op.s = B.size;
    bool swapped = r.y.empty();  // u is the image of a_{i+1}; the path ends at a_i
    op.swapped = swapped;
    int p_u = swapped ? (edge_i + 1) % L : edge_i;
    op.b = pb.chain(swapped ? r.x : r.y);
    op.ntab = B.node_child[p_u];
    op.tab = B.edge_child[edge_i];
    // u's end is the child's first boundary?
    op.tab_src_first = op.tab >= 0 ? (swapped ? !B.edge_first_lo[edge_i] : B.edge_first_lo[edge_i]) : 0;
    // u's end is the block's first boundary?
    op.first = swapped ? !first_is_lo : first_is_lo;
    pb.prog.ops.push_back(op);
  }
  // register lifetimes and depths
  Program &P = pb.prog;
  P.reg_depth.assign(P.reg_s.size(), 0);
  for (auto &o : P.ops) {
    if (o.kind == OP_INIT) P.reg_depth[o.dst] = 1;
    else if (o.kind == OP_EJ) P.reg_depth[o.dst] = P.reg_depth[o.a] + 1;
    else if (o.kind == OP_NJ || o.kind == OP_AXPY) P.reg_depth[o.dst] = P.reg_depth[o.a];
  }
  for (int d : P.reg_depth) P.max_depth = std::max(P.max_depth, d);
  P.last_use.assign(P.reg_s.size(), -1);
  for (int i = 0; i < (int)P.ops.size(); i++) {
    const Op &o = P.ops[i];
    for (int r : {o.dst, o.a, o.b})
      if (r >= 0) P.last_use[r] = i;
  }
  return P;
}

}  // namespace

Plan make_plan(int k, const std::vector<std::pair<int, int>> &edges, int mode, int tree) {
  if (k < 2 || k > 12) fail(CC_E_K_RANGE, "k must be in [2, 12]");
  WQ w;
  w.k = k;
  w.alive.assign(k, 1);
  w.adj.assign(k, {});
  w.node_ann.assign(k, -1);
  for (auto &e : edges) {
    int a = e.first, b = e.second;
    if (a < 0 || b < 0 || a >= k || b >= k) fail(CC_E_ARG, "query edge endpoint out of range");
    if (a == b) fail(CC_E_ARG, "query self-loop");
    if (w.adj[a].count(b)) fail(CC_E_ARG, "duplicate query edge");
    w.adj[a].insert(b);
    w.adj[b].insert(a);
  }
  // connectivity
  {
    std::vector<int> seen(k, 0), st{0};
    seen[0] = 1;
    while (!st.empty()) {
      int x = st.back();
      st.pop_back();
      for (int y : w.adj[x])
        if (!seen[y]) {
          seen[y] = 1;
          st.push_back(y);
        }
    }
    for (int x = 0; x < k; x++)
      if (!seen[x]) fail(CC_E_QUERY_DISCONNECTED, "query is not connected");
  }
  if (mode != PLAN_DB && mode != PLAN_PS) fail(CC_E_ARG, "unknown plan mode");
  Plan plan;
  plan.k = k;
  plan.mode = mode;
  plan.edges = edges;
  plan.aut = count_aut(k, w.adj);
  Search S;
  S.rec(w, Tree());
  if (!S.have) fail(CC_E_QUERY_TW, "no decomposition into leaf edges and contractible cycles: treewidth > 2");
  plan.num_trees = (int)S.trees.size();
  const Tree *pick = &S.best;
  TreeScore sc = S.best_score;
  plan.tree = S.best_index;
  if (tree >= 0) {
    if (tree >= (int)S.trees.size()) fail(CC_E_ARG, "no decomposition tree of that index");
    pick = &S.trees[tree];
    sc = S.scores[tree];
    plan.tree = tree;
  }
  plan.blocks = pick->blocks;
  plan.longest_cycle = sc.longest;
  plan.sum_boundary = sc.sumbd;
  plan.num_annotations = sc.nann;
  // children come before parents, so a flag is final when a parent reads it
  for (auto &B : plan.blocks) {
    if (B.kind != BK_CYCLE && B.kind != BK_ROOT_CYCLE) continue;
    if (B.boundary.size() == 2) {
      if (!adjacent_in_cycle(B.nodes, B.boundary[0], B.boundary[1])) {
        B.pair_keyed = true;
      } else {
        // adjacent boundary nodes joined by an edge that is itself a pair
        // table's: the block's table is keyed by those pairs as well
        const int L = (int)B.nodes.size();
        for (int i = 0; i < L; i++) {
          const int x = B.nodes[i], y = B.nodes[(i + 1) % L];
          const bool bedge = (x == B.boundary[0] && y == B.boundary[1]) || (x == B.boundary[1] && y == B.boundary[0]);
          if (bedge && B.edge_child[i] >= 0 && plan.blocks[B.edge_child[i]].pair_keyed) B.pair_keyed = true;
        }
      }
    }
    B.ps = mode == PLAN_PS || B.pair_keyed;
  }
  plan.programs.assign(plan.blocks.size(), Program());
  for (size_t i = 0; i < plan.blocks.size(); i++)
    if (plan.blocks[i].kind == BK_CYCLE || plan.blocks[i].kind == BK_ROOT_CYCLE)
      plan.programs[i] = build_program(plan, (int)i);
  return plan;
}

std::vector<int32_t> describe_plan(const Plan &p) {
  std::vector<int32_t> v;
  v.push_back((int32_t)p.blocks.size());
  for (auto &B : p.blocks) {
    v.push_back(B.kind);
    v.push_back(B.size);
    v.push_back((int32_t)B.nodes.size());
    for (int x : B.nodes) v.push_back(x);
    v.push_back((int32_t)B.boundary.size());
    for (int x : B.boundary) v.push_back(x);
    std::vector<int> ch;
    for (int c : B.node_child)
      if (c >= 0) ch.push_back(c);
    for (int c : B.edge_child)
      if (c >= 0) ch.push_back(c);
    if (B.kind == BK_ROOT_SINGLE) {
      ch.clear();
      if (B.single_child >= 0) ch.push_back(B.single_child);
    }
    v.push_back((int32_t)ch.size());
    for (int c : ch) v.push_back(c);
  }
  return v;
}

}  // namespace cc
