// Graph residency: validate the CSR, order vertices by degree (Section 5.1,
// degree ordering: ascending degree, ties by id), relabel every vertex by its
// rank and sort each neighbour list by rank, so that the neighbours lower than
// any given vertex form a prefix of its list.  Also builds the reverse-slot
// index (slot of (v,u) for the slot of (u,v)), the lower-neighbour counts and
// a two-step reach estimate used to schedule sources.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <functional>
#include <numeric>
#include <thread>

#include "cc_internal.h"

namespace cc {

DevGraph::~DevGraph() {
  if (rp) (void)hipFree(rp);
  if (col) (void)hipFree(col);
  if (rev) (void)hipFree(rev);
  if (orig) (void)hipFree(orig);
  if (lowcnt) (void)hipFree(lowcnt);
  if (deg) (void)hipFree(deg);
  if (split_items) (void)hipFree(split_items);
}

void DevGraph::split_range(int64_t n_lim, const int32_t **items, int *count) const {
  // h_split_w is descending: the items of vertices below n_lim are a suffix
  // (with greater<>, upper_bound finds the first item whose vertex is < n_lim)
  auto it = std::upper_bound(h_split_w.begin(), h_split_w.end(), (int32_t)std::min<int64_t>(n_lim, INT32_MAX),
                             std::greater<int32_t>());
  const int64_t first = it - h_split_w.begin();
  *count = (int)((int64_t)h_split_w.size() - first);
  *items = split_items ? split_items + 2 * first : nullptr;
}

template <typename F>
static void parallel_for(int64_t n, F f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 100000) nt = 1;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; t++)
    th.emplace_back([&, t]() {
      int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
      for (int64_t i = lo; i < hi; i++) f(i);
    });
  for (auto &x : th) x.join();
}

std::unique_ptr<DevGraph> make_graph(int64_t n, const int64_t *row_ptr, const int32_t *col, uint32_t flags,
                                     hipStream_t stream) {
  if (n < 1 || n >= (int64_t(1) << 31)) fail(CC_E_ARG, "n must be in [1, 2^31)");
  if (!row_ptr || (!col && row_ptr[n] > 0)) fail(CC_E_ARG, "null CSR array");
  if (row_ptr[0] != 0) fail(CC_E_GRAPH, "row_ptr[0] must be 0");
  for (int64_t v = 0; v < n; v++)
    if (row_ptr[v + 1] < row_ptr[v]) fail(CC_E_GRAPH, "row_ptr is not non-decreasing");
  int64_t nnz = row_ptr[n];
  bool clean = flags & CC_GRAPH_CLEAN;
  // sorted, validated copy of each row (original ids)
  std::vector<int64_t> rp0(n + 1, 0);
  std::vector<int32_t> c0(nnz);
  std::vector<int64_t> rowlen(n, 0);
  std::vector<int> bad(n, 0);
  parallel_for(n, [&](int64_t v) {
    int64_t s = row_ptr[v], e = row_ptr[v + 1];
    int32_t *dst = c0.data() + s;
    int64_t len = 0;
    for (int64_t i = s; i < e; i++) {
      int32_t x = col[i];
      if (x < 0 || x >= n) {
        bad[v] = 1;
        return;
      }
      if (x == v) {
        if (!clean) {
          bad[v] = 2;
          return;
        }
        continue;
      }
      dst[len++] = x;
    }
    std::sort(dst, dst + len);
    int64_t u = len ? 1 : 0;
    for (int64_t i = 1; i < len; i++) {
      if (dst[i] == dst[i - 1]) {
        if (!clean) {
          bad[v] = 3;
          return;
        }
        continue;
      }
      dst[u++] = dst[i];
    }
    rowlen[v] = u;
  });
  for (int64_t v = 0; v < n; v++) {
    if (bad[v] == 1) fail(CC_E_GRAPH, "neighbour id out of range");
    if (bad[v] == 2) fail(CC_E_GRAPH, "self-loop");
    if (bad[v] == 3) fail(CC_E_GRAPH, "duplicate edge");
  }
  // symmetry: every (v, x) must have (x, v)
  parallel_for(n, [&](int64_t v) {
    const int32_t *s = c0.data() + row_ptr[v];
    for (int64_t i = 0; i < rowlen[v]; i++) {
      int32_t x = s[i];
      const int32_t *xs = c0.data() + row_ptr[x];
      if (!std::binary_search(xs, xs + rowlen[x], (int32_t)v)) {
        bad[v] = 4;
        return;
      }
    }
  });
  for (int64_t v = 0; v < n; v++)
    if (bad[v] == 4) fail(CC_E_GRAPH, "CSR is not symmetric");

  auto G = std::make_unique<DevGraph>();
  G->n = n;
  G->flags = flags;
  // degree order
  std::vector<int32_t> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  bool rev_ties = flags & CC_GRAPH_REVERSE_TIES;
  std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
    if (rowlen[a] != rowlen[b]) return rowlen[a] < rowlen[b];
    return rev_ties ? a > b : a < b;
  });
  G->h_orig = ord;
  G->h_rank.assign(n, 0);
  for (int64_t r = 0; r < n; r++) G->h_rank[ord[r]] = (int32_t)r;
  G->h_rp.assign(n + 1, 0);
  for (int64_t r = 0; r < n; r++) G->h_rp[r + 1] = G->h_rp[r] + rowlen[ord[r]];
  G->m2 = G->h_rp[n];
  G->h_col.assign(G->m2, 0);
  G->h_lowcnt.assign(n, 0);
  int64_t maxd = 0;
  for (int64_t v = 0; v < n; v++) maxd = std::max(maxd, rowlen[v]);
  G->max_degree = maxd;
  parallel_for(n, [&](int64_t r) {
    int32_t v = ord[r];
    const int32_t *s = c0.data() + row_ptr[v];
    int32_t *d = G->h_col.data() + G->h_rp[r];
    int64_t len = rowlen[v];
    for (int64_t i = 0; i < len; i++) d[i] = G->h_rank[s[i]];
    std::sort(d, d + len);
    G->h_lowcnt[r] = (int32_t)(std::lower_bound(d, d + len, (int32_t)r) - d);
  });
  std::vector<int64_t> rev(G->m2);
  parallel_for(n, [&](int64_t r) {
    for (int64_t e = G->h_rp[r]; e < G->h_rp[r + 1]; e++) {
      int32_t x = G->h_col[e];
      const int32_t *xs = G->h_col.data() + G->h_rp[x];
      int64_t pos = std::lower_bound(xs, xs + (G->h_rp[x + 1] - G->h_rp[x]), (int32_t)r) - xs;
      rev[e] = G->h_rp[x] + pos;
    }
  });
  // R2(u): number of two-edge high-starting walks u -> v -> w (v, w < u)
  G->h_r2.assign(n, 0);
  parallel_for(n, [&](int64_t r) {
    int64_t s = 0;
    for (int64_t e = G->h_rp[r]; e < G->h_rp[r] + G->h_lowcnt[r]; e++) s += rev[e] - G->h_rp[G->h_col[e]];
    G->h_r2[r] = s;
  });

  // hub schedule of the dense EdgeJoin (a per-degree bucket: vertices of
  // degree above twice the chunk are cut into chunks of that many neighbours)
  G->split_chunk = 512;
  if (const char *ev = getenv("CC_SPLIT_CHUNK")) G->split_chunk = std::max(0, atoi(ev));
  std::vector<int32_t> items;
  G->split_lo = n;
  if (G->split_chunk > 0) {
    for (int64_t r = n - 1; r >= 0; r--) {
      const int64_t d = G->h_rp[r + 1] - G->h_rp[r];
      if (d <= 2 * (int64_t)G->split_chunk) break;  // ranks ascend with degree
      G->split_lo = r;
      for (int64_t off = 0; off < d; off += G->split_chunk) {
        items.push_back((int32_t)r);
        items.push_back((int32_t)off);
        G->h_split_w.push_back((int32_t)r);
      }
    }
  }

  HIP_CHECK(hipGetDevice(&G->device));
  if (!items.empty()) {
    HIP_CHECK(hipMalloc(&G->split_items, sizeof(int32_t) * items.size()));
    HIP_CHECK(hipMemcpyAsync(G->split_items, items.data(), sizeof(int32_t) * items.size(), hipMemcpyHostToDevice,
                             stream));
  }
  HIP_CHECK(hipMalloc(&G->rp, sizeof(int64_t) * (n + 1)));
  HIP_CHECK(hipMalloc(&G->col, sizeof(int32_t) * std::max<int64_t>(1, G->m2)));
  HIP_CHECK(hipMalloc(&G->rev, sizeof(int64_t) * std::max<int64_t>(1, G->m2)));
  HIP_CHECK(hipMalloc(&G->orig, sizeof(int32_t) * n));
  HIP_CHECK(hipMalloc(&G->lowcnt, sizeof(int32_t) * n));
  HIP_CHECK(hipMalloc(&G->deg, sizeof(int32_t) * n));
  G->h_deg.resize(n);
  for (int64_t r = 0; r < n; r++) G->h_deg[r] = (int32_t)(G->h_rp[r + 1] - G->h_rp[r]);
  HIP_CHECK(hipMemcpyAsync(G->rp, G->h_rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, stream));
  if (G->m2) {
    HIP_CHECK(hipMemcpyAsync(G->col, G->h_col.data(), sizeof(int32_t) * G->m2, hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(G->rev, rev.data(), sizeof(int64_t) * G->m2, hipMemcpyHostToDevice, stream));
  }
  HIP_CHECK(hipMemcpyAsync(G->orig, G->h_orig.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
  HIP_CHECK(hipMemcpyAsync(G->lowcnt, G->h_lowcnt.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
  HIP_CHECK(hipMemcpyAsync(G->deg, G->h_deg.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
  HIP_CHECK(hipStreamSynchronize(stream));
  return G;
}

}  // namespace cc
