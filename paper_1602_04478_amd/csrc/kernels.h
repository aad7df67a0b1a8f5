// Launch wrappers for the device kernels (kernels.hip).  Host code only sees
// plain pointers and sizes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cc {

// Frontier program operations (see planner.cpp).
enum OpKind {
  OP_INIT = 0,   // dst[x] = A_h[u] (x) E(u,x), x a lower neighbour of u
  OP_NJ = 1,     // dst[v] = a[v] (x) A[v]                      (NodeJoin)
  OP_EJ = 2,     // dst[w] = sum_{v in N(w), v < u} a[v] (x) E(v,w)   (EdgeJoin)
  OP_AXPY = 3,   // dst += w * a   (dst fresh on its first AXPY)
  OP_MROOT = 4,  // count += w * sum_v a[v] (x) b[v], signatures covering all k colours
  OP_MU = 5,     // U[u]  += w * sum_v a[v] (x) b[v]
  OP_MV = 6,     // U[v]  += w * a[v] (x) b[v]
  OP_MEDGE = 7,  // T[x,y] += w * a[x] (x) E(x,y) (x) b[y]
  OP_MEDGE_T = 8, // T[u,y] += w * A[u] (x) E(u,y) (x) b[y]   (or T[y,u] when swapped)
  OP_MPAIR = 9   // P[u,v] += w * a[v] (x) b[v]               (pair-keyed table, u the source)
};

// The entries of one path length (depth) for a group: the (vertex, source)
// pairs reachable by a high-starting walk of that length.  In dense mode the
// entry of (v, b) is v * B + b for every v < n_lim; in sparse mode entries are
// listed (v * 64 + b) and idx maps (v, b) to its entry or -1.
struct LevelDev {
  uint64_t *mb;     // [n_lim][2]: marks (bit b: (v, b) is an entry), then the index of v's first
                    // entry (entries numbered in (v, b) order) -- one 16-byte load per vertex
  int64_t *list;    // [entries] v * 64 + b
  uint32_t *cnt;    // [0] number of entries, [1] number of marked vertices
  uint32_t *bcnt;   // [2][chunks] compaction scratch: entries, then marked vertices, per chunk
  int32_t *vlist;   // the marked vertices, ascending (cnt[1] of them)
};

// A frontier register: one row of T * C slots per entry of its level.
struct RegDev {
  uint64_t *val;
  uint64_t *mask;  // dense groups: per vertex, bit b set when row (v, b) may be nonzero
  int C;           // slots per (entry, trial)
  int s;           // signature size
};

// The group being processed.
// EdgeJoin work counters (profiling): PROF_LANES triples summed by the host
constexpr int PROF_LANES = 64;

struct GroupDev {
  const int32_t *src;  // source ranks, [B]
  int B;
  int T;
  int k;
  int64_t n_lim;      // every frontier vertex is below this rank
  int dense;          // 1: domain = all (v, b) with v < n_lim; 0: the register's list
  int nofilter;       // 1: path vertices are not required to lie below their source (path splitting)
  uint64_t *prof;     // optional work counters of the launch (profiling)
  // Dense EdgeJoin hub schedule: output vertices of rank >= split_lo (below
  // n_lim) have their neighbour lists cut into chunks of split_chunk
  // neighbours, one work item each (hitems: (vertex, first neighbour offset)
  // pairs, nh of them, heaviest first); the others are one item per vertex.
  // nh = 0: no split.
  const int32_t *hitems;
  int nh;
  int split_chunk;
  int64_t split_lo;
};

struct GraphDev {
  const int64_t *rp;
  const int32_t *col;
  const int64_t *rev;
  int64_t n;
  int64_t m2;
};

// Tables of child blocks.
struct TabDev {
  const uint64_t *val;  // unary: [x][t][slot]; edge: [slot e][t][slot]
  int C;
  int s;
};

// Per-launch outputs / accumulators.
struct AccDev {
  uint64_t *sum;       // per trial: lo, hi (2 x u64)
  uint32_t *ovf;       // per trial overflow flag
  uint64_t *per_src;   // optional [n][T] x (lo, hi) by rank, or null
};

// Row-local ops fused after a vertex-major EdgeJoin: they run on the rows of
// the output vertex while its EdgeJoin row is still in LDS.  Operands are
// registers of the epilogue: register 0 is the EdgeJoin's output; a register
// with an LDS block lives in LDS (and is written out when `write` is set); a
// register without one is read from global memory at its own level.
enum EpiKind { EPI_NJ = 0, EPI_AXPY = 1, EPI_MROOT = 2 };
constexpr int EPI_MAX_OPS = 8, EPI_MAX_REGS = 8;
struct EpiReg {
  RegDev r;        // global storage (val unused for an LDS-only register)
  LevelDev L;      // its level (rows are found there when read from global memory)
  int col;         // first LDS column of its block, or -1
  int write;       // 1: written to r at the end of the vertex
};
struct EpiOp {
  int kind, dst, a, b;  // register indices (dst unused for MROOT)
  TabDev nt;            // NodeJoin's node table
  uint64_t w;           // AXPY / MROOT weight
  int first;            // AXPY: dst starts at zero
};
struct Epilogue {
  int nops, nregs, ncols;
  EpiOp ops[EPI_MAX_OPS];
  EpiReg regs[EPI_MAX_REGS];
  // a second EdgeJoin on the same scan (packed launches only): input in2 at
  // the same level as the first input, output regs[1], slot map map2
  RegDev in2;
  const uint32_t *map2;
  int map2_w, map2_cp;
  // annotated EdgeJoins with one trial: 1 = a pair's output slots spread
  // over the lanes, 0 = one source per lane (set by the launch)
  int ann_lanes;
};

const uint16_t *lut_device(int device);
// Bytes of the constant-table pool (static device memory) on the current
// device, 256-byte aligned; null when the pool is full or the lookup fails.
void *table_pool_alloc(size_t bytes);
// copy host -> device on a private non-blocking stream and wait (one-time table uploads)
bool upload_sync(void *d, const void *h, size_t bytes);
// trials x slots of one frontier row: EdgeJoin keeps two accumulator words per
// slot in LDS, within 64 KiB per workgroup with its rank tables
inline int max_row_slots() { return 3584; }

void launch_colour(const int32_t *orig, int64_t n, int k, uint64_t seed, int t0, int T, uint8_t *out,
                   hipStream_t st);
// param = {seed, first trial} in device memory
void launch_colour_dev(const int32_t *orig, int64_t n, int k, const uint64_t *param, int T, uint8_t *out,
                       hipStream_t st);
void launch_copy16(const void *a, void *b, int64_t n16, hipStream_t st);  // n16 16-byte words
void launch_permute_colours(const uint8_t *by_orig, const int32_t *orig, int64_t n, int T, uint8_t *out,
                            hipStream_t st);
void launch_fill_u8(uint8_t *p, int64_t n, hipStream_t st, uint8_t x = 0);
void launch_fill_u64(uint64_t *p, int64_t n, hipStream_t st);

// grouped path (heavy.hip)
void launch_level_init(const GraphDev &g, const GroupDev &grp, const int32_t *lowcnt, int max_low, LevelDev L,
                       hipStream_t st);
void launch_level_next(const GraphDev &g, const GroupDev &grp, LevelDev Lin, LevelDev Lout, hipStream_t st);
void launch_level_compact(const GroupDev &grp, LevelDev L, hipStream_t st);
void launch_level_reset(const GroupDev &grp, LevelDev L, hipStream_t st);
int64_t level_chunks(int64_t n_lim);  // size of LevelDev::bcnt
void launch_init(const GraphDev &g, const GroupDev &grp, const int32_t *lowcnt, int max_low, const uint8_t *colr,
                 LevelDev L, RegDev dst, TabDev etab, int e_src_first, TabDev ntab, uint32_t *ovf, hipStream_t st);
void launch_ej(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev Lin, LevelDev Lout, RegDev a,
               RegDev dst, TabDev etab, int e_src_first, uint32_t *ovf, hipStream_t st);
// Two data-edge EdgeJoins a1 -> d1 and a2 -> d2 whose inputs share a level, in
// one packed launch over one neighbour scan (one colouring); false when that
// launch does not apply (then nothing was launched)
bool launch_ej_dual(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev Lin, LevelDev Lout,
                    RegDev a1, RegDev d1, RegDev a2, RegDev d2, uint32_t *ovf, hipStream_t st);
// EdgeJoin with a fused epilogue (vertex-major kernel only; see epi_fits)
void launch_ej_epi(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev Lin, RegDev a,
                   const Epilogue &epi, TabDev etab, int e_src_first, uint32_t *ovf, AccDev acc, hipStream_t st);
bool epi_fits(int ncols, int T, int etab_C);
// build (once per device and k) the EdgeJoin slot maps the vertex-major kernel
// reads instead of the slot arithmetic; false on a device error
bool ejmaps_prepare(int k);
void launch_nj(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev L, RegDev a, RegDev dst,
               TabDev ntab, uint32_t *ovf, hipStream_t st);
void launch_axpy(const GroupDev &grp, LevelDev L, RegDev a, RegDev dst, uint64_t w, int first, uint32_t *ovf,
                 hipStream_t st);
void launch_fill_u64v(uint64_t *p, int64_t n, uint64_t x, hipStream_t st);
// dst = sum over q < nterms (<= 4) of w[q] * term q, rows of level L (one pass for an AXPY chain);
// term q is a[q], or NodeJoin(a[q], nt[q]) when nt && nt[q].val (that NodeJoin's output is not stored)
void launch_axpyn(const GroupDev &grp, int64_t n, const uint8_t *colr, LevelDev L, const RegDev *a,
                  const TabDev *nt, const uint64_t *w, int nterms, RegDev dst, uint32_t *ovf, hipStream_t st);
void launch_mroot(const GroupDev &grp, int64_t n, const uint8_t *colr, LevelDev La, LevelDev Lb, RegDev a, RegDev b,
                  uint64_t w, AccDev acc, hipStream_t st);
// root merge whose first operand is an AXPY chain (terms as launch_axpyn's;
// the chain's signature size sa, slots Ca) computed in the pass; false (nothing
// launched) when a NodeJoin term has no split map or the chain does not fit
bool launch_mroot_terms(const GroupDev &grp, int64_t n, const uint8_t *colr, LevelDev La, LevelDev Lb,
                        const RegDev *a, const TabDev *nt, const uint64_t *wq, int nterms, int Ca, int sa, RegDev b,
                        uint64_t w, AccDev acc, hipStream_t st);
void launch_munary(const GroupDev &grp, int64_t n, const uint8_t *colr, LevelDev La, LevelDev Lb, RegDev a,
                   RegDev b, uint64_t w, int at_u, uint64_t *out, int s_out, int C_out, uint32_t *ovf, hipStream_t st);
void launch_medge(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev La, LevelDev Lb, RegDev a,
                  RegDev b, TabDev etab, int e_src_first, int out_first_is_x, uint64_t w, uint64_t *out, int s_out,
                  int C_out, uint32_t *ovf, hipStream_t st);
void launch_medge_t(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, const int32_t *lowcnt,
                    int max_low, TabDev ntab, LevelDev Lb, RegDev b, TabDev etab, int e_src_first,
                    int out_first_is_u, uint64_t w, uint64_t *out, int s_out, int C_out, uint32_t *ovf,
                    hipStream_t st);
// pair-keyed merge (dense groups): rows of P[(u_b, v)] staged in `stage`
// (rows v * B + b, activity words), the nonzero ones appended to the entry
// list (keys (u, v), values [T][C]) through the counter cnt (capacity cap)
void launch_mpair(const GroupDev &grp, int64_t n, const uint8_t *colr, RegDev a, RegDev b, uint64_t w, RegDev stage,
                  int32_t *keys, uint64_t *vals, uint64_t cap, unsigned long long *cnt, uint32_t *ovf,
                  hipStream_t st);
// table rows aligned to a pair graph's slots: slot e <- entry idx[e] (or zeros when -1)
void launch_pair_gather(const int64_t *idx, int64_t m2, const uint64_t *vals, int64_t per, uint64_t *tab,
                        hipStream_t st);
void launch_leaf(const GraphDev &g, int T, int k, const uint8_t *colr, TabDev na, TabDev ea, int e_src_first,
                 TabDev nb, uint64_t *out, int s_out, int C_out, uint32_t *ovf, hipStream_t st);
void launch_root_single(int64_t n, int T, TabDev u, AccDev acc, hipStream_t st);

// ------------------------------------------------------------------ one workgroup per source
struct LOp {
  int kind, dst, a, b, tab, tab_src_first, ntab, s, first, swapped;
  uint64_t w;
};

struct LightArgs {
  GraphDev g;
  const int32_t *lowcnt;  // lower neighbours per vertex (the degree with nofilter)
  int nofilter;           // 1: path vertices need not lie below the source
  const uint8_t *colr;
  int T, k;
  const int32_t *src;   // candidate sources (ranks)
  int nsrc;
  uint32_t *next;       // work counter (zero before launch)
  int32_t *fail;        // sources handed back
  uint32_t *nfail;
  const LOp *ops;
  int nops;
  const int32_t *reg_depth, *reg_C, *reg_s;
  int nregs, D;
  const TabDev *tabs;   // per block id (null val: no table)
  uint64_t *out;        // the block's output table (non-root)
  int s_out, C_out;
  AccDev acc;
  uint8_t *scratch;
  int64_t scratch_per_wg;
  const uint16_t *lut;
  uint64_t *prof;       // profiling: PROF_LANES (read, written, 0) byte triples, or null
};

int light_max_depth();
int light_max_regs();
// large: the variant with the big LDS key pool (one workgroup per compute unit)
void launch_light(const LightArgs &a, int grid, bool large, hipStream_t st);

}  // namespace cc
