// engine.hpp -- batched Kuhn-Munkres on one workgroup (gfx950).
//
// Method: "Batched KM" (Section 2.3.1 of the paper).  Alternating trees grow
// from every free row at once inside the tight-edge subgraph; every
// vertex-disjoint augmenting path found is applied (one per tree that reached
// a free column); when no tree can grow and none has reached a free column,
// the duals move across the cut (reached rows up, reached columns down) by
// the smallest slack, exactly as in KM.  The loop stops when every row is
// matched.
//
// Organisation on the device (one workgroup = one instance):
//   * Column j is owned by thread j % BLOCK (CPT columns per thread, strided
//     so that a cost-row read is one coalesced sweep across the workgroup).
//     The owner keeps in registers: its dual v_j, the level at which the
//     column was reached, and the column's two smallest reduced costs from
//     distinct trees ("top-2 keys", each packed as value << 24 | row).
//   * Row state lives in LDS: match arrays, the tree a row belongs to, the
//     forest row list, and h_i = u_i - D_i (the row dual relative to the
//     level D_i at which the row joined; non-forest rows store u_i).  Dual
//     changes across the cut are therefore lazy: raising every reached row by
//     delta is just raising the running level D (Dijkstra-style potentials),
//     and a key stores reduced cost + D, which stays valid while the forest
//     grows.
//   * When a tree augments, its rows and columns leave the forest and their
//     duals are materialised.  A column whose best key came from a dead tree
//     falls back to its second key (best from another tree); keys that are
//     still unknown are kept as lower bounds ("stale") and recomputed
//     ("gathered") only when they could be the next minimum.  This avoids
//     re-reading the whole forest after every augmentation.
//   * Workgroup minima use DPP row rotations inside a wavefront and one LDS
//     atomic per wavefront; the level loop needs two barriers per level.
//
// Integer ranges (int32 costs with max - min = R <= 2^31 - 1): u only rises,
// v only falls, free columns keep v >= 0, so u_i <= max C and v_j >= -R; a
// reduced cost is in [0, 2R] and the running level D is at most R.  A key
// value (reduced cost + D) is therefore below 3 * 2^31 < 2^40 and fits with a
// 24-bit row index in 64 bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "otkm.h"

namespace otkm {

constexpr int kRowBits = 24;
constexpr uint64_t kRowMask = (1ull << kRowBits) - 1;
constexpr uint64_t kInf = ~0ull;
constexpr int kNoEnd = 0x7fffffff;

// int control words in LDS
enum Ctl { CNT0 = 0, CNT1 = 1, NAUG = 2, GCNT = 3, ERR = 4, FCNT = 5, ERRA0 = 6, ERRA1 = 7, ERRB0 = 8, ERRB1 = 9,
           GAB = 10, LCNT = 11, NCTL = 12 };

// Global state of one instance spread over G <= kMaxWgs workgroups, in 64-bit
// words (all zero before the launch): barrier arrivals and abort flag; per
// slot set and workgroup the local minimum pair and a tag word (level << 32 |
// error); per workgroup gathers and final error; then per level parity and
// workgroup a list of settled columns: a tag word (level << 32 | count) and at
// most `per` (columns owned by a workgroup) entries.
constexpr int kMaxWgs = 16;
constexpr int kGBar = 0, kGAbort = 1, kGMin = 2, kGGath = kGMin + 4 * kMaxWgs * 3, kGFin = kGGath + kMaxWgs,
              kGList = 256;
static_assert(kGFin + kMaxWgs <= kGList, "grid state header overlaps the lists");
__host__ __device__ inline size_t grid_ws_u64(int G, int per) { return kGList + 2 * (size_t)G * (size_t)(per + 1); }

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }
__host__ __device__ inline int gather_cap(int n) { return n / 16 < 32 ? 32 : n / 16; }

struct LdsLayout {
  size_t hrow, mrow, mcol, rtree, par, fst, fr, alive, gcol, gv, gk1, gk2, gt1, gt2, red, ctl, total;
};

// Byte offsets of every LDS array for an instance of size n (host and device).
// grid: the engine runs one instance over several workgroups, whose settle
// exchange stages the other workgroups' entries in red (128 words instead of 80).
__host__ __device__ inline LdsLayout lds_layout(int n, bool grid = false) {
  LdsLayout L;
  const size_t N = (size_t)n, G = (size_t)gather_cap(n);
  size_t o = 0;
  L.hrow = o;  o = align16(o + 8 * N);
  L.mrow = o;  o = align16(o + 4 * N);
  L.mcol = o;  o = align16(o + 4 * N);
  L.rtree = o; o = align16(o + 4 * N);
  L.par = o;   o = align16(o + 2 * N);  // 16-bit row ids (n <= OT_MAX_N)
  L.fst = o;   o = align16(o + 4 * N);
  L.fr = o;    o = align16(o + 8 * N);
  L.alive = o; o = align16(o + N);
  L.gcol = o;  o = align16(o + 4 * G);
  L.gv = o;    o = align16(o + 8 * G);
  L.gk1 = o;   o = align16(o + 8 * G);
  L.gk2 = o;   o = align16(o + 8 * G);
  L.gt1 = o;   o = align16(o + 4 * G);
  L.gt2 = o;   o = align16(o + 4 * G);
  // slots [0, 8), per-wave words [16, 32), refresh partials [32, 32 + 3 NW);
  // the grid exchange: [16, 112) entries, [112, 121) counts
  L.red = o;   o = align16(o + 8 * (grid ? 128 : 80));
  L.ctl = o;   o = align16(o + 4 * NCTL);
  L.total = o;
  return L;
}

// Global scratch per workgroup: list of trees that augment this step and the
// smallest free column reached per tree (both touched only at augmentations).
__host__ __device__ inline size_t ws_ints(int n) { return 2 * (size_t)n; }

struct Problem {
  const int32_t *C;   // nr x n (rows x columns), row stride ld
  int n, ld;
  int nr = 0;         // rows, 1 <= nr <= n; 0 = n (square).  With nr < n every row is matched and
                      // the column duals start at 0 (no column reduction), so they end <= 0 and
                      // exactly 0 on the columns left unmatched: the rectangular LP's dual
  const int32_t *CT;  // transpose of C (n x nr, row stride ldt), or null; only read to refresh single columns
  int ldt = 0;        // row stride of CT; 0 = nr
  const int32_t *Cout;  // costs the reported total is taken over (row stride ldo), or null for C
  int ldo;
  int dscale;         // reported duals are dscale * (duals of C); 1 unless C holds scaled-down costs
  // Optional results of the grid-wide initial sweeps (k_init_rows / k_init_cols /
  // k_init_merge), or null to run them inside the workgroup:
  const int64_t *init_u;     // [nr] row minima u_i = min_j C_ij
  const uint64_t *init_b;    // [n][2] per column the two smallest keys pack(C_ij - u_i, i)
  const int32_t *init_rmax;  // [nr] row maxima (with the row minima: the cost range)

  int max_paths;      // 0 = all free rows
  int flags;          // OT_FLAG_* bits
  int32_t *plan;      // [nr]
  int64_t *cost;      // [1]
  int64_t *u, *v;     // [nr], [n] or null
  ot_stats *stats;    // [1] or null
  int32_t *ws;        // [ws_ints(n)] per workgroup
  uint64_t *grid_ws = nullptr;  // several workgroups per instance: [grid_ws_u64(G, per)], zeroed
};

__device__ __forceinline__ uint64_t pack(int64_t val, int row) {
  return ((uint64_t)val << kRowBits) | (uint32_t)row;
}
__device__ __forceinline__ int64_t kval(uint64_t k) { return (int64_t)(k >> kRowBits); }
__device__ __forceinline__ int krow(uint64_t k) { return (int)(k & kRowMask); }

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return b < a ? b : a; }

template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t x) {
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)x, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(x >> 32), CTRL, 0xf, 0xf, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ uint64_t readlane64(uint64_t x, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// Minimum over a full wavefront (all 64 lanes active): rotations inside each
// 16-lane row, then the four row results through scalar reads.  The result is
// wave-uniform.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
  x = umin64(x, dpp64<0x121>(x));  // row_ror:1
  x = umin64(x, dpp64<0x122>(x));  // row_ror:2
  x = umin64(x, dpp64<0x124>(x));  // row_ror:4
  x = umin64(x, dpp64<0x128>(x));  // row_ror:8
  return umin64(umin64(readlane64(x, 0), readlane64(x, 16)), umin64(readlane64(x, 32), readlane64(x, 48)));
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
  // the rotations read inside each 16-lane row, so no lane keeps the old
  // value (the identity); passing it lets the compiler fold each move into
  // the minimum (v_min_u32 with a DPP operand)
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x121, 0xf, 0xf, false));  // row_ror:1
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x122, 0xf, 0xf, false));  // row_ror:2
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x124, 0xf, 0xf, false));  // row_ror:4
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x128, 0xf, 0xf, false));  // row_ror:8
  const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 0), r1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 16);
  const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 32), r3 = (uint32_t)__builtin_amdgcn_readlane((int)x, 48);
  return min(min(r0, r1), min(r2, r3));
}
__device__ __forceinline__ int wave_min_i32(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off, 64));
  return x;
}
__device__ __forceinline__ int wave_max_i32(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Insert candidate c (from a row of tree t >= 0) into a column's top-2:
// a1 = best key overall (tree ta1), a2 = best key among trees != ta1.
template <class K>
__device__ __forceinline__ void top2_push(K &a1, int &ta1, K &a2, int &ta2, K c, int t) {
  // same tree as the best: only the best can improve; another tree: c may
  // become the best (the old best moves to second) or the second.  a1 <= a2,
  // so c < a1 implies c < a2 and the second changes exactly when c is from
  // another tree and below a2.  Flat selects only (no divergent branches).
  const bool same = t == ta1, lt1 = c < a1, lt2 = c < a2;
  const bool ch2 = !same && lt2;
  const K x = lt1 ? a1 : c;
  const int tx = lt1 ? ta1 : t;
  a2 = ch2 ? x : a2;
  ta2 = ch2 ? tx : ta2;
  a1 = lt1 ? c : a1;
  ta1 = lt1 ? t : ta1;
}

// Merge two exact top-2 summaries (symmetric, so both butterfly partners agree).
template <class K>
__device__ __forceinline__ void top2_merge(K &a1, int &ta1, K &a2, int &ta2, K b1, int tb1, K b2, int tb2) {
  if (b1 < a1) {
    K x1 = a1, x2 = a2; int y1 = ta1, y2 = ta2;
    a1 = b1; ta1 = tb1; a2 = b2; ta2 = tb2;
    b1 = x1; tb1 = y1; b2 = x2; tb2 = y2;
  }
  K c = (tb1 != ta1) ? b1 : b2;
  int tc = (tb1 != ta1) ? tb1 : tb2;
  if (c < a2) { a2 = c; ta2 = tc; }
}

__device__ __forceinline__ int64_t now_ticks() { return (int64_t)wall_clock64(); }

// LONG: also sweep long frontiers in chunks of 2U rows (more registers; used by
// the one-instance kernel, where occupancy does not matter).
// RECT: the rows may be fewer than the columns (Problem::nr); the batched
// kernel is square and keeps n in their place.
// Column keys are value << bits | row.  Wide keys (64-bit, 24 row bits) hold
// every value the method reaches with int32 costs.  Compact keys (32-bit, 12
// row bits, n <= 4096) hold values below 2^20, which is enough when the cost
// range R is below 2^18: a key value is at most 3R (a reduced cost in
// [0, 2R] plus a level in [0, R]), as long as every free row is a root (with
// a tree cap the level adds up over stages).  Compact keys halve the
// instructions of every key comparison and selection.
template <bool COMPACT>
struct KeyOf {
  using T = uint64_t;
  static constexpr int kBits = kRowBits;
};
template <>
struct KeyOf<true> {
  using T = uint32_t;
  static constexpr int kBits = 12;
};
constexpr int64_t kCompactRange = 1 << 18;  // cost ranges below this use compact keys
constexpr int kCompactMaxN = 1 << 12;

// GRID: one instance over gridDim.x workgroups.  Rows, matches and the forest
// are replicated in every workgroup's LDS and updated identically; the columns
// (keys in registers) are split.  Per level the workgroups exchange their
// minimum keys and the columns they settled through global memory, with a
// grid barrier after each.
template <int BLOCK, int CPT, bool LONG = false, bool GRID = false, bool RECT = false, bool COMPACT = false>
struct Engine {
  static constexpr int NW = BLOCK / 64;
  using Key = typename KeyOf<COMPACT>::T;
  static constexpr int KB = KeyOf<COMPACT>::kBits;
  static constexpr Key KINF = (Key)~(Key)0;
  static __device__ __forceinline__ Key kpack(int64_t val, int row) { return ((Key)val << KB) | (Key)(uint32_t)row; }
  static __device__ __forceinline__ int64_t kv(Key k) { return (int64_t)(k >> KB); }
  static __device__ __forceinline__ int kr(Key k) { return (int)(k & (((Key)1 << KB) - 1)); }

  // problem
  const int32_t *__restrict__ C;
  const int32_t *__restrict__ CT;
  int n, ld;
  int nr_;   // RECT: rows (n columns)
  int ldt;   // row stride of CT
  // rows: n unless RECT (the batched kernel is square and saves the register)
  __device__ __forceinline__ int rows() const {
    if constexpr (RECT) return nr_;
    else return n;
  }
  // LDS
  int64_t *hrow;
  int32_t *mrow, *mcol, *rtree, *fst, *gcol, *gt1, *gt2, *ctl;
  int16_t *par;  // parent row of each reached column
  int2 *fr;  // frontier records of the next sweep: (row | tree << 16, low 32 bits of h)
  uint8_t *alive;
  int64_t *gv;
  uint64_t *gk1, *gk2, *red;
  int gcap;
  // global scratch
  int32_t *auglist, *bend;
  // buffer resource over C and the byte offset of every owned column (clamped
  // to the last column) for the narrow sweep's loads
  __amdgpu_buffer_rsrc_t crsrc;
  int voff[CPT];
  // per-column registers
  Key k1[CPT], k2[CPT];
  int t1[CPT], t2[CPT], ctree[CPT];
  // v_j lies in [-R, R] and the level at which a column is reached in [0, R]
  // (R = max C - min C < 2^31), so both fit 32 bits.
  int32_t vj[CPT], dcol[CPT];
  bool narrow;          // cost range below 2^30
  uint32_t vis;   // bit k: column k has been reached (is in a tree)
  uint32_t stl;   // bit k: k1 is only a lower bound (its tree is gone)
  int tid, lane, wid;
  int err_local;  // this thread's first error (0 = none); reduced at every level
  // GRID
  int G, g, epoch;
  uint32_t lev;  // current level, the tag of this level's exchanges (from 1)
  uint64_t *gws;

  __device__ __forceinline__ int col(int k) const {
    if constexpr (GRID) return tid + g * BLOCK + k * BLOCK * G;
    else return tid + k * BLOCK;
  }
  // Always-valid column for loads: loads are issued unconditionally (a guarded
  // load becomes a branch plus a full wait for memory), values of columns past
  // n are ignored afterwards.
  __device__ __forceinline__ int lcol(int k) const { return col(k) < n ? col(k) : n - 1; }
  __device__ __forceinline__ bool stale(int k) const { return (stl >> k) & 1u; }
  __device__ __forceinline__ void fail(int code) { if (err_local == 0) err_local = code; }

  // exact iff the best key's tree is still alive (or there is no candidate at all)
  __device__ __forceinline__ void recompute_stale(int k) {
    const bool ok = k1[k] == KINF || (t1[k] >= 0 && alive[t1[k]]);
    if (ok) stl &= ~(1u << k); else stl |= 1u << k;
  }

  // Fold cost rows list[0..cnt) (forest rows; rows no longer in the forest
  // are skipped) into every owned column's top-2 keys.  Rows go in chunks of U
  // whose loads are all issued before any is used, so a short frontier costs
  // one memory latency.  With NARROW (cost range below 2^30) every key value
  // is below 2^32, so reduced costs are formed in 32-bit modular arithmetic
  // (exact there) and each chunk is reduced to its own top-2 per column before
  // one merge.  Returns rows used.
  // Rows per chunk, measured on MI355X (geometric n = 512..4096): U * CPT = 8
  // loads per lane (two rows at 4 columns per lane) beat 16 and 4 on the short
  // frontiers that dominate; on long frontiers the next chunk's loads are
  // issued before the current chunk is folded.
  static constexpr int U = CPT >= 8 ? 2 : 8 / CPT;  // U * CPT <= 32 pass bits
  static constexpr int GU = 8;  // forest rows in flight per lane when recomputing a stale column
  // One chunk of UU rows list[f .. f+UU) (slots past cnt are skipped).  REC:
  // list holds frontier records (row, tree and the low word of h, written when
  // the row joined, so no dependent LDS read of rtree / hrow is needed in the
  // narrow case); otherwise plain row ids.
  // Narrow cost range: one chunk of up to UN rows, all of its loads in flight
  // at once.  A row's record is the same for every lane, so the row, its tree
  // and -h live in scalar registers: a cost row is a buffer load with the row
  // offset in the scalar offset, and a reduced cost is one three-operand add,
  // exact in 32-bit modular arithmetic because every key value is below 2^32
  // here.  The chunk is reduced per column to its own top-2 (best, then best
  // from another tree) on 32-bit values with the row and tree beside them
  // (ties keep the earlier row), and merged once into the column's keys.
  static constexpr int UN = CPT >= 8 ? 4 : (CPT >= 4 ? 8 : 16);
  template <int S, bool REC>
  __device__ __forceinline__ int sweep_chunk_narrow(const int32_t *list, int f, int cnt) {
    constexpr int UN = S;
    const int nv = min(UN, cnt - f);  // uniform
    uint32_t id[UN], nh[UN];
    int soff[UN];
    bool live[UN];
    int32_t c[UN][CPT];
    int used = 0, first = -1;
#pragma unroll
    for (int q = 0; q < UN; ++q) {
      live[q] = false; id[q] = 0; nh[q] = 0; soff[q] = 0;
      if (q >= nv) continue;
      int row, tr;
      uint32_t h32;
      if (REC) {
        const int2 e = ((const int2 *)list)[f + q];
        row = __builtin_amdgcn_readfirstlane(e.x & 0xffff);
        tr = __builtin_amdgcn_readfirstlane(e.x >> 16);  // negative: the row's tree has gone
        h32 = (uint32_t)__builtin_amdgcn_readfirstlane(e.y);
      } else {
        row = __builtin_amdgcn_readfirstlane(list[f + q]);
        if ((unsigned)row >= (unsigned)rows()) row = 0;
        tr = __builtin_amdgcn_readfirstlane(rtree[row]);
        h32 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)hrow[row]);
      }
      if ((unsigned)row >= (unsigned)rows()) { fail(OT_EINTERNAL); row = 0; tr = -1; }
      live[q] = tr >= 0;
      used += live[q];
      if (live[q] && first < 0) first = q;
      id[q] = ((uint32_t)row << 16) | (uint32_t)tr;  // rows are distinct: ids order as rows
      nh[q] = 0u - h32;
      soff[q] = row * ld * 4;
    }
    if (first < 0) return 0;  // every row of the chunk left the forest
    // A slot without a live row repeats the first live one: a duplicate of a
    // candidate changes neither the best nor the best from another tree, so
    // the reduction below needs no per-slot predicate.
#pragma unroll
    for (int q = 0; q < UN; ++q) {
      if (!live[q]) { id[q] = id[first]; nh[q] = nh[first]; soff[q] = soff[first]; }
#pragma unroll
      for (int k = 0; k < CPT; ++k)
        c[q][k] = __builtin_amdgcn_raw_buffer_load_b32(crsrc, voff[k], __builtin_amdgcn_readfirstlane(soff[q]), 0);
    }
    uint32_t clr = 0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const uint32_t nvj = 0u - (uint32_t)vj[k];
      uint32_t v[UN];
      uint32_t b1 = ~0u, b2 = ~0u, i1 = ~0u, i2 = ~0u;
#pragma unroll
      for (int q = 0; q < UN; ++q) {
        // (value, row) order, as the packed keys: the result does not depend on
        // the order of the rows in the chunk, or on how a sweep is chunked
        v[q] = (uint32_t)c[q][k] + nh[q] + nvj;
        const bool lt = (v[q] < b1) | ((v[q] == b1) & (id[q] < i1));
        b1 = lt ? v[q] : b1;
        i1 = lt ? id[q] : i1;
      }
      const uint32_t ti1 = i1 & 0xffffu;
#pragma unroll
      for (int q = 0; q < UN; ++q) {
        const bool ok = ((id[q] & 0xffffu) != ti1) & ((v[q] < b2) | ((v[q] == b2) & (id[q] < i2)));
        b2 = ok ? v[q] : b2;
        i2 = ok ? id[q] : i2;
      }
      // merge (b1, b2) into (k1, k2): the smaller best wins, and the second is
      // the better of the loser's best (when it is from another tree) or its
      // second, and the winner's second
      const uint64_t c1 = b1 == ~0u ? kInf : (((uint64_t)b1 << kRowBits) | (i1 >> 16));
      const uint64_t c2 = b2 == ~0u ? kInf : (((uint64_t)b2 << kRowBits) | (i2 >> 16));
      const int tb1 = b1 == ~0u ? -1 : (int)(i1 & 0xffffu), tb2 = b2 == ~0u ? -1 : (int)(i2 & 0xffffu);
      const bool sw = c1 < k1[k];
      const uint64_t x1 = sw ? c1 : k1[k], x2 = sw ? c2 : k2[k];
      const int tx1 = sw ? tb1 : t1[k], tx2 = sw ? tb2 : t2[k];
      const uint64_t y1 = sw ? k1[k] : c1, y2 = sw ? k2[k] : c2;
      const int ty1 = sw ? t1[k] : tb1, ty2 = sw ? t2[k] : tb2;
      const bool d = ty1 != tx1;
      const uint64_t cc = d ? y1 : y2;
      const int tc = d ? ty1 : ty2;
      const bool lt = cc < x2;
      k1[k] = x1; t1[k] = tx1;
      k2[k] = lt ? cc : x2; t2[k] = lt ? tc : tx2;
      clr |= sw ? (1u << k) : 0u;  // best key now from a live tree
    }
    stl &= ~clr;
    return used;
  }

  // The last rows of a sweep go in the smallest chunk that holds them.
  template <int S, bool REC>
  __device__ __forceinline__ int sweep_narrow_tail(const int32_t *list, int f, int cnt) {
    if constexpr (S > 1) {
      if (cnt - f <= S / 2) return sweep_narrow_tail<S / 2, REC>(list, f, cnt);
    }
    return sweep_chunk_narrow<S, REC>(list, f, cnt);
  }

  // One chunk's rows, trees, row duals and cost entries (the loads of the
  // entries may still be in flight).
  template <int UU>
  struct Chunk {
    int r[UU], t[UU];
    int64_t h[UU];
    uint32_t h32[UU];
    int32_t c[UU][CPT];
  };

  // Read chunk list[f .. f+UU) (slots past cnt are skipped) and issue its
  // cost loads; nothing here waits for them.
  template <bool NARROW, int UU, bool REC>
  __device__ __forceinline__ void chunk_load(const int32_t *list, int f, int cnt, Chunk<UU> &X) {
#pragma unroll
    for (int q = 0; q < UU; ++q) {
      if (REC) {
        const int2 e = ((const int2 *)list)[f + q < cnt ? f + q : cnt - 1];
        X.r[q] = e.x & 0xffff;
        if ((unsigned)X.r[q] >= (unsigned)rows()) { fail(OT_EINTERNAL); X.r[q] = 0; }
        X.t[q] = (f + q < cnt && e.x >= 0) ? (e.x >> 16) : -1;  // sign bit: the row's tree has gone
        X.h32[q] = (uint32_t)e.y;
        X.h[q] = NARROW ? 0 : hrow[X.r[q]];
      } else {
        X.r[q] = f + q < cnt ? list[f + q] : 0;
        if ((unsigned)X.r[q] >= (unsigned)rows()) { fail(OT_EINTERNAL); X.r[q] = 0; }
        X.t[q] = f + q < cnt ? rtree[X.r[q]] : -1;
        X.h[q] = hrow[X.r[q]];
        X.h32[q] = (uint32_t)X.h[q];
      }
    }
#pragma unroll
    for (int q = 0; q < UU; ++q) {
      const int32_t *row = C + (size_t)X.r[q] * (size_t)ld;
#pragma unroll
      for (int k = 0; k < CPT; ++k) X.c[q][k] = row[lcol(k)];
    }
  }

  // Merge a chunk's top-2 (b1, tb1, b2, tb2) into column k's (k1, t1, k2,
  // t2): the smaller best wins, and the second is the better of the loser's
  // best (when it is from another tree) or its second, and the winner's
  // second.  Returns whether the best changed (it is then from a live tree).
  __device__ __forceinline__ bool merge_top2(int k, Key b1, int tb1, Key b2, int tb2) {
    const bool sw = b1 < k1[k];
    const Key x1 = sw ? b1 : k1[k], x2 = sw ? b2 : k2[k];
    const int tx1 = sw ? tb1 : t1[k], tx2 = sw ? tb2 : t2[k];
    const Key y1 = sw ? k1[k] : b1, y2 = sw ? k2[k] : b2;
    const int ty1 = sw ? t1[k] : tb1, ty2 = sw ? t2[k] : tb2;
    const bool d = ty1 != tx1;
    const Key cc = d ? y1 : y2;
    const int tc = d ? ty1 : ty2;
    const bool lt = cc < x2;
    k1[k] = x1; t1[k] = tx1;
    k2[k] = lt ? cc : x2; t2[k] = lt ? tc : tx2;
    return sw;
  }

  // Compact keys: each candidate of the chunk is one packed 32-bit key
  // (value << KB | row), so a column's best over the chunk is a chain of
  // minima, and the tree of the winner is read back from rtree (a live row
  // of the chunk is a forest row, and rtree holds the tree of its record).
  // The best from another tree is the minimum over the candidates whose
  // tree differs.  The columns go in phases so that the CPT tree reads of a
  // phase are in flight together.  The results equal the generic fold's.
  template <int UU>
  __device__ __forceinline__ int chunk_fold_compact(const Chunk<UU> &X) {
    int rs[UU], ts[UU];
    uint32_t nh[UU];
    int used = 0;
#pragma unroll
    for (int q = 0; q < UU; ++q) {
      rs[q] = __builtin_amdgcn_readfirstlane(X.r[q]);
      ts[q] = __builtin_amdgcn_readfirstlane(X.t[q]);
      nh[q] = 0u - (uint32_t)__builtin_amdgcn_readfirstlane((int)X.h32[q]);
      used += ts[q] >= 0;
    }
    if (used == 0) return 0;
    const int rmax = rows() - 1;
    Key kk[UU][CPT], b1[CPT], b2[CPT];
    int tb1[CPT], tb2[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const uint32_t nvj = 0u - (uint32_t)vj[k];
      Key m = KINF;
#pragma unroll
      for (int q = 0; q < UU; ++q) {
        // exact: every key value is below 2^20 with compact keys
        const uint32_t v = (uint32_t)X.c[q][k] + nh[q] + nvj;
        kk[q][k] = ts[q] >= 0 ? ((v << KB) | (uint32_t)rs[q]) : KINF;
        m = min(m, kk[q][k]);
      }
      b1[k] = m;
    }
    // the low bits of a live candidate are its row (clamped for lanes past n)
#pragma unroll
    for (int k = 0; k < CPT; ++k) tb1[k] = rtree[min(kr(b1[k]), rmax)];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      Key m = KINF;
#pragma unroll
      for (int q = 0; q < UU; ++q) m = min(m, ts[q] != tb1[k] ? kk[q][k] : KINF);
      b2[k] = m;
    }
#pragma unroll
    for (int k = 0; k < CPT; ++k) tb2[k] = rtree[min(kr(b2[k]), rmax)];
    uint32_t clr = 0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const bool in = col(k) < n;
      const Key c1 = in ? b1[k] : KINF, c2 = in ? b2[k] : KINF;
      const int u1 = in ? tb1[k] : -1, u2 = c2 == KINF ? -1 : tb2[k];
      clr |= merge_top2(k, c1, u1, c2, u2) ? (1u << k) : 0u;  // best key now from a live tree
    }
    stl &= ~clr;
    return used;
  }

  // Fold a loaded chunk into every owned column's top-2 keys; returns the rows used.
  template <bool NARROW, int UU>
  __device__ __forceinline__ int chunk_fold(const Chunk<UU> &X) {
    int used = 0;
    {
      constexpr int U = UU;
      const int *r = X.r, *t = X.t;
      const int64_t *h = X.h;
      const uint32_t *h32 = X.h32;
      const int32_t(*c)[CPT] = X.c;
#pragma unroll
      for (int q = 0; q < U; ++q) used += t[q] >= 0;
      if constexpr (COMPACT) return chunk_fold_compact<UU>(X);
      if (NARROW) {
        // Per column: the exact top-2 of this chunk's candidates (the best, then
        // the best from another tree), merged once into the column's top-2.
        // Select-only: a few lanes of a wavefront improve a key in a typical
        // chunk, and divergent branches cost more than they skip.
        uint32_t clr = 0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
          Key key[U];
          Key b1 = KINF, b2 = KINF;
          int tb1 = -1, tb2 = -1;
#pragma unroll
          for (int q = 0; q < U; ++q) {
            // exact: every key value is below 2^32 here, so 32-bit wrap-around cannot occur
            const uint32_t v = (uint32_t)c[q][k] - (h32[q] + (uint32_t)vj[k]);
            const bool ok = (t[q] >= 0) & (col(k) < n);
            key[q] = ok ? (((Key)v << KB) | (Key)(uint32_t)r[q]) : KINF;
            const bool lt = key[q] < b1;
            b1 = lt ? key[q] : b1;
            tb1 = lt ? t[q] : tb1;
          }
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const bool ok = (t[q] != tb1) & (key[q] < b2);
            b2 = ok ? key[q] : b2;
            tb2 = ok ? t[q] : tb2;
          }
          // merge (b1, tb1, b2, tb2) into (k1, t1, k2, t2): the smaller best
          // wins, and the second is the better of the loser's best (when it
          // is from another tree) or its second, and the winner's second
          const bool sw = b1 < k1[k];
          const Key x1 = sw ? b1 : k1[k], x2 = sw ? b2 : k2[k];
          const int tx1 = sw ? tb1 : t1[k], tx2 = sw ? tb2 : t2[k];
          const Key y1 = sw ? k1[k] : b1, y2 = sw ? k2[k] : b2;
          const int ty1 = sw ? t1[k] : tb1, ty2 = sw ? t2[k] : tb2;
          const bool d = ty1 != tx1;
          const Key cc = d ? y1 : y2;
          const int tc = d ? ty1 : ty2;
          const bool lt = cc < x2;
          k1[k] = x1; t1[k] = tx1;
          k2[k] = lt ? cc : x2; t2[k] = lt ? tc : tx2;
          clr |= sw ? (1u << k) : 0u;  // best key now from a live tree
        }
        stl &= ~clr;
        return used;
      }
      // Wide cost range: filter against the second key without branching,
      // then exact 64-bit updates on the (rare) slots where some lane passes.
      uint32_t pass = 0;
#pragma unroll
      for (int q = 0; q < U; ++q) {
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
          const int64_t v = (int64_t)c[q][k] - h[q] - vj[k];
          const bool p = v <= kv(k2[k]);
          pass |= (p & (t[q] >= 0) & (col(k) < n)) ? (1u << (q * CPT + k)) : 0u;
        }
      }
      // Slots nobody in the wavefront needs are skipped with one scalar branch.
      if (__builtin_amdgcn_ballot_w64(pass != 0) != 0) {
        uint32_t clr = 0;
#pragma unroll
        for (int q = 0; q < U; ++q) {
#pragma unroll
          for (int k = 0; k < CPT; ++k) {
            const bool p = (pass >> (q * CPT + k)) & 1u;
            if (__builtin_amdgcn_ballot_w64(p) == 0) continue;
            // Divergent from here on: typically a few lanes of the wavefront
            // take each branch, and a branch no lane takes is skipped whole.
            if (p) {
              int64_t val = (int64_t)c[q][k] - h[q] - vj[k];
              if (val < 0) { fail(OT_EINTERNAL); val = 0; }
              const Key key = kpack(val, r[q]);
              const int tq = t[q];
              if (key < k1[k]) {
                // new best; the old best stays second unless it is from the same tree
                if (tq != t1[k]) { k2[k] = k1[k]; t2[k] = t1[k]; }
                k1[k] = key; t1[k] = tq;
                clr |= 1u << k;  // best key now from a live tree
              } else if (tq != t1[k] && key < k2[k]) {
                k2[k] = key; t2[k] = tq;
              }
            }
          }
        }
        stl &= ~clr;
      }
    }
    return used;
  }


  template <bool NARROW, int UU, bool REC>
  __device__ __forceinline__ int sweep_chunk(const int32_t *list, int f, int cnt) {
    Chunk<UU> X;
    chunk_load<NARROW, UU, REC>(list, f, cnt, X);
    return chunk_fold<NARROW, UU>(X);
  }

  // Compact keys in the one-instance kernels: up to UL rows per chunk (the
  // packed-key fold costs little per row, so longer chunks spread each
  // column's merge over more rows); a frontier of at most UL rows goes in one
  // chunk of the smallest power-of-two size that holds it.
  static constexpr int UL = CPT >= 8 ? 4 : 8;
  template <int S, bool REC>
  __device__ __forceinline__ int sweep_short(const int32_t *list, int cnt) {
    if constexpr (S > 1) {
      if (cnt <= S / 2) return sweep_short<S / 2, REC>(list, cnt);
    }
    Chunk<S> X;
    chunk_load<true, S, REC>(list, 0, cnt, X);
    return chunk_fold_compact<S>(X);
  }

  // Rows go in chunks of U.  In the one-instance kernel the chunks are
  // pipelined: a short frontier pays one small chunk, a long one about one
  // memory latency in all.
  template <bool NARROW, bool REC>
  __device__ __forceinline__ int sweep_t(const int32_t *list, int cnt) {
    int used = 0;
    int f = 0;
    if constexpr (COMPACT && LONG) {
      if (cnt <= 0) return 0;
      if (cnt <= UL) return sweep_short<UL, REC>(list, cnt);
      Chunk<UL> a;
      chunk_load<true, UL, REC>(list, 0, cnt, a);
      for (f = UL; f < cnt; f += UL) {
        Chunk<UL> b;
        chunk_load<true, UL, REC>(list, f, cnt, b);
        used += chunk_fold_compact<UL>(a);
        a = b;
      }
      return used + chunk_fold_compact<UL>(a);
    }
#ifndef OTKM_SWEEP32
#define OTKM_SWEEP32 0
#endif
    if constexpr (NARROW && OTKM_SWEEP32) {
      for (; f + UN <= cnt; f += UN) used += sweep_chunk_narrow<UN, REC>(list, f, cnt);
      if (f < cnt) used += sweep_narrow_tail<UN, REC>(list, f, cnt);
      return used;
    }
    if (LONG) {
      // the next chunk's cost loads are in flight while this chunk is folded,
      // so a long frontier pays about one memory latency, not one per chunk
      if (f < cnt) {
        Chunk<U> a;
        chunk_load<NARROW, U, REC>(list, f, cnt, a);
        for (f += U; f < cnt; f += U) {
          Chunk<U> b;
          chunk_load<NARROW, U, REC>(list, f, cnt, b);
          used += chunk_fold<NARROW, U>(a);
          a = b;
        }
        used += chunk_fold<NARROW, U>(a);
      }
      return used;
    }
    for (; f < cnt; f += U) used += sweep_chunk<NARROW, U, REC>(list, f, cnt);
    return used;
  }

  __device__ __forceinline__ int sweep(const int32_t *list, int cnt) {
    if constexpr (COMPACT) return sweep_t<true, false>(list, cnt);
    else return narrow ? sweep_t<true, false>(list, cnt) : sweep_t<false, false>(list, cnt);
  }
  __device__ __forceinline__ int sweep_frontier(int cnt) {
    const int32_t *list = (const int32_t *)fr;
    if constexpr (COMPACT) return sweep_t<true, true>(list, cnt);
    else return narrow ? sweep_t<true, true>(list, cnt) : sweep_t<false, true>(list, cnt);
  }
  __device__ __forceinline__ static int2 frontier_rec(int row, int tree, int64_t h) {
    return make_int2(row | (tree << 16), (int)(uint32_t)h);
  }

  // Workgroup minimum of valid / stale keys over unreached owned columns plus
  // the error code, into slot set `s` (u64 pair at red[2s], int at ctl[es]).
  // The slots must hold (kInf, kInf, 0) beforehand; the caller issues the barrier.
  // Only key values are used downstream (the level, the refresh limit), so the
  // slots receive value << kRowBits.  With NARROW every value is below 2^32 - 1
  // and the wavefront reduction runs on 32-bit words.
  __device__ __forceinline__ void reduce_min(int s, int es) {
    if (COMPACT || narrow) {
      uint32_t a = 0xffffffffu, b = 0xffffffffu;
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        const bool open = (col(k) < n) & !((vis >> k) & 1u);
        const uint32_t v = (open && k1[k] != KINF) ? (uint32_t)kv(k1[k]) : 0xffffffffu;
        const bool st = stale(k);
        a = st ? a : min(a, v);
        b = st ? min(b, v) : b;
      }
      a = wave_min_u32(a);
      b = wave_min_u32(b);
      if (lane == 0) {
        if (a != 0xffffffffu) atomicMin((unsigned long long *)&red[2 * s], (unsigned long long)a << kRowBits);
        if (b != 0xffffffffu) atomicMin((unsigned long long *)&red[2 * s + 1], (unsigned long long)b << kRowBits);
      }
    } else if constexpr (!COMPACT) {
      uint64_t a = kInf, b = kInf;
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        if (col(k) >= n || ((vis >> k) & 1u)) continue;
        if (stale(k)) b = umin64(b, k1[k]);
        else a = umin64(a, k1[k]);
      }
      a = wave_min_u64(a);
      b = wave_min_u64(b);
      if (lane == 0) {
        if (a != kInf) atomicMin((unsigned long long *)&red[2 * s], (unsigned long long)a);
        if (b != kInf) atomicMin((unsigned long long *)&red[2 * s + 1], (unsigned long long)b);
      }
    }
    if (err_local != 0) atomicMin(&ctl[es], err_local);  // rare: only lanes that saw an error
  }
  // GRID: barrier over the instance's workgroups (thread 0 arrives and waits).
  // Every wait is bounded: one that runs out raises the abort flag, a raised
  // flag ends every other wait, and the caller leaves its loop, so the kernel
  // always finishes.  Returns true on abort.
  static constexpr int kSpinLimit = 1 << 21;  // polls (a round trip and a short sleep each): about a second
  __device__ __forceinline__ bool grid_sync() {
    __syncthreads();
    if (tid == 0) {
      int *bar = (int *)(gws + kGBar), *ab = (int *)(gws + kGAbort);
      int stop = __hip_atomic_load(ab, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!stop) {
        ++epoch;
        __hip_atomic_fetch_add(bar, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const int target = epoch * G;
        for (int s = 0; __hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target; ++s) {
          if (__hip_atomic_load(ab, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { stop = 1; break; }
          if (s > kSpinLimit) { __hip_atomic_store(ab, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); stop = 1; break; }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      ctl[GAB] = stop;
    }
    __syncthreads();
    return ctl[GAB] != 0;
  }

  // GRID exchanges.  Every word a workgroup publishes carries the level it
  // belongs to, so a reader fetches tags and data in one round and polls until
  // all of them show the current level: minimum words hold (level mod 2^31) <<
  // 33 | key value (33 bits), the error word level << 32 | error, settled
  // columns (level mod 2^28) << 36 | column << 24 | row << 12 | tree, and a
  // list's count word level << 32 | count.  Polls are bounded and end on the
  // abort flag.
  __device__ __forceinline__ bool poll_abort(int s) {
    int ab = 0;
    if ((s & 31) == 31) {
      ab = lane == 0 ? __hip_atomic_load((int *)(gws + kGAbort), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
      ab = __builtin_amdgcn_readfirstlane(ab);
    }
    if (s > kSpinLimit) {
      if (lane == 0) __hip_atomic_store((int *)(gws + kGAbort), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ab = 1;
    }
    return ab != 0;
  }
  // A key value is below 3 * 2^31 < 2^33 - 1, so 33 bits hold it with all ones
  // for "no key", and the remaining 31 bits tag the level.
  static constexpr uint64_t kMinVal = (1ull << 33) - 1;
  static constexpr uint32_t kLevTag = 0x7fffffffu;
  static __device__ __forceinline__ uint64_t enc_min(uint64_t key, uint32_t lv) {
    const uint64_t v = key == kInf ? kMinVal : (key >> kRowBits);
    return ((uint64_t)(lv & kLevTag) << 33) | v;
  }
  static __device__ __forceinline__ uint64_t dec_min(uint64_t w) {
    const uint64_t v = w & kMinVal;
    return v == kMinVal ? kInf : v << kRowBits;
  }

  // GRID: publish this workgroup's slot set s (minimum pair, error es), read
  // every workgroup's, and replace the local values by the minima over all of
  // them.  The caller has issued the barrier after reduce_min.  Returns true on
  // abort.
  __device__ __forceinline__ bool grid_min(int s, int es) {
    uint64_t *slot = gws + kGMin + ((size_t)s * kMaxWgs) * 3;
    if (wid == 0) {
      if (lane == 0) {
        __hip_atomic_store(&slot[3 * g], enc_min(red[2 * s], lev), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&slot[3 * g + 1], enc_min(red[2 * s + 1], lev), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&slot[3 * g + 2], ((uint64_t)lev << 32) | (uint32_t)ctl[es], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
      const int w = lane / 3, k = lane - 3 * (lane / 3);
      uint64_t x = 0;
      bool stop = false;
      for (int it = 0;; ++it) {
        if (w < G) x = __hip_atomic_load(&slot[3 * w + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool ok = w >= G || (k < 2 ? (uint32_t)(x >> 33) == (lev & kLevTag) : (uint32_t)(x >> 32) == lev);
        if (__builtin_amdgcn_ballot_w64(!ok) == 0) break;
        if (poll_abort(it)) { stop = true; break; }
        __builtin_amdgcn_s_sleep(1);
      }
      const uint64_t a = wave_min_u64(w < G && k == 0 ? dec_min(x) : kInf);
      const uint64_t b = wave_min_u64(w < G && k == 1 ? dec_min(x) : kInf);
      const int ee = wave_min_i32(w < G && k == 2 ? (int)(uint32_t)x : 0);
      if (lane == 0) { red[2 * s] = a; red[2 * s + 1] = b; ctl[es] = ee; ctl[GAB] = stop ? 1 : 0; }
    }
    __syncthreads();
    return ctl[GAB] != 0;
  }

  __device__ __forceinline__ void reset_slots(int s, int es) {
    red[2 * s] = kInf;
    red[2 * s + 1] = kInf;
    ctl[es] = 0;
  }

  // One round of a stale column's gather: GU forest rows per lane (list
  // entries f0, f0 + stride, ...), their trees and duals, and their entries
  // of the column (loads possibly still in flight).
  struct GatherSet {
    int i[GU], t[GU];
    int64_t h[GU];
    int32_t c[GU];
  };
  __device__ __forceinline__ void gather_load(GatherSet &X, const int32_t *colp, size_t cstride, int f0, int stride,
                                              int nf) {
#pragma unroll
    for (int q = 0; q < GU; ++q) {
      const int f = f0 + q * stride;
      X.i[q] = f < nf ? fst[f] : 0;
      if ((unsigned)X.i[q] >= (unsigned)rows()) { fail(OT_EINTERNAL); X.i[q] = 0; }
      X.t[q] = f < nf ? rtree[X.i[q]] : -1;
      X.h[q] = hrow[X.i[q]];
    }
#pragma unroll
    for (int q = 0; q < GU; ++q) X.c[q] = colp[(size_t)X.i[q] * cstride];
  }
  __device__ __forceinline__ void gather_fold(const GatherSet &X, int64_t v, Key &a1, int &ta1, Key &a2, int &ta2) {
#pragma unroll
    for (int q = 0; q < GU; ++q) {
      if (X.t[q] < 0) continue;
      int64_t val = (int64_t)X.c[q] - X.h[q] - v;
      if (val < 0) { fail(OT_EINTERNAL); val = 0; }
      top2_push(a1, ta1, a2, ta2, kpack(val, X.i[q]), X.t[q]);
    }
  }
  static __device__ __forceinline__ Key wmin_key(Key x) {
    if constexpr (COMPACT) return wave_min_u32(x);
    else return wave_min_u64(x);
  }

  // Recompute stale keys that could be the next minimum.  Returns cost
  // entries read; sets `resweep` when a full re-sweep of the forest was used.
  __device__ __forceinline__ int64_t refresh_stale(uint64_t mv, bool &resweep, int &swept) {
    const int64_t lim = (mv == kInf) ? INT64_MAX : kval(mv);
    uint32_t req = 0;
    int slot[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      slot[k] = -1;
      if (col(k) >= n || ((vis >> k) & 1u) || !stale(k)) continue;
      if (kv(k1[k]) > lim) continue;
      int s = atomicAdd(&ctl[GCNT], 1);
      slot[k] = s;
      req |= 1u << k;
      if (s < gcap) { gcol[s] = col(k); gv[s] = vj[k]; }
    }
    __syncthreads();
    const int g = ctl[GCNT];
    const int nf = ctl[FCNT];
    resweep = false;
    swept = 0;
    if (g > gcap) {
      // too many: one coalesced re-sweep of every forest row fixes all keys
#pragma unroll
      for (int k = 0; k < CPT; ++k) { k1[k] = KINF; k2[k] = KINF; t1[k] = -1; t2[k] = -1; }
      stl = 0;
      swept = sweep(fst, nf);
      resweep = true;
      return 0;
    }
    // Each stale column gets wpc wavefronts that split the forest rows; partial
    // top-2 summaries meet in LDS and one thread per column merges them.
    const int wpc = g >= NW ? 1 : NW / g;
    const int per_round = NW / wpc;
    uint64_t *pk1 = red + 32, *pk2 = red + 32 + NW;
    int32_t *pt = (int32_t *)(red + 32 + 2 * NW);
    for (int base = 0; base < g; base += per_round) {
      const int s = base + wid / wpc;
      const int slice = wid % wpc;
      if (s < g) {
        const int j = gcol[s];
        const int64_t v = gv[s];
        // column j of C: a contiguous row of the transpose when there is one,
        // else one entry per cost row
        const int32_t *colp = CT ? CT + (size_t)j * (size_t)ldt : C + j;
        const size_t cstride = CT ? 1 : (size_t)ld;
        Key a1 = KINF, a2 = KINF;
        int ta1 = -1, ta2 = -1;
        const int stride = 64 * wpc;
        // GU forest rows per lane at a time; the next GU rows' reads are issued
        // before the current ones are folded, so a long forest list pays about
        // one memory latency instead of one per round
        // (one-instance kernels; the batched kernels keep one round in flight
        // to spare registers)
        const int f00 = slice * 64 + lane;
        if constexpr (LONG) {
          if (f00 - lane < nf) {
            GatherSet a;
            gather_load(a, colp, cstride, f00, stride, nf);
            for (int f0 = f00 + GU * stride; f0 - lane < nf; f0 += GU * stride) {
              GatherSet b;
              gather_load(b, colp, cstride, f0, stride, nf);
              gather_fold(a, v, a1, ta1, a2, ta2);
              a = b;
            }
            gather_fold(a, v, a1, ta1, a2, ta2);
          }
        } else {
          for (int f0 = f00; f0 - lane < nf; f0 += GU * stride) {
            GatherSet a;
            gather_load(a, colp, cstride, f0, stride, nf);
            gather_fold(a, v, a1, ta1, a2, ta2);
          }
        }
        // the wavefront's top-2: its best key, then the best over the lanes of
        // the candidates outside the best key's tree (a lane's own best when
        // that is from another tree, else its second); the trees of the two
        // winners are read back from rtree
        {
          const Key w1 = wmin_key(a1);
          const int tw1 = w1 == KINF ? -1 : rtree[kr(w1)];
          const Key w2 = wmin_key(ta1 != tw1 ? a1 : a2);
          const int tw2 = w2 == KINF ? -1 : rtree[kr(w2)];
          a1 = w1; ta1 = tw1; a2 = w2; ta2 = tw2;
        }
        if (lane == 0) {
          if (wpc == 1) { gk1[s] = a1; gt1[s] = ta1; gk2[s] = a2; gt2[s] = ta2; }
          else { pk1[wid] = a1; pk2[wid] = a2; pt[2 * wid] = ta1; pt[2 * wid + 1] = ta2; }
        }
      }
      __syncthreads();
      if (wpc > 1 && tid < per_round && base + tid < g) {
        const int w0 = tid * wpc;
        Key a1 = (Key)pk1[w0], a2 = (Key)pk2[w0];
        int ta1 = pt[2 * w0], ta2 = pt[2 * w0 + 1];
        for (int w = w0 + 1; w < w0 + wpc; ++w) top2_merge(a1, ta1, a2, ta2, (Key)pk1[w], pt[2 * w], (Key)pk2[w], pt[2 * w + 1]);
        const int s = base + tid;
        gk1[s] = a1; gt1[s] = ta1; gk2[s] = a2; gt2[s] = ta2;
      }
      if (wpc > 1) __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      if (!((req >> k) & 1u)) continue;
      const int s = slot[k];
      k1[k] = (Key)gk1[s]; t1[k] = gt1[s]; k2[k] = (Key)gk2[s]; t2[k] = gt2[s];
      stl &= ~(1u << k);
    }
    return (int64_t)g * (int64_t)nf;
  }

  __device__ __forceinline__ void run(const Problem &P, char *smem) {
    C = P.C; CT = P.CT; n = P.n; ld = P.ld;
    nr_ = (RECT && P.nr > 0 && P.nr < P.n) ? P.nr : P.n;
    const int nr = rows();
    ldt = (RECT && P.ldt > 0) ? P.ldt : nr;
    const bool colred = nr == n;  // column reduction: square problems only
    tid = threadIdx.x; lane = tid & 63; wid = tid >> 6;
    {
      // the row offset goes in the (unchecked) scalar offset and the clamped
      // column in the checked vector offset, so the extent only bounds columns
      const int64_t extent = ((int64_t)(nr - 1) * ld + n) * 4;
      crsrc = __builtin_amdgcn_make_buffer_rsrc((void *)C, (short)0, (int)(extent < 0x7fffffff ? extent : 0x7fffffff),
                                                0x00020000);
    }
    err_local = 0;
    const LdsLayout L = lds_layout(n, GRID);
    hrow = (int64_t *)(smem + L.hrow);
    mrow = (int32_t *)(smem + L.mrow);
    mcol = (int32_t *)(smem + L.mcol);
    rtree = (int32_t *)(smem + L.rtree);
    par = (int16_t *)(smem + L.par);
    fst = (int32_t *)(smem + L.fst);
    fr = (int2 *)(smem + L.fr);
    alive = (uint8_t *)(smem + L.alive);
    gcol = (int32_t *)(smem + L.gcol);
    gv = (int64_t *)(smem + L.gv);
    gk1 = (uint64_t *)(smem + L.gk1);
    gk2 = (uint64_t *)(smem + L.gk2);
    gt1 = (int32_t *)(smem + L.gt1);
    gt2 = (int32_t *)(smem + L.gt2);
    red = (uint64_t *)(smem + L.red);
    ctl = (int32_t *)(smem + L.ctl);
    gcap = gather_cap(n);
    if constexpr (GRID) {
      G = gridDim.x; g = blockIdx.x; epoch = 0; lev = 0;
      gws = P.grid_ws;
      auglist = P.ws + (size_t)g * ws_ints(n);
    } else {
      auglist = P.ws;
    }
#pragma unroll
    for (int k = 0; k < CPT; ++k) voff[k] = lcol(k) * 4;
    bend = auglist + n;

    const int K = (P.max_paths <= 0 || P.max_paths > nr) ? nr : P.max_paths;
    int64_t st_levels = 0, st_dual = 0, st_aug = 0, st_paths = 0, st_rows = 0, st_gath = 0, st_resw = 0;
    int64_t st_refresh = 0, st_rcols = 0, tm_refresh = 0;
    int64_t tm_sweep = 0, tm_select = 0, tm_settle = 0, tm_aug = 0;

    if (tid < NCTL) ctl[tid] = 0;
    if (tid < 8) red[tid] = kInf;

    // ---- initialisation: u_i = min_j C_ij (one wavefront per row) and the cost range
    const bool pre = P.init_u && P.init_b && P.init_rmax;
    int gmin = 0x7fffffff, gmax = (int)0x80000000;
    if (pre) {
      for (int i = tid; i < nr; i += BLOCK) {
        const int64_t mn = P.init_u[i];
        hrow[i] = mn;
        gmin = min(gmin, (int)mn);
        gmax = max(gmax, P.init_rmax[i]);
      }
    }
    for (int i = pre ? nr : wid; i < nr; i += NW) {
      const int32_t *row = C + (size_t)i * (size_t)ld;
      int mn = 0x7fffffff, mx = (int)0x80000000;
      for (int j0 = 0; j0 < n; j0 += 64 * 16) {
        int c[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int j = j0 + lane + 64 * q;
          c[q] = row[j < n ? j : n - 1];  // clamped: duplicates do not change min / max
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) { mn = min(mn, c[q]); mx = max(mx, c[q]); }
      }
      mn = wave_min_i32(mn);
      mx = wave_max_i32(mx);
      if (lane == 0) hrow[i] = mn;
      gmin = min(gmin, mn);
      gmax = max(gmax, mx);
    }
    for (int i = tid; i < n; i += BLOCK) {
      mrow[i] = -1; mcol[i] = -1; bend[i] = kNoEnd;
      const bool root = i < K;
      alive[i] = root ? 1 : 0;
      rtree[i] = root ? i : -1;
      if (root) fst[i] = i;
    }
    gmin = wave_min_i32(gmin);
    gmax = wave_max_i32(gmax);
    int *ired = (int *)(red + 16);
    if (lane == 0) { ired[wid] = gmin; ired[NW + wid] = gmax; }
    __syncthreads();
    gmin = 0x7fffffff; gmax = (int)0x80000000;
    for (int w = 0; w < NW; ++w) { gmin = min(gmin, ired[w]); gmax = max(gmax, ired[NW + w]); }
    narrow = (int64_t)gmax - (int64_t)gmin < (1ll << 30);
    if (COMPACT && ((int64_t)gmax - (int64_t)gmin >= kCompactRange || n > kCompactMaxN)) {
      // the caller chose compact keys for a range they cannot hold
      if (P.stats && tid == 0) { ot_stats s = {}; s.status = OT_EINTERNAL; *P.stats = s; }
      return;
    }
    if ((int64_t)gmax - (int64_t)gmin > 0x7fffffffll) {
      if (P.stats && tid == 0) { ot_stats s = {}; s.status = OT_ERANGE; *P.stats = s; }
      return;
    }

    // ---- v_j = min_i (C_ij - u_i) (square; else v_j = 0); with every row a root, keep
    // the two best rows as keys
    vis = 0;
    stl = 0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      k1[k] = KINF; k2[k] = KINF; t1[k] = -1; t2[k] = -1; vj[k] = 0; dcol[k] = 0; ctree[k] = -1;
    }
    {
      uint64_t b1[CPT], b2[CPT];
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        b1[k] = pre ? P.init_b[2 * (size_t)lcol(k)] : kInf;
        b2[k] = pre ? P.init_b[2 * (size_t)lcol(k) + 1] : kInf;
      }
      int i = pre ? nr : 0;
      for (; i + 4 <= nr; i += 4) {
        int32_t c[4][CPT];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int32_t *row = C + (size_t)(i + q) * (size_t)ld;
#pragma unroll
          for (int k = 0; k < CPT; ++k) c[q][k] = row[lcol(k)];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t h = hrow[i + q];
#pragma unroll
          for (int k = 0; k < CPT; ++k) {
            uint64_t key = pack((int64_t)c[q][k] - h, i + q);
            if (key < b1[k]) { b2[k] = b1[k]; b1[k] = key; }
            else if (key < b2[k]) b2[k] = key;
          }
        }
      }
      for (; i < nr; ++i) {
        const int32_t *row = C + (size_t)i * (size_t)ld;
        const int64_t h = hrow[i];
        int32_t c[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) c[k] = row[lcol(k)];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
          if (col(k) >= n) continue;
          uint64_t key = pack((int64_t)c[k] - h, i);
          if (key < b1[k]) { b2[k] = b1[k]; b1[k] = key; }
          else if (key < b2[k]) b2[k] = key;
        }
      }
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        if (col(k) >= n) continue;
        vj[k] = colred ? (int32_t)kval(b1[k]) : 0;
        if (K == nr) {
          k1[k] = kpack(kval(b1[k]) - vj[k], krow(b1[k]));
          t1[k] = krow(b1[k]);
          if (b2[k] != kInf) { k2[k] = kpack(kval(b2[k]) - vj[k], krow(b2[k])); t2[k] = krow(b2[k]); }
        }
      }
    }
    st_rows = 2 * (int64_t)nr;
    int cur = 0;
    if (tid == 0) {
      ctl[CNT0] = 0; ctl[CNT1] = 0; ctl[FCNT] = K;
    }
    if (K < nr) {
      for (int i = tid; i < K; i += BLOCK) fr[i] = frontier_rec(i, i, hrow[i]);
      if (tid == 0) ctl[CNT0] = K;
    }
    __syncthreads();

    int nfree = nr, nalive = K, cursor = K;
    int64_t D = 0;
    // (n + 2)^2 + 64 <= 16,793,668 for n <= 4096: below every exchange tag's
    // range (31 bits on minimum words, 28 on settled columns), so tags never wrap
    const int64_t watchdog = (int64_t)(n + 2) * (int64_t)(n + 2) + 64;
    const bool timers = (P.flags & OT_FLAG_PHASE_TIMERS) != 0;
    int64_t tprev = timers ? now_ticks() : 0;

    while (nfree > 0) {
      const int ps = cur;  // slot parity of this level
      if constexpr (GRID) ++lev;
      // (1) fold the rows that joined last step into the keys
      const int nf = ctl[cur == 0 ? CNT0 : CNT1];
      st_rows += sweep_frontier(nf);
      const int64_t t0 = timers ? now_ticks() : 0;
      tm_sweep += t0 - tprev;
      // (2) smallest key over unreached columns
      reduce_min(ps, ERRA0 + ps);
      if (tid == 0) {
        ctl[cur == 0 ? CNT1 : CNT0] = 0; ctl[NAUG] = 0; ctl[GCNT] = 0; ctl[LCNT] = 0;
        reset_slots(ps ^ 1, ERRA0 + (ps ^ 1));
        reset_slots(2 + (ps ^ 1), ERRB0 + (ps ^ 1));
      }
      __syncthreads();
      if constexpr (GRID) {
        if (grid_min(ps, ERRA0 + ps)) { fail(OT_EINTERNAL); break; }
      }
      uint64_t mv = red[2 * ps], ms = red[2 * ps + 1];
      int berr = ctl[ERRA0 + ps];
      if (berr == 0 && ms != kInf && (mv == kInf || kval(ms) <= kval(mv))) {
        bool resweep;
        int swept;
        const int64_t tr0 = timers ? now_ticks() : 0;
        st_gath += refresh_stale(mv, resweep, swept);
        ++st_refresh;
        st_rcols += ctl[GCNT];
        if (timers) tm_refresh += now_ticks() - tr0;
        if (resweep) { ++st_resw; st_rows += swept; }
        reduce_min(2 + ps, ERRB0 + ps);
        __syncthreads();
        if constexpr (GRID) {
          if (grid_min(2 + ps, ERRB0 + ps)) { fail(OT_EINTERNAL); break; }
        }
        mv = red[2 * (2 + ps)];
        berr = ctl[ERRB0 + ps];
      }
      if (berr != 0) break;
      if (mv == kInf) { fail(OT_EINTERNAL); break; }
      const int64_t level = kval(mv);
      if (level > D) { D = level; ++st_dual; }
      // the watchdog; and with a tree cap the level adds up over stages and
      // could in principle leave the 32-bit range of the per-column levels
      // (compact keys hold levels below 2^20; the cost range bounds the level
      // by R < 2^18 unless a tree cap lets it add up over stages)
      if (++st_levels > watchdog || D > (COMPACT ? (1ll << 20) - 1 : 0x7ffffffell)) { fail(OT_EINTERNAL); break; }
      const int64_t t1_ = timers ? now_ticks() : 0;
      tm_select += t1_ - t0;

      // (3) settle every unreached column at the current level
      // the next frontier overwrites this one: every wavefront finished
      // reading it before the barrier above
      int *nxtcnt = &ctl[cur == 0 ? CNT1 : CNT0];
      if constexpr (GRID) {
        // settle the owned columns, publish them, and apply every workgroup's
        // list to the replicated state
        const int per = BLOCK * CPT;
        uint64_t *lists = gws + kGList + (size_t)ps * G * (per + 1);  // this parity's lists
        uint64_t *lst = lists + (size_t)g * (per + 1);                // count word, then entries
        const uint64_t etag = (uint64_t)(lev & 0xfffffffu) << 36;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
          const int j = col(k);
          if (j >= n || ((vis >> k) & 1u) || k1[k] == KINF || stale(k) || kv(k1[k]) != D) continue;
          vis |= 1u << k;
          dcol[k] = (int32_t)D;
          ctree[k] = t1[k];
          const uint64_t e = etag | ((uint64_t)j << 24) | ((uint64_t)kr(k1[k]) << 12) | (uint64_t)(uint32_t)t1[k];
          __hip_atomic_store(&lst[1 + atomicAdd(&ctl[LCNT], 1)], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        // wavefront 0 reads every workgroup's count word and its first L - 1
        // entries in one round (L lanes per workgroup); later entries, if any,
        // are polled one by one below
        const int L = 64 / G;
        uint64_t *spec = red + 16;     // [G][L - 1] entries read with the counts
        int *gc = (int *)(red + 112);  // gc[w] = first entry of workgroup w, gc[G] = total
        if (wid == 0) {
          if (lane == 0)
            __hip_atomic_store(lst, ((uint64_t)lev << 32) | (uint32_t)ctl[LCNT], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
          const int w = lane / L, k = lane - w * L;
          uint64_t x = 0;
          int cnt = 0;
          bool stop = false;
          for (int it = 0;; ++it) {
            if (w < G) x = __hip_atomic_load(lists + (size_t)w * (per + 1) + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t hdr = __shfl(x, w < G ? w * L : 0, 64);
            const bool hok = w >= G || (uint32_t)(hdr >> 32) == lev;
            cnt = (w < G && hok) ? (int)(uint32_t)hdr : 0;
            const bool ok = hok && (w >= G || k == 0 || k - 1 >= cnt || (x >> 36) == (lev & 0xfffffffu));
            if (__builtin_amdgcn_ballot_w64(!ok) == 0) break;
            if (poll_abort(it)) { stop = true; break; }
            __builtin_amdgcn_s_sleep(1);
          }
          if (!stop && w < G && k >= 1 && k - 1 < cnt) spec[w * (L - 1) + (k - 1)] = x;
          if (lane == 0) {
            int acc = 0;
            for (int v = 0; v < G; ++v) {
              gc[v] = acc;
              acc += __builtin_amdgcn_readlane(cnt, v * L);
            }
            gc[G] = acc;
            ctl[GAB] = stop ? 1 : 0;
          }
        }
        __syncthreads();
        if (ctl[GAB]) { fail(OT_EINTERNAL); break; }
        const int tot = gc[G];
        for (int q = tid; q < tot; q += BLOCK) {
          int w = 0;
          while (w + 1 < G && gc[w + 1] <= q) ++w;
          const int idx = q - gc[w];
          if (idx >= per) { fail(OT_EINTERNAL); continue; }
          uint64_t e;
          if (idx < L - 1) {
            e = spec[w * (L - 1) + idx];
          } else {
            const uint64_t *src = lists + (size_t)w * (per + 1) + 1 + idx;
            int it = 0;
            for (;; ++it) {
              e = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              if ((e >> 36) == (lev & 0xfffffffu) || it > kSpinLimit) break;
              __builtin_amdgcn_s_sleep(1);
            }
            if (it > kSpinLimit) { fail(OT_EINTERNAL); continue; }
          }
          const int j = (int)((e >> 24) & 0xfff), p = (int)((e >> 12) & 0xfff), tr = (int)(e & 0xfff);
          if (j >= n || p >= nr || tr >= nr) { fail(OT_EINTERNAL); continue; }
          par[j] = (int16_t)p;
          const int mc = mcol[j];
          if (mc < 0) {
            if (atomicMin(&bend[tr], j) == kNoEnd) {
              const int s = atomicAdd(&ctl[NAUG], 1);
              auglist[s] = tr;
            }
          } else {
            rtree[mc] = tr;
            const int64_t hm = hrow[mc] - D;
            hrow[mc] = hm;
            fr[atomicAdd(nxtcnt, 1)] = frontier_rec(mc, tr, hm);
            fst[atomicAdd(&ctl[FCNT], 1)] = mc;
          }
        }
      } else {
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        const int j = col(k);
        if (j >= n || ((vis >> k) & 1u) || k1[k] == KINF || stale(k) || kv(k1[k]) != D) continue;
        const int p = kr(k1[k]);
        const int tr = t1[k];
        vis |= 1u << k;
        dcol[k] = (int32_t)D;
        ctree[k] = tr;
        par[j] = (int16_t)p;
        const int mc = mcol[j];
        if (mc < 0) {
          if (atomicMin(&bend[tr], j) == kNoEnd) {
            const int s = atomicAdd(&ctl[NAUG], 1);
            auglist[s] = tr;
          }
        } else {
          // the matched row joins the tree (undone below if the tree augments now)
          rtree[mc] = tr;
          const int64_t hm = hrow[mc] - D;
          hrow[mc] = hm;
          fr[atomicAdd(nxtcnt, 1)] = frontier_rec(mc, tr, hm);
          fst[atomicAdd(&ctl[FCNT], 1)] = mc;
        }
      }
      }
      __syncthreads();
      const int naug = ctl[NAUG];
      const int64_t t2_ = timers ? now_ticks() : 0;
      tm_settle += t2_ - t1_;
      if (naug > 0) {
        // (4) flip one path per tree that reached a free column (trees are disjoint)
        for (int a = tid; a < naug; a += BLOCK) {
          const int tr = auglist[a];
          int j = bend[tr];
          bend[tr] = kNoEnd;
          for (int steps = 0;; ++steps) {
            if (steps > n || (unsigned)j >= (unsigned)n) { fail(OT_EINTERNAL); break; }
            const int p = par[j];
            if ((unsigned)p >= (unsigned)nr) { fail(OT_EINTERNAL); break; }
            const int before = mrow[p];
            mrow[p] = j;
            mcol[j] = p;
            if (p == tr) break;
            j = before;
          }
          alive[tr] = 0;
        }
        ++st_aug;
        st_paths += naug;
        nfree -= naug;
        nalive -= naug;
        __syncthreads();
        // (5) rows and columns of finished trees leave the forest with their duals materialised
        for (int i = tid; i < nr; i += BLOCK) {
          const int t = rtree[i];
          if (t >= 0 && !alive[t]) { hrow[i] += D; rtree[i] = -1; }
        }
        // rows that joined this step in a tree that just finished leave the next sweep
        for (int q = tid; q < *nxtcnt; q += BLOCK) {
          const int2 e = fr[q];
          if (e.x >= 0 && !alive[e.x >> 16]) fr[q].x = e.x | (int)0x80000000;
        }
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
          if (col(k) >= n) continue;
          if (((vis >> k) & 1u) && !alive[ctree[k]]) {
            const int64_t d = D - dcol[k];
            vj[k] -= (int32_t)d;
            const Key sh = (Key)d << KB;
            if (k1[k] != KINF) k1[k] += sh;
            if (k2[k] != KINF) k2[k] += sh;
            vis &= ~(1u << k);
            ctree[k] = -1;
          }
          if (t1[k] >= 0 && !alive[t1[k]]) {
            // best key came from a finished tree: fall back to the best other tree;
            // what lies behind it is unknown, so keep it only as a lower bound
            k1[k] = k2[k]; t1[k] = t2[k]; t2[k] = -1;
          } else if (t2[k] >= 0 && !alive[t2[k]]) {
            t2[k] = -1;
          }
          if (nalive == 0) { k1[k] = KINF; k2[k] = KINF; t1[k] = -1; t2[k] = -1; }
          recompute_stale(k);
        }
        if (tid == 0) ctl[FCNT] = 0;
        __syncthreads();
        // (6) rebuild the forest list (one LDS atomic per wavefront and 64 rows,
        // each lane's slot from its rank among the lanes that keep a row); with
        // a tree cap, start new trees from the next free rows
        for (int i0 = wid * 64; i0 < nr; i0 += BLOCK) {
          const int i = i0 + lane;
          const bool keep = i < nr && rtree[i] >= 0;
          const uint64_t m = __builtin_amdgcn_ballot_w64(keep);
          int base = 0;
          if (lane == 0 && m != 0) base = atomicAdd(&ctl[FCNT], (int)__builtin_popcountll(m));
          base = __builtin_amdgcn_readfirstlane(base);
          const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
          if (keep) fst[base + rank] = i;
        }
        const int need = min(K - nalive, nr - cursor);
        if (need > 0) {
          __syncthreads();  // the scan above must not see the new roots
          for (int q = tid; q < need; q += BLOCK) {
            const int r = cursor + q;
            rtree[r] = r;
            alive[r] = 1;
            const int64_t hr = hrow[r] - D;
            hrow[r] = hr;
            fr[atomicAdd(nxtcnt, 1)] = frontier_rec(r, r, hr);
            fst[atomicAdd(&ctl[FCNT], 1)] = r;
          }
          cursor += need;
          nalive += need;
        }
        __syncthreads();
        tprev = timers ? now_ticks() : 0;
        tm_aug += tprev - t2_;
      } else {
        tprev = t2_;
      }
      cur ^= 1;
    }

    __syncthreads();
    if (err_local != 0) atomicMin(&ctl[ERR], err_local);
    __syncthreads();
    int err = ctl[ERR];
    if constexpr (GRID) {
      // one error and the gathers over all workgroups (every workgroup left the
      // loop at the same level; after an abort the barrier returns at once)
      if (tid == 0) {
        __hip_atomic_store(gws + kGFin + g, (uint64_t)(uint32_t)err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(gws + kGGath + g, (uint64_t)st_gath, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      const bool aborted = grid_sync();
      if (tid == 0) {
        int e = aborted ? OT_EINTERNAL : 0;
        int64_t gath = 0;
        if (!aborted)
          for (int w = 0; w < G; ++w) {
            e = min(e, (int)(uint32_t)__hip_atomic_load(gws + kGFin + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            gath += (int64_t)__hip_atomic_load(gws + kGGath + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        ctl[ERR] = e;
        red[0] = (uint64_t)gath;
      }
      __syncthreads();
      err = ctl[ERR];
      st_gath = (int64_t)red[0];
      __syncthreads();
    }
    if (err == 0 && (!GRID || g == 0)) {
      int64_t part = 0;
      const int32_t *Cr = P.Cout ? P.Cout : C;
      const size_t ldr = P.Cout ? (size_t)P.ldo : (size_t)ld;
      for (int i = tid; i < nr; i += BLOCK) {
        const int j = mrow[i];
        P.plan[i] = j;
        if (P.u) P.u[i] = hrow[i] * P.dscale;
        part += (j >= 0 && j < n) ? (int64_t)Cr[(size_t)i * ldr + j] : 0;
      }
      part = wave_sum_i64(part);
      int64_t *sred = (int64_t *)(red + 16);
      if (lane == 0) sred[wid] = part;
      __syncthreads();
      if (tid == 0) {
        int64_t tot = 0;
        for (int w = 0; w < NW; ++w) tot += sred[w];
        *P.cost = tot;
      }
    }
    if (err == 0 && P.v) {
#pragma unroll
      for (int k = 0; k < CPT; ++k)
        if (col(k) < n) P.v[col(k)] = (int64_t)vj[k] * P.dscale;
    }
    if (P.stats && tid == 0 && (!GRID || g == 0)) {
      ot_stats s;
      s.levels = st_levels; s.dual_adjusts = st_dual; s.aug_events = st_aug; s.paths = st_paths;
      s.rows_swept = st_rows; s.gathers = st_gath; s.resweeps = st_resw; s.status = err;
      s.t_sweep_ns = 10 * tm_sweep; s.t_select_ns = 10 * tm_select;  // wall clock ticks are 10 ns
      s.t_settle_ns = 10 * tm_settle; s.t_augment_ns = 10 * tm_aug;
      s.refreshes = st_refresh; s.refresh_cols = st_rcols; s.t_refresh_ns = 10 * tm_refresh;
      *P.stats = s;
    }
  }
};

}  // namespace otkm
