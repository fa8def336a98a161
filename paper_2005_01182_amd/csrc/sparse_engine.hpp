// sparse_engine.hpp -- Batched KM on a sparse cost graph, one workgroup per
// instance.
//
// The graph is given in CSR: row i's edges go to the columns
// idx[ptr[i] .. ptr[i+1]) at costs cost[...]; an entry missing from the graph
// cannot be used.  Every row must be matched (n <= m); columns may stay free.
// Same method as the dense engine (Section 2.3.1): alternating trees grow at
// once from every free row over tight edges, each tree that reaches a free
// column augments along one path, and when no tree can grow the duals move
// across the cut by the smallest slack.  Organisation:
//   * one phase ("round") grows the forest from every free row with
//     Dijkstra-style levels: a row that joined at level D keeps
//     h_i = u_i - D, and column j's key is the smallest c_ij - h_i - v_j over
//     the forest rows next to it (its distance), packed with the row;
//   * a level sweeps the edge lists of the rows that joined last (atomic
//     minimum into the keys in LDS), takes the smallest key over unreached
//     columns and settles every column at that value; a settled matched
//     column brings its row into the same tree;
//   * the round ends at the first level whose settled columns include a free
//     one, after every column at that level has been settled (so every tree
//     that reaches a free column at the level augments); the duals are then
//     materialised (u_i += D - d_i on forest rows, v_j -= D - d_j on settled
//     columns), one path per such tree (its smallest free column) is flipped,
//     and the next round starts from the remaining free rows -- the forest is
//     rebuilt each round, which is what the method does after augmenting;
//   * when no column can be reached and no tree has found a free column, the
//     forest's rows have fewer neighbours than rows (Hall's condition fails):
//     no matching covers every row (OT_EINFEASIBLE).
// Duals start at u_i = the cheapest edge of row i and v = 0; v only falls,
// and only on settled columns, so v <= 0 and every column left free keeps
// v_j = 0: (u, v) is an optimal solution of the dual LP (u_i + v_j <= c_e on
// every edge, v <= 0).
//
// Ranges: costs are int32, so every dual stays within n * 2^32 <= 2^44 and a
// key value (a distance, at most the largest reduced cost along a path) fits
// 47 bits above the 16-bit row index.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.hpp"
#include "otkm.h"

namespace otkm {

constexpr int kSpRowBits = 16;
constexpr uint64_t kSpRowMask = (1ull << kSpRowBits) - 1;
constexpr uint64_t kSpSettled = 1ull << 63;
constexpr uint64_t kSpInf = kSpSettled - 1;  // an unreached column (no key yet); kInf would read as settled
constexpr int kSpGroup = 16;  // lanes that share one row's edge list in a sweep

enum SpCtl { SP_LCNT = 0, SP_FOUND = 1, SP_NAUG = 2, SP_ERR = 3, SP_NCTL = 4 };

struct SparseLds {
  size_t key, v, h, bend, mcol, mrow, rtree, list, red, ctl, total;
};
// Byte offsets of the LDS arrays for n rows and m columns (host and device).
__host__ __device__ inline SparseLds sparse_lds(int n, int m) {
  SparseLds L;
  const size_t N = (size_t)n, M = (size_t)m;
  size_t o = 0;
  L.key = o;   o = align16(o + 8 * M);
  L.v = o;     o = align16(o + 8 * M);
  L.h = o;     o = align16(o + 8 * N);
  L.bend = o;  o = align16(o + 4 * N);
  L.mcol = o;  o = align16(o + 2 * M);
  L.mrow = o;  o = align16(o + 2 * N);
  L.rtree = o; o = align16(o + 2 * N);
  L.list = o;  o = align16(o + 2 * N);
  L.red = o;   o = align16(o + 8 * 32);
  L.ctl = o;   o = align16(o + 4 * SP_NCTL);
  L.total = o;
  return L;
}

struct SparseProblem {
  const int64_t *ptr;   // [n + 1]
  const int32_t *idx;   // [ptr[n]]
  const int32_t *cost;  // [ptr[n]]
  int n, m;
  int32_t *plan;        // [n]
  int64_t *total;       // [1]
  int64_t *u, *v;       // [n], [m] or null
  ot_stats *stats;      // [1] or null
};

template <int BLOCK>
struct SparseEngine {
  static constexpr int NW = BLOCK / 64;
  uint64_t *key;
  int64_t *v, *h;
  int32_t *bend, *ctl;
  int16_t *mcol, *mrow, *rtree, *list;
  uint64_t *red;
  int tid, lane, wid;

  // smallest 64-bit value over the workgroup (every thread gets it)
  __device__ __forceinline__ uint64_t block_min(uint64_t x) {
    x = wave_min_u64(x);
    if (lane == 0) red[wid] = x;
    __syncthreads();
    uint64_t r = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) r = umin64(r, red[w]);
    return r;
  }

  __device__ __forceinline__ int64_t block_sum(int64_t x) {
    x = wave_sum_i64(x);
    __syncthreads();  // red may still be read by a block_min
    if (lane == 0) red[wid] = (uint64_t)x;
    __syncthreads();
    int64_t r = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) r += (int64_t)red[w];
    return r;
  }

  __device__ __forceinline__ void run(const SparseProblem &P, char *smem) {
    const int n = P.n, m = P.m;
    tid = threadIdx.x; lane = tid & 63; wid = tid >> 6;
    const SparseLds L = sparse_lds(n, m);
    key = (uint64_t *)(smem + L.key);
    v = (int64_t *)(smem + L.v);
    h = (int64_t *)(smem + L.h);
    bend = (int32_t *)(smem + L.bend);
    mcol = (int16_t *)(smem + L.mcol);
    mrow = (int16_t *)(smem + L.mrow);
    rtree = (int16_t *)(smem + L.rtree);
    list = (int16_t *)(smem + L.list);
    red = (uint64_t *)(smem + L.red);
    ctl = (int32_t *)(smem + L.ctl);
    if (tid < SP_NCTL) ctl[tid] = 0;
    for (int j = tid; j < m; j += BLOCK) { v[j] = 0; mcol[j] = -1; }
    __syncthreads();
    // ---- u_i = the cheapest edge of row i; the graph's shape is checked here
    // (a column out of range or a row with its end before its start: OT_EINVAL;
    // a row without edges can never be matched: OT_EINFEASIBLE)
    for (int i = wid; i < n; i += NW) {
      const int64_t b = P.ptr[i], e = P.ptr[i + 1];
      int mn = 0x7fffffff;
      bool bad = e < b;
      for (int64_t q = b + lane; q < e; q += 64) {
        const int j = P.idx[q];
        bad |= (unsigned)j >= (unsigned)m;
        mn = min(mn, P.cost[q]);
      }
      mn = wave_min_i32(mn);
      const bool anybad = __builtin_amdgcn_ballot_w64(bad) != 0;
      if (lane == 0) {
        h[i] = mn;
        mrow[i] = -1;
        if (anybad) atomicMax(&ctl[SP_ERR], 2);
        else if (e == b) atomicMax(&ctl[SP_ERR], 1);
      }
    }
    __syncthreads();
    int err = ctl[SP_ERR] == 2 ? OT_EINVAL : ctl[SP_ERR] == 1 ? OT_EINFEASIBLE : OT_OK;
    int64_t st_levels = 0, st_dual = 0, st_rounds = 0, st_paths = 0, st_rows = 0, st_edges = 0;
    int nfree = n;
    const int64_t watchdog = (int64_t)(n + 1) * (int64_t)(m + 2) + 64;
    while (err == OT_OK && nfree > 0) {
      // ---- a new round: every free row is the root of its own tree
      __syncthreads();
      for (int j = tid; j < m; j += BLOCK) key[j] = kSpInf;
      for (int i = tid; i < n; i += BLOCK) {
        bend[i] = 0x7fffffff;
        rtree[i] = mrow[i] < 0 ? (int16_t)i : (int16_t)-1;
      }
      if (tid == 0) { ctl[SP_LCNT] = 0; ctl[SP_FOUND] = 0; ctl[SP_NAUG] = 0; }
      __syncthreads();
      for (int i = tid; i < n; i += BLOCK)
        if (mrow[i] < 0) list[atomicAdd(&ctl[SP_LCNT], 1)] = (int16_t)i;
      __syncthreads();
      int s0 = 0, s1 = ctl[SP_LCNT];
      int64_t D = 0;
      for (;;) {
        if (++st_levels > watchdog) { err = OT_EINTERNAL; break; }
        st_rows += s1 - s0;
        // (1) the rows that joined last: keys of their unreached neighbours
        {
          const int sub = lane / kSpGroup, sl = lane % kSpGroup;
          for (int p = s0 + wid * (64 / kSpGroup) + sub; p < s1; p += NW * (64 / kSpGroup)) {
            const int i = list[p];
            const int64_t hi = h[i];
            const int64_t b = P.ptr[i], e = P.ptr[i + 1];
            if (sl == 0) st_edges += e - b;
            for (int64_t q = b + sl; q < e; q += kSpGroup) {
              const int j = P.idx[q];
              const uint64_t k = key[j];
              if (k & kSpSettled) continue;
              const uint64_t nk = ((uint64_t)((int64_t)P.cost[q] - hi - v[j]) << kSpRowBits) | (uint64_t)i;
              if (nk < k) atomicMin((unsigned long long *)&key[j], (unsigned long long)nk);
            }
          }
        }
        __syncthreads();
        // (2) the smallest key over unreached columns
        uint64_t mv = kSpInf;
        for (int j = tid; j < m; j += BLOCK) {
          const uint64_t k = key[j];
          if (!(k & kSpSettled)) mv = umin64(mv, k);
        }
        mv = block_min(mv);
        const bool found = ctl[SP_FOUND] != 0;
        if (mv == kSpInf) {
          if (!found) err = OT_EINFEASIBLE;
          break;
        }
        const int64_t level = (int64_t)(mv >> kSpRowBits);
        if (found && level > D) break;
        if (level > D) { D = level; ++st_dual; }
        // (3) settle every unreached column at the level
        for (int j = tid; j < m; j += BLOCK) {
          const uint64_t k = key[j];
          if ((k & kSpSettled) || (int64_t)(k >> kSpRowBits) != D) continue;
          key[j] = k | kSpSettled;
          const int i2 = mcol[j];
          if (i2 >= 0) {
            rtree[i2] = rtree[(int)(k & kSpRowMask)];
            h[i2] -= D;
            list[atomicAdd(&ctl[SP_LCNT], 1)] = (int16_t)i2;
          } else {
            ctl[SP_FOUND] = 1;
          }
        }
        __syncthreads();
        s0 = s1;
        s1 = ctl[SP_LCNT];
      }
      if (err != OT_OK) break;
      ++st_rounds;
      // ---- end of the round at level D: materialise the duals and claim one
      // free column per tree (the smallest)
      __syncthreads();
      const int nl = ctl[SP_LCNT];
      for (int p = tid; p < nl; p += BLOCK) h[list[p]] += D;
      for (int j = tid; j < m; j += BLOCK) {
        const uint64_t k = key[j];
        if (!(k & kSpSettled)) continue;
        v[j] -= D - (int64_t)((k & ~kSpSettled) >> kSpRowBits);
        if (mcol[j] < 0) atomicMin(&bend[rtree[(int)(k & kSpRowMask)]], j);
      }
      __syncthreads();
      // ---- flip each claimed path (the trees are disjoint, so are the paths)
      for (int j0 = tid; j0 < m; j0 += BLOCK) {
        const uint64_t k0 = key[j0];
        if (!(k0 & kSpSettled) || mcol[j0] >= 0 || bend[rtree[(int)(k0 & kSpRowMask)]] != j0) continue;
        int j = j0;
        for (int guard = 0; guard <= n; ++guard) {
          const int i = (int)(key[j] & kSpRowMask);
          const int prev = mrow[i];
          mrow[i] = (int16_t)j;
          mcol[j] = (int16_t)i;
          if (prev < 0) break;
          j = prev;
        }
        atomicAdd(&ctl[SP_NAUG], 1);
      }
      __syncthreads();
      const int naug = ctl[SP_NAUG];
      st_paths += naug;
      nfree -= naug;
      if (naug == 0) err = OT_EINTERNAL;  // a round that found a free column augments
    }
    __syncthreads();
    // ---- results: plan, duals, and the total over the plan's edges (the
    // cheapest copy when a column repeats in a row)
    int64_t part = 0;
    if (err == OT_OK) {
      for (int i = wid; i < n; i += NW) {
        const int j = mrow[i];
        const int64_t b = P.ptr[i], e = P.ptr[i + 1];
        int c = 0x7fffffff;
        for (int64_t q = b + lane; q < e; q += 64)
          if (P.idx[q] == j) c = min(c, P.cost[q]);
        c = wave_min_i32(c);
        if (lane == 0) {
          P.plan[i] = j;
          if (P.u) P.u[i] = h[i];
          part += c;
        }
      }
      if (P.v)
        for (int j = tid; j < m; j += BLOCK) P.v[j] = v[j];
    }
    const int64_t total = block_sum(part);
    const int64_t edges = block_sum(st_edges);
    if (tid == 0) {
      if (err == OT_OK) *P.total = total;
      if (P.stats) {
        ot_stats s = {};
        s.levels = st_levels;
        s.dual_adjusts = st_dual;
        s.aug_events = st_rounds;
        s.paths = st_paths;
        s.rows_swept = st_rows;
        s.gathers = edges;  // edge entries (column and cost) read by the sweeps
        s.status = err;
        *P.stats = s;
      }
    }
  }
};

}  // namespace otkm
