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
//   * at the first level whose settled columns include a free one, after
//     every column at that level has been settled, each tree that reached a
//     free column flips one path (to its smallest such column);
//   * two ways to go on from there (template parameter KEEP):
//       - restart (the batch kernel): the duals are materialised
//         (u_i += D - d_i on forest rows, v_j -= D - d_j on settled columns)
//         and the next round grows a new forest from the remaining free rows;
//       - kept forest (the one-instance kernel, the dense engine's
//         organisation): only the trees that augmented leave, with their
//         duals materialised; the other trees keep growing at the same level.
//         A column whose key came from a leaving row, or that a leaving tree
//         had settled, gets its key recomputed from its incoming edges (a
//         column-major copy of the graph the kernel builds first in global
//         scratch).  On a 4096 x 4096 k-NN graph this reads a quarter of the
//         edges the restarts read and takes two thirds of the levels;
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
constexpr uint64_t kSpRecompute = kSpInf - 1;  // a key to recompute from the live forest (kept forest only)
constexpr int kSpGroup = 16;  // lanes that share one row's edge list in a sweep

enum SpCtl { SP_LCNT = 0, SP_FOUND = 1, SP_NAUG = 2, SP_ERR = 3, SP_NLCNT = 4, SP_NCTL = 5 };

struct SparseLds {
  size_t key, v, h, bend, mcol, mrow, rtree, list, nlist, alive, red, ctl, total;
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
  L.nlist = o; o = align16(o + 2 * N);
  L.alive = o; o = align16(o + N);
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
  // kept forest only: global scratch for the graph by columns, written by the
  // kernel (colptr [m + 1], crow and ccost [nnz])
  int32_t *colptr = nullptr, *crow = nullptr, *ccost = nullptr;
  int64_t cap = 0;  // entries crow and ccost hold
};

// KEEP: the trees that did not augment stay (the dense engine's organisation);
// a column whose best row left the forest, or that a finished tree releases,
// gets its key recomputed from its incoming edges (a column-major copy of the
// graph the kernel builds first).  Without KEEP the forest is regrown from
// the free rows after every augmentation round.
template <int BLOCK, bool KEEP = false>
struct SparseEngine {
  static constexpr int NW = BLOCK / 64;
  uint64_t *key;
  int64_t *v, *h;
  int32_t *bend, *ctl;
  int16_t *mcol, *mrow, *rtree, *list, *nlist;
  uint8_t *alive;
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

  // The graph by columns: column j's incoming edges are rows
  // crow[colptr[j] .. colptr[j+1]) at costs ccost[...] (global scratch).
  __device__ __forceinline__ void build_csc(const SparseProblem &P) {
    const int n = P.n, m = P.m;
    int32_t *cnt = (int32_t *)key;  // m counters in the keys' space (reset afterwards)
    for (int j = tid; j < m; j += BLOCK) cnt[j] = 0;
    __syncthreads();
    for (int i = wid; i < n; i += NW)
      for (int64_t q = P.ptr[i] + lane; q < P.ptr[i + 1]; q += 64) atomicAdd(&cnt[P.idx[q]], 1);
    __syncthreads();
    if (wid == 0) {  // exclusive prefix sum, 64 columns at a time
      int carry = 0;
      for (int b = 0; b < m; b += 64) {
        const int j = b + lane;
        const int x = j < m ? cnt[j] : 0;
        int incl = x;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const int y = __shfl_up(incl, off, 64);
          if (lane >= off) incl += y;
        }
        if (j < m) { P.colptr[j] = carry + incl - x; cnt[j] = carry + incl - x; }
        carry += __shfl(incl, 63, 64);
      }
      if (lane == 0) P.colptr[m] = carry;
    }
    __syncthreads();
    for (int i = wid; i < n; i += NW)
      for (int64_t q = P.ptr[i] + lane; q < P.ptr[i + 1]; q += 64) {
        const int pos = atomicAdd(&cnt[P.idx[q]], 1);
        P.crow[pos] = i;
        P.ccost[pos] = P.cost[q];
      }
    __threadfence();  // read back by other threads of this workgroup
    __syncthreads();
  }

  // Column j's key from the rows of live trees next to it; returns edges read.
  __device__ __forceinline__ int64_t recompute(const SparseProblem &P, int j) {
    uint64_t best = kSpInf;
    const int b = P.colptr[j], e = P.colptr[j + 1];
    for (int q = b; q < e; ++q) {
      const int i = P.crow[q];
      if (rtree[i] < 0) continue;
      const uint64_t nk = ((uint64_t)((int64_t)P.ccost[q] - h[i] - v[j]) << kSpRowBits) | (uint64_t)i;
      best = umin64(best, nk);
    }
    key[j] = best;
    return e - b;
  }

  // Batched KM with the forest kept across augmentations: every free row is a
  // root from the start; a tree that reaches a free column augments at once
  // (its smallest such column) and leaves the forest with its duals
  // materialised; the others keep growing at the same level.
  __device__ __forceinline__ int kept_loop(const SparseProblem &P, int64_t &st_levels, int64_t &st_dual,
                                           int64_t &st_aug, int64_t &st_paths, int64_t &st_rows,
                                           int64_t &st_edges) {
    const int n = P.n, m = P.m;
    build_csc(P);
    for (int j = tid; j < m; j += BLOCK) key[j] = kSpInf;
    for (int i = tid; i < n; i += BLOCK) {
      rtree[i] = (int16_t)i;
      alive[i] = 1;
      bend[i] = 0x7fffffff;
      list[i] = (int16_t)i;
    }
    if (tid == 0) { ctl[SP_FOUND] = 0; ctl[SP_NAUG] = 0; ctl[SP_NLCNT] = 0; }
    __syncthreads();
    int cnt = n, nfree = n, err = OT_OK;
    int64_t D = 0;
    const int64_t watchdog = (int64_t)(n + 1) * (int64_t)(m + 2) + 64;
    while (nfree > 0) {
      if (++st_levels > watchdog) { err = OT_EINTERNAL; break; }
      st_rows += cnt;
      // (1) the rows that joined last (those of finished trees are skipped)
      {
        const int sub = lane / kSpGroup, sl = lane % kSpGroup;
        for (int p = wid * (64 / kSpGroup) + sub; p < cnt; p += NW * (64 / kSpGroup)) {
          const int i = list[p];
          if (rtree[i] < 0) continue;
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
      if (mv == kSpInf) { err = OT_EINFEASIBLE; break; }  // live trees and nothing to reach
      const int64_t level = (int64_t)(mv >> kSpRowBits);
      if (level > D) { D = level; ++st_dual; }
      // (3) settle every unreached column at the level
      for (int j = tid; j < m; j += BLOCK) {
        const uint64_t k = key[j];
        if ((k & kSpSettled) || (int64_t)(k >> kSpRowBits) != D) continue;
        key[j] = k | kSpSettled;
        const int t = rtree[(int)(k & kSpRowMask)];
        const int i2 = mcol[j];
        if (i2 >= 0) {
          rtree[i2] = (int16_t)t;
          h[i2] -= D;
          nlist[atomicAdd(&ctl[SP_NLCNT], 1)] = (int16_t)i2;
        } else {
          atomicMin(&bend[t], j);
          ctl[SP_FOUND] = 1;
        }
      }
      __syncthreads();
      if (ctl[SP_FOUND]) {
        // (4) one path per tree that reached a free column (its smallest one);
        // trees are disjoint, so are the paths
        for (int j0 = tid; j0 < m; j0 += BLOCK) {
          const uint64_t k0 = key[j0];
          if (!(k0 & kSpSettled) || mcol[j0] >= 0) continue;
          const int t = rtree[(int)(k0 & kSpRowMask)];
          if (bend[t] != j0) continue;
          int j = j0;
          for (int guard = 0; guard <= n; ++guard) {
            const int i = (int)(key[j] & kSpRowMask);
            const int prev = mrow[i];
            mrow[i] = (int16_t)j;
            mcol[j] = (int16_t)i;
            if (prev < 0) break;
            j = prev;
          }
          alive[t] = 0;
          atomicAdd(&ctl[SP_NAUG], 1);
        }
        __syncthreads();
        const int naug = ctl[SP_NAUG];
        if (naug == 0) { err = OT_EINTERNAL; break; }
        st_paths += naug;
        ++st_aug;
        nfree -= naug;
        // (5) finished trees leave: their columns are released with v
        // materialised, and a key whose row leaves is recomputed below
        for (int j = tid; j < m; j += BLOCK) {
          const uint64_t k = key[j];
          if (k == kSpInf) continue;
          const int t = rtree[(int)(k & kSpRowMask)];
          if (t >= 0 && alive[t]) continue;
          if (k & kSpSettled) v[j] -= D - (int64_t)((k & ~kSpSettled) >> kSpRowBits);
          key[j] = kSpRecompute;
        }
        __syncthreads();
        for (int i = tid; i < n; i += BLOCK) {
          const int t = rtree[i];
          if (t >= 0 && !alive[t]) { h[i] += D; rtree[i] = -1; }
        }
        __syncthreads();
        for (int j = tid; j < m; j += BLOCK)
          if (key[j] == kSpRecompute) st_edges += recompute(P, j);
        if (tid == 0) { ctl[SP_FOUND] = 0; ctl[SP_NAUG] = 0; }
        __syncthreads();
      }
      // the next frontier: the rows that joined at this level
      cnt = ctl[SP_NLCNT];
      int16_t *tmp = list; list = nlist; nlist = tmp;
      __syncthreads();
      if (tid == 0) ctl[SP_NLCNT] = 0;
    }
    __syncthreads();
    // every row is matched: materialise the live forest's duals (none left
    // when all trees finished; a row of a live tree only remains on error)
    for (int i = tid; i < n; i += BLOCK)
      if (rtree[i] >= 0) { h[i] += D; rtree[i] = -1; }
    __syncthreads();
    return err;
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
    nlist = (int16_t *)(smem + L.nlist);
    alive = (uint8_t *)(smem + L.alive);
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
    // the graph by columns must fit the workspace it is built in
    if (KEEP && P.ptr[n] - P.ptr[0] > P.cap) err = OT_EINVAL;
    int64_t st_levels = 0, st_dual = 0, st_rounds = 0, st_paths = 0, st_rows = 0, st_edges = 0;
    int nfree = n;
    const int64_t watchdog = (int64_t)(n + 1) * (int64_t)(m + 2) + 64;
    if constexpr (KEEP) {
      if (err == OT_OK) err = kept_loop(P, st_levels, st_dual, st_rounds, st_paths, st_rows, st_edges);
      nfree = 0;
    }
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
        s.gathers = edges;  // edge entries (column and cost) read by the sweeps and key recomputes
        s.status = err;
        *P.stats = s;
      }
    }
  }
};

}  // namespace otkm
