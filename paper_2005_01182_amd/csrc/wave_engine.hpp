// wave_engine.hpp -- batched Kuhn-Munkres for instances of at most 64 rows,
// on one wavefront with every piece of state in registers.
//
// The method and every choice it makes are the workgroup engine's (Engine in
// engine.hpp): trees from every free row (or from the first max_paths rows),
// exact per-column top-2 keys of (reduced cost + level, row) from distinct
// trees, a level D that rises to the smallest key, columns settled at D, one
// path per tree that reached a free column (its smallest such column), the
// forest kept across augmentations with the duals of finished trees
// materialised, stale keys recomputed when they could be the next minimum.
// So the results are the same, bit for bit.  The organisation differs:
//   * lane j holds column j's state and lane i row i's (dual, match, tree),
//     so a row that joins a tree, a path flip or a finished tree is a few
//     lane selects, ballots and cross-lane reads: no barrier and no LDS
//     atomic anywhere in the level loop;
//   * the frontier, the forest and the live trees are 64-bit lane masks;
//   * the cost matrix sits in LDS (rows padded to n + 1 words, so a row and a
//     column both read without bank conflicts): a sweep row is one LDS read
//     per lane, and a stale column is recomputed by all 64 lanes at once (one
//     row each) with two wavefront minima: the best key, then the best key of
//     the rows outside the best key's tree;
//   * keys are 32-bit (value << 12 | row) when the cost range is below 2^18
//     and every free row is a root, as in the workgroup engine, else 64-bit;
//     the order of keys, and so every choice, is the same either way.
#pragma once

#include "engine.hpp"

namespace otkm {

constexpr int kWaveMaxN = 64;

// LDS bytes of the wave engine for an n x n instance.
// C with rows padded to n + 1 words, then a 64-word row map used when paths flip.
__host__ __device__ inline size_t wave_lds_bytes(int n) { return ((size_t)n * (size_t)(n + 1) + 64) * 4; }

template <bool COMPACT>
struct WaveCore {
  using Key = typename KeyOf<COMPACT>::T;
  static constexpr int KB = KeyOf<COMPACT>::kBits;
  static constexpr Key KINF = (Key)~(Key)0;
  // compact keys hold values below 2^20 (3 x the cost range at most); with
  // 64-bit keys only the level is bounded (by the cost range, below 2^31)
  static constexpr int64_t kValMax = (1ll << 20) - 1;
  static constexpr int64_t kLevelMax = COMPACT ? kValMax : 0x7ffffffell;
  static __device__ __forceinline__ Key kpk(int64_t val, int row) { return ((Key)val << KB) | (Key)(uint32_t)row; }
  static __device__ __forceinline__ int64_t kv(Key k) { return (int64_t)(k >> KB); }
  static __device__ __forceinline__ int kr(Key k) { return (int)(k & (((Key)1 << KB) - 1)); }
  static __device__ __forceinline__ Key wmin(Key x) {
    if constexpr (COMPACT) return wave_min_u32(x);
    else return wave_min_u64(x);
  }

  int n, lane;
  bool cl;  // this lane holds a column and a row of the instance
  int32_t *rmap;  // [64] in LDS: the new column of each row on a flipped path
  // column state (lane j)
  Key k1, k2;
  int t1, t2, ctree, par, mcol, dcol;
  int32_t vj;
  bool vis, stl;
  bool bad;  // an invariant failed in this lane (reported as OT_EINTERNAL)
  // row state (lane i)
  int64_t h;   // u_i - D_i in a tree, u_i outside
  int mrow, rtree, bend;
  // lane masks
  uint64_t alive, forest, front;

  static __device__ __forceinline__ int bit_of(uint64_t m) { return __builtin_ctzll(m); }
  __device__ __forceinline__ bool alive_tree(int t) const { return t >= 0 && ((alive >> t) & 1ull); }

  // c - h_r - v_j for row r's entry c of this lane's column (the reduced cost
  // plus the level at which r joined).  With compact keys the cost range R is
  // below 2^18 and the result lies in [-R, 5R], so 32-bit wrapping arithmetic
  // gives it exactly.
  __device__ __forceinline__ int64_t reduced(int32_t c, int r, int32_t vjj) const {
    if constexpr (COMPACT) {
      const uint32_t hr = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)h, r);
      return (int32_t)((uint32_t)c - hr - (uint32_t)vjj);
    } else {
      return (int64_t)c - (int64_t)readlane64((uint64_t)h, r) - vjj;
    }
  }

  // Fold row r's entries (c in this lane's column) into the column keys.
  __device__ __forceinline__ void fold_row(int32_t c, int r) {
    const int tr = __builtin_amdgcn_readlane(rtree, r);
    const int64_t val = reduced(c, r, vj);
    bad |= cl && (val < 0 || (COMPACT && val > kValMax));  // a negative reduced cost: infeasible duals
    const Key key = cl ? kpk(val < 0 ? 0 : val, r) : KINF;
    stl = stl && !(key < k1);  // the best key now comes from a live tree
    top2_push(k1, t1, k2, t2, key, tr);
  }

  // Fold rows `rows` (a uniform mask) into the column keys, two rows at a
  // time with both LDS reads issued first (lanes past n read column 0 and keep
  // no key).  An odd last row is paired with itself: a candidate folded twice
  // changes nothing.
  __device__ __forceinline__ void sweep(const int32_t *Cs, int S, uint64_t rows) {
    const int lc = cl ? lane : 0;
    while (rows) {
      const int r0 = bit_of(rows);
      rows &= rows - 1;
      const int r1 = rows ? bit_of(rows) : r0;
      rows &= rows - 1;
      const int32_t c0 = Cs[r0 * S + lc], c1 = Cs[r1 * S + lc];
      fold_row(c0, r0);
      fold_row(c1, r1);
    }
  }

  // Exact top-2 of G columns js[] over the forest rows, every lane taking one
  // row: the best key, then the best key among rows of other trees.  The G
  // columns' reductions are independent, so their latencies overlap.  The
  // results are uniform.
  template <int G>
  __device__ __forceinline__ void columns_top2(const int32_t *Cs, int S, const int *js, Key *a1, int *ta1, Key *a2,
                                               int *ta2) {
    const bool in = cl && ((forest >> lane) & 1ull);
    const int li = in ? lane : 0;
    Key a[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int32_t vjj = __builtin_amdgcn_readlane(vj, js[g]);
      const int32_t c = Cs[li * S + js[g]];
      int64_t val;
      if constexpr (COMPACT) val = (int32_t)((uint32_t)c - (uint32_t)(uint64_t)h - (uint32_t)vjj);
      else val = (int64_t)c - h - vjj;
      bad |= in && (val < 0 || (COMPACT && val > kValMax));
      a[g] = in ? kpk(val < 0 ? 0 : val, lane) : KINF;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) a1[g] = wmin(a[g]);
#pragma unroll
    for (int g = 0; g < G; ++g) ta1[g] = a1[g] == KINF ? -1 : __builtin_amdgcn_readlane(rtree, kr(a1[g]));
#pragma unroll
    for (int g = 0; g < G; ++g) a2[g] = wmin(in && rtree != ta1[g] ? a[g] : KINF);
#pragma unroll
    for (int g = 0; g < G; ++g) ta2[g] = a2[g] == KINF ? -1 : __builtin_amdgcn_readlane(rtree, kr(a2[g]));
  }

  // Refresh the stale columns in mask R (two at a time).
  __device__ __forceinline__ void refresh(const int32_t *Cs, int S, uint64_t R) {
    while (R) {
      int js[2];
      js[0] = bit_of(R);
      R &= R - 1;
      Key a1[2], a2[2];
      int ta1[2], ta2[2];
      if (R) {
        js[1] = bit_of(R);
        R &= R - 1;
        columns_top2<2>(Cs, S, js, a1, ta1, a2, ta2);
      } else {
        columns_top2<1>(Cs, S, js, a1, ta1, a2, ta2);
        js[1] = js[0]; a1[1] = a1[0]; ta1[1] = ta1[0]; a2[1] = a2[0]; ta2[1] = ta2[0];
      }
#pragma unroll
      for (int g = 0; g < 2; ++g)
        if (lane == js[g]) { k1 = a1[g]; t1 = ta1[g]; k2 = a2[g]; t2 = ta2[g]; stl = false; }
    }
  }

  // Solve with C in LDS (row i at Cs[i * (n + 1)]) and mn = row minimum u_i
  // in lane i.
  __device__ __forceinline__ void solve(const Problem &P, int32_t *Cs, int mn) {
    n = P.n;
    lane = threadIdx.x & 63;
    cl = lane < n;
    const int S = n + 1;
    rmap = Cs + n * S;
    h = cl ? (int64_t)mn : 0;
    // ---- v_j = min_i (C_ij - u_i) and the two best rows of column j
    Key b1 = KINF, b2 = KINF;
    const int lc = cl ? lane : 0;
    for (int i0 = 0; i0 < n; i0 += 4) {
      int32_t c[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) c[q] = Cs[min(i0 + q, n - 1) * S + lc];  // four reads in flight
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (i0 + q >= n) break;
        const int ui = __builtin_amdgcn_readlane(mn, i0 + q);
        const Key key = kpk((int64_t)c[q] - ui, i0 + q);
        const bool lt1 = key < b1, lt2 = key < b2;
        b2 = lt1 ? b1 : (lt2 ? key : b2);
        b1 = lt1 ? key : b1;
      }
    }
    const int K = (P.max_paths <= 0 || P.max_paths > n) ? n : P.max_paths;
    vj = cl ? (int32_t)kv(b1) : 0;
    k1 = KINF; k2 = KINF; t1 = -1; t2 = -1;
    if (cl && K == n) {
      k1 = kpk(kv(b1) - vj, kr(b1));
      t1 = kr(b1);
      if (b2 != KINF) { k2 = kpk(kv(b2) - vj, kr(b2)); t2 = kr(b2); }
    }
    vis = false; stl = false; bad = false; dcol = 0; ctree = -1; par = -1; mcol = -1;
    mrow = -1; bend = kNoEnd;
    const uint64_t roots = K == 64 ? ~0ull : ((1ull << K) - 1);
    rtree = (cl && lane < K) ? lane : -1;
    alive = roots;
    forest = roots;
    front = K == n ? 0 : roots;  // with every row a root the keys above already hold the first sweep

    // counters fit 32 bits at n <= 64 (levels are at most 66^2 + 64), and
    // keeping them narrow keeps the loop's scalar registers from spilling
    int st_levels = 0, st_dual = 0, st_aug = 0, st_paths = 0, st_rows = 2 * n, st_gath = 0;
    int st_resw = 0, st_refresh = 0, st_rcols = 0;
    int err = 0;
    int nfree = n, nalive = K, cursor = K;
    int64_t D = 0;
    const int watchdog = (n + 2) * (n + 2) + 64;
    const int gcap = gather_cap(n);
    const bool timers = (P.flags & OT_FLAG_PHASE_TIMERS) != 0;
    // phase times in wall clock ticks (10 ns), 32-bit differences
    uint32_t tm_sweep = 0, tm_select = 0, tm_settle = 0, tm_aug = 0, tm_refresh = 0;

    while (nfree > 0) {
      // (1) fold the rows that joined last step into the keys
      const uint32_t tA = timers ? (uint32_t)now_ticks() : 0;
      st_rows += __builtin_popcountll(front);
      sweep(Cs, S, front);
      front = 0;
      const uint32_t tB = timers ? (uint32_t)now_ticks() : 0;
      tm_sweep += tB - tA;
      // (2) smallest key over unreached columns (stale keys are lower bounds)
      const bool open = cl && !vis && k1 != KINF;
      Key mv = wmin(open && !stl ? k1 : KINF);
      // stale keys are rare: their minimum only when there is one
      const Key ms = __builtin_amdgcn_ballot_w64(open && stl) ? wmin(open && stl ? k1 : KINF) : KINF;
      if (ms != KINF && (mv == KINF || kv(ms) <= kv(mv))) {
        const int64_t lim = mv == KINF ? INT64_MAX : kv(mv);
        uint64_t R = __builtin_amdgcn_ballot_w64(open && stl && kv(k1) <= lim);
        const int g = __builtin_popcountll(R);
        const uint32_t tR = timers ? (uint32_t)now_ticks() : 0;
        ++st_refresh;
        st_rcols += g;
        if (g > gcap) {
          // too many: one sweep of every forest row fixes all keys
          if (cl) { k1 = KINF; k2 = KINF; t1 = -1; t2 = -1; }
          stl = false;
          ++st_resw;
          st_rows += __builtin_popcountll(forest);
          sweep(Cs, S, forest);
        } else {
          st_gath += g * __builtin_popcountll(forest);
          refresh(Cs, S, R);
        }
        if (timers) tm_refresh += (uint32_t)now_ticks() - tR;
        const bool open2 = cl && !vis && k1 != KINF;
        mv = wmin(open2 && !stl ? k1 : KINF);
      }
      if (mv == KINF) { err = OT_EINTERNAL; break; }
      const int64_t level = kv(mv);
      if (level > D) { D = level; ++st_dual; }
      if (++st_levels > watchdog || D > kLevelMax) { err = OT_EINTERNAL; break; }
      const uint32_t tC = timers ? (uint32_t)now_ticks() : 0;
      tm_select += tC - tB;

      // (3) settle every unreached column at the current level
      const bool settle = cl && !vis && !stl && k1 != KINF && kv(k1) == D;
      const uint64_t Sm = __builtin_amdgcn_ballot_w64(settle);
      if (settle) { vis = true; dcol = (int32_t)D; ctree = t1; par = kr(k1); }
      // matched rows of settled columns join their column's tree
      const int src = (cl && mrow >= 0) ? mrow : lane;
      const int ttree = __builtin_amdgcn_ds_bpermute(src * 4, t1);
      const bool joins = cl && mrow >= 0 && ((Sm >> mrow) & 1ull);
      if (joins) { rtree = ttree; h -= D; }
      const uint64_t J = __builtin_amdgcn_ballot_w64(joins);
      front |= J;
      forest |= J;
      // free settled columns end paths: per tree its smallest such column
      uint64_t E = Sm & __builtin_amdgcn_ballot_w64(cl && mcol < 0), augm = 0;
      while (E) {
        const int j = bit_of(E);
        E &= E - 1;
        const int tr = __builtin_amdgcn_readlane(t1, j);
        if (!((augm >> tr) & 1ull)) {
          augm |= 1ull << tr;
          if (lane == tr) bend = j;
        }
      }
      const uint32_t tD = timers ? (uint32_t)now_ticks() : 0;
      tm_settle += tD - tC;
      if (augm) {
        // (4) flip one path per such tree (trees are disjoint).  The walks
        // only read (par, and the matches as they were before this step), so
        // each step is two lane reads with no write in between; the flips
        // are applied after all walks: every path column takes its parent
        // row, and that row takes the column (through the row map in LDS).
        const int naug = __builtin_popcountll(augm);
        uint64_t pcols = 0, prows = 0;
        for (uint64_t A = augm; A; A &= A - 1) {
          const int tr = bit_of(A);
          int j = __builtin_amdgcn_readlane(bend, tr);
          for (int steps = 0;; ++steps) {
            if (steps > n || (unsigned)j >= (unsigned)n) { err = OT_EINTERNAL; break; }
            const int p = __builtin_amdgcn_readlane(par, j);
            if ((unsigned)p >= (unsigned)n) { err = OT_EINTERNAL; break; }
            pcols |= 1ull << j;
            prows |= 1ull << p;
            if (lane == 0) rmap[p] = j;
            if (p == tr) break;
            j = __builtin_amdgcn_readlane(mrow, p);
          }
        }
        if (err) break;
        if ((pcols >> lane) & 1ull) mcol = par;
        if ((prows >> lane) & 1ull) mrow = rmap[lane];
        if ((augm >> lane) & 1ull) bend = kNoEnd;
        alive &= ~augm;
        ++st_aug;
        st_paths += naug;
        nfree -= naug;
        nalive -= naug;
        // (5) rows and columns of finished trees leave the forest with their duals materialised
        if (cl && rtree >= 0 && !alive_tree(rtree)) { h += D; rtree = -1; }
        forest = __builtin_amdgcn_ballot_w64(cl && rtree >= 0);
        front &= forest;  // rows that joined this step a tree that just finished
        if (cl) {
          if (vis && !alive_tree(ctree)) {
            const int64_t d = D - dcol;
            vj -= (int32_t)d;
            const Key sh = (Key)d << KB;
            if (k1 != KINF) k1 += sh;
            if (k2 != KINF) k2 += sh;
            vis = false;
            ctree = -1;
          }
          if (t1 >= 0 && !alive_tree(t1)) { k1 = k2; t1 = t2; t2 = -1; }
          else if (t2 >= 0 && !alive_tree(t2)) t2 = -1;
          if (nalive == 0) { k1 = KINF; k2 = KINF; t1 = -1; t2 = -1; }
          stl = !(k1 == KINF || alive_tree(t1));
        }
        // (6) with a tree cap, start new trees from the next free rows
        const int need = min(K - nalive, n - cursor);
        if (need > 0) {
          const uint64_t nr = (need == 64 ? ~0ull : ((1ull << need) - 1)) << cursor;
          if ((nr >> lane) & 1ull) { rtree = lane; h -= D; }
          alive |= nr;
          forest |= nr;
          front |= nr;
          cursor += need;
          nalive += need;
        }
        if (timers) tm_aug += (uint32_t)now_ticks() - tD;
      }
    }
    if (err == 0 && __builtin_amdgcn_ballot_w64(bad) != 0) err = OT_EINTERNAL;

    if (err == 0) {
      int64_t part = 0;
      if (cl) {
        P.plan[lane] = mrow;
        if (P.u) P.u[lane] = h * P.dscale;
        if (P.v) P.v[lane] = (int64_t)vj * P.dscale;
        if (mrow >= 0 && mrow < n)  // the total over C is read from its copy in LDS
          part = P.Cout ? (int64_t)P.Cout[(size_t)lane * (size_t)P.ldo + mrow] : (int64_t)Cs[lane * S + mrow];
      }
      part = wave_sum_i64(part);
      if (lane == 0) *P.cost = part;
    }
    if (P.stats && lane == 0) {
      ot_stats s = {};
      s.levels = st_levels; s.dual_adjusts = st_dual; s.aug_events = st_aug; s.paths = st_paths;
      s.rows_swept = st_rows; s.gathers = st_gath; s.resweeps = st_resw; s.status = err;
      s.refreshes = st_refresh; s.refresh_cols = st_rcols;
      s.t_sweep_ns = 10 * (int64_t)tm_sweep; s.t_select_ns = 10 * (int64_t)tm_select;
      s.t_settle_ns = 10 * (int64_t)tm_settle; s.t_augment_ns = 10 * (int64_t)tm_aug;
      s.t_refresh_ns = 10 * (int64_t)tm_refresh;
      *P.stats = s;
    }
  }
};

struct WaveEngine {
  __device__ __forceinline__ void run(const Problem &P, char *smem) {
    const int n = P.n, lane = threadIdx.x & 63;
    const bool cl = lane < n;
    const int S = n + 1;
    int32_t *Cs = (int32_t *)smem;
    // ---- C into LDS (row i at Cs[i * S])
    // sixteen rows' loads in flight at a time (every lane loads: rows and
    // columns past n read entry (0, 0) and store nothing)
    for (int i0 = 0; i0 < n; i0 += 16) {
      int32_t c[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const bool in = i0 + q < n && cl;
        c[q] = P.C[in ? (size_t)(i0 + q) * (size_t)P.ld + lane : 0];
      }
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (i0 + q < n && cl) Cs[(i0 + q) * S + lane] = c[q];
    }
    __syncthreads();
    // ---- u_i = min_j C_ij (lane i) and the cost range
    int mn = 0x7fffffff, mx = (int)0x80000000;
    if (cl)
      for (int k = 0; k < n; ++k) {
        const int32_t c = Cs[lane * S + k];
        mn = min(mn, c);
        mx = max(mx, c);
      }
    const int gmin = wave_min_i32(cl ? mn : 0x7fffffff), gmax = wave_max_i32(cl ? mx : (int)0x80000000);
    const int64_t range = (int64_t)gmax - (int64_t)gmin;
    if (range > 0x7fffffffll) {
      if (P.stats && lane == 0) { ot_stats s = {}; s.status = OT_ERANGE; *P.stats = s; }
      return;
    }
    // compact keys: a key value stays below 3 x the range when every free row is a root
    const bool all_roots = P.max_paths <= 0 || P.max_paths >= n;
    if (range < kCompactRange && all_roots && !(P.flags & OT_FLAG_WIDE_KEYS)) {
      WaveCore<true> W;
      W.solve(P, Cs, mn);
    } else {
      WaveCore<false> W;
      W.solve(P, Cs, mn);
    }
  }
};

}  // namespace otkm
