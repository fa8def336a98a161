// bins_engine.hpp -- Batched KM on bins: the integer transportation problem of
// Eq. (1) solved on the supply and demand bins themselves, without expanding
// every unit of mass into its own vertex.
//
// It is the primal-dual (Hungarian) method for the transportation problem,
// organised as Batched KM (Section 2.3.1): alternating trees grow at once from
// every row bin that still has supply, over tight edges; a tree that reaches a
// column bin with demand left ships along its path as much as the path allows
// (the root's supply left, the end's demand left, and the flow on every
// backward arc); when no tree can grow, the duals move across the cut by the
// smallest slack.  Compared with the assignment engine:
//   * a column is left through every row that already ships to it (backward
//     arcs of positive flow, which are tight), not through one matched row;
//   * a path carries an integer amount, so its root may keep supply and then
//     starts a new tree at the current level, and its end may keep demand;
//   * flows live in global memory, column-major (XT[j * n + i] = x_ij), so a
//     column's backward arcs are one contiguous read.
// The sweep, minimum selection, stale-key refresh and lazy duals are the
// assignment engine's (Engine), unchanged.
//
// Ranges: with the KM reduction as the start, a column with demand left has
// never moved, so a row with supply left satisfies u_i <= max C and the level
// D (the rise of such a row) stays below R = max C - min C, as in the
// assignment engine: keys and per-column values fit the same words.
#pragma once

#include "engine.hpp"

namespace otkm {

// LDS of the bin engine: the assignment engine's layout for max(n, m) bins,
// then the supply left per row, the number of positive flows per column, the
// columns to leave through their flows at one level (all int32), and three
// control words (a count and a 64-bit total).
struct BinsLds {
  size_t rs, cflow, xlist, bctl, total;
};
__host__ __device__ inline BinsLds bins_lds(int n, int m) {
  BinsLds L;
  size_t o = lds_layout(n > m ? n : m).total;
  L.rs = o;    o = align16(o + 4 * (size_t)n);
  L.cflow = o; o = align16(o + 4 * (size_t)m);
  L.xlist = o; o = align16(o + 4 * (size_t)m);
  L.bctl = o;  o = align16(o + 16);
  L.total = o;
  return L;
}

struct BinsProblem {
  const int32_t *C;        // n x m costs, row stride ld
  const int32_t *CT;       // its transpose (m x n, row stride n), or null
  int n, m, ld;
  // the KM reduction's sweeps (k_init_rows / k_init_cols / k_init_merge over C):
  const int64_t *init_u;     // [n] row minima
  const uint64_t *init_b;    // [m][2] per column the two smallest keys pack(C_ij - u_i, i)
  const int32_t *init_rmax;  // [n] row maxima
  const int32_t *r, *c;    // [n], [m] masses (>= 0, equal sums: checked before the launch)
  int32_t *XT;             // [m][n] flows, zero before the launch
  int64_t *u, *v;          // [n], [m] duals out
  ot_stats *stats;         // [1] or null
  int32_t *ws;             // ws_ints(max(n, m))
};

template <int BLOCK, int CPT>
struct BinEngine : Engine<BLOCK, CPT, true, false, true> {
  using E = Engine<BLOCK, CPT, true, false, true>;
  using E::C; using E::CT; using E::n; using E::ld; using E::nr_; using E::ldt; using E::hrow; using E::mrow;
  using E::mcol; using E::rtree; using E::par; using E::fst; using E::fr; using E::alive; using E::gcol; using E::gv;
  using E::gk1; using E::gk2; using E::gt1; using E::gt2; using E::red; using E::ctl; using E::gcap; using E::auglist;
  using E::bend; using E::k1; using E::k2; using E::t1; using E::t2; using E::ctree; using E::vj; using E::dcol;
  using E::narrow; using E::vis; using E::stl; using E::tid; using E::lane; using E::wid; using E::err_local;
  using E::crsrc; using E::voff; using E::NW;
  using E::col; using E::lcol; using E::stale; using E::fail; using E::recompute_stale; using E::sweep_frontier;
  using E::reduce_min; using E::reset_slots; using E::refresh_stale; using E::frontier_rec;

  int32_t *rs;     // [n] supply left per row
  int32_t *cflow;  // [m] positive flows per column
  int32_t *xlist;  // [m] columns settled this level that are left through their flows
  int32_t *xcnt;   // its length
  unsigned long long *shipped;  // units shipped at this level
  int32_t *XT;

  // x_ij: column j's flows are contiguous
  __device__ __forceinline__ int32_t &x(int i, int j) { return XT[(size_t)j * (size_t)nr_ + (size_t)i]; }

  __device__ __forceinline__ void run(const BinsProblem &P, char *smem) {
    C = P.C; CT = P.CT; n = P.m; ld = P.ld; nr_ = P.n; ldt = P.n;
    const int nr = nr_, nc = n;
    XT = P.XT;
    tid = threadIdx.x; lane = tid & 63; wid = tid >> 6;
    err_local = 0;
    {
      const int64_t extent = ((int64_t)(nr - 1) * ld + nc) * 4;
      crsrc = __builtin_amdgcn_make_buffer_rsrc((void *)C, (short)0, (int)(extent < 0x7fffffff ? extent : 0x7fffffff),
                                                0x00020000);
    }
    const int B = nr > nc ? nr : nc;
    const LdsLayout L = lds_layout(B);
    hrow = (int64_t *)(smem + L.hrow);
    mrow = (int32_t *)(smem + L.mrow);   // row -> the column it joined through (rpar)
    mcol = (int32_t *)(smem + L.mcol);   // column -> demand left
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
    const BinsLds BL = bins_lds(nr, nc);
    rs = (int32_t *)(smem + BL.rs);
    cflow = (int32_t *)(smem + BL.cflow);
    xlist = (int32_t *)(smem + BL.xlist);
    shipped = (unsigned long long *)(smem + BL.bctl);
    xcnt = (int32_t *)(smem + BL.bctl + 8);
    int32_t *rpar = mrow, *rd = mcol;
    gcap = gather_cap(nc);
    auglist = P.ws;
    bend = auglist + B;
#pragma unroll
    for (int k = 0; k < CPT; ++k) voff[k] = lcol(k) * 4;

    int64_t st_levels = 0, st_dual = 0, st_aug = 0, st_paths = 0, st_rows = 0, st_gath = 0, st_resw = 0;
    int64_t st_refresh = 0, st_rcols = 0;
    if (tid < NCTL) ctl[tid] = 0;
    if (tid == 0) { *shipped = 0; *xcnt = 0; }
    if (tid < 8) red[tid] = kInf;

    // ---- u_i = min_j C_ij and the cost range, from the reduction's row sweep
    int gmin = 0x7fffffff, gmax = (int)0x80000000;
    for (int i = tid; i < nr; i += BLOCK) {
      const int64_t mn = P.init_u[i];
      hrow[i] = mn;
      gmin = min(gmin, (int)mn);
      gmax = max(gmax, P.init_rmax[i]);
    }
    int64_t left_part = 0;
    for (int i = tid; i < nr; i += BLOCK) {
      const int ri = P.r[i];
      rs[i] = ri;
      left_part += ri;
      mrow[i] = -1;
      rtree[i] = ri > 0 ? i : -1;
      alive[i] = ri > 0 ? 1 : 0;
    }
    for (int j = tid; j < nc; j += BLOCK) { rd[j] = P.c[j]; cflow[j] = 0; par[j] = (int16_t)-1; }
    for (int j = tid; j < B; j += BLOCK) bend[j] = kNoEnd;
    gmin = wave_min_i32(gmin);
    gmax = wave_max_i32(gmax);
    left_part = wave_sum_i64(left_part);
    int *ired = (int *)(red + 16);
    int64_t *lred = (int64_t *)(red + 32);
    if (lane == 0) { ired[wid] = gmin; ired[NW + wid] = gmax; lred[wid] = left_part; }
    __syncthreads();
    gmin = 0x7fffffff; gmax = (int)0x80000000;
    int64_t left = 0;
    for (int w = 0; w < NW; ++w) { gmin = min(gmin, ired[w]); gmax = max(gmax, ired[NW + w]); left += lred[w]; }
    narrow = (int64_t)gmax - (int64_t)gmin < (1ll << 30);
    if ((int64_t)gmax - (int64_t)gmin > 0x7fffffffll) {
      if (P.stats && tid == 0) { ot_stats s = {}; s.status = OT_ERANGE; *P.stats = s; }
      return;
    }

    // ---- v_j = min_i (C_ij - u_i); the keys start empty (the first level sweeps every root)
    vis = 0;
    stl = 0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      k1[k] = kInf; k2[k] = kInf; t1[k] = -1; t2[k] = -1; dcol[k] = 0; ctree[k] = -1;
      vj[k] = col(k) < nc ? (int32_t)kval(P.init_b[2 * (size_t)col(k)]) : 0;
    }
    st_rows = 2 * (int64_t)nr;
    // roots: every row with supply, listed by a ballot per 64 rows
    if (tid == 0) { ctl[CNT0] = 0; ctl[CNT1] = 0; ctl[FCNT] = 0; }
    __syncthreads();
    for (int i0 = wid * 64; i0 < nr; i0 += BLOCK) {
      const int i = i0 + lane;
      const bool root = i < nr && rs[i] > 0;
      const uint64_t msk = __builtin_amdgcn_ballot_w64(root);
      int base = 0;
      if (lane == 0 && msk != 0) base = atomicAdd(&ctl[FCNT], (int)__builtin_popcountll(msk));
      base = __builtin_amdgcn_readfirstlane(base);
      const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(msk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)msk, 0));
      if (root) { fst[base + rank] = i; fr[base + rank] = frontier_rec(i, i, hrow[i]); }
    }
    __syncthreads();
    if (tid == 0) ctl[CNT0] = ctl[FCNT];
    __syncthreads();

    int cur = 0;
    int64_t D = 0;
    // every nc + 1 levels at least one path ships at least one unit
    const int64_t watchdog = (left + nr + nc) * (int64_t)(nc + 2) + 4096;

    while (left > 0) {
      const int ps = cur;
      // (1) fold the rows that joined last step into the keys
      const int nf = ctl[cur == 0 ? CNT0 : CNT1];
      st_rows += sweep_frontier(nf);
      // (2) smallest key over unreached columns
      reduce_min(ps, ERRA0 + ps);
      if (tid == 0) {
        ctl[cur == 0 ? CNT1 : CNT0] = 0; ctl[NAUG] = 0; ctl[GCNT] = 0; *xcnt = 0;
        reset_slots(ps ^ 1, ERRA0 + (ps ^ 1));
        reset_slots(2 + (ps ^ 1), ERRB0 + (ps ^ 1));
      }
      __syncthreads();
      uint64_t mv = red[2 * ps], ms = red[2 * ps + 1];
      int berr = ctl[ERRA0 + ps];
      if (berr == 0 && ms != kInf && (mv == kInf || kval(ms) <= kval(mv))) {
        bool resweep;
        int swept;
        st_gath += refresh_stale(mv, resweep, swept);
        ++st_refresh;
        st_rcols += ctl[GCNT];
        if (resweep) { ++st_resw; st_rows += swept; }
        reduce_min(2 + ps, ERRB0 + ps);
        __syncthreads();
        mv = red[2 * (2 + ps)];
        berr = ctl[ERRB0 + ps];
      }
      if (berr != 0) break;
      if (mv == kInf) { fail(OT_EINTERNAL); break; }
      const int64_t level = kval(mv);
      if (level > D) { D = level; ++st_dual; }
      if (++st_levels > watchdog || D > 0x7ffffffell) { fail(OT_EINTERNAL); break; }

      // (3) settle every unreached column at the current level: a column with
      // demand left ends its tree's path; a column with flows is left through
      // them (listed for (3b)); the list of the next sweep is rebuilt below
      int *nxtcnt = &ctl[cur == 0 ? CNT1 : CNT0];
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        const int j = col(k);
        if (j >= nc || ((vis >> k) & 1u) || k1[k] == kInf || stale(k) || kval(k1[k]) != D) continue;
        const int tr = t1[k];
        vis |= 1u << k;
        dcol[k] = (int32_t)D;
        ctree[k] = tr;
        par[j] = (int16_t)krow(k1[k]);
        if (rd[j] > 0) {
          if (atomicMin(&bend[tr], j) == kNoEnd) auglist[atomicAdd(&ctl[NAUG], 1)] = tr;
        } else if (cflow[j] > 0) {
          xlist[atomicAdd(xcnt, 1)] = j;
        }
      }
      __syncthreads();
      // (3b) rows that ship to a settled column join its tree (one wavefront
      // per column; a row reached through two columns joins once)
      const int nx = *xcnt;
      for (int q = wid; q < nx; q += NW) {
        const int j = xlist[q];
        const int tr = rtree[par[j]];
        const int32_t *xc = XT + (size_t)j * (size_t)nr;
        for (int i = lane; i < nr; i += 64) {
          if (xc[i] <= 0 || rtree[i] >= 0) continue;
          if (atomicCAS(&rtree[i], -1, tr) != -1) continue;
          mrow[i] = j;
          const int64_t h = hrow[i] - D;
          hrow[i] = h;
          fr[atomicAdd(nxtcnt, 1)] = frontier_rec(i, tr, h);
          fst[atomicAdd(&ctl[FCNT], 1)] = i;
        }
      }
      __syncthreads();
      const int naug = ctl[NAUG];
      if (naug > 0) {
        // (4) ship along one path per tree that reached a column with demand
        // (trees are disjoint, so are their paths)
        for (int a = tid; a < naug; a += BLOCK) {
          const int tr = auglist[a];
          const int je = bend[tr];
          bend[tr] = kNoEnd;
          bool ok = (unsigned)je < (unsigned)nc;
          int64_t amt = ok ? rd[je] : 0;
          int j = je, steps = 0;
          while (ok) {  // bottleneck: the end's demand, every backward arc, the root's supply
            const int p = par[j];
            if ((unsigned)p >= (unsigned)nr || ++steps > nr + nc) { ok = false; break; }
            if (p == tr) { amt = min(amt, (int64_t)rs[p]); break; }
            const int jp = rpar[p];
            if ((unsigned)jp >= (unsigned)nc) { ok = false; break; }
            amt = min(amt, (int64_t)x(p, jp));
            j = jp;
          }
          if (!ok || amt <= 0) { fail(OT_EINTERNAL); alive[tr] = 0; continue; }
          for (j = je;;) {
            const int p = par[j];
            if (x(p, j) == 0) atomicAdd(&cflow[j], 1);
            x(p, j) += (int32_t)amt;
            if (p == tr) { rs[p] -= (int32_t)amt; break; }
            const int jp = rpar[p];
            x(p, jp) -= (int32_t)amt;
            if (x(p, jp) == 0) atomicAdd(&cflow[jp], -1);
            j = jp;
          }
          rd[je] -= (int32_t)amt;
          atomicAdd(shipped, (unsigned long long)amt);
          alive[tr] = 0;
        }
        ++st_aug;
        st_paths += naug;
        __syncthreads();
        left -= (int64_t)*shipped;
        __syncthreads();
        if (tid == 0) *shipped = 0;
        // (5) every tree leaves the forest with its duals materialised, not only
        // those that shipped: a row can ship to several columns, and once one of
        // them leaves while the row stays (or the reverse), the next dual move
        // would take that flow off a tight edge.  So each round that ships ends
        // the forest, as a phase of the primal-dual method ends its labels.
        for (int i = tid; i < nr; i += BLOCK) {
          if (rtree[i] >= 0) { hrow[i] += D; rtree[i] = -1; }
          alive[i] = 0;
        }
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
          if (col(k) < nc && ((vis >> k) & 1u)) vj[k] -= (int32_t)(D - dcol[k]);
          k1[k] = kInf; k2[k] = kInf; t1[k] = -1; t2[k] = -1; ctree[k] = -1;
        }
        vis = 0;
        stl = 0;
        if (tid == 0) { ctl[FCNT] = 0; *nxtcnt = 0; }
        __syncthreads();
        // (6) every row with supply left starts a new tree at the current level
        for (int i0 = wid * 64; i0 < nr; i0 += BLOCK) {
          const int i = i0 + lane;
          const bool root = i < nr && rs[i] > 0;
          const uint64_t msk = __builtin_amdgcn_ballot_w64(root);
          int base = 0;
          if (lane == 0 && msk != 0) base = atomicAdd(&ctl[FCNT], (int)__builtin_popcountll(msk));
          base = __builtin_amdgcn_readfirstlane(base);
          const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(msk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)msk, 0));
          if (root) {
            rtree[i] = i;
            alive[i] = 1;
            const int64_t h = hrow[i] - D;
            hrow[i] = h;
            fst[base + rank] = i;
            fr[base + rank] = frontier_rec(i, i, h);
          }
        }
        __syncthreads();
        if (tid == 0) *nxtcnt = ctl[FCNT];
        __syncthreads();
      }
      cur ^= 1;
    }

    __syncthreads();
    if (err_local != 0) atomicMin(&ctl[ERR], err_local);
    __syncthreads();
    const int err = ctl[ERR];
    if (err == 0) {
      for (int i = tid; i < nr; i += BLOCK) P.u[i] = hrow[i];
#pragma unroll
      for (int k = 0; k < CPT; ++k)
        if (col(k) < nc) P.v[col(k)] = (int64_t)vj[k];
    }
    if (P.stats && tid == 0) {
      ot_stats s = {};
      s.levels = st_levels; s.dual_adjusts = st_dual; s.aug_events = st_aug; s.paths = st_paths;
      s.rows_swept = st_rows; s.gathers = st_gath; s.resweeps = st_resw; s.status = err;
      s.refreshes = st_refresh; s.refresh_cols = st_rcols;
      *P.stats = s;
    }
  }
};

}  // namespace otkm
