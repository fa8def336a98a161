// auction.hip -- the auction algorithm with epsilon-scaling (Section 2.3.3):
// kernel and the C-ABI calls ot_auction and ot_auction_dev.
//
// Rows bid for columns with rewards R_ij = -C_ij, scaled by (n + 1) so that
// all arithmetic is exact integer and a slack of eps = 1 on that scale is
// eps < 1/n on the costs (the paper's condition for an exact result with
// integer weights; in general the plan is within n * eps of the optimum).
//
// One workgroup of 1024 threads solves one instance with every piece of
// state in LDS (prices, pending bids, owners, the row -> column map and the
// lists of unassigned rows: 36n + 576 bytes, 148.0 KB at n = 4096).  Bidding
// is Jacobi style, the parallel form the paper points to: in a round every
// unassigned row bids at once (one wavefront per bidder scans its cost row,
// coalesced), a bid is one 64-bit LDS atomic maximum of (price << 12 | row)
// on its column, and after one barrier each bidder learns whether it won.
// Two barriers a round; the rows that lost or were evicted form the next
// round's list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <mutex>

#include "otkm.h"
#include "runtime.hpp"

namespace otkm {
namespace {

constexpr int kAucBlock = 1024;
constexpr int kAucWaves = kAucBlock / 64;
constexpr int kAucRowBits = 12;                         // n <= 4096
constexpr int kAucLoads = 32;                           // cost loads in flight per lane
constexpr int64_t kAucBidLimit = (int64_t)1 << 51;      // a packed bid is price << 12 | row
constexpr int64_t kAucRoundLimit = (int64_t)1 << 22;    // every launch ends
constexpr int64_t kAucEpsLimit = (int64_t)1 << 50;

struct AuctionArgs {
  const int32_t *C;
  int n, ld;
  int64_t eps0, eps_final;
  int theta;
  int32_t *plan;
  int64_t *cost, *price;  // price may be null
  ot_stats *stats;        // may be null
};

__host__ __device__ inline size_t auction_lds_bytes(int n) { return (size_t)n * 36 + 576; }

// Wavefront reductions (all 64 lanes active): rotations inside each 16-lane
// row (DPP), then the four row results through scalar reads; uniform result.
template <int CTRL>
__device__ __forceinline__ int64_t dpp_i64(int64_t x) {
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)(uint64_t)x, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)((uint64_t)x >> 32), CTRL, 0xf, 0xf, false);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int64_t lane_i64(int64_t x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int64_t wave_max_i64(int64_t x) {
  x = max(x, dpp_i64<0x121>(x));  // row_ror:1
  x = max(x, dpp_i64<0x122>(x));  // row_ror:2
  x = max(x, dpp_i64<0x124>(x));  // row_ror:4
  x = max(x, dpp_i64<0x128>(x));  // row_ror:8
  return max(max(lane_i64(x, 0), lane_i64(x, 16)), max(lane_i64(x, 32), lane_i64(x, 48)));
}
__device__ __forceinline__ int wave_min_int(int x) {
  x = min(x, __builtin_amdgcn_update_dpp(INT_MAX, x, 0x121, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(INT_MAX, x, 0x122, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(INT_MAX, x, 0x124, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(INT_MAX, x, 0x128, 0xf, 0xf, false));
  return min(min(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16)),
             min(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48)));
}

// One lane's running best value (column j1) and best value over its other
// columns; columns arrive in increasing order, so a tie keeps the smaller.
struct Top2 {
  int64_t b1 = INT64_MIN, b2 = INT64_MIN;
  int j1 = INT_MAX;
  __device__ __forceinline__ void push(int64_t val, int j) {
    if (val > b1) { b2 = b1; b1 = val; j1 = j; }
    else if (val > b2) b2 = val;
  }
  // merge another lane-local summary (a tie goes to the smaller column)
  __device__ __forceinline__ void merge(const Top2 &o) {
    if (o.b1 > b1 || (o.b1 == b1 && o.j1 < j1)) {
      b2 = max(o.b2, b1); b1 = o.b1; j1 = o.j1;
    } else {
      b2 = max(b2, o.b1);
    }
  }
};

// One lane's top-2 over the columns [js, je) of a cost row: all its loads
// (up to 32 a lane) issued before any is used, two independent chains.
__device__ __forceinline__ Top2 scan_row(const int32_t *row, int js, int je, int n, int lane, const int64_t *price,
                                         int64_t scale) {
  Top2 ta, tb;
  for (int j0 = js; j0 < je; j0 += kAucLoads * 64) {
    int32_t c[kAucLoads];
#pragma unroll
    for (int q = 0; q < kAucLoads; ++q) {
      const int j = j0 + q * 64 + lane;
      c[q] = row[j < je ? j : n - 1];
    }
#pragma unroll
    for (int q = 0; q < kAucLoads; ++q) {
      const int j = j0 + q * 64 + lane;
      if (j < je) {
        const int64_t val = -(int64_t)c[q] * scale - price[j];
        if (q & 1) tb.push(val, j);
        else ta.push(val, j);
      }
    }
  }
  ta.merge(tb);
  return ta;
}

// The wavefront's best value v1, its smallest column jb, and the best value
// over the other columns v2 (uniform).
__device__ __forceinline__ void wave_top2(const Top2 &t, int64_t &v1, int &jb, int64_t &v2) {
  v1 = wave_max_i64(t.b1);
  jb = wave_min_int(t.b1 == v1 ? t.j1 : INT_MAX);
  v2 = wave_max_i64(t.j1 == jb ? t.b2 : t.b1);
}

// Bid of list entry e (row i) for column jb: the price rises by the gap to
// the second-best value plus eps, as an atomic maximum of price << 12 | row.
__device__ __forceinline__ void place_bid(int e, int i, int jb, int64_t v1, int64_t v2, int64_t eps,
                                          const int64_t *price, unsigned long long *bid, int32_t *bidobj, int *ctl,
                                          int64_t *red) {
  const int64_t nb = price[jb] + (v1 - v2) + eps;
  if (nb >= kAucBidLimit) {
    atomicOr(&ctl[2], 1);
    bidobj[e] = -1;
  } else {
    atomicMax(&bid[jb], ((unsigned long long)nb << kAucRowBits) | (unsigned long long)i);
    bidobj[e] = jb;
  }
  atomicAdd((unsigned long long *)&red[16], 1ull);
}

__global__ __launch_bounds__(kAucBlock) void k_auction(AuctionArgs A) {
  extern __shared__ __align__(16) char smem[];
  const int n = A.n;
  int64_t *price = (int64_t *)smem;                                  // [n]
  unsigned long long *bid = (unsigned long long *)(smem + 8 * (size_t)n);  // [n], 0 = none
  int64_t *red = (int64_t *)(smem + 16 * (size_t)n);                 // [24]: cost partials, [16] bids
  int64_t *pv1 = red + 24, *pv2 = red + 40;                          // [16] each: slice top-2 values
  int32_t *pj = (int32_t *)(red + 56);                               // [16]: slice best columns
  int32_t *owner = (int32_t *)(smem + 16 * (size_t)n + 512);         // [n] row holding column j
  int32_t *rowobj = owner + n;                                       // [n] column held by row i
  int32_t *list0 = rowobj + n;                                       // [n] unassigned rows
  int32_t *list1 = list0 + n;                                        // [n]
  int32_t *bidobj = list1 + n;                                       // [n] column bid by list entry e
  int *ctl = bidobj + n;                                             // [16]
  // ctl[0], ctl[1]: entry counts of list0 / list1; ctl[2]: error
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t scale = (int64_t)n + 1;

  for (int j = tid; j < n; j += kAucBlock) { price[j] = 0; bid[j] = 0; }
  if (tid == 0) { ctl[2] = 0; red[16] = 0; }
  int64_t eps = A.eps0, rounds = 0;
  int phases = 0, err = 0;
  for (;;) {
    // a phase: every row unassigned, the prices of the previous phase kept
    for (int j = tid; j < n; j += kAucBlock) { owner[j] = -1; rowobj[j] = -1; list0[j] = j; }
    if (tid == 0) { ctl[0] = n; ctl[1] = 0; }
    __syncthreads();
    ++phases;
    int cur = 0, cnt = n;
    while (cnt > 0) {
      if (++rounds > kAucRoundLimit) { err = OT_EINTERNAL; break; }  // uniform
      const int32_t *lc = cur ? list1 : list0;
      int32_t *ln = cur ? list0 : list1;
      // the next round's count: last read before the previous round's end
      if (tid == 0) ctl[cur ^ 1] = 0;
      if (cnt * 2 <= kAucWaves && n > kAucLoads * 64) {
        // (1a) few bidders on rows longer than one batch of loads: G
        // wavefronts share each bidder's row (G a power of two, cnt * G <=
        // 16), each scanning one contiguous slice, and publish their slice's
        // top-2; then one thread per bidder merges the slices in column order
        // and bids (measured: 1252 -> 1029 ms at n = 4096; at n <= 2048 the
        // extra barrier costs more than the shorter scan saves)
        int G = kAucWaves;
        while (cnt * G > kAucWaves) G >>= 1;
        if (wid < cnt * G) {
          const int e = wid / G, g = wid % G;
          const int seg = (n + G - 1) / G;
          const int js = min(n, g * seg), je = min(n, js + seg);
          const Top2 t = scan_row(A.C + (size_t)lc[e] * (size_t)A.ld, js, je, n, lane, price, scale);
          int64_t v1, v2;
          int jb;
          wave_top2(t, v1, jb, v2);
          if (lane == 0) { pv1[wid] = v1; pv2[wid] = v2; pj[wid] = jb; }
        }
        __syncthreads();
        if (tid < cnt) {
          const int e = tid;
          int64_t v1 = pv1[e * G], v2 = pv2[e * G];
          int jb = pj[e * G];
          for (int g = 1; g < G; ++g) {  // slices in increasing column order: a tie keeps the earlier column
            const int64_t o1 = pv1[e * G + g], o2 = pv2[e * G + g];
            if (o1 > v1) { v2 = max(o2, v1); v1 = o1; jb = pj[e * G + g]; }
            else v2 = max(v2, o1);
          }
          place_bid(e, lc[e], jb, v1, n == 1 ? v1 : v2, eps, price, bid, bidobj, ctl, red);
        }
      } else {
        // (1b) bids: wavefront w takes the entries w, w + 16, ...
        for (int e = wid; e < cnt; e += kAucWaves) {
          const Top2 t = scan_row(A.C + (size_t)lc[e] * (size_t)A.ld, 0, n, n, lane, price, scale);
          int64_t v1, v2;
          int jb;
          wave_top2(t, v1, jb, v2);
          if (lane == 0) place_bid(e, lc[e], jb, v1, n == 1 ? v1 : v2, eps, price, bid, bidobj, ctl, red);
        }
      }
      __syncthreads();
      if (ctl[2]) { err = OT_ERANGE; break; }  // uniform
      // (2) each bidder learns its result; the winner of a column reads the
      // bid before clearing it, so a bidder that reads 0 or another row lost
      for (int e = tid; e < cnt; e += kAucBlock) {
        const int i = lc[e];
        const int jb = bidobj[e];
        const unsigned long long b = bid[jb];
        if (b != 0 && (int)(b & ((1u << kAucRowBits) - 1)) == i) {
          bid[jb] = 0;
          const int old = owner[jb];
          if (old >= 0) {
            rowobj[old] = -1;
            ln[atomicAdd(&ctl[cur ^ 1], 1)] = old;  // evicted: bids again
          }
          owner[jb] = i;
          rowobj[i] = jb;
          price[jb] = (int64_t)(b >> kAucRowBits);
        } else {
          ln[atomicAdd(&ctl[cur ^ 1], 1)] = i;  // outbid: bids again
        }
      }
      __syncthreads();
      cnt = ctl[cur ^ 1];
      cur ^= 1;
    }
    if (err || eps == A.eps_final) break;
    eps = max(A.eps_final, eps / A.theta);
    __syncthreads();  // the next phase rewrites the lists and counts read above
  }

  if (err == 0) {
    int64_t part = 0;
    for (int i = tid; i < n; i += kAucBlock) {
      const int j = rowobj[i];
      A.plan[i] = j;
      part += A.C[(size_t)i * (size_t)A.ld + (size_t)j];
    }
    if (A.price)
      for (int j = tid; j < n; j += kAucBlock) A.price[j] = price[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += (int64_t)__shfl_xor((long long)part, off, 64);
    if (lane == 0) red[wid] = part;
    __syncthreads();
    if (tid == 0) {
      int64_t total = 0;
      for (int w = 0; w < kAucWaves; ++w) total += red[w];
      *A.cost = total;
    }
  }
  if (tid == 0 && A.stats) {
    ot_stats s = {};
    s.levels = rounds;
    s.aug_events = phases;
    s.paths = err ? 0 : n;
    s.rows_swept = red[16];
    s.status = err;
    *A.stats = s;
  }
}

int auction_check(int32_t n, int64_t eps0, int32_t theta, int64_t eps_final) {
  if (n <= 0 || theta < 2 || eps_final < 1 || eps0 < eps_final) return OT_EINVAL;
  if (n > OT_MAX_N) return OT_ETOOBIG;
  if (eps0 >= kAucEpsLimit) return OT_ERANGE;
  return OT_OK;
}

hipError_t launch_auction(const AuctionArgs &A, hipStream_t s) {
  const size_t lds = auction_lds_bytes(A.n);
  hipError_t e = hipFuncSetAttribute((const void *)k_auction, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_auction, dim3(1), dim3(kAucBlock), lds, s, A);
  return hipGetLastError();
}

}  // namespace
}  // namespace otkm

using namespace otkm;

extern "C" {

int ot_auction_dev(const int32_t *dC, int32_t n, int32_t ld, int64_t eps0, int32_t theta, int64_t eps_final,
                   int32_t *dplan, int64_t *dcost, int64_t *dprice, ot_stats *dstats, void *stream) {
  if (!dC || !dplan || !dcost || ld < n) return OT_EINVAL;
  int rc = auction_check(n, eps0, theta, eps_final);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(lib_mutex());
  if ((rc = init_locked())) return rc;
  AuctionArgs A;
  A.C = dC; A.n = n; A.ld = ld; A.eps0 = eps0; A.eps_final = eps_final; A.theta = theta;
  A.plan = dplan; A.cost = dcost; A.price = dprice; A.stats = dstats;
  return map_hip(launch_auction(A, stream ? (hipStream_t)stream : lib_stream()));
}

int ot_auction(const int32_t *C, int32_t n, int64_t eps0, int32_t theta, int64_t eps_final, int32_t *plan,
               int64_t *cost, int64_t *price, ot_stats *stats) {
  if (!C || !plan || !cost) return OT_EINVAL;
  int rc = auction_check(n, eps0, theta, eps_final);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(lib_mutex());
  if ((rc = init_locked())) return rc;
  hipStream_t s = lib_stream();
  int err = OT_OK;
  const size_t N = (size_t)n;
  auto *dC = (int32_t *)pool_get(220, 4 * N * N, &err);
  auto *dplan = (int32_t *)pool_get(221, 4 * N, &err);
  auto *dcost = (int64_t *)pool_get(222, 8, &err);
  auto *dprice = (int64_t *)pool_get(223, 8 * N, &err);
  auto *dst = (ot_stats *)pool_get(224, sizeof(ot_stats), &err);
  if (err) return err;
  hipError_t e = hipMemcpyAsync(dC, C, 4 * N * N, hipMemcpyHostToDevice, s);
  AuctionArgs A;
  A.C = dC; A.n = n; A.ld = n; A.eps0 = eps0; A.eps_final = eps_final; A.theta = theta;
  A.plan = dplan; A.cost = dcost; A.price = dprice; A.stats = dst;
  if (e == hipSuccess) e = launch_auction(A, s);
  ot_stats hs{};
  if (e == hipSuccess) e = hipMemcpyAsync(&hs, dst, sizeof hs, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return map_hip(e);
  if (stats) *stats = hs;
  if (hs.status != OT_OK) return (int)hs.status;
  e = hipMemcpyAsync(plan, dplan, 4 * N, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(cost, dcost, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && price) e = hipMemcpyAsync(price, dprice, 8 * N, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return map_hip(e);
}

}  // extern "C"
