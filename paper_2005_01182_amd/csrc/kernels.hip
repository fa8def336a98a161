// kernels.hip -- gfx950 kernels around the batched-KM engine and their launchers.
//
// The engine's own kernels live in solve_kernels.hpp (instantiated by the
// solve_*.hip files); this file dispatches to them and holds the rest:
//   k_fill_i32        queue/flag reset (a kernel, so launches stay graph-capturable)
//   k_tr_prep         transport: check masses, unit -> bin maps (Eq. (1), r/c integer)
//   k_tr_expand       transport: S x S unit cost matrix
//   k_tr_aggregate    transport: unit plan -> bin plan X
//   k_tr_duals_*      transport: bin duals from unit duals (+ zero-mass bins)
//   k_grid_cost       serving: integer-point Euclidean costs, exactly rounded
#include <hip/hip_runtime.h>

#include "engine.hpp"
#include "gridcost.hpp"
#include "launch.hpp"

namespace otkm {

// ---------------------------------------------------------------------------
// batch: which instances compact keys hold
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_batch_flags(BatchArgs A) {
  const int idx = blockIdx.x;
  if (idx >= A.nq) return;
  const int k = A.order ? A.order[idx] : idx;
  if ((unsigned)k >= (unsigned)A.count) return;
  const int n = A.n[k];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __shared__ int s_lo[4], s_hi[4];
  int lo = 0x7fffffff, hi = (int)0x80000000;
  const bool sized = n >= 1 && n <= kCompactMaxN && n <= A.max_n && A.max_paths <= 0;
  const int32_t *C = A.C + A.coff[k];
  if (A.ctw && n >= 1 && n <= A.max_n) {
    // 64 x 64 tiles through LDS: each wavefront reads 16 rows of a tile
    // (64 consecutive entries per row) and writes 16 rows of its transpose;
    // the range is taken from the entries as they are read
    __shared__ int32_t tile[64][65];
    int32_t *T = A.ctw + A.coff[k];
    const int nt = (n + 63) / 64;
    for (int ti = 0; ti < nt; ++ti)
      for (int tj = 0; tj < nt; ++tj) {
        const int j = tj * 64 + lane;
        int32_t x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = ti * 64 + wid * 16 + r;
          x[r] = (i < n && j < n) ? C[(size_t)i * n + j] : 0;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = ti * 64 + wid * 16 + r;
          if (i < n && j < n) { lo = min(lo, x[r]); hi = max(hi, x[r]); }
          tile[wid * 16 + r][lane] = x[r];
        }
        __syncthreads();
        const int i = ti * 64 + lane;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int jj = tj * 64 + wid * 16 + r;  // row jj of the transpose, column i
          if (jj < n && i < n) T[(size_t)jj * n + i] = tile[lane][wid * 16 + r];
        }
        __syncthreads();
      }
  } else if (sized) {
    const int64_t total = (int64_t)n * n;
    int64_t q = threadIdx.x;
    for (; q + 768 < total; q += 1024) {
      const int a = C[q], b = C[q + 256], c = C[q + 512], d = C[q + 768];
      lo = min(lo, min(min(a, b), min(c, d)));
      hi = max(hi, max(max(a, b), max(c, d)));
    }
    for (; q < total; q += 256) { lo = min(lo, C[q]); hi = max(hi, C[q]); }
  }
  lo = wave_min_i32(lo);
  hi = wave_max_i32(hi);
  if (lane == 0) { s_lo[wid] = lo; s_hi[wid] = hi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) { lo = min(lo, s_lo[w]); hi = max(hi, s_hi[w]); }
    A.kflags[k] = (sized && (int64_t)hi - (int64_t)lo < kCompactRange) ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// grid-wide initial sweeps of one instance (the two full passes over C that the
// KM reduction needs: row minima, then per column the two smallest C_ij - u_i)
// ---------------------------------------------------------------------------
// u_i = min_j C_ij and rmax_i = max_j C_ij, one wavefront per row (the cost
// range min_i u_i .. max_i rmax_i is reduced by the solver; no global atomics).
// C has nr rows of n columns.
__global__ __launch_bounds__(256) void k_init_rows(const int32_t *C, int nr, int n, int ld, int64_t *u,
                                                   int32_t *rmax) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= nr) return;
  const int32_t *row = C + (size_t)i * (size_t)ld;
  int mn = 0x7fffffff, mx = (int)0x80000000;
  if ((ld & 3) == 0 && ((uintptr_t)C & 15) == 0) {
    // 16-byte loads: four columns per lane per step, four steps in flight (a
    // cold matrix comes from HBM, whose latency needs that many bytes in flight)
    int j = lane * 4;
    for (; j + 768 + 3 < n; j += 1024) {
      const int4 a = *(const int4 *)(row + j);
      const int4 b = *(const int4 *)(row + j + 256);
      const int4 c = *(const int4 *)(row + j + 512);
      const int4 d = *(const int4 *)(row + j + 768);
      mn = min(mn, min(min(min(a.x, a.y), min(a.z, a.w)), min(min(b.x, b.y), min(b.z, b.w))));
      mx = max(mx, max(max(max(a.x, a.y), max(a.z, a.w)), max(max(b.x, b.y), max(b.z, b.w))));
      mn = min(mn, min(min(min(c.x, c.y), min(c.z, c.w)), min(min(d.x, d.y), min(d.z, d.w))));
      mx = max(mx, max(max(max(c.x, c.y), max(c.z, c.w)), max(max(d.x, d.y), max(d.z, d.w))));
    }
    for (; j + 256 + 3 < n; j += 512) {
      const int4 a = *(const int4 *)(row + j);
      const int4 b = *(const int4 *)(row + j + 256);
      mn = min(mn, min(min(min(a.x, a.y), min(a.z, a.w)), min(min(b.x, b.y), min(b.z, b.w))));
      mx = max(mx, max(max(max(a.x, a.y), max(a.z, a.w)), max(max(b.x, b.y), max(b.z, b.w))));
    }
    for (; j + 3 < n; j += 256) {
      const int4 a = *(const int4 *)(row + j);
      mn = min(mn, min(min(a.x, a.y), min(a.z, a.w)));
      mx = max(mx, max(max(a.x, a.y), max(a.z, a.w)));
    }
    for (int t = j; t < n && t < j + 4; ++t) { mn = min(mn, row[t]); mx = max(mx, row[t]); }
  } else {
    for (int t = lane; t < n; t += 64) { mn = min(mn, row[t]); mx = max(mx, row[t]); }
  }
  mn = wave_min_i32(mn);
  mx = wave_max_i32(mx);
  if (lane == 0) {
    u[i] = mn;
    rmax[i] = mx;
  }
}

__device__ __forceinline__ void two_smallest(uint64_t &b1, uint64_t &b2, uint64_t key) {
  const bool l1 = key < b1, l2 = key < b2;
  b2 = l1 ? b1 : (l2 ? key : b2);
  b1 = l1 ? key : b1;
}

// Partial top-2 per column over one slice of kInitSliceRows rows:
// part[(y * n + j) * 2 + {0,1}] = the two smallest pack(C_ij - u_i, i), i in
// slice y.  A workgroup covers 64 columns; its four wavefronts split the slice
// (each row a coalesced 256-byte read) and merge through LDS.
constexpr int kInitSliceRows = 128;
__global__ __launch_bounds__(256) void k_init_cols(const int32_t *C, int nr, int n, int ld, const int64_t *u,
                                                   uint64_t *part) {
  __shared__ uint64_t sb[4][64][2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const int jc = j < n ? j : n - 1;
  const int i0 = blockIdx.y * kInitSliceRows + w * (kInitSliceRows / 4);
  const int i1 = min(nr, i0 + kInitSliceRows / 4);
  uint64_t b1 = kInf, b2 = kInf;
  int i = i0;
  for (; i + 8 <= i1; i += 8) {
    int32_t c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = C[(size_t)(i + q) * (size_t)ld + jc];
#pragma unroll
    for (int q = 0; q < 8; ++q) two_smallest(b1, b2, pack((int64_t)c[q] - u[i + q], i + q));
  }
  for (; i < i1; ++i) two_smallest(b1, b2, pack((int64_t)C[(size_t)i * (size_t)ld + jc] - u[i], i));
  sb[w][lane][0] = b1;
  sb[w][lane][1] = b2;
  __syncthreads();
  if (w == 0 && j < n) {
#pragma unroll
    for (int v = 1; v < 4; ++v) {
      two_smallest(b1, b2, sb[v][lane][0]);
      two_smallest(b1, b2, sb[v][lane][1]);
    }
    part[((size_t)blockIdx.y * n + j) * 2] = b1;
    part[((size_t)blockIdx.y * n + j) * 2 + 1] = b2;
  }
}

// b[j][0..1] = the two smallest keys of column j over all slices.
__global__ __launch_bounds__(256) void k_init_merge(const uint64_t *part, int slices, int n, uint64_t *b) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  uint64_t b1 = kInf, b2 = kInf;
  for (int y = 0; y < slices; ++y) {
    two_smallest(b1, b2, part[((size_t)y * n + j) * 2]);
    two_smallest(b1, b2, part[((size_t)y * n + j) * 2 + 1]);
  }
  b[2 * (size_t)j] = b1;
  b[2 * (size_t)j + 1] = b2;
}

// CT = C^T (n x nr, row stride nr) from C (nr x n, row stride ld): 64 x 64
// tiles through LDS so that both the read and the write are coalesced.
__global__ __launch_bounds__(256) void k_transpose(const int32_t *C, int nr, int n, int ld, int32_t *CT) {
  __shared__ int32_t tile[64][65];
  const int bj = blockIdx.x * 64, bi = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int i = bi + r, j = bj + tx;
    if (i < nr && j < n) tile[r][tx] = C[(size_t)i * (size_t)ld + j];
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int j = bj + r, i = bi + tx;
    if (i < nr && j < n) CT[(size_t)j * (size_t)nr + i] = tile[tx][r];
  }
}

// The transposes of a batch's matrices (instance k: n[k] x n[k] at offset
// coff[k] in both buffers), 64 x 64 tiles through LDS; blockIdx.z is the
// instance, tiles outside it return at once.
__global__ __launch_bounds__(256) void k_transpose_batch(const int32_t *C, const int64_t *coff, const int32_t *nn,
                                                         int32_t *CT) {
  __shared__ int32_t tile[64][65];
  const int k = blockIdx.z;
  const int n = nn[k];
  const int bj = blockIdx.x * 64, bi = blockIdx.y * 64;
  if (bi >= n || bj >= n) return;
  const int32_t *A = C + coff[k];
  int32_t *AT = CT + coff[k];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int i = bi + r, j = bj + tx;
    if (i < n && j < n) tile[r][tx] = A[(size_t)i * (size_t)n + j];
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int j = bj + r, i = bi + tx;
    if (i < n && j < n) AT[(size_t)j * (size_t)n + i] = tile[tx][r];
  }
}

// lb = sum_i u_i + sum_j v_j for the KM reduction's duals (u_i = row minimum,
// v_j = smallest C_ij - u_i, the value of the column's best key b[2j]): a
// feasible dual, so a lower bound on the optimum.  One workgroup.
__global__ __launch_bounds__(1024) void k_lower_bound(const int64_t *u, const uint64_t *b, int n, int64_t *lb) {
  __shared__ int64_t red[1024];
  int64_t s = 0;
  for (int k = threadIdx.x; k < n; k += 1024) s += u[k] + kval(b[2 * (size_t)k]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *lb = red[0];
}

// Cs = floor(C / s) element-wise (row stride ld in, n out): the scaled costs of
// the single-scaling-factor mode.  floor(C/s) * s <= C, so duals feasible for
// Cs become feasible for C when multiplied by s.
__global__ void k_floor_div(const int32_t *C, int n, int ld, int32_t s, int32_t *Cs) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const int32_t c = C[(size_t)i * (size_t)ld + j];
    const int32_t q = c / s;  // truncates toward zero; step down for negative non-multiples
    Cs[(size_t)i * (size_t)n + j] = (c % s != 0 && c < 0) ? q - 1 : q;
  }
}

// ---------------------------------------------------------------------------
// rectangular assignment (n x m, n != m): Eq. (1) with unit masses, the smaller
// side matched completely and the larger side at most once
// ---------------------------------------------------------------------------
// The solver runs on rows = the smaller side: C itself when n <= m, else C^T
// (trans).  Its outputs (plan pq over its rows, duals uq over its rows and vq
// over its columns, status in sq) become the caller's: when trans, rows and
// columns swap back, so plan[i] = the column whose solver row took row i, or
// -1.  Without a column reduction the larger side's potentials end <= 0 and 0
// where unmatched; with equal sides (square, column-reduced) they are shifted
// by their maximum V (u += V, v -= V keeps every u_i + v_j and the objective),
// which gives the same sign condition.  One workgroup.
__global__ __launch_bounds__(1024) void k_rect_finish(int n, int m, int trans, const int32_t *pq, const int64_t *uq,
                                                      const int64_t *vq, const int64_t *cq, const ot_stats *sq,
                                                      int32_t *plan, int64_t *cost, int64_t *u, int64_t *v,
                                                      ot_stats *stats) {
  __shared__ int64_t red[1024];
  const int tid = threadIdx.x;
  const int status = sq->status;
  if (stats && tid == 0) *stats = *sq;
  if (status != 0) return;
  const int cols = trans ? n : m;  // the solver's columns
  int64_t mx = INT64_MIN;
  for (int k = tid; k < cols; k += 1024) mx = vq[k] > mx ? vq[k] : mx;
  red[tid] = mx;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w && red[tid + w] > red[tid]) red[tid] = red[tid + w];
    __syncthreads();
  }
  const int64_t V = red[0];  // solver rows' duals + V, solver columns' duals - V
  if (!trans) {
    for (int i = tid; i < n; i += 1024) {
      plan[i] = pq[i];
      if (u) u[i] = uq[i] + V;
    }
    if (v)
      for (int j = tid; j < m; j += 1024) v[j] = vq[j] - V;
  } else {
    for (int i = tid; i < n; i += 1024) {
      plan[i] = -1;
      if (u) u[i] = vq[i] - V;
    }
    if (v)
      for (int j = tid; j < m; j += 1024) v[j] = uq[j] + V;
    __syncthreads();  // the -1 fill is visible to the workgroup before the scatter
    for (int j = tid; j < m; j += 1024) {
      const int i = pq[j];
      if ((unsigned)i < (unsigned)n) plan[i] = j;
    }
  }
  if (tid == 0) *cost = *cq;
}

__global__ void k_fill_i32(int32_t *p, int32_t value, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// ---------------------------------------------------------------------------
// transport by unit expansion
// ---------------------------------------------------------------------------
// One workgroup: validate masses, then rowbin[a] / colbin[b] = bin of unit a / b
// and rfirst[i] / cfirst[j] = first unit of bin (or -1 for zero mass).
__global__ __launch_bounds__(1024) void k_tr_prep(const int32_t *r, const int32_t *c, int n, int m, int S,
                                                  int32_t *rowbin, int32_t *colbin, int32_t *rfirst,
                                                  int32_t *cfirst, int32_t *gate, ot_stats *stats) {
  __shared__ unsigned long long s_sum[2];
  __shared__ int s_neg;
  __shared__ int s_off[1024];
  if (threadIdx.x == 0) { s_sum[0] = 0; s_sum[1] = 0; s_neg = 0; }
  __syncthreads();
  long long a = 0, b = 0;
  int neg = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) { int x = r[i]; neg |= x < 0; a += x; }
  for (int j = threadIdx.x; j < m; j += blockDim.x) { int x = c[j]; neg |= x < 0; b += x; }
  atomicAdd(&s_sum[0], (unsigned long long)a);  // two's complement: wraps to the signed sum
  atomicAdd(&s_sum[1], (unsigned long long)b);
  if (neg) atomicOr(&s_neg, 1);
  __syncthreads();
  const long long sr = (long long)s_sum[0], sc = (long long)s_sum[1];
  int status = 0;
  if (s_neg) status = OT_ENEGMASS;
  else if (sr != sc || sr < 1 || sr != (long long)S) status = OT_EUNBALANCED;
  if (status != 0) {
    if (threadIdx.x == 0) {
      *gate = status;
      if (stats) { ot_stats s = {}; s.status = status; *stats = s; }
    }
    return;
  }
  // exclusive prefix sums, sequential over chunks of blockDim entries
  for (int side = 0; side < 2; ++side) {
    const int32_t *w = side == 0 ? r : c;
    const int len = side == 0 ? n : m;
    int32_t *bin = side == 0 ? rowbin : colbin;
    int32_t *first = side == 0 ? rfirst : cfirst;
    int base = 0;
    for (int start = 0; start < len; start += blockDim.x) {
      const int i = start + threadIdx.x;
      const int x = i < len ? w[i] : 0;
      s_off[threadIdx.x] = x;
      __syncthreads();
      // Hillis-Steele inclusive scan over the chunk
      for (int d = 1; d < (int)blockDim.x; d <<= 1) {
        int y = threadIdx.x >= (unsigned)d ? s_off[threadIdx.x - d] : 0;
        __syncthreads();
        s_off[threadIdx.x] += y;
        __syncthreads();
      }
      const int incl = s_off[threadIdx.x];
      const int excl = base + incl - x;
      if (i < len) {
        first[i] = x > 0 ? excl : -1;
        for (int q = 0; q < x; ++q) bin[excl + q] = i;
      }
      const int total = s_off[blockDim.x - 1];
      __syncthreads();
      base += total;
    }
  }
  if (threadIdx.x == 0) *gate = 0;
}

__global__ void k_tr_expand(const int32_t *C, int m, int S, const int32_t *rowbin, const int32_t *colbin,
                            int32_t *Cx, const int32_t *gate) {
  if (*gate != 0) return;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (b >= S || a >= S) return;
  Cx[(size_t)a * S + b] = C[(size_t)rowbin[a] * m + colbin[b]];
}

__global__ void k_tr_aggregate(const int32_t *plan, int S, int m, const int32_t *rowbin, const int32_t *colbin,
                               int32_t *X, const int32_t *gate, const ot_stats *stats) {
  if (*gate != 0 || (stats && stats->status != 0)) return;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= S) return;
  const int b = plan[a];
  if ((unsigned)b >= (unsigned)S) return;
  atomicAdd(&X[(size_t)rowbin[a] * m + colbin[b]], 1);
}

// Bins with mass take the dual of their first unit (all units of a bin carry
// the same dual in an optimal unit solution).
__global__ void k_tr_duals_copy(const int64_t *U, const int64_t *V, int n, int m, const int32_t *rfirst,
                                const int32_t *cfirst, int64_t *u, int64_t *v, const int32_t *gate,
                                const ot_stats *stats) {
  if (*gate != 0 || (stats && stats->status != 0)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && rfirst[i] >= 0) u[i] = U[rfirst[i]];
  if (i < m && cfirst[i] >= 0) v[i] = V[cfirst[i]];
}

// Zero-mass row i: u_i = min over columns with mass of C_ij - v_j (one wavefront per row).
__global__ __launch_bounds__(256) void k_tr_duals_zero_rows(const int32_t *C, const int32_t *r, const int32_t *c,
                                                            int n, int m, int64_t *u, const int64_t *v,
                                                            const int32_t *gate, const ot_stats *stats) {
  if (*gate != 0 || (stats && stats->status != 0)) return;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= n || r[i] != 0) return;
  int64_t best = INT64_MAX;
  for (int j = lane; j < m; j += 64)
    if (c[j] > 0) best = min(best, (int64_t)C[(size_t)i * m + j] - v[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) best = min(best, (int64_t)__shfl_xor(best, off, 64));
  if (lane == 0) u[i] = best;
}

// Zero-mass column j: v_j = min over all rows of C_ij - u_i (one thread per column, coalesced rows).
__global__ void k_tr_duals_zero_cols(const int32_t *C, const int32_t *c, int n, int m, const int64_t *u,
                                     int64_t *v, const int32_t *gate, const ot_stats *stats) {
  if (*gate != 0 || (stats && stats->status != 0)) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m || c[j] != 0) return;
  int64_t best = INT64_MAX;
  for (int i = 0; i < n; ++i) best = min(best, (int64_t)C[(size_t)i * m + j] - u[i]);
  v[j] = best;
}

// ---------------------------------------------------------------------------
// serving: C_ij = round(sqrt(|p_i - q_j|^2)) for integer points, exact
// ---------------------------------------------------------------------------
__global__ void k_grid_cost(const int32_t *ps, const int32_t *pt, int n, int32_t *Cout) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n || i >= n) return;
  const int64_t dx = (int64_t)ps[2 * i] - pt[2 * j];
  const int64_t dy = (int64_t)ps[2 * i + 1] - pt[2 * j + 1];
  Cout[(size_t)i * n + j] = grid_isqrt_round(dx * dx + dy * dy);
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int cpt_for(int n, int block) {
  const int need = (n + block - 1) / block;
  return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : need <= 8 ? 8 : 0;
}

hipError_t launch_assign_one(const Problem &P, int block, const int32_t *gate, hipStream_t s) {
  const int cpt = cpt_for(P.n, block);
  return block <= 256 ? launch_assign_one_lo(P, block, cpt, gate, s) : launch_assign_one_hi(P, block, cpt, gate, s);
}

int batch_occupancy(int block, int max_n) {
  const int cpt = cpt_for(max_n, block);
  const int o = block <= 256 ? batch_occupancy_lo(block, cpt, max_n) : batch_occupancy_hi(block, cpt, max_n);
  return o < 0 ? 0 : o;
}

hipError_t launch_assign_batch(const BatchArgs &A, int block, int grid, hipStream_t s) {
  const int cpt = cpt_for(A.max_n, block);
  return block <= 256 ? launch_assign_batch_lo(A, block, cpt, grid, s) : launch_assign_batch_hi(A, block, cpt, grid, s);
}

hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s, p, value, count);
  return hipGetLastError();
}

hipError_t launch_transport(const TransportArgs &T, int block, hipStream_t s) {
  hipLaunchKernelGGL(k_tr_prep, dim3(1), dim3(1024), 0, s, T.r, T.c, T.n, T.m, T.S, T.rowbin, T.colbin, T.rfirst,
                     T.cfirst, T.gate, T.stats);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tr_expand, dim3((T.S + 255) / 256, T.S), dim3(256), 0, s, T.C, T.m, T.S, T.rowbin, T.colbin,
                     T.Cx, T.gate);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (T.CxT && (e = launch_transpose(T.Cx, T.S, T.S, T.S, T.CxT, s)) != hipSuccess) return e;
  Problem P;
  P.C = T.Cx; P.n = T.S; P.ld = T.S; P.max_paths = T.max_paths; P.flags = 0; P.CT = T.CxT;
  P.Cout = nullptr; P.ldo = T.S; P.dscale = 1;
  P.init_u = nullptr; P.init_b = nullptr; P.init_rmax = nullptr;
  P.plan = T.plan; P.cost = T.cost; P.u = T.U; P.v = T.V; P.stats = T.stats; P.ws = T.ws;
  if ((e = launch_assign_one(P, block, T.gate, s)) != hipSuccess) return e;
  if ((e = launch_fill_i32(T.X, 0, (int64_t)T.n * T.m, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_tr_aggregate, dim3((T.S + 255) / 256), dim3(256), 0, s, T.plan, T.S, T.m, T.rowbin, T.colbin,
                     T.X, T.gate, T.stats);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nm = T.n > T.m ? T.n : T.m;
  hipLaunchKernelGGL(k_tr_duals_copy, dim3((nm + 255) / 256), dim3(256), 0, s, T.U, T.V, T.n, T.m, T.rfirst, T.cfirst,
                     T.u, T.v, T.gate, T.stats);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_tr_duals_zero_rows, dim3((T.n + 3) / 4), dim3(256), 0, s, T.C, T.r, T.c, T.n, T.m, T.u, T.v,
                     T.gate, T.stats);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_tr_duals_zero_cols, dim3((T.m + 255) / 256), dim3(256), 0, s, T.C, T.c, T.n, T.m, T.u, T.v,
                     T.gate, T.stats);
  return hipGetLastError();
}

size_t init_part_bytes(int nr, int n) {
  return (size_t)((nr + kInitSliceRows - 1) / kInitSliceRows) * (size_t)n * 16;
}

hipError_t launch_init_sweeps(const int32_t *C, int nr, int n, int ld, int64_t *u, int32_t *rmax, uint64_t *part,
                              uint64_t *b, hipStream_t st) {
  hipError_t e;
  hipLaunchKernelGGL(k_init_rows, dim3((nr + 3) / 4), dim3(256), 0, st, C, nr, n, ld, u, rmax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int slices = (nr + kInitSliceRows - 1) / kInitSliceRows;
  hipLaunchKernelGGL(k_init_cols, dim3((n + 63) / 64, slices), dim3(256), 0, st, C, nr, n, ld, u, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_init_merge, dim3((n + 255) / 256), dim3(256), 0, st, part, slices, n, b);
  return hipGetLastError();
}

hipError_t launch_floor_div(const int32_t *C, int n, int ld, int32_t s, int32_t *Cs, hipStream_t st) {
  const int bx = (n + 255) / 256;
  hipLaunchKernelGGL(k_floor_div, dim3(bx < 8 ? bx : 8, n), dim3(256), 0, st, C, n, ld, s, Cs);
  return hipGetLastError();
}

hipError_t launch_transpose(const int32_t *C, int nr, int n, int ld, int32_t *CT, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose, dim3((n + 63) / 64, (nr + 63) / 64), dim3(256), 0, s, C, nr, n, ld, CT);
  return hipGetLastError();
}

hipError_t launch_transpose_batch(const int32_t *C, const int64_t *coff, const int32_t *n, int count, int max_n,
                                  int32_t *CT, hipStream_t s) {
  const int t = (max_n + 63) / 64;
  for (int k0 = 0; k0 < count; k0 += 65535) {  // grid z holds at most 65535 instances per launch
    const int c = count - k0 < 65535 ? count - k0 : 65535;
    hipLaunchKernelGGL(k_transpose_batch, dim3(t, t, c), dim3(256), 0, s, C, coff + k0, n + k0, CT);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_lower_bound(const int64_t *u, const uint64_t *b, int n, int64_t *lb, hipStream_t s) {
  hipLaunchKernelGGL(k_lower_bound, dim3(1), dim3(1024), 0, s, u, b, n, lb);
  return hipGetLastError();
}

hipError_t launch_rect_finish(int n, int m, bool trans, const int32_t *pq, const int64_t *uq, const int64_t *vq,
                              const int64_t *cq, const ot_stats *sq, int32_t *plan, int64_t *cost, int64_t *u,
                              int64_t *v, ot_stats *stats, hipStream_t s) {
  hipLaunchKernelGGL(k_rect_finish, dim3(1), dim3(1024), 0, s, n, m, trans ? 1 : 0, pq, uq, vq, cq, sq, plan, cost,
                     u, v, stats);
  return hipGetLastError();
}

hipError_t launch_grid_cost(const int32_t *ps, const int32_t *pt, int n, int32_t *Cout, hipStream_t s) {
  hipLaunchKernelGGL(k_grid_cost, dim3((n + 255) / 256, n), dim3(256), 0, s, ps, pt, n, Cout);
  return hipGetLastError();
}

}  // namespace otkm
