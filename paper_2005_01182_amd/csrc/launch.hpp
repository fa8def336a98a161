// launch.hpp -- host-side launch helpers shared by the runtime (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.hpp"

namespace otkm {

struct BatchArgs {
  const int32_t *C;       // base of all cost matrices
  const int32_t *CT = nullptr;  // their transposes at the same offsets, or null (refreshes then gather from C)
  const int64_t *coff;    // [count] element offset of instance k's matrix
  const int32_t *n;       // [count]
  const int64_t *voff;    // [count] element offset of instance k's plan/u/v
  const int32_t *order;   // [count] processing order, or null
  int count;             // instances (bound for indices in order[])
  int nq;                // queue length: entries of order[] (or instances) this launch solves
  int max_n, max_paths;
  int32_t *plan;
  int64_t *cost, *u, *v;
  ot_stats *stats;
  int32_t *ws;            // grid * ws_ints(max_n)
  int32_t *head;          // queue head (reset to 0 before the launch)
  int32_t *done;          // [count] or null: done[k] = tag once instance k's outputs are visible to the host
  int32_t tag;
  // Optional: per instance whether compact keys hold it ([count] bytes, set by
  // the launch) and a second queue head; with both, the launch runs the
  // compact-key kernel over those instances and the 64-bit-key kernel over the
  // rest, one after the other on the stream.
  uint8_t *kflags = nullptr;
  int32_t *head2 = nullptr;
  // Optional, with kflags: the flag pass, which reads every matrix anyway,
  // also writes its transpose here (same offsets as C), and the solve kernels
  // then read these transposes to refresh single stale columns.
  int32_t *ctw = nullptr;
};

struct TransportArgs {
  const int32_t *C, *r, *c;
  int n, m, S, max_paths;
  int32_t *rowbin, *colbin, *rfirst, *cfirst, *gate;  // [S], [S], [n], [m], [1]
  int32_t *Cx;                                        // [S*S]
  int32_t *CxT;                                       // [S*S] transpose of Cx, or null
  int32_t *plan;                                      // [S]
  int64_t *U, *V;                                     // [S] unit duals
  int32_t *ws;                                        // ws_ints(S)
  int32_t *X;                                         // [n*m]
  int64_t *cost, *u, *v;                              // [1], [n], [m]
  ot_stats *stats;                                    // [1]
};

int cpt_for(int n, int block);
// per-file dispatchers of the engine's instantiations (solve_*.hip)
hipError_t launch_assign_one_lo(const Problem &P, int block, int cpt, const int32_t *gate, hipStream_t s);
hipError_t launch_assign_one_hi(const Problem &P, int block, int cpt, const int32_t *gate, hipStream_t s);
hipError_t launch_assign_batch_lo(const BatchArgs &A, int block, int cpt, int grid, hipStream_t s);
hipError_t launch_assign_batch_hi(const BatchArgs &A, int block, int cpt, int grid, hipStream_t s);
int batch_occupancy_lo(int block, int cpt, int max_n);
int batch_occupancy_hi(int block, int cpt, int max_n);
int batch_occupancy(int block, int max_n);
hipError_t launch_assign_one(const Problem &P, int block, const int32_t *gate, hipStream_t s);
hipError_t launch_assign_grid(const Problem &P, int block, int wgs, hipStream_t s);
hipError_t launch_assign_batch(const BatchArgs &A, int block, int grid, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t count, hipStream_t s);
hipError_t launch_transport(const TransportArgs &T, int block, hipStream_t s);
size_t init_part_bytes(int nr, int n);
hipError_t launch_init_sweeps(const int32_t *C, int nr, int n, int ld, int64_t *u, int32_t *rmax, uint64_t *part,
                              uint64_t *b, hipStream_t st);
hipError_t launch_lower_bound(const int64_t *u, const uint64_t *b, int n, int64_t *lb, hipStream_t s);
hipError_t launch_floor_div(const int32_t *C, int n, int ld, int32_t s, int32_t *Cs, hipStream_t st);
hipError_t launch_transpose(const int32_t *C, int nr, int n, int ld, int32_t *CT, hipStream_t s);
hipError_t launch_transpose_batch(const int32_t *C, const int64_t *coff, const int32_t *n, int count, int max_n,
                                  int32_t *CT, hipStream_t s);
hipError_t launch_rect_finish(int n, int m, bool trans, const int32_t *pq, const int64_t *uq, const int64_t *vq,
                              const int64_t *cq, const ot_stats *sq, int32_t *plan, int64_t *cost, int64_t *u,
                              int64_t *v, ot_stats *stats, hipStream_t s);
hipError_t launch_grid_cost(const int32_t *ps, const int32_t *pt, int n, int32_t *Cout, hipStream_t s);
// Serving: one persistent kernel over a queue in host memory (serve_kernel.hip)
struct ServeArgs {
  const int32_t *h_tail, *h_quit;  // host (mapped): published entries; the epoch at or below which launches end
  const int32_t *desc;             // host (mapped): entry p at [p % qcap][4] = {slot, n, coff low, coff high}
  const int32_t *pts;              // host (mapped): [slots][4 max_n] points, src (2n) then dst (2n)
  int32_t *head, *tail, *quit;     // device: entries taken; mirrors of the two host words
  uint64_t *polled;                // device: s_memrealtime of the last read of the host words
  int qcap, slots, max_n, epoch, linger;
  int32_t *C;                      // device: cost matrices (element offset coff per entry)
  int32_t *plan;                   // host (mapped): [slots][max_n]
  int64_t *cost, *u, *v;           // host (mapped): [slots], [slots][max_n] x 2
  ot_stats *stats;                 // host (mapped): [slots]
  int32_t *done;                   // host (mapped): [slots], entry p's slot gets p + 1 when its results are out
  int32_t *ws;                     // device: grid * ws_ints(max_n)
};
size_t serve_lds_bytes(int max_n);
int serve_occupancy(int max_n);
hipError_t launch_serve(const ServeArgs &A, int grid, hipStream_t s);

}  // namespace otkm
