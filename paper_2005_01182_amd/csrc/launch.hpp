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
  // Live queue (serving): with live_tail set, order is a ring of qcap entries
  // filled while the kernel runs (entry p at order[p % qcap], published once
  // *live_tail > p; device memory written by a kernel on another stream),
  // head is the first entry not yet taken (set before the launch), nq is
  // unused, and done[k] = p + 1 for entry p.
  const int32_t *live_tail = nullptr;
  int32_t qcap = 0;
  int32_t linger = 0;                  // empty polls (a few microseconds each) before a workgroup leaves
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
// Serving: entries [first, first + count) of a live queue (each {slot, n, coff
// low, coff high} in host memory at staging[p % qcap]) into the device
// descriptors and ring, then the tail to first + count.
hipError_t launch_serve_publish(const int4 *staging, int first, int count, int qcap, int64_t vstride,
                                int32_t *ring, int32_t *n, int64_t *coff, int64_t *voff, int32_t *tail,
                                hipStream_t s);

}  // namespace otkm
