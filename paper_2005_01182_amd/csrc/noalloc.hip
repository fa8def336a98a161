// noalloc.hip -- the allocation-free variant of ot_assign_dev.
//
// Its scratch (the engine's per-workgroup lists and the outputs of the
// grid-wide reduction sweeps) lives in one file-scope device array instead of
// the library's stream workspaces, so a call never allocates device memory:
// callers under graph capture or in tight serving loops can use it.  Each
// device holds its own copy of the array; host code reaches it only through
// the address hipGetSymbolAddress returns on that device.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "launch.hpp"
#include "otkm.h"
#include "runtime.hpp"

namespace otkm {
namespace {

// ws (8n) + row minima (8n) + row maxima (4n) + per-slice column top-2
// (16 n ceil(n / 128)) + merged column top-2 (16n), each 256-byte aligned:
// 2,244,608 bytes at n = 4096, the largest size (OT_NOALLOC_SCRATCH_BYTES).
constexpr size_t kScratchBytes = OT_NOALLOC_SCRATCH_BYTES;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, unsigned char *> g_ptr;  // device -> address of its copy of `scratch`

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t ws, u0, rmax, part, b, total;
};

Layout layout(int n) {
  Layout L;
  const size_t N = (size_t)n;
  size_t o = 0;
  L.ws = o;   o = up256(o + 4 * ws_ints(n));
  L.u0 = o;   o = up256(o + 8 * N);
  L.rmax = o; o = up256(o + 4 * N);
  L.part = o; o = up256(o + init_part_bytes(n, n));
  L.b = o;    o = up256(o + 16 * N);
  L.total = o;
  return L;
}

// Address of this device's scratch, looked up once per device with that
// device current.
int scratch_ptr(unsigned char **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OT_ENODEV;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ptr.find(dev);
  if (it == g_ptr.end()) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return map_hip(e == hipSuccess ? hipErrorInvalidSymbol : e);
    it = g_ptr.emplace(dev, (unsigned char *)p).first;
  }
  *out = it->second;
  return OT_OK;
}

}  // namespace
}  // namespace otkm

using namespace otkm;

extern "C" int ot_assign_dev_noalloc(const int32_t *dC, int32_t n, int32_t ld, const ot_options *opt,
                                     int32_t *dplan, int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats,
                                     void *stream) {
  if (!dC || !dplan || !dcost || n <= 0 || ld < n) return OT_EINVAL;
  if (n > OT_MAX_N || layout(n).total > kScratchBytes) return OT_ETOOBIG;
  int block = default_block(n), max_paths = 0, flags = 0;
  if (opt) {
    for (int k = 0; k < 3; ++k)
      if (opt->reserved[k] != 0) return OT_EINVAL;
    // one workgroup on the exact costs: no exchange state, no scaled copy
    if (opt->max_paths < 0 || (opt->flags & ~(OT_FLAG_PHASE_TIMERS | OT_FLAG_WIDE_KEYS)) != 0 || opt->scale > 1 || opt->scale < 0 ||
        opt->wgs > 1 || opt->wgs < 0)
      return OT_EINVAL;
    if (opt->block != 0) {
      if ((opt->block != 64 && opt->block != 256 && opt->block != 512 && opt->block != 1024) ||
          cpt_for(n, opt->block) == 0)
        return OT_EINVAL;
      block = opt->block;
    }
    max_paths = opt->max_paths;
    flags = opt->flags;
  }
  {
    std::lock_guard<std::mutex> lk(lib_mutex());
    const int rc = init_locked();
    if (rc) return rc;
  }
  unsigned char *base = nullptr;
  int rc = scratch_ptr(&base);
  if (rc) return rc;
  const Layout L = layout(n);
  hipStream_t s = stream ? (hipStream_t)stream : lib_stream();
  auto *u0 = (int64_t *)(base + L.u0);
  auto *rmax = (int32_t *)(base + L.rmax);
  auto *part = (uint64_t *)(base + L.part);
  auto *b = (uint64_t *)(base + L.b);
  // every scratch word is written before it is read (the sweeps fill u0, rmax,
  // part and b; the engine initialises its lists), so nothing is cleared
  Problem P;
  P.C = dC; P.n = n; P.ld = ld; P.CT = nullptr; P.max_paths = max_paths; P.flags = flags;
  P.Cout = nullptr; P.ldo = ld; P.dscale = 1;
  P.init_u = nullptr; P.init_b = nullptr; P.init_rmax = nullptr;
  if (!(block == 64 && n <= 64)) {  // one wavefront reads C itself
    const hipError_t e = launch_init_sweeps(dC, n, n, ld, u0, rmax, part, b, s);
    if (e != hipSuccess) return map_hip(e);
    P.init_u = u0; P.init_b = b; P.init_rmax = rmax;
  }
  P.plan = dplan; P.cost = dcost; P.u = du; P.v = dv; P.stats = dstats;
  P.ws = (int32_t *)(base + L.ws);
  return map_hip(launch_assign_one(P, block, nullptr, s));
}
