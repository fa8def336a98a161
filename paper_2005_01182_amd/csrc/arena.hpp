// arena.hpp -- first-fit allocator of byte ranges inside one device arena.
// Plain C++ (no HIP): the server keeps every admitted request's cost matrix in
// one device allocation and carves it with this allocator.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace otkm {

class Arena {
 public:
  static constexpr int64_t kAlign = 256;
  explicit Arena(int64_t size) : size_(size) {
    if (size > 0) free_[0] = size;
  }
  static int64_t round(int64_t bytes) { return (bytes + kAlign - 1) & ~(kAlign - 1); }

  // Offset of a free range of at least `bytes` (rounded up to kAlign), or -1.
  int64_t alloc(int64_t bytes) {
    bytes = round(bytes);
    if (bytes <= 0) return -1;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const int64_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest > 0) free_[off + bytes] = rest;
      used_ += bytes;
      return off;
    }
    return -1;
  }

  // Return a range obtained from alloc(bytes) with the same `bytes`.
  void release(int64_t off, int64_t bytes) {
    bytes = round(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

  int64_t used() const { return used_; }
  int64_t size() const { return size_; }
  const std::map<int64_t, int64_t> &free_ranges() const { return free_; }

 private:
  std::map<int64_t, int64_t> free_;  // offset -> size, disjoint and non-adjacent
  int64_t size_ = 0, used_ = 0;
};

}  // namespace otkm
