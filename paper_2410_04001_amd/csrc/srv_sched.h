// Host-side bookkeeping of the serving engine, free of HIP so that it can be
// built and tested on a machine without a GPU: the device-arena allocator
// and the footprint of one request.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <iterator>
#include <map>

namespace lrnr {
namespace srv {

constexpr int64_t kAlign = 256;

inline int64_t align_up(int64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) with coalescing of free neighbours.
// Offsets and sizes are multiples of kAlign.
class Arena {
 public:
  explicit Arena(int64_t size = 0) { reset(size); }

  void reset(int64_t size) {
    size_ = size & ~(kAlign - 1);
    free_.clear();
    used_ = 0;
    peak_ = 0;
    if (size_ > 0) free_[0] = size_;
  }

  // Offset of a new block of at least `bytes`, or -1 when no free block fits.
  int64_t alloc(int64_t bytes) {
    const int64_t n = align_up(bytes > 0 ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const int64_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      used_ += n;
      if (used_ > peak_) peak_ = used_;
      return off;
    }
    return -1;
  }

  // Returns a block; `bytes` must be the size it was allocated with.
  void release(int64_t off, int64_t bytes) {
    const int64_t n = align_up(bytes > 0 ? bytes : 1);
    used_ -= n;
    auto next = free_.lower_bound(off);
    int64_t start = off, len = n;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && next->first == off + n) {
      len += next->second;
      free_.erase(next);
    }
    free_[start] = len;
  }

  int64_t size() const { return size_; }
  int64_t used() const { return used_; }
  int64_t peak() const { return peak_; }
  int64_t largest_free() const {
    int64_t m = 0;
    for (const auto& kv : free_)
      if (kv.second > m) m = kv.second;
    return m;
  }
  size_t free_blocks() const { return free_.size(); }

 private:
  int64_t size_ = 0, used_ = 0, peak_ = 0;
  std::map<int64_t, int64_t> free_;  // offset -> length
};

// Layout of one request's state in the arena (byte offsets from its block).
struct Footprint {
  int64_t xt, x0, tb;      // points
  int64_t s, m, v;         // coefficients and Adam moments [r_total]
  int64_t mu, loss, step;  // [4], [4], one int (padded)
  int64_t partials;        // [tiles][P] per-tile records
  int64_t u;               // [grid] evaluation output
  int64_t total;
  int tiles;
};

// pts_per_tile / bc_pairs_per_tile: the kernels' tile sizes; record_floats:
// the record length P of the request's net.
inline Footprint footprint(int64_t n_r, int64_t n_0, int64_t n_b, int r_total,
                           int record_floats, int64_t grid_points, int pts_per_tile,
                           int bc_pairs_per_tile) {
  Footprint f{};
  const int64_t G = (n_r + pts_per_tile - 1) / pts_per_tile +
                    (n_0 + pts_per_tile - 1) / pts_per_tile +
                    (n_b + bc_pairs_per_tile - 1) / bc_pairs_per_tile;
  int64_t off = 0;
  auto take = [&off](int64_t bytes) {
    const int64_t o = off;
    off += align_up(bytes > 0 ? bytes : 1);
    return o;
  };
  f.xt = take(n_r * 8);
  f.x0 = take(n_0 * 4);
  f.tb = take(n_b * 4);
  f.s = take((int64_t)r_total * 4);
  f.m = take((int64_t)r_total * 4);
  f.v = take((int64_t)r_total * 4);
  f.mu = take(16);
  f.loss = take(16);
  f.step = take(16);
  f.partials = take(G * record_floats * 4);
  f.u = take(grid_points * 4);
  f.total = off;
  f.tiles = (int)G;
  return f;
}

}  // namespace srv
}  // namespace lrnr
