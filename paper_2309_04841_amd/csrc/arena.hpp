// arena.hpp -- offset bookkeeping of the request loop's device arena.
//
// Host-only (no HIP types): the server owns one device allocation and uses
// this class to carve it.  Two placement rules keep request space contiguous:
// requests take the lowest block that fits (first fit from the bottom), and
// the resident cost vectors take the highest (last fit from the top), so cost
// vectors added while requests are in flight do not split the space below
// them.  Blocks are multiples of 256 bytes.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace qaoa_arena {

constexpr size_t kGranule = 256;
constexpr size_t kNone = SIZE_MAX;

inline size_t round_up(size_t bytes) { return (bytes + kGranule - 1) & ~(kGranule - 1); }

class ArenaMap {
 public:
  explicit ArenaMap(size_t bytes = 0) { reset(bytes); }

  void reset(size_t bytes) {
    size_ = bytes & ~(kGranule - 1);
    used_ = peak_ = 0;
    free_.clear();
    if (size_) free_[0] = size_;
  }

  // Lowest-addressed block of `bytes` (rounded up), or kNone.
  size_t alloc_low(size_t bytes) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        take(bytes);
        return off;
      }
    }
    return kNone;
  }

  // Highest-addressed block of `bytes` (rounded up), carved from the top end
  // of the highest free range that fits, or kNone.
  size_t alloc_high(size_t bytes) {
    bytes = round_up(bytes);
    for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
      if (it->second >= bytes) {
        const size_t start = it->first, len = it->second;
        const size_t off = start + len - bytes;
        free_.erase(std::next(it).base());
        if (len > bytes) free_[start] = len - bytes;
        take(bytes);
        return off;
      }
    }
    return kNone;
  }

  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
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

  size_t largest_free() const {
    size_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t free_ranges() const { return free_.size(); }
  void reset_peak() { peak_ = used_; }

 private:
  void take(size_t bytes) {
    used_ += bytes;
    peak_ = std::max(peak_, used_);
  }
  size_t size_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length, disjoint, coalesced
};

// What the scheduler does with the request at the head of the queue when its
// block could not be allocated: wait while other requests are in flight (they
// free memory as they finish), reject it when nothing is in flight (no
// finishing request will ever make room), so the queue always drains.
enum class HeadAction { kWait, kReject };
inline HeadAction head_blocked(size_t in_flight) { return in_flight ? HeadAction::kWait : HeadAction::kReject; }

}  // namespace qaoa_arena
