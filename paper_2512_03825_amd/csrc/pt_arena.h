// pt_arena.h -- first-fit allocator of offsets inside one device arena, used by
// the served form to admit jobs by memory budget.  Plain C++ (no HIP), so the
// CPU tests can exercise it directly.  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace ptmi {

class Arena {
 public:
  explicit Arena(size_t bytes = 0, size_t align = 256) { reset(bytes, align); }

  void reset(size_t bytes, size_t align) {
    align_ = align ? align : 1;
    size_ = bytes - bytes % align_;
    free_.clear();
    if (size_) free_[0] = size_;
    used_ = peak_ = 0;
  }

  // Lowest-addressed free range that holds n bytes (rounded up to the
  // alignment).  Returns false, changing nothing, when none does.
  bool alloc(size_t n, size_t *off) {
    n = round(n);
    if (n == 0 || n > size_) return false;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, at = it->first + n;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += n;
      if (used_ > peak_) peak_ = used_;
      return true;
    }
    return false;
  }

  // Give back a range returned by alloc(off, n) with the same n; neighbouring
  // free ranges merge.  Returns false (changing nothing) for a range that
  // overlaps free space or lies outside the arena.
  bool release(size_t off, size_t n) {
    n = round(n);
    if (n == 0 || off % align_ || off + n > size_ || off + n < off) return false;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first < off + n) return false;
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second > off) return false;
    }
    auto it = free_.emplace(off, n).first;
    nx = std::next(it);
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
    used_ -= n;
    return true;
  }

  // Whether n bytes could ever be allocated (the arena is large enough).
  bool could_fit(size_t n) const { return n && round(n) <= size_; }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto &f : free_) m = f.second > m ? f.second : m;
    return m;
  }
  size_t free_ranges() const { return free_.size(); }

 private:
  size_t round(size_t n) const { return (n + align_ - 1) / align_ * align_; }
  std::map<size_t, size_t> free_; // offset -> length, disjoint and never adjacent
  size_t size_ = 0, align_ = 256, used_ = 0, peak_ = 0;
};

}  // namespace ptmi
