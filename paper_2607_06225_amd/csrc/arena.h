// arena.h -- first-fit sub-allocator over one fixed range of offsets.
//
// The request server reserves its whole device budget once and carves each
// micro-batch's memory (sequences, workspace with traceback codes, results,
// CIGAR words) out of it with this allocator.  Admission of work is then
// exactly "the arena has a free block this large".  Host code only: the
// allocator hands out offsets and never touches the memory.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace alnrt {

class Arena {
 public:
  // Manage offsets [0, size rounded down to align); align is a power of two.
  void reset(uint64_t size, uint64_t align) {
    align_ = align ? align : 1;
    size_ = size / align_ * align_;
    free_.clear();
    used_.clear();
    used_bytes_ = 0;
    if (size_) free_[0] = size_;
  }

  // Lowest-offset free block of at least `bytes` (rounded up to align).
  bool alloc(uint64_t bytes, uint64_t *off) {
    const uint64_t need = round_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const uint64_t start = it->first, rest = it->second - need;
      free_.erase(it);
      if (rest) free_[start + need] = rest;
      used_[start] = need;
      used_bytes_ += need;
      *off = start;
      return true;
    }
    return false;
  }

  // Return the block that starts at `off`; neighbours merge.  False if `off`
  // is not the start of a live block.
  bool release(uint64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    uint64_t start = off, len = u->second;
    used_.erase(u);
    used_bytes_ -= len;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && start + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
    return true;
  }

  // Whether a block of `bytes` could be allocated right now.
  bool fits(uint64_t bytes) const { return largest_free() >= round_up(bytes ? bytes : 1); }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (const auto &f : free_) m = f.second > m ? f.second : m;
    return m;
  }
  uint64_t size() const { return size_; }
  uint64_t used() const { return used_bytes_; }
  size_t free_blocks() const { return free_.size(); }
  size_t live_blocks() const { return used_.size(); }
  uint64_t round_up(uint64_t v) const { return (v + align_ - 1) / align_ * align_; }

 private:
  uint64_t size_ = 0, align_ = 1, used_bytes_ = 0;
  std::map<uint64_t, uint64_t> free_; // start -> length, disjoint, never adjacent
  std::map<uint64_t, uint64_t> used_; // start -> length
};

} // namespace alnrt
