/*
 * lk_arena.hpp -- best-fit allocator over one slice of a device arena (byte offsets only;
 * it never touches the memory).  Used by the serving loop to carve request outputs out of
 * the caller's device-memory budget.
 *
 * Free blocks are indexed twice: by offset (to merge a freed block with its neighbours)
 * and by (length, offset) (to find the smallest block that fits).  Allocation and release
 * are O(log #free blocks), so a fragmented arena does not slow admission down.
 */
#ifndef LK_ARENA_HPP
#define LK_ARENA_HPP

#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>
#include <set>
#include <utility>

namespace lksrv {

class Arena {
 public:
  static constexpr uint64_t kGranule = 256;  // every block starts and ends 256-byte aligned

  Arena(uint64_t base, uint64_t size) : base_(base), size_(size / kGranule * kGranule) {
    if (size_) insert(0, size_);
  }

  // Best fit: the smallest free block that holds `bytes` (rounded up to the granule),
  // lowest offset among equals.  Returns false, changing nothing, if none does.
  bool alloc(uint64_t bytes, uint64_t *addr) {
    bytes = round(bytes);
    if (bytes == 0) bytes = kGranule;
    auto it = by_len_.lower_bound({bytes, 0});
    if (it == by_len_.end()) return false;
    const uint64_t len = it->first, off = it->second;
    erase(off, len);
    if (len > bytes) insert(off + bytes, len - bytes);
    used_ += bytes;
    peak_ = std::max(peak_, used_);
    *addr = base_ + off;
    return true;
  }

  // Return a block obtained from alloc with the same `bytes`; merges with free neighbours.
  void release(uint64_t addr, uint64_t bytes) {
    bytes = round(bytes);
    if (bytes == 0) bytes = kGranule;
    uint64_t off = addr - base_;
    used_ -= bytes;
    auto next = by_off_.lower_bound(off);
    if (next != by_off_.end() && off + bytes == next->first) {
      const uint64_t nlen = next->second;
      erase(next->first, nlen);
      bytes += nlen;
    }
    next = by_off_.lower_bound(off);
    if (next != by_off_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        const uint64_t poff = prev->first, plen = prev->second;
        erase(poff, plen);
        off = poff;
        bytes += plen;
      }
    }
    insert(off, bytes);
  }

  uint64_t size() const { return size_; }
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }
  size_t free_blocks() const { return by_off_.size(); }
  // Largest free block (0 if none).
  uint64_t largest_free() const { return by_len_.empty() ? 0 : by_len_.rbegin()->first; }
  // Visit free blocks in offset order: f(offset, length).
  template <class F>
  void for_each_free(F f) const {
    for (const auto &b : by_off_) f(b.first, b.second);
  }
  static uint64_t round(uint64_t b) { return (b + kGranule - 1) / kGranule * kGranule; }

 private:
  void insert(uint64_t off, uint64_t len) {
    by_off_[off] = len;
    by_len_.insert({len, off});
  }
  void erase(uint64_t off, uint64_t len) {
    by_off_.erase(off);
    by_len_.erase({len, off});
  }

  uint64_t base_, size_, used_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> by_off_;            // offset -> length
  std::set<std::pair<uint64_t, uint64_t>> by_len_;  // (length, offset)
};

}  // namespace lksrv

#endif  // LK_ARENA_HPP
