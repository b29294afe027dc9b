// Workspace arena of a context: first-fit allocation of byte ranges of the
// caller's workspace.  Every user of the workspace -- blocking calls and
// serving requests alike -- takes its range from here under the context
// mutex, so ranges in use never overlap.  Offsets are multiples of 256 bytes.
// Host-only code (no HIP), so the bookkeeping can be checked on the CPU.
#pragma once
#include <cstddef>
#include <utility>
#include <vector>

namespace corutv {

class Arena {
 public:
  explicit Arena(size_t capacity = 0) : cap_(capacity) {}
  void reset(size_t capacity) {
    cap_ = capacity;
    used_.clear();
  }
  size_t capacity() const { return cap_; }
  // First range of `bytes` bytes at a 256-aligned offset that overlaps no
  // range in use; false if none is free.
  bool alloc(size_t bytes, size_t* off) {
    size_t cur = 0;
    for (size_t i = 0; i <= used_.size(); ++i) {
      const size_t end = i < used_.size() ? used_[i].first : cap_;
      if (end >= cur && end - cur >= bytes) {
        used_.insert(used_.begin() + i, {cur, cur + bytes});
        *off = cur;
        return true;
      }
      if (i < used_.size()) cur = align(used_[i].second);
    }
    return false;
  }
  // Release the range that starts at off (no-op for an unknown offset).
  bool release(size_t off) {
    for (size_t i = 0; i < used_.size(); ++i)
      if (used_[i].first == off) {
        used_.erase(used_.begin() + i);
        return true;
      }
    return false;
  }
  const std::vector<std::pair<size_t, size_t>>& ranges() const { return used_; }

 private:
  static size_t align(size_t x) { return (x + 255) / 256 * 256; }
  size_t cap_;
  std::vector<std::pair<size_t, size_t>> used_;  // [begin, end), sorted by begin
};

}  // namespace corutv
