// Ring allocator over a byte range [0, size): space is handed out in
// allocation order (first-in, first-out), like the admission queue of a
// server, and comes back when released, in any order; the oldest live
// allocation bounds the free space, so space released out of order is reused
// once everything allocated before it has been released too.  Host-only, no
// locking (the owner serialises calls).  Offsets are multiples of `align`.
#pragma once

#include <stdint.h>

#include <deque>

namespace cm {

class RingAlloc {
 public:
  explicit RingAlloc(uint64_t size, uint64_t align = 256) : size_(size - size % align), align_(align) {}

  uint64_t size() const { return size_; }
  uint64_t used() const { return used_; }  // bytes of the allocations not yet released
  bool empty() const { return live_.empty(); }

  // Offset of `bytes` (rounded up to the alignment) or -1 if they do not fit
  // now.  Zero bytes always succeed at offset 0 and take no space.
  int64_t alloc(uint64_t bytes, uint64_t id) {
    if (bytes == 0) return 0;
    const uint64_t len = (bytes + align_ - 1) / align_ * align_;
    if (len > size_) return -1;
    uint64_t off;
    if (live_.empty()) {
      off = 0;
    } else {
      const Entry& front = live_.front();
      const Entry& back = live_.back();
      const uint64_t end = back.off + back.len;
      if (back.off >= front.off) {  // live range [front.off, end) does not wrap
        if (end + len <= size_)
          off = end;
        else if (len <= front.off)
          off = 0;  // wrap; [end, size) stays unused until the ring drains past it
        else
          return -1;
      } else {  // wrapped: free space is [end, front.off)
        if (end + len <= front.off)
          off = end;
        else
          return -1;
      }
    }
    live_.push_back(Entry{off, len, id, false});
    used_ += len;
    return (int64_t)off;
  }

  // Returns false if id is not live.
  bool release(uint64_t id) {
    for (Entry& e : live_) {
      if (e.id == id && !e.released) {
        e.released = true;
        used_ -= e.len;
        while (!live_.empty() && live_.front().released) live_.pop_front();
        return true;
      }
    }
    return false;
  }

 private:
  struct Entry {
    uint64_t off, len, id;
    bool released;
  };
  uint64_t size_, align_;
  uint64_t used_ = 0;
  std::deque<Entry> live_;
};

}  // namespace cm
