// Offset bookkeeping of a first-fit arena: one contiguous block of `capacity`
// bytes handed out in 256-byte aligned pieces; free pieces are kept sorted by
// offset and merged with their neighbours on release.  No device calls here:
// the serving loop maps offsets onto one device allocation, which keeps
// hipMalloc / hipFree (and the device-wide synchronisation of hipFree) out of
// the loop.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <mutex>
#include <unordered_map>

namespace pico {

class OffsetArena {
 public:
  static constexpr size_t kAlign = 256;
  static constexpr size_t kNone = ~size_t(0);

  static size_t round_up(size_t bytes) { return ((bytes ? bytes : 1) + kAlign - 1) / kAlign * kAlign; }

  explicit OffsetArena(size_t capacity = 0) { reset(capacity); }

  void reset(size_t capacity) {
    cap_ = capacity / kAlign * kAlign;
    used_ = 0;
    free_.clear();
    live_.clear();
    if (cap_) free_[0] = cap_;
  }

  // offset of a piece of at least `bytes`, or kNone when no free piece fits
  size_t alloc(size_t bytes) {
    const size_t need = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const size_t off = it->first, rest = it->second - need;
      free_.erase(it);
      if (rest) free_[off + need] = rest;
      live_[off] = need;
      used_ += need;
      return off;
    }
    return kNone;
  }

  // returns false for an offset that is not a live piece
  bool release(size_t off) {
    auto lv = live_.find(off);
    if (lv == live_.end()) return false;
    size_t start = off, len = lv->second;
    used_ -= len;
    live_.erase(lv);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
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

  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }
  size_t free_pieces() const { return free_.size(); }
  size_t live_pieces() const { return live_.size(); }

 private:
  size_t cap_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;            // offset -> length, disjoint, merged
  std::unordered_map<size_t, size_t> live_;  // offset -> length
};

// One device allocation carved by an OffsetArena; thread-safe.
struct DeviceArena {
  OffsetArena book;
  char* base = nullptr;
  std::mutex mu;

  void* alloc(size_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    const size_t off = book.alloc(bytes);
    return off == OffsetArena::kNone ? nullptr : base + off;
  }
  bool release(void* p) {
    std::lock_guard<std::mutex> lk(mu);
    return book.release(static_cast<size_t>(static_cast<char*>(p) - base));
  }
};

}  // namespace pico
