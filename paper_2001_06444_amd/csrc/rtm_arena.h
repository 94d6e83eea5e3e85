// rtm_arena.h -- first-fit sub-allocator over one device buffer (host code).
//
// The library never calls hipMalloc on its working paths: every wavefield,
// boundary/snapshot store, image and statistics array is carved out of one
// caller-provided device arena.  Blocks are 256-byte aligned (rows of the
// wavefields are 256-byte aligned relative to the block), free ranges are
// kept sorted by offset and merged with both neighbours on release.  Plain
// C++ (no HIP): the host-side unit test builds it with the sanitizers.
#pragma once

#include <stddef.h>

#include <algorithm>
#include <iterator>
#include <map>
#include <mutex>

namespace rtm {

inline size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

class Arena {
 public:
  void init(void* base, size_t size) {
    base_ = static_cast<char*>(base);
    size_ = size;
    free_.clear();
    free_[0] = size;
    used_ = peak_ = 0;
  }
  void* alloc(size_t n) {
    std::lock_guard<std::mutex> lk(mu_);
    n = align256(n ? n : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        size_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > n) free_[off + n] = sz - n;
        used_ += n;
        peak_ = std::max(peak_, used_);
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(void* p, size_t n) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    n = align256(n ? n : 1);
    size_t off = static_cast<char*>(p) - base_;
    used_ -= n;
    auto it = free_.emplace(off, n).first;
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
  size_t size() const { return size_; }
  size_t used() {
    std::lock_guard<std::mutex> lk(mu_);
    return used_;
  }
  size_t peak() {
    std::lock_guard<std::mutex> lk(mu_);
    return peak_;
  }

 private:
  std::mutex mu_;
  char* base_ = nullptr;
  size_t size_ = 0;
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

}  // namespace rtm
