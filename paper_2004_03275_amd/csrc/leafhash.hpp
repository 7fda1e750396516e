// leafhash.hpp -- open-addressing hash from a leaf key (level, block
// coordinates at that level) to the leaf's index, for the host-side forest,
// regrid and transfer code.  Linear probing in a power-of-two table at most
// half full; a key never equals the empty marker.
#pragma once
#include <stdint.h>

#include <vector>

namespace amrv {

class LeafHash {
 public:
  // coordinates below 2^19 blocks a side, levels below 64
  static constexpr int64_t kMaxBlocks = int64_t(1) << 19;

  explicit LeafHash(size_t n) {
    size_t cap = 16;
    while (cap < 2 * n + 16) cap <<= 1;
    tab_.assign(cap, Entry{kEmpty, -1, 0});
    mask_ = cap - 1;
  }

  static uint64_t key(int l, int64_t i, int64_t j, int64_t k) {
    return (uint64_t(l) << 57) | (uint64_t(i) << 38) | (uint64_t(j) << 19) | uint64_t(k);
  }

  void put(uint64_t k, int32_t v) {
    size_t h = slot(k);
    while (tab_[h].key != kEmpty && tab_[h].key != k) h = (h + 1) & mask_;
    tab_[h] = Entry{k, v, 0};
  }

  // the leaf index, or -1
  int32_t get(uint64_t k) const {
    for (size_t h = slot(k);; h = (h + 1) & mask_) {
      const Entry& e = tab_[h];
      if (e.key == k) return e.val;
      if (e.key == kEmpty) return -1;
    }
  }

  // (level, coordinates) lookup with the range checks of a block position
  int32_t find(int l, int64_t i, int64_t j, int64_t k) const {
    if (l < 1 || i < 0 || j < 0 || k < 0 || i >= kMaxBlocks || j >= kMaxBlocks || k >= kMaxBlocks) return -1;
    return get(key(l, i, j, k));
  }

 private:
  static constexpr uint64_t kEmpty = ~uint64_t(0);
  struct Entry {  // 16 bytes: key and value in one cache line
    uint64_t key;
    int32_t val;
    int32_t unused;
  };
  size_t slot(uint64_t k) const {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    return size_t(k) & mask_;
  }
  std::vector<Entry> tab_;
  size_t mask_ = 0;
};

}  // namespace amrv
