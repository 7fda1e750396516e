// parallel.hpp -- split a host loop over [0, n) into contiguous chunks on a
// few threads (forest tables and regrid plans of large leaf lists).
#pragma once
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

namespace amrv {

// fn(chunk, begin, end) for chunks [begin, end) of [0, n), chunk = 0, 1, ...
// in order; returns the number of chunks.  Serial below two grains.  An
// exception inside a chunk is caught and reported as false in *ok.
template <class Fn>
int parallel_chunks(int64_t n, Fn&& fn, bool* ok, int64_t grain = 2048) {
  const unsigned hw = std::thread::hardware_concurrency();
  const int64_t want = std::min<int64_t>(std::min<int64_t>(hw ? hw : 1, 16), (n + grain - 1) / grain);
  const int nt = (int)std::max<int64_t>(1, want);
  const int64_t chunk = (n + nt - 1) / std::max(nt, 1);
  std::atomic<bool> good{true};
  auto run = [&](int i) {
    const int64_t b = (int64_t)i * chunk, e = std::min(n, b + chunk);
    try {
      if (b < e) fn(i, b, e);
    } catch (...) {
      good = false;
    }
  };
  if (nt == 1) {
    run(0);
  } else {
    std::vector<std::thread> th;
    th.reserve((size_t)nt - 1);
    try {
      for (int i = 1; i < nt; i++) th.emplace_back(run, i);
    } catch (...) {
      good = false;
    }
    run(0);
    for (auto& t : th) t.join();
    // chunks whose thread could not be started run here
    for (int i = (int)th.size() + 1; i < nt; i++) run(i);
  }
  if (ok) *ok = good.load();
  return nt;
}

}  // namespace amrv
