// regrid.cpp -- host-side regrid plan of a block forest (arXiv 2004.03275,
// Sec. 1.3: refinement ratio 2, a block is refined when flagged, coarsened
// only when all of its cells are below the coarsening fraction of the
// tolerance, i.e. when all 2^d siblings of a parent are flagged -1).
//
// Rules (the balance of the result is 2:1 over faces, edges and corners):
//   1. a leaf flagged +1 below max_level is split into its 2^d children;
//   2. every leaf touching a splitting leaf from one level coarser is split
//      as well, repeated until nothing changes (worklist over the touching-
//      leaf lists below);
//   3. a complete group of 2^d sibling leaves, all flagged -1, none split,
//      above level 1, is merged into its parent unless a leaf touching the
//      group ends (after steps 1-2, other merges ignored) finer than the
//      group's level;
//   4. new order: unchanged leaves in place, a split leaf replaced by its
//      children (child index ox + 2 oy + 4 oz), a merged group by its parent
//      at the position of its first member.
#include "regrid.hpp"

#include <algorithm>

#include "leafhash.hpp"
#include "parallel.hpp"

namespace amrv {

namespace {

struct LeafIndex {
  LeafHash h;
  explicit LeafIndex(const Tables& t) : h((size_t)t.n) {
    for (int64_t b = 0; b < t.n; b++)
      h.put(LeafHash::key(t.lvl[b], t.ijk[3 * b], t.ijk[3 * b + 1], t.ijk[3 * b + 2]), (int32_t)b);
  }
  int32_t at(int l, const int64_t c[3]) const { return h.find(l, c[0], c[1], c[2]); }
};

}  // namespace

int regrid_plan(const amrv_config& c, const Tables& t, const int8_t* flags, std::vector<int32_t>& out_lev,
                std::vector<int32_t>& out_ijk, std::string& err) {
  const int nd = t.nd, nch = 1 << nd;
  const int64_t n = t.n;
  const LeafIndex ix(t);
  auto blocks = [&](int l, int d) -> int64_t { return d < nd ? (int64_t)c.base_blocks[d] << (l - 1) : 1; };

  // touching leaves of every leaf: for each of the 3^d - 1 neighbouring block
  // positions, the leaf covering it (same level or one coarser) or the finer
  // leaves of that position adjacent to this leaf
  // built in chunks of the leaf list on a few threads, then concatenated in
  // leaf order (toff[b] .. toff[b+1] in tlist)
  constexpr int MAXCH = 16;
  std::vector<int32_t> clist[MAXCH];
  std::vector<int64_t> toff((size_t)n + 1, 0);
  int nofs = 1;
  for (int d = 0; d < nd; d++) nofs *= 3;
  bool ok = true;
  const int nchunks = parallel_chunks(n, [&](int ci, int64_t b0, int64_t b1) {
    std::vector<int32_t>& tl = clist[ci];
    tl.reserve((size_t)(b1 - b0) * 32);
    for (int64_t b = b0; b < b1; b++) {
      const int l = t.lvl[b];
      const size_t t0 = tl.size();
      for (int q = 0; q < nofs; q++) {
        int o[3] = {0, 0, 0};
        bool zero = true;
        for (int d = 0, r = q; d < nd; d++, r /= 3) {
          o[d] = r % 3 - 1;
          zero = zero && o[d] == 0;
        }
        if (zero) continue;
        int64_t x[3] = {0, 0, 0};
        bool inside = true;
        for (int d = 0; d < nd; d++) {
          x[d] = t.ijk[3 * b + d] + o[d];
          const int64_t ext = blocks(l, d);
          if (x[d] < 0 || x[d] >= ext) {
            if (c.bc[d][0] != AMRV_BC_PERIODIC) inside = false;
            x[d] = ((x[d] % ext) + ext) % ext;
          }
        }
        if (!inside) continue;
        int32_t a = ix.at(l, x);
        if (a < 0) {
          const int64_t p[3] = {x[0] >> 1, x[1] >> 1, x[2] >> 1};
          a = ix.at(l - 1, p);
        }
        if (a >= 0) {
          tl.push_back(a);
          continue;
        }
        for (int ch = 0; ch < nch; ch++) {
          int64_t y[3] = {0, 0, 0};
          bool adj = true;
          for (int d = 0; d < nd; d++) {
            const int bit = (ch >> d) & 1;
            if ((o[d] > 0 && bit) || (o[d] < 0 && !bit)) adj = false;
            y[d] = 2 * x[d] + bit;
          }
          if (!adj) continue;
          const int32_t f = ix.at(l + 1, y);
          if (f >= 0) tl.push_back(f);
        }
      }
      // duplicates (a coarser leaf touching along a face and its edges) and
      // the leaf itself (periodic wrap of a one-block domain) may remain: the
      // closure and the merge test below give the same result with them
      toff[(size_t)b + 1] = (int64_t)(tl.size() - t0);  // count, summed below
    }
  }, &ok);
  if (!ok) {
    err = "host out of memory";
    return AMRV_ENOMEM;
  }
  std::vector<int32_t> tlist;
  size_t total = 0;
  for (int ci = 0; ci < nchunks; ci++) total += clist[ci].size();
  tlist.reserve(total);
  for (int ci = 0; ci < nchunks; ci++) tlist.insert(tlist.end(), clist[ci].begin(), clist[ci].end());
  for (int64_t b = 0; b < n; b++) toff[(size_t)b + 1] += toff[(size_t)b];
  auto touching = [&](int32_t b) {
    return std::make_pair(tlist.data() + toff[(size_t)b], tlist.data() + toff[(size_t)b + 1]);
  };

  // steps 1-2: final level of every leaf after splitting
  std::vector<int32_t> fin(t.lvl.begin(), t.lvl.end());
  std::vector<int32_t> work;
  for (int64_t b = 0; b < n; b++)
    if (flags[b] > 0 && t.lvl[b] < c.max_level) {
      fin[b] = t.lvl[b] + 1;
      work.push_back((int32_t)b);
    }
  while (!work.empty()) {
    const int32_t b = work.back();
    work.pop_back();
    const auto tb = touching(b);
    for (const int32_t* p = tb.first; p != tb.second; p++) {
      const int32_t a = *p;
      if (t.lvl[a] == t.lvl[b] - 1 && fin[a] == t.lvl[a]) {
        fin[a] = t.lvl[a] + 1;
        work.push_back(a);
      }
    }
  }

  // step 3: merges; head[b] = first member (list order) of b's merged group
  std::vector<int32_t> head((size_t)n, -1);
  std::vector<int8_t> seen((size_t)n, 0);  // the leaf's sibling group was examined
  for (int64_t b = 0; b < n; b++) {
    const int l = t.lvl[b];
    if (flags[b] >= 0 || l <= 1 || fin[b] != l || seen[b]) continue;
    int32_t mem[8];
    bool ok = true;
    for (int ch = 0; ch < nch && ok; ch++) {
      int64_t y[3] = {0, 0, 0};
      for (int d = 0; d < nd; d++) y[d] = 2 * (t.ijk[3 * b + d] >> 1) + ((ch >> d) & 1);
      mem[ch] = ix.at(l, y);
      ok = mem[ch] >= 0 && flags[mem[ch]] < 0 && fin[mem[ch]] == l;
    }
    if (!ok) continue;
    for (int ch = 0; ch < nch; ch++) seen[mem[ch]] = 1;
    for (int ch = 0; ch < nch && ok; ch++) {
      const auto tm = touching(mem[ch]);
      for (const int32_t* p = tm.first; p != tm.second; p++) {
        const int32_t a = *p;
        if (std::find(mem, mem + nch, a) != mem + nch) continue;
        if (fin[a] > l) {
          ok = false;
          break;
        }
      }
    }
    if (!ok) continue;
    const int32_t first = *std::min_element(mem, mem + nch);
    for (int ch = 0; ch < nch; ch++) head[mem[ch]] = first;
  }

  // step 4: the new leaf list
  out_lev.clear();
  out_ijk.clear();
  for (int64_t b = 0; b < n; b++) {
    const int l = t.lvl[b];
    const int32_t* x = &t.ijk[3 * b];
    if (head[b] >= 0) {
      if (head[b] != b) continue;
      out_lev.push_back(l - 1);
      for (int d = 0; d < 3; d++) out_ijk.push_back(d < nd ? x[d] >> 1 : 0);
    } else if (fin[b] > l) {
      for (int ch = 0; ch < nch; ch++) {
        out_lev.push_back(l + 1);
        for (int d = 0; d < 3; d++) out_ijk.push_back(d < nd ? 2 * x[d] + ((ch >> d) & 1) : 0);
      }
    } else {
      out_lev.push_back(l);
      for (int d = 0; d < 3; d++) out_ijk.push_back(x[d]);
    }
  }
  (void)err;
  return AMRV_OK;
}

int regrid_sources(const Tables& from, const Tables& to, std::vector<int32_t>& src, std::string& err) {
  const int nd = from.nd, nch = 1 << nd;
  const LeafIndex ix(from);
  src.assign((size_t)to.n * XFER_STRIDE, -1);
  for (int64_t b = 0; b < to.n; b++) {
    const int l = to.lvl[b];
    const int64_t x[3] = {to.ijk[3 * b], to.ijk[3 * b + 1], to.ijk[3 * b + 2]};
    int32_t* s = &src[(size_t)b * XFER_STRIDE];
    if ((s[1] = ix.at(l, x)) >= 0) {
      s[0] = XFER_COPY;
      continue;
    }
    const int64_t p[3] = {x[0] >> 1, x[1] >> 1, x[2] >> 1};
    if ((s[1] = ix.at(l - 1, p)) >= 0) {
      s[0] = XFER_PROLONG;
      continue;
    }
    s[0] = XFER_RESTRICT;
    for (int ch = 0; ch < nch; ch++) {
      int64_t y[3] = {0, 0, 0};
      for (int d = 0; d < nd; d++) y[d] = 2 * x[d] + ((ch >> d) & 1);
      if ((s[1 + ch] = ix.at(l + 1, y)) < 0) {
        err = "the target forest is not a one-level regrid of the source forest";
        return AMRV_EINVAL;
      }
    }
  }
  return AMRV_OK;
}

}  // namespace amrv
