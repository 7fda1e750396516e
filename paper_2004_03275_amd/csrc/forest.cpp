// forest.cpp -- host-side block forest: validation and neighbour tables.
//
// A forest is a list of leaves (level, block coordinates at that level) of a
// quadtree/octree with refinement ratio 2 (arXiv 2004.03275, Sec. 1.3).  The
// tables built here tell every kernel, per leaf face, whether the neighbour is
// on the same level, coarser, finer or a physical boundary, and give each
// coarse-fine face a slot in the ghost / flux slab arrays.
#include "forest.hpp"

#include <cstdio>

#include "leafhash.hpp"
#include "parallel.hpp"

namespace amrv {

int build_tables(const amrv_config& c, int64_t n, const int32_t* lev, const int32_t* ijk, Tables& t) {
  t = Tables();
  auto fail = [&](int code, const char* msg) {
    t.err = msg;
    return code;
  };
  if (n <= 0 || !lev || !ijk) return fail(AMRV_EINVAL, "empty or null leaf list");
  if (n > (int64_t)1 << 30) return fail(AMRV_EINVAL, "too many leaves");
  if (c.ndim < 1 || c.ndim > 3) return fail(AMRV_EINVAL, "ndim must be 1, 2 or 3");
  if (c.nghost != 2) return fail(AMRV_EINVAL, "nghost must be 2");
  if (c.max_level < 1 || c.max_level > MAXLEV - 1) return fail(AMRV_EINVAL, "max_level out of range");
  if (c.physics != AMRV_EULER && c.physics != AMRV_MHD_GLM && c.physics != AMRV_POLYTROPE)
    return fail(AMRV_EINVAL, "unknown physics");
  if (c.flux < AMRV_TVDLF || c.flux > AMRV_HLLC) return fail(AMRV_EINVAL, "unknown flux");
  if (c.limiter != AMRV_MINMOD && c.limiter != AMRV_VANLEER && c.limiter != AMRV_MC && c.limiter != AMRV_KOREN &&
      c.limiter != AMRV_CADA)
    return fail(AMRV_EINVAL, "unknown limiter");
  if (c.rk_stages != 2 && c.rk_stages != 3) return fail(AMRV_EINVAL, "rk_stages must be 2 or 3");
  if (!(c.cada_radius >= 0.0) || !(c.cada_radius < 1e300)) return fail(AMRV_EINVAL, "bad Cada radius");
  if (c.physics == AMRV_POLYTROPE) {
    if (!(c.gamma >= 1.0) || !(c.cad > 0.0) || !(c.cfl > 0.0))
      return fail(AMRV_EINVAL, "the polytrope needs gamma >= 1, c_ad > 0 and a positive cfl");
    if (c.flux == AMRV_HLLC) return fail(AMRV_EINVAL, "HLLC needs the energy equation (not the polytrope)");
  } else if (!(c.gamma > 1.0) || !(c.cfl > 0.0)) {
    return fail(AMRV_EINVAL, "gamma must exceed 1 and cfl be positive");
  }
  const int nd = c.ndim;
  for (int d = 0; d < nd; d++) {
    if (c.block_nx[d] < 4 || (c.block_nx[d] & 1)) return fail(AMRV_EINVAL, "block_nx must be even and >= 4");
    if (c.base_blocks[d] < 1) return fail(AMRV_EINVAL, "base_blocks must be >= 1");
    if (!(c.xmax[d] > c.xmin[d])) return fail(AMRV_EINVAL, "xmax must exceed xmin");
    if (c.bc[d][0] != c.bc[d][1] || c.bc[d][0] < 0 || c.bc[d][0] > 1)
      return fail(AMRV_EINVAL, "bc must be periodic or zero-gradient on both sides");
  }
  if (nd > 1) {
    for (int d = 0; d < nd; d++)
      if (c.block_nx[d] != 16) return fail(AMRV_ENOTSUP, "2D/3D kernels use 16-cell blocks");
  } else if (c.block_nx[0] > (1 << 20)) {
    return fail(AMRV_ENOTSUP, "1D block too large");
  }

  t.nd = nd;
  t.nx = c.block_nx[0];
  t.n = n;
  t.ncell = 1;
  for (int d = 0; d < nd; d++) t.ncell *= c.block_nx[d];
  t.T = t.ncell / t.nx;
  t.nvar = c.physics == AMRV_MHD_GLM ? 3 + 2 * nd : c.physics == AMRV_POLYTROPE ? 1 + nd : 2 + nd;

  auto nblk = [&](int l, int d) -> int64_t { return d < nd ? (int64_t)c.base_blocks[d] << (l - 1) : 1; };
  auto periodic = [&](int d) { return c.bc[d][0] == AMRV_BC_PERIODIC; };

  for (int d = 0; d < nd; d++)
    if (nblk(c.max_level, d) >= LeafHash::kMaxBlocks) return fail(AMRV_EINVAL, "domain too large in blocks");
  LeafHash idx((size_t)n);
  t.lvl.assign(lev, lev + n);
  t.ijk.assign(ijk, ijk + 3 * n);
  for (int64_t b = 0; b < n; b++) {
    const int l = lev[b];
    if (l < 1 || l > c.max_level) return fail(AMRV_EINVAL, "leaf level out of range");
    for (int d = 0; d < 3; d++)
      if (ijk[3 * b + d] < 0 || ijk[3 * b + d] >= nblk(l, d)) return fail(AMRV_EINVAL, "leaf coordinate out of range");
    const uint64_t key = LeafHash::key(l, ijk[3 * b], ijk[3 * b + 1], ijk[3 * b + 2]);
    if (idx.get(key) >= 0) return fail(AMRV_EUNBALANCED, "duplicate leaf");
    idx.put(key, (int32_t)b);
  }
  // The checks and tables below run over chunks of the leaf list on a few
  // threads.  A chunk stops at its first failing leaf; the failure of the
  // lowest chunk is reported, i.e. the first failing leaf in list order,
  // as a serial pass would.
  struct ChunkErr {
    int code = AMRV_OK;
    const char* msg = nullptr;
  };
  constexpr int MAXCH = 16;
  ChunkErr errs[MAXCH];
  bool ok = true;
  auto first_error = [&]() -> int {
    if (!ok) return fail(AMRV_ENOMEM, "host out of memory");
    for (const ChunkErr& e : errs)
      if (e.msg) return fail(e.code, e.msg);
    return AMRV_OK;
  };

  // cover without overlap: no leaf below another, total volume = domain
  int64_t dom = 1;
  for (int d = 0; d < nd; d++) dom *= c.base_blocks[d];
  dom <<= nd * (c.max_level - 1);
  int64_t vols[MAXCH] = {0};
  parallel_chunks(n, [&](int ci, int64_t b0, int64_t b1) {
    int64_t v = 0;
    for (int64_t b = b0; b < b1; b++) {
      const int l = lev[b];
      for (int a = 1; a < l; a++) {
        const int sh = l - a;
        if (idx.find(a, ijk[3 * b] >> sh, nd > 1 ? ijk[3 * b + 1] >> sh : 0, nd > 2 ? ijk[3 * b + 2] >> sh : 0) >= 0) {
          errs[ci] = {AMRV_EUNBALANCED, "leaf overlaps a coarser leaf"};
          return;
        }
      }
      v += (int64_t)1 << (nd * (c.max_level - l));
    }
    vols[ci] = v;
  }, &ok);
  if (int rc = first_error()) return rc;
  int64_t vol = 0;
  for (int64_t v : vols) vol += v;
  if (vol != dom) return fail(AMRV_EUNBALANCED, "leaves do not cover the domain");

  // 2:1 balance over faces, edges and corners
  auto wrapc = [&](int d, int64_t& x, int64_t ext) {
    if (x >= 0 && x < ext) return true;
    if (!periodic(d)) return false;
    x = ((x % ext) + ext) % ext;
    return true;
  };
  int nofs = 1;
  for (int d = 0; d < nd; d++) nofs *= 3;
  parallel_chunks(n, [&](int ci, int64_t b0, int64_t b1) {
    for (int64_t b = b0; b < b1; b++) {
      const int l = lev[b];
      for (int q = 0; q < nofs; q++) {
        int o[3] = {0, 0, 0}, r = q;
        bool zero = true;
        for (int d = 0; d < nd; d++) {
          o[d] = r % 3 - 1;
          r /= 3;
          zero = zero && o[d] == 0;
        }
        if (zero) continue;
        int64_t x[3] = {0, 0, 0};
        bool in = true;
        for (int d = 0; d < nd; d++) {
          x[d] = ijk[3 * b + d] + o[d];
          in = in && wrapc(d, x[d], nblk(l, d));
        }
        if (!in) continue;
        if (idx.find(l, x[0], x[1], x[2]) >= 0) continue;
        if (l > 1 && idx.find(l - 1, x[0] >> 1, x[1] >> 1, x[2] >> 1) >= 0) continue;
        bool bad = l + 1 > c.max_level;
        for (int ch = 0; ch < (1 << nd) && !bad; ch++) {
          int64_t y[3] = {0, 0, 0};
          bool touch = true;
          for (int d = 0; d < nd; d++) {
            const int bit = (ch >> d) & 1;
            if ((o[d] == 1 && bit) || (o[d] == -1 && !bit)) touch = false;
            y[d] = 2 * x[d] + bit;
          }
          bad = touch && idx.find(l + 1, y[0], y[1], y[2]) < 0;
        }
        if (bad) {
          errs[ci] = {AMRV_EUNBALANCED, "forest is not 2:1 balanced"};
          return;
        }
      }
    }
  }, &ok);
  if (int rc = first_error()) return rc;

  // faces: kind and neighbour (per leaf), then slots in leaf and face order
  t.kind.assign((size_t)6 * n, (int8_t)NB_BND);
  t.nbr.assign((size_t)6 * n, -1);
  t.slot.assign((size_t)6 * n, -1);
  parallel_chunks(n, [&](int, int64_t b0, int64_t b1) {
    for (int64_t b = b0; b < b1; b++) {
      const int l = lev[b];
      for (int f = 0; f < 2 * nd; f++) {
        const int d = f >> 1, s = (f & 1) ? 1 : -1;
        int64_t x[3] = {ijk[3 * b], ijk[3 * b + 1], ijk[3 * b + 2]};
        x[d] += s;
        int8_t k;
        int32_t nb;
        if (!wrapc(d, x[d], nblk(l, d))) {
          k = NB_BND;
          nb = (int32_t)b;
        } else if ((nb = idx.find(l, x[0], x[1], x[2])) >= 0) {
          k = NB_SAME;
        } else if (l > 1 && (nb = idx.find(l - 1, x[0] >> 1, x[1] >> 1, x[2] >> 1)) >= 0) {
          k = NB_COARSER;
        } else {
          k = NB_FINER;
          nb = -1;
        }
        t.kind[6 * b + f] = k;
        t.nbr[6 * b + f] = nb;
      }
    }
  }, &ok);
  if (int rc = first_error()) return rc;
  for (int64_t b = 0; b < n; b++)
    for (int f = 0; f < 2 * nd; f++) {
      const int8_t k = t.kind[6 * b + f];
      if (k != NB_COARSER && k != NB_FINER) continue;
      t.slot[6 * b + f] = (int32_t)t.sleaf.size();
      t.sleaf.push_back((int32_t)b);
      t.sface.push_back(f);
      if (k == NB_FINER)
        t.rlist.push_back(t.slot[6 * b + f]);
      else
        t.plist.push_back(t.slot[6 * b + f]);
    }
  t.nslot = (int)t.sleaf.size();
  t.fslot.assign((size_t)4 * t.nslot, -1);
  parallel_chunks(t.nslot, [&](int ci, int64_t s0, int64_t s1) {
    for (int64_t s = s0; s < s1; s++) {
      const int64_t b = t.sleaf[s];
      const int f = t.sface[s];
      if (t.kind[6 * b + f] != NB_FINER) continue;
      const int l = lev[b];
      const int d = f >> 1, side = (f & 1) ? 1 : -1;
      int64_t x[3] = {ijk[3 * b], ijk[3 * b + 1], ijk[3 * b + 2]};
      x[d] += side;
      wrapc(d, x[d], nblk(l, d));
      const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
      const int nq = 1 << (nd - 1);
      for (int q = 0; q < nq; q++) {
        int64_t y[3] = {2 * x[0], nd > 1 ? 2 * x[1] : 0, nd > 2 ? 2 * x[2] : 0};
        y[d] += side < 0 ? 1 : 0;
        if (nd > 1) y[e1] += q & 1;
        if (nd > 2) y[e2] += (q >> 1) & 1;
        const int32_t fl = idx.find(l + 1, y[0], y[1], y[2]);
        if (fl < 0) {
          errs[ci] = {AMRV_EUNBALANCED, "finer neighbour is not a leaf"};
          return;
        }
        const int back = 2 * d + (side < 0 ? 1 : 0);
        if (t.kind[6 * fl + back] != NB_COARSER) {
          errs[ci] = {AMRV_EUNBALANCED, "inconsistent coarse-fine face"};
          return;
        }
        t.fslot[4 * s + q] = t.slot[6 * fl + back];
      }
    }
  }, &ok);
  if (int rc = first_error()) return rc;
  return AMRV_OK;
}

}  // namespace amrv
