// fmg.hip -- Helmholtz solver on a 2D or 3D block-adaptive forest
// (declared in include/amrv_mg.h; the multigrid of Sec. 1.4 on the block-
// adaptive quadtree / octree grid), by full-approximation-scheme V-cycles
// over the block tree.
//
// The problem on the leaf cells: lap(u) - lambda u = f, the (2d+1)-point lap
// of a cell at its own level, the value across a face from
//   a leaf cell at the same level;
//   the zero-Neumann mirror at a non-periodic domain face (periodic faces
//     wrap through the neighbour table);
//   the fine side of a coarse-fine face: (u + 2 u_c) / 3, u_c the coarse
//     leaf's cell across the face moved a quarter coarse cell along it in
//     each tangential direction with the coarse block's own difference there
//     (central, one-sided at its edges);
//   the coarse side: u + (4/3) (m - u), m the mean of the 2^(d-1) fine cells
//     touching the face -- the mean of the fine fluxes, so the scheme is
//     conservative.
//
// The tree: every leaf and every ancestor of a leaf is a block of 16^d
// cells, the blocks of a level stored one after another (level 1 first).  A
// parent holds the mean of its children's 2^d cells.  The grid of level l
// is every block of that level, relaxed with the plain stencil (a refined
// neighbour's own cells in place of the coarse side of a coarse-fine face;
// on the finest level this is the problem's stencil) and the right-hand
// side of the full approximation scheme L(u) + r: r the restricted residual
// of a parent, the problem's residual of a leaf (f itself where the plain
// stencil is the problem's).  So a coarse leaf and the refined block beside
// it relax one operator, and the fixed point is the problem's solution.
//
// A V-cycle: from the finest level down to level 2, `pre` red-black sweeps,
// the residual, its restriction with the state's into the parents, and the
// parents' coarse right-hand side; on level 1 (complete: base^d blocks)
// `pre` sweeps, then one V-cycle of the uniform-grid solver of multigrid.hip
// on the level-1 grid for the correction L(e) = r (from e = 0), then `post`
// sweeps; back up, every block adds the bi/trilinear interpolation (within
// its parent) of the parent's change since restriction, then `post` sweeps.
// A cycle has no host wait: a solve enqueues as many cycles as the previous
// solve needed, less one, before it first reads back the problem's residual
// over the leaves, then checks after every cycle (the stopping rule max |r|
// <= tol max |f|).  Kernels are templated on the dimension; a 256-thread
// workgroup walks a block plane by plane.
//
// Layout in the caller's workspace (256-byte aligned arrays):
//   tables   lvl, ij[3], nbr[6], chi[8], cnb[6], par per block (2D uses the
//            first entries); leaf -> block
//   u, f, fu, r, uo  [block][16^d] doubles (state, relaxation right-hand
//                 side, the problem's f, residual or restricted residual,
//                 restricted state)
//   the uniform solver's own workspace (its finest right-hand side and
//                 solution arrays are the level-1 grid, fgrid and vgrid)
//   red, tmp, part  two 64-bit maxima, eight leaf fields (reaction-diffusion
//                 and projection temporaries), per-leaf sums
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <array>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/amrv_mg.h"
#include "errors.hpp"
#include "mg_internal.hpp"

namespace {

using amrv::set_error;

constexpr int NB = 16;
constexpr int WG = 256;  // threads per workgroup: one 16 x 16 plane of a block at a time
constexpr int FMG_MAXL = 16;
constexpr int NBR_NONE = -1;  // no block of the same level across the face (a coarser leaf is)
constexpr int NBR_WALL = -2;  // a non-periodic domain face
constexpr int TS = 3, FS = 6, CS = 8;  // table strides per block: coordinates, faces, children (2D uses the first)
constexpr size_t ALIGN = 256;

template <int ND>
constexpr int ncb() {  // cells per block
  return ND == 3 ? NB * NB * NB : NB * NB;
}
template <int ND>
constexpr int nplanes() {
  return ND == 3 ? NB : 1;
}

struct FmgDev {
  const int* lvl;
  const int* ij;   // [block][TS]: block coordinates at its level
  const int* nbr;  // [block][FS]: -x, +x, -y, +y, -z, +z; a block index, NBR_NONE or NBR_WALL
  const int* chi;  // [block][CS]: children (x fastest), -1 for a leaf
  const int* cnb;  // [block][FS]: the coarser leaf across a face whose nbr is NBR_NONE
  const int* par;  // [block]: parent, -1 on level 1
  double* u;
  double* f;   // right-hand side of the relaxation: the problem's f on the finest level, else L(u) + r
  double* fu;  // the problem's f on the leaves
  double* r;
  double* uo;
  double lam;
  double ih2[FMG_MAXL + 1];  // 1/h^2 per level (1-based)
  double rh[FMG_MAXL + 1];   // 1/h per level
};

// a cell's index in its block, (x, y, z) with x fastest (z = 0 in 2D)
__host__ __device__ inline int cidx(const int* c) { return c[0] + NB * (c[1] + NB * c[2]); }

// a neighbour value in the form cv + w u(c)
struct Across {
  double cv, w;
};

// the value across face `face` (2d: -d, 2d + 1: +d) of cell c of block b, as
// cv + w u(c) (host-callable too, for checks of the tables on the CPU); the
// pair is returned by value: written through references, the compiler kept
// it in private memory, whose reload waits for every load in flight
template <int ND>
__host__ __device__ inline Across across(const FmgDev& g, int b, bool leaf, const int* c, int face) {
  constexpr int NCB = ncb<ND>();
  const int nb = g.nbr[FS * b + face];
  if (nb == NBR_WALL) {
    return {0.0, 1.0};
  }
  const int d = face >> 1;
  const bool lo = (face & 1) == 0;
  int C[3] = {c[0], c[1], c[2]};  // the neighbouring cell in the neighbouring block
  C[d] = lo ? NB - 1 : 0;
  if (nb >= 0) {
    const int* ch = g.chi + CS * nb;
    if (!leaf || ch[0] < 0) {
      return {g.u[(size_t)nb * NCB + cidx(C)], 0.0};
    }
    // the coarse side: the 2^(ND-1) fine cells of the neighbour's children
    // that touch the face, in its grid of 32^ND child cells
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < (1 << (ND - 1)); t++) {
      int F[3] = {0, 0, 0};
      int bit = 0;
#pragma unroll
      for (int e = 0; e < ND; e++) {
        if (e == d) {
          F[e] = 2 * C[e] + (lo ? 1 : 0);
        } else {
          F[e] = 2 * C[e] + ((t >> bit) & 1);
          bit++;
        }
      }
      const int fb = ch[(F[0] >> 4) + 2 * (F[1] >> 4) + 4 * (F[2] >> 4)];
      const int Fl[3] = {F[0] & (NB - 1), F[1] & (NB - 1), F[2] & (NB - 1)};
      s += g.u[(size_t)fb * NCB + cidx(Fl)];
    }
    return {((4.0 / 3.0) / (1 << (ND - 1))) * s, -1.0 / 3.0};
  }
  // the fine side: the coarser leaf across the face, its cell moved a quarter
  // cell toward this one along each tangential direction
  const int Cb = g.cnb[FS * b + face];
  int gc[3] = {0, 0, 0}, K[3] = {0, 0, 0};
#pragma unroll
  for (int e = 0; e < ND; e++) {
    gc[e] = g.ij[TS * b + e] * NB + c[e];
    K[e] = (gc[e] >> 1) - g.ij[TS * Cb + e] * NB;
  }
  K[d] = lo ? NB - 1 : 0;
  const double* p = g.u + (size_t)Cb * NCB + cidx(K);
  double val = p[0];
#pragma unroll
  for (int e = 0; e < ND; e++) {
    if (e == d) continue;
    const int st = e == 0 ? 1 : (e == 1 ? NB : NB * NB);
    const int t = K[e];
    double slope;
    if (t == 0)
      slope = p[st] - p[0];
    else if (t == NB - 1)
      slope = p[0] - p[-st];
    else
      slope = 0.5 * p[st] - 0.5 * p[-st];
    val += ((gc[e] & 1) ? 0.25 : -0.25) * slope;
  }
  return {(2.0 / 3.0) * val, 1.0 / 3.0};
}

// the neighbour sums of cell c of block b: sum of the 2 ND values as sc + sw u(c)
template <int ND>
__host__ __device__ inline void stencil(const FmgDev& g, int b, bool leaf, const int* c, double& sc, double& sw) {
  const double* ub = g.u + (size_t)b * ncb<ND>();
  // local sums, each face's value selected (not the address it is added
  // to), so both stay in registers
  double s = 0.0, ws = 0.0;
#pragma unroll
  for (int face = 0; face < 2 * ND; face++) {
    int cn[3] = {c[0], c[1], c[2]};
    cn[face >> 1] += (face & 1) ? 1 : -1;
    double av, aw = 0.0;
    if (cn[face >> 1] >= 0 && cn[face >> 1] < NB) {
      av = ub[cidx(cn)];
    } else {
      const Across a = across<ND>(g, b, leaf, c, face);
      av = a.cv;
      aw = a.w;
    }
    s += av;
    ws += aw;
  }
  sc = s;
  sw = ws;
}

// stencil for K cells of block b at once, the same sums in the same order:
// every neighbour load that needs no rule (a cell of this block, or of a
// same-level neighbour block whose own cell stands in: the face type is
// uniform per block, so a lane on the face only changes the address) is
// issued before any other face is resolved, so the K cells' loads are in
// flight together; the lanes on a wall or coarse-fine face then take across()
template <int ND, int K>
__host__ __device__ inline void stencil_k(const FmgDev& g, int b, bool leaf, const int (*c)[3], double* sc,
                                          double* sw) {
  constexpr int NCB = ncb<ND>();
  double v[K][2 * ND];
  bool rule[2 * ND];  // the face needs across() for the lanes on it
#pragma unroll
  for (int face = 0; face < 2 * ND; face++) {
    const int d = face >> 1, s1 = (face & 1) ? 1 : -1;
    const int nb = g.nbr[FS * b + face];
    const bool plain = nb >= 0 && (!leaf || g.chi[CS * nb] < 0);
    rule[face] = !plain;
#pragma unroll
    for (int k = 0; k < K; k++) {
      int cn[3] = {c[k][0], c[k][1], c[k][2]};
      const int x = cn[d] + s1;
      const bool out = x < 0 || x > NB - 1;
      // in the block: the neighbour; out with a plain face: the neighbour
      // block's cell; out otherwise: the cell itself (discarded)
      cn[d] = out ? (plain ? (s1 > 0 ? 0 : NB - 1) : cn[d]) : x;
      const int blk = out && plain ? nb : b;
      v[k][face] = g.u[(size_t)blk * NCB + cidx(cn)];
    }
  }
#pragma unroll
  for (int k = 0; k < K; k++) {
    double s = 0.0, ws = 0.0;  // as in stencil
#pragma unroll
    for (int face = 0; face < 2 * ND; face++) {
      const int x = c[k][face >> 1] + ((face & 1) ? 1 : -1);
      double av = v[k][face], aw = 0.0;
      if (!((x >= 0 && x < NB) || !rule[face])) {
        const Across a = across<ND>(g, b, leaf, c[k], face);
        av = a.cv;
        aw = a.w;
      }
      s += av;
      ws += aw;
    }
    sc[k] = s;
    sw[k] = ws;
  }
}

// Every kernel below applies one per-cell function (host-callable too, so a
// host loop over the same functions checks a cycle on the CPU); a 256-thread
// workgroup walks a block plane by plane, thread t at (t & 15, t >> 4).

// lap(u) - lambda u at cell c of block b: the problem's rules (leaf), or the
// plain stencil, the refined neighbours' own (restricted) cells in place of
// the coarse side of a coarse-fine face
template <int ND>
__host__ __device__ inline double apply_cell(const FmgDev& g, int b, bool leaf, const int* c) {
  double sc, sw;
  stencil<ND>(g, b, leaf, c, sc, sw);
  const double u = g.u[(size_t)b * ncb<ND>() + cidx(c)];
  return g.ih2[g.lvl[b]] * (sc + sw * u - (2.0 * ND) * u) - g.lam * u;
}

// red-black relaxation of cell c of block b with the plain stencil (the
// problem's rules on the finest level, which has no refined neighbour): a
// cell of colour (x + y + z) & 1 reads cells of the other colour only (the
// block edge is even, so the colour is global) and coarser levels, none of
// which a sweep of one level writes
template <int ND>
__host__ __device__ inline void smooth_cell(const FmgDev& g, int b, const int* c) {
  const double ih2 = g.ih2[g.lvl[b]];
  double sc, sw;
  stencil<ND>(g, b, false, c, sc, sw);
  const size_t i = (size_t)b * ncb<ND>() + cidx(c);
  g.u[i] = (g.f[i] - ih2 * sc) / (ih2 * (sw - 2.0 * ND) - g.lam);
}

// the residual of the relaxation (plain stencil)
template <int ND>
__host__ __device__ inline void resid_cell(const FmgDev& g, int b, const int* c) {
  const size_t i = (size_t)b * ncb<ND>() + cidx(c);
  g.r[i] = g.f[i] - apply_cell<ND>(g, b, false, c);
}

// the problem's residual at a leaf cell
template <int ND>
__host__ __device__ inline double residual(const FmgDev& g, int b, const int* c) {
  return g.fu[(size_t)b * ncb<ND>() + cidx(c)] - apply_cell<ND>(g, b, true, c);
}

// the right-hand side of a level below the finest: L(u) + r with L the plain
// stencil, r the restricted residual (a parent) or the problem's residual (a
// leaf; where the plain stencil is the problem's, exactly f).  A leaf next to
// a refined block thereby relaxes with the same stencil as that block's
// cells, and is left unchanged once the problem's residual vanishes.
template <int ND>
__host__ __device__ inline void fas_cell(const FmgDev& g, int b, const int* c) {
  const size_t i = (size_t)b * ncb<ND>() + cidx(c);
  if (g.chi[CS * b] >= 0) {
    g.f[i] = apply_cell<ND>(g, b, false, c) + g.r[i];
    return;
  }
  bool refined = false;  // a refined same-level neighbour (else both stencils agree)
#pragma unroll
  for (int face = 0; face < 2 * ND; face++) {
    const int nb = g.nbr[FS * b + face];
    refined = refined || (nb >= 0 && g.chi[CS * nb] >= 0);
  }
  if (!refined) {
    g.f[i] = g.fu[i];
    return;
  }
  const double lp = apply_cell<ND>(g, b, false, c);
  const double lc = apply_cell<ND>(g, b, true, c);
  g.f[i] = lp == lc ? g.fu[i] : lp + (g.fu[i] - lc);
}

// a block of level >= 2 adds the bi/trilinear interpolation of its parent's
// change e = u - uo: weights 9, 3, 3, 1 (/16) in 2D, 27, 9, 3, 1 (/64) in 3D,
// from the parent cell and its neighbours toward the fine cell, the parent's
// own cell where that neighbour lies outside the parent
template <int ND>
__host__ __device__ inline double prolong_delta(const FmgDev& g, int b, const int* c) {
  constexpr int NCB = ncb<ND>();
  const int p = g.par[b];
  int I[3] = {0, 0, 0}, I2[3] = {0, 0, 0};
#pragma unroll
  for (int e = 0; e < ND; e++) {
    I[e] = (g.ij[TS * b + e] & 1) * 8 + (c[e] >> 1);
    const int n2 = I[e] + ((c[e] & 1) ? 1 : -1);
    I2[e] = n2 < 0 ? 0 : (n2 > NB - 1 ? NB - 1 : n2);
  }
  const double* up = g.u + (size_t)p * NCB;
  const double* uq = g.uo + (size_t)p * NCB;
  auto e = [&](int a, int bb, int cc) {
    const int k[3] = {a ? I2[0] : I[0], bb ? I2[1] : I[1], cc ? I2[2] : I[2]};
    const int i = cidx(k);
    return up[i] - uq[i];
  };
  double d;
  if constexpr (ND == 2) {
    d = (9.0 * e(0, 0, 0) + 3.0 * e(1, 0, 0) + 3.0 * e(0, 1, 0) + e(1, 1, 0)) * (1.0 / 16.0);
  } else {
    d = (27.0 * e(0, 0, 0) + 9.0 * (e(1, 0, 0) + e(0, 1, 0) + e(0, 0, 1)) +
         3.0 * (e(1, 1, 0) + e(1, 0, 1) + e(0, 1, 1)) + e(1, 1, 1)) *
        (1.0 / 64.0);
  }
  return d;
}

template <int ND>
__host__ __device__ inline void prolong_cell(const FmgDev& g, int b, const int* c) {
  g.u[(size_t)b * ncb<ND>() + cidx(c)] += prolong_delta<ND>(g, b, c);
}

// index of cell c of level-1 block b in the n^ND grid
template <int ND>
__host__ __device__ inline size_t grid_index(const FmgDev& g, int b, const int* c, int n) {
  size_t i = 0;
#pragma unroll
  for (int e = ND - 1; e >= 0; e--) i = i * n + (size_t)(g.ij[TS * b + e] * NB + c[e]);
  return i;
}

// a level-1 cell to the n^ND grid: the correction problem L(e) = r, from e = 0
template <int ND>
__host__ __device__ inline void to_grid_cell(const FmgDev& g, int b, const int* c, int n, double* fgrid,
                                             double* vgrid) {
  const size_t i = (size_t)b * ncb<ND>() + cidx(c);
  const size_t gi = grid_index<ND>(g, b, c, n);
  fgrid[gi] = g.r[i];
  vgrid[gi] = 0.0;
}

// the block a workgroup of a 3D launch over n blocks takes: workgroups are
// dealt to the 8 XCDs round robin (workgroup i to XCD i % 8), so each XCD is
// given a contiguous range of the blocks instead, and blocks next to each
// other in the tree's order read each other's faces through one L2
__device__ inline int xcd_block(int i, int n) {
  const int q = n >> 3, r = n & 7, x = i & 7;
  return x * q + (x < r ? x : r) + (i >> 3);
}

#define FMG_PLANES(ND)                                        \
  const int tx = threadIdx.x & (NB - 1), ty = threadIdx.x >> 4; \
  for (int tz = 0; tz < nplanes<ND>(); tz++)

// a colour sweep over the blocks [b0, b0 + gridDim.x); in 3D the 256 threads
// take the 128 cells of the colour in each of two planes at a time (x = 2 hx
// + the parity that gives the colour), so no lane idles
template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_smooth(FmgDev g, int b0, int colour) {
  if constexpr (ND == 2) {
    const int tx = threadIdx.x & (NB - 1), ty = threadIdx.x >> 4;
    const int c[3] = {tx, ty, 0};
    if (((tx + ty) & 1) == colour) smooth_cell<2>(g, b0 + blockIdx.x, c);
  } else {
    // the cells of four plane pairs at a time (stencil_k): the same update
    // as smooth_cell, its loads batched
    constexpr int K = 4;
    const int hx = threadIdx.x & 7, ty = (threadIdx.x >> 3) & (NB - 1), pz = threadIdx.x >> 7;
    const int b = b0 + xcd_block(blockIdx.x, gridDim.x);
    const double ih2 = g.ih2[g.lvl[b]];
    const int span = NB / gridDim.y;  // the planes of this workgroup's part of the block
    for (int z0 = blockIdx.y * span; z0 < (int)(blockIdx.y + 1) * span; z0 += 2 * K) {
      int c[K][3];
      size_t i[K];
      double fv[K], sc[K], sw[K];
#pragma unroll
      for (int k = 0; k < K; k++) {
        const int tz = z0 + 2 * k + pz;
        c[k][0] = 2 * hx + ((ty + tz + colour) & 1);
        c[k][1] = ty;
        c[k][2] = tz;
        i[k] = (size_t)b * ncb<3>() + cidx(c[k]);
        fv[k] = g.f[i[k]];
      }
      stencil_k<3, K>(g, b, false, c, sc, sw);
#pragma unroll
      for (int k = 0; k < K; k++) g.u[i[k]] = (fv[k] - ih2 * sc[k]) / (ih2 * (sw[k] - 2.0 * 3) - g.lam);
    }
  }
}

// lap(u) - lambda u at K cells of block b (u their values): apply_cell's
// arithmetic with the loads batched as in stencil_k
template <int ND, int K>
__host__ __device__ inline void apply_k(const FmgDev& g, int b, bool leaf, const int (*c)[3], const double* u,
                                        double* out) {
  double sc[K], sw[K];
  stencil_k<ND, K>(g, b, leaf, c, sc, sw);
  const double ih2 = g.ih2[g.lvl[b]];
#pragma unroll
  for (int k = 0; k < K; k++) out[k] = ih2 * (sc[k] + sw[k] * u[k] - (2.0 * ND) * u[k]) - g.lam * u[k];
}

template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_resid(FmgDev g, int b0) {
  if constexpr (ND == 2) {
    FMG_PLANES(ND) {
      const int c[3] = {tx, ty, tz};
      resid_cell<ND>(g, b0 + blockIdx.x, c);
    }
  } else {
    // four planes at a time (apply_k)
    constexpr int K = 4;
    const int tx = threadIdx.x & (NB - 1), ty = threadIdx.x >> 4;
    const int b = b0 + xcd_block(blockIdx.x, gridDim.x);
    const int span = NB / gridDim.y;
    for (int z0 = blockIdx.y * span; z0 < (int)(blockIdx.y + 1) * span; z0 += K) {
      int c[K][3];
      size_t i[K];
      double fv[K], uv[K], a[K];
#pragma unroll
      for (int k = 0; k < K; k++) {
        c[k][0] = tx;
        c[k][1] = ty;
        c[k][2] = z0 + k;
        i[k] = (size_t)b * ncb<3>() + cidx(c[k]);
        fv[k] = g.f[i[k]];
        uv[k] = g.u[i[k]];
      }
      apply_k<3, K>(g, b, false, c, uv, a);
#pragma unroll
      for (int k = 0; k < K; k++) g.r[i[k]] = fv[k] - a[k];
    }
  }
}

// a child block's residual restricted together with its state, so the fine
// residual is never stored: parent cell t of the child's quadrant / octant
// takes the means of u and of f - L(u) (L the plain stencil) over its 2^ND
// cells (into the parent's u and uo, and r), the residual as resid_cell's; in
// 3D 256 threads take the 512 parent cells (on levels of few blocks split
// over gridDim.y workgroups), in 2D 64 threads the 64
template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_resid_restrict(FmgDev g, int b0) {
  constexpr int NCB = ncb<ND>(), NP = ND == 3 ? 512 : 64, NC = 1 << ND;
  const int b = b0 + (ND == 3 ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x);
  const int p = g.par[b];
  const int q[3] = {g.ij[TS * b] & 1, g.ij[TS * b + 1] & 1, ND == 3 ? (g.ij[TS * b + 2] & 1) : 0};
  const int span = NP / gridDim.y;
  for (int t = blockIdx.y * span + threadIdx.x; t < (int)(blockIdx.y + 1) * span; t += blockDim.x) {
    const int xx = t & 7, yy = (t >> 3) & 7, zz = ND == 3 ? t >> 6 : 0;
    int c[NC][3];
    double uv[NC], fv[NC], a[NC], r[NC];
#pragma unroll
    for (int k = 0; k < NC; k++) {
      c[k][0] = 2 * xx + (k & 1);
      c[k][1] = 2 * yy + ((k >> 1) & 1);
      c[k][2] = ND == 3 ? 2 * zz + (k >> 2) : 0;
      const size_t i = (size_t)b * NCB + cidx(c[k]);
      uv[k] = g.u[i];
      fv[k] = g.f[i];
    }
    apply_k<ND, NC>(g, b, false, c, uv, a);
#pragma unroll
    for (int k = 0; k < NC; k++) r[k] = fv[k] - a[k];
    double um, rm;
    if constexpr (ND == 2) {
      um = 0.25 * ((uv[0] + uv[1]) + (uv[2] + uv[3]));
      rm = 0.25 * ((r[0] + r[1]) + (r[2] + r[3]));
    } else {
      um = 0.125 * (((uv[0] + uv[1]) + (uv[2] + uv[3])) + ((uv[4] + uv[5]) + (uv[6] + uv[7])));
      rm = 0.125 * (((r[0] + r[1]) + (r[2] + r[3])) + ((r[4] + r[5]) + (r[6] + r[7])));
    }
    const int pc[3] = {q[0] * 8 + xx, q[1] * 8 + yy, q[2] * 8 + zz};
    const size_t ip = (size_t)p * NCB + cidx(pc);
    g.u[ip] = um;
    g.uo[ip] = um;
    g.r[ip] = rm;
  }
}


// a parent block in 3D: L(u) + r (fas_cell's first case) four planes at a
// time (apply_k)
__device__ inline void fas_parent_3d(const FmgDev& g, int b) {
  constexpr int K = 4;
  const int tx = threadIdx.x & (NB - 1), ty = threadIdx.x >> 4;
  const int span = NB / gridDim.y;
  for (int z0 = blockIdx.y * span; z0 < (int)(blockIdx.y + 1) * span; z0 += K) {
    int c[K][3];
    size_t i[K];
    double rv[K], uv[K], a[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
      c[k][0] = tx;
      c[k][1] = ty;
      c[k][2] = z0 + k;
      i[k] = (size_t)b * ncb<3>() + cidx(c[k]);
      rv[k] = g.r[i[k]];
      uv[k] = g.u[i[k]];
    }
    apply_k<3, K>(g, b, false, c, uv, a);
#pragma unroll
    for (int k = 0; k < K; k++) g.f[i[k]] = a[k] + rv[k];
  }
}

// a leaf block below the finest level in 3D (fas_cell's other cases): f
// copied from the problem's f where no same-level neighbour is refined, else
// lp + (f - lc) with both stencils, four planes at a time
__device__ inline void fas_leaf_3d(const FmgDev& g, int b) {
  const int tx = threadIdx.x & (NB - 1), ty = threadIdx.x >> 4;
  const size_t base = (size_t)b * ncb<3>() + tx + NB * ty;
  bool refined = false;  // uniform per workgroup
#pragma unroll
  for (int face = 0; face < 6; face++) {
    const int nb = g.nbr[FS * b + face];
    refined = refined || (nb >= 0 && g.chi[CS * nb] >= 0);
  }
  constexpr int K = 4;
  const int span = NB / gridDim.y;
  const int zlo = blockIdx.y * span, zhi = zlo + span;
  if (!refined) {
    for (int z0 = zlo; z0 < zhi; z0 += K) {
      double v[K];
#pragma unroll
      for (int k = 0; k < K; k++) v[k] = g.fu[base + (size_t)NB * NB * (z0 + k)];
#pragma unroll
      for (int k = 0; k < K; k++) g.f[base + (size_t)NB * NB * (z0 + k)] = v[k];
    }
    return;
  }
  for (int z0 = zlo; z0 < zhi; z0 += K) {
    int c[K][3];
    double fv[K], uv[K], lp[K], lc[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
      c[k][0] = tx;
      c[k][1] = ty;
      c[k][2] = z0 + k;
      fv[k] = g.fu[base + (size_t)NB * NB * (z0 + k)];
      uv[k] = g.u[base + (size_t)NB * NB * (z0 + k)];
    }
    apply_k<3, K>(g, b, false, c, uv, lp);
    apply_k<3, K>(g, b, true, c, uv, lc);
#pragma unroll
    for (int k = 0; k < K; k++)
      g.f[base + (size_t)NB * NB * (z0 + k)] = lp[k] == lc[k] ? fv[k] : lp[k] + (fv[k] - lc[k]);
  }
}

template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_fas(FmgDev g, int b0) {
  if constexpr (ND == 3) {
    const int b = b0 + xcd_block(blockIdx.x, gridDim.x);
    if (g.chi[CS * b] >= 0)
      fas_parent_3d(g, b);
    else
      fas_leaf_3d(g, b);
    return;
  }
  FMG_PLANES(ND) {
    const int c[3] = {tx, ty, tz};
    fas_cell<ND>(g, b0 + blockIdx.x, c);
  }
}

template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_prolong(FmgDev g, int b0) {
  if constexpr (ND == 2) {
    FMG_PLANES(ND) {
      const int c[3] = {tx, ty, tz};
      prolong_cell<ND>(g, b0 + blockIdx.x, c);
    }
  } else {
    // four planes at a time: the parent's values (shared by neighbouring
    // planes) and the cells' own values loaded before any store
    constexpr int K = 4;
    const int tx = threadIdx.x & (NB - 1), ty = threadIdx.x >> 4;
    const int b = b0 + xcd_block(blockIdx.x, gridDim.x);
    for (int z0 = 0; z0 < NB; z0 += K) {
      double d[K], uv[K];
      size_t i[K];
#pragma unroll
      for (int k = 0; k < K; k++) {
        const int c[3] = {tx, ty, z0 + k};
        i[k] = (size_t)b * ncb<3>() + cidx(c);
        uv[k] = g.u[i[k]];
        d[k] = prolong_delta<3>(g, b, c);
      }
#pragma unroll
      for (int k = 0; k < K; k++) g.u[i[k]] = uv[k] + d[k];
    }
  }
}

template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_to_grid(FmgDev g, int b0, int n, double* fgrid, double* vgrid) {
  FMG_PLANES(ND) {
    const int c[3] = {tx, ty, tz};
    to_grid_cell<ND>(g, b0 + blockIdx.x, c, n, fgrid, vgrid);
  }
}

template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_from_grid(FmgDev g, int b0, int n, const double* vgrid) {
  const int b = b0 + blockIdx.x;
  FMG_PLANES(ND) {
    const int c[3] = {tx, ty, tz};
    g.u[(size_t)b * ncb<ND>() + cidx(c)] += vgrid[grid_index<ND>(g, b, c, n)];
  }
}

// block maximum of v >= 0 into *out (the bits of non-negative doubles order
// as the values)
__device__ __forceinline__ void fold_max(double v, unsigned long long* out) {
  __shared__ double sm[WG / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sm[0];
    for (int i = 1; i < WG / 64; i++) m = fmax(m, sm[i]);
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
  }
}

// max |r| of the problem over the leaves into out[0] and, with fmax, max |f|
// (the problem's f as solved) into out[1] (every block launched; parents skip)
template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_resmax(FmgDev g, unsigned long long* out, int with_f) {
  const int b = ND == 3 ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  if (g.chi[CS * b] >= 0) return;  // uniform per workgroup
  double mr = 0.0, mf = 0.0;
  if constexpr (ND == 2) {
    FMG_PLANES(ND) {
      const int c[3] = {tx, ty, tz};
      const double r = residual<ND>(g, b, c);
      const double f = g.fu[(size_t)b * ncb<ND>() + cidx(c)];
      mr = fmax(mr, isnan(r) ? INFINITY : fabs(r));
      mf = fmax(mf, isnan(f) ? INFINITY : fabs(f));
    }
  } else {
    // residual() four planes at a time (stencil_k with the problem's rules)
    constexpr int K = 4;
    const int tx = threadIdx.x & (NB - 1), ty = threadIdx.x >> 4;
    const double ih2 = g.ih2[g.lvl[b]];
    for (int z0 = 0; z0 < NB; z0 += K) {
      int c[K][3];
      double fv[K], uv[K], sc[K], sw[K];
#pragma unroll
      for (int k = 0; k < K; k++) {
        c[k][0] = tx;
        c[k][1] = ty;
        c[k][2] = z0 + k;
        const size_t i = (size_t)b * ncb<3>() + cidx(c[k]);
        fv[k] = g.fu[i];
        uv[k] = g.u[i];
      }
      stencil_k<3, K>(g, b, true, c, sc, sw);
#pragma unroll
      for (int k = 0; k < K; k++) {
        const double r = fv[k] - (ih2 * (sc[k] + sw[k] * uv[k] - (2.0 * 3) * uv[k]) - g.lam * uv[k]);
        mr = fmax(mr, isnan(r) ? INFINITY : fabs(r));
        mf = fmax(mf, isnan(fv[k]) ? INFINITY : fabs(fv[k]));
      }
    }
  }
  fold_max(mr, out);
  if (with_f) {
    __syncthreads();
    fold_max(mf, out + 1);
  }
}

// leaf fields <-> block arrays; dir 0: f and phi in, 1: phi out
template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_leaves(FmgDev g, const int* leafblk, const double* f, double* phi,
                                                  int dir) {
  constexpr int NCB = ncb<ND>();
  const int k = blockIdx.x;
  for (int t = threadIdx.x; t < NCB; t += WG) {
    const size_t i = (size_t)leafblk[k] * NCB + t, o = (size_t)k * NCB + t;
    if (dir == 0) {
      g.f[i] = f[o];
      g.fu[i] = f[o];
      g.u[i] = phi[o];
    } else {
      phi[o] = g.u[i];
    }
  }
}

__global__ void k_fmg_maxabs(const double* v, long long count, unsigned long long* out) {
  double m = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    m = fmax(m, isnan(v[i]) ? INFINITY : fabs(v[i]));
  fold_max(m, out);
}

__global__ void k_fmg_zero2(unsigned long long* p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0ull;
}

// ---- Poisson (lambda = 0) and the divergence control (Sec. 2.4) ------------

// volume-weighted sum of a leaf block's cells of `which` (0: g.f, 1: g.u)
// into part[k] (a fixed reduction order: the same bits on every run)
template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_wsum(FmgDev g, const int* leafblk, int which, double* part) {
  constexpr int NCB = ncb<ND>();
  __shared__ double sm[WG / 64];
  const int b = leafblk[blockIdx.x];
  const double* a = which ? g.u : g.f;
  double v = 0.0;
  for (int t = threadIdx.x; t < NCB; t += WG) v += a[(size_t)b * NCB + t];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  const int l = g.lvl[b];
  if (threadIdx.x == 0)
    part[blockIdx.x] = ((sm[0] + sm[1]) + (sm[2] + sm[3])) / (ND == 3 ? g.ih2[l] * g.rh[l] : g.ih2[l]);
}

// mean = sum(part) / volume, one workgroup, a fixed order
__global__ void __launch_bounds__(WG) k_fmg_wmean(const double* part, int n, double vol, double* mean) {
  __shared__ double sm[WG];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += WG) v += part[i];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int o = WG / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *mean = sm[0] / vol;
}

// subtract *mean from the leaf blocks' g.f and g.fu (which 0) or g.u (which 1)
template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_submean(FmgDev g, const int* leafblk, int which, const double* mean) {
  constexpr int NCB = ncb<ND>();
  const double m = *mean;
  for (int t = threadIdx.x; t < NCB; t += WG) {
    const size_t i = (size_t)leafblk[blockIdx.x] * NCB + t;
    if (which == 0) {
      g.f[i] -= m;
      g.fu[i] -= m;
    } else {
      g.u[i] -= m;
    }
  }
}

// the value one cell over from cell c of leaf block b across face `face`
template <int ND>
__host__ __device__ inline double face_value(const FmgDev& g, int b, const int* c, int face) {
  constexpr int NCB = ncb<ND>();
  int cn[3] = {c[0], c[1], c[2]};
  cn[face >> 1] += (face & 1) ? 1 : -1;
  if (cn[face >> 1] >= 0 && cn[face >> 1] < NB) return g.u[(size_t)b * NCB + cidx(cn)];
  const Across a = across<ND>(g, b, true, c, face);
  return a.cv + a.w * g.u[(size_t)b * NCB + cidx(c)];
}

// central difference along d of the loaded leaf field: (w(+1) - w(-1)) (n_l / 2L),
// into out (acc 0) or added to it (acc 1)
template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_diff(FmgDev g, const int* leafblk, int d, int acc, double* out) {
  constexpr int NCB = ncb<ND>();
  const int b = leafblk[blockIdx.x];
  FMG_PLANES(ND) {
    const int c[3] = {tx, ty, tz};
    const double v =
        (face_value<ND>(g, b, c, 2 * d + 1) - face_value<ND>(g, b, c, 2 * d)) * (0.5 * g.rh[g.lvl[b]]);
    const size_t o = (size_t)blockIdx.x * NCB + cidx(c);
    out[o] = acc ? out[o] + v : v;
  }
}

__global__ void k_fmg_sub(long long n, double* a, const double* da) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t < n) a[t] = a[t] - da[t];
}

__global__ void k_fmg_zero(long long n, double* a) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t < n) a[t] = 0.0;
}

// ---- reaction-diffusion on the leaves (Sec. 2.5) ---------------------------

struct RdF {
  int model;
  double Du, Dv, p1, p2, p3;
};

// (F0_u, F0_v) of Eqs. schnakenberg / gray-scott
__device__ __forceinline__ void react(const RdF& p, double u, double v, double& ru, double& rv) {
  if (p.model == AMRV_RD_SCHNAKENBERG) {
    const double uuv = (u * u) * v;
    ru = p.p1 * ((p.p2 - u) + uuv);
    rv = p.p1 * (p.p3 - uuv);
  } else {
    const double uvv = u * (v * v);
    ru = p.p1 * (1.0 - u) - uvv;
    rv = uvv - (p.p1 + p.p2) * v;
  }
}

// a leaf field into the state of the leaf blocks
template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_load(FmgDev g, const int* leafblk, const double* w) {
  constexpr int NCB = ncb<ND>();
  for (int t = threadIdx.x; t < NCB; t += WG)
    g.u[(size_t)leafblk[blockIdx.x] * NCB + t] = w[(size_t)blockIdx.x * NCB + t];
}

// D lap(w) at the leaf cells of the loaded field (the problem's rules; g.lam = 0)
template <int ND>
__global__ void __launch_bounds__(WG) k_fmg_lap(FmgDev g, const int* leafblk, double D, double* out) {
  FMG_PLANES(ND) {
    const int c[3] = {tx, ty, tz};
    out[(size_t)blockIdx.x * ncb<ND>() + cidx(c)] = D * apply_cell<ND>(g, leafblk[blockIdx.x], true, c);
  }
}

// o = b + c (F0(s) + l), l = D lap(s) (explicit Euler and midpoint stages)
__global__ void k_fmg_rd_explicit(RdF p, long long n, const double* bu, const double* bv, const double* su,
                                  const double* sv, const double* lu, const double* lv, double* ou, double* ov,
                                  double c) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  double ru, rv;
  react(p, su[t], sv[t], ru, rv);
  const double fu = ru + lu[t], fv = rv + lv[t];
  ou[t] = bu[t] + c * fu;
  ov[t] = bv[t] + c * fv;
}

// split: f = -lambda (w + dt F0(w)) per species
__global__ void k_fmg_rd_split_rhs(RdF p, long long n, const double* u, const double* v, double lu_, double lv_,
                                   double dt, double* fu, double* fv) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  double ru, rv;
  react(p, u[t], v[t], ru, rv);
  fu[t] = -lu_ * (u[t] + dt * ru);
  fv[t] = -lv_ * (v[t] + dt * rv);
}

// IMEX first stage: E = F(w), f = -lambda ((w + dt F0(w)) + (dt/2) D lap(w)),
// initial guess w + dt F(w)
__global__ void k_fmg_rd_imex_rhs(RdF p, long long n, const double* u, const double* v, const double* du,
                                  const double* dv, double lu_, double lv_, double dt, double* Eu, double* Ev,
                                  double* fu, double* fv, double* su, double* sv) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  double ru, rv;
  react(p, u[t], v[t], ru, rv);
  Eu[t] = ru + du[t];
  Ev[t] = rv + dv[t];
  const double hdt = 0.5 * dt;
  fu[t] = -lu_ * ((u[t] + dt * ru) + hdt * du[t]);
  fv[t] = -lv_ * ((v[t] + dt * rv) + hdt * dv[t]);
  su[t] = u[t] + dt * (ru + du[t]);
  sv[t] = v[t] + dt * (rv + dv[t]);
}

// IMEX second stage: w1 = w + (dt/2) (E + F(w*)), l = D lap(w*)
__global__ void k_fmg_rd_imex_final(RdF p, long long n, double* u, double* v, const double* Eu, const double* Ev,
                                    const double* su, const double* sv, const double* lu, const double* lv,
                                    double dt) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  double ru, rv;
  react(p, su[t], sv[t], ru, rv);
  const double hdt = 0.5 * dt;
  u[t] = u[t] + hdt * (Eu[t] + (ru + lu[t]));
  v[t] = v[t] + hdt * (Ev[t] + (rv + lv[t]));
}

// ---------------------------------------------------------------------------
// host: the block tree
// ---------------------------------------------------------------------------

struct Tree {
  int nd = 2, nblk = 0, nlev = 0;
  int lstart[FMG_MAXL + 2] = {};
  std::vector<int> lvl, ij, nbr, chi, cnb, par, leafblk;
};

int fmg_ndim(const amrv_fmg_config* c) { return c->ndim == 0 ? 2 : c->ndim; }

int validate(const amrv_fmg_config* c) {
  if (!c) return set_error(AMRV_EINVAL, "null config");
  const int nd = fmg_ndim(c);
  if (nd != 2 && nd != 3) return set_error(AMRV_EINVAL, "ndim must be 2 or 3");
  if (c->nleaves < 1) return set_error(AMRV_EINVAL, "nleaves must be >= 1");
  if (c->base < 1 || c->base > 512 || (c->base & (c->base - 1)))
    return set_error(AMRV_EINVAL, "base must be a power of two in 1..512");
  if (c->max_level < 1 || c->max_level > FMG_MAXL) return set_error(AMRV_EINVAL, "max_level must be in 1..16");
  if ((long long)c->base * NB > (nd == 2 ? 8192 : 512))
    return set_error(AMRV_EINVAL, "base * 16 must be <= 8192 (2D) or 512 (3D)");
  if (c->bc != AMRV_MG_PERIODIC && c->bc != AMRV_MG_NEUMANN) return set_error(AMRV_EINVAL, "bc must be periodic or Neumann");
  if (c->pre_sweeps < 1 || c->pre_sweeps > 8 || c->post_sweeps < 1 || c->post_sweeps > 8)
    return set_error(AMRV_EINVAL, "pre_sweeps and post_sweeps must be in 1..8");
  if (!(c->length > 0.0) || !std::isfinite(c->length)) return set_error(AMRV_EINVAL, "length must be > 0");
  return 0;
}

int build_tree(const amrv_fmg_config* c, const int32_t* level, const int32_t* ijk, Tree& T) {
  if (!level || !ijk) return set_error(AMRV_EINVAL, "null leaf arrays");
  const int nd = fmg_ndim(c), nf = 2 * nd, nch = 1 << nd;
  using Key = std::array<int, 4>;  // level, i, j, k
  std::map<Key, int> leaf;
  std::map<Key, int> blocks;  // value: 1 for a leaf
  for (long long k = 0; k < c->nleaves; k++) {
    const int l = level[k];
    const long long nl = (long long)c->base << (l - 1);
    bool ok = l >= 1 && l <= c->max_level;
    for (int e = 0; e < 3 && ok; e++) {
      const int v = ijk[3 * k + e];
      ok = e < nd ? (v >= 0 && v < nl) : v == 0;
    }
    if (!ok) return set_error(AMRV_EINVAL, "leaf level or block coordinates out of range");
    if (!leaf.emplace(Key{l, ijk[3 * k], ijk[3 * k + 1], ijk[3 * k + 2]}, (int)k).second)
      return set_error(AMRV_EUNBALANCED, "leaves overlap (a leaf appears twice)");
  }
  for (const auto& kv : leaf) blocks[kv.first] = 1;
  for (const auto& kv : leaf) {
    Key a = kv.first;
    while (a[0] > 1) {
      a = Key{a[0] - 1, a[1] >> 1, a[2] >> 1, a[3] >> 1};
      auto it = blocks.find(a);
      if (it != blocks.end()) {
        if (it->second == 1) return set_error(AMRV_EUNBALANCED, "leaves overlap");
        break;  // its ancestors are in already
      }
      blocks[a] = 0;
    }
  }
  // blocks ordered by level, then z, y, x
  std::vector<Key> keys;
  for (const auto& kv : blocks) keys.push_back(kv.first);
  std::sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
    return std::make_tuple(a[0], a[3], a[2], a[1]) < std::make_tuple(b[0], b[3], b[2], b[1]);
  });
  std::map<Key, int> index;
  for (size_t b = 0; b < keys.size(); b++) index[keys[b]] = (int)b;
  const int nblk = (int)keys.size();
  T.nd = nd;
  T.nblk = nblk;
  T.lvl.assign(nblk, 0);
  T.ij.assign(TS * nblk, 0);
  T.nbr.assign(FS * nblk, NBR_NONE);
  T.chi.assign(CS * nblk, -1);
  T.cnb.assign(FS * nblk, -1);
  T.par.assign(nblk, -1);
  T.leafblk.assign(c->nleaves, -1);
  T.nlev = 0;
  for (int b = 0; b < nblk; b++) T.nlev = std::max(T.nlev, keys[b][0]);
  // blocks of level l: [lstart[l], lstart[l + 1])
  for (int l = 0; l <= FMG_MAXL + 1; l++) T.lstart[l] = 0;
  for (int b = 0; b < nblk; b++) T.lstart[keys[b][0] + 1]++;
  for (int l = 1; l <= FMG_MAXL + 1; l++) T.lstart[l] += T.lstart[l - 1];
  long long nbase = 1;
  for (int e = 0; e < nd; e++) nbase *= c->base;
  if (T.lstart[2] - T.lstart[1] != nbase) return set_error(AMRV_EUNBALANCED, "the leaves do not cover the base grid");
  auto find = [&](int l, long long i, long long j, long long k) {
    auto it = index.find(Key{l, (int)i, (int)j, (int)k});
    return it == index.end() ? -1 : it->second;
  };
  for (int b = 0; b < nblk; b++) {
    const Key& K = keys[b];
    const int l = K[0];
    T.lvl[b] = l;
    for (int e = 0; e < 3; e++) T.ij[TS * b + e] = K[1 + e];
    if (l > 1) T.par[b] = find(l - 1, K[1] >> 1, K[2] >> 1, K[3] >> 1);
    const long long nl = (long long)c->base << (l - 1);
    const bool isleaf = blocks[K] == 1;
    int nchild = 0;
    for (int q = 0; q < nch; q++) {
      T.chi[CS * b + q] = find(l + 1, 2 * K[1] + (q & 1), 2 * K[2] + ((q >> 1) & 1), 2 * K[3] + ((q >> 2) & 1));
      nchild += T.chi[CS * b + q] >= 0;
    }
    if (isleaf ? nchild != 0 : nchild != nch) return set_error(AMRV_EUNBALANCED, "leaves overlap or leave gaps");
    for (int f = 0; f < nf; f++) {
      const int d = f >> 1;
      long long n3[3] = {K[1], K[2], K[3]};
      n3[d] += (f & 1) ? 1 : -1;
      if (n3[d] < 0 || n3[d] >= nl) {
        if (c->bc == AMRV_MG_NEUMANN) {
          T.nbr[FS * b + f] = NBR_WALL;
          continue;
        }
        n3[d] = (n3[d] + nl) % nl;
      }
      const int nb = find(l, n3[0], n3[1], n3[2]);
      T.nbr[FS * b + f] = nb;
      if (nb >= 0) {
        // a refined neighbour of a leaf: its children along the face must be leaves
        if (isleaf && blocks[keys[nb]] == 0)
          for (int q = 0; q < nch; q++) {
            if (((q >> d) & 1) != ((f & 1) ? 0 : 1)) continue;
            const int cq = find(l + 1, 2 * n3[0] + (q & 1), 2 * n3[1] + ((q >> 1) & 1), 2 * n3[2] + ((q >> 2) & 1));
            if (cq < 0 || blocks[keys[cq]] != 1) return set_error(AMRV_EUNBALANCED, "2:1 balance across a face broken");
          }
        continue;
      }
      // no block of this level across the face: only a leaf may see a coarser leaf there
      const long long nl1 = nl >> 1;
      long long cc[3] = {n3[0] >> 1, n3[1] >> 1, n3[2] >> 1};
      for (int e = 0; e < nd; e++) cc[e] = (cc[e] + nl1) % nl1;
      const int C = l > 1 ? find(l - 1, cc[0], cc[1], cc[2]) : -1;
      if (!isleaf || C < 0 || blocks[keys[C]] != 1)
        return set_error(AMRV_EUNBALANCED, "2:1 balance across a face broken");
      T.cnb[FS * b + f] = C;
    }
  }
  for (const auto& kv : leaf) T.leafblk[kv.second] = index[kv.first];
  return 0;
}

// the uniform solver of the level-1 grid: one field, the forest's boundary,
// per-colour sweeps (its smoother choice does not change its result)
amrv_mg_config base_config(const amrv_fmg_config* c) {
  amrv_mg_config mc{};
  mc.ndim = fmg_ndim(c);
  mc.n = c->base * NB;
  mc.bc = c->bc;
  mc.nfields = 1;
  mc.pre_sweeps = 2;
  mc.post_sweeps = 2;
  mc.use_graph = 0;
  mc.smoother = AMRV_MG_PER_COLOUR;
  mc.length = c->length;
  return mc;
}

struct FmgLayout {
  size_t off_tab[7], off_u, off_f, off_fu, off_r, off_uo, off_red, off_tmp[8], off_part, off_mg, total;
  size_t mg_bytes;
};

FmgLayout layout(const amrv_fmg_config* c, const Tree& T) {
  FmgLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += (bytes + ALIGN - 1) / ALIGN * ALIGN;
    return at;
  };
  const int nd = fmg_ndim(c);
  const size_t nb = (size_t)T.nblk, cb = nd == 3 ? (size_t)NB * NB * NB : (size_t)NB * NB;
  L.off_tab[0] = take(sizeof(int) * nb);        // lvl
  L.off_tab[1] = take(sizeof(int) * TS * nb);   // ij
  L.off_tab[2] = take(sizeof(int) * FS * nb);   // nbr
  L.off_tab[3] = take(sizeof(int) * CS * nb);   // chi
  L.off_tab[4] = take(sizeof(int) * FS * nb);   // cnb
  L.off_tab[5] = take(sizeof(int) * nb);        // par
  L.off_tab[6] = take(sizeof(int) * (size_t)c->nleaves);  // leaf -> block
  L.off_u = take(sizeof(double) * cb * nb);
  L.off_f = take(sizeof(double) * cb * nb);
  L.off_fu = take(sizeof(double) * cb * nb);
  L.off_r = take(sizeof(double) * cb * nb);
  L.off_uo = take(sizeof(double) * cb * nb);
  L.off_red = take(sizeof(unsigned long long) * 2);
  for (int i = 0; i < 8; i++) L.off_tmp[i] = take(sizeof(double) * cb * (size_t)c->nleaves);  // RD temporaries
  L.off_part = take(sizeof(double) * ((size_t)c->nleaves + 1));  // per-leaf sums and their mean
  amrv_mg_config mc = base_config(c);
  L.mg_bytes = amrv_mg_workspace_bytes(&mc);
  L.off_mg = take(L.mg_bytes);
  L.total = o;
  return L;
}

}  // namespace

struct amrv_fmg {
  amrv_fmg_config cfg{};
  int nd = 2;      // dimension
  long long ncb = 0;  // cells per block
  hipStream_t st = nullptr;
  Tree T;
  FmgLayout L{};
  FmgDev g{};
  int* leafblk = nullptr;
  double* fgrid = nullptr;
  double* vgrid = nullptr;
  double* tmp[8] = {};  // leaf fields of the reaction-diffusion steps
  double* part = nullptr;  // per-leaf area-weighted sums, then [nleaves] = their mean
  double area = 0.0;       // L^nd (the domain's area or volume)
  unsigned long long* red = nullptr;
  unsigned long long* hred = nullptr;  // pinned
  amrv_mg* base = nullptr;
  int last_cycles = 0;  // cycles of the previous solve
};

namespace {

int hip_fail(hipError_t e, const char* what) {
  return set_error(AMRV_EDEVICE, (std::string(what) + ": " + hipGetErrorString(e)).c_str());
}

#define FMGCHK(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);  \
  } while (0)

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, 8);
  return d;
}

int nblocks(const amrv_fmg* m, int l) { return m->T.lstart[l + 1] - m->T.lstart[l]; }

// a launch of the ND = 2 or 3 instance of a kernel template on m's stream
#define FMG_LAUNCH(kern, grid, block, ...)                                           \
  do {                                                                               \
    if (m->nd == 2)                                                                  \
      hipLaunchKernelGGL((kern<2>), dim3(grid), dim3(block), 0, m->st, __VA_ARGS__); \
    else                                                                             \
      hipLaunchKernelGGL((kern<3>), dim3(grid), dim3(block), 0, m->st, __VA_ARGS__); \
  } while (0)

// the launch grid of a per-block kernel over level l: in 3D a level of few
// blocks gives each block up to `parts` workgroups, each taking an equal
// share of its planes, so that small levels still fill the chip
dim3 level_grid(const amrv_fmg* m, int l, int parts) {
  const int n = nblocks(m, l);
  int s = 1;
  while (m->nd == 3 && s < parts && (long long)n * s < 4096) s *= 2;
  return dim3(n, s);
}

int sweeps(amrv_fmg* m, int l, int count) {
  for (int s = 0; s < count; s++)
    for (int c = 0; c < 2; c++)
      FMG_LAUNCH(k_fmg_smooth, level_grid(m, l, 2), WG, m->g, m->T.lstart[l], c);
  FMGCHK(hipGetLastError());
  return 0;
}

// one V-cycle (enqueued; the level-1 solve synchronises inside)
int vcycle(amrv_fmg* m) {
  const int L = m->T.nlev;
  const int pre = m->cfg.pre_sweeps, post = m->cfg.post_sweeps;
  for (int l = L; l >= 2; l--) {
    if (int rc = sweeps(m, l, pre)) return rc;
    FMG_LAUNCH(k_fmg_resid_restrict, level_grid(m, l, 2), m->nd == 3 ? WG : 64, m->g, m->T.lstart[l]);
    FMG_LAUNCH(k_fmg_fas, level_grid(m, l - 1, 4), WG, m->g, m->T.lstart[l - 1]);
    FMGCHK(hipGetLastError());
  }
  if (int rc = sweeps(m, 1, pre)) return rc;
  const int n = m->cfg.base * NB;
  FMG_LAUNCH(k_fmg_resid, level_grid(m, 1, 4), WG, m->g, m->T.lstart[1]);
  FMG_LAUNCH(k_fmg_to_grid, nblocks(m, 1), WG, m->g, m->T.lstart[1], n, m->fgrid, m->vgrid);
  FMGCHK(hipGetLastError());
  // the level-1 correction: one of the uniform solver's V-cycles from zero
  // (it cuts the error by 20 or more; solved as a correction, what is left
  // shrinks with the residual from cycle to cycle), enqueued without a host
  // wait
  if (int rc = amrv::mg_enqueue_correction(m->base, m->fgrid, m->vgrid, m->g.lam, 1, true)) return rc;
  FMG_LAUNCH(k_fmg_from_grid, nblocks(m, 1), WG, m->g, m->T.lstart[1], n, m->vgrid);
  FMGCHK(hipGetLastError());
  if (int rc2 = sweeps(m, 1, post)) return rc2;
  for (int l = 2; l <= L; l++) {
    FMG_LAUNCH(k_fmg_prolong, nblocks(m, l), WG, m->g, m->T.lstart[l]);
    FMGCHK(hipGetLastError());
    if (int rc2 = sweeps(m, l, post)) return rc2;
  }
  return 0;
}

// max |r| over the leaves (and, with fmax, max |f| of the problem as solved)
int norms(amrv_fmg* m, double* res, double* fmax) {
  hipLaunchKernelGGL(k_fmg_zero2, dim3(1), dim3(64), 0, m->st, m->red);
  FMG_LAUNCH(k_fmg_resmax, m->T.nblk, WG, m->g, m->red, fmax ? 1 : 0);
  FMGCHK(hipGetLastError());
  FMGCHK(hipMemcpyAsync(m->hred, m->red, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, m->st));
  FMGCHK(hipStreamSynchronize(m->st));
  *res = bits_to_double(m->hred[0]);
  if (fmax) *fmax = bits_to_double(m->hred[1]);
  return 0;
}

// subtract the area-weighted mean of the leaves' f (which 0: g.f and g.fu) or u (1)
int remove_mean(amrv_fmg* m, int which) {
  const int nl = (int)m->cfg.nleaves;
  FMG_LAUNCH(k_fmg_wsum, nl, WG, m->g, m->leafblk, which, m->part);
  hipLaunchKernelGGL(k_fmg_wmean, dim3(1), dim3(WG), 0, m->st, m->part, nl, m->area, m->part + nl);
  FMG_LAUNCH(k_fmg_submean, nl, WG, m->g, m->leafblk, which, m->part + nl);
  FMGCHK(hipGetLastError());
  return 0;
}

}  // namespace

extern "C" {

size_t amrv_fmg_workspace_bytes(const amrv_fmg_config* cfg, const int32_t* leaf_level, const int32_t* leaf_ijk) {
  if (validate(cfg)) return 0;
  Tree T;
  if (build_tree(cfg, leaf_level, leaf_ijk, T)) return 0;
  return layout(cfg, T).total;
}

int amrv_fmg_create(const amrv_fmg_config* cfg, const int32_t* leaf_level, const int32_t* leaf_ijk,
                    void* workspace, size_t bytes, void* stream, amrv_fmg** out) {
  if (!out) return set_error(AMRV_EINVAL, "null argument");
  *out = nullptr;
  if (int rc = validate(cfg)) return rc;
  if (!workspace) return set_error(AMRV_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % ALIGN) return set_error(AMRV_EINVAL, "workspace must be 256-byte aligned");
  amrv_fmg* m = new amrv_fmg;
  m->cfg = *cfg;
  m->st = static_cast<hipStream_t>(stream);
  if (int rc = build_tree(cfg, leaf_level, leaf_ijk, m->T)) {
    delete m;
    return rc;
  }
  m->L = layout(cfg, m->T);
  if (bytes < m->L.total) {
    delete m;
    return set_error(AMRV_ENOMEM, ("workspace too small: need " + std::to_string(m->L.total)).c_str());
  }
  char* base = static_cast<char*>(workspace);
  const Tree& T = m->T;
  const std::vector<int>* tabs[7] = {&T.lvl, &T.ij, &T.nbr, &T.chi, &T.cnb, &T.par, &T.leafblk};
  int* dtab[7];
  hipError_t e = hipSuccess;
  for (int i = 0; i < 7 && e == hipSuccess; i++) {
    dtab[i] = reinterpret_cast<int*>(base + m->L.off_tab[i]);
    e = hipMemcpyAsync(dtab[i], tabs[i]->data(), sizeof(int) * tabs[i]->size(), hipMemcpyHostToDevice, m->st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(m->st);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&m->hred), 2 * sizeof(unsigned long long));
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "amrv_fmg_create");
  }
  FmgDev& g = m->g;
  g.lvl = dtab[0];
  g.ij = dtab[1];
  g.nbr = dtab[2];
  g.chi = dtab[3];
  g.cnb = dtab[4];
  g.par = dtab[5];
  m->leafblk = dtab[6];
  g.u = reinterpret_cast<double*>(base + m->L.off_u);
  g.f = reinterpret_cast<double*>(base + m->L.off_f);
  g.fu = reinterpret_cast<double*>(base + m->L.off_fu);
  g.r = reinterpret_cast<double*>(base + m->L.off_r);
  g.uo = reinterpret_cast<double*>(base + m->L.off_uo);
  for (int l = 1; l <= FMG_MAXL; l++) {
    const double q = (double)((long long)cfg->base * NB << (l - 1)) / cfg->length;
    g.ih2[l] = q * q;
    g.rh[l] = q;
  }
  m->red = reinterpret_cast<unsigned long long*>(base + m->L.off_red);
  for (int i = 0; i < 8; i++) m->tmp[i] = reinterpret_cast<double*>(base + m->L.off_tmp[i]);
  m->part = reinterpret_cast<double*>(base + m->L.off_part);
  m->nd = m->T.nd;
  m->ncb = m->nd == 3 ? (long long)NB * NB * NB : (long long)NB * NB;
  m->area = m->nd == 3 ? cfg->length * cfg->length * cfg->length : cfg->length * cfg->length;
  const amrv_mg_config mc = base_config(cfg);
  if (int rc = amrv_mg_create(&mc, base + m->L.off_mg, m->L.mg_bytes, stream, &m->base)) {
    (void)hipHostFree(m->hred);
    delete m;
    return rc;
  }
  // the level-1 grid is the uniform solver's own right-hand side and
  // solution: k_fmg_to_grid fills the one and zeroes the other
  amrv::mg_correction_grids(m->base, &m->fgrid, &m->vgrid);
  // parents start from zero (every parent is restricted before it is read)
  e = hipMemsetAsync(g.u, 0, sizeof(double) * m->ncb * (size_t)T.nblk, m->st);
  if (e == hipSuccess) e = hipStreamSynchronize(m->st);
  if (e != hipSuccess) {
    amrv_mg_destroy(m->base);
    (void)hipHostFree(m->hred);
    delete m;
    return hip_fail(e, "amrv_fmg_create");
  }
  *out = m;
  return 0;
}

int amrv_fmg_destroy(amrv_fmg* m) {
  if (!m) return 0;
  int rc = amrv_mg_destroy(m->base);
  if (m->hred) (void)hipHostFree(m->hred);
  delete m;
  return rc;
}

int amrv_fmg_levels(const amrv_fmg* m, int32_t* nblocks_per_level) {
  if (!m || !nblocks_per_level) return set_error(AMRV_EINVAL, "null argument");
  for (int l = 1; l <= FMG_MAXL; l++) nblocks_per_level[l - 1] = l <= m->T.nlev ? nblocks(m, l) : 0;
  return 0;
}

int amrv_fmg_solve(amrv_fmg* m, const double* f, double* phi, double lambda, double tol, int32_t max_cycles,
                   int32_t* cycles, double* res_max, double* f_max) {
  if (!m || !f || !phi) return set_error(AMRV_EINVAL, "null argument");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return set_error(AMRV_EINVAL, "lambda must be >= 0 and finite");
  if (!(tol > 0.0) || max_cycles < 0) return set_error(AMRV_EINVAL, "tol must be > 0 and max_cycles >= 0");
  m->g.lam = lambda;
  FMG_LAUNCH(k_fmg_leaves, m->cfg.nleaves, WG, m->g, m->leafblk, f, phi, 0);
  FMGCHK(hipGetLastError());
  // Poisson: lap has the constants as null space and its area-weighted sums
  // vanish, so the problem solved is lap(phi) = f - mean(f), and phi is
  // returned with zero mean (means area-weighted)
  const bool poisson = lambda == 0.0;
  if (poisson)
    if (int rc = remove_mean(m, 0)) return rc;
  double res = 0.0, fmax = 0.0;
  if (int rc = norms(m, &res, &fmax)) return rc;
  int c = 0;
  bool ok = res <= tol * fmax;
  // cycles the previous solve needed, less one, before the next host check
  for (int i = 0; !ok && i < std::min(max_cycles, m->last_cycles - 1) && !std::isnan(res); i++) {
    if (int rc = vcycle(m)) return rc;
    c++;
  }
  if (c > 0) {
    if (int rc = norms(m, &res, nullptr)) return rc;
    ok = res <= tol * fmax;
  }
  while (!ok && c < max_cycles && !std::isnan(res)) {
    if (int rc = vcycle(m)) return rc;
    c++;
    if (int rc = norms(m, &res, nullptr)) return rc;
    ok = res <= tol * fmax;
  }
  m->last_cycles = c;
  if (poisson)
    if (int rc = remove_mean(m, 1)) return rc;
  FMG_LAUNCH(k_fmg_leaves, m->cfg.nleaves, WG, m->g, m->leafblk, f, phi, 1);
  FMGCHK(hipGetLastError());
  FMGCHK(hipStreamSynchronize(m->st));
  if (cycles) *cycles = c;
  if (res_max) *res_max = res;
  if (f_max) *f_max = fmax;
  if (std::isnan(res) || std::isinf(res) || std::isinf(fmax))
    return set_error(AMRV_ENONPHYSICAL, "NaN or infinity in the forest multigrid right-hand side or residual");
  if (!ok) return set_error(AMRV_ENOTCONVERGED, "forest multigrid residual above tol after max_cycles V-cycles");
  return 0;
}

int amrv_fmg_rd_step(amrv_fmg* m, const amrv_rd_params* p, int32_t scheme, double dt, int32_t nsteps, double* u,
                     double* v, double tol, int32_t max_cycles, int32_t* cycles_total, double* res_max) {
  if (!m || !p || !u || !v) return set_error(AMRV_EINVAL, "null argument");
  if (p->model != AMRV_RD_SCHNAKENBERG && p->model != AMRV_RD_GRAY_SCOTT) return set_error(AMRV_EINVAL, "unknown model");
  if (!(p->Du > 0.0) || !(p->Dv > 0.0)) return set_error(AMRV_EINVAL, "diffusion coefficients must be positive");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(AMRV_EINVAL, "dt must be positive and finite");
  if (nsteps < 0) return set_error(AMRV_EINVAL, "nsteps must be >= 0");
  if (scheme < AMRV_RD_EULER || scheme > AMRV_RD_IMEX) return set_error(AMRV_EINVAL, "unknown scheme");
  const bool implicit = scheme == AMRV_RD_SPLIT || scheme == AMRV_RD_IMEX;
  if (implicit && (!(tol > 0.0) || max_cycles < 0)) return set_error(AMRV_EINVAL, "bad tol or max_cycles");
  const RdF k{p->model, p->Du, p->Dv, p->p1, p->p2, p->p3};
  const long long n = (long long)m->cfg.nleaves * m->ncb;
  const int nb = (int)((n + 255) / 256);
  const int nl = (int)m->cfg.nleaves;
  FmgDev g0 = m->g;
  g0.lam = 0.0;
  double* const* T = m->tmp;
  // D lap of a leaf field into out
  auto lap = [&](const double* w, double D, double* out) {
    FMG_LAUNCH(k_fmg_load, nl, WG, g0, m->leafblk, w);
    FMG_LAUNCH(k_fmg_lap, nl, WG, g0, m->leafblk, D, out);
  };
  int total = 0;
  double rmax = 0.0;
  auto solve = [&](const double* f, double* phi, double lam) {
    int32_t c = 0;
    double r = 0.0;
    const int rc = amrv_fmg_solve(m, f, phi, lam, tol, max_cycles, &c, &r, nullptr);
    total += c;
    rmax = std::max(rmax, r);
    return rc;
  };
  for (int s = 0; s < nsteps; s++) {
    if (scheme == AMRV_RD_EULER || scheme == AMRV_RD_MIDPOINT) {
      lap(u, k.Du, T[0]);
      lap(v, k.Dv, T[1]);
      if (scheme == AMRV_RD_EULER) {
        hipLaunchKernelGGL(k_fmg_rd_explicit, dim3(nb), dim3(256), 0, m->st, k, n, u, v, u, v, T[0], T[1], u, v, dt);
      } else {
        hipLaunchKernelGGL(k_fmg_rd_explicit, dim3(nb), dim3(256), 0, m->st, k, n, u, v, u, v, T[0], T[1], T[2], T[3],
                           0.5 * dt);
        lap(T[2], k.Du, T[0]);
        lap(T[3], k.Dv, T[1]);
        hipLaunchKernelGGL(k_fmg_rd_explicit, dim3(nb), dim3(256), 0, m->st, k, n, u, v, T[2], T[3], T[0], T[1], u, v,
                           dt);
      }
      FMGCHK(hipGetLastError());
      continue;
    }
    if (scheme == AMRV_RD_SPLIT) {
      const double lu = 1.0 / (dt * k.Du), lv = 1.0 / (dt * k.Dv);
      hipLaunchKernelGGL(k_fmg_rd_split_rhs, dim3(nb), dim3(256), 0, m->st, k, n, u, v, lu, lv, dt, T[0], T[1]);
      FMGCHK(hipGetLastError());
      if (int rc = solve(T[0], u, lu)) return rc;
      if (int rc = solve(T[1], v, lv)) return rc;
      continue;
    }
    const double lu = 2.0 / (dt * k.Du), lv = 2.0 / (dt * k.Dv);
    lap(u, k.Du, T[0]);
    lap(v, k.Dv, T[1]);
    hipLaunchKernelGGL(k_fmg_rd_imex_rhs, dim3(nb), dim3(256), 0, m->st, k, n, u, v, T[0], T[1], lu, lv, dt, T[2],
                       T[3], T[4], T[5], T[6], T[7]);
    FMGCHK(hipGetLastError());
    if (int rc = solve(T[4], T[6], lu)) return rc;
    if (int rc = solve(T[5], T[7], lv)) return rc;
    lap(T[6], k.Du, T[0]);
    lap(T[7], k.Dv, T[1]);
    hipLaunchKernelGGL(k_fmg_rd_imex_final, dim3(nb), dim3(256), 0, m->st, k, n, u, v, T[2], T[3], T[6], T[7], T[0],
                       T[1], dt);
    FMGCHK(hipGetLastError());
  }
  FMGCHK(hipStreamSynchronize(m->st));
  if (cycles_total) *cycles_total = total;
  if (res_max) *res_max = rmax;
  return 0;
}

int amrv_fmg_divb_project(amrv_fmg* m, double* bx, double* by, double* bz, double tol, int32_t max_cycles,
                          int32_t* cycles, double* div_before, double* div_after) {
  if (!m || !bx || !by || (m->nd == 3 && !bz)) return set_error(AMRV_EINVAL, "null argument");
  if (!(tol > 0.0) || max_cycles < 0) return set_error(AMRV_EINVAL, "bad tol or max_cycles");
  const long long n = (long long)m->cfg.nleaves * m->ncb;
  const int nb = (int)((n + 255) / 256);
  const int nl = (int)m->cfg.nleaves;
  double* const* T = m->tmp;
  double* const B[3] = {bx, by, bz};
  // the central divergence of B into out, directions added x, y (, z)
  auto div = [&](double* out) {
    for (int d = 0; d < m->nd; d++) {
      FMG_LAUNCH(k_fmg_load, nl, WG, m->g, m->leafblk, B[d]);
      FMG_LAUNCH(k_fmg_diff, nl, WG, m->g, m->leafblk, d, d > 0 ? 1 : 0, out);
    }
  };
  auto maxabs = [&](const double* v, double* out) -> int {
    hipLaunchKernelGGL(k_fmg_zero2, dim3(1), dim3(64), 0, m->st, m->red);
    hipLaunchKernelGGL(k_fmg_maxabs, dim3(std::min(1024, nb)), dim3(WG), 0, m->st, v, n, m->red);
    FMGCHK(hipGetLastError());
    FMGCHK(hipMemcpyAsync(m->hred, m->red, sizeof(unsigned long long), hipMemcpyDeviceToHost, m->st));
    FMGCHK(hipStreamSynchronize(m->st));
    *out = bits_to_double(m->hred[0]);
    return 0;
  };
  div(T[0]);
  if (div_before)
    if (int rc = maxabs(T[0], div_before)) return rc;
  hipLaunchKernelGGL(k_fmg_zero, dim3(nb), dim3(256), 0, m->st, n, T[1]);
  FMGCHK(hipGetLastError());
  // phi: the zero-mean solution of lap(phi) = div B* - mean
  const int rc = amrv_fmg_solve(m, T[0], T[1], 0.0, tol, max_cycles, cycles, nullptr, nullptr);
  if (rc) return rc;
  FMG_LAUNCH(k_fmg_load, nl, WG, m->g, m->leafblk, T[1]);
  for (int d = 0; d < m->nd; d++) FMG_LAUNCH(k_fmg_diff, nl, WG, m->g, m->leafblk, d, 0, T[2 + d]);
  for (int d = 0; d < m->nd; d++) hipLaunchKernelGGL(k_fmg_sub, dim3(nb), dim3(256), 0, m->st, n, B[d], T[2 + d]);
  FMGCHK(hipGetLastError());
  if (div_after) {
    div(T[0]);
    if (int rc2 = maxabs(T[0], div_after)) return rc2;
  }
  FMGCHK(hipStreamSynchronize(m->st));
  return 0;
}

}  // extern "C"
