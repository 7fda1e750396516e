// kernels.hip -- gfx950 kernels of the block-forest finite-volume update.
//
// One SSP Runge-Kutta stage (arXiv 2004.03275, Sec. 2.1-2.4) on a forest of
// 16^d blocks (Sec. 1.3) is:
//   k_restrict   coarse-side ghost slabs of coarse-fine faces: mean of the
//                2^d finer cells (pairwise sum, times 2^-d)
//   k_prolong_flux  fine-side ghost slabs (coarse value plus a quarter of
//                its minmod slope per dimension) and the fine-side face
//                fluxes of the same faces (the coarse side replaces its own
//                flux by their mean: conservation)
//   k_stage      per leaf: primitive variables, MUSCL states, Riemann fluxes,
//                flux divergence and the SSP combination.  Same-level and
//                boundary ghosts are gathered straight from the neighbour's
//                interior, so only coarse-fine faces touch the slabs above.
// plus k_cfl (Courant reduction, Sec. 2.1) and k_lohner (Sec. 1.3 flags).
//
// The stencil work is FP64 VALU and HBM traffic: there is no matrix-core
// contraction here.  The 2D/3D stage kernel streams a 16^3 block through a
// 16x16 workgroup plane by plane: z-direction data stays in registers, the
// x/y planes of primitive values, face states and fluxes in LDS.
#include <float.h>

#include <type_traits>

#include "internal.hpp"
#include "physics.hpp"
#include "bf16.hpp"
#include "stage_common.hpp"

namespace amrv {

// ---------------------------------------------------------------------------
// ghost slabs of coarse-fine faces
// ---------------------------------------------------------------------------

// one thread per coarse ghost cell (slot, transverse position t, layer); the
// two children along x of every restricted cell are adjacent in memory (x is
// the fastest index, the pair starts at an even x), so they come in one
// 16-byte load, and the two layers of one position are neighbouring lanes:
// on an x face the pair of lanes reads 32 contiguous bytes of each fine row
template <int ND, int NV>
__global__ void __launch_bounds__(WGS) k_restrict(Geo g, const double* __restrict__ U, const int32_t* __restrict__ list,
                                                  int nlist) {
  const long long i = (long long)blockIdx.x * WGS + threadIdx.x;
  if (i >= (long long)nlist * 2 * g.T) return;
  const int slot = list[i / (2 * g.T)];
  const int rem = (int)(i % (2 * g.T));
  const int layer = rem & 1, t = rem >> 1;
  const int a1 = ND > 1 ? t % g.nx : 0, a2 = ND > 2 ? t / g.nx : 0;
  const int f = g.sface[slot];
  const int d = f >> 1, hi = f & 1;
  const int half = g.nx >> 1;
  const int q = (ND > 1 ? (a1 >= half) : 0) + (ND > 2 ? 2 * (a2 >= half) : 0);
  const int fine = g.sleaf[g.fslot[slot * 4 + q]];
  const size_t vs = (size_t)g.n * g.ncell;
  const double* base = U + (size_t)fine * g.ncell;
  double acc[8][NV];
#pragma unroll
  for (int o = 0; o < (1 << ND); o += 2) {
    int c[3] = {0, 0, 0};
#pragma unroll
    for (int e = 0; e < ND; e++) {
      const int oe = (o >> e) & 1;
      if (e == d)
        c[e] = hi ? 2 * layer + oe : g.nx - 2 - 2 * layer + oe;
      else
        c[e] = (2 * ((e == (d == 0 ? 1 : 0)) ? a1 : a2) + oe) % g.nx;
    }
    const int cell = cell_index(g, c[0], c[1], c[2]);
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double2 pr = *reinterpret_cast<const double2*>(base + v * vs + cell);
      acc[o][v] = pr.x;
      acc[o + 1][v] = pr.y;
    }
  }
  const size_t out = (size_t)slot * NV * 2 * g.T + (size_t)layer * g.T + t;
#pragma unroll
  for (int v = 0; v < NV; v++) {
    double r;
    if constexpr (ND == 1)
      r = (acc[0][v] + acc[1][v]) * 0.5;
    else if constexpr (ND == 2)
      r = ((acc[0][v] + acc[1][v]) + (acc[2][v] + acc[3][v])) * 0.25;
    else
      r = (((acc[0][v] + acc[1][v]) + (acc[2][v] + acc[3][v])) + ((acc[4][v] + acc[5][v]) + (acc[6][v] + acc[7][v]))) *
          0.125;
    g.G[out + (size_t)v * 2 * g.T] = r;
  }
}

// Fine side of a coarse-fine face, one thread per transverse position t:
// both prolonged ghost layers (they lie in the same coarse cell and differ
// only in the half along the face normal, so they share the coarse value and
// its limited slopes), and with `fluxes` the face flux from the two interior
// cells and the two ghosts.  Prolongation never reads a prolonged value:
// with 2:1 balance over edges and corners the coarse stencil only touches
// coarse interior cells and restricted or same-level ghosts.
template <int ND, int PH, int FLUX, int LIM>
__global__ void __launch_bounds__(WGS) k_prolong_flux(Geo g, const double* __restrict__ U,
                                                      const double* __restrict__ pp,
                                                      const int32_t* __restrict__ list, int nlist, int fluxes) {
  using S = Sys<ND, PH>;
  constexpr int NV = S::NV;
  const long long i = (long long)blockIdx.x * WGS + threadIdx.x;
  if (i >= (long long)nlist * g.T) return;
  const int slot = list[i / g.T];
  const int t = (int)(i % g.T);
  const int a1 = ND > 1 ? t % g.nx : 0, a2 = ND > 2 ? t / g.nx : 0;
  const int fine = g.sleaf[slot];
  const int f = g.sface[slot];
  const int d = f >> 1, hi = f & 1;
  const int C = g.nbr[fine * 6 + f];
  int cc[3] = {0, 0, 0}, par0[3] = {0, 0, 0}, par1[3] = {0, 0, 0};
#pragma unroll
  for (int e = 0; e < ND; e++) {
    const int loc0 = e == d ? (hi ? g.nx : -1) : ((e == (d == 0 ? 1 : 0)) ? a1 : a2);
    const int loc1 = e == d ? (hi ? g.nx + 1 : -2) : loc0;
    const long long gl0 = (long long)g.ijk[fine * 3 + e] * g.nx + loc0;  // fine global coordinates
    const long long gl1 = (long long)g.ijk[fine * 3 + e] * g.nx + loc1;
    const long long gc = gl0 >> 1;                                         // the coarse cell (floor)
    cc[e] = (int)(((gc % g.nx) + g.nx) % g.nx);
    par0[e] = (int)(gl0 & 1);
    par1[e] = (int)(gl1 & 1);
  }
  double u0[NV], r0[NV], r1[NV];
  fetch_cons<NV, ND>(g, U, C, cc[0], cc[1], cc[2], u0);
#pragma unroll
  for (int v = 0; v < NV; v++) {
    r0[v] = u0[v];
    r1[v] = u0[v];
  }
#pragma unroll
  for (int e = 0; e < ND; e++) {
    double um[NV], up[NV];
    int lo[3] = {cc[0], cc[1], cc[2]}, hi3[3] = {cc[0], cc[1], cc[2]};
    lo[e] -= 1;
    hi3[e] += 1;
    fetch_cons<NV, ND>(g, U, C, lo[0], lo[1], lo[2], um);
    fetch_cons<NV, ND>(g, U, C, hi3[0], hi3[1], hi3[2], up);
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double tq = 0.25 * minmod(u0[v] - um[v], up[v] - u0[v]);
      r0[v] = par0[e] ? r0[v] + tq : r0[v] - tq;
      r1[v] = par1[e] ? r1[v] + tq : r1[v] - tq;
    }
  }
  const size_t base = (size_t)slot * NV * 2 * g.T + t;
#pragma unroll
  for (int v = 0; v < NV; v++) {
    g.G[base + (size_t)v * 2 * g.T] = r0[v];
    g.G[base + (size_t)v * 2 * g.T + g.T] = r1[v];
  }
  if (!fluxes) return;
  // face between cells m-1 and m along d: interior cells m-2, m-1 (hi) or
  // m, m+1 (lo), ghosts layer 0 next to the face, layer 1 beyond it
  const PhysParams P = load_phys(pp);
  double W[4][NV];  // interior cells (nearer the face last), then ghost layers 0, 1
  const int m = hi ? g.nx : 0;
#pragma unroll
  for (int j = 0; j < 2; j++) {
    int c[3] = {0, 0, 0};
    c[d] = hi ? m - 2 + j : m + 1 - j;
    if (ND > 1) c[d == 0 ? 1 : 0] = a1;
    if (ND > 2) c[d == 2 ? 1 : 2] = a2;
    double u[NV];
    const int cell = cell_index(g, c[0], c[1], c[2]);
#pragma unroll
    for (int v = 0; v < NV; v++) u[v] = U[uidx(g, v, fine, cell)];
    cons2prim<ND, PH>(u, W[j], P);
  }
  cons2prim<ND, PH>(r0, W[2], P);
  cons2prim<ND, PH>(r1, W[3], P);
  // the four cells in increasing coordinate along d
  double V0[NV], V1[NV], V2[NV], V3[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) {
    V0[v] = hi ? W[0][v] : W[3][v];
    V1[v] = hi ? W[1][v] : W[2][v];
    V2[v] = hi ? W[2][v] : W[1][v];
    V3[v] = hi ? W[3][v] : W[0][v];
  }
  double lo_[NV], vl[NV], vr[NV], hi_[NV], F[NV];
  const double th = pp[PP_CTHR + 3 * g.lvl[fine] + d];
  muscl<NV, LIM>(V0, V1, V2, lo_, vl, th);
  muscl<NV, LIM>(V1, V2, V3, vr, hi_, th);
  riemann_dir<ND, PH, FLUX>(d, vl, vr, F, P);
  const size_t fb = (size_t)slot * NV * g.T + t;
#pragma unroll
  for (int v = 0; v < NV; v++) g.FF[fb + (size_t)v * g.T] = F[v];
}

// ---------------------------------------------------------------------------
// regrid transfer (Sec. 1.3, refinement ratio 2): one workgroup per new leaf.
// A copied leaf takes its old cells; a child of a split leaf takes, per cell,
// the parent cell plus a quarter of its minmod slope per dimension (x, y, z
// order, added on the upper half), with the parent's ghost cells at its
// boundary; a merged parent takes the pairwise-tree sum of the 2^d child
// cells times 2^-d.  The same formulas as the coarse-fine ghost slabs.
// ---------------------------------------------------------------------------

template <int ND, int NV>
__global__ void __launch_bounds__(WGS) k_transfer(Geo gf, const double* __restrict__ Uf, Geo gt,
                                                  double* __restrict__ Ut, const int32_t* __restrict__ xf) {
  const int leaf = blockIdx.x;
  if (leaf >= gt.n) return;
  const int how = xf[leaf * 9];
  const int nx = gt.nx, h = nx / 2;
  const size_t vst = (size_t)gt.n * gt.ncell;
  int off[3] = {0, 0, 0};
#pragma unroll
  for (int e = 0; e < ND; e++) off[e] = gt.ijk[3 * leaf + e] & 1;
  for (int cell = threadIdx.x; cell < gt.ncell; cell += WGS) {
    int x[3] = {cell % nx, ND > 1 ? (cell / nx) % nx : 0, ND > 2 ? cell / (nx * nx) : 0};
    double r[NV];
    if (how == 0) {
      const int src = xf[leaf * 9 + 1];
#pragma unroll
      for (int v = 0; v < NV; v++) r[v] = Uf[uidx(gf, v, src, cell)];
    } else if (how == 1) {
      const int par = xf[leaf * 9 + 1];
      int pc[3] = {0, 0, 0};
#pragma unroll
      for (int e = 0; e < ND; e++) pc[e] = off[e] * h + x[e] / 2;
      double u0[NV];
      fetch_cons<NV, ND>(gf, Uf, par, pc[0], pc[1], pc[2], u0);
#pragma unroll
      for (int v = 0; v < NV; v++) r[v] = u0[v];
#pragma unroll
      for (int e = 0; e < ND; e++) {
        int lo[3] = {pc[0], pc[1], pc[2]}, hi[3] = {pc[0], pc[1], pc[2]};
        lo[e] -= 1;
        hi[e] += 1;
        double um[NV], up[NV];
        fetch_cons<NV, ND>(gf, Uf, par, lo[0], lo[1], lo[2], um);
        fetch_cons<NV, ND>(gf, Uf, par, hi[0], hi[1], hi[2], up);
#pragma unroll
        for (int v = 0; v < NV; v++) {
          const double tq = 0.25 * minmod(u0[v] - um[v], up[v] - u0[v]);
          r[v] = (x[e] & 1) ? r[v] + tq : r[v] - tq;
        }
      }
    } else {
      int q = 0, y[3] = {0, 0, 0};
#pragma unroll
      for (int e = 0; e < ND; e++) {
        const int qe = x[e] / h;
        q |= qe << e;
        y[e] = 2 * (x[e] - qe * h);
      }
      const int src = xf[leaf * 9 + 1 + q];
      double c8[1 << ND][NV];
#pragma unroll
      for (int a = 0; a < (1 << ND); a++) {
        const int z0 = y[0] + (a & 1), z1 = y[1] + (ND > 1 ? (a >> 1) & 1 : 0), z2 = y[2] + (ND > 2 ? (a >> 2) & 1 : 0);
        const int fc = cell_index(gf, z0, z1, z2);
#pragma unroll
        for (int v = 0; v < NV; v++) c8[a][v] = Uf[uidx(gf, v, src, fc)];
      }
#pragma unroll
      for (int v = 0; v < NV; v++) {
        if constexpr (ND == 1)
          r[v] = (c8[0][v] + c8[1][v]) * 0.5;
        else if constexpr (ND == 2)
          r[v] = ((c8[0][v] + c8[1][v]) + (c8[2][v] + c8[3][v])) * 0.25;
        else
          r[v] = (((c8[0][v] + c8[1][v]) + (c8[2][v] + c8[3][v])) + ((c8[4][v] + c8[5][v]) + (c8[6][v] + c8[7][v]))) *
                 0.125;
      }
    }
#pragma unroll
    for (int v = 0; v < NV; v++) Ut[v * vst + (size_t)leaf * gt.ncell + cell] = r[v];
  }
}

// ---------------------------------------------------------------------------
// stage update, 2D / 3D: one 16x16 workgroup per leaf, streaming z-planes
// ---------------------------------------------------------------------------

// Stage update of 16^2 / 16^3 leaves.  One 256-thread workgroup owns a leaf;
// thread (tx, ty) owns the z-column of cells (tx, ty, *).  Per z-plane:
//   (1) z direction in registers: slope of cell k+1, flux of face k+1/2;
//   (2) the plane's primitive values (plus the 2-cell x/y ghost ring) to LDS;
//   (3) limited slopes of all cells of the plane along x and y (LDS);
//   (4) x and y face fluxes from the slopes (LDS);
//   (5) flux divergence, summed x, y, z, and the SSP combination.
// Global loads are issued one phase or one plane ahead of their use, so the
// memory latency overlaps the FP64 work of the current plane.
//
// SPLIT = false: x and y share the slope and flux phases (3 barriers per
// plane, separate x/y LDS arrays).  SPLIT = true: x, then y, through one set
// of LDS arrays (5 barriers per plane, 40% less LDS, so more workgroups fit
// on a compute unit).  Both evaluate identical expressions.
//
// AR names the arithmetic the instance was compiled with (0: correctly
// rounded, no contraction; 1: the fast-arithmetic unit, stage_fast.hip); the
// body is the same text.
template <int ND, int PH, int FLUX, int LIM, bool SPLIT, int AR>
__global__ void __launch_bounds__(WGS, (Sys<ND, PH>::NV > 5) ? 1 : (SPLIT ? (lim_asym<LIM>() ? 1 : 3) : (lim_asym<LIM>() && AR == 0 ? 2 : 1))) k_stage_tile(Geo g, StageArgs a, const double* __restrict__ pp,
                                                                  Sched sc) {
  using S = Sys<ND, PH>;
  constexpr int NV = S::NV;
  constexpr int PW = NB + 4;
  constexpr int NZ = ND == 3 ? NB : 1;
  constexpr int NSX = NB * 18;  // x slopes: 16 rows x cells -1..16, [row][cell+1]
  constexpr int NFX = NB * 17;  // x faces: 16 rows x faces 0..16, [row][face]
  constexpr int NSB = SPLIT ? 1 : 2;
  // an asymmetric limiter keeps two half slopes per cell (toward the upper
  // and toward the lower face) and runs the split variant only
  constexpr bool ASYM = lim_asym<LIM>();
  // the combined variant with an asymmetric limiter forms each face's two
  // states in the flux phase from four primitives (each half slope serves that
  // one face only, so nothing is computed twice), with no slope phase
  constexpr bool RCF = ASYM && !SPLIT;
  constexpr int NSS = (SPLIT && !ASYM) ? 1 : 2;
  __shared__ double sP[NV][PW * PW];  // primitive plane incl. x/y ghost ring, (y+2)*PW + x+2
  __shared__ double sS[RCF ? 1 : NSS][NV][RCF ? 1 : NSX]; // half slopes 0.5*phi: x [row][cell+1]; y [cell+1][column]
                                      // (asymmetric: [0] toward the upper, [1] toward the lower face)
  __shared__ double sF[NSB][NV][NFX]; // fluxes: x [row][face]; y [face][column]
  auto& sSx = sS[0];
  auto& sSy = sS[RCF ? 0 : NSS - 1];
  auto& sFx = sF[0];
  auto& sFy = sF[NSB - 1];
  __shared__ double sZF[ND == 3 ? NV : 1][ND == 3 ? NB * NB : 1];  // +z coarse-fine face flux of the own column
  __shared__ int sLeaf;
  // fused features of the learned flagger (3D combined hydrodynamics, last
  // stage): rho and p of the output plane, and the running sums of the 16
  // sub-blocks (4^3 cells) of the current layer of sub-blocks, then their sums
  constexpr bool FEAT = ND == 3 && !SPLIT && PH != PH_MHD;
  __shared__ double sQ[FEAT ? 2 : 1][FEAT ? NB * NB : 1];
  __shared__ double sAcc[FEAT ? 2 : 1][FEAT ? 64 : 1];
  // add the output plane kp (in sQ) to its sub-blocks' sums, cells in y, x
  // order (planes arrive in z order): 32 threads, one per (variable, sub-block
  // column)
  auto pool_plane = [&](int kp) {
    if constexpr (FEAT) {
      const int t = threadIdx.x;
      if (t >= 32) return;
      const int var = t >> 4, bx = t & 3, by = (t >> 2) & 3;
      const int sb = bx + 4 * by + 16 * (kp >> 2);
      double acc = (kp & 3) == 0 ? 0.0 : sAcc[var][sb];
      for (int j = 0; j < 4; j++)
        for (int i = 0; i < 4; i++) acc = acc + sQ[var][(4 * by + j) * NB + 4 * bx + i];
      sAcc[var][sb] = acc;
    }
  };

  const PhysParams P = load_phys(pp);
  const double dt = pp[PP_DT];
  if (dt == 0.0) return;  // a device-timed run that has reached its end time
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const size_t vs = (size_t)g.n * g.ncell;  // variable stride of the state
  unsigned long long csmax = 0, ccmax = 0;
  int cbad = 0;

  // ring cell of this thread (tid < 128): x ring then y ring
  int rx = 0, ry = 0, rface = 0, rlayer = 0, ra1 = 0;
  if (tid < 64) {
    const int c = tid >> 4;
    ry = tid & 15;
    rx = c < 2 ? c - 2 : 14 + c;
    rface = rx < 0 ? 0 : 1;
    rlayer = rx < 0 ? -1 - rx : rx - NB;
    ra1 = ry;
  } else if (tid < 128) {
    const int u = tid - 64, c = u >> 4;
    rx = u & 15;
    ry = c < 2 ? c - 2 : 14 + c;
    rface = ry < 0 ? 2 : 3;
    rlayer = ry < 0 ? -1 - ry : ry - NB;
    ra1 = rx;
  }
  const bool ring = tid < 128;
  const int rdst = (ry + 2) * PW + rx + 2;

  for (int iter = 0;; iter++) {
    int leaf;
    if (sc.mode == 2) {
      if (tid == 0) sLeaf = queue_next(sc, g.n);
      __syncthreads();
      leaf = sLeaf;
      __syncthreads();
    } else {
      if (iter) break;
      leaf = pick_leaf(sc, blockIdx.x);
    }
    if (leaf >= g.n) break;

    const int lvl = g.lvl[leaf];
    const double rdx = g.rdx[lvl][0], rdy = g.rdx[lvl][1], rdz = ND == 3 ? g.rdx[lvl][2] : 0.0;
    // (r dx)^2 of Cada's smoothness switch per direction (0: none)
    const double thx = pp[PP_CTHR + 3 * lvl], thy = pp[PP_CTHR + 3 * lvl + 1],
                 thz = ND == 3 ? pp[PP_CTHR + 3 * lvl + 2] : 0.0;
    int kinds[2 * ND];
#pragma unroll
    for (int f = 0; f < 2 * ND; f++) kinds[f] = g.kind[leaf * 6 + f];

    const size_t col = (size_t)leaf * g.ncell + tx + NB * ty;
    const double* own = a.Uin + col;   // var 0 of cell (tx, ty, 0); plane stride NB*NB
    const double* ownn = a.Un + col;
    double* out = a.Uout + col;

    // source of this thread's ring cell: var 0 at plane 0, plane and var strides
    const double* rptr = a.Uin;
    int rks = 0;
    size_t rvs = vs;
    if (ring) {
      const int kd = kinds[rface];
      const int d = rface >> 1, hi = rface & 1;
      if (kd == NB_SAME || kd == NB_BND) {
        const int src = g.nbr[leaf * 6 + rface];
        const int along = kd == NB_SAME ? (hi ? rlayer : NB - 1 - rlayer) : (hi ? NB - 1 : 0);
        const int cell0 = d == 0 ? along + NB * ra1 : ra1 + NB * along;
        rptr = a.Uin + (size_t)src * g.ncell + cell0;
        rks = NB * NB;
        rvs = vs;
      } else {
        const int sl = g.slot[leaf * 6 + rface];
        rptr = g.G + (size_t)sl * NV * 2 * g.T + (size_t)rlayer * g.T + ra1;
        rks = NB;
        rvs = 2 * (size_t)g.T;
      }
    }

    // +z face source of this thread's column (ghost planes 16, 17)
    const double* zptr = a.Uin;
    int zls = 0;
    size_t zvs = vs;
    if constexpr (ND == 3) {
      const int kd = kinds[5];
      if (kd == NB_SAME) {
        zptr = a.Uin + (size_t)g.nbr[leaf * 6 + 5] * g.ncell + tx + NB * ty;
        zls = NB * NB;
      } else if (kd == NB_BND) {
        zptr = own + (NB - 1) * NB * NB;
        zls = 0;
      } else {
        zptr = g.G + (size_t)g.slot[leaf * 6 + 5] * NV * 2 * g.T + tx + NB * ty;
        zls = g.T;
        zvs = 2 * (size_t)g.T;
      }
    }

    double V0[NV], V1[NV], C2[NV], VLz[NV], Flo[NV], Cr[NV];
    double Cq0[NV], Cq1[NV];  // conserved planes k, k+1 (the update operands)
    if constexpr (ND == 3) {
      // a coarse-fine +z face: its flux comes from the fine-flux slabs, staged
      // here once per leaf so that no plane issues a load it waits for at once
      if (!(kinds[5] == NB_SAME || kinds[5] == NB_BND)) {
        double F[NV];
        cf_flux<NV, ND>(g, leaf, 5, kinds[5], tx, ty, F);
#pragma unroll
        for (int v = 0; v < NV; v++) sZF[v][tid] = F[v];
      }
      double vm2[NV], vm1[NV], c[NV], lo[NV], hi[NV], vlm1[NV];
      own_prim<ND, PH>(g, a.Uin, leaf, tx, ty, -2, vm2, P);
      own_prim<ND, PH>(g, a.Uin, leaf, tx, ty, -1, vm1, P);
      load_strided<NV>(own, vs, Cq0);
      cons2prim<ND, PH>(Cq0, V0, P);
      load_strided<NV>(own + NB * NB, vs, Cq1);
      cons2prim<ND, PH>(Cq1, V1, P);
      load_strided<NV>(own + 2 * NB * NB, vs, C2);
      muscl<NV, LIM>(vm2, vm1, V0, lo, vlm1, thz);
      muscl<NV, LIM>(vm1, V0, V1, lo, hi, thz);
      if (kinds[4] == NB_SAME || kinds[4] == NB_BND) {
        riemann<ND, PH, FLUX, (ND == 3 ? 2 : 0)>(vlm1, lo, Flo, P);
      } else {
        cf_flux<NV, ND>(g, leaf, 4, kinds[4], tx, ty, Flo);
      }
#pragma unroll
      for (int v = 0; v < NV; v++) VLz[v] = hi[v];
    } else {
      double c[NV];
      load_strided<NV>(own, vs, c);
      cons2prim<ND, PH>(c, V0, P);
    }
    if (ring) load_strided<NV>(rptr, rvs, Cr);
    // vmcnt(0) once before the plane loop: the first planes' loads are all
    // needed at once.  Inside the loop the compiler's own waits apply: the
    // loads of plane k+1 are issued during plane k, and the stores of plane
    // k are not waited for before the next plane's work
    __builtin_amdgcn_s_waitcnt(0x0F70);

    double Ui[NV], Uo[NV];
    for (int k = 0; k < NZ; k++) {
      double zd[NV];
      if constexpr (ND == 3) {
        // (1) z direction: prefetched plane k+2, slope of cell k+1, face k+1/2
        double V2[NV], VR1[NV], VL1[NV], Fhi[NV];
        cons2prim<ND, PH>(C2, V2, P);
        if constexpr (!SPLIT) {
          // the conserved values of plane k, loaded two planes ago for its
          // primitives, stay in registers as the update operand (no reload)
#pragma unroll
          for (int v = 0; v < NV; v++) {
            Ui[v] = Cq0[v];
            Cq0[v] = Cq1[v];
            Cq1[v] = C2[v];
          }
        }
        const int pn = k + 3;
        if (pn < NB)
          load_strided<NV>(own + pn * NB * NB, vs, C2);
        else if (pn < NB + 2)
          load_strided<NV>(zptr + (pn - NB) * zls, zvs, C2);
        muscl<NV, LIM>(V0, V1, V2, VR1, VL1, thz);
        if (k == NB - 1 && !(kinds[5] == NB_SAME || kinds[5] == NB_BND)) {
#pragma unroll
          for (int v = 0; v < NV; v++) Fhi[v] = sZF[v][tid];
        } else {
          riemann<ND, PH, FLUX, (ND == 3 ? 2 : 0)>(VLz, VR1, Fhi, P);
        }
#pragma unroll
        for (int v = 0; v < NV; v++) {
          zd[v] = (Fhi[v] - Flo[v]) * rdz;
          Flo[v] = Fhi[v];
          VLz[v] = VL1[v];
        }
        // (2) plane k to LDS; V1, V2 move down the queue
#pragma unroll
        for (int v = 0; v < NV; v++) {
          sP[v][(ty + 2) * PW + tx + 2] = V0[v];
          V0[v] = V1[v];
          V1[v] = V2[v];
        }
      } else {
#pragma unroll
        for (int v = 0; v < NV; v++) sP[v][(ty + 2) * PW + tx + 2] = V0[v];
      }
      if (ring) {
        double w[NV];
        cons2prim<ND, PH>(Cr, w, P);
#pragma unroll
        for (int v = 0; v < NV; v++) sP[v][rdst] = w[v];
        if (k + 1 < NZ) load_strided<NV>(rptr + (k + 1) * rks, rvs, Cr);
      }
      // operands of this plane's update (loaded early, consumed in phase 5;
      // in 3D the combined variant already holds U_in of the plane)
      if constexpr (!SPLIT) {
        if constexpr (ND != 3) load_strided<NV>(own + k * NB * NB, vs, Ui);
        if (a.stage > 1) load_strided<NV>(ownn + k * NB * NB, vs, Uo);
      }
      __syncthreads();
      if constexpr (FEAT) {
        if (a.Xout && k > 0) pool_plane(k - 1);
      }

      // The items of the slope and flux phases do not divide evenly over the
      // four waves (576 and 544 per plane); the remainder goes to the threads
      // of one wave, which changes from plane to plane (and leaf to leaf), so
      // that it is spread over the SIMDs instead of always falling on the
      // first wave's.  Each item is computed the same way by any thread.
      const int rs = (tid + 64 * (k + leaf)) & (WGS - 1);
      const int rf = (tid + 64 * (k + leaf + 2)) & (WGS - 1);
      // (3) limited slopes of the plane's cells (and the first ghost layer)
      auto slopes = [&](int t0, int t1) {
        if constexpr (RCF) return;  // no slope phase (above)
#pragma unroll
        for (int j = 0; j < 3; j++) {
          const int t = t0 + rs + j * WGS;
          if (t >= t1) break;
          const bool yd = t >= NSX;
          const int u = yd ? t - NSX : t;
          int b, st;
          if (!yd) {
            const int r = u / 18, c = u % 18 - 1;
            b = (r + 2) * PW + c + 2;
            st = 1;
          } else {
            const int c = u / NB - 1, r = u % NB;
            b = (c + 2) * PW + r + 2;
            st = PW;
          }
#pragma unroll
          for (int v = 0; v < NV; v++) {
            const double vm = sP[v][b - st], v0 = sP[v][b], vp = sP[v][b + st];
            // the half slope, formed once per cell: both face states of the
            // cell add or subtract the same product 0.5*phi
            const double sa = v0 - vm, sb = vp - v0;
            const double th = yd ? thy : thx;
            const double sl = 0.5 * limiter<LIM>(sa, sb, th);
            if constexpr (ASYM && !RCF) {
              sS[0][v][u] = sl;
              sS[1][v][u] = 0.5 * limiter<LIM>(sb, sa, th);
            } else if (!yd) {
              sSx[v][u] = sl;
            } else {
              sSy[v][u] = sl;
            }
          }
        }
      };
      // (4) face fluxes from the limited states.  A y face is solved as an x
      // face of the state with its x and y components exchanged (and the
      // flux exchanged back): the arithmetic is the same up to the order of
      // the first two terms of the v.v and B.B sums, and IEEE addition is
      // commutative, so the results are identical while a wave holding both
      // x and y faces runs one Riemann solver instead of two.
      auto fluxes = [&](int t0, int t1) {
        for (int t = t0 + rf; t < t1; t += WGS) {
          const bool yd = t >= NFX;
          const int u = yd ? t - NFX : t;
          int r, m, bl, st, s0, s1;
          if (!yd) {
            r = u / 17;
            m = u % 17;
            bl = (r + 2) * PW + m + 1;
            st = 1;
            s0 = r * 18 + m;
            s1 = s0 + 1;
          } else {
            m = u / NB;
            r = u % NB;
            bl = (m + 1) * PW + r + 2;
            st = PW;
            s0 = m * NB + r;
            s1 = s0 + NB;
          }
          const int bf = m == 0 ? 2 * yd : (m == NB ? 2 * yd + 1 : -1);
          double F[NV];
          if (bf >= 0 && !(kinds[bf] == NB_SAME || kinds[bf] == NB_BND)) {
            cf_flux<NV, ND>(g, leaf, bf, kinds[bf], r, k, F);
          } else {
            double vl[NV], vr[NV];
            if constexpr (RCF) {
              // cells a (lower) and b (upper) of the face and their outer
              // neighbours: a's half slope toward its upper face phi(a - a0,
              // b - a), b's toward its lower face phi(b1 - b, b - a), as the
              // slope phase forms them
              const double th = yd ? thy : thx;
#pragma unroll
              for (int v = 0; v < NV; v++) {
                const double pa0 = sP[v][bl - st], pa = sP[v][bl], pb = sP[v][bl + st], pb1 = sP[v][bl + 2 * st];
                const double da = pa - pa0, dab = pb - pa, db = pb1 - pb;
                vl[v] = pa + 0.5 * limiter<LIM>(da, dab, th);
                vr[v] = pb - 0.5 * limiter<LIM>(db, dab, th);
              }
            } else {
              const double* slu = &sS[ASYM ? 0 : (yd ? NSS - 1 : 0)][0][0];  // toward the upper face
              const double* sll = &sS[ASYM ? 1 : (yd ? NSS - 1 : 0)][0][0];  // toward the lower face
#pragma unroll
              for (int v = 0; v < NV; v++) {
                vl[v] = sP[v][bl] + slu[v * NSX + s0];
                vr[v] = sP[v][bl + st] - sll[v * NSX + s1];
              }
            }
            if (yd) {
              swap_xy<ND, PH>(vl);
              swap_xy<ND, PH>(vr);
            }
            riemann<ND, PH, FLUX, 0>(vl, vr, F, P);
            if (yd) swap_xy<ND, PH>(F);
          }
          double* fo = &sF[yd ? NSB - 1 : 0][0][0];
#pragma unroll
          for (int v = 0; v < NV; v++) fo[v * NFX + u] = F[v];
        }
      };
      double accx[NV];
      if constexpr (!SPLIT) {
        if constexpr (!RCF) {
          slopes(0, 2 * NSX);
          __syncthreads();
        }
        fluxes(0, 2 * NFX);
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NV; v++) accx[v] = (sFx[v][ty * 17 + tx + 1] - sFx[v][ty * 17 + tx]) * rdx;
      } else {
        slopes(0, NSX);
        __syncthreads();
        fluxes(0, NFX);
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NV; v++) accx[v] = (sFx[v][ty * 17 + tx + 1] - sFx[v][ty * 17 + tx]) * rdx;
        slopes(NSX, 2 * NSX);
        __syncthreads();
        load_strided<NV>(own + k * NB * NB, vs, Ui);
        if (a.stage > 1) load_strided<NV>(ownn + k * NB * NB, vs, Uo);
        fluxes(NFX, 2 * NFX);
        __syncthreads();
      }

      // (5) divergence (x, then y, then z) and the SSP combination
#pragma unroll
      for (int v = 0; v < NV; v++) {
        double acc = accx[v];
        acc = acc + (sFy[v][(ty + 1) * NB + tx] - sFy[v][ty * NB + tx]) * rdy;
        if constexpr (ND == 3) acc = acc + zd[v];
        const double tmp = Ui[v] - dt * acc;
        const double res = combine<NV>(a.stage, a.rk, a.stage > 1 ? Uo[v] : 0.0, tmp);
        out[v * vs + (size_t)k * NB * NB] = res;
        Ui[v] = res;
      }
      if (a.cflred) {
        const double rd[3] = {rdx, rdy, rdz};
        cfl_cell<ND, PH>(Ui, P, rd, csmax, ccmax, cbad);
      }
      if constexpr (FEAT) {
        if (a.Xout) {
          double w[NV];
          cons2prim<ND, PH>(Ui, w, P);
          sQ[0][tid] = Ui[0];
          sQ[1][tid] = pressure<ND, PH>(w, P);
        }
      }
    }
    if constexpr (FEAT) {
      // the last plane's sums, then the 128 features of the leaf: sub-block
      // means over their leaf mean (summed in sub-block order), minus one
      if (a.Xout) {
        __syncthreads();
        pool_plane(NB - 1);
        __syncthreads();
        if (tid < 128) {
          const int var = tid >> 6, sb = tid & 63;
          double m = 0.0;
          for (int i = 0; i < 64; i++) m = m + sAcc[var][i] / 64.0;
          const double mtot = m / 64.0;
          const float fv = (float)(sAcc[var][sb] / 64.0 / mtot - 1.0);
          a.Xout[(size_t)leaf * 128 + 64 * var + sb] = to_bf16(fv);
        }
      }
    }
    if constexpr (ND == 3 && !SPLIT && PH != PH_MHD) {
      bool rany = false;
#pragma unroll
      for (int f = 0; f < 6; f++) rany = rany || (a.Gw && kinds[f] == NB_COARSER);
      if (rany) {
        __threadfence_block();
        __syncthreads();
        restrict_leaf<NV>(g, a, leaf, tid);
      }
    }
  }
  if (a.cflred) cfl_fold(a.cflred, csmax, ccmax, cbad);
}

// ---------------------------------------------------------------------------
// stage update of 16^3 leaves in two launches (variant 2, 3D MHD): the z
// direction of every column first (k_stage_zcol), then the x/y planes with
// the z flux divergence read back (k_stage_xy).  The 9-variable z queue of
// the one-launch kernel keeps it at one workgroup per CU; split, each launch
// fits two.  Same expressions in the same order as k_stage_tile, so the
// results are identical bit for bit.  AR names the arithmetic of the unit
// that instantiates them (0: correctly rounded, stage_zsplit.hip; 1: fast,
// stage_zsplit_fast.hip), as for k_stage_tile.
// ---------------------------------------------------------------------------

// (1) of the stage update for whole columns: thread (tx, ty) streams its
// column through the planes, with the z slope of cell k+1 and the flux of face
// k+1/2 in registers, and writes (F_{k+1/2} - F_{k-1/2}) * rdz of every cell
// to a.Zd (the state layout).  No LDS, no barrier.
template <int PH, int FLUX, int LIM, int AR>
__global__ void __launch_bounds__(WGS, 2) k_stage_zcol(Geo g, StageArgs a, const double* __restrict__ pp, Sched sc) {
  constexpr int ND = 3;
  constexpr int NV = Sys<ND, PH>::NV;
  const PhysParams P = load_phys(pp);
  if (pp[PP_DT] == 0.0) return;  // a device-timed run that has reached its end time
  const int leaf = pick_leaf(sc, blockIdx.x);
  if (leaf >= g.n) return;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const size_t vs = (size_t)g.n * g.ncell;
  const int lvl = g.lvl[leaf];
  const double rdz = g.rdx[lvl][2];
  const double thz = pp[PP_CTHR + 3 * lvl + 2];
  const int kd4 = g.kind[leaf * 6 + 4], kd5 = g.kind[leaf * 6 + 5];
  const size_t col = (size_t)leaf * g.ncell + tx + NB * ty;
  const double* own = a.Uin + col;
  double* zo = a.Zd + col;

  // +z face source of this thread's column (ghost planes 16, 17)
  const double* zptr = a.Uin;
  int zls = 0;
  size_t zvs = vs;
  if (kd5 == NB_SAME) {
    zptr = a.Uin + (size_t)g.nbr[leaf * 6 + 5] * g.ncell + tx + NB * ty;
    zls = NB * NB;
  } else if (kd5 == NB_BND) {
    zptr = own + (NB - 1) * NB * NB;
    zls = 0;
  } else {
    zptr = g.G + (size_t)g.slot[leaf * 6 + 5] * NV * 2 * g.T + tx + NB * ty;
    zls = g.T;
    zvs = 2 * (size_t)g.T;
  }

  double V0[NV], V1[NV], C2[NV], VLz[NV], Flo[NV];
  {
    double vm2[NV], vm1[NV], c[NV], lo[NV], hi[NV], vlm1[NV];
    own_prim<ND, PH>(g, a.Uin, leaf, tx, ty, -2, vm2, P);
    own_prim<ND, PH>(g, a.Uin, leaf, tx, ty, -1, vm1, P);
    load_strided<NV>(own, vs, c);
    cons2prim<ND, PH>(c, V0, P);
    load_strided<NV>(own + NB * NB, vs, c);
    cons2prim<ND, PH>(c, V1, P);
    load_strided<NV>(own + 2 * NB * NB, vs, C2);
    muscl<NV, LIM>(vm2, vm1, V0, lo, vlm1, thz);
    muscl<NV, LIM>(vm1, V0, V1, lo, hi, thz);
    if (kd4 == NB_SAME || kd4 == NB_BND) {
      riemann<ND, PH, FLUX, 2>(vlm1, lo, Flo, P);
    } else {
      cf_flux<NV, ND>(g, leaf, 4, kd4, tx, ty, Flo);
    }
#pragma unroll
    for (int v = 0; v < NV; v++) VLz[v] = hi[v];
  }
  for (int k = 0; k < NB; k++) {
    double V2[NV], VR1[NV], VL1[NV], Fhi[NV];
    cons2prim<ND, PH>(C2, V2, P);
    const int pn = k + 3;
    if (pn < NB)
      load_strided<NV>(own + pn * NB * NB, vs, C2);
    else if (pn < NB + 2)
      load_strided<NV>(zptr + (pn - NB) * zls, zvs, C2);
    muscl<NV, LIM>(V0, V1, V2, VR1, VL1, thz);
    if (k == NB - 1 && !(kd5 == NB_SAME || kd5 == NB_BND)) {
      cf_flux<NV, ND>(g, leaf, 5, kd5, tx, ty, Fhi);
    } else {
      riemann<ND, PH, FLUX, 2>(VLz, VR1, Fhi, P);
    }
#pragma unroll
    for (int v = 0; v < NV; v++) {
      zo[v * vs + (size_t)k * NB * NB] = (Fhi[v] - Flo[v]) * rdz;
      Flo[v] = Fhi[v];
      VLz[v] = VL1[v];
      V0[v] = V1[v];
      V1[v] = V2[v];
    }
  }
}

// (2)-(5) of the stage update on x/y planes, the z divergence from a.Zd: per
// plane the primitives (with the 2-cell x/y ghost ring) to LDS, then every x
// and y face flux with the face's two limited states formed in place from
// four primitives (the half slope of the lower cell toward the face and of the
// upper cell toward it: each is needed by that one face only, so no slope is
// stored and no slope phase or barrier is needed), then the divergence and
// the SSP combination.  Two barriers per plane, 68 KB of LDS for MHD.
template <int PH, int FLUX, int LIM, int AR>
__global__ void __launch_bounds__(WGS, 2) k_stage_xy(Geo g, StageArgs a, const double* __restrict__ pp, Sched sc) {
  constexpr int ND = 3;
  using S = Sys<ND, PH>;
  constexpr int NV = S::NV;
  constexpr int PW = NB + 4;
  constexpr int NFX = NB * 17;  // x faces: 16 rows x faces 0..16, [row][face]
  __shared__ double sP[NV][PW * PW];  // primitive plane incl. x/y ghost ring, (y+2)*PW + x+2
  __shared__ double sF[2][NV][NFX];   // fluxes: x [row][face]; y [face][column]
  __shared__ int sLeaf;

  const PhysParams P = load_phys(pp);
  const double dt = pp[PP_DT];
  if (dt == 0.0) return;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const size_t vs = (size_t)g.n * g.ncell;
  unsigned long long csmax = 0, ccmax = 0;
  int cbad = 0;

  // ring cell of this thread (tid < 128): x ring then y ring
  int rx = 0, ry = 0, rface = 0, rlayer = 0, ra1 = 0;
  if (tid < 64) {
    const int c = tid >> 4;
    ry = tid & 15;
    rx = c < 2 ? c - 2 : 14 + c;
    rface = rx < 0 ? 0 : 1;
    rlayer = rx < 0 ? -1 - rx : rx - NB;
    ra1 = ry;
  } else if (tid < 128) {
    const int u = tid - 64, c = u >> 4;
    rx = u & 15;
    ry = c < 2 ? c - 2 : 14 + c;
    rface = ry < 0 ? 2 : 3;
    rlayer = ry < 0 ? -1 - ry : ry - NB;
    ra1 = rx;
  }
  const bool ring = tid < 128;
  const int rdst = (ry + 2) * PW + rx + 2;

  for (int iter = 0;; iter++) {
    int leaf;
    if (sc.mode == 2) {
      if (tid == 0) sLeaf = queue_next(sc, g.n);
      __syncthreads();
      leaf = sLeaf;
      __syncthreads();
    } else {
      if (iter) break;
      leaf = pick_leaf(sc, blockIdx.x);
    }
    if (leaf >= g.n) break;

    const int lvl = g.lvl[leaf];
    const double rdx = g.rdx[lvl][0], rdy = g.rdx[lvl][1], rdz = g.rdx[lvl][2];
    const double thx = pp[PP_CTHR + 3 * lvl], thy = pp[PP_CTHR + 3 * lvl + 1];
    int kinds[4];
#pragma unroll
    for (int f = 0; f < 4; f++) kinds[f] = g.kind[leaf * 6 + f];

    const size_t col = (size_t)leaf * g.ncell + tx + NB * ty;
    const double* own = a.Uin + col;
    const double* ownn = a.Un + col;
    const double* zdp = a.Zd + col;
    double* out = a.Uout + col;

    // source of this thread's ring cell: var 0 at plane 0, plane and var strides
    const double* rptr = a.Uin;
    int rks = 0;
    size_t rvs = vs;
    if (ring) {
      const int kd = kinds[rface];
      const int d = rface >> 1, hi = rface & 1;
      if (kd == NB_SAME || kd == NB_BND) {
        const int src = g.nbr[leaf * 6 + rface];
        const int along = kd == NB_SAME ? (hi ? rlayer : NB - 1 - rlayer) : (hi ? NB - 1 : 0);
        const int cell0 = d == 0 ? along + NB * ra1 : ra1 + NB * along;
        rptr = a.Uin + (size_t)src * g.ncell + cell0;
        rks = NB * NB;
        rvs = vs;
      } else {
        const int sl = g.slot[leaf * 6 + rface];
        rptr = g.G + (size_t)sl * NV * 2 * g.T + (size_t)rlayer * g.T + ra1;
        rks = NB;
        rvs = 2 * (size_t)g.T;
      }
    }

    double Cq[NV], Cr[NV], Ui[NV], Uo[NV], Zk[NV];
    load_strided<NV>(own, vs, Cq);
    if (ring) load_strided<NV>(rptr, rvs, Cr);

    for (int k = 0; k < NB; k++) {
      // (2) plane k (own cell and ring cell) to LDS; the next plane's loads,
      // U^n and the z divergence of this plane issued for phase 5
      {
        double w[NV];
        cons2prim<ND, PH>(Cq, w, P);
#pragma unroll
        for (int v = 0; v < NV; v++) {
          sP[v][(ty + 2) * PW + tx + 2] = w[v];
          Ui[v] = Cq[v];
        }
      }
      if (k + 1 < NB) load_strided<NV>(own + (k + 1) * NB * NB, vs, Cq);
      if (ring) {
        double w[NV];
        cons2prim<ND, PH>(Cr, w, P);
#pragma unroll
        for (int v = 0; v < NV; v++) sP[v][rdst] = w[v];
        if (k + 1 < NB) load_strided<NV>(rptr + (k + 1) * rks, rvs, Cr);
      }
      if (a.stage > 1) load_strided<NV>(ownn + k * NB * NB, vs, Uo);
      load_strided<NV>(zdp + k * NB * NB, vs, Zk);
      __syncthreads();

      // (3)+(4) face fluxes; a y face is solved as an x face of the state
      // with its x and y components exchanged (as in k_stage_tile)
      for (int t = tid; t < 2 * NFX; t += WGS) {
        const bool yd = t >= NFX;
        const int u = yd ? t - NFX : t;
        int r, m, bl, st;
        if (!yd) {
          r = u / 17;
          m = u % 17;
          bl = (r + 2) * PW + m + 1;
          st = 1;
        } else {
          m = u / NB;
          r = u % NB;
          bl = (m + 1) * PW + r + 2;
          st = PW;
        }
        const int bf = m == 0 ? 2 * yd : (m == NB ? 2 * yd + 1 : -1);
        double F[NV];
        if (bf >= 0 && !(kinds[bf] == NB_SAME || kinds[bf] == NB_BND)) {
          cf_flux<NV, ND>(g, leaf, bf, kinds[bf], r, k, F);
        } else {
          const double th = yd ? thy : thx;
          double vl[NV], vr[NV];
#pragma unroll
          for (int v = 0; v < NV; v++) {
            // cells a (lower) and b (upper) of the face and their outer neighbours
            const double pa0 = sP[v][bl - st], pa = sP[v][bl], pb = sP[v][bl + st], pb1 = sP[v][bl + 2 * st];
            // the half slopes as the slope phase of k_stage_tile forms them: a
            // toward its upper face phi(a - a0, b - a), b toward its lower face
            // phi(b1 - b, b - a) (asymmetric limiters) or phi(b - a, b1 - b)
            const double da = pa - pa0, dab = pb - pa, db = pb1 - pb;
            const double su = 0.5 * limiter<LIM>(da, dab, th);
            const double sl = lim_asym<LIM>() ? 0.5 * limiter<LIM>(db, dab, th) : 0.5 * limiter<LIM>(dab, db, th);
            vl[v] = pa + su;
            vr[v] = pb - sl;
          }
          if (yd) {
            swap_xy<ND, PH>(vl);
            swap_xy<ND, PH>(vr);
          }
          riemann<ND, PH, FLUX, 0>(vl, vr, F, P);
          if (yd) swap_xy<ND, PH>(F);
        }
        double* fo = &sF[yd ? 1 : 0][0][0];
#pragma unroll
        for (int v = 0; v < NV; v++) fo[v * NFX + u] = F[v];
      }
      __syncthreads();

      // (5) divergence (x, then y, then z) and the SSP combination
#pragma unroll
      for (int v = 0; v < NV; v++) {
        double acc = (sF[0][v][ty * 17 + tx + 1] - sF[0][v][ty * 17 + tx]) * rdx;
        acc = acc + (sF[1][v][(ty + 1) * NB + tx] - sF[1][v][ty * NB + tx]) * rdy;
        acc = acc + Zk[v];
        const double tmp = Ui[v] - dt * acc;
        const double res = combine<NV>(a.stage, a.rk, a.stage > 1 ? Uo[v] : 0.0, tmp);
        out[v * vs + (size_t)k * NB * NB] = res;
        Ui[v] = res;
      }
      if (a.cflred) {
        const double rd[3] = {rdx, rdy, rdz};
        cfl_cell<ND, PH>(Ui, P, rd, csmax, ccmax, cbad);
      }
    }
  }
  if (a.cflred) cfl_fold(a.cflred, csmax, ccmax, cbad);
}

// ---------------------------------------------------------------------------
// stage update, 1D: a leaf of nx cells in chunks of 256, one workgroup each
// ---------------------------------------------------------------------------

template <int PH, int FLUX, int LIM>
__global__ void __launch_bounds__(WGS) k_stage_line(Geo g, StageArgs a, const double* __restrict__ pp, Sched sc) {
  using S = Sys<1, PH>;
  constexpr int NV = S::NV;
  constexpr int CH = WGS;
  __shared__ double sP[NV][CH + 4];
  __shared__ double sL[NV][CH + 2];
  __shared__ double sR[NV][CH + 2];
  __shared__ double sF[NV][CH + 1];
  const PhysParams P = load_phys(pp);
  const double dt = pp[PP_DT];
  if (dt == 0.0) return;
  const int tid = threadIdx.x;
  const int nch = (g.nx + CH - 1) / CH;
  const int leaf = sc.mode == 0 ? sc.leaf0 : (int)(blockIdx.x / nch);
  const int c0 = (int)(blockIdx.x % nch) * CH;
  if (leaf >= g.n) return;
  const int lvl = g.lvl[leaf];
  const double rdx = g.rdx[lvl][0];
  const int kind0 = g.kind[leaf * 6 + 0], kind1 = g.kind[leaf * 6 + 1];

  for (int t = tid; t < CH + 4; t += WGS) {
    const int x = c0 - 2 + t;
    if (x > g.nx + 1) continue;
    double u[NV], w[NV];
    fetch_cons<NV, 1>(g, a.Uin, leaf, x, 0, 0, u);
    cons2prim<1, PH>(u, w, P);
#pragma unroll
    for (int v = 0; v < NV; v++) sP[v][t] = w[v];
  }
  __syncthreads();
  for (int t = tid; t < CH + 2; t += WGS) {
    const int x = c0 - 1 + t;
    if (x > g.nx) continue;
    double vm[NV], v0[NV], vp[NV], lo[NV], hi[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
      vm[v] = sP[v][t];
      v0[v] = sP[v][t + 1];
      vp[v] = sP[v][t + 2];
    }
    muscl<NV, LIM>(vm, v0, vp, lo, hi, pp[PP_CTHR + 3 * lvl]);
#pragma unroll
    for (int v = 0; v < NV; v++) {
      sL[v][t] = hi[v];
      sR[v][t] = lo[v];
    }
  }
  __syncthreads();
  for (int t = tid; t < CH + 1; t += WGS) {
    const int m = c0 + t;
    if (m > g.nx) continue;
    double F[NV];
    if (m == 0 && !(kind0 == NB_SAME || kind0 == NB_BND)) {
      cf_flux<NV, 1>(g, leaf, 0, kind0, 0, 0, F);
    } else if (m == g.nx && !(kind1 == NB_SAME || kind1 == NB_BND)) {
      cf_flux<NV, 1>(g, leaf, 1, kind1, 0, 0, F);
    } else {
      double vl[NV], vr[NV];
#pragma unroll
      for (int v = 0; v < NV; v++) {
        vl[v] = sL[v][t];
        vr[v] = sR[v][t + 1];
      }
      riemann<1, PH, FLUX, 0>(vl, vr, F, P);
    }
#pragma unroll
    for (int v = 0; v < NV; v++) sF[v][t] = F[v];
  }
  __syncthreads();
  const int x = c0 + tid;
  unsigned long long csmax = 0, ccmax = 0;
  int cbad = 0;
  if (x < g.nx) {
    double res[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double acc = (sF[v][tid + 1] - sF[v][tid]) * rdx;
      const size_t id = uidx(g, v, leaf, x);
      const double tmp = a.Uin[id] - dt * acc;
      const double un = a.stage == 1 ? 0.0 : a.Un[id];
      res[v] = combine<NV>(a.stage, a.rk, un, tmp);
      a.Uout[id] = res[v];
    }
    if (a.cflred) {
      const double rd[3] = {rdx, 0.0, 0.0};
      cfl_cell<1, PH>(res, P, rd, csmax, ccmax, cbad);
    }
  }
  if (a.cflred) cfl_fold(a.cflred, csmax, ccmax, cbad);
}

// ---------------------------------------------------------------------------
// Courant reduction and validation (Sec. 2.1)
// ---------------------------------------------------------------------------


// red[0] = bits of max_cells sum_d (|v_d|+c_d)/dx_d, red[1] = bits of the max
// signal speed (GLM c_h), red[2] = non-physical flag.  Non-negative doubles
// order like their bit patterns, so integer atomics give the exact maximum.
template <int ND, int PH>
__global__ void __launch_bounds__(WGS) k_cfl(Geo g, const double* __restrict__ U, const double* __restrict__ pp,
                                             unsigned long long* red) {
  constexpr int NV = Sys<ND, PH>::NV;
  const PhysParams P = load_phys(pp);
  const long long total = (long long)g.n * g.ncell;
  unsigned long long smax = 0, cmax = 0;
  int bad = 0;
  for (long long i = (long long)blockIdx.x * WGS + threadIdx.x; i < total; i += (long long)gridDim.x * WGS) {
    const int leaf = (int)(i / g.ncell), cell = (int)(i % g.ncell);
    double u[NV], v[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) u[k] = U[uidx(g, k, leaf, cell)];
    cons2prim<ND, PH>(u, v, P);
    if (nonphysical<ND, PH>(v)) {
      bad = 1;
      continue;
    }
    const int lvl = g.lvl[leaf];
    double s = 0.0, cm = 0.0;
#pragma unroll
    for (int d = 0; d < ND; d++) {
      const double w = fabs(v[1 + d]) + wave_speed_dir<ND, PH>(v, d, P);
      const double tq = w * g.rdx[lvl][d];
      s = d == 0 ? tq : s + tq;
      cm = w > cm ? w : cm;
    }
    const unsigned long long sb = (unsigned long long)__double_as_longlong(s);
    const unsigned long long cb = (unsigned long long)__double_as_longlong(cm);
    smax = sb > smax ? sb : smax;
    cmax = cb > cmax ? cb : cmax;
  }
  smax = wave_max_u64(smax);
  cmax = wave_max_u64(cmax);
  bad = __any(bad);
  if ((threadIdx.x & 63) == 0) {
    if (smax) atomicMax(&red[0], smax);
    if (cmax) atomicMax(&red[1], cmax);
    if (bad) atomicOr(&red[2], 1ull);
  }
}

// ---------------------------------------------------------------------------
// Loehner flags (Sec. 1.3): one workgroup per leaf
// ---------------------------------------------------------------------------

template <int ND, int PH>
__device__ __forceinline__ void rho_p(const Geo& g, const double* __restrict__ U, int leaf, int x, int y, int z,
                                      const PhysParams& P, double& rho, double& p) {
  constexpr int NV = Sys<ND, PH>::NV;
  double u[NV], v[NV];
  fetch_cons<NV, ND>(g, U, leaf, x, y, z, u);
  cons2prim<ND, PH>(u, v, P);
  rho = v[0];
  p = pressure<ND, PH>(v, P);
}

template <int ND, int PH>
__global__ void __launch_bounds__(WGS) k_lohner(Geo g, const double* __restrict__ U, const double* __restrict__ pp,
                                                const double* __restrict__ lp, int max_level, double* emax_out,
                                                int8_t* flags, const int8_t* __restrict__ only) {
  __shared__ double red[WGS / 64];
  const int leaf = blockIdx.x;
  if (only && !only[leaf]) return;
  const PhysParams P = load_phys(pp);
  const double eps = lp[LP_EPS], wr = lp[LP_WRHO], wp = lp[LP_WP];
  double m = 0.0;
  for (int cell = threadIdx.x; cell < g.ncell; cell += WGS) {
    const int x = cell % g.nx;
    const int y = ND > 1 ? (cell / g.nx) % g.nx : 0;
    const int z = ND > 2 ? cell / (g.nx * g.nx) : 0;
    double r0, p0;
    rho_p<ND, PH>(g, U, leaf, x, y, z, P, r0, p0);
    double nr = 0.0, dr = 0.0, np = 0.0, dp = 0.0;
#pragma unroll
    for (int d = 0; d < ND; d++) {
      int lo[3] = {x, y, z}, hi[3] = {x, y, z};
      lo[d] -= 1;
      hi[d] += 1;
      double rm, pm, rp, pq;
      rho_p<ND, PH>(g, U, leaf, lo[0], lo[1], lo[2], P, rm, pm);
      rho_p<ND, PH>(g, U, leaf, hi[0], hi[1], hi[2], P, rp, pq);
      const double d2r = rp - 2.0 * r0 + rm;
      const double ddr = fabs(rp - r0) + fabs(r0 - rm) + eps * (fabs(rp) + 2.0 * fabs(r0) + fabs(rm));
      const double d2p = pq - 2.0 * p0 + pm;
      const double ddp = fabs(pq - p0) + fabs(p0 - pm) + eps * (fabs(pq) + 2.0 * fabs(p0) + fabs(pm));
      nr = d == 0 ? d2r * d2r : nr + d2r * d2r;
      dr = d == 0 ? ddr * ddr : dr + ddr * ddr;
      np = d == 0 ? d2p * d2p : np + d2p * d2p;
      dp = d == 0 ? ddp * ddp : dp + ddp * ddp;
    }
    const double er = dr > 0.0 ? sqrt(nr / dr) : 0.0;
    const double ep = dp > 0.0 ? sqrt(np / dp) : 0.0;
    const double e = wr * er + wp * ep;
    if (e > m) m = e;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double y = __shfl_xor(m, o, 64);
    m = y > m ? y : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = red[0];
    for (int w = 1; w < WGS / 64; w++) mm = red[w] > mm ? red[w] : mm;
    const int l = g.lvl[leaf];
    int8_t fl = 0;
    if (l < max_level && mm > lp[LP_TOL])
      fl = 1;
    else if (l > 1 && mm < lp[LP_CTOL])
      fl = -1;
    flags[leaf] = fl;
    emax_out[leaf] = mm;
  }
}

#ifndef AMRV_STAGE_UNIT
// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__global__ void k_set_scalars(double* dst, double a0, double a1, double a2, double a3, int n) {
  const int i = threadIdx.x;
  const double v = i == 0 ? a0 : (i == 1 ? a1 : (i == 2 ? a2 : a3));
  if (i < n) dst[i] = v;
}

__global__ void k_reset_u32(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_scale(double* U, const double* __restrict__ facp, long long count) {
  const double fac = *facp;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    U[i] = U[i] * fac;
}

// ---------------------------------------------------------------------------
// launchers: dispatch runtime configuration onto template instances
// ---------------------------------------------------------------------------

#endif  // AMRV_STAGE_UNIT

template <int V>
using IC = std::integral_constant<int, V>;

// call fn(IC<ndim>, IC<physics>, IC<flux>, IC<limiter>) for the runtime
// configuration; the polytrope has no HLLC instance
template <class Fn>
static void dispatch(const LaunchCfg& c, Fn&& fn) {
  auto lim = [&](auto nd, auto ph, auto fl) {
    if (c.lim == LIM_MINMOD)
      fn(nd, ph, fl, IC<LIM_MINMOD>{});
    else if (c.lim == LIM_MC)
      fn(nd, ph, fl, IC<LIM_MC>{});
    else if (c.lim == LIM_KOREN)
      fn(nd, ph, fl, IC<LIM_KOREN>{});
    else if (c.lim == LIM_CADA)
      fn(nd, ph, fl, IC<LIM_CADA>{});
    else
      fn(nd, ph, fl, IC<LIM_VANLEER>{});
  };
  auto flx = [&](auto nd, auto ph) {
    if (c.flux == FLX_TVDLF)
      lim(nd, ph, IC<FLX_TVDLF>{});
    else if (c.flux == FLX_HLL)
      lim(nd, ph, IC<FLX_HLL>{});
    else
      lim(nd, ph, IC<FLX_HLLC>{});
  };
  auto poly_flx = [&](auto nd) {
    if (c.flux == FLX_TVDLF)
      lim(nd, IC<PH_POLY>{}, IC<FLX_TVDLF>{});
    else
      lim(nd, IC<PH_POLY>{}, IC<FLX_HLL>{});
  };
  auto phys = [&](auto nd) {
    if (c.phys == PH_MHD)
      flx(nd, IC<PH_MHD>{});
    else if (c.phys == PH_POLY)
      poly_flx(nd);
    else
      flx(nd, IC<PH_EULER>{});
  };
  if (c.ndim == 1)
    phys(IC<1>{});
  else if (c.ndim == 2)
    phys(IC<2>{});
  else
    phys(IC<3>{});
}

static inline unsigned blocks_for(long long work) { return (unsigned)((work + WGS - 1) / WGS); }

// The combined-variant stage kernels of 2D/3D non-MHD physics are compiled
// in units of their own with LLVM's ILP-maximising scheduler, which helps
// them at two waves per SIMD and slows the others: stage_ilp.hip (correctly
// rounded, no contraction) and stage_fast.hip (fast arithmetic, AR = 1);
// each instantiation exists in one unit only.
hipError_t launch_stage_combined(const Geo& g, const LaunchCfg& c, const StageArgs& a, const double* physp,
                                 const Sched& s, int grid, hipStream_t st);
hipError_t launch_stage_combined_fast(const Geo& g, const LaunchCfg& c, const StageArgs& a, const double* physp,
                                      const Sched& s, int grid, hipStream_t st);
// the two-launch stage update of the 3D MHD forests (variant 2), in units of
// their own (stage_zsplit.hip, and stage_zsplit_fast.hip in fast arithmetic)
hipError_t launch_stage_zsplit(const Geo& g, const LaunchCfg& c, const StageArgs& a, const double* physp,
                               const Sched& s, int grid, hipStream_t st);
hipError_t launch_stage_zsplit_fast(const Geo& g, const LaunchCfg& c, const StageArgs& a, const double* physp,
                                    const Sched& s, int grid, hipStream_t st);
template <int ND, int PH, int LM>
constexpr bool in_ilp_unit() {
  return ND >= 2 && PH != PH_MHD;
}

#ifdef AMRV_STAGE_UNIT
#if AMRV_STAGE_UNIT >= 2
#if AMRV_STAGE_UNIT == 3
#define AMRV_ZSPLIT_LAUNCHER launch_stage_zsplit_fast
#define AMRV_ZSPLIT_AR 1
#else
#define AMRV_ZSPLIT_LAUNCHER launch_stage_zsplit
#define AMRV_ZSPLIT_AR 0
#endif
// z columns over every leaf (one workgroup per leaf, XCD remap as the
// schedule's), then the x/y planes in the schedule the forest uses
hipError_t AMRV_ZSPLIT_LAUNCHER(const Geo& g, const LaunchCfg& c, const StageArgs& a, const double* physp,
                                const Sched& s, int grid, hipStream_t st) {
  Sched zs = s;
  int zgrid = 1;
  if (s.mode != 0) {
    zs.mode = 1;
    zgrid = s.xcd_remap ? 8 * ((g.n + 7) / 8) : g.n;
  }
  dispatch(c, [&](auto nd, auto ph, auto fl, auto lm) {
    constexpr int ND = decltype(nd)::value, FL = decltype(fl)::value, LM = decltype(lm)::value;
    constexpr int PH = decltype(ph)::value;
    if constexpr (ND == 3 && PH == PH_MHD) {
      hipLaunchKernelGGL((k_stage_zcol<PH, FL, LM, AMRV_ZSPLIT_AR>), dim3(zgrid), dim3(WGS), 0, st, g, a, physp, zs);
      hipLaunchKernelGGL((k_stage_xy<PH, FL, LM, AMRV_ZSPLIT_AR>), dim3(grid), dim3(WGS), 0, st, g, a, physp, s);
    }
  });
  return hipGetLastError();
}
#undef AMRV_ZSPLIT_LAUNCHER
#undef AMRV_ZSPLIT_AR
#else
#if AMRV_STAGE_UNIT == 1
#define AMRV_UNIT_LAUNCHER launch_stage_combined_fast
#else
#define AMRV_UNIT_LAUNCHER launch_stage_combined
#endif
hipError_t AMRV_UNIT_LAUNCHER(const Geo& g, const LaunchCfg& c, const StageArgs& a, const double* physp,
                              const Sched& s, int grid, hipStream_t st) {
  dispatch(c, [&](auto nd, auto ph, auto fl, auto lm) {
    constexpr int ND = decltype(nd)::value, FL = decltype(fl)::value, LM = decltype(lm)::value;
    constexpr int PH = decltype(ph)::value;
    if constexpr (in_ilp_unit<ND, PH, LM>())
      hipLaunchKernelGGL((k_stage_tile<ND, PH, FL, LM, false, AMRV_STAGE_UNIT>), dim3(grid), dim3(WGS), 0, st, g, a,
                         physp, s);
  });
  return hipGetLastError();
}
#undef AMRV_UNIT_LAUNCHER
#endif  // AMRV_STAGE_UNIT >= 2
#else

hipError_t launch_restrict(const Geo& g, const LaunchCfg& c, const double* U, const int32_t* list, int nlist,
                           hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  const unsigned nb = blocks_for((long long)nlist * 2 * g.T);
#define BODY_R                                                                                                        \
  if (c.phys == PH_MHD) {                                                                                             \
    hipLaunchKernelGGL((k_restrict<ND, Sys<ND, PH_MHD>::NV>), dim3(nb), dim3(WGS), 0, st, g, U, list, nlist);         \
  } else if (c.phys == PH_POLY) {                                                                                     \
    hipLaunchKernelGGL((k_restrict<ND, Sys<ND, PH_POLY>::NV>), dim3(nb), dim3(WGS), 0, st, g, U, list, nlist);        \
  } else {                                                                                                            \
    hipLaunchKernelGGL((k_restrict<ND, Sys<ND, PH_EULER>::NV>), dim3(nb), dim3(WGS), 0, st, g, U, list, nlist);       \
  }
  if (c.ndim == 1) {
    constexpr int ND = 1;
    BODY_R
  } else if (c.ndim == 2) {
    constexpr int ND = 2;
    BODY_R
  } else {
    constexpr int ND = 3;
    BODY_R
  }
#undef BODY_R
  return hipGetLastError();
}

hipError_t launch_transfer(const Geo& from, const double* Uf, const Geo& to, double* Ut, const int32_t* xfer,
                           const LaunchCfg& c, hipStream_t st) {
  if (to.n <= 0) return hipSuccess;
#define BODY_T                                                                                                        \
  if (c.phys == PH_MHD) {                                                                                             \
    hipLaunchKernelGGL((k_transfer<ND, Sys<ND, PH_MHD>::NV>), dim3(to.n), dim3(WGS), 0, st, from, Uf, to, Ut, xfer);  \
  } else if (c.phys == PH_POLY) {                                                                                     \
    hipLaunchKernelGGL((k_transfer<ND, Sys<ND, PH_POLY>::NV>), dim3(to.n), dim3(WGS), 0, st, from, Uf, to, Ut, xfer); \
  } else {                                                                                                            \
    hipLaunchKernelGGL((k_transfer<ND, Sys<ND, PH_EULER>::NV>), dim3(to.n), dim3(WGS), 0, st, from, Uf, to, Ut, xfer); \
  }
  if (c.ndim == 1) {
    constexpr int ND = 1;
    BODY_T
  } else if (c.ndim == 2) {
    constexpr int ND = 2;
    BODY_T
  } else {
    constexpr int ND = 3;
    BODY_T
  }
#undef BODY_T
  return hipGetLastError();
}

hipError_t launch_prolong(const Geo& g, const LaunchCfg& c, const double* U, const double* physp,
                          const int32_t* list, int nlist, bool fluxes, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  const unsigned nb = blocks_for((long long)nlist * g.T);
  dispatch(c, [&](auto nd, auto ph, auto fl, auto lm) {
    constexpr int ND = decltype(nd)::value, FL = decltype(fl)::value, LM = decltype(lm)::value;
    constexpr int PH = decltype(ph)::value;
    hipLaunchKernelGGL((k_prolong_flux<ND, PH, FL, LM>), dim3(nb), dim3(WGS), 0, st, g, U, physp, list, nlist,
                       fluxes ? 1 : 0);
  });
  return hipGetLastError();
}

hipError_t launch_stage(const Geo& g, const LaunchCfg& c, const StageArgs& a, const double* physp, const Sched& s,
                        int grid, hipStream_t st) {
  bool combined = false;
  if (c.variant == 2) {
    if (c.ndim != 3 || c.phys != PH_MHD || a.Zd == nullptr) return hipErrorInvalidValue;
    return c.arith == 1 ? launch_stage_zsplit_fast(g, c, a, physp, s, grid, st)
                        : launch_stage_zsplit(g, c, a, physp, s, grid, st);
  }
  dispatch(c, [&](auto nd, auto ph, auto fl, auto lm) {
    constexpr int ND = decltype(nd)::value, FL = decltype(fl)::value, LM = decltype(lm)::value;
    constexpr int PH = decltype(ph)::value;
    if constexpr (ND == 1)
      hipLaunchKernelGGL((k_stage_line<PH, FL, LM>), dim3(grid), dim3(WGS), 0, st, g, a, physp, s);
    else if (c.variant == 1 || (lim_asym<LM>() && !in_ilp_unit<ND, PH, LM>()))
      hipLaunchKernelGGL((k_stage_tile<ND, PH, FL, LM, true, 0>), dim3(grid), dim3(WGS), 0, st, g, a, physp, s);
    else if constexpr (in_ilp_unit<ND, PH, LM>())
      combined = true;
    else if constexpr (!lim_asym<LM>())
      hipLaunchKernelGGL((k_stage_tile<ND, PH, FL, LM, false, 0>), dim3(grid), dim3(WGS), 0, st, g, a, physp, s);
  });
  if (combined && c.arith == 1) return launch_stage_combined_fast(g, c, a, physp, s, grid, st);
  if (combined) return launch_stage_combined(g, c, a, physp, s, grid, st);
  return hipGetLastError();
}

hipError_t launch_cfl(const Geo& g, const LaunchCfg& c, const double* U, const double* physp,
                      unsigned long long* red, hipStream_t st) {
  const long long total = (long long)g.n * g.ncell;
  long long nb = (total + WGS - 1) / WGS;
  if (nb > 4096) nb = 4096;
#define BODY_C(ND)                                                                                                    \
  if (c.phys == PH_MHD)                                                                                               \
    hipLaunchKernelGGL((k_cfl<ND, PH_MHD>), dim3((unsigned)nb), dim3(WGS), 0, st, g, U, physp, red);                  \
  else if (c.phys == PH_POLY)                                                                                         \
    hipLaunchKernelGGL((k_cfl<ND, PH_POLY>), dim3((unsigned)nb), dim3(WGS), 0, st, g, U, physp, red);                 \
  else                                                                                                                \
    hipLaunchKernelGGL((k_cfl<ND, PH_EULER>), dim3((unsigned)nb), dim3(WGS), 0, st, g, U, physp, red);
  if (c.ndim == 1) {
    BODY_C(1)
  } else if (c.ndim == 2) {
    BODY_C(2)
  } else {
    BODY_C(3)
  }
#undef BODY_C
  return hipGetLastError();
}

hipError_t launch_lohner(const Geo& g, const LaunchCfg& c, const double* U, const double* physp, const double* lohp,
                         int max_level, double* emax, int8_t* flags, const int8_t* only, hipStream_t st) {
#define BODY_L(ND)                                                                                                    \
  if (c.phys == PH_MHD)                                                                                               \
    hipLaunchKernelGGL((k_lohner<ND, PH_MHD>), dim3(g.n), dim3(WGS), 0, st, g, U, physp, lohp, max_level, emax, flags, \
                       only);                                                                                         \
  else if (c.phys == PH_POLY)                                                                                         \
    hipLaunchKernelGGL((k_lohner<ND, PH_POLY>), dim3(g.n), dim3(WGS), 0, st, g, U, physp, lohp, max_level, emax, flags, \
                       only);                                                                                         \
  else                                                                                                                \
    hipLaunchKernelGGL((k_lohner<ND, PH_EULER>), dim3(g.n), dim3(WGS), 0, st, g, U, physp, lohp, max_level, emax, flags, \
                       only);
  if (c.ndim == 1) {
    BODY_L(1)
  } else if (c.ndim == 2) {
    BODY_L(2)
  } else {
    BODY_L(3)
  }
#undef BODY_L
  return hipGetLastError();
}

__global__ void k_dt_update(unsigned long long* red, double* pp, double* t, unsigned* err, double cfl, double t_end,
                            double glm_cr, int mhd) {
  if (threadIdx.x != 0) return;
  const unsigned long long sb = red[0], cb = red[1];
  if (red[2]) *err = 1u;
  const double smax = __longlong_as_double((long long)sb);
  const double ch = __longlong_as_double((long long)cb);
  const double tn = *t;
  double dt = 0.0;
  if (tn < t_end && smax > 0.0 && !red[2]) {
    dt = cfl / smax;
    const double rem = t_end - tn;
    if (rem < dt) dt = rem;
    err[CNT_TAKEN - CNT_ERR] += 1u;
  }
  *t = tn + dt;
  pp[PP_DT] = dt;
  if (mhd) {
    pp[PP_CH] = ch;
    pp[PP_DAMP] = exp(-(dt * ch) / glm_cr);
  }
  red[0] = 0ull;
  red[1] = 0ull;
  red[2] = 0ull;
}

hipError_t launch_dt_update(unsigned long long* red, double* pp, double* t, unsigned* err, double cfl, double t_end,
                            double glm_cr, int mhd, hipStream_t st) {
  hipLaunchKernelGGL(k_dt_update, dim3(1), dim3(64), 0, st, red, pp, t, err, cfl, t_end, glm_cr, mhd);
  return hipGetLastError();
}

hipError_t launch_set_scalars(double* dst, const double* vals, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, st, dst, vals[0], n > 1 ? vals[1] : 0.0,
                     n > 2 ? vals[2] : 0.0, n > 3 ? vals[3] : 0.0, n);
  return hipGetLastError();
}

hipError_t launch_reset_u32(unsigned* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_u32, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_scale_var(double* U, const double* facp, long long count, hipStream_t st) {
  long long nb = (count + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_scale, dim3((unsigned)nb), dim3(256), 0, st, U, facp, count);
  return hipGetLastError();
}

#endif  // AMRV_STAGE_UNIT

}  // namespace amrv
