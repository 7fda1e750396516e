// stage_common.hpp -- device helpers shared by the stage-update kernels
// (kernels.hip, stage3d.hip): state indexing, ghost cells of a leaf from its
// neighbours or the coarse-fine slabs, coarse-fine face fluxes, the Courant
// fold, the persistent work queues, the SSP combination and the fused
// restriction of a 3D leaf's result.
#pragma once
#include "internal.hpp"
#include "physics.hpp"

namespace amrv {

constexpr int NB = 16;   // block edge in 2D/3D
constexpr int WGS = 256; // workgroup size

__device__ __forceinline__ size_t uidx(const Geo& g, int v, int leaf, int cell) {
  return ((size_t)v * g.n + leaf) * g.ncell + cell;
}

__device__ __forceinline__ int cell_index(const Geo& g, int x, int y, int z) { return x + g.nx * (y + g.nx * z); }

// conserved values of ghost cell (layer, a1, a2) across face f of `leaf`
template <int NV>
__device__ __forceinline__ void ghost_cons(const Geo& g, const double* __restrict__ U, int leaf, int f, int layer,
                                           int a1, int a2, double* u) {
  const int kind = g.kind[leaf * 6 + f];
  const int d = f >> 1, hi = f & 1;
  if (kind == NB_SAME || kind == NB_BND) {
    const int src = g.nbr[leaf * 6 + f];
    const int along = (kind == NB_SAME) ? (hi ? layer : g.nx - 1 - layer) : (hi ? g.nx - 1 : 0);
    int c[3] = {0, 0, 0};
    c[d] = along;
    if (g.ndim > 1) c[d == 0 ? 1 : 0] = a1;
    if (g.ndim > 2) c[d == 2 ? 1 : 2] = a2;
    const int cell = cell_index(g, c[0], c[1], c[2]);
#pragma unroll
    for (int v = 0; v < NV; v++) u[v] = U[uidx(g, v, src, cell)];
  } else {
    const int s = g.slot[leaf * 6 + f];
    const size_t base = (size_t)s * NV * 2 * g.T + (size_t)layer * g.T + a2 * g.nx + a1;
#pragma unroll
    for (int v = 0; v < NV; v++) u[v] = g.G[base + (size_t)v * 2 * g.T];
  }
}

// conserved values of a cell of `leaf` given in local coordinates; at most one
// coordinate may lie in the two face-ghost layers
template <int NV, int ND>
__device__ __forceinline__ void fetch_cons(const Geo& g, const double* __restrict__ U, int leaf, int x, int y, int z,
                                           double* u) {
  int c[3] = {x, y, z};
  int f = -1, layer = 0;
#pragma unroll
  for (int d = 0; d < ND; d++) {
    if (c[d] < 0) {
      f = 2 * d;
      layer = -1 - c[d];
    } else if (c[d] >= g.nx) {
      f = 2 * d + 1;
      layer = c[d] - g.nx;
    }
  }
  if (f < 0) {
    const int cell = cell_index(g, x, y, z);
#pragma unroll
    for (int v = 0; v < NV; v++) u[v] = U[uidx(g, v, leaf, cell)];
    return;
  }
  const int d = f >> 1;
  const int a1 = ND > 1 ? c[d == 0 ? 1 : 0] : 0;
  const int a2 = ND > 2 ? c[d == 2 ? 1 : 2] : 0;
  ghost_cons<NV>(g, U, leaf, f, layer, a1, a2, u);
}

// face flux of a coarse-fine face taken from the fine-side flux slabs: the
// fine leaf's own value, or on the coarse side the mean of the 2^(d-1) fine
// fluxes covering the coarse face
template <int NV, int ND>
__device__ __forceinline__ void cf_flux(const Geo& g, int leaf, int f, int kind, int a1, int a2, double* F) {
  const int s = g.slot[leaf * 6 + f];
  if (kind == NB_COARSER) {
    const size_t base = (size_t)s * NV * g.T + a2 * g.nx + a1;
#pragma unroll
    for (int v = 0; v < NV; v++) F[v] = g.FF[base + (size_t)v * g.T];
    return;
  }
  if constexpr (ND == 1) {
    const int fs = g.fslot[s * 4];
#pragma unroll
    for (int v = 0; v < NV; v++) F[v] = g.FF[(size_t)fs * NV + v];
  } else if constexpr (ND == 2) {
    const int fs = g.fslot[s * 4 + (a1 >= NB / 2)];
    const size_t base = (size_t)fs * NV * g.T;
    const int t0 = (2 * a1) & (NB - 1), t1 = (2 * a1 + 1) & (NB - 1);
#pragma unroll
    for (int v = 0; v < NV; v++) F[v] = (g.FF[base + (size_t)v * g.T + t0] + g.FF[base + (size_t)v * g.T + t1]) * 0.5;
  } else {
    const int fs = g.fslot[s * 4 + (a1 >= NB / 2) + 2 * (a2 >= NB / 2)];
    const size_t base = (size_t)fs * NV * g.T;
    const int x0 = (2 * a1) & (NB - 1), x1 = (2 * a1 + 1) & (NB - 1);
    const int y0 = (2 * a2) & (NB - 1), y1 = (2 * a2 + 1) & (NB - 1);
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double* p = g.FF + base + (size_t)v * g.T;
      F[v] = ((p[y0 * NB + x0] + p[y0 * NB + x1]) + (p[y1 * NB + x0] + p[y1 * NB + x1])) * 0.25;
    }
  }
}

__device__ __forceinline__ PhysParams load_phys(const double* __restrict__ pp) {
  PhysParams P;
  P.gamma = pp[PP_GAMMA];
  P.gm1 = pp[PP_GM1];
  P.igm1 = pp[PP_IGM1];
  P.ch = pp[PP_CH];
  P.cad = pp[PP_CAD];
  P.gcad = pp[PP_GCAD];
  return P;
}

template <int ND, int PH, int FLUX>
__device__ __forceinline__ void riemann_dir(int d, double* vl, double* vr, double* F, const PhysParams& P) {
  if (d == 0) {
    riemann<ND, PH, FLUX, 0>(vl, vr, F, P);
  } else if constexpr (ND > 1) {
    if (d == 1) {
      riemann<ND, PH, FLUX, (ND > 1 ? 1 : 0)>(vl, vr, F, P);
    } else if constexpr (ND > 2) {
      riemann<ND, PH, FLUX, (ND > 2 ? 2 : 0)>(vl, vr, F, P);
    }
  }
}

// Courant quantities of one cell (Sec. 2.1): sum_d (|v_d| + c_d) / dx_d and
// max_d (|v_d| + c_d), with the non-physical test; same arithmetic as k_cfl
template <int ND, int PH>
__device__ __forceinline__ void cfl_cell(const double* u, const PhysParams& P, const double* rd,
                                         unsigned long long& smax, unsigned long long& cmax, int& bad) {
  constexpr int NV = Sys<ND, PH>::NV;
  double v[NV];
  cons2prim<ND, PH>(u, v, P);
  if (nonphysical<ND, PH>(v)) {
    bad = 1;
    return;
  }
  double s = 0.0, cm = 0.0;
#pragma unroll
  for (int d = 0; d < ND; d++) {
    const double w = fabs(v[1 + d]) + wave_speed_dir<ND, PH>(v, d, P);
    const double tq = w * rd[d];
    s = d == 0 ? tq : s + tq;
    cm = w > cm ? w : cm;
  }
  const unsigned long long sb = (unsigned long long)__double_as_longlong(s);
  const unsigned long long cb = (unsigned long long)__double_as_longlong(cm);
  smax = sb > smax ? sb : smax;
  cmax = cb > cmax ? cb : cmax;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  return x;
}

// fold per-thread Courant maxima into the reduction words (one atomic per wave)
__device__ __forceinline__ void cfl_fold(unsigned long long* red, unsigned long long smax, unsigned long long cmax,
                                         int bad) {
  smax = wave_max_u64(smax);
  cmax = wave_max_u64(cmax);
  bad = __any(bad);
  if ((threadIdx.x & 63) == 0) {
    if (smax) atomicMax(&red[0], smax);
    if (cmax) atomicMax(&red[1], cmax);
    if (bad) atomicOr(&red[2], 1ull);
  }
}


__device__ __forceinline__ int pick_leaf(const Sched& sc, int b) {
  if (sc.mode == 0) return sc.leaf0;
  if (sc.xcd_remap) return (b & 7) * sc.per_xcd + (b >> 3);
  return b;
}

// next leaf of a persistent workgroup (n when all are taken).  Workgroups are
// dealt to the 8 XCDs round robin by index; with xcd_remap each XCD first
// drains its own queue over a contiguous eighth of the (Morton-ordered)
// leaves, so neighbouring leaves, whose ghost cells each reads from the
// other, pass through the same L2, then helps with the others' queues.
__device__ __forceinline__ int queue_next(const Sched& sc, int n) {
  if (!sc.xcd_remap) return (int)atomicAdd(sc.counter, 1u);
  const int home = blockIdx.x & 7;
  for (int j = 0; j < 8; j++) {
    const int q = (home + j) & 7;
    const int lo = q * sc.per_xcd;
    const int len = min(sc.per_xcd, n - lo);
    if (len <= 0 || __atomic_load_n(sc.counter + q, __ATOMIC_RELAXED) >= (unsigned)len) continue;
    const unsigned i = atomicAdd(sc.counter + q, 1u);
    if (i < (unsigned)len) return lo + (int)i;
  }
  return n;
}

template <int ND, int PH>
__device__ __forceinline__ void own_prim(const Geo& g, const double* __restrict__ U, int leaf, int x, int y, int z,
                                         double* v, const PhysParams& P) {
  constexpr int NV = Sys<ND, PH>::NV;
  double u[NV];
  fetch_cons<NV, ND>(g, U, leaf, x, y, z, u);
  cons2prim<ND, PH>(u, v, P);
}

// exchange the x and y components (velocity or momentum, magnetic field) of a
// state or flux vector
template <int ND, int PH>
__device__ __forceinline__ void swap_xy(double* q) {
  using S = Sys<ND, PH>;
  double t = q[1];
  q[1] = q[2];
  q[2] = t;
  if constexpr (PH == PH_MHD) {
    t = q[S::IB];
    q[S::IB] = q[S::IB + 1];
    q[S::IB + 1] = t;
  }
}

template <int NV>
__device__ __forceinline__ double combine(int stage, int rk, double un, double tmp) {
  if (stage == 1) return tmp;
  if (rk == 2) return 0.5 * un + 0.5 * tmp;
  if (stage == 2) return 0.75 * un + 0.25 * tmp;
  return (1.0 / 3.0) * un + (2.0 / 3.0) * tmp;
}

template <int NV>
__device__ __forceinline__ void load_strided(const double* __restrict__ p, size_t vs, double* u) {
#pragma unroll
  for (int v = 0; v < NV; v++) u[v] = p[v * vs];
}

// (6) of the 3D stage update: restriction of a leaf's new state onto the
// ghost slabs of its coarser neighbours (buffer a.Gw): after all planes are
// stored, the 2 layers x 8 x 8 coarse ghost cells of each such face, one
// thread each (tid < 128), from the 2x2x2 fine cells just written
// (cache-hot), summed in the order of the separate restriction pass.
template <int NV>
__device__ __forceinline__ void restrict_leaf(const Geo& g, const StageArgs& a, int leaf, int tid) {
  constexpr int NB = 16;
  if (tid >= 128) return;
  const size_t vs = (size_t)g.n * g.ncell;
  const double* src = a.Uout + (size_t)leaf * g.ncell;
  const int lay = tid >> 6, c1 = tid & 7, c2 = (tid >> 3) & 7;
  for (int f = 0; f < 6; f++) {
    if (g.kind[leaf * 6 + f] != NB_COARSER) continue;
    const int d = f >> 1, e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
    const int rs = g.slot[g.nbr[leaf * 6 + f] * 6 + (f ^ 1)];
    if (rs < 0) continue;
    int cc[3];
    cc[d] = (f & 1) ? NB / 2 - 1 - lay : lay;
    cc[e1] = c1;
    cc[e2] = c2;
    const int tt = 8 * (g.ijk[leaf * 3 + e1] & 1) + NB * 8 * (g.ijk[leaf * 3 + e2] & 1) + c1 + NB * c2;
    double* o = a.Gw + (size_t)rs * NV * 2 * g.T + (size_t)lay * g.T + tt;
    const double* p0 = src + 2 * cc[0] + NB * (2 * cc[1] + NB * 2 * cc[2]);
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double* p = p0 + v * vs;
      const double2 q0 = *reinterpret_cast<const double2*>(p);
      const double2 q1 = *reinterpret_cast<const double2*>(p + NB);
      const double2 q2 = *reinterpret_cast<const double2*>(p + NB * NB);
      const double2 q3 = *reinterpret_cast<const double2*>(p + NB * NB + NB);
      o[(size_t)v * 2 * g.T] = (((q0.x + q0.y) + (q1.x + q1.y)) + ((q2.x + q2.y) + (q3.x + q3.y))) * 0.125;
    }
  }
}

}  // namespace amrv
