// multigrid.hip -- geometric multigrid Helmholtz solver on one uniform
// cell-centred grid and the reaction-diffusion time steps built on it
// (declared in include/amrv_mg.h; the method's multigrid of Sec. 1.4 and the
// reaction-diffusion schemes of Sec. 2.5).
//
// Layout in the caller's workspace (every array 256-byte aligned):
//   phi[field][level], f[field][level]   n_l^d doubles each, n_l = n >> l,
//                                         x fastest; level 0 is the grid
//   tmp[4]                                n^d doubles (reaction-diffusion
//                                         temporaries)
//   par                                   lambda per field, 1/diagonal per
//                                         field and level, 1/h^2 per level
// plus pinned host memory for the per-block residual maxima, folded on the
// host after each cycle.
//
// A V-cycle: on each level above the tail, `pre` red-black sweeps and a
// launch that forms the residual on the 2^d children of every coarse cell,
// averages it into the coarse right-hand side and zeroes the coarse
// correction (in 2D both in one tiled launch, k_mg_down2d); the coarse
// levels of at most 4,096 cells are solved by one workgroup per field with
// every level resident in LDS (the whole descent, the exact solve on the
// 2-per-side grid and the ascent in one launch); back up, a launch adds the
// bi/trilinear interpolation of the coarse correction, then `post` sweeps
// (again one tiled launch in 2D, the finest one also folding the residual
// norms).  Fields (u and v of the reaction-diffusion steps) are solved by the
// same launches (grid y = field).  These grids are small (a 256^2 field is
// 512 KiB), so the cycle is bound by launch and synchronisation latency, not
// by HBM: a solve enqueues several cycles before its first host check, and
// each cycle can be replayed from a captured HIP graph (use_graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/amrv_mg.h"
#include "errors.hpp"
#include "mg_internal.hpp"

namespace {

constexpr int MG_MAXL = 14;   // n <= 8192: 13 levels down to 2 cells per side
constexpr int NFMAX = 2;
constexpr int TAIL_CELLS = 4096;
constexpr int TAIL_THREADS = 1024;
constexpr int TK = TAIL_CELLS / 2 / TAIL_THREADS;  // colour cells per tail thread on its top level
constexpr int PAR_LAM = 0;
constexpr int PAR_IDIAG = NFMAX;                       // + field * MG_MAXL + level
constexpr int PAR_IH2 = NFMAX + NFMAX * MG_MAXL;       // + level
constexpr int PAR_COUNT = PAR_IH2 + MG_MAXL;

struct MgDev {
  int nd, bc, nlev, nf;
  int n[MG_MAXL];
  int lg[MG_MAXL];              // log2(n[l])
  int cells[MG_MAXL];
  int loff[MG_MAXL];            // LDS offset (doubles) of the tail's phi_l; f_l follows it
  int loffv[MG_MAXL];           // the same with a coefficient: phi_l, f_l, eps_l
  const double* eps[MG_MAXL];   // cell coefficient per level (variable-coefficient solves)
  double* phi[NFMAX][MG_MAXL];
  double* f[NFMAX][MG_MAXL];
  double* phi2[NFMAX][MG_MAXL]; // 2D levels above the tail: the tiled launches'
                                // second buffer (down writes it, up reads it)
  const double* par;
  unsigned long long* hpart;  // pinned host slots of per-block maxima: [2][NFMAX][maxb]
  int maxb;
};

struct MgPar {
  double v[PAR_COUNT];
};

struct RdK {
  int model;
  double Du, Dv, p1, p2, p3;
};

// neighbours with the boundary rule: periodic wrap, or (Neumann) the cell
// itself, whose value is the mirrored ghost
__device__ __forceinline__ int im(int i, int n, int bc) { return i > 0 ? i - 1 : (bc == AMRV_MG_PERIODIC ? n - 1 : 0); }
__device__ __forceinline__ int ip(int i, int n, int bc) { return i < n - 1 ? i + 1 : (bc == AMRV_MG_PERIODIC ? 0 : n - 1); }

// cell t of a level with n = 2^lg cells per side
template <int ND>
__device__ __forceinline__ void decode(int t, int n, int lg, int& x, int& y, int& z) {
  x = t & (n - 1);
  const int r = t >> lg;
  y = ND == 3 ? (r & (n - 1)) : r;
  z = ND == 3 ? (r >> lg) : 0;
}

// Laplacian: per direction ((w- + w+) - 2 w) * (1/h^2), added x, y, z
template <int ND>
__device__ __forceinline__ double lap_at(const double* a, int x, int y, int z, int n, int bc, double ih2) {
  const int row = (z * n + y) * n;
  const double w = a[row + x];
  double out = ((a[row + im(x, n, bc)] + a[row + ip(x, n, bc)]) - 2.0 * w) * ih2;
  out = out + ((a[(z * n + im(y, n, bc)) * n + x] + a[(z * n + ip(y, n, bc)) * n + x]) - 2.0 * w) * ih2;
  if constexpr (ND == 3)
    out = out + ((a[(im(z, n, bc) * n + y) * n + x] + a[(ip(z, n, bc) * n + y) * n + x]) - 2.0 * w) * ih2;
  return out;
}

// Gauss-Seidel update of one cell: phi = (sum of neighbours / h^2 - f) / (2 d / h^2 + lambda)
template <int ND>
__device__ __forceinline__ void gs_cell(double* p, const double* rhs, int x, int y, int z, int n, int bc, double ih2,
                                        double idiag) {
  const int row = (z * n + y) * n;
  double s = (p[row + im(x, n, bc)] + p[row + ip(x, n, bc)]) +
             (p[(z * n + im(y, n, bc)) * n + x] + p[(z * n + ip(y, n, bc)) * n + x]);
  if constexpr (ND == 3) s = s + (p[(im(z, n, bc) * n + y) * n + x] + p[(ip(z, n, bc) * n + y) * n + x]);
  p[row + x] = (s * ih2 - rhs[row + x]) * idiag;
}

// cell t of colour c among the cells with (x + y + z) % 2 == c
template <int ND>
__device__ __forceinline__ void colour_cell(int t, int n, int lg, int c, int& x, int& y, int& z) {
  const int xh = t & ((n >> 1) - 1);
  const int r = t >> (lg - 1);
  y = ND == 3 ? (r & (n - 1)) : r;
  z = ND == 3 ? (r >> lg) : 0;
  x = 2 * xh + ((y + z + c) & 1);
}

// residual f - (lap(phi) - lambda phi) of one fine cell
template <int ND>
__device__ __forceinline__ double resid(const double* p, const double* rhs, int x, int y, int z, int n, int bc,
                                        double ih2, double lam) {
  const int i = (z * n + y) * n + x;
  return rhs[i] - (lap_at<ND>(p, x, y, z, n, bc, ih2) - lam * p[i]);
}

// coarse cell (xc, yc, zc): mean of the children's residuals
template <int ND>
__device__ __forceinline__ double restrict_cell(const double* p, const double* rhs, int xc, int yc, int zc, int n,
                                                int bc, double ih2, double lam) {
  double s = 0.0;
#pragma unroll
  for (int dz = 0; dz < (ND == 3 ? 2 : 1); dz++)
#pragma unroll
    for (int dy = 0; dy < 2; dy++)
#pragma unroll
      for (int dx = 0; dx < 2; dx++) s += resid<ND>(p, rhs, 2 * xc + dx, 2 * yc + dy, 2 * zc + dz, n, bc, ih2, lam);
  return s * (ND == 3 ? 0.125 : 0.25);
}

// ---- variable coefficient: div(eps grad phi) - lambda phi, face coefficient
// the mean of the two cells; a neighbour that is the cell itself (a Neumann
// face) contributes no flux -----------------------------------------------

template <int ND>
__device__ __forceinline__ void nbr_list(int x, int y, int z, int n, int bc, int* j) {
  const int row = (z * n + y) * n;
  j[0] = row + im(x, n, bc);
  j[1] = row + ip(x, n, bc);
  j[2] = (z * n + im(y, n, bc)) * n + x;
  j[3] = (z * n + ip(y, n, bc)) * n + x;
  if constexpr (ND == 3) {
    j[4] = (im(z, n, bc) * n + y) * n + x;
    j[5] = (ip(z, n, bc) * n + y) * n + x;
  }
}

template <int ND>
__device__ __forceinline__ void gs_cell_var(double* p, const double* rhs, const double* e, int x, int y, int z, int n,
                                            int bc, double ih2, double lam) {
  const int i = (z * n + y) * n + x;
  int j[2 * ND];
  nbr_list<ND>(x, y, z, n, bc, j);
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int k = 0; k < 2 * ND; k++)
    if (j[k] != i) {
      const double ef = 0.5 * (e[i] + e[j[k]]);
      num += ef * p[j[k]];
      den += ef;
    }
  p[i] = (num * ih2 - rhs[i]) / (den * ih2 + lam);
}

template <int ND>
__device__ __forceinline__ double resid_var(const double* p, const double* rhs, const double* e, int x, int y, int z,
                                            int n, int bc, double ih2, double lam) {
  const int i = (z * n + y) * n + x;
  int j[2 * ND];
  nbr_list<ND>(x, y, z, n, bc, j);
  double a = 0.0;
#pragma unroll
  for (int k = 0; k < 2 * ND; k++)
    if (j[k] != i) a += 0.5 * (e[i] + e[j[k]]) * (p[j[k]] - p[i]);
  return rhs[i] - (a * ih2 - lam * p[i]);
}

template <int ND>
__device__ __forceinline__ double restrict_cell_var(const double* p, const double* rhs, const double* e, int xc, int yc,
                                                    int zc, int n, int bc, double ih2, double lam) {
  double s = 0.0;
#pragma unroll
  for (int dz = 0; dz < (ND == 3 ? 2 : 1); dz++)
#pragma unroll
    for (int dy = 0; dy < 2; dy++)
#pragma unroll
      for (int dx = 0; dx < 2; dx++)
        s += resid_var<ND>(p, rhs, e, 2 * xc + dx, 2 * yc + dy, 2 * zc + dz, n, bc, ih2, lam);
  return s * (ND == 3 ? 0.125 : 0.25);
}

// bi/trilinear interpolation of the coarse correction at fine cell (x, y, z):
// weight 3/4 on the parent and 1/4 on the parent's neighbour on the side of
// the fine cell, per direction (boundary rule as for the stencil)
template <int ND>
__device__ __forceinline__ double prolong_cell(const double* e, int x, int y, int z, int nc, int bc) {
  const int xc = x >> 1, yc = y >> 1, zc = z >> 1;
  const int xn = (x & 1) ? ip(xc, nc, bc) : im(xc, nc, bc);
  const int yn = (y & 1) ? ip(yc, nc, bc) : im(yc, nc, bc);
  auto plane = [&](int zz) {
    const double a = 0.75 * e[(zz * nc + yc) * nc + xc] + 0.25 * e[(zz * nc + yc) * nc + xn];
    const double b = 0.75 * e[(zz * nc + yn) * nc + xc] + 0.25 * e[(zz * nc + yn) * nc + xn];
    return 0.75 * a + 0.25 * b;
  };
  if constexpr (ND == 2) {
    return plane(0);
  } else {
    const int zn = (z & 1) ? ip(zc, nc, bc) : im(zc, nc, bc);
    return 0.75 * plane(zc) + 0.25 * plane(zn);
  }
}

__device__ __forceinline__ double par_ih2(const MgDev& g, int l) { return g.par[PAR_IH2 + l]; }
__device__ __forceinline__ double par_idiag(const MgDev& g, int f, int l) { return g.par[PAR_IDIAG + f * MG_MAXL + l]; }
__device__ __forceinline__ double par_lam(const MgDev& g, int f) { return g.par[PAR_LAM + f]; }

// ---- level kernels (HBM levels above the tail) ---------------------------

template <int ND, bool VAR>
__global__ void __launch_bounds__(256) k_mg_smooth(MgDev g, int l, int c) {
  const int f = blockIdx.y;
  const int n = g.n[l];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (g.cells[l] >> 1)) return;
  int x, y, z;
  colour_cell<ND>(t, n, g.lg[l], c, x, y, z);
  if constexpr (VAR)
    gs_cell_var<ND>(g.phi[f][l], g.f[f][l], g.eps[l], x, y, z, n, g.bc, par_ih2(g, l), par_lam(g, f));
  else
    gs_cell<ND>(g.phi[f][l], g.f[f][l], x, y, z, n, g.bc, par_ih2(g, l), par_idiag(g, f, l));
}

template <int ND, bool VAR>
__global__ void __launch_bounds__(256) k_mg_restrict(MgDev g, int l) {
  const int f = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.cells[l + 1]) return;
  int x, y, z;
  decode<ND>(t, g.n[l + 1], g.lg[l + 1], x, y, z);
  if constexpr (VAR)
    g.f[f][l + 1][t] = restrict_cell_var<ND>(g.phi[f][l], g.f[f][l], g.eps[l], x, y, z, g.n[l], g.bc, par_ih2(g, l),
                                             par_lam(g, f));
  else
    g.f[f][l + 1][t] =
        restrict_cell<ND>(g.phi[f][l], g.f[f][l], x, y, z, g.n[l], g.bc, par_ih2(g, l), par_lam(g, f));
  g.phi[f][l + 1][t] = 0.0;
}

// coefficient of level l + 1: the mean of the 2^d children
template <int ND>
__global__ void __launch_bounds__(256) k_mg_eps_restrict(MgDev g, int l, double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.cells[l + 1]) return;
  int x, y, z;
  decode<ND>(t, g.n[l + 1], g.lg[l + 1], x, y, z);
  const int n = g.n[l];
  const double* e = g.eps[l];
  double s = 0.0;
  for (int dz = 0; dz < (ND == 3 ? 2 : 1); dz++)
    for (int dy = 0; dy < 2; dy++)
      for (int dx = 0; dx < 2; dx++) s += e[((2 * z + dz) * n + 2 * y + dy) * n + 2 * x + dx];
  out[t] = s * (ND == 3 ? 0.125 : 0.25);
}

template <int ND>
__global__ void __launch_bounds__(256) k_mg_prolong(MgDev g, int l) {
  const int f = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.cells[l]) return;
  int x, y, z;
  decode<ND>(t, g.n[l], g.lg[l], x, y, z);
  g.phi[f][l][t] += prolong_cell<ND>(g.phi[f][l + 1], x, y, z, g.n[l + 1], g.bc);
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// Block maxima of non-negative doubles as bit patterns (NaN sorts above every
// number), written by each block into its own slot of the pinned host buffer
// (the residual maxima of field f in row f, the |f| maxima in row NFMAX + f);
// the host folds the launch's slots once it has completed.  No atomics: many
// blocks folding into one address serialise.
__device__ void fold_norms(const MgDev& g, int f, unsigned long long a, unsigned long long b, int with_f) {
  __shared__ unsigned long long sr[16], sf[16];
  a = wave_max_u64(a);
  b = wave_max_u64(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sr[w] = a;
    sf[w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); i++) {
      a = sr[i] > a ? sr[i] : a;
      b = sf[i] > b ? sf[i] : b;
    }
    g.hpart[(size_t)f * g.maxb + blockIdx.x] = a;
    if (with_f) g.hpart[(size_t)(NFMAX + f) * g.maxb + blockIdx.x] = b;
  }
}

// max |residual| (and with with_f, max |f|) of level 0 per field
template <int ND, bool VAR>
__global__ void __launch_bounds__(256) k_mg_resnorm(MgDev g, int with_f) {
  const int f = blockIdx.y;
  unsigned long long br = 0, bf = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < g.cells[0]; t += gridDim.x * blockDim.x) {
    int x, y, z;
    decode<ND>(t, g.n[0], g.lg[0], x, y, z);
    double r;
    if constexpr (VAR)
      r = resid_var<ND>(g.phi[f][0], g.f[f][0], g.eps[0], x, y, z, g.n[0], g.bc, par_ih2(g, 0), par_lam(g, f));
    else
      r = resid<ND>(g.phi[f][0], g.f[f][0], x, y, z, g.n[0], g.bc, par_ih2(g, 0), par_lam(g, f));
    const unsigned long long a = (unsigned long long)__double_as_longlong(fabs(r));
    const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(g.f[f][0][t]));
    br = a > br ? a : br;
    bf = b > bf ? b : bf;
  }
  fold_norms(g, f, br, bf, with_f);
}


__global__ void k_mg_set(double* dst, MgPar v) {
  const int i = threadIdx.x;
  if (i < PAR_COUNT) dst[i] = v.v[i];
}

// ---- tiled 2D level kernels ---------------------------------------------
// One workgroup per 32x32 tile of a level above the tail: the tile and a halo
// ring of H cells (clipped at Neumann domain faces, wrapped on periodic ones)
// are staged in LDS and the red-black sweeps are repeated over the whole
// staged region; a cell whose neighbours are not all staged (the open edge
// of the halo) is never updated, so after k half-sweeps every cell at least
// k cells from the open edge holds exactly the value the global sweeps give
// it (same neighbours, same arithmetic).  `down` sweeps pre times, forms the
// residual on the tile, restricts it and clears the coarse correction (H =
// 2 pre + 1); `up` adds the interpolated coarse correction over the region,
// sweeps post times (H = 2 post, + 1 when it also folds the residual norm
// of the finest level).  A launch never writes the array it stages from
// (blocks that start late would read a neighbour's new tile): down reads phi
// and writes phi2, up reads phi2 and writes phi.

constexpr int TS = 32;                 // tile side
constexpr int RP = 64;                 // LDS row pitch of a staged region
constexpr int HMAX = 9;                // largest halo: pre, post <= 4
constexpr int RMAX = TS + 2 * HMAX;    // largest staged rows and columns

struct Region {
  int gx0, gy0, w, h;
  bool open[4];  // x-, x+, y-, y+ edges that cut the domain (not a Neumann face)
};

__device__ __forceinline__ Region region2d(int x0, int y0, int n, int H, int bc) {
  Region r;
  if (bc == AMRV_MG_PERIODIC) {
    r.gx0 = x0 - H;
    r.gy0 = y0 - H;
    r.w = r.h = TS + 2 * H;
    r.open[0] = r.open[1] = r.open[2] = r.open[3] = true;
  } else {
    r.gx0 = max(x0 - H, 0);
    r.gy0 = max(y0 - H, 0);
    const int x1 = min(x0 + TS + H, n), y1 = min(y0 + TS + H, n);
    r.w = x1 - r.gx0;
    r.h = y1 - r.gy0;
    r.open[0] = r.gx0 > 0;
    r.open[1] = x1 < n;
    r.open[2] = r.gy0 > 0;
    r.open[3] = y1 < n;
  }
  return r;
}

__device__ __forceinline__ int wrapn(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// The coarse cells a region's interpolation reads: parents (gx >> 1 of the
// unwrapped fine coordinate) and their neighbours, staged with the boundary
// rule applied (wrap, or the mirrored cell at a Neumann face) in an
// EP-pitched LDS block, so each fine cell interpolates from LDS with the
// weights and order of prolong_cell.
constexpr int EP = 32;
constexpr int EMAX = RMAX / 2 + 3;

struct CoarseWin {
  int cx0, cy0;
};

__device__ __forceinline__ CoarseWin stage_coarse(double* E, const Region& r, int nc, const double* e, int bc) {
  CoarseWin c;
  c.cx0 = (r.gx0 >> 1) - 1;
  c.cy0 = (r.gy0 >> 1) - 1;
  const int cw = ((r.gx0 + r.w - 1) >> 1) - c.cx0 + 2, ch = ((r.gy0 + r.h - 1) >> 1) - c.cy0 + 2;
  constexpr int K = (EMAX * EP + 255) / 256;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int i = threadIdx.x + 256 * k;
    const int lx = i & (EP - 1), ly = i >> 5;
    v[k] = 0.0;
    if (lx < cw && ly < ch) {
      int gx = c.cx0 + lx, gy = c.cy0 + ly;
      if (bc == AMRV_MG_PERIODIC) {
        gx = wrapn(gx, nc);
        gy = wrapn(gy, nc);
      } else {
        gx = min(max(gx, 0), nc - 1);
        gy = min(max(gy, 0), nc - 1);
      }
      v[k] = e[gy * nc + gx];
    }
  }
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int i = threadIdx.x + 256 * k;
    const int lx = i & (EP - 1), ly = i >> 5;
    if (lx < cw && ly < ch) E[ly * EP + lx] = v[k];
  }
  return c;
}

// prolong_cell's interpolation at the unwrapped fine cell (ux, uy) from the
// staged coarse block
__device__ __forceinline__ double prolong_lds(const double* E, const CoarseWin& c, int ux, int uy) {
  const int xc = (ux >> 1) - c.cx0, yc = (uy >> 1) - c.cy0;
  const int xn = (ux & 1) ? xc + 1 : xc - 1, yn = (uy & 1) ? yc + 1 : yc - 1;
  const double a = 0.75 * E[yc * EP + xc] + 0.25 * E[yc * EP + xn];
  const double b = 0.75 * E[yn * EP + xc] + 0.25 * E[yn * EP + xn];
  return 0.75 * a + 0.25 * b;
}

// stage phi (+ the interpolated coarse correction when E != null) and f of
// the region into LDS (row pitch RP); every global load is issued before the
// first one is waited for
__device__ __forceinline__ void stage_region(double* P, double* F, const Region& r, int n, const double* phi,
                                             const double* rhs, const double* E, const CoarseWin& cw) {
  constexpr int K = (RMAX * RP + 255) / 256;
  double pv[K], fv[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int i = threadIdx.x + 256 * k;
    const int lx = i & (RP - 1), ly = i >> 6;
    pv[k] = fv[k] = 0.0;
    if (lx < r.w && ly < r.h) {
      const int gx = wrapn(r.gx0 + lx, n), gy = wrapn(r.gy0 + ly, n);
      pv[k] = phi[gy * n + gx];
      fv[k] = rhs[gy * n + gx];
    }
  }
  if (E) {
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int i = threadIdx.x + 256 * k;
      const int lx = i & (RP - 1), ly = i >> 6;
      if (lx < r.w && ly < r.h) pv[k] = pv[k] + prolong_lds(E, cw, r.gx0 + lx, r.gy0 + ly);
    }
  }
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int i = threadIdx.x + 256 * k;
    const int lx = i & (RP - 1), ly = i >> 6;
    if (lx < r.w && ly < r.h) {
      P[i] = pv[k];
      F[i] = fv[k];
    }
  }
}

// one half-sweep of colour c over the staged region: 32 lanes per row take
// the row's cells of that colour; every new value is computed before any is
// stored (a half-sweep reads only the other colour, so no barrier is needed
// between the two passes).  A cell with a neighbour beyond an open edge is
// left alone.
__device__ __forceinline__ void tile_halfsweep(double* P, const double* F, const Region& r, int c, double ih2,
                                               double idiag) {
  constexpr int K = (RMAX + 7) / 8;
  const int j = threadIdx.x & 31, r0 = threadIdx.x >> 5;
  double nv[K];
  bool ok[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int ly = r0 + 8 * k;
    const int lx = 2 * j + ((c + r.gx0 + r.gy0 + ly) & 1);
    const int i = ly * RP + lx;
    ok[k] = ly < r.h && lx < r.w && !(lx == 0 && r.open[0]) && !(lx == r.w - 1 && r.open[1]) &&
            !(ly == 0 && r.open[2]) && !(ly == r.h - 1 && r.open[3]);
    nv[k] = 0.0;
    if (ok[k]) {
      const int xm = lx == 0 ? i : i - 1, xp = lx == r.w - 1 ? i : i + 1;
      const int ym = ly == 0 ? i : i - RP, yp = ly == r.h - 1 ? i : i + RP;
      const double sum = (P[xm] + P[xp]) + (P[ym] + P[yp]);
      nv[k] = (sum * ih2 - F[i]) * idiag;
    }
  }
#pragma unroll
  for (int k = 0; k < K; k++) {
    const int ly = r0 + 8 * k;
    const int lx = 2 * j + ((c + r.gx0 + r.gy0 + ly) & 1);
    if (ok[k]) P[ly * RP + lx] = nv[k];
  }
}

// residual at a staged cell whose neighbours are all staged
__device__ __forceinline__ double tile_resid(const double* P, const double* F, const Region& r, int lx, int ly,
                                             double ih2, double lam) {
  const int i = ly * RP + lx;
  const int xm = lx == 0 ? i : i - 1, xp = lx == r.w - 1 ? i : i + 1;
  const int ym = ly == 0 ? i : i - RP, yp = ly == r.h - 1 ? i : i + RP;
  const double w = P[i];
  double lap = ((P[xm] + P[xp]) - 2.0 * w) * ih2;
  lap = lap + ((P[ym] + P[yp]) - 2.0 * w) * ih2;
  return F[i] - (lap - lam * w);
}

__global__ void __launch_bounds__(256) k_mg_down2d(MgDev g, int l, int pre) {
  __shared__ double P[RMAX * RP], F[RMAX * RP];
  const int f = blockIdx.y, n = g.n[l], nt = n / TS;
  const int x0 = (blockIdx.x % nt) * TS, y0 = (blockIdx.x / nt) * TS;
  const Region r = region2d(x0, y0, n, 2 * pre + 1, g.bc);
  stage_region(P, F, r, n, g.phi[f][l], g.f[f][l], nullptr, CoarseWin{0, 0});
  __syncthreads();
  const double ih2 = par_ih2(g, l), idg = par_idiag(g, f, l), lam = par_lam(g, f);
  for (int s = 0; s < pre; s++)
    for (int c = 0; c < 2; c++) {
      tile_halfsweep(P, F, r, c, ih2, idg);
      __syncthreads();
    }
  {
    const int cx = threadIdx.x & (TS / 2 - 1), cy = threadIdx.x >> 4;
    const int bx = x0 - r.gx0 + 2 * cx, by = y0 - r.gy0 + 2 * cy;
    double sum = 0.0;
#pragma unroll
    for (int dy = 0; dy < 2; dy++)
#pragma unroll
      for (int dx = 0; dx < 2; dx++) sum += tile_resid(P, F, r, bx + dx, by + dy, ih2, lam);
    const int nc = n >> 1;
    const int ci = (y0 / 2 + cy) * nc + (x0 / 2 + cx);
    g.f[f][l + 1][ci] = sum * 0.25;
    g.phi[f][l + 1][ci] = 0.0;
  }
  double* out = g.phi2[f][l];  // other blocks of this launch still stage phi
#pragma unroll
  for (int k = 0; k < TS * TS / 256; k++) {
    const int tx = threadIdx.x & (TS - 1), ty = (threadIdx.x >> 5) + 8 * k;
    out[(y0 + ty) * n + x0 + tx] = P[(y0 + ty - r.gy0) * RP + (x0 + tx - r.gx0)];
  }
}

__global__ void __launch_bounds__(256) k_mg_up2d(MgDev g, int l, int post, int norm) {
  __shared__ double P[RMAX * RP], F[RMAX * RP], E[EMAX * EP];
  const int f = blockIdx.y, n = g.n[l], nt = n / TS;
  const int x0 = (blockIdx.x % nt) * TS, y0 = (blockIdx.x / nt) * TS;
  const Region r = region2d(x0, y0, n, 2 * post + (norm ? 1 : 0), g.bc);
  const CoarseWin cw = stage_coarse(E, r, n >> 1, g.phi[f][l + 1], g.bc);
  __syncthreads();
  stage_region(P, F, r, n, g.phi2[f][l], g.f[f][l], E, cw);
  __syncthreads();
  const double ih2 = par_ih2(g, l), idg = par_idiag(g, f, l), lam = par_lam(g, f);
  for (int s = 0; s < post; s++)
    for (int c = 0; c < 2; c++) {
      tile_halfsweep(P, F, r, c, ih2, idg);
      __syncthreads();
    }
  double* out = g.phi[f][l];
  unsigned long long br = 0;
#pragma unroll
  for (int k = 0; k < TS * TS / 256; k++) {
    const int tx = threadIdx.x & (TS - 1), ty = (threadIdx.x >> 5) + 8 * k;
    const int lx = x0 + tx - r.gx0, ly = y0 + ty - r.gy0;
    out[(y0 + ty) * n + x0 + tx] = P[ly * RP + lx];
    if (norm) {
      const unsigned long long a =
          (unsigned long long)__double_as_longlong(fabs(tile_resid(P, F, r, lx, ly, ih2, lam)));
      br = a > br ? a : br;
    }
  }
  if (norm) fold_norms(g, f, br, 0ull, 0);
}

// ---- the coarse tail: every level from `top` down, one workgroup per field,
// all levels in LDS -------------------------------------------------------

template <int ND>
__device__ void tail_sweeps(const MgDev& g, double* P, const double* F, int l, int sweeps, double ih2, double idg) {
  const int n = g.n[l], lg = g.lg[l], half = g.cells[l] >> 1;
  for (int s = 0; s < sweeps; s++)
    for (int c = 0; c < 2; c++) {
      // TK cells per thread per pass: every new value before any store
      for (int t0 = threadIdx.x; t0 < half; t0 += TK * blockDim.x) {
        double nv[TK];
        int idx[TK];
#pragma unroll
        for (int k = 0; k < TK; k++) {
          const int t = t0 + k * blockDim.x;
          idx[k] = -1;
          if (t < half) {
            int x, y, z;
            colour_cell<ND>(t, n, lg, c, x, y, z);
            const int row = (z * n + y) * n;
            double sum = (P[row + im(x, n, g.bc)] + P[row + ip(x, n, g.bc)]) +
                         (P[(z * n + im(y, n, g.bc)) * n + x] + P[(z * n + ip(y, n, g.bc)) * n + x]);
            if constexpr (ND == 3)
              sum = sum + (P[(im(z, n, g.bc) * n + y) * n + x] + P[(ip(z, n, g.bc) * n + y) * n + x]);
            idx[k] = row + x;
            nv[k] = (sum * ih2 - F[row + x]) * idg;
          }
        }
#pragma unroll
        for (int k = 0; k < TK; k++)
          if (idx[k] >= 0) P[idx[k]] = nv[k];
      }
      __syncthreads();
    }
}

// exact solve on the coarsest grid (2 cells per side): per direction the
// operator couples the two cells as c [[-1, 1], [1, -1]] (c = 1/h^2 with the
// mirrored Neumann ghost, 2/h^2 with the periodic wrap), so the 2^d Walsh
// patterns (-1)^popcount(k & cell) are its eigenvectors, with eigenvalue
// -2c per set bit of k, minus lambda.  For lambda = 0 the constant pattern
// has eigenvalue 0 and the correction gets no constant part.
template <int ND>
__device__ void coarse_exact(const MgDev& g, double* P, const double* F, double ih2, double lam) {
  constexpr int C = 1 << ND;
  if (threadIdx.x == 0) {
    const double c2 = 2.0 * (g.bc == AMRV_MG_PERIODIC ? 2.0 : 1.0) * ih2;
    double hat[C];
#pragma unroll
    for (int k = 0; k < C; k++) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < C; c++) s += (__popc(k & c) & 1) ? -F[c] : F[c];
      double mu = -lam;
#pragma unroll
      for (int d = 0; d < ND; d++)
        if ((k >> d) & 1) mu -= c2;
      hat[k] = mu == 0.0 ? 0.0 : s / (mu * C);
    }
#pragma unroll
    for (int c = 0; c < C; c++) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < C; k++) s += (__popc(k & c) & 1) ? -hat[k] : hat[k];
      P[c] = s;
    }
  }
  __syncthreads();
}

template <int ND>
__device__ void tail_sweeps_var(const MgDev& g, double* P, const double* F, const double* E, int l, int sweeps,
                                double ih2, double lam) {
  const int n = g.n[l], lg = g.lg[l], half = g.cells[l] >> 1;
  for (int s = 0; s < sweeps; s++)
    for (int c = 0; c < 2; c++) {
      for (int t = threadIdx.x; t < half; t += blockDim.x) {
        int x, y, z;
        colour_cell<ND>(t, n, lg, c, x, y, z);
        gs_cell_var<ND>(P, F, E, x, y, z, n, g.bc, ih2, lam);
      }
      __syncthreads();
    }
}

// exact solve on the 2-per-side grid with a coefficient: the 2^d x 2^d
// system of the operator, strictly diagonally dominant (lambda > 0), by
// Gaussian elimination without pivoting in one thread
template <int ND>
__device__ void coarse_exact_var(const MgDev& g, double* P, const double* F, const double* E, double ih2, double lam) {
  constexpr int C = 1 << ND;
  if (threadIdx.x == 0) {
    double A[C][C + 1];
    for (int r = 0; r < C; r++) {
      for (int c = 0; c <= C; c++) A[r][c] = 0.0;
      const int x = r & 1, y = (r >> 1) & 1, z = ND == 3 ? (r >> 2) & 1 : 0;
      int j[2 * ND];
      nbr_list<ND>(x, y, z, 2, g.bc, j);
      double diag = -lam;
      for (int k = 0; k < 2 * ND; k++)
        if (j[k] != r) {
          const double ef = 0.5 * (E[r] + E[j[k]]) * ih2;
          A[r][j[k]] += ef;
          diag -= ef;
        }
      A[r][r] += diag;
      A[r][C] = F[r];
    }
    for (int k = 0; k < C; k++)
      for (int r = k + 1; r < C; r++) {
        const double m = A[r][k] / A[k][k];
        for (int c = k; c <= C; c++) A[r][c] -= m * A[k][c];
      }
    for (int r = C - 1; r >= 0; r--) {
      double s = A[r][C];
      for (int c = r + 1; c < C; c++) s -= A[r][c] * P[c];
      P[r] = s / A[r][r];
    }
  }
  __syncthreads();
}

template <int ND, bool VAR>
__global__ void __launch_bounds__(TAIL_THREADS) k_mg_tail(MgDev g, int top, int pre, int post) {
  extern __shared__ double lds[];
  __shared__ double s_ih2[MG_MAXL], s_idg[MG_MAXL];
  const int f = blockIdx.x;
  if (threadIdx.x < MG_MAXL) {
    s_ih2[threadIdx.x] = par_ih2(g, threadIdx.x);
    s_idg[threadIdx.x] = par_idiag(g, f, threadIdx.x);
  }
  const double lam = par_lam(g, f);
  auto P = [&](int l) { return lds + (VAR ? g.loffv[l] : g.loff[l]); };
  auto F = [&](int l) { return P(l) + g.cells[l]; };
  auto E = [&](int l) { return P(l) + 2 * g.cells[l]; };  // with a coefficient only
  const int last = g.nlev - 1;
  for (int i = threadIdx.x; i < g.cells[top]; i += blockDim.x) {
    P(top)[i] = g.phi[f][top][i];
    F(top)[i] = g.f[f][top][i];
  }
  if constexpr (VAR)
    for (int l = top; l <= last; l++)
      for (int i = threadIdx.x; i < g.cells[l]; i += blockDim.x) E(l)[i] = g.eps[l][i];
  __syncthreads();
  for (int l = top; l < last; l++) {
    if constexpr (VAR)
      tail_sweeps_var<ND>(g, P(l), F(l), E(l), l, pre, s_ih2[l], lam);
    else
      tail_sweeps<ND>(g, P(l), F(l), l, pre, s_ih2[l], s_idg[l]);
    const double ih2 = s_ih2[l];
    for (int t = threadIdx.x; t < g.cells[l + 1]; t += blockDim.x) {
      int x, y, z;
      decode<ND>(t, g.n[l + 1], g.lg[l + 1], x, y, z);
      if constexpr (VAR)
        F(l + 1)[t] = restrict_cell_var<ND>(P(l), F(l), E(l), x, y, z, g.n[l], g.bc, ih2, lam);
      else
        F(l + 1)[t] = restrict_cell<ND>(P(l), F(l), x, y, z, g.n[l], g.bc, ih2, lam);
      P(l + 1)[t] = 0.0;
    }
    __syncthreads();
  }
  if constexpr (VAR)
    coarse_exact_var<ND>(g, P(last), F(last), E(last), s_ih2[last], lam);
  else
    coarse_exact<ND>(g, P(last), F(last), s_ih2[last], lam);
  for (int l = last - 1; l >= top; l--) {
    for (int t = threadIdx.x; t < g.cells[l]; t += blockDim.x) {
      int x, y, z;
      decode<ND>(t, g.n[l], g.lg[l], x, y, z);
      P(l)[t] += prolong_cell<ND>(P(l + 1), x, y, z, g.n[l + 1], g.bc);
    }
    __syncthreads();
    if constexpr (VAR)
      tail_sweeps_var<ND>(g, P(l), F(l), E(l), l, post, s_ih2[l], lam);
    else
      tail_sweeps<ND>(g, P(l), F(l), l, post, s_ih2[l], s_idg[l]);
  }
  for (int i = threadIdx.x; i < g.cells[top]; i += blockDim.x) g.phi[f][top][i] = P(top)[i];
}

// ---- divergence control of the MHD runs (Sec. 2.4): lap(phi) = div B*,
// B = B* - grad phi, central differences (w(+1) - w(-1)) * (n / 2L) ---------

template <int ND>
__device__ __forceinline__ double cdiff(const double* w, int x, int y, int z, int n, int bc, int d, double c) {
  if (d == 0) return (w[(z * n + y) * n + ip(x, n, bc)] - w[(z * n + y) * n + im(x, n, bc)]) * c;
  if (d == 1) return (w[(z * n + ip(y, n, bc)) * n + x] - w[(z * n + im(y, n, bc)) * n + x]) * c;
  return (w[(ip(z, n, bc) * n + y) * n + x] - w[(im(z, n, bc) * n + y) * n + x]) * c;
}

template <int ND>
__device__ __forceinline__ double cdiv(const double* b0, const double* b1, const double* b2, int x, int y, int z,
                                       int n, int bc, double c) {
  double d = cdiff<ND>(b0, x, y, z, n, bc, 0, c);
  d = d + cdiff<ND>(b1, x, y, z, n, bc, 1, c);
  if constexpr (ND == 3) d = d + cdiff<ND>(b2, x, y, z, n, bc, 2, c);
  return d;
}

// right-hand side div B*, initial guess 0
template <int ND>
__global__ void __launch_bounds__(256) k_mg_divb(MgDev g, const double* b0, const double* b1, const double* b2,
                                                 double c) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.cells[0]) return;
  int x, y, z;
  decode<ND>(t, g.n[0], g.lg[0], x, y, z);
  g.f[0][0][t] = cdiv<ND>(b0, b1, b2, x, y, z, g.n[0], g.bc, c);
  g.phi[0][0][t] = 0.0;
}

template <int ND>
__global__ void __launch_bounds__(256) k_mg_gradsub(MgDev g, double* b0, double* b1, double* b2, double c) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.cells[0]) return;
  int x, y, z;
  decode<ND>(t, g.n[0], g.lg[0], x, y, z);
  const double* phi = g.phi[0][0];
  b0[t] = b0[t] - cdiff<ND>(phi, x, y, z, g.n[0], g.bc, 0, c);
  b1[t] = b1[t] - cdiff<ND>(phi, x, y, z, g.n[0], g.bc, 1, c);
  if constexpr (ND == 3) b2[t] = b2[t] - cdiff<ND>(phi, x, y, z, g.n[0], g.bc, 2, c);
}

// max |div B| into the host slots of row 0
template <int ND>
__global__ void __launch_bounds__(256) k_mg_divnorm(MgDev g, const double* b0, const double* b1, const double* b2,
                                                    double c) {
  unsigned long long m = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < g.cells[0]; t += gridDim.x * blockDim.x) {
    int x, y, z;
    decode<ND>(t, g.n[0], g.lg[0], x, y, z);
    const unsigned long long a =
        (unsigned long long)__double_as_longlong(fabs(cdiv<ND>(b0, b1, b2, x, y, z, g.n[0], g.bc, c)));
    m = a > m ? a : m;
  }
  fold_norms(g, 0, m, 0ull, 0);
}

// ---- reaction-diffusion (Sec. 2.5) ---------------------------------------

__device__ __forceinline__ void react(const RdK& p, double u, double v, double& ru, double& rv) {
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

// out = base + c F(src), F = F0 + D lap (explicit Euler and midpoint stages)
template <int ND>
__global__ void __launch_bounds__(256) k_rd_explicit(MgDev g, RdK p, const double* bu, const double* bv,
                                                     const double* su, const double* sv, double* ou, double* ov,
                                                     double c) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.cells[0]) return;
  int x, y, z;
  decode<ND>(t, g.n[0], g.lg[0], x, y, z);
  const double ih2 = par_ih2(g, 0);
  double ru, rv;
  react(p, su[t], sv[t], ru, rv);
  const double fu = ru + p.Du * lap_at<ND>(su, x, y, z, g.n[0], g.bc, ih2);
  const double fv = rv + p.Dv * lap_at<ND>(sv, x, y, z, g.n[0], g.bc, ih2);
  ou[t] = bu[t] + c * fu;
  ov[t] = bv[t] + c * fv;
}

// split scheme: f = -lambda (w + dt F0(w)), initial guess w
template <int ND>
__global__ void __launch_bounds__(256) k_rd_split_rhs(MgDev g, RdK p, const double* u, const double* v, double dt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.cells[0]) return;
  double ru, rv;
  react(p, u[t], v[t], ru, rv);
  g.f[0][0][t] = -par_lam(g, 0) * (u[t] + dt * ru);
  g.f[1][0][t] = -par_lam(g, 1) * (v[t] + dt * rv);
  g.phi[0][0][t] = u[t];
  g.phi[1][0][t] = v[t];
}

// IMEX first stage: f = -lambda ((w + dt F0(w)) + (dt/2) D lap(w)), initial
// guess the explicit Euler predictor w + dt F(w); F(w) kept for the second
// stage
template <int ND>
__global__ void __launch_bounds__(256) k_rd_imex_rhs(MgDev g, RdK p, const double* u, const double* v, double* Eu,
                                                     double* Ev, double dt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.cells[0]) return;
  int x, y, z;
  decode<ND>(t, g.n[0], g.lg[0], x, y, z);
  const double ih2 = par_ih2(g, 0);
  double ru, rv;
  react(p, u[t], v[t], ru, rv);
  const double du = p.Du * lap_at<ND>(u, x, y, z, g.n[0], g.bc, ih2);
  const double dv = p.Dv * lap_at<ND>(v, x, y, z, g.n[0], g.bc, ih2);
  Eu[t] = ru + du;
  Ev[t] = rv + dv;
  const double hdt = 0.5 * dt;
  g.f[0][0][t] = -par_lam(g, 0) * ((u[t] + dt * ru) + hdt * du);
  g.f[1][0][t] = -par_lam(g, 1) * ((v[t] + dt * rv) + hdt * dv);
  g.phi[0][0][t] = u[t] + dt * (ru + du);
  g.phi[1][0][t] = v[t] + dt * (rv + dv);
}

// IMEX second stage: w1 = w + (dt/2) (F(w) + F(w*)), w* = the solve's phi
template <int ND>
__global__ void __launch_bounds__(256) k_rd_imex_final(MgDev g, RdK p, double* u, double* v, const double* Eu,
                                                       const double* Ev, double dt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.cells[0]) return;
  int x, y, z;
  decode<ND>(t, g.n[0], g.lg[0], x, y, z);
  const double ih2 = par_ih2(g, 0);
  const double* su = g.phi[0][0];
  const double* sv = g.phi[1][0];
  double ru, rv;
  react(p, su[t], sv[t], ru, rv);
  const double fu = ru + p.Du * lap_at<ND>(su, x, y, z, g.n[0], g.bc, ih2);
  const double fv = rv + p.Dv * lap_at<ND>(sv, x, y, z, g.n[0], g.bc, ih2);
  const double hdt = 0.5 * dt;
  u[t] = u[t] + hdt * (Eu[t] + fu);
  v[t] = v[t] + hdt * (Ev[t] + fv);
}

int blocks_of(int n) { return (n + 255) / 256; }

}  // namespace

struct amrv_mg {
  amrv_mg_config cfg{};
  MgDev g{};
  hipStream_t st = nullptr;
  double* par = nullptr;
  unsigned long long* hpart = nullptr;  // pinned slots of per-block maxima
  int nb_cycle = 0, nb_init = 0;        // blocks folding norms: a V-cycle's last launch, the initial norms
  double* tmp[4] = {nullptr, nullptr, nullptr, nullptr};
  int tail = 0;
  size_t tail_lds = 0;
  hipGraphExec_t gexec = nullptr;
  bool profile = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double prof_ms = 0.0;
  int64_t prof_cycles = 0;
  int last_cycles = 0;  // V-cycles of the last reaction-diffusion solve
  bool var = false;     // a cell coefficient is set (div(eps grad phi) - lambda phi)
  size_t tail_lds_var = 0;
  int par_nf = 0;         // fields of the last parameter block set (0: none yet)
  double par_lam0 = 0.0;  // its field-0 lambda
  double* eps[MG_MAXL] = {};
};

namespace {

using amrv::set_error;

int hip_err(hipError_t e, const char* where) {
  return set_error(AMRV_EDEVICE, (std::string(where) + ": " + hipGetErrorString(e)).c_str());
}

#define MGCHK(expr)                                \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_err(e_, #expr); \
  } while (0)

constexpr size_t ALIGN = 256;
size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

int validate(const amrv_mg_config* c) {
  if (!c) return set_error(AMRV_EINVAL, "null config");
  if (c->ndim != 2 && c->ndim != 3) return set_error(AMRV_EINVAL, "ndim must be 2 or 3");
  const int nmax = c->ndim == 2 ? 8192 : 512;
  if (!is_pow2(c->n) || c->n < 4 || c->n > nmax)
    return set_error(AMRV_EINVAL, "n must be a power of two in 4..8192 (2D) or 4..512 (3D)");
  if (c->bc != AMRV_MG_PERIODIC && c->bc != AMRV_MG_NEUMANN) return set_error(AMRV_EINVAL, "unknown boundary");
  if (c->nfields < 1 || c->nfields > NFMAX) return set_error(AMRV_EINVAL, "nfields must be 1 or 2");
  if (c->pre_sweeps < 1 || c->pre_sweeps > 8 || c->post_sweeps < 1 || c->post_sweeps > 8)
    return set_error(AMRV_EINVAL, "pre and post sweeps must be in 1..8");
  if (c->smoother != AMRV_MG_TILED && c->smoother != AMRV_MG_PER_COLOUR) return set_error(AMRV_EINVAL, "unknown smoother");
  if (!(c->length > 0.0) || !std::isfinite(c->length)) return set_error(AMRV_EINVAL, "length must be positive");
  return 0;
}

struct MgLayout {
  int nlev = 0;
  size_t off_phi[NFMAX][MG_MAXL]{}, off_f[NFMAX][MG_MAXL]{}, off_phi2[NFMAX][MG_MAXL]{}, off_eps[MG_MAXL]{},
      off_tmp[4]{}, off_par = 0, total = 0;
};

MgLayout layout(const amrv_mg_config* c) {
  MgLayout L;
  int lv = 0;
  for (int n = c->n; n >= 2; n >>= 1) lv++;
  L.nlev = lv;
  size_t o = 0;
  for (int f = 0; f < c->nfields; f++)
    for (int l = 0; l < lv; l++) {
      size_t cells = 1;
      for (int d = 0; d < c->ndim; d++) cells *= (size_t)(c->n >> l);
      L.off_phi[f][l] = o;
      o += up(cells * 8);
      L.off_f[f][l] = o;
      o += up(cells * 8);
      if (c->ndim == 2 && cells > (size_t)TAIL_CELLS) {
        L.off_phi2[f][l] = o;
        o += up(cells * 8);
      }
    }
  for (int l = 0; l < lv; l++) {
    size_t cells = 1;
    for (int d = 0; d < c->ndim; d++) cells *= (size_t)(c->n >> l);
    L.off_eps[l] = o;
    o += up(cells * 8);
  }
  size_t c0 = 1;
  for (int d = 0; d < c->ndim; d++) c0 *= (size_t)c->n;
  for (int i = 0; i < 4; i++) {
    L.off_tmp[i] = o;
    o += up(c0 * 8);
  }
  L.off_par = o;
  o += up(PAR_COUNT * 8);
  L.total = o;
  return L;
}

bool tiled(const amrv_mg* m) {
  return !m->var && m->g.nd == 2 && m->cfg.smoother == AMRV_MG_TILED && m->tail > 0 &&
         2 * std::max(m->cfg.pre_sweeps, m->cfg.post_sweeps) + 1 <= HMAX;
}

// residual norms of level 0 (with_f: also max |f|), published to the pinned
// host copy by the launch's last block
template <int ND>
void enqueue_norms_nd(amrv_mg* m, int with_f) {
  const MgDev& g = m->g;
  if (m->var)
    hipLaunchKernelGGL((k_mg_resnorm<ND, true>), dim3(m->nb_init, g.nf), dim3(256), 0, m->st, g, with_f);
  else
    hipLaunchKernelGGL((k_mg_resnorm<ND, false>), dim3(m->nb_init, g.nf), dim3(256), 0, m->st, g, with_f);
}

// one V-cycle, ending with the residual norms of its result
template <int ND>
void enqueue_vcycle_nd(amrv_mg* m) {
  const MgDev& g = m->g;
  const int nf = g.nf;
  const int pre = m->cfg.pre_sweeps, post = m->cfg.post_sweeps;
  if (tiled(m)) {
    for (int l = 0; l < m->tail; l++)
      hipLaunchKernelGGL(k_mg_down2d, dim3((g.n[l] / TS) * (g.n[l] / TS), nf), dim3(256), 0, m->st, g, l, pre);
  } else {
    for (int l = 0; l < m->tail; l++) {
      for (int s = 0; s < pre; s++)
        for (int c = 0; c < 2; c++)
          if (m->var)
            hipLaunchKernelGGL((k_mg_smooth<ND, true>), dim3(blocks_of(g.cells[l] >> 1), nf), dim3(256), 0, m->st, g,
                               l, c);
          else
            hipLaunchKernelGGL((k_mg_smooth<ND, false>), dim3(blocks_of(g.cells[l] >> 1), nf), dim3(256), 0, m->st,
                               g, l, c);
      if (m->var)
        hipLaunchKernelGGL((k_mg_restrict<ND, true>), dim3(blocks_of(g.cells[l + 1]), nf), dim3(256), 0, m->st, g, l);
      else
        hipLaunchKernelGGL((k_mg_restrict<ND, false>), dim3(blocks_of(g.cells[l + 1]), nf), dim3(256), 0, m->st, g,
                           l);
    }
  }
  if (m->var)
    hipLaunchKernelGGL((k_mg_tail<ND, true>), dim3(nf), dim3(TAIL_THREADS), m->tail_lds_var, m->st, g, m->tail, pre,
                       post);
  else
    hipLaunchKernelGGL((k_mg_tail<ND, false>), dim3(nf), dim3(TAIL_THREADS), m->tail_lds, m->st, g, m->tail, pre,
                       post);
  if (tiled(m)) {
    for (int l = m->tail - 1; l >= 0; l--)
      hipLaunchKernelGGL(k_mg_up2d, dim3((g.n[l] / TS) * (g.n[l] / TS), nf), dim3(256), 0, m->st, g, l, post,
                         l == 0 ? 1 : 0);
    return;  // the finest level's up launch folded the norms
  }
  for (int l = m->tail - 1; l >= 0; l--) {
    hipLaunchKernelGGL(k_mg_prolong<ND>, dim3(blocks_of(g.cells[l]), nf), dim3(256), 0, m->st, g, l);
    for (int s = 0; s < post; s++)
      for (int c = 0; c < 2; c++)
        if (m->var)
          hipLaunchKernelGGL((k_mg_smooth<ND, true>), dim3(blocks_of(g.cells[l] >> 1), nf), dim3(256), 0, m->st, g,
                             l, c);
        else
          hipLaunchKernelGGL((k_mg_smooth<ND, false>), dim3(blocks_of(g.cells[l] >> 1), nf), dim3(256), 0, m->st, g,
                             l, c);
  }
  enqueue_norms_nd<ND>(m, 0);
}

void enqueue_vcycle(amrv_mg* m) {
  if (m->g.nd == 2)
    enqueue_vcycle_nd<2>(m);
  else
    enqueue_vcycle_nd<3>(m);
}

int set_params(amrv_mg* m, const double* lam) {
  MgPar P{};
  const double L = m->cfg.length;
  for (int l = 0; l < m->g.nlev; l++) {
    const double r = m->g.n[l] / L;
    P.v[PAR_IH2 + l] = r * r;
  }
  for (int f = 0; f < m->g.nf; f++) {
    P.v[PAR_LAM + f] = lam[f];
    for (int l = 0; l < m->g.nlev; l++)
      P.v[PAR_IDIAG + f * MG_MAXL + l] = 1.0 / (2.0 * m->g.nd * P.v[PAR_IH2 + l] + lam[f]);
  }
  hipLaunchKernelGGL(k_mg_set, dim3(1), dim3(64), 0, m->st, m->par, P);
  MGCHK(hipGetLastError());
  m->par_nf = m->g.nf;
  m->par_lam0 = lam[0];
  return 0;
}

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, 8);
  return d;
}

int launch_cycle(amrv_mg* m) {
  if (m->cfg.use_graph) {
    if (!m->gexec) {
      hipGraph_t gr;
      MGCHK(hipStreamBeginCapture(m->st, hipStreamCaptureModeThreadLocal));
      enqueue_vcycle(m);
      MGCHK(hipStreamEndCapture(m->st, &gr));
      hipError_t e = hipGraphInstantiate(&m->gexec, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      MGCHK(e);
    }
    MGCHK(hipGraphLaunch(m->gexec, m->st));
  } else {
    enqueue_vcycle(m);
    MGCHK(hipGetLastError());
  }
  return 0;
}

// the V-cycle loop on level-0 buffers already filled: `unchecked` cycles
// are enqueued behind the initial norms before the host first waits (each
// host check is a synchronisation), then the residual is checked after every
// cycle.  Returns 0, or AMRV_ENOTCONVERGED / AMRV_ENONPHYSICAL.
int run_cycles(amrv_mg* m, double tol, int max_cycles, int unchecked, int* cycles, double* res_out,
               double* f_out) {
  const int nf = m->g.nf;
  if (m->profile) unchecked = 0;  // profiling times each cycle on its own
  unchecked = std::max(0, std::min(unchecked, max_cycles));
  // the norms of the initial guess (max |f| is taken from these)
  if (m->g.nd == 2)
    enqueue_norms_nd<2>(m, 1);
  else
    enqueue_norms_nd<3>(m, 1);
  MGCHK(hipGetLastError());
  for (int i = 0; i < unchecked; i++)
    if (int rc = launch_cycle(m)) return rc;
  MGCHK(hipStreamSynchronize(m->st));
  double fmax[NFMAX] = {0, 0}, res[NFMAX] = {0, 0};
  auto fold = [&](int row, int nb) {
    unsigned long long v = 0;
    const unsigned long long* p = m->hpart + (size_t)row * m->g.maxb;
    for (int b = 0; b < nb; b++) v = p[b] > v ? p[b] : v;
    return bits_to_double(v);
  };
  for (int f = 0; f < nf; f++) fmax[f] = fold(NFMAX + f, m->nb_init);
  int nb = unchecked ? m->nb_cycle : m->nb_init;
  auto done = [&]() {
    bool ok = true;
    for (int f = 0; f < nf; f++) {
      res[f] = fold(f, nb);
      ok = ok && (res[f] <= tol * fmax[f]);
    }
    return ok;
  };
  int c = unchecked;
  bool ok = done();
  for (int f = 0; f < nf; f++)
    if (std::isnan(res[f]) || std::isnan(fmax[f])) {
      if (cycles) *cycles = c;
      return set_error(AMRV_ENONPHYSICAL, "NaN in the multigrid right-hand side, initial guess or residual");
    }
  while (!ok && c < max_cycles) {
    if (m->profile) MGCHK(hipEventRecord(m->e0, m->st));
    if (int rc = launch_cycle(m)) return rc;
    if (m->profile) MGCHK(hipEventRecord(m->e1, m->st));
    MGCHK(hipStreamSynchronize(m->st));
    if (m->profile) {
      float ms = 0.0f;
      MGCHK(hipEventElapsedTime(&ms, m->e0, m->e1));
      m->prof_ms += ms;
      m->prof_cycles++;
    }
    c++;
    nb = m->nb_cycle;
    ok = done();
    for (int f = 0; f < nf; f++)
      if (std::isnan(res[f])) {
        if (cycles) *cycles = c;
        return set_error(AMRV_ENONPHYSICAL, "NaN in the multigrid residual");
      }
  }
  if (cycles) *cycles = c;
  for (int f = 0; f < nf; f++) {
    if (res_out) res_out[f] = res[f];
    if (f_out) f_out[f] = fmax[f];
  }
  if (!ok) return set_error(AMRV_ENOTCONVERGED, "multigrid residual above tol after max_cycles V-cycles");
  return 0;
}

}  // namespace

namespace amrv {

int mg_correction_grids(amrv_mg* m, double** f, double** e) {
  if (!m || !f || !e) return set_error(AMRV_EINVAL, "null argument");
  *f = m->g.f[0][0];
  *e = m->g.phi[0][0];
  return 0;
}

int mg_enqueue_correction(amrv_mg* m, const double* f, double* out, double lambda, int cycles, bool e_zeroed) {
  if (!m || !f || !out) return set_error(AMRV_EINVAL, "null argument");
  if (m->g.nf != 1 || m->var) return set_error(AMRV_EINVAL, "a correction solve needs one field and the constant coefficient");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return set_error(AMRV_EINVAL, "lambda must be non-negative and finite");
  if (m->par_nf != 1 || m->par_lam0 != lambda)
    if (int rc = set_params(m, &lambda)) return rc;
  const size_t bytes = (size_t)m->g.cells[0] * sizeof(double);
  if (f != m->g.f[0][0]) MGCHK(hipMemcpyAsync(m->g.f[0][0], f, bytes, hipMemcpyDeviceToDevice, m->st));
  if (!e_zeroed) MGCHK(hipMemsetAsync(m->g.phi[0][0], 0, bytes, m->st));
  for (int c = 0; c < cycles; c++)
    if (int rc = launch_cycle(m)) return rc;
  if (out != m->g.phi[0][0]) MGCHK(hipMemcpyAsync(out, m->g.phi[0][0], bytes, hipMemcpyDeviceToDevice, m->st));
  return 0;
}

}  // namespace amrv

extern "C" {

size_t amrv_mg_workspace_bytes(const amrv_mg_config* cfg) {
  if (validate(cfg)) return 0;
  return layout(cfg).total;
}

int amrv_mg_create(const amrv_mg_config* cfg, void* workspace, size_t bytes, void* stream, amrv_mg** out) {
  if (!out) return set_error(AMRV_EINVAL, "null argument");
  *out = nullptr;
  if (int rc = validate(cfg)) return rc;
  if (!workspace) return set_error(AMRV_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % ALIGN) return set_error(AMRV_EINVAL, "workspace must be 256-byte aligned");
  const MgLayout L = layout(cfg);
  if (bytes < L.total) return set_error(AMRV_ENOMEM, ("workspace too small: need " + std::to_string(L.total)).c_str());
  if (cfg->use_graph && !stream) return set_error(AMRV_EINVAL, "graph replay needs a stream other than the null stream");
  amrv_mg* m = new amrv_mg;
  m->cfg = *cfg;
  m->st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(workspace);
  MgDev& g = m->g;
  g.nd = cfg->ndim;
  g.bc = cfg->bc;
  g.nlev = L.nlev;
  g.nf = cfg->nfields;
  for (int l = 0; l < L.nlev; l++) {
    g.n[l] = cfg->n >> l;
    long long c = 1;
    for (int d = 0; d < cfg->ndim; d++) c *= g.n[l];
    g.cells[l] = (int)c;
    g.lg[l] = 0;
    while ((1 << g.lg[l]) < g.n[l]) g.lg[l]++;
    for (int f = 0; f < cfg->nfields; f++) {
      g.phi[f][l] = reinterpret_cast<double*>(base + L.off_phi[f][l]);
      g.f[f][l] = reinterpret_cast<double*>(base + L.off_f[f][l]);
      g.phi2[f][l] = L.off_phi2[f][l] ? reinterpret_cast<double*>(base + L.off_phi2[f][l]) : nullptr;
    }
  }
  for (int i = 0; i < 4; i++) m->tmp[i] = reinterpret_cast<double*>(base + L.off_tmp[i]);
  for (int l = 0; l < L.nlev; l++) {
    m->eps[l] = reinterpret_cast<double*>(base + L.off_eps[l]);
    g.eps[l] = m->eps[l];
  }
  m->par = reinterpret_cast<double*>(base + L.off_par);
  g.par = m->par;
  // the tail: the first level of at most TAIL_CELLS cells, and every level below
  int tail = 0;
  while (g.cells[tail] > TAIL_CELLS) tail++;
  m->tail = tail;
  int off = 0;
  for (int l = tail; l < L.nlev; l++) {
    g.loff[l] = off;
    off += 2 * g.cells[l];
  }
  m->tail_lds = (size_t)off * sizeof(double);
  int offv = 0;
  for (int l = tail; l < L.nlev; l++) {
    g.loffv[l] = offv;
    offv += 3 * g.cells[l];
  }
  m->tail_lds_var = (size_t)offv * sizeof(double);
  hipError_t e = cfg->ndim == 2
                     ? hipFuncSetAttribute(reinterpret_cast<const void*>(k_mg_tail<2, false>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)m->tail_lds)
                     : hipFuncSetAttribute(reinterpret_cast<const void*>(k_mg_tail<3, false>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)m->tail_lds);
  if (e == hipSuccess)
    e = cfg->ndim == 2 ? hipFuncSetAttribute(reinterpret_cast<const void*>(k_mg_tail<2, true>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)m->tail_lds_var)
                       : hipFuncSetAttribute(reinterpret_cast<const void*>(k_mg_tail<3, true>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)m->tail_lds_var);
  m->nb_init = std::min(blocks_of(g.cells[0]), 256);
  m->nb_cycle = tiled(m) ? (g.n[0] / TS) * (g.n[0] / TS) : m->nb_init;
  g.maxb = std::max(m->nb_init, m->nb_cycle);
  const size_t hbytes = (size_t)2 * NFMAX * g.maxb * sizeof(unsigned long long);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&m->hpart), hbytes);
  if (e == hipSuccess) {
    std::memset(m->hpart, 0, hbytes);
    g.hpart = m->hpart;
  }
  if (e == hipSuccess) e = hipEventCreate(&m->e0);
  if (e == hipSuccess) e = hipEventCreate(&m->e1);
  if (e != hipSuccess) {
    int rc = hip_err(e, "amrv_mg_create");
    amrv_mg_destroy(m);
    return rc;
  }
  *out = m;
  return 0;
}

int amrv_mg_destroy(amrv_mg* m) {
  if (!m) return 0;
  if (m->st) (void)hipStreamSynchronize(m->st);
  if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
  if (m->hpart) (void)hipHostFree(m->hpart);
  if (m->e0) (void)hipEventDestroy(m->e0);
  if (m->e1) (void)hipEventDestroy(m->e1);
  delete m;
  return 0;
}

int amrv_mg_solve(amrv_mg* m, const double* f, double* phi, const double* lambda, double tol, int32_t max_cycles,
                  int32_t* cycles, double* res_max, double* f_max) {
  if (!m || !f || !phi || !lambda) return set_error(AMRV_EINVAL, "null argument");
  if (!(tol > 0.0)) return set_error(AMRV_EINVAL, "tol must be positive");
  if (max_cycles < 0) return set_error(AMRV_EINVAL, "max_cycles must be >= 0");
  for (int i = 0; i < m->g.nf; i++)
    if (!(lambda[i] >= 0.0) || !std::isfinite(lambda[i]))
      return set_error(AMRV_EINVAL, "lambda must be non-negative and finite");
  for (int i = 0; i < m->g.nf; i++)
    if (m->var && !(lambda[i] > 0.0)) return set_error(AMRV_EINVAL, "a solve with a coefficient needs lambda > 0");
  if (int rc = set_params(m, lambda)) return rc;
  const size_t bytes = (size_t)m->g.cells[0] * sizeof(double);
  for (int i = 0; i < m->g.nf; i++) {
    MGCHK(hipMemcpyAsync(m->g.f[i][0], f + (size_t)i * m->g.cells[0], bytes, hipMemcpyDeviceToDevice, m->st));
    MGCHK(hipMemcpyAsync(m->g.phi[i][0], phi + (size_t)i * m->g.cells[0], bytes, hipMemcpyDeviceToDevice, m->st));
  }
  int c = 0;
  const int rc = run_cycles(m, tol, max_cycles, 0, &c, res_max, f_max);
  if (cycles) *cycles = c;
  for (int i = 0; i < m->g.nf; i++)
    MGCHK(hipMemcpyAsync(phi + (size_t)i * m->g.cells[0], m->g.phi[i][0], bytes, hipMemcpyDeviceToDevice, m->st));
  MGCHK(hipStreamSynchronize(m->st));
  return rc;
}

int amrv_mg_divb_project(amrv_mg* m, double* bx, double* by, double* bz, double tol, int32_t max_cycles,
                         int32_t* cycles, double* div_before, double* div_after) {
  if (!m || !bx || !by || (m->g.nd == 3 && !bz)) return set_error(AMRV_EINVAL, "null argument");
  if (m->g.nf != 1) return set_error(AMRV_EINVAL, "the projection needs a solver created with nfields = 1");
  if (m->var) return set_error(AMRV_EINVAL, "the projection needs the constant coefficient");
  if (m->g.bc != AMRV_MG_PERIODIC) return set_error(AMRV_EINVAL, "the projection needs periodic faces");
  if (!(tol > 0.0) || max_cycles < 0) return set_error(AMRV_EINVAL, "bad tol or max_cycles");
  const double lam0 = 0.0;
  if (int rc = set_params(m, &lam0)) return rc;
  const MgDev& g = m->g;
  const double c = 0.5 * g.n[0] / m->cfg.length;
  const bool d2 = g.nd == 2;
  const int nb = blocks_of(g.cells[0]);
  double* b2 = d2 ? bx : bz;  // not read in 2D
  auto divmax = [&](double* out) -> int {
    hipLaunchKernelGGL(d2 ? k_mg_divnorm<2> : k_mg_divnorm<3>, dim3(m->nb_init), dim3(256), 0, m->st, g, bx, by, b2,
                       c);
    MGCHK(hipGetLastError());
    MGCHK(hipStreamSynchronize(m->st));
    unsigned long long v = 0;
    for (int b = 0; b < m->nb_init; b++) v = m->hpart[b] > v ? m->hpart[b] : v;
    if (out) *out = bits_to_double(v);
    return 0;
  };
  if (int rc = divmax(div_before)) return rc;
  hipLaunchKernelGGL(d2 ? k_mg_divb<2> : k_mg_divb<3>, dim3(nb), dim3(256), 0, m->st, g, bx, by, b2, c);
  MGCHK(hipGetLastError());
  int cyc = 0;
  const int rc = run_cycles(m, tol, max_cycles, 0, &cyc, nullptr, nullptr);
  if (cycles) *cycles = cyc;
  if (rc) return rc;
  hipLaunchKernelGGL(d2 ? k_mg_gradsub<2> : k_mg_gradsub<3>, dim3(nb), dim3(256), 0, m->st, g, bx, by, b2, c);
  MGCHK(hipGetLastError());
  return divmax(div_after);
}

int amrv_rd_step(amrv_mg* m, const amrv_rd_params* p, int32_t scheme, double dt, int32_t nsteps, double* u, double* v,
                 double tol, int32_t max_cycles, int32_t* cycles_total, double* res_max) {
  if (!m || !p || !u || !v) return set_error(AMRV_EINVAL, "null argument");
  if (p->model != AMRV_RD_SCHNAKENBERG && p->model != AMRV_RD_GRAY_SCOTT) return set_error(AMRV_EINVAL, "unknown model");
  if (!(p->Du > 0.0) || !(p->Dv > 0.0)) return set_error(AMRV_EINVAL, "diffusion coefficients must be positive");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(AMRV_EINVAL, "dt must be positive and finite");
  if (nsteps < 0) return set_error(AMRV_EINVAL, "nsteps must be >= 0");
  if (scheme < AMRV_RD_EULER || scheme > AMRV_RD_IMEX) return set_error(AMRV_EINVAL, "unknown scheme");
  if (m->var) return set_error(AMRV_EINVAL, "reaction-diffusion steps need the constant coefficient");
  const bool implicit = scheme == AMRV_RD_SPLIT || scheme == AMRV_RD_IMEX;
  if (implicit && m->g.nf != 2) return set_error(AMRV_EINVAL, "split and IMEX steps need a solver with nfields = 2");
  if (implicit && (!(tol > 0.0) || max_cycles < 0)) return set_error(AMRV_EINVAL, "bad tol or max_cycles");
  RdK k{p->model, p->Du, p->Dv, p->p1, p->p2, p->p3};
  const MgDev& g = m->g;
  const int nb = blocks_of(g.cells[0]);
  const size_t bytes = (size_t)g.cells[0] * sizeof(double);
  double lam[2] = {1.0, 1.0};
  if (scheme == AMRV_RD_SPLIT) {
    lam[0] = 1.0 / (dt * p->Du);
    lam[1] = 1.0 / (dt * p->Dv);
  } else if (scheme == AMRV_RD_IMEX) {
    lam[0] = 2.0 / (dt * p->Du);
    lam[1] = 2.0 / (dt * p->Dv);
  }
  if (int rc = set_params(m, lam)) return rc;
  int total = 0;
  const bool d2 = g.nd == 2;
  double *cu = u, *cv = v, *au = m->tmp[0], *av = m->tmp[1];  // explicit schemes: current and other buffer
  for (int s = 0; s < nsteps; s++) {
    if (scheme == AMRV_RD_EULER || scheme == AMRV_RD_MIDPOINT) {
      // the new state goes to the other buffer of the pair (the caller's
      // arrays and tmp[0..1] alternate); one copy at the end if needed
      if (scheme == AMRV_RD_EULER) {
        hipLaunchKernelGGL(d2 ? k_rd_explicit<2> : k_rd_explicit<3>, dim3(nb), dim3(256), 0, m->st, g, k, cu, cv, cu,
                           cv, au, av, dt);
      } else {
        double *hu = m->tmp[2], *hv = m->tmp[3];
        hipLaunchKernelGGL(d2 ? k_rd_explicit<2> : k_rd_explicit<3>, dim3(nb), dim3(256), 0, m->st, g, k, cu, cv, cu,
                           cv, hu, hv, 0.5 * dt);
        hipLaunchKernelGGL(d2 ? k_rd_explicit<2> : k_rd_explicit<3>, dim3(nb), dim3(256), 0, m->st, g, k, cu, cv, hu,
                           hv, au, av, dt);
      }
      MGCHK(hipGetLastError());
      std::swap(cu, au);
      std::swap(cv, av);
      if (s + 1 == nsteps && cu != u) {
        MGCHK(hipMemcpyAsync(u, cu, bytes, hipMemcpyDeviceToDevice, m->st));
        MGCHK(hipMemcpyAsync(v, cv, bytes, hipMemcpyDeviceToDevice, m->st));
      }
      continue;
    }
    if (scheme == AMRV_RD_SPLIT)
      hipLaunchKernelGGL(d2 ? k_rd_split_rhs<2> : k_rd_split_rhs<3>, dim3(nb), dim3(256), 0, m->st, g, k, u, v, dt);
    else
      hipLaunchKernelGGL(d2 ? k_rd_imex_rhs<2> : k_rd_imex_rhs<3>, dim3(nb), dim3(256), 0, m->st, g, k, u, v,
                         m->tmp[0], m->tmp[1], dt);
    MGCHK(hipGetLastError());
    int c = 0;
    // the previous solve's cycle count, less one, runs before the first check
    const int rc = run_cycles(m, tol, max_cycles, m->last_cycles - 1, &c, res_max, nullptr);
    m->last_cycles = c;
    total += c;
    if (rc) {
      if (cycles_total) *cycles_total = total;
      return rc;
    }
    if (scheme == AMRV_RD_SPLIT) {
      MGCHK(hipMemcpyAsync(u, g.phi[0][0], bytes, hipMemcpyDeviceToDevice, m->st));
      MGCHK(hipMemcpyAsync(v, g.phi[1][0], bytes, hipMemcpyDeviceToDevice, m->st));
    } else {
      hipLaunchKernelGGL(d2 ? k_rd_imex_final<2> : k_rd_imex_final<3>, dim3(nb), dim3(256), 0, m->st, g, k, u, v,
                         m->tmp[0], m->tmp[1], dt);
      MGCHK(hipGetLastError());
    }
  }
  if (cycles_total) *cycles_total = total;
  MGCHK(hipStreamSynchronize(m->st));
  return 0;
}

int amrv_mg_set_coefficient(amrv_mg* m, const double* eps) {
  if (!m) return set_error(AMRV_EINVAL, "null argument");
  if (m->gexec) {  // the captured cycle belongs to the other operator
    MGCHK(hipGraphExecDestroy(m->gexec));
    m->gexec = nullptr;
  }
  if (!eps) {
    m->var = false;
    m->g.eps[0] = m->eps[0];
    return 0;
  }
  const MgDev& g = m->g;
  MGCHK(hipMemcpyAsync(m->eps[0], eps, (size_t)g.cells[0] * sizeof(double), hipMemcpyDeviceToDevice, m->st));
  for (int l = 0; l + 1 < g.nlev; l++) {
    if (g.nd == 2)
      hipLaunchKernelGGL(k_mg_eps_restrict<2>, dim3(blocks_of(g.cells[l + 1])), dim3(256), 0, m->st, g, l,
                         m->eps[l + 1]);
    else
      hipLaunchKernelGGL(k_mg_eps_restrict<3>, dim3(blocks_of(g.cells[l + 1])), dim3(256), 0, m->st, g, l,
                         m->eps[l + 1]);
    MGCHK(hipGetLastError());
  }
  MGCHK(hipStreamSynchronize(m->st));
  m->var = true;
  return 0;
}

int amrv_mg_profile(amrv_mg* m, int32_t enable) {
  if (!m) return set_error(AMRV_EINVAL, "null argument");
  m->profile = enable != 0;
  return 0;
}

int amrv_mg_profile_read(amrv_mg* m, double* ms_total, int64_t* cycles) {
  if (!m || !ms_total || !cycles) return set_error(AMRV_EINVAL, "null argument");
  *ms_total = m->prof_ms;
  *cycles = m->prof_cycles;
  m->prof_ms = 0.0;
  m->prof_cycles = 0;
  return 0;
}

}  // extern "C"
