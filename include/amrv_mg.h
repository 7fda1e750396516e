/* amrv_mg.h -- C-ABI of libamrv's geometric multigrid Helmholtz solver and
 * the reaction-diffusion time steps built on it.
 *
 * Method (arXiv 2004.03275): the multigrid functionality of Sec. 1.4 solves
 * Poisson/Helmholtz problems; Sec. 2.5 uses it for the reaction-diffusion
 * models (Eqs. gray-scott and schnakenberg): the split scheme's backward-
 * Euler diffusion step leads to the Helmholtz problem of Eq. diff-helmholtz,
 * and the first stage of the IMEX scheme (Eq. imex, the trapezoidal pair) to
 * another one.  This library solves them on one uniform cell-centred grid.
 *
 * Grid and layout: n cells per side (a power of two), ndim = 2 or 3, on
 * [0, L]^ndim, h = L / n.  A field is n^ndim binary64 values in device
 * memory, x fastest: index x + n (y + n z).  Boundaries: periodic, or zero
 * Neumann (the ghost value beyond a face equals the adjacent interior cell).
 * Discrete Laplacian: per direction ((w_minus + w_plus) - 2 w) / h^2, the
 * directions summed in the order x, y, z.
 *
 * Helmholtz problem: lap(phi) - lambda phi = f with lambda > 0, or the
 * Poisson problem (lambda = 0) of the divergence control of the paper's MHD
 * runs (Sec. 2.4), whose solution is fixed up to a constant.  The solver
 * runs V-cycles (red-black Gauss-Seidel smoothing with `pre` and `post`
 * sweeps, residual restriction by averaging the 2^ndim children, correction
 * prolongation by bi/trilinear interpolation, coarse grids rediscretised
 * down to 2 cells per side and solved exactly there) until the maximum
 * residual |f - (lap(phi) - lambda phi)| is at most tol times max |f| -- the
 * paper's stopping rule, Sec. 2.5.2, with tol = 1e-7 there.  Since lambda I - lap is an M-matrix
 * whose rows sum to lambda, the returned solution differs from the exact
 * discrete one by at most (max residual) / lambda in every cell (lambda = 0:
 * up to a constant, by at most sqrt(cells) (max residual) / mu_1 with mu_1
 * the smallest non-zero eigenvalue magnitude of lap).
 *
 * Conventions: as in amrv.h (0 on success, negative AMRV_E* codes,
 * amrv_last_error() for the message).  All device pointers belong to the
 * caller; the handle keeps only its workspace and stream.  Calls enqueue on
 * the handle's stream and return after it has completed (the solver reads
 * the residual after every cycle).
 */
#ifndef AMRV_MG_H
#define AMRV_MG_H

#include <stddef.h>
#include <stdint.h>

#include "amrv.h"

#ifdef __cplusplus
extern "C" {
#endif

#define AMRV_ENOTCONVERGED (-7) /* the residual did not reach tol within max_cycles */

#define AMRV_MG_PERIODIC 0
#define AMRV_MG_NEUMANN 1

/* Smoother launches of the levels above the LDS-resident coarse tail.  In 2D
 * TILED stages 32x32 tiles with a halo in LDS and repeats the red-black
 * sweeps over the halo, so one launch per level smooths and restricts (and
 * one prolongs and smooths); PER_COLOUR launches every colour sweep over the
 * whole level.  Both compute every cell from the same neighbour values in
 * the same order and agree bit for bit; 3D always uses PER_COLOUR. */
#define AMRV_MG_TILED 0
#define AMRV_MG_PER_COLOUR 1

#define AMRV_RD_SCHNAKENBERG 0 /* F0 = (kappa (a - u + u^2 v), kappa (b - u^2 v)) */
#define AMRV_RD_GRAY_SCOTT 1   /* F0 = (-u v^2 + F (1 - u), u v^2 - (F + k) v) */

#define AMRV_RD_EULER 0    /* w1 = w + dt F(w), F = F0 + D lap: explicit */
#define AMRV_RD_MIDPOINT 1 /* explicit midpoint: w + dt F(w + dt/2 F(w)) */
#define AMRV_RD_SPLIT 2    /* w* = w + dt F0(w); w1 = w* + dt D lap(w1) (Helmholtz, lambda = 1/(dt D)) */
#define AMRV_RD_IMEX 3     /* Eq. imex: w* - dt/2 D lap(w*) = w + dt F0(w) + dt/2 D lap(w)
                              (Helmholtz, lambda = 2/(dt D)); w1 = w + dt/2 (F(w) + F(w*)) */

typedef struct amrv_mg amrv_mg;

typedef struct {
  int32_t ndim;          /* 2 or 3 */
  int32_t n;             /* cells per side: power of two, 4..8192 (2D), 4..512 (3D) */
  int32_t bc;            /* AMRV_MG_PERIODIC or AMRV_MG_NEUMANN */
  int32_t nfields;       /* 1 or 2 fields solved together (2 for the RD steps) */
  int32_t pre_sweeps;    /* red-black sweeps before restriction (1..8) */
  int32_t post_sweeps;   /* red-black sweeps after prolongation (1..8) */
  int32_t use_graph;     /* replay each V-cycle from a captured HIP graph (needs a stream) */
  int32_t smoother;      /* AMRV_MG_TILED or AMRV_MG_PER_COLOUR (same results, bit for bit) */
  double length;         /* L > 0 */
} amrv_mg_config;

typedef struct {
  int32_t model; /* AMRV_RD_SCHNAKENBERG or AMRV_RD_GRAY_SCOTT */
  int32_t pad;
  double Du, Dv; /* diffusion coefficients, > 0 */
  double p1, p2, p3; /* Schnakenberg: kappa, a, b; Gray-Scott: F, k, unused */
} amrv_rd_params;

/* Bytes of device workspace for this configuration (256-byte aligned
 * start), or 0 with amrv_last_error() set for an invalid one. */
size_t amrv_mg_workspace_bytes(const amrv_mg_config* cfg);

/* Creates a solver in the caller's workspace (device memory of at least
 * amrv_mg_workspace_bytes, owned by the caller, alive until destroy) on the
 * given HIP stream (NULL: the null stream).  Allocates only pinned host
 * memory for the residual read-back. */
int amrv_mg_create(const amrv_mg_config* cfg, void* workspace, size_t bytes, void* stream, amrv_mg** out);
int amrv_mg_destroy(amrv_mg* m);

/* Solves lap(phi) - lambda phi = f (Sec. 1.4; Sec. 2.5.1, Eq. diff-helmholtz) for
 * nfields fields stored one after another (f and phi: nfields * n^ndim
 * doubles each, device; phi holds the initial guess on entry and the
 * solution on return; lambda: nfields host values, each >= 0; with
 * lambda = 0 the right-hand side must sum to zero, or the residual cannot
 * fall below |mean f| and the call ends with AMRV_ENOTCONVERGED).  Stops when
 * every field's max residual <= tol * its max |f| (tol > 0), or after
 * max_cycles V-cycles (then AMRV_ENOTCONVERGED, phi holding the last
 * iterate).  cycles, res_max and f_max (host, may be NULL) receive the
 * cycle count and, per field, the final max residual and max |f|. */
int amrv_mg_solve(amrv_mg* m, const double* f, double* phi, const double* lambda, double tol, int32_t max_cycles,
                  int32_t* cycles, double* res_max, double* f_max);

/* Variable coefficient (Sec. 1.4: Helmholtz problems with variable
 * coefficients): with eps != NULL (device, n^ndim doubles, each > 0; copied)
 * later amrv_mg_solve calls solve div(eps grad phi) - lambda phi = f, the
 * coefficient of a face the arithmetic mean of its two cells (none across a
 * Neumann face), coarse levels carrying the mean of their children's eps, the
 * 2-per-side grid solved by elimination; lambda must be > 0 (the operator
 * stays an M-matrix with row sums lambda, so the residual bound above
 * holds).  These solves use the per-colour launches.  eps = NULL returns to
 * eps = 1.  amrv_rd_step and amrv_mg_divb_project need eps = 1. */
int amrv_mg_set_coefficient(amrv_mg* m, const double* eps);

/* Divergence control of the MHD runs (Sec. 2.4) on one uniform periodic
 * grid: solves lap(phi) = div B* (central differences (w(+1) - w(-1)) n/(2L),
 * directions added x, y, z) to tol, then sets B = B* - grad phi with the
 * same differences -- an approximate projection: it removes the divergence
 * up to the difference between the 5/7-point lap and div(grad).  bx, by, bz:
 * device arrays of n^ndim doubles (bz unused in 2D), updated in place.  Needs
 * a solver with nfields = 1 and periodic faces (the central divergence of a
 * field with mirrored Neumann faces does not sum to zero).  div_before and
 * div_after (host, may be NULL) receive max |div B| before and after;
 * cycles the V-cycle count. */
int amrv_mg_divb_project(amrv_mg* m, double* bx, double* by, double* bz, double tol, int32_t max_cycles,
                         int32_t* cycles, double* div_before, double* div_after);

/* nsteps time steps of the reaction-diffusion model (Sec. 2.5) on the
 * device fields u, v (n^ndim doubles each, updated in place) with step dt
 * and the given scheme.  SPLIT and IMEX need a solver created with
 * nfields = 2: both species' Helmholtz problems are solved together, each
 * to tol, at most max_cycles V-cycles per step (initial guess: the current
 * state for SPLIT, the explicit Euler predictor w + dt F(w) for IMEX).  To
 * save host synchronisations a solve runs the previous solve's cycle count
 * less one before its first residual check, so it may run a cycle or two
 * more than tol demands (never fewer).  If
 * a solve does not converge (AMRV_ENOTCONVERGED) or meets a NaN
 * (AMRV_ENONPHYSICAL), u and v hold the state after the last completed
 * step.  cycles_total (may be NULL) receives the V-cycles summed over the
 * steps; res_max (may be NULL, 2 doubles) the last solve's residuals. */
int amrv_rd_step(amrv_mg* m, const amrv_rd_params* p, int32_t scheme, double dt, int32_t nsteps, double* u, double* v,
                 double tol, int32_t max_cycles, int32_t* cycles_total, double* res_max);

/* V-cycle timing: with enable != 0, every V-cycle of amrv_mg_solve and
 * amrv_rd_step (graph replay or direct launches, residual read-back
 * included) is bracketed by HIP events on the handle's stream;
 * amrv_mg_profile_read returns the summed time (ms) and the cycle count
 * since the last read, and resets both. */
int amrv_mg_profile(amrv_mg* m, int32_t enable);
int amrv_mg_profile_read(amrv_mg* m, double* ms_total, int64_t* cycles);

/* ---------------------------------------------------------------------------
 * Helmholtz problem on a 2D or 3D block-adaptive forest (Sec. 1.4: the
 * geometric multigrid on the block-adaptive quadtree / octree grid).
 *
 * Grid: the leaves of a quadtree (ndim 2) or octree (ndim 3) forest of
 * 16^ndim-cell blocks on [0, L]^ndim, base^ndim blocks at level 1 (base a
 * power of two), leaf k at level leaf_level[k] (1..max_level) with block
 * coordinates leaf_ijk[3k .. 3k + 2] at that level (the third 0 in 2D), the
 * leaves covering the domain without overlap and 2:1 balanced across faces.
 * A field is one binary64 value per leaf cell, [leaf][(z)][y][x] with x
 * fastest (the forest's state layout of one variable), in device memory.
 *
 * Problem: lap(u) - lambda u = f, lap of a cell the (2 ndim + 1)-point sum at
 * the cell's own level, (sum of the 2 ndim values across its faces - 2 ndim
 * u) / h_l^2, h_l = L / (16 base 2^(l-1)).  The value across a face is the
 * same-level leaf's cell; at a domain face the periodic image or the
 * zero-Neumann mirror (the cell itself); on the fine side of a coarse-fine
 * face (u + 2 u_c) / 3, u_c the coarse cell across the face moved a quarter
 * coarse cell along the face in each tangential direction with the coarse
 * block's own difference there (central, one-sided at its edges); on the
 * coarse side u + (4/3) (m - u), m the mean of the 2^(ndim-1) fine cells
 * touching the face (the mean of the fine fluxes: the scheme is
 * conservative and second order).  The coarse-fine stencils are this
 * library's reading: the paper defers them to its multigrid library.
 *
 * Solver: V-cycles of the full approximation scheme over the block tree
 * (every ancestor of a leaf is a block holding the mean of its children),
 * red-black Gauss-Seidel with pre_sweeps / post_sweeps sweeps per level,
 * bi/trilinear interpolation of the coarse change within each parent, and
 * the uniform solver above on the complete level-1 grid (base * 16 <= 8192
 * in 2D, <= 512 in 3D).  Stops when the
 * maximum residual of the problem over the leaf cells is at most tol times
 * max |f|, or after max_cycles cycles (AMRV_ENOTCONVERGED, phi holding the
 * last iterate).  Host-synchronous: every cycle reads its residual back. */

typedef struct amrv_fmg amrv_fmg;

typedef struct {
  int64_t nleaves;     /* leaves, >= 1 */
  int32_t base;        /* level-1 blocks per side: a power of two, 1..512 */
  int32_t max_level;   /* 1..16 */
  int32_t bc;          /* AMRV_MG_PERIODIC or AMRV_MG_NEUMANN */
  int32_t pre_sweeps;  /* red-black sweeps per level on the way down (1..8) */
  int32_t post_sweeps; /* and on the way up (1..8) */
  int32_t ndim;        /* 2 (quadtree, also for 0) or 3 (octree) */
  double length;       /* L > 0 */
} amrv_fmg_config;

/* Bytes of device workspace for this forest (256-byte aligned start), or 0
 * with amrv_last_error() set (AMRV_EINVAL for a bad configuration,
 * AMRV_EUNBALANCED for leaves that overlap, leave gaps or break 2:1
 * balance).  leaf_level [nleaves], leaf_ijk [nleaves][3]: host. */
size_t amrv_fmg_workspace_bytes(const amrv_fmg_config* cfg, const int32_t* leaf_level, const int32_t* leaf_ijk);

/* Builds the block tree and its tables in the caller's workspace (device
 * memory of at least amrv_fmg_workspace_bytes, owned by the caller, alive
 * until destroy), on the given HIP stream (NULL: the null stream).
 * Allocates only pinned host memory for the residual read-back (and the
 * level-1 solver's).  Returns 0 or a negative AMRV_E* code. */
int amrv_fmg_create(const amrv_fmg_config* cfg, const int32_t* leaf_level, const int32_t* leaf_ijk,
                    void* workspace, size_t bytes, void* stream, amrv_fmg** out);
int amrv_fmg_destroy(amrv_fmg* m);

/* Blocks per level of the tree (levels 1..16; 0 beyond the finest), host
 * array of 16. */
int amrv_fmg_levels(const amrv_fmg* m, int32_t* nblocks_per_level);

/* Solves lap(phi) - lambda phi = f on the leaf cells (f, phi: device fields
 * of nleaves * 256 doubles; phi holds the initial guess on entry and the
 * solution on return).  lambda = 0 (Poisson, the divergence control of
 * Sec. 2.4): lap is singular on a periodic or Neumann domain (constants are
 * its null space, the area-weighted sum of lap(phi) vanishes), so the
 * problem solved is lap(phi) = f - mean(f) and phi is returned with zero
 * mean, means weighted by cell area.  cycles, res_max, f_max (host, may be
 * NULL) receive the V-cycle count, the final maximum residual and max |f|
 * of the problem solved.  Returns 0, AMRV_ENOTCONVERGED, AMRV_ENONPHYSICAL
 * (NaN or infinity in f, phi or the residual), AMRV_EINVAL (lambda < 0,
 * tol <= 0, max_cycles < 0) or AMRV_EDEVICE. */
int amrv_fmg_solve(amrv_fmg* m, const double* f, double* phi, double lambda, double tol, int32_t max_cycles,
                   int32_t* cycles, double* res_max, double* f_max);

/* nsteps reaction-diffusion steps on the forest's leaf fields u, v (device,
 * nleaves * 256 doubles each, updated in place), the schemes and models of
 * amrv_rd_step with this forest's Laplacian (the rules above, lambda = 0):
 * EULER and MIDPOINT explicit (the paper's Gray-Scott AMR run uses
 * MIDPOINT), SPLIT and IMEX through amrv_fmg_solve per species (tol,
 * max_cycles as there).  cycles_total and res_max (host, may be NULL)
 * receive the V-cycles summed over the solves and the largest final
 * residual.  Returns 0 or the first failing solve's code. */
int amrv_fmg_rd_step(amrv_fmg* m, const amrv_rd_params* p, int32_t scheme, double dt, int32_t nsteps, double* u,
                     double* v, double tol, int32_t max_cycles, int32_t* cycles_total, double* res_max);

/* The divergence control of Sec. 2.4 on a forest's leaf fields bx, by, bz
 * (device, nleaves * 16^ndim doubles each, updated in place; bz unused and
 * may be NULL in 2D, required in 3D): phi is the
 * zero-mean solution of lap(phi) = div B* (amrv_fmg_solve with lambda = 0,
 * tol and max_cycles as there), then B = B* - grad phi; div and grad are
 * central differences (w(+1) - w(-1)) / (2 h_l) at each cell's level with
 * the neighbour values of the rules above (exact for linear data), added x,
 * y then z.  An approximate projection: it removes the divergence up to what
 * the compact lap and div(grad) disagree on (O(h^2) away from coarse-fine
 * faces, O(1) next to them).  div_before, div_after (host, may be NULL)
 * receive max |div B| before and after; cycles the V-cycle count. */
int amrv_fmg_divb_project(amrv_fmg* m, double* bx, double* by, double* bz, double tol, int32_t max_cycles,
                          int32_t* cycles, double* div_before, double* div_after);

#ifdef __cplusplus
}
#endif
#endif
