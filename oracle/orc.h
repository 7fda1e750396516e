/* orc.h -- CPU oracle for the block-forest conservative finite-volume update.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of bench.py may load this library.  The product path (the HIP library)
 * never links, loads or calls it, and the two share no source, header, table
 * or helper.
 *
 * What it computes follows MPI-AMRVAC (Keppens et al., arXiv 2004.03275):
 *   conservation law dU/dt + div F(U) = 0 (Sec. 1.1, Eq. (eq)), HD variables
 *   (rho, rho v, E) with E = rho v^2/2 + p/(gamma-1) (Sec. 1.1); primitive
 *   conversion and signal speeds (Sec. 1.2, phys_to_primitive, phys_get_cmax,
 *   phys_get_cbounds); TVDLF / HLL / HLLC approximate Riemann fluxes (Sec. 1.2,
 *   Sec. 2.4); block quadtree/octree with refinement ratio 2 and the Loehner
 *   refine/coarsen rule (Sec. 1.3); three-step / SSP Runge-Kutta (Sec. 2.1,
 *   2.3.2, 2.4); Courant-limited time step (Sec. 2.1).  The paper prints none
 *   of the scheme formulas; where it is silent the reading used is stated at
 *   the function that implements it.
 *
 * All arithmetic is IEEE binary64 with round-to-nearest, built with
 * -ffp-contract=off and without fast-math, so every expression is evaluated
 * exactly in the order written.
 *
 * State layout (host memory, caller owned, copied in/out):
 *   U[var][leaf][z][y][x], interior cells only, leaves in the caller's order.
 * Error codes: 0 ok, -1 invalid argument, -2 unbalanced / non-covering forest,
 *   -3 non-physical state (rho <= 0, p <= 0 or NaN), -4 out of memory.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_forest orc_forest;

/* Field order is part of the contract: 20 int32 then 13 double. */
typedef struct {
  int32_t ndim;            /* 1, 2 or 3 */
  int32_t block_nx[3];     /* interior cells per block and dimension (1 if unused) */
  int32_t nghost;          /* ghost layers; must be 2 */
  int32_t base_blocks[3];  /* level-1 blocks per dimension */
  int32_t max_level;       /* refine_max_level of Sec. 1.3 (1 = pure decomposition) */
  int32_t physics;         /* 0 = Euler (HD), 1 = ideal MHD with GLM cleaning, 2 = polytrope
                              p = c_ad rho^gamma without energy equation (shallow water:
                              c_ad = 1/2, gamma = 2; TVDLF or HLL) */
  int32_t flux;            /* 0 = TVDLF, 1 = HLL, 2 = HLLC */
  int32_t limiter;         /* 0 = minmod, 1 = van Leer, 2 = monotonized central, 3 = Koren, 4 = Cada */
  int32_t rk_stages;       /* 2 = SSP-RK2, 3 = SSP-RK3 */
  int32_t bc[3][2];        /* per dimension, low/high side: 0 periodic, 1 zero gradient */
  int32_t pad_;
  double xmin[3], xmax[3]; /* xprobmin/xprobmax of Sec. 1.3 */
  double gamma, cfl;
  double lohner_tol, lohner_coarsen_frac, lohner_eps, lohner_w_rho, lohner_w_p;
  double glm_cr;
  double cad;              /* c_ad of the polytrope */
  double cada_radius;      /* r of Cada's smoothness switch (0: no switch) */
} orc_config;

int orc_forest_create(const orc_config* cfg, int64_t nleaves,
                      const int32_t* leaf_level, const int32_t* leaf_ijk,
                      orc_forest** out);
int orc_forest_destroy(orc_forest* f);
int orc_nvar(const orc_forest* f);
int orc_set_state(orc_forest* f, const double* U, int64_t n_doubles);
int orc_get_state(const orc_forest* f, double* U, int64_t n_doubles);
/* Courant time step of the current state; also validates positivity and, for
 * MHD, records the GLM cleaning speed used by the next advance calls. */
int orc_max_dt(orc_forest* f, double* dt_out);
/* GLM cleaning speed recorded by the last orc_max_dt (0 if none). */
double orc_glm_ch(const orc_forest* f);
/* One full SSP Runge-Kutta step of size dt. */
int orc_advance(orc_forest* f, double dt);
/* Loehner refine (+1) / keep (0) / coarsen (-1) flags, one per leaf; emax_out
 * (optional, may be NULL) receives the per-leaf max of the weighted estimator. */
int orc_flag_blocks(orc_forest* f, int8_t* flags_out, double* emax_out);
/* Test hook: the ghost-filled block of leaf `leaf` for the current state,
 * layout [var][pz][py][px] with px = nx + 2*nghost on active dimensions.
 * Edge and corner ghost cells are never filled and hold NaN. */
int orc_padded_block(orc_forest* f, int64_t leaf, double* out, int64_t n_doubles);
/* Test hook: neighbour kind per face of a leaf: 0 same level, 1 coarser,
 * 2 finer, 3 physical boundary. faces = 2*ndim entries (-x,+x,-y,+y,-z,+z). */
int orc_face_kinds(const orc_forest* f, int64_t leaf, int32_t* kinds);
/* Test hook: per-cell weighted Loehner estimator of one leaf, [cell]. */
/* The forest's Riemann flux across a face normal to dir (0..ndim-1) for the
 * primitive face states vl, vr (nvar values each; MHD uses the GLM speed of
 * the last orc_max_dt) into F (nvar). */
int orc_face_flux(orc_forest* f, const double* vl, const double* vr, int dir, double* F);
int orc_lohner_cells(orc_forest* f, int64_t leaf, double* out, int64_t n_doubles);
/* Regrid plan (Sec. 1.3, refinement ratio 2): leaves flagged +1 (below
 * max_level) are split into 2^ndim children; a complete group of 2^ndim
 * sibling leaves all flagged -1 (above level 1) is merged into its parent;
 * 2:1 balance over faces, edges and corners is kept by refining every leaf
 * that touches a refined leaf from one level coarser (repeated until
 * nothing changes) and by keeping a group whose parent would touch a leaf
 * ending more than one level finer (other coarsenings ignored).  New order:
 * unchanged leaves in place, a refined leaf replaced by its children (child
 * index ox + 2 oy + 4 oz), a merged group by its parent at the position of
 * the group's first member.  Writes up to `cap` leaves to new_level /
 * new_ijk [cap][3]; *new_n is the new leaf count (ORC_ENOMEM if > cap). */
int orc_regrid_plan(const orc_forest* f, const int8_t* flags, int64_t cap, int64_t* new_n, int32_t* new_level,
                    int32_t* new_ijk);
/* State of `from` onto `to` (a one-level regrid of it, same configuration):
 * copied leaves, children by conservative linear prolongation of the parent
 * (coarse value plus a quarter minmod slope per dimension, the parent's ghost
 * cells at its boundary), parents by restriction of their children. */
int orc_regrid_transfer(orc_forest* from, orc_forest* to);
/* Test hook: the limited slope of a cell toward a face from the difference a
 * away from the face and b toward it (limiter 0 minmod, 1 van Leer,
 * 2 monotonized central, 3 Koren). */
double orc_limiter_value(int limiter, double a, double b, double thr2);
void orc_set_threads(int n);
int orc_get_threads(void);
const char* orc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
