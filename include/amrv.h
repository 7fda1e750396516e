/* amrv.h -- C-ABI of the MI355X block-forest finite-volume library (libamrv.so).
 *
 * The library advances the conservative finite-volume discretisation of
 *   dU/dt + div F(U) = 0                       (arXiv 2004.03275, Sec. 1.1, Eq. (eq))
 * on a quadtree/octree forest of fixed-size blocks with refinement ratio 2
 * (Sec. 1.3): ghost-cell fill (same-level copy, fine-to-coarse restriction,
 * coarse-to-fine prolongation), limited MUSCL reconstruction in primitive
 * variables (Sec. 1.2 phys_to_primitive), TVDLF / HLL / HLLC fluxes (Sec. 1.2,
 * Sec. 2.4), coarse-fine flux replacement for conservation (Sec. 1.1), SSP
 * Runge-Kutta stages (Sec. 2.1-2.4), the Courant time step (Sec. 2.1,
 * phys_get_cmax) and the Loehner refine/coarsen flags (Sec. 1.3).  Ideal MHD
 * uses HLL or HLLC (after Li 2005, Sec. 2.4) with mixed GLM divergence
 * cleaning; the polytrope without energy equation (Sec. 2.2) gives the
 * shallow water equations.  Limiters: minmod, van Leer, monotonized central,
 * Koren and Cada's third-order limiter (Sec. 2.2-2.4).
 *
 * Every operation runs in hand-written HIP kernels for gfx950 in binary64.
 *
 * Conventions for every entry point:
 *  - Return 0 on success or a negative AMRV_E* code; amrv_last_error() gives a
 *    thread-local message.  No entry point aborts the process.
 *  - Host arrays passed in are owned by the caller and copied; the library
 *    keeps no pointer to them after the call returns.
 *  - Device memory: the caller allocates ONE device workspace of
 *    amrv_workspace_bytes() bytes (e.g. a torch uint8 tensor) and keeps it
 *    alive until amrv_forest_destroy; the library allocates no device memory
 *    of its own (its one static array, the training scratch of
 *    amrv_mlp_train_noalloc, is part of the loaded code object).  The HIP
 *    stream is borrowed; all work is enqueued on it.
 *  - State layout: conserved binary64 U[var][leaf][z][y][x], interior cells
 *    only, leaves in the caller's order.  Hydrodynamics: var = (rho, m_x,
 *    [m_y, m_z,] E); MHD: (rho, m.., E, B.., psi); polytrope: (rho, m..).
 */
#ifndef AMRV_H
#define AMRV_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AMRV_OK 0
#define AMRV_EINVAL (-1)        /* bad config, argument, size or dt */
#define AMRV_EUNBALANCED (-2)   /* leaves overlap, leave gaps or break 2:1 balance */
#define AMRV_ENONPHYSICAL (-3)  /* rho <= 0, p <= 0 or NaN in the state */
#define AMRV_ENOMEM (-4)        /* workspace too small */
#define AMRV_EDEVICE (-5)       /* HIP runtime error */
#define AMRV_ENOTSUP (-6)       /* configuration valid but not supported by the kernels */

#define AMRV_EULER 0
#define AMRV_MHD_GLM 1
/* polytrope without energy equation (Sec. 2.2): state (rho, m), p = c_ad rho^gamma,
   c^2 = gamma c_ad rho^(gamma-1); the shallow water equations for rho = h,
   c_ad = 1/2, gamma = 2.  TVDLF or HLL. */
#define AMRV_POLYTROPE 2
#define AMRV_TVDLF 0
#define AMRV_HLL 1
#define AMRV_HLLC 2
#define AMRV_MINMOD 0
#define AMRV_VANLEER 1
#define AMRV_MC 2 /* monotonized central ('woodward', Sec. 2.3.1) */
#define AMRV_KOREN 3 /* Koren (Sec. 2.2, 2.3.2); asymmetric: two half slopes per cell */
#define AMRV_CADA 4  /* Cada's third order (Sec. 2.4 blast runs; LimO3 of Cada and Torrilhon 2009;
                        its smoothness switch with cada_radius > 0); asymmetric */
#define AMRV_BC_PERIODIC 0
#define AMRV_BC_ZERO_GRADIENT 1

/* schedules of the stage update (amrv_set_schedule) */
#define AMRV_SCHED_PER_BLOCK 0    /* one kernel launch per leaf per stage */
#define AMRV_SCHED_GRID 1         /* one launch per stage, one workgroup per leaf */
#define AMRV_SCHED_PERSISTENT 2   /* one launch per stage, persistent workgroups */

/* flag modes (amrv_flag_blocks) */
#define AMRV_FLAG_LOHNER 0        /* Loehner estimator (Sec. 1.3) */
#define AMRV_FLAG_MLP 1           /* learned flagger: +1 where its logit > 0, else 0 */
#define AMRV_FLAG_MLP_FALLBACK 2  /* learned flagger, Loehner where |logit| < margin */

typedef struct amrv_forest amrv_forest;

/* Problem description (par-file keys of Sec. 1.3: block size, base domain
 * size in blocks, refine_max_level, xprobmin/xprobmax; Courant number of
 * Sec. 2.1; scheme choice of Sec. 1.3; Loehner tolerances of Sec. 1.3).
 * Field order is part of the ABI: 20 int32 followed by 16 double. */
typedef struct {
  int32_t ndim;            /* 1, 2 or 3 */
  int32_t block_nx[3];     /* cells per block; 1D: any even nx >= 4; 2D/3D: 16 */
  int32_t nghost;          /* must be 2 */
  int32_t base_blocks[3];  /* level-1 blocks per dimension */
  int32_t max_level;       /* 1 = pure domain decomposition */
  int32_t physics;         /* AMRV_EULER, AMRV_MHD_GLM or AMRV_POLYTROPE */
  int32_t flux;            /* AMRV_TVDLF, AMRV_HLL, AMRV_HLLC (HLLC: not the polytrope) */
  int32_t limiter;         /* AMRV_MINMOD, AMRV_VANLEER, AMRV_MC, AMRV_KOREN or AMRV_CADA */
  int32_t rk_stages;       /* 2 (SSP-RK2) or 3 (SSP-RK3) */
  int32_t bc[3][2];        /* AMRV_BC_*, same value on both sides of a dimension */
  int32_t pad_;
  double xmin[3], xmax[3];
  double gamma, cfl;
  double lohner_tol;           /* refine if the block max estimator exceeds it */
  double lohner_coarsen_frac;  /* coarsen if the block max is below frac*tol */
  double lohner_eps;           /* noise filter of the estimator */
  double lohner_w_rho, lohner_w_p;
  double glm_cr;               /* GLM damping length c_r */
  double cad;                  /* c_ad of the polytrope (> 0; read only for AMRV_POLYTROPE) */
  double cada_radius;          /* r >= 0 of Cada's smoothness switch: with AMRV_CADA the unlimited
                                  third-order slope (a+2b)/3 where a^2+b^2 <= (r dx)^2 (0: never) */
} amrv_config;

/* Device bytes the forest needs for this leaf list (three state copies,
 * neighbour tables, ghost and flux slabs of coarse-fine faces, scratch).
 * Returns 0 and sets the error message on an invalid config or forest. */
size_t amrv_workspace_bytes(const amrv_config* cfg, int64_t nleaves, const int32_t* leaf_level,
                            const int32_t* leaf_ijk);

/* Validate the leaf list (levels 1..max_level, block coordinates at that
 * level in leaf_ijk[3*i..3*i+2], cover without overlap, 2:1 balance across
 * faces, edges and corners), build neighbour and coarse-fine tables and bind
 * the workspace.  hip_stream is a hipStream_t (NULL = default stream). */
int amrv_forest_create(const amrv_config* cfg, int64_t nleaves, const int32_t* leaf_level,
                       const int32_t* leaf_ijk, void* d_workspace, size_t ws_bytes,
                       void* hip_stream, amrv_forest** out);
int amrv_forest_destroy(amrv_forest* f);

int amrv_nvar(const amrv_forest* f);
int64_t amrv_state_doubles(const amrv_forest* f);

/* Copy the state in/out.  on_device = 0: U is host memory (the call
 * synchronises the stream); 1: U is device memory (asynchronous). */
int amrv_set_state(amrv_forest* f, const double* U, int64_t n_doubles, int32_t on_device);
int amrv_get_state(amrv_forest* f, double* U, int64_t n_doubles, int32_t on_device);

/* Courant time step dt = cfl / max_cells sum_d (|v_d| + c_d)/dx_d of the
 * current state (Sec. 2.1; c = sound speed, the fast speed for MHD, or
 * sqrt(gamma c_ad rho^(gamma-1)) for the polytrope).  Synchronises; returns
 * AMRV_ENONPHYSICAL if any cell has rho <= 0, p <= 0 or NaN (the polytrope:
 * rho <= 0 or a velocity that is NaN or overflows).  For MHD it also records the GLM speed c_h = max |v_d| + c_f,d used by
 * the following amrv_advance calls. */
int amrv_max_dt(amrv_forest* f, double* dt_out);
/* GLM cleaning speed recorded by the last amrv_max_dt (0 before any). */
double amrv_glm_ch(const amrv_forest* f);

/* One full SSP Runge-Kutta step of size dt (Sec. 2.1-2.4), asynchronous on
 * the forest's stream.  dt must be positive and finite (else AMRV_EINVAL).
 * A non-physical result is reported by the next amrv_max_dt. */
int amrv_advance(amrv_forest* f, double dt);

/* nsteps full SSP-RK steps whose time steps are computed on the device:
 * each step takes dt = min(cfl / max_cells sum_d (|v_d| + c_d)/dx_d, t_end - t)
 * from the Courant reduction of the state it starts from (the last stage of
 * each step folds the reduction of its result into the same pass), so the
 * host does not synchronise between steps; the steps replay one captured
 * HIP graph.  *t (host) is the time before and after; a step starting at or
 * after t_end does nothing.  *taken (may be NULL) counts the steps with
 * dt > 0.  Synchronises at the end; AMRV_ENONPHYSICAL if a step met a
 * non-physical state (the steps after it do nothing).  The same arithmetic
 * as amrv_max_dt + amrv_advance, except that the MHD damping factor is
 * evaluated on the device.  The Courant reduction of the starting state is
 * computed first unless the previous amrv_advance_cfl (all steps taken) or
 * amrv_max_dt already left it for the current state; the state must then
 * not have been changed other than through this API since. */
int amrv_advance_cfl(amrv_forest* f, int32_t nsteps, double t_end, double* t, int32_t* taken);

/* Refinement flags, one int8 per leaf into host memory.
 * AMRV_FLAG_LOHNER (Sec. 1.3): +1 refine (level < max_level and block max
 * estimator > tol), -1 coarsen (level > 1 and max < frac * tol), else 0;
 * emax_out (host, may be NULL) receives each leaf's max estimator.
 * AMRV_FLAG_MLP: the learned flagger's two logits (z_r, z_c): +1 where
 * z_r > 0 (and level < max_level), -1 where z_r <= 0 and z_c > 0 (and
 * level > 1), else 0; emax_out receives z_r (amrv_mlp_logits gives both).
 * Needs amrv_mlp_set_weights.  AMRV_FLAG_MLP_FALLBACK: as AMRV_FLAG_MLP, but
 * leaves with |z_r| < margin or |z_c| < margin (amrv_mlp_set_margin) get the
 * Loehner flag, and emax_out the Loehner maximum for them.  Synchronises. */
int amrv_flag_blocks(amrv_forest* f, int32_t mode, int8_t* flags_out, double* emax_out);

/* ---- learned refinement flagger (a 128-64-64-2 perceptron, bfloat16 MFMA
 * products with binary32 accumulation; not part of the paper, which flags
 * with the Loehner estimator of Sec. 1.3) ----
 * Parameters: 12,546 binary32 values, W1 [64][128], b1 [64], W2 [64][64],
 * b2 [64], W3 [2][64], b3 [2]; output 0 is the refine logit (trained on
 * Loehner's block maximum > tol), output 1 the coarsen logit (maximum <
 * frac * tol).  Features of a leaf: the means of rho and p over 64
 * sub-blocks (4^3 cells in 3D, 2^2 in 2D), each divided by the leaf's mean of
 * them minus one, as bfloat16 bit patterns [128] (rho first). */
#define AMRV_MLP_NPARAM 12546
#define AMRV_MLP_NIN 128
int amrv_mlp_set_weights(amrv_forest* f, const float* w_host, int64_t n);
int amrv_mlp_set_margin(amrv_forest* f, float margin);
/* Features of the current state, [nleaves][128] bfloat16 bits; out is host
 * (on_device = 0, synchronises) or device memory. */
int amrv_mlp_features(amrv_forest* f, uint16_t* out, int32_t on_device);
/* enable != 0: the last stage of every step also pools the flagger's
 * features of its result (the same sums, in the same order, as
 * amrv_mlp_features), so that the next AMRV_FLAG_MLP / AMRV_FLAG_MLP_FALLBACK
 * flagging of that state runs only the network.  3D hydrodynamic forests on
 * the combined stage-kernel variant with minmod, van Leer or MC; elsewhere
 * the flaggings compute the features as before.  Disabled by default. */
int amrv_mlp_fuse_features(amrv_forest* f, int32_t enable);
/* The logits of the last AMRV_FLAG_MLP / AMRV_FLAG_MLP_FALLBACK flagging,
 * [nleaves][2] binary32 (refine, coarsen) into host memory.  Synchronises. */
int amrv_mlp_logits(amrv_forest* f, float* out);

typedef struct {
  float lr, beta1, beta2, eps;  /* Adam (binary32) */
  float pos_weight;             /* weight of the refine output's positive samples in its loss */
  float pos_weight_c;           /* weight of the coarsen output's positive samples in its loss */
  int32_t t0;                   /* Adam steps already taken */
} amrv_train_cfg;
/* Device scratch bytes of amrv_mlp_train for batch size `batch`. */
size_t amrv_mlp_train_workspace_bytes(int32_t batch);
/* nbatch optimisation steps on device data, all pointers device memory:
 * X [n][128] bfloat16 features, y [n] labels (Loehner's class: +1 refine,
 * -1 coarsen, 0 keep; the targets of the refine and coarsen outputs), order
 * [n] sample order (batch b uses order[b*batch .. b*batch+batch-1]; the
 * caller draws the permutation), w [12,546] binary32 master weights updated
 * in place, m and v [12,546] Adam moments.  The loss of a sample is the sum
 * of both outputs' class-weighted binary cross-entropies.  Steps first_batch .. first_batch+nbatch-1; a last
 * partial batch is padded with zero-weight rows.  loss (may be NULL):
 * per-batch mean loss, indexed by batch number.  grad (may be NULL): the last
 * step's gradient.  batch must be a positive multiple of 32 <= 4096.
 * Asynchronous on the stream. */
int amrv_mlp_train(const uint16_t* X, const float* y, const int32_t* order, int64_t n, int32_t batch,
                   int32_t first_batch, int32_t nbatch, float* w, float* m, float* v, const amrv_train_cfg* cfg,
                   void* d_workspace, size_t ws_bytes, void* hip_stream, float* loss, float* grad);

/* amrv_mlp_train without the workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid hipMalloc).  Same arguments,
 * arithmetic and results as amrv_mlp_train; the scratch lives in a
 * library-held static device array of amrv_mlp_train_workspace_bytes(4096)
 * bytes (about 6.1 MiB), one per GPU, resolved on the first call on a
 * device and kept until the process ends.  batch <= 4096 (larger:
 * AMRV_ENOMEM).  The call allocates nothing: no hipMalloc, no hipFree.
 * Every call on one GPU shares that GPU's scratch and leaves its contents
 * behind; each call overwrites every scratch value before reading it, so
 * nothing needs clearing, but calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.
 * Asynchronous on the stream. */
int amrv_mlp_train_noalloc(const uint16_t* X, const float* y, const int32_t* order, int64_t n, int32_t batch,
                           int32_t first_batch, int32_t nbatch, float* w, float* m, float* v,
                           const amrv_train_cfg* cfg, void* hip_stream, float* loss, float* grad);

/* Regrid plan (Sec. 1.3: refinement ratio 2; a block is refined when one of
 * its cells exceeds the tolerance and coarsened when all of them lie below a
 * fraction of it).  Host-only, reads no device data.
 * flags: host int8[nleaves] as from amrv_flag_blocks (+1 split, 0 keep,
 *   -1 merge).  A leaf flagged +1 below max_level is split into its 2^ndim
 *   children; a complete group of 2^ndim sibling leaves, all flagged -1 and
 *   above level 1, is merged into its parent.  2:1 balance over faces, edges
 *   and corners is kept by also splitting every leaf that touches a split
 *   leaf from one level coarser (until nothing changes), and by keeping a
 *   group whose parent would touch a leaf ending more than one level finer
 *   (other merges not counted).
 * Order of the new list: unchanged leaves in place, a split leaf replaced by
 *   its children (child index ox + 2 oy + 4 oz), a merged group by its parent
 *   at the position of the group's first member; a Morton-ordered forest
 *   stays Morton ordered.
 * new_level [capacity], new_ijk [capacity][3]: host arrays owned by the
 *   caller; *new_n receives the new leaf count.  If it exceeds capacity,
 *   nothing else is written and AMRV_ENOMEM is returned (query with
 *   capacity 0 first). */
int amrv_regrid_plan(const amrv_forest* f, const int8_t* flags, int64_t capacity, int64_t* new_n,
                     int32_t* new_level, int32_t* new_ijk);
/* The same plan for a leaf list given on the host (cfg, n, level, ijk as
 * for amrv_forest_create), without a forest or a GPU. */
int amrv_regrid_plan_leaves(const amrv_config* cfg, int64_t nleaves, const int32_t* leaf_level,
                            const int32_t* leaf_ijk, const int8_t* flags, int64_t capacity, int64_t* new_n,
                            int32_t* new_level, int32_t* new_ijk);
/* Move the current state U^n of `from` onto `to`, a forest created (same
 * configuration, its own workspace) on a one-level regrid of `from`'s leaves
 * (e.g. the list of amrv_regrid_plan).  A leaf of `to` that is a leaf of
 * `from` is copied; a child of a leaf of `from` gets the parent cell plus a
 * quarter of its minmod-limited slope per dimension, added on the cell's
 * upper half (conservative linear prolongation, the parent's ghost cells at
 * its boundary); a parent of 2^ndim leaves of `from` gets the pairwise-tree
 * sum of its children's cells times 2^-ndim (restriction).  Runs on both
 * forests' streams and returns after the transfer has completed; `from` is
 * unchanged apart from its ghost slabs.  AMRV_EINVAL if the configurations
 * differ or a leaf of `to` has no source. */
int amrv_regrid_transfer(amrv_forest* from, amrv_forest* to);

/* Select the schedule of the stage update (AMRV_SCHED_*).  xcd_remap != 0
 * keeps consecutive leaves on the same XCD (grid: the workgroup-to-leaf map;
 * persistent: one work queue per XCD over an eighth of the leaves, drained
 * by that XCD's workgroups first); persistent_wgs is the persistent grid size
 * (0 = 2 per compute unit).  The default is AMRV_SCHED_GRID with
 * the remap on, or the result of amrv_autotune. */
int amrv_set_schedule(amrv_forest* f, int32_t sched, int32_t xcd_remap, int32_t persistent_wgs);
int amrv_get_schedule(const amrv_forest* f, int32_t* sched, int32_t* xcd_remap, int32_t* persistent_wgs);

/* Stage-kernel variant for 2D/3D leaves: 0 = x and y share the slope and
 * flux phases (fewer barriers, more LDS), 1 = x then y through one set of
 * LDS arrays (less LDS, more workgroups per compute unit), 2 = (3D MHD
 * forests only; others get AMRV_EINVAL) two launches per stage: the z
 * direction of every column, whose flux divergence goes to a workspace
 * buffer that amrv_workspace_bytes includes for these forests, then the x/y
 * planes with the face states formed in place (no stored slopes), so that
 * each launch fits two workgroups per compute unit.  All give identical
 * results. */
int amrv_set_variant(amrv_forest* f, int32_t variant);
int amrv_get_variant(const amrv_forest* f, int32_t* variant);

/* Arithmetic of the stage update.  AMRV_ARITH_EXACT (the default): every
 * operation correctly rounded, no contraction, in the oracle's order, so
 * results equal the oracle's bit for bit.  AMRV_ARITH_FAST: the combined-
 * variant stage kernels of the 2D/3D hydrodynamic systems (Euler, polytrope;
 * every limiter) with multiply-adds contracted into FMAs, and
 * division, reciprocal, square root and the sound speed sqrt(gamma p/rho)
 * from the hardware reciprocal (square root) estimates refined by Newton
 * steps: each within a few ulp of the correctly rounded value, the stage
 * results within the 1e-10 relative-L1 bar of the oracle, not bit for bit;
 * likewise the two-launch update of 3D MHD forests (variant 2).  Other
 * configurations (1D, 2D MHD, the one-launch MHD kernels, the split variant)
 * run exact in either mode.  Ghost prolongation, the Courant reduction outside
 * the stage kernel and Loehner flags are always exact. */
#define AMRV_ARITH_EXACT 0
#define AMRV_ARITH_FAST 1
int amrv_set_arithmetic(amrv_forest* f, int32_t mode);
int amrv_get_arithmetic(const amrv_forest* f, int32_t* mode);

/* Time the candidate schedules and kernel variants on the current state
 * (first-stage kernel, state unchanged) and keep the fastest.  Synchronises. */
int amrv_autotune(amrv_forest* f, int32_t reps);
/* Text table of the last amrv_autotune: one line per candidate with its
 * median first-stage kernel time.  Valid until the next call on f. */
const char* amrv_autotune_report(const amrv_forest* f);

/* Capture one advance step in a HIP graph and replay it on later
 * amrv_advance calls (enable != 0), or launch kernels directly (0). */
int amrv_use_graph(amrv_forest* f, int32_t enable);

/* Stage-kernel timing: with enable != 0, every batched stage-update launch
 * is bracketed by HIP events on the forest's stream (graph replay is
 * bypassed while enabled).  amrv_profile_read synchronises and returns the
 * summed event time of those launches (ms), their count, and their
 * algorithmic HBM bytes: per launch, the interior state read and written
 * (2 passes in the first stage, 3 in later ones, nvar * 8 bytes per cell
 * and pass).  Reading resets the counters. */
int amrv_profile(amrv_forest* f, int32_t enable);
int amrv_profile_read(amrv_forest* f, double* ms_total, int64_t* launches, double* bytes);

/* Uniform forests (every leaf on one level, so the leaves tile the domain
 * as one grid): copies state variable var (0 <= var < nvar) between the
 * forest's current state and a device grid array of
 * (base_blocks[d] * 2^(level-1) * block_nx) cells per dimension, x fastest
 * (to_grid != 0: forest -> grid; else grid -> forest, which then counts as
 * a new state).  This lets grid solvers act on forest states, e.g. the
 * multigrid divergence control of the MHD runs (Sec. 2.4, amrv_mg.h) on the
 * magnetic field of a uniform MHD forest.  Synchronises.  EINVAL for a
 * forest with leaves on several levels. */
int amrv_uniform_grid_copy(amrv_forest* f, int32_t var, double* grid, int32_t to_grid);

int amrv_synchronize(amrv_forest* f);
const char* amrv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
