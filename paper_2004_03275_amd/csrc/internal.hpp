// internal.hpp -- device tables and kernel launch interface of libamrv.
//
// Data layout in HBM (all inside the caller's workspace):
//   state   U[var][leaf][z][y][x]           binary64, interior cells only (3 copies:
//                                           U^n, U^(1), U^(2) of the SSP stages)
//   tables  per leaf: level, block coords, per face: neighbour kind / index /
//           coarse-fine slot (int32 / int8)
//   slabs   G[slot][var][layer][t]          ghost cells of coarse-fine faces only
//                                           (restricted on the coarse side,
//                                           prolonged on the fine side)
//           FF[slot][var][t]                fine-side face fluxes of coarse-fine faces
//   where t = a2 * NB + a1 indexes the face's transverse cells (a1 along the
//   lower-numbered transverse axis).  Same-level and boundary ghosts are never
//   stored: kernels read them from the neighbour's (or own) interior.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amrv {

enum { NB_SAME = 0, NB_COARSER = 1, NB_FINER = 2, NB_BND = 3 };
constexpr int MAXLEV = 16;

struct Geo {
  int n;          // leaves
  int ndim;
  int nx;         // cells per block per dimension (16 in 2D/3D; 1D: any even >= 4)
  int ncell;      // cells per block
  int T;          // transverse cells per face slab
  int nslot;      // coarse-fine face slots
  int nvar;
  const int32_t* lvl;    // [n]
  const int32_t* ijk;    // [n][3]
  const int32_t* nbr;    // [n][6] same-level or coarser neighbour, own index at a boundary
  const int8_t* kind;    // [n][6] NB_*
  const int32_t* slot;   // [n][6] coarse-fine slot or -1
  const int32_t* fslot;  // [nslot][4] FINER slots: the fine leaves' slots, transverse order
  const int32_t* sleaf;  // [nslot] leaf owning the slot
  const int32_t* sface;  // [nslot] face of the slot
  double* G;             // [nslot][nvar][2][T]
  double* FF;            // [nslot][nvar][T]
  double rdx[MAXLEV][3]; // 1/dx per level and dimension
};

struct Sched {
  int mode;            // 0 per-block launch, 1 grid, 2 persistent
  int xcd_remap;       // map consecutive leaves onto one XCD
  int leaf0;           // per-block mode: the leaf
  int per_xcd;         // ceil(n / 8) for the remap
  unsigned* counter;   // persistent work queues of this stage: [0] the global queue, or with
                       // xcd_remap [x] the queue of XCD x over leaves [x*per_xcd, (x+1)*per_xcd)
};

struct StageArgs {
  const double* Uin;   // stage input U^(s-1)
  const double* Un;    // step initial state U^n
  double* Uout;        // stage output
  const double* dtp;   // device-resident dt
  int stage;           // 1..rk
  int rk;              // 2 or 3
  unsigned long long* cflred;  // last stage: fold the Courant reduction of the new state here (or null)
  double* Gw;          // 3D combined variant: restrict the stage output onto the coarse neighbours'
                       // ghost slabs of this buffer (the G layout), or null
  uint16_t* Xout;      // 3D combined variant, last stage: the learned flagger's features of the
                       // stage output [n][128] bfloat16 bits, or null
  double* Zd;          // variant 2 (3D MHD): the z flux divergence of every cell (the state
                       // layout), written by the z-column launch and read by the x/y launch
};

struct Kernels;  // forward

// physics: Euler (energy equation), ideal MHD with GLM cleaning, and the
// polytrope p = c_ad rho^gamma without energy equation (shallow water for
// rho = h, c_ad = 1/2, gamma = 2); the values of AMRV_EULER, AMRV_MHD_GLM and
// AMRV_POLYTROPE
enum { PH_EULER = 0, PH_MHD = 1, PH_POLY = 2 };

// launchers (kernels.hip)
struct LaunchCfg {
  int ndim, phys, flux, lim;  // phys: PH_EULER, PH_MHD or PH_POLY
  int variant;  // stage kernel: 0 combined x/y phases, 1 split x then y, 2 (3D MHD) z columns, then x/y
  int arith;    // 0 correctly rounded (default), 1 fast arithmetic where the stage kernel has that form
};

hipError_t launch_restrict(const Geo& g, const LaunchCfg& c, const double* U, const int32_t* list, int nlist,
                           hipStream_t st);
// fine-side ghost slabs (prolongation) and, with fluxes, the fine-side face
// fluxes of the same coarse-fine faces
hipError_t launch_prolong(const Geo& g, const LaunchCfg& c, const double* U, const double* physp,
                          const int32_t* list, int nlist, bool fluxes, hipStream_t st);
hipError_t launch_stage(const Geo& g, const LaunchCfg& c, const StageArgs& a, const double* physp, const Sched& s,
                        int grid, hipStream_t st);
hipError_t launch_cfl(const Geo& g, const LaunchCfg& c, const double* U, const double* physp,
                      unsigned long long* red, hipStream_t st);
hipError_t launch_lohner(const Geo& g, const LaunchCfg& c, const double* U, const double* physp,
                         const double* lohp, int max_level, double* emax, int8_t* flags, const int8_t* only,
                         hipStream_t st);
// regrid: state of the leaves of `to` from the state Uf of `from` (whose
// coarse-fine ghost slabs must hold Uf's ghosts); xfer[n_to][9] per new leaf:
// how (0 copy, 1 prolong from the parent, 2 restrict the children) and sources
hipError_t launch_transfer(const Geo& from, const double* Uf, const Geo& to, double* Ut, const int32_t* xfer,
                           const LaunchCfg& c, hipStream_t st);
hipError_t launch_set_scalars(double* dst, const double* src_host_vals, int n, hipStream_t st);
hipError_t launch_reset_u32(unsigned* p, int n, hipStream_t st);
hipError_t launch_scale_var(double* U, const double* facp, long long count, hipStream_t st);
// device-side time step from a Courant reduction: dt = min(cfl / smax, t_end - t),
// t += dt, c_h and the GLM damping factor into the parameter block, then the
// reduction words are cleared for the next fold
hipError_t launch_dt_update(unsigned long long* red, double* pp, double* t, unsigned* err, double cfl, double t_end,
                            double glm_cr, int mhd, hipStream_t st);
// device counters: [8s .. 8s+7] the work queues of stage s = 1..3 (cleared
// before every step), [CNT_ERR] non-physical flag, [CNT_TAKEN] steps taken
constexpr int CNT_QUEUES = 32, CNT_ERR = 40, CNT_TAKEN = 41, CNT_COUNT = 64;

// device parameter block (written once per forest, plus dt / ch per step)
// layout: [0] gamma [1] gm1 [2] igm1 [3] ch [4] dt [5] glm damping factor
// [6] time [7] c_ad [8] gamma * c_ad; from [16]: (r dx)^2 of Cada's smoothness
// switch per level and dimension, [16 + 3 l + d] (0: none)
constexpr int PP_GAMMA = 0, PP_GM1 = 1, PP_IGM1 = 2, PP_CH = 3, PP_DT = 4, PP_DAMP = 5, PP_T = 6, PP_CAD = 7,
              PP_GCAD = 8, PP_CTHR = 16, PP_COUNT = PP_CTHR + 3 * MAXLEV;
// Loehner parameters: [0] eps [1] w_rho [2] w_p [3] tol [4] coarsen tol
constexpr int LP_EPS = 0, LP_WRHO = 1, LP_WP = 2, LP_TOL = 3, LP_CTOL = 4, LP_COUNT = 8;

}  // namespace amrv
