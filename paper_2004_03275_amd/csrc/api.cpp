// api.cpp -- the C-ABI of libamrv (declared in include/amrv.h): workspace
// layout, stage scheduling (per-block launches, one grid launch, or persistent
// workgroups on an atomic leaf queue), HIP-graph replay of a whole step, the
// schedule autotuner, and the synchronising queries (max_dt, flag_blocks).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/amrv.h"
#include "errors.hpp"
#include "forest.hpp"
#include "gridcopy.hpp"
#include "regrid.hpp"
#include "internal.hpp"
#include "mlp.hpp"

using namespace amrv;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(AMRV_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                             \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

constexpr size_t ALIGN = 256;

struct Layout {
  size_t off_U[3], off_G, off_FF, off_lvl, off_ijk, off_nbr, off_slot, off_kind, off_fslot, off_sleaf, off_sface,
      off_rlist, off_plist, off_pp, off_lp, off_red, off_cnt, off_emax, off_flags, off_mw, off_mwb, off_mx, off_mz,
      off_munc, off_xfer, off_zd, total;
};

// 3D MHD forests carry a buffer for the z flux divergence of stage-kernel
// variant 2 (one state-sized array)
bool zsplit_capable(const amrv_config& c, const Tables& t) { return c.physics == AMRV_MHD_GLM && t.nd == 3; }

Layout plan(const amrv_config& c, const Tables& t) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += (bytes + ALIGN - 1) / ALIGN * ALIGN;
    return at;
  };
  const size_t state = sizeof(double) * (size_t)t.nvar * (size_t)t.n * (size_t)t.ncell;
  for (int i = 0; i < 3; i++) L.off_U[i] = take(state);
  // three ghost-slab buffers: stage s of a step reads buffer s-1 and, in the
  // 3D combined variant, writes the restriction of its result to buffer s mod S
  L.off_G = take(3 * sizeof(double) * (size_t)std::max(1, t.nslot) * t.nvar * 2 * t.T);
  L.off_FF = take(sizeof(double) * (size_t)std::max(1, t.nslot) * t.nvar * t.T);
  L.off_lvl = take(sizeof(int32_t) * t.n);
  L.off_ijk = take(sizeof(int32_t) * 3 * t.n);
  L.off_nbr = take(sizeof(int32_t) * 6 * t.n);
  L.off_slot = take(sizeof(int32_t) * 6 * t.n);
  L.off_kind = take(sizeof(int8_t) * 6 * t.n);
  L.off_fslot = take(sizeof(int32_t) * 4 * std::max(1, t.nslot));
  L.off_sleaf = take(sizeof(int32_t) * std::max(1, t.nslot));
  L.off_sface = take(sizeof(int32_t) * std::max(1, t.nslot));
  L.off_rlist = take(sizeof(int32_t) * std::max<size_t>(1, t.rlist.size()));
  L.off_plist = take(sizeof(int32_t) * std::max<size_t>(1, t.plist.size()));
  L.off_pp = take(sizeof(double) * PP_COUNT);
  L.off_lp = take(sizeof(double) * LP_COUNT);
  L.off_red = take(sizeof(unsigned long long) * 4);
  L.off_cnt = take(sizeof(unsigned) * CNT_COUNT);
  L.off_emax = take(sizeof(double) * t.n);
  L.off_flags = take(sizeof(int8_t) * t.n);
  L.off_mw = take(sizeof(float) * MLP_NPARAM);
  L.off_mwb = take(sizeof(uint16_t) * MLP_WB_COUNT);
  L.off_mx = take(sizeof(uint16_t) * MLP_NIN * t.n);
  L.off_mz = take(sizeof(float) * MLP_NOUT * t.n);
  L.off_munc = take(sizeof(int8_t) * t.n);
  L.off_xfer = take(sizeof(int32_t) * XFER_STRIDE * t.n);
  L.off_zd = take(zsplit_capable(c, t) ? state : 1);
  L.total = o;
  return L;
}

}  // namespace

namespace amrv {
// the error channel shared with the multigrid entry points (amrv_last_error)
int set_error(int code, const char* msg) { return fail(code, msg); }
}  // namespace amrv

struct amrv_forest {
  amrv_config cfg{};
  Tables tab;
  Layout lay{};
  Geo geo{};
  LaunchCfg lc{};
  hipStream_t st = nullptr;
  char* ws = nullptr;
  double* U[3] = {nullptr, nullptr, nullptr};
  double* pp = nullptr;
  double* lp = nullptr;
  unsigned long long* red = nullptr;
  unsigned* cnt = nullptr;
  double* emax = nullptr;
  int8_t* flags = nullptr;
  int32_t* rlist = nullptr;
  int32_t* plist = nullptr;
  int sched = AMRV_SCHED_GRID, xcd = 1, pwgs = 0, ncu = 256;
  double ch = 0.0;
  bool graph_on = false, graph_valid = false;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t dexec = nullptr;  // device-timed step
  hipGraph_t dgraph = nullptr;
  double dt_tend = 0.0;            // t_end baked into the captured device-timed step
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;  // recorded pairs
  std::vector<hipEvent_t> ev_free;
  double prof_bytes = 0.0;
  bool have_mlp = false;
  float margin = 2.0f;
  std::string tune_report;  // the last autotune's timing table
  std::vector<int32_t> xfer_host;  // regrid sources while their upload is in flight
  bool fold_valid = false;         // the reduction words hold the Courant fold of U^n
  double* Gb[3] = {nullptr, nullptr, nullptr};  // ghost-slab buffers (geo.G = Gb[0])
  bool rvalid = false;             // Gb[0]'s coarse-side slots hold the restriction of U^n
  bool fuse_feat = false;          // the last stage writes the flagger's features (amrv_mlp_fuse_features)
  bool fvalid = false;             // the feature buffer holds the features of U^n
};

namespace {

int set_scalars(amrv_forest* f, int at, const std::vector<double>& v) {
  HIPCHK(launch_set_scalars(f->pp + at, v.data(), (int)v.size(), f->st));
  return AMRV_OK;
}

Sched make_sched(const amrv_forest* f, int mode, int leaf0) {
  Sched s{};
  s.mode = mode;
  s.xcd_remap = f->xcd;
  s.leaf0 = leaf0;
  s.per_xcd = (int)((f->tab.n + 7) / 8);
  s.counter = f->cnt;
  return s;
}

int stage_grid(const amrv_forest* f, int mode) {
  const Tables& t = f->tab;
  if (t.nd == 1) {
    const int nch = (t.nx + 255) / 256;
    return mode == AMRV_SCHED_PER_BLOCK ? nch : (int)(t.n * nch);
  }
  if (mode == AMRV_SCHED_PER_BLOCK) return 1;
  if (mode == AMRV_SCHED_PERSISTENT) return f->pwgs > 0 ? f->pwgs : 2 * f->ncu;
  return f->xcd ? 8 * (int)((t.n + 7) / 8) : (int)t.n;
}

// enqueue the coarse-fine pre-pass on state U into geo's ghost-slab buffer;
// restriction skipped when the buffer already holds it
int enqueue_ghosts(amrv_forest* f, const Geo& geo, const double* U, bool fluxes, bool restrict_too = true) {
  const int nr = (int)f->tab.rlist.size(), np = (int)f->tab.plist.size();
  if (nr && restrict_too) HIPCHK(launch_restrict(geo, f->lc, U, f->rlist, nr, f->st));
  if (np) HIPCHK(launch_prolong(geo, f->lc, U, f->pp, f->plist, np, fluxes, f->st));
  return AMRV_OK;
}

// the stage kernel restricts its own result (3D combined variant, not MHD,
// whose damping of psi after the step would make the restriction stale)
bool fused_restriction(const amrv_forest* f) {
  return f->tab.nd == 3 && f->lc.variant == 0 && f->lc.phys != PH_MHD && !f->tab.rlist.empty();
}

// the last stage writes the learned flagger's features of its result (3D
// combined variant of the hydrodynamic systems)
bool fused_features(const amrv_forest* f) {
  return f->fuse_feat && f->tab.nd == 3 && f->lc.variant == 0 && f->lc.phys != PH_MHD;
}

int enqueue_stage_update(amrv_forest* f, const Geo& geo, const StageArgs& a, int mode) {
  const Tables& t = f->tab;
  int m = mode;
  if (t.nd == 1 && m == AMRV_SCHED_PERSISTENT) m = AMRV_SCHED_GRID;
  if (m == AMRV_SCHED_PER_BLOCK) {
    const int grid = stage_grid(f, m);
    for (int64_t b = 0; b < t.n; b++) {
      Sched s = make_sched(f, 0, (int)b);
      HIPCHK(launch_stage(geo, f->lc, a, f->pp, s, grid, f->st));
    }
    return AMRV_OK;
  }
  Sched s = make_sched(f, m == AMRV_SCHED_PERSISTENT ? 2 : 1, 0);
  if (t.nd == 1) s.xcd_remap = 0;
  if (m == AMRV_SCHED_PERSISTENT) s.counter = f->cnt + 8 * a.stage;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (f->prof) {
    for (hipEvent_t* e : {&e0, &e1}) {
      if (!f->ev_free.empty()) {
        *e = f->ev_free.back();
        f->ev_free.pop_back();
      } else {
        HIPCHK(hipEventCreate(e));
      }
    }
    HIPCHK(hipEventRecord(e0, f->st));
  }
  HIPCHK(launch_stage(geo, f->lc, a, f->pp, s, stage_grid(f, m), f->st));
  if (f->prof) {
    HIPCHK(hipEventRecord(e1, f->st));
    f->ev.emplace_back(e0, e1);
    const double passes = a.stage == 1 ? 2.0 : 3.0;
    f->prof_bytes += passes * 8.0 * (double)t.nvar * (double)t.n * (double)t.ncell;
  }
  return AMRV_OK;
}

// one full SSP step on the forest's stream; dt and the damping factor are
// read from the device parameter block.  fold != null: the last stage folds
// the Courant reduction of the new state into it.  With the fused restriction
// stage s reads ghost-slab buffer s-1 and restricts its result into buffer
// s mod S, so only the first stage after a state change runs the separate
// restriction (assume_valid: the caller guarantees Gb[0] holds it, as before
// a captured step).
int enqueue_step(amrv_forest* f, unsigned long long* fold = nullptr, bool assume_valid = false) {
  const int S = f->cfg.rk_stages;
  const bool fused = fused_restriction(f), feat = fused_features(f);
  if (f->sched == AMRV_SCHED_PERSISTENT && f->tab.nd > 1) HIPCHK(launch_reset_u32(f->cnt, CNT_QUEUES, f->st));
  for (int s = 1; s <= S; s++) {
    const double* in = s == 1 ? f->U[0] : (s == 2 ? f->U[1] : f->U[2]);
    double* out = s == S ? f->U[0] : (s == 1 ? f->U[1] : f->U[2]);
    Geo geo = f->geo;
    if (fused) geo.G = f->Gb[s - 1];
    const bool restrict_too = !fused || (s == 1 && !assume_valid && !f->rvalid);
    int rc = enqueue_ghosts(f, geo, in, true, restrict_too);
    if (rc) return rc;
    StageArgs a{};
    a.Uin = in;
    a.Un = f->U[0];
    a.Uout = out;
    a.dtp = f->pp + PP_DT;
    a.stage = s;
    a.rk = S;
    a.cflred = s == S ? fold : nullptr;
    a.Gw = fused ? f->Gb[s % S] : nullptr;
    a.Xout = feat && s == S ? (uint16_t*)(f->ws + f->lay.off_mx) : nullptr;
    a.Zd = zsplit_capable(f->cfg, f->tab) ? (double*)(f->ws + f->lay.off_zd) : nullptr;
    rc = enqueue_stage_update(f, geo, a, f->sched);
    if (rc) return rc;
  }
  f->rvalid = fused;
  f->fvalid = feat;
  if (f->cfg.physics == AMRV_MHD_GLM) {
    const int ip = 2 + 2 * f->tab.nd;
    double* psi = f->U[0] + (size_t)ip * f->tab.n * f->tab.ncell;
    HIPCHK(launch_scale_var(psi, f->pp + PP_DAMP, (long long)f->tab.n * f->tab.ncell, f->st));
  }
  return AMRV_OK;
}

void drop_graph(amrv_forest* f) {
  if (f->gexec) (void)hipGraphExecDestroy(f->gexec);
  if (f->graph) (void)hipGraphDestroy(f->graph);
  if (f->dexec) (void)hipGraphExecDestroy(f->dexec);
  if (f->dgraph) (void)hipGraphDestroy(f->dgraph);
  f->gexec = nullptr;
  f->graph = nullptr;
  f->dexec = nullptr;
  f->dgraph = nullptr;
  f->graph_valid = false;
}

// a device-timed step: dt from the previous fold, then the step with a fold
int enqueue_device_step(amrv_forest* f, double t_end, bool assume_valid = false) {
  HIPCHK(launch_dt_update(f->red, f->pp, f->pp + PP_T, f->cnt + CNT_ERR, f->cfg.cfl, t_end, f->cfg.glm_cr,
                          f->cfg.physics == AMRV_MHD_GLM, f->st));
  return enqueue_step(f, f->red, assume_valid);
}

// before replaying a captured step (which assumes it): the restriction of
// U^n in ghost-slab buffer 0
int ensure_restricted(amrv_forest* f) {
  if (!fused_restriction(f) || f->rvalid) return AMRV_OK;
  HIPCHK(launch_restrict(f->geo, f->lc, f->U[0], f->rlist, (int)f->tab.rlist.size(), f->st));
  f->rvalid = true;
  return AMRV_OK;
}

int capture_graph(amrv_forest* f) {
  drop_graph(f);
  HIPCHK(hipStreamBeginCapture(f->st, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_step(f, nullptr, true);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(f->st, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  f->graph = g;
  HIPCHK(hipGraphInstantiate(&f->gexec, g, nullptr, nullptr, 0));
  f->graph_valid = true;
  return AMRV_OK;
}

// The tables of the last amrv_workspace_bytes call on this thread, kept for
// the amrv_forest_create call that normally follows with the same leaf list
// (the pair is how a caller sizes and then creates a forest; building the
// tables once saves a pass over the leaves).  Reused only on an exact match
// of the configuration and the leaf arrays.
struct TableCache {
  bool valid = false;
  amrv_config cfg{};
  std::vector<int32_t> lev, ijk;
  Tables tab;
};
thread_local TableCache g_tables;

bool cache_matches(const amrv_config& c, int64_t n, const int32_t* lev, const int32_t* ijk) {
  const TableCache& k = g_tables;
  return k.valid && std::memcmp(&k.cfg, &c, sizeof c) == 0 && (int64_t)k.lev.size() == n && lev && ijk &&
         std::memcmp(k.lev.data(), lev, sizeof(int32_t) * (size_t)n) == 0 &&
         std::memcmp(k.ijk.data(), ijk, sizeof(int32_t) * 3 * (size_t)n) == 0;
}

}  // namespace

extern "C" {

const char* amrv_last_error(void) { return g_err.c_str(); }

size_t amrv_workspace_bytes(const amrv_config* cfg, int64_t n, const int32_t* lev, const int32_t* ijk) {
  if (!cfg) {
    g_err = "null config";
    return 0;
  }
  g_tables.valid = false;
  Tables t;
  const int rc = build_tables(*cfg, n, lev, ijk, t);
  if (rc) {
    g_err = t.err;
    return 0;
  }
  const size_t total = plan(*cfg, t).total;
  g_tables.cfg = *cfg;
  g_tables.lev.assign(lev, lev + n);
  g_tables.ijk.assign(ijk, ijk + 3 * n);
  g_tables.tab = std::move(t);
  g_tables.valid = true;
  return total;
}

int amrv_forest_create(const amrv_config* cfg, int64_t n, const int32_t* lev, const int32_t* ijk, void* d_ws,
                       size_t ws_bytes, void* stream, amrv_forest** out) {
  if (!cfg || !out) return fail(AMRV_EINVAL, "null argument");
  *out = nullptr;
  amrv_forest* f = new amrv_forest();
  f->cfg = *cfg;
  int rc = AMRV_OK;
  if (cache_matches(*cfg, n, lev, ijk)) {
    f->tab = std::move(g_tables.tab);
    g_tables.valid = false;
  } else {
    rc = build_tables(*cfg, n, lev, ijk, f->tab);
  }
  if (rc) {
    std::string m = f->tab.err;
    delete f;
    return fail(rc, m);
  }
  f->lay = plan(f->cfg, f->tab);
  if (!d_ws) {
    delete f;
    return fail(AMRV_EINVAL, "null workspace");
  }
  if (ws_bytes < f->lay.total) {
    delete f;
    return fail(AMRV_ENOMEM, "workspace too small: need " + std::to_string(f->lay.total) + " bytes");
  }
  if (((uintptr_t)d_ws) % ALIGN) {
    delete f;
    return fail(AMRV_EINVAL, "workspace must be 256-byte aligned");
  }
  f->st = (hipStream_t)stream;
  f->ws = (char*)d_ws;
  const Tables& t = f->tab;
  const Layout& L = f->lay;
  for (int i = 0; i < 3; i++) f->U[i] = (double*)(f->ws + L.off_U[i]);
  f->pp = (double*)(f->ws + L.off_pp);
  f->lp = (double*)(f->ws + L.off_lp);
  f->red = (unsigned long long*)(f->ws + L.off_red);
  f->cnt = (unsigned*)(f->ws + L.off_cnt);
  f->emax = (double*)(f->ws + L.off_emax);
  f->flags = (int8_t*)(f->ws + L.off_flags);
  f->rlist = (int32_t*)(f->ws + L.off_rlist);
  f->plist = (int32_t*)(f->ws + L.off_plist);

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&f->ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    delete f;
    return hip_fail(e, "device query");
  }

  Geo& g = f->geo;
  g.n = (int)t.n;
  g.ndim = t.nd;
  g.nx = t.nx;
  g.ncell = t.ncell;
  g.T = t.T;
  g.nslot = t.nslot;
  g.nvar = t.nvar;
  g.lvl = (const int32_t*)(f->ws + L.off_lvl);
  g.ijk = (const int32_t*)(f->ws + L.off_ijk);
  g.nbr = (const int32_t*)(f->ws + L.off_nbr);
  g.slot = (const int32_t*)(f->ws + L.off_slot);
  g.kind = (const int8_t*)(f->ws + L.off_kind);
  g.fslot = (const int32_t*)(f->ws + L.off_fslot);
  g.sleaf = (const int32_t*)(f->ws + L.off_sleaf);
  g.sface = (const int32_t*)(f->ws + L.off_sface);
  g.G = (double*)(f->ws + L.off_G);
  for (int i = 0; i < 3; i++) f->Gb[i] = g.G + (size_t)i * std::max(1, t.nslot) * t.nvar * 2 * t.T;
  g.FF = (double*)(f->ws + L.off_FF);
  for (int l = 0; l < MAXLEV; l++)
    for (int d = 0; d < 3; d++) {
      g.rdx[l][d] = 0.0;
      if (d < t.nd && l >= 1 && l <= cfg->max_level) {
        const double cells = (double)(((int64_t)cfg->base_blocks[d] << (l - 1)) * cfg->block_nx[d]);
        const double dx = (cfg->xmax[d] - cfg->xmin[d]) / cells;
        g.rdx[l][d] = 1.0 / dx;
      }
    }
  f->lc.ndim = t.nd;
  static_assert(AMRV_EULER == PH_EULER && AMRV_MHD_GLM == PH_MHD && AMRV_POLYTROPE == PH_POLY, "physics codes");
  f->lc.phys = cfg->physics;
  f->lc.flux = cfg->flux;
  f->lc.lim = cfg->limiter;
  f->lc.variant = 0;
  f->lc.arith = AMRV_ARITH_EXACT;

  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    if (!bytes) return hipSuccess;
    return hipMemcpyAsync(f->ws + off, src, bytes, hipMemcpyHostToDevice, f->st);
  };
  const size_t nsl = (size_t)t.nslot;
  double pp[PP_COUNT] = {0};
  pp[PP_GAMMA] = cfg->gamma;
  pp[PP_GM1] = cfg->gamma - 1.0;
  pp[PP_IGM1] = 1.0 / (cfg->gamma - 1.0);
  pp[PP_CAD] = cfg->cad;
  pp[PP_GCAD] = cfg->gamma * cfg->cad;
  for (int l = 1; l <= cfg->max_level && l < MAXLEV; l++)
    for (int d = 0; d < t.nd; d++)
      if (cfg->cada_radius > 0.0) {
        const double cells = (double)(((int64_t)cfg->base_blocks[d] << (l - 1)) * cfg->block_nx[d]);
        const double rd = cfg->cada_radius * ((cfg->xmax[d] - cfg->xmin[d]) / cells);
        pp[PP_CTHR + 3 * l + d] = rd * rd;
      }
  double lp[LP_COUNT] = {0};
  lp[LP_EPS] = cfg->lohner_eps;
  lp[LP_WRHO] = cfg->lohner_w_rho;
  lp[LP_WP] = cfg->lohner_w_p;
  lp[LP_TOL] = cfg->lohner_tol;
  lp[LP_CTOL] = cfg->lohner_coarsen_frac * cfg->lohner_tol;
  hipError_t es[] = {up(L.off_lvl, t.lvl.data(), 4 * t.n),
                     up(L.off_ijk, t.ijk.data(), 12 * t.n),
                     up(L.off_nbr, t.nbr.data(), 24 * t.n),
                     up(L.off_slot, t.slot.data(), 24 * t.n),
                     up(L.off_kind, t.kind.data(), 6 * t.n),
                     up(L.off_fslot, t.fslot.data(), 16 * nsl),
                     up(L.off_sleaf, t.sleaf.data(), 4 * nsl),
                     up(L.off_sface, t.sface.data(), 4 * nsl),
                     up(L.off_rlist, t.rlist.data(), 4 * t.rlist.size()),
                     up(L.off_plist, t.plist.data(), 4 * t.plist.size()),
                     up(L.off_pp, pp, sizeof pp),
                     up(L.off_lp, lp, sizeof lp),
                     hipStreamSynchronize(f->st)};
  for (hipError_t x : es)
    if (x != hipSuccess) {
      delete f;
      return hip_fail(x, "table upload");
    }
  *out = f;
  return AMRV_OK;
}

int amrv_forest_destroy(amrv_forest* f) {
  if (!f) return AMRV_OK;
  drop_graph(f);
  delete f;
  return AMRV_OK;
}

int amrv_nvar(const amrv_forest* f) { return f ? f->tab.nvar : 0; }

int64_t amrv_state_doubles(const amrv_forest* f) {
  return f ? (int64_t)f->tab.nvar * f->tab.n * f->tab.ncell : 0;
}

int amrv_set_state(amrv_forest* f, const double* U, int64_t nd, int32_t on_device) {
  if (!f || !U) return fail(AMRV_EINVAL, "null argument");
  if (nd != amrv_state_doubles(f)) return fail(AMRV_EINVAL, "state size mismatch");
  HIPCHK(hipMemcpyAsync(f->U[0], U, sizeof(double) * nd, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        f->st));
  if (!on_device) HIPCHK(hipStreamSynchronize(f->st));
  f->fold_valid = false;
  f->rvalid = false;
  f->fvalid = false;
  return AMRV_OK;
}

int amrv_uniform_grid_copy(amrv_forest* f, int32_t var, double* grid, int32_t to_grid) {
  if (!f || !grid) return fail(AMRV_EINVAL, "null argument");
  if (var < 0 || var >= f->tab.nvar) return fail(AMRV_EINVAL, "variable out of range");
  const int nd = f->tab.nd, l0 = f->tab.lvl[0];
  for (int64_t b = 0; b < f->tab.n; b++)
    if (f->tab.lvl[b] != l0) return fail(AMRV_EINVAL, "the forest is not uniform (leaves on several levels)");
  int ext[3] = {1, 1, 1};
  for (int d = 0; d < nd; d++) ext[d] = (f->cfg.base_blocks[d] << (l0 - 1)) * f->tab.nx;
  double* Uvar = f->U[0] + (size_t)var * f->tab.n * f->tab.ncell;
  HIPCHK(launch_grid_copy(Uvar, grid, f->geo.ijk, (int)f->tab.n, nd, f->tab.nx, f->tab.ncell, ext[0], ext[1],
                          to_grid ? 1 : 0, f->st));
  if (!to_grid) {
    f->fold_valid = false;
    f->rvalid = false;
    f->fvalid = false;
  }
  HIPCHK(hipStreamSynchronize(f->st));
  return AMRV_OK;
}

int amrv_get_state(amrv_forest* f, double* U, int64_t nd, int32_t on_device) {
  if (!f || !U) return fail(AMRV_EINVAL, "null argument");
  if (nd != amrv_state_doubles(f)) return fail(AMRV_EINVAL, "state size mismatch");
  HIPCHK(hipMemcpyAsync(U, f->U[0], sizeof(double) * nd, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        f->st));
  if (!on_device) HIPCHK(hipStreamSynchronize(f->st));
  return AMRV_OK;
}

int amrv_max_dt(amrv_forest* f, double* dt_out) {
  if (!f || !dt_out) return fail(AMRV_EINVAL, "null argument");
  HIPCHK(launch_reset_u32((unsigned*)f->red, 8, f->st));
  HIPCHK(launch_cfl(f->geo, f->lc, f->U[0], f->pp, f->red, f->st));
  unsigned long long h[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(h, f->red, sizeof h, hipMemcpyDeviceToHost, f->st));
  HIPCHK(hipStreamSynchronize(f->st));
  f->fold_valid = true;
  if (h[2]) return fail(AMRV_ENONPHYSICAL, "non-physical state (rho <= 0, p <= 0 or NaN)");
  double smax, cmax;
  std::memcpy(&smax, &h[0], 8);
  std::memcpy(&cmax, &h[1], 8);
  if (!(smax > 0.0)) return fail(AMRV_ENONPHYSICAL, "zero signal speed");
  f->ch = cmax;
  int rc = set_scalars(f, PP_CH, {cmax});
  if (rc) return rc;
  *dt_out = f->cfg.cfl / smax;
  return AMRV_OK;
}

double amrv_glm_ch(const amrv_forest* f) { return f ? f->ch : 0.0; }

int amrv_advance(amrv_forest* f, double dt) {
  if (!f) return fail(AMRV_EINVAL, "null forest");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(AMRV_EINVAL, "dt must be positive and finite");
  if (f->cfg.physics == AMRV_MHD_GLM && !(f->ch > 0.0)) return fail(AMRV_EINVAL, "MHD needs amrv_max_dt first");
  const double damp = f->cfg.physics == AMRV_MHD_GLM ? std::exp(-(dt * f->ch) / f->cfg.glm_cr) : 1.0;
  f->fold_valid = false;
  int rc = set_scalars(f, PP_DT, {dt, damp});
  if (rc) return rc;
  if (f->graph_on && !f->prof) {
    rc = ensure_restricted(f);
    if (rc) return rc;
    if (!f->graph_valid) {
      rc = capture_graph(f);
      if (rc) return rc;
    }
    HIPCHK(hipGraphLaunch(f->gexec, f->st));
    f->rvalid = fused_restriction(f);
    f->fvalid = fused_features(f);
    return AMRV_OK;
  }
  return enqueue_step(f);
}

int amrv_advance_cfl(amrv_forest* f, int32_t nsteps, double t_end, double* t, int32_t* taken) {
  if (!f || !t) return fail(AMRV_EINVAL, "null argument");
  if (nsteps < 0) return fail(AMRV_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(*t) || std::isnan(t_end)) return fail(AMRV_EINVAL, "bad time");
  // initial fold: the Courant reduction of the current state, unless the
  // last step of the previous call (or amrv_max_dt) left it in place
  HIPCHK(launch_reset_u32(f->cnt + CNT_ERR, 2, f->st));
  int rc = set_scalars(f, PP_T, {*t});
  if (rc) return rc;
  if (!f->fold_valid) {
    HIPCHK(launch_reset_u32((unsigned*)f->red, 8, f->st));
    HIPCHK(launch_cfl(f->geo, f->lc, f->U[0], f->pp, f->red, f->st));
  }
  f->fold_valid = false;
  const bool graph = f->st != nullptr && f->sched != AMRV_SCHED_PER_BLOCK && !f->prof;
  if (graph) {
    rc = ensure_restricted(f);
    if (rc) return rc;
  }
  if (graph && (!f->dexec || f->dt_tend != t_end)) {
    if (f->dexec) (void)hipGraphExecDestroy(f->dexec);
    if (f->dgraph) (void)hipGraphDestroy(f->dgraph);
    f->dexec = nullptr;
    f->dgraph = nullptr;
    HIPCHK(hipStreamBeginCapture(f->st, hipStreamCaptureModeThreadLocal));
    rc = enqueue_device_step(f, t_end, true);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(f->st, &gr);
    if (rc) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    f->dgraph = gr;
    HIPCHK(hipGraphInstantiate(&f->dexec, gr, nullptr, nullptr, 0));
    f->dt_tend = t_end;
  }
  for (int i = 0; i < nsteps; i++) {
    if (graph) {
      HIPCHK(hipGraphLaunch(f->dexec, f->st));
      f->rvalid = fused_restriction(f);
      f->fvalid = fused_features(f);
    } else {
      rc = enqueue_device_step(f, t_end);
      if (rc) return rc;
    }
  }
  double th = 0.0;
  unsigned cw[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(&th, f->pp + PP_T, sizeof th, hipMemcpyDeviceToHost, f->st));
  HIPCHK(hipMemcpyAsync(cw, f->cnt + CNT_ERR, sizeof cw, hipMemcpyDeviceToHost, f->st));
  HIPCHK(hipStreamSynchronize(f->st));
  *t = th;
  if (taken) *taken = (int32_t)cw[1];
  // every step folded the Courant reduction of its result: it stays valid
  f->fold_valid = (int64_t)cw[1] == (int64_t)nsteps && !cw[0];
  // the GLM speed of the latest fold (the next amrv_advance needs it)
  if (f->cfg.physics == AMRV_MHD_GLM) {
    double ch = 0.0;
    HIPCHK(hipMemcpy(&ch, f->pp + PP_CH, sizeof ch, hipMemcpyDeviceToHost));
    f->ch = ch;
  }
  if (cw[0]) return fail(AMRV_ENONPHYSICAL, "non-physical state during a device-timed run");
  return AMRV_OK;
}

int amrv_flag_blocks(amrv_forest* f, int32_t mode, int8_t* flags_out, double* emax_out) {
  if (!f || !flags_out) return fail(AMRV_EINVAL, "null argument");
  if (mode != AMRV_FLAG_LOHNER && mode != AMRV_FLAG_MLP && mode != AMRV_FLAG_MLP_FALLBACK)
    return fail(AMRV_EINVAL, "unknown flag mode");
  const int n = (int)f->tab.n;
  const int8_t* only = nullptr;
  if (mode != AMRV_FLAG_LOHNER) {
    if (!f->have_mlp) return fail(AMRV_EINVAL, "flag mode needs amrv_mlp_set_weights");
    if (f->tab.nd < 2) return fail(AMRV_ENOTSUP, "the learned flagger is defined for 2D and 3D leaves");
    uint16_t* X = (uint16_t*)(f->ws + f->lay.off_mx);
    float* z = (float*)(f->ws + f->lay.off_mz);
    int8_t* unc = (int8_t*)(f->ws + f->lay.off_munc);
    if (!(f->fvalid && fused_features(f))) HIPCHK(launch_mlp_features(f->geo, f->lc, f->U[0], f->pp, X, f->st));
    HIPCHK(launch_mlp_infer(X, n, (const uint16_t*)(f->ws + f->lay.off_mwb), (const float*)(f->ws + f->lay.off_mw), z,
                            f->geo.lvl, f->cfg.max_level, f->margin, f->flags,
                            mode == AMRV_FLAG_MLP_FALLBACK ? unc : nullptr, f->emax, f->st));
    if (mode == AMRV_FLAG_MLP_FALLBACK) only = unc;
  }
  if (mode != AMRV_FLAG_MLP) {
    int rc = enqueue_ghosts(f, f->geo, f->U[0], false);
    f->rvalid = true;  // buffer 0 now restricts U^n
    if (rc) return rc;
    HIPCHK(launch_lohner(f->geo, f->lc, f->U[0], f->pp, f->lp, f->cfg.max_level, f->emax, f->flags, only, f->st));
  }
  HIPCHK(hipMemcpyAsync(flags_out, f->flags, n, hipMemcpyDeviceToHost, f->st));
  if (emax_out) HIPCHK(hipMemcpyAsync(emax_out, f->emax, sizeof(double) * n, hipMemcpyDeviceToHost, f->st));
  HIPCHK(hipStreamSynchronize(f->st));
  return AMRV_OK;
}

int amrv_mlp_set_weights(amrv_forest* f, const float* w, int64_t n) {
  if (!f || !w) return fail(AMRV_EINVAL, "null argument");
  if (n != MLP_NPARAM) return fail(AMRV_EINVAL, "expected 12546 parameters");
  float* dw = (float*)(f->ws + f->lay.off_mw);
  HIPCHK(hipMemcpyAsync(dw, w, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, f->st));
  HIPCHK(launch_mlp_prep(dw, (uint16_t*)(f->ws + f->lay.off_mwb), f->st));
  HIPCHK(hipStreamSynchronize(f->st));
  f->have_mlp = true;
  return AMRV_OK;
}

int amrv_mlp_set_margin(amrv_forest* f, float margin) {
  if (!f) return fail(AMRV_EINVAL, "null forest");
  if (!(margin >= 0.0f)) return fail(AMRV_EINVAL, "margin must be >= 0");
  f->margin = margin;
  return AMRV_OK;
}

int amrv_mlp_features(amrv_forest* f, uint16_t* out, int32_t on_device) {
  if (!f || !out) return fail(AMRV_EINVAL, "null argument");
  if (f->tab.nd < 2) return fail(AMRV_ENOTSUP, "features are defined for 2D and 3D leaves");
  uint16_t* X = (uint16_t*)(f->ws + f->lay.off_mx);
  HIPCHK(launch_mlp_features(f->geo, f->lc, f->U[0], f->pp, X, f->st));
  const size_t bytes = sizeof(uint16_t) * MLP_NIN * (size_t)f->tab.n;
  HIPCHK(hipMemcpyAsync(out, X, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, f->st));
  if (!on_device) HIPCHK(hipStreamSynchronize(f->st));
  return AMRV_OK;
}

int amrv_mlp_fuse_features(amrv_forest* f, int32_t enable) {
  if (!f) return fail(AMRV_EINVAL, "null forest");
  f->fuse_feat = enable != 0;
  f->fvalid = false;
  drop_graph(f);
  return AMRV_OK;
}

int amrv_mlp_logits(amrv_forest* f, float* out) {
  if (!f || !out) return fail(AMRV_EINVAL, "null argument");
  HIPCHK(hipMemcpyAsync(out, f->ws + f->lay.off_mz, sizeof(float) * MLP_NOUT * f->tab.n, hipMemcpyDeviceToHost,
                        f->st));
  HIPCHK(hipStreamSynchronize(f->st));
  return AMRV_OK;
}

size_t amrv_mlp_train_workspace_bytes(int32_t batch) {
  if (batch <= 0 || batch % 32 || batch > 4096) {
    g_err = "batch must be a positive multiple of 32 <= 4096";
    return 0;
  }
  return mlp_train_scratch_bytes(batch);
}

namespace {
// argument checks shared by both training entry points
int check_train_args(const uint16_t* X, const float* y, const int32_t* order, int64_t n, int32_t batch,
                     int32_t first_batch, int32_t nbatch, const float* w, const float* m, const float* v,
                     const amrv_train_cfg* cfg) {
  if (!X || !y || !order || !w || !m || !v || !cfg) return fail(AMRV_EINVAL, "null argument");
  if (n <= 0 || n > (1 << 30)) return fail(AMRV_EINVAL, "bad sample count");
  if (batch <= 0 || batch % 32 || batch > 4096) return fail(AMRV_EINVAL, "batch must be a positive multiple of 32 <= 4096");
  const int64_t nb_total = (n + batch - 1) / batch;
  if (first_batch < 0 || nbatch < 0 || first_batch + nbatch > nb_total) return fail(AMRV_EINVAL, "batch range outside the data");
  if (!(cfg->lr >= 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
      !(cfg->eps > 0.0f) || !(cfg->pos_weight > 0.0f) || !(cfg->pos_weight_c > 0.0f) || cfg->t0 < 0)
    return fail(AMRV_EINVAL, "bad training hyper-parameters");
  return AMRV_OK;
}
}  // namespace

int amrv_mlp_train(const uint16_t* X, const float* y, const int32_t* order, int64_t n, int32_t batch,
                   int32_t first_batch, int32_t nbatch, float* w, float* m, float* v, const amrv_train_cfg* cfg,
                   void* ws, size_t ws_bytes, void* stream, float* loss, float* grad) {
  int rc = check_train_args(X, y, order, n, batch, first_batch, nbatch, w, m, v, cfg);
  if (rc) return rc;
  if (!ws) return fail(AMRV_EINVAL, "null argument");
  if (ws_bytes < mlp_train_scratch_bytes(batch)) return fail(AMRV_ENOMEM, "training workspace too small");
  if (((uintptr_t)ws) % 256) return fail(AMRV_EINVAL, "workspace must be 256-byte aligned");
  TrainHyper hp{cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, cfg->pos_weight, cfg->pos_weight_c};
  HIPCHK(launch_mlp_train(X, y, order, (int)n, batch, first_batch, nbatch, w, m, v, hp, cfg->t0, ws, loss, grad,
                          (hipStream_t)stream));
  return AMRV_OK;
}

int amrv_mlp_train_noalloc(const uint16_t* X, const float* y, const int32_t* order, int64_t n, int32_t batch,
                           int32_t first_batch, int32_t nbatch, float* w, float* m, float* v,
                           const amrv_train_cfg* cfg, void* stream, float* loss, float* grad) {
  int rc = check_train_args(X, y, order, n, batch, first_batch, nbatch, w, m, v, cfg);
  if (rc) return rc;
  if (mlp_train_scratch_bytes(batch) > MLP_STATIC_SCRATCH_BYTES)
    return fail(AMRV_ENOMEM, "batch needs more than the library's training scratch");
  void* ws = nullptr;
  HIPCHK(mlp_static_scratch(&ws));
  TrainHyper hp{cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, cfg->pos_weight, cfg->pos_weight_c};
  HIPCHK(launch_mlp_train(X, y, order, (int)n, batch, first_batch, nbatch, w, m, v, hp, cfg->t0, ws, loss, grad,
                          (hipStream_t)stream));
  return AMRV_OK;
}

int amrv_regrid_plan(const amrv_forest* f, const int8_t* flags, int64_t capacity, int64_t* new_n,
                     int32_t* new_level, int32_t* new_ijk) {
  if (!f || !flags || !new_n || capacity < 0 || (capacity > 0 && (!new_level || !new_ijk)))
    return fail(AMRV_EINVAL, "null argument");
  std::vector<int32_t> lev, ijk;
  std::string err;
  const int rc = regrid_plan(f->cfg, f->tab, flags, lev, ijk, err);
  if (rc) return fail(rc, err);
  *new_n = (int64_t)lev.size();
  if (*new_n > capacity)
    return fail(AMRV_ENOMEM, "capacity " + std::to_string(capacity) + " below the new leaf count " +
                                 std::to_string(*new_n));
  std::copy(lev.begin(), lev.end(), new_level);
  std::copy(ijk.begin(), ijk.end(), new_ijk);
  return AMRV_OK;
}

int amrv_regrid_plan_leaves(const amrv_config* cfg, int64_t n, const int32_t* lev, const int32_t* ijk,
                            const int8_t* flags, int64_t capacity, int64_t* new_n, int32_t* new_level,
                            int32_t* new_ijk) {
  if (!cfg || !flags || !new_n || capacity < 0 || (capacity > 0 && (!new_level || !new_ijk)))
    return fail(AMRV_EINVAL, "null argument");
  Tables t;
  int rc = build_tables(*cfg, n, lev, ijk, t);
  if (rc) return fail(rc, t.err);
  std::vector<int32_t> nl, nijk;
  std::string err;
  rc = regrid_plan(*cfg, t, flags, nl, nijk, err);
  if (rc) return fail(rc, err);
  *new_n = (int64_t)nl.size();
  if (*new_n > capacity)
    return fail(AMRV_ENOMEM, "capacity " + std::to_string(capacity) + " below the new leaf count " +
                                 std::to_string(*new_n));
  std::copy(nl.begin(), nl.end(), new_level);
  std::copy(nijk.begin(), nijk.end(), new_ijk);
  return AMRV_OK;
}

int amrv_regrid_transfer(amrv_forest* from, amrv_forest* to) {
  if (!from || !to || from == to) return fail(AMRV_EINVAL, "two distinct forests are needed");
  const amrv_config &a = from->cfg, &b = to->cfg;
  bool same = a.ndim == b.ndim && a.physics == b.physics && a.max_level == b.max_level;
  for (int d = 0; d < 3; d++)
    same = same && a.block_nx[d] == b.block_nx[d] && a.base_blocks[d] == b.base_blocks[d] && a.bc[d][0] == b.bc[d][0];
  if (!same) return fail(AMRV_EINVAL, "the two forests differ in their configuration");
  std::string err;
  int rc = regrid_sources(from->tab, to->tab, to->xfer_host, err);
  if (rc) return fail(rc, err);
  int32_t* xf = (int32_t*)(to->ws + to->lay.off_xfer);
  // ghost slabs of the source state (coarse-fine faces), then the transfer
  rc = enqueue_ghosts(from, from->geo, from->U[0], false);
  from->rvalid = true;
  to->rvalid = false;
  to->fvalid = false;
  if (rc) return rc;
  if (from->st != to->st) HIPCHK(hipStreamSynchronize(from->st));
  HIPCHK(hipMemcpyAsync(xf, to->xfer_host.data(), sizeof(int32_t) * to->xfer_host.size(), hipMemcpyHostToDevice,
                        to->st));
  HIPCHK(launch_transfer(from->geo, from->U[0], to->geo, to->U[0], xf, to->lc, to->st));
  to->fold_valid = false;
  HIPCHK(hipStreamSynchronize(to->st));
  to->ch = from->ch;
  return AMRV_OK;
}

int amrv_set_schedule(amrv_forest* f, int32_t sched, int32_t xcd_remap, int32_t pwgs) {
  if (!f) return fail(AMRV_EINVAL, "null forest");
  if (sched < AMRV_SCHED_PER_BLOCK || sched > AMRV_SCHED_PERSISTENT) return fail(AMRV_EINVAL, "unknown schedule");
  if (pwgs < 0 || pwgs > 1 << 20) return fail(AMRV_EINVAL, "bad persistent grid size");
  f->sched = sched;
  f->xcd = xcd_remap ? 1 : 0;
  f->pwgs = pwgs;
  drop_graph(f);
  return AMRV_OK;
}

int amrv_get_schedule(const amrv_forest* f, int32_t* sched, int32_t* xcd, int32_t* pwgs) {
  if (!f || !sched || !xcd || !pwgs) return fail(AMRV_EINVAL, "null argument");
  *sched = f->sched;
  *xcd = f->xcd;
  *pwgs = f->pwgs;
  return AMRV_OK;
}

int amrv_set_variant(amrv_forest* f, int32_t variant) {
  if (!f) return fail(AMRV_EINVAL, "null forest");
  if (variant < 0 || variant > 2) return fail(AMRV_EINVAL, "unknown stage-kernel variant");
  if (variant == 2 && !zsplit_capable(f->cfg, f->tab))
    return fail(AMRV_EINVAL, "stage-kernel variant 2 is the two-launch update of 3D MHD forests");
  f->lc.variant = variant;
  drop_graph(f);
  return AMRV_OK;
}

int amrv_set_arithmetic(amrv_forest* f, int32_t mode) {
  if (!f) return fail(AMRV_EINVAL, "null forest");
  if (mode != AMRV_ARITH_EXACT && mode != AMRV_ARITH_FAST) return fail(AMRV_EINVAL, "unknown arithmetic mode");
  f->lc.arith = mode;
  drop_graph(f);
  return AMRV_OK;
}

int amrv_get_arithmetic(const amrv_forest* f, int32_t* mode) {
  if (!f || !mode) return fail(AMRV_EINVAL, "null argument");
  *mode = f->lc.arith;
  return AMRV_OK;
}

int amrv_get_variant(const amrv_forest* f, int32_t* variant) {
  if (!f || !variant) return fail(AMRV_EINVAL, "null argument");
  *variant = f->lc.variant;
  return AMRV_OK;
}

int amrv_autotune(amrv_forest* f, int32_t reps) {
  if (!f) return fail(AMRV_EINVAL, "null forest");
  if (reps < 1) reps = 3;
  struct Cand {
    int sched, xcd, pwgs, var;
  };
  std::vector<Cand> cands;
  std::vector<int> vars = f->tab.nd > 1 ? std::vector<int>{0, 1} : std::vector<int>{0};
  if (zsplit_capable(f->cfg, f->tab)) vars.push_back(2);
  for (int var : vars) {
    cands.push_back({AMRV_SCHED_GRID, 0, 0, var});
    cands.push_back({AMRV_SCHED_GRID, 1, 0, var});
    if (f->tab.nd > 1)
      for (int x : {0, 1})
        for (int k : {2, 3, 4}) cands.push_back({AMRV_SCHED_PERSISTENT, x, k * f->ncu, var});
  }
  const int s0 = f->sched, x0 = f->xcd, p0 = f->pwgs, v0 = f->lc.variant;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // time the first stage U^n -> U^(1) as a step runs it (coarse-fine
  // pre-pass, with the separate restriction where the kernel does not fuse
  // it, and the stage update, writing the fused restriction into ghost-slab
  // buffer 1 as stage 1 does); it writes only the stage buffer and ghost
  // slabs, so the state is untouched (dt must be > 0: dt = 0 marks a
  // finished run)
  int rc = set_scalars(f, PP_DT, {1.0e-12, 1.0});
  double best = 1e300;
  std::string report;
  Cand bc = {s0, x0, p0, v0};
  for (const Cand& c : cands) {
    if (rc) break;
    f->sched = c.sched;
    f->xcd = c.xcd;
    f->pwgs = c.pwgs;
    f->lc.variant = c.var;
    const bool fused = fused_restriction(f);
    StageArgs a{};
    a.Uin = f->U[0];
    a.Un = f->U[0];
    a.Uout = f->U[1];
    a.dtp = f->pp + PP_DT;
    a.stage = 1;
    a.rk = f->cfg.rk_stages;
    a.Gw = fused ? f->Gb[1] : nullptr;
    a.Zd = zsplit_capable(f->cfg, f->tab) ? (double*)(f->ws + f->lay.off_zd) : nullptr;
    std::vector<float> ts;
    for (int r = 0; r < reps + 1 && !rc; r++) {
      if (c.sched == AMRV_SCHED_PERSISTENT) {
        hipError_t e = launch_reset_u32(f->cnt, CNT_QUEUES, f->st);
        if (e != hipSuccess) rc = hip_fail(e, "reset");
      }
      (void)hipEventRecord(e0, f->st);
      if (!rc) rc = enqueue_ghosts(f, f->geo, f->U[0], true, !fused);
      if (!rc) rc = enqueue_stage_update(f, f->geo, a, c.sched);
      (void)hipEventRecord(e1, f->st);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (r) ts.push_back(ms);
    }
    if (rc) break;
    std::sort(ts.begin(), ts.end());
    const double med = ts[ts.size() / 2];
    char line[160];
    snprintf(line, sizeof line, "sched=%d xcd=%d wgs=%d variant=%d: median %.4f ms (min %.4f)\n", c.sched, c.xcd,
             c.pwgs, c.var, med, (double)ts.front());
    report += line;
    if (med < best) {
      best = med;
      bc = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  f->sched = bc.sched;
  f->xcd = bc.xcd;
  f->pwgs = bc.pwgs;
  f->lc.variant = bc.var;
  f->tune_report = report;
  drop_graph(f);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(f->st));
  return AMRV_OK;
}

const char* amrv_autotune_report(const amrv_forest* f) { return f ? f->tune_report.c_str() : ""; }

int amrv_use_graph(amrv_forest* f, int32_t enable) {
  if (!f) return fail(AMRV_EINVAL, "null forest");
  if (enable && f->st == nullptr) return fail(AMRV_EINVAL, "graph capture needs a non-default stream");
  if (enable && f->sched == AMRV_SCHED_PER_BLOCK) return fail(AMRV_EINVAL, "graphs replay the batched schedules only");
  f->graph_on = enable != 0;
  drop_graph(f);
  return AMRV_OK;
}

int amrv_profile(amrv_forest* f, int32_t enable) {
  if (!f) return fail(AMRV_EINVAL, "null forest");
  f->prof = enable != 0;
  return AMRV_OK;
}

int amrv_profile_read(amrv_forest* f, double* ms_total, int64_t* launches, double* bytes) {
  if (!f || !ms_total || !launches || !bytes) return fail(AMRV_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(f->st));
  double tot = 0.0;
  for (auto& pr : f->ev) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
    tot += ms;
    f->ev_free.push_back(pr.first);
    f->ev_free.push_back(pr.second);
  }
  *ms_total = tot;
  *launches = (int64_t)f->ev.size();
  *bytes = f->prof_bytes;
  f->ev.clear();
  f->prof_bytes = 0.0;
  return AMRV_OK;
}

int amrv_synchronize(amrv_forest* f) {
  if (!f) return fail(AMRV_EINVAL, "null forest");
  HIPCHK(hipStreamSynchronize(f->st));
  return AMRV_OK;
}

}  // extern "C"
