/* orc.c -- plain, slow CPU oracle of the block-forest finite-volume update.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, the smoke check and the CPU
 * baseline of bench.py; never by the product library.  It shares no code with
 * the HIP path.  Every function states the passage of arXiv 2004.03275
 * (MPI-AMRVAC) it follows, or the reading taken where the paper is silent.
 *
 * Structure of one step (readings of Sec. 1.3 and Sec. 2.1-2.4):
 *   for every Runge-Kutta stage
 *     1. ghost fill of each leaf from the stage input: same-level copy, fine to
 *        coarse restriction, physical boundary, then coarse to fine
 *        prolongation from the coarse leaf's filled cells;
 *     2. per leaf and direction: primitive variables, limited MUSCL face
 *        states, approximate Riemann flux at every face;
 *     3. at a coarse face next to finer leaves the coarse flux is replaced by
 *        the mean of the fine face fluxes of the same stage (conservation);
 *     4. flux divergence and the SSP Runge-Kutta combination.
 *   then (MHD) GLM damping of psi.
 *
 * Formula order is fixed and written out; the build uses -ffp-contract=off.
 */
#include "orc.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EUNBALANCED (-2)
#define ORC_ENONPHYSICAL (-3)
#define ORC_ENOMEM (-4)

#define NVMAX 9

enum { NB_SAME = 0, NB_COARSER = 1, NB_FINER = 2, NB_BND = 3 };
enum { PHYS_EULER = 0, PHYS_MHD = 1, PHYS_POLY = 2 };
enum { FLUX_TVDLF = 0, FLUX_HLL = 1, FLUX_HLLC = 2 };
enum { LIM_MINMOD = 0, LIM_VANLEER = 1, LIM_MC = 2, LIM_KOREN = 3, LIM_CADA = 4 };

static __thread char g_err[512];

static int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

const char* orc_last_error(void) { return g_err; }

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

struct orc_forest {
  orc_config c;
  int nd, nvar, ng, mhd, poly;
  int64_t n;
  int32_t* lev;
  int32_t* ijk;
  int nx[3], gs[3], px[3];
  int64_t ncell, npad;
  uint64_t* hkey;
  int64_t* hval;
  uint64_t hmask;
  int32_t* kind;   /* [n][6] neighbour kind per face */
  int64_t* nbr;    /* [n][6] same-level or coarser neighbour leaf, else -1 */
  double* U;       /* current state, [var][leaf][cell] */
  double* U1;      /* Runge-Kutta stage buffers */
  double* U2;
  double** ffine;  /* [n*6] fine-side boundary flux slab at coarse-fine faces */
  double ch;       /* GLM cleaning speed from the last max_dt */
};

/* ------------------------------------------------------------------ */
/* leaf lookup: open-addressing hash of (level, i, j, k)               */
/* ------------------------------------------------------------------ */

static uint64_t key_of(int l, int64_t i, int64_t j, int64_t k) {
  return ((uint64_t)l << 60) | ((uint64_t)i << 40) | ((uint64_t)j << 20) | (uint64_t)k;
}

static uint64_t mix(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

static int64_t lookup(const orc_forest* f, int l, const int64_t c[3]) {
  if (l < 1 || l > 15) return -1;
  for (int d = 0; d < 3; d++)
    if (c[d] < 0 || c[d] >= (1 << 20)) return -1;
  uint64_t k = key_of(l, c[0], c[1], c[2]) + 1;
  uint64_t h = mix(k) & f->hmask;
  while (f->hkey[h]) {
    if (f->hkey[h] == k) return f->hval[h];
    h = (h + 1) & f->hmask;
  }
  return -1;
}

static int insert(orc_forest* f, int l, const int64_t c[3], int64_t v) {
  uint64_t k = key_of(l, c[0], c[1], c[2]) + 1;
  uint64_t h = mix(k) & f->hmask;
  while (f->hkey[h]) {
    if (f->hkey[h] == k) return 0; /* duplicate */
    h = (h + 1) & f->hmask;
  }
  f->hkey[h] = k;
  f->hval[h] = v;
  return 1;
}

/* blocks per dimension at level l (Sec. 1.3: refinement ratio 2) */
static int64_t nblk(const orc_forest* f, int l, int d) {
  if (d >= f->nd) return 1;
  return (int64_t)f->c.base_blocks[d] << (l - 1);
}

/* cells per dimension of the whole domain at level l */
static int64_t ncells_dom(const orc_forest* f, int l, int d) {
  return nblk(f, l, d) * f->nx[d];
}

static int periodic(const orc_forest* f, int d) { return f->c.bc[d][0] == 0; }

/* wrap a global block or cell coordinate periodically; returns 0 if the
 * coordinate lies outside a non-periodic domain */
static int wrap(const orc_forest* f, int d, int64_t* x, int64_t extent) {
  if (*x >= 0 && *x < extent) return 1;
  if (!periodic(f, d)) return 0;
  *x = ((*x % extent) + extent) % extent;
  return 1;
}

/* ------------------------------------------------------------------ */
/* physics: Sec. 1.1 (HD variables), Sec. 1.2 (primitive conversion,   */
/* fluxes, signal speeds), ideal MHD with mu0 = 1 (Sec. 2.4)           */
/* ------------------------------------------------------------------ */

/* index of energy / pressure; magnetic field; psi */
static int iE(const orc_forest* f) { return 1 + f->nd; }
static int iB(const orc_forest* f) { return 2 + f->nd; }
static int iPsi(const orc_forest* f) { return 2 + 2 * f->nd; }

/* Polytropic closure without an energy equation (Sec. 2.2): p = c_ad rho^gamma,
 * c^2 = gamma c_ad rho^(gamma-1); with rho = h, c_ad = 1/2, gamma = 2 these
 * are the shallow water equations.  The exponents 0, 1 and 2 are exact
 * (rho^2 = rho*rho); others go through pow. */
static double rpow(double r, double e) { return e == 1.0 ? r : e == 2.0 ? r * r : pow(r, e); }
static double poly_p(const orc_forest* f, double rho) { return f->c.cad * rpow(rho, f->c.gamma); }

/* phys_to_primitive: v = m / rho (via 1/rho), p = (gamma-1)(E - m.m/(2 rho) [- B.B/2]);
 * the polytrope's primitive vector is (rho, v) (its pressure follows from rho) */
static void to_prim(const orc_forest* f, const double* u, double* v) {
  const int nd = f->nd;
  const double gm1 = f->c.gamma - 1.0;
  double rho = u[0];
  double inv = 1.0 / rho;
  double mm = 0.0;
  v[0] = rho;
  for (int d = 0; d < nd; d++) {
    v[1 + d] = u[1 + d] * inv;
    mm = mm + u[1 + d] * u[1 + d];
  }
  if (f->poly) return;
  if (!f->mhd) {
    v[iE(f)] = gm1 * (u[iE(f)] - 0.5 * mm * inv);
  } else {
    double bb = 0.0;
    for (int d = 0; d < nd; d++) {
      bb = bb + u[iB(f) + d] * u[iB(f) + d];
      v[iB(f) + d] = u[iB(f) + d];
    }
    v[iE(f)] = gm1 * (u[iE(f)] - 0.5 * mm * inv - 0.5 * bb);
    v[iPsi(f)] = u[iPsi(f)];
  }
}

/* phys_to_conserved: m = rho v, E = p/(gamma-1) + rho v.v/2 [+ B.B/2];
 * 1/(gamma-1) is formed once and multiplied. */
static void to_cons(const orc_forest* f, const double* v, double* u) {
  const int nd = f->nd;
  const double igm1 = 1.0 / (f->c.gamma - 1.0);
  double rho = v[0];
  double vv = 0.0;
  u[0] = rho;
  for (int d = 0; d < nd; d++) {
    u[1 + d] = rho * v[1 + d];
    vv = vv + v[1 + d] * v[1 + d];
  }
  if (f->poly) return;
  if (!f->mhd) {
    u[iE(f)] = v[iE(f)] * igm1 + 0.5 * rho * vv;
  } else {
    double bb = 0.0;
    for (int d = 0; d < nd; d++) {
      bb = bb + v[iB(f) + d] * v[iB(f) + d];
      u[iB(f) + d] = v[iB(f) + d];
    }
    u[iE(f)] = v[iE(f)] * igm1 + 0.5 * rho * vv + 0.5 * bb;
    u[iPsi(f)] = v[iPsi(f)];
  }
}

/* phys_get_flux in direction n (Sec. 1.1-1.2).  HD: F = v_n U + p (0, e_n, v_n).
 * MHD: total pressure p + B^2/2, Maxwell stress -B B_n, induction v_n B - B_n v.
 * The normal-field and psi components are supplied by the GLM face solve. */
static void phys_flux(const orc_forest* f, const double* v, const double* u, int n, double* F) {
  const int nd = f->nd;
  const double vn = v[1 + n];
  F[0] = u[1 + n];
  if (f->poly) {
    const double p = poly_p(f, v[0]);
    for (int d = 0; d < nd; d++) {
      F[1 + d] = u[1 + d] * vn;
      if (d == n) F[1 + d] = F[1 + d] + p;
    }
    return;
  }
  const double p = v[iE(f)];
  if (!f->mhd) {
    for (int d = 0; d < nd; d++) {
      F[1 + d] = u[1 + d] * vn;
      if (d == n) F[1 + d] = F[1 + d] + p;
    }
    F[iE(f)] = (u[iE(f)] + p) * vn;
  } else {
    const double* B = v + iB(f);
    double bb = 0.0, vB = 0.0;
    for (int d = 0; d < nd; d++) {
      bb = bb + B[d] * B[d];
      vB = vB + v[1 + d] * B[d];
    }
    double pt = p + 0.5 * bb;
    for (int d = 0; d < nd; d++) {
      F[1 + d] = u[1 + d] * vn - B[d] * B[n];
      if (d == n) F[1 + d] = F[1 + d] + pt;
    }
    F[iE(f)] = (u[iE(f)] + pt) * vn - B[n] * vB;
    for (int d = 0; d < nd; d++) F[iB(f) + d] = (d == n) ? 0.0 : B[d] * vn - B[n] * v[1 + d];
    F[iPsi(f)] = 0.0;
  }
}

/* phys_get_cmax (Sec. 1.2): HD sound speed sqrt(gamma p / rho); MHD fast
 * magnetosonic speed in direction n; the polytrope's sqrt(gamma c_ad rho^(gamma-1)). */
static double speed(const orc_forest* f, const double* v, int n) {
  const double g = f->c.gamma;
  if (f->poly) return sqrt(g * f->c.cad * rpow(v[0], g - 1.0));
  if (!f->mhd) return sqrt(g * v[iE(f)] / v[0]);
  const int nd = f->nd;
  double irho = 1.0 / v[0];
  double bb = 0.0;
  for (int d = 0; d < nd; d++) bb = bb + v[iB(f) + d] * v[iB(f) + d];
  double a2 = g * v[iE(f)] * irho;
  double b2 = bb * irho;
  double bn2 = v[iB(f) + n] * v[iB(f) + n] * irho;
  double s = a2 + b2;
  double disc = s * s - 4.0 * a2 * bn2;
  if (!(disc > 0.0)) disc = 0.0;
  return sqrt(0.5 * (s + sqrt(disc)));
}

static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

/* Approximate Riemann flux across a face normal to n with left/right
 * primitive states (Sec. 1.2 phys_get_cbounds; TVDLF, HLL, HLLC of Sec. 1.2,
 * 2.2, 2.4).  Readings: Rusanov speed max(|v_n|+c) over the two states; Davis
 * wave-speed estimates for HLL/HLLC; HLLC star states of the Toro textbook
 * with the branch order S_L>=0, S_M>=0, S_R>0.  MHD (HLL/TVDLF only) uses the
 * mixed GLM face solve of Dedner et al. for the normal field and psi. */
static void riemann(const orc_forest* f, const double* vl_in, const double* vr_in, int n,
                    double* F) {
  const int nv = f->nvar;
  double vl[NVMAX], vr[NVMAX], ul[NVMAX], ur[NVMAX], fl[NVMAX], fr[NVMAX];
  memcpy(vl, vl_in, sizeof(double) * nv);
  memcpy(vr, vr_in, sizeof(double) * nv);
  double bns = 0.0, psis = 0.0;
  const double ch = f->ch;
  if (f->mhd) {
    const int ib = iB(f) + n, ip = iPsi(f);
    bns = 0.5 * (vl[ib] + vr[ib]) - 0.5 * (vr[ip] - vl[ip]) / ch;
    psis = 0.5 * (vl[ip] + vr[ip]) - 0.5 * ch * (vr[ib] - vl[ib]);
    vl[ib] = bns;
    vr[ib] = bns;
  }
  to_cons(f, vl, ul);
  to_cons(f, vr, ur);
  phys_flux(f, vl, ul, n, fl);
  phys_flux(f, vr, ur, n, fr);
  const double cl = speed(f, vl, n), cr = speed(f, vr, n);
  const double unl = vl[1 + n], unr = vr[1 + n];

  if (f->c.flux == FLUX_TVDLF) {
    double cmax = dmax(fabs(unl) + cl, fabs(unr) + cr);
    for (int k = 0; k < nv; k++) F[k] = 0.5 * ((fl[k] + fr[k]) - cmax * (ur[k] - ul[k]));
  } else if (f->c.flux == FLUX_HLL) {
    double sl = dmin(unl - cl, unr - cr);
    double sr = dmax(unl + cl, unr + cr);
    if (sl >= 0.0) {
      for (int k = 0; k < nv; k++) F[k] = fl[k];
    } else if (sr <= 0.0) {
      for (int k = 0; k < nv; k++) F[k] = fr[k];
    } else {
      double ids = 1.0 / (sr - sl);
      for (int k = 0; k < nv; k++)
        F[k] = ((sr * fl[k] - sl * fr[k]) + (sl * sr) * (ur[k] - ul[k])) * ids;
    }
  } else if (f->mhd) {
    /* HLLC for MHD, after Li (2005) as cited by the paper (Sec. 2.4): total
     * pressure p_T = p + B.B/2 in the contact speed and the star pressure,
     * normal field B_n from the GLM sub-solve on both sides; in the star
     * region the transverse velocity and field come from the HLL state
     * (the same on both sides), or, where B_n = 0, from the side's own
     * velocity and its field compressed like the density; star energy
     * E* = ((S_K - u_K) E_K - p_TK u_K + p_T* S_M + B_n (v_K.B_K - v*.B*)) / (S_K - S_M). */
    const int ie = iE(f), ib = iB(f), nd = f->nd;
    double sl = dmin(unl - cl, unr - cr);
    double sr = dmax(unl + cl, unr + cr);
    if (sl >= 0.0) {
      for (int k = 0; k < nv; k++) F[k] = fl[k];
    } else if (sr <= 0.0) {
      for (int k = 0; k < nv; k++) F[k] = fr[k];
    } else {
      double bbl = vl[ib] * vl[ib], bbr = vr[ib] * vr[ib];
      for (int d = 1; d < nd; d++) {
        bbl = bbl + vl[ib + d] * vl[ib + d];
        bbr = bbr + vr[ib + d] * vr[ib + d];
      }
      double ptl = vl[ie] + 0.5 * bbl, ptr = vr[ie] + 0.5 * bbr;
      double rl = vl[0] * (sl - unl);
      double rr = vr[0] * (sr - unr);
      double sm = ((ptr - ptl) + unl * rl - unr * rr) / (rl - rr);
      double ids = 1.0 / (sr - sl);
      double uh[NVMAX]; /* HLL state: density, momenta, field */
      for (int k = 0; k <= nd; k++) uh[k] = ((sr * ur[k] - sl * ul[k]) - (fr[k] - fl[k])) * ids;
      for (int d = 0; d < nd; d++)
        uh[ib + d] = ((sr * ur[ib + d] - sl * ul[ib + d]) - (fr[ib + d] - fl[ib + d])) * ids;
      const int left = sm >= 0.0;
      const double* vk = left ? vl : vr;
      const double* uk = left ? ul : ur;
      const double* fk = left ? fl : fr;
      double sk = left ? sl : sr;
      double rk = left ? rl : rr;
      double unk = vk[1 + n], ptk = left ? ptl : ptr;
      double inv = 1.0 / (sk - sm);
      double coef = rk * inv;
      double pts = ptk + rk * (sm - unk);
      double bn = bns;
      double vs[3] = {0.0, 0.0, 0.0}, bs[3] = {0.0, 0.0, 0.0};
      for (int d = 0; d < nd; d++) {
        if (d == n) {
          vs[d] = sm;
          bs[d] = bn;
        } else if (bn == 0.0) {
          vs[d] = vk[1 + d];
          bs[d] = vk[ib + d] * ((sk - unk) * inv);
        } else {
          vs[d] = uh[1 + d] / uh[0];
          bs[d] = uh[ib + d];
        }
      }
      double vbk = vk[1] * vk[ib], vbs = vs[0] * bs[0];
      for (int d = 1; d < nd; d++) {
        vbk = vbk + vk[1 + d] * vk[ib + d];
        vbs = vbs + vs[d] * bs[d];
      }
      double us[NVMAX];
      us[0] = coef;
      for (int d = 0; d < nd; d++) {
        us[1 + d] = coef * vs[d];
        us[ib + d] = bs[d];
      }
      us[ie] = ((sk - unk) * uk[ie] - ptk * unk + pts * sm + bn * (vbk - vbs)) * inv;
      us[iPsi(f)] = uk[iPsi(f)];
      for (int k = 0; k < nv; k++) F[k] = fk[k] + sk * (us[k] - uk[k]);
    }
  } else { /* HLLC, hydrodynamics */
    const int ie = iE(f);
    double sl = dmin(unl - cl, unr - cr);
    double sr = dmax(unl + cl, unr + cr);
    double pl = vl[ie], pr = vr[ie];
    double rl = vl[0] * (sl - unl);
    double rr = vr[0] * (sr - unr);
    double sm = ((pr - pl) + unl * rl - unr * rr) / (rl - rr);
    if (sl >= 0.0) {
      for (int k = 0; k < nv; k++) F[k] = fl[k];
    } else if (sm >= 0.0 || sr > 0.0) {
      const int left = sm >= 0.0;
      const double* vk = left ? vl : vr;
      const double* uk = left ? ul : ur;
      const double* fk = left ? fl : fr;
      double sk = left ? sl : sr;
      double rk = left ? rl : rr; /* rho_K (S_K - u_K) */
      double unk = vk[1 + n], pk = vk[ie];
      /* star state U*_K = rho_K (S_K - u_K)/(S_K - S_M) (1, S_M, v_t, .) with
       * the energy in the star-pressure form p* = p_K + rho_K (S_K - u_K)(S_M - u_K),
       * E* = ((S_K - u_K) E_K - p_K u_K + p* S_M) / (S_K - S_M) */
      double inv = 1.0 / (sk - sm);
      double coef = rk * inv;
      double ps = pk + rk * (sm - unk);
      double us[NVMAX];
      us[0] = coef;
      for (int d = 0; d < f->nd; d++) us[1 + d] = (d == n) ? coef * sm : coef * vk[1 + d];
      us[ie] = ((sk - unk) * uk[ie] - pk * unk + ps * sm) * inv;
      for (int k = 0; k < nv; k++) F[k] = fk[k] + sk * (us[k] - uk[k]);
    } else {
      for (int k = 0; k < nv; k++) F[k] = fr[k];
    }
  }
  if (f->mhd) {
    F[iB(f) + n] = psis;
    F[iPsi(f)] = ch * ch * bns;
  }
}

/* Limited slope of a cell toward one of its faces, from the difference a
 * on the side away from that face and the difference b toward it (the paper
 * names minmod-type and other limited reconstructions, Sec. 2.2-2.4, with the
 * textbook formulas): minmod picks the smaller magnitude, van Leer the
 * harmonic mean 2ab/(a+b), the monotonized central limiter of Sec. 2.3.1
 * ('woodward') the smallest in magnitude of 2a, the central difference
 * (a+b)/2 and 2b, Koren's limiter (Sec. 2.2, 2.3.2) the smallest of 2a, the
 * third-order (kappa = 1/3) combination (a+2b)/3 and 2b.  All vanish at
 * extrema (a b <= 0).  The first three are symmetric in a and b; Koren's is
 * not, so a cell's two faces get different slopes.
 *
 * Cada's third-order limiter (Sec. 2.4 MHD blast runs; Cada and Torrilhon
 * 2009, the limited function 'LimO3'): with theta = a/b the slope is
 * b H(theta), H(theta) = max(0, min(p3, max(-theta/2, min(2 theta, p3,
 * 1.6)))) and p3 = (2 + theta)/3 the unlimited third-order value.  It is
 * not zero at extrema (-2 < theta < 0) and not symmetric.  With the
 * smoothness switch of that paper (radius r > 0), the unlimited third-order
 * slope (a + 2b)/3 is taken where a^2 + b^2 <= (r dx)^2 (the switch without
 * its blending width); thr2 = (r dx)^2, 0 for no switch.  Written here
 * without the division: for b > 0 every candidate of H times b is a
 * candidate in a and b (p3 b = (a + 2b)/3), and b < 0 follows from
 * s(-a, -b) = -s(a, b); b = 0 gives 0 (H is bounded), and so does a = 0
 * (H(0) = 0).  The smoothness switch above applies only for thr2 > 0
 * (cada_radius > 0); with thr2 = 0 the limited function is used alone. */
static double smaller(double x, double y) { return y < x ? y : x; }
static double larger(double x, double y) { return y > x ? y : x; }

static double cada(double a, double b, double thr2) {
  if (a == 0.0 && b == 0.0) return 0.0; /* flat: every branch gives 0 */
  if (thr2 > 0.0 && a * a + b * b <= thr2) return (a + 2.0 * b) / 3.0;
  if (a == 0.0 || b == 0.0) return 0.0; /* H bounded, H(0) = 0 */
  const double sg = b > 0.0 ? 1.0 : -1.0;
  const double ap = sg * a, bp = sg * b;
  const double p3 = (ap + 2.0 * bp) / 3.0;
  const double in = smaller(smaller(2.0 * ap, p3), 1.6 * bp);
  const double r = larger(0.0, smaller(p3, larger(-0.5 * ap, in)));
  return sg * r;
}

static double limit_ab(int kind, double a, double b, double thr2) {
  if (kind == LIM_CADA) return cada(a, b, thr2);
  if (a * b <= 0.0) return 0.0;
  if (kind == LIM_MINMOD) return fabs(a) < fabs(b) ? a : b;
  if (kind == LIM_MC || kind == LIM_KOREN) {
    double ta = 2.0 * a, tb = 2.0 * b;
    double c = kind == LIM_MC ? 0.5 * (a + b) : (a + 2.0 * b) / 3.0;
    double m = fabs(ta) < fabs(tb) ? ta : tb;
    return fabs(c) < fabs(m) ? c : m;
  }
  return 2.0 * a * b / (a + b);
}

static double limiter(const orc_forest* f, double a, double b, double thr2) {
  return limit_ab(f->c.limiter, a, b, thr2);
}

double orc_limiter_value(int kind, double a, double b, double thr2) { return limit_ab(kind, a, b, thr2); }

static double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

/* 1/dx of dimension d at level l: dx = (xmax - xmin) / (cells at level l) */
static double rdx(const orc_forest* f, int l, int d) {
  double dx = (f->c.xmax[d] - f->c.xmin[d]) / (double)ncells_dom(f, l, d);
  return 1.0 / dx;
}

/* (r dx)^2 of Cada's smoothness switch along d at level l; 0 without it */
static double cada_thr2(const orc_forest* f, int l, int d) {
  if (!(f->c.cada_radius > 0.0)) return 0.0;
  double dx = (f->c.xmax[d] - f->c.xmin[d]) / (double)ncells_dom(f, l, d);
  double rd = f->c.cada_radius * dx;
  return rd * rd;
}

static int64_t pidx(const orc_forest* f, int i, int j, int k) {
  return ((int64_t)(k + f->gs[2]) * f->px[1] + (j + f->gs[1])) * f->px[0] + (i + f->gs[0]);
}

static int64_t cidx(const orc_forest* f, int i, int j, int k) {
  return ((int64_t)k * f->nx[1] + j) * f->nx[0] + i;
}

static double st(const orc_forest* f, const double* S, int v, int64_t leaf, int64_t cell) {
  return S[((int64_t)v * f->n + leaf) * f->ncell + cell];
}

/* ------------------------------------------------------------------ */
/* forest construction and validation (Sec. 1.3)                       */
/* ------------------------------------------------------------------ */

/* classify the neighbour of leaf b across face (d, s): same level, coarser,
 * finer (then the 2^(ndim-1) adjacent children are leaves), or boundary */
static int classify(const orc_forest* f, int64_t b, int d, int s, int64_t* nb) {
  int l = f->lev[b];
  int64_t c[3] = {f->ijk[3 * b], f->ijk[3 * b + 1], f->ijk[3 * b + 2]};
  c[d] += s;
  *nb = -1;
  if (!wrap(f, d, &c[d], nblk(f, l, d))) return NB_BND;
  int64_t x = lookup(f, l, c);
  if (x >= 0) {
    *nb = x;
    return NB_SAME;
  }
  if (l > 1) {
    int64_t p[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
    for (int e = f->nd; e < 3; e++) p[e] = 0;
    x = lookup(f, l - 1, p);
    if (x >= 0) {
      *nb = x;
      return NB_COARSER;
    }
  }
  return NB_FINER;
}

/* the region of block (l, c) must be covered by one leaf at level l or l-1,
 * or by leaves at level l+1 wherever it touches the leaf at offset -o */
static int region_balanced(const orc_forest* f, int l, const int64_t c[3], const int o[3]) {
  if (lookup(f, l, c) >= 0) return 1;
  if (l > 1) {
    int64_t p[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
    for (int e = f->nd; e < 3; e++) p[e] = 0;
    if (lookup(f, l - 1, p) >= 0) return 1;
  }
  if (l + 1 > f->c.max_level) return 0;
  int nch = 1 << f->nd;
  for (int q = 0; q < nch; q++) {
    int64_t ch[3] = {0, 0, 0};
    int ok = 1;
    for (int e = 0; e < f->nd; e++) {
      int qe = (q >> e) & 1;
      if (o[e] == 1 && qe != 0) ok = 0;  /* neighbour on the +side: its low half touches */
      if (o[e] == -1 && qe != 1) ok = 0; /* neighbour on the -side: its high half touches */
      ch[e] = 2 * c[e] + qe;
    }
    if (!ok) continue;
    if (lookup(f, l + 1, ch) < 0) return 0;
  }
  return 1;
}

int orc_forest_create(const orc_config* cfg, int64_t n, const int32_t* lev, const int32_t* ijk,
                      orc_forest** out) {
  if (!cfg || !lev || !ijk || !out || n <= 0) return fail(ORC_EINVAL, "null argument or n <= 0");
  *out = NULL;
  const orc_config* c = cfg;
  if (c->ndim < 1 || c->ndim > 3) return fail(ORC_EINVAL, "ndim must be 1..3");
  if (c->nghost != 2) return fail(ORC_EINVAL, "nghost must be 2");
  if (c->max_level < 1 || c->max_level > 12) return fail(ORC_EINVAL, "max_level out of range");
  if (c->physics != PHYS_EULER && c->physics != PHYS_MHD && c->physics != PHYS_POLY)
    return fail(ORC_EINVAL, "bad physics");
  if (c->flux < 0 || c->flux > 2) return fail(ORC_EINVAL, "bad flux");
  if (c->limiter < 0 || c->limiter > 4) return fail(ORC_EINVAL, "bad limiter");
  if (!(c->cada_radius >= 0.0) || !(c->cada_radius < INFINITY)) return fail(ORC_EINVAL, "bad Cada radius");
  if (c->rk_stages != 2 && c->rk_stages != 3) return fail(ORC_EINVAL, "rk_stages must be 2 or 3");
  if (c->physics == PHYS_POLY) {
    if (!(c->gamma >= 1.0) || !(c->cad > 0.0) || !(c->cfl > 0.0))
      return fail(ORC_EINVAL, "polytrope needs gamma >= 1, c_ad > 0, cfl > 0");
    if (c->flux == FLUX_HLLC) return fail(ORC_EINVAL, "HLLC needs the energy equation (not the polytrope)");
  } else if (!(c->gamma > 1.0) || !(c->cfl > 0.0)) {
    return fail(ORC_EINVAL, "gamma must be > 1, cfl > 0");
  }
  for (int d = 0; d < c->ndim; d++) {
    if (c->block_nx[d] < 4 || (c->block_nx[d] & 1))
      return fail(ORC_EINVAL, "block_nx must be even and >= 4");
    if (c->base_blocks[d] < 1) return fail(ORC_EINVAL, "base_blocks must be >= 1");
    if (!(c->xmax[d] > c->xmin[d])) return fail(ORC_EINVAL, "xmax must exceed xmin");
    if (c->bc[d][0] < 0 || c->bc[d][0] > 1 || c->bc[d][1] != c->bc[d][0])
      return fail(ORC_EINVAL, "bc must be periodic or zero-gradient, same on both sides");
  }
  orc_forest* f = (orc_forest*)calloc(1, sizeof(orc_forest));
  if (!f) return fail(ORC_ENOMEM, "out of memory");
  f->c = *c;
  f->nd = c->ndim;
  f->mhd = c->physics == PHYS_MHD;
  f->poly = c->physics == PHYS_POLY;
  f->nvar = f->mhd ? 3 + 2 * f->nd : f->poly ? 1 + f->nd : 2 + f->nd;
  f->ng = c->nghost;
  f->n = n;
  f->ncell = 1;
  f->npad = 1;
  for (int d = 0; d < 3; d++) {
    int act = d < f->nd;
    f->nx[d] = act ? c->block_nx[d] : 1;
    f->gs[d] = act ? f->ng : 0;
    f->px[d] = f->nx[d] + 2 * f->gs[d];
    f->ncell *= f->nx[d];
    f->npad *= f->px[d];
  }
  f->lev = (int32_t*)malloc(sizeof(int32_t) * n);
  f->ijk = (int32_t*)malloc(sizeof(int32_t) * 3 * n);
  uint64_t cap = 16;
  while (cap < (uint64_t)(4 * n)) cap <<= 1;
  f->hkey = (uint64_t*)calloc(cap, sizeof(uint64_t));
  f->hval = (int64_t*)calloc(cap, sizeof(int64_t));
  f->hmask = cap - 1;
  f->kind = (int32_t*)malloc(sizeof(int32_t) * 6 * n);
  f->nbr = (int64_t*)malloc(sizeof(int64_t) * 6 * n);
  size_t sz = sizeof(double) * (size_t)f->nvar * (size_t)n * (size_t)f->ncell;
  f->U = (double*)calloc(1, sz);
  f->U1 = (double*)calloc(1, sz);
  f->U2 = (double*)calloc(1, sz);
  f->ffine = (double**)calloc((size_t)n * 6, sizeof(double*));
  if (!f->lev || !f->ijk || !f->hkey || !f->hval || !f->kind || !f->nbr || !f->U || !f->U1 ||
      !f->U2 || !f->ffine) {
    orc_forest_destroy(f);
    return fail(ORC_ENOMEM, "out of memory");
  }
  memcpy(f->lev, lev, sizeof(int32_t) * n);
  memcpy(f->ijk, ijk, sizeof(int32_t) * 3 * n);

  /* leaves: level and coordinates in range, no duplicates */
  for (int64_t b = 0; b < n; b++) {
    int l = lev[b];
    if (l < 1 || l > c->max_level) {
      orc_forest_destroy(f);
      return fail(ORC_EINVAL, "leaf %lld: level %d out of range", (long long)b, l);
    }
    int64_t x[3];
    for (int d = 0; d < 3; d++) {
      x[d] = ijk[3 * b + d];
      if (x[d] < 0 || x[d] >= nblk(f, l, d)) {
        orc_forest_destroy(f);
        return fail(ORC_EINVAL, "leaf %lld: coordinate out of range", (long long)b);
      }
    }
    if (!insert(f, l, x, b)) {
      orc_forest_destroy(f);
      return fail(ORC_EUNBALANCED, "leaf %lld duplicates another leaf", (long long)b);
    }
  }
  /* no leaf has a leaf ancestor; volumes add up to the domain */
  int64_t vol = 0, dom = 1;
  for (int d = 0; d < f->nd; d++) dom *= c->base_blocks[d];
  dom <<= f->nd * (c->max_level - 1);
  for (int64_t b = 0; b < n; b++) {
    int l = lev[b];
    for (int la = l - 1; la >= 1; la--) {
      int64_t a[3];
      for (int d = 0; d < 3; d++) a[d] = d < f->nd ? ((int64_t)ijk[3 * b + d] >> (l - la)) : 0;
      if (lookup(f, la, a) >= 0) {
        orc_forest_destroy(f);
        return fail(ORC_EUNBALANCED, "leaf %lld overlaps a coarser leaf", (long long)b);
      }
    }
    vol += (int64_t)1 << (f->nd * (c->max_level - l));
  }
  if (vol != dom) {
    orc_forest_destroy(f);
    return fail(ORC_EUNBALANCED, "leaves do not cover the domain");
  }
  /* 2:1 balance across faces, edges and corners (reading of Sec. 1.3) */
  int nofs = 1;
  for (int d = 0; d < f->nd; d++) nofs *= 3;
  for (int64_t b = 0; b < n; b++) {
    int l = lev[b];
    for (int q = 0; q < nofs; q++) {
      int o[3] = {0, 0, 0}, t = q, zero = 1;
      for (int d = 0; d < f->nd; d++) {
        o[d] = t % 3 - 1;
        t /= 3;
        if (o[d]) zero = 0;
      }
      if (zero) continue;
      int64_t x[3] = {0, 0, 0};
      int inside = 1;
      for (int d = 0; d < f->nd; d++) {
        x[d] = (int64_t)ijk[3 * b + d] + o[d];
        if (!wrap(f, d, &x[d], nblk(f, l, d))) inside = 0;
      }
      if (!inside) continue;
      if (!region_balanced(f, l, x, o)) {
        orc_forest_destroy(f);
        return fail(ORC_EUNBALANCED, "leaf %lld violates 2:1 balance", (long long)b);
      }
    }
  }
  for (int64_t b = 0; b < n; b++)
    for (int fc = 0; fc < 6; fc++) {
      f->kind[6 * b + fc] = NB_BND;
      f->nbr[6 * b + fc] = -1;
      if (fc / 2 < f->nd) f->kind[6 * b + fc] = classify(f, b, fc / 2, (fc & 1) ? 1 : -1, &f->nbr[6 * b + fc]);
    }
  /* storage for fine-side boundary fluxes at coarse-fine faces */
  for (int64_t b = 0; b < n; b++)
    for (int fc = 0; fc < 2 * f->nd; fc++)
      if (f->kind[6 * b + fc] == NB_COARSER) {
        int d = fc / 2;
        int64_t m = (int64_t)f->nvar * (f->ncell / f->nx[d]);
        f->ffine[6 * b + fc] = (double*)malloc(sizeof(double) * m);
        if (!f->ffine[6 * b + fc]) {
          orc_forest_destroy(f);
          return fail(ORC_ENOMEM, "out of memory");
        }
      }
  *out = f;
  return ORC_OK;
}

int orc_forest_destroy(orc_forest* f) {
  if (!f) return ORC_OK;
  if (f->ffine)
    for (int64_t i = 0; i < f->n * 6; i++) free(f->ffine[i]);
  free(f->ffine);
  free(f->lev);
  free(f->ijk);
  free(f->hkey);
  free(f->hval);
  free(f->kind);
  free(f->nbr);
  free(f->U);
  free(f->U1);
  free(f->U2);
  free(f);
  return ORC_OK;
}

int orc_nvar(const orc_forest* f) { return f ? f->nvar : 0; }
double orc_glm_ch(const orc_forest* f) { return f ? f->ch : 0.0; }

int orc_set_state(orc_forest* f, const double* U, int64_t nd) {
  if (!f || !U) return fail(ORC_EINVAL, "null argument");
  if (nd != (int64_t)f->nvar * f->n * f->ncell) return fail(ORC_EINVAL, "state size mismatch");
  memcpy(f->U, U, sizeof(double) * nd);
  return ORC_OK;
}

int orc_get_state(const orc_forest* f, double* U, int64_t nd) {
  if (!f || !U) return fail(ORC_EINVAL, "null argument");
  if (nd != (int64_t)f->nvar * f->n * f->ncell) return fail(ORC_EINVAL, "state size mismatch");
  memcpy(U, f->U, sizeof(double) * nd);
  return ORC_OK;
}

int orc_face_kinds(const orc_forest* f, int64_t leaf, int32_t* kinds) {
  if (!f || !kinds || leaf < 0 || leaf >= f->n) return fail(ORC_EINVAL, "bad argument");
  for (int fc = 0; fc < 2 * f->nd; fc++) kinds[fc] = f->kind[6 * leaf + fc];
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* ghost fill (Sec. 1.3 block tree, ratio 2; ghost layers per stencil  */
/* width, Sec. 2.1).  Face ghosts only, 2 layers.                      */
/* ------------------------------------------------------------------ */

/* global cell coordinate of local coordinate x (may be a ghost index) */
static int64_t gcoord(const orc_forest* f, int64_t b, int d, int x) {
  return (int64_t)f->ijk[3 * b + d] * f->nx[d] + x;
}

/* value of cell with global coordinates g at level l (after periodic wrap),
 * found by leaf lookup; used by restriction */
static double cell_at(const orc_forest* f, const double* S, int v, int l, int64_t g[3]) {
  int64_t blk[3] = {0, 0, 0};
  int loc[3] = {0, 0, 0};
  for (int d = 0; d < f->nd; d++) {
    wrap(f, d, &g[d], ncells_dom(f, l, d));
    blk[d] = g[d] / f->nx[d];
    loc[d] = (int)(g[d] % f->nx[d]);
  }
  int64_t leaf = lookup(f, l, blk);
  if (leaf < 0) return NAN; /* cannot happen on a validated forest */
  return st(f, S, v, leaf, cidx(f, loc[0], loc[1], loc[2]));
}

/* local coordinates of cell t (0 <= t < cells per slab) of ghost layer
 * `layer` across face (d, s): transverse coordinates run over the interior */
static void slab_cell(const orc_forest* f, int d, int s, int layer, int64_t t, int x[3]) {
  for (int e = 0; e < 3; e++) {
    if (e == d) continue;
    x[e] = (int)(t % f->nx[e]);
    t /= f->nx[e];
  }
  x[d] = s < 0 ? -1 - layer : f->nx[d] + layer;
}

/* Fill a padded block: interior copy, then the faces whose ghosts need no
 * prolongation: same-level copy (with periodic wrap), restriction of the
 * 2^ndim finer cells as a pairwise-tree sum times 2^-ndim, and zero-gradient
 * physical boundaries (copy of the nearest interior cell into both layers).
 * Edge and corner ghosts stay NaN: the stencil never reads them. */
static void fill_basic(const orc_forest* f, const double* S, int64_t b, double* W) {
  const int nv = f->nvar, l = f->lev[b];
  for (int64_t i = 0; i < (int64_t)nv * f->npad; i++) W[i] = NAN;
  for (int v = 0; v < nv; v++)
    for (int k = 0; k < f->nx[2]; k++)
      for (int j = 0; j < f->nx[1]; j++)
        for (int i = 0; i < f->nx[0]; i++)
          W[v * f->npad + pidx(f, i, j, k)] = st(f, S, v, b, cidx(f, i, j, k));
  for (int fc = 0; fc < 2 * f->nd; fc++) {
    int d = fc / 2, s = (fc & 1) ? 1 : -1;
    int kind = f->kind[6 * b + fc];
    int64_t nb = f->nbr[6 * b + fc];
    if (kind == NB_COARSER) continue;
    int64_t nt = f->ncell / f->nx[d];
    for (int layer = 0; layer < f->ng; layer++) {
      for (int64_t t = 0; t < nt; t++) {
        int x[3];
        slab_cell(f, d, s, layer, t, x);
        int64_t dst = pidx(f, x[0], x[1], x[2]);
        if (kind == NB_SAME) {
          int y[3] = {x[0], x[1], x[2]};
          y[d] = s < 0 ? f->nx[d] - 1 - layer : layer;
          for (int v = 0; v < nv; v++) W[v * f->npad + dst] = st(f, S, v, nb, cidx(f, y[0], y[1], y[2]));
        } else if (kind == NB_BND) {
          int y[3] = {x[0], x[1], x[2]};
          y[d] = s < 0 ? 0 : f->nx[d] - 1;
          for (int v = 0; v < nv; v++) W[v * f->npad + dst] = st(f, S, v, b, cidx(f, y[0], y[1], y[2]));
        } else { /* NB_FINER: restriction */
          int64_t G[3];
          for (int e = 0; e < 3; e++) G[e] = e < f->nd ? gcoord(f, b, e, x[e]) : 0;
          for (int v = 0; v < nv; v++) {
            double c8[8];
            int nch = 1 << f->nd;
            for (int q = 0; q < nch; q++) {
              int64_t g[3] = {0, 0, 0};
              for (int e = 0; e < f->nd; e++) g[e] = 2 * G[e] + ((q >> e) & 1);
              c8[q] = cell_at(f, S, v, l + 1, g);
            }
            double r;
            if (f->nd == 1)
              r = (c8[0] + c8[1]) * 0.5;
            else if (f->nd == 2)
              r = ((c8[0] + c8[1]) + (c8[2] + c8[3])) * 0.25;
            else
              r = (((c8[0] + c8[1]) + (c8[2] + c8[3])) + ((c8[4] + c8[5]) + (c8[6] + c8[7]))) * 0.125;
            W[v * f->npad + dst] = r;
          }
        }
      }
    }
  }
}

/* Prolongation into the ghosts of faces whose neighbour is coarser: the
 * coarse cell value plus, per dimension in order x, y, z, a quarter of its
 * minmod-limited slope, added or subtracted by which half of the coarse cell
 * the fine cell lies in (conservative linear prolongation).  The coarse
 * leaf's own ghosts come from fill_basic. */
static void fill_prolong(const orc_forest* f, const double* S, int64_t b, double* W, double* Wc) {
  const int nv = f->nvar, l = f->lev[b];
  for (int fc = 0; fc < 2 * f->nd; fc++) {
    if (f->kind[6 * b + fc] != NB_COARSER) continue;
    int d = fc / 2, s = (fc & 1) ? 1 : -1;
    int64_t C = f->nbr[6 * b + fc];
    fill_basic(f, S, C, Wc);
    int64_t nt = f->ncell / f->nx[d];
    for (int layer = 0; layer < f->ng; layer++) {
      for (int64_t t = 0; t < nt; t++) {
        int x[3];
        slab_cell(f, d, s, layer, t, x);
        int64_t g[3] = {0, 0, 0};
        int cc[3] = {0, 0, 0};
        for (int e = 0; e < f->nd; e++) {
          g[e] = gcoord(f, b, e, x[e]);
          wrap(f, e, &g[e], ncells_dom(f, l, e));
          int64_t gc = g[e] / 2;
          cc[e] = (int)(gc % f->nx[e]);
        }
        int64_t dst = pidx(f, x[0], x[1], x[2]);
        for (int v = 0; v < nv; v++) {
          const double* w = Wc + (int64_t)v * f->npad;
          double u0 = w[pidx(f, cc[0], cc[1], cc[2])];
          double u = u0;
          for (int e = 0; e < f->nd; e++) {
            int lo[3] = {cc[0], cc[1], cc[2]}, hi[3] = {cc[0], cc[1], cc[2]};
            lo[e] -= 1;
            hi[e] += 1;
            double sl = minmod(u0 - w[pidx(f, lo[0], lo[1], lo[2])], w[pidx(f, hi[0], hi[1], hi[2])] - u0);
            double t = 0.25 * sl;
            u = (g[e] & 1) ? u + t : u - t;
          }
          W[v * f->npad + dst] = u;
        }
      }
    }
  }
}

static void fill_all(const orc_forest* f, const double* S, int64_t b, double* W, double* Wc) {
  fill_basic(f, S, b, W);
  fill_prolong(f, S, b, W, Wc);
}

/* ------------------------------------------------------------------ */
/* fluxes                                                              */
/* ------------------------------------------------------------------ */

/* primitive variables of every padded cell */
static void padded_prim(const orc_forest* f, const double* W, double* P) {
  const int nv = f->nvar;
  for (int64_t c = 0; c < f->npad; c++) {
    double u[NVMAX], v[NVMAX];
    for (int k = 0; k < nv; k++) u[k] = W[k * f->npad + c];
    to_prim(f, u, v);
    for (int k = 0; k < nv; k++) P[k * f->npad + c] = v[k];
  }
}

/* MUSCL face states and flux at the face normal to d lying on the low side
 * of local cell x (x[d] in 0..nx): left state from cell x-e_d extrapolated by
 * half its limited slope, right state from cell x likewise (Sec. 2.2 limited
 * reconstruction in primitive variables). */
static void face_flux(const orc_forest* f, const double* P, int d, const int x[3], double thr2, double* F) {
  const int nv = f->nvar;
  int m2[3] = {x[0], x[1], x[2]}, m1[3] = {x[0], x[1], x[2]}, p1[3] = {x[0], x[1], x[2]};
  m2[d] -= 2;
  m1[d] -= 1;
  p1[d] += 1;
  int64_t im2 = pidx(f, m2[0], m2[1], m2[2]), im1 = pidx(f, m1[0], m1[1], m1[2]);
  int64_t i0 = pidx(f, x[0], x[1], x[2]), ip1 = pidx(f, p1[0], p1[1], p1[2]);
  double vl[NVMAX], vr[NVMAX];
  for (int k = 0; k < nv; k++) {
    const double* p = P + (int64_t)k * f->npad;
    /* left state: cell m-1 toward its upper face (away: backward difference);
     * right state: cell m toward its lower face (away: forward difference) */
    double sl = limiter(f, p[im1] - p[im2], p[i0] - p[im1], thr2);
    double sr = limiter(f, p[ip1] - p[i0], p[i0] - p[im1], thr2);
    vl[k] = p[im1] + 0.5 * sl;
    vr[k] = p[i0] - 0.5 * sr;
  }
  riemann(f, vl, vr, d, F);
}

/* number of faces normal to d in a block and their linear index */
static int64_t nfaces(const orc_forest* f, int d) { return (f->ncell / f->nx[d]) * (f->nx[d] + 1); }

static int64_t fidx(const orc_forest* f, int d, const int x[3]) {
  int e[3] = {f->nx[0], f->nx[1], f->nx[2]};
  e[d] += 1;
  return ((int64_t)x[2] * e[1] + x[1]) * e[0] + x[0];
}

/* transverse index of a cell within a face slab normal to d */
static int64_t tidx(const orc_forest* f, int d, const int x[3]) {
  int e[3] = {f->nx[0], f->nx[1], f->nx[2]};
  int y[3] = {x[0], x[1], x[2]};
  e[d] = 1;
  y[d] = 0;
  return ((int64_t)y[2] * e[1] + y[1]) * e[0] + y[0];
}

/* ------------------------------------------------------------------ */
/* one Runge-Kutta stage (Sec. 2.1, 2.3.2, 2.4: three-step / SSP RK)    */
/* ------------------------------------------------------------------ */

typedef struct {
  double* W;
  double* Wc;
  double* P;
  double* F[3];
} scratch;

static int scratch_alloc(const orc_forest* f, scratch* s) {
  memset(s, 0, sizeof *s);
  s->W = (double*)malloc(sizeof(double) * f->nvar * f->npad);
  s->Wc = (double*)malloc(sizeof(double) * f->nvar * f->npad);
  s->P = (double*)malloc(sizeof(double) * f->nvar * f->npad);
  int ok = s->W && s->Wc && s->P;
  for (int d = 0; d < f->nd; d++) {
    s->F[d] = (double*)malloc(sizeof(double) * f->nvar * nfaces(f, d));
    ok = ok && s->F[d];
  }
  return ok;
}

static void scratch_free(scratch* s) {
  free(s->W);
  free(s->Wc);
  free(s->P);
  for (int d = 0; d < 3; d++) free(s->F[d]);
}

/* Pass A: fine leaves record the fluxes on their faces that touch a coarser
 * leaf, for the coarse side's replacement in pass B. */
static void record_fine_fluxes(const orc_forest* f, const double* S, int64_t b, scratch* w) {
  int any = 0;
  for (int fc = 0; fc < 2 * f->nd; fc++) any |= f->kind[6 * b + fc] == NB_COARSER;
  if (!any) return;
  fill_all(f, S, b, w->W, w->Wc);
  padded_prim(f, w->W, w->P);
  const int nv = f->nvar;
  for (int fc = 0; fc < 2 * f->nd; fc++) {
    if (f->kind[6 * b + fc] != NB_COARSER) continue;
    int d = fc / 2, s = (fc & 1) ? 1 : -1;
    double* out = f->ffine[6 * b + fc];
    int64_t nt = f->ncell / f->nx[d];
    for (int k = 0; k < f->nx[2]; k++)
      for (int j = 0; j < f->nx[1]; j++)
        for (int i = 0; i < f->nx[0]; i++) {
          int x[3] = {i, j, k};
          if (x[d] != 0) continue;
          x[d] = s < 0 ? 0 : f->nx[d];
          double F[NVMAX];
          face_flux(f, w->P, d, x, cada_thr2(f, f->lev[b], d), F);
          int64_t t = tidx(f, d, x);
          for (int v = 0; v < nv; v++) out[v * nt + t] = F[v];
        }
  }
}

/* Pass B: all fluxes of leaf b, coarse-fine replacement, divergence and the
 * SSP combination.  stage counts from 1; Un is the step's initial state. */
static void update_leaf(const orc_forest* f, const double* S, const double* Un, double* Out, int64_t b,
                        int stage, double dt, scratch* w) {
  const int nv = f->nvar, nd = f->nd, l = f->lev[b];
  fill_all(f, S, b, w->W, w->Wc);
  padded_prim(f, w->W, w->P);
  for (int d = 0; d < nd; d++) {
    int e[3] = {f->nx[0], f->nx[1], f->nx[2]};
    e[d] += 1;
    int64_t nf = nfaces(f, d);
    for (int k = 0; k < e[2]; k++)
      for (int j = 0; j < e[1]; j++)
        for (int i = 0; i < e[0]; i++) {
          int x[3] = {i, j, k};
          double F[NVMAX];
          face_flux(f, w->P, d, x, cada_thr2(f, l, d), F);
          int64_t q = fidx(f, d, x);
          for (int v = 0; v < nv; v++) w->F[d][v * nf + q] = F[v];
        }
  }
  /* conservative coarse-fine coupling: coarse face flux := mean of the fine
   * face fluxes of the same stage */
  for (int fc = 0; fc < 2 * nd; fc++) {
    if (f->kind[6 * b + fc] != NB_FINER) continue;
    int d = fc / 2, s = (fc & 1) ? 1 : -1;
    int64_t nf = nfaces(f, d);
    for (int k = 0; k < f->nx[2]; k++)
      for (int j = 0; j < f->nx[1]; j++)
        for (int i = 0; i < f->nx[0]; i++) {
          int x[3] = {i, j, k};
          if (x[d] != 0) continue;
          x[d] = s < 0 ? 0 : f->nx[d];
          /* the fine cell just across the face, in global fine coordinates */
          int64_t gf[3] = {0, 0, 0};
          for (int e = 0; e < nd; e++) gf[e] = 2 * gcoord(f, b, e, x[e]);
          gf[d] = 2 * gcoord(f, b, d, s < 0 ? -1 : f->nx[d]) + (s < 0 ? 1 : 0);
          double vals[4][NVMAX];
          int nsub = 1 << (nd - 1), qi = 0;
          for (int q = 0; q < (1 << nd); q++) {
            if ((q >> d) & 1) continue;
            int64_t g[3] = {gf[0], gf[1], gf[2]};
            for (int e = 0; e < nd; e++)
              if (e != d) g[e] += (q >> e) & 1;
            int64_t blk[3] = {0, 0, 0};
            int loc[3] = {0, 0, 0};
            for (int e = 0; e < nd; e++) {
              wrap(f, e, &g[e], ncells_dom(f, l + 1, e));
              blk[e] = g[e] / f->nx[e];
              loc[e] = (int)(g[e] % f->nx[e]);
            }
            int64_t fl = lookup(f, l + 1, blk);
            const double* ff = f->ffine[6 * fl + 2 * d + (s < 0 ? 1 : 0)];
            int64_t nt = f->ncell / f->nx[d];
            int64_t t = tidx(f, d, loc);
            for (int v = 0; v < nv; v++) vals[qi][v] = ff[v * nt + t];
            qi++;
          }
          int64_t q = fidx(f, d, x);
          for (int v = 0; v < nv; v++) {
            double m;
            if (nsub == 1)
              m = vals[0][v];
            else if (nsub == 2)
              m = (vals[0][v] + vals[1][v]) * 0.5;
            else
              m = ((vals[0][v] + vals[1][v]) + (vals[2][v] + vals[3][v])) * 0.25;
            w->F[d][v * nf + q] = m;
          }
        }
  }
  double r[3];
  for (int d = 0; d < nd; d++) r[d] = rdx(f, l, d);
  const int S3 = f->c.rk_stages;
  for (int k = 0; k < f->nx[2]; k++)
    for (int j = 0; j < f->nx[1]; j++)
      for (int i = 0; i < f->nx[0]; i++) {
        int x[3] = {i, j, k};
        int64_t cell = cidx(f, i, j, k);
        for (int v = 0; v < nv; v++) {
          double acc = 0.0;
          for (int d = 0; d < nd; d++) {
            int y[3] = {i, j, k};
            y[d] += 1;
            int64_t nf = nfaces(f, d);
            double diff = (w->F[d][v * nf + fidx(f, d, y)] - w->F[d][v * nf + fidx(f, d, x)]) * r[d];
            acc = (d == 0) ? diff : acc + diff;
          }
          int64_t a = ((int64_t)v * f->n + b) * f->ncell + cell;
          double tmp = S[a] - dt * acc; /* U + dt L(U), L = -div F */
          double un = Un[a];
          double res;
          if (stage == 1)
            res = tmp;
          else if (S3 == 2)
            res = 0.5 * un + 0.5 * tmp;
          else if (stage == 2)
            res = 0.75 * un + 0.25 * tmp;
          else
            res = (1.0 / 3.0) * un + (2.0 / 3.0) * tmp;
          Out[a] = res;
        }
      }
}

static int check_physical(const orc_forest* f, const double* S);

int orc_advance(orc_forest* f, double dt) {
  if (!f) return fail(ORC_EINVAL, "null forest");
  if (!(dt > 0.0) || !isfinite(dt)) return fail(ORC_EINVAL, "dt must be positive and finite");
  if (f->mhd && !(f->ch > 0.0)) return fail(ORC_EINVAL, "MHD needs orc_max_dt before advancing");
  const int S = f->c.rk_stages;
  int err = 0;
  for (int stage = 1; stage <= S; stage++) {
    const double* in = stage == 1 ? f->U : (stage == 2 ? f->U1 : f->U2);
    double* out = stage == S ? f->U : (stage == 1 ? f->U1 : f->U2);
#pragma omp parallel
    {
      scratch w;
      int ok = scratch_alloc(f, &w);
      if (!ok) {
#pragma omp atomic write
        err = 1;
      }
#pragma omp for schedule(dynamic, 1)
      for (int64_t b = 0; b < f->n; b++)
        if (ok) record_fine_fluxes(f, in, b, &w);
#pragma omp for schedule(dynamic, 1)
      for (int64_t b = 0; b < f->n; b++)
        if (ok) update_leaf(f, in, f->U, out, b, stage, dt, &w);
      scratch_free(&w);
    }
    if (err) return fail(ORC_ENOMEM, "out of memory");
  }
  if (f->mhd) {
    /* GLM damping of psi once per step: psi *= exp(-dt c_h / c_r) */
    double fac = exp(-(dt * f->ch) / f->c.glm_cr);
    double* psi = f->U + (int64_t)iPsi(f) * f->n * f->ncell;
    for (int64_t i = 0; i < f->n * f->ncell; i++) psi[i] = psi[i] * fac;
  }
  return check_physical(f, f->U);
}

/* ------------------------------------------------------------------ */
/* Courant time step (Sec. 2.1: Courant number, phys_get_cmax)          */
/* ------------------------------------------------------------------ */

/* rho <= 0, p <= 0 or NaN (the polytrope: rho <= 0 or a velocity that is
 * NaN or overflows, its pressure being positive with rho) */
static int nonphysical(const orc_forest* f, const double* v) {
  if (!(v[0] > 0.0)) return 1;
  if (!f->poly) return !(v[iE(f)] > 0.0);
  double vv = 0.0;
  for (int d = 0; d < f->nd; d++) vv = vv + v[1 + d] * v[1 + d];
  return !(vv < INFINITY);
}

static int check_physical(const orc_forest* f, const double* S) {
  int bad = 0;
#pragma omp parallel for reduction(| : bad) schedule(static)
  for (int64_t b = 0; b < f->n; b++)
    for (int64_t c = 0; c < f->ncell; c++) {
      double u[NVMAX], v[NVMAX];
      for (int k = 0; k < f->nvar; k++) u[k] = st(f, S, k, b, c);
      to_prim(f, u, v);
      if (nonphysical(f, v)) bad = 1;
    }
  if (bad) return fail(ORC_ENONPHYSICAL, "non-physical state (rho <= 0, p <= 0 or NaN)");
  return ORC_OK;
}

/* dt = cfl / max over cells of sum_d (|v_d| + c_d) / dx_d; the maximum is
 * exact, so the thread count does not change the result.  For MHD the GLM
 * cleaning speed c_h is the maximum over cells and directions of |v_d|+c_f,d. */
int orc_max_dt(orc_forest* f, double* dt_out) {
  if (!f || !dt_out) return fail(ORC_EINVAL, "null argument");
  double smax = 0.0, chmax = 0.0;
  int bad = 0;
#pragma omp parallel for reduction(max : smax, chmax) reduction(| : bad) schedule(static)
  for (int64_t b = 0; b < f->n; b++) {
    int l = f->lev[b];
    double r[3];
    for (int d = 0; d < f->nd; d++) r[d] = rdx(f, l, d);
    for (int64_t c = 0; c < f->ncell; c++) {
      double u[NVMAX], v[NVMAX];
      for (int k = 0; k < f->nvar; k++) u[k] = st(f, f->U, k, b, c);
      to_prim(f, u, v);
      if (nonphysical(f, v)) {
        bad = 1;
        continue;
      }
      double s = 0.0;
      for (int d = 0; d < f->nd; d++) {
        double w = fabs(v[1 + d]) + speed(f, v, d);
        double t = w * r[d];
        s = (d == 0) ? t : s + t;
        if (w > chmax) chmax = w;
      }
      if (s > smax) smax = s;
    }
  }
  if (bad) return fail(ORC_ENONPHYSICAL, "non-physical state (rho <= 0, p <= 0 or NaN)");
  f->ch = chmax;
  *dt_out = f->c.cfl / smax;
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Loehner refinement flags (Sec. 1.3)                                 */
/* ------------------------------------------------------------------ */

/* Sec. 1.3: weighted second derivatives (Loehner), refine when any cell
 * exceeds the tolerance, coarsen when all cells are below a fraction of it.
 * Reading: per variable u in {rho, p}, with axis neighbours only,
 *   E = sqrt( sum_d (u+ - 2u0 + u-)^2 /
 *             sum_d (|u+ - u0| + |u0 - u-| + eps (|u+| + 2|u0| + |u-|))^2 ),
 * E = 0 where the denominator vanishes; block value = max over interior
 * cells of w_rho E_rho + w_p E_p. */
static double lohner_cell(const orc_forest* f, const double* q, const int x[3]) {
  const double eps = f->c.lohner_eps;
  double num = 0.0, den = 0.0;
  for (int d = 0; d < f->nd; d++) {
    int a[3] = {x[0], x[1], x[2]}, b[3] = {x[0], x[1], x[2]};
    a[d] -= 1;
    b[d] += 1;
    double um = q[pidx(f, a[0], a[1], a[2])];
    double u0 = q[pidx(f, x[0], x[1], x[2])];
    double up = q[pidx(f, b[0], b[1], b[2])];
    double d2 = up - 2.0 * u0 + um;
    double dd = fabs(up - u0) + fabs(u0 - um) + eps * (fabs(up) + 2.0 * fabs(u0) + fabs(um));
    num = num + d2 * d2;
    den = den + dd * dd;
  }
  if (!(den > 0.0)) return 0.0;
  return sqrt(num / den);
}

int orc_flag_blocks(orc_forest* f, int8_t* flags, double* emax_out) {
  if (!f || !flags) return fail(ORC_EINVAL, "null argument");
  int err = 0;
  const double tol = f->c.lohner_tol, ctol = f->c.lohner_coarsen_frac * f->c.lohner_tol;
#pragma omp parallel
  {
    scratch w;
    int ok = scratch_alloc(f, &w);
    double* rho = (double*)malloc(sizeof(double) * f->npad);
    double* prs = (double*)malloc(sizeof(double) * f->npad);
    if (!ok || !rho || !prs) {
#pragma omp atomic write
      err = 1;
    }
#pragma omp for schedule(dynamic, 1)
    for (int64_t b = 0; b < f->n; b++) {
      if (err) continue;
      fill_all(f, f->U, b, w.W, w.Wc);
      padded_prim(f, w.W, w.P);
      for (int64_t c = 0; c < f->npad; c++) {
        rho[c] = w.P[c];
        prs[c] = f->poly ? poly_p(f, w.P[c]) : w.P[(int64_t)iE(f) * f->npad + c];
      }
      double emax = 0.0;
      for (int k = 0; k < f->nx[2]; k++)
        for (int j = 0; j < f->nx[1]; j++)
          for (int i = 0; i < f->nx[0]; i++) {
            int x[3] = {i, j, k};
            double e = f->c.lohner_w_rho * lohner_cell(f, rho, x) + f->c.lohner_w_p * lohner_cell(f, prs, x);
            if (e > emax) emax = e;
          }
      int l = f->lev[b];
      int8_t fl = 0;
      if (l < f->c.max_level && emax > tol)
        fl = 1;
      else if (l > 1 && emax < ctol)
        fl = -1;
      flags[b] = fl;
      if (emax_out) emax_out[b] = emax;
    }
    scratch_free(&w);
    free(rho);
    free(prs);
  }
  if (err) return fail(ORC_ENOMEM, "out of memory");
  return ORC_OK;
}

int orc_padded_block(orc_forest* f, int64_t leaf, double* out, int64_t n_doubles) {
  if (!f || !out || leaf < 0 || leaf >= f->n) return fail(ORC_EINVAL, "bad argument");
  if (n_doubles != (int64_t)f->nvar * f->npad) return fail(ORC_EINVAL, "size mismatch");
  double* Wc = (double*)malloc(sizeof(double) * f->nvar * f->npad);
  if (!Wc) return fail(ORC_ENOMEM, "out of memory");
  fill_all(f, f->U, leaf, out, Wc);
  free(Wc);
  return ORC_OK;
}

int orc_face_flux(orc_forest* f, const double* vl, const double* vr, int dir, double* F) {
  if (!f || !vl || !vr || !F || dir < 0 || dir >= f->nd) return fail(ORC_EINVAL, "bad argument");
  riemann(f, vl, vr, dir, F);
  return ORC_OK;
}

int orc_lohner_cells(orc_forest* f, int64_t leaf, double* out, int64_t n_doubles) {
  if (!f || !out || leaf < 0 || leaf >= f->n) return fail(ORC_EINVAL, "bad argument");
  if (n_doubles != f->ncell) return fail(ORC_EINVAL, "size mismatch");
  scratch w;
  double* rho = (double*)malloc(sizeof(double) * f->npad);
  double* prs = (double*)malloc(sizeof(double) * f->npad);
  int ok = scratch_alloc(f, &w) && rho && prs;
  if (ok) {
    fill_all(f, f->U, leaf, w.W, w.Wc);
    padded_prim(f, w.W, w.P);
    for (int64_t c = 0; c < f->npad; c++) {
      rho[c] = w.P[c];
      prs[c] = f->poly ? poly_p(f, w.P[c]) : w.P[(int64_t)iE(f) * f->npad + c];
    }
    for (int k = 0; k < f->nx[2]; k++)
      for (int j = 0; j < f->nx[1]; j++)
        for (int i = 0; i < f->nx[0]; i++) {
          int x[3] = {i, j, k};
          out[cidx(f, i, j, k)] =
              f->c.lohner_w_rho * lohner_cell(f, rho, x) + f->c.lohner_w_p * lohner_cell(f, prs, x);
        }
  }
  scratch_free(&w);
  free(rho);
  free(prs);
  return ok ? ORC_OK : fail(ORC_ENOMEM, "out of memory");
}

/* ------------------------------------------------------------------ */
/* regridding (Sec. 1.3): refine flagged blocks into 2^ndim children,   */
/* coarsen complete sibling groups whose members are all flagged for    */
/* coarsening, keep the forest 2:1 balanced                             */
/* ------------------------------------------------------------------ */

/* Leaves touching block (l, c) across offset o (each o_d in -1, 0, 1): the
 * leaf covering the neighbouring block region at level l, l-1 or l-2, or the
 * leaves at levels l+1 and l+2 inside it that touch block (l, c).  Calls
 * visit(leaf) for each; returns 0 if the region lies outside a non-periodic
 * domain. */
typedef void (*leaf_visit)(const orc_forest* f, int64_t leaf, void* ctx);

static void touching_finer(const orc_forest* f, int l, const int64_t r[3], const int o[3], int depth,
                           leaf_visit visit, void* ctx) {
  /* leaves at level l+depth inside region (l, r) that touch its side facing -o */
  int64_t span = (int64_t)1 << depth;
  int64_t lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  for (int e = 0; e < f->nd; e++) {
    lo[e] = r[e] * span;
    hi[e] = lo[e] + span;
    if (o[e] == 1) hi[e] = lo[e] + 1;         /* neighbour on the +side: its low layer touches */
    if (o[e] == -1) lo[e] = hi[e] - 1;        /* neighbour on the -side: its high layer touches */
  }
  for (int64_t k = lo[2]; k < hi[2]; k++)
    for (int64_t j = lo[1]; j < hi[1]; j++)
      for (int64_t i = lo[0]; i < hi[0]; i++) {
        int64_t c[3] = {i, j, k};
        int64_t x = lookup(f, l + depth, c);
        if (x >= 0) visit(f, x, ctx);
      }
}

static int touching_leaves(const orc_forest* f, int l, const int64_t c[3], const int o[3], leaf_visit visit,
                           void* ctx) {
  int64_t r[3] = {c[0], c[1], c[2]};
  for (int e = 0; e < f->nd; e++) {
    r[e] += o[e];
    if (!wrap(f, e, &r[e], nblk(f, l, e))) return 0;
  }
  for (int up = 0; up <= 2 && l - up >= 1; up++) {
    int64_t p[3] = {r[0] >> up, r[1] >> up, r[2] >> up};
    for (int e = f->nd; e < 3; e++) p[e] = 0;
    int64_t x = lookup(f, l - up, p);
    if (x >= 0) {
      visit(f, x, ctx);
      return 1;
    }
  }
  for (int depth = 1; depth <= 2; depth++) touching_finer(f, l, r, o, depth, visit, ctx);
  return 1;
}

typedef struct {
  int32_t* tgt;
  int lvl;       /* refine: the refining leaf's level; coarsen: the group's level */
  int changed;   /* refine: a coarser neighbour was marked */
  int violates;  /* coarsen: a neighbour ends finer than the group level */
} regrid_ctx;

/* refining a leaf of level l puts children at l+1: a touching leaf of level
 * l-1 must refine too (2:1 balance over faces, edges and corners) */
static void visit_refine(const orc_forest* f, int64_t a, void* p) {
  regrid_ctx* x = (regrid_ctx*)p;
  if (f->lev[a] == x->lvl - 1 && x->tgt[a] == f->lev[a]) {
    x->tgt[a] = f->lev[a] + 1;
    x->changed = 1;
  }
}

/* a group of level l coarsens to l-1: every touching leaf must end at a
 * level <= l */
static void visit_coarsen(const orc_forest* f, int64_t a, void* p) {
  regrid_ctx* x = (regrid_ctx*)p;
  (void)f;
  if (x->tgt[a] > x->lvl) x->violates = 1;
}

static void offsets(int nd, int idx, int o[3]) {
  /* idx in 0 .. 3^nd - 1 -> offset vector in {-1,0,1}^nd */
  for (int e = 0; e < 3; e++) {
    o[e] = e < nd ? idx % 3 - 1 : 0;
    idx /= 3;
  }
}

int orc_regrid_plan(const orc_forest* f, const int8_t* flags, int64_t cap, int64_t* new_n, int32_t* new_lev,
                    int32_t* new_ijk) {
  if (!f || !flags || !new_n || cap < 0 || (cap > 0 && (!new_lev || !new_ijk)))
    return fail(ORC_EINVAL, "null argument");
  const int nd = f->nd, nch = 1 << nd, noff = nd == 1 ? 3 : (nd == 2 ? 9 : 27);
  int32_t* tgt = (int32_t*)malloc(sizeof(int32_t) * f->n);
  int64_t* grp = (int64_t*)malloc(sizeof(int64_t) * f->n); /* first member of the coarsening group, or -1 */
  if (!tgt || !grp) {
    free(tgt);
    free(grp);
    return fail(ORC_ENOMEM, "out of memory");
  }
  /* 1. requested refinements */
  for (int64_t b = 0; b < f->n; b++) {
    tgt[b] = f->lev[b] + ((flags[b] > 0 && f->lev[b] < f->c.max_level) ? 1 : 0);
    grp[b] = -1;
  }
  /* 2. balance: refine coarser touching leaves until nothing changes */
  regrid_ctx x = {tgt, 0, 1, 0};
  while (x.changed) {
    x.changed = 0;
    for (int64_t b = 0; b < f->n; b++) {
      if (tgt[b] == f->lev[b]) continue;
      int64_t c[3] = {f->ijk[3 * b], f->ijk[3 * b + 1], f->ijk[3 * b + 2]};
      x.lvl = f->lev[b];
      for (int i = 0; i < noff; i++) {
        int o[3];
        offsets(nd, i, o);
        if (o[0] == 0 && o[1] == 0 && o[2] == 0) continue;
        touching_leaves(f, f->lev[b], c, o, visit_refine, &x);
      }
    }
  }
  /* 3. coarsening: complete sibling groups, all flagged -1, none refining,
   * whose parent would stay balanced against the final levels of step 2 */
  for (int64_t b = 0; b < f->n; b++) {
    int l = f->lev[b];
    if (flags[b] >= 0 || l <= 1 || tgt[b] != l || grp[b] >= 0) continue;
    int64_t P[3] = {f->ijk[3 * b] >> 1, f->ijk[3 * b + 1] >> 1, f->ijk[3 * b + 2] >> 1};
    for (int e = nd; e < 3; e++) P[e] = 0;
    int64_t mem[8];
    int ok = 1;
    for (int q = 0; q < nch && ok; q++) {
      int64_t ch[3] = {0, 0, 0};
      for (int e = 0; e < nd; e++) ch[e] = 2 * P[e] + ((q >> e) & 1);
      mem[q] = lookup(f, l, ch);
      if (mem[q] < 0 || flags[mem[q]] >= 0 || tgt[mem[q]] != l) ok = 0;
    }
    if (!ok) continue;
    regrid_ctx y = {tgt, l, 0, 0};
    for (int i = 0; i < noff; i++) {
      int o[3];
      offsets(nd, i, o);
      if (o[0] == 0 && o[1] == 0 && o[2] == 0) continue;
      touching_leaves(f, l - 1, P, o, visit_coarsen, &y);
    }
    if (y.violates) continue;
    int64_t first = mem[0];
    for (int q = 1; q < nch; q++)
      if (mem[q] < first) first = mem[q];
    for (int q = 0; q < nch; q++) grp[mem[q]] = first;
  }
  /* 4. the new leaf list: unchanged leaves in place, a refined leaf replaced
   * by its children (child index ox + 2 oy + 4 oz), a coarsened group by its
   * parent at the position of the group's first member */
  int64_t m = 0;
  for (int64_t b = 0; b < f->n; b++) {
    if (grp[b] >= 0 && grp[b] != b) continue;
    int cnt = (tgt[b] > f->lev[b]) ? nch : 1;
    for (int q = 0; q < cnt; q++, m++) {
      if (m >= cap) continue;
      if (grp[b] == b) {
        new_lev[m] = f->lev[b] - 1;
        for (int e = 0; e < 3; e++) new_ijk[3 * m + e] = e < nd ? f->ijk[3 * b + e] >> 1 : 0;
      } else if (cnt > 1) {
        new_lev[m] = f->lev[b] + 1;
        for (int e = 0; e < 3; e++) new_ijk[3 * m + e] = e < nd ? 2 * f->ijk[3 * b + e] + ((q >> e) & 1) : 0;
      } else {
        new_lev[m] = f->lev[b];
        for (int e = 0; e < 3; e++) new_ijk[3 * m + e] = f->ijk[3 * b + e];
      }
    }
  }
  free(tgt);
  free(grp);
  *new_n = m;
  if (m > cap) return fail(ORC_ENOMEM, "capacity %lld below the new leaf count %lld", (long long)cap, (long long)m);
  return ORC_OK;
}

/* Move the state of `from` onto the leaves of `to`, a forest whose every leaf
 * is a leaf of `from`, a child of one (refinement: conservative linear
 * prolongation of the parent's cells, the same formula as for coarse-fine
 * ghosts, with the parent's ghost cells for its boundary cells), or the
 * parent of 2^ndim leaves of `from` (coarsening: restriction, the pairwise
 * tree sum of the children's cells times 2^-ndim). */
int orc_regrid_transfer(orc_forest* from, orc_forest* to) {
  if (!from || !to) return fail(ORC_EINVAL, "null argument");
  const orc_config *a = &from->c, *b = &to->c;
  int same = a->ndim == b->ndim && a->physics == b->physics && a->max_level == b->max_level;
  for (int d = 0; d < 3; d++)
    same = same && a->block_nx[d] == b->block_nx[d] && a->base_blocks[d] == b->base_blocks[d] &&
           a->bc[d][0] == b->bc[d][0];
  if (!same) return fail(ORC_EINVAL, "the two forests differ in their configuration");
  const orc_forest* f = from;
  const int nd = f->nd, nv = f->nvar, nch = 1 << nd;
  /* classify every new leaf first, so that a bad target changes nothing */
  int64_t* src = (int64_t*)malloc(sizeof(int64_t) * to->n * 8);
  int8_t* how = (int8_t*)malloc(to->n);
  double* W = (double*)malloc(sizeof(double) * nv * f->npad);
  double* Wc = (double*)malloc(sizeof(double) * nv * f->npad);
  double* out = (double*)malloc(sizeof(double) * nv * to->n * to->ncell);
  if (!src || !how || !W || !Wc || !out) {
    free(src), free(how), free(W), free(Wc), free(out);
    return fail(ORC_ENOMEM, "out of memory");
  }
  int bad = 0;
  for (int64_t n = 0; n < to->n && !bad; n++) {
    int l = to->lev[n];
    int64_t c[3] = {to->ijk[3 * n], to->ijk[3 * n + 1], to->ijk[3 * n + 2]};
    int64_t x = lookup(f, l, c);
    if (x >= 0) {
      how[n] = 0;
      src[8 * n] = x;
      continue;
    }
    int64_t p[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
    for (int e = nd; e < 3; e++) p[e] = 0;
    x = l > 1 ? lookup(f, l - 1, p) : -1;
    if (x >= 0) {
      how[n] = 1;
      src[8 * n] = x;
      continue;
    }
    how[n] = 2;
    for (int q = 0; q < nch; q++) {
      int64_t ch[3] = {0, 0, 0};
      for (int e = 0; e < nd; e++) ch[e] = 2 * c[e] + ((q >> e) & 1);
      src[8 * n + q] = lookup(f, l + 1, ch);
      if (src[8 * n + q] < 0) bad = 1;
    }
  }
  if (bad) {
    free(src), free(how), free(W), free(Wc), free(out);
    return fail(ORC_EINVAL, "the target forest is not a one-level regrid of the source forest");
  }
  const int h[3] = {f->nx[0] / 2, nd > 1 ? f->nx[1] / 2 : 0, nd > 2 ? f->nx[2] / 2 : 0};
  free(W);
  free(Wc);
  int oom = 0;
#pragma omp parallel
  {
    double* W = (double*)malloc(sizeof(double) * nv * f->npad);
    double* Wc = (double*)malloc(sizeof(double) * nv * f->npad);
    if (!W || !Wc) {
#pragma omp atomic write
      oom = 1;
    }
#pragma omp for schedule(dynamic, 4)
  for (int64_t n = 0; n < to->n; n++) {
    if (oom) continue;
    if (how[n] == 1) fill_all(f, f->U, src[8 * n], W, Wc);
    for (int k = 0; k < f->nx[2]; k++)
      for (int j = 0; j < f->nx[1]; j++)
        for (int i = 0; i < f->nx[0]; i++) {
          int x[3] = {i, j, k};
          int64_t dst = cidx(f, i, j, k);
          for (int v = 0; v < nv; v++) {
            double r;
            if (how[n] == 0) {
              r = st(f, f->U, v, src[8 * n], dst);
            } else if (how[n] == 1) {
              /* child offset within the parent and the parent cell */
              int pc[3] = {0, 0, 0};
              for (int e = 0; e < nd; e++) pc[e] = (int)(to->ijk[3 * n + e] & 1) * h[e] + x[e] / 2;
              const double* w = W + (int64_t)v * f->npad;
              double u0 = w[pidx(f, pc[0], pc[1], pc[2])];
              r = u0;
              for (int e = 0; e < nd; e++) {
                int lo[3] = {pc[0], pc[1], pc[2]}, hi[3] = {pc[0], pc[1], pc[2]};
                lo[e] -= 1;
                hi[e] += 1;
                double t = 0.25 * minmod(u0 - w[pidx(f, lo[0], lo[1], lo[2])], w[pidx(f, hi[0], hi[1], hi[2])] - u0);
                r = (x[e] & 1) ? r + t : r - t;
              }
            } else {
              /* the child holding this cell, and its 2^ndim fine cells */
              int q = 0, y[3] = {0, 0, 0};
              for (int e = 0; e < nd; e++) {
                int qe = x[e] / h[e];
                q |= qe << e;
                y[e] = 2 * (x[e] - qe * h[e]);
              }
              double c8[8];
              for (int a2 = 0; a2 < nch; a2++) {
                int z[3] = {y[0], y[1], y[2]};
                for (int e = 0; e < nd; e++) z[e] += (a2 >> e) & 1;
                c8[a2] = st(f, f->U, v, src[8 * n + q], cidx(f, z[0], z[1], z[2]));
              }
              if (nd == 1)
                r = (c8[0] + c8[1]) * 0.5;
              else if (nd == 2)
                r = ((c8[0] + c8[1]) + (c8[2] + c8[3])) * 0.25;
              else
                r = (((c8[0] + c8[1]) + (c8[2] + c8[3])) + ((c8[4] + c8[5]) + (c8[6] + c8[7]))) * 0.125;
            }
            out[((int64_t)v * to->n + n) * to->ncell + dst] = r;
          }
        }
  }
    free(W);
    free(Wc);
  }
  if (oom) {
    free(src), free(how), free(out);
    return fail(ORC_ENOMEM, "out of memory");
  }
  memcpy(to->U, out, sizeof(double) * nv * to->n * to->ncell);
  free(src), free(how), free(out);
  return ORC_OK;
}
