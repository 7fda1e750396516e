// physics.hpp -- device-side physics of the finite-volume update (gfx950, binary64).
//
// Hydrodynamics: U = (rho, rho v, E), E = rho v^2/2 + p/(gamma-1)
// (arXiv 2004.03275, Sec. 1.1); primitive V = (rho, v, p) (Sec. 1.2,
// phys_to_primitive / phys_to_conserved).  Ideal MHD (mu0 = 1) adds B and the
// GLM scalar psi.  Fluxes: TVDLF (Rusanov), HLL, HLLC (Sec. 1.2, Sec. 2.4),
// all with the textbook formulas; the expression order below is fixed so that
// every result is reproducible bit for bit (built with -ffp-contract=off).
//
// Division, reciprocal, square root and the sound speed of the hydrodynamic
// systems go through ddiv, drcp, dsqrt and dsound.  They are the correctly
// rounded operations, except in the fast-arithmetic unit (AMRV_FAST_MATH,
// stage_fast.hip, built with contraction on), where they come from the
// hardware reciprocal and reciprocal square root refined by Newton steps:
// each result within a few ulp of the correctly rounded one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace amrv {

enum { FLX_TVDLF = 0, FLX_HLL = 1, FLX_HLLC = 2 };
enum { LIM_MINMOD = 0, LIM_VANLEER = 1, LIM_MC = 2, LIM_KOREN = 3, LIM_CADA = 4 };

// limiters whose slope toward a face depends on which face (not symmetric in
// the two differences): a cell keeps two slopes
template <int LIM>
constexpr bool lim_asym() { return LIM == LIM_KOREN || LIM == LIM_CADA; }

struct PhysParams {
  double gamma;
  double gm1;   // gamma - 1
  double igm1;  // 1 / (gamma - 1)
  double ch;    // GLM cleaning speed (MHD)
  double cad;   // c_ad of the polytrope
  double gcad;  // gamma * c_ad
};

template <int ND, int PH>
struct Sys {
  static constexpr int NV = PH == PH_MHD ? 3 + 2 * ND : PH == PH_POLY ? 1 + ND : 2 + ND;
  static constexpr int IE = 1 + ND;   // energy / pressure (Euler, MHD)
  static constexpr int IB = 2 + ND;   // first magnetic component
  static constexpr int IP = 2 + 2 * ND;  // psi
};

#ifdef AMRV_FAST_MATH
// 1/b: hardware reciprocal, then two Newton steps y += y (1 - b y)
__device__ __forceinline__ double drcp(double b) {
  double y = __builtin_amdgcn_rcp(b);
  y = __builtin_fma(y, __builtin_fma(-b, y, 1.0), y);
  y = __builtin_fma(y, __builtin_fma(-b, y, 1.0), y);
  return y;
}
// a/b: a times the refined reciprocal, then one residual correction
// q += y (a - b q) (Markstein's final step)
__device__ __forceinline__ double ddiv(double a, double b) {
  const double y = drcp(b);
  const double q = a * y;
  return __builtin_fma(y, __builtin_fma(-b, q, a), q);
}
// x^(-1/2) for x > 0: hardware estimate, then two Newton steps
// y += (y/2)(1 - x y^2)
__device__ __forceinline__ double drsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
  y = __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
  return y;
}
// sqrt(x) for x > 0: g = x y with y ~ x^(-1/2), then the residual
// correction g += (y/2)(x - g^2)
__device__ __forceinline__ double dsqrt(double x) {
  const double y = drsq(x);
  const double g = x * y;
  return __builtin_fma(0.5 * y, __builtin_fma(-g, g, x), g);
}
// sqrt(gp / rho) = gp (gp rho)^(-1/2): one reciprocal square root instead of
// a division and a square root
__device__ __forceinline__ double dsound(double gp, double rho) { return gp * drsq(gp * rho); }
// sqrt(x) for x >= 0 (the estimate alone would give 0 * inf at 0)
__device__ __forceinline__ double dsqrt0(double x) { return x == 0.0 ? x : dsqrt(x); }
#else
__device__ __forceinline__ double drcp(double b) { return 1.0 / b; }
__device__ __forceinline__ double ddiv(double a, double b) { return a / b; }
__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ double dsound(double gp, double rho) { return sqrt(gp / rho); }
__device__ __forceinline__ double dsqrt0(double x) { return sqrt(x); }
#endif

__device__ __forceinline__ double dmin(double a, double b) { return a < b ? a : b; }
__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }

// rho^e of the polytrope: the exponents 1 and 2 are exact (rho*rho), others
// go through pow (exponent 0 gives 1)
__device__ __forceinline__ double rpow(double r, double e) { return e == 1.0 ? r : e == 2.0 ? r * r : pow(r, e); }

// pressure of a primitive state: its own entry, or c_ad rho^gamma
template <int ND, int PH>
__device__ __forceinline__ double pressure(const double* v, const PhysParams& P) {
  if constexpr (PH == PH_POLY)
    return P.cad * rpow(v[0], P.gamma);
  else
    return v[Sys<ND, PH>::IE];
}

// rho <= 0, p <= 0 or NaN; the polytrope (whose pressure is positive with
// rho): rho <= 0 or a velocity that is NaN or overflows
template <int ND, int PH>
__device__ __forceinline__ bool nonphysical(const double* v) {
  if constexpr (PH == PH_POLY) {
    double vv = v[1] * v[1];
#pragma unroll
    for (int d = 1; d < ND; d++) vv = vv + v[1 + d] * v[1 + d];
    return !(v[0] > 0.0) || !(vv < __builtin_huge_val());
  } else {
    return !(v[0] > 0.0) || !(v[Sys<ND, PH>::IE] > 0.0);
  }
}

// conserved -> primitive: 1/rho once, v = m * (1/rho),
// p = (gamma-1) * ((E - (0.5*m.m)*(1/rho)) [- 0.5*B.B]); the polytrope's
// primitive state is (rho, v)
template <int ND, int PH>
__device__ __forceinline__ void cons2prim(const double* u, double* v, const PhysParams& P) {
  using S = Sys<ND, PH>;
  const double rho = u[0];
  const double inv = drcp(rho);
  double mm = u[1] * u[1];
  v[0] = rho;
  v[1] = u[1] * inv;
#pragma unroll
  for (int d = 1; d < ND; d++) {
    v[1 + d] = u[1 + d] * inv;
    mm = mm + u[1 + d] * u[1 + d];
  }
  if constexpr (PH == PH_POLY) {
    return;
  } else if constexpr (PH == PH_EULER) {
    v[S::IE] = P.gm1 * (u[S::IE] - 0.5 * mm * inv);
  } else {
    double bb = u[S::IB] * u[S::IB];
    v[S::IB] = u[S::IB];
#pragma unroll
    for (int d = 1; d < ND; d++) {
      bb = bb + u[S::IB + d] * u[S::IB + d];
      v[S::IB + d] = u[S::IB + d];
    }
    v[S::IE] = P.gm1 * (u[S::IE] - 0.5 * mm * inv - 0.5 * bb);
    v[S::IP] = u[S::IP];
  }
}

// primitive -> conserved: m = rho v, E = p*(1/(gamma-1)) + (0.5*rho)*v.v [+ 0.5*B.B]
template <int ND, int PH>
__device__ __forceinline__ void prim2cons(const double* v, double* u, const PhysParams& P) {
  using S = Sys<ND, PH>;
  const double rho = v[0];
  double vv = v[1] * v[1];
  u[0] = rho;
  u[1] = rho * v[1];
#pragma unroll
  for (int d = 1; d < ND; d++) {
    u[1 + d] = rho * v[1 + d];
    vv = vv + v[1 + d] * v[1 + d];
  }
  if constexpr (PH == PH_POLY) {
    return;
  } else if constexpr (PH == PH_EULER) {
    u[S::IE] = v[S::IE] * P.igm1 + 0.5 * rho * vv;
  } else {
    double bb = v[S::IB] * v[S::IB];
    u[S::IB] = v[S::IB];
#pragma unroll
    for (int d = 1; d < ND; d++) {
      bb = bb + v[S::IB + d] * v[S::IB + d];
      u[S::IB + d] = v[S::IB + d];
    }
    u[S::IE] = v[S::IE] * P.igm1 + 0.5 * rho * vv + 0.5 * bb;
    u[S::IP] = v[S::IP];
  }
}

// physical flux normal to direction n (compile-time)
template <int ND, int PH, int N>
__device__ __forceinline__ void phys_flux(const double* v, const double* u, double* F, const PhysParams& P) {
  using S = Sys<ND, PH>;
  const double vn = v[1 + N];
  const double p = pressure<ND, PH>(v, P);
  F[0] = u[1 + N];
  if constexpr (PH == PH_POLY) {
#pragma unroll
    for (int d = 0; d < ND; d++) {
      F[1 + d] = u[1 + d] * vn;
      if (d == N) F[1 + d] = F[1 + d] + p;
    }
  } else if constexpr (PH == PH_EULER) {
#pragma unroll
    for (int d = 0; d < ND; d++) {
      F[1 + d] = u[1 + d] * vn;
      if (d == N) F[1 + d] = F[1 + d] + p;
    }
    F[S::IE] = (u[S::IE] + p) * vn;
  } else {
    const double* B = v + S::IB;
    double bb = B[0] * B[0];
    double vB = v[1] * B[0];
#pragma unroll
    for (int d = 1; d < ND; d++) {
      bb = bb + B[d] * B[d];
      vB = vB + v[1 + d] * B[d];
    }
    const double pt = p + 0.5 * bb;
#pragma unroll
    for (int d = 0; d < ND; d++) {
      F[1 + d] = u[1 + d] * vn - B[d] * B[N];
      if (d == N) F[1 + d] = F[1 + d] + pt;
    }
    F[S::IE] = (u[S::IE] + pt) * vn - B[N] * vB;
#pragma unroll
    for (int d = 0; d < ND; d++) F[S::IB + d] = (d == N) ? 0.0 : B[d] * vn - B[N] * v[1 + d];
    F[S::IP] = 0.0;
  }
}

// signal speed: sound speed sqrt((gamma*p)/rho), the polytrope's
// sqrt((gamma*c_ad) * rho^(gamma-1)), or the MHD fast speed along N
template <int ND, int PH, int N>
__device__ __forceinline__ double wave_speed(const double* v, const PhysParams& P) {
  using S = Sys<ND, PH>;
  if constexpr (PH == PH_POLY) {
    return dsqrt(P.gcad * rpow(v[0], P.gm1));
  } else if constexpr (PH == PH_EULER) {
    return dsound(P.gamma * v[S::IE], v[0]);
  } else {
    const double irho = drcp(v[0]);
    double bb = v[S::IB] * v[S::IB];
#pragma unroll
    for (int d = 1; d < ND; d++) bb = bb + v[S::IB + d] * v[S::IB + d];
    const double a2 = P.gamma * v[S::IE] * irho;
    const double b2 = bb * irho;
    const double bn2 = v[S::IB + N] * v[S::IB + N] * irho;
    const double s = a2 + b2;
    double disc = s * s - 4.0 * a2 * bn2;
    if (!(disc > 0.0)) disc = 0.0;
    return dsqrt0(0.5 * (s + dsqrt0(disc)));
  }
}

// runtime-direction wrapper
template <int ND, int PH>
__device__ __forceinline__ double wave_speed_dir(const double* v, int n, const PhysParams& P) {
  if (n == 0) return wave_speed<ND, PH, 0>(v, P);
  if constexpr (ND > 1) {
    if (n == 1) return wave_speed<ND, PH, (ND > 1 ? 1 : 0)>(v, P);
  }
  if constexpr (ND > 2) return wave_speed<ND, PH, (ND > 2 ? 2 : 0)>(v, P);
  return 0.0;
}

// limited slope of a cell toward a face from the difference a away from it
// and b toward it: minmod (smaller magnitude), van Leer (harmonic mean
// 2ab/(a+b)), monotonized central (smallest magnitude of 2a, (a+b)/2, 2b),
// Koren (smallest of 2a, (a+2b)/3, 2b); zero at extrema.  All but Koren are
// symmetric in a and b, bit for bit.  Cada's third-order limiter (LimO3 of
// Cada and Torrilhon 2009) is b H(a/b) with
// H(t) = max(0, min(p3, max(-t/2, min(2t, p3, 1.6)))), p3 = (2 + t)/3: for
// b > 0 the candidates scale by b exactly, b < 0 is the odd mirror, b = 0
// gives 0, as does a = 0; it keeps a slope at extrema (-2 < a/b < 0).  With
// that paper's smoothness switch (thr2 = (r dx)^2 > 0) it is the unlimited
// third-order slope (a + 2b)/3 where a^2 + b^2 <= thr2.
template <int LIM>
__device__ __forceinline__ double limiter(double a, double b, double thr2 = 0.0) {
  if constexpr (LIM == LIM_CADA) {
    if (a == 0.0 && b == 0.0) return 0.0;  // flat: every branch gives 0
    if (thr2 > 0.0 && a * a + b * b <= thr2) return ddiv(a + 2.0 * b, 3.0);
    if (a == 0.0 || b == 0.0) return 0.0;  // H bounded, H(0) = 0
    const double sg = b > 0.0 ? 1.0 : -1.0;
    const double ap = sg * a, bp = sg * b;
    const double p3 = ddiv(ap + 2.0 * bp, 3.0);
    double in = 2.0 * ap;
    in = p3 < in ? p3 : in;
    in = 1.6 * bp < in ? 1.6 * bp : in;
    double m = -0.5 * ap;
    m = in > m ? in : m;
    m = m < p3 ? m : p3;
    m = m > 0.0 ? m : 0.0;
    return sg * m;
  }
  if (a * b <= 0.0) return 0.0;
  if constexpr (LIM == LIM_MINMOD) {
    return fabs(a) < fabs(b) ? a : b;
  } else if constexpr (LIM == LIM_MC || LIM == LIM_KOREN) {
    const double ta = 2.0 * a, tb = 2.0 * b;
    const double c = LIM == LIM_MC ? 0.5 * (a + b) : ddiv(a + 2.0 * b, 3.0);
    const double m = fabs(ta) < fabs(tb) ? ta : tb;
    return fabs(c) < fabs(m) ? c : m;
  } else {
    return ddiv(2.0 * a * b, a + b);
  }
}

__device__ __forceinline__ double minmod(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  return fabs(a) < fabs(b) ? a : b;
}

// HLLC flux (hydrodynamics) normal to N.  Every branch needs the conserved
// state and physical flux of one side only (F_L and F*_L use the left state,
// F*_R and F_R the right one), so the side is chosen first from the wave
// speeds and only its state and flux are formed.  The arithmetic of each
// quantity is the textbook one in a fixed order.
template <int ND, int N>
__device__ __forceinline__ void hllc_flux(const double* vl, const double* vr, double* F, const PhysParams& P) {
  using S = Sys<ND, PH_EULER>;
  constexpr int NV = S::NV, ie = S::IE;
  const double cl = wave_speed<ND, PH_EULER, N>(vl, P);
  const double cr = wave_speed<ND, PH_EULER, N>(vr, P);
  const double unl = vl[1 + N], unr = vr[1 + N];
  const double sl = dmin(unl - cl, unr - cr);
  const double sr = dmax(unl + cl, unr + cr);
  const double pl = vl[ie], pr = vr[ie];
  const double rl = vl[0] * (sl - unl);
  const double rr = vr[0] * (sr - unr);
  const double sm = ddiv((pr - pl) + unl * rl - unr * rr, rl - rr);
  const bool left = sl >= 0.0 || sm >= 0.0;
  const bool star = !(sl >= 0.0) && (sm >= 0.0 || sr > 0.0);
  double vk[NV];
#pragma unroll
  for (int k = 0; k < NV; k++) vk[k] = left ? vl[k] : vr[k];
  double uk[NV], fk[NV];
  prim2cons<ND, PH_EULER>(vk, uk, P);
  phys_flux<ND, PH_EULER, N>(vk, uk, fk, P);
  if (star) {
    // star state rho_K (S_K - u_K)/(S_K - S_M) (1, S_M, v_t, .); energy in the
    // star-pressure form E* = ((S_K - u_K) E_K - p_K u_K + p* S_M)/(S_K - S_M),
    // p* = p_K + rho_K (S_K - u_K)(S_M - u_K): one reciprocal serves both
    const double sk = left ? sl : sr;
    const double rk = left ? rl : rr;
    const double unk = vk[1 + N], pk = vk[ie];
    const double inv = drcp(sk - sm);
    const double coef = rk * inv;
    const double ps = pk + rk * (sm - unk);
    double us[NV];
    us[0] = coef;
#pragma unroll
    for (int d = 0; d < ND; d++) us[1 + d] = (d == N) ? coef * sm : coef * vk[1 + d];
    us[ie] = ((sk - unk) * uk[ie] - pk * unk + ps * sm) * inv;
#pragma unroll
    for (int k = 0; k < NV; k++) F[k] = fk[k] + sk * (us[k] - uk[k]);
  } else {
#pragma unroll
    for (int k = 0; k < NV; k++) F[k] = fk[k];
  }
}

// HLLC for MHD after Li (2005): total pressure p_T = p + B.B/2 in the
// contact speed and star pressure, the GLM normal field on both sides
// (already in vl, vr); in the star region the transverse velocity and field
// are the HLL state's (the same on both sides), or where B_n = 0 the side's
// own velocity and its field compressed like the density; star energy
// E* = ((S_K-u_K) E_K - p_TK u_K + p_T* S_M + B_n (v_K.B_K - v*.B*)) / (S_K-S_M).
template <int ND, int N>
__device__ __forceinline__ void hllc_mhd(const double* vl, const double* vr, const double* ul, const double* ur,
                                         const double* fl, const double* fr, double cl, double cr, double* F) {
  using S = Sys<ND, PH_MHD>;
  constexpr int NV = S::NV, ie = S::IE, ib = S::IB;
  const double unl = vl[1 + N], unr = vr[1 + N];
  const double sl = dmin(unl - cl, unr - cr);
  const double sr = dmax(unl + cl, unr + cr);
  if (sl >= 0.0) {
#pragma unroll
    for (int k = 0; k < NV; k++) F[k] = fl[k];
    return;
  }
  if (sr <= 0.0) {
#pragma unroll
    for (int k = 0; k < NV; k++) F[k] = fr[k];
    return;
  }
  double bbl = vl[ib] * vl[ib], bbr = vr[ib] * vr[ib];
#pragma unroll
  for (int d = 1; d < ND; d++) {
    bbl = bbl + vl[ib + d] * vl[ib + d];
    bbr = bbr + vr[ib + d] * vr[ib + d];
  }
  const double ptl = vl[ie] + 0.5 * bbl, ptr = vr[ie] + 0.5 * bbr;
  const double rl = vl[0] * (sl - unl);
  const double rr = vr[0] * (sr - unr);
  const double sm = ddiv((ptr - ptl) + unl * rl - unr * rr, rl - rr);
  const double ids = drcp(sr - sl);
  double uh[NV];  // HLL state of density, momenta and field
#pragma unroll
  for (int k = 0; k <= ND; k++) uh[k] = ((sr * ur[k] - sl * ul[k]) - (fr[k] - fl[k])) * ids;
#pragma unroll
  for (int d = 0; d < ND; d++) uh[ib + d] = ((sr * ur[ib + d] - sl * ul[ib + d]) - (fr[ib + d] - fl[ib + d])) * ids;
  const bool left = sm >= 0.0;
  double vk[NV], uk[NV], fk[NV];
#pragma unroll
  for (int k = 0; k < NV; k++) {
    vk[k] = left ? vl[k] : vr[k];
    uk[k] = left ? ul[k] : ur[k];
    fk[k] = left ? fl[k] : fr[k];
  }
  const double sk = left ? sl : sr;
  const double rk = left ? rl : rr;
  const double unk = vk[1 + N], ptk = left ? ptl : ptr;
  const double inv = drcp(sk - sm);
  const double coef = rk * inv;
  const double pts = ptk + rk * (sm - unk);
  const double bn = vk[ib + N];
  double vs[ND], bs[ND];
#pragma unroll
  for (int d = 0; d < ND; d++) {
    if (d == N) {
      vs[d] = sm;
      bs[d] = bn;
    } else if (bn == 0.0) {
      vs[d] = vk[1 + d];
      bs[d] = vk[ib + d] * ((sk - unk) * inv);
    } else {
      vs[d] = ddiv(uh[1 + d], uh[0]);
      bs[d] = uh[ib + d];
    }
  }
  double vbk = vk[1] * vk[ib], vbs = vs[0] * bs[0];
#pragma unroll
  for (int d = 1; d < ND; d++) {
    vbk = vbk + vk[1 + d] * vk[ib + d];
    vbs = vbs + vs[d] * bs[d];
  }
  double us[NV];
  us[0] = coef;
#pragma unroll
  for (int d = 0; d < ND; d++) {
    us[1 + d] = coef * vs[d];
    us[ib + d] = bs[d];
  }
  us[ie] = ((sk - unk) * uk[ie] - ptk * unk + pts * sm + bn * (vbk - vbs)) * inv;
  us[S::IP] = uk[S::IP];
#pragma unroll
  for (int k = 0; k < NV; k++) F[k] = fk[k] + sk * (us[k] - uk[k]);
}

// Approximate Riemann flux normal to N from left/right primitive face states.
// vl/vr are modified only for MHD (normal field replaced by the GLM value).
template <int ND, int PH, int FLUX, int N>
__device__ __forceinline__ void riemann(double* vl, double* vr, double* F, const PhysParams& P) {
  using S = Sys<ND, PH>;
  constexpr int NV = S::NV;
  static_assert(!(PH == PH_POLY && FLUX == FLX_HLLC), "HLLC needs the energy equation");
  if constexpr (FLUX == FLX_HLLC && PH == PH_EULER) {
    hllc_flux<ND, N>(vl, vr, F, P);
    return;
  } else {
    double bns = 0.0, psis = 0.0;
    if constexpr (PH == PH_MHD) {
      constexpr int ib = S::IB + N, ip = S::IP;
      bns = 0.5 * (vl[ib] + vr[ib]) - ddiv(0.5 * (vr[ip] - vl[ip]), P.ch);
      psis = 0.5 * (vl[ip] + vr[ip]) - 0.5 * P.ch * (vr[ib] - vl[ib]);
      vl[ib] = bns;
      vr[ib] = bns;
    }
    double ul[NV], ur[NV], fl[NV], fr[NV];
    prim2cons<ND, PH>(vl, ul, P);
    prim2cons<ND, PH>(vr, ur, P);
    phys_flux<ND, PH, N>(vl, ul, fl, P);
    phys_flux<ND, PH, N>(vr, ur, fr, P);
    const double cl = wave_speed<ND, PH, N>(vl, P);
    const double cr = wave_speed<ND, PH, N>(vr, P);
    const double unl = vl[1 + N], unr = vr[1 + N];
    if constexpr (FLUX == FLX_TVDLF) {
      const double cmax = dmax(fabs(unl) + cl, fabs(unr) + cr);
#pragma unroll
      for (int k = 0; k < NV; k++) F[k] = 0.5 * ((fl[k] + fr[k]) - cmax * (ur[k] - ul[k]));
    } else if constexpr (FLUX == FLX_HLLC && PH == PH_MHD) {
      hllc_mhd<ND, N>(vl, vr, ul, ur, fl, fr, cl, cr, F);
    } else {
      const double sl = dmin(unl - cl, unr - cr);
      const double sr = dmax(unl + cl, unr + cr);
      if (sl >= 0.0) {
#pragma unroll
        for (int k = 0; k < NV; k++) F[k] = fl[k];
      } else if (sr <= 0.0) {
#pragma unroll
        for (int k = 0; k < NV; k++) F[k] = fr[k];
      } else {
        const double ids = drcp(sr - sl);
#pragma unroll
        for (int k = 0; k < NV; k++) F[k] = ((sr * fl[k] - sl * fr[k]) + (sl * sr) * (ur[k] - ul[k])) * ids;
      }
    }
    if constexpr (PH == PH_MHD) {
      F[S::IB + N] = psis;
      F[S::IP] = P.ch * P.ch * bns;
    }
  }
}

// limited face states of a cell from its two neighbours along one direction:
// hi = v0 + 0.5*phi(backward, forward) (value at the cell's upper face),
// lo = v0 - 0.5*phi(forward, backward) (lower face; the same phi unless the
// limiter is asymmetric)
template <int NV, int LIM>
__device__ __forceinline__ void muscl(const double* vm, const double* v0, const double* vp, double* lo, double* hi,
                                      double thr2 = 0.0) {
#pragma unroll
  for (int k = 0; k < NV; k++) {
    const double a = v0[k] - vm[k], b = vp[k] - v0[k];
    const double s = limiter<LIM>(a, b, thr2);
    hi[k] = v0[k] + 0.5 * s;
    if constexpr (lim_asym<LIM>())
      lo[k] = v0[k] - 0.5 * limiter<LIM>(b, a, thr2);
    else
      lo[k] = v0[k] - 0.5 * s;
  }
}

}  // namespace amrv
