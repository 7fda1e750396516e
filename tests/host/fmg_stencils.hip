// Host check of the forest multigrid's batched stencils (csrc/fmg.hip): for
// every block of a forest read from argv[1], stencil_k and apply_k give the
// same sums, bit for bit, as stencil and apply_cell cell by cell, with the
// plain stencil on every block and the problem's rules on the leaves: in 3D
// the batch layouts of the colour sweep and of the residual kernels (K = 4)
// and the fused residual-restriction's 2x2x2 cube (K = 8), in 2D its 2x2
// square (K = 4).
// Input: "nleaves base max_level bc ndim", then "level i j k" per leaf.
// Prints "checked N mismatches M"; exit status 0 iff M == 0.
#include "fmg.hip"

#include <cstdio>
#include <cstring>
#include <fstream>
#include <random>

namespace {

bool same(double a, double b) { return std::memcmp(&a, &b, sizeof(double)) == 0; }

}  // namespace

template <int ND>
int check(const Tree& T, const amrv_fmg_config& c) {
  constexpr int NCB = ncb<ND>();
  std::vector<double> u((size_t)T.nblk * NCB);
  std::mt19937_64 rng(5);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (auto& v : u) v = U(rng);
  FmgDev g{};
  g.lvl = T.lvl.data();
  g.ij = T.ij.data();
  g.nbr = T.nbr.data();
  g.chi = T.chi.data();
  g.cnb = T.cnb.data();
  g.par = T.par.data();
  g.u = u.data();
  g.lam = 7.0;
  for (int l = 1; l <= FMG_MAXL; l++) {
    const double q = (double)((long long)c.base * NB << (l - 1)) / c.length;
    g.ih2[l] = q * q;
    g.rh[l] = q;
  }
  long long bad = 0, tot = 0;
  for (int b = 0; b < T.nblk; b++) {
    if constexpr (ND == 3) {
      // the colour sweep's batch: cells (2 hx + parity, y, z0 + 2k + pz)
      for (int colour = 0; colour < 2; colour++)
        for (int t = 0; t < 256; t++)
          for (int z0 = 0; z0 < NB; z0 += 8) {
            const int hx = t & 7, ty = (t >> 3) & 15, pz = t >> 7;
            int cc[4][3];
            double sc[4], sw[4];
            for (int k = 0; k < 4; k++) {
              const int tz = z0 + 2 * k + pz;
              cc[k][0] = 2 * hx + ((ty + tz + colour) & 1);
              cc[k][1] = ty;
              cc[k][2] = tz;
            }
            stencil_k<3, 4>(g, b, false, cc, sc, sw);
            for (int k = 0; k < 4; k++) {
              double s1, w1;
              stencil<3>(g, b, false, cc[k], s1, w1);
              tot++;
              bad += !(same(s1, sc[k]) && same(w1, sw[k]));
            }
          }
      // the residual kernels' batch: cells (x, y, z0 + k), both rule sets on leaves
      for (int leaf = 0; leaf < (T.chi[CS * b] < 0 ? 2 : 1); leaf++)
        for (int t = 0; t < 256; t++)
          for (int z0 = 0; z0 < NB; z0 += 4) {
            int cc[4][3];
            double uv[4], a[4];
            for (int k = 0; k < 4; k++) {
              cc[k][0] = t & 15;
              cc[k][1] = t >> 4;
              cc[k][2] = z0 + k;
              uv[k] = u[(size_t)b * NCB + cidx(cc[k])];
            }
            apply_k<3, 4>(g, b, leaf != 0, cc, uv, a);
            for (int k = 0; k < 4; k++) {
              tot++;
              bad += !same(apply_cell<3>(g, b, leaf != 0, cc[k]), a[k]);
            }
          }
    }
    // the fused residual-restriction's batch: the 2^ND cells of a parent cell
    constexpr int NC = 1 << ND;
    for (int t = 0; t < (ND == 3 ? 512 : 64); t++) {
      int cc[NC][3];
      double uv[NC], a[NC];
      for (int k = 0; k < NC; k++) {
        cc[k][0] = 2 * (t & 7) + (k & 1);
        cc[k][1] = 2 * ((t >> 3) & 7) + ((k >> 1) & 1);
        cc[k][2] = ND == 3 ? 2 * (t >> 6) + (k >> 2) : 0;
        uv[k] = u[(size_t)b * NCB + cidx(cc[k])];
      }
      apply_k<ND, NC>(g, b, false, cc, uv, a);
      for (int k = 0; k < NC; k++) {
        tot++;
        bad += !same(apply_cell<ND>(g, b, false, cc[k]), a[k]);
      }
    }
  }
  std::printf("blocks %d checked %lld mismatches %lld\n", T.nblk, tot, bad);
  return bad != 0;
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  std::ifstream in(argv[1]);
  amrv_fmg_config c{};
  long long n;
  in >> n >> c.base >> c.max_level >> c.bc >> c.ndim;
  if (!in || (c.ndim != 2 && c.ndim != 3)) return 2;
  c.nleaves = n;
  c.pre_sweeps = c.post_sweeps = 2;
  c.length = 1.0;
  std::vector<int32_t> lev(n), ijk(3 * n);
  for (long long k = 0; k < n; k++) in >> lev[k] >> ijk[3 * k] >> ijk[3 * k + 1] >> ijk[3 * k + 2];
  Tree T;
  if (build_tree(&c, lev.data(), ijk.data(), T)) {
    std::printf("build_tree: %s\n", amrv_last_error());
    return 1;
  }
  return c.ndim == 3 ? check<3>(T, c) : check<2>(T, c);
}
