// forest.hpp -- host-side forest tables (see forest.cpp).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/amrv.h"
#include "internal.hpp"

namespace amrv {

struct Tables {
  int nd = 0, nx = 0, ncell = 0, T = 0, nvar = 0, nslot = 0;
  int64_t n = 0;
  std::vector<int32_t> lvl, ijk, nbr, slot, fslot, sleaf, sface, rlist, plist;
  std::vector<int8_t> kind;
  std::string err;
};

// Validate a leaf list and build the per-face tables. Returns AMRV_OK or an
// AMRV_E* code with t.err set.
int build_tables(const amrv_config& c, int64_t n, const int32_t* lev, const int32_t* ijk, Tables& t);

}  // namespace amrv
