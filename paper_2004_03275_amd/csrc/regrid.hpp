// regrid.hpp -- host-side regrid plan and transfer sources (see regrid.cpp).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "forest.hpp"

namespace amrv {

// per new leaf: [0] how (XFER_*), [1..8] source leaves of the old forest
// (copy / prolong: [1] the leaf or parent; restrict: [1 + child] the children)
constexpr int XFER_STRIDE = 9;
enum { XFER_COPY = 0, XFER_PROLONG = 1, XFER_RESTRICT = 2 };

// New leaf list for the flags (+1 split, 0 keep, -1 merge) of forest t.
int regrid_plan(const amrv_config& c, const Tables& t, const int8_t* flags, std::vector<int32_t>& out_lev,
                std::vector<int32_t>& out_ijk, std::string& err);

// Where each leaf of `to` takes its state from in `from`.
int regrid_sources(const Tables& from, const Tables& to, std::vector<int32_t>& src, std::string& err);

}  // namespace amrv
