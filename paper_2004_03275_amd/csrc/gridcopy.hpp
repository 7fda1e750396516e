// gridcopy.hpp -- launcher of the uniform-forest <-> grid copy (gridcopy.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amrv {

// Uvar: one variable's block of the state ([leaf][cells]); grid: gx * gy * gz
// doubles, x fastest; ijk: device block coordinates of the leaves
hipError_t launch_grid_copy(double* Uvar, double* grid, const int32_t* ijk, int nleaves, int ndim, int nx, int ncell,
                            int gx, int gy, int to_grid, hipStream_t st);

}  // namespace amrv
