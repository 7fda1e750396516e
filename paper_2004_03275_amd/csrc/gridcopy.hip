// gridcopy.hip -- one variable of a uniform forest's state (every leaf at
// one level) to or from a global grid array, x fastest, so that grid-based
// solvers (the multigrid divergence control) can act on forest states.
#include <hip/hip_runtime.h>

#include "gridcopy.hpp"

namespace amrv {

// one workgroup per leaf; cell (x, y, z) of leaf b sits at global cell
// ijk_b * nx + (x, y, z)
__global__ void __launch_bounds__(256) k_grid_copy(double* U, double* grid, const int32_t* ijk, int nleaves, int ndim,
                                                   int nx, int ncell, int gx, int gy, int to_grid) {
  const int b = blockIdx.x;
  if (b >= nleaves) return;
  const int bx = ijk[3 * b], by = ijk[3 * b + 1], bz = ijk[3 * b + 2];
  double* u = U + (size_t)b * ncell;
  for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
    const int x = i % nx;
    const int y = ndim > 1 ? (i / nx) % nx : 0;
    const int z = ndim > 2 ? i / (nx * nx) : 0;
    const size_t gi = ((size_t)(bz * nx + z) * gy + (by * nx + y)) * gx + (bx * nx + x);
    if (to_grid)
      grid[gi] = u[i];
    else
      u[i] = grid[gi];
  }
}

hipError_t launch_grid_copy(double* Uvar, double* grid, const int32_t* ijk, int nleaves, int ndim, int nx, int ncell,
                            int gx, int gy, int to_grid, hipStream_t st) {
  hipLaunchKernelGGL(k_grid_copy, dim3(nleaves), dim3(256), 0, st, Uvar, grid, ijk, nleaves, ndim, nx, ncell, gx, gy,
                     to_grid);
  return hipGetLastError();
}

}  // namespace amrv
