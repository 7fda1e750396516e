// mg_internal.hpp -- entry points of the uniform multigrid solver
// (multigrid.hip) for the library's own use.
#pragma once

#include "../../include/amrv_mg.h"

namespace amrv {

// Enqueues, on the solver's stream and without any host synchronisation,
// `cycles` V-cycles for lap(e) - lambda e = f from e = 0, then copies e to
// out (f, out: n^d device doubles).  For a solver with one field and the
// constant coefficient; lambda >= 0.  Returns 0 or a negative AMRV_E* code.
int mg_enqueue_correction(amrv_mg* m, const double* f, double* out, double lambda, int cycles);

}  // namespace amrv
