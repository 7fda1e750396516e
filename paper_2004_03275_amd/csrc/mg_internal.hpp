// mg_internal.hpp -- entry points of the uniform multigrid solver
// (multigrid.hip) for the library's own use.
#pragma once

#include "../../include/amrv_mg.h"

namespace amrv {

// The solver's own finest-level right-hand side and solution arrays (field
// 0, n^d device doubles each): a caller that fills *f and zeroes *e itself
// and passes them to mg_enqueue_correction saves its copies and its fill.
int mg_correction_grids(amrv_mg* m, double** f, double** e);

// Enqueues, on the solver's stream and without any host synchronisation,
// `cycles` V-cycles for lap(e) - lambda e = f from e = 0, then copies e to
// out (f, out: n^d device doubles; no copy where f or out is the solver's own
// array).  e_zeroed: the solver's solution array already holds zeros (else
// it is cleared here).  The parameter block is uploaded only when lambda
// differs from the last one set.  For a solver with one field and the
// constant coefficient; lambda >= 0.  Returns 0 or a negative AMRV_E* code.
int mg_enqueue_correction(amrv_mg* m, const double* f, double* out, double lambda, int cycles, bool e_zeroed);

}  // namespace amrv
