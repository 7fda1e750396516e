// stage_fast.hip -- the combined-variant stage kernels of 2D/3D non-MHD
// physics in fast arithmetic (launch_stage_combined_fast, AR = 1): built with
// contraction of multiply-adds into FMAs and with the division, reciprocal,
// square root and sound speed of physics.hpp taken from the hardware
// reciprocal and reciprocal square root plus Newton steps (AMRV_FAST_MATH).
// Same expressions otherwise; results within a few ulp per operation of the
// correctly rounded kernels, held to the 1e-10 relative-L1 bar against the
// oracle instead of bit-for-bit equality.
#define AMRV_STAGE_UNIT 1
#define AMRV_FAST_MATH
#include "kernels.hip"
