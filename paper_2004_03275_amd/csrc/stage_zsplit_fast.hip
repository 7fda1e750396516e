// stage_zsplit_fast.hip -- the two-launch stage update of 3D MHD forests
// (stage-kernel variant 2) in fast arithmetic (launch_stage_zsplit_fast,
// AR = 1): multiply-adds contracted into FMAs, divisions, reciprocals and
// square roots from the hardware estimates refined by Newton steps
// (AMRV_FAST_MATH, physics.hpp).  Held to the 1e-10 relative-L1 bar against
// the oracle instead of bit-for-bit equality.
#define AMRV_STAGE_UNIT 3
#define AMRV_FAST_MATH
#include "kernels.hip"
