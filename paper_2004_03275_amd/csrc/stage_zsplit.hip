// stage_zsplit.hip -- the two-launch stage update of 3D MHD forests
// (launch_stage_zsplit, stage-kernel variant 2): k_stage_zcol streams the z
// direction of every column and stores its flux divergence, k_stage_xy then
// updates the x/y planes.  Correctly rounded, like the one-launch kernel whose
// results it reproduces bit for bit; default scheduler.
#define AMRV_STAGE_UNIT 2
#include "kernels.hip"
