// stage_ilp.hip -- the combined-variant stage kernels of 2D/3D non-MHD
// physics (launch_stage_combined), compiled on their own with LLVM's
// ILP-maximising scheduler; everything else of kernels.hip stays in that unit.
#define AMRV_STAGE_UNIT 0
#include "kernels.hip"
