// mlp.hpp -- parameter layout and launchers of the learned flagger (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace amrv {

// binary32 master parameter vector: W1 [64][128], b1 [64], W2 [64][64], b2 [64],
// W3 [2][64], b3 [2]; output 0 is the refine logit, output 1 the coarsen logit
constexpr int MLP_NIN = 128, MLP_NH = 64, MLP_NOUT = 2;
constexpr int MLP_W1 = 0;
constexpr int MLP_B1 = MLP_W1 + MLP_NH * MLP_NIN;
constexpr int MLP_W2 = MLP_B1 + MLP_NH;
constexpr int MLP_B2 = MLP_W2 + MLP_NH * MLP_NH;
constexpr int MLP_W3 = MLP_B2 + MLP_NH;
constexpr int MLP_B3 = MLP_W3 + MLP_NOUT * MLP_NH;
constexpr int MLP_NPARAM = MLP_B3 + MLP_NOUT;  // 12,546
// bfloat16 operand copies: W1b [64][128], W2b [64][64], W2bT [64][64], W3b [2][64]
constexpr int MLP_WB_W1 = 0;
constexpr int MLP_WB_W2 = MLP_WB_W1 + MLP_NH * MLP_NIN;
constexpr int MLP_WB_W2T = MLP_WB_W2 + MLP_NH * MLP_NH;
constexpr int MLP_WB_W3 = MLP_WB_W2T + MLP_NH * MLP_NH;
constexpr int MLP_WB_COUNT = MLP_WB_W3 + MLP_NOUT * MLP_NH;

struct TrainHyper {
  float lr, beta1, beta2, eps, pos_weight, pos_weight_c;
};

hipError_t launch_mlp_features(const Geo& g, const LaunchCfg& c, const double* U, const double* physp, uint16_t* X,
                               hipStream_t st);
hipError_t launch_mlp_prep(const float* w, uint16_t* wb, hipStream_t st);
// z [n][2]: refine and coarsen logits; flags [n]: the three-way decision;
// uncertain, zout (may be null): the fallback marks and the refine logits
hipError_t launch_mlp_infer(const uint16_t* X, int n, const uint16_t* wb, const float* w, float* z, const int32_t* lvl,
                            int max_level, float margin, int8_t* flags, int8_t* uncertain, double* zout,
                            hipStream_t st);
// device scratch of one training call with batch B (256-byte aligned pieces)
constexpr size_t mlp_align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t mlp_train_scratch_bytes_c(int B) {
  return 2 * mlp_align256(2 * (size_t)B * MLP_NIN)       // xg, xgT
         + 6 * mlp_align256(2 * (size_t)B * MLP_NH)      // h1 h1T h2 dh2 dh2T dh1T
         + mlp_align256(4 * (size_t)B * MLP_NH)          // dh1
         + 2 * mlp_align256(4 * (size_t)MLP_NOUT * B)    // z, dz [B][2]
         + mlp_align256(4 * (size_t)B)                   // loss
         + mlp_align256(4 * (size_t)MLP_NPARAM)          // grad
         + mlp_align256(2 * (size_t)MLP_WB_COUNT)        // wb
         + mlp_align256(16);                             // step counter
}
size_t mlp_train_scratch_bytes(int B);
// the library-held scratch of amrv_mlp_train_noalloc: the largest batch
constexpr int MLP_MAX_BATCH = 4096;
constexpr size_t MLP_STATIC_SCRATCH_BYTES = mlp_train_scratch_bytes_c(MLP_MAX_BATCH);
constexpr int MLP_MAX_DEVICES = 64;
// this device's address of that scratch (resolved once per device)
hipError_t mlp_static_scratch(void** out);
hipError_t launch_mlp_train(const uint16_t* X, const float* Y, const int32_t* order, int n, int B, int first_batch,
                            int nbatch, float* w, float* am, float* av, const TrainHyper& hp, int t0, void* ws,
                            float* loss_out, float* grad_out, hipStream_t st);

}  // namespace amrv
