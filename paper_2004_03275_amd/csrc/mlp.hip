// mlp.hip -- learned refinement flagger on gfx950.
//
// The paper refines blocks where the Loehner estimator exceeds a tolerance
// (arXiv 2004.03275, Sec. 1.3).  This file adds a small multilayer perceptron
// (128-64-64-2) that predicts those decisions from pooled block features, so
// most blocks can be flagged without the estimator's ghost fill and
// second-derivative pass:
//   k_mlp_features  per leaf: means of rho and p over 64 sub-blocks (4^3 cells
//                   in 3D, 2^2 in 2D), normalised by the leaf mean, to bfloat16
//   k_mlp_infer     refine and coarsen logits of all leaves: bfloat16 MFMA
//                   products (v_mfma_f32_16x16x32_bf16), binary32 accumulation,
//                   and each leaf's three-way flag from its two logits
//   k_mlp_train     one optimisation step on a batch: forward, class-weighted
//                   binary cross-entropy, backward (weight gradients again as
//                   bfloat16 MFMA products with binary32 accumulation), Adam
// Reductions run in a fixed order, so results are deterministic.
#include <type_traits>

#include <mutex>

#include "bf16.hpp"
#include "internal.hpp"
#include "mlp.hpp"
#include "physics.hpp"

namespace amrv {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// 8 consecutive bfloat16 values (16 bytes, 16-byte aligned) as an MFMA operand
__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  bf16x8 r;
  __builtin_memcpy(&r, p, 16);
  return r;
}

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 r;
  const uint4 z = make_uint4(0, 0, 0, 0);
  __builtin_memcpy(&r, &z, 16);
  return r;
}

// gather 8 bfloat16 values with a stride (in elements)
__device__ __forceinline__ bf16x8 gather8(const uint16_t* p, int stride) {
  uint16_t t[8];
#pragma unroll
  for (int j = 0; j < 8; j++) t[j] = p[j * stride];
  bf16x8 r;
  __builtin_memcpy(&r, t, 16);
  return r;
}

// Operand layout of v_mfma_f32_16x16x32_bf16 (64 lanes): lane l holds
// A[m = l % 16][k = 8 (l / 16) .. +7], B[k = 8 (l / 16) .. +7][n = l % 16], and
// receives D[m = 4 (l / 16) + i][n = l % 16], i = 0..3.
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------

template <int ND, int PH>
__global__ void __launch_bounds__(128) k_mlp_features(Geo g, const double* __restrict__ U,
                                                      const double* __restrict__ pp, uint16_t* __restrict__ X) {
  using S = Sys<ND, PH>;
  constexpr int NV = S::NV;
  __shared__ double means[2][64];
  __shared__ double mtot[2];
  const int leaf = blockIdx.x;
  const int t = threadIdx.x;
  const int var = t >> 6, sb = t & 63;  // var 0: rho, 1: p
  PhysParams P;
  P.gamma = pp[PP_GAMMA];
  P.gm1 = pp[PP_GM1];
  P.igm1 = pp[PP_IGM1];
  P.ch = 0.0;
  P.cad = pp[PP_CAD];
  P.gcad = pp[PP_GCAD];
  const size_t vs = (size_t)g.n * g.ncell;
  const double* base = U + (size_t)leaf * g.ncell;
  double s = 0.0;
  if constexpr (ND == 3) {
    const int bx = sb & 3, by = (sb >> 2) & 3, bz = sb >> 4;
    for (int k = 0; k < 4; k++)
      for (int j = 0; j < 4; j++)
        for (int i = 0; i < 4; i++) {
          const int cell = (4 * bx + i) + 16 * ((4 * by + j) + 16 * (4 * bz + k));
          double q;
          if (var == 0) {
            q = base[cell];
          } else {
            double u[NV], v[NV];
#pragma unroll
            for (int c = 0; c < NV; c++) u[c] = base[c * vs + cell];
            cons2prim<ND, PH>(u, v, P);
            q = pressure<ND, PH>(v, P);
          }
          s = s + q;
        }
    means[var][sb] = s / 64.0;
  } else {
    const int bx = sb & 7, by = sb >> 3;
    for (int j = 0; j < 2; j++)
      for (int i = 0; i < 2; i++) {
        const int cell = (2 * bx + i) + 16 * (2 * by + j);
        double q;
        if (var == 0) {
          q = base[cell];
        } else {
          double u[NV], v[NV];
#pragma unroll
          for (int c = 0; c < NV; c++) u[c] = base[c * vs + cell];
          cons2prim<ND, PH>(u, v, P);
          q = pressure<ND, PH>(v, P);
        }
        s = s + q;
      }
    means[var][sb] = s / 4.0;
  }
  __syncthreads();
  if (sb == 0) {
    double m = 0.0;
    for (int i = 0; i < 64; i++) m = m + means[var][i];
    mtot[var] = m / 64.0;
  }
  __syncthreads();
  const float f = (float)(means[var][sb] / mtot[var] - 1.0);
  X[(size_t)leaf * MLP_NIN + 64 * var + sb] = to_bf16(f);
}

// ---------------------------------------------------------------------------
// parameters: binary32 master vector -> bfloat16 operand copies
// ---------------------------------------------------------------------------

// W1b [64][128], W2b [64][64], W2bT [64][64] (transposed), W3b [2][64]
__global__ void k_mlp_prep(const float* __restrict__ w, uint16_t* __restrict__ wb) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < MLP_NH * MLP_NIN; i += gridDim.x * blockDim.x)
    wb[MLP_WB_W1 + i] = to_bf16(w[MLP_W1 + i]);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < MLP_NH * MLP_NH; i += gridDim.x * blockDim.x) {
    const uint16_t b = to_bf16(w[MLP_W2 + i]);
    wb[MLP_WB_W2 + i] = b;
    const int n2 = i / MLP_NH, n1 = i % MLP_NH;  // W2[n2][n1]
    wb[MLP_WB_W2T + n1 * MLP_NH + n2] = b;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < MLP_NOUT * MLP_NH; i += gridDim.x * blockDim.x)
    wb[MLP_WB_W3 + i] = to_bf16(w[MLP_W3 + i]);
}

// ---------------------------------------------------------------------------
// forward pass of one 16-row tile by one wave
// ---------------------------------------------------------------------------

// rows of X: xrow(r) -> pointer to 128 bfloat16 features, or nullptr (zeros)
// h1t, h2t: the wave's LDS tiles [16][64] bfloat16.  Returns, in lane l < 16,
// the refine logit of row l and, in lane 16 + l, the coarsen logit of row l
// (other lanes: undefined).
template <class XRow>
__device__ __forceinline__ float tile_forward(XRow xrow, const uint16_t* __restrict__ wb, const float* __restrict__ w,
                                              uint16_t* h1t, uint16_t* h2t) {
  const int l = threadIdx.x & 63;
  const int lm = l & 15, lk = 8 * (l >> 4);
  const uint16_t* xr = xrow(lm);
  bf16x8 xa[4];
#pragma unroll
  for (int kt = 0; kt < 4; kt++) xa[kt] = xr ? load8(xr + kt * 32 + lk) : zero8();
#pragma unroll
  for (int nt = 0; nt < 4; nt++) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; kt++)
      acc = mfma(xa[kt], load8(wb + MLP_WB_W1 + (nt * 16 + lm) * MLP_NIN + kt * 32 + lk), acc);
    const int n = nt * 16 + lm;
    const float bias = w[MLP_B1 + n];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const float a = acc[i] + bias;
      h1t[(4 * (l >> 4) + i) * MLP_NH + n] = to_bf16(a > 0.f ? a : 0.f);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int nt = 0; nt < 4; nt++) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 2; kt++)
      acc = mfma(load8(h1t + lm * MLP_NH + kt * 32 + lk), load8(wb + MLP_WB_W2 + (nt * 16 + lm) * MLP_NH + kt * 32 + lk),
                 acc);
    const int n = nt * 16 + lm;
    const float bias = w[MLP_B2 + n];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const float a = acc[i] + bias;
      h2t[(4 * (l >> 4) + i) * MLP_NH + n] = to_bf16(a > 0.f ? a : 0.f);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  float z = 0.f;
  if (l < 32) {
    const int o = l >> 4, r = l & 15;
    for (int k = 0; k < MLP_NH; k++)
      z = z + from_bf16(h2t[r * MLP_NH + k]) * from_bf16(wb[MLP_WB_W3 + o * MLP_NH + k]);
    z = z + w[MLP_B3 + o];
  }
  return z;
}

// logits of n rows of X [n][128] into z [n][2], and each leaf's flag from
// its logits (z_r, z_c): +1 where z_r > 0 below the finest level, -1 where
// z_r <= 0 and z_c > 0 above level 1, else 0; `uncertain` (optional) marks
// leaves with |z_r| < margin or |z_c| < margin (fallback mode), `zout`
// (optional) receives z_r.  256 threads = 4 waves x 16 rows.
__global__ void __launch_bounds__(256) k_mlp_infer(const uint16_t* __restrict__ X, int n, const uint16_t* __restrict__ wb,
                                                   const float* __restrict__ w, float* __restrict__ z,
                                                   const int32_t* __restrict__ lvl, int max_level, float margin,
                                                   int8_t* __restrict__ flags, int8_t* __restrict__ uncertain,
                                                   double* __restrict__ zout) {
  __shared__ __attribute__((aligned(16))) uint16_t h1[4][16 * MLP_NH];
  __shared__ __attribute__((aligned(16))) uint16_t h2[4][16 * MLP_NH];
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int r0 = blockIdx.x * 64 + wave * 16;
  auto xrow = [&](int m) -> const uint16_t* { return r0 + m < n ? X + (size_t)(r0 + m) * MLP_NIN : nullptr; };
  const float zz = tile_forward(xrow, wb, w, h1[wave], h2[wave]);
  const int r = l & 15, o = l >> 4;
  const float zc = __shfl(zz, r + 16, 64);  // lane r (< 16) gets the coarsen logit of its row
  if (l < 32 && r0 + r < n) z[(size_t)(r0 + r) * MLP_NOUT + o] = zz;
  if (l < 16 && r0 + r < n) {
    const int i = r0 + r;
    const float zr = zz;
    const int lv = lvl[i];
    flags[i] = (zr > 0.f && lv < max_level) ? 1 : ((!(zr > 0.f) && zc > 0.f && lv > 1) ? -1 : 0);
    if (uncertain) uncertain[i] = (fabsf(zr) < margin || fabsf(zc) < margin) ? 1 : 0;
    if (zout) zout[i] = (double)zr;
  }
}

// ---------------------------------------------------------------------------
// training step: one workgroup, one batch
// ---------------------------------------------------------------------------

// scratch layout (bytes offsets computed by mlp_train_layout)
struct TrainScratch {
  uint16_t* xg;    // [B][128] gathered batch features
  uint16_t* xgT;   // [128][B]
  uint16_t* h1;    // [B][64]
  uint16_t* h1T;   // [64][B]
  uint16_t* h2;    // [B][64]
  uint16_t* dh2;   // [B][64] bfloat16
  uint16_t* dh2T;  // [64][B]
  uint16_t* dh1T;  // [64][B]
  float* dh1;      // [B][64] binary32 (bias gradient)
  float* z;        // [B][2]
  float* dz;       // [B][2]
  float* grad;     // [NPARAM]
  float* loss;     // [B] per-row loss
  uint16_t* wb;    // bfloat16 operand copies
  int* tstep;      // Adam step counter
};

__global__ void __launch_bounds__(256) k_mlp_train(const uint16_t* __restrict__ X, const float* __restrict__ Y,
                                                   const int32_t* __restrict__ order, int n, int B, int batch,
                                                   float* __restrict__ w, float* __restrict__ am, float* __restrict__ av,
                                                   TrainHyper hp, TrainScratch s, float* __restrict__ loss_out) {
  __shared__ __attribute__((aligned(16))) uint16_t h1t[4][16 * MLP_NH];
  __shared__ __attribute__((aligned(16))) uint16_t h2t[4][16 * MLP_NH];
  __shared__ float red[256];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
  const int lm = l & 15, lk = 8 * (l >> 4);
  const int b0 = batch * B;
  int nvalid = n - b0;
  if (nvalid > B) nvalid = B;

  // P0: gather the batch (padding rows are zero with zero weight)
  for (int i = tid; i < B * MLP_NIN; i += 256) {
    const int r = i / MLP_NIN, c = i % MLP_NIN;
    const uint16_t v = r < nvalid ? X[(size_t)order[b0 + r] * MLP_NIN + c] : (uint16_t)0;
    s.xg[i] = v;
    s.xgT[(size_t)c * B + r] = v;
  }
  __threadfence_block();
  __syncthreads();

  // P1: forward, 16-row tiles round-robin over the waves
  for (int rt = wave; rt < B / 16; rt += 4) {
    const int r0 = rt * 16;
    auto xrow = [&](int m) -> const uint16_t* { return s.xg + (size_t)(r0 + m) * MLP_NIN; };
    const float z = tile_forward(xrow, s.wb, w, h1t[wave], h2t[wave]);
    // activations for the backward pass
    for (int i = l; i < 16 * MLP_NH; i += 64) {
      const int m = i / MLP_NH, c = i % MLP_NH;
      s.h1[(size_t)(r0 + m) * MLP_NH + c] = h1t[wave][i];
      s.h1T[(size_t)c * B + r0 + m] = h1t[wave][i];
      s.h2[(size_t)(r0 + m) * MLP_NH + c] = h2t[wave][i];
    }
    if (l < 32) s.z[(size_t)(r0 + (l & 15)) * MLP_NOUT + (l >> 4)] = z;
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  __threadfence_block();
  __syncthreads();

  // P2: logit gradients and loss per row.  The label is Loehner's class
  // (+1 refine, -1 coarsen, 0 keep): target 1 of the refine output for +1,
  // of the coarsen output for -1; each output's class-weighted binary
  // cross-entropy, summed
  const float Bv = (float)nvalid;
  for (int r = tid; r < B; r += 256) {
    float dzr = 0.f, dzc = 0.f, lr = 0.f;
    if (r < nvalid) {
      const float lab = Y[order[b0 + r]];
#pragma unroll
      for (int o = 0; o < MLP_NOUT; o++) {
        const float z = s.z[(size_t)r * MLP_NOUT + o];
        const float y = o == 0 ? (lab > 0.5f ? 1.f : 0.f) : (lab < -0.5f ? 1.f : 0.f);
        const float pw = o == 0 ? hp.pos_weight : hp.pos_weight_c;
        const float sg = 1.f / (1.f + expf(-z));
        const float dz = ((1.f - y) * sg - pw * y * (1.f - sg)) / Bv;
        // -(pw y log s + (1-y) log(1-s)) with log s = -softplus(-z)
        const float sp_neg = fmaxf(-z, 0.f) + log1pf(expf(-fabsf(z)));
        const float sp_pos = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));
        lr = lr + (pw * y * sp_neg + (1.f - y) * sp_pos);
        if (o == 0)
          dzr = dz;
        else
          dzc = dz;
      }
    }
    s.dz[(size_t)r * MLP_NOUT] = dzr;
    s.dz[(size_t)r * MLP_NOUT + 1] = dzc;
    s.loss[r] = lr;
  }
  __threadfence_block();
  __syncthreads();

  // P3: W3, b3, b2 gradients; dh2 = (dz_r w3_r + dz_c w3_c) * [h2 > 0]
  // (binary32, then bfloat16)
  if (tid < MLP_NOUT * MLP_NH) {
    const int o = tid / MLP_NH, c = tid % MLP_NH;
    float g3 = 0.f;
    for (int r = 0; r < B; r++) g3 = g3 + s.dz[(size_t)r * MLP_NOUT + o] * from_bf16(s.h2[(size_t)r * MLP_NH + c]);
    s.grad[MLP_W3 + tid] = g3;
  } else if (tid < MLP_NOUT * MLP_NH + MLP_NOUT) {
    const int o = tid - MLP_NOUT * MLP_NH;
    float g = 0.f, L = 0.f;
    for (int r = 0; r < B; r++) {
      g = g + s.dz[(size_t)r * MLP_NOUT + o];
      L = L + s.loss[r];
    }
    s.grad[MLP_B3 + o] = g;
    if (loss_out && o == 0) loss_out[batch] = L / Bv;
  }
  auto dh2_of = [&](int r, int c) -> float {
    return from_bf16(s.h2[(size_t)r * MLP_NH + c]) > 0.f
               ? s.dz[(size_t)r * MLP_NOUT] * from_bf16(s.wb[MLP_WB_W3 + c]) +
                     s.dz[(size_t)r * MLP_NOUT + 1] * from_bf16(s.wb[MLP_WB_W3 + MLP_NH + c])
               : 0.f;
  };
  for (int i = tid; i < B * MLP_NH; i += 256) {
    const int r = i / MLP_NH, c = i % MLP_NH;
    const uint16_t db = to_bf16(dh2_of(r, c));
    s.dh2[i] = db;
    s.dh2T[(size_t)c * B + r] = db;
  }
  __threadfence_block();
  __syncthreads();
  if (tid < MLP_NH) {
    float g = 0.f;
    for (int r = 0; r < B; r++) g = g + dh2_of(r, tid);
    s.grad[MLP_B2 + tid] = g;
  }

  // P4a: dW2 = dh2^T h1  (64 x 64, K = B): 16 output tiles, 4 per wave
  for (int tt = wave; tt < 16; tt += 4) {
    const int mt = tt >> 2, nt = tt & 3;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < B / 32; kt++)
      acc = mfma(load8(s.dh2T + (size_t)(mt * 16 + lm) * B + kt * 32 + lk),
                 load8(s.h1T + (size_t)(nt * 16 + lm) * B + kt * 32 + lk), acc);
#pragma unroll
    for (int i = 0; i < 4; i++) s.grad[MLP_W2 + (mt * 16 + 4 * (l >> 4) + i) * MLP_NH + nt * 16 + lm] = acc[i];
  }
  // P4b: dh1 = dh2 W2 * [h1 > 0]  (B x 64, K = 64)
  for (int tt = wave; tt < (B / 16) * 4; tt += 4) {
    const int rt = tt >> 2, nt = tt & 3;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 2; kt++)
      acc = mfma(load8(s.dh2 + (size_t)(rt * 16 + lm) * MLP_NH + kt * 32 + lk),
                 load8(s.wb + MLP_WB_W2T + (nt * 16 + lm) * MLP_NH + kt * 32 + lk), acc);
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int r = rt * 16 + 4 * (l >> 4) + i, c = nt * 16 + lm;
      const float d = from_bf16(s.h1[(size_t)r * MLP_NH + c]) > 0.f ? acc[i] : 0.f;
      s.dh1[(size_t)r * MLP_NH + c] = d;
      s.dh1T[(size_t)c * B + r] = to_bf16(d);
    }
  }
  __threadfence_block();
  __syncthreads();

  // P5: dW1 = dh1^T X (64 x 128, K = B): 32 tiles; b1 gradient
  for (int tt = wave; tt < 32; tt += 4) {
    const int mt = tt >> 3, nt = tt & 7;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kt = 0; kt < B / 32; kt++)
      acc = mfma(load8(s.dh1T + (size_t)(mt * 16 + lm) * B + kt * 32 + lk),
                 load8(s.xgT + (size_t)(nt * 16 + lm) * B + kt * 32 + lk), acc);
#pragma unroll
    for (int i = 0; i < 4; i++) s.grad[MLP_W1 + (mt * 16 + 4 * (l >> 4) + i) * MLP_NIN + nt * 16 + lm] = acc[i];
  }
  if (tid < MLP_NH) {
    float g = 0.f;
    for (int r = 0; r < B; r++) g = g + s.dh1[(size_t)r * MLP_NH + tid];
    s.grad[MLP_B1 + tid] = g;
  }
  __threadfence_block();
  __syncthreads();

  // P6: Adam (binary32 master weights), then fresh bfloat16 copies
  const int t = *s.tstep + 1;
  const float c1 = (float)(1.0 - pow((double)hp.beta1, (double)t));
  const float c2 = (float)(1.0 - pow((double)hp.beta2, (double)t));
  for (int i = tid; i < MLP_NPARAM; i += 256) {
    const float gr = s.grad[i];
    const float m = hp.beta1 * am[i] + (1.f - hp.beta1) * gr;
    const float v = hp.beta2 * av[i] + (1.f - hp.beta2) * gr * gr;
    am[i] = m;
    av[i] = v;
    w[i] = w[i] - hp.lr * (m / c1) / (sqrtf(v / c2) + hp.eps);
  }
  __threadfence_block();
  __syncthreads();
  for (int i = tid; i < MLP_NH * MLP_NIN; i += 256) s.wb[MLP_WB_W1 + i] = to_bf16(w[MLP_W1 + i]);
  for (int i = tid; i < MLP_NH * MLP_NH; i += 256) {
    const uint16_t b = to_bf16(w[MLP_W2 + i]);
    s.wb[MLP_WB_W2 + i] = b;
    s.wb[MLP_WB_W2T + (i % MLP_NH) * MLP_NH + i / MLP_NH] = b;
  }
  if (tid < MLP_NOUT * MLP_NH) s.wb[MLP_WB_W3 + tid] = to_bf16(w[MLP_W3 + tid]);
  if (tid == 0) *s.tstep = t;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_mlp_features(const Geo& g, const LaunchCfg& c, const double* U, const double* physp, uint16_t* X,
                               hipStream_t st) {
  auto go = [&](auto nd) {
    constexpr int ND = decltype(nd)::value;
    if (c.phys == PH_MHD)
      hipLaunchKernelGGL((k_mlp_features<ND, PH_MHD>), dim3(g.n), dim3(128), 0, st, g, U, physp, X);
    else if (c.phys == PH_POLY)
      hipLaunchKernelGGL((k_mlp_features<ND, PH_POLY>), dim3(g.n), dim3(128), 0, st, g, U, physp, X);
    else
      hipLaunchKernelGGL((k_mlp_features<ND, PH_EULER>), dim3(g.n), dim3(128), 0, st, g, U, physp, X);
  };
  if (c.ndim == 2) {
    go(std::integral_constant<int, 2>{});
  } else if (c.ndim == 3) {
    go(std::integral_constant<int, 3>{});
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_mlp_prep(const float* w, uint16_t* wb, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_prep, dim3(16), dim3(256), 0, st, w, wb);
  return hipGetLastError();
}

hipError_t launch_mlp_infer(const uint16_t* X, int n, const uint16_t* wb, const float* w, float* z, const int32_t* lvl,
                            int max_level, float margin, int8_t* flags, int8_t* uncertain, double* zout,
                            hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_infer, dim3((n + 63) / 64), dim3(256), 0, st, X, n, wb, w, z, lvl, max_level, margin, flags,
                     uncertain, zout);
  return hipGetLastError();
}

size_t mlp_train_scratch_bytes(int B) { return mlp_train_scratch_bytes_c(B); }

static TrainScratch carve(char* ws, int B) {
  TrainScratch s;
  size_t o = 0;
  auto take = [&](size_t b) {
    char* p = ws + o;
    o += (b + 255) / 256 * 256;
    return p;
  };
  s.xg = (uint16_t*)take(2 * (size_t)B * MLP_NIN);
  s.xgT = (uint16_t*)take(2 * (size_t)B * MLP_NIN);
  s.h1 = (uint16_t*)take(2 * (size_t)B * MLP_NH);
  s.h1T = (uint16_t*)take(2 * (size_t)B * MLP_NH);
  s.h2 = (uint16_t*)take(2 * (size_t)B * MLP_NH);
  s.dh2 = (uint16_t*)take(2 * (size_t)B * MLP_NH);
  s.dh2T = (uint16_t*)take(2 * (size_t)B * MLP_NH);
  s.dh1T = (uint16_t*)take(2 * (size_t)B * MLP_NH);
  s.dh1 = (float*)take(4 * (size_t)B * MLP_NH);
  s.z = (float*)take(4 * (size_t)MLP_NOUT * B);
  s.dz = (float*)take(4 * (size_t)MLP_NOUT * B);
  s.grad = (float*)take(4 * (size_t)MLP_NPARAM);
  s.loss = (float*)take(4 * (size_t)B);
  s.wb = (uint16_t*)take(2 * (size_t)MLP_WB_COUNT);
  s.tstep = (int*)take(16);
  return s;
}

__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

hipError_t launch_mlp_train(const uint16_t* X, const float* Y, const int32_t* order, int n, int B, int first_batch,
                            int nbatch, float* w, float* am, float* av, const TrainHyper& hp, int t0, void* ws,
                            float* loss_out, float* grad_out, hipStream_t st) {
  TrainScratch s = carve((char*)ws, B);
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, s.tstep, t0);
  hipLaunchKernelGGL(k_mlp_prep, dim3(16), dim3(256), 0, st, w, s.wb);
  for (int b = 0; b < nbatch; b++)
    hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(256), 0, st, X, Y, order, n, B, first_batch + b, w, am, av, hp, s,
                       loss_out);
  if (grad_out) {
    hipError_t e = hipMemcpyAsync(grad_out, s.grad, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// Training scratch held by the library for callers that cannot allocate
// (amrv_mlp_train_noalloc): room for the largest batch, one copy per device
// for the life of the process.  Host code never passes the array's name to a
// kernel: it resolves each device's address with hipGetSymbolAddress once,
// with that device current, and uses that address only.
static __device__ __align__(256) char scratch[MLP_STATIC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[MLP_MAX_DEVICES] = {};
}  // namespace

hipError_t mlp_static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MLP_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace amrv
