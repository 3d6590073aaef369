// Host launchers of the learned-correction kernels (learned.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"

namespace stgv {

hipError_t mlp_launch_pack(const float* theta, const float* norm, void* packed, hipStream_t st);
hipError_t mlp_launch_forward(const void* packed, const float* x, int64_t rows, float* y, hipStream_t st);
hipError_t mlp_launch_grad(const void* packed, const float* x, const float* y, const int64_t* idx,
                           int64_t batch, float* gpart, double* lpart, float* grad, double* loss,
                           hipStream_t st);
hipError_t mlp_launch_adam(float* theta, float* m, float* v, const float* grad, float lr, float b1,
                           float b2, float omb1, float omb2, float eps, float c1, float c2, hipStream_t st);
hipError_t mlp_launch_norm(const float* x, const float* y, int64_t rows, double* part, int nblocks,
                           float* norm, hipStream_t st);
hipError_t mlp_launch_restrict(int storage, const void* fine, int mode, Geometry gf, PhysConsts cf,
                               int nc, float sf, float sg, float* out, hipStream_t st);
hipError_t mlp_launch_pairs(int forcing, const float* a, const float* b, const float* c, int nc,
                            PhysConsts pc, float* x, float* y, hipStream_t st);
// The fused learned step of a D3Q27 x D3Q19 FP32 state, n % 64 == 0 (learned_step.hip);
// flags & K_PARTIALS selects the diagnostic variant.
hipError_t launch_learned_step(int forcing, int mode, int flags, int n, hipStream_t st, float* pop,
                               float* dst, Geometry geo, PhysConsts c, float* fields, double* partials,
                               const void* packed);

}  // namespace stgv
