// The fused learned step: D3Q27 x D3Q19, FP32 populations and arithmetic, with
// the network's moment correction (K_LEARNED) and optionally the diagnostics.
#include "lbm_kernels.hpp"
#include "learned.hpp"

namespace stgv {
namespace {

template <int FORCE, int MODE, int FLAGS>
hipError_t go(int n, hipStream_t st, float* pop, float* dst, Geometry geo, PhysConsts c,
              float* fields, double* partials, const void* net) {
  const dim3 block(64, 1, 1), grid(n / 64, n, n);
  hipLaunchKernelGGL((lbm_step_kernel<27, 19, FORCE, float, float, MODE, FLAGS>), grid, block, 0, st,
                     pop, dst, geo, c, fields, partials, net);
  return hipGetLastError();
}

template <int FORCE>
hipError_t by_mode(int mode, bool diag, int n, hipStream_t st, float* pop, float* dst, Geometry geo,
                   PhysConsts c, float* fields, double* partials, const void* net) {
  constexpr int S = K_COLLIDE | K_LEARNED;
  constexpr int D = K_COLLIDE | K_FIELDS | K_PARTIALS | K_LEARNED;
  switch (mode) {
    case MODE_EVEN: return diag ? go<FORCE, MODE_EVEN, D>(n, st, pop, dst, geo, c, fields, partials, net)
                                : go<FORCE, MODE_EVEN, S>(n, st, pop, dst, geo, c, fields, partials, net);
    case MODE_ODD: return diag ? go<FORCE, MODE_ODD, D>(n, st, pop, dst, geo, c, fields, partials, net)
                               : go<FORCE, MODE_ODD, S>(n, st, pop, dst, geo, c, fields, partials, net);
    default: return diag ? go<FORCE, MODE_AB, D>(n, st, pop, dst, geo, c, fields, partials, net)
                         : go<FORCE, MODE_AB, S>(n, st, pop, dst, geo, c, fields, partials, net);
  }
}

}  // namespace

hipError_t launch_learned_step(int forcing, int mode, int flags, int n, hipStream_t st, float* pop,
                               float* dst, Geometry geo, PhysConsts c, float* fields, double* partials,
                               const void* packed) {
  const bool diag = (flags & K_PARTIALS) != 0;
  if (forcing == FORCE_GUO) return by_mode<FORCE_GUO>(mode, diag, n, st, pop, dst, geo, c, fields, partials, packed);
  return by_mode<FORCE_SHIFT>(mode, diag, n, st, pop, dst, geo, c, fields, partials, packed);
}

}  // namespace stgv
