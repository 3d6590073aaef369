// Template instances of the node kernels for one storage type STGV_T and one
// compute type STGV_C.  Included once per (storage, compute) pair by the
// lbm_*.hip translation units; the layout kernels (init, canonicalise, load)
// are instantiated by the FP32-compute unit of each storage type
// (STGV_LAYOUT_KERNELS).
#pragma once
#include "lbm_kernels.hpp"
#include "lbm_launch.hpp"

namespace stgv {
// Internal linkage: every (storage, compute) translation unit has its own
// helpers, whose template arguments do not name the compute type.
namespace {

template <int QF, int QG, int FORCE, typename T, int MODE, int FLAGS>
hipError_t go_step(const LaunchShape& sh, hipStream_t st, T* pop, T* dst, Geometry geo,
                   PhysConsts c, float* fields, double* partials) {
  const size_t lds = (MODE == MODE_EVEN && FLAGS == K_COLLIDE) ? even_step_lds(sizeof(T), geo.n) : 0;
  hipLaunchKernelGGL((lbm_step_kernel<QF, QG, FORCE, T, STGV_C, MODE, FLAGS>), sh.grid, sh.block,
                     lds, st, pop, dst, geo, c, fields, partials);
  return hipGetLastError();
}

template <int QF, int QG, int FORCE, typename T>
hipError_t step_force(int mode, bool diag, const LaunchShape& sh, hipStream_t st, T* pop, T* dst,
                      Geometry geo, PhysConsts c, float* fields, double* partials) {
  constexpr int STEP = K_COLLIDE;
  constexpr int STEP_DIAG = K_COLLIDE | K_FIELDS | K_PARTIALS;
#define STGV_GO(M) \
  return diag ? go_step<QF, QG, FORCE, T, M, STEP_DIAG>(sh, st, pop, dst, geo, c, fields, partials) \
              : go_step<QF, QG, FORCE, T, M, STEP>(sh, st, pop, dst, geo, c, fields, partials)
  if (mode == MODE_EVEN) STGV_GO(MODE_EVEN);
  if constexpr (sizeof(STGV_C) == 4 && ring_pair<QF, QG>(sizeof(T))) {
    if (mode == MODE_ODD && !diag && ring_shape(sh, geo.n, sizeof(T))) {
      const size_t lds = ring_step_lds(sizeof(T), (size_t)(x_moving<QF>() + x_moving<QG>()) * 256 * sizeof(T));
      if (ring_whole_shape(sh, geo.n, sizeof(T)))
        hipLaunchKernelGGL((lbm_step_ring_kernel<QF, QG, FORCE, T, STGV_C, false>), sh.grid, sh.block, lds,
                           st, pop, geo, c);
      else
        hipLaunchKernelGGL((lbm_step_ring_kernel<QF, QG, FORCE, T, STGV_C, true>), sh.grid, sh.block, lds,
                           st, pop, geo, c);
      return hipGetLastError();
    }
  }
  if (mode == MODE_ODD) STGV_GO(MODE_ODD);
  if (mode == MODE_AB) STGV_GO(MODE_AB);
#undef STGV_GO
  return hipErrorInvalidValue;
}

template <int QF, int QG, typename T>
hipError_t step_pair(int force, int mode, int flags, const LaunchShape& sh, hipStream_t st, T* pop,
                     T* dst, Geometry geo, PhysConsts c, float* fields, double* partials) {
  constexpr int STEP = K_COLLIDE;
  constexpr int STEP_DIAG = K_COLLIDE | K_FIELDS | K_PARTIALS;
  constexpr int SAMPLE = K_FIELDS | K_PARTIALS;
  constexpr int FIELDS = K_FIELDS;
  if (flags == STEP || flags == STEP_DIAG) {
    const bool d = flags == STEP_DIAG;
    switch (force) {
      case FORCE_GUO: return step_force<QF, QG, FORCE_GUO, T>(mode, d, sh, st, pop, dst, geo, c, fields, partials);
      case FORCE_SHIFT: return step_force<QF, QG, FORCE_SHIFT, T>(mode, d, sh, st, pop, dst, geo, c, fields, partials);
      case FORCE_EDM: return step_force<QF, QG, FORCE_EDM, T>(mode, d, sh, st, pop, dst, geo, c, fields, partials);
      case FORCE_HCZ: return step_force<QF, QG, FORCE_HCZ, T>(mode, d, sh, st, pop, dst, geo, c, fields, partials);
      default: return hipErrorInvalidValue;
    }
  }
  // Moment-only passes read the natural layout (MODE_EVEN, also the AB lattice)
  // or the odd AA layout; the physical velocity does not depend on the forcing.
#define STGV_GO(M, FL) return go_step<QF, QG, FORCE_GUO, T, M, FL>(sh, st, pop, dst, geo, c, fields, partials)
  const int gm = (mode == MODE_ODD) ? MODE_ODD : MODE_EVEN;
  if (flags == SAMPLE) {
    if (gm == MODE_EVEN) STGV_GO(MODE_EVEN, SAMPLE);
    STGV_GO(MODE_ODD, SAMPLE);
  }
  if (flags == FIELDS) {
    if (gm == MODE_EVEN) STGV_GO(MODE_EVEN, FIELDS);
    STGV_GO(MODE_ODD, FIELDS);
  }
#undef STGV_GO
  return hipErrorInvalidValue;
}

}  // namespace

template <>
hipError_t launch_step<STGV_T, STGV_C>(int qf, int qg, int force, int mode, int flags,
                               const LaunchShape& sh, hipStream_t st, STGV_T* pop, STGV_T* dst,
                               Geometry geo, PhysConsts c, float* fields, double* partials) {
#define STGV_STEP_PAIR(A, B) \
  if (qf == A && qg == B) return step_pair<A, B, STGV_T>(force, mode, flags, sh, st, pop, dst, geo, c, fields, partials);
  STGV_FOR_EACH_PAIR(STGV_STEP_PAIR)
#undef STGV_STEP_PAIR
  return hipErrorInvalidValue;
}

#ifdef STGV_LAYOUT_KERNELS
template <>
hipError_t launch_init<STGV_T>(int qf, int qg, const LaunchShape& sh, hipStream_t st, STGV_T* pop,
                               Geometry geo, double u0, double noise_amp, uint64_t seed) {
#define STGV_INIT(A, B) \
  if (qf == A && qg == B) { \
    hipLaunchKernelGGL((lbm_init_tgv_kernel<A, B, STGV_T>), sh.grid, sh.block, 0, st, pop, geo, u0, noise_amp, seed); \
    return hipGetLastError(); }
  STGV_FOR_EACH_PAIR(STGV_INIT)
#undef STGV_INIT
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_stream<STGV_T>(int qf, int qg, int mode, const LaunchShape& sh, hipStream_t st,
                                 STGV_T* pop, STGV_T* dst, Geometry geo) {
  const bool ring = mode == MODE_ODD && ring_shape(sh, geo.n, sizeof(STGV_T));
  const bool whole = ring_whole_shape(sh, geo.n, sizeof(STGV_T));
#define STGV_STREAM(A, B) \
  if (qf == A && qg == B) { \
    if constexpr (ring_pair<A, B>(sizeof(STGV_T))) { \
      if (ring) { \
        const size_t lds = ring_step_lds(sizeof(STGV_T), (size_t)(x_moving<A>() + x_moving<B>()) * 256 * sizeof(STGV_T)); \
        if (whole) hipLaunchKernelGGL((lbm_stream_ring_kernel<A, B, STGV_T, false>), sh.grid, sh.block, lds, st, pop, geo); \
        else hipLaunchKernelGGL((lbm_stream_ring_kernel<A, B, STGV_T, true>), sh.grid, sh.block, lds, st, pop, geo); \
        return hipGetLastError(); \
      } \
    } \
    if (mode == MODE_EVEN) hipLaunchKernelGGL((lbm_stream_kernel<A, B, STGV_T, MODE_EVEN>), sh.grid, sh.block, even_step_lds(sizeof(STGV_T), geo.n), st, pop, dst, geo); \
    else if (mode == MODE_ODD) hipLaunchKernelGGL((lbm_stream_kernel<A, B, STGV_T, MODE_ODD>), sh.grid, sh.block, 0, st, pop, dst, geo); \
    else if (mode == MODE_AB) hipLaunchKernelGGL((lbm_stream_kernel<A, B, STGV_T, MODE_AB>), sh.grid, sh.block, 0, st, pop, dst, geo); \
    else return hipErrorInvalidValue; \
    return hipGetLastError(); }
  STGV_FOR_EACH_PAIR(STGV_STREAM)
#undef STGV_STREAM
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_canon<STGV_T>(int qf, int qg, int mode, const LaunchShape& sh, hipStream_t st,
                                const STGV_T* pop, Geometry geo, float* out) {
#define STGV_CANON(A, B) \
  if (qf == A && qg == B) { \
    if (mode == MODE_ODD) hipLaunchKernelGGL((lbm_canon_kernel<A, B, STGV_T, MODE_ODD>), sh.grid, sh.block, 0, st, pop, geo, out); \
    else hipLaunchKernelGGL((lbm_canon_kernel<A, B, STGV_T, MODE_EVEN>), sh.grid, sh.block, 0, st, pop, geo, out); \
    return hipGetLastError(); }
  STGV_FOR_EACH_PAIR(STGV_CANON)
#undef STGV_CANON
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_load<STGV_T>(int qf, int qg, const LaunchShape& sh, hipStream_t st, STGV_T* pop,
                               Geometry geo, const float* in) {
#define STGV_LOAD(A, B) \
  if (qf == A && qg == B) { \
    hipLaunchKernelGGL((lbm_load_kernel<A, B, STGV_T>), sh.grid, sh.block, 0, st, pop, geo, in); \
    return hipGetLastError(); }
  STGV_FOR_EACH_PAIR(STGV_LOAD)
#undef STGV_LOAD
  return hipErrorInvalidValue;
}
#endif  // STGV_LAYOUT_KERNELS

}  // namespace stgv
