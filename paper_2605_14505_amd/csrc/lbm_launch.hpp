// Host-side launchers: map run-time choices (stencil pair, forcing, layout mode,
// kernel flags) onto the kernel template instances of one storage type.
#pragma once
#include <hip/hip_runtime.h>

#include "lbm_device.hpp"

namespace stgv {

struct LaunchShape {
  dim3 grid, block;
};

// The stencil pairs (momentum Q_f x scalar Q_g) with kernel instances: those of the
// stencil comparisons of Sections 3.2-3.3 and of the D3Q7-scalar sweep.  X(qf, qg) is applied
// to each.
#define STGV_FOR_EACH_PAIR(X) X(27, 19) X(27, 7) X(19, 7) X(27, 27) X(19, 19) X(19, 15) X(15, 7) X(7, 27)

// Launch shape of the node kernels: block (bx, by) over x and y, grid over
// (x, y, z).  Blocks are 256 threads except when a row is shorter than a
// wavefront; every block is a whole number of 64-wide wavefronts.
#ifndef STGV_BLOCK_X
#define STGV_BLOCK_X 256
#endif
inline LaunchShape node_shape(int n) {
  int bx, by;
  if (n <= 64 && 64 % n == 0) {
    bx = n;
    by = 256 / n;
  } else if (n % 64 != 0 && n % 32 == 0) {
    bx = 32;                      // whole 128-byte lines per row, no idle lanes (n = 96, 160, ...)
    by = 8;
  } else if (n % 64 == 0) {
    bx = n % 256 == 0 ? 256 : (n % 128 == 0 ? 128 : 64);   // rows split evenly (n = 320, 384, 448)
    by = 256 / bx;
  } else {
    bx = ((n + 63) / 64) * 64;
    if (bx > STGV_BLOCK_X) bx = STGV_BLOCK_X;
    by = 256 / bx;
  }
  LaunchShape s;
  s.block = dim3(bx, by, 1);
  s.grid = dim3((n + bx - 1) / bx, (n + by - 1) / by, n);
  return s;
}

// Whether the plain odd step runs row-aligned through an LDS ring (lbm_step_ring_kernel):
// on blocks of whole rows that tile the box or on 256-node blocks holding part of one
// row (n a multiple of 256, from 512); whole rows from n = 128 for 2-byte storage, from
// n = 256 for FP32 (FP32 at 128^3 and 64^3 lost 13 % and 2.5 % with it).  Only for the
// stencil pairs where it measured faster (ring_pair).  Measured on gfx950 (odd step, ms,
// shifted loads and stores -> ring): 256^3 FP32 27x19 1.141 -> 1.090 (2 blocks per CU,
// ring_step_lds), 19x19 0.957 -> 0.871, 7x27 0.819 -> 0.805; FP16 27x19 0.567 -> 0.549,
// 27x7 0.403 -> 0.396; 512^3 27x19 FP32 9.61 -> 9.22, FP16 4.80 and BF16 4.82 against 5.22
// and 9.5 for LDS-staged stores alone.  Slower with the ring, so shifted: FP32 27x27
// (1.377 -> 1.822), 19x15, 15x7, 19x7, 27x7 (within 1 %); FP16 19x7 (0.294 -> 0.308).
template <int QF, int QG>
constexpr bool ring_pair(size_t elem) {
  return elem == 4 ? ((QF == 27 && QG == 19) || (QF == 19 && QG == 19) || (QF == 7 && QG == 27))
                   : ((QF == 27 && QG == 19) || (QF == 27 && QG == 7));
}
inline bool ring_whole_shape(const LaunchShape& sh, int n, size_t elem) {
  const int bx = (int)sh.block.x, by = (int)sh.block.y;
  return n >= (elem == 4 ? 256 : 128) && bx == n && sh.grid.x == 1 && bx * by == 256 && n % by == 0;
}
inline bool ring_part_shape(const LaunchShape& sh, int n) {
  return n >= 512 && sh.block.x == 256 && sh.block.y == 1 && n % 256 == 0;
}
inline bool ring_shape(const LaunchShape& sh, int n, size_t elem) {
  return ring_whole_shape(sh, n, elem) || ring_part_shape(sh, n);
}

// Blocks resident per CU for the plain even step (0 = as many as the registers allow), set
// by requesting unused dynamic LDS (160 KiB per CU): FP32 storage for n >= 256, 2-byte
// storage for n >= 512.  The even step keeps every population array of its resident
// wavefronts open at once; past ~70-95 KB of loads in flight per CU more wavefronts only
// add open streams.  Measured on gfx950 (D3Q27 x D3Q19 even step, ms): FP32 at 2 blocks
// instead of 4, 256^3 1.137 -> 1.080, 384^3 4.02 -> 3.84, 512^3 9.26 -> 8.98 (3 blocks:
// 1.131 at 256^3); 2-byte storage at 3 blocks instead of 4, 512^3 FP16 4.67 -> 4.42, BF16
// 5.00 -> 4.92 (before its loads were batched), while 256^3 and 128^3 lose with any cap.  The shifted odd step, whose
// x-shifted lines neighbouring wavefronts share, gains nothing from a cap; the ring odd
// step has its own (ring_step_lds).
// The caps assume a step that issues its loads in two batches; the BF16 even step is made
// to (lbm_step_kernel), and is then best with FP16's caps.
#ifndef STGV_EVEN_CAP_FP32
#define STGV_EVEN_CAP_FP32 2
#endif
#ifndef STGV_EVEN_CAP_2B
#define STGV_EVEN_CAP_2B 3
#endif
inline size_t even_step_lds(size_t elem, int n) {
  const int cap = elem == 4 ? (n >= 256 ? STGV_EVEN_CAP_FP32 : 0) : (n >= 512 ? STGV_EVEN_CAP_2B : 0);
  if (cap <= 0) return 0;
  // just over a (cap + 1)-th of the CU's LDS, so that cap blocks fit and cap + 1 do not
  size_t b = (160u * 1024u) / (size_t)(cap + 1) + 1024u;
  return b > 65536u ? 65536u : b;
}

// Blocks resident per CU for the ring odd step (0 = as many as registers and its LDS
// allow), counting the kernel's own LDS of `static_lds` bytes: FP32 at 2 (256^3 odd step
// 1.103 -> 1.088 ms, 512^3 9.37 -> 9.22 against no cap; at 3, 1.106); 2-byte storage lost
// with a cap of 2 (256^3 0.553 -> 0.600), gained nothing at 3 or 4 (512^3), and keeps none.
#ifndef STGV_ODD_CAP_FP32
#define STGV_ODD_CAP_FP32 2
#endif
#ifndef STGV_ODD_CAP_2B
#define STGV_ODD_CAP_2B 0
#endif
inline size_t ring_step_lds(size_t elem, size_t static_lds) {
  const int cap = elem == 4 ? STGV_ODD_CAP_FP32 : STGV_ODD_CAP_2B;
  if (cap <= 0) return 0;
  const size_t want = (160u * 1024u) / (size_t)(cap + 1) + 1024u;
  if (want <= static_lds) return 0;
  return want > 65536u ? 65536u - static_lds : want - static_lds;
}

// Every function returns the launch error (hipSuccess when queued).
template <typename T, typename C>
hipError_t launch_step(int qf, int qg, int force, int mode, int flags, const LaunchShape& sh,
                       hipStream_t st, T* pop, T* dst, Geometry geo, PhysConsts c,
                       float* fields, double* partials);

template <typename T>
hipError_t launch_init(int qf, int qg, const LaunchShape& sh, hipStream_t st, T* pop, Geometry geo,
                       double u0, double noise_amp, uint64_t seed);

// Free streaming (lbm_stream_kernel) in layout MODE, from pop into dst.
template <typename T>
hipError_t launch_stream(int qf, int qg, int mode, const LaunchShape& sh, hipStream_t st, T* pop,
                         T* dst, Geometry geo);

template <typename T>
hipError_t launch_canon(int qf, int qg, int mode, const LaunchShape& sh, hipStream_t st,
                        const T* pop, Geometry geo, float* out);

template <typename T>
hipError_t launch_load(int qf, int qg, const LaunchShape& sh, hipStream_t st, T* pop,
                       Geometry geo, const float* in);

}  // namespace stgv
