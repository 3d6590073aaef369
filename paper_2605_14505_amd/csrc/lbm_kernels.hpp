// Kernels of the DDF lattice Boltzmann step and its diagnostics (gfx950).
#pragma once
#include "lbm_device.hpp"

namespace stgv {

// ---------------------------------------------------------------------------
// Fused stream-collide-force step (optionally with the diagnostic moments)
//
// Block (bx, by) threads over x and y; grid (ceil(n/bx), ceil(n/by), n).
// `pop` is the population array (AA) or the source lattice (AB); `dst` is the
// AB destination and equals `pop` otherwise.
// ---------------------------------------------------------------------------
// Minimum resident 256-thread blocks per CU requested from the register allocator
// (0 = compiler's choice): STGV_EVEN_MIN_BLOCKS for the plain even step with 4-byte
// storage and arithmetic (the instance that fits a tighter register budget without
// spilling), STGV_STEP_MIN_BLOCKS for every other step instance.
#ifndef STGV_STEP_MIN_BLOCKS
#define STGV_STEP_MIN_BLOCKS 0
#endif
#ifndef STGV_EVEN_MIN_BLOCKS
#define STGV_EVEN_MIN_BLOCKS STGV_STEP_MIN_BLOCKS
#endif
template <int MODE, int FLAGS, typename T, typename C>
constexpr int step_min_blocks() {
  const int b = (MODE == MODE_EVEN && FLAGS == K_COLLIDE && sizeof(T) == 4 && sizeof(C) == 4)
                    ? STGV_EVEN_MIN_BLOCKS : STGV_STEP_MIN_BLOCKS;
  return b > 0 ? b : 1;
}
#define STGV_STEP_BOUNDS_FOR(MODE, FLAGS, T, C) __launch_bounds__(256, (step_min_blocks<MODE, FLAGS, T, C>()))
#define STGV_STEP_BOUNDS STGV_STEP_BOUNDS_FOR(MODE_ODD, K_COLLIDE, T, C)

// Block coordinates of a node kernel.  The hardware hands consecutive workgroups to the
// 8 XCDs in turn, each with its own L2, so the blocks that split one row along x sit on
// different XCDs; the steps whose loads or stores are shifted along x (odd AA, A-B) share
// a line at every block seam, and then fetch it from HBM twice (at 512^3 FP16, 15 % more
// than the algorithmic bytes).  For those steps, when rows are split, the workgroups are
// renumbered so that the blocks of one row group are 8 apart in dispatch order, i.e. on
// one XCD: workgroup L = 8 (nbx q + h) + k holds x-block h of row group 8 q + k.  A
// bijection whenever the row groups (gridDim.y gridDim.z) are a multiple of 8.
struct BlockXYZ { int bx, by, bz; };

template <int MODE>
__device__ __forceinline__ BlockXYZ node_block() {
  BlockXYZ b{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z};
  const int gx = (int)gridDim.x, gy = (int)gridDim.y;
  if (MODE != MODE_EVEN && gx > 1 && ((gy * (int)gridDim.z) & 7) == 0) {
    const int L = b.bx + gx * (b.by + gy * b.bz);
    const int k = L & 7, rest = L >> 3;
    const int rg = (rest / gx) * 8 + k;
    b.bx = rest % gx;
    b.by = rg % gy;
    b.bz = rg / gy;
  }
  return b;
}

// Left alone, the compiler has the BF16 even step issue all 46 loads before its first
// wait, where the FP16 one issues 32, waits, then the rest; at the occupancy caps of
// even_step_lds that keeps more bytes in flight than the step can use.  An empty asm that
// takes the 27 f values makes the wavefront wait for them before it issues the g loads.  BF16 even step,
// ms: 512^3 4.75 -> 4.50 (at FP16's 3 blocks per CU; with a cap of 2 and all loads first
// 4.59-4.75), 256^3 0.548 -> 0.549.
template <int MODE, int FLAGS, typename T, int QF>
constexpr bool kBatchBf16 = MODE == MODE_EVEN && FLAGS == K_COLLIDE && std::is_same<T, bf16_t>::value && QF == 27;
#define STGV_OPERANDS_27(a) "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]), "+v"(a[7]), "+v"(a[8]), "+v"(a[9]), "+v"(a[10]), "+v"(a[11]), "+v"(a[12]), "+v"(a[13]), "+v"(a[14]), "+v"(a[15]), "+v"(a[16]), "+v"(a[17]), "+v"(a[18]), "+v"(a[19]), "+v"(a[20]), "+v"(a[21]), "+v"(a[22]), "+v"(a[23]), "+v"(a[24]), "+v"(a[25]), "+v"(a[26])

template <int QF, int QG, int FORCE, typename T, typename C, int MODE, int FLAGS>
__global__ STGV_STEP_BOUNDS_FOR(MODE, FLAGS, T, C) void lbm_step_kernel(T* pop, T* dst, Geometry geo,
                                                       PhysConsts c, float* __restrict__ fields,
                                                       double* __restrict__ partials) {
  const int n = geo.n;
  const BlockXYZ blk = node_block<MODE>();
  const int x = blk.bx * blockDim.x + threadIdx.x;
  const int y = blk.by * blockDim.y + threadIdx.y;
  const int z = blk.bz;
  const bool active = (x < n) && (y < n);
  constexpr bool kPart = (FLAGS & K_PARTIALS) != 0;
  if (!kPart && !active) return;

  double acc[NPART];
#pragma unroll
  for (int k = 0; k < NPART; ++k) acc[k] = 0.0;

  if (active) {
    const NodeIndex ix = make_index(x, y, z, n);
    C f[QF], g[QG];
    gather<QF, T, MODE, true>(f, pop, 0, ix, geo.stride);
    if constexpr (kBatchBf16<MODE, FLAGS, T, QF>) asm volatile("" : STGV_OPERANDS_27(f) :: "memory");
    gather<QG, T, MODE, true>(g, pop, QF, ix, geo.stride);
    StepMacro<C> m;
    step_macro<QF, QG, FORCE, sizeof(T) == 4>(f, g, c, m);
    if (FLAGS & (K_FIELDS | K_PARTIALS)) {
      const NodeMacro<C> dm = diag_macro(m);
      if (FLAGS & K_FIELDS) write_fields(dm, fields, ix.base, (int64_t)n * n * n);
      if (kPart) node_partials(dm, c, acc);
    }
    if (FLAGS & K_COLLIDE) {
      step_collide<QF, QG, FORCE, sizeof(T) == 4>(f, g, c, m);
      scatter<QF, T, MODE>(f, dst, 0, ix, geo.stride);
      scatter<QG, T, MODE>(g, dst, QF, ix, geo.stride);
    }
  }
  if (kPart) {
    const int64_t b = blk.bx + (int64_t)gridDim.x * (blk.by + (int64_t)gridDim.y * blk.bz);
    block_reduce_store<NPART, (1u << P_UMAX2)>(acc, partials + b * NPART);
  }
}

// The plain odd step row-aligned, its x-shift taken through a ring in LDS per block row
// (row_load / row_pick / row_put / row_store), on the shapes of ring_shape (blocks of
// whole rows, or 256-node blocks holding part of one row), which tile the box exactly,
// so every lane is active and reaches the barriers.
// PART: blocks holding part of a row, whose x-moving loads and stores use the cache
// policy STGV_RING_PART_NT_XLOAD / STGV_RING_PART_NT_XSTORE (1 = bypass); whole-row
// blocks bypass the caches for every access.  A seam lane's load shares its line with
// the neighbouring block's aligned load, which finds it in L2 only if it was loaded
// cached: 512^3 odd step FP16 5.21 -> 4.80 ms, BF16 5.67 -> 4.82 ms with cached x-moving
// loads; cached x-moving stores changed nothing further (4.80 / 4.80) and alone gave
// 4.90 / 4.96.
#ifndef STGV_RING_PART_NT_XLOAD
#define STGV_RING_PART_NT_XLOAD 0
#endif
#ifndef STGV_RING_PART_NT_XSTORE
#define STGV_RING_PART_NT_XSTORE 1
#endif
template <int QF, int QG, int FORCE, typename T, typename C, bool PART>
__global__ STGV_STEP_BOUNDS void lbm_step_ring_kernel(T* pop, Geometry geo, PhysConsts c) {
  constexpr bool NL = !PART || STGV_RING_PART_NT_XLOAD, NS = !PART || STGV_RING_PART_NT_XSTORE;
  constexpr int KF = x_moving<QF>(), KG = x_moving<QG>();
  __shared__ T xs[KF + KG][256];
  const int n = geo.n;
  const BlockXYZ blk = node_block<MODE_ODD>();
  const int x = blk.bx * blockDim.x + threadIdx.x;
  const int y = blk.by * blockDim.y + threadIdx.y;
  const NodeIndex ix = make_index(x, y, blk.bz, n);
  const RowLane l = make_rowlane(x, n);
  C f[QF], g[QG];
  row_load<QF, T, NL>(f, xs, 0, pop, 0, ix, geo.stride, l, std::make_integer_sequence<int, QF>{});
  row_load<QG, T, NL>(g, xs, KF, pop, QF, ix, geo.stride, l, std::make_integer_sequence<int, QG>{});
  __syncthreads();
  row_pick<QF>(f, (const T(*)[256])xs, 0, l, std::make_integer_sequence<int, QF>{});
  row_pick<QG>(g, (const T(*)[256])xs, KF, l, std::make_integer_sequence<int, QG>{});
  __syncthreads();                      // every lane has taken its values before any put
  StepMacro<C> m;
  step_macro<QF, QG, FORCE, sizeof(T) == 4>(f, g, c, m);
  step_collide<QF, QG, FORCE, sizeof(T) == 4>(f, g, c, m);
  row_put<QF>(f, xs, 0, l, std::make_integer_sequence<int, QF>{});
  row_put<QG>(g, xs, KF, l, std::make_integer_sequence<int, QG>{});
  __syncthreads();
  row_store<QF, T, NS>(f, (const T(*)[256])xs, 0, pop, 0, ix, geo.stride, l, std::make_integer_sequence<int, QF>{});
  row_store<QG, T, NS>(g, (const T(*)[256])xs, KF, pop, QF, ix, geo.stride, l, std::make_integer_sequence<int, QG>{});
}

// ---------------------------------------------------------------------------
// Free streaming: the step's loads, stores, launch shape and block order with the
// identity in place of the collision, so every population moves one link along its
// velocity per call (the streaming half of Eqs. (5) and (11) alone).  Values pass
// through FP32, which holds every FP16 / BF16 value exactly, so a stream is exact in
// every storage type.  It is the ceiling of the step's own access pattern.
// ---------------------------------------------------------------------------
template <int QF, int QG, typename T, int MODE>
__global__ __launch_bounds__(256) void lbm_stream_kernel(T* pop, T* dst, Geometry geo) {
  const int n = geo.n;
  const BlockXYZ blk = node_block<MODE>();
  const int x = blk.bx * blockDim.x + threadIdx.x;
  const int y = blk.by * blockDim.y + threadIdx.y;
  if (x >= n || y >= n) return;
  const NodeIndex ix = make_index(x, y, blk.bz, n);
  float f[QF], g[QG];
  gather<QF, T, MODE, true>(f, pop, 0, ix, geo.stride);
  gather<QG, T, MODE, true>(g, pop, QF, ix, geo.stride);
  scatter<QF, T, MODE>(f, dst, 0, ix, geo.stride);
  scatter<QG, T, MODE>(g, dst, QF, ix, geo.stride);
}

// The odd free-streaming step row-aligned, on the shapes where the odd step runs
// row-aligned (ring_shape; every lane active).
template <int QF, int QG, typename T, bool PART>
__global__ __launch_bounds__(256) void lbm_stream_ring_kernel(T* pop, Geometry geo) {
  constexpr bool NL = !PART || STGV_RING_PART_NT_XLOAD, NS = !PART || STGV_RING_PART_NT_XSTORE;
  constexpr int KF = x_moving<QF>(), KG = x_moving<QG>();
  __shared__ T xs[KF + KG][256];
  const int n = geo.n;
  const BlockXYZ blk = node_block<MODE_ODD>();
  const int x = blk.bx * blockDim.x + threadIdx.x;
  const int y = blk.by * blockDim.y + threadIdx.y;
  const NodeIndex ix = make_index(x, y, blk.bz, n);
  const RowLane l = make_rowlane(x, n);
  float f[QF], g[QG];
  row_load<QF, T, NL>(f, xs, 0, pop, 0, ix, geo.stride, l, std::make_integer_sequence<int, QF>{});
  row_load<QG, T, NL>(g, xs, KF, pop, QF, ix, geo.stride, l, std::make_integer_sequence<int, QG>{});
  __syncthreads();
  row_pick<QF>(f, (const T(*)[256])xs, 0, l, std::make_integer_sequence<int, QF>{});
  row_pick<QG>(g, (const T(*)[256])xs, KF, l, std::make_integer_sequence<int, QG>{});
  __syncthreads();
  row_put<QF>(f, xs, 0, l, std::make_integer_sequence<int, QF>{});
  row_put<QG>(g, xs, KF, l, std::make_integer_sequence<int, QG>{});
  __syncthreads();
  row_store<QF, T, NS>(f, (const T(*)[256])xs, 0, pop, 0, ix, geo.stride, l, std::make_integer_sequence<int, QF>{});
  row_store<QG, T, NS>(g, (const T(*)[256])xs, KF, pop, QF, ix, geo.stride, l, std::make_integer_sequence<int, QG>{});
}

// ---------------------------------------------------------------------------
// Taylor-Green initial state (Eqs. (20)-(21)) in natural order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  // one output of SplitMix64 (Steele, Lea & Flood 2014) from state x
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// One rounding of an FP64 value into the storage type.  FP32 rounds directly; FP16 and
// BF16 go through FP32 rounded to odd (truncate, then set the last bit when inexact),
// which carries at least two more significand bits than either, so the final
// round-to-nearest-even of the hardware conversion equals a direct rounding of the
// FP64 value.
__device__ __forceinline__ float round_to_odd_f32(double d) {
  float r = (float)d;
  if ((double)r != d) {
    uint32_t b = __float_as_uint(r);
    if (fabs((double)r) > fabs(d)) b -= 1u;     // step back toward zero (sign-magnitude)
    r = __uint_as_float(b | 1u);
  }
  return r;
}
__device__ __forceinline__ void store_once(float* p, double d) { store_as(p, (float)d); }
__device__ __forceinline__ void store_once(_Float16* p, double d) { store_as(p, round_to_odd_f32(d)); }
__device__ __forceinline__ void store_once(bf16_t* p, double d) { store_as(p, round_to_odd_f32(d)); }

template <int QF, int QG, typename T>
__global__ __launch_bounds__(256) void lbm_init_tgv_kernel(T* pop, Geometry geo, double u0,
                                                           double noise_amp, uint64_t seed) {
  using SF = Stencil<QF>;
  using SG = Stencil<QG>;
  const int n = geo.n;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= n || y >= n) return;
  const int64_t node = (int64_t)x + (int64_t)n * (y + (int64_t)n * z);
  const double h = 2.0 * M_PI / n;
  const double X = h * x, Y = h * y, Z = h * z;
  const double vx = u0 * sin(X) * cos(Y) * cos(Z);
  const double vy = -u0 * cos(X) * sin(Y) * cos(Z);
  const double vz = 0.0;
  const double p0 = u0 * u0 / 16.0 * (cos(2.0 * X) + cos(2.0 * Y)) * (cos(2.0 * Z) + 2.0);
  const double drho = p0 / SF::cs2;
  const double rho = 1.0 + drho;
  const uint64_t ctr = (seed << 40) + (uint64_t)node;
  const double xi = (double)(splitmix64(ctr) >> 11) * 0x1.0p-53;
  const double rho_p = noise_amp * (2.0 * xi - 1.0);
  const double usq = vx * vx + vy * vy + vz * vz;
#pragma unroll
  for (int i = 0; i < QF; ++i) {
    const double eu = SF::ex[i] * vx + SF::ey[i] * vy + SF::ez[i] * vz;
    const double d = SF::w[i] * (drho + rho * (eu / SF::cs2 + eu * eu / (2.0 * SF::cs2 * SF::cs2)
                                               - usq / (2.0 * SF::cs2)));
    store_once(pop + (int64_t)i * geo.stride + node, d);
  }
#pragma unroll
  for (int j = 0; j < QG; ++j) {
    const double eu = SG::ex[j] * vx + SG::ey[j] * vy + SG::ez[j] * vz;
    const double poly = eu / SG::cs2 + eu * eu / (2.0 * SG::cs2 * SG::cs2) - usq / (2.0 * SG::cs2);
    const double d = SG::w[j] * (rho_p + (1.0 + rho_p) * poly);
    store_once(pop + (int64_t)(QF + j) * geo.stride + node, d);
  }
}

// ---------------------------------------------------------------------------
// Layout conversion: current layout -> natural FP32 deviations, and back.
// ---------------------------------------------------------------------------
template <int QF, int QG, typename T, int MODE>
__global__ __launch_bounds__(256) void lbm_canon_kernel(const T* pop, Geometry geo,
                                                        float* __restrict__ out) {
  const int n = geo.n;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= n || y >= n) return;
  const NodeIndex ix = make_index(x, y, z, n);
  const int64_t n3 = (int64_t)n * n * n;
  float f[QF], g[QG];
  gather<QF, T, MODE>(f, pop, 0, ix, geo.stride);
  gather<QG, T, MODE>(g, pop, QF, ix, geo.stride);
#pragma unroll
  for (int i = 0; i < QF; ++i) out[i * n3 + ix.base] = f[i];
#pragma unroll
  for (int j = 0; j < QG; ++j) out[(QF + j) * n3 + ix.base] = g[j];
}

template <int QF, int QG, typename T>
__global__ __launch_bounds__(256) void lbm_load_kernel(T* pop, Geometry geo,
                                                       const float* __restrict__ in) {
  const int n = geo.n;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= n || y >= n) return;
  const int64_t n3 = (int64_t)n * n * n;
  const int64_t node = (int64_t)x + (int64_t)n * (y + (int64_t)n * z);
#pragma unroll
  for (int i = 0; i < QF + QG; ++i)
    store_as(pop + (int64_t)i * geo.stride + node, in[i * n3 + node]);
}

}  // namespace stgv
