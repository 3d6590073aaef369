// Device code of the fused stream-collide-force step (gfx950).
//
// One thread owns one lattice node.  Populations are stored as deviations from
// their lattice weights (df_i = f_i - w_i, dg_j = g_j - w^g_j), structure of
// arrays: array i holds df_i for every node, x fastest, arrays `stride`
// elements apart; the Q_f momentum arrays come first, then the Q_g scalar
// arrays.  All collision and forcing arithmetic is FP32 on the deviations (no
// "1 -" cancellation); storage is FP32, FP16 or BF16.
//
// Streaming (LHS of Eqs. (5) and (11), periodic box) uses the AA in-place
// pattern: an even step reads slot i of its own node and writes the
// post-collision value into slot opp(i) of the same node; an odd step reads
// slot opp(i) at x - e_i and writes slot i at x + e_i.  Both touch exactly the
// same addresses a thread reads, so the update is race-free in place.  After
// an even number of steps the array is in natural (pre-collision, streamed)
// order.  MODE_AB is a two-lattice push variant (read natural at x, write
// natural at x + e_i into a second array) kept for bitwise cross-checking.
#pragma once
#include <type_traits>
#include <utility>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stencil.hpp"

namespace stgv {

enum Mode : int { MODE_EVEN = 0, MODE_ODD = 1, MODE_AB = 2 };
// Guo source term, Shan-Chen velocity shift (Eq. (10)), exact difference method
// (Kupershtokh), He-Shan-Doolen source term: the four schemes of the forcing comparison.
enum Forcing : int { FORCE_GUO = 0, FORCE_SHIFT = 1, FORCE_EDM = 2, FORCE_HCZ = 3 };
enum KernelFlags : int {
  K_COLLIDE = 1,    // collide and stream (the time step)
  K_FIELDS = 2,     // write rho - 1, u_x, u_y, u_z, rho' per node
  K_PARTIALS = 4,   // write per-block diagnostic partials
};

// Per-block diagnostic partials written by the diagnostic step / moments kernels.
enum Partial : int {
  P_EK = 0,     // sum 1/2 |u|^2
  P_EP,         // sum 1/2 ((G/N) rho')^2
  P_DRHO,       // sum (rho - 1)
  P_DSIG,       // sum (sum_j g_j - 1)
  P_MX, P_MY, P_MZ,  // sum rho u
  P_UMAX2,      // max |u|^2
  P_NONFINITE,  // count of nodes with a non-finite moment
  NPART
};
enum FdPartial : int { FD_CURL2 = 0, FD_GRAD2, NFD };

// Record layout in the device diagnostics ring (doubles).
enum Record : int {
  R_STEP = 0, R_EK, R_EP, R_CURL2, R_GRAD2, R_DRHO, R_DSIG, R_MX, R_MY, R_MZ, R_UMAX2,
  R_NONFINITE, NREC = 16
};

struct PhysConsts {
  double omega_f;     // 1 / tau_f
  double omega_g;     // 1 / tau_g
  double tau_f;       // Shan-Chen shift
  double G;           // Boussinesq gravity (lattice units)
  double beta;        // (d rho_b / dz)_LU
  double g_over_n;    // G / N for the potential energy
};

struct Geometry {
  int n;             // box edge
  int64_t stride;    // elements between population arrays
};

// ---------------------------------------------------------------------------
// storage <-> compute conversion (compute type C is float or double)
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };

// Population loads that bypass the caches, per layout mode (bit MODE of the mask), and in
// the odd step for the directions with e_x = 0 (whose lines no neighbouring wavefront
// shares) where the kernel asks for it.  Every value is read once per step; measured on
// gfx950 (256^3 D3Q27 x D3Q19, FP32 / FP16 storage), non-temporal loads of the even step
// and of the odd step's x-aligned directions take 7-8 % off both steps, while
// non-temporal loads of the x-shifted directions, whose lines two wavefronts share, make
// the odd step 20-30 % slower.  (The row-aligned odd step, lbm_step_ring_kernel, sets
// its own cache policy.)
#ifndef STGV_NT_LOAD_MODES
#define STGV_NT_LOAD_MODES 1
#endif
#ifndef STGV_NT_LOAD_ODD_XALIGNED
#define STGV_NT_LOAD_ODD_XALIGNED 1
#endif
template <bool NT, typename T>
__device__ __forceinline__ T get(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename C, bool NT = false> __device__ __forceinline__ C load_as(const float* p) { return (C)get<NT>(p); }
template <typename C, bool NT = false> __device__ __forceinline__ C load_as(const _Float16* p) { return (C)(float)get<NT>(p); }
template <typename C, bool NT = false> __device__ __forceinline__ C load_as(const bf16_t* p) {
  return (C)__uint_as_float(((uint32_t)get<NT>(&p->bits)) << 16);
}

// Population stores bypass the caches by default (each value is read again only
// one step later, after the whole ~GB state has streamed through).
#ifndef STGV_NT_STORE
#define STGV_NT_STORE 1
#endif
template <typename T>
__device__ __forceinline__ void put(T* p, T v) {
#if STGV_NT_STORE
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}
// Rounding to the storage type is round-to-nearest-even in every case (a double
// is rounded once, straight to FP32; FP16 / BF16 stores take FP32 values, and
// the BF16 conversion is gfx950's own, v_cvt_pk_bf16_f32).
__device__ __forceinline__ void store_as(float* p, float v) { put(p, v); }
__device__ __forceinline__ void store_as(float* p, double v) { put(p, (float)v); }
__device__ __forceinline__ void store_as(_Float16* p, float v) { put(p, (_Float16)v); }
__device__ __forceinline__ void store_as(bf16_t* p, float v) {
  put(&p->bits, __builtin_bit_cast(uint16_t, (__bf16)v));   // gfx950 converts in hardware
}

// ---------------------------------------------------------------------------
// neighbour addressing on the periodic box
//
// Per-thread offsets are 32-bit node indices (n^3 * element size < 2^32); the
// base of each population array is uniform across the wavefront, so a load is
// a scalar base plus a 32-bit vector offset and the per-node state costs no
// 64-bit address registers.
// ---------------------------------------------------------------------------
struct NodeIndex {
  uint32_t base;                // linear index x + n (y + n z)
  uint32_t xo[3], yo[3], zo[3]; // x -/0/+ 1, n (y -/0/+ 1), n^2 (z -/0/+ 1)
  __device__ __forceinline__ uint32_t at(int dx, int dy, int dz) const {
    return xo[dx + 1] + yo[dy + 1] + zo[dz + 1];
  }
};

__device__ __forceinline__ NodeIndex make_index(int x, int y, int z, int n) {
  NodeIndex ix;
  const uint32_t un = (uint32_t)n, n2 = un * un;
  ix.xo[0] = x == 0 ? un - 1 : x - 1;
  ix.xo[1] = x;
  ix.xo[2] = x == n - 1 ? 0 : x + 1;
  ix.yo[0] = un * (y == 0 ? un - 1 : y - 1);
  ix.yo[1] = un * y;
  ix.yo[2] = un * (y == n - 1 ? 0 : y + 1);
  ix.zo[0] = n2 * (z == 0 ? un - 1 : z - 1);
  ix.zo[1] = n2 * z;
  ix.zo[2] = n2 * (z == n - 1 ? 0 : z + 1);
  ix.base = ix.xo[1] + ix.yo[1] + ix.zo[1];
  return ix;
}

template <typename T>
__device__ __forceinline__ const T* at_node(const T* array, uint32_t node) {
  return (const T*)((const char*)array + node * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T* at_node(T* array, uint32_t node) {
  return (T*)((char*)array + node * (uint32_t)sizeof(T));
}

// Gather the pre-collision populations of one lattice (Q directions starting at
// array `first`) in the layout given by MODE.  The direction is a compile-time index, so
// the choice of load (cached or non-temporal) is fixed per direction.
template <int Q, typename T, int MODE, bool NTX, int I, typename C>
__device__ __forceinline__ void gather_one(C* v, const T* pop, int first, const NodeIndex& ix,
                                           int64_t stride) {
  using S = Stencil<Q>;
  constexpr bool odd = MODE == MODE_ODD;   // post-collision value of x - e_i sits in slot opp(i)
  constexpr bool nt = ((STGV_NT_LOAD_MODES >> MODE) & 1) != 0 ||
                      (odd && NTX && STGV_NT_LOAD_ODD_XALIGNED && S::ex[I] == 0);
  const uint32_t off = odd ? ix.at(-S::ex[I], -S::ey[I], -S::ez[I]) : ix.base;
  const int slot = odd ? opp(I) : I;
  v[I] = load_as<C, nt>(at_node(pop + (int64_t)(first + slot) * stride, off));
}
template <int Q, typename T, int MODE, bool NTX, typename C, int... I>
__device__ __forceinline__ void gather_seq(C* v, const T* pop, int first, const NodeIndex& ix,
                                           int64_t stride, std::integer_sequence<int, I...>) {
  (gather_one<Q, T, MODE, NTX, I>(v, pop, first, ix, stride), ...);
}
// NTX: non-temporal loads for the odd step's x-aligned directions.
template <int Q, typename T, int MODE, bool NTX = false, typename C>
__device__ __forceinline__ void gather(C* v, const T* pop, int first, const NodeIndex& ix,
                                       int64_t stride) {
  gather_seq<Q, T, MODE, NTX>(v, pop, first, ix, stride, std::make_integer_sequence<int, Q>{});
}

// Scatter post-collision populations for MODE (AB writes into `dst`), one compile-time
// direction at a time like gather.
template <int Q, typename T, int MODE, int I, typename C>
__device__ __forceinline__ void scatter_one(const C* v, T* dst, int first, const NodeIndex& ix,
                                            int64_t stride) {
  using S = Stencil<Q>;
  constexpr bool even = MODE == MODE_EVEN;   // even: kept at x, swapped into slot opp(i);
                                             // odd / AB push: natural slot i at x + e_i
  const uint32_t off = even ? ix.base : ix.at(S::ex[I], S::ey[I], S::ez[I]);
  const int slot = even ? opp(I) : I;
  store_as(at_node(dst + (int64_t)(first + slot) * stride, off), v[I]);
}
template <int Q, typename T, int MODE, typename C, int... I>
__device__ __forceinline__ void scatter_seq(const C* v, T* dst, int first, const NodeIndex& ix,
                                            int64_t stride, std::integer_sequence<int, I...>) {
  (scatter_one<Q, T, MODE, I>(v, dst, first, ix, stride), ...);
}
template <int Q, typename T, int MODE, typename C>
__device__ __forceinline__ void scatter(const C* v, T* dst, int first, const NodeIndex& ix,
                                        int64_t stride) {
  scatter_seq<Q, T, MODE>(v, dst, first, ix, stride, std::make_integer_sequence<int, Q>{});
}

// ---------------------------------------------------------------------------
// Helpers of the row-aligned odd step
// ---------------------------------------------------------------------------
template <int Q>
constexpr int x_moving() {
  int k = 0;
  for (int i = 0; i < Q; ++i) k += Stencil<Q>::ex[i] != 0;
  return k;
}

__device__ __forceinline__ _Float16 rounded(const _Float16*, float v) { return (_Float16)v; }
__device__ __forceinline__ bf16_t rounded(const bf16_t*, float v) {
  return bf16_t{__builtin_bit_cast(uint16_t, (__bf16)v)};
}
__device__ __forceinline__ void put_rounded(_Float16* p, _Float16 v) { put(p, v); }
__device__ __forceinline__ void put_rounded(bf16_t* p, bf16_t v) { put(&p->bits, v.bits); }

// ---------------------------------------------------------------------------
// Row-aligned odd step
//
// The odd step's x-shift of +-1 taken through LDS.  For each direction with e_x != 0 the
// lanes of a block row treat their LDS row as a ring of bx places: lane t loads at its
// own x from the row of (y - e_y, z - e_z) and leaves the value at place t; after a
// barrier it takes the value at place t - e_x (mod bx), i.e. that of node x - e_x.  The
// post-collision values go the other way: lane t leaves its value at place t + e_x and,
// after a barrier, stores what sits at place t at its own x.  Where a block holds whole
// rows (bx = n) the ring is the row itself.  Where it holds part of a row, the ring's
// seam is the block's edge: the lane whose own value no lane of the block needs (the
// last lane for e_x = +1, the first for e_x = -1) loads instead the node across the
// edge, x -+ bx, which its ring neighbour needs; and the lane whose place receives the
// value that belongs across the edge stores it there, at x +- bx.  Every lane does one
// load and one store per direction, every destination is written once, and the node
// that reads a location before the step is the one that writes it, as in the plain AA
// step.  All accesses are whole aligned lines except the two seam lanes', and bypass the
// caches.
// ---------------------------------------------------------------------------
template <int Q>
constexpr int x_slot(int i) {     // index of direction i among those with e_x != 0
  int k = 0;
  for (int j = 0; j < i; ++j) k += Stencil<Q>::ex[j] != 0;
  return k;
}

__device__ __forceinline__ float rounded(const float*, float v) { return v; }
__device__ __forceinline__ void put_rounded(float* p, float v) { put(p, v); }
template <bool NT> __device__ __forceinline__ float raw_load(const float* p) { return get<NT>(p); }
template <bool NT> __device__ __forceinline__ _Float16 raw_load(const _Float16* p) { return get<NT>(p); }
template <bool NT> __device__ __forceinline__ bf16_t raw_load(const bf16_t* p) { return bf16_t{get<NT>(&p->bits)}; }
template <bool NT, typename T> __device__ __forceinline__ void raw_store(T* p, T v) {
  if constexpr (NT) put_rounded(p, v);
  else if constexpr (sizeof(T) == 4) *p = v;
  else if constexpr (std::is_same_v<T, bf16_t>) p->bits = v.bits;
  else *p = v;
}

struct RowLane {
  int lid;          // thread index in the block
  int place_m;      // ring place t - 1 (mod bx) in the block's LDS rows
  int place_p;      // ring place t + 1 (mod bx)
  uint32_t x_own;   // the lane's node x
  uint32_t x_a;     // x + bx (mod n) for the first lane of the row, else x
  uint32_t x_b;     // x - bx (mod n) for the last lane of the row, else x
};

__device__ __forceinline__ RowLane make_rowlane(int x, int n) {
  const int tx = threadIdx.x, bx = blockDim.x;
  RowLane l;
  l.lid = threadIdx.y * bx + tx;
  const int row0 = l.lid - tx;
  l.place_m = row0 + (tx == 0 ? bx - 1 : tx - 1);
  l.place_p = row0 + (tx == bx - 1 ? 0 : tx + 1);
  l.x_own = (uint32_t)x;
  l.x_a = (uint32_t)(tx == 0 ? (x + bx) % n : x);
  l.x_b = (uint32_t)(tx == bx - 1 ? (x - bx + n) % n : x);
  return l;
}

template <int Q, typename T, bool NTX, int I, typename C>
__device__ __forceinline__ void row_load_one(C* v, T (*xs)[256], int k0, const T* pop, int first,
                                             const NodeIndex& ix, int64_t stride, const RowLane& l) {
  using S = Stencil<Q>;
  constexpr int ex = S::ex[I];
  // the ring's seam lane for e_x = +1 is the last, for e_x = -1 the first
  const uint32_t xl = ex > 0 ? l.x_b : (ex < 0 ? l.x_a : l.x_own);
  const T* p = at_node(pop + (int64_t)(first + opp(I)) * stride, xl + ix.yo[1 - S::ey[I]] + ix.zo[1 - S::ez[I]]);
  if constexpr (ex == 0) v[I] = load_as<C, true>(p);
  else xs[k0 + x_slot<Q>(I)][l.lid] = raw_load<NTX>(p);
}
template <int Q, typename T, int I, typename C>
__device__ __forceinline__ void row_pick_one(C* v, const T (*xs)[256], int k0, const RowLane& l) {
  using S = Stencil<Q>;
  if constexpr (S::ex[I] != 0) v[I] = load_as<C>(&xs[k0 + x_slot<Q>(I)][S::ex[I] > 0 ? l.place_m : l.place_p]);
}
template <int Q, typename T, int I, typename C>
__device__ __forceinline__ void row_put_one(const C* v, T (*xs)[256], int k0, const RowLane& l) {
  using S = Stencil<Q>;
  if constexpr (S::ex[I] != 0)
    xs[k0 + x_slot<Q>(I)][S::ex[I] > 0 ? l.place_p : l.place_m] = rounded((const T*)nullptr, v[I]);
}
template <int Q, typename T, bool NTX, int I, typename C>
__device__ __forceinline__ void row_store_one(const C* v, const T (*xs)[256], int k0, T* dst, int first,
                                              const NodeIndex& ix, int64_t stride, const RowLane& l) {
  using S = Stencil<Q>;
  constexpr int ex = S::ex[I];
  // the place that receives the value belonging across the seam: the first lane's for
  // e_x = +1, the last lane's for e_x = -1
  const uint32_t xd = ex > 0 ? l.x_a : (ex < 0 ? l.x_b : l.x_own);
  T* p = at_node(dst + (int64_t)(first + I) * stride, xd + ix.yo[1 + S::ey[I]] + ix.zo[1 + S::ez[I]]);
  if constexpr (ex == 0) store_as(p, v[I]);
  else raw_store<NTX>(p, xs[k0 + x_slot<Q>(I)][l.lid]);
}

template <int Q, typename T, bool NTX, typename C, int... I>
__device__ __forceinline__ void row_load(C* v, T (*xs)[256], int k0, const T* pop, int first,
                                         const NodeIndex& ix, int64_t stride, const RowLane& l,
                                         std::integer_sequence<int, I...>) {
  (row_load_one<Q, T, NTX, I>(v, xs, k0, pop, first, ix, stride, l), ...);
}
template <int Q, typename T, typename C, int... I>
__device__ __forceinline__ void row_pick(C* v, const T (*xs)[256], int k0, const RowLane& l,
                                         std::integer_sequence<int, I...>) {
  (row_pick_one<Q, T, I>(v, xs, k0, l), ...);
}
template <int Q, typename T, typename C, int... I>
__device__ __forceinline__ void row_put(const C* v, T (*xs)[256], int k0, const RowLane& l,
                                        std::integer_sequence<int, I...>) {
  (row_put_one<Q, T, I>(v, xs, k0, l), ...);
}
template <int Q, typename T, bool NTX, typename C, int... I>
__device__ __forceinline__ void row_store(const C* v, const T (*xs)[256], int k0, T* dst, int first,
                                          const NodeIndex& ix, int64_t stride, const RowLane& l,
                                          std::integer_sequence<int, I...>) {
  (row_store_one<Q, T, NTX, I>(v, xs, k0, dst, first, ix, stride, l), ...);
}

// ---------------------------------------------------------------------------
// node-local physics
// ---------------------------------------------------------------------------
// Moments over a lattice whose directions come in opposite pairs (i, i + 1):
// sum a_i = a_0 + sum_pairs (a_i + a_{i+1}) and
// sum e_i a_i = sum_pairs e_i (a_i - a_{i+1}); pairing first keeps the
// rounding of the sums at the scale of the moments rather than of the
// individual (larger, velocity-carrying) deviations.
template <int Q, typename C>
__device__ __forceinline__ void pair_moments(const C* a, C& m0, C& mx, C& my, C& mz) {
  using S = Stencil<Q>;
  C s = a[0], x = C(0), y = C(0), z = C(0);
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    s += a[i] + a[i + 1];
    const C dlt = a[i] - a[i + 1];
    if (S::ex[i] != 0) x += S::ex[i] > 0 ? dlt : -dlt;
    if (S::ey[i] != 0) y += S::ey[i] > 0 ? dlt : -dlt;
    if (S::ez[i] != 0) z += S::ez[i] > 0 ? dlt : -dlt;
  }
  m0 = s; mx = x; my = y; mz = z;
}

template <int Q, typename C>
__device__ __forceinline__ C pair_sum(const C* a) {
  C s = a[0];
#pragma unroll
  for (int i = 1; i < Q; i += 2) s += a[i] + a[i + 1];
  return s;
}

__device__ __forceinline__ float fma_c(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_c(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename C>
__device__ __forceinline__ C dot_e(int ex, int ey, int ez, C vx, C vy, C vz) {
  C eu = C(0);
  if (ex != 0) eu += ex > 0 ? vx : -vx;
  if (ey != 0) eu += ey > 0 ? vy : -vy;
  if (ez != 0) eu += ez > 0 ? vz : -vz;
  return eu;
}

template <typename C>
struct NodeMacro {
  C drho;       // rho - 1
  C rho;
  C jx, jy, jz; // sum e f
  C dsig;       // sum g - 1
  C rho_p;      // rho'
  C s;          // -u'_z (d rho_b/dz)_LU
  C Fz;         // -G rho'
  C ux, uy, uz; // physical velocity, Eq. (7)
  C vx, vy, vz; // velocity of the momentum equilibrium the collision relaxes to
};

// The node's moments from its population sums: drho = sum f - 1 (deviations),
// j = sum e f, dsig = sum g - 1.
template <int FORCE, typename C>
__device__ __forceinline__ void macro_from_sums(C drho, C jx, C jy, C jz, C dsig, const PhysConsts& c,
                                                NodeMacro<C>& m) {
  const C rho = C(1) + drho;                  // Eq. (6), rho_0 = 1 plus deviation
  const C inv_rho = C(1) / rho;
  const C upz = jz * inv_rho;
  const C s = -upz * (C)c.beta;               // Eqs. (12)-(13), bare u_z
  const C rho_p = dsig + C(0.5) * s;          // Eqs. (16)-(17): sum g + S/2 - rho_0
  const C Fz = -(C)c.G * rho_p;               // Eq. (18)
  m.drho = drho; m.rho = rho; m.jx = jx; m.jy = jy; m.jz = jz;
  m.dsig = dsig; m.rho_p = rho_p; m.s = s; m.Fz = Fz;
  m.ux = jx * inv_rho;
  m.uy = jy * inv_rho;
  m.uz = upz + C(0.5) * Fz * inv_rho;         // Eq. (7)
  m.vx = m.ux;
  m.vy = m.uy;
  if (FORCE == FORCE_SHIFT) m.vz = upz + (C)c.tau_f * Fz * inv_rho;  // Shan-Chen shift, Eq. (10) (tau F / rho)
  else if (FORCE == FORCE_EDM) m.vz = upz;                            // EDM relaxes to f^eq(u')
  else m.vz = m.uz;                                                   // Guo, HCZ: u of Eq. (7)
}

template <int QF, int QG, int FORCE, typename C>
__device__ __forceinline__ void node_macro(const C* f, const C* g, const PhysConsts& c,
                                           NodeMacro<C>& m) {
  C drho, jx, jy, jz;
  pair_moments<QF>(f, drho, jx, jy, jz);
  const C dsig = pair_sum<QG>(g);
  macro_from_sums<FORCE>(drho, jx, jy, jz, dsig, c, m);
}

template <int QF, int QG, int FORCE, typename C>
struct Collision {
  using SF = Stencil<QF>;
  using SG = Stencil<QG>;
  static constexpr C icf = C(1.0 / SF::cs2);
  static constexpr C icg = C(1.0 / SG::cs2);
  const NodeMacro<C>& m;
  C vx, vy, vz, usq, omega_f, omega_g, tau_f, base_f, conc, base_g;
  C tx, ty, tz;   // velocity of the scalar equilibrium

  __device__ __forceinline__ Collision(const PhysConsts& c, const NodeMacro<C>& mm) : m(mm) {
    vx = m.vx; vy = m.vy; vz = m.vz;
    usq = vx * vx + vy * vy + vz * vz;
    omega_f = (C)c.omega_f; omega_g = (C)c.omega_g; tau_f = (C)c.tau_f;
    base_f = m.drho - C(0.5) * icf * m.rho * usq;
    conc = C(1) + m.rho_p;
    // the scalar equilibrium moves with the velocity of the momentum equilibrium,
    // except under EDM, whose fluid velocity is u of Eq. (7)
    if (FORCE == FORCE_EDM) {
      tx = m.ux; ty = m.uy; tz = m.uz;
      base_g = -C(0.5) * icg * (tx * tx + ty * ty + tz * tz);
    } else {
      tx = vx; ty = vy; tz = vz;
      base_g = -C(0.5) * icg * usq;
    }
  }
  // momentum lattice: df_eq = w [drho + rho (xi + xi^2/2 - u^2/(2 c^2))], xi = e.u / c^2
  __device__ __forceinline__ C feq(int i) const {
    const C xi = icf * dot_e(SF::ex[i], SF::ey[i], SF::ez[i], vx, vy, vz);
    return C(SF::w[i]) * (base_f + m.rho * xi * (C(1) + C(0.5) * xi));
  }
  // scalar lattice: dg_eq = w [rho' + (1 + rho') (xi + xi^2/2 - u^2/(2 c^2))]
  __device__ __forceinline__ C geq(int j) const {
    const C xi = icg * dot_e(SG::ex[j], SG::ey[j], SG::ez[j], tx, ty, tz);
    return C(SG::w[j]) * (m.rho_p + conc * (base_g + xi * (C(1) + C(0.5) * xi)));
  }
  // the same equilibria from e.v_eq (f) or e.v_theta (g) and the weight w
  __device__ __forceinline__ C feq_of(C eu, C w) const {
    const C xi = icf * eu;
    return w * (base_f + m.rho * xi * (C(1) + C(0.5) * xi));
  }
  __device__ __forceinline__ C geq_of(C eu, C w) const {
    const C xi = icg * eu;
    return w * (m.rho_p + conc * (base_g + xi * (C(1) + C(0.5) * xi)));
  }
  // f[i] <- d_i = f_i^eq - f_i and g[j] <- h_j = g_j^eq - g_j
  __device__ __forceinline__ void relaxation_increments(C* f, C* g) const {
#pragma unroll
    for (int i = 0; i < QF; ++i) f[i] = feq(i) - f[i];
#pragma unroll
    for (int j = 0; j < QG; ++j) g[j] = geq(j) - g[j];
  }
  // From the increments to the post-collision populations.
  //   f*_i = f_i + omega (d_i - p_i) + G_i = f_i^eq + [(omega - 1) d_i - omega p_i + G_i]
  // with p_i = w_i (r_0 + e_i . r / c^2) the projection of the moment residual
  // and G_i the force term of the scheme; the bracket is formed with fused
  // multiply-adds so the small terms (p_i, G_i ~ 1e-12) shift its single rounding
  // instead of deciding ties of the final sum: ties broken by a term whose sign
  // follows e_i . F would bias the node mass a little every step.
  //   Guo: G_i = (1 - omega/2) w [(e_z - u_z) / c^2 + (e.u) e_z / c^4] Fz;
  //   EDM: G_i = f^eq_i(u' + F/rho) - f^eq_i(u'), which for the second-order
  //        equilibrium is exactly w [(e_z - u_z) / c^2 + (e.u) e_z / c^4] Fz with
  //        u = u' + F/(2 rho): the Guo bracket without the factor (1 - omega/2);
  //   HCZ: G_i = (1 - omega/2) (e_z - u_z) Fz / (rho c^2) f^eq_i(u).
  // The increments carry the momentum rho u_eq - j: F/2 (Guo, HCZ), tau F
  // (shift), 0 (EDM).
  __device__ __forceinline__ void finish(C* f, C* g) const {
    C r0, rx, ry, rz;
    pair_moments<QF>(f, r0, rx, ry, rz);
    if (FORCE == FORCE_GUO || FORCE == FORCE_HCZ) rz -= C(0.5) * m.Fz;
    else if (FORCE == FORCE_SHIFT) rz -= tau_f * m.Fz;
    const C half_c = (C(1) - C(0.5) * omega_f) * m.Fz;
    const C bracket_c = (FORCE == FORCE_GUO) ? half_c : m.Fz;          // Guo / EDM
    const C hcz_c = icf * half_c / m.rho;                               // HCZ
#pragma unroll
    for (int i = 0; i < QF; ++i) {
      const C p = C(SF::w[i]) * (r0 + icf * dot_e(SF::ex[i], SF::ey[i], SF::ez[i], rx, ry, rz));
      C small = -omega_f * p;
      if (FORCE == FORCE_GUO || FORCE == FORCE_EDM) {
        const C eu = dot_e(SF::ex[i], SF::ey[i], SF::ez[i], m.ux, m.uy, m.uz);
        C br = -icf * m.uz;
        if (SF::ez[i] != 0) br += SF::ez[i] > 0 ? icf * (C(1) + icf * eu) : -icf * (C(1) + icf * eu);
        small = fma_c(-omega_f, p, C(SF::w[i]) * bracket_c * br);
      } else if (FORCE == FORCE_HCZ) {
        const C ez_u = C(SF::ez[i]) - m.uz;
        small = fma_c(-omega_f, p, hcz_c * ez_u * (C(SF::w[i]) + feq(i)));
      }
      f[i] = feq(i) + fma_c(omega_f - C(1), f[i], small);
    }
    const C r0g = pair_sum<QG>(g) - C(0.5) * m.s;
    const C src = (C(1) - C(0.5) * omega_g) * m.s - omega_g * r0g;
#pragma unroll
    for (int j = 0; j < QG; ++j) g[j] = geq(j) + fma_c(omega_g - C(1), g[j], C(SG::w[j]) * src);
  }
};

// BGK collision of both lattices in place (Eqs. (5), (8), (9), (11), (14), (15)).
//
// The relaxation increment d_i = f_i^eq - f_i has, in exact arithmetic, zeroth
// moment 0 and first moment rho u_eq - j (= F/2 for Guo, tau_f F for the shift);
// the scalar increment has zeroth moment S/2.  Rounding breaks those identities
// at the level of the velocity-carrying deviations, which at tau ~ 1/2 acts
// as a spurious local mass / momentum source every step.  The increments are
// therefore projected back onto their exact conserved moments
// (d_i -= w_i (r_0 + e_i . r / c_s^2) with r the moment residual), which is the
// identity in exact arithmetic.
template <int QF, int QG, int FORCE, typename C>
__device__ __forceinline__ void node_collide(C* f, C* g, const PhysConsts& c,
                                             const NodeMacro<C>& m) {
  const Collision<QF, QG, FORCE, C> col(c, m);
  col.relaxation_increments(f, g);
  col.finish(f, g);
}

// ---------------------------------------------------------------------------
// The time step's collision in split arithmetic
//
// Why: the scalar lattice carries rho_0 + rho' = 1 + rho', so its equilibrium
// flux (1 + rho') u moves the background density with the velocity, and an
// error of one FP32 ulp in u (or in the velocity-linear equilibrium term
// 3 w e.u, the largest part of every deviation) moves background mass between
// nodes: rho' (~1e-3 - 1e-2) sees it at ~1e-5 relative within 100 steps.  The
// density deviation is hit the same way through the momentum lattice's linear
// term.  So the step keeps those two quantities exact or nearly so, in FP32:
//
// * every population is split as df = hi + lo with hi on the grid of 2^-23
//   (`grid_split`); sums of grid values below 2 in magnitude are exact in FP32,
//   so drho = sum df, j = sum e df and sum dg are held as an exact grid part plus
//   a small lo sum whose own rounding is ~2^-24 of 2^-23 (when the split of N^2
//   puts most of it in the background gradient, rho' reaches 0.1 - 1 and an FP32
//   rounding of sum dg or of rho' itself is ~1e-8 per node and step);
// * the stratification source s = -beta u'_z is an exact product pair, and rho'
//   = sum dg + s/2 a grid part plus a remainder;
// * the velocities are jh + a small lo part (u' = j/rho = j - j drho/rho:
//   no rounding of 1 + drho enters it);
// * the linear equilibrium terms w (drho + 3 e.J) and w (rho' + 3 e.(1 + rho')t)
//   are formed from grid parts (exact sums), an error-free product with the
//   weight (the fused multiply-add residual) and small remainders; the
//   quadratic terms, two orders smaller, are plain FP32.  The weight's own FP32
//   residual (w - fl(w), ~1e-8 relative) multiplies the whole equilibrium:
//   without it the sum of the equilibria misses rho' (or drho) by
//   ~1e-8 (3/2) u^2 at every node and step, always with the same sign, a
//   steady drift of the scalar and momentum masses.
// The increment d_i = f^eq_i - f_i is thus rounded at the scale of d rather than
// of f, and the population is updated once:
// f*_i = f_i + (omega d_i + G_i).  The only rounding at the scale of the
// population is the final one, the one FP32 storage makes anyway.
// ---------------------------------------------------------------------------
// x = hi + lo exactly, hi on the grid of ulp(1.5): 2^-23 in FP32, 2^-52 in FP64
// (exact for |x| < 0.5; beyond it hi + lo still equals x, on a coarser grid).
template <typename C>
__device__ __forceinline__ void grid_split(C x, C& hi, C& lo) {
  const C k = C(1.5);
  hi = (x + k) - k;
  lo = x - hi;
}

// e . v for a lattice direction, summed in a fixed order (x, y, z); -0 is the
// neutral start so that a single term is passed through unchanged.
template <typename C>
__device__ __forceinline__ C edot(int ex, int ey, int ez, const C* v) {
  C r = C(-0.0);
  if (ex != 0) r += ex > 0 ? v[0] : -v[0];
  if (ey != 0) r += ey > 0 ? v[1] : -v[1];
  if (ez != 0) r += ez > 0 ? v[2] : -v[2];
  return r;
}

// Zeroth moment m0 = sum df and momentum j = sum e df, each as a grid part (an exact
// sum) plus the sum of the small remainders.
template <int Q, typename C>
__device__ __forceinline__ void split_moments(const C* a, C& m0h, C& m0l, C* jh, C* jl) {
  using S = Stencil<Q>;
  grid_split(a[0], m0h, m0l);
#pragma unroll
  for (int k = 0; k < 3; ++k) { jh[k] = C(-0.0); jl[k] = C(-0.0); }
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    C h0, l0, h1, l1;
    grid_split(a[i], h0, l0);
    grid_split(a[i + 1], h1, l1);
    m0h += h0 + h1;
    m0l += l0 + l1;
    const C dh = h0 - h1, dl = l0 - l1;    // e_{i+1} = -e_i
    const int e[3] = {S::ex[i], S::ey[i], S::ez[i]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (e[k] == 0) continue;
      jh[k] += e[k] > 0 ? dh : -dh;
      jl[k] += e[k] > 0 ? dl : -dl;
    }
  }
}

// Zeroth moment only, as grid part plus remainder.
template <int Q, typename C>
__device__ __forceinline__ void split_sum(const C* a, C& mh, C& ml) {
  grid_split(a[0], mh, ml);
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    C h0, l0, h1, l1;
    grid_split(a[i], h0, l0);
    grid_split(a[i + 1], h1, l1);
    mh += h0 + h1;
    ml += l0 + l1;
  }
}

template <typename C>
struct StepMacro {
  C drho, rho, inv, dsig, rho_p, s, Fz;   // FP32 values
  C dr_h, dr_l;  // drho = dr_h + dr_l: grid part (exact sum) and remainder
  C rp_h, rp_l;  // rho' likewise (sum g - 1 + s/2 with s as an exact product pair)
  C jh[3];      // grid part of j = sum e df, shared by every velocity below
  C j[3];       // j (FP32 value), for the diagnostics
  C jeq_l[3];   // rho v_eq - jh: the equilibrium momentum's remainder (j + k F e_z)
  C u[3];       // physical velocity, Eq. (7) (FP32 value)
  C ul[3];      // u - jh
  C v[3];       // velocity of the momentum equilibrium (FP32 value)
  C t[3];       // velocity of the scalar equilibrium (FP32 value)
  C fl[3];      // (1 + rho') t - jh: remainder of the scalar equilibrium's flux
};

// EXACT: the moment sums in split form (FP32 storage).  With 2-byte storage the store
// rounds each deviation at 2^-11 (FP16) or 2^-8 (BF16) of itself, far above anything the
// exact sums save, so those steps take plain pair sums (the remainders are then zero)
// and keep only the cheap error-free parts (the fused increments, the source pair).
template <int QF, int QG, int FORCE, bool EXACT, typename C>
__device__ __forceinline__ void step_macro(const C* f, const C* g, const PhysConsts& c,
                                           StepMacro<C>& m) {
  C jl[3];
  C sg_h, sg_l;
  if constexpr (EXACT) {
    split_moments<QF>(f, m.dr_h, m.dr_l, m.jh, jl);
    split_sum<QG>(g, sg_h, sg_l);
  } else {
    pair_moments<QF>(f, m.dr_h, m.jh[0], m.jh[1], m.jh[2]);
    m.dr_l = C(0);
    jl[0] = jl[1] = jl[2] = C(0);
    sg_h = pair_sum<QG>(g);
    sg_l = C(0);
  }
  m.drho = m.dr_h + m.dr_l;
  m.dsig = sg_h + sg_l;
  m.rho = C(1) + m.drho;                          // Eq. (6)
  m.inv = C(1) / m.rho;
  const C q = m.drho * m.inv;                     // u' = j / rho = j - j drho / rho
  C upl[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) upl[k] = jl[k] - (m.jh[k] + jl[k]) * q;
  // Eqs. (12)-(13), bare u_z: s = -beta u'_z = s_h + s_l, s_h = fl(-beta jh_z) and the
  // product's exact residual carried in s_l
  const C beta = (C)c.beta;
  const C s_h = -beta * m.jh[2];
  const C s_l = fma_c(-beta, upl[2], fma_c(-beta, m.jh[2], -s_h));
  m.s = s_h + s_l;
  // Eqs. (16)-(17): rho' = sum g - 1 + s/2, grid part exact
  m.rp_h = sg_h;
  m.rp_l = fma_c(C(0.5), s_h, fma_c(C(0.5), s_l, sg_l));
  m.rho_p = m.rp_h + m.rp_l;
  m.Fz = -(C)c.G * m.rho_p;                       // Eq. (18)
  const C fz_inv = m.Fz * m.inv;
  m.ul[0] = upl[0];
  m.ul[1] = upl[1];
  m.ul[2] = upl[2] + C(0.5) * fz_inv;             // Eq. (7)
  C vl[3] = {upl[0], upl[1], upl[2]};             // EDM relaxes to f^eq(u')
  m.jeq_l[0] = jl[0];
  m.jeq_l[1] = jl[1];
  m.jeq_l[2] = jl[2];
  if (FORCE == FORCE_SHIFT) {                     // Eq. (10), shift tau F / rho
    vl[2] = upl[2] + (C)c.tau_f * fz_inv;
    m.jeq_l[2] = jl[2] + (C)c.tau_f * m.Fz;
  } else if (FORCE == FORCE_GUO || FORCE == FORCE_HCZ) {
    vl[2] = m.ul[2];
    m.jeq_l[2] = jl[2] + C(0.5) * m.Fz;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    m.j[k] = m.jh[k] + jl[k];
    m.u[k] = m.jh[k] + m.ul[k];
    m.v[k] = m.jh[k] + vl[k];
    // the scalar equilibrium moves with the momentum equilibrium's velocity,
    // except under EDM, whose fluid velocity is u of Eq. (7)
    const C tl = FORCE == FORCE_EDM ? m.ul[k] : vl[k];
    m.t[k] = m.jh[k] + tl;
    m.fl[k] = tl + m.rho_p * m.t[k];
  }
}

// The relaxation increment w (y + rq) - p of one population p, y the exact grid part.
// EXACT: w y = ph + pe exactly (the fused multiply-add residual), ph - p exact, and the
// remainders, the residual and the weight's FP32 residual on all of it summed at the
// increment's scale, so the only rounding of that size is the last one.  (A chain of
// three fused multiply-adds, fma(wl, y + rq, fma(w, rq, fma(w, y, -p))), rounds three
// times at that size and measurably loses accuracy at tau ~ 1/2.)  Otherwise the chain,
// for 2-byte storage whose store rounding is far larger.
template <bool EXACT, typename C>
__device__ __forceinline__ C increment(C w, C wl, C y, C rq, C p) {
  if constexpr (EXACT) {
    const C ph = w * y;
    C pe = fma_c(w, y, -ph);
    pe = fma_c(wl, y + rq, pe);
    return (ph - p) + fma_c(w, rq, pe);
  } else {
    return fma_c(wl, y + rq, fma_c(w, rq, fma_c(w, y, -p)));
  }
}

// Post-collision populations of both lattices, in place (Eqs. (5), (8)-(11),
// (14)-(15) with the forcing scheme's term).
template <int QF, int QG, int FORCE, bool EXACT, typename C>
__device__ __forceinline__ void step_collide(C* f, C* g, const PhysConsts& c, const StepMacro<C>& m) {
  using SF = Stencil<QF>;
  using SG = Stencil<QG>;
  constexpr C icf = C(1.0 / SF::cs2);
  constexpr C icg = C(1.0 / SG::cs2);
  const C omega_f = (C)c.omega_f, omega_g = (C)c.omega_g;
  const C dr_h = m.dr_h, dr_l = m.dr_l;
  const C vsq = m.v[0] * m.v[0] + m.v[1] * m.v[1] + m.v[2] * m.v[2];
  const C qb_f = -C(0.5) * icf * vsq;
  const C half_c = (C(1) - C(0.5) * omega_f) * m.Fz;
  const C bracket_c = (FORCE == FORCE_GUO) ? half_c : m.Fz;          // Guo / EDM
  const C hcz_c = icf * half_c * m.inv;                               // HCZ
  // momentum lattice, by opposite pairs (the rest direction is its own pair)
#pragma unroll
  for (int i = 0; i < QF; i += (i == 0 ? 1 : 2)) {
    const int ex = SF::ex[i], ey = SF::ey[i], ez = SF::ez[i];
    const C w = C(SF::w[i]);
    const C wl = C(SF::w[i] - (double)w);              // the weight's FP32 residual
    const C ejh = edot(ex, ey, ez, m.jh);
    const C ejl = edot(ex, ey, ez, m.jeq_l);
    const C xi = icf * edot(ex, ey, ez, m.v);
    const C qv = m.rho * fma_c(C(0.5) * xi, xi, qb_f);  // rho (xi^2/2 - v^2/(2c^2)), even in e
    const C eu = edot(ex, ey, ez, m.u);
#pragma unroll
    for (int sgn = 1; sgn >= (i == 0 ? 1 : -1); sgn -= 2) {
      const int k = sgn > 0 ? i : i + 1;
      const C y = fma_c(C(sgn) * icf, ejh, dr_h);          // drho + 3 e.J, grid parts: exact
      const C r = fma_c(C(sgn) * icf, ejl, dr_l);          // remainders
      const C rq = r + qv;
      const C d = increment<EXACT>(w, wl, y, rq, f[k]);    // f^eq - f
      C force = C(0);
      if (FORCE == FORCE_GUO || FORCE == FORCE_EDM) {
        //   Guo: G_i = (1 - omega/2) w [(e_z - u_z) / c^2 + (e.u) e_z / c^4] Fz;
        //   EDM: G_i = f^eq_i(u' + F/rho) - f^eq_i(u'), for the second-order
        //        equilibrium exactly w [(e_z - u_z) / c^2 + (e.u) e_z / c^4] Fz
        //        with u = u' + F/(2 rho): the Guo bracket without (1 - omega/2)
        C br = -icf * m.u[2];
        const int ezk = sgn * ez;
        if (ezk != 0) {
          const C t = icf * fma_c(C(sgn) * icf, eu, C(1));
          br += ezk > 0 ? t : -t;
        }
        force = w * bracket_c * br;
      } else if (FORCE == FORCE_HCZ) {
        //   HCZ: G_i = (1 - omega/2) (e_z - u_z) Fz / (rho c^2) f^eq_i(u)
        force = hcz_c * (C(sgn * ez) - m.u[2]) * fma_c(w, y + rq, w);
      }
      f[k] = f[k] + fma_c(omega_f, d, force);
    }
  }
  // scalar lattice: g^eq_j = w [rho' + 3 e.(1 + rho') t + (1 + rho')(xi^2/2 - t^2/(2c^2))]
  const C rp_h = m.rp_h, rp_l = m.rp_l;
  const C conc = C(1) + m.rho_p;
  const C tsq = (FORCE == FORCE_EDM) ? m.t[0] * m.t[0] + m.t[1] * m.t[1] + m.t[2] * m.t[2] : vsq;
  const C qb_g = -C(0.5) * icg * tsq;
  const C src = (C(1) - C(0.5) * omega_g) * m.s;       // (1 - 1/(2 tau_g)) S / w
#pragma unroll
  for (int j = 0; j < QG; j += (j == 0 ? 1 : 2)) {
    const int ex = SG::ex[j], ey = SG::ey[j], ez = SG::ez[j];
    const C w = C(SG::w[j]);
    const C wl = C(SG::w[j] - (double)w);
    const C ejh = edot(ex, ey, ez, m.jh);
    const C ejl = edot(ex, ey, ez, m.fl);
    const C xi = icg * edot(ex, ey, ez, m.t);
    const C qv = conc * fma_c(C(0.5) * xi, xi, qb_g);
    const C ws = w * src;
#pragma unroll
    for (int sgn = 1; sgn >= (j == 0 ? 1 : -1); sgn -= 2) {
      const int k = sgn > 0 ? j : j + 1;
      const C y = fma_c(C(sgn) * icg, ejh, rp_h);
      const C r = fma_c(C(sgn) * icg, ejl, rp_l);
      const C rq = r + qv;
      const C h = increment<EXACT>(w, wl, y, rq, g[k]);    // g^eq - g
      g[k] = g[k] + fma_c(omega_g, h, ws);
    }
  }
}

// The step's moments in the form the diagnostics take.
template <typename C>
__device__ __forceinline__ NodeMacro<C> diag_macro(const StepMacro<C>& s) {
  NodeMacro<C> m;
  m.drho = s.drho; m.rho = s.rho; m.dsig = s.dsig; m.rho_p = s.rho_p; m.s = s.s; m.Fz = s.Fz;
  m.jx = s.j[0]; m.jy = s.j[1]; m.jz = s.j[2];
  m.ux = s.u[0]; m.uy = s.u[1]; m.uz = s.u[2];
  m.vx = s.v[0]; m.vy = s.v[1]; m.vz = s.v[2];
  return m;
}

// Diagnostic outputs of one node: the five fields (rho - 1, u, rho') and its
// contributions to the block partials.
template <typename C>
__device__ __forceinline__ void write_fields(const NodeMacro<C>& m, float* __restrict__ fields, uint32_t node,
                                             int64_t n3) {
  fields[node] = (float)m.drho;
  fields[n3 + node] = (float)m.ux;
  fields[2 * n3 + node] = (float)m.uy;
  fields[3 * n3 + node] = (float)m.uz;
  fields[4 * n3 + node] = (float)m.rho_p;
}

template <typename C>
__device__ __forceinline__ void node_partials(const NodeMacro<C>& m, const PhysConsts& c, double* acc) {
  const C u2 = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
  const C ep = (C)c.g_over_n * m.rho_p;
  acc[P_EK] = 0.5 * (double)u2;
  acc[P_EP] = 0.5 * (double)(ep * ep);
  acc[P_DRHO] = (double)m.drho;
  acc[P_DSIG] = (double)m.dsig;
  acc[P_MX] = (double)m.jx;
  acc[P_MY] = (double)m.jy;
  acc[P_MZ] = (double)(m.jz + C(0.5) * m.Fz);
  acc[P_UMAX2] = (double)u2;
  acc[P_NONFINITE] = (isfinite(m.rho) && isfinite(u2) && isfinite(m.rho_p)) ? 0.0 : 1.0;
}

// ---------------------------------------------------------------------------
// block reductions (fixed order: deterministic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Reduce NV per-thread values over the block and write them to out[0..NV).
// Bit k of MAXMASK selects a maximum instead of a sum for entry k.  Every
// thread of the block must call this (masked-out threads pass neutral values);
// the block size must be a multiple of 64 and at most 1024.
template <int NV, unsigned MAXMASK>
__device__ __forceinline__ void block_reduce_store(const double* vals, double* __restrict__ out) {
  __shared__ double lds[16][NV];
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthreads = blockDim.x * blockDim.y * blockDim.z;
  const int lane = tid & 63, wid = tid >> 6, nw = nthreads >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double r = ((MAXMASK >> k) & 1u) ? wave_max(vals[k]) : wave_sum(vals[k]);
    if (lane == 0) lds[wid][k] = r;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double acc = lds[0][k];
      for (int w = 1; w < nw; ++w)
        acc = ((MAXMASK >> k) & 1u) ? fmax(acc, lds[w][k]) : acc + lds[w][k];
      out[k] = acc;
    }
  }
}

}  // namespace stgv
