// Learned per-node correction of a coarse run: moment basis, network layout and
// the BF16 MFMA layers (gfx950).
//
// Moment basis: monomials e_x^a e_y^b e_z^c, exponents in {0, 1, 2}; all 27 for
// the D3Q27 momentum lattice, the 19 with at least one zero exponent for the
// D3Q19 scalar lattice.  Slot order: conserved moments first ((000), (100),
// (010), (001) for f; (000) for g), the others in lexicographic order.  The
// network maps the 47 node features [M (f - f^eq), M (g - g^eq), rho'] to
// corrections of the 41 non-conserved moments; the post-collision populations
// gain M^-1 [0, dm].  Network 47 -> 64 -> 64 -> 41, tanh hidden layers, inputs
// normalised as (x - mean) * iscale, outputs scaled by y_scale.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"
#include "stencil.hpp"

namespace stgv {
namespace mlp {

constexpr int N_IN = 47, N_HID = 64, N_OUT = 41;
constexpr int K_IN = 48;               // input width padded to the MFMA k-step (16)
constexpr int M_OUT = 64;              // output rows padded to two 32-row tiles
constexpr int NCF = 4, NCG = 1;        // conserved slots of f and g
constexpr int N_PARAMS = N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_OUT * N_HID + N_OUT;

// ---------------------------------------------------------------------------
// moment basis
// ---------------------------------------------------------------------------
struct Exps { int a[27], b[27], c[27]; int n; };

constexpr Exps make_exps(bool full) {
  Exps e{};
  const int head[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  const int nhead = full ? 4 : 1;
  int k = 0;
  for (int h = 0; h < nhead; ++h) { e.a[k] = head[h][0]; e.b[k] = head[h][1]; e.c[k] = head[h][2]; ++k; }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        if (!full && a != 0 && b != 0 && c != 0) continue;
        bool is_head = false;
        for (int h = 0; h < nhead; ++h)
          if (head[h][0] == a && head[h][1] == b && head[h][2] == c) is_head = true;
        if (is_head) continue;
        e.a[k] = a; e.b[k] = b; e.c[k] = c; ++k;
      }
  e.n = k;
  return e;
}
constexpr Exps EXP_F = make_exps(true);
constexpr Exps EXP_G = make_exps(false);

constexpr int ipow(int v, int p) { return p == 0 ? 1 : (p == 1 ? v : v * v); }

template <int Q>
constexpr int mom_entry(int k, int i) {   // M[k][i]
  using S = Stencil<Q>;
  const Exps& E = (Q == 27) ? EXP_F : EXP_G;
  return ipow(S::ex[i], E.a[k]) * ipow(S::ey[i], E.b[k]) * ipow(S::ez[i], E.c[k]);
}

// Exact inverse by Gauss-Jordan elimination on rationals (compile time).
struct Frac { long long n, d; };
constexpr long long gcd_ll(long long a, long long b) {
  a = a < 0 ? -a : a; b = b < 0 ? -b : b;
  while (b) { long long t = a % b; a = b; b = t; }
  return a == 0 ? 1 : a;
}
constexpr Frac mk(long long n, long long d) {
  if (d < 0) { n = -n; d = -d; }
  const long long g = gcd_ll(n, d);
  return Frac{n / g, d / g};
}
constexpr Frac fsub(Frac x, Frac y) { return mk(x.n * y.d - y.n * x.d, x.d * y.d); }
constexpr Frac fmul(Frac x, Frac y) { return mk(x.n * y.n, x.d * y.d); }
constexpr Frac fdiv(Frac x, Frac y) { return mk(x.n * y.d, x.d * y.n); }

template <int Q>
struct Inverse { float v[Q][Q]; };

template <int Q>
struct InverseFrac { Frac v[Q][Q]; };

template <int Q>
constexpr InverseFrac<Q> make_inverse_frac() {
  Frac A[Q][2 * Q] = {};
  for (int r = 0; r < Q; ++r)
    for (int c = 0; c < 2 * Q; ++c)
      A[r][c] = c < Q ? Frac{mom_entry<Q>(r, c), 1} : Frac{r == c - Q ? 1 : 0, 1};
  for (int col = 0; col < Q; ++col) {
    int piv = col;
    while (A[piv][col].n == 0) ++piv;
    for (int c = 0; c < 2 * Q; ++c) { const Frac t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t; }
    const Frac pv = A[col][col];
    for (int c = 0; c < 2 * Q; ++c) A[col][c] = fdiv(A[col][c], pv);
    for (int r = 0; r < Q; ++r) {
      if (r == col || A[r][col].n == 0) continue;
      const Frac fac = A[r][col];
      for (int c = 0; c < 2 * Q; ++c) A[r][c] = fsub(A[r][c], fmul(fac, A[col][c]));
    }
  }
  InverseFrac<Q> out{};
  for (int r = 0; r < Q; ++r)
    for (int c = 0; c < Q; ++c) out.v[r][c] = A[r][Q + c];
  return out;
}
constexpr InverseFrac<27> MINV_F_FRAC = make_inverse_frac<27>();
constexpr InverseFrac<19> MINV_G_FRAC = make_inverse_frac<19>();

template <int Q>
constexpr Frac inverse_entry(int r, int c) { return Q == 27 ? MINV_F_FRAC.v[r][c] : MINV_G_FRAC.v[r][c]; }

template <int Q>
constexpr Inverse<Q> make_inverse() {
  Inverse<Q> out{};
  for (int r = 0; r < Q; ++r)
    for (int c = 0; c < Q; ++c) out.v[r][c] = (float)inverse_entry<Q>(r, c).n / (float)inverse_entry<Q>(r, c).d;
  return out;
}
constexpr Inverse<27> MINV_F = make_inverse<27>();
constexpr Inverse<19> MINV_G = make_inverse<19>();

// moments m[k] = sum_i M[k][i] a[i] (additions only: M has entries in {-1, 0, 1})
template <int Q, typename C>
__device__ __forceinline__ C moment(int k, const C* a) {
  C s = C(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int m = mom_entry<Q>(k, i);
    if (m > 0) s += a[i];
    else if (m < 0) s -= a[i];
  }
  return s;
}

// Raw features of a node from its relaxation increments d = f^eq - f and
// h = g^eq - g: x[k] = -(M d)[k], x[27 + k] = -(M h)[k], x[46] = rho'.  The
// conserved slots take their exact values instead of the rounding residue of
// the sums: the mass of f - f^eq is 0, its momentum is rho (u' - u_eq) =
// (0, 0, -F_z / 2) with Guo forcing and (0, 0, -tau_f F_z) with the velocity
// shift, and the zeroth moment of g - g^eq is -s / 2 (Eqs. (6), (7), (10),
// (16)).
template <int FORCE, typename C, typename Out>
__device__ __forceinline__ void node_features(const C* d, const C* h, const NodeMacro<C>& m, C tau_f,
                                              Out emit) {
  static_assert(FORCE == FORCE_GUO || FORCE == FORCE_SHIFT, "learned form: Guo or velocity shift");
  emit(0, 0.f);
  emit(1, 0.f);
  emit(2, 0.f);
  emit(3, (float)((FORCE == FORCE_GUO) ? -C(0.5) * m.Fz : -tau_f * m.Fz));
#pragma unroll
  for (int k = NCF; k < 27; ++k) emit(k, (float)-moment<27>(k, d));
  emit(27, (float)(-C(0.5) * m.s));
#pragma unroll
  for (int k = NCG; k < 19; ++k) emit(27 + k, (float)-moment<19>(k, h));
  emit(46, (float)m.rho_p);
}

// ---------------------------------------------------------------------------
// layout of the fused learned step: one node on two lanes of a wavefront
// ---------------------------------------------------------------------------
// In a 32x32x16 MFMA, lane (c, h) (c = lane % 32, h = lane / 32) supplies the
// B operand rows k = 16 ks + 8 h + q and receives the result rows
// 8 j + 4 h + q' (q' < 4) of each 32-row tile.  Storing logical row k of a
// weight matrix at physical row perm_row(k) (bits 2 and 3 of k swapped) makes
// the result registers of one layer, in order, the B operand of the next:
// B[ks][q] = D[tile ks / 2][8 (ks % 2) + q].
constexpr int perm_row(int k) { return (k & ~12) | ((k & 4) << 1) | ((k & 8) >> 1); }
// result row of register r of tile mt in lane half h
constexpr int d_row_of(int mt, int r, int h) { return 32 * mt + 8 * (r >> 2) + 4 * h + (r & 3); }
// B-operand row (K index) of slot b (ks = b / 8, q = b % 8) in lane half h
constexpr int slot_k(int h, int b) { return 16 * (b >> 3) + 8 * h + (b & 7); }

// Populations owned by lane half h: slot s < 13 holds the f pair (2s + 1, 2s + 2),
// half 0 the first and half 1 its opposite; slot 13 the f rest direction (half 0);
// slots 14..22 the g pairs likewise; slot 23 the g rest direction (half 0).  -1
// marks the two empty slots of half 1.  Global index: f_i = i, g_j = 27 + j.  The
// two halves' directions at a slot are opposite, so one sign per lane turns the
// half-0 direction into this lane's.
constexpr int NSLOT = 24, NSLOT_F = 14;
constexpr int owned_pop(int h, int s) {
  if (s < NSLOT_F - 1) return 2 * s + 1 + h;
  if (s == NSLOT_F - 1) return h ? -1 : 0;
  if (s < NSLOT - 1) return 27 + 2 * (s - NSLOT_F) + 1 + h;
  if (s == NSLOT - 1) return h ? -1 : 27;
  return -1;
}

// BF16 bits of a dyadic rational num / den (den a power of two, |num| < 256): exact.
constexpr uint16_t bf16_dyadic(long long num, long long den) {
  if (num == 0) return 0;
  const uint16_t sign = num < 0 ? 0x8000 : 0;
  long long a = num < 0 ? -num : num;
  int e = 0;                                         // value = a / den = m * 2^e, 1 <= m < 2
  while (a >= 2 * den) { den *= 2; ++e; }
  while (a < den) { a *= 2; --e; }
  // mantissa: 7 bits of (a - den) / den
  const long long frac = ((a - den) << 7) / den;
  return (uint16_t)(sign | ((uint16_t)(e + 127) << 7) | (uint16_t)frac);
}

// Constant A operands of the fused step:
//  feat: [physical row perm_row(k)][K index] = -(moment k of the owned population at
//        that K index), k a non-conserved moment; features are M (f - f^eq) = -M d;
//  minv: [result row of slot s of half h][output k] = M^-1 entry mapping the
//        non-conserved moment correction dm_k onto population owned_pop(h, s).
struct StepTables {
  uint16_t feat[64 * K_IN];
  uint16_t minv[64 * K_IN];
};

constexpr bool conserved_feature(int k) { return k < NCF || k == 27 || k >= N_IN - 1; }

constexpr StepTables make_step_tables() {
  StepTables t{};
  for (int row = 0; row < 64; ++row) {
    const int k = perm_row(row);
    for (int kk = 0; kk < K_IN; ++kk) {
      const int h = (kk >> 3) & 1, b = 8 * (kk >> 4) + (kk & 7);
      const int p = owned_pop(h, b);
      int v = 0;
      if (p >= 0 && k < N_IN && !conserved_feature(k)) {
        if (k < 27 && p < 27) v = -mom_entry<27>(k, p);
        if (k >= 27 && p >= 27) v = -mom_entry<19>(k - 27, p - 27);
      }
      t.feat[row * K_IN + kk] = bf16_dyadic(v, 1);
    }
  }
  const Frac zero{0, 1};
  for (int row = 0; row < 64; ++row) {
    const int mt = row >> 5, h = (row >> 2) & 1, r = 4 * ((row >> 3) & 3) + (row & 3);
    const int p = owned_pop(h, 16 * mt + r);
    for (int k = 0; k < K_IN; ++k) {
      Frac v = zero;
      if (p >= 0 && p < 27 && k < 27 - NCF) v = inverse_entry<27>(p, NCF + k);
      if (p >= 27 && k >= 27 - NCF && k < N_OUT) v = inverse_entry<19>(p - 27, NCG + k - (27 - NCF));
      t.minv[row * K_IN + k] = bf16_dyadic(v.n, v.d);
    }
  }
  return t;
}

// ---------------------------------------------------------------------------
// packed network (device): BF16 weights in MFMA-friendly row-major tiles,
// FP32 biases and normalisation
// ---------------------------------------------------------------------------
struct Packed {
  uint16_t w1[N_HID * K_IN];        // [hidden][input], input 47 zero
  uint16_t w2[N_HID * N_HID];       // [hidden][hidden]
  uint16_t w3[M_OUT * N_HID];       // [output][hidden], outputs >= 41 zero
  uint16_t w2t[N_HID * N_HID];      // W2^T
  uint16_t w3t[N_HID * M_OUT];      // W3^T: [hidden][output], outputs >= 41 zero
  float b1[N_HID], b2[N_HID], b3[M_OUT];
  float x_mean[K_IN], x_iscale[K_IN], y_scale[M_OUT];
  float zero[M_OUT];                // a zero bias for the backward products
  // the fused step's copies: rows at perm_row(logical row), W3 and b3 times y_scale
  alignas(16) uint16_t w1p[64 * K_IN];
  alignas(16) uint16_t w2p[64 * N_HID];
  alignas(16) uint16_t w3p[64 * N_HID];
  alignas(16) StepTables tab;
  alignas(16) float b1p[64], b2p[64], b3p[64], x_mean_p[64], x_iscale_p[64];
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t bf16_bits(float v) {   // round to nearest even
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_float(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// Activation buffers in LDS hold 64 nodes (one wavefront) x up to 64 values,
// node-major, rows padded to 72 entries to spread the 16-byte operand reads
// over the LDS banks.
constexpr int LDS_PITCH = 72;

// 32x32x16 BF16 MFMA operand layouts (checked on gfx950): lane l holds
// A[l % 32][8 (l / 32) + q] and B[8 (l / 32) + q][l % 32], q = 0..7; result
// register r of lane l is D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
__device__ __forceinline__ int d_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {   // 16-byte aligned
  return *reinterpret_cast<const bf16x8*>(p);
}

// out^T = W act^T for the 64 nodes of this wavefront: W is [MROWS][KW] row-major
// in global memory, act is LDS [node][LDS_PITCH] (k < KW used); the result for
// (row, node) is handed to emit(row, node, value) with the bias added.
template <int MROWS, int KW, typename Emit>
__device__ __forceinline__ void mfma_layer(const uint16_t* __restrict__ W, const float* __restrict__ bias,
                                           const uint16_t* act, Emit emit) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5, col = lane & 31;
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
#pragma unroll
    for (int mt = 0; mt < MROWS / 32; ++mt) {
      f32x16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = bias[32 * mt + d_row(r, lane)];
#pragma unroll
      for (int ks = 0; ks < KW / 16; ++ks) {
        const bf16x8 a = load8(W + (32 * mt + col) * KW + 16 * ks + 8 * half);
        const bf16x8 b = load8(act + (32 * nt + col) * LDS_PITCH + 16 * ks + 8 * half);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) emit(32 * mt + d_row(r, lane), 32 * nt + col, acc[r]);
    }
  }
}

// The network on the 64 node feature rows in LDS buffer x (normalised, BF16,
// columns 47.. zero).  h is a second LDS buffer; the de-normalised outputs
// go to o[node * N_OUT + k] (LDS, FP32).  Every wavefront of the block must call
// it (it synchronises the block between layers).
__device__ __forceinline__ void mlp_forward_wave(const Packed* __restrict__ P, uint16_t* x, uint16_t* h,
                                                 float* o) {
  mfma_layer<N_HID, K_IN>(P->w1, P->b1, x, [&](int row, int node, float v) {
    h[node * LDS_PITCH + row] = bf16_bits(tanhf(v));
  });
  __syncthreads();
  mfma_layer<N_HID, N_HID>(P->w2, P->b2, h, [&](int row, int node, float v) {
    x[node * LDS_PITCH + row] = bf16_bits(tanhf(v));
  });
  __syncthreads();
  mfma_layer<M_OUT, N_HID>(P->w3, P->b3, x, [&](int row, int node, float v) {
    if (row < N_OUT) o[node * N_OUT + row] = v * P->y_scale[row];
  });
  __syncthreads();
}

}  // namespace mlp
}  // namespace stgv
