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
constexpr Inverse<Q> make_inverse() {
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
  Inverse<Q> out{};
  for (int r = 0; r < Q; ++r)
    for (int c = 0; c < Q; ++c) out.v[r][c] = (float)A[r][Q + c].n / (float)A[r][Q + c].d;
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
