// The fused learned step: D3Q27 x D3Q19, FP32 populations and arithmetic, with the
// network's moment correction added to the post-collision populations.
//
// One node lives on two lanes of a wavefront, lane (c, h) with c = lane % 32 the node
// of the wavefront's 32 and h = lane / 32 the half: each half loads, relaxes and
// stores the 24 populations owned_pop(h, s) lists (mlp_device.hpp), and the halves
// exchange five partial sums for the moments and five for the projection of the
// relaxation increments.  Everything per node that is a product with a matrix runs
// on 32x32x16 BF16 MFMA with the 32 nodes as the columns:
//   features   x = -M d (the non-equilibrium moments), d in two BF16 halves;
//   network    three layers, tanh, weights stored at permuted rows so that each
//              layer's result registers are the next layer's B operand;
//   correction dF = M^-1 [0, dm], dm in two BF16 halves, whose result rows are the
//              populations the lane owns.
// The MFMA A operands (the two moment tables and the three weight matrices, 34 KB of
// BF16) are staged in LDS once per block behind one barrier; the diagnostic reduction
// adds its own.  Launched with 256-thread blocks on an (n / 64, n / 2, n) grid, each block
// two 32-node runs in each of two x-rows (n % 64 == 0, n <= 256).
#include "lbm_kernels.hpp"
#include "learned.hpp"
#include "mlp_device.hpp"

namespace stgv {
namespace {
using namespace mlp;
using SF = Stencil<27>;
using SG = Stencil<19>;

__device__ __forceinline__ float xor32(float v) { return __shfl_xor(v, 32, 64); }

// Row pitch padding (bf16 elements) of the MFMA A-operand tables held in LDS.  Padding by 8
// (pitches 112 B and 144 B, which spread the lanes of each 16-byte read phase over distinct
// bank groups) measured 1 % slower on gfx950 (64^3 step 33.9 -> 34.3 us): bank conflicts
// on these reads do not limit the kernel.
#ifndef STGV_LEARNED_W_PAD
#define STGV_LEARNED_W_PAD 0
#endif
constexpr int PW_IN = K_IN + STGV_LEARNED_W_PAD, PW_HID = N_HID + STGV_LEARNED_W_PAD;

// A ROWS x COLS BF16 table (COLS a multiple of 8), row-major in global memory, on its way
// to LDS rows of pitch PITCH: this thread's 16-byte pieces of the 256-thread block's share
// are loaded into registers first (load) and written to LDS later (put), so that a block
// issues the loads of every table before it waits for any of them.
constexpr int kStageThreads = 256;
using u32x4 = unsigned int __attribute__((ext_vector_type(4)));
template <int ROWS, int COLS, int PITCH>
struct Staged {
  static constexpr int per_row = COLS / 8, pieces = ROWS * per_row;
  static_assert(pieces > kStageThreads && pieces <= 2 * kStageThreads, "two pieces per thread");
  u32x4 t0, t1;   // named registers: an array member here was placed in scratch memory
  __device__ __forceinline__ void load(const uint16_t* __restrict__ g) {
    const int i = (int)threadIdx.x;
    t0 = reinterpret_cast<const u32x4*>(g)[i];
    // unconditional (past the end: the last piece again), so no load waits on a branch
    t1 = reinterpret_cast<const u32x4*>(g)[min(i + kStageThreads, pieces - 1)];
  }
  __device__ __forceinline__ void put(uint16_t* d) const {
    auto at = [d](int i) {
      const int r = i / per_row, c = i - r * per_row;
      return reinterpret_cast<u32x4*>(d + r * PITCH + 8 * c);
    };
    const int i = (int)threadIdx.x;
    *at(i) = t0;
    if (i + kStageThreads < pieces) *at(i + kStageThreads) = t1;
  }
};

__device__ __forceinline__ f32x16 mfma16(const bf16x8& a, const bf16x8& b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// FP32 -> BF16 conversions in the fused step use gfx950's packed convert (round to
// nearest even), one instruction per pair of values.
__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }

// v = hi + lo with hi, lo in BF16 (|v - hi - lo| ~ 2^-16 |v|)
__device__ __forceinline__ void split_bf16(float v, __bf16& hi, __bf16& lo) {
  hi = to_bf16(v);
  lo = to_bf16(v - (float)hi);
}

// tanh x = 1 - 2 / (1 + e^(2x)) with the hardware exp2 and reciprocal: absolute error
// ~1e-7, far below the BF16 rounding (2^-9 relative) the activation goes through next.
// Saturates to +-1 for large |x| (e^(2x) -> inf or 0).
__device__ __forceinline__ float fast_tanh(float x) {
  return 1.f - 2.f * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(2.8853900817779268f * x));
}

// direction data of population p (global index: f_i = i, g_j = 27 + j; -1: none)
struct Dir {
  int ex, ey, ez, opp;
  float w;
};
__device__ __forceinline__ Dir dir_of(int p) {
  Dir d{0, 0, 0, 0, 0.f};
  if (p >= 0 && p < 27) d = Dir{SF::ex[p], SF::ey[p], SF::ez[p], opp(p), (float)SF::w[p]};
  if (p >= 27) d = Dir{SG::ex[p - 27], SG::ey[p - 27], SG::ez[p - 27], 27 + opp(p - 27), (float)SG::w[p - 27]};
  return d;
}

// A population is addressed as a base uniform across the wavefront (the lower of the
// two neighbouring arrays a slot's halves own) plus a 32-bit byte offset: the node's
// offset and, for the half owning the upper array, one array stride.
__device__ __forceinline__ const float* at_byte(const float* base, uint32_t bytes) {
  return (const float*)((const char*)base + bytes);
}
__device__ __forceinline__ float* at_byte(float* base, uint32_t bytes) {
  return (float*)((char*)base + bytes);
}

// array (population slot) and node offset of the load (GATHER) or store of population p
template <int MODE, bool GATHER>
__device__ __forceinline__ void address_of(int p, const NodeIndex& ix, int& arr, uint32_t& off) {
  const Dir d = dir_of(p);
  if (GATHER) {
    if (MODE == MODE_ODD) { arr = d.opp; off = ix.at(-d.ex, -d.ey, -d.ez); }
    else { arr = p; off = ix.base; }
  } else {
    if (MODE == MODE_EVEN) { arr = d.opp; off = ix.base; }
    else { arr = p; off = ix.at(d.ex, d.ey, d.ez); }
  }
}

// the analytic value of conserved feature k, or NaN if k is not one
template <int FORCE>
__device__ __forceinline__ float analytic_feature(int k, const NodeMacro<float>& m, float tau_f) {
  if (k < NCF - 1) return 0.f;                                            // mass, x, y momentum
  if (k == NCF - 1) return FORCE == FORCE_GUO ? -0.5f * m.Fz : -tau_f * m.Fz;
  if (k == 27) return -0.5f * m.s;
  if (k == N_IN - 1) return m.rho_p;
  return __builtin_nanf("");
}
constexpr bool is_analytic(int k) { return k < NCF || k == 27 || k == N_IN - 1; }

// tanh of the 16 results of a tile into two 8-wide B operands
__device__ __forceinline__ void tanh_to_b(const f32x16& t, bf16x8& lo8, bf16x8& hi8) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    lo8[q] = to_bf16(fast_tanh(t[q]));
    hi8[q] = to_bf16(fast_tanh(t[8 + q]));
  }
}

__device__ __forceinline__ f32x16 bias_tile(const float* b, int mt, int h) {
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = b[d_row_of(mt, r, h)];
  return acc;
}

template <int FORCE, int MODE, bool DIAG>
__global__ __launch_bounds__(256) void learned_step_kernel(float* __restrict__ pop, float* __restrict__ dst,
                                                           Geometry geo, PhysConsts c,
                                                           float* __restrict__ fields,
                                                           double* __restrict__ partials,
                                                           const Packed* __restrict__ P) {
  static_assert(FORCE == FORCE_GUO || FORCE == FORCE_SHIFT, "learned form: Guo or velocity shift");
  const int n = geo.n;
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5, col = lane & 31;
  // A wavefront holds 32 consecutive nodes of one x-row (rows are a whole number of
  // 64-node segments), a block two such runs in each of two rows; the row and plane are
  // the wavefront's own, so only x is per lane and nothing is divided.
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int y = 2 * (int)blockIdx.y + (wv >> 1), z = (int)blockIdx.z;
  const int x0 = 64 * (int)blockIdx.x + 32 * (wv & 1);
  const NodeIndex ix = make_index(x0 + col, y, z, n);
  const float* src = pop;

  // ---- this half's populations.  The halves of a slot read neighbouring arrays
  // (a1 = a0 +- 1): the address is the lower array's base, uniform, plus the node offset
  // and, for the half owning the upper array, one array stride.
  const uint32_t S = (uint32_t)geo.stride;
  const uint32_t upper_h1 = h ? S : 0u, upper_h0 = h ? 0u : S;
  auto slot_address = [&](auto* base, int p0, int p1, int a0, int a1, uint32_t off) {
    int lower;
    uint32_t extra;
    if (p1 < 0) { lower = a0; extra = 0u; }                       // half 0 only
    else if (a1 == a0 + 1) { lower = a0; extra = upper_h1; }
    else if (a0 == a1 + 1) { lower = a1; extra = upper_h0; }
    else { lower = 0; extra = (uint32_t)(h ? a1 : a0) * S; }
    return at_byte(base + (size_t)lower * S, (off + extra) * 4u);
  };
  float v[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int p0 = owned_pop(0, s), p1 = owned_pop(1, s);
    int a0 = 0, a1 = 0;
    uint32_t o0 = 0, o1 = 0;
    if (p0 >= 0) address_of<MODE, true>(p0, ix, a0, o0);
    if (p1 >= 0) address_of<MODE, true>(p1, ix, a1, o1);
    v[s] = 0.f;
    if ((h ? p1 : p0) >= 0) v[s] = load_as<float>(slot_address(src, p0, p1, a0, a1, h ? o1 : o0));
  }

  // The MFMA A operands (feature and correction tables, the three permuted weight
  // matrices, 34 KB unpadded) are shared by every node: staged in LDS once per block, they
  // are read there instead of through the vector cache (64^3 step 40.2 -> 33.9 us).  Their
  // loads are issued behind the population loads and before any wait, so the block pays
  // one memory latency for both.
  __shared__ alignas(16) uint16_t s_feat[64 * PW_IN], s_minv[64 * PW_IN], s_w1p[64 * PW_IN];
  __shared__ alignas(16) uint16_t s_w2p[64 * PW_HID], s_w3p[64 * PW_HID];
  {
    Staged<64, K_IN, PW_IN> feat, minv, w1;
    Staged<64, N_HID, PW_HID> w2, w3;
    feat.load(P->tab.feat);
    minv.load(P->tab.minv);
    w1.load(P->w1p);
    w2.load(P->w2p);
    w3.load(P->w3p);
    // every staged value is an input here, so the wave waits once, for all of the loads,
    // and no LDS write is scheduled above a load still to be issued
    asm volatile("" ::"v"(feat.t0), "v"(feat.t1), "v"(minv.t0), "v"(minv.t1), "v"(w1.t0), "v"(w1.t1),
                 "v"(w2.t0), "v"(w2.t1), "v"(w3.t0), "v"(w3.t1));
    feat.put(s_feat);
    minv.put(s_minv);
    w1.put(s_w1p);
    w2.put(s_w2p);
    w3.put(s_w3p);
  }
  __syncthreads();
  // Direction of slot s in this half: sg * e0(s), e0 the half-0 direction; the
  // weight is the same in both halves except for half 1's two empty slots.
  const float sg = h ? -1.f : 1.f;
  auto e0 = [](int s) { return dir_of(owned_pop(0, s)); };
  auto weight = [&](int s) {
    const float w0 = e0(s).w;
    return owned_pop(1, s) >= 0 ? w0 : (h ? 0.f : w0);
  };

  // ---- moments: partial sums over the half, completed with the other half's
  float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f, dsig = 0.f;
#pragma unroll
  for (int s = 0; s < NSLOT_F; ++s) {
    const Dir d = e0(s);
    drho += v[s];
    jx = d.ex ? (d.ex > 0 ? jx + v[s] : jx - v[s]) : jx;
    jy = d.ey ? (d.ey > 0 ? jy + v[s] : jy - v[s]) : jy;
    jz = d.ez ? (d.ez > 0 ? jz + v[s] : jz - v[s]) : jz;
  }
#pragma unroll
  for (int s = NSLOT_F; s < NSLOT; ++s) dsig += v[s];
  jx *= sg;
  jy *= sg;
  jz *= sg;
  drho += xor32(drho);
  jx += xor32(jx);
  jy += xor32(jy);
  jz += xor32(jz);
  dsig += xor32(dsig);
  NodeMacro<float> m;
  macro_from_sums<FORCE>(drho, jx, jy, jz, dsig, c, m);
  const Collision<27, 19, FORCE, float> cl(c, m);
  // e.(a, b, c) for this lane's direction of slot s
  auto edot = [&](int s, float a, float b, float cc) {
    const Dir d = e0(s);
    return sg * dot_e(d.ex, d.ey, d.ez, a, b, cc);
  };
  auto feq_s = [&](int s) { return cl.feq_of(edot(s, cl.vx, cl.vy, cl.vz), weight(s)); };
  auto geq_s = [&](int s) { return cl.geq_of(edot(s, cl.tx, cl.ty, cl.tz), weight(s)); };

  // ---- relaxation increments d = f^eq - f and their conserved moments
  float r0 = 0.f, rx = 0.f, ry = 0.f, rz = 0.f, r0g = 0.f;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    if (s < NSLOT_F) {
      const Dir d = e0(s);
      v[s] = feq_s(s) - v[s];
      r0 += v[s];
      rx = d.ex ? (d.ex > 0 ? rx + v[s] : rx - v[s]) : rx;
      ry = d.ey ? (d.ey > 0 ? ry + v[s] : ry - v[s]) : ry;
      rz = d.ez ? (d.ez > 0 ? rz + v[s] : rz - v[s]) : rz;
    } else {
      v[s] = geq_s(s) - v[s];
      r0g += v[s];
    }
  }
  rx *= sg;
  ry *= sg;
  rz *= sg;
  r0 += xor32(r0);
  rx += xor32(rx);
  ry += xor32(ry);
  rz += xor32(rz);
  r0g += xor32(r0g);

  // ---- features: -M d on MFMA, d in two BF16 halves
  bf16x8 dhi[3], dlo[3];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    __bf16 hi, lo;
    split_bf16(v[s], hi, lo);
    dhi[s >> 3][s & 7] = hi;
    dlo[s >> 3][s & 7] = lo;
  }
  f32x16 xf[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f32x16 acc = {0};
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) {
      const bf16x8 a = load8(s_feat + (32 * mt + col) * PW_IN + 16 * ks + 8 * h);
      acc = mfma16(a, dhi[ks], acc);
      acc = mfma16(a, dlo[ks], acc);
    }
    xf[mt] = acc;
  }

  // ---- finish the collision (the increments are no longer needed)
  {
    rz -= (FORCE == FORCE_GUO) ? 0.5f * m.Fz : cl.tau_f * m.Fz;
    r0g -= 0.5f * m.s;
    const float om = cl.omega_f, og = cl.omega_g;
    const float guo_c = (1.f - 0.5f * om) * m.Fz;
    const float src_g = (1.f - 0.5f * og) * m.s - og * r0g;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      if (s < NSLOT_F) {
        constexpr float icf = Collision<27, 19, FORCE, float>::icf;
        const float pr = weight(s) * (r0 + icf * edot(s, rx, ry, rz));
        float small = -om * pr;
        if (FORCE == FORCE_GUO) {
          const int ez0 = e0(s).ez;
          float br = -icf * m.uz;
          if (ez0 != 0) br += (ez0 > 0 ? sg : -sg) * (icf * (1.f + icf * edot(s, m.ux, m.uy, m.uz)));
          small = fma_c(-om, pr, weight(s) * guo_c * br);
        }
        v[s] = feq_s(s) + fma_c(om - 1.f, v[s], small);
      } else {
        v[s] = geq_s(s) + fma_c(og - 1.f, v[s], weight(s) * src_g);
      }
    }
  }

  // ---- normalised features -> layer-1 operand (logical feature k at physical row perm_row(k))
  bf16x8 b1[3];
#pragma unroll
  for (int ks = 0; ks < 3; ++ks) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int mt = ks >> 1, r = 8 * (ks & 1) + q;
      float val = xf[mt][r];
      const int k0 = perm_row(d_row_of(mt, r, 0)), k1 = perm_row(d_row_of(mt, r, 1));
      if (is_analytic(k0) || is_analytic(k1)) {
        const float v0 = is_analytic(k0) ? analytic_feature<FORCE>(k0, m, cl.tau_f) : val;
        const float v1 = is_analytic(k1) ? analytic_feature<FORCE>(k1, m, cl.tau_f) : val;
        val = h ? v1 : v0;
      }
      const int row = d_row_of(mt, r, h);
      b1[ks][q] = to_bf16((val - P->x_mean_p[row]) * P->x_iscale_p[row]);
    }
  }

  // ---- the network
  bf16x8 hb[4];
  {
    f32x16 t[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      t[mt] = bias_tile(P->b1p, mt, h);
#pragma unroll
      for (int ks = 0; ks < 3; ++ks)
        t[mt] = mfma16(load8(s_w1p + (32 * mt + col) * PW_IN + 16 * ks + 8 * h), b1[ks], t[mt]);
    }
    tanh_to_b(t[0], hb[0], hb[1]);
    tanh_to_b(t[1], hb[2], hb[3]);
  }
  {
    f32x16 t[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      t[mt] = bias_tile(P->b2p, mt, h);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        t[mt] = mfma16(load8(s_w2p + (32 * mt + col) * PW_HID + 16 * ks + 8 * h), hb[ks], t[mt]);
    }
    tanh_to_b(t[0], hb[0], hb[1]);
    tanh_to_b(t[1], hb[2], hb[3]);
  }
  bf16x8 mhi[3], mlo[3];
  {
    f32x16 t[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      t[mt] = bias_tile(P->b3p, mt, h);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        t[mt] = mfma16(load8(s_w3p + (32 * mt + col) * PW_HID + 16 * ks + 8 * h), hb[ks], t[mt]);
    }
#pragma unroll
    for (int ks = 0; ks < 3; ++ks)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        __bf16 hi, lo;
        split_bf16(t[ks >> 1][8 * (ks & 1) + q], hi, lo);
        mhi[ks][q] = hi;
        mlo[ks][q] = lo;
      }
  }

  // ---- correction M^-1 [0, dm]: result rows are this half's populations
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f32x16 acc = {0};
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) {
      const bf16x8 a = load8(s_minv + (32 * mt + col) * PW_IN + 16 * ks + 8 * h);
      acc = mfma16(a, mhi[ks], acc);
      acc = mfma16(a, mlo[ks], acc);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r)
      if (16 * mt + r < NSLOT) v[16 * mt + r] += acc[r];
  }

  // ---- store, addressed as the loads (the node's neighbour offsets are recomputed here
  // rather than kept live through the network: the empty asm hides that the lane's x is
  // unchanged)
  int col_s = col;
  asm volatile("" : "+v"(col_s));
  const NodeIndex ixs = make_index(x0 + col_s, y, z, n);
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int p0 = owned_pop(0, s), p1 = owned_pop(1, s);
    int a0 = 0, a1 = 0;
    uint32_t o0 = 0, o1 = 0;
    if (p0 >= 0) address_of<MODE, false>(p0, ixs, a0, o0);
    if (p1 >= 0) address_of<MODE, false>(p1, ixs, a1, o1);
    if ((h ? p1 : p0) >= 0) store_as(slot_address(dst, p0, p1, a0, a1, h ? o1 : o0), v[s]);
  }

  if constexpr (DIAG) {
    double acc[NPART];
#pragma unroll
    for (int k = 0; k < NPART; ++k) acc[k] = 0.0;
    if (h == 0) {
      write_fields(m, fields, ixs.base, (int64_t)n * n * n);
      node_partials(m, c, acc);
    }
    const int64_t blk = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
    block_reduce_store<NPART, (1u << P_UMAX2)>(acc, partials + blk * NPART);
  }
}

template <int FORCE, int MODE>
hipError_t go(bool diag, int n, hipStream_t st, float* pop, float* dst, Geometry geo, PhysConsts c,
              float* fields, double* partials, const void* net) {
  const dim3 block(256), grid((unsigned)(n / 64), (unsigned)(n / 2), (unsigned)n);   // n^3 / 128 blocks
  const Packed* P = static_cast<const Packed*>(net);
  if (diag)
    hipLaunchKernelGGL((learned_step_kernel<FORCE, MODE, true>), grid, block, 0, st, pop, dst, geo, c, fields,
                       partials, P);
  else
    hipLaunchKernelGGL((learned_step_kernel<FORCE, MODE, false>), grid, block, 0, st, pop, dst, geo, c, fields,
                       partials, P);
  return hipGetLastError();
}

template <int FORCE>
hipError_t by_mode(int mode, bool diag, int n, hipStream_t st, float* pop, float* dst, Geometry geo,
                   PhysConsts c, float* fields, double* partials, const void* net) {
  switch (mode) {
    case MODE_EVEN: return go<FORCE, MODE_EVEN>(diag, n, st, pop, dst, geo, c, fields, partials, net);
    case MODE_ODD: return go<FORCE, MODE_ODD>(diag, n, st, pop, dst, geo, c, fields, partials, net);
    default: return go<FORCE, MODE_AB>(diag, n, st, pop, dst, geo, c, fields, partials, net);
  }
}

}  // namespace

hipError_t launch_learned_step(int forcing, int mode, int flags, int n, hipStream_t st, float* pop,
                               float* dst, Geometry geo, PhysConsts c, float* fields, double* partials,
                               const void* packed) {
  if (n % 64 != 0 || n > 256) return hipErrorInvalidValue;     // the boxes lbm_set_mlp accepts
  const bool diag = (flags & K_PARTIALS) != 0;
  if (forcing == FORCE_GUO) return by_mode<FORCE_GUO>(mode, diag, n, st, pop, dst, geo, c, fields, partials, packed);
  if (forcing == FORCE_SHIFT) return by_mode<FORCE_SHIFT>(mode, diag, n, st, pop, dst, geo, c, fields, partials, packed);
  return hipErrorInvalidValue;
}

}  // namespace stgv
