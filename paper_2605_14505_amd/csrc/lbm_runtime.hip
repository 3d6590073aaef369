// Host runtime and C ABI of the stratified-TGV DDF lattice Boltzmann step
// (declared in include/stgv.h), plus the diagnostic reduction kernels and the
// streaming-bandwidth probe.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/stgv.h"
#include "learned.hpp"
#include "postproc.hpp"
#include "lbm_device.hpp"
#include "lbm_launch.hpp"
#include "mlp_device.hpp"

namespace stgv {

// ---------------------------------------------------------------------------
// Dissipation stencil: eps_k needs |curl u|^2 and eps_p needs |grad rho'|^2 by
// second-order central differences (periodic).  A 64 x 4 tile of x-y columns
// marches up a chunk of z.  Each z-plane of the tile plus a one-node halo is
// staged in LDS (double-buffered, one barrier per plane) for the in-plane
// derivatives while the next plane is already on its way into registers; the
// z-derivatives of a plane are taken one plane later, when the plane above has
// arrived, from the column's values kept in registers.  Node by node, the
// arithmetic and the order of each thread's sum (planes z0, z0 + 1, ...) are
// those of the plain definition.
//
// The hardware hands consecutive blocks to the 8 XCDs in turn, each with its own
// L2; left so, a tile's halo rows belong to tiles on other XCDs and are fetched
// from HBM again.  The tiles of a z-chunk are therefore remapped so that every
// XCD owns a contiguous band of rows, whose inner halos its own L2 then serves.
// ---------------------------------------------------------------------------
#ifndef STGV_FD_ZC
#define STGV_FD_ZC 32
#endif
constexpr int FD_TX = 64, FD_TY = 4, FD_ZC = STGV_FD_ZC;
constexpr int FD_W = FD_TX + 2, FD_H = FD_TY + 2;
constexpr int FD_CELLS = FD_W * FD_H;
constexpr int FD_SLOTS = (FD_CELLS + FD_TX * FD_TY - 1) / (FD_TX * FD_TY);
constexpr int kXcds = 8;

__global__ __launch_bounds__(256) void lbm_fd_kernel(const float* __restrict__ fields, int n,
                                                     double* __restrict__ partials) {
  __shared__ float plane[2][4][FD_H][FD_W];     // u_x, u_y, u_z, rho'
  const int64_t n2 = (int64_t)n * n, n3 = n2 * n;
  const float* ux = fields + n3;
  const float* uy = fields + 2 * n3;
  const float* uz = fields + 3 * n3;
  const float* rp = fields + 4 * n3;
  int bx = blockIdx.x, by = blockIdx.y;
  if (gridDim.y % kXcds == 0) {            // the chunk's tiles, in dispatch order, by XCD
    const int lin = blockIdx.x + gridDim.x * blockIdx.y;
    const int xcd = lin % kXcds, j = lin / kXcds;
    by = xcd * (gridDim.y / kXcds) + j / gridDim.x;
    bx = j % gridDim.x;
  }
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = tx + FD_TX * ty;
  const int x0 = bx * FD_TX, y0 = by * FD_TY;
  const bool active = (x0 + tx < n) && (y0 + ty < n);
  const int z0 = blockIdx.z * FD_ZC;
  const int z1 = min(z0 + FD_ZC, n);
  auto zwrap = [n](int z) { return z < 0 ? z + n : (z >= n ? z - n : z); };

  // this thread's cells of the staged tile and their in-plane offsets, wrapped once
  int64_t off[FD_SLOTS];
  int cell[FD_SLOTS];
#pragma unroll
  for (int s = 0; s < FD_SLOTS; ++s) {
    const int c = tid + FD_TX * FD_TY * s;
    cell[s] = c < FD_CELLS ? c : -1;
    const int ly = c / FD_W, lx = c % FD_W;
    const int gx = ((x0 + lx - 1) % n + n) % n, gy = ((y0 + ly - 1) % n + n) % n;
    off[s] = c < FD_CELLS ? gx + (int64_t)n * gy : 0;
  }
  float r[FD_SLOTS][4];
  auto fetch = [&](int z) {
    const int64_t zo = n2 * zwrap(z);
#pragma unroll
    for (int s = 0; s < FD_SLOTS; ++s) {
      if (cell[s] < 0) continue;
      r[s][0] = ux[zo + off[s]];
      r[s][1] = uy[zo + off[s]];
      r[s][2] = uz[zo + off[s]];
      r[s][3] = rp[zo + off[s]];
    }
  };

  // per column: centres of the two planes below, in-plane terms of the plane below
  float cx_2 = 0.f, cy_2 = 0.f, cr_2 = 0.f, cx_1 = 0.f, cy_1 = 0.f, cr_1 = 0.f;
  float duz_dy = 0.f, duz_dx = 0.f, duy_dx = 0.f, dux_dy = 0.f, gx = 0.f, gy = 0.f;
  double curl2 = 0.0, grad2 = 0.0;
  const int lx = tx + 1, ly = ty + 1;

  fetch(z0 - 1);
  for (int z = z0 - 1; z <= z1; ++z) {
    const int b = (z - z0 + 1) & 1;
#pragma unroll
    for (int s = 0; s < FD_SLOTS; ++s) {
      if (cell[s] < 0) continue;
#pragma unroll
      for (int f = 0; f < 4; ++f) (&plane[b][f][0][0])[cell[s]] = r[s][f];
    }
    if (z < z1) fetch(z + 1);
    __syncthreads();
    const float cx_0 = plane[b][0][ly][lx], cy_0 = plane[b][1][ly][lx], cr_0 = plane[b][3][ly][lx];
    if (active && z >= z0 + 1) {          // plane z - 1 is complete
      const float dux_dz = 0.5f * (cx_0 - cx_2);
      const float duy_dz = 0.5f * (cy_0 - cy_2);
      const float wx = duz_dy - duy_dz, wy = dux_dz - duz_dx, wz = duy_dx - dux_dy;
      curl2 += (double)(wx * wx + wy * wy + wz * wz);
      const float gz = 0.5f * (cr_0 - cr_2);
      grad2 += (double)(gx * gx + gy * gy + gz * gz);
    }
    // in-plane terms of plane z, used when plane z + 1 arrives
    duz_dx = 0.5f * (plane[b][2][ly][lx + 1] - plane[b][2][ly][lx - 1]);
    duz_dy = 0.5f * (plane[b][2][ly + 1][lx] - plane[b][2][ly - 1][lx]);
    duy_dx = 0.5f * (plane[b][1][ly][lx + 1] - plane[b][1][ly][lx - 1]);
    dux_dy = 0.5f * (plane[b][0][ly + 1][lx] - plane[b][0][ly - 1][lx]);
    gx = 0.5f * (plane[b][3][ly][lx + 1] - plane[b][3][ly][lx - 1]);
    gy = 0.5f * (plane[b][3][ly + 1][lx] - plane[b][3][ly - 1][lx]);
    cx_2 = cx_1; cy_2 = cy_1; cr_2 = cr_1;
    cx_1 = cx_0; cy_1 = cy_0; cr_1 = cr_0;
  }
  // partials in dispatch order, so the reduction order does not depend on the remap
  const double v[NFD] = {curl2, grad2};
  const int64_t blk = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
  block_reduce_store<NFD, 0u>(v, partials + blk * NFD);
}

// ---------------------------------------------------------------------------
// Fixed-order FP64 reduction of the per-block partials into one record, in two
// launches: kMidBlocks blocks each reduce an even share of the step and stencil
// partials into one row of NPART + NFD values, then one block reduces the rows
// and writes the record.  Both orders depend only on the box size, so records
// are bitwise reproducible.
// ---------------------------------------------------------------------------
constexpr int kMidBlocks = 256;
constexpr int kNV = NPART + NFD;
constexpr unsigned kMaxMask = 1u << P_UMAX2;

__global__ __launch_bounds__(256) void lbm_mid_kernel(const double* __restrict__ sp, int64_t nsp,
                                                      const double* __restrict__ fp, int64_t nfp,
                                                      double* __restrict__ mid) {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  double v[kNV];
#pragma unroll
  for (int k = 0; k < kNV; ++k) v[k] = 0.0;
  for (int64_t i = nsp * b / nb + threadIdx.x; i < nsp * (b + 1) / nb; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NPART; ++k)
      v[k] = ((kMaxMask >> k) & 1u) ? fmax(v[k], sp[i * NPART + k]) : v[k] + sp[i * NPART + k];
  }
  for (int64_t i = nfp * b / nb + threadIdx.x; i < nfp * (b + 1) / nb; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NFD; ++k) v[NPART + k] += fp[i * NFD + k];
  }
  block_reduce_store<kNV, kMaxMask>(v, mid + b * kNV);
}

__global__ __launch_bounds__(256) void lbm_final_kernel(const double* __restrict__ mid, int64_t rows,
                                                        double* __restrict__ rec, int64_t step) {
  constexpr int NV = kNV;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  for (int64_t b = threadIdx.x; b < rows; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
      v[k] = ((kMaxMask >> k) & 1u) ? fmax(v[k], mid[b * NV + k]) : v[k] + mid[b * NV + k];
  }
  __shared__ double out[NV];
  block_reduce_store<NV, kMaxMask>(v, out);
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[NREC] = {0};
    r[R_STEP] = (double)step;
    r[R_EK] = out[P_EK];
    r[R_EP] = out[P_EP];
    r[R_CURL2] = out[NPART + FD_CURL2];
    r[R_GRAD2] = out[NPART + FD_GRAD2];
    r[R_DRHO] = out[P_DRHO];
    r[R_DSIG] = out[P_DSIG];
    r[R_MX] = out[P_MX];
    r[R_MY] = out[P_MY];
    r[R_MZ] = out[P_MZ];
    r[R_UMAX2] = out[P_UMAX2];
    r[R_NONFINITE] = out[P_NONFINITE];
    for (int k = 0; k < NREC; ++k) rec[k] = r[k];
  }
}

// ---------------------------------------------------------------------------
// Streaming-bandwidth probe: the achievable HBM ceiling for long unit-stride
// streams.  Each 256-thread block moves one 16 KiB chunk: four coalesced
// 16-byte vectors per thread, all loads issued before the stores.
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int BW_UNROLL = 4;

__global__ __launch_bounds__(256) void bw_copy_kernel(v4f* __restrict__ dst,
                                                      const v4f* __restrict__ src, int64_t nv) {
  const int64_t base = (int64_t)blockIdx.x * (256 * BW_UNROLL) + threadIdx.x;
  v4f v[BW_UNROLL];
#pragma unroll
  for (int k = 0; k < BW_UNROLL; ++k) {
    const int64_t i = base + k * 256;
    if (i < nv) v[k] = __builtin_nontemporal_load(src + i);
  }
#pragma unroll
  for (int k = 0; k < BW_UNROLL; ++k) {
    const int64_t i = base + k * 256;
    if (i < nv) __builtin_nontemporal_store(v[k], dst + i);
  }
}
__global__ __launch_bounds__(256) void bw_read_kernel(float* __restrict__ dst,
                                                      const v4f* __restrict__ src, int64_t nv) {
  const int64_t base = (int64_t)blockIdx.x * (256 * BW_UNROLL) + threadIdx.x;
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < BW_UNROLL; ++k) {
    const int64_t i = base + k * 256;
    if (i < nv) {
      const v4f v = __builtin_nontemporal_load(src + i);
      acc += v.x + v.y + v.z + v.w;
    }
  }
  // keep the loads live; one value per block
  __shared__ float red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) dst[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(256) void bw_write_kernel(v4f* __restrict__ dst, int64_t nv) {
  const int64_t base = (int64_t)blockIdx.x * (256 * BW_UNROLL) + threadIdx.x;
  const v4f v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < BW_UNROLL; ++k) {
    const int64_t i = base + k * 256;
    if (i < nv) __builtin_nontemporal_store(v, dst + i);
  }
}

}  // namespace stgv

// ===========================================================================
// Host side
// ===========================================================================
using namespace stgv;

namespace {

constexpr int kRingCap = 4096;
constexpr size_t kAlign = 256;

thread_local char g_err[512] = "";

struct Derived {
  double L, nu, D, tau_f, tau_g, nb, G, beta, cs2_f, cs2_g;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

void set_err(char* buf, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, 512, fmt, ap);
  va_end(ap);
}

double lattice_cs2(int q) { return q == 7 ? 0.25 : 1.0 / 3.0; }

bool valid_pair(int qf, int qg) {
#define STGV_IS_PAIR(A, B) if (qf == A && qg == B) return true;
  STGV_FOR_EACH_PAIR(STGV_IS_PAIR)
#undef STGV_IS_PAIR
  return false;
}

// Parameter checks and the lattice-unit constants of Eqs. (8), (13), (14), (19)
// with U = u0, L = n / (2 pi), rho_0 = 1 and G = (G/N) N.
int derive(const lbm_params* p, Derived* d, char* err) {
  if (!p) { set_err(err, "params is NULL"); return LBM_EINVAL; }
  if (p->n < 4 || p->n > 1024) { set_err(err, "n = %d outside [4, 1024]", p->n); return LBM_EINVAL; }
  if (!valid_pair(p->q_f, p->q_g)) {
    set_err(err, "stencil pair D3Q%d x D3Q%d not supported (27x19, 27x7, 19x7, 27x27, 19x19, 19x15, "
                 "15x7, 7x27)", p->q_f, p->q_g);
    return LBM_EINVAL;
  }
  if (p->forcing < LBM_FORCE_GUO || p->forcing > LBM_FORCE_HCZ) {
    set_err(err, "forcing = %d invalid", p->forcing); return LBM_EINVAL;
  }
  if (p->storage < LBM_FP32 || p->storage > LBM_BF16) {
    set_err(err, "storage = %d invalid", p->storage); return LBM_EINVAL;
  }
  if (p->compute != LBM_COMPUTE_FP32 && p->compute != LBM_COMPUTE_FP64) {
    set_err(err, "compute = %d invalid", p->compute); return LBM_EINVAL;
  }
  if (p->compute == LBM_COMPUTE_FP64 && p->storage != LBM_FP32) {
    set_err(err, "FP64 arithmetic is available with FP32 storage only"); return LBM_EINVAL;
  }
  if (p->reserved != 0) { set_err(err, "reserved field must be 0"); return LBM_EINVAL; }
  if (p->layout != LBM_LAYOUT_AA && p->layout != LBM_LAYOUT_AB) {
    set_err(err, "layout = %d invalid", p->layout); return LBM_EINVAL;
  }
  if (p->diag_every < 0) { set_err(err, "diag_every = %d < 0", p->diag_every); return LBM_EINVAL; }
  if (!(std::isfinite(p->u0) && p->u0 > 0.0 && p->u0 < 0.3)) {
    set_err(err, "u0 = %g outside (0, 0.3)", p->u0); return LBM_EINVAL;
  }
  if (!(std::isfinite(p->re) && p->re > 0.0)) { set_err(err, "re = %g must be > 0", p->re); return LBM_EINVAL; }
  if (!(std::isfinite(p->sc) && p->sc > 0.0)) { set_err(err, "sc = %g must be > 0", p->sc); return LBM_EINVAL; }
  if (!(p->fr > 0.0) || std::isnan(p->fr)) { set_err(err, "fr = %g must be > 0 (inf allowed)", p->fr); return LBM_EINVAL; }
  if (!(std::isfinite(p->g_over_n) && p->g_over_n > 0.0)) {
    set_err(err, "g_over_n = %g must be finite and > 0", p->g_over_n); return LBM_EINVAL;
  }
  if (!(std::isfinite(p->noise_amp) && p->noise_amp >= 0.0)) {
    set_err(err, "noise_amp = %g must be finite and >= 0", p->noise_amp); return LBM_EINVAL;
  }
  Derived o;
  o.cs2_f = lattice_cs2(p->q_f);
  o.cs2_g = lattice_cs2(p->q_g);
  o.L = p->n / (2.0 * M_PI);
  o.nu = p->u0 * o.L / p->re;
  o.D = o.nu / p->sc;
  o.tau_f = o.nu / o.cs2_f + 0.5;
  o.tau_g = o.D / o.cs2_g + 0.5;
  o.nb = std::isinf(p->fr) ? 0.0 : p->u0 / (p->fr * o.L);
  o.G = p->g_over_n * o.nb;
  o.beta = o.G != 0.0 ? -o.nb * o.nb / o.G : 0.0;
  if (!(o.tau_f > 0.5) || !(o.tau_g > 0.5) || !std::isfinite(o.tau_f) || !std::isfinite(o.tau_g)) {
    set_err(err, "relaxation times tau_f = %.17g, tau_g = %.17g must exceed 1/2", o.tau_f, o.tau_g);
    return LBM_EINVAL;
  }
  if (d) *d = o;
  return LBM_OK;
}

struct Sizes {
  int64_t n3, stride;
  size_t elem, pop_bytes;
  size_t off_fields, off_sp, off_fp, off_mid, off_ring, work_bytes;
  int64_t nsp, nfp, nsp_learned;
};

size_t elem_size(int storage) { return storage == LBM_FP32 ? 4 : 2; }

Sizes sizes_of(const lbm_params* p) {
  Sizes s;
  const int64_t n = p->n;
  s.n3 = n * n * n;
  s.elem = elem_size(p->storage);
  // Arrays start on 256-byte boundaries; the default pad of 1 KiB (plus the
  // alignment) keeps the Q_f + Q_g streams off a power-of-two stride.
  const int64_t per_line = (int64_t)(kAlign / s.elem);
  const int64_t pad = p->pad >= 0 ? p->pad : (int64_t)(1024 / s.elem);
  s.stride = ((s.n3 + pad + per_line - 1) / per_line) * per_line;
  const int64_t arrays = (int64_t)(p->q_f + p->q_g) * (p->layout == LBM_LAYOUT_AB ? 2 : 1);
  s.pop_bytes = (size_t)(arrays * s.stride) * s.elem;
  const LaunchShape sh = node_shape(p->n);
  s.nsp = (int64_t)sh.grid.x * sh.grid.y * sh.grid.z;
  // the learned step runs 256-thread blocks of 128 nodes
  s.nsp_learned = (p->n % 64 == 0) ? (int64_t)p->n * p->n * p->n / 128 : 0;
  const int64_t nsp_max = s.nsp > s.nsp_learned ? s.nsp : s.nsp_learned;
  s.nfp = (int64_t)((p->n + FD_TX - 1) / FD_TX) * ((p->n + FD_TY - 1) / FD_TY) * ((p->n + FD_ZC - 1) / FD_ZC);
  size_t off = 0;
  s.off_fields = off; off = align_up(off + (size_t)(5 * s.n3) * sizeof(float), kAlign);
  s.off_sp = off;     off = align_up(off + (size_t)(nsp_max * NPART) * sizeof(double), kAlign);
  s.off_fp = off;     off = align_up(off + (size_t)(s.nfp * NFD) * sizeof(double), kAlign);
  s.off_mid = off;    off = align_up(off + (size_t)kMidBlocks * kNV * sizeof(double), kAlign);
  s.off_ring = off;   off = align_up(off + (size_t)kRingCap * NREC * sizeof(double), kAlign);
  s.work_bytes = off;
  return s;
}

}  // namespace

struct lbm_ctx {
  lbm_params p;
  Derived d;
  Sizes sz;
  LaunchShape sh;
  PhysConsts c;
  Geometry geo;
  char* pop;           // AA array, or the first AB lattice
  char* pop_b;         // second AB lattice (nullptr for AA)
  char* work;
  hipStream_t stream;
  int64_t step;
  int odd;             // AA: the array holds the odd-step layout; AB: pop_b is current
  int64_t ring_head;   // records queued
  int64_t ring_tail;   // records drained
  const void* mlp;     // attached packed network (learned step) or nullptr
  char err[512];
};

namespace {

int hip_fail(lbm_ctx* ctx, hipError_t e, const char* what) {
  char* buf = ctx ? ctx->err : g_err;
  set_err(buf, "%s: %s", what, hipGetErrorString(e));
  return LBM_EHIP;
}

template <typename F>
hipError_t by_storage(int storage, F&& f) {
  switch (storage) {
    case LBM_FP32: return f((float*)nullptr);
    case LBM_FP16: return f((_Float16*)nullptr);
    default: return f((bf16_t*)nullptr);
  }
}

// Node-kernel launch for the context's storage and compute types.
hipError_t launch_node(lbm_ctx* c, int mode, int flags, char* src, char* dst, float* fields,
                       double* partials);

float* fields_buf(lbm_ctx* c) { return (float*)(c->work + c->sz.off_fields); }
double* sp_buf(lbm_ctx* c) { return (double*)(c->work + c->sz.off_sp); }
double* fp_buf(lbm_ctx* c) { return (double*)(c->work + c->sz.off_fp); }
double* mid_buf(lbm_ctx* c) { return (double*)(c->work + c->sz.off_mid); }
double* ring_buf(lbm_ctx* c) { return (double*)(c->work + c->sz.off_ring); }

// Layout of the current state for the gather of a moment-only pass.
int current_mode(const lbm_ctx* c) {
  if (c->p.layout == LBM_LAYOUT_AB) return MODE_EVEN;
  return c->odd ? MODE_ODD : MODE_EVEN;
}
char* current_array(const lbm_ctx* c) {
  return (c->p.layout == LBM_LAYOUT_AB && c->odd) ? c->pop_b : c->pop;
}

// Queue the dissipation stencil and the final reduction into the next ring slot.
hipError_t queue_record(lbm_ctx* c, int64_t step, bool learned) {
  const dim3 fblock(FD_TX, FD_TY, 1);
  const dim3 fgrid((c->p.n + FD_TX - 1) / FD_TX, (c->p.n + FD_TY - 1) / FD_TY,
                   (c->p.n + FD_ZC - 1) / FD_ZC);
  hipLaunchKernelGGL(lbm_fd_kernel, fgrid, fblock, 0, c->stream, fields_buf(c), c->p.n, fp_buf(c));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double* slot = ring_buf(c) + (c->ring_head % kRingCap) * NREC;
  hipLaunchKernelGGL(lbm_mid_kernel, dim3(kMidBlocks), dim3(256), 0, c->stream, sp_buf(c),
                     learned ? c->sz.nsp_learned : c->sz.nsp, fp_buf(c), c->sz.nfp, mid_buf(c));
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lbm_final_kernel, dim3(1), dim3(256), 0, c->stream, mid_buf(c),
                     (int64_t)kMidBlocks, slot, step);
  e = hipGetLastError();
  if (e == hipSuccess) c->ring_head++;
  return e;
}

}  // namespace

namespace {
hipError_t launch_node(lbm_ctx* c, int mode, int flags, char* src, char* dst, float* fields,
                       double* partials) {
  const int qf = c->p.q_f, qg = c->p.q_g, fo = c->p.forcing;
  switch (c->p.storage) {
    case LBM_FP32:
      if (c->p.compute == LBM_COMPUTE_FP64)
        return launch_step<float, double>(qf, qg, fo, mode, flags, c->sh, c->stream, (float*)src,
                                          (float*)dst, c->geo, c->c, fields, partials);
      return launch_step<float, float>(qf, qg, fo, mode, flags, c->sh, c->stream, (float*)src,
                                       (float*)dst, c->geo, c->c, fields, partials);
    case LBM_FP16:
      return launch_step<_Float16, float>(qf, qg, fo, mode, flags, c->sh, c->stream, (_Float16*)src,
                                          (_Float16*)dst, c->geo, c->c, fields, partials);
    default:
      return launch_step<bf16_t, float>(qf, qg, fo, mode, flags, c->sh, c->stream, (bf16_t*)src,
                                        (bf16_t*)dst, c->geo, c->c, fields, partials);
  }
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int lbm_query_sizes(const lbm_params* p, size_t* pop_bytes, size_t* work_bytes) {
  const int rc = derive(p, nullptr, g_err);
  if (rc != LBM_OK) return rc;
  const Sizes s = sizes_of(p);
  if (pop_bytes) *pop_bytes = s.pop_bytes;
  if (work_bytes) *work_bytes = s.work_bytes;
  return LBM_OK;
}

int lbm_derived(const lbm_params* p, double* out) {
  Derived d;
  const int rc = derive(p, &d, g_err);
  if (rc != LBM_OK) return rc;
  if (!out) { set_err(g_err, "out is NULL"); return LBM_EINVAL; }
  const double v[8] = {d.L, d.nu, d.D, d.tau_f, d.tau_g, d.nb, d.G, d.beta};
  memcpy(out, v, sizeof(v));
  return LBM_OK;
}

int lbm_init_tgv(const lbm_params* p, void* pop_dev, size_t pop_bytes, void* work_dev,
                 size_t work_bytes, void* hip_stream, lbm_ctx** out) {
  if (!out) { set_err(g_err, "out is NULL"); return LBM_EINVAL; }
  *out = nullptr;
  Derived d;
  int rc = derive(p, &d, g_err);
  if (rc != LBM_OK) return rc;
  const Sizes s = sizes_of(p);
  if (!pop_dev || !work_dev) { set_err(g_err, "device buffer is NULL"); return LBM_EINVAL; }
  if (((uintptr_t)pop_dev % kAlign) || ((uintptr_t)work_dev % kAlign)) {
    set_err(g_err, "device buffers must be %zu-byte aligned", kAlign); return LBM_EINVAL;
  }
  if (pop_bytes < s.pop_bytes) {
    set_err(g_err, "population buffer has %zu bytes, needs %zu", pop_bytes, s.pop_bytes);
    return LBM_ESIZE;
  }
  if (work_bytes < s.work_bytes) {
    set_err(g_err, "work buffer has %zu bytes, needs %zu", work_bytes, s.work_bytes);
    return LBM_ESIZE;
  }
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) { set_err(g_err, "out of host memory"); return LBM_EINVAL; }
  c->p = *p;
  c->d = d;
  c->sz = s;
  c->sh = node_shape(p->n);
  c->c.omega_f = 1.0 / d.tau_f;
  c->c.omega_g = 1.0 / d.tau_g;
  c->c.tau_f = d.tau_f;
  c->c.G = d.G;
  c->c.beta = d.beta;
  c->c.g_over_n = p->g_over_n;
  c->geo.n = p->n;
  c->geo.stride = s.stride;
  c->pop = (char*)pop_dev;
  c->pop_b = p->layout == LBM_LAYOUT_AB
                 ? (char*)pop_dev + (size_t)(p->q_f + p->q_g) * s.stride * s.elem
                 : nullptr;
  c->work = (char*)work_dev;
  c->stream = (hipStream_t)hip_stream;
  c->step = 0;
  c->odd = 0;
  c->ring_head = c->ring_tail = 0;
  c->mlp = nullptr;
  c->err[0] = 0;
  hipError_t e = by_storage(p->storage, [&](auto* tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return launch_init<T>(p->q_f, p->q_g, c->sh, c->stream, (T*)c->pop, c->geo, p->u0,
                          p->noise_amp, p->seed);
  });
  if (e != hipSuccess) {
    hip_fail(nullptr, e, "init kernel");
    delete c;
    return LBM_EHIP;
  }
  *out = c;
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t nsteps) {
  if (!c) { set_err(g_err, "ctx is NULL"); return LBM_EINVAL; }
  if (nsteps < 0) { set_err(c->err, "n = %lld < 0", (long long)nsteps); return LBM_EINVAL; }
  const int64_t k = c->p.diag_every;
  if (k > 0 && nsteps > 0) {
    // records in [step, step + n): multiples of k
    const int64_t first = (c->step + k - 1) / k, last = (c->step + nsteps - 1) / k;
    const int64_t count = last - first + 1;
    if (c->ring_head - c->ring_tail + count > kRingCap) {
      set_err(c->err, "diagnostics ring would overflow (%lld pending + %lld new > %d): drain it first",
              (long long)(c->ring_head - c->ring_tail), (long long)count, kRingCap);
      return LBM_ESTATE;
    }
  }
  for (int64_t s = 0; s < nsteps; ++s) {
    const bool diag = k > 0 && (c->step % k) == 0;
    const int flags = diag ? (K_COLLIDE | K_FIELDS | K_PARTIALS) : K_COLLIDE;
    int mode;
    char *src, *dst;
    if (c->p.layout == LBM_LAYOUT_AB) {
      mode = MODE_AB;
      src = c->odd ? c->pop_b : c->pop;
      dst = c->odd ? c->pop : c->pop_b;
    } else {
      mode = c->odd ? MODE_ODD : MODE_EVEN;
      src = dst = c->pop;
    }
    hipError_t e = c->mlp
        ? launch_learned_step(c->p.forcing, mode, flags, c->p.n, c->stream, (float*)src, (float*)dst,
                              c->geo, c->c, fields_buf(c), sp_buf(c), c->mlp)
        : launch_node(c, mode, flags, src, dst, fields_buf(c), sp_buf(c));
    if (e != hipSuccess) return hip_fail(c, e, "step kernel");
    if (diag) {
      e = queue_record(c, c->step, c->mlp != nullptr);
      if (e != hipSuccess) return hip_fail(c, e, "diagnostic kernels");
    }
    c->step++;
    c->odd ^= 1;
  }
  return LBM_OK;
}

int lbm_stream(lbm_ctx* c, int64_t nsteps) {
  if (!c) { set_err(g_err, "ctx is NULL"); return LBM_EINVAL; }
  if (nsteps < 0) { set_err(c->err, "n = %lld < 0", (long long)nsteps); return LBM_EINVAL; }
  for (int64_t s = 0; s < nsteps; ++s) {
    int mode;
    char *src, *dst;
    if (c->p.layout == LBM_LAYOUT_AB) {
      mode = MODE_AB;
      src = c->odd ? c->pop_b : c->pop;
      dst = c->odd ? c->pop : c->pop_b;
    } else {
      mode = c->odd ? MODE_ODD : MODE_EVEN;
      src = dst = c->pop;
    }
    hipError_t e = by_storage(c->p.storage, [&](auto* tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      return launch_stream<T>(c->p.q_f, c->p.q_g, mode, c->sh, c->stream, (T*)src, (T*)dst, c->geo);
    });
    if (e != hipSuccess) return hip_fail(c, e, "free-streaming kernel");
    c->step++;
    c->odd ^= 1;
  }
  return LBM_OK;
}

int lbm_sample(lbm_ctx* c) {
  if (!c) { set_err(g_err, "ctx is NULL"); return LBM_EINVAL; }
  if (c->ring_head - c->ring_tail + 1 > kRingCap) {
    set_err(c->err, "diagnostics ring full: drain it first");
    return LBM_ESTATE;
  }
  const int mode = current_mode(c);
  char* src = current_array(c);
  hipError_t e = launch_node(c, mode, K_FIELDS | K_PARTIALS, src, src, fields_buf(c), sp_buf(c));
  if (e != hipSuccess) return hip_fail(c, e, "moments kernel");
  e = queue_record(c, c->step, false);
  if (e != hipSuccess) return hip_fail(c, e, "diagnostic kernels");
  return LBM_OK;
}

int lbm_diagnostics(lbm_ctx* c, lbm_diag* out, int32_t max, int32_t* n_out) {
  if (!c) { set_err(g_err, "ctx is NULL"); return LBM_EINVAL; }
  if (n_out) *n_out = 0;
  if (max < 0 || (max > 0 && !out)) { set_err(c->err, "invalid output array"); return LBM_EINVAL; }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  const int64_t pending = c->ring_head - c->ring_tail;
  const int64_t take = pending < max ? pending : max;
  const double n3 = (double)c->sz.n3;
  const double u0 = c->p.u0, L = c->d.L;
  const double e_scale = 1.0 / (n3 * u0 * u0);
  const double eps_scale = L / (n3 * u0 * u0 * u0);
  const double cs = std::sqrt(c->d.cs2_f);
  int rc = LBM_OK;
  double rec[NREC];
  for (int64_t r = 0; r < take; ++r) {
    const int64_t slot = (c->ring_tail + r) % kRingCap;
    e = hipMemcpy(rec, ring_buf(c) + slot * NREC, sizeof(rec), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy ring");
    lbm_diag& o = out[r];
    o.step = (int64_t)rec[R_STEP];
    o.t = o.step * u0 / L;
    o.ek = rec[R_EK] * e_scale;
    o.ep = c->d.G != 0.0 ? rec[R_EP] * e_scale : 0.0;
    o.eps_k = c->d.nu * rec[R_CURL2] * eps_scale;
    o.eps_p = c->d.G != 0.0 ? c->d.D * c->p.g_over_n * c->p.g_over_n * rec[R_GRAD2] * eps_scale : 0.0;
    o.mass = n3 + rec[R_DRHO];
    o.scalar = n3 + rec[R_DSIG];
    o.mom[0] = rec[R_MX];
    o.mom[1] = rec[R_MY];
    o.mom[2] = rec[R_MZ];
    o.umax = std::sqrt(rec[R_UMAX2]);
    o.nonfinite = (int64_t)rec[R_NONFINITE];
    if (o.nonfinite > 0 || !(o.umax <= cs)) {
      set_err(c->err, "unstable state at step %lld: %lld non-finite nodes, max|u| = %g",
              (long long)o.step, (long long)o.nonfinite, o.umax);
      rc = LBM_EUNSTABLE;
    }
  }
  c->ring_tail += take;
  if (n_out) *n_out = (int32_t)take;
  return rc;
}

int lbm_read_fields(lbm_ctx* c, float* dev_out) {
  if (!c) { set_err(g_err, "ctx is NULL"); return LBM_EINVAL; }
  if (!dev_out) { set_err(c->err, "dev_out is NULL"); return LBM_EINVAL; }
  const int mode = current_mode(c);
  char* src = current_array(c);
  hipError_t e = launch_node(c, mode, K_FIELDS, src, src, dev_out, nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "fields kernel");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  return LBM_OK;
}

int lbm_read_populations(lbm_ctx* c, float* dev_out) {
  if (!c) { set_err(g_err, "ctx is NULL"); return LBM_EINVAL; }
  if (!dev_out) { set_err(c->err, "dev_out is NULL"); return LBM_EINVAL; }
  const int mode = current_mode(c);
  char* src = current_array(c);
  hipError_t e = by_storage(c->p.storage, [&](auto* tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return launch_canon<T>(c->p.q_f, c->p.q_g, mode, c->sh, c->stream, (const T*)src, c->geo, dev_out);
  });
  if (e != hipSuccess) return hip_fail(c, e, "canonicalise kernel");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  return LBM_OK;
}

int lbm_load_populations(lbm_ctx* c, const float* dev_in, int64_t step) {
  if (!c) { set_err(g_err, "ctx is NULL"); return LBM_EINVAL; }
  if (!dev_in) { set_err(c->err, "dev_in is NULL"); return LBM_EINVAL; }
  if (step < 0) { set_err(c->err, "step = %lld < 0", (long long)step); return LBM_EINVAL; }
  hipError_t e = by_storage(c->p.storage, [&](auto* tag) {
    using T = std::remove_pointer_t<decltype(tag)>;
    return launch_load<T>(c->p.q_f, c->p.q_g, c->sh, c->stream, (T*)c->pop, c->geo, dev_in);
  });
  if (e != hipSuccess) return hip_fail(c, e, "load kernel");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  c->odd = 0;
  c->step = step;
  return LBM_OK;
}

int lbm_stencil_info(int32_t q, int32_t* e, double* w, double* cs2) {
  auto fill = [&](auto S) {
    using St = decltype(S);
    for (int i = 0; i < St::q; ++i) {
      if (e) { e[3 * i] = St::ex[i]; e[3 * i + 1] = St::ey[i]; e[3 * i + 2] = St::ez[i]; }
      if (w) w[i] = St::w[i];
    }
    if (cs2) *cs2 = St::cs2;
    return LBM_OK;
  };
  switch (q) {
    case 7: return fill(Stencil<7>{});
    case 15: return fill(Stencil<15>{});
    case 19: return fill(Stencil<19>{});
    case 27: return fill(Stencil<27>{});
    default: set_err(g_err, "no D3Q%d stencil", q); return LBM_EINVAL;
  }
}

int lbm_bw_probe(int32_t kind, void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (bytes == 0 || bytes % 16) { set_err(g_err, "bytes must be a positive multiple of 16"); return LBM_EINVAL; }
  if (!dst || (kind != 2 && !src)) { set_err(g_err, "NULL buffer"); return LBM_EINVAL; }
  const int64_t nv = (int64_t)(bytes / 16);
  const int64_t blocks = (nv + 256 * BW_UNROLL - 1) / (256 * BW_UNROLL);
  if (blocks > 0x7fffffff) { set_err(g_err, "bytes too large"); return LBM_EINVAL; }
  hipStream_t st = (hipStream_t)hip_stream;
  switch (kind) {
    case 0: hipLaunchKernelGGL(bw_copy_kernel, dim3(blocks), dim3(256), 0, st, (v4f*)dst, (const v4f*)src, nv); break;
    case 1: hipLaunchKernelGGL(bw_read_kernel, dim3(blocks), dim3(256), 0, st, (float*)dst, (const v4f*)src, nv); break;
    case 2: hipLaunchKernelGGL(bw_write_kernel, dim3(blocks), dim3(256), 0, st, (v4f*)dst, nv); break;
    default: set_err(g_err, "kind = %d invalid", kind); return LBM_EINVAL;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(nullptr, e, "bandwidth probe");
  return LBM_OK;
}

// ---------------------------------------------------------------------------
// learned correction
// ---------------------------------------------------------------------------
size_t lbm_mlp_packed_bytes(void) { return sizeof(mlp::Packed); }

int lbm_mlp_pack(const float* params, const float* norm, void* packed, void* stream) {
  if (!params || !norm || !packed) { set_err(g_err, "NULL buffer"); return LBM_EINVAL; }
  if ((uintptr_t)packed % 16) { set_err(g_err, "packed buffer must be 16-byte aligned"); return LBM_EINVAL; }
  hipError_t e = mlp_launch_pack(params, norm, packed, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "pack kernel");
  return LBM_OK;
}

int lbm_mlp_forward(const void* packed, const float* x, int64_t rows, float* y, void* stream) {
  if (!packed || !x || !y || rows < 0) { set_err(g_err, "invalid argument"); return LBM_EINVAL; }
  if (rows == 0) return LBM_OK;
  if ((rows + 63) / 64 > 0x7fffffff) { set_err(g_err, "too many rows"); return LBM_EINVAL; }
  hipError_t e = mlp_launch_forward(packed, x, rows, y, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "forward kernel");
  return LBM_OK;
}

size_t lbm_mlp_grad_work_bytes(int64_t batch) {
  const int64_t blocks = batch > 0 ? (batch + 63) / 64 : 0;
  return align_up((size_t)blocks * mlp::N_PARAMS * sizeof(float), kAlign) +
         align_up((size_t)blocks * sizeof(double), kAlign);
}

int lbm_mlp_grad(const void* packed, const float* x, const float* y, const int64_t* idx, int64_t batch,
                 float* grad, double* loss, void* work, size_t work_bytes, void* stream) {
  if (!packed || !x || !y || !idx || !grad || !work || batch <= 0) {
    set_err(g_err, "invalid argument"); return LBM_EINVAL;
  }
  if (work_bytes < lbm_mlp_grad_work_bytes(batch)) {
    set_err(g_err, "work buffer has %zu bytes, needs %zu", work_bytes, lbm_mlp_grad_work_bytes(batch));
    return LBM_ESIZE;
  }
  const int64_t blocks = (batch + 63) / 64;
  float* gpart = (float*)work;
  double* lpart = (double*)((char*)work + align_up((size_t)blocks * mlp::N_PARAMS * sizeof(float), kAlign));
  hipError_t e = mlp_launch_grad(packed, x, y, idx, batch, gpart, lpart, grad, loss, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "gradient kernels");
  return LBM_OK;
}

// ---------------------------------------------------------------------------
// The gradient without a caller workspace: its per-block partial sums live in a
// file-scope device array of fixed size, one copy per GPU for the whole process.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kStaticGradBlocks = (LBM_MLP_STATIC_MAX_BATCH + 63) / 64;
constexpr size_t kStaticGpartBytes = ((size_t)kStaticGradBlocks * mlp::N_PARAMS * sizeof(float) + 255) / 256 * 256;
constexpr size_t kStaticScratchBytes = kStaticGpartBytes + (size_t)kStaticGradBlocks * sizeof(double);
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

// The partial gradients (kStaticGradBlocks x LBM_MLP_PARAMS FP32) and losses (FP64)
// of lbm_mlp_grad_static.  Host code never uses this name as an address: it takes the
// device address that hipGetSymbolAddress returns for the current GPU (scratch_address).
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Device address of `scratch` on the current GPU, looked up once per device (with that
// device current) and kept.
static int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) { set_err(g_err, "device %d beyond the library's %d", dev, kMaxDevices); return LBM_EINVAL; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress of the gradient scratch");
    if (!ptr) { set_err(g_err, "hipGetSymbolAddress returned no address for the gradient scratch"); return LBM_EHIP; }
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return LBM_OK;
}

int lbm_mlp_grad_static(const void* packed, const float* x, const float* y, const int64_t* idx,
                        int64_t batch, float* grad, double* loss, void* stream) {
  if (!packed || !x || !y || !idx || !grad || batch <= 0) { set_err(g_err, "invalid argument"); return LBM_EINVAL; }
  if (batch > LBM_MLP_STATIC_MAX_BATCH) {
    set_err(g_err, "batch of %lld rows exceeds the %d rows of the built-in gradient scratch",
            (long long)batch, (int)LBM_MLP_STATIC_MAX_BATCH);
    return LBM_ESIZE;
  }
  void* base = nullptr;
  const int st = scratch_address(&base);
  if (st != LBM_OK) return st;
  // every block writes all of its partials before the reduction reads them, so nothing
  // left by an earlier call needs clearing
  float* gpart = static_cast<float*>(base);
  double* lpart = reinterpret_cast<double*>(static_cast<char*>(base) + kStaticGpartBytes);
  hipError_t e = mlp_launch_grad(packed, x, y, idx, batch, gpart, lpart, grad, loss, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "gradient kernels");
  return LBM_OK;
}

int lbm_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t t, double lr, void* stream) {
  if (!params || !m || !v || !grad || t < 1 || !(lr > 0.0)) { set_err(g_err, "invalid argument"); return LBM_EINVAL; }
  const double b1 = 0.9, b2 = 0.999;
  const double c1 = 1.0 / (1.0 - std::pow(b1, (double)t)), c2 = 1.0 / (1.0 - std::pow(b2, (double)t));
  // 1 - beta and the bias corrections in double: 1 - 0.999f in FP32 is off by 1.3e-5
  hipError_t e = mlp_launch_adam(params, m, v, grad, (float)lr, (float)b1, (float)b2, (float)(1.0 - b1),
                                 (float)(1.0 - b2), 1e-8f, (float)c1, (float)c2, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "adam kernel");
  return LBM_OK;
}

static constexpr int kNormBlocks = 256;
size_t lbm_mlp_norm_work_bytes(void) { return (size_t)kNormBlocks * (2 * mlp::N_IN + mlp::N_OUT) * sizeof(double); }

int lbm_mlp_norm(const float* x, const float* y, int64_t rows, float* norm, void* work, size_t work_bytes,
                 void* stream) {
  if (!x || !y || !norm || !work || rows <= 0) { set_err(g_err, "invalid argument"); return LBM_EINVAL; }
  if (work_bytes < lbm_mlp_norm_work_bytes()) { set_err(g_err, "work buffer too small"); return LBM_ESIZE; }
  hipError_t e = mlp_launch_norm(x, y, rows, (double*)work, kNormBlocks, norm, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "normalisation kernels");
  return LBM_OK;
}

static bool learned_forcing(const lbm_ctx* c) {
  return c->p.forcing == LBM_FORCE_GUO || c->p.forcing == LBM_FORCE_SHIFT;
}

int lbm_restrict(lbm_ctx* fine, const lbm_ctx* coarse, float* out) {
  if (!fine || !coarse || !out) { set_err(g_err, "invalid argument"); return LBM_EINVAL; }
  if (fine->p.q_f != 27 || fine->p.q_g != 19 || coarse->p.q_f != 27 || coarse->p.q_g != 19) {
    set_err(fine->err, "restriction is defined for D3Q27 x D3Q19"); return LBM_EINVAL;
  }
  if (!learned_forcing(fine) || !learned_forcing(coarse)) {
    set_err(fine->err, "the learned form is defined for Guo and velocity-shift forcing"); return LBM_EINVAL;
  }
  if (fine->p.n != 4 * coarse->p.n) {
    set_err(fine->err, "fine n = %d must be 4 x coarse n = %d", fine->p.n, coarse->p.n); return LBM_EINVAL;
  }
  const float sf = (float)(4.0 * coarse->d.tau_f / fine->d.tau_f);
  const float sg = (float)(4.0 * coarse->d.tau_g / fine->d.tau_g);
  hipError_t e = mlp_launch_restrict(fine->p.storage, current_array(fine), current_mode(fine), fine->geo,
                                     fine->c, coarse->p.n, sf, sg, out, fine->stream);
  if (e != hipSuccess) return hip_fail(fine, e, "restriction kernel");
  return LBM_OK;
}

int lbm_training_pairs(lbm_ctx* c, const float* a, const float* b, const float* cc, float* x, float* y) {
  if (!c || !a || !b || !cc || !x || !y) { set_err(g_err, "invalid argument"); return LBM_EINVAL; }
  if (c->p.q_f != 27 || c->p.q_g != 19) { set_err(c->err, "training pairs need D3Q27 x D3Q19"); return LBM_EINVAL; }
  if (!learned_forcing(c)) {
    set_err(c->err, "the learned form is defined for Guo and velocity-shift forcing"); return LBM_EINVAL;
  }
  hipError_t e = mlp_launch_pairs(c->p.forcing, a, b, cc, c->p.n, c->c, x, y, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "training-pair kernel");
  return LBM_OK;
}

int lbm_set_mlp(lbm_ctx* c, const void* packed) {
  if (!c) { set_err(g_err, "ctx is NULL"); return LBM_EINVAL; }
  if (packed) {
    if (c->p.q_f != 27 || c->p.q_g != 19 || c->p.storage != LBM_FP32 || c->p.compute != LBM_COMPUTE_FP32 ||
        c->p.n % 64 != 0 || c->p.n > 256 || !learned_forcing(c)) {
      set_err(c->err, "the learned step needs D3Q27 x D3Q19, Guo or velocity-shift forcing, FP32 storage "
                      "and arithmetic, n %% 64 == 0 and n <= 256");
      return LBM_EINVAL;
    }
    if ((uintptr_t)packed % 16) { set_err(c->err, "packed network must be 16-byte aligned"); return LBM_EINVAL; }
  }
  c->mlp = packed;
  return LBM_OK;
}

int lbm_postprocess(const lbm_diag* recs, int32_t count, double re, double fr, double t_end, double* r_out,
                    double* gamma_out, lbm_post* out) {
  if (!recs || !out || count < 2 || !(re > 0.0) || !(fr > 0.0) || std::isnan(t_end)) {
    set_err(g_err, "invalid argument"); return LBM_EINVAL;
  }
  for (int32_t i = 1; i < count; ++i)
    if (!(recs[i].t > recs[i - 1].t)) { set_err(g_err, "record times must increase (record %d)", i); return LBM_EINVAL; }
  const double nu = 1.0 / re, nb = 1.0 / fr;          // fr = +inf gives N = 0
  lbm_post post{};
  post.r_max = -1.0;
  for (int32_t i = 0; i < count; ++i) {
    const double r = recs[i].eps_k / (nu * nb * nb);
    if (r_out) r_out[i] = r;
    if (gamma_out) gamma_out[i] = recs[i].eps_p / recs[i].eps_k;
    if (r > post.r_max) { post.r_max = r; post.t_r_max = recs[i].t; }
  }
  double ip = 0.0, ik = 0.0, ie = 0.0;
  int32_t used = 1;
  for (int32_t i = 1; i < count && recs[i].t <= t_end; ++i, ++used) {
    const double h = 0.5 * (recs[i].t - recs[i - 1].t);
    ip += h * (recs[i].eps_p + recs[i - 1].eps_p);
    ik += h * (recs[i].eps_k + recs[i - 1].eps_k);
    ie += h * (recs[i].ek + recs[i - 1].ek);
  }
  post.gamma_b = ip / ik;
  post.fr_t = ik / (nb * ie);
  post.used = used;
  *out = post;
  return LBM_OK;
}

int32_t lbm_spectrum_shells(int32_t n) { return (n < 4 || n > 1024) ? -1 : spectrum_shells(n); }

static size_t spectrum_fields_bytes(int n) { return align_up((size_t)5 * n * n * n * sizeof(float), kAlign); }

int lbm_spectrum_work_bytes(int32_t n, size_t* bytes) {
  if (!bytes || n < 4 || n > 1024) { set_err(g_err, "invalid argument"); return LBM_EINVAL; }
  char err[512] = {0};
  const size_t extra = spectrum_extra_bytes(n, err);
  if (!extra) { set_err(g_err, "%s", err); return LBM_EHIP; }
  *bytes = spectrum_fields_bytes(n) + extra;
  return LBM_OK;
}

int lbm_ke_spectrum(lbm_ctx* c, void* work, size_t work_bytes, double* shells) {
  if (!c) { set_err(g_err, "ctx is NULL"); return LBM_EINVAL; }
  if (!work || !shells || (uintptr_t)work % kAlign) {
    set_err(c->err, "work (256-byte aligned) and shells must be device buffers"); return LBM_EINVAL;
  }
  const int n = c->p.n;
  const size_t fb = spectrum_fields_bytes(n);
  if (work_bytes < fb) { set_err(c->err, "spectrum work buffer too small"); return LBM_ESIZE; }
  float* fields = static_cast<float*>(work);
  const int mode = current_mode(c);
  char* src = current_array(c);
  hipError_t e = launch_node(c, mode, K_FIELDS, src, src, fields, nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "fields kernel");
  const size_t n3 = (size_t)n * n * n;
  char err[512] = {0};
  e = spectrum_launch(fields + n3, fields + 2 * n3, fields + 3 * n3, n, c->p.u0, static_cast<char*>(work) + fb,
                      work_bytes - fb, shells, c->stream, err);
  if (e == hipErrorInvalidValue && err[0]) { set_err(c->err, "%s", err); return LBM_ESIZE; }
  if (e == hipErrorUnknown && err[0]) { set_err(c->err, "%s", err); return LBM_EHIP; }
  if (e != hipSuccess) return hip_fail(c, e, "spectrum kernels");
  return LBM_OK;
}

int64_t lbm_get_step(const lbm_ctx* c) { return c ? c->step : -1; }

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err : g_err; }

const char* lbm_status_string(int s) {
  switch (s) {
    case LBM_OK: return "LBM_OK";
    case LBM_EINVAL: return "LBM_EINVAL";
    case LBM_ESIZE: return "LBM_ESIZE";
    case LBM_EHIP: return "LBM_EHIP";
    case LBM_EUNSTABLE: return "LBM_EUNSTABLE";
    case LBM_ESTATE: return "LBM_ESTATE";
    default: return "unknown status";
  }
}

void lbm_destroy(lbm_ctx* c) { delete c; }

}  // extern "C"
