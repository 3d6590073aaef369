// Learned correction of a coarse run: restriction of a fine state, training
// pairs, the network's forward / backward / Adam kernels on BF16 MFMA.
#include <hip/hip_runtime.h>

#include "learned.hpp"
#include "lbm_device.hpp"
#include "mlp_device.hpp"

namespace stgv {
namespace mlp {

__constant__ StepTables kStepTables = make_step_tables();

// ---------------------------------------------------------------------------
// packing: FP32 master parameters (W1 [64][47], b1, W2 [64][64], b2, W3 [41][64],
// b3) and the normalisation (x_mean[47], x_iscale[47], y_scale[41]) -> Packed
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ theta,
                                                   const float* __restrict__ norm,
                                                   Packed* __restrict__ P) {
  const float* W1 = theta;
  const float* b1 = W1 + N_HID * N_IN;
  const float* W2 = b1 + N_HID;
  const float* b2 = W2 + N_HID * N_HID;
  const float* W3 = b2 + N_HID;
  const float* b3 = W3 + N_OUT * N_HID;
  for (int t = threadIdx.x; t < N_HID * K_IN; t += blockDim.x) {
    const int r = t / K_IN, c = t % K_IN;
    P->w1[t] = c < N_IN ? bf16_bits(W1[r * N_IN + c]) : 0;
  }
  for (int t = threadIdx.x; t < N_HID * N_HID; t += blockDim.x) {
    const int r = t / N_HID, c = t % N_HID;
    P->w2[t] = bf16_bits(W2[t]);
    P->w2t[t] = bf16_bits(W2[c * N_HID + r]);
  }
  for (int t = threadIdx.x; t < M_OUT * N_HID; t += blockDim.x) {
    const int r = t / N_HID, c = t % N_HID;               // w3: [output r][hidden c]
    P->w3[t] = r < N_OUT ? bf16_bits(W3[r * N_HID + c]) : 0;
    const int h = t / M_OUT, o = t % M_OUT;               // w3t: [hidden h][output o]
    P->w3t[t] = o < N_OUT ? bf16_bits(W3[o * N_HID + h]) : 0;
  }
  for (int t = threadIdx.x; t < M_OUT; t += blockDim.x) {
    P->b1[t] = t < N_HID ? b1[t] : 0.f;
    P->b2[t] = t < N_HID ? b2[t] : 0.f;
    P->b3[t] = t < N_OUT ? b3[t] : 0.f;
    P->y_scale[t] = t < N_OUT ? norm[2 * N_IN + t] : 0.f;
    P->zero[t] = 0.f;
  }
  for (int t = threadIdx.x; t < K_IN; t += blockDim.x) {
    P->x_mean[t] = t < N_IN ? norm[t] : 0.f;
    P->x_iscale[t] = t < N_IN ? norm[N_IN + t] : 0.f;
  }
  // the fused step's copies: logical row k at physical row perm_row(k); the output
  // layer carries y_scale so that its result is the moment correction itself
  for (int t = threadIdx.x; t < 64 * K_IN; t += blockDim.x) {
    const int row = t / K_IN, c = t % K_IN, k = perm_row(row);
    P->w1p[t] = c < N_IN ? bf16_bits(W1[k * N_IN + c]) : 0;
    P->tab.feat[t] = kStepTables.feat[t];
    P->tab.minv[t] = kStepTables.minv[t];
  }
  for (int t = threadIdx.x; t < 64 * N_HID; t += blockDim.x) {
    const int row = t / N_HID, c = t % N_HID, k = perm_row(row);
    P->w2p[t] = bf16_bits(W2[k * N_HID + c]);
    P->w3p[t] = k < N_OUT ? bf16_bits(norm[2 * N_IN + k] * W3[k * N_HID + c]) : 0;
  }
  for (int row = threadIdx.x; row < 64; row += blockDim.x) {
    const int k = perm_row(row);
    P->b1p[row] = b1[k];
    P->b2p[row] = b2[k];
    P->b3p[row] = k < N_OUT ? norm[2 * N_IN + k] * b3[k] : 0.f;
    P->x_mean_p[row] = k < N_IN ? norm[k] : 0.f;
    P->x_iscale_p[row] = k < N_IN ? norm[N_IN + k] : 0.f;
  }
}

// Normalised features of one row into an LDS activation row (BF16, zero padded to 64).
__device__ __forceinline__ void put_features(const Packed* P, const float* x, uint16_t* row) {
  for (int k = 0; k < 64; ++k)
    row[k] = k < N_IN ? bf16_bits((x[k] - P->x_mean[k]) * P->x_iscale[k]) : (uint16_t)0;
}

// ---------------------------------------------------------------------------
// batch inference: rows of raw features -> de-normalised moment corrections
// one wavefront (64 rows) per block
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void forward_kernel(const Packed* __restrict__ P,
                                                     const float* __restrict__ x, int64_t rows,
                                                     float* __restrict__ y) {
  __shared__ __attribute__((aligned(16))) uint16_t xs[64 * LDS_PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t hs[64 * LDS_PITCH];
  __shared__ float os[64 * N_OUT];
  const int lane = threadIdx.x;
  const int64_t row = (int64_t)blockIdx.x * 64 + lane;
  float xr[N_IN];
  for (int k = 0; k < N_IN; ++k) xr[k] = row < rows ? x[row * N_IN + k] : 0.f;
  put_features(P, xr, xs + lane * LDS_PITCH);
  __syncthreads();
  mlp_forward_wave(P, xs, hs, os);
  if (row < rows)
    for (int k = 0; k < N_OUT; ++k) y[row * N_OUT + k] = os[lane * N_OUT + k];
}

// ---------------------------------------------------------------------------
// gradient of the mean squared error over a batch (rows idx[0..batch)), one
// wavefront of 64 samples per block; per-block partial gradients in the
// master-parameter order and a partial loss
// ---------------------------------------------------------------------------
// sum_n A[n][i] B[n][j] for i, j < 64 over the 64 nodes (rows) of two LDS buffers.
template <typename Emit>
__device__ __forceinline__ void outer_over_nodes(const uint16_t* A, const uint16_t* B, Emit emit) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5, col = lane & 31;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      f32x16 acc = {0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        bf16x8 a, b;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int n = 16 * ks + 8 * half + q;
          a[q] = __builtin_bit_cast(__bf16, A[n * LDS_PITCH + 32 * mt + col]);
          b[q] = __builtin_bit_cast(__bf16, B[n * LDS_PITCH + 32 * nt + col]);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) emit(32 * mt + d_row(r, lane), 32 * nt + col, acc[r]);
    }
}

__global__ __launch_bounds__(64) void grad_kernel(const Packed* __restrict__ P,
                                                  const float* __restrict__ x,
                                                  const float* __restrict__ y,
                                                  const int64_t* __restrict__ idx, int64_t batch,
                                                  float* __restrict__ gpart,
                                                  double* __restrict__ lpart) {
  __shared__ __attribute__((aligned(16))) uint16_t X[64 * LDS_PITCH], H1[64 * LDS_PITCH],
      H2[64 * LDS_PITCH], D0[64 * LDS_PITCH], D12[2 * 64 * LDS_PITCH];
  __shared__ float lsum[64];
  uint16_t* D1 = D12;
  uint16_t* D2 = D12 + 64 * LDS_PITCH;
  // the normalised targets live in D1/D2 until the output layer has used them
  float* yn = reinterpret_cast<float*>(D12);
  static_assert(sizeof(D12) >= 64 * N_OUT * sizeof(float), "target staging does not fit");
  const int lane = threadIdx.x;
  const int64_t s = (int64_t)blockIdx.x * 64 + lane;
  const bool live = s < batch;
  const int64_t row = live ? idx[s] : 0;
  const float inv_count = 1.0f / (float)(batch * N_OUT);
  {
    float xr[N_IN];
    for (int k = 0; k < N_IN; ++k) xr[k] = live ? x[row * N_IN + k] : 0.f;
    put_features(P, xr, X + lane * LDS_PITCH);
    for (int k = 0; k < N_OUT; ++k) yn[lane * N_OUT + k] = live ? y[row * N_OUT + k] / P->y_scale[k] : 0.f;
    for (int k = 0; k < LDS_PITCH; ++k) D0[lane * LDS_PITCH + k] = 0;
  }
  __syncthreads();
  // forward
  mfma_layer<N_HID, K_IN>(P->w1, P->b1, X, [&](int r, int n, float v) {
    H1[n * LDS_PITCH + r] = bf16_bits(tanhf(v));
  });
  __syncthreads();
  mfma_layer<N_HID, N_HID>(P->w2, P->b2, H1, [&](int r, int n, float v) {
    H2[n * LDS_PITCH + r] = bf16_bits(tanhf(v));
  });
  __syncthreads();
  float lacc = 0.f;
  // output layer and dL/do = 2 (o - y) / (batch * 41); padded samples contribute nothing
  mfma_layer<M_OUT, N_HID>(P->w3, P->b3, H2, [&](int r, int n, float v) {
    if (r < N_OUT && (int64_t)blockIdx.x * 64 + n < batch) {
      const float d = v - yn[n * N_OUT + r];
      lacc += d * d;
      D0[n * LDS_PITCH + r] = bf16_bits(2.f * d * inv_count);
    }
  });
  lsum[lane] = lacc;
  __syncthreads();
  // back through the hidden layers (transposed weights), tanh' = 1 - h^2
  mfma_layer<N_HID, M_OUT>(P->w3t, P->zero, D0, [&](int r, int n, float v) {
    const float h = bf16_float(H2[n * LDS_PITCH + r]);
    D1[n * LDS_PITCH + r] = bf16_bits(v * (1.f - h * h));
  });
  __syncthreads();
  mfma_layer<N_HID, N_HID>(P->w2t, P->zero, D1, [&](int r, int n, float v) {
    const float h = bf16_float(H1[n * LDS_PITCH + r]);
    D2[n * LDS_PITCH + r] = bf16_bits(v * (1.f - h * h));
  });
  __syncthreads();
  // weight gradients: sums over the block's samples of outer products
  float* g = gpart + (int64_t)blockIdx.x * N_PARAMS;
  float* gW1 = g;
  float* gb1 = gW1 + N_HID * N_IN;
  float* gW2 = gb1 + N_HID;
  float* gb2 = gW2 + N_HID * N_HID;
  float* gW3 = gb2 + N_HID;
  float* gb3 = gW3 + N_OUT * N_HID;
  outer_over_nodes(D2, X, [&](int i, int j, float v) { if (j < N_IN) gW1[i * N_IN + j] = v; });
  outer_over_nodes(D1, H1, [&](int i, int j, float v) { gW2[i * N_HID + j] = v; });
  outer_over_nodes(D0, H2, [&](int i, int j, float v) { if (i < N_OUT) gW3[i * N_HID + j] = v; });
  {
    float a = 0.f, b = 0.f, c = 0.f;
    for (int n = 0; n < 64; ++n) {
      a += bf16_float(D2[n * LDS_PITCH + lane]);
      b += bf16_float(D1[n * LDS_PITCH + lane]);
      c += bf16_float(D0[n * LDS_PITCH + lane]);
    }
    gb1[lane] = a;
    gb2[lane] = b;
    if (lane < N_OUT) gb3[lane] = c;
  }
  if (lane == 0) {
    double t = 0.0;
    for (int n = 0; n < 64; ++n) t += (double)lsum[n];
    lpart[blockIdx.x] = t;
  }
}

// Fixed-order sums of the per-block partials: the gradient and the batch loss.
__global__ __launch_bounds__(256) void grad_reduce_kernel(const float* __restrict__ gpart,
                                                          const double* __restrict__ lpart,
                                                          int64_t nblocks, int64_t batch,
                                                          float* __restrict__ grad,
                                                          double* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < N_PARAMS) {
    double s = 0.0;
    for (int64_t b = 0; b < nblocks; ++b) s += (double)gpart[b * N_PARAMS + p];
    grad[p] = (float)s;
  }
  if (p == 0 && loss) {
    double s = 0.0;
    for (int64_t b = 0; b < nblocks; ++b) s += lpart[b];
    *loss = s / ((double)batch * N_OUT);
  }
}

// Adam (Kingma & Ba 2015); c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ theta, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ grad,
                                                   float lr, float beta1, float beta2, float omb1,
                                                   float omb2, float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N_PARAMS) return;
  const float gr = grad[p];
  const float mm = beta1 * m[p] + omb1 * gr;
  const float vv = beta2 * v[p] + omb2 * gr * gr;
  m[p] = mm;
  v[p] = vv;
  theta[p] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
}

// ---------------------------------------------------------------------------
// normalisation: column means / variances of the features and mean squares of
// the targets over all rows, two-stage FP64
// ---------------------------------------------------------------------------
constexpr int NSTAT = 2 * N_IN + N_OUT;    // sum x, sum x^2, sum y^2

__global__ __launch_bounds__(256) void stats_kernel(const float* __restrict__ x,
                                                    const float* __restrict__ y, int64_t rows,
                                                    double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t chunk = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * chunk, r1 = min(rows, r0 + chunk);
  for (int c = 0; c < NSTAT; ++c) {
    double s = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
      if (c < N_IN) s += (double)x[r * N_IN + c];
      else if (c < 2 * N_IN) { const double v = x[r * N_IN + c - N_IN]; s += v * v; }
      else { const double v = y[r * N_OUT + c - 2 * N_IN]; s += v * v; }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * NSTAT + c] = red[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void norm_kernel(const double* __restrict__ part, int nblocks,
                                                   int64_t rows, float* __restrict__ norm) {
  const int c = threadIdx.x;
  if (c >= N_IN + N_OUT) return;
  if (c < N_IN) {
    double s = 0.0, s2 = 0.0;
    for (int b = 0; b < nblocks; ++b) { s += part[b * NSTAT + c]; s2 += part[b * NSTAT + N_IN + c]; }
    const double mean = s / rows;
    const double var = s2 / rows - mean * mean;
    norm[c] = (float)mean;
    norm[N_IN + c] = var > 1e-300 ? (float)(1.0 / sqrt(var)) : 0.f;
  } else {
    const int k = c - N_IN;
    double s2 = 0.0;
    for (int b = 0; b < nblocks; ++b) s2 += part[b * NSTAT + 2 * N_IN + k];
    const double ms = s2 / rows;
    norm[2 * N_IN + k] = ms > 1e-300 ? (float)sqrt(ms) : 1.f;
  }
}

// ---------------------------------------------------------------------------
// restriction of a fine D3Q27 x D3Q19 state to the coarse grid (ratio 4)
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(256) void restrict_kernel(const T* __restrict__ fine, Geometry gf,
                                                       PhysConsts cf, int nc, float sf, float sg,
                                                       float* __restrict__ out) {
  const int64_t nc3 = (int64_t)nc * nc * nc;
  const int64_t J = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= nc3) return;
  const int X = (int)(J % nc), Y = (int)((J / nc) % nc), Z = (int)(J / ((int64_t)nc * nc));
  const int n = gf.n;
  auto wf = [](int d) { return (d == -2 || d == 2) ? 0.125f : 0.25f; };   // [1,2,2,2,1] / 8
  float fb[27] = {0}, gb[19] = {0}, fn[27] = {0}, gn[19] = {0};
  for (int dz = -2; dz <= 2; ++dz)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        const int x = (4 * X + dx + n) % n, y = (4 * Y + dy + n) % n, z = (4 * Z + dz + n) % n;
        const float w = wf(dx) * wf(dy) * wf(dz);
        const NodeIndex ix = make_index(x, y, z, n);
        float f[27], g[19];
        gather<27, T, MODE>(f, fine, 0, ix, gf.stride);
        gather<19, T, MODE>(g, fine, 27, ix, gf.stride);
        NodeMacro<float> m;
        node_macro<27, 19, FORCE_GUO>(f, g, cf, m);
        m.vx = m.ux; m.vy = m.uy; m.vz = m.uz;           // equilibria at the physical velocity
        const Collision<27, 19, FORCE_GUO, float> col(cf, m);
#pragma unroll
        for (int i = 0; i < 27; ++i) { fb[i] += w * f[i]; fn[i] += w * (f[i] - col.feq(i)); }
#pragma unroll
        for (int j = 0; j < 19; ++j) { gb[j] += w * g[j]; gn[j] += w * (g[j] - col.geq(j)); }
      }
  // non-conserved moments of the filtered non-equilibrium part, rescaled by (s - 1)
  float mf[27], mg[19];
#pragma unroll
  for (int k = 0; k < 27; ++k) mf[k] = k < NCF ? 0.f : (sf - 1.f) * moment<27>(k, fn);
#pragma unroll
  for (int k = 0; k < 19; ++k) mg[k] = k < NCG ? 0.f : (sg - 1.f) * moment<19>(k, gn);
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    float a = fb[i];
#pragma unroll
    for (int k = NCF; k < 27; ++k)
      if (MINV_F.v[i][k] != 0.f) a += MINV_F.v[i][k] * mf[k];
    out[i * nc3 + J] = a;
  }
#pragma unroll
  for (int j = 0; j < 19; ++j) {
    float a = gb[j];
#pragma unroll
    for (int k = NCG; k < 19; ++k)
      if (MINV_G.v[j][k] != 0.f) a += MINV_G.v[j][k] * mg[k];
    out[(27 + j) * nc3 + J] = a;
  }
}

// ---------------------------------------------------------------------------
// training pairs on the coarse grid: features of state a; targets from the
// residual b - c (b: restricted fine state one coarse step later, c: the
// coarse step of a), returned to the source node and projected on the
// non-conserved moments.  a, b, c: natural-order FP32 deviations.
// ---------------------------------------------------------------------------
template <int FORCE>
__global__ __launch_bounds__(256) void pairs_kernel(const float* __restrict__ a,
                                                    const float* __restrict__ b,
                                                    const float* __restrict__ c, int nc,
                                                    PhysConsts pc, float* __restrict__ xo,
                                                    float* __restrict__ yo) {
  using SF = Stencil<27>;
  using SG = Stencil<19>;
  const int64_t nc3 = (int64_t)nc * nc * nc;
  const int64_t J = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= nc3) return;
  const int X = (int)(J % nc), Y = (int)((J / nc) % nc), Z = (int)(J / ((int64_t)nc * nc));
  const NodeIndex ix = make_index(X, Y, Z, nc);
  float f[27], g[19];
#pragma unroll
  for (int i = 0; i < 27; ++i) f[i] = a[i * nc3 + J];
#pragma unroll
  for (int j = 0; j < 19; ++j) g[j] = a[(27 + j) * nc3 + J];
  NodeMacro<float> m;
  node_macro<27, 19, FORCE>(f, g, pc, m);
  const Collision<27, 19, FORCE, float> col(pc, m);
  col.relaxation_increments(f, g);       // f <- f^eq - f, g <- g^eq - g
  float* xr = xo + J * N_IN;
  node_features<FORCE>(f, g, m, (float)pc.tau_f, [&](int k, float v) { xr[k] = v; });
  float rf[27], rg[19];
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const uint32_t o = ix.at(SF::ex[i], SF::ey[i], SF::ez[i]);
    rf[i] = b[i * nc3 + o] - c[i * nc3 + o];
  }
#pragma unroll
  for (int j = 0; j < 19; ++j) {
    const uint32_t o = ix.at(SG::ex[j], SG::ey[j], SG::ez[j]);
    rg[j] = b[(27 + j) * nc3 + o] - c[(27 + j) * nc3 + o];
  }
  float* yr = yo + J * N_OUT;
#pragma unroll
  for (int k = NCF; k < 27; ++k) yr[k - NCF] = moment<27>(k, rf);
#pragma unroll
  for (int k = NCG; k < 19; ++k) yr[27 - NCF + k - NCG] = moment<19>(k, rg);
}

}  // namespace mlp

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t mlp_launch_pack(const float* theta, const float* norm, void* packed, hipStream_t st) {
  hipLaunchKernelGGL(mlp::pack_kernel, dim3(1), dim3(256), 0, st, theta, norm, (mlp::Packed*)packed);
  return hipGetLastError();
}

hipError_t mlp_launch_forward(const void* packed, const float* x, int64_t rows, float* y, hipStream_t st) {
  const int64_t blocks = (rows + 63) / 64;
  hipLaunchKernelGGL(mlp::forward_kernel, dim3((unsigned)blocks), dim3(64), 0, st,
                     (const mlp::Packed*)packed, x, rows, y);
  return hipGetLastError();
}

hipError_t mlp_launch_grad(const void* packed, const float* x, const float* y, const int64_t* idx,
                           int64_t batch, float* gpart, double* lpart, float* grad, double* loss,
                           hipStream_t st) {
  const int64_t blocks = (batch + 63) / 64;
  hipLaunchKernelGGL(mlp::grad_kernel, dim3((unsigned)blocks), dim3(64), 0, st,
                     (const mlp::Packed*)packed, x, y, idx, batch, gpart, lpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp::grad_reduce_kernel, dim3((mlp::N_PARAMS + 255) / 256), dim3(256), 0, st,
                     gpart, lpart, blocks, batch, grad, loss);
  return hipGetLastError();
}

hipError_t mlp_launch_adam(float* theta, float* m, float* v, const float* grad, float lr, float b1,
                           float b2, float omb1, float omb2, float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(mlp::adam_kernel, dim3((mlp::N_PARAMS + 255) / 256), dim3(256), 0, st, theta,
                     m, v, grad, lr, b1, b2, omb1, omb2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_launch_norm(const float* x, const float* y, int64_t rows, double* part, int nblocks,
                           float* norm, hipStream_t st) {
  hipLaunchKernelGGL(mlp::stats_kernel, dim3(nblocks), dim3(256), 0, st, x, y, rows, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp::norm_kernel, dim3(1), dim3(256), 0, st, part, nblocks, rows, norm);
  return hipGetLastError();
}

template <typename T>
static hipError_t restrict_t(const void* fine, int mode, Geometry gf, PhysConsts cf, int nc, float sf,
                             float sg, float* out, hipStream_t st) {
  const int64_t nc3 = (int64_t)nc * nc * nc;
  const dim3 grid((unsigned)((nc3 + 255) / 256));
  if (mode == MODE_ODD)
    hipLaunchKernelGGL((mlp::restrict_kernel<T, MODE_ODD>), grid, dim3(256), 0, st, (const T*)fine, gf, cf, nc, sf, sg, out);
  else
    hipLaunchKernelGGL((mlp::restrict_kernel<T, MODE_EVEN>), grid, dim3(256), 0, st, (const T*)fine, gf, cf, nc, sf, sg, out);
  return hipGetLastError();
}

hipError_t mlp_launch_restrict(int storage, const void* fine, int mode, Geometry gf, PhysConsts cf,
                               int nc, float sf, float sg, float* out, hipStream_t st) {
  switch (storage) {
    case 0: return restrict_t<float>(fine, mode, gf, cf, nc, sf, sg, out, st);
    case 1: return restrict_t<_Float16>(fine, mode, gf, cf, nc, sf, sg, out, st);
    default: return restrict_t<bf16_t>(fine, mode, gf, cf, nc, sf, sg, out, st);
  }
}

hipError_t mlp_launch_pairs(int forcing, const float* a, const float* b, const float* c, int nc,
                            PhysConsts pc, float* x, float* y, hipStream_t st) {
  const int64_t nc3 = (int64_t)nc * nc * nc;
  const dim3 grid((unsigned)((nc3 + 255) / 256));
  if (forcing == FORCE_GUO)
    hipLaunchKernelGGL((mlp::pairs_kernel<FORCE_GUO>), grid, dim3(256), 0, st, a, b, c, nc, pc, x, y);
  else
    hipLaunchKernelGGL((mlp::pairs_kernel<FORCE_SHIFT>), grid, dim3(256), 0, st, a, b, c, nc, pc, x, y);
  return hipGetLastError();
}

}  // namespace stgv
