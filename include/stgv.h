/*
 * stgv.h - C ABI of the MI355X (gfx950) stratified Taylor-Green double-
 * distribution-function lattice Boltzmann step.
 *
 * The method is the paper's Section 2: a D3Q<q_f> momentum lattice f (LBE
 * Eq. (5), moments Eqs. (6)-(7), BGK Eq. (8), equilibrium Eq. (9)) coupled to a
 * D3Q<q_g> scalar lattice g for the density perturbation rho' (LBE Eq. (11),
 * source Eqs. (12)-(13), BGK Eq. (14), equilibrium Eq. (15), zeroth moment
 * Eqs. (16)-(17)) through the Boussinesq force F = (0, 0, -G rho') (Eq. (18)),
 * applied by the Guo source term or the Shan-Chen velocity shift (Eq. (10)),
 * on the periodic box [0, 2 pi)^3 (Section 2.4) with the Taylor-Green initial
 * state of Eqs. (20)-(21) and the energy / dissipation diagnostics of
 * Eqs. (22)-(26).  Stencils are those of Table 1.
 *
 * Conventions shared by every call:
 *  - Memory: the caller allocates and owns every device buffer and the HIP
 *    stream.  A context keeps non-owning pointers, which must stay valid until
 *    lbm_destroy.  lbm_destroy frees host memory only.
 *  - Errors: every int-returning call returns an lbm_status and never aborts
 *    or throws.  lbm_last_error(ctx) (or lbm_last_error(NULL) for calls that
 *    failed before a context existed) gives a message.  Parameter errors are
 *    reported before any device work is queued.
 *  - Streams: all device work is queued on the caller's stream, in order.
 *    lbm_diagnostics, lbm_read_fields, lbm_read_populations and
 *    lbm_load_populations synchronise that stream before they return.
 *  - Threading: one host thread per context at a time.
 *  - Determinism: identical parameters give bit-identical populations and
 *    diagnostics (fixed-order FP64 reductions, no atomics).  The spectrum of
 *    lbm_ke_spectrum bins with LDS atomics and is reproducible to rounding.
 *  - Units: lattice units (dx = dt = 1) inside; lbm_diag reports the paper's
 *    non-dimensional values (E / U^2, eps L / U^3, t = step U / L) with
 *    L = n / (2 pi) nodes per unit length and U = u0.
 */
#ifndef STGV_H
#define STGV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx; /* opaque, host side */

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* invalid parameter or argument (nothing was queued) */
  LBM_ESIZE = -2,     /* a buffer is smaller than lbm_query_sizes requires */
  LBM_EHIP = -3,      /* a HIP call failed; the message carries hipGetErrorString */
  LBM_EUNSTABLE = -4, /* a drained diagnostic record is non-finite or has max|u| > c_s */
  LBM_ESTATE = -5     /* call not valid in the current state (e.g. diagnostics ring full) */
} lbm_status;

typedef enum {
  LBM_FORCE_GUO = 0,   /* Guo-Zheng-Shi discrete source term (cited with Eq. (5)) */
  LBM_FORCE_SHIFT = 1, /* Shan-Chen velocity shift u_eq = u' + tau_f F / rho (Eq. (10)) */
  LBM_FORCE_EDM = 2,   /* exact difference method (Kupershtokh), compared in Section 3.6:
                          relax to f^eq(u'), add f^eq(u' + F/rho) - f^eq(u') */
  LBM_FORCE_HCZ = 3    /* He-Shan-Doolen source term, compared in Section 3.6: relax to
                          f^eq(u), add (1 - 1/2tau)(e - u).F/(rho c_s^2) f^eq(u) */
} lbm_forcing;

typedef enum {
  LBM_FP32 = 0,       /* populations stored as FP32 deviations f_i - w_i */
  LBM_FP16 = 1,       /* ... as IEEE half deviations, round-to-nearest-even */
  LBM_BF16 = 2        /* ... as bfloat16 deviations, round-to-nearest-even */
} lbm_storage;

typedef enum {
  LBM_COMPUTE_FP32 = 0, /* collision and forcing arithmetic in FP32 (every storage type) */
  LBM_COMPUTE_FP64 = 1  /* ... in FP64 (FP32 storage only) */
} lbm_compute;

typedef enum {
  LBM_LAYOUT_AA = 0,  /* one population array, AA in-place streaming */
  LBM_LAYOUT_AB = 1   /* two population arrays (push), for cross-checks */
} lbm_layout;

/* Problem statement (Section 2.4: Re_0 = U L / nu, Fr_0 = U / (N L), Sc = nu / D). */
typedef struct {
  int32_t n;           /* periodic box n^3 nodes, 4 <= n <= 1024 */
  int32_t q_f, q_g;    /* stencil pair D3Q{q_f} x D3Q{q_g} (Table 1 stencils): (27,19), (27,7),
                          (19,7), or one of the paper's other compared pairs (27,27), (19,19),
                          (19,15), (15,7), (7,27) */
  int32_t forcing;     /* lbm_forcing */
  int32_t storage;     /* lbm_storage */
  int32_t compute;     /* lbm_compute */
  int32_t layout;      /* lbm_layout */
  int32_t diag_every;  /* a diagnostic record every k steps (at steps 0, k, 2k, ...); 0 = none */
  int32_t pad;         /* extra elements between population arrays; < 0 = library default */
  int32_t reserved;    /* must be 0 */
  double u0;           /* Taylor-Green amplitude U in lattice units, 0 < u0 < 0.3 */
  double re;           /* Re_0 > 0 */
  double fr;           /* Fr_0 > 0; +inf = unstratified (G = 0) */
  double sc;           /* Sc > 0 (Pr for a thermal scalar) */
  double g_over_n;     /* G / N > 0: split of N^2 between G and d rho_b / dz (rho_0 = 1) */
  double noise_amp;    /* rho'(t=0) = A (2 xi - 1), xi uniform from SplitMix64; A >= 0 */
  uint64_t seed;       /* key of the noise: xi(node) = splitmix64(seed * 2^40 + x + n (y + n z)) */
} lbm_params;

/* One diagnostic record, in the paper's non-dimensional units. */
typedef struct {
  int64_t step;        /* time step the moments belong to (pre-collision state of that step) */
  double t;            /* step * U / L */
  double ek;           /* Eq. (22) / U^2 */
  double ep;           /* Eq. (23) / U^2 (0 when G = 0) */
  double eps_k;        /* Eq. (25) * L / U^3, central differences */
  double eps_p;        /* Eq. (26) * L / U^3 (0 when G = 0) */
  double mass;         /* sum over nodes of rho */
  double scalar;       /* sum over nodes and directions of g */
  double mom[3];       /* sum over nodes of rho u (lattice units) */
  double umax;         /* max |u| (lattice units) */
  int64_t nonfinite;   /* nodes with a non-finite rho, |u|^2 or rho' */
} lbm_diag;

/* Validate parameters and report the device bytes the caller must provide:
 * pop_bytes for the populations, work_bytes for fields, partial sums and the
 * diagnostics ring.  CPU only: touches no device.  Returns LBM_EINVAL with a
 * message for any invalid parameter. */
int lbm_query_sizes(const lbm_params* p, size_t* pop_bytes, size_t* work_bytes);

/* Derived lattice constants (Eqs. (8), (13), (14), (19)) as 8 doubles:
 * [L, nu, D, tau_f, tau_g, N, G, beta] with beta = (d rho_b/dz)_LU.  CPU only. */
int lbm_derived(const lbm_params* p, double* out8);

/* Create a context and queue the Taylor-Green initial state (Eqs. (20)-(21),
 * pure equilibrium, rho'(0) = seeded noise) on `hip_stream` (a hipStream_t,
 * NULL = default stream).  pop_dev / work_dev: device buffers of at least
 * lbm_query_sizes bytes, 256-byte aligned, owned by the caller.  On success
 * *out receives the context and the step counter is 0. */
int lbm_init_tgv(const lbm_params* p, void* pop_dev, size_t pop_bytes, void* work_dev,
                 size_t work_bytes, void* hip_stream, lbm_ctx** out);

/* Queue n >= 0 fused stream-collide-force steps.  A step whose index is a
 * multiple of diag_every also queues its diagnostic record.  Returns
 * LBM_ESTATE without queueing anything if the records would overflow the
 * ring (4096 records); drain it with lbm_diagnostics. */
int lbm_step(lbm_ctx* ctx, int64_t n);

/* Queue n >= 0 free-streaming steps: the streaming half of Eqs. (5) and (11)
 * alone (no collision, no force), with the step's own loads, stores, launch
 * shape, block order and resident-block caps.  Every population moves one
 * link along its velocity per step, exactly (values are moved, never
 * rounded), and the step counter and layout parity advance as in lbm_step.
 * Afterwards the state is no longer the method's; the call measures the
 * memory-access ceiling of the step and checks the streaming layout.  Queues
 * no diagnostics. */
int lbm_stream(lbm_ctx* ctx, int64_t n);

/* Queue a diagnostic record of the current state (without stepping). */
int lbm_sample(lbm_ctx* ctx);

/* Synchronise the stream and move up to `max` pending records, oldest first,
 * into out[0..*n_out).  Returns LBM_EUNSTABLE if any returned record is
 * non-finite or has max|u| above the lattice speed of sound. */
int lbm_diagnostics(lbm_ctx* ctx, lbm_diag* out, int32_t max, int32_t* n_out);

/* Write the current moments as five FP32 device arrays of n^3 values, x
 * fastest: rho - 1, u_x, u_y, u_z (physical velocity, Eq. (7)), rho'
 * (Eq. (16)).  dev_out must hold 5 n^3 floats.  Synchronises. */
int lbm_read_fields(lbm_ctx* ctx, float* dev_out);

/* Write the current pre-collision populations as FP32 deviations in natural
 * order: (q_f + q_g) arrays of n^3 values (f_i - w_i, then g_j - w^g_j),
 * whatever the layout and step parity.  Synchronises. */
int lbm_read_populations(lbm_ctx* ctx, float* dev_out);

/* Replace the state by the populations in dev_in (same layout as
 * lbm_read_populations, rounded to the storage type) and set the step
 * counter to `step`.  Synchronises. */
int lbm_load_populations(lbm_ctx* ctx, const float* dev_in, int64_t step);

/* Velocity set of D3Q{q}, q in {7, 15, 19, 27} (Table 1, in this library's
 * order): e[3 q] as (x, y, z) triples, w[q], *cs2.  CPU only. */
int lbm_stencil_info(int32_t q, int32_t* e, double* w, double* cs2);

/* Streaming-bandwidth probe: kind 0 copies `bytes` from src to dst, kind 1
 * reads src (writes one float per 16 KiB of src to dst), kind 2 writes dst.
 * Queued on hip_stream; bytes must be a multiple of 16. */
int lbm_bw_probe(int32_t kind, void* dst, const void* src, size_t bytes, void* hip_stream);

/* ------------------------------------------------------------------------
 * Learned correction of a coarse D3Q27 x D3Q19 run (this library's extension of
 * the method; not in the paper).  A per-node network maps 47 features (the
 * non-equilibrium moments M (f - f^eq), M (g - g^eq) in the monomial basis
 * e_x^a e_y^b e_z^c, a, b, c in {0, 1, 2}, and rho') to corrections dm of the 41
 * non-conserved moments; the post-collision populations gain M^-1 [0, dm], which
 * leaves mass, momentum and the scalar untouched.  Network 47 -> 64 -> 64 -> 41,
 * tanh, BF16 MFMA with FP32 accumulation.
 *
 * Parameters ("params", LBM_MLP_PARAMS FP32 on the device, the master copy):
 * W1 [64][47], b1 [64], W2 [64][64], b2 [64], W3 [41][64], b3 [41], row-major.
 * Normalisation ("norm", 135 FP32): x_mean [47], x_iscale [47], y_scale [41];
 * the network sees (x - x_mean) * x_iscale and its output times y_scale is dm.
 * Feature rows are [rows][47] FP32, target rows [rows][41] FP32.  All buffers
 * are caller-owned device memory; work is queued on hip_stream.
 * ------------------------------------------------------------------------ */
enum { LBM_MLP_IN = 47, LBM_MLP_HIDDEN = 64, LBM_MLP_OUT = 41, LBM_MLP_PARAMS = 9897,
       LBM_MLP_NORM = 135 };

/* Bytes of the packed network (BF16 weight tiles, FP32 biases and normalisation). */
size_t lbm_mlp_packed_bytes(void);

/* Pack params + norm into packed_dev (>= lbm_mlp_packed_bytes(), 16-byte aligned). */
int lbm_mlp_pack(const float* params_dev, const float* norm_dev, void* packed_dev, void* hip_stream);

/* dm for `rows` feature rows (de-normalised network output). */
int lbm_mlp_forward(const void* packed_dev, const float* x_dev, int64_t rows, float* y_dev,
                    void* hip_stream);

/* Work bytes of lbm_mlp_grad for a batch. */
size_t lbm_mlp_grad_work_bytes(int64_t batch);

/* Gradient (LBM_MLP_PARAMS FP32, parameter order) and loss (one FP64) of the mean
 * squared error between the normalised output and y / y_scale over the batch
 * rows idx_dev[0..batch) of x_dev / y_dev.  Deterministic (fixed-order sums). */
int lbm_mlp_grad(const void* packed_dev, const float* x_dev, const float* y_dev,
                 const int64_t* idx_dev, int64_t batch, float* grad_dev, double* loss_dev,
                 void* work_dev, size_t work_bytes, void* hip_stream);

/* lbm_mlp_grad for callers that cannot allocate (code under HIP graph capture, tight
 * training loops, hosts that forbid hipMalloc): the same kernels and the same result,
 * bit for bit, with the per-block partial sums in a device array built into the
 * library (about 10 MB per GPU, held until the process ends) instead of a workspace.
 * batch <= LBM_MLP_STATIC_MAX_BATCH, else LBM_ESIZE before any device work.  Runs on
 * the current device (the one hip_stream and the buffers belong to); allocates
 * nothing.  Calls that overlap on one GPU (other streams or host threads) share the
 * array and race: serialise them. */
#define LBM_MLP_STATIC_MAX_BATCH 16384
int lbm_mlp_grad_static(const void* packed_dev, const float* x_dev, const float* y_dev,
                        const int64_t* idx_dev, int64_t batch, float* grad_dev, double* loss_dev,
                        void* hip_stream);

/* One Adam step (Kingma & Ba; beta1 0.9, beta2 0.999, eps 1e-8) at step t >= 1 on
 * params / m / v (FP32, LBM_MLP_PARAMS each). */
int lbm_mlp_adam(float* params_dev, float* m_dev, float* v_dev, const float* grad_dev, int64_t t,
                 double lr, void* hip_stream);

/* Normalisation from data: x_mean, x_iscale = 1 / std (0 for a constant
 * column), y_scale = root mean square (1 if zero), over `rows` rows. */
size_t lbm_mlp_norm_work_bytes(void);
int lbm_mlp_norm(const float* x_dev, const float* y_dev, int64_t rows, float* norm_dev,
                 void* work_dev, size_t work_bytes, void* hip_stream);

/* Restrict the current state of a fine D3Q27 x D3Q19 context to the grid of a
 * coarse one (fine n = 4 coarse n): separable [1,2,2,2,1]/8 filter sampled at
 * every 4th node, non-conserved filtered non-equilibrium moments rescaled by
 * 4 tau_coarse / tau_fine (Guo or velocity-shift contexts).  coarse_dev: (q_f + q_g) n_c^3 FP32 deviations in the
 * layout of lbm_read_populations.  Queued on the fine context's stream. */
int lbm_restrict(lbm_ctx* fine, const lbm_ctx* coarse, float* coarse_dev);

/* Training pairs on a coarse grid: features x_dev [n^3][47] of state a_dev and
 * targets y_dev [n^3][41]: the non-conserved moments of (b - c) returned to the
 * node each population streamed from, where b is the restricted fine state one
 * coarse step later and c the coarse step of a (all in the layout of
 * lbm_read_populations).  Queued on the context's stream. */
int lbm_training_pairs(lbm_ctx* coarse, const float* a_dev, const float* b_dev, const float* c_dev,
                       float* x_dev, float* y_dev);

/* Attach (or, with NULL, detach) a packed network to a D3Q27 x D3Q19 context
 * with Guo or velocity-shift forcing, FP32 storage and arithmetic, n % 64 == 0 and n <= 256
 * (a coarse grid: 64^3 to 256^3); later lbm_step calls run the fused learned step.
 * packed_dev must stay valid while attached.  Returns LBM_EINVAL otherwise. */
int lbm_set_mlp(lbm_ctx* ctx, const void* packed_dev);

/* ------------------------------------------------------------------------
 * Post-processing (Sections 3.4-3.5): the quantities derived from the diagnostic
 * histories and the kinetic-energy spectrum.  Physical units (U = L = 1 on the
 * 2 pi box): nu = 1/Re, N = 1/Fr.
 * ------------------------------------------------------------------------ */
typedef struct {
  double gamma_b;      /* bulk flux coefficient int eps_p dt / int eps_k dt over [0, t_end] */
  double fr_t;         /* turbulent Froude number int eps_k dt / (N int E_k dt) over [0, t_end] */
  double r_max;        /* largest buoyancy Reynolds number eps_k / (nu N^2) among the records */
  double t_r_max;      /* its time */
  int32_t used;        /* records with t <= t_end entering the integrals */
  int32_t reserved;
} lbm_post;

/* From `count` >= 2 records with increasing t: per-record buoyancy Reynolds
 * number R = eps_k / (nu N^2) into r_out and flux coefficient Gamma = eps_p /
 * eps_k into gamma_out (either may be NULL), and the bulk quantities into *out;
 * integrals are trapezoid sums over the records with t <= t_end.  fr may be
 * +inf (N = 0: R and Fr_t are +inf).  Host memory only, CPU only.  LBM_EINVAL
 * for a bad argument or non-increasing times. */
int lbm_postprocess(const lbm_diag* recs, int32_t count, double re, double fr, double t_end,
                    double* r_out, double* gamma_out, lbm_post* out);

/* Number of spectral shells for an n^3 box: k = 0 .. round(sqrt(3) n / 2), or -1
 * for n outside [4, 1024]. */
int32_t lbm_spectrum_shells(int32_t n);

/* Device work bytes of lbm_ke_spectrum for an n^3 box (velocity fields, the FFT's
 * complex output and work space, per-block partial sums).  Creates and caches the
 * rocFFT plan for n, so it needs the GPU; LBM_EHIP if rocFFT fails. */
int lbm_spectrum_work_bytes(int32_t n, size_t* bytes);

/* Kinetic-energy spectrum of the current state, E(k) = sum over wavevectors with
 * round(|k|) = k of |u_hat|^2 / 2, u_hat = FFT(u / U) / n^3 (u of Eq. (7)), so that
 * sum_k E(k) = E_k.  shells_dev: lbm_spectrum_shells(n) FP64 values (device); work:
 * lbm_spectrum_work_bytes bytes (device, 256-byte aligned), both caller-owned.
 * Queued on the context's stream (the result is valid after it synchronises). */
int lbm_ke_spectrum(lbm_ctx* ctx, void* work_dev, size_t work_bytes, double* shells_dev);

int64_t lbm_get_step(const lbm_ctx* ctx);
const char* lbm_last_error(const lbm_ctx* ctx);
const char* lbm_status_string(int status);
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* STGV_H */
