// stgv_run: a stratified Taylor-Green run through the C ABI alone (no Python, no torch).
//
//   stgv_run [--n 128] [--qf 27] [--qg 19] [--forcing shift|guo|edm|hcz]
//            [--storage fp32|fp16|bf16] [--compute fp32|fp64] [--layout aa|ab]
//            [--re 1600] [--fr 1] [--sc 0.7] [--u0 0.05] [--gn 0.02] [--noise 1e-6]
//            [--seed 0] [--steps 1000] [--diag 50] [--spectrum FILE]
//            [--checkpoint FILE] [--resume FILE] [--mlp FILE]
//
// Allocates the population and work buffers with hipMalloc, queues the initial state
// and the steps, drains the diagnostic records (printed as CSV: step, t, E_k, E_p,
// eps_k, eps_p, mass, max|u|) and reports the run's MLUPS from HIP events.  With two
// or more records it also prints the post-processing of Sections 3.4-3.5 over the whole run
// (bulk flux coefficient, turbulent Froude number, peak buoyancy Reynolds number);
// --spectrum writes the kinetic-energy spectrum of the final state (k, E(k) per line).
// --checkpoint writes the final state (header + the FP32 populations of
// lbm_read_populations) and --resume continues from such a file for --steps more
// steps; a resumed run reproduces the uninterrupted one bit for bit.  --mlp attaches a
// trained network (the raw file `python -m paper_2605_14505_amd.learned --export`
// writes), so the steps are the fused learned step.
// Exit status: 0 on success, 2 for bad arguments (a resume file that is not a
// checkpoint of the run's box included), 1 for a library or HIP error.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/stgv.h"

namespace {

void usage() {
  std::fprintf(stderr,
               "usage: stgv_run [--n N] [--qf Q] [--qg Q] [--forcing shift|guo|edm|hcz]\n"
               "                [--storage fp32|fp16|bf16] [--compute fp32|fp64] [--layout aa|ab]\n"
               "                [--re RE] [--fr FR] [--sc SC] [--u0 U0] [--gn G/N] [--noise A]\n"
               "                [--seed S] [--steps K] [--diag D] [--spectrum FILE]\n"
               "                [--checkpoint FILE] [--resume FILE] [--mlp FILE]\n");
}

bool pick(const char* v, const char* const* names, int count, int32_t* out) {
  for (int i = 0; i < count; ++i)
    if (std::strcmp(v, names[i]) == 0) { *out = i; return true; }
  return false;
}

int fail(const char* what, int status, const lbm_ctx* ctx) {
  std::fprintf(stderr, "stgv_run: %s: %s (%s)\n", what, lbm_status_string(status), lbm_last_error(ctx));
  return 1;
}

// The kinetic-energy spectrum of the current state into `path` (k, E(k) per line).
int write_spectrum(lbm_ctx* ctx, int n, const char* path) {
  const int32_t shells = lbm_spectrum_shells(n);
  size_t work_bytes = 0;
  int st = lbm_spectrum_work_bytes(n, &work_bytes);
  if (st != LBM_OK) return fail("spectrum work size", st, nullptr);
  void *work = nullptr, *dev = nullptr;
  if (hipMalloc(&work, work_bytes) != hipSuccess || hipMalloc(&dev, (size_t)shells * sizeof(double)) != hipSuccess) {
    std::fprintf(stderr, "stgv_run: hipMalloc for the spectrum failed\n");
    return 1;
  }
  int rc = 0;
  std::vector<double> e((size_t)shells);
  st = lbm_ke_spectrum(ctx, work, work_bytes, static_cast<double*>(dev));
  if (st != LBM_OK) {
    rc = fail("spectrum", st, ctx);
  } else if (hipMemcpy(e.data(), dev, e.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    std::fprintf(stderr, "stgv_run: copying the spectrum failed\n");
    rc = 1;
  } else {
    FILE* f = std::fopen(path, "w");
    if (!f) {
      std::fprintf(stderr, "stgv_run: cannot write %s\n", path);
      rc = 1;
    } else {
      for (int32_t k = 0; k < shells; ++k) std::fprintf(f, "%d %.12e\n", k, e[(size_t)k]);
      std::fclose(f);
    }
  }
  (void)hipFree(work);
  (void)hipFree(dev);
  return rc;
}

// Checkpoint file: this header, then (q_f + q_g) n^3 FP32 population deviations in the
// order of lbm_read_populations.  The header keeps the run's whole parameter set, so a
// resume with another box, stencil pair, forcing, storage, arithmetic, layout or physics
// is refused (the diagnostic cadence and the array padding may change).
struct CkptHeader {
  char magic[8];       // "STGVCKP2"
  lbm_params params;
  int64_t step;
};
constexpr char kMagic[8] = {'S', 'T', 'G', 'V', 'C', 'K', 'P', '2'};

// The first parameter in which a checkpoint's run differs from this one, or nullptr.
const char* params_mismatch(const lbm_params& a, const lbm_params& b) {
  if (a.n != b.n) return "box size";
  if (a.q_f != b.q_f || a.q_g != b.q_g) return "stencil pair";
  if (a.forcing != b.forcing) return "forcing";
  if (a.storage != b.storage) return "storage";
  if (a.compute != b.compute) return "arithmetic";
  if (a.layout != b.layout) return "layout";
  if (a.u0 != b.u0) return "u0";
  if (a.re != b.re) return "Re";
  if (a.fr != b.fr) return "Fr";
  if (a.sc != b.sc) return "Sc";
  if (a.g_over_n != b.g_over_n) return "G/N";
  if (a.noise_amp != b.noise_amp || a.seed != b.seed) return "initial noise";
  return nullptr;
}

int save_state(lbm_ctx* ctx, const lbm_params& p, const char* path) {
  const size_t count = (size_t)(p.q_f + p.q_g) * p.n * p.n * p.n;
  void* dev = nullptr;
  if (hipMalloc(&dev, count * sizeof(float)) != hipSuccess) {
    std::fprintf(stderr, "stgv_run: hipMalloc for the checkpoint failed\n");
    return 1;
  }
  std::vector<float> host(count);
  int rc = 0;
  const int st = lbm_read_populations(ctx, static_cast<float*>(dev));
  if (st != LBM_OK) {
    rc = fail("reading the populations", st, ctx);
  } else if (hipMemcpy(host.data(), dev, count * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
    std::fprintf(stderr, "stgv_run: copying the populations failed\n");
    rc = 1;
  } else {
    CkptHeader hd{};
    std::memcpy(hd.magic, kMagic, sizeof(kMagic));
    hd.params = p;
    hd.step = lbm_get_step(ctx);
    FILE* f = std::fopen(path, "wb");
    if (!f || std::fwrite(&hd, sizeof(hd), 1, f) != 1 || std::fwrite(host.data(), sizeof(float), count, f) != count) {
      std::fprintf(stderr, "stgv_run: cannot write %s\n", path);
      rc = 1;
    }
    if (f) std::fclose(f);
  }
  (void)hipFree(dev);
  return rc;
}

// Read a checkpoint of this run's box and stencils into host memory (before any GPU
// work, so that a wrong file is an argument error); returns 0 or prints why not.
int read_checkpoint(const lbm_params& p, const char* path, std::vector<float>& host, int64_t& step) {
  FILE* f = std::fopen(path, "rb");
  if (!f) { std::fprintf(stderr, "stgv_run: cannot read %s\n", path); return 2; }
  CkptHeader hd{};
  const size_t count = (size_t)(p.q_f + p.q_g) * p.n * p.n * p.n;
  host.resize(count);
  const bool head = std::fread(&hd, sizeof(hd), 1, f) == 1 && std::memcmp(hd.magic, kMagic, sizeof(kMagic)) == 0 &&
                   hd.step >= 0;
  const char* differs = head ? params_mismatch(hd.params, p) : nullptr;
  const bool ok = head && !differs && std::fread(host.data(), sizeof(float), count, f) == count;
  std::fclose(f);
  if (!ok) {
    if (differs)
      std::fprintf(stderr, "stgv_run: %s is a checkpoint of another run (its %s differs)\n", path, differs);
    else
      std::fprintf(stderr, "stgv_run: %s is not a checkpoint of a %d^3 D3Q%dxD3Q%d run\n", path, p.n, p.q_f, p.q_g);
    return 2;
  }
  step = hd.step;
  return 0;
}

int load_state(lbm_ctx* ctx, const std::vector<float>& host, int64_t step) {
  void* dev = nullptr;
  if (hipMalloc(&dev, host.size() * sizeof(float)) != hipSuccess) {
    std::fprintf(stderr, "stgv_run: hipMalloc for the checkpoint failed\n");
    return 1;
  }
  int rc = 0;
  if (hipMemcpy(dev, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    std::fprintf(stderr, "stgv_run: copying the populations failed\n");
    rc = 1;
  } else {
    const int st = lbm_load_populations(ctx, static_cast<const float*>(dev), step);
    if (st != LBM_OK) rc = fail("loading the populations", st, ctx);
  }
  (void)hipFree(dev);
  return rc;
}

// A network file: "STGVMLP1", int32 parameter and normalisation counts, then the FP32
// master parameters and normalisation in the layout lbm_mlp_pack reads.
int read_network(const char* path, std::vector<float>& params, std::vector<float>& norm) {
  FILE* f = std::fopen(path, "rb");
  if (!f) { std::fprintf(stderr, "stgv_run: cannot read %s\n", path); return 2; }
  char magic[8] = {0};
  int32_t counts[2] = {0, 0};
  params.resize(LBM_MLP_PARAMS);
  norm.resize(LBM_MLP_NORM);
  const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "STGVMLP1", 8) == 0 &&
                  std::fread(counts, sizeof(int32_t), 2, f) == 2 && counts[0] == LBM_MLP_PARAMS &&
                  counts[1] == LBM_MLP_NORM &&
                  std::fread(params.data(), sizeof(float), params.size(), f) == params.size() &&
                  std::fread(norm.data(), sizeof(float), norm.size(), f) == norm.size();
  std::fclose(f);
  if (!ok) { std::fprintf(stderr, "stgv_run: %s is not a network file\n", path); return 2; }
  return 0;
}

// Pack the network on the device and attach it; *packed stays allocated while attached.
int attach_network(lbm_ctx* ctx, hipStream_t stream, const std::vector<float>& params,
                   const std::vector<float>& norm, void** packed) {
  void *dp = nullptr, *dn = nullptr;
  if (hipMalloc(&dp, params.size() * sizeof(float)) != hipSuccess ||
      hipMalloc(&dn, norm.size() * sizeof(float)) != hipSuccess ||
      hipMalloc(packed, lbm_mlp_packed_bytes()) != hipSuccess) {
    std::fprintf(stderr, "stgv_run: hipMalloc for the network failed\n");
    return 1;
  }
  int rc = 0;
  if (hipMemcpy(dp, params.data(), params.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dn, norm.data(), norm.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    std::fprintf(stderr, "stgv_run: copying the network failed\n");
    rc = 1;
  } else {
    int st = lbm_mlp_pack(static_cast<const float*>(dp), static_cast<const float*>(dn), *packed, stream);
    if (st == LBM_OK && hipStreamSynchronize(stream) != hipSuccess) st = LBM_EHIP;
    if (st != LBM_OK) rc = fail("packing the network", st, nullptr);
    else if ((st = lbm_set_mlp(ctx, *packed)) != LBM_OK) rc = fail("attaching the network", st, ctx);
  }
  (void)hipFree(dp);
  (void)hipFree(dn);
  return rc;
}

}  // namespace

int main(int argc, char** argv) {
  lbm_params p{};
  p.n = 128; p.q_f = 27; p.q_g = 19; p.forcing = LBM_FORCE_SHIFT; p.storage = LBM_FP32;
  p.compute = LBM_COMPUTE_FP32; p.layout = LBM_LAYOUT_AA; p.diag_every = 50; p.pad = -1;
  p.u0 = 0.05; p.re = 1600.0; p.fr = 1.0; p.sc = 0.7; p.g_over_n = 0.02; p.noise_amp = 1e-6; p.seed = 0;
  long long steps = 1000;
  const char* spectrum_path = nullptr;
  const char* checkpoint_path = nullptr;
  const char* resume_path = nullptr;
  const char* mlp_path = nullptr;
  static const char* const forcings[] = {"guo", "shift", "edm", "hcz"};
  static const char* const storages[] = {"fp32", "fp16", "bf16"};
  static const char* const computes[] = {"fp32", "fp64"};
  static const char* const layouts[] = {"aa", "ab"};
  for (int i = 1; i < argc; ++i) {
    const std::string a = argv[i];
    if (a == "--help" || a == "-h") { usage(); return 0; }
    if (i + 1 >= argc) { usage(); return 2; }
    const char* v = argv[++i];
    bool ok = true;
    if (a == "--n") p.n = std::atoi(v);
    else if (a == "--qf") p.q_f = std::atoi(v);
    else if (a == "--qg") p.q_g = std::atoi(v);
    else if (a == "--forcing") ok = pick(v, forcings, 4, &p.forcing);
    else if (a == "--storage") ok = pick(v, storages, 3, &p.storage);
    else if (a == "--compute") ok = pick(v, computes, 2, &p.compute);
    else if (a == "--layout") ok = pick(v, layouts, 2, &p.layout);
    else if (a == "--re") p.re = std::atof(v);
    else if (a == "--fr") p.fr = std::atof(v);
    else if (a == "--sc") p.sc = std::atof(v);
    else if (a == "--u0") p.u0 = std::atof(v);
    else if (a == "--gn") p.g_over_n = std::atof(v);
    else if (a == "--noise") p.noise_amp = std::atof(v);
    else if (a == "--seed") p.seed = std::strtoull(v, nullptr, 10);
    else if (a == "--steps") steps = std::atoll(v);
    else if (a == "--diag") p.diag_every = std::atoi(v);
    else if (a == "--spectrum") spectrum_path = v;
    else if (a == "--checkpoint") checkpoint_path = v;
    else if (a == "--resume") resume_path = v;
    else if (a == "--mlp") mlp_path = v;
    else ok = false;
    if (!ok) { std::fprintf(stderr, "stgv_run: bad option %s %s\n", a.c_str(), v); usage(); return 2; }
  }
  if (steps < 0) { usage(); return 2; }

  size_t pop_bytes = 0, work_bytes = 0;
  int st = lbm_query_sizes(&p, &pop_bytes, &work_bytes);     // validates every parameter on the CPU
  if (st != LBM_OK) return fail("parameters", st, nullptr);
  std::vector<float> resume_state;
  int64_t resume_step = 0;
  if (resume_path) {
    const int r = read_checkpoint(p, resume_path, resume_state, resume_step);
    if (r != 0) return r;
  }
  std::vector<float> mlp_params, mlp_norm;
  if (mlp_path) {
    const int r = read_network(mlp_path, mlp_params, mlp_norm);
    if (r != 0) return r;
  }
  void *pop = nullptr, *work = nullptr;
  if (hipMalloc(&pop, pop_bytes) != hipSuccess || hipMalloc(&work, work_bytes) != hipSuccess) {
    std::fprintf(stderr, "stgv_run: hipMalloc of %zu + %zu bytes failed\n", pop_bytes, work_bytes);
    return 1;
  }
  hipStream_t stream = nullptr;
  if (hipStreamCreate(&stream) != hipSuccess) { std::fprintf(stderr, "stgv_run: hipStreamCreate failed\n"); return 1; }
  lbm_ctx* ctx = nullptr;
  st = lbm_init_tgv(&p, pop, pop_bytes, work, work_bytes, stream, &ctx);
  if (st != LBM_OK) return fail("initial state", st, nullptr);
  if (resume_path) {
    const int r = load_state(ctx, resume_state, resume_step);
    if (r != 0) { lbm_destroy(ctx); return r; }
    std::vector<float>().swap(resume_state);
  }
  void* packed = nullptr;
  if (mlp_path) {
    const int r = attach_network(ctx, stream, mlp_params, mlp_norm, &packed);
    if (r != 0) { lbm_destroy(ctx); return r; }
  }

  std::printf("step,t,ek,ep,eps_k,eps_p,mass,umax\n");
  std::vector<lbm_diag> recs(4096), all;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipEventRecord(e0, stream);
  int rc = 0;
  // chunks that cannot overflow the 4096-record ring between drains
  const long long chunk = p.diag_every > 0 ? 4000LL * p.diag_every : steps;
  for (long long done = 0; done < steps && rc == 0;) {
    const long long k = std::min(chunk, steps - done);
    st = lbm_step(ctx, k);
    if (st != LBM_OK) { rc = fail("step", st, ctx); break; }
    done += k;
    int32_t got = 0;
    st = lbm_diagnostics(ctx, recs.data(), (int32_t)recs.size(), &got);
    for (int32_t r = 0; r < got; ++r) {
      std::printf("%lld,%.6f,%.10e,%.10e,%.10e,%.10e,%.10e,%.6e\n", (long long)recs[r].step, recs[r].t,
                  recs[r].ek, recs[r].ep, recs[r].eps_k, recs[r].eps_p, recs[r].mass, recs[r].umax);
      all.push_back(recs[r]);
    }
    if (st != LBM_OK) rc = fail("diagnostics", st, ctx);
  }
  (void)hipEventRecord(e1, stream);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  const double n3 = (double)p.n * p.n * p.n;
  std::fprintf(stderr, "stgv_run: %lld steps of %d^3 D3Q%dxD3Q%d in %.1f ms: %.1f MLUPS\n", steps, p.n, p.q_f,
               p.q_g, ms, steps > 0 && ms > 0.f ? n3 * steps / (ms * 1e-3) / 1e6 : 0.0);
  if (rc == 0 && all.size() >= 2) {
    lbm_post post{};
    st = lbm_postprocess(all.data(), (int32_t)all.size(), p.re, p.fr, all.back().t, nullptr, nullptr, &post);
    if (st != LBM_OK) rc = fail("post-processing", st, nullptr);
    else
      std::fprintf(stderr, "stgv_run: t <= %.4f (%d records): Gamma_b %.10e  Fr_t %.10e  R_max %.10e at t = %.4f\n",
                   all.back().t, post.used, post.gamma_b, post.fr_t, post.r_max, post.t_r_max);
  }
  if (rc == 0 && spectrum_path) rc = write_spectrum(ctx, p.n, spectrum_path);
  if (rc == 0 && checkpoint_path) rc = save_state(ctx, p, checkpoint_path);
  lbm_destroy(ctx);
  if (packed) (void)hipFree(packed);
  (void)hipStreamDestroy(stream);
  (void)hipFree(pop);
  (void)hipFree(work);
  return rc;
}
