// Kinetic-energy spectrum of a velocity field on the GPU: three rocFFT real-to-complex
// transforms and a shell-binning reduction (Section 3.5, spectra at peak activity).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace stgv {

// Shells 0 .. round(sqrt(3) n / 2): every wavevector of the n^3 box has one.
int spectrum_shells(int n);

// Device bytes the spectrum needs besides the velocity fields (complex buffer, per-block
// partials, rocFFT work).  Creates (and caches) the FFT plan for n; returns 0 and fills
// err when rocFFT fails.
size_t spectrum_extra_bytes(int n, char* err);

// E(k) of u = (ux, uy, uz) / u0 (each n^3 FP32, x fastest) into out[spectrum_shells(n)]
// (FP64, device).  work: spectrum_extra_bytes(n) bytes, 256-byte aligned.  Queued on st.
// Returns a HIP error, or hipErrorUnknown with err filled when rocFFT fails.
hipError_t spectrum_launch(const float* ux, const float* uy, const float* uz, int n, double u0,
                           void* work, size_t work_bytes, double* out, hipStream_t st, char* err);

}  // namespace stgv
