"""Post-processing of a stratified Taylor-Green run (FP64, NumPy): the quantities the paper
derives from the energy and dissipation histories and from the velocity field.

Test infrastructure only (part of the CPU oracle).  Definitions, in the paper's
physical units (U = L = 1 on the 2 pi box, so nu = 1/Re and N = 1/Fr):

* buoyancy Reynolds number R = eps_k / (nu N^2)  (Section 3.4, buoyancy Reynolds number);
* flux coefficient Gamma = eps_p / eps_k  (Section 3.5, Froude number effects);
* bulk flux coefficient Gamma_b = int_0^T eps_p dt / int_0^T eps_k dt, T = 30;
* turbulent Froude number Fr_t = int_0^T eps_k dt / (N int_0^T E_k dt);
* kinetic-energy spectrum E(k) = sum over integer wavevectors with round(|k|) = k of
  |u_hat(k)|^2 / 2, u_hat the discrete Fourier coefficients of u / U
  (u_hat = FFT(u) / n^3), so that sum_k E(k) = <|u|^2> / 2 = E_k.

Readings where the paper is silent: the time integrals are trapezoid sums over the
diagnostic records with t <= T; spectral shells are the integers nearest |k| and run
to round(sqrt(3) n / 2), so that no mode is dropped.
"""
import numpy as np


def buoyancy_reynolds(eps_k, re, fr):
    """R = eps_k / (nu N^2) with nu = 1/Re and N = 1/Fr (physical units)."""
    nu, nb = 1.0 / re, 1.0 / fr
    return np.asarray(eps_k, dtype=np.float64) / (nu * nb * nb)


def flux_coefficient(eps_k, eps_p):
    """Gamma = eps_p / eps_k."""
    return np.asarray(eps_p, dtype=np.float64) / np.asarray(eps_k, dtype=np.float64)


def _trapezoid(t, y, t_end):
    """Trapezoid sum of y over the samples with t <= t_end, written out."""
    total = 0.0
    for i in range(1, len(t)):
        if t[i] > t_end:
            break
        total += 0.5 * (t[i] - t[i - 1]) * (y[i] + y[i - 1])
    return total


def bulk_flux_coefficient(t, eps_k, eps_p, t_end=30.0):
    """Gamma_b = int eps_p dt / int eps_k dt over [0, t_end]."""
    return _trapezoid(t, eps_p, t_end) / _trapezoid(t, eps_k, t_end)


def turbulent_froude(t, eps_k, ek, fr, t_end=30.0):
    """Fr_t = int eps_k dt / (N int E_k dt) over [0, t_end], N = 1/Fr."""
    return _trapezoid(t, eps_k, t_end) / ((1.0 / fr) * _trapezoid(t, ek, t_end))


def spectrum_shells(n):
    """Number of shells 0 .. round(sqrt(3) n / 2)."""
    return int(np.floor(np.sqrt(3.0) * n / 2.0 + 0.5)) + 1


def ke_spectrum(u, u0):
    """E(k) of the velocity field u (3, n, n, n) (lattice units, arrays [c, z, y, x]) scaled by u0."""
    u = np.asarray(u, dtype=np.float64) / u0
    n = u.shape[-1]
    k1 = np.fft.fftfreq(n, d=1.0 / n)                    # integer wavenumbers, -n/2 .. n/2 - 1
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    shell = np.floor(np.sqrt(kx * kx + ky * ky + kz * kz) + 0.5).astype(np.int64)
    energy = np.zeros(spectrum_shells(n))
    for c in range(3):
        uh = np.fft.fftn(u[c]) / n ** 3
        np.add.at(energy, shell.ravel(), 0.5 * (uh.real ** 2 + uh.imag ** 2).ravel())
    return energy
