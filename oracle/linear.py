"""Linear (small-amplitude) analysis of the lattice Boltzmann step.

Test infrastructure only (part of the CPU oracle).  Around the rest state
rho = 1, u = 0 with no force, the BGK step of Eqs. (5), (8) and (9) is linear in
the deviation h = f - w.  For a plane wave exp(i k.x) the collision is the
matrix (1 - omega) I + omega E with E_ij = w_i (1 + e_i.e_j / c_s^2) (the
linearised equilibrium), and streaming multiplies direction i by
exp(-i k.e_i).  The eigenvalues of that product give the exact per-step decay
of every linear mode on the lattice.  The shear-mode eigenvalue is what a
small-amplitude unstratified Taylor-Green mode decays with; the time-stepping
oracle has to reproduce it.
"""
import numpy as np

from . import lattice as lat


def propagator(q, tau, k):
    L = lat.BY_Q[q]
    e = L.e.astype(np.float64)
    E = L.w[:, None] * (1.0 + (e @ e.T) / L.cs2)
    omega = 1.0 / tau
    C = (1.0 - omega) * np.eye(q) + omega * E
    phase = np.exp(-1j * (e @ np.asarray(k, dtype=np.float64)))
    return phase[:, None] * C


def shear_eigenvalue(q, tau, k):
    """Eigenvalue of the transverse (shear) mode: |lambda| near 1 and the smallest |arg lambda|."""
    lam = np.linalg.eigvals(propagator(q, tau, k))
    near = lam[np.abs(lam) > 0.5]
    return near[np.argmin(np.abs(np.angle(near)))]


def shear_energy_rate(q, tau, k):
    """Per-step decay rate of the kinetic energy of a shear mode: -2 ln |lambda|."""
    return -2.0 * np.log(np.abs(shear_eigenvalue(q, tau, k)))
