"""Pins of the time-stepping oracle against theory it does not contain.

* Viscous decay: a small-amplitude unstratified Taylor-Green mode loses kinetic
  energy at the rate of the least-damped shear eigenvalue of the linearised
  lattice propagator (computed by a separate route: a 27x27 eigenproblem), and
  that rate approaches the Navier-Stokes value 2 nu |k|^2 as the grid is refined.
* Internal waves: a small standing density perturbation in a stratified fluid
  at rest oscillates at the Boussinesq frequency N k_h / |k|.  This also
  separates the readings of the Shan-Chen shift (as printed it halves the force,
  frequency off by a factor 1/sqrt(2)) and of the scalar source placement (as
  printed it biases N^2 at tau_g = 0.6 by about 12 %).
* The TGV state at t = 0: closed forms of E_k, eps_k (with the central
  difference), E_p, and the total mass.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy.optimize import curve_fit

from oracle import lattice as lat, linear, model


# ---------------------------------------------------------------------------
# viscous decay
# ---------------------------------------------------------------------------
def _decay_rate(n, tau, q_f, steps=250, skip=50):
    L = n / (2 * math.pi)
    u0 = 1e-4
    nu = (tau - 0.5) / 3.0
    p = model.Params(n=n, q_f=q_f, q_g=7, u0=u0, re=u0 * L / nu, fr=math.inf, sc=1.0)
    U = model.units(p)
    assert abs(U.tau_f - tau) < 1e-12
    (_, _), ser = model.run(p, steps, diag_every=1)
    ek = np.array([d.ek for d in ser])
    s = np.arange(steps)
    rate = -np.polyfit(s[skip:], np.log(ek[skip:]), 1)[0]
    return rate, U


@pytest.mark.parametrize("q_f,tau", [(27, 0.6), (27, 0.8), (19, 0.6)])
def test_tgv_decay_matches_linear_lattice_eigenvalue(q_f, tau):
    n = 32
    rate, U = _decay_rate(n, tau, q_f)
    k = np.array([1.0, 1.0, 1.0]) * 2 * math.pi / n
    lam_rate = linear.shear_energy_rate(q_f, U.tau_f, k)
    # Residual sources: the O(Re) nonlinearity (Re ~ 1e-2 here) and the transient.
    assert abs(rate / lam_rate - 1.0) < 1e-4
    # and the lattice rate is Navier-Stokes' 2 nu |k|^2 up to O((k dx)^2)
    cont = 2.0 * U.nu * float(k @ k)
    assert abs(lam_rate / cont - 1.0) < 0.02


def test_decay_error_against_navier_stokes_shrinks_with_resolution():
    errs = []
    for n in (16, 32, 64):
        k = np.array([1.0, 1.0, 1.0]) * 2 * math.pi / n
        tau = 0.6
        errs.append(abs(linear.shear_energy_rate(27, tau, k) / (2 * (tau - 0.5) / 3 * float(k @ k)) - 1))
    for coarse, fine in zip(errs, errs[1:]):                 # second order in k dx
        assert 3.0 < coarse / fine < 5.0


# ---------------------------------------------------------------------------
# internal gravity waves
# ---------------------------------------------------------------------------
def _internal_wave(n=32, nb=0.01, tau_f=0.6, tau_g=0.6, forcing="guo", q_f=27, q_g=19,
                   steps=1800, g_over_n=0.01, **flags):
    """Standing wave rho' = A cos(k x) cos(k z) in fluid at rest; returns the fitted frequency / (N/sqrt 2)."""
    lf, lg = lat.BY_Q[q_f], lat.BY_Q[q_g]
    k = 2 * math.pi / n
    x = np.arange(n)
    Z, X = np.meshgrid(x, x, indexing="ij")
    A = 1e-4 / g_over_n
    basis = np.cos(k * X) * np.cos(k * Z)
    f = lf.w.reshape(-1, 1, 1, 1) * np.ones((1, n, 1, n))                 # box n x 1 x n
    g = lg.w.reshape(-1, 1, 1, 1) * (1.0 + A * basis[:, None, :])[None]
    U = dataclasses.replace(model.raw_units(tau_f, tau_g, nb=nb, forcing=forcing,
                                            g_over_n=g_over_n), **flags)
    amp = []
    for _ in range(steps):
        fs, gs, m = model.collide(f, g, lf, lg, U)
        amp.append(4.0 * (m.rho_p[:, 0, :] * basis).mean() / A)
        f, g = model.stream(fs, lf), model.stream(gs, lg)
    t = np.arange(steps, dtype=float)
    w0 = nb / math.sqrt(2.0)            # N k_h / |k| with k_h = k_z
    fn = lambda t, a0, w, ph, gam: a0 * np.cos(w * t + ph) * np.exp(-gam * t)
    p, _ = curve_fit(fn, t, np.array(amp), p0=[1.0, w0, 0.0, 1e-3])
    return p[1] / w0


@pytest.mark.parametrize("forcing,q_f,q_g", [("guo", 27, 19), ("shift", 27, 19), ("shift", 19, 7),
                                             ("edm", 27, 19), ("hcz", 27, 19)])
def test_internal_wave_frequency(forcing, q_f, q_g):
    r = _internal_wave(forcing=forcing, q_f=q_f, q_g=q_g)
    assert abs(r - 1.0) < 0.01


def test_printed_shan_chen_shift_gives_the_wrong_wave_frequency():
    r = _internal_wave(forcing="shift", shift_half=True, steps=1200)
    assert abs(r * math.sqrt(2.0) - 1.0) < 0.01          # force halved -> omega / sqrt(2)


def test_printed_source_placement_biases_the_wave_frequency():
    r = _internal_wave(source_as_printed=True) / _internal_wave()
    # scalar gain per step (1 + a - a^2) s with a = 1 - 1/(2 tau_g) = 1/6  ->  omega up by ~6.7 %
    a = 1.0 - 1.0 / 1.2
    assert abs(r - math.sqrt(1 + a - a * a)) < 2e-3


# ---------------------------------------------------------------------------
# the Taylor-Green set-up at t = 0
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,q_f,q_g", [(8, 27, 19), (12, 27, 7), (16, 19, 7)])
def test_tgv_closed_forms_at_t0(n, q_f, q_g):
    p = model.Params(n=n, q_f=q_f, q_g=q_g, u0=0.05, re=800, fr=1.0, sc=1.0, noise_amp=0.0)
    f, g = model.init_tgv(p)
    U = model.units(p)
    d = model.state_diag(f, g, p, 0)
    assert d.ek == pytest.approx(1.0 / 8.0, rel=1e-13)                    # (U^2/8) / U^2
    h = 2 * math.pi / n
    eps_k_lb = U.nu * 0.75 * p.u0 ** 2 * math.sin(h) ** 2
    assert d.eps_k == pytest.approx(eps_k_lb * U.L / p.u0 ** 3, rel=1e-12)
    assert d.ep < 1e-25 and d.eps_p < 1e-25                                 # rho' = 0 up to rounding
    assert d.mass == pytest.approx(n ** 3, rel=1e-14)
    assert d.scalar == pytest.approx(n ** 3, rel=1e-14)
    fl = model.state_fields(f, g, p)
    u_expect, p0 = model.tgv_fields(n, p.u0)
    np.testing.assert_allclose(fl[1:4], u_expect, rtol=0, atol=1e-16)      # a few ulps of 0.05
    # rho - 1 from sum f ~ 1 carries a few FP64 ulps of 1
    np.testing.assert_allclose(fl[0], p0 / lat.BY_Q[q_f].cs2, rtol=0, atol=2e-15)


def test_tgv_units_match_the_stated_dimensionless_numbers():
    p = model.Params(n=256, u0=0.05, re=1600, fr=0.3, sc=0.7)
    U = model.units(p)
    assert U.L == pytest.approx(256 / (2 * math.pi))
    assert p.u0 * U.L / U.nu == pytest.approx(1600)                        # Re = U L / nu
    assert U.nu / U.D == pytest.approx(0.7)                                # Sc = nu / D
    assert p.u0 / (U.nb * U.L) == pytest.approx(0.3)                       # Fr = U / (N L)
    assert math.sqrt(-U.G * U.beta) == pytest.approx(U.nb)                 # Eq. (19), rho0 = 1
    assert U.tau_f == pytest.approx(3 * U.nu + 0.5)
    assert U.tau_g == pytest.approx(3 * U.D + 0.5)
    u7 = model.units(dataclasses.replace(p, q_g=7))
    assert u7.tau_g == pytest.approx(4 * U.D + 0.5)                        # D3Q7: c_s^2 = 1/4


def test_noise_generator_is_splitmix64():
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")))
    assert int(model.splitmix64(np.array([0], dtype=np.uint64))[0]) == int(gold["seed_0_first"], 16)
    seed = 1234567
    got = [int(model.splitmix64(np.array([(seed + k * model.SM_GAMMA) % 2 ** 64], dtype=np.uint64))[0])
           for k in range(5)]
    assert got == gold["seed_1234567_first5"]
    a = model.noise(16, 1e-6, 0)
    assert np.abs(a).max() <= 1e-6 and abs(a.mean()) < 1e-7 and a.std() == pytest.approx(1e-6 / math.sqrt(3), rel=0.05)
    assert not np.array_equal(a, model.noise(16, 1e-6, 1))


def test_unstratified_limit_decouples_the_scalar():
    """Fr -> inf (G = 0): f evolves exactly as with no scalar lattice at all (any q_g)."""
    base = dict(n=8, u0=0.05, re=100, fr=math.inf, sc=1.0, noise_amp=1e-3, seed=3)
    (f1, _), _ = model.run(model.Params(q_g=19, **base), 5)
    (f2, _), _ = model.run(model.Params(q_g=7, **base), 5)
    np.testing.assert_array_equal(f1, f2)


# ---------------------------------------------------------------------------
# potential energy and its dissipation on a prescribed density perturbation
# (Section 3.2, Eq. (23); Section 3.3, Eq. (26))
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m_x,m_z", [(1, 1), (2, 3)])
def test_potential_energy_and_dissipation_closed_forms(m_x, m_z):
    # rho' = A cos(k_x x) cos(k_z z) on the nodes, fluid at rest.  Discrete orthogonality
    # gives <rho'^2> = A^2 / 4, so E_p = (G/N)^2 A^2 / 8; the periodic central difference
    # of cos(k x) is -sin(k) sin(k x), so <|grad rho'|^2> = A^2 (sin^2 k_x + sin^2 k_z) / 4
    # and eps_p = D (G/N)^2 A^2 (sin^2 k_x + sin^2 k_z) / 4 (lattice units, k per node).
    # G/N = 0.3 and N = 0.01 make G = 0.003 distinct from G/N, and Sc = 0.7 makes D
    # distinct from nu: squaring G/N wrongly, using G for G/N, or dropping D fails.
    n, amp, g_over_n = 24, 3e-3, 0.3
    p = model.Params(n=n, u0=0.05, re=400.0, fr=1.0, sc=0.7, g_over_n=g_over_n)
    U = dataclasses.replace(model.units(p), nb=0.01, G=g_over_n * 0.01)
    j = np.arange(n)
    Z, Y, X = np.meshgrid(j, j, j, indexing="ij")
    kx, kz = 2 * math.pi * m_x / n, 2 * math.pi * m_z / n
    rho_p = amp * np.cos(kx * X) * np.cos(kz * Z)
    zero = np.zeros((3, n, n, n))
    m = model.Macro(rho=np.ones((n, n, n)), up=zero, sigma=rho_p + 1.0, s=np.zeros((n, n, n)),
                    rho_p=rho_p, F=zero, u=zero, ueq=zero, utheta=zero)
    d = model.diagnostics(m, U, 0)
    ep = g_over_n ** 2 * amp ** 2 / 8.0
    eps_p = U.D * g_over_n ** 2 * amp ** 2 * (math.sin(kx) ** 2 + math.sin(kz) ** 2) / 4.0
    assert d.ep * U.u0 ** 2 == pytest.approx(ep, rel=1e-12)
    assert d.eps_p * U.u0 ** 3 / U.L == pytest.approx(eps_p, rel=1e-12)
    assert d.ek == 0.0 and d.eps_k == 0.0


# ---------------------------------------------------------------------------
# the initial pressure, Eq. (21), as read
# ---------------------------------------------------------------------------
def _poisson_pressure(u, h):
    """Pressure of an incompressible velocity field on the periodic box: the solution of
    lap p = -rho_0 d_i u_j d_j u_i with zero mean, all derivatives spectral."""
    n = u.shape[-1]
    k = np.fft.fftfreq(n, d=h) * 2 * math.pi
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    K = (KX, KY, KZ)
    uh = [np.fft.fftn(c) for c in u]
    du = [[np.real(np.fft.ifftn(1j * K[i] * uh[j])) for j in range(3)] for i in range(3)]   # du[i][j] = d_i u_j
    rhs = -model.RHO0 * sum(du[i][j] * du[j][i] for i in range(3) for j in range(3))
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    k2[0, 0, 0] = 1.0
    ph = -np.fft.fftn(rhs) / k2
    ph[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(ph))


def test_initial_pressure_solves_the_taylor_green_poisson_equation():
    # The paper's Eq. (21) prints the z factor garbled as cos(2z + 2); the reading
    # (cos 2x + cos 2y)(cos 2z + 2) U^2 / 16 is the pressure of the initial velocity of
    # Eq. (20).  The spectral Poisson solution of lap p = -rho_0 d_i u_j d_j u_i must equal
    # it to rounding (up to the constant a Poisson solution leaves free); the printed form
    # must not.
    n, u0 = 32, 0.05
    u, p0 = model.tgv_fields(n, u0)
    p = _poisson_pressure(u, 2 * math.pi / n)
    read = p0 - p0.mean()
    assert np.abs(p - read).max() <= 1e-13 * np.abs(read).max() + 1e-18
    j = np.arange(n)
    Z, Y, X = np.meshgrid(j, j, j, indexing="ij")
    x, y, z = (2 * math.pi / n * a for a in (X, Y, Z))
    printed = model.RHO0 * u0 ** 2 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * np.cos(2 * z + 2)
    printed -= printed.mean()
    assert np.abs(p - printed).max() > 0.3 * np.abs(read).max()


# ---------------------------------------------------------------------------
# -dE/dt of the energy history (Section 3.1: second-order central differences in time)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("a,dt", [(0.3, 0.05), (1.0, 0.02)])
def test_dissipation_series_of_an_exponential_decay(a, dt):
    # E = exp(-a t): the central difference gives -dE/dt = a exp(-a t) sinh(a dt) / (a dt),
    # a relative error (a dt)^2 / 6 + O((a dt)^4), at the interior times t_1 .. t_{m-2}.
    # A forward difference (error a dt / 2), a sign slip or a wrong denominator fail.
    ts = np.arange(0.0, 10.0, dt)
    t, rate = model.dissipation_series(ts, np.exp(-a * ts))
    assert np.array_equal(t, ts[1:-1])
    exact = a * np.exp(-a * t)
    rel = rate / exact - 1.0
    x = a * dt
    assert np.allclose(rel, math.sinh(x) / x - 1.0, rtol=1e-6, atol=1e-12)
    assert 0.9 * x * x / 6 < rel.max() < 1.1 * x * x / 6
