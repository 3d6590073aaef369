"""Pins of the post-processing oracle: the spectrum of the Taylor-Green initial field
(all energy in shell round(sqrt 3) = 2), Parseval, single modes, and the time integrals
against closed forms."""
import math

import numpy as np
import pytest

from oracle import lattice as lat, model, postproc


def test_taylor_green_spectrum_is_one_shell():
    # u = U0 (sin x cos y cos z, -cos x sin y cos z, 0): wavevectors (+-1, +-1, +-1), |k| = sqrt 3
    n = 16
    p = model.Params(n=n, u0=0.05, fr=math.inf)
    f, g = model.init_tgv(p)
    u = model.fields(model.macro(f, g, lat.D3Q27, lat.D3Q19, model.units(p)))[1:4]
    e = postproc.ke_spectrum(u, 0.05)
    assert e.size == postproc.spectrum_shells(n) == round(math.sqrt(3) * 8) + 1
    # E_k = <|u|^2>/2 / U0^2 = 1/8 up to the rounding of u = u' + F/(2 rho) at t = 0 (F = 0 here)
    assert abs(e[2] - 0.125) < 1e-12
    assert np.abs(np.delete(e, 2)).max() < 1e-28


def test_parseval_on_a_random_field():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((3, 12, 12, 12))
    e = postproc.ke_spectrum(u, 2.0)
    assert math.isclose(e.sum(), 0.5 * (u * u).sum(0).mean() / 4.0, rel_tol=1e-12)


@pytest.mark.parametrize("kvec,shell", [((0, 0, 5), 5), ((3, 4, 0), 5), ((1, 1, 1), 2), ((4, 4, 4), 7)])
def test_single_mode_lands_in_its_shell(kvec, shell):
    n = 16
    x = np.arange(n) * 2 * np.pi / n
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    kx, ky, kz = kvec
    u = np.zeros((3, n, n, n))
    u[1] = np.cos(kx * xx + ky * y + kz * z)              # <u_y^2>/2 = 1/4
    e = postproc.ke_spectrum(u, 1.0)
    assert abs(e[shell] - 0.25) < 1e-13
    assert np.abs(np.delete(e, shell)).max() < 1e-25


def test_time_integrals_against_closed_forms():
    t = np.linspace(0.0, 40.0, 4001)                        # records past t_end are ignored
    eps_k = np.exp(-t / 10.0)
    eps_p = 0.5 * np.exp(-t / 10.0) * (1.0 + 0.1 * np.sin(t))
    ek = 2.0 + 0.0 * t
    ik = 10.0 * (1.0 - math.exp(-3.0))
    ip = 0.5 * (ik + 0.1 * (10.0 / 101.0) * (10.0 - math.exp(-3.0) * (math.sin(30.0) + 10.0 * math.cos(30.0))))
    h = t[1] - t[0]
    assert math.isclose(postproc.bulk_flux_coefficient(t, eps_k, eps_p), ip / ik, rel_tol=h * h)
    assert math.isclose(postproc.turbulent_froude(t, eps_k, ek, fr=0.5), ik / (2.0 * 2.0 * 30.0), rel_tol=h * h)
    # R and Gamma are pointwise
    assert postproc.buoyancy_reynolds(2e-3, re=1600.0, fr=0.5) == pytest.approx(2e-3 * 1600.0 * 0.25)
    assert postproc.flux_coefficient(4.0, 1.0) == 0.25
