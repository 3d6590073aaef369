"""Pins of the learned-correction oracle: the moment basis, the conservation of the
correction, the network gradient against finite differences, Adam's first step, the
zero-output identity, restriction of equilibria, and the training-pair construction."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import lattice as lat, learned as L, model


@pytest.mark.parametrize("q", [27, 19])
def test_moment_matrix_inverse_is_exact(q):
    M = L.moment_matrix(q)
    Mi = L.moment_inverse_exact(q)
    for r in range(q):
        for c in range(q):
            assert sum(Fraction(int(M[r][k])) * Mi[k][c] for k in range(q)) == (1 if r == c else 0)
    # every entry is dyadic (exact in FP32): denominators divide 8
    assert all(8 % v.denominator == 0 for row in Mi for v in row)
    # the conserved slots are the mass and momentum (and scalar) moments
    e = lat.BY_Q[q].e
    assert np.array_equal(M[0], np.ones(q, dtype=np.int64))
    if q == 27:
        for a in range(3):
            assert np.array_equal(M[1 + a], e[:, a])


def test_correction_changes_only_non_conserved_moments():
    rng = np.random.default_rng(0)
    dm = rng.standard_normal((41, 5))
    cf, cg = L.correction(dm)
    e = lat.D3Q27.e.astype(float)
    np.testing.assert_allclose(cf.sum(0), 0.0, atol=1e-14)
    np.testing.assert_allclose(e.T @ cf, 0.0, atol=1e-14)
    np.testing.assert_allclose(cg.sum(0), 0.0, atol=1e-14)
    np.testing.assert_allclose(L.project(cf, cg), dm, rtol=1e-13, atol=1e-14)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    theta = L.init_params(3) + 0.05 * rng.standard_normal(L.N_PARAMS)
    xn = rng.standard_normal((7, L.N_IN))
    yn = rng.standard_normal((7, L.N_OUT))
    _, g = L.loss_and_grad(theta, xn, yn)
    idx = rng.choice(L.N_PARAMS, 60, replace=False)
    h = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (L.loss_and_grad(tp, xn, yn)[0] - L.loss_and_grad(tm, xn, yn)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-3), (k, fd, g[k])


def test_adam_first_step_moves_by_lr_times_sign():
    theta = np.array([1.0, -2.0, 0.5])
    grad = np.array([3.0, -1e-3, 0.25])
    new, m, v = L.adam_step(theta, grad, np.zeros(3), np.zeros(3), 1, lr=1e-2)
    # bias-corrected m / sqrt(v) = g / |g| at t = 1
    np.testing.assert_allclose(theta - new, 1e-2 * np.sign(grad) * np.abs(grad) / (np.abs(grad) + 1e-8),
                               rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * grad)
    np.testing.assert_allclose(v, 0.001 * grad * grad)


def test_zero_output_layer_gives_the_plain_step():
    p = model.Params(n=6, forcing="shift", re=100, noise_amp=1e-3, g_over_n=0.5)
    f, g = model.init_tgv(p)
    (f, g), _ = model.run(p, 2, state=(f, g))
    U = model.units(p)
    theta = L.unpack(L.init_params(0))
    theta["W3"][:] = 0.0
    theta["b3"][:] = 0.0
    norm = (np.zeros(47), np.ones(47), np.ones(41))
    fs, gs, _ = L.learned_collide(f, g, U, L.pack(theta), norm)
    fp, gp, _ = model.collide(f, g, lat.D3Q27, lat.D3Q19, U)
    np.testing.assert_array_equal(fs, fp)
    np.testing.assert_array_equal(gs, gp)


def test_features_of_an_unforced_equilibrium_vanish():
    p = model.Params(n=8, fr=math.inf, noise_amp=1e-3)
    f, g = model.init_tgv(p)
    x = L.features(f, g, model.units(p))
    np.testing.assert_allclose(x[:46], 0.0, atol=2e-15)          # FP64 rounding of O(0.3) sums
    np.testing.assert_allclose(x[46], model.noise(8, 1e-3, 0), rtol=0, atol=1e-15)


def test_restriction_of_a_uniform_equilibrium_is_the_coarse_equilibrium():
    # G = 0: the equilibrium velocity is the physical velocity, so no non-equilibrium part
    pf = model.Params(n=16, fr=math.inf)
    pc = model.Params(n=4, fr=math.inf)
    u = np.zeros((3, 16, 16, 16))
    u[0], u[1], u[2] = 0.02, -0.01, 0.0
    rho = np.full((16, 16, 16), 1.003)
    f = model.f_equilibrium(lat.D3Q27, rho, u)
    g = 1.002 * model.theta(lat.D3Q19, u)
    fc, gc = L.restrict(f, g, pf, pc)
    np.testing.assert_allclose(fc, f[:, ::4, ::4, ::4], rtol=1e-14)
    np.testing.assert_allclose(gc, g[:, ::4, ::4, ::4], rtol=1e-14)


def test_restriction_keeps_the_filtered_conserved_moments():
    pf = model.Params(n=16, forcing="guo", fr=1.0, noise_amp=1e-3)
    pc = model.Params(n=4, forcing="guo", fr=1.0)
    (f, g), _ = model.run(pf, 3)
    fc, gc = L.restrict(f, g, pf, pc)
    e = lat.D3Q27.e.astype(float)
    np.testing.assert_allclose(fc.sum(0), L.filter_sample(f.sum(0), 4), rtol=1e-13)
    np.testing.assert_allclose(np.tensordot(e.T, fc, axes=(1, 0)),
                               L.filter_sample(np.tensordot(e.T, f, axes=(1, 0)), 4), atol=1e-15)
    np.testing.assert_allclose(gc.sum(0), L.filter_sample(g.sum(0), 4), rtol=1e-13)
    assert np.abs(fc - L.filter_sample(f, 4)).max() > 0       # the non-equilibrium part was rescaled


def test_filter_weights_and_unstream():
    assert L.FILTER.sum() == 1.0
    a = np.random.default_rng(2).standard_normal((27, 5, 6, 7))
    np.testing.assert_array_equal(L.unstream(model.stream(a, lat.D3Q27), lat.D3Q27), a)


def test_training_targets_vanish_for_an_exact_coarse_step():
    pc = model.Params(n=6, forcing="shift", re=200, fr=1.0, noise_amp=1e-3, g_over_n=0.5)
    a = model.init_tgv(pc)
    (b_f, b_g), _ = model.run(pc, 1, state=a)
    x, y = L.training_pair(a, (b_f, b_g), pc)
    assert x.shape == (47, 6, 6, 6) and y.shape == (41, 6, 6, 6)
    np.testing.assert_allclose(y, 0.0, atol=1e-16)
    # and a perturbation of b shows up as its non-conserved moments at the source node
    rng = np.random.default_rng(3)
    dm = 1e-6 * rng.standard_normal((41, 6, 6, 6))
    cf, cg = L.correction(dm)
    _, y2 = L.training_pair(a, (b_f + model.stream(cf, lat.D3Q27), b_g + model.stream(cg, lat.D3Q19)), pc)
    np.testing.assert_allclose(y2, dm, rtol=1e-7, atol=1e-16)


@pytest.mark.parametrize("forcing", ["guo", "shift"])
def test_conserved_feature_slots_are_the_full_moments(forcing):
    # the closed forms of the conserved slots agree with the moments of f - f^eq, g - g^eq
    # summed in full, and carry the forcing: -F_z/2 (Guo) or -tau_f F_z (shift)
    p = model.Params(n=6, forcing=forcing, re=100, fr=0.5, noise_amp=1e-3, g_over_n=0.5)
    (f, g), _ = model.run(p, 3)
    U = model.units(p)
    x = L.features(f, g, U)
    m = model.macro(f, g, lat.D3Q27, lat.D3Q19, U)
    feq = model.f_equilibrium(lat.D3Q27, m.rho, m.ueq)
    geq = (m.rho_p + model.RHO0) * model.theta(lat.D3Q19, m.utheta)
    e = lat.D3Q27.e.astype(float)
    np.testing.assert_allclose(x[0], (f - feq).sum(0), rtol=0, atol=1e-15)
    np.testing.assert_allclose(x[1:4], np.tensordot(e.T, f - feq, axes=(1, 0)), rtol=0, atol=1e-16)
    np.testing.assert_allclose(x[27], (g - geq).sum(0), rtol=0, atol=1e-15)
    fz = -U.G * m.rho_p
    np.testing.assert_allclose(x[3], -0.5 * fz if forcing == "guo" else -U.tau_f * fz, rtol=1e-9)
    np.testing.assert_allclose(x[27], -0.5 * m.s, rtol=1e-9, atol=1e-18)
    assert np.abs(x[3]).max() > 0 and np.all(x[0:3] == 0.0)


def test_restriction_rescales_a_relaxed_shear_wave_to_the_coarse_run():
    # A shear wave u_x = U sin z relaxes on the fine grid (32^3, tau_f = 1) and on the
    # coarse grid (8^3, the same physical viscosity, so tau_c = 0.625) from equilibrium.
    # After the same physical time (64 fine, 16 coarse steps) the restricted fine state
    # must carry the coarse run's own non-equilibrium shear stress Pi_xz: the lattice
    # gradient is 4 x larger on the coarse grid and Pi_neq ~ tau c_s^2 du, hence the
    # rescale 4 tau_c / tau_f (2.5 here).  Without it the stress is 0.40 of the coarse
    # run's; with 4 alone, tau_c / tau_f alone or the inverted ratio it is off by a
    # factor 1.6, 0.25 or 2.6.  Measured agreement: 0.8 %.
    lf, lg = lat.D3Q27, lat.D3Q19
    u0, nf, nc, tau_f = 0.05, 32, 8, 1.0
    re = u0 * (nf / (2 * math.pi)) / ((tau_f - 0.5) / 3.0)
    pf = model.Params(n=nf, forcing="guo", u0=u0, re=re, fr=math.inf, sc=1.0)
    pc = model.Params(n=nc, forcing="guo", u0=u0, re=re, fr=math.inf, sc=1.0)
    assert model.units(pf).tau_f == pytest.approx(1.0) and model.units(pc).tau_f == pytest.approx(0.625)

    def shear(p):
        z = 2 * math.pi * np.arange(p.n) / p.n
        u = np.zeros((3, p.n, p.n, p.n))
        u[0] = u0 * np.sin(z)[:, None, None]
        return model.f_equilibrium(lf, np.ones((p.n,) * 3), u), model.theta(lg, u)

    def stress_amplitude(f, g, p):
        m = model.macro(f, g, lf, lg, model.units(p))
        neq = f - model.f_equilibrium(lf, m.rho, m.u)
        pi = np.tensordot((lf.e[:, 0] * lf.e[:, 2]).astype(float), neq, axes=(0, 0))
        z = 2 * math.pi * np.arange(p.n) / p.n
        return 2.0 * np.mean(pi * np.cos(z)[:, None, None])

    (ff, gf), _ = model.run(pf, 64, state=shear(pf))
    (fc, gc), _ = model.run(pc, 16, state=shear(pc))
    fr, gr = L.restrict(ff, gf, pf, pc)
    ratio = stress_amplitude(fr, gr, pc) / stress_amplitude(fc, gc, pc)
    assert abs(ratio - 1.0) < 0.05, ratio


def test_forward_pass_of_a_hand_computed_network():
    # Two rows through a network with a handful of non-zero weights, worked out with
    # scalar tanh: tanh on both hidden layers, none on the output, W rows index outputs.
    p = {name: np.zeros(shape) for name, shape in L.SHAPES}
    p["W1"][0, 0], p["b1"][1] = 0.5, -0.25
    p["W1"][2, 46], p["W1"][2, 3] = 1.0, 0.5
    p["W2"][0, 0], p["W2"][0, 1], p["b2"][0] = 1.0, 2.0, 0.1
    p["W2"][1, 0], p["W2"][1, 2] = -1.0, 0.75
    p["W3"][0, 0], p["W3"][0, 1], p["b3"][0] = 3.0, 1.0, 2.0
    p["W3"][40, 1], p["b3"][7] = -2.0, -0.3
    x = np.zeros((2, L.N_IN))
    x[0, 0] = 1.0
    x[1, 46], x[1, 3], x[1, 0] = 2.0, -1.0, -2.0
    out, _ = L.forward(L.pack(p), x)
    th = math.tanh
    for r in range(2):
        h1 = [th(0.5 * x[r, 0]), th(-0.25), th(x[r, 46] + 0.5 * x[r, 3])]
        h2 = [th(h1[0] + 2.0 * h1[1] + 0.1), th(-h1[0] + 0.75 * h1[2])]
        want = np.zeros(L.N_OUT)
        want[0] = 3.0 * h2[0] + h2[1] + 2.0
        want[40] = -2.0 * h2[1]
        want[7] = -0.3
        assert np.allclose(out[r], want, rtol=0, atol=1e-15), (r, out[r][[0, 7, 40]], want[[0, 7, 40]])
    assert abs(out[0, 0]) > 1.5          # large enough that a tanh on the output would show


def test_normalisation_statistics_of_known_columns():
    # columns with exactly known statistics: a +- d alternating (mean a, standard deviation
    # d), a constant column (scale 0), targets of root mean square r, and a zero target
    # column (scale 1): a variance taken with the wrong mean, a missing square root or an
    # inverted scale fails
    n = 64
    sign = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    x = np.zeros((n, L.N_IN))
    y = np.zeros((n, L.N_OUT))
    for k in range(L.N_IN):
        x[:, k] = 0.25 * k - 3.0 + (0.5 + 0.125 * k) * sign
    x[:, 5] = 7.0
    for k in range(L.N_OUT - 1):
        y[:, k] = (1.0 + k) * 1e-4 * sign
    mean, iscale, yscale = L.norm_from_data(x, y)
    for k in range(L.N_IN):
        assert mean[k] == pytest.approx(0.25 * k - 3.0 if k != 5 else 7.0, abs=1e-13)
        if k == 5:
            assert iscale[k] == 0.0
        else:
            assert iscale[k] == pytest.approx(1.0 / (0.5 + 0.125 * k), rel=1e-12)
    for k in range(L.N_OUT - 1):
        assert yscale[k] == pytest.approx((1.0 + k) * 1e-4, rel=1e-12)
    assert yscale[L.N_OUT - 1] == 1.0
