"""Host-side logic of the learned-form driver (no GPU): parameter layout and initial
weights, units, and the error metrics applied to the energy histories."""
import math

import numpy as np
import pytest

learned = pytest.importorskip("paper_2605_14505_amd.learned")


def test_initial_network_is_the_plain_method():
    theta = learned.init_params(0)
    assert theta.dtype == np.float32 and theta.size == learned.NPARAM == 9897
    w1 = theta[:64 * 47].reshape(64, 47)
    out = theta[-(41 * 64 + 41):]
    assert np.all(out == 0.0)                                  # zero output layer and bias
    assert abs(w1).max() <= math.sqrt(6.0 / (47 + 64)) and w1.std() > 0.05
    assert np.array_equal(theta, learned.init_params(0))       # seeded
    assert not np.array_equal(theta, learned.init_params(1))


def test_steps_per_unit_time():
    # L = n / 2 pi lattice units, U = u0: 256^3 at u0 = 0.05 takes 814.9 steps per L/U
    assert math.isclose(learned.steps_per_unit_time(256), 256 / (2 * math.pi) / 0.05)
    assert math.isclose(learned.steps_per_unit_time(256), 4 * learned.steps_per_unit_time(64))


def _records(ts, ek, ep, eps=None):
    return [{"t": t, "ek": a, "ep": b, "eps_k": (eps[i] if eps is not None else 0.0), "eps_p": 0.0,
             "nonfinite": 0} for i, (t, a, b) in enumerate(zip(ts, ek, ep))]


def test_decay_rate_of_an_exponential_energy():
    t = np.linspace(0.0, 5.0, 201)
    e = np.exp(-0.3 * t)
    tt, rate = learned.decay_rate(_records(t, 0.5 * e, 0.5 * e))
    np.testing.assert_allclose(tt, t[1:-1])
    # central differences of exp(-a t): a e sinh(a h)/(a h), h = 0.025
    h = t[1] - t[0]
    np.testing.assert_allclose(rate, 0.3 * e[1:-1] * math.sinh(0.3 * h) / (0.3 * h), rtol=1e-12)


def test_series_errors_on_known_offsets():
    t = np.linspace(0.0, 3.0, 31)
    d = np.exp(-t)
    ref = _records(t, 2.0 * d, 1.0 * d, eps=np.full(31, 0.5))
    run = _records(t, 2.2 * d, 0.9 * d, eps=np.full(31, 0.5))
    e = learned.series_errors(run, ref)
    assert e["finite"] and e["records"] == 31
    assert math.isclose(e["ek"], 0.1) and math.isclose(e["ep"], 0.1) and e["eps_k"] == 0.0
    # E = 3.1 d against 3 d: the decay rate is off by 1/30
    assert math.isclose(e["dEdt"], 0.1 / 3.0, rel_tol=1e-12)
    assert e["eps_p"] == 0.0                                   # zero reference, exact match
    assert math.isclose(learned.score(e), e["ek"] + e["ep"] + e["dEdt"])
    # a non-finite record makes every error infinite
    bad = [dict(r) for r in run]
    bad[5]["ek"] = math.nan
    assert learned.series_errors(bad, ref)["ek"] == math.inf
    # only common record times are compared
    assert learned.series_errors(run[::2], ref)["records"] == 16
