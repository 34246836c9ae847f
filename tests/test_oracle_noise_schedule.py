"""Pins of the oracle's noise stream and switching schedules.

The Philox bit stream is pinned by the generator's published known-answer
vectors (tests/golden/philox4x32_10_kat.txt), the Gaussian deviates by their
statistics and by their determinism.  The schedules are pinned by the properties the paper
states for lambda(tau): end points, vanishing end slopes, the closed-form
slope 630 tau^4 (1-tau)^4 of the polynomial, and the RS form giving a
temperature linear in tau."""
import os

import numpy as np
import pytest
from scipy import stats


def _draws(O, n, seed=0, step=0, stream=0):
    return np.array([O.gauss3(seed, i, step, stream) for i in range(n)])


def test_philox_known_answers(oracle_lib):
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(v, 16) for v in r]
        assert list(oracle_lib.philox(w[0:4], w[4:6])) == w[6:10]


def test_gaussian_moments(oracle_lib):
    z = _draws(oracle_lib, 40000).ravel()
    assert abs(z.mean()) < 0.01
    assert z.var() == pytest.approx(1.0, abs=0.015)
    assert abs(stats.skew(z)) < 0.03
    assert stats.kurtosis(z, fisher=False) == pytest.approx(3.0, abs=0.06)
    # Kolmogorov-Smirnov against the standard normal
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_gaussian_independence(oracle_lib):
    a = _draws(oracle_lib, 20000, seed=3, step=10)
    b = _draws(oracle_lib, 20000, seed=3, step=11)
    c = _draws(oracle_lib, 20000, seed=3, step=10, stream=1)
    d = _draws(oracle_lib, 20000, seed=4, step=10)
    for u, v in ((a, b), (a, c), (a, d)):
        assert abs(np.corrcoef(u.ravel(), v.ravel())[0, 1]) < 0.02
    cc = np.corrcoef(a.T)
    assert np.abs(cc - np.eye(3)).max() < 0.03


def test_noise_is_counter_based(oracle_lib):
    z1 = oracle_lib.gauss3(123456789012, 77, 4242, 0)
    z2 = oracle_lib.gauss3(123456789012, 77, 4242, 0)
    assert np.array_equal(z1, z2)
    assert not np.array_equal(z1, oracle_lib.gauss3(123456789012, 77, 4243, 0))
    assert not np.array_equal(z1, oracle_lib.gauss3(123456789013, 77, 4242, 0))
    # high bits of the step and of the seed are part of the key / counter
    assert not np.array_equal(oracle_lib.gauss3(0, 1, 5, 0), oracle_lib.gauss3(0, 1, 5 + (1 << 32), 0))
    assert not np.array_equal(oracle_lib.gauss3(1, 1, 5, 0), oracle_lib.gauss3(1 + (1 << 32), 1, 5, 0))


def test_philox_words_uniform(oracle_lib):
    words = np.array([oracle_lib.philox([i, 7, 0, 0], [99, 0]) for i in range(10000)], dtype=np.uint64).ravel()
    top = (words >> np.uint64(24)).astype(np.int64)
    counts = np.bincount(top, minlength=256)
    assert stats.chisquare(counts).pvalue > 1e-3
    low = (words & np.uint64(0xFF)).astype(np.int64)
    assert stats.chisquare(np.bincount(low, minlength=256)).pvalue > 1e-3


def test_fl_polynomial_properties(oracle_lib):
    f = lambda t: oracle_lib.lambda_fl(2, t)
    assert f(0.0) == 0.0
    assert f(1.0) == pytest.approx(1.0, abs=1e-14)
    taus = np.linspace(0.0, 1.0, 101)
    for t in taus:
        assert f(1.0 - t) == pytest.approx(1.0 - f(t), abs=1e-13)
    # five-point stencil: the power-basis form loses ~1e-13 to cancellation near tau = 1
    h = 1e-3
    for t in np.linspace(0.01, 0.99, 49):
        slope = (f(t - 2 * h) - 8 * f(t - h) + 8 * f(t + h) - f(t + 2 * h)) / (12 * h)
        assert slope == pytest.approx(630.0 * t ** 4 * (1.0 - t) ** 4, abs=1e-8)
    assert (f(1e-3) - f(0.0)) / 1e-3 < 1e-9 and (f(1.0) - f(1.0 - 1e-3)) / 1e-3 < 1e-9
    vals = [f(t) for t in taus]
    assert np.all(np.diff(vals) >= 0)
    assert oracle_lib.lambda_fl(1, 0.37) == 0.37


def test_rs_temperature_is_linear_in_tau(oracle_lib):
    T0, Tf = 100.0, 1600.0
    lf = T0 / Tf
    for t in np.linspace(0, 1, 21):
        lam = oracle_lib.lambda_rs(lf, t)
        assert T0 / lam == pytest.approx(T0 + t * (Tf - T0), rel=1e-13)


def test_schedule_layout(oracle_lib):
    lam = oracle_lib.schedule("fl", 10, 20, 5, 7, function=2)
    assert len(lam) == 10 + 40 + 5 + 7 + 1
    assert np.all(lam[:11] == 0.0)
    assert lam[30] == pytest.approx(1.0, abs=1e-14)
    assert np.all(np.abs(lam[30:36] - 1.0) < 1e-14)
    assert lam[55] == pytest.approx(0.0, abs=1e-14)
    assert np.all(lam[55:] == 0.0)
    # backward branch is the time reverse of the forward one
    assert np.allclose(lam[35:56], lam[10:31][::-1], atol=1e-14)
    rs = oracle_lib.schedule("rs", 4, 8, 2, 0, lambda_f=0.25)
    assert rs[0] == 1.0 and rs[4] == 1.0
    assert rs[12] == pytest.approx(0.25) and rs[14] == pytest.approx(0.25)
    assert rs[-1] == pytest.approx(1.0)
    assert np.allclose(rs[14:23], rs[4:13][::-1])
