"""Pins of the oracle's efficient-global-optimisation model (no GPU): the kriging predictor
interpolates, its error variance is the diffuse-mean limit of a plain Gaussian-process
posterior, the concentrated likelihood is the full likelihood at its optimum, EI equals its
defining integral, and the loop finds the Branin minimum; the space-filling start is a Latin
hypercube."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import ego as E
from paper_1603_09493_amd import inputs as I


def _data(n=14, d=3, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.random((n, d))
    y = np.sin(3 * X[:, 0]) + X[:, 1] ** 2 - 0.5 * X[:, 2] + 0.1 * np.cos(7 * X[:, 1])
    return X, y


def test_predictor_interpolates():
    X, y = _data()
    m = E.fit(X, y)
    yh, s = E.predict(X, y, m, X)
    assert np.abs(yh - y).max() <= 1e-6 * np.abs(y).max()
    assert s.max() <= 1e-3 * math.sqrt(m["sigma2"])


def test_variance_is_the_diffuse_mean_limit():
    X, y = _data(seed=1)
    m = dict(theta=np.array([2.0, 5.0, 1.0]), mu=None, sigma2=None)
    lnL, mu, s2, R = E.concentrated(X, y, m["theta"])
    m.update(mu=mu, sigma2=s2)
    x = np.random.default_rng(5).random((7, 3))
    yh, s = E.predict(X, y, m, x)
    # plain GP with covariance s2 R + V 1 1' (mean ~ N(0, V)), V large
    V = 1e7 * s2
    n = len(y)
    K = s2 * R + V * np.ones((n, n))
    k = s2 * E.corr(x, X, m["theta"]) + V
    kss = s2 * (1 + E.NUGGET) + V
    mean = k @ np.linalg.solve(K, y)
    var = kss - (k * np.linalg.solve(K, k.T).T).sum(1) - s2 * E.NUGGET
    assert np.abs(mean - yh).max() <= 1e-5 * np.abs(y).max()
    assert np.abs(var - s ** 2).max() <= 1e-4 * s2


def test_concentrated_likelihood_is_the_full_optimum():
    X, y = _data(seed=2)
    th = np.array([1.5, 3.0, 0.7])
    lnL, mu, s2, R = E.concentrated(X, y, th)
    n = len(y)
    Ri = np.linalg.inv(R)
    logdet = np.linalg.slogdet(R)[1]

    def full(mu_, s2_):
        e = y - mu_
        return -0.5 * n * math.log(2 * math.pi * s2_) - 0.5 * logdet - (e @ Ri @ e) / (2 * s2_)

    top = full(mu, s2)
    assert abs(top - (lnL - 0.5 * n * (math.log(2 * math.pi) + 1))) < 1e-9 * abs(top)
    for dm, ds in ((1e-3, 0), (-1e-3, 0), (0, 1e-3), (0, -1e-3)):
        assert full(mu + dm, s2 * (1 + ds)) < top


@pytest.mark.parametrize("mu,s,fmin", [(0.3, 0.2, 0.1), (-1.0, 0.5, 0.0), (2.0, 0.1, 0.0), (0.0, 1.0, 0.0)])
def test_ei_matches_its_integral(mu, s, fmin):
    ref, _ = integrate.quad(lambda t: (fmin - t) * math.exp(-0.5 * ((t - mu) / s) ** 2) / (s * math.sqrt(2 * math.pi)),
                            -np.inf, fmin, epsabs=1e-14, epsrel=1e-12)
    got = E.expected_improvement([mu], [s], fmin)[0]
    assert abs(got - ref) <= 1e-9 * max(abs(ref), 1e-300) + 1e-15
    assert E.expected_improvement([mu], [0.0], fmin)[0] == max(fmin - mu, 0.0)


def _branin(u):
    x1, x2 = 15 * u[0] - 5, 15 * u[1]
    return (x2 - 5.1 / (4 * math.pi ** 2) * x1 ** 2 + 5 / math.pi * x1 - 6) ** 2 + 10 * (1 - 1 / (8 * math.pi)) * math.cos(x1) + 10


def test_loop_finds_the_branin_minimum():
    X0 = I.lhs_maximin(10, 2, seed=3)
    X, y = E.minimize(_branin, 2, X0, iters=25, n_cand=4000, seed=1)
    assert y.min() < 0.397887 + 0.05, y.min()
    assert y[:10].min() > y.min()          # the EI steps improved on the start


def test_lhs_maximin_is_a_latin_hypercube():
    n, d = 30, 4
    U = I.lhs_maximin(n, d, seed=9, sweeps=40)
    for j in range(d):
        assert np.array_equal(np.sort((U[:, j] * n).astype(int)), np.arange(n))
    def mind(A):
        D = np.sqrt(((A[:, None] - A[None]) ** 2).sum(-1)); np.fill_diagonal(D, np.inf); return D.min()
    U0 = I.lhs_maximin(n, d, seed=9, sweeps=0)
    assert mind(U) > mind(U0)
