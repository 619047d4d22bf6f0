"""Host side of the GPU optimiser (no GPU): its likelihood fit reaches the oracle's optimum, and
the arrays it hands to the EI kernel reproduce the oracle's predictor and error estimate when the
kernel's formulas (v = G r; yhat = mu + v_n; s^2 = sigma^2 (1 - |v_<n|^2 + (1 - v_n+1)^2 / c)) are
applied to them on the CPU."""
import math

import numpy as np
import pytest

from oracle import ego as OE
from paper_1603_09493_amd import ego


def _data(seed, n, d):
    rng = np.random.default_rng(seed)
    X = rng.random((n, d))
    return X, np.cos(3 * X[:, 0]) + X.sum(1) ** 2 / d


@pytest.mark.parametrize("seed,n,d", [(0, 14, 3), (1, 25, 2)])
def test_fit_reaches_the_oracle_likelihood(seed, n, d):
    X, y = _data(seed, n, d)
    m = ego.fit(X, y)
    mo = OE.fit(X, y)
    got = OE.concentrated(X, y, m.theta)[0]
    assert got >= mo["lnL"] - 1e-6 * abs(mo["lnL"])
    assert abs(m.lnL - got) <= 1e-6 * abs(got)      # R is nearly singular at small theta


def test_kernel_arrays_reproduce_the_predictor():
    X, y = _data(3, 30, 4)
    theta = np.array([1.3, 0.4, 2.2, 0.9])
    _, mu, s2, _ = OE.concentrated(X, y, theta)
    pm = ego.model_arrays(X, y, theta)
    assert abs(pm.mu - mu) <= 1e-12 * abs(mu) and abs(pm.sigma2 - s2) <= 1e-10 * s2
    n = len(y)
    assert np.array_equal(pm.G[:n], np.tril(pm.G[:n]))
    C = np.random.default_rng(4).random((500, 4))
    r = np.exp(-(((C[:, None, :] - X[None]) ** 2) * theta).sum(-1))
    v = r @ pm.G.T
    yh = pm.mu + v[:, n]
    var = pm.sigma2 * (1 - (v[:, :n] ** 2).sum(1) + (1 - v[:, n + 1]) ** 2 / pm.c)
    yo, so = OE.predict(X, y, dict(theta=theta, mu=mu, sigma2=s2), C)
    assert np.abs(yh - yo).max() <= 1e-10 * np.abs(yo).max()
    assert np.abs(np.sqrt(np.maximum(var, 0)) - so).max() <= 1e-7 * math.sqrt(s2)


def test_unit_to_design_spans_the_box():
    from paper_1603_09493_amd import inputs as I
    assert np.allclose(ego.unit_to_design(np.zeros(4)), I.OPT_LO)
    assert np.allclose(ego.unit_to_design(np.ones(4)), I.OPT_HI)
