"""Efficient global optimisation (Jones, Schonlau and Welch 1998), the optimiser of Sec. II.A --
TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the bench's CPU baseline may import this module.

The model is the one of that method: the objective y(x) on the unit box is a constant mu plus a
Gaussian process with variance sigma^2 and correlation
    R(a, b) = exp(-sum_l theta_l (a_l - b_l)^2)          (+ g on the diagonal, g a tiny nugget)
whose parameters maximise the concentrated log-likelihood
    ln L(theta) = -(n/2) ln sigma^2(theta) - (1/2) ln |R(theta)|,
    mu(theta) = 1' R^-1 y / 1' R^-1 1,  sigma^2(theta) = (y - 1 mu)' R^-1 (y - 1 mu) / n.
At a new point x with correlations r to the n training points the predictor and its mean squared
error are
    yhat(x) = mu + r' R^-1 (y - 1 mu),
    s^2(x)  = sigma^2 [1 - r' R^-1 r + (1 - 1' R^-1 r)^2 / (1' R^-1 1)],
and the expected improvement over the best value f_min found so far is
    EI(x) = (f_min - yhat) Phi(z) + s phi(z),  z = (f_min - yhat) / s     (max(f_min - yhat, 0) if s = 0).
The optimiser evaluates the point of largest EI, adds it and refits, until the largest EI is small.
Every formula here is written out with dense solves, in FP64.
"""
from __future__ import annotations

import math

import numpy as np

NUGGET = 1e-10


def corr(A, B, theta):
    A = np.atleast_2d(A)
    B = np.atleast_2d(B)
    d2 = ((A[:, None, :] - B[None, :, :]) ** 2 * np.asarray(theta)[None, None, :]).sum(-1)
    return np.exp(-d2)


def concentrated(X, y, theta, g: float = NUGGET):
    """(ln L, mu, sigma^2, R) at correlation parameters theta."""
    n = len(y)
    R = corr(X, X, theta) + g * np.eye(n)
    one = np.ones(n)
    Ri1 = np.linalg.solve(R, one)
    Riy = np.linalg.solve(R, y)
    mu = (one @ Riy) / (one @ Ri1)
    e = y - mu
    s2 = (e @ np.linalg.solve(R, e)) / n
    sign, logdet = np.linalg.slogdet(R)
    if sign <= 0 or s2 <= 0:
        return -np.inf, mu, s2, R
    return -0.5 * n * math.log(s2) - 0.5 * logdet, mu, s2, R


def fit(X, y, starts: int = 8, seed: int = 0, lo: float = 1e-2, hi: float = 1e3):
    """theta maximising ln L (log-space search from several starts, Nelder-Mead)."""
    from scipy.optimize import minimize
    d = X.shape[1]
    rng = np.random.default_rng(seed)
    best = None
    for s in range(starts):
        z0 = rng.uniform(math.log(lo), math.log(hi), d) if s else np.full(d, math.log(1.0))
        f = lambda z: -concentrated(X, y, np.exp(np.clip(z, math.log(lo), math.log(hi))))[0]
        r = minimize(f, z0, method="Nelder-Mead", options=dict(maxiter=400 * d, xatol=1e-6, fatol=1e-9))
        if best is None or r.fun < best.fun:
            best = r
    theta = np.exp(np.clip(best.x, math.log(lo), math.log(hi)))
    lnL, mu, s2, _ = concentrated(X, y, theta)
    return dict(theta=theta, mu=mu, sigma2=s2, lnL=lnL)


def predict(X, y, model, x, g: float = NUGGET):
    """(yhat, s) at the rows of x."""
    theta, mu, s2 = model["theta"], model["mu"], model["sigma2"]
    n = len(y)
    R = corr(X, X, theta) + g * np.eye(n)
    one = np.ones(n)
    r = corr(x, X, theta)                                  # [m][n]
    Rir = np.linalg.solve(R, r.T)                          # [n][m]
    yhat = mu + r @ np.linalg.solve(R, y - mu)
    Ri1 = np.linalg.solve(R, one)
    var = s2 * (1.0 - (r * Rir.T).sum(1) + (1.0 - one @ Rir) ** 2 / (one @ Ri1))
    return yhat, np.sqrt(np.maximum(var, 0.0))


def expected_improvement(yhat, s, f_min):
    yhat = np.asarray(yhat, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    imp = f_min - yhat
    out = np.maximum(imp, 0.0)
    pos = s > 0
    z = imp[pos] / s[pos]
    Phi = 0.5 * np.array([math.erfc(-v / math.sqrt(2.0)) for v in z])
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    out[pos] = imp[pos] * Phi + s[pos] * phi
    return out


def minimize(f, d: int, X0, iters: int, n_cand: int = 20000, seed: int = 0, ei_tol: float = 0.0):
    """The optimisation loop: evaluate the start points X0, then repeatedly fit, pick the random
    candidate (n_cand uniform points) of largest EI, evaluate it, until iters points were added
    or the largest EI is <= ei_tol.  Returns (X, y)."""
    rng = np.random.default_rng(seed)
    X = np.array(X0, dtype=np.float64)
    y = np.array([f(x) for x in X])
    for it in range(iters):
        model = fit(X, y, seed=it)
        C = rng.random((n_cand, d))
        yh, s = predict(X, y, model, C)
        ei = expected_improvement(yh, s, y.min())
        k = int(np.argmax(ei))
        if ei[k] <= ei_tol:
            break
        X = np.vstack([X, C[k]])
        y = np.append(y, f(C[k]))
    return X, y
