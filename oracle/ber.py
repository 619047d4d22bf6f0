"""Bit-error-rate formulas of the paper (Sec. II.C) -- TEST INFRASTRUCTURE ONLY.

* switching-field distribution: sigma = 0.015 H_A with H_A = 2 K_1,hard / J_S (Sec. II.C),
  expressed here in tesla (mu0 H_A = 2 mu0 K_1,hard / J_S = 2 K_1,hard / Ms_hard);
* Eqs. (1)/(2): BER = 1/2 [1 - erf(H_crit / sqrt(2 sigma^2))];
* Eq. (3): BER_adj = t_write / tau with tau = exp(E_B / kB T) / f0, f0 = 130 GHz, t_write = 1 ns;
* BER_tot is the sum of the three.
"""
from __future__ import annotations

import math

MU0 = 4e-7 * math.pi
F0 = 130e9          # attempt frequency (Sec. II.C)
T_WRITE = 1e-9      # field exposure time during writing (Sec. II.C)


def sigma_T(K_hard: float, Js: float) -> float:
    """sigma of the switching-field distribution in tesla: 0.015 mu0 H_A, H_A = 2 K / J_S (A/m)."""
    return 0.015 * MU0 * 2.0 * K_hard / Js


def ber_crit(H_crit: float, sigma: float) -> float:
    """Eqs. (1)/(2): tail of the Gaussian SFD beyond the critical field (same units)."""
    return 0.5 * (1.0 - math.erf(H_crit / math.sqrt(2.0 * sigma * sigma)))


def ber_adj(E_B_over_kT: float) -> float:
    """Eq. (3) with tau = f0^-1 exp(E_B / kB T)."""
    return T_WRITE * F0 * math.exp(-E_B_over_kT)


def p_switch(H_crit: float, sigma: float) -> float:
    """Probability that the target island is written: 1 - BER_targ."""
    return 1.0 - ber_crit(H_crit, sigma)


def h_crit_from_ber(ber: float, sigma: float) -> float:
    """Inverse of Eq. (1) by bisection (monotone in H_crit)."""
    lo, hi = 0.0, 40.0 * sigma
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if ber_crit(mid, sigma) > ber:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
