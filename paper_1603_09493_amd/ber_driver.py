"""Critical-field search and write bit-error rate (Sec. II.C, Fig. 4, Eqs. (1)-(2)) on top of the
batched solver.

For one design the paper runs 12 recording simulations side by side, each with a different
global field H_ext working against the head field, on a grid of half the switching-field
distribution width sigma = 0.015 mu0 H_A (mu0 H_A = 2 K_1,hard / J_S), and refines the bracket
between the last field that still lets the target switch and the first that prevents it twice.
BER_targ = 1/2 [1 - erf(H_crit / sqrt(2 sigma^2))].  If the head cannot switch the target even
without H_ext the evaluation is aborted with BER = 1 (Fig. 1).

Here the 12 simulations of a level are 12 instances of one batched launch (one mesh group).
The paper states the critical field was always inside {0..4 sigma}, yet its shingled designs of
Table III imply about 5.4 and 6.0 sigma through Eq. (1); the first level therefore spans
{0, sigma/2, ..., 5.5 sigma} and is extended while every field still switches.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import bpm


def sigma_T(K_hard: float, Ms_hard: float) -> float:
    """sigma in tesla: 0.015 * 2 K_1,hard / Ms_hard (= 0.015 mu0 H_A with J_S = mu0 Ms)."""
    return 0.015 * 2.0 * K_hard / Ms_hard


def ber_from_hcrit(h: float, sigma: float) -> float:
    return 0.5 * (1.0 - math.erf(h / math.sqrt(2.0 * sigma * sigma)))


@dataclasses.dataclass
class Search:
    h_crit: float            # tesla (midpoint of the final bracket)
    lo: float                # largest field that still writes (tesla)
    hi: float                # smallest field that no longer writes (tesla)
    sigma: float             # tesla
    ber: float
    levels: list             # [(fields [12], switched [12])]
    aborted: bool


def _level(ctx, mid, mat, fld, fields, t_end, precision, previous):
    """One level: 12 instances with H_ext along -dir (target) or +dir (previous bit)."""
    ctx.clear_instances()
    d = np.asarray(fld.dir, dtype=np.float64)
    sign = 1.0 if previous else -1.0
    ids = []
    for h in fields:
        f = dataclasses.replace(fld, B_ext=tuple(sign * h * d))
        ids.append(ctx.instance_add(mid, mat, f))
    ctx.run(t_end=t_end, precision=precision, rtol=1e-5 if precision == 32 else 1e-6)
    ctx.sync()
    res = ctx.results(ids)
    return np.array([bool(r["switched"]) for r in res])


def critical_field(ctx: bpm.Context, mid: int, mat, fld, t_end: float = 1e-9, precision: int = 32,
                   previous: bool = False, n_par: int = 12, refinements: int = 2, max_extend: int = 4) -> Search:
    """H_crit for the target bit (previous=False: switching must still happen) or for the
    previous bit (previous=True: it must stay unswitched)."""
    sig = sigma_T(mat.K[1], mat.Ms[1])
    want = (lambda sw: ~sw) if previous else (lambda sw: sw)   # True where writing succeeds
    fields = 0.5 * sig * np.arange(n_par)
    levels = []
    ok = want(_level(ctx, mid, mat, fld, fields, t_end, precision, previous))
    levels.append((fields.copy(), ok.copy()))
    if not ok[0]:
        return Search(0.0, 0.0, 0.0, sig, 1.0, levels, True)
    ext = 0
    while ok.all() and ext < max_extend:
        fields = fields[-1] + 0.5 * sig * np.arange(1, n_par + 1)
        ok = want(_level(ctx, mid, mat, fld, fields, t_end, precision, previous))
        levels.append((fields.copy(), ok.copy()))
        ext += 1
    if ok.all():
        h = float(fields[-1])
        return Search(h, h, math.inf, sig, ber_from_hcrit(h, sig), levels, False)
    # bracket: last success before the first failure
    first_fail = int(np.argmax(~ok))
    lo = float(fields[first_fail - 1]) if first_fail > 0 else float(levels[-2][0][-1])
    hi = float(fields[first_fail])
    for _ in range(refinements):
        fields = lo + (hi - lo) * np.arange(1, n_par + 1) / (n_par + 1)
        ok = want(_level(ctx, mid, mat, fld, fields, t_end, precision, previous))
        levels.append((fields.copy(), ok.copy()))
        if ok.all():
            lo = float(fields[-1])
        else:
            ff = int(np.argmax(~ok))
            hi = float(fields[ff])
            lo = float(fields[ff - 1]) if ff > 0 else lo
    h = 0.5 * (lo + hi)
    return Search(h, lo, hi, sig, ber_from_hcrit(h, sig), levels, False)
