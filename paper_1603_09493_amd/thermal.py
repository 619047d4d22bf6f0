"""Thermally induced erasure of an island in a stray field, by direct sampling of the stochastic
LLG equation on the GPU.

The paper obtains the erasure rate of a neighbouring bit from an energy barrier and an attempt
frequency that it takes from stochastic LLG simulations (Sec. II.C, Eq. (3)).  Here the
stochastic LLG itself is sampled: R realizations of one island (one mesh group, Philox keys
differing per realization) start along +z and are exposed to a static field along -z at a
temperature T; the erasure probability is the fraction whose hard-layer volume-averaged m_z ends
below zero.  Direct sampling resolves probabilities down to about 1/R, which is why the paper's
small bit-error rates need the barrier route instead.

The stochastic Heun integration and the observables run in the library (bpm_run with BPM_HEUN);
this module only builds the instances and counts.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import bpm
from . import inputs as I


@dataclasses.dataclass
class Erasure:
    n: int                 # realizations
    k: int                 # realizations whose hard layer reversed
    p: float               # k / n
    label: float           # logit of (k + 1/2) / (n + 1): finite at k = 0 and k = n
    status_ok: int         # realizations that ended with status 0
    kernel_ms: float
    wall_s: float


def logit_label(k: int, n: int) -> float:
    """Logit of the smoothed fraction (k + 1/2) / (n + 1), the surrogate's erasure label."""
    q = (k + 0.5) / (n + 1.0)
    return math.log(q / (1.0 - q))


def count_erased(results) -> tuple:
    """(erased, finished) over bpm results: erased = hard-layer <m_z> < 0 at the end."""
    ok = [r for r in results if r["status"] == 0]
    return sum(1 for r in ok if r["mz_hard"] < 0.0), len(ok)


def run_erasure(ctx: bpm.Context, mesh, mat, B_stray: float, realizations: int, t_end: float, dt: float,
                temperature: float = 300.0, key_base: int = 0, S=None, precision: int = 32,
                mesh_id: int | None = None) -> Erasure:
    """Exposes `realizations` copies of one island (from m = +z) to a static field B_stray along -z
    at `temperature` for t_end (stochastic Heun at dt); Philox key of realization r = key_base + r.
    S (optional) replaces the island's demag operator (e.g. zeros for a demag-free check)."""
    ctx.clear_instances()
    mid = ctx.mesh_add(mesh, S, keep=2 if precision == 32 else 1) if mesh_id is None else mesh_id
    fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=B_stray, dir=(0.0, 0.0, -1.0), t_rise=0.0)
    ids = [ctx.instance_add(mid, mat, fld, seed=key_base + r) for r in range(realizations)]
    t0 = time.perf_counter()
    ctx.run(t_end=t_end, precision=precision, integrator=bpm.HEUN, dt_fixed=dt, temperature=temperature)
    ctx.sync()
    wall = time.perf_counter() - t0
    res = ctx.results(ids)
    k, n_ok = count_erased(res)
    return Erasure(n=realizations, k=k, p=k / realizations, label=logit_label(k, realizations), status_ok=n_ok,
                   kernel_ms=ctx.last_run_info()["kernel_ms"], wall_s=wall)
