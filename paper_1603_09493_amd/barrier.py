"""Energy barrier of an island in a static head field and the adjacent-track error rate
(Sec. II.C, Eq. (3)) on the batched GPU solver.

The paper computes the barrier with a minimum-energy-path method (nudged elastic band) for the
adjacent bit 2 nm from the trailing edge, and turns it into BER_adj = t_write / tau with
tau = exp(E_B / kB T) / f0, f0 = 130 GHz, t_write = 1 ns, T = 300 K.  Here the minimum energy path
comes from the simplified string method (E, Ren and Vanden-Eijnden 2007) on the library's own
field and energy kernels:

* the P images of the chain are P instances of one mesh group;
* one iteration relaxes all of them in one launch (bpm_run with BPM_FLAG_RELAX: the LLG
  equation without its precession term, which descends the total energy) for a pseudo-time
  dtau, then bpm_string_reparam moves them back to equal spacing along the chain on the GPU and
  makes the result the next starting state;
* after the last iteration the energies of the relaxed images at their arc lengths give E_B
  (highest image minus the first, an interior maximum refined by the parabola through it and its
  two neighbours).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import bpm
from . import inputs as I

K_BOLTZMANN = 1.380649e-23
ATTEMPT_FREQUENCY = 130e9      # f0 (Sec. II.C)
WRITE_TIME = 1e-9              # t_write (Sec. II.C)


@dataclasses.dataclass
class Barrier:
    E_B: float                 # J
    energies: np.ndarray       # [P] J, relaxed images of the last iteration
    arclen: np.ndarray         # [P] arc length of those images along the chain
    images: list               # [P] of [3][n] relaxed images
    history: list              # E_B after every iteration
    kernel_ms: float


def profile_barrier(s, E) -> float:
    """Highest energy along the chain minus the first image's; an interior maximum is lifted to
    the vertex of the parabola through it and its two neighbours (s, E)."""
    s = np.asarray(s, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    k = int(np.argmax(E))
    top = float(E[k])
    if 0 < k < len(E) - 1:
        xs = s[k - 1:k + 2]
        A = np.stack([xs * xs, xs, np.ones(3)], axis=1)
        a, b, c = np.linalg.solve(A, E[k - 1:k + 2])
        if a < 0.0:
            xv = -b / (2.0 * a)
            if xs[0] <= xv <= xs[2]:
                top = max(top, float(c - b * b / (4.0 * a)))
    return top - float(E[0])


def string_barrier(ctx: bpm.Context, mid: int, n: int, mat, fld, chain, offset=(0.0, 0.0, 0.0),
                   dtau: float = 2e-12, iters: int = 60, precision: int = 64, rtol: float | None = None,
                   wg_per_group: int = 0, relax_alpha: float | None = 1.0) -> Barrier:
    """Simplified string method from `chain` ([P][3][n] initial images, e.g.
    inputs.rotation_chain) for one island on mesh group `mid` in the static field `fld`.  The
    relaxation runs use damping relax_alpha (the energy landscape does not depend on it; None
    keeps the material's)."""
    chain = np.asarray(chain, dtype=np.float64)
    P = chain.shape[0]
    if iters < 1 or not 3 <= P <= 64:
        raise ValueError("need iters >= 1 and 3..64 images")
    if rtol is None:
        rtol = 1e-6 if precision == 64 else 1e-5
    if relax_alpha is not None:
        mat = dataclasses.replace(mat, alpha=float(relax_alpha))
    ctx.clear_instances()
    ids = [ctx.instance_add(mid, mat, fld, offset=offset, m0=chain[k]) for k in range(P)]
    hist, ms = [], 0.0
    E = s = None
    for _ in range(iters):
        ctx.run(t_end=dtau, precision=precision, rtol=rtol, flags=bpm.FLAG_RELAX, wg_per_group=wg_per_group)
        ctx.sync()
        ms += ctx.last_run_info()["kernel_ms"]
        res = ctx.results(ids)
        bad = [r["status"] for r in res if r["status"] != 0]
        if bad:
            raise RuntimeError(f"string relaxation failed: statuses {bad}")
        E = np.array([r["energy"] for r in res])
        s = ctx.string_reparam(ids)
        hist.append(profile_barrier(s, E))
    images = [ctx.get_m(i, n) for i in ids]
    return Barrier(hist[-1], E, s, images, hist, ms)


def ber_adj(E_B: float, T: float = 300.0, f0: float = ATTEMPT_FREQUENCY, t_write: float = WRITE_TIME) -> float:
    """Eq. (3): the probability that the adjacent bit reverses during one write, t_write / tau."""
    return t_write * f0 * math.exp(-E_B / (K_BOLTZMANN * T))


def adjacent_error(ctx: bpm.Context, mesh, mid: int, mat, grid, g_origin, g_h, layout=None,
                   cross_offset: float = 0.0, P: int = 16, iters: int = 60, dtau: float = 2e-12,
                   precision: int = 64, T: float = 300.0):
    """(BER_adj, Barrier) of the adjacent island of `layout` in the head field `grid` (the island
    starts along +z, the head field points down)."""
    layout = I.recording_layout() if layout is None else layout
    fld = I.adjacent_field(grid, g_origin, g_h, layout=layout, cross_offset=cross_offset)
    b = string_barrier(ctx, mid, mesh.n, mat, fld, I.rotation_chain(mesh.n, P), offset=layout["adjacent"],
                       dtau=dtau, iters=iters, precision=precision)
    return ber_adj(b.E_B, T=T), b


def string_barrier_many(ctx: bpm.Context, mesh, mats, flds, chains, offsets, dtau: float = 2e-12, iters: int = 60,
                        precision: int = 64, rtol: float | None = None, relax_alpha: float | None = 1.0,
                        mids: list | None = None) -> list:
    """string_barrier for many strings of one island mesh in lock step: every iteration relaxes
    all images of all strings in one launch (64 // P strings per copy of the mesh group), then
    redistributes each string."""
    from .ber_driver import group_slots
    q = len(mats)
    chains = [np.asarray(c, dtype=np.float64) for c in chains]
    P = chains[0].shape[0]
    if iters < 1 or not 3 <= P <= 64 or q < 1:
        raise ValueError("need iters >= 1, 3..64 images and at least one string")
    if rtol is None:
        rtol = 1e-6 if precision == 64 else 1e-5
    mids = [] if mids is None else mids
    groups = group_slots(ctx, mesh, mids, q, P)
    ctx.clear_instances()
    ids = []
    for k in range(q):
        m = mats[k] if relax_alpha is None else dataclasses.replace(mats[k], alpha=float(relax_alpha))
        ids.append([ctx.instance_add(groups[k], m, flds[k], offset=tuple(offsets[k]), m0=chains[k][j]) for j in range(P)])
    hist = [[] for _ in range(q)]
    ms = 0.0
    E = [None] * q
    s = [None] * q
    for _ in range(iters):
        ctx.run(t_end=dtau, precision=precision, rtol=rtol, flags=bpm.FLAG_RELAX)
        ctx.sync()
        ms += ctx.last_run_info()["kernel_ms"]
        res = ctx.results([i for row in ids for i in row])
        bad = [r["status"] for r in res if r["status"] != 0]
        if bad:
            raise RuntimeError(f"string relaxation failed: statuses {bad[:8]}")
        for k in range(q):
            E[k] = np.array([r["energy"] for r in res[k * P:(k + 1) * P]])
            s[k] = ctx.string_reparam(ids[k])
            hist[k].append(profile_barrier(s[k], E[k]))
    n = mesh.n
    return [Barrier(hist[k][-1], E[k], s[k], [ctx.get_m(i, n) for i in ids[k]], hist[k], ms) for k in range(q)]


def adjacent_errors_many(ctx: bpm.Context, mesh, mats, grid, g_origin, g_h, cross_offsets, layout=None,
                         P: int = 16, iters: int = 60, dtau: float = 2e-12, precision: int = 64, T: float = 300.0,
                         mids: list | None = None):
    """adjacent_error for many designs (materials and cross-track offsets) in lock step:
    returns [(BER_adj, Barrier)]."""
    layout = I.recording_layout() if layout is None else layout
    flds = [I.adjacent_field(grid, g_origin, g_h, layout=layout, cross_offset=c) for c in cross_offsets]
    chains = [I.rotation_chain(mesh.n, P)] * len(mats)
    bs = string_barrier_many(ctx, mesh, mats, flds, chains, [layout["adjacent"]] * len(mats), dtau=dtau,
                             iters=iters, precision=precision, mids=mids)
    return [(ber_adj(b.E_B, T=T), b) for b in bs]
