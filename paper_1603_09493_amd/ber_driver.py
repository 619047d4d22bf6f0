"""Critical-field search and write bit-error rate (Sec. II.C, Fig. 4, Eqs. (1)-(2)) on top of the
batched solver.

For one design the paper runs 12 recording simulations side by side, each with a different
global field H_ext working against the head field, on a grid of half the switching-field
distribution width sigma = 0.015 mu0 H_A (mu0 H_A = 2 K_1,hard / J_S), and refines the bracket
between the last field that still lets the target switch and the first that prevents it twice.
BER_targ = 1/2 [1 - erf(H_crit / sqrt(2 sigma^2))].  If the head cannot switch the target even
without H_ext the evaluation is aborted with BER = 1 (Fig. 1).

Here the 12 simulations of a level are 12 instances of one batched launch (one mesh group).
The target and the previous bit are the islands of the pseudo-hexagonal layout at their own
positions under the same moving head field (inputs.recording_layout / recording_field); H_ext
points along the head field at the island's centre, taken where that field is strongest during
the write period (for a uniform or pole field: its `dir`).  Evaluation is sequential with early
abort (Sec. II.C): a head that cannot write the target, or that rewrites the previous bit even
without H_ext, gives BER_tot = 1 and the later error rates are not computed.
The paper states the critical field was always inside {0..4 sigma}, yet its shingled designs of
Table III imply about 5.4 and 6.0 sigma through Eq. (1); the first level therefore spans
{0, sigma/2, ..., 5.5 sigma} and is extended while every field still switches.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import bpm
from . import inputs as I


def sigma_T(K_hard: float, Ms_hard: float) -> float:
    """sigma in tesla: 0.015 * 2 K_1,hard / Ms_hard (= 0.015 mu0 H_A with J_S = mu0 Ms)."""
    return 0.015 * 2.0 * K_hard / Ms_hard


def ber_from_hcrit(h: float, sigma: float) -> float:
    """Eqs. (1)-(2), written with erfc so that rates far in the tail keep their digits."""
    return 0.5 * math.erfc(h / math.sqrt(2.0 * sigma * sigma))


@dataclasses.dataclass
class Search:
    h_crit: float            # tesla (midpoint of the final bracket)
    lo: float                # largest field that still writes (tesla)
    hi: float                # smallest field that no longer writes (tesla)
    sigma: float             # tesla
    ber: float
    levels: list             # [(fields [12], switched [12])]
    aborted: bool


def _trilinear(grid, origin, h, p):
    """Trilinear sample of a [3][nz][ny][nx] grid at point p (zero outside the grid)."""
    nz, ny, nx = grid.shape[1:]
    u = (np.asarray(p, dtype=np.float64) - np.asarray(origin, dtype=np.float64)) / h
    n = np.array([nx, ny, nz])
    if np.any(u < 0.0) or np.any(u > n - 1):
        return np.zeros(3)
    i = np.minimum(np.floor(u).astype(int), n - 2)
    f = u - i
    out = np.zeros(3)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = (f[0] if dx else 1 - f[0]) * (f[1] if dy else 1 - f[1]) * (f[2] if dz else 1 - f[2])
                out += w * grid[:, i[2] + dz, i[1] + dy, i[0] + dx]
    return out


def head_direction(fld, centre, t_end: float, samples: int = 128) -> np.ndarray:
    """Unit vector of the head field (without B_ext) at `centre`, where its magnitude peaks over
    [0, t_end]; the field's `dir` for the uniform and pole kinds."""
    if fld.kind != I.FIELD_GRID:
        d = np.asarray(fld.dir, dtype=np.float64)
        return d / np.linalg.norm(d)
    best, bn = None, -1.0
    c = np.asarray(centre, dtype=np.float64)
    for t in np.linspace(0.0, t_end, samples):
        s = c - np.asarray(fld.x_off) - np.asarray(fld.v) * t
        b = _trilinear(fld.grid, fld.g_origin, fld.g_h, s)
        nb = float(np.linalg.norm(b))
        if nb > bn:
            best, bn = b, nb
    if bn <= 0.0:
        raise ValueError("the head field is zero at the island along its whole path")
    return best / bn


def _level(ctx, mid, mat, fld, fields, t_end, precision, previous, offset, hdir):
    """One level: len(fields) instances with H_ext along -hdir (target) or +hdir (previous bit)."""
    ctx.clear_instances()
    sign = 1.0 if previous else -1.0
    ids = []
    for h in fields:
        f = dataclasses.replace(fld, B_ext=tuple(np.asarray(fld.B_ext) + sign * h * hdir))
        ids.append(ctx.instance_add(mid, mat, f, offset=offset))
    ctx.run(t_end=t_end, precision=precision, rtol=1e-5 if precision == 32 else 1e-6)
    ctx.sync()
    res = ctx.results(ids)
    if any(r["status"] != 0 for r in res):
        raise RuntimeError(f"recording simulation failed: statuses {[r['status'] for r in res]}")
    return np.array([bool(r["switched"]) for r in res])


class HcritSearch:
    """The critical-field search of one island as a state machine, so that the searches of many
    designs can share launches: next_fields() is the H_ext of the next level (None when done),
    feed() takes that level's switched flags; result holds the Search when done.

    First level {0, sigma/2, ..., 5.5 sigma}: abort if H_ext = 0 already fails; extended by 12
    further steps of sigma/2 while every field writes (at most max_extend times); then the bracket
    between the last field that writes and the first that fails is refined `refinements` times
    on 12 interior points."""

    def __init__(self, mat, fld, t_end: float = 1e-9, previous: bool = False, n_par: int = 12,
                 refinements: int = 2, max_extend: int = 4, offset=(0.0, 0.0, 0.0), centre=None):
        self.sig = sigma_T(mat.K[1], mat.Ms[1])
        self.hdir = head_direction(fld, offset if centre is None else centre, t_end)
        self.mat, self.fld, self.previous, self.offset = mat, fld, previous, tuple(offset)
        self.n_par, self.refinements, self.max_extend = n_par, refinements, max_extend
        self.levels = []
        self.phase = "first"
        self.fields = 0.5 * self.sig * np.arange(n_par)
        self.ext = self.ref = 0
        self.lo = self.hi = 0.0
        self.result = None

    def next_fields(self):
        return None if self.result is not None else self.fields

    def _finish(self):
        h = 0.5 * (self.lo + self.hi)
        self.result = Search(h, self.lo, self.hi, self.sig, ber_from_hcrit(h, self.sig), self.levels, False)

    def _refine_grid(self):
        self.fields = self.lo + (self.hi - self.lo) * np.arange(1, self.n_par + 1) / (self.n_par + 1)

    def feed(self, switched):
        sw = np.asarray(switched, dtype=bool)
        ok = ~sw if self.previous else sw          # True where writing succeeds
        f = self.fields
        self.levels.append((f.copy(), ok.copy()))
        if self.phase == "first":
            if not ok[0]:
                self.result = Search(0.0, 0.0, 0.0, self.sig, 1.0, self.levels, True)
                return
            self.phase = "extend"
        if self.phase == "extend":
            if ok.all():
                if self.ext < self.max_extend:
                    self.ext += 1
                    self.fields = f[-1] + 0.5 * self.sig * np.arange(1, self.n_par + 1)
                    return
                h = float(f[-1])
                self.result = Search(h, h, math.inf, self.sig, ber_from_hcrit(h, self.sig), self.levels, False)
                return
            ff = int(np.argmax(~ok))
            self.lo = float(f[ff - 1]) if ff > 0 else float(self.levels[-2][0][-1])
            self.hi = float(f[ff])
            self.phase = "refine"
            if self.refinements == 0:
                self._finish()
            else:
                self._refine_grid()
            return
        # refinement level
        if ok.all():
            self.lo = float(f[-1])
        else:
            ff = int(np.argmax(~ok))
            self.hi = float(f[ff])
            self.lo = float(f[ff - 1]) if ff > 0 else self.lo
        self.ref += 1
        if self.ref >= self.refinements:
            self._finish()
        else:
            self._refine_grid()


def critical_field(ctx: bpm.Context, mid: int, mat, fld, t_end: float = 1e-9, precision: int = 32,
                   previous: bool = False, n_par: int = 12, refinements: int = 2, max_extend: int = 4,
                   offset=(0.0, 0.0, 0.0), centre=None) -> Search:
    """H_crit for the target bit (previous=False: switching must still happen) or for the
    previous bit (previous=True: it must stay unswitched), the island placed at `offset`.
    `centre` (default: offset) is where the H_ext direction is taken."""
    srch = HcritSearch(mat, fld, t_end, previous, n_par, refinements, max_extend, offset, centre)
    while (fields := srch.next_fields()) is not None:
        srch.feed(_level(ctx, mid, mat, fld, fields, t_end, precision, previous, srch.offset, srch.hdir))
    return srch.result


def group_slots(ctx: bpm.Context, mesh, mids: list, need: int, per_group: int, keep: int = 3) -> list:
    """Mesh groups (copies of `mesh`) for `need` jobs of per_group instances each, at most 64
    instances per group: returns the group of every job, adding copies to `mids` as needed."""
    jobs_per_group = max(1, 64 // per_group)
    while len(mids) * jobs_per_group < need:
        mids.append(ctx.mesh_add(mesh, keep=keep))
    return [mids[j // jobs_per_group] for j in range(need)]


def _levels_many(ctx, groups, searches, t_end, precision):
    """One launch for the pending level of every search (12 instances each, on its own group)."""
    ctx.clear_instances()
    ids = []
    for g, s in zip(groups, searches):
        sign = 1.0 if s.previous else -1.0
        ids.append([ctx.instance_add(g, s.mat, dataclasses.replace(
            s.fld, B_ext=tuple(np.asarray(s.fld.B_ext) + sign * h * s.hdir)), offset=s.offset)
            for h in s.next_fields()])
    ctx.run(t_end=t_end, precision=precision, rtol=1e-5 if precision == 32 else 1e-6)
    ctx.sync()
    flat = ctx.results([i for row in ids for i in row])
    bad = [r["status"] for r in flat if r["status"] != 0]
    if bad:
        raise RuntimeError(f"recording simulation failed: statuses {bad[:8]}")
    out, k = [], 0
    for row in ids:
        out.append(np.array([bool(r["switched"]) for r in flat[k:k + len(row)]]))
        k += len(row)
    return out


def run_searches(ctx: bpm.Context, mesh, mids: list, searches: list, t_end: float, precision: int) -> int:
    """Advances every search to its end, all pending levels in one launch per round; returns the
    number of launches."""
    rounds = 0
    while True:
        live = [s for s in searches if s.next_fields() is not None]
        if not live:
            return rounds
        groups = group_slots(ctx, mesh, mids, len(live), live[0].n_par)
        for s, sw in zip(live, _levels_many(ctx, groups, live, t_end, precision)):
            s.feed(sw)
        rounds += 1


@dataclasses.dataclass
class WriteErrors:
    ber_targ: float
    ber_prev: float          # 1.0 when aborted at the target stage (not evaluated)
    ber_tot: float           # BER_targ + BER_prev, + BER_adj when given; 1 on abort
    stage: str               # "done", or the stage that aborted: "targ" / "prev"
    targ: Search
    prev: Search | None


def write_errors(ctx: bpm.Context, mesh, mid: int, mat, fld, layout=None, t_end: float = I.BIT_PERIOD,
                 precision: int = 32, ber_adj=None, **search) -> WriteErrors:
    """BER_targ, then BER_prev (Eqs. (1)-(2)) for one design, with the early abort of Sec. II.C.

    The target and the previous island (layout: inputs.recording_layout()) see the same moving
    head field `fld` over one write period.  ber_adj, when given, is a callable returning BER_adj
    (Eq. (3)); it is called only when both write stages passed."""
    layout = I.recording_layout() if layout is None else layout
    zc = 0.5 * (float(mesh.xyz[2].min()) + float(mesh.xyz[2].max()))
    at = lambda p: (float(p[0]), float(p[1]), float(p[2]))
    ctr = lambda p: (float(p[0]), float(p[1]), float(p[2]) + zc)
    targ = critical_field(ctx, mid, mat, fld, t_end=t_end, precision=precision, previous=False,
                          offset=at(layout["target"]), centre=ctr(layout["target"]), **search)
    if targ.aborted:
        return WriteErrors(1.0, 1.0, 1.0, "targ", targ, None)
    prev = critical_field(ctx, mid, mat, fld, t_end=t_end, precision=precision, previous=True,
                          offset=at(layout["previous"]), centre=ctr(layout["previous"]), **search)
    if prev.aborted:
        return WriteErrors(targ.ber, 1.0, 1.0, "prev", targ, prev)
    tot = targ.ber + prev.ber
    if ber_adj is not None:
        tot += float(ber_adj())
    return WriteErrors(targ.ber, prev.ber, min(1.0, tot), "done", targ, prev)


def write_errors_many(ctx: bpm.Context, mesh, designs, layout=None, t_end: float = I.BIT_PERIOD,
                      precision: int = 32, adjacent=None, mids: list | None = None, **search) -> list:
    """write_errors for many designs [(mat, fld), ...] of one island mesh, in lock step: every
    round runs the pending level of every design's search in one launch (12 instances per design,
    five designs per copy of the mesh group), so the GPU holds 12 q islands instead of 12.  The
    stages stay sequential per design with the early abort.  adjacent, when given, is a callable
    taking the list of indices of the designs that passed both write stages and returning their
    BER_adj values (e.g. from barrier.string_barrier_many)."""
    layout = I.recording_layout() if layout is None else layout
    mids = [] if mids is None else mids
    zc = 0.5 * (float(mesh.xyz[2].min()) + float(mesh.xyz[2].max()))
    at = lambda p: (float(p[0]), float(p[1]), float(p[2]))
    ctr = lambda p: (float(p[0]), float(p[1]), float(p[2]) + zc)
    targ = [HcritSearch(m, f, t_end, False, offset=at(layout["target"]), centre=ctr(layout["target"]), **search)
            for m, f in designs]
    run_searches(ctx, mesh, mids, targ, t_end, precision)
    ok_t = [i for i, s in enumerate(targ) if not s.result.aborted]
    prev = {i: HcritSearch(designs[i][0], designs[i][1], t_end, True, offset=at(layout["previous"]),
                           centre=ctr(layout["previous"]), **search) for i in ok_t}
    run_searches(ctx, mesh, mids, list(prev.values()), t_end, precision)
    ok_p = [i for i in ok_t if not prev[i].result.aborted]
    adj = dict(zip(ok_p, adjacent(ok_p))) if (adjacent is not None and ok_p) else {}
    out = []
    for i, t in enumerate(targ):
        if t.result.aborted:
            out.append(WriteErrors(1.0, 1.0, 1.0, "targ", t.result, None))
            continue
        p = prev[i].result
        if p.aborted:
            out.append(WriteErrors(t.result.ber, 1.0, 1.0, "prev", t.result, p))
            continue
        tot = t.result.ber + p.ber + float(adj.get(i, 0.0))
        out.append(WriteErrors(t.result.ber, p.ber, min(1.0, tot), "done", t.result, p))
    return out
