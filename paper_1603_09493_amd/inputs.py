"""Seeded synthetic inputs: island meshes, materials, head-field schedules and design batches.

This module produces *inputs* only.  It holds none of the method's arithmetic: no finite-element
quantities, no fields, no time stepping.  Both the GPU library (through its Python binding) and
the CPU oracle consume exactly the arrays it returns, so that a parity test compares two
independent solvers on the same bytes.

Geometry follows the media description of the paper (Sec. II.B and Fig. 3): a cylindrical or
elliptic exchange-coupled-composite island, soft layer on top (nearest the head, which is the
reading that makes "9 nm below the air bearing surface is the middle of the soft phase" in
Sec. III consistent with the 6 nm spacing), hard layer below, both easy axes along z.  The paper
meshes with NETGEN; here a seeded extruded mesher stands in for it:

* a 2-D Delaunay triangulation of boundary samples plus a jittered hexagonal interior lattice,
* extruded into z-levels (the soft/hard interface is a level),
* each prism cut into three tetrahedra by a rule that depends only on the global 2-D node
  indices, which keeps neighbouring prisms conforming,
* interface nodes duplicated: the soft copy and the hard copy carry the same coordinates and are
  listed as pairs, so each node belongs to exactly one layer.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial import Delaunay

NM = 1e-9

# Field kinds understood by both solvers.
FIELD_UNIFORM = 0
FIELD_POLE = 1
FIELD_GRID = 2

LAYER_SOFT = 0
LAYER_HARD = 1


@dataclasses.dataclass
class Mesh:
    """P1 tetrahedral island mesh (SI units)."""
    xyz: np.ndarray          # [3][n] float64, metres
    tet: np.ndarray          # [ntet][4] int32, positively oriented
    layer: np.ndarray        # [n] int32, 0 = soft (top), 1 = hard (bottom)
    iface: np.ndarray        # [nif][2] int32, (soft node, hard node) with equal coordinates
    n2d: int = 0             # 2-D nodes per level (informational)

    @property
    def n(self) -> int:
        return int(self.xyz.shape[1])

    @property
    def ntet(self) -> int:
        return int(self.tet.shape[0])


@dataclasses.dataclass
class Material:
    """Per-instance material: index 0 = soft layer, 1 = hard layer (SI)."""
    Ms: tuple = (1.0e6, 0.6e6)          # A/m
    K: tuple = (0.2e6, 1.2e6)           # J/m^3
    A: tuple = (10e-12, 10e-12)         # J/m
    axis: tuple = ((0.0, 0.0, 1.0), (0.0, 0.0, 1.0))
    A_int: float = 3e-12                # J/m, interlayer exchange constant
    delta_int: float = 1e-9             # m, interlayer thickness
    alpha: float = 0.1


@dataclasses.dataclass
class Field:
    """Applied-field schedule (tesla, seconds, metres).

    kind = FIELD_UNIFORM:  B(t) = B_peak * r(t) * dir + B_ext
    kind = FIELD_POLE:     B(x, t) = B_peak * r(t) * fx(x - x_off - v t) * fy(y - y_off - v_y t) * dir + B_ext
    kind = FIELD_GRID:     B(x, t) = B_peak * r(t) * G(x - x_off - v t) + B_ext, G the trilinear
                           interpolation of `grid` ([3][nz][ny][nx] float32, node (i, j, k) at
                           g_origin + g_h (i, j, k); zero outside)
    with r(t) = min(t / t_rise, 1).
    """
    kind: int = FIELD_UNIFORM
    B_peak: float = 1.2
    dir: tuple = (0.0, 0.0, -1.0)
    t_rise: float = 0.1e-9
    v: tuple = (0.0, 0.0, 0.0)
    x_off: tuple = (0.0, 0.0, 0.0)
    L_grad: float = 10e-9
    W_pole: float = 13e-9
    B_ext: tuple = (0.0, 0.0, 0.0)
    grid: object = None                 # FIELD_GRID: float32 [3][nz][ny][nx]
    g_origin: tuple = (0.0, 0.0, 0.0)
    g_h: float = 2.5e-9


def pole_field_grid(B_peak: float, dir, L_grad: float, W_pole: float, lo, hi, h: float = 2.5e-9):
    """The synthetic pole head field sampled on a grid in its own frame: node values
    B_peak * fx(s_x) * fy(s_y) * dir (tesla) with fx = (1 - tanh(s_x / L)) / 2 and
    fy = (tanh((s_y + W/2) / L) - tanh((s_y - W/2) / L)) / 2 -- the form in which a precomputed
    head field is handed to the recording simulation, here at the paper's 2.5 nm spacing.
    Returns (grid float32 [3][nz][ny][nx], origin, h) covering the box [lo, hi]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    n = np.maximum(2, np.ceil((hi - lo) / h).astype(int) + 1)
    xs, ys = lo[0] + h * np.arange(n[0]), lo[1] + h * np.arange(n[1])
    fx = 0.5 * (1.0 - np.tanh(xs / L_grad))
    fy = 0.5 * (np.tanh((ys + 0.5 * W_pole) / L_grad) - np.tanh((ys - 0.5 * W_pole) / L_grad))
    prof = B_peak * fy[:, None] * fx[None, :]                     # [ny][nx]
    g = np.empty((3, n[2], n[1], n[0]), dtype=np.float32)
    for d in range(3):
        g[d] = (dir[d] * prof)[None, :, :]
    return g, tuple(float(v) for v in lo), float(h)


# ----------------------------------------------------------------------------------------------
# 2-D triangulation of an ellipse
# ----------------------------------------------------------------------------------------------

def _ellipse_boundary(a: float, b: float, h: float) -> np.ndarray:
    """Points on the ellipse x^2/a^2 + y^2/b^2 = 1 at (almost) equal arc-length spacing ~h."""
    th = np.linspace(0.0, 2.0 * np.pi, 4097)
    x, y = a * np.cos(th), b * np.sin(th)
    seg = np.hypot(np.diff(x), np.diff(y))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    perim = s[-1]
    nb = max(6, int(round(perim / h)))
    targets = np.arange(nb) * perim / nb
    tq = np.interp(targets, s, th)
    return np.stack([a * np.cos(tq), b * np.sin(tq)], axis=1)


def _disk_points(a: float, b: float, h: float, rng: np.random.Generator, jitter: float):
    bnd = _ellipse_boundary(a, b, h)
    dy = h * math.sqrt(3.0) / 2.0
    pts = []
    ny = int(math.ceil(b / dy)) + 1
    nx = int(math.ceil(a / h)) + 1
    for j in range(-ny, ny + 1):
        y = j * dy
        off = 0.5 * h if (j % 2) else 0.0
        for i in range(-nx, nx + 1):
            x = i * h + off
            if (x / a) ** 2 + (y / b) ** 2 >= 1.0:
                continue
            pts.append((x, y))
    inner = np.array(pts, dtype=np.float64).reshape(-1, 2)
    if inner.shape[0]:
        d = np.min(np.hypot(inner[:, None, 0] - bnd[None, :, 0], inner[:, None, 1] - bnd[None, :, 1]), axis=1)
        inner = inner[d >= 0.6 * h]
    if inner.shape[0]:
        inner = inner + rng.uniform(-jitter * h, jitter * h, size=inner.shape)
    return bnd, inner


def _triangulate(a: float, b: float, h: float, seed: int, jitter: float):
    rng = np.random.default_rng(seed)
    bnd, inner = _disk_points(a, b, h, rng, jitter)
    p2 = np.concatenate([bnd, inner], axis=0) if inner.shape[0] else bnd
    tri = Delaunay(p2).simplices.astype(np.int64)
    # drop slivers that Delaunay may create between nearly collinear boundary samples
    e1 = p2[tri[:, 1]] - p2[tri[:, 0]]
    e2 = p2[tri[:, 2]] - p2[tri[:, 0]]
    area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    tri = tri[area > 1e-3 * h * h]
    used = np.unique(tri)
    remap = -np.ones(p2.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    return p2[used], remap[tri]


# ----------------------------------------------------------------------------------------------
# Extrusion
# ----------------------------------------------------------------------------------------------

def _levels(t: float, hz: float) -> np.ndarray:
    nl = max(1, int(round(t / hz)))
    return np.linspace(0.0, t, nl + 1)


def island_mesh(a: float, b: float, t_soft: float, t_hard: float, h: float, seed: int = 0,
                jitter: float = 0.15, renumber: bool = True) -> Mesh:
    """Extruded ECC island: hard layer z in [0, t_hard], soft layer z in [t_hard, t_hard+t_soft].

    a, b are the semi-axes (a = b for a cylinder); h is the target edge length.
    """
    p2, tri = _triangulate(a, b, h, seed, jitter)
    n2 = p2.shape[0]
    zh = _levels(t_hard, h)
    zs = t_hard + _levels(t_soft, h)
    levels = [(z, LAYER_HARD) for z in zh] + [(z, LAYER_SOFT) for z in zs]
    nlev = len(levels)
    n = nlev * n2
    xyz = np.empty((3, n), dtype=np.float64)
    layer = np.empty(n, dtype=np.int32)
    for k, (z, L) in enumerate(levels):
        xyz[0, k * n2:(k + 1) * n2] = p2[:, 0]
        xyz[1, k * n2:(k + 1) * n2] = p2[:, 1]
        xyz[2, k * n2:(k + 1) * n2] = z
        layer[k * n2:(k + 1) * n2] = L
    tri_sorted = np.sort(tri, axis=1)
    tets = []
    nh = len(zh)
    # cells inside the hard block: levels 0..nh-1; inside the soft block: levels nh..nlev-1
    for k in range(nlev - 1):
        if k == nh - 1:
            continue  # the interface: no cells between the duplicated planes
        lo, hi = k * n2, (k + 1) * n2
        v0, v1, v2 = tri_sorted[:, 0], tri_sorted[:, 1], tri_sorted[:, 2]
        B0, B1, B2 = lo + v0, lo + v1, lo + v2
        T0, T1, T2 = hi + v0, hi + v1, hi + v2
        tets.append(np.stack([B0, B1, B2, T2], axis=1))
        tets.append(np.stack([B0, B1, T1, T2], axis=1))
        tets.append(np.stack([B0, T0, T1, T2], axis=1))
    tet = np.concatenate(tets, axis=0).astype(np.int64)
    # orient positively
    P = xyz.T
    d1 = P[tet[:, 1]] - P[tet[:, 0]]
    d2 = P[tet[:, 2]] - P[tet[:, 0]]
    d3 = P[tet[:, 3]] - P[tet[:, 0]]
    det = np.einsum("ij,ij->i", d1, np.cross(d2, d3))
    neg = det < 0
    tet[neg, 2], tet[neg, 3] = tet[neg, 3].copy(), tet[neg, 2].copy()
    iface = np.stack([nh * n2 + np.arange(n2), (nh - 1) * n2 + np.arange(n2)], axis=1)
    # Renumber the nodes by reverse Cuthill-McKee over the graph of tet edges and interface pairs
    # (the level-major numbering above puts every row's neighbours a whole level apart): nodes
    # that share a tet, or an interface pair, get nearby indices.  Relabelling changes nothing
    # physical.
    perm = _rcm_order(n, tet, iface) if renumber else np.arange(n)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    xyz = xyz[:, perm]
    layer = layer[perm]
    tet = inv[tet]
    iface = inv[iface]
    return Mesh(xyz=np.ascontiguousarray(xyz), tet=np.ascontiguousarray(tet.astype(np.int32)),
                layer=layer, iface=np.ascontiguousarray(iface.astype(np.int32)), n2d=n2)


def _rcm_order(n: int, tet: np.ndarray, iface: np.ndarray) -> np.ndarray:
    """Reverse Cuthill-McKee order of the node graph (edges of the tets and interface pairs)."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    pairs = [tet[:, [a, b]] for a in range(4) for b in range(a + 1, 4)] + [iface]
    e = np.concatenate(pairs, axis=0)
    r = np.concatenate([e[:, 0], e[:, 1]])
    c = np.concatenate([e[:, 1], e[:, 0]])
    g = coo_matrix((np.ones(r.size, dtype=np.int8), (r, c)), shape=(n, n)).tocsr()
    return np.asarray(reverse_cuthill_mckee(g, symmetric_mode=True), dtype=np.int64)


def island_mesh_target(a: float, b: float, t_soft: float, t_hard: float, n_target: int,
                       seed: int = 0, tol: float = 0.12) -> Mesh:
    """Mesh whose node count is within `tol` of n_target (bisection on the edge length)."""
    vol = math.pi * a * b * (t_soft + t_hard)
    h = (vol / n_target) ** (1.0 / 3.0)
    lo, hi = 0.3 * h, 3.0 * h
    best = None
    for _ in range(40):
        m = island_mesh(a, b, t_soft, t_hard, h, seed)
        err = m.n / n_target - 1.0
        if best is None or abs(err) < abs(best[0]):
            best = (err, m)
        if abs(err) <= tol:
            return m
        if m.n > n_target:
            lo = h
        else:
            hi = h
        h = 0.5 * (lo + hi)
    return best[1]


# ----------------------------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------------------------

def single_island_workload(seed: int = 0, n_target: int = 500):
    """A single two-layer cylinder: d = 8 nm, t = 10 nm (soft 3 nm on top, hard 7 nm),
    uniform field 30 degrees from -z ramped 0 -> 1.2 T in 0.1 ns, alpha = 0.1."""
    mesh = island_mesh_target(4 * NM, 4 * NM, 3 * NM, 7 * NM, n_target, seed=seed)
    mat = Material()
    psi = math.radians(30.0)
    fld = Field(kind=FIELD_UNIFORM, B_peak=1.2, dir=(math.sin(psi), 0.0, -math.cos(psi)),
                t_rise=0.1e-9)
    return mesh, mat, fld


def patch_workload(seed: int = 1, n_target: int = 2000, sigma_rel: float = 0.05):
    """3x3 patch of elliptic islands (18 x 4.5 nm, t = 10 nm), 25 nm down-track by 6.5 nm
    cross-track pitch, per-island per-layer Ms and K scaled by (1 + 0.05 N(0,1)), analytic
    pole field 1.5 T, gradient length 10 nm, 20 m/s, rise 0.1 ns.

    Returns (mesh, [Material]*9, [Field]*9, offsets[9][3]).
    """
    mesh = patch_island_mesh(seed, n_target)
    rng = np.random.default_rng(seed)
    base = Material()
    mats, flds, offs = [], [], []
    px, py = 25 * NM, 6.5 * NM
    psi = math.radians(20.0)
    for i in range(3):
        for j in range(3):
            sc = 1.0 + sigma_rel * rng.standard_normal(4)
            mats.append(dataclasses.replace(
                base, Ms=(base.Ms[0] * sc[0], base.Ms[1] * sc[1]),
                K=(base.K[0] * sc[2], base.K[1] * sc[3])))
            offs.append(((i - 1) * px, (j - 1) * py, 0.0))
    for _ in range(9):
        flds.append(Field(kind=FIELD_POLE, B_peak=1.5, dir=(math.sin(psi), 0.0, -math.cos(psi)),
                          t_rise=0.1e-9, v=(20.0, 0.0, 0.0), x_off=(-10 * NM, 0.0, 0.0),
                          L_grad=10 * NM, W_pole=2 * py))
    return mesh, mats, flds, np.array(offs, dtype=np.float64)


# Recording geometry of the 4 Tb/in^2 media (Sec. II.B, Fig. 3) and of the write simulations
# (Sec. II.C): pseudo-hexagonal islands, 13.5 nm down-track and 11.7 nm cross-track pitch, 12 nm
# dots of 12 nm height (6 nm soft on top, 1 nm interlayer, 5 nm hard, as Fig. 3 labels them; the
# middle of the soft phase then lies 9 nm below the air-bearing surface at 6 nm spacing),
# J_S = 0.7 T in both phases, K_1,soft = 0.2 K_1,hard; the head moves at 13.5 m/s, so one bit
# period is 1 ns.
MEDIA_PITCH_DOWN = 13.5 * NM
MEDIA_PITCH_CROSS = 11.7 * NM
MEDIA_DOT = 12.0 * NM
MEDIA_INTERLAYER = 1.0 * NM
MEDIA_SOFT = 6.0 * NM
MEDIA_HARD = 5.0 * NM
MEDIA_JS = 0.7                                          # tesla
HEAD_VELOCITY = 13.5                                    # m/s, down-track (+x)
BIT_PERIOD = MEDIA_PITCH_DOWN / HEAD_VELOCITY           # 1 ns
HEAD_RISE = 0.1e-9


def recording_layout(p_down: float = MEDIA_PITCH_DOWN, p_cross: float = MEDIA_PITCH_CROSS) -> dict:
    """Island centres (x down-track, y cross-track, metres) relative to the target bit.

    The head travels in +x, so the previously written bit lies one down-track pitch behind the
    target.  Neighbouring tracks of the pseudo-hexagonal pattern are shifted by half a
    down-track pitch; `adjacent` is the nearest island of the next track."""
    return {"target": (0.0, 0.0, 0.0), "previous": (-p_down, 0.0, 0.0),
            "adjacent": (0.5 * p_down, p_cross, 0.0)}


def media_mesh(n_target: int = 600, seed: int = 0, d: float = MEDIA_DOT, t_soft: float = MEDIA_SOFT,
               t_hard: float = MEDIA_HARD) -> Mesh:
    """One cylindrical island of the media (hard layer z in [0, t_hard], soft on top)."""
    return island_mesh_target(0.5 * d, 0.5 * d, t_soft, t_hard, n_target, seed=seed)


def media_material(K_hard: float = 0.8e6, A_int: float = 2e-12, alpha: float = 0.1,
                   A: float = 10e-12) -> Material:
    """Material of the media islands: J_S = 0.7 T in both phases, K_1,soft = K_1,hard / 5, the
    interlayer coupling A_int acting across a 1 nm interlayer (K_1,hard and A_int are design
    parameters of the optimisation; the paper's initial values are the defaults)."""
    Ms = MEDIA_JS / (4e-7 * math.pi)
    return Material(Ms=(Ms, Ms), K=(0.2 * K_hard, K_hard), A=(A, A), A_int=A_int,
                    delta_int=MEDIA_INTERLAYER, alpha=alpha)


def write_head_grid(B_peak: float, dir, L_grad: float, W_pole: float, P_len: float, z_top: float,
                    z_decay: float, lo, hi, h: float = 2.5e-9):
    """A synthetic write-head field sampled on a grid in the head's own frame, standing in for the
    precomputed head field of Sec. II.A (same 2.5 nm spacing).  Node values are
    B_peak * fx(s_x) * fy(s_y) * fz(s_z) * dir with a pole of down-track length P_len whose
    trailing edge sits at s_x = 0 (the head moves in +x):
      fx = (tanh(s_x / L) - tanh((s_x - P_len) / L)) / 2,
      fy = (tanh((s_y + W/2) / L) - tanh((s_y - W/2) / L)) / 2,
      fz = exp((s_z - z_top) / z_decay)  (the field weakens away from the air-bearing surface).
    Returns (grid float32 [3][nz][ny][nx], origin, h) covering the box [lo, hi]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    n = np.maximum(2, np.ceil((hi - lo) / h).astype(int) + 1)
    xs, ys, zs = (lo[d] + h * np.arange(n[d]) for d in range(3))
    fx = 0.5 * (np.tanh(xs / L_grad) - np.tanh((xs - P_len) / L_grad))
    fy = 0.5 * (np.tanh((ys + 0.5 * W_pole) / L_grad) - np.tanh((ys - 0.5 * W_pole) / L_grad))
    fz = np.exp((zs - z_top) / z_decay)
    prof = B_peak * fz[:, None, None] * fy[None, :, None] * fx[None, None, :]      # [nz][ny][nx]
    g = np.empty((3, n[2], n[1], n[0]), dtype=np.float32)
    for d in range(3):
        g[d] = dir[d] * prof
    return g, tuple(float(v) for v in lo), float(h)


def default_head_grid(B_peak: float = 2.2, psi_deg: float = 25.0):
    """The synthetic head used by the write-error driver: 2.2 T peak, tilted psi from -z toward
    +x, 10 nm pole length and width, 4 nm edge length, 25 nm decay below the soft-layer top,
    sampled over [-40, 50] x [-30, 30] x [-2.5, 15] nm."""
    psi = math.radians(psi_deg)
    d = (math.sin(psi), 0.0, -math.cos(psi))
    return write_head_grid(B_peak, d, 4 * NM, 10 * NM, 10 * NM, MEDIA_SOFT + MEDIA_HARD, 25 * NM,
                           lo=(-40 * NM, -30 * NM, -2.5 * NM), hi=(50 * NM, 30 * NM, 15 * NM))


def recording_field(grid, g_origin, g_h, down_offset: float = 6.8 * NM, cross_offset: float = 0.0,
                    p_down: float = MEDIA_PITCH_DOWN, v: float = HEAD_VELOCITY, t_rise: float = HEAD_RISE,
                    B_ext=(0.0, 0.0, 0.0)) -> Field:
    """The moving head field of one write period: the field switches on at t = 0 (rise t_rise)
    and the trailing edge travels from down_offset - p_down to down_offset (relative to the target
    centre) at speed v, so that it ends the period down_offset past the target, where it started
    relative to the previous bit.  cross_offset shifts the head across the track (Table I's
    down- and cross-track offsets)."""
    return Field(kind=FIELD_GRID, B_peak=1.0, dir=(0.0, 0.0, -1.0), t_rise=t_rise, v=(v, 0.0, 0.0),
                 x_off=(down_offset - p_down, cross_offset, 0.0), B_ext=tuple(B_ext), grid=grid,
                 g_origin=tuple(g_origin), g_h=g_h)


def adjacent_field(grid, g_origin, g_h, layout=None, cross_offset: float = 0.0,
                   te_distance: float = 2.0 * NM) -> Field:
    """The static head field seen by the adjacent island (Sec. II.C): the head stands with its
    trailing edge te_distance behind the island's centre in the flight direction (so the island
    sits 2 nm inside the pole's down-track extent by default), shifted across the track by
    cross_offset; the island itself is placed at layout["adjacent"]."""
    layout = recording_layout() if layout is None else layout
    xa = layout["adjacent"][0]
    return Field(kind=FIELD_GRID, B_peak=1.0, dir=(0.0, 0.0, -1.0), t_rise=0.0, v=(0.0, 0.0, 0.0),
                 x_off=(xa - te_distance, cross_offset, 0.0), grid=grid, g_origin=tuple(g_origin), g_h=g_h)


def rotation_chain(n: int, P: int, via=(1.0, 0.0, 0.0)) -> np.ndarray:
    """Initial string of P uniform states turning from +z to -z through the unit direction `via`
    (perpendicular to z): image k at polar angle pi k / (P - 1).  Returns [P][3][n]."""
    v = np.asarray(via, dtype=np.float64)
    th = math.pi * np.arange(P) / (P - 1)
    d = np.cos(th)[:, None] * np.array([0.0, 0.0, 1.0]) + np.sin(th)[:, None] * v      # [P][3]
    return np.ascontiguousarray(np.repeat(d[:, :, None], n, axis=2))


def lhs_maximin(n: int, d: int, seed: int = 0, sweeps: int = 200) -> np.ndarray:
    """Seeded Latin hypercube of n points in [0, 1]^d with a larger smallest pairwise distance:
    each coordinate takes one point in each of the n strata (at a uniform position inside it);
    random swaps of two points' coordinate in one dimension are kept when they do not shrink the
    smallest pairwise distance (the space-filling start of the global optimiser, Sec. II.A)."""
    rng = np.random.default_rng(seed)
    P = np.stack([rng.permutation(n) for _ in range(d)], axis=1)
    U = (P + rng.random((n, d))) / n

    def mindist(A):
        D = np.sqrt(((A[:, None, :] - A[None, :, :]) ** 2).sum(-1))
        D[np.arange(len(A)), np.arange(len(A))] = np.inf
        return D.min()

    best = mindist(U)
    for _ in range(sweeps * n):
        j = rng.integers(d)
        a, b = rng.choice(n, 2, replace=False)
        V = U.copy()
        V[a, j], V[b, j] = U[b, j], U[a, j]
        m = mindist(V)
        if m >= best:
            U, best = V, m
    return U


# Free media and placement parameters of the write-error optimisation (Table I without the head
# geometry): K_1,hard (J/m^3), A_ex,int (J/m), down-track offset (m), cross-track offset (m).
OPT_NAMES = ("K_hard", "A_int", "down_offset", "cross_offset")
OPT_LO = np.array([0.5e6, 1e-12, 0.0, -8e-9])
OPT_HI = np.array([1.2e6, 10e-12, 8e-9, 8e-9])


# Design-vector layout used by the batched designs and the surrogate:
DESIGN_NAMES = ("d", "t_soft", "t_hard", "Ms_soft", "Ms_hard", "K_soft", "K_hard", "A_int",
                "psi", "B_peak", "alpha", "t_rise")
DESIGN_LO = np.array([6e-9, 2e-9, 2e-9, 0.4e6, 0.4e6, 0.1e6, 0.1e6, 0.5e-12, 0.0, 0.8, 0.02,
                      0.05e-9])
DESIGN_HI = np.array([12e-9, 8e-9, 8e-9, 1.2e6, 1.2e6, 1.5e6, 1.5e6, 10e-12,
                      math.radians(45.0), 2.0, 0.2, 0.2e-9])


# parameters with a positive lower bound can be sampled log-uniformly (psi starts at 0: linear)
DESIGN_LOG = DESIGN_LO > 0


def design_of_unit(u: np.ndarray, log_prior: bool) -> np.ndarray:
    """Designs from unit coordinates u in [0, 1]^12: lo + (hi - lo) u, or lo (hi / lo)^u for the
    parameters in DESIGN_LOG when log_prior."""
    u = np.asarray(u, dtype=np.float64)
    x = DESIGN_LO + (DESIGN_HI - DESIGN_LO) * u
    if log_prior:
        lo, hi = DESIGN_LO[DESIGN_LOG], DESIGN_HI[DESIGN_LOG]
        x[..., DESIGN_LOG] = lo * (hi / lo) ** u[..., DESIGN_LOG]
    return x


def unit_of_design(x: np.ndarray, log_prior: bool) -> np.ndarray:
    """Inverse of design_of_unit."""
    x = np.asarray(x, dtype=np.float64)
    u = (x - DESIGN_LO) / (DESIGN_HI - DESIGN_LO)
    if log_prior:
        lo, hi = DESIGN_LO[DESIGN_LOG], DESIGN_HI[DESIGN_LOG]
        u[..., DESIGN_LOG] = np.log(x[..., DESIGN_LOG] / lo) / np.log(hi / lo)
    return u


def sample_designs(n: int, seed: int = 2, fixed_alpha_rise: bool = True, log_prior: bool = False) -> np.ndarray:
    """Designs in the batched-island ranges, uniform (or log-uniform in the parameters with a
    positive lower bound when log_prior); returns [n][12] float64.

    With fixed_alpha_rise the last two entries are alpha = 0.1 and t_rise = 0.1 ns (the ranges
    of the batched-island workload do not include them)."""
    rng = np.random.default_rng(seed)
    u = rng.random((n, len(DESIGN_NAMES)))
    x = design_of_unit(u, log_prior)
    if fixed_alpha_rise:
        x[:, 10] = 0.1
        x[:, 11] = 0.1e-9
    return x


# Node density of the batched designs: the largest island of the design box (d = 12 nm, t_soft +
# t_hard = 16 nm, 1809.6 nm^3) gets 3000 nodes; the count is proportional to the volume and
# clipped to [300, 3000] (the smallest islands, 113 nm^3, would otherwise get ~190).
DESIGN_NODES_MIN, DESIGN_NODES_MAX = 300, 3000
DESIGN_NODE_DENSITY = DESIGN_NODES_MAX / (math.pi * (0.5 * DESIGN_HI[0]) ** 2 * (DESIGN_HI[1] + DESIGN_HI[2]))


def design_node_target(x: np.ndarray, density: float = DESIGN_NODE_DENSITY) -> int:
    """Node count proportional to island volume, clipped to [300, 3000]."""
    vol = math.pi * (x[0] / 2) ** 2 * (x[1] + x[2])
    return int(min(DESIGN_NODES_MAX, max(DESIGN_NODES_MIN, round(density * vol))))


def design_inputs(x: np.ndarray, seed: int = 0):
    """(mesh, Material, Field) for one design vector x (see DESIGN_NAMES)."""
    r = 0.5 * x[0]
    mesh = island_mesh_target(r, r, x[1], x[2], design_node_target(x), seed=seed)
    mat = Material(Ms=(x[3], x[4]), K=(x[5], x[6]), A_int=x[7], alpha=x[10])
    psi = x[8]
    fld = Field(kind=FIELD_UNIFORM, B_peak=x[9], dir=(math.sin(psi), 0.0, -math.cos(psi)),
                t_rise=x[11])
    return mesh, mat, fld


def _design_inputs_job(args):
    x, seed = args
    return design_inputs(x, seed)


def _pool_map(fn, jobs, workers: int = 0, chunksize: int = 16):
    """[fn(j) for j in jobs] on a pool of worker processes started with 'spawn' (workers = 0: up to
    16, bounded by the CPUs this process may use); serial for short lists.  Call it before any GPU
    work in the process."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    if workers <= 0:
        try:
            avail = len(os.sched_getaffinity(0))
        except AttributeError:
            avail = os.cpu_count() or 1
        workers = max(1, min(16, avail))
    if workers == 1 or len(jobs) < 8:
        return [fn(j) for j in jobs]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(fn, jobs, chunksize=max(1, min(chunksize, len(jobs) // workers))))


def design_inputs_many(X: np.ndarray, seeds=None, workers: int = 0):
    """design_inputs for every row of X (mesh seed = row index unless seeds is given), meshed by a
    pool of worker processes.  Call it before any GPU work in the process."""
    X = np.asarray(X, dtype=np.float64)
    seeds = list(range(X.shape[0])) if seeds is None else list(seeds)
    return _pool_map(_design_inputs_job, [(X[q], int(seeds[q])) for q in range(X.shape[0])], workers)


def patch_island_mesh(seed: int, n_target: int = 2000) -> Mesh:
    """The island of the 3x3 patch (elliptic 18 x 4.5 nm, soft 3 nm on hard 7 nm) with mesh seed
    `seed`."""
    return island_mesh_target(9 * NM, 2.25 * NM, 3 * NM, 7 * NM, n_target, seed=seed)


def patch_island_meshes(seeds, workers: int = 0):
    """patch_island_mesh for every seed, on a pool of worker processes (before any GPU work)."""
    return _pool_map(patch_island_mesh, [int(s) for s in seeds], workers, chunksize=2)


def random_unit_m(n: int, seed: int, cone: float = math.pi) -> np.ndarray:
    """[3][n] unit vectors within `cone` radians of +z (seeded)."""
    rng = np.random.default_rng(seed)
    ct = 1.0 - (1.0 - math.cos(cone)) * rng.random(n)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = 2.0 * math.pi * rng.random(n)
    return np.ascontiguousarray(np.stack([st * np.cos(ph), st * np.sin(ph), ct]))


def mlp_init_params(seed: int) -> np.ndarray:
    """Seeded initial parameters of the 12 -> 4x256 -> 3 surrogate, flat FP32 vector in the
    library's parameter layout (per layer W [out][in], then b [out]): weights and biases uniform
    in +-1/sqrt(fan-in).  (On 1792 solver labels this gives a held-out switching-field error of
    2.6 % against 3.9 % with He-uniform weights and zero biases.)"""
    sizes = (12, 256, 256, 256, 256, 3)
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(sizes) - 1):
        ni, no = sizes[i], sizes[i + 1]
        lim = 1.0 / math.sqrt(ni)
        parts.append(rng.uniform(-lim, lim, size=no * ni))
        parts.append(rng.uniform(-lim, lim, size=no))
    return np.concatenate(parts).astype(np.float32)
