"""ctypes wrapper around the FP64 CPU oracle (liboracle.so) -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may import this
module.  It shares nothing with the GPU library; the arrays both consume come from the seeded
input generators.  The arithmetic lives in bpm_oracle.c (see its header for the passages of the
paper it follows).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

DP45, DP5_FIXED, HEUN = 0, 1, 2
FIELD_UNIFORM, FIELD_POLE, FIELD_GRID = 0, 1, 2
OK, EINVAL, ENOMEM, ENONFINITE, ESTEPUNDERFLOW, EMAXSTEPS = 0, -1, -2, -5, -6, -7

# Smear factor of the Gaussian charge blobs of the demag operator (std = beta * V_tet^(1/3)):
# the blob whose Coulomb self-energy equals that of a uniformly charged ball of the tet's volume,
# beta = 5/(6 sqrt(pi)) * (3/(4 pi))^(1/3).
DEMAG_BETA = 5.0 / (6.0 * np.sqrt(np.pi)) * (3.0 / (4.0 * np.pi)) ** (1.0 / 3.0)


class Material(C.Structure):
    _fields_ = [("Ms", C.c_double * 2), ("K", C.c_double * 2), ("A", C.c_double * 2),
                ("axis", (C.c_double * 3) * 2), ("A_int", C.c_double), ("delta_int", C.c_double),
                ("alpha", C.c_double)]


class Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad_", C.c_int32), ("B_peak", C.c_double),
                ("dir", C.c_double * 3), ("t_rise", C.c_double), ("v", C.c_double * 3),
                ("x_off", C.c_double * 3), ("L_grad", C.c_double), ("W_pole", C.c_double),
                ("B_ext", C.c_double * 3), ("grid", C.c_void_p), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("pad2_", C.c_int32), ("g_origin", C.c_double * 3), ("g_h", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("integrator", C.c_int32), ("save_every", C.c_int32), ("t_end", C.c_double),
                ("dt0", C.c_double), ("dt_fixed", C.c_double), ("rtol", C.c_double),
                ("atol", C.c_double), ("dt_min", C.c_double), ("temperature", C.c_double),
                ("max_steps", C.c_int64), ("relax", C.c_int32), ("pad_", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("switched", C.c_int32), ("t_sw", C.c_double),
                ("B_sw", C.c_double), ("mz_soft", C.c_double), ("mz_hard", C.c_double),
                ("t_reached", C.c_double), ("energy", C.c_double), ("n_accept", C.c_int64),
                ("n_reject", C.c_int64), ("dt_min_used", C.c_double), ("dt_max_used", C.c_double),
                ("max_norm_dev", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def build():
    subprocess.check_call([os.path.join(_HERE, "build.sh")])


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        L.or_mesh_create.restype = P
        L.or_mesh_create.argtypes = [C.c_int, C.c_int, P, P, P, C.c_int, P]
        L.or_mesh_free.argtypes = [P]
        L.or_mesh_nnz.restype = C.c_int
        L.or_mesh_nnz.argtypes = [P]
        L.or_mesh_export.argtypes = [P] * 9
        L.or_demag_S.restype = C.c_int
        L.or_demag_S.argtypes = [P, C.c_double, P]
        L.or_demag_S_entry.restype = C.c_double
        L.or_demag_S_entry.argtypes = [P, C.c_double, C.c_int, C.c_int]
        L.or_fields.restype = C.c_int
        L.or_fields.argtypes = [P, P, P, P, P, C.c_double, P, P, P, P, P]
        L.or_llg_rhs.argtypes = [C.c_int, C.c_double, P, P, P]
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_gauss3.argtypes = [P, C.c_uint64, C.c_uint32, P]
        L.or_dp5_tableau.argtypes = [P, P, P]
        L.or_run.restype = C.c_int
        L.or_run.argtypes = [P, P, C.c_int, P, P, P, C.c_int, P, P, P, P, P, C.c_int64, P]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def material(m) -> Material:
    """From an inputs.Material (or any object with the same attributes)."""
    s = Material()
    for i in range(2):
        s.Ms[i], s.K[i], s.A[i] = m.Ms[i], m.K[i], m.A[i]
        for c in range(3):
            s.axis[i][c] = m.axis[i][c]
    s.A_int, s.delta_int, s.alpha = m.A_int, m.delta_int, m.alpha
    return s


_GRIDS = []   # float32 copies of field grids handed to the oracle (kept alive for its calls)


def field(f) -> Field:
    s = Field()
    s.kind = f.kind
    s.B_peak, s.t_rise, s.L_grad, s.W_pole = f.B_peak, f.t_rise, f.L_grad, f.W_pole
    for c in range(3):
        s.dir[c], s.v[c], s.x_off[c], s.B_ext[c] = f.dir[c], f.v[c], f.x_off[c], f.B_ext[c]
    grid = getattr(f, "grid", None)
    if grid is not None:
        g = np.ascontiguousarray(grid, dtype=np.float32)
        _GRIDS.append(g)
        del _GRIDS[:-64]
        s.grid = g.ctypes.data
        s.nz, s.ny, s.nx = (int(v) for v in g.shape[1:])
        s.g_h = f.g_h
        for c in range(3):
            s.g_origin[c] = f.g_origin[c]
    return s


class OracleMesh:
    """Mesh quantities of the P1 discretisation, built by the oracle."""

    def __init__(self, mesh):
        L = lib()
        self.mesh = mesh
        self.n = mesh.n
        self._xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
        self._tet = np.ascontiguousarray(mesh.tet, dtype=np.int32)
        self._layer = np.ascontiguousarray(mesh.layer, dtype=np.int32)
        self._iface = np.ascontiguousarray(mesh.iface, dtype=np.int32)
        self.h = L.or_mesh_create(self.n, self._tet.shape[0], _p(self._xyz), _p(self._tet),
                                  _p(self._layer), self._iface.shape[0], _p(self._iface))
        if not self.h:
            raise ValueError("oracle rejected the mesh")
        self.nnz = L.or_mesh_nnz(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_mesh_free(self.h)
            self.h = None

    def export(self):
        n, nnz, nif, nt = self.n, self.nnz, self._iface.shape[0], self._tet.shape[0]
        V = np.empty(n); rp = np.empty(n + 1, np.int32); col = np.empty(nnz, np.int32)
        K = np.empty(nnz); D = np.empty((nnz, 3)); a = np.empty(max(nif, 1)); tv = np.empty(nt)
        cen = np.empty(3)
        lib().or_mesh_export(self.h, _p(V), _p(rp), _p(col), _p(K), _p(D), _p(a), _p(tv), _p(cen))
        return dict(V=V, rowptr=rp, col=col, K=K, D=D, aif=a[:nif], tetV=tv, centroid=cen)

    def K_dense(self):
        e = self.export()
        Kd = np.zeros((self.n, self.n))
        for i in range(self.n):
            for q in range(e["rowptr"][i], e["rowptr"][i + 1]):
                Kd[i, e["col"][q]] = e["K"][q]
        return Kd

    def D_dense(self):
        """[n][3][n]: D[k, alpha, j]."""
        e = self.export()
        Dd = np.zeros((self.n, 3, self.n))
        for k in range(self.n):
            for q in range(e["rowptr"][k], e["rowptr"][k + 1]):
                Dd[k, :, e["col"][q]] = e["D"][q]
        return Dd

    def demag_S(self, beta: float = DEMAG_BETA) -> np.ndarray:
        S = np.empty((self.n, self.n))
        rc = lib().or_demag_S(self.h, beta, _p(S))
        if rc != 0:
            raise MemoryError("or_demag_S failed")
        return S

    def demag_S_entry(self, k: int, l: int, beta: float = DEMAG_BETA) -> float:
        return lib().or_demag_S_entry(self.h, beta, int(k), int(l))

    def fields(self, S, mat, fld, m, t=0.0, offset=(0.0, 0.0, 0.0), Bdip=None):
        """Returns (B_total [3][n], terms [5][3][n] = ex, an, int, demag, zeeman, E[5])."""
        n = self.n
        m = np.ascontiguousarray(m, dtype=np.float64)
        Bt = np.empty((3, n)); terms = np.empty((5, 3, n)); E = np.empty(5)
        off = np.ascontiguousarray(offset, dtype=np.float64)
        bd = None if Bdip is None else np.ascontiguousarray(Bdip, dtype=np.float64)
        Sa = None if S is None else np.ascontiguousarray(S, dtype=np.float64)
        ms, fs = material(mat), field(fld)
        lib().or_fields(self.h, _p(Sa), C.byref(ms), C.byref(fs), _p(off), float(t), _p(m),
                        _p(bd), _p(Bt), _p(terms), _p(E))
        return Bt, terms, E

    def run(self, S, mats, flds, opts: dict, m0=None, offsets=None, coupled=False, seeds=None,
            traj_cap=0):
        """Integrates R instances.  Returns (m [R][3][n], [result dicts], traj list)."""
        R = len(mats)
        n = self.n
        marr = (Material * R)(*[material(x) for x in mats])
        farr = (Field * R)(*[field(x) for x in flds])
        off = np.zeros((R, 3)) if offsets is None else np.ascontiguousarray(offsets, dtype=np.float64)
        if m0 is None:
            m = np.zeros((R, 3, n)); m[:, 2, :] = 1.0
        else:
            m = np.array(np.broadcast_to(m0, (R, 3, n)), dtype=np.float64, order="C")
        sd = np.zeros(R, np.uint64) if seeds is None else np.ascontiguousarray(seeds, dtype=np.uint64)
        o = Opts()
        o.integrator = opts.get("integrator", DP45)
        o.save_every = opts.get("save_every", 1)
        o.t_end = opts["t_end"]
        o.dt0 = opts.get("dt0", 1e-15)
        o.dt_fixed = opts.get("dt_fixed", 0.0)
        o.rtol = opts.get("rtol", 1e-6)
        o.atol = opts.get("atol", o.rtol)
        o.dt_min = opts.get("dt_min", 1e-19)
        o.temperature = opts.get("temperature", 0.0)
        o.max_steps = opts.get("max_steps", 0)
        o.relax = 1 if opts.get("relax", False) else 0
        res = (Result * R)()
        cap = int(traj_cap)
        traj = np.zeros((R, max(cap, 1), 9))
        nt = np.zeros(R, np.int64)
        Sa = None if S is None else np.ascontiguousarray(S, dtype=np.float64)
        rc = lib().or_run(self.h, _p(Sa), R, marr, farr, _p(off), int(bool(coupled)), _p(sd),
                          C.byref(o), _p(m), res, _p(traj) if cap > 0 else None, cap,
                          _p(nt) if cap > 0 else None)
        if rc != 0:
            raise ValueError(f"or_run failed: {rc}")
        trajs = [traj[r, :nt[r]].copy() for r in range(R)] if cap > 0 else []
        return m, [r.as_dict() for r in res], trajs


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def gauss3(key, step, node):
    k = np.ascontiguousarray(key, dtype=np.uint32)
    g = np.empty(3)
    lib().or_gauss3(_p(k), C.c_uint64(step), C.c_uint32(node), _p(g))
    return g


def dp5_tableau():
    c = np.empty(7); a = np.empty((7, 6)); e = np.empty(7)
    lib().or_dp5_tableau(_p(c), _p(a), _p(e))
    return c, a, e


def llg_rhs(alpha, m, B):
    m = np.ascontiguousarray(m, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    dm = np.empty_like(m)
    lib().or_llg_rhs(m.shape[1], float(alpha), _p(m), _p(B), _p(dm))
    return dm


def num_threads():
    return lib().or_num_threads()
