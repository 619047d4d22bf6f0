"""Thin ctypes binding of libbpmllg.so (include/bpm_llg.h).

Argument marshalling only: every step of the simulation runs in the library's HIP kernels.
The library must have been built (paper_1603_09493_amd.build_lib); importing this module on a
machine without it raises immediately -- there is no CPU fallback.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbpmllg.so")

BPM_OK, BPM_EINVAL, BPM_ENOMEM, BPM_EHIP, BPM_ESTATE = 0, -1, -2, -3, -4
BPM_ENONFINITE, BPM_ESTEPUNDERFLOW, BPM_EMAXSTEPS = -5, -6, -7
FIELD_UNIFORM, FIELD_POLE, FIELD_GRID = 0, 1, 2
FLAG_SYMMETRIC_DEMAG = 1
FLAG_WG512 = 2
FLAG_STREAM_S = 4
FLAG_WG256 = 8
FLAG_CONTINUE = 16
FLAG_RELAX = 32
KEEP_S64, KEEP_S32, KEEP_S32_TILES, KEEP_S16_TILES = 1, 2, 4, 8
DP45, DP5_FIXED, HEUN = 0, 1, 2


class BpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class bpm_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_tets", C.c_int32), ("n_iface", C.c_int32), ("pad_", C.c_int32),
                ("xyz", C.c_void_p), ("tet", C.c_void_p), ("node_layer", C.c_void_p), ("iface", C.c_void_p)]


class bpm_material(C.Structure):
    _fields_ = [("Ms", C.c_double * 2), ("K", C.c_double * 2), ("A", C.c_double * 2),
                ("axis", (C.c_double * 3) * 2), ("A_int", C.c_double), ("delta_int", C.c_double),
                ("alpha", C.c_double)]


class bpm_field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad_", C.c_int32), ("B_peak", C.c_double), ("dir", C.c_double * 3),
                ("t_rise", C.c_double), ("v", C.c_double * 3), ("x_off", C.c_double * 3),
                ("L_grad", C.c_double), ("W_pole", C.c_double), ("B_ext", C.c_double * 3),
                ("grid", C.c_void_p), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad2_", C.c_int32),
                ("g_origin", C.c_double * 3), ("g_h", C.c_double)]


class bpm_gp(C.Structure):
    _fields_ = [("n", C.c_int32), ("d", C.c_int32), ("mu", C.c_double), ("sigma2", C.c_double),
                ("c", C.c_double), ("f_min", C.c_double), ("X", C.c_void_p), ("theta", C.c_void_p),
                ("G", C.c_void_p)]


class bpm_run_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("integrator", C.c_int32), ("t_end", C.c_double),
                ("dt0", C.c_double), ("dt_fixed", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
                ("dt_min", C.c_double), ("temperature", C.c_double), ("max_steps", C.c_int64),
                ("save_every", C.c_int32), ("traj_cap", C.c_int32), ("wg_per_group", C.c_int32),
                ("flags", C.c_int32)]


class bpm_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("switched", C.c_int32), ("t_sw", C.c_double), ("B_sw", C.c_double),
                ("mz_soft", C.c_double), ("mz_hard", C.c_double), ("t_reached", C.c_double),
                ("energy", C.c_double), ("n_accept", C.c_int64), ("n_reject", C.c_int64),
                ("dt_min_used", C.c_double), ("dt_max_used", C.c_double), ("max_norm_dev", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol declared in include/bpm_llg.h (the load test checks them all)
SYMBOLS = [
    "bpm_create", "bpm_destroy", "bpm_last_error", "bpm_mesh_add", "bpm_mesh_add_ex", "bpm_mesh_get_S",
    "bpm_mesh_get_assembly", "bpm_instance_add", "bpm_couple_dipoles", "bpm_clear_instances",
    "bpm_run", "bpm_sync", "bpm_autotune", "bpm_get_results", "bpm_get_trajectory", "bpm_get_m", "bpm_last_run_info",
    "bpm_last_run_layout", "bpm_string_reparam",
]

EXTRA_SYMBOLS = [
    "bpm_mlp_num_params", "bpm_mlp_create", "bpm_mlp_destroy", "bpm_mlp_set_params", "bpm_mlp_get_params",
    "bpm_mlp_predict", "bpm_mlp_grads", "bpm_mlp_train_step", "bpm_sample_designs", "bpm_topk", "bpm_screen",
    "bpm_topk_noalloc", "bpm_gp_ei", "bpm_argmax",
]

_lib = None


def lib():
    """Loads libbpmllg.so; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1603_09493_amd.build_lib")
    # PyTorch ships its own HIP runtime under the same soname; loading it first makes this library
    # bind to that one, so that one process holds a single HIP runtime and torch's device buffers
    # and streams are valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.bpm_create.argtypes = [C.POINTER(P), C.c_int, C.c_char_p]
    L.bpm_destroy.argtypes = [P]
    L.bpm_destroy.restype = None
    L.bpm_last_error.argtypes = [P]
    L.bpm_last_error.restype = C.c_char_p
    L.bpm_mesh_add.argtypes = [P, C.POINTER(bpm_mesh), P, D, C.POINTER(I32)]
    L.bpm_mesh_add_ex.argtypes = [P, C.POINTER(bpm_mesh), P, D, I32, C.POINTER(I32)]
    L.bpm_mesh_get_S.argtypes = [P, I32, P]
    L.bpm_mesh_get_assembly.argtypes = [P, I32, C.POINTER(I32), P, P, P, P, P, P]
    L.bpm_instance_add.argtypes = [P, I32, C.POINTER(bpm_material), C.POINTER(bpm_field), P, P, C.c_uint64,
                                   C.POINTER(I32)]
    L.bpm_couple_dipoles.argtypes = [P, I32, P]
    L.bpm_clear_instances.argtypes = [P]
    L.bpm_run.argtypes = [P, C.POINTER(bpm_run_opts), P]
    L.bpm_sync.argtypes = [P]
    L.bpm_autotune.argtypes = [P, C.POINTER(bpm_run_opts), I32, P, I64, C.POINTER(I32), P]
    L.bpm_get_results.argtypes = [P, I32, P, P]
    L.bpm_get_trajectory.argtypes = [P, I32, P, I64, C.POINTER(I64)]
    L.bpm_get_m.argtypes = [P, I32, P, I32]
    L.bpm_string_reparam.argtypes = [P, I32, P, P]
    L.bpm_gp_ei.argtypes = [P, C.POINTER(bpm_gp), I64, P, C.c_uint64, P, P, P, P]
    L.bpm_argmax.argtypes = [P, P, I64, P, P]
    L.bpm_last_run_info.argtypes = [P, C.POINTER(D), C.POINTER(I32), C.POINTER(I32)]
    L.bpm_last_run_layout.argtypes = [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32), C.POINTER(I32), C.POINTER(I64)]
    L.bpm_mlp_num_params.argtypes = []
    L.bpm_mlp_create.argtypes = [P, I32, P, C.POINTER(P)]
    L.bpm_mlp_destroy.argtypes = [P]
    L.bpm_mlp_destroy.restype = None
    L.bpm_mlp_set_params.argtypes = [P, P]
    L.bpm_mlp_get_params.argtypes = [P, P]
    L.bpm_mlp_predict.argtypes = [P, P, P, I64, P]
    L.bpm_mlp_grads.argtypes = [P, P, P, P, I32, P, P]
    L.bpm_mlp_train_step.argtypes = [P, P, P, P, I32, C.c_float, P, P]
    L.bpm_sample_designs.argtypes = [P, C.c_uint64, I64, P, P]
    L.bpm_topk.argtypes = [P, P, I64, I64, P, P]
    L.bpm_screen.argtypes = [P, C.c_uint64, I64, I64, P, P, D, P, P, P, P, P]
    L.bpm_topk_noalloc.argtypes = [P, P, I64, I64, P, P]
    for name in SYMBOLS + EXTRA_SYMBOLS:
        fn = getattr(L, name)
        if name not in ("bpm_destroy", "bpm_last_error", "bpm_mlp_destroy"):
            fn.restype = C.c_int
    _lib = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def material_struct(m) -> bpm_material:
    s = bpm_material()
    for i in range(2):
        s.Ms[i], s.K[i], s.A[i] = m.Ms[i], m.K[i], m.A[i]
        for c in range(3):
            s.axis[i][c] = m.axis[i][c]
    s.A_int, s.delta_int, s.alpha = m.A_int, m.delta_int, m.alpha
    return s


def field_struct(f) -> bpm_field:
    s = bpm_field()
    s.kind = f.kind
    s.B_peak, s.t_rise, s.L_grad, s.W_pole = f.B_peak, f.t_rise, f.L_grad, f.W_pole
    for c in range(3):
        s.dir[c], s.v[c], s.x_off[c], s.B_ext[c] = f.dir[c], f.v[c], f.x_off[c], f.B_ext[c]
    grid = getattr(f, "grid", None)
    if grid is not None:
        g = np.ascontiguousarray(grid, dtype=np.float32)
        if g.ndim != 4 or g.shape[0] != 3:
            raise ValueError("field grid must be [3][nz][ny][nx]")
        s._grid_keep = g                    # alive until the call that copies it returns
        s.grid = g.ctypes.data
        s.nz, s.ny, s.nx = (int(v) for v in g.shape[1:])
        s.g_h = f.g_h
        for c in range(3):
            s.g_origin[c] = f.g_origin[c]
    return s


class Context:
    """One bpm_ctx on a HIP device."""

    def __init__(self, device: int = 0, tune_cache=None):
        self.L = lib()
        self.h = C.c_void_p()
        rc = self.L.bpm_create(C.byref(self.h), int(device), None if tune_cache is None else tune_cache.encode())
        if rc != 0:
            raise BpmError(rc, "bpm_create failed (no HIP device?)")
        self.mesh_n = {}

    def close(self):
        if self.h:
            self.L.bpm_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise BpmError(rc, self.L.bpm_last_error(self.h).decode())
        return rc

    # meshes -------------------------------------------------------------------------------------
    def mesh_add(self, mesh, S=None, beta=0.0, keep=3) -> int:
        """keep (bits): 1 = row-major FP64 demag operator, 2 = row-major FP32, 4 = FP32 upper-triangle
        packed tiles (for the upper-triangle product of FP32 batches), 8 = the same tiles in FP16
        (scaled by a power of two; used when the FP32 tiles are not kept)."""
        xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
        tet = np.ascontiguousarray(mesh.tet, dtype=np.int32)
        layer = np.ascontiguousarray(mesh.layer, dtype=np.int32)
        iface = np.ascontiguousarray(mesh.iface, dtype=np.int32)
        s = bpm_mesh(int(xyz.shape[1]), int(tet.shape[0]), int(iface.shape[0]), 0, _p(xyz), _p(tet), _p(layer),
                     _p(iface) if iface.shape[0] else None)
        Sa = None if S is None else np.ascontiguousarray(S, dtype=np.float64)
        mid = C.c_int32()
        self._check(self.L.bpm_mesh_add_ex(self.h, C.byref(s), _p(Sa), float(beta), int(keep), C.byref(mid)))
        self.mesh_n[mid.value] = int(xyz.shape[1])
        return mid.value

    def mesh_get_S(self, mid):
        n = self.mesh_n[mid]
        S = np.empty((n, n))
        self._check(self.L.bpm_mesh_get_S(self.h, mid, _p(S)))
        return S

    def mesh_get_assembly(self, mid, pattern_only=False):
        """Host-assembled quantities of a group (dict), or only the pattern size nnz."""
        n = self.mesh_n[mid]
        nnz = C.c_int32()
        self._check(self.L.bpm_mesh_get_assembly(self.h, mid, C.byref(nnz), None, None, None, None, None, None))
        if pattern_only:
            return nnz.value
        V = np.empty(n); rp = np.empty(n + 1, np.int32); col = np.empty(nnz.value, np.int32)
        K = np.empty(nnz.value); D = np.empty((nnz.value, 3)); aif = np.empty(n)
        self._check(self.L.bpm_mesh_get_assembly(self.h, mid, C.byref(nnz), _p(V), _p(rp), _p(col), _p(K), _p(D),
                                                 _p(aif)))
        return dict(V=V, rowptr=rp, col=col, K=K, D=D, aif=aif)

    # instances ----------------------------------------------------------------------------------
    def instance_add(self, mid, mat, fld, offset=None, m0=None, seed=0) -> int:
        ms, fs = material_struct(mat), field_struct(fld)
        off = None if offset is None else np.ascontiguousarray(offset, dtype=np.float64)
        m0a = None if m0 is None else np.ascontiguousarray(m0, dtype=np.float64)
        if m0a is not None and m0a.shape != (3, self.mesh_n[mid]):
            raise ValueError("m0 must be [3][n]")
        iid = C.c_int32()
        self._check(self.L.bpm_instance_add(self.h, mid, C.byref(ms), C.byref(fs), _p(off), _p(m0a),
                                            C.c_uint64(int(seed)), C.byref(iid)))
        return iid.value

    def couple_dipoles(self, ids):
        a = np.ascontiguousarray(ids, dtype=np.int32)
        self._check(self.L.bpm_couple_dipoles(self.h, len(a), _p(a)))

    def clear_instances(self):
        self._check(self.L.bpm_clear_instances(self.h))

    # runs ---------------------------------------------------------------------------------------
    def run(self, t_end, precision=64, integrator=DP45, dt0=1e-15, dt_fixed=0.0, rtol=1e-6, atol=None,
            dt_min=1e-19, temperature=0.0, max_steps=0, save_every=0, traj_cap=0, wg_per_group=0,
            flags=0, stream=None):
        o = bpm_run_opts()
        o.precision, o.integrator, o.t_end, o.dt0, o.dt_fixed = precision, integrator, t_end, dt0, dt_fixed
        o.rtol, o.atol = rtol, (rtol if atol is None else atol)
        o.dt_min, o.temperature, o.max_steps = dt_min, temperature, max_steps
        o.save_every, o.traj_cap, o.wg_per_group, o.flags = save_every, traj_cap, wg_per_group, flags
        self._check(self.L.bpm_run(self.h, C.byref(o), None if stream is None else C.c_void_p(stream)))

    def autotune(self, candidates, probe_attempts=60, t_end=1e-9, precision=32, integrator=DP45, rtol=1e-5,
                 dt0=1e-15, dt_fixed=0.0, flags=0):
        o = bpm_run_opts()
        o.precision, o.integrator, o.t_end, o.dt0, o.dt_fixed = precision, integrator, t_end, dt0, dt_fixed
        o.rtol, o.atol, o.dt_min, o.flags = rtol, rtol, 1e-19, flags
        cand = np.ascontiguousarray(candidates, dtype=np.int32)
        ms = np.empty(len(cand))
        best = C.c_int32()
        self._check(self.L.bpm_autotune(self.h, C.byref(o), len(cand), _p(cand), int(probe_attempts),
                                        C.byref(best), _p(ms)))
        return best.value, ms

    def sync(self):
        self._check(self.L.bpm_sync(self.h))

    def results(self, ids):
        a = np.ascontiguousarray(ids, dtype=np.int32)
        out = (bpm_result * len(a))()
        self._check(self.L.bpm_get_results(self.h, len(a), _p(a), out))
        return [r.as_dict() for r in out]

    def trajectory(self, iid, cap):
        out = np.zeros((max(cap, 1), 9))
        nw = C.c_int64()
        self._check(self.L.bpm_get_trajectory(self.h, iid, _p(out), cap, C.byref(nw)))
        return out[:nw.value]

    def get_m(self, iid, n, out=None):
        """Final magnetisation [3][n] FP64: into a new host array, or into `out` (a device tensor
        of 3n doubles)."""
        if out is not None:
            self._check(self.L.bpm_get_m(self.h, iid, _dp(out), 1))
            return out
        host = np.empty((3, n))
        self._check(self.L.bpm_get_m(self.h, iid, _p(host), 0))
        return host

    def string_reparam(self, ids):
        """Moves the images `ids` (chain order, final states of the last run) back to equal spacing
        along the chain and stores them as the instances' m0; returns the arc lengths of the
        images before the move."""
        a = np.ascontiguousarray(ids, dtype=np.int32)
        s = np.empty(len(a))
        self._check(self.L.bpm_string_reparam(self.h, len(a), _p(a), _p(s)))
        return s

    def last_run_info(self):
        ms = C.c_double(); grid = C.c_int32(); G = C.c_int32()
        self._check(self.L.bpm_last_run_info(self.h, C.byref(ms), C.byref(grid), C.byref(G)))
        return dict(kernel_ms=ms.value, grid=grid.value, wg_per_group=G.value)

    def last_run_layout(self):
        """Threads per workgroup, rows of S kept in LDS (0 = streamed), CSR entries staged in LDS,
        instances per staged right-hand-side block and dynamic LDS bytes of the last DP5 run."""
        v = [C.c_int32() for _ in range(4)]
        b = C.c_int64()
        self._check(self.L.bpm_last_run_layout(self.h, *(C.byref(x) for x in v), C.byref(b)))
        return dict(threads=v[0].value, s_rows_lds=v[1].value, csr_cap=v[2].value, rhs_block=v[3].value,
                    lds_bytes=b.value)


def _dp(x):
    """Device pointer of a torch tensor (or an int address)."""
    return C.c_void_p(x if isinstance(x, int) else x.data_ptr())


_SIDE = None


@contextlib.contextmanager
def _ts(stream):
    """Stream argument for calls on torch tensors: the given HIP stream, else one ordered after
    the torch work that produced the inputs and before torch's later work (and any reuse of the
    buffers by its allocator): torch's current stream, or -- when that is the default stream,
    whose handle 0 the library would read as its own stream -- a side stream that waits on it
    before the call and that it waits on after the call."""
    if stream is not None:
        yield C.c_void_p(stream)
        return
    import torch
    global _SIDE
    cur = torch.cuda.current_stream()
    if cur.cuda_stream:
        yield C.c_void_p(cur.cuda_stream)
        return
    if _SIDE is None:
        _SIDE = torch.cuda.Stream()
    _SIDE.wait_stream(cur)
    try:
        yield C.c_void_p(_SIDE.cuda_stream)
    finally:
        cur.wait_stream(_SIDE)


class Mlp:
    """Surrogate MLP 12 -> 4 x 256 -> 3 on the GPU (bpm_mlp).  Device buffers are torch tensors;
    calls run on torch's current stream unless a HIP stream is given."""

    def __init__(self, ctx: Context, max_batch: int = 4096, theta=None):
        self.ctx, self.L = ctx, ctx.L
        self.h = C.c_void_p()
        th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float32)
        ctx._check(self.L.bpm_mlp_create(ctx.h, int(max_batch), _p(th), C.byref(self.h)))
        self.n_params = self.L.bpm_mlp_num_params()

    def close(self):
        if self.h:
            self.L.bpm_mlp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        assert th.size == self.n_params
        self.ctx._check(self.L.bpm_mlp_set_params(self.h, _p(th)))

    def get_params(self):
        out = np.empty(self.n_params, np.float32)
        self.ctx._check(self.L.bpm_mlp_get_params(self.h, _p(out)))
        return out

    def predict(self, X, Y, n=None, stream=None):
        n = X.shape[0] if n is None else n
        with _ts(stream) as st:
            self.ctx._check(self.L.bpm_mlp_predict(self.h, _dp(X), _dp(Y), int(n), st))

    def grads(self, X, T, mask, batch=None):
        import torch
        batch = X.shape[0] if batch is None else batch
        loss = C.c_float()
        g = np.empty(self.n_params, np.float32)
        torch.cuda.current_stream().synchronize()    # the call runs on the library's own stream
        self.ctx._check(self.L.bpm_mlp_grads(self.h, _dp(X), _dp(T), _dp(mask), int(batch), C.byref(loss), _p(g)))
        return loss.value, g

    def train_step(self, X, T, mask, lr, batch=None, want_loss=True, stream=None):
        batch = X.shape[0] if batch is None else batch
        loss = C.c_float()
        with _ts(stream) as st:
            self.ctx._check(self.L.bpm_mlp_train_step(self.h, _dp(X), _dp(T), _dp(mask), int(batch), float(lr),
                                                      C.byref(loss) if want_loss else None, st))
        return loss.value if want_loss else None

    def topk(self, score, k, idx, n=None, stream=None):
        n = score.shape[0] if n is None else n
        with _ts(stream) as st:
            self.ctx._check(self.L.bpm_topk(self.h, _dp(score), int(n), int(k), _dp(idx), st))

    def screen(self, seed, n, k, lo, hi, min_stability, X, Y, score, idx, stream=None):
        lo = np.ascontiguousarray(lo, dtype=np.float64); hi = np.ascontiguousarray(hi, dtype=np.float64)
        with _ts(stream) as st:
            self.ctx._check(self.L.bpm_screen(self.h, C.c_uint64(int(seed)), int(n), int(k), _p(lo), _p(hi),
                                              float(min_stability), _dp(X), _dp(Y), _dp(score), _dp(idx), st))


def topk_noalloc(ctx: Context, score, k, idx, n=None, stream=None):
    """bpm_topk_noalloc: indices of the k largest of n device scores into the device int64 idx,
    with the library's fixed scratch area (no allocation)."""
    n = score.shape[0] if n is None else n
    with _ts(stream) as st:
        ctx._check(ctx.L.bpm_topk_noalloc(ctx.h, _dp(score), int(n), int(k), _dp(idx), st))


def gp_ei(ctx: Context, model: bpm_gp, m, cand, ei, seed=0, yhat=None, sd=None, stream=None):
    """bpm_gp_ei on device tensors: EI (and yhat, s) of the kriging model at m candidates
    (generated into cand when seed != 0)."""
    with _ts(stream) as st:
        ctx._check(ctx.L.bpm_gp_ei(ctx.h, C.byref(model), int(m), _dp(cand), C.c_uint64(int(seed)),
                                   None if yhat is None else _dp(yhat), None if sd is None else _dp(sd), _dp(ei), st))


def argmax(ctx: Context, v, idx, m=None, stream=None):
    """bpm_argmax: index of the largest of the device FP64 values v into the device int64 idx."""
    m = v.shape[0] if m is None else m
    with _ts(stream) as st:
        ctx._check(ctx.L.bpm_argmax(ctx.h, _dp(v), int(m), _dp(idx), st))


def sample_designs(ctx: Context, seed, n, X, stream=None):
    with _ts(stream) as st:
        ctx._check(ctx.L.bpm_sample_designs(ctx.h, C.c_uint64(int(seed)), int(n), _dp(X), st))


def nan_to_none(x):
    return None if (x is None or (isinstance(x, float) and math.isnan(x))) else x
