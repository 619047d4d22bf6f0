"""Learned screen driver: label designs with the batched solver, train the MLP on the GPU with the
library's own kernels, screen candidate rounds, and verify the picks with the solver.

The paper's optimizer (Sec. II.A) fits a surrogate (a Gaussian process) to the evaluated designs
and always evaluates the most promising proposal next; the solver's answer is the ground truth.
Here the surrogate is the MLP of the C ABI and a round proposes k designs out of n candidates at
once; the batched solver stays the judge of every pick.

Design vector (12): d, t_soft, t_hard, Ms_soft, Ms_hard, K_soft, K_hard, A_int, psi, B_peak,
alpha, t_rise -- inputs.DESIGN_LO/HI give the ranges.  Designs are uniform in the box; the
network inputs are log coordinates (psi linear) scaled to [-1, 1] -- the screening round maps its
uniform samples the same way on the GPU.  Targets are z-scored log B_sw, z-scored log t_sw and the
switched flag (masked regression where the design did not switch).
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import bpm
from . import inputs as I

KB = 1.380649e-23


def scale(x: np.ndarray) -> np.ndarray:
    """Network inputs of designs x: log coordinates (linear for psi) mapped to [-1, 1]."""
    return 2.0 * I.unit_of_design(x, log_prior=True) - 1.0


def unscale(X: np.ndarray) -> np.ndarray:
    return I.design_of_unit(0.5 * (np.asarray(X, dtype=np.float64) + 1.0), log_prior=True)


def sample(n: int, seed: int) -> np.ndarray:
    """n designs from the surrogate's prior (uniform in the box, alpha and the rise time varying)."""
    return I.sample_designs(n, seed=seed, fixed_alpha_rise=False)


def stability(x: np.ndarray) -> np.ndarray:
    """Thermal-stability proxy (K_s V_s + K_h V_h) / (kB 300 K) of design rows x."""
    x = np.atleast_2d(x)
    area = math.pi * 0.25 * x[:, 0] ** 2
    return (x[:, 5] * area * x[:, 1] + x[:, 6] * area * x[:, 2]) / (KB * 300.0)


@dataclasses.dataclass
class Labels:
    switched: np.ndarray   # [n] bool
    B_sw: np.ndarray       # [n] tesla (NaN where not switched)
    t_sw: np.ndarray       # [n] seconds (NaN where not switched)
    status: np.ndarray     # [n] int
    kernel_ms: float
    wall_s: float


def label_designs(ctx: bpm.Context, x: np.ndarray, t_end: float = 0.5e-9, precision: int = 32,
                  mesh_seed: int = 0, clear: bool = True, chunk: int = 512, work: float = 1.0e9,
                  progress=None) -> Labels:
    """Runs every design (rows of x) as one island, in batched launches of designs of similar size,
    each launch holding at most `chunk` designs and at most `work` summed N^2 (so that the launcher
    can give large islands several workgroups).  Every design is meshed with the same jitter seed,
    so that its mesh (and label) is a function of the design alone.  `progress` (optional) receives
    one line per launch."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    built = []
    for row in x:
        mesh, mat, fld = I.design_inputs(row, seed=mesh_seed)
        built.append((mesh, mat, fld))
    if progress is not None:
        progress(f"meshed {n} designs ({sum(b[0].n for b in built)} nodes)")
    order = np.argsort([b[0].n for b in built], kind="stable")
    sw = np.zeros(n, bool)
    tsw = np.full(n, np.nan)
    bsw = np.full(n, np.nan)
    st = np.zeros(n, np.int64)
    kernel_ms = 0.0
    wall = 0.0
    keep = 2 if precision == 32 else 1
    chunks, cur, w = [], [], 0.0
    for q in order:
        nq2 = float(built[q][0].n) ** 2
        if cur and (len(cur) >= chunk or w + nq2 > work):
            chunks.append(cur)
            cur, w = [], 0.0
        cur.append(q)
        w += nq2
    if cur:
        chunks.append(cur)
    for c0, idx in enumerate(chunks):
        if clear or c0 > 0:
            ctx.clear_instances()
        ids = []
        for q in idx:
            mesh, mat, fld = built[q]
            mid = ctx.mesh_add(mesh, keep=keep)
            ids.append(ctx.instance_add(mid, mat, fld))
        t0 = time.perf_counter()
        # FP32 launches read only the upper triangle of each island's symmetric demag operator
        ctx.run(t_end=t_end, precision=precision, rtol=1e-5 if precision == 32 else 1e-6,
                flags=bpm.FLAG_SYMMETRIC_DEMAG if precision == 32 else 0)
        ctx.sync()
        wall += time.perf_counter() - t0
        kernel_ms += ctx.last_run_info()["kernel_ms"]
        for q, r in zip(idx, ctx.results(ids)):
            sw[q], tsw[q], bsw[q], st[q] = bool(r["switched"]), r["t_sw"], r["B_sw"], r["status"]
        if progress is not None:
            progress(f"labelled chunk {c0 + 1}/{len(chunks)}: {len(idx)} designs, "
                     f"{ctx.last_run_info()['kernel_ms']:.0f} ms")
    ok = sw & np.isfinite(tsw) & np.isfinite(bsw) & (tsw > 0)
    return Labels(switched=ok, B_sw=np.where(ok, bsw, np.nan), t_sw=np.where(ok, tsw, np.nan), status=st,
                  kernel_ms=kernel_ms, wall_s=wall)


@dataclasses.dataclass
class TargetScaler:
    """z-scores of log B_sw and log t_sw (a squared error in log B_sw is a relative error)."""
    b_mu: float
    b_sd: float
    t_mu: float
    t_sd: float

    @staticmethod
    def fit(lab: Labels) -> "TargetScaler":
        b = np.log(lab.B_sw[lab.switched])
        t = np.log(lab.t_sw[lab.switched])
        return TargetScaler(float(b.mean()), float(b.std() + 1e-12), float(t.mean()), float(t.std() + 1e-12))

    def targets(self, lab: Labels):
        T = np.zeros((lab.switched.size, 3), np.float32)
        m = lab.switched
        T[m, 0] = (np.log(lab.B_sw[m]) - self.b_mu) / self.b_sd
        T[m, 1] = (np.log(lab.t_sw[m]) - self.t_mu) / self.t_sd
        T[:, 2] = m.astype(np.float32)
        return T, m.astype(np.uint8)

    def B_of(self, y0):
        return np.exp(self.b_mu + self.b_sd * np.asarray(y0, dtype=np.float64))


def train(net: bpm.Mlp, X: np.ndarray, T: np.ndarray, mask: np.ndarray, epochs: int = 200, batch: int = 512,
          lr: float = 1e-3, seed: int = 0, lr_final: float = 1e-5):
    """Minibatch Adam on device tensors (torch provides the buffers); cosine-decayed step size."""
    import torch
    rng = np.random.default_rng(seed)
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    Td = torch.from_numpy(np.ascontiguousarray(T, np.float32)).cuda()
    md = torch.from_numpy(np.ascontiguousarray(mask, np.uint8)).cuda()
    n = X.shape[0]
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    losses = []
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            xb, tb, mb = Xd[idx].contiguous(), Td[idx].contiguous(), md[idx].contiguous()
            a = 0.5 * (1 + math.cos(math.pi * step / total))
            cur = lr_final + (lr - lr_final) * a
            want = (s == steps_per_epoch - 1)
            L = net.train_step(xb, tb, mb, cur, batch=xb.shape[0], want_loss=want)
            if want:
                losses.append(L)
            step += 1
    return losses


def predict(net: bpm.Mlp, X: np.ndarray) -> np.ndarray:
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    Yd = torch.empty((X.shape[0], 3), dtype=torch.float32, device="cuda")
    net.predict(Xd, Yd)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


def bsw_predicted(sc: TargetScaler, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Switching field predicted for designs X (scaled) from the network outputs Y.  B_sw is the
    applied field at the island at t_sw; for the uniform ramped field of the design workload that
    is B_peak * min(t_sw / t_rise, 1).  The estimate is the geometric mean of that expression at
    the predicted t_sw (output 1) and of the predicted B_sw (output 0): the two heads' errors are
    partly independent."""
    x = unscale(X)
    t = np.exp(sc.t_mu + sc.t_sd * np.asarray(Y[:, 1], dtype=np.float64))
    b_t = x[:, 9] * np.minimum(t / x[:, 11], 1.0)
    return np.sqrt(b_t * sc.B_of(Y[:, 0]))


def bsw_error(net: bpm.Mlp, sc: TargetScaler, X: np.ndarray, lab: Labels):
    """Mean and 95th percentile of |relative error| of the predicted switching field over the
    designs that switched."""
    Y = predict(net, X)
    m = lab.switched
    rel = np.abs(bsw_predicted(sc, X[m], Y[m]) / lab.B_sw[m] - 1.0)
    return float(rel.mean()), float(np.percentile(rel, 95)), Y


def screen_round(net: bpm.Mlp, seed: int, n: int, k: int, min_stability: float):
    """One fused screening round on the GPU; returns (picked scaled designs [k][12], seconds)."""
    import torch
    X = torch.empty((n, 12), dtype=torch.float32, device="cuda")
    Y = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    sc = torch.empty(n, dtype=torch.float32, device="cuda")
    idx = torch.empty(k, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.screen(seed, n, k, I.DESIGN_LO, I.DESIGN_HI, min_stability, X, Y, sc, idx)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    picks = X[idx].cpu().numpy()
    return picks, dt, sc[idx].cpu().numpy()


def active_round(ctx: bpm.Context, net: bpm.Mlp, sc: TargetScaler, X: np.ndarray, T: np.ndarray, mask: np.ndarray,
                 seed: int, n: int, k: int, min_stability: float, t_end: float = 0.3e-9, epochs: int = 60,
                 lr: float = 5e-4, progress=None):
    """One closed round of the screen: score n candidates on the GPU, let the batched solver judge
    the k best, append the judged designs to the training set and continue training on it.
    Returns (X, T, mask) of the grown training set, the judged designs' Labels, their scaled
    inputs and the screen time."""
    picks, secs, _ = screen_round(net, seed=seed, n=n, k=k, min_stability=min_stability)
    lab = label_designs(ctx, unscale(picks), t_end=t_end, progress=progress)
    ok = lab.status == 0
    Tn, mn = sc.targets(Labels(lab.switched[ok], lab.B_sw[ok], lab.t_sw[ok], lab.status[ok], 0, 0))
    X2 = np.concatenate([X, picks[ok]]).astype(np.float32)
    T2 = np.concatenate([T, Tn]).astype(np.float32)
    m2 = np.concatenate([mask, mn])
    train(net, X2, T2, m2, epochs=epochs, batch=64, lr=lr, seed=seed)
    return X2, T2, m2, lab, picks, secs
