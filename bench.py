"""Benchmark of the batched FE-LLG island solver on one MI355X.

Default workload: the 3x3 patch of dipole-coupled elliptic ECC islands (18 x 4.5 nm, t = 10 nm,
~2k-node P1 mesh each, 25 nm x 6.5 nm pitch, per-island Ms/K spread), driven by the synthetic
pole field (1.5 T, 10 nm gradient length, 20 m/s, 0.1 ns rise), integrated for 1 ns with
adaptive Dormand-Prince 5(4) in FP32.  One step = one full 1 ns run of the 9 islands (the whole
stepping path: exchange, anisotropy, interlayer, demag, Zeeman, dipoles, RK45 control and
observables) -- plus, when the surrogate is built, one screening round of the MLP.

Prints one JSON line (see the keys below).  Inputs are resident on the GPU before timing.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "island-ns simulated/s (batched LLG) + surrogate designs/s at ≤2% Hsw error"


def _device_sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except Exception:
        pass


def cpu_baseline_patch(mesh, mats, flds, offs, t_sample=2e-12):
    """The FP64 oracle on the same patch for a short window (its dipole-coupled system is one
    serial integration: one core)."""
    from oracle import oracle as O
    om = O.OracleMesh(mesh)
    S = om.demag_S()
    t0 = time.perf_counter()
    _, res, _ = om.run(S, mats, flds, dict(t_end=t_sample, rtol=1e-6), offsets=offs, coupled=True)
    wall = time.perf_counter() - t0
    return {"value": len(mats) * t_sample * 1e9 / wall, "unit": "island-ns/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle, same 9-island patch, first {t_sample*1e12:.1f} ps of the run "
                      f"({res[0]['n_accept']} DP5 steps, {wall:.1f} s wall), rate extrapolated"}


def surrogate_leg(n_train=8192, n_test=512, t_end=0.3e-9, n_cand=1_000_000, k=10_000, epochs=100, log=None):
    """Label designs with the batched FP32 solver, train the MLP with the library's kernels,
    report the held-out switching-field error and time a 1M-candidate screening round."""
    import numpy as np
    import torch

    from paper_1603_09493_amd import bpm
    from paper_1603_09493_amd import inputs as I
    from paper_1603_09493_amd import surrogate as SG
    ctx = bpm.Context(0)
    x = SG.sample(n_train + n_test, seed=12)
    lab = SG.label_designs(ctx, x, t_end=t_end, progress=log)
    solver_designs_per_s = x.shape[0] / lab.wall_s
    X = SG.scale(x).astype(np.float32)
    tr, te = slice(0, n_train), slice(n_train, None)
    lab_tr = SG.Labels(lab.switched[tr], lab.B_sw[tr], lab.t_sw[tr], lab.status[tr], 0, 0)
    lab_te = SG.Labels(lab.switched[te], lab.B_sw[te], lab.t_sw[te], lab.status[te], 0, 0)
    sc = SG.TargetScaler.fit(lab_tr)
    T, mask = sc.targets(lab_tr)
    net = bpm.Mlp(ctx, 512, I.mlp_init_params(3))
    t0 = time.perf_counter()
    SG.train(net, X[tr], T, mask, epochs=epochs, batch=64, lr=2e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    err, p95, _ = SG.bsw_error(net, sc, X[te], lab_te)
    SG.screen_round(net, seed=1, n=n_cand, k=k, min_stability=40.0)       # warm-up
    times = [SG.screen_round(net, seed=2 + i, n=n_cand, k=k, min_stability=40.0)[1] for i in range(3)]
    dt = min(times)
    net.close()
    ctx.close()
    return {"designs_per_s": n_cand / dt, "candidates": n_cand, "top_k": k, "screen_ms": dt * 1e3,
            "hsw_mean_rel_err": err, "hsw_p95_rel_err": p95, "n_train": n_train, "n_test": n_test,
            "train_s": train_s, "label_t_end_ns": t_end * 1e9,
            "solver_designs_per_s": solver_designs_per_s,
            "screen_vs_solver": (n_cand / dt) / solver_designs_per_s,
            "valid_at_2pct": bool(err <= 0.02)}


def batch_leg(n_islands=4096, t_end=1e-11, steps=1, log=None):
    """Batched independent islands of uneven size (designs uniform in the batched ranges, N
    proportional to volume in [300, 3000], FP32 demag only), one persistent launch, per-island
    adaptive steps."""
    from paper_1603_09493_amd import bpm, roofline
    from paper_1603_09493_amd import inputs as I
    ctx = bpm.Context(0)
    x = I.sample_designs(n_islands, seed=2)
    t0 = time.perf_counter()
    sizes, nnzs, ids = [], [], []
    for q, row in enumerate(x):
        mesh, mat, fld = I.design_inputs(row, seed=q)
        mid = ctx.mesh_add(mesh, keep=2)
        ids.append(ctx.instance_add(mid, mat, fld))
        sizes.append(mesh.n)
        nnzs.append(int(ctx.mesh_get_assembly(mid)["rowptr"][-1]) if q < 64 else None)
        if log and q % 1024 == 1023:
            log(f"batch: {q + 1} islands set up")
    setup_s = time.perf_counter() - t0
    ctx.run(t_end=t_end, precision=32, rtol=1e-5)      # warm-up
    ctx.sync()
    _device_sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run(t_end=t_end, precision=32, rtol=1e-5)
        ctx.sync()
    wall = time.perf_counter() - t0
    info = ctx.last_run_info()
    res = ctx.results(ids)
    att = [r["n_accept"] + r["n_reject"] for r in res]
    nnz_per_node = sum(v for v in nnzs if v) / sum(sizes[:64])
    by = sum(roofline.eval_bytes(n, int(n * nnz_per_node), 1, 4) * (6 * a + 1) for n, a in zip(sizes, att))
    ctx.close()
    return {"islands": n_islands, "simulated_ns": t_end * 1e9, "value": n_islands * t_end * 1e9 * steps / wall,
            "unit": "island-ns/s", "setup_s": setup_s, "kernel_ms": info["kernel_ms"], "grid": info["grid"],
            "nodes_total": int(sum(sizes)), "nodes_min": int(min(sizes)), "nodes_max": int(max(sizes)),
            "attempts_min": int(min(att)), "attempts_max": int(max(att)),
            "achieved_GBs": by / (info["kernel_ms"] * 1e-3) / 1e9,
            "status_ok": int(sum(1 for r in res if r["status"] == 0))}


def heun_leg(n_designs=64, realizations=1024, steps=40, dt=5e-15, temperature=300.0, log=None):
    """Thermal workload: n_designs patch-island meshes (the patch island, one mesh seed each), each
    with `realizations` Philox streams, a static stray field U(0.3, 0.6) T along -z at 300 K,
    stochastic Heun at fixed dt, FP32.  Reports realization-ns/s and the FP32 matrix-core use of
    the demag products (2 N^2 R flops per field evaluation, two evaluations per step)."""
    import dataclasses
    import numpy as np
    from paper_1603_09493_amd import bpm, roofline
    from paper_1603_09493_amd import inputs as I
    ctx = bpm.Context(0)
    rng = np.random.default_rng(3)
    base_mesh, mats, flds, _ = I.patch_workload()
    mat0 = mats[0]
    n_total, flops_per_step = 0, 0.0
    t0 = time.perf_counter()
    for dsg in range(n_designs):
        mesh = base_mesh if dsg == 0 else I.patch_workload(seed=1 + dsg)[0]
        mid = ctx.mesh_add(mesh, keep=2)
        B = float(rng.uniform(0.3, 0.6))
        fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=B, dir=(0.0, 0.0, -1.0), t_rise=0.0)
        for r in range(realizations):
            ctx.instance_add(mid, mat0, fld, seed=(3 << 48) | (dsg << 20) | r)
        n_total += mesh.n
        flops_per_step += 2 * 2.0 * mesh.n * mesh.n * realizations
        if log and dsg % 16 == 15:
            log(f"heun: {dsg + 1} designs set up")
    setup_s = time.perf_counter() - t0
    kw = dict(t_end=steps * dt, precision=32, integrator=bpm.HEUN, dt_fixed=dt, temperature=temperature)
    ctx.run(**dict(kw, t_end=2 * dt))      # warm-up (graph capture, first touch)
    ctx.sync()
    _device_sync()
    t0 = time.perf_counter()
    ctx.run(**kw)
    ctx.sync()
    wall = time.perf_counter() - t0
    k_ms = ctx.last_run_info()["kernel_ms"]
    ctx.close()
    tf = flops_per_step * steps / (k_ms * 1e-3) / 1e12
    return {"designs": n_designs, "realizations": realizations, "nodes_per_island_mean": n_total / n_designs,
            "steps": steps, "dt_fs": dt * 1e15, "value": n_designs * realizations * steps * dt * 1e9 / wall,
            "unit": "realization-ns/s", "kernel_ms": k_ms, "setup_s": setup_s,
            "demag_gemm_tflops": tf, "demag_gemm_frac_fp32_mfma": tf / roofline.MI355X_FP32_TFLOPS}


COUNTERS = os.path.join(ROOT, "profiles", "dp5_kernel_patch_counters.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1603_09493_amd", "csrc", "llg_kernels.hip")


def kernel_source_sha():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_per_eval():
    """HBM bytes per field evaluation of the stepping kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE of one profiled launch, each scaled by what the counter
    reads for a device copy of known size), or None when the summary is missing or was taken on a
    different kernel source."""
    if not os.path.exists(COUNTERS):
        return None
    kv = {}
    with open(COUNTERS) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv["kernel_source_sha256"] != kernel_source_sha():
            return None
        evals = float(kv["evals_per_launch"])
        fetch = float(kv["fetch_kib_per_launch"]) * 1024 * float(kv["fetch_scale"])
        write = float(kv["write_kib_per_launch"]) * 1024 * float(kv["write_scale"])
    except (KeyError, ValueError):
        return None
    return (fetch + write) / evals


def copy_calibration(mib=512, reps=3):
    """A plain device copy of known size (for scaling the profiler's byte counters)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"bytes_read": n * 4, "bytes_written": n * 4, "reps": reps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--t-end", type=float, default=1e-9)
    ap.add_argument("--precision", type=int, default=32)
    ap.add_argument("--wg", type=int, default=0,
                    help="workgroups per mesh group (0 = autotune; negative = that many 512-thread workgroups)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--copy-calib", action="store_true", help="also run a 512 MiB device copy (profiling)")
    ap.add_argument("--batch", type=int, default=0, help="also run N batched uneven islands (0 = skip)")
    ap.add_argument("--batch-t-end", type=float, default=1e-11)
    ap.add_argument("--heun", type=int, default=0, help="also run the thermal workload with N designs (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design in DESIGN.md, not an implemented path.", file=sys.stderr)
        sys.exit(2)

    from paper_1603_09493_amd import bpm, roofline
    from paper_1603_09493_amd import inputs as I

    mesh, mats, flds, offs = I.patch_workload()
    ctx = bpm.Context(0)
    t0 = time.perf_counter()
    mid = ctx.mesh_add(mesh)          # host assembly + GPU demag assembly (setup, not timed below)
    setup_s = time.perf_counter() - t0
    ids = [ctx.instance_add(mid, m, f, offset=o) for m, f, o in zip(mats, flds, offs)]
    ctx.couple_dipoles(ids)
    asm = ctx.mesh_get_assembly(mid)
    nnz = int(asm["rowptr"][-1])
    rtol = 1e-5 if args.precision == 32 else 1e-6
    run_kw = dict(t_end=args.t_end, precision=args.precision, rtol=rtol, wg_per_group=abs(args.wg),
                  flags=bpm.FLAG_WG512 if args.wg < 0 else 0)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    log(f"patch: {len(ids)} islands x {mesh.n} nodes, setup {setup_s:.1f} s")
    tuned = None
    if args.wg == 0:
        # workgroups per group; negative = 512-thread workgroups
        cands = [32, 64, 96, 128, 192, 256, -48, -64, -96, -112, -128, -136, -144, -160, -192, -256]
        tuned, ms = ctx.autotune(cands, probe_attempts=80, t_end=args.t_end, precision=args.precision, rtol=rtol)
        log("autotune (us/attempt): " + ", ".join(f"{c}:{1e3*m:.0f}" for c, m in zip(cands, ms)) + f" -> {tuned}")
    for w in range(args.warmup):
        ctx.run(**dict(run_kw, t_end=args.t_end / 10))     # warm-up: same launch, shorter window
        ctx.sync()
        log(f"warmup {w}: kernel {ctx.last_run_info()['kernel_ms']:.0f} ms")
    _device_sync()
    kernel_ms, attempts, wall = [], [], 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.run(**run_kw)
        ctx.sync()
        info = ctx.last_run_info()
        kernel_ms.append(info["kernel_ms"])
        r = ctx.results(ids)
        attempts.append(r[0]["n_accept"] + r[0]["n_reject"])
        log(f"step: kernel {info['kernel_ms']:.0f} ms, {attempts[-1]} attempts")
    _device_sync()
    wall = time.perf_counter() - t0
    res = ctx.results(ids)
    ms_per_step = 1e3 * wall / args.steps
    value = len(ids) * args.t_end * 1e9 * args.steps / wall

    p = args.precision // 8
    evals = 6 * attempts[-1] + 1
    by = roofline.eval_bytes(mesh.n, nnz, len(ids), p) * evals
    fl = roofline.eval_flops(mesh.n, nnz, len(ids)) * evals
    k_ms = kernel_ms[-1]
    achieved = by / (k_ms * 1e-3) / 1e9
    tpe = traffic_per_eval()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "island-ns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": "3x3 dipole-coupled ECC island patch (elliptic 18x4.5 nm, t=10 nm, "
                        "25x6.5 nm pitch), 9 x %d-node P1 meshes, pole field 1.5 T / 10 nm / 20 m/s / "
                        "0.1 ns rise, %.2g ns, DP5(4) rtol %.0e" % (mesh.n, args.t_end * 1e9, rtol),
            "islands": len(ids),
            "nodes_per_island": mesh.n,
            "nnz": nnz,
            "simulated_ns": args.t_end * 1e9,
            "wg_per_group": ctx.last_run_info()["wg_per_group"],
            "threads_per_wg": ctx.last_run_layout()["threads"],
            "autotuned_wg_per_group": tuned,
            "grid": ctx.last_run_info()["grid"],
            "attempts": attempts[-1],
            "n_reject": res[0]["n_reject"],
            "switched": [int(x["switched"]) for x in res],
            "setup_s": setup_s,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "dp5_kernel",
            "achieved": achieved,
            "peak": roofline.MI355X_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / roofline.MI355X_HBM_GBS,
            "traffic": None if tpe is None else tpe * evals,
            "algorithmic_bytes_per_launch": by,
            "evals_per_launch": evals,
            "kernel_ms": k_ms,
            "achieved_tflops": fl / (k_ms * 1e-3) / 1e12,
        },
    }
    ctx.close()
    if not args.no_surrogate:
        out["surrogate"] = surrogate_leg(log=log)
    if args.copy_calib:
        out["copy_calibration"] = copy_calibration()
    if args.batch > 0:
        out["batch"] = batch_leg(args.batch, args.batch_t_end, log=log)
    if args.heun > 0:
        out["heun"] = heun_leg(args.heun, log=log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_patch(mesh, mats, flds, offs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
