"""Benchmark of the batched FE-LLG island solver on one MI355X.

Headline workload: a batch of 4096 independent exchange-coupled-composite islands from designs
drawn uniformly in the design box (d 6-12 nm, soft/hard thickness 2-8 nm, Ms 0.4-1.2 MA/m and
K 0.1-1.5 MJ/m^3 per layer, interlayer exchange 0.5-10 pJ/m, field angle 0-45 deg, peak field
0.8-2.0 T; seed 2), meshed with a node count proportional to the island volume in [300, 3000],
each with its own FP32 dense demag operator, driven by a uniform field ramped over 0.1 ns, and
integrated with adaptive Dormand-Prince 5(4) (FP32, rtol 1e-5) in one persistent launch.

One step = one slice of that run: every island is advanced by --slice-ps picoseconds through the
whole stepping path (exchange SpMV, anisotropy, interlayer coupling, Zeeman, demag product on the
upper triangle of S, LLG right-hand side, error norm, step control, |m| renormalisation and the
switching observables); the first timed step starts the run at t = 0 and every later step
continues it (BPM_FLAG_CONTINUE).  --steps 67 --slice-ps 15 covers the configured 1 ns.  The
default (20 steps of 15 ps, 0.3 ns) fits a ten-minute job; a wall-clock guard stops stepping
early rather than overrun --budget-s, and the line says how much was simulated.

Also reported: the roofline of the stepping kernel (algorithmic bytes / its HIP-event time), HBM
traffic from the committed rocprofv3 counter summary, the learned screen (trained on the batch's
own solver labels, held-out switching-field error, 1M-candidate screening rounds), the
optimiser's expected-improvement kernel, the write-error evaluation (BER_tot of 16 designs in lock
step), the stochastic path, and the FP64 oracle on a subsample of the same designs on the host
cores.  --demag-storage fp16 runs the headline on FP16 tiles of S.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import signal
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

T_PROCESS = time.time()
METRIC = "island-ns simulated/s (batched LLG) + surrogate designs/s at ≤2% Hsw error"
COUNTERS = os.path.join(ROOT, "profiles", "dp5_kernel_batch4096_%stiles_counters.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1603_09493_amd", "csrc", "llg_kernels.hip")


def log(msg):
    print(f"[bench {time.time() - T_PROCESS:6.1f}s] {msg}", file=sys.stderr, flush=True)


def cpu_info():
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def kernel_source_sha():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_ratio(storage="fp32"):
    """(FETCH_SIZE + WRITE_SIZE) of the profiled stepping launch, scaled by the counters' reading
    for a device copy of known size, per algorithmic byte of that launch -- or None when the
    summary is missing or was taken on another kernel source or storage of S."""
    path = COUNTERS % storage
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv["kernel_source_sha256"] != kernel_source_sha() or kv.get("demag_storage", storage) != storage:
            return None
        fetch = float(kv["fetch_kib_per_launch"]) * 1024 * float(kv["fetch_scale"])
        write = float(kv["write_kib_per_launch"]) * 1024 * float(kv["write_scale"])
        return (fetch + write) / float(kv["algorithmic_bytes_per_launch"])
    except (KeyError, ValueError, ZeroDivisionError):
        return None


def cpu_baseline(rows, slice_s, cores):
    """The FP64 oracle on the first `cores` designs of the batch, one design per thread (the
    oracle runs one island per call; ctypes releases the GIL), for slice_s of simulated time each,
    same tolerance as the GPU run."""
    import concurrent.futures as cf
    from oracle import oracle as O
    from paper_1603_09493_amd import inputs as I

    def one(q):
        mesh, mat, fld = I.design_inputs(rows[q], seed=q)
        om = O.OracleMesh(mesh)
        t0 = time.perf_counter()
        S = om.demag_S()
        _, res, _ = om.run(S, [mat], [fld], dict(t_end=slice_s, rtol=1e-5))
        return mesh.n, time.perf_counter() - t0, res[0]["n_accept"] + res[0]["n_reject"]

    k = min(cores, len(rows))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=k) as ex:
        out = list(ex.map(one, range(k)))
    wall = time.perf_counter() - t0
    return {"value": k * slice_s * 1e9 / wall, "unit": "island-ns/s", "cores": k, "kind": "oracle",
            "sample": f"FP64 oracle (rtol 1e-5), the first {k} designs of the same batch "
                      f"({min(o[0] for o in out)}-{max(o[0] for o in out)} nodes), one island per thread, "
                      f"{slice_s * 1e12:.1f} ps each from t = 0 (demag operator assembly included), "
                      f"{wall:.1f} s wall"}


def copy_calibration(mib, reps=3):
    """Plain device copies of known size, for scaling the profiler's FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"bytes_read": n * 4, "bytes_written": n * 4, "reps": reps}


def surrogate_leg(ctx, rows, res, n_test=512, n_cand=1_000_000, k=10_000, epochs=250):
    """Trains the MLP on the batch's own solver labels (switched flag, switching time and field
    after the timed window), reports the held-out switching-field error and times 1M-candidate
    screening rounds over the same design box."""
    import numpy as np
    import torch
    from paper_1603_09493_amd import bpm
    from paper_1603_09493_amd import inputs as I
    from paper_1603_09493_amd import surrogate as SG
    n = len(res)
    sw = np.array([bool(r["switched"]) and math.isfinite(r["t_sw"]) and r["t_sw"] > 0 for r in res])
    lab = SG.Labels(sw, np.array([r["B_sw"] if s else np.nan for r, s in zip(res, sw)]),
                    np.array([r["t_sw"] if s else np.nan for r, s in zip(res, sw)]),
                    np.array([r["status"] for r in res]), 0.0, 0.0)
    X = SG.scale(rows).astype(np.float32)
    tr, te = slice(0, n - n_test), slice(n - n_test, n)
    pick = lambda L, s: SG.Labels(L.switched[s], L.B_sw[s], L.t_sw[s], L.status[s], 0, 0)
    lab_tr, lab_te = pick(lab, tr), pick(lab, te)
    sc = SG.TargetScaler.fit(lab_tr)
    T, mask = sc.targets(lab_tr)
    net = bpm.Mlp(ctx, 512, I.mlp_init_params(3))
    t0 = time.perf_counter()
    SG.train(net, X[tr], T, mask, epochs=epochs, batch=64, lr=2e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    Y = SG.predict(net, X[te])
    m = lab_te.switched
    head = np.abs(sc.B_of(Y[m, 0]) / lab_te.B_sw[m] - 1.0)
    comb = np.abs(SG.bsw_predicted(sc, X[te][m], Y[m]) / lab_te.B_sw[m] - 1.0)
    ramp = lab_te.t_sw[m] < rows[te][m, 11]
    acc = float(np.mean((Y[:, 2] > 0) == lab_te.switched))
    # the design box of the batch (damping and rise time fixed at 0.1 and 0.1 ns)
    lo, hi = I.DESIGN_LO.copy(), I.DESIGN_HI.copy()
    for f in (10, 11):
        lo[f] = rows[0, f]
        hi[f] = rows[0, f] * (1 + 1e-9)
    Xd = torch.empty((n_cand, 12), dtype=torch.float32, device="cuda")
    Yd = torch.empty((n_cand, 3), dtype=torch.float32, device="cuda")
    sd = torch.empty(n_cand, dtype=torch.float32, device="cuda")
    idx = torch.empty(k, dtype=torch.int64, device="cuda")
    times = []
    for i in range(4):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        net.screen(100 + i, n_cand, k, lo, hi, 40.0, Xd, Yd, sd, idx)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
    net.close()
    dt = min(times[1:])
    return {"designs_per_s": n_cand / dt, "candidates": n_cand, "top_k": k, "screen_ms": dt * 1e3,
            "n_train": n - n_test, "n_test": n_test, "train_s": train_s, "epochs": epochs,
            "labels": "switched flag, t_sw, B_sw of the timed batch run itself",
            "hsw_mean_rel_err": float(head.mean()) if head.size else None,
            "hsw_p95_rel_err": float(np.percentile(head, 95)) if head.size else None,
            "hsw_mean_rel_err_switch_during_ramp": float(head[ramp].mean()) if ramp.any() else None,
            "n_test_switched": int(m.sum()), "n_test_switch_during_ramp": int(ramp.sum()),
            "hsw_mean_rel_err_two_head_estimate": float(comb.mean()) if comb.size else None,
            "switch_classification_accuracy": acc,
            "valid_at_2pct": bool(head.size and head.mean() <= 0.02)}


def ego_ei_leg(ctx, n=128, d=4, m=1 << 22, reps=5):
    """Expected improvement of a fitted kriging model (n training points in d dimensions) at m
    Philox candidates per call, and its argmax: the GPU step of the global optimiser.  Algorithmic
    FP64 work per candidate: the n correlations (3d + 2 flops each, the exponential counted as
    one), the triangular L^-1 r (n (n + 1) flops), alpha' r and w' r (4n), the n squares (2n) and
    about 40 for the EI formula."""
    import numpy as np
    import torch
    from paper_1603_09493_amd import bpm as B, ego, roofline
    from paper_1603_09493_amd import inputs as I
    X = I.lhs_maximin(n, d, seed=5, sweeps=5)
    y = np.sin(5 * X[:, 0]) * np.cos(3 * X[:, 1]) + (X ** 2).sum(1)
    t0 = time.perf_counter()
    model = ego.fit(X, y, starts=4)
    fit_s = time.perf_counter() - t0
    prop = ego.Proposer(ctx, d, m)
    idx = torch.empty(1, dtype=torch.int64, device="cuda")
    dm = prop.evaluate(model, float(y.min()), 1)
    torch.cuda.synchronize()
    # a stream of its own, so that the events bracket exactly the library's launches on it
    st = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(st)
    for r in range(reps):
        B.gp_ei(ctx, dm.desc, m, prop.cand, prop.ei, seed=2 + r, yhat=prop.yhat, sd=prop.sd, stream=st.cuda_stream)
        B.argmax(ctx, prop.ei, idx, stream=st.cuda_stream)
    ev[1].record(st)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    flops = m * (n * (3 * d + 2) + n * (n + 1) + 6 * n + 40)
    del dm
    return {"n_train": n, "d": d, "candidates": m, "ms_per_call": ms, "candidates_per_s": m / ms * 1e3,
            "fit_s": fit_s, "bound": "mfma", "achieved_tflops": flops / ms / 1e9,
            "peak_tflops": roofline.MI355X_FP64_TFLOPS, "frac": flops / ms / 1e9 / roofline.MI355X_FP64_TFLOPS,
            "kernel": "gp_ei_kernel + argmax (L^-1 r on FP64 matrix cores, 16x16x4; peak: FP64 78.6 TFLOP/s)"}


def write_error_leg(ctx, designs=16, nodes=300):
    """BER_tot of `designs` start designs of the optimiser (maximin Latin hypercube over K_1,hard,
    A_ex,int and the down- and cross-track offsets, seed 1) on the synthetic 2.2 T head, FP32,
    judged in lock step: the critical-field searches of the target and previous bit (12 fields
    per level on a sigma/2 grid, two refinements) and the adjacent island's string (13 images,
    30 iterations) of every design share launches."""
    from paper_1603_09493_amd import ego
    from paper_1603_09493_amd import inputs as I
    mesh = I.media_mesh(n_target=nodes)
    det = []
    f = ego.ber_objective_many(ctx, mesh, I.default_head_grid(), precision=32, details=det)
    U = I.lhs_maximin(designs, 4, seed=1)
    t0 = time.perf_counter()
    y = f(list(U))
    dt = time.perf_counter() - t0
    stages = [d["stage"] for d in det]
    return {"designs": designs, "nodes": mesh.n, "precision": "f32", "wall_s": dt, "designs_per_s": designs / dt,
            "stages": {k: stages.count(k) for k in sorted(set(stages))}, "best_log10_ber_tot": float(min(y)),
            "search": "12 fields per level, sigma/2 grid, up to 4 extensions, 2 refinements, 1 ns write period",
            "barrier": "string method, 13 images, 30 relaxation launches of 2 ps"}


def thermal_leg(ctx, meshes, realizations=1024, steps=40, dt=5e-15, temperature=300.0):
    """Thermal-erasure workload: each mesh (the patch island, one mesh seed per design) carries
    `realizations` Philox streams of the single-island material in a static stray field drawn
    uniformly in 0.3-0.6 T along -z, at 300 K, integrated with stochastic Heun in FP32 at dt for
    `steps` steps.  Reports realization-ns/s, the FP32 matrix-core rate of the demag products
    (2 N^2 R flops per field evaluation, two evaluations per step) divided by the whole step time
    (exchange and field phases included; the GEMM kernel alone is in the profile) and the erased
    fractions."""
    import numpy as np
    from paper_1603_09493_amd import bpm, roofline, thermal
    from paper_1603_09493_amd import inputs as I
    rng = np.random.default_rng(3)
    mat = I.Material()
    ctx.clear_instances()
    ids, flops, B = [], 0.0, []
    t0 = time.perf_counter()
    for dsg, mesh in enumerate(meshes):
        mid = ctx.mesh_add(mesh, keep=2)
        B.append(float(rng.uniform(0.3, 0.6)))
        fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=B[-1], dir=(0.0, 0.0, -1.0), t_rise=0.0)
        ids.append([ctx.instance_add(mid, mat, fld, seed=(3 << 48) | (dsg << 20) | r) for r in range(realizations)])
        flops += 2 * 2.0 * mesh.n * mesh.n * realizations
    setup_s = time.perf_counter() - t0
    kw = dict(precision=32, integrator=bpm.HEUN, dt_fixed=dt, temperature=temperature)
    ctx.run(t_end=2 * dt, **kw)        # warm-up: graph capture, first touch
    ctx.sync()
    t0 = time.perf_counter()
    ctx.run(t_end=steps * dt, **kw)
    ctx.sync()
    wall = time.perf_counter() - t0
    k_ms = ctx.last_run_info()["kernel_ms"]
    erased = []
    for grp in ids:
        k, n_ok = thermal.count_erased(ctx.results(grp))
        erased.append(k / realizations)
    ctx.clear_instances()
    tf = flops * steps / (k_ms * 1e-3) / 1e12
    n_real = len(meshes) * realizations
    return {"designs": len(meshes), "realizations_per_design": realizations,
            "nodes_per_island_mean": float(np.mean([m.n for m in meshes])), "steps": steps, "dt_fs": dt * 1e15,
            "temperature_K": temperature, "stray_field_T": [min(B), max(B)],
            "value": n_real * steps * dt * 1e9 / wall, "unit": "realization-ns/s", "kernel_ms": k_ms,
            "ms_per_heun_step": k_ms / steps, "setup_s": setup_s,
            "demag_tflops_over_step_time": tf,
            "demag_flops_per_step_over_step_time_frac_fp32_mfma": tf / roofline.MI355X_FP32_TFLOPS,
            "erased_fraction_max": max(erased),
            "exposure_ns": steps * dt * 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--slice-ps", type=float, default=15.0, help="simulated time per step (ps)")
    ap.add_argument("--islands", type=int, default=4096)
    ap.add_argument("--budget-s", type=float, default=500.0,
                    help="wall-clock budget of the whole process; stepping stops early to keep it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-ego", action="store_true", help="skip the optimiser's EI kernel leg")
    ap.add_argument("--no-ber", action="store_true", help="skip the write-error (BER_tot) leg")
    ap.add_argument("--full-demag", action="store_true", help="read all of S (default: its upper triangle)")
    ap.add_argument("--demag-storage", choices=["fp32", "fp16"], default="fp32",
                    help="storage of the packed upper-triangle tiles of S (arithmetic stays FP32)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="also run three device copies of this many MiB (scales the profiler's byte counters)")
    ap.add_argument("--cpu-slice-ps", type=float, default=16.0, help="simulated time per oracle island (ps)")
    ap.add_argument("--thermal", type=int, default=64,
                    help="designs of the thermal-erasure leg (x 1024 realizations each; 0 = skip)")
    ap.add_argument("--thermal-steps", type=int, default=40)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design, not an implemented path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from paper_1603_09493_amd import inputs as I
    cores, cpu_model = cpu_info()
    rows = I.sample_designs(args.islands, seed=2)
    # meshing first (worker processes started before any GPU work in this process)
    ins = I.design_inputs_many(rows)
    log(f"meshed {len(ins)} islands ({sum(m.n for m, _, _ in ins)} nodes, "
        f"{min(m.n for m, _, _ in ins)}-{max(m.n for m, _, _ in ins)} per island)")
    thermal_meshes = I.patch_island_meshes([1 + d for d in range(args.thermal)]) if args.thermal > 0 else []
    from paper_1603_09493_amd import bpm, roofline
    ctx = bpm.Context(0)
    t0 = time.perf_counter()
    ids, sizes, nnzs = [], [], []
    # the batch keeps its operators as FP32 packed upper-triangle tiles only (about half the bytes
    # of row-major S); --full-demag keeps the row-major FP32 copy for the full product
    # (--demag-storage fp16: the tiles in FP16, widened to FP32 in the product)
    if args.full_demag and args.demag_storage != "fp32":
        ap.error("--full-demag reads the row-major FP32 copy")
    keep = bpm.KEEP_S32 if args.full_demag else (bpm.KEEP_S16_TILES if args.demag_storage == "fp16" else bpm.KEEP_S32_TILES)
    s_entry = 2 if args.demag_storage == "fp16" else 4
    for q, (mesh, mat, fld) in enumerate(ins):
        mid = ctx.mesh_add(mesh, keep=keep)
        ids.append(ctx.instance_add(mid, mat, fld))
        sizes.append(mesh.n)
        nnzs.append(int(ctx.mesh_get_assembly(mid, pattern_only=True)))
        if q % 1024 == 1023:
            log(f"set up {q + 1} islands")
    setup_s = time.perf_counter() - t0
    log(f"setup {setup_s:.1f} s (host assembly + GPU demag operators)")
    flags = 0 if args.full_demag else bpm.FLAG_SYMMETRIC_DEMAG
    sl = args.slice_ps * 1e-12
    kw = dict(precision=32, rtol=1e-5)

    # launch shape tuned on the batch itself: one 256-thread workgroup per island (two islands per
    # compute unit) or one 512-thread workgroup per island
    t0 = time.perf_counter()
    cands = [1, -1]
    tuned, tune_ms = ctx.autotune(cands, probe_attempts=12, t_end=sl, precision=32, rtol=1e-5, flags=flags)
    tune_info = {"candidates": ["256 threads x 1 wg/island", "512 threads x 1 wg/island"],
                 "ms_per_attempt": [float(x) for x in tune_ms], "chosen": int(tuned),
                 "tune_s": time.perf_counter() - t0}
    log(f"autotune: {dict(zip(tune_info['candidates'], [round(x, 2) for x in tune_info['ms_per_attempt']]))}")
    for w in range(args.warmup):
        ctx.run(t_end=sl / 10, flags=flags, **kw)
        ctx.sync()
        log(f"warmup {w}: kernel {ctx.last_run_info()['kernel_ms']:.0f} ms")

    state = {"done": 0, "kernel_ms": 0.0, "wall": 0.0}
    out = {}

    def emit(partial_reason=None):
        done = state["done"]
        res = ctx.results(ids) if done else []
        att = np.array([r["n_accept"] + r["n_reject"] for r in res]) if res else np.zeros(1)
        sim_ns = done * args.slice_ps * 1e-3
        wall = state["wall"]
        by = sum(roofline.eval_bytes(n, z, 1, 4, symmetric=not args.full_demag, ps=s_entry) * (6 * a + 1)
                 for n, z, a in zip(sizes, nnzs, att)) if res else 0.0
        fl = sum(roofline.eval_flops(n, z, 1) * (6 * a + 1) for n, z, a in zip(sizes, nnzs, att)) if res else 0.0
        k_s = state["kernel_ms"] * 1e-3
        achieved = by / k_s / 1e9 if k_s > 0 else 0.0
        tr = traffic_ratio(args.demag_storage)
        out.update({
            "metric": METRIC,
            "value": args.islands * sim_ns / wall if wall > 0 else 0.0,
            "unit": "island-ns/s",
            "n_gpus": 1,
            "steps": done,
            "warmup": args.warmup,
            "ms_per_step": 1e3 * wall / done if done else None,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32",
            "data": "synthetic",
            "config": {
                "workload": "batch of %d independent ECC islands, designs uniform in the design box "
                            "(seed 2), P1 meshes of 300-3000 nodes proportional to volume, per-island "
                            "FP32 dense demag, ramped uniform field, adaptive DP5(4) rtol 1e-5, 1 ns "
                            "configured" % args.islands,
                "islands": args.islands,
                "nodes_total": int(sum(sizes)), "nodes_min": int(min(sizes)), "nodes_max": int(max(sizes)),
                "configured_ns": 1.0,
                "simulated_ns": sim_ns,
                "slice_ps": args.slice_ps,
                "steps_requested": args.steps,
                "demag_product": "full S" if args.full_demag else "upper triangle of S, packed 64x64 tiles",
                "demag_storage": args.demag_storage,
                "switched_fraction": float(np.mean([r["switched"] for r in res])) if res else None,
                "attempts_mean": float(att.mean()), "attempts_max": int(att.max()),
                "status_ok": int(sum(r["status"] == 0 for r in res)) if res else 0,
                "setup_s": setup_s,
                "grid": ctx.last_run_info()["grid"],
                "threads_per_wg": ctx.last_run_layout()["threads"],
                "autotune": tune_info,
            },
            "roofline": {
                "bound": "hbm",
                "kernel": "dp5_kernel (FP32, one %d-thread workgroup per island)" % ctx.last_run_layout()["threads"],
                "achieved": achieved,
                "peak": roofline.MI355X_HBM_GBS,
                "unit": "GB/s",
                "frac": achieved / roofline.MI355X_HBM_GBS,
                "traffic": None if tr is None else tr * by,
                "algorithmic_bytes": by,
                "kernel_s": k_s,
                "launches": done,
                "achieved_tflops": fl / k_s / 1e12 if k_s > 0 else 0.0,
            },
        })
        if partial_reason:
            out["config"]["stopped_early"] = partial_reason
        return out

    def on_term(signum, frame):
        emit(f"signal {signum} after {state['done']} steps")
        print(json.dumps(out), flush=True)
        os._exit(0)

    signal.signal(signal.SIGTERM, on_term)
    # wall time kept for what follows the timed steps (measured: surrogate ~10 s, thermal leg
    # ~3 s, oracle sample ~15 s, write-error leg ~41 s), with margin
    reserve = (20.0 + (0.0 if args.no_surrogate else 25.0) + (0.0 if args.no_cpu_baseline else 30.0)
               + (0.0 if args.thermal <= 0 else 10.0 + 0.1 * args.thermal) + (0.0 if args.no_ber else 60.0))
    stop = None
    t_step = None
    for k in range(args.steps):
        elapsed = time.time() - T_PROCESS
        if t_step is not None and elapsed + 1.3 * t_step + reserve > args.budget_s:
            stop = f"wall-clock budget: {k} of {args.steps} steps in {args.budget_s:.0f} s"
            log(stop)
            break
        t1 = time.perf_counter()
        ctx.run(t_end=(k + 1) * sl, flags=flags | (bpm.FLAG_CONTINUE if k else 0), **kw)
        ctx.sync()
        t_step = time.perf_counter() - t1
        state["wall"] += t_step
        state["kernel_ms"] += ctx.last_run_info()["kernel_ms"]
        state["done"] = k + 1
        log(f"step {k + 1}/{args.steps}: t = {(k + 1) * args.slice_ps:.0f} ps, {t_step:.2f} s")
    emit(stop)
    log(f"value {out['value']:.3f} island-ns/s, HBM {out['roofline']['frac']:.3f} of peak")
    res = ctx.results(ids)
    if args.copy_calib > 0:
        out["copy_calibration"] = copy_calibration(args.copy_calib)
    if not args.no_surrogate:
        try:
            out["surrogate"] = surrogate_leg(ctx, rows, res)
            log(f"surrogate: {out['surrogate']['designs_per_s']:.3g} designs/s, "
                f"held-out Hsw error {out['surrogate']['hsw_mean_rel_err']}")
            solver_rate = args.islands / out["ms_per_step"] / args.steps * 1e3 if out["ms_per_step"] else None
            out["surrogate"]["solver_designs_per_s"] = solver_rate
            out["surrogate"]["screen_vs_solver"] = (out["surrogate"]["designs_per_s"] / solver_rate
                                                    if solver_rate else None)
        except Exception as e:   # the line is still printed
            out["surrogate"] = {"error": repr(e)}
    if not args.no_ego:
        try:
            out["ego_ei"] = ego_ei_leg(ctx)
            log(f"ego EI: {out['ego_ei']['candidates_per_s']:.3g} candidates/s, "
                f"{out['ego_ei']['achieved_tflops']:.2f} TFLOP/s FP64")
        except Exception as e:
            out["ego_ei"] = {"error": repr(e)}
    if not args.no_ber:
        try:
            out["write_errors"] = write_error_leg(ctx)
            log(f"write errors: {out['write_errors']['designs_per_s']:.3g} designs/s in lock step")
        except Exception as e:
            out["write_errors"] = {"error": repr(e)}
    if args.thermal > 0:
        try:
            out["thermal"] = thermal_leg(ctx, thermal_meshes, steps=args.thermal_steps)
            log(f"thermal: {out['thermal']['value']:.3g} realization-ns/s, demag flops over step time "
                f"{out['thermal']['demag_tflops_over_step_time']:.1f} TFLOP/s")
        except Exception as e:
            out["thermal"] = {"error": repr(e)}
    ctx.close()
    if not args.no_cpu_baseline:
        try:
            cb = cpu_baseline(rows, args.cpu_slice_ps * 1e-12, cores)
            cb["nproc"] = cores
            cb["cpu_model"] = cpu_model
            out["cpu_baseline"] = cb
            log(f"cpu baseline {cb['value']:.3g} island-ns/s on {cb['cores']} cores")
        except Exception as e:
            out["cpu_baseline"] = {"error": repr(e), "nproc": cores, "cpu_model": cpu_model}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
