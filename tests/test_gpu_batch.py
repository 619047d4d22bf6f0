"""GPU parity of the batched path (independent uneven islands, one workgroup each) and of
continued runs, through the C ABI.

* The demag product that reads only the upper triangle of S (64 x 64 tiles, FP32) against the
  FP64 oracle and against the full product, element by element, on islands of 266-2898 nodes
  (ragged last tiles, the largest island of the design box).
* Continued runs (BPM_FLAG_CONTINUE) against one run: identical for fixed steps on their grid,
  the same switching for adaptive steps; misuse rejected.
* 64 designs of the 4096-island batch, FP32 adaptive in one launch, against the FP64 oracle's
  switching time and field (stored by tests/golden/make_batch_switching.py, which calls only the
  oracle).
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1603_09493_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch4096_switching.json")


@pytest.fixture(scope="module")
def ctx():
    from paper_1603_09493_amd import bpm
    c = bpm.Context(0)
    yield c
    c.close()


def _case(name, **kw):
    print(f"[gpu-case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _batch_rows():
    """Rows of the 4096-design batch: the smallest and largest island and two whose node counts
    leave ragged 64-node tiles."""
    X = I.sample_designs(4096, seed=2)
    n = np.array([I.design_node_target(x) for x in X])
    order = np.argsort(n, kind="stable")
    rows = [int(order[0]), int(order[-1])]
    for q in order[len(order) // 3:]:
        if n[q] % 64 not in (0, 63) and len(rows) < 4 and int(q) not in rows:
            rows.append(int(q))
    return X, rows


@pytest.mark.parametrize("keep", [3, 6, 4, 8])
def test_tiled_symmetric_product_against_oracle(ctx, oracle_mod, keep):
    """FP32 fixed-step DP5 (200 steps of 5 fs) of four batch islands in one launch, one workgroup
    each, upper-triangle demag product, from seeded states within 0.6 rad of +z: every node within
    1e-4 of the FP64 oracle, and within 2e-5 of the same launch with the full product.  keep 3:
    tiles read from the row-major S; 6: from the packed upper-triangle tiles; 4: the group keeps
    only the packed tiles (the full product is then refused), whose unpacked copy equals S to FP32
    rounding; 8: only the FP16 tiles, whose unpacked copy is within FP16 rounding (2^-11
    relative) of every entry."""
    from paper_1603_09493_amd import bpm
    X, rows = _batch_rows()
    T, dt = 1e-12, 5e-15
    ctx.clear_instances()
    cases = []
    for q in rows:
        mesh, mat, fld = I.design_inputs(X[q], seed=q)
        om = oracle_mod.OracleMesh(mesh)
        S = om.demag_S()
        mid = ctx.mesh_add(mesh, S, keep=keep)
        if keep == 4:
            Sg = ctx.mesh_get_S(mid)
            assert np.array_equal(Sg, Sg.T)
            assert np.abs(Sg - S).max() <= 2 ** -23 * np.abs(S).max(), np.abs(Sg - S).max()
        if keep == 8:
            Sg = ctx.mesh_get_S(mid)
            assert np.array_equal(Sg, Sg.T)
            assert np.all(np.abs(Sg - S) <= 2 ** -11 * np.abs(S)), np.abs((Sg - S) / S).max()
            assert np.abs(Sg - S).max() > 0.0
        m0 = I.random_unit_m(mesh.n, seed=100 + q, cone=0.6)
        cases.append((mesh, mat, fld, om, S, ctx.instance_add(mid, mat, fld, m0=m0), m0))
    _case("tiled-symmetric", keep=keep, sizes=[c[0].n for c in cases])
    assert min(c[0].n for c in cases) < 300 and max(c[0].n for c in cases) > 2800
    got, energy = {}, {}
    for name, flags in (("sym", bpm.FLAG_SYMMETRIC_DEMAG), ("full", 0)):
        if keep in (4, 8) and name == "full":
            with pytest.raises(bpm.BpmError) as e:
                ctx.run(t_end=T, precision=32, integrator=bpm.DP5_FIXED, dt_fixed=dt, wg_per_group=1, flags=flags)
            assert e.value.code == bpm.BPM_EINVAL
            continue
        ctx.run(t_end=T, precision=32, integrator=bpm.DP5_FIXED, dt_fixed=dt, wg_per_group=1, flags=flags)
        ctx.sync()
        assert ctx.last_run_info()["wg_per_group"] == 1
        got[name] = [ctx.get_m(c[5], c[0].n) for c in cases]
        res = ctx.results([c[5] for c in cases])
        assert all(r["status"] == 0 and r["n_accept"] == 200 for r in res)
        energy[name] = [r["energy"] for r in res]
    for idx, (mesh, mat, fld, om, S, iid, m0) in enumerate(cases):
        ms = got["sym"][idx]
        mo, ro, _ = om.run(S, [mat], [fld], dict(t_end=T, integrator=oracle_mod.DP5_FIXED, dt_fixed=dt), m0=m0)
        assert np.abs(mo[0] - m0).max() > 1e-2          # the state moved
        assert np.abs(ms - mo[0]).max() <= 1e-4, (mesh.n, np.abs(ms - mo[0]).max())
        assert abs(energy["sym"][idx] / ro[0]["energy"] - 1) <= 1e-3, (energy["sym"][idx], ro[0]["energy"])
        if "full" in got:
            assert np.abs(ms - got["full"][idx]).max() <= 2e-5, (mesh.n, np.abs(ms - got["full"][idx]).max())


def test_continued_fixed_step_run_is_identical(ctx, oracle_mod):
    """FP64 fixed step on the single-island workload: 0 -> 1 ps -> 2 ps -> 3 ps in three runs
    takes the same 300 steps as one 3 ps run and lands on the same state and trajectory (to the
    rounding of the grid time at the splits), and both match the oracle."""
    from paper_1603_09493_amd import bpm
    mesh, mat, fld = I.single_island_workload()
    om = oracle_mod.OracleMesh(mesh)
    S = om.demag_S()
    dt = 10e-15
    ctx.clear_instances()
    mid = ctx.mesh_add(mesh, S)
    iid = ctx.instance_add(mid, mat, fld)
    _case("continue-fixed", n=mesh.n)
    kw = dict(precision=64, integrator=bpm.DP5_FIXED, dt_fixed=dt, save_every=25, traj_cap=64)
    ctx.run(t_end=3e-12, **kw)
    ctx.sync()
    m1, r1, t1 = ctx.get_m(iid, mesh.n), ctx.results([iid])[0], ctx.trajectory(iid, 64)
    for k, T in enumerate((1e-12, 2e-12, 3e-12)):
        ctx.run(t_end=T, flags=bpm.FLAG_CONTINUE if k else 0, **kw)
        ctx.sync()
    m3, r3, t3 = ctx.get_m(iid, mesh.n), ctx.results([iid])[0], ctx.trajectory(iid, 64)
    assert r3["status"] == r1["status"] == 0, (r1, r3)
    assert r3["n_accept"] == r1["n_accept"] == 300, (r1["n_accept"], r3["n_accept"])
    assert abs(r3["t_reached"] - 3e-12) <= 1e-24 and abs(r1["t_reached"] - 3e-12) <= 1e-24
    assert np.abs(m1 - m3).max() <= 1e-13, np.abs(m1 - m3).max()
    assert t1.shape == t3.shape, (t1.shape, t3.shape)
    assert np.abs(t1 - t3).max() <= 1e-13, np.abs(t1 - t3).max(axis=0)
    mo, ro, _ = om.run(S, [mat], [fld], dict(t_end=3e-12, integrator=oracle_mod.DP5_FIXED, dt_fixed=dt))
    assert np.abs(m3 - mo[0]).max() <= 1e-9


def test_continued_adaptive_batch_switches_alike(ctx):
    """FP32 adaptive, upper-triangle product, eight batch islands driven hard enough to switch:
    ten continued 20 ps slices give the same switching as one 0.2 ns run (the only difference is
    the step shortened to land on each slice end)."""
    from paper_1603_09493_amd import bpm
    X = I.sample_designs(8, seed=21)
    X[:, 9] = 2.0                        # peak field at the top of the range
    X[:, 5:7] = np.minimum(X[:, 5:7], 0.6e6)
    ctx.clear_instances()
    ids = []
    for q, x in enumerate(X):
        mesh, mat, fld = I.design_inputs(x, seed=q)
        ids.append(ctx.instance_add(ctx.mesh_add(mesh, keep=2), mat, fld))
    _case("continue-adaptive", islands=len(ids))
    kw = dict(precision=32, rtol=1e-5, flags=bpm.FLAG_SYMMETRIC_DEMAG)
    ctx.run(t_end=0.2e-9, **kw)
    ctx.sync()
    one = ctx.results(ids)
    for k in range(10):
        ctx.run(t_end=0.2e-9 * (k + 1) / 10, **dict(kw, flags=kw["flags"] | (bpm.FLAG_CONTINUE if k else 0)))
        ctx.sync()
    sl = ctx.results(ids)
    print("[continue-adaptive]", [(a["switched"], a["t_sw"], b["t_sw"], a["n_accept"], b["n_accept"])
                                  for a, b in zip(one, sl)], flush=True)
    assert sum(r["switched"] for r in one) >= 4
    for a, b in zip(one, sl):
        assert a["status"] == b["status"] == 0 and abs(b["t_reached"] - 0.2e-9) <= 1e-21, (a, b)
        assert a["switched"] == b["switched"], (a, b)
        if a["switched"]:
            assert abs(a["t_sw"] / b["t_sw"] - 1) <= 1e-3, (a, b)
        assert abs(a["mz_hard"] - b["mz_hard"]) <= 5e-3, (a, b)
        assert abs(a["n_accept"] - b["n_accept"]) <= 20, (a, b)


def test_continue_misuse_is_rejected(ctx):
    from paper_1603_09493_amd import bpm
    mesh, mat, fld = I.single_island_workload(n_target=300)
    ctx.clear_instances()
    mid = ctx.mesh_add(mesh)
    iid = ctx.instance_add(mid, mat, fld)
    ctx.run(t_end=1e-12, precision=64, integrator=bpm.DP5_FIXED, dt_fixed=10e-15)
    ctx.sync()
    for bad, code in ((dict(t_end=0.5e-12), bpm.BPM_EINVAL),
                      (dict(t_end=2e-12, precision=32), bpm.BPM_EINVAL),
                      (dict(t_end=2e-12, dt_fixed=7e-15), bpm.BPM_EINVAL)):
        kw = dict(precision=64, integrator=bpm.DP5_FIXED, dt_fixed=10e-15, flags=bpm.FLAG_CONTINUE)
        kw.update(bad)
        with pytest.raises(bpm.BpmError) as e:
            ctx.run(**kw)
        assert e.value.code == code
    assert ctx.results([iid])[0]["t_reached"] == 1e-12   # the failed calls left the results alone
    ctx.instance_add(mid, mat, fld)      # the instance set changed
    with pytest.raises(bpm.BpmError) as e:
        ctx.run(t_end=2e-12, precision=64, integrator=bpm.DP5_FIXED, dt_fixed=10e-15, flags=bpm.FLAG_CONTINUE)
    assert e.value.code == bpm.BPM_ESTATE


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="tests/golden/batch4096_switching.json not generated")
@pytest.mark.parametrize("keep", ["KEEP_S32_TILES", "KEEP_S16_TILES"])
def test_batch_switching_parity_64_designs(keep):
    """64 designs of the batch (266-2898 nodes) in one FP32 adaptive launch, one workgroup per
    island, upper-triangle demag product on the packed FP32 tiles (the bench's storage) or on the
    FP16 tiles, 0.3 ns: the switched flag agrees with the FP64 oracle wherever the oracle's final
    hard-layer <m_z> is clear of zero, and the switching time and field agree within 1 %."""
    from paper_1603_09493_amd import bpm
    with open(GOLDEN) as f:
        gold = json.load(f)
    X = I.sample_designs(4096, seed=2)
    c = bpm.Context(0)
    try:
        ids = []
        for d in gold["designs"]:
            mesh, mat, fld = I.design_inputs(X[d["row"]], seed=d["row"])
            assert mesh.n == d["n"]
            ids.append(c.instance_add(c.mesh_add(mesh, keep=getattr(bpm, keep)), mat, fld))
        _case("batch-64", keep=keep, sizes=f"{min(d['n'] for d in gold['designs'])}-{max(d['n'] for d in gold['designs'])}")
        # one workgroup per island, as in the 4096-island launch (64 groups alone would get a
        # cooperative share of the GPU each)
        c.run(t_end=gold["t_end"], precision=32, rtol=1e-5, flags=bpm.FLAG_SYMMETRIC_DEMAG, wg_per_group=1)
        c.sync()
        assert c.last_run_info()["wg_per_group"] == 1
        res = c.results(ids)
    finally:
        c.close()
    n_sw = 0
    for d, r in zip(gold["designs"], res):
        assert r["status"] == 0
        if abs(d["mz_hard"]) > 0.2:
            assert bool(r["switched"]) == bool(d["switched"]), d
        if d["switched"] and r["switched"]:
            n_sw += 1
            assert abs(r["t_sw"] / d["t_sw"] - 1) <= 0.01, (d, r["t_sw"])
            assert abs(r["B_sw"] / d["B_sw"] - 1) <= 0.01, (d, r["B_sw"])
    assert n_sw >= 16


def test_batch_autotune_and_tune_cache(tmp_path):
    """The launch-shape tuner on a batch of islands: one 256-thread workgroup per island (two
    islands per compute unit) or one 512-thread workgroup; it keeps the faster, a run that names
    no shape uses it, and a new context given the same cache file uses it without tuning."""
    from paper_1603_09493_amd import bpm
    X = I.sample_designs(48, seed=2)
    cache = str(tmp_path / "tune.txt")

    def setup(c):
        ids = []
        for q, x in enumerate(X):
            mesh, mat, fld = I.design_inputs(x, seed=q)
            ids.append(c.instance_add(c.mesh_add(mesh, keep=2), mat, fld))
        return ids

    c = bpm.Context(0, tune_cache=cache)
    try:
        ids = setup(c)
        _case("batch-autotune", islands=len(ids))
        best, ms = c.autotune([1, -1], probe_attempts=12, t_end=1e-11, precision=32, rtol=1e-5,
                              flags=bpm.FLAG_SYMMETRIC_DEMAG)
        assert np.all(np.isfinite(ms)) and best == [1, -1][int(np.argmin(ms))], (best, ms)
        c.run(t_end=1e-13, precision=32, rtol=1e-5, flags=bpm.FLAG_SYMMETRIC_DEMAG)
        c.sync()
        assert c.last_run_info()["wg_per_group"] == 1
        assert c.last_run_layout()["threads"] == (512 if best < 0 else 256)
        assert all(r["status"] == 0 for r in c.results(ids))
    finally:
        c.close()
    line = open(cache).read().split()
    assert len(line) == 4 and int(line[3]) == best
    c2 = bpm.Context(0, tune_cache=cache)
    try:
        setup(c2)
        c2.run(t_end=1e-13, precision=32, rtol=1e-5, flags=bpm.FLAG_SYMMETRIC_DEMAG)
        c2.sync()
        assert c2.last_run_layout()["threads"] == (512 if best < 0 else 256)
    finally:
        c2.close()


@pytest.mark.parametrize("precision,integrator", [(64, 1), (32, 0), (32, 2)])
def test_get_m_into_device_memory(ctx, precision, integrator):
    """bpm_get_m into a device buffer equals the host copy, for both state layouts (stepping runs
    [R][3][n], thermal runs [3][n][R]) and both precisions."""
    import torch
    from paper_1603_09493_amd import bpm
    mesh, mat, fld = I.single_island_workload(n_target=300)
    ctx.clear_instances()
    mid = ctx.mesh_add(mesh)
    ids = [ctx.instance_add(mid, mat, fld, m0=I.random_unit_m(mesh.n, 40 + r, cone=0.5), seed=r) for r in range(3)]
    _case("get-m-device", precision=precision, integrator=integrator)
    kw = dict(t_end=0.2e-12, precision=precision, integrator=integrator)
    if integrator != 0:
        kw.update(dt_fixed=2e-15, temperature=300.0 if integrator == 2 else 0.0)
    ctx.run(**kw)
    ctx.sync()
    for i in ids:
        host = ctx.get_m(i, mesh.n)
        dev = torch.empty(3 * mesh.n, dtype=torch.float64, device="cuda")
        ctx.get_m(i, mesh.n, out=dev)
        assert np.array_equal(dev.cpu().numpy().reshape(3, mesh.n), host)
        assert np.abs(np.sqrt((host ** 2).sum(0)) - 1).max() < 1e-5
