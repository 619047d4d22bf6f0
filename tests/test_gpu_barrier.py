"""Energy barrier by the string method on the GPU solver (Sec. II.C, Eq. (3)), against the oracle.

FP64: the GPU string (relaxation launches with the precession term dropped, redistribution
kernel) follows the oracle's string iteration by iteration: energies and arc lengths to 1e-9
relative, images to 1e-8, E_B to 1e-8.  FP32: E_B within 1 % of the FP64 oracle.  The coherent
island's barrier matches the closed form K V (1 - h)^2 on the GPU path too, and BER_adj closes
BER_tot with the write errors.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_1603_09493_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def adj(oracle_mod):
    mesh = I.media_mesh(n_target=300)
    om = oracle_mod.OracleMesh(mesh)
    S = om.demag_S()
    mat = dataclasses.replace(I.media_material(), alpha=1.0)
    g, org, h = I.default_head_grid(B_peak=2.2)
    lay = I.recording_layout()
    fld = I.adjacent_field(g, org, h, layout=lay, cross_offset=-3e-9)
    return mesh, om, S, mat, fld, lay, (g, org, h)


def _gpu_string(mesh, S, mat, fld, chain, offset, precision, **kw):
    from paper_1603_09493_amd import barrier as B, bpm
    ctx = bpm.Context(0)
    try:
        mid = ctx.mesh_add(mesh, S)
        return B.string_barrier(ctx, mid, mesh.n, mat, fld, chain, offset=offset, precision=precision, **kw)
    finally:
        ctx.close()


def test_string_fp64_parity(adj):
    from oracle import barrier as OBar
    mesh, om, S, mat, fld, lay, _ = adj
    P, iters, dtau = 13, 30, 2e-12
    chain = I.rotation_chain(mesh.n, P)
    print(f"[gpu-case] string-fp64 n={mesh.n} P={P} iters={iters}", flush=True)
    ro = OBar.string_barrier(om, S, mat, fld, chain, offset=lay["adjacent"], dtau=dtau, iters=iters)
    rg = _gpu_string(mesh, S, mat, fld, chain, lay["adjacent"], 64, dtau=dtau, iters=iters)
    Emax = np.abs(ro["energies"]).max()
    assert np.abs(rg.energies - ro["energies"]).max() <= 1e-9 * Emax
    assert np.abs(rg.arclen - ro["arclen"]).max() <= 1e-9 * ro["arclen"][-1]
    assert max(np.abs(a - b).max() for a, b in zip(rg.images, ro["images"])) <= 1e-8
    assert abs(rg.E_B / ro["E_B"] - 1) <= 1e-8
    kT = 1.380649e-23 * 300
    assert 60 < ro["E_B"] / kT < 200            # an ECC island of this size: ~10^2 kT


def test_string_fp32_barrier_within_one_percent(adj):
    from oracle import barrier as OBar
    mesh, om, S, mat, fld, lay, _ = adj
    P, iters, dtau = 13, 30, 2e-12
    chain = I.rotation_chain(mesh.n, P)
    print(f"[gpu-case] string-fp32 n={mesh.n}", flush=True)
    ro = OBar.string_barrier(om, S, mat, fld, chain, offset=lay["adjacent"], dtau=dtau, iters=iters)
    rg = _gpu_string(mesh, S, mat, fld, chain, lay["adjacent"], 32, dtau=dtau, iters=iters)
    assert abs(rg.E_B / ro["E_B"] - 1) <= 0.01


@pytest.mark.parametrize("h", [0.0, 0.5])
def test_string_coherent_island_closed_form(oracle_mod, h):
    mesh = I.island_mesh(2e-9, 2e-9, 2e-9, 2e-9, 1.0e-9, seed=3)
    V = oracle_mod.OracleMesh(mesh).export()["V"].sum()
    K, Ms = 0.5e6, 0.5e6
    mat = I.Material(Ms=(Ms, Ms), K=(K, K), A=(1e-10, 1e-10), A_int=1e-10, alpha=1.0)
    fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=h * 2 * K / Ms, dir=(0.0, 0.0, -1.0), t_rise=0.0)
    print(f"[gpu-case] string-macrospin h={h}", flush=True)
    r = _gpu_string(mesh, np.zeros((mesh.n, mesh.n)), mat, fld, I.rotation_chain(mesh.n, 13), (0.0, 0.0, 0.0),
                    64, dtau=1e-12, iters=8)
    assert abs(r.E_B / (K * V * (1 - h) ** 2) - 1) < 2e-3


def test_ber_tot_with_adjacent_barrier(adj):
    """BER_targ + BER_prev + BER_adj for one design: the adjacent stage runs only after both write
    stages passed, and its rate matches Eq. (3) on the oracle's barrier."""
    from oracle import barrier as OBar
    from paper_1603_09493_amd import barrier as B, ber_driver as D, bpm
    mesh, om, S, mat, _, lay, (g, org, h) = adj
    wmat = I.media_material()
    fld = I.recording_field(g, org, h, down_offset=4e-9)
    got = {}

    def adj_rate():
        got["ber"], got["b"] = B.adjacent_error(ctx, mesh, mid_adj, dataclasses.replace(wmat, alpha=1.0), g, org, h,
                                                layout=lay, cross_offset=0.0, P=13, iters=30)
        return got["ber"]

    ctx = bpm.Context(0)
    try:
        mid = ctx.mesh_add(mesh, S)
        mid_adj = mid
        print(f"[gpu-case] ber-tot n={mesh.n}", flush=True)
        w = D.write_errors(ctx, mesh, mid, wmat, fld, layout=lay, precision=64, ber_adj=adj_rate)
    finally:
        ctx.close()
    assert w.stage == "done" and "ber" in got
    assert w.ber_tot == pytest.approx(w.ber_targ + w.ber_prev + got["ber"], rel=1e-12)
    fa = I.adjacent_field(g, org, h, layout=lay, cross_offset=0.0)
    ro = OBar.string_barrier(om, S, dataclasses.replace(wmat, alpha=1.0), fa, I.rotation_chain(mesh.n, 13),
                             offset=lay["adjacent"], dtau=2e-12, iters=30)
    assert abs(got["b"].E_B / ro["E_B"] - 1) <= 1e-8
    assert abs(got["ber"] / OBar.ber_adj(ro["E_B"]) - 1) <= 1e-5
