"""GPU stochastic Heun path (many realizations per island) against the oracle and against
closed-form statistics.

Bars: FP64 with the same Philox noise -- max |dm| <= 1e-9 over a short run; FP32 statistics of
free rotational diffusion and of the Boltzmann equilibrium in a uniaxial well within their
sampling error.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from paper_1603_09493_amd import inputs as I

pytestmark = pytest.mark.gpu

GAMMA = 1.76085963023e11
KB = 1.380649e-23


@pytest.fixture(scope="module")
def ctx():
    from paper_1603_09493_amd import bpm
    c = bpm.Context(0)
    yield c
    c.close()


def _case(name, **kw):
    print(f"[gpu-case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def test_heun_fp64_parity_with_noise(ctx, oracle_mod):
    from paper_1603_09493_amd import bpm
    O = oracle_mod
    mesh, mat, fld = I.single_island_workload(n_target=300)
    om = O.OracleMesh(mesh)
    S = om.demag_S()
    R = 5
    seeds = [(3 << 32) | (100 + r) for r in range(R)]
    T, dt, Temp = 1.0e-12, 5e-15, 300.0
    _case("heun-fp64", n=mesh.n, R=R, steps=int(T / dt))
    mo, ro, _ = om.run(S, [mat] * R, [fld] * R, dict(t_end=T, integrator=O.HEUN, dt_fixed=dt, temperature=Temp),
                       seeds=seeds)
    ctx.clear_instances()
    mid = ctx.mesh_add(mesh, S)
    ids = [ctx.instance_add(mid, mat, fld, seed=sd) for sd in seeds]
    ctx.run(t_end=T, precision=64, integrator=bpm.HEUN, dt_fixed=dt, temperature=Temp)
    ctx.sync()
    for r, i in enumerate(ids):
        mg = ctx.get_m(i, mesh.n)
        assert np.abs(mg - mo[r]).max() <= 1e-9, r
    res = ctx.results(ids)
    for a, b in zip(res, ro):
        assert a["status"] == 0 and a["n_accept"] == b["n_accept"]
        assert abs(a["mz_hard"] - b["mz_hard"]) < 1e-9
    # different seeds give different paths; the noise did act
    assert np.abs(mo[0] - mo[1]).max() > 1e-6


def test_heun_fp64_parity_in_moving_grid_field(ctx, oracle_mod):
    """The stochastic path in the gridded moving head field (the adjacent island of the
    pseudo-hexagonal layout, cross-track offset 2 nm, the head moving during the run), FP64 with
    the same noise: every node within 1e-9 of the oracle."""
    from paper_1603_09493_amd import bpm
    O = oracle_mod
    mesh = I.media_mesh(n_target=300)
    om = O.OracleMesh(mesh)
    S = om.demag_S()
    mat = I.media_material()
    g, org, h = I.default_head_grid()
    lay = I.recording_layout()
    fld = I.recording_field(g, org, h, down_offset=4e-9, cross_offset=2e-9)
    R = 3
    seeds = [(5 << 32) | (7 + r) for r in range(R)]
    offs = np.array([lay["target"], lay["adjacent"], lay["previous"]])
    T, dt, Temp = 1.0e-12, 5e-15, 300.0
    _case("heun-fp64-grid", n=mesh.n, R=R, steps=int(T / dt))
    mo, ro, _ = om.run(S, [mat] * R, [fld] * R, dict(t_end=T, integrator=O.HEUN, dt_fixed=dt, temperature=Temp),
                       seeds=seeds, offsets=offs)
    ctx.clear_instances()
    mid = ctx.mesh_add(mesh, S)
    ids = [ctx.instance_add(mid, mat, fld, offset=tuple(offs[r]), seed=sd) for r, sd in enumerate(seeds)]
    ctx.run(t_end=T, precision=64, integrator=bpm.HEUN, dt_fixed=dt, temperature=Temp)
    ctx.sync()
    for r, i in enumerate(ids):
        assert np.abs(ctx.get_m(i, mesh.n) - mo[r]).max() <= 1e-9, r
    # the head field reached the islands differently: their states differ beyond the noise
    assert np.abs(mo[0] - mo[1]).max() > 1e-6


def test_heun_clipped_last_step_and_graph_replay(ctx, oracle_mod):
    """t_end not a multiple of dt: graph-replayed regular steps plus one shorter final step."""
    from paper_1603_09493_amd import bpm
    O = oracle_mod
    mesh, mat, fld = I.single_island_workload(n_target=300)
    om = O.OracleMesh(mesh)
    S = om.demag_S()
    T, dt = 0.2035e-12, 5e-15
    _case("heun-clip", n=mesh.n)
    mo, ro, _ = om.run(S, [mat], [fld], dict(t_end=T, integrator=O.HEUN, dt_fixed=dt, temperature=300.0), seeds=[9])
    ctx.clear_instances()
    mid = ctx.mesh_add(mesh, S)
    i = ctx.instance_add(mid, mat, fld, seed=9)
    ctx.run(t_end=T, precision=64, integrator=bpm.HEUN, dt_fixed=dt, temperature=300.0)
    ctx.sync()
    assert np.abs(ctx.get_m(i, mesh.n) - mo[0]).max() <= 1e-9
    assert ctx.results([i])[0]["n_accept"] == ro[0]["n_accept"] == 41


@pytest.mark.parametrize("R,steps,mixed", [(64, 7.0, True), (64, 7.5, False), (70, 0.6, True), (128, 2.0, False)])
def test_heun_fp64_parity_step_parity_and_wave_layouts(ctx, oracle_mod, R, steps, mixed):
    """Odd and even step counts (the state alternates between two buffers), a clipped final
    step with no regular step before it, R a multiple of 64 (one node per wave) or not, and
    realizations with shared or differing constants -- each against the oracle, every node."""
    import dataclasses
    from paper_1603_09493_amd import bpm
    O = oracle_mod
    mesh, mat, fld = I.single_island_workload(n_target=300)
    om = O.OracleMesh(mesh)
    S = om.demag_S()
    dt = 5e-15
    T = steps * dt
    seeds = [(7 << 32) | (R << 12) | r for r in range(R)]
    flds = [dataclasses.replace(fld, B_peak=fld.B_peak * (0.8 if (mixed and r % 3 == 1) else 1.0)) for r in range(R)]
    _case("heun-fp64-layout", n=mesh.n, R=R, steps=steps, mixed=mixed)
    mo, ro, _ = om.run(S, [mat] * R, flds, dict(t_end=T, integrator=O.HEUN, dt_fixed=dt, temperature=300.0),
                       seeds=seeds)
    ctx.clear_instances()
    mid = ctx.mesh_add(mesh, S)
    ids = [ctx.instance_add(mid, mat, f, seed=sd) for f, sd in zip(flds, seeds)]
    ctx.run(t_end=T, precision=64, integrator=bpm.HEUN, dt_fixed=dt, temperature=300.0)
    ctx.sync()
    res = ctx.results(ids)
    for r, i in enumerate(ids):
        assert np.abs(ctx.get_m(i, mesh.n) - mo[r]).max() <= 1e-9, r
        assert res[r]["n_accept"] == ro[r]["n_accept"] == math.ceil(steps - 1e-9)
        assert abs(res[r]["mz_hard"] - ro[r]["mz_hard"]) < 1e-9


@pytest.mark.parametrize("R", [200, 256])
def test_heun_fp32_matrix_core_path_against_oracle(ctx, oracle_mod, R):
    """FP32 runs use the 128 x 128 matrix-core demag product (ragged in both dimensions here:
    N = 324 rows in tiles of 128, R = 200 columns = 128 + 72; R = 256 also takes the wave-uniform
    field kernels) and FP32 noise transforms: every node of every realization against the FP64
    oracle with the same Philox noise.  Bar: 2e-4 after 10 steps at 300 K (FP32 rounding; a wrong
    tile or lane mapping of the product gives errors of order 1e-2 and more)."""
    from paper_1603_09493_amd import bpm
    O = oracle_mod
    mesh, mat, fld = I.single_island_workload(n_target=300)
    om = O.OracleMesh(mesh)
    S = om.demag_S()
    seeds = [(11 << 32) | (R << 12) | r for r in range(R)]
    T, dt, Temp = 10 * 5e-15, 5e-15, 300.0
    _case("heun-fp32-mfma", n=mesh.n, R=R, steps=10)
    mo, ro, _ = om.run(S, [mat] * R, [fld] * R, dict(t_end=T, integrator=O.HEUN, dt_fixed=dt, temperature=Temp),
                       seeds=seeds)
    ctx.clear_instances()
    mid = ctx.mesh_add(mesh, S, keep=3)
    ids = [ctx.instance_add(mid, mat, fld, seed=sd) for sd in seeds]
    ctx.run(t_end=T, precision=32, integrator=bpm.HEUN, dt_fixed=dt, temperature=Temp)
    ctx.sync()
    worst = max(float(np.abs(ctx.get_m(i, mesh.n) - mo[r]).max()) for r, i in enumerate(ids))
    print(f"[heun-fp32] R={R}: max |dm| = {worst:.2e}", flush=True)
    assert worst <= 2e-4
    # the noise acted: realizations differ far beyond the bar
    assert np.abs(mo[0] - mo[1]).max() > 1e-3


def test_free_rotational_diffusion_many_realizations(ctx):
    from paper_1603_09493_amd import bpm
    mesh = I.island_mesh(4e-9, 4e-9, 2e-9, 3e-9, 1.0e-9, seed=2)
    Ms, alpha, Temp = 1.0e6, 0.5, 300.0
    mat = I.Material(Ms=(Ms, Ms), K=(0.0, 0.0), A=(0.0, 0.0), A_int=0.0, alpha=alpha)
    fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=0.0, t_rise=0.0)
    R, t = 64, 1.0e-12
    _case("heun-diffusion", n=mesh.n, R=R)
    ctx.clear_instances()
    mid = ctx.mesh_add(mesh)
    ids = [ctx.instance_add(mid, mat, fld, seed=1000 + r) for r in range(R)]
    ctx.run(t_end=t, precision=32, integrator=bpm.HEUN, dt_fixed=1e-15, temperature=Temp)
    ctx.sync()
    V = ctx.mesh_get_assembly(mid)["V"]
    mz = np.array([ctx.get_m(i, mesh.n)[2] for i in ids])
    D = alpha * GAMMA * KB * Temp / ((1 + alpha ** 2) * Ms * V)
    e1 = np.exp(-2 * D * t)
    e2 = 1 / 3 + 2 / 3 * np.exp(-6 * D * t)
    z1 = ((mz - e1) / np.sqrt(e2 - e1 ** 2)).mean() * math.sqrt(mz.size)
    assert abs(z1) < 4.0, z1
    assert abs((mz ** 2 - e2).mean()) < 0.01


def _mz2_boltzmann(s):
    Z = quad(lambda x: math.exp(s * x * x), -1, 1)[0]
    return math.exp(s) / (s * Z) - 1 / (2 * s)


def test_boltzmann_equilibrium_many_realizations(ctx):
    """Independent macrospins (no exchange, no demag) in a uniaxial well at 300 K: the ensemble
    <m_z^2> of every node matches the Boltzmann value for s = K V_i / kB T."""
    from paper_1603_09493_amd import bpm
    mesh = I.island_mesh(4e-9, 4e-9, 2e-9, 3e-9, 1.0e-9, seed=2)
    Ms, K, alpha, Temp = 1.0e6, 2.0e7, 1.0, 300.0
    mat = I.Material(Ms=(Ms, Ms), K=(K, K), A=(0.0, 0.0), A_int=0.0, alpha=alpha)
    fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=0.0, t_rise=0.0)
    R = 256
    _case("heun-boltzmann", n=mesh.n, R=R)
    ctx.clear_instances()
    S0 = np.zeros((mesh.n, mesh.n))
    mid = ctx.mesh_add(mesh, S0)
    ids = [ctx.instance_add(mid, mat, fld, seed=(7 << 32) | r) for r in range(R)]
    ctx.run(t_end=60e-12, precision=32, integrator=bpm.HEUN, dt_fixed=2e-15, temperature=Temp)
    ctx.sync()
    V = ctx.mesh_get_assembly(mid)["V"]
    mz = np.array([ctx.get_m(i, mesh.n)[2] for i in ids])
    s = K * V / (KB * Temp)
    ref = np.array([_mz2_boltzmann(x) for x in s])
    assert abs((mz ** 2 - ref[None, :]).mean()) < 0.01
    # both wells populated (barrier crossings happened): the sign of m_z is balanced
    assert abs(np.sign(mz).mean()) < 0.1


def _reversed_fraction_boltzmann(s, h):
    """Macrospin in a uniaxial well (barrier parameter s = K V / kB T) with a field along -z
    (h = Ms V B / kB T): P(m_z < 0) with the Boltzmann density exp(s x^2 - h x) in x = cos(theta)
    (sin(theta) d(theta) = dx)."""
    w = lambda x: math.exp(s * x * x - h * x)
    return quad(w, -1, 0)[0] / quad(w, -1, 1)[0]


def test_erasure_fraction_matches_boltzmann(ctx):
    """Thermally induced erasure (stochastic LLG, Heun, FP32): 4096 realizations of a small
    rigid island (exchange and interlayer coupling far stiffer than kB T, no demag) from +z in a
    static field along -z at 300 K, barrier about 3 kB T.  After about ten relaxation times the
    erased fraction (hard-layer <m_z> < 0) matches the Boltzmann reversed fraction of the
    macrospin within four standard errors."""
    from paper_1603_09493_amd import bpm, thermal
    mesh = I.island_mesh(1.5e-9, 1.5e-9, 1e-9, 1e-9, 1.0e-9, seed=4)
    Ms, Temp, R = 1.0e6, 300.0, 4096
    ctx.clear_instances()
    mid = ctx.mesh_add(mesh, np.zeros((mesh.n, mesh.n)), keep=2)
    V = ctx.mesh_get_assembly(mid)["V"].sum()
    K = 3.0 * KB * Temp / V              # s = 3
    B = 0.5 * KB * Temp / (Ms * V)       # h = 0.5
    mat = I.Material(Ms=(Ms, Ms), K=(K, K), A=(200e-12, 200e-12), A_int=200e-12, alpha=1.0)
    _case("heun-erasure", n=mesh.n, R=R, K=f"{K:.3g}", B=f"{B:.4f}")
    er = thermal.run_erasure(ctx, mesh, mat, B, R, t_end=0.6e-9, dt=1.5e-15, temperature=Temp,
                             key_base=(11 << 32), mesh_id=mid)
    p_ref = _reversed_fraction_boltzmann(3.0, 0.5)
    z = (er.p - p_ref) / math.sqrt(p_ref * (1 - p_ref) / R)
    print(f"[heun-erasure] erased {er.k}/{er.n} = {er.p:.4f}, Boltzmann {p_ref:.4f}, z = {z:.2f}, "
          f"label {er.label:.3f}, {er.wall_s:.1f} s", flush=True)
    assert er.status_ok == R
    assert 0.5 < p_ref < 0.9
    assert abs(z) < 4.0, z
    assert abs(er.label - thermal.logit_label(er.k, er.n)) == 0.0
