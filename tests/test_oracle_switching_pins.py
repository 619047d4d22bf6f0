"""Pins of the oracle's switching observables, inter-island dipoles and ECC coupling (no GPU).

Each reference here is computed without the oracle's formulas:
* switching time and field: the macrospin in a field along -z has a closed-form polar angle,
  tan(theta'/2) = tan(theta'_0/2) exp(-alpha gamma' int B dt) with theta' measured from -z, so the
  hard layer's <m_z> crosses zero where int_0^t B = ln(cot(theta_0/2)) / (alpha gamma');
* point dipoles: B = mu0 (3 (mu.r^) r^ - mu) / (4 pi r^3), i.e. 2 mu0 mu / (4 pi r^3) on the axis
  and -mu0 mu / (4 pi r^3) transverse, read back from one precession step of a uniform island;
  the pair energy -mu0 / (4 pi r^3) [3 (mu_I.r^)(mu_J.r^) - mu_I.mu_J];
* exchange-coupled-composite switching (paper Sec. II.B, Fig. 3: soft layer on hard layer through
  an interlayer exchange): a two-spin model of the two rigid layers, minimised by continuation
  here, which reduces to the Stoner-Wohlfarth field of each layer at J = 0 and of the averaged
  anisotropy 2 (K_s t_s + K_h t_h) / (Ms_s t_s + Ms_h t_h) as J grows (1.3100 T at 30 degrees
  for the single-island layers);
* Stoner-Wohlfarth astroid h(psi) = (cos^2/3 psi + sin^2/3 psi)^-3/2 at 1 %.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from paper_1603_09493_amd import inputs as I

MU0 = 4e-7 * math.pi
GAMMA = 1.76085963023e11


def _macrospin(alpha, B, dir_z=-1.0, t_rise=0.0):
    """A small two-layer island with no exchange, anisotropy, interlayer coupling or demag: every
    node follows the same macrospin equation exactly."""
    mesh = I.island_mesh(2e-9, 2e-9, 1e-9, 1e-9, 1.0e-9, seed=0)
    mat = I.Material(K=(0.0, 0.0), A=(0.0, 0.0), A_int=0.0, alpha=alpha)
    fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=B, dir=(0.0, 0.0, dir_z), t_rise=t_rise)
    return mesh, mat, fld


def _m_at(n, theta):
    m = np.zeros((3, n))
    m[0] = math.sin(theta)
    m[2] = math.cos(theta)
    return m


def test_switching_time_in_static_reverse_field(oracle_mod):
    alpha, B, th0 = 0.1, 1.0, 0.3
    mesh, mat, fld = _macrospin(alpha, B)
    om = oracle_mod.OracleMesh(mesh)
    gp = GAMMA / (1 + alpha ** 2)
    t_cross = -math.log(math.tan(th0 / 2)) / (alpha * gp * B)
    m, res, _ = om.run(None, [mat], [fld], dict(t_end=1.6 * t_cross, rtol=1e-10, dt0=1e-15), m0=_m_at(om.n, th0))
    r = res[0]
    assert r["status"] == 0 and r["switched"] and r["mz_hard"] < -0.5
    assert abs(r["t_sw"] / t_cross - 1) < 1e-3, (r["t_sw"], t_cross)
    assert abs(r["B_sw"] - B) < 1e-12


@pytest.mark.parametrize("th0,B_peak,during_ramp", [(1.45, 2.0, True), (0.3, 1.5, False)])
def test_switching_time_and_field_in_ramped_field(oracle_mod, th0, B_peak, during_ramp):
    """B(t) = B_peak min(t / t_rise, 1) along -z: t_sw from int_0^t B = L and B_sw = B(t_sw)."""
    alpha, t_rise = 0.1, 0.1e-9
    mesh, mat, fld = _macrospin(alpha, B_peak, t_rise=t_rise)
    om = oracle_mod.OracleMesh(mesh)
    gp = GAMMA / (1 + alpha ** 2)
    L = -math.log(math.tan(th0 / 2)) / (alpha * gp)
    if L <= B_peak * t_rise / 2:
        t_cross = math.sqrt(2 * L * t_rise / B_peak)
    else:
        t_cross = t_rise / 2 + L / B_peak
    assert (t_cross < t_rise) == during_ramp
    m, res, _ = om.run(None, [mat], [fld], dict(t_end=1.5 * t_cross, rtol=1e-10, dt0=1e-15), m0=_m_at(om.n, th0))
    r = res[0]
    assert r["status"] == 0 and r["switched"]
    assert abs(r["t_sw"] / t_cross - 1) < 1e-3, (r["t_sw"], t_cross)
    B_expect = B_peak * min(t_cross / t_rise, 1.0)
    assert abs(r["B_sw"] / B_expect - 1) < 1e-3, (r["B_sw"], B_expect)
    # the oracle's B_sw is the applied field at its own t_sw
    assert abs(r["B_sw"] - B_peak * min(r["t_sw"] / t_rise, 1.0)) < 1e-12


# ------------------------------------------------------------------------------------------
# inter-island point dipoles
# ------------------------------------------------------------------------------------------

def _dipole_pair():
    mesh = I.island_mesh(2e-9, 2e-9, 1e-9, 1.5e-9, 1.0e-9, seed=3)
    mat = I.Material(Ms=(0.9e6, 0.5e6), K=(0.0, 0.0), A=(10e-12, 10e-12), A_int=0.0, alpha=0.0)
    fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=0.0, t_rise=0.0)
    return mesh, mat, fld


def _moment(mesh, mat):
    """|mu| of a uniformly magnetised island from its tet volumes (computed here from the node
    coordinates) and the layer of each tet."""
    P = mesh.xyz.T
    t = mesh.tet
    vol = np.abs(np.einsum("ij,ij->i", P[t[:, 1]] - P[t[:, 0]],
                           np.cross(P[t[:, 2]] - P[t[:, 0]], P[t[:, 3]] - P[t[:, 0]]))) / 6
    lay = mesh.layer[t[:, 0]]
    return float(sum(mat.Ms[L] * vol[lay == L].sum() for L in (0, 1)))


@pytest.mark.parametrize("axis", ["on_axis", "transverse"])
def test_point_dipole_field_closed_form(oracle_mod, axis):
    """Island I at the origin along +z, island J at distance r (along z or along x) along +x, no
    other field: J precesses about the dipole field of I, which one step of 0.1 fs reads back."""
    mesh, mat, fld = _dipole_pair()
    om = oracle_mod.OracleMesh(mesh)
    r = 9e-9
    offs = np.array([[0, 0, 0], [0, 0, r] if axis == "on_axis" else [r, 0, 0]], dtype=np.float64)
    mI = _m_at(om.n, 0.0)
    mJ = _m_at(om.n, math.pi / 2)
    dt = 1e-16
    m, res, _ = om.run(None, [mat, mat], [fld, fld], dict(t_end=dt, integrator=oracle_mod.DP5_FIXED, dt_fixed=dt),
                       m0=np.stack([mI, mJ]), offsets=offs, coupled=True)
    mu = _moment(mesh, mat)
    Bz = (2 if axis == "on_axis" else -1) * MU0 * mu / (4 * math.pi * r ** 3)
    # dm/dt = -gamma m x B with m = x^, B = Bz z^: m rotates toward +y at rate gamma Bz
    my = m[1, 1]
    assert np.allclose(my, my[0], rtol=1e-12, atol=0)        # the field is uniform on J
    B_read = math.asin(my[0]) / (GAMMA * dt)
    assert abs(B_read / Bz - 1) < 1e-6, (B_read, Bz)


def test_point_dipole_pair_energy_and_gradient(oracle_mod):
    """Zero-length run: the total energy of two uniformly magnetised islands (no exchange,
    anisotropy, interlayer, demag or Zeeman energy) is the point-dipole pair energy; its
    derivative with respect to a rotation of J is -mu_J' . B_J."""
    mesh, mat, fld = _dipole_pair()
    om = oracle_mod.OracleMesh(mesh)
    mu = _moment(mesh, mat)
    rv = np.array([6e-9, 4e-9, -3e-9])
    r = np.linalg.norm(rv)
    e = rv / r
    offs = np.array([[0, 0, 0], rv])
    uI = np.array([0.3, -0.4, 0.866])
    uI /= np.linalg.norm(uI)

    def energy(th):
        uJ = np.array([math.sin(th), 0.0, math.cos(th)])
        m0 = np.stack([np.repeat(uI[:, None], om.n, 1), np.repeat(uJ[:, None], om.n, 1)])
        _, res, _ = om.run(None, [mat, mat], [fld, fld], dict(t_end=0.0), m0=m0, offsets=offs, coupled=True)
        return res[0]["energy"] + res[1]["energy"], uJ

    th = 0.7
    E, uJ = energy(th)
    c = MU0 / (4 * math.pi * r ** 3)
    E_ref = -c * mu * mu * (3 * (uI @ e) * (uJ @ e) - uI @ uJ)
    assert abs(E / E_ref - 1) < 1e-10, (E, E_ref)
    h = 1e-5
    dE = (energy(th + h)[0] - energy(th - h)[0]) / (2 * h)
    BJ = c * mu * (3 * (uI @ e) * e - uI)
    duJ = np.array([math.cos(th), 0.0, -math.sin(th)])
    assert abs(dE / (-mu * duJ @ BJ) - 1) < 1e-6


# ------------------------------------------------------------------------------------------
# exchange-coupled composite switching
# ------------------------------------------------------------------------------------------

def _sw_h(psi):
    return (math.cos(psi) ** (2 / 3) + math.sin(psi) ** (2 / 3)) ** -1.5


def _two_spin_switch(Ms, K, t, J, psi, B_max, nB=5000):
    """Field at which the hard spin of the up state of two rigid layers (energy per area
    -K_s t_s cos^2 th_s - K_h t_h cos^2 th_h - J cos(th_s - th_h) - B sum Ms t cos(th - phi_B),
    field at phi_B = pi - psi from +z) first leaves the upper hemisphere, following the local
    minimum from B = 0 upward."""
    phB = math.pi - psi

    def E(x, B):
        a, b = x
        return (-K[0] * t[0] * math.cos(a) ** 2 - K[1] * t[1] * math.cos(b) ** 2 - J * math.cos(a - b)
                - B * (Ms[0] * t[0] * math.cos(a - phB) + Ms[1] * t[1] * math.cos(b - phB)))

    def G(x, B):
        a, b = x
        return np.array([K[0] * t[0] * math.sin(2 * a) + J * math.sin(a - b) + B * Ms[0] * t[0] * math.sin(a - phB),
                         K[1] * t[1] * math.sin(2 * b) - J * math.sin(a - b) + B * Ms[1] * t[1] * math.sin(b - phB)])

    x = np.array([1e-6, 1e-6])
    for B in np.linspace(0.0, B_max, nB):
        x = minimize(E, x, args=(B,), jac=G, method="BFGS", options=dict(gtol=1e-14)).x
        if math.cos(x[1]) < 0:
            return B
    return None


ECC_MS, ECC_K = (1.0e6, 0.6e6), (0.2e6, 1.2e6)     # the single-island layers: soft, hard
ECC_T = (1.5e-9, 3.5e-9)                            # the single-island thickness ratio 3 : 7


def test_two_spin_model_limits():
    psi = math.radians(30)
    # J = 0: the hard layer at its own Stoner-Wohlfarth field 2 K_h / Ms_h h(psi) = 2.0961 T
    assert abs(_two_spin_switch(ECC_MS, ECC_K, ECC_T, 0.0, psi, 2.5) / (2 * 1.2e6 / 0.6e6 * _sw_h(psi)) - 1) < 1e-3
    # J -> infinity: the averaged anisotropy, 2.5 T * 0.52402 = 1.3100 T
    avg = 2 * (ECC_K[0] * ECC_T[0] + ECC_K[1] * ECC_T[1]) / (ECC_MS[0] * ECC_T[0] + ECC_MS[1] * ECC_T[1])
    assert abs(avg - 2.5) < 1e-12
    assert abs(_two_spin_switch(ECC_MS, ECC_K, ECC_T, 100.0, psi, 2.0) / (avg * _sw_h(psi)) - 1) < 1e-3
    assert abs(avg * _sw_h(psi) - 1.3100) < 1e-4


@pytest.mark.parametrize("J", [0.0, 3e-3, 0.1])
def test_ecc_switching_against_two_spin_model(oracle_mod, J):
    """Two-layer island with the single-island layers (3 : 7 thickness), exchange stiff enough to
    keep each layer uniform, no demag, alpha = 1, static field at 30 degrees from -z: the hard
    layer stays up at 0.99 of the two-spin switching field and reverses at 1.01 of it.  J = 0:
    the soft layer reverses alone at its own field (0.4 T * 0.52402 = 0.2096 T); J = 0.1 J/m^2
    (40 times K_h t_h) is within 0.2 % of the rigid limit 1.3100 T."""
    psi = math.radians(30)
    mesh = I.island_mesh(2e-9, 2e-9, ECC_T[0], ECC_T[1], 2e-9, seed=0)
    om = oracle_mod.OracleMesh(mesh)
    A = 2e-9 if J > 0.05 else 300e-12
    ref = _two_spin_switch(ECC_MS, ECC_K, ECC_T, J, psi, 2.5)
    if J == 0.1:
        assert abs(ref / 1.3100 - 1) < 2.5e-3
    out = []
    for fac in (0.99, 1.01):
        mat = I.Material(Ms=ECC_MS, K=ECC_K, A=(A, A), A_int=J * 1e-9, delta_int=1e-9, alpha=1.0)
        fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=fac * ref, dir=(math.sin(psi), 0.0, -math.cos(psi)), t_rise=0.0)
        _, res, _ = om.run(None, [mat], [fld], dict(t_end=0.25e-9, rtol=1e-6))
        out.append((res[0]["mz_soft"], res[0]["mz_hard"]))
    assert out[0][1] > 0.5 and out[1][1] < -0.5, (ref, out)
    if J == 0.0:
        Bs = 2 * ECC_K[0] / ECC_MS[0] * _sw_h(psi)
        soft = []
        for fac in (0.99, 1.01):
            mat = I.Material(Ms=ECC_MS, K=ECC_K, A=(A, A), A_int=0.0, alpha=1.0)
            fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=fac * Bs, dir=(math.sin(psi), 0.0, -math.cos(psi)), t_rise=0.0)
            # the soft layer's anisotropy field is only 0.4 T: its reversal takes longer
            _, res, _ = om.run(None, [mat], [fld], dict(t_end=1e-9, rtol=1e-6))
            soft.append((res[0]["mz_soft"], res[0]["mz_hard"]))
        assert soft[0][0] > 0.5 and soft[1][0] < -0.5 and soft[1][1] > 0.9, soft


@pytest.mark.parametrize("psi_deg", [5.0, 10.0, 20.0, 30.0, 45.0])
def test_stoner_wohlfarth_astroid_one_percent(oracle_mod, psi_deg):
    """Uniform macrospin island (one material in both layers, no demag): a static field 1 % below
    the Stoner-Wohlfarth field leaves it up, 1 % above reverses it."""
    psi = math.radians(psi_deg)
    Ms, K = 0.8e6, 0.5e6
    BK = 2 * K / Ms
    mesh = I.island_mesh(2e-9, 2e-9, 1e-9, 1e-9, 1.0e-9, seed=0)
    om = oracle_mod.OracleMesh(mesh)
    mat = I.Material(Ms=(Ms, Ms), K=(K, K), A_int=10e-12, alpha=1.0)
    out = []
    for fac in (0.99, 1.01):
        B = fac * _sw_h(psi) * BK
        fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=B, dir=(math.sin(psi), 0.0, -math.cos(psi)), t_rise=0.0)
        m, res, _ = om.run(None, [mat], [fld], dict(t_end=0.5e-9, rtol=1e-7))
        out.append(res[0]["mz_hard"])
    assert out[0] > 0.0 and out[1] < 0.0, out
