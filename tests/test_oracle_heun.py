"""Pins of the oracle's stochastic Heun integrator (no GPU).

* T = 0: the scheme is deterministic Heun, second order on the macrospin closed form.
* Free rotational diffusion (no exchange, anisotropy, field or demag; each node is then an
  independent macrospin of moment w_i = Ms V_i): <m_z>(t) = exp(-2 D_i t) and
  <m_z^2>(t) = 1/3 + 2/3 exp(-6 D_i t) with Brown's D_i = alpha gamma kB T / ((1 + alpha^2) w_i).
  This fixes the variance of the thermal field (a wrong factor changes D).
* Equilibrium in a uniaxial well: <m_z^2> = e^s / (s Z) - 1 / (2 s), Z = int_-1^1 e^{s x^2} dx,
  s = K V_i / kB T (Boltzmann distribution of a macrospin).
"""
import math

import numpy as np
from scipy.integrate import quad

from paper_1603_09493_amd import inputs as I

GAMMA = 1.76085963023e11
KB = 1.380649e-23


def _free_mesh():
    return I.island_mesh(4e-9, 4e-9, 2e-9, 3e-9, 1.0e-9, seed=2)


def test_heun_zero_temperature_is_second_order(oracle_mod):
    O = oracle_mod
    mesh = I.island_mesh(2e-9, 2e-9, 1e-9, 1e-9, 1.0e-9, seed=0)
    om = O.OracleMesh(mesh)
    alpha, B, th0, T = 0.2, 2.0, 2.0, 20e-12
    mat = I.Material(K=(0.0, 0.0), A=(0.0, 0.0), A_int=0.0, alpha=alpha)
    fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=B, dir=(0.0, 0.0, 1.0), t_rise=0.0)
    m0 = np.zeros((3, om.n)); m0[0] = math.sin(th0); m0[2] = math.cos(th0)
    gp = GAMMA / (1 + alpha ** 2)
    th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-alpha * gp * B * T))
    ex = np.array([math.sin(th) * math.cos(gp * B * T), math.sin(th) * math.sin(gp * B * T), math.cos(th)])
    errs = []
    for dt in (2e-14, 1e-14, 5e-15):
        m, res, _ = om.run(None, [mat], [fld], dict(t_end=T, integrator=O.HEUN, dt_fixed=dt, temperature=0.0),
                           m0=m0, seeds=[1])
        errs.append(np.abs(m[0, :, 0] - ex).max())
    o1, o2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert 1.7 < o1 < 2.5 and 1.7 < o2 < 2.5, (errs, o1, o2)


def test_free_rotational_diffusion(oracle_mod):
    O = oracle_mod
    mesh = _free_mesh()
    om = O.OracleMesh(mesh)
    V = om.export()["V"]
    Ms, alpha, Temp = 1.0e6, 0.5, 300.0
    mat = I.Material(Ms=(Ms, Ms), K=(0.0, 0.0), A=(0.0, 0.0), A_int=0.0, alpha=alpha)
    fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=0.0, t_rise=0.0)
    R = 8
    t = 1.0e-12
    m, res, _ = om.run(None, [mat] * R, [fld] * R, dict(t_end=t, integrator=O.HEUN, dt_fixed=1e-15,
                                                        temperature=Temp), seeds=np.arange(R) + 11)
    D = alpha * GAMMA * KB * Temp / ((1 + alpha ** 2) * Ms * V)
    mz = m[:, 2, :]                         # [R][n]
    e1 = np.exp(-2 * D * t)
    e2 = 1 / 3 + 2 / 3 * np.exp(-6 * D * t)
    # centred and scaled residuals over every (realization, node)
    var1 = e2 - e1 ** 2
    z1 = ((mz - e1) / np.sqrt(var1)).mean() * math.sqrt(mz.size)
    assert abs(z1) < 4.0, z1
    assert abs(((mz ** 2) - e2).mean()) < 0.02
    # the rate is in the regime where both moments moved substantially
    assert 0.2 < e1.mean() < 0.9


def _mz2_boltzmann(s):
    Z = quad(lambda x: math.exp(s * x * x), -1, 1)[0]
    return math.exp(s) / (s * Z) - 1 / (2 * s)


def test_equilibrium_in_uniaxial_well(oracle_mod):
    O = oracle_mod
    mesh = _free_mesh()
    om = O.OracleMesh(mesh)
    V = om.export()["V"]
    Ms, K, alpha, Temp = 1.0e6, 2.0e7, 1.0, 300.0
    mat = I.Material(Ms=(Ms, Ms), K=(K, K), A=(0.0, 0.0), A_int=0.0, alpha=alpha)
    fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=0.0, t_rise=0.0)
    R = 4
    m, res, _ = om.run(None, [mat] * R, [fld] * R, dict(t_end=60e-12, integrator=O.HEUN, dt_fixed=2e-15,
                                                        temperature=Temp), seeds=np.arange(R) + 21)
    s = K * V / (KB * Temp)
    ref = np.array([_mz2_boltzmann(x) for x in s])
    mz2 = (m[:, 2, :] ** 2)
    assert abs((mz2 - ref[None, :]).mean()) < 0.02, ((mz2 - ref).mean(), ref.mean())
    # anisotropy pushes the moments toward the axis compared with the isotropic 1/3
    assert mz2.mean() > 0.5
