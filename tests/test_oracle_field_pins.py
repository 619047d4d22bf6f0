"""Pins of the oracle's gridded head field (no GPU).

The paper samples the precomputed head field on a grid and moves it over the bit with a rise
(Sec. II.A).  Trilinear interpolation reproduces any affine field exactly, so a grid sampled
from B(s) = B0 + G s must give back that field at every node inside the grid (to the FP32
rounding of the stored node values), in the moving frame s = x - x_off - v t and scaled by the
rise; outside the grid only B_ext acts.  The synthetic pole sampled at 2.5 nm must stay within the
trilinear error bound (h^2 / 8) max|f''| of the analytic pole.
"""
import math

import numpy as np

from paper_1603_09493_amd import inputs as I


def _zeeman(om, fld, t, off=(0.0, 0.0, 0.0)):
    mat = I.Material(K=(0.0, 0.0), A=(0.0, 0.0), A_int=0.0)
    m = np.zeros((3, om.n)); m[2] = 1.0
    _, terms, _ = om.fields(None, mat, fld, m, t=t, offset=off)
    return terms[4]


def test_grid_reproduces_affine_field(oracle_mod):
    mesh = I.island_mesh(4e-9, 4e-9, 3e-9, 4e-9, 1.0e-9, seed=6)
    om = oracle_mod.OracleMesh(mesh)
    B0 = np.array([0.1, -0.2, -0.9])
    G = np.array([[2e7, -1e7, 3e6], [5e6, 1.5e7, -2e7], [-3e7, 1e7, 2.5e7]])     # T/m
    lo, h, n = np.array([-30e-9, -20e-9, -10e-9]), 2.5e-9, (25, 17, 11)          # nx, ny, nz
    xs = [lo[d] + h * np.arange(n[d]) for d in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    grid = np.stack([B0[c] + G[c, 0] * X + G[c, 1] * Y + G[c, 2] * Z for c in range(3)]).astype(np.float32)
    v, x_off, t, t_rise, B_ext = np.array([-13.5, 2.0, 0.0]), np.array([1e-9, -2e-9, 0.5e-9]), 0.2e-9, 0.25e-9, (0.01, 0.0, -0.02)
    fld = I.Field(kind=I.FIELD_GRID, B_peak=1.3, t_rise=t_rise, v=tuple(v), x_off=tuple(x_off), B_ext=B_ext,
                  grid=grid, g_origin=tuple(lo), g_h=h)
    off = (1.5e-9, -0.5e-9, 0.0)
    Bz = _zeeman(om, fld, t, off)
    P = mesh.xyz.T + np.asarray(off)
    s = P - x_off - v * t
    assert np.all(s > lo) and np.all(s < lo + h * (np.array(n) - 1))     # inside the grid
    ref = (1.3 * min(t / t_rise, 1.0)) * (B0[None, :] + s @ G.T) + np.asarray(B_ext)
    scale = np.abs(grid).max() * 1.3
    assert np.abs(Bz.T - ref).max() <= 2e-7 * scale, np.abs(Bz.T - ref).max() / scale


def test_grid_is_zero_outside(oracle_mod):
    mesh = I.island_mesh(3e-9, 3e-9, 2e-9, 2e-9, 1.0e-9, seed=7)
    om = oracle_mod.OracleMesh(mesh)
    grid = np.ones((3, 4, 4, 4), dtype=np.float32)
    B_ext = (0.0, 0.05, -0.1)
    # the grid lies entirely beyond the island in x
    fld = I.Field(kind=I.FIELD_GRID, B_peak=1.0, t_rise=0.0, B_ext=B_ext, grid=grid, g_origin=(20e-9, 0, 0), g_h=1e-9)
    Bz = _zeeman(om, fld, 0.0)
    assert np.array_equal(Bz.T, np.broadcast_to(np.asarray(B_ext), (om.n, 3)))


def test_sampled_pole_matches_analytic_pole(oracle_mod):
    mesh = I.island_mesh(6e-9, 6e-9, 3e-9, 7e-9, 1.2e-9, seed=8)
    om = oracle_mod.OracleMesh(mesh)
    psi = math.radians(20)
    d = (math.sin(psi), 0.0, -math.cos(psi))
    L, W, Bp = 10e-9, 13e-9, 1.5
    pole = I.Field(kind=I.FIELD_POLE, B_peak=Bp, dir=d, t_rise=0.0, x_off=(-3e-9, 1e-9, 0), L_grad=L, W_pole=W)
    g, org, h = I.pole_field_grid(Bp, d, L, W, lo=(-40e-9, -30e-9, -5e-9), hi=(40e-9, 30e-9, 15e-9), h=2.5e-9)
    gridf = I.Field(kind=I.FIELD_GRID, B_peak=1.0, t_rise=0.0, x_off=(-3e-9, 1e-9, 0), grid=g, g_origin=org, g_h=h)
    a, b = _zeeman(om, pole, 0.0), _zeeman(om, gridf, 0.0)
    # trilinear error <= h^2/8 * (|f_xx| + |f_yy|) with |f''| <= 0.77 / L^2 per tanh factor
    bound = Bp * (2.5e-9) ** 2 / 8 * 2 * 0.77 / L ** 2
    assert np.abs(a - b).max() <= bound + 1e-6, (np.abs(a - b).max(), bound)
    assert np.abs(a - b).max() > 0.0
