"""Pins of the oracle's string-method energy barrier and of Eq. (3) (no GPU).

* Macrospin limit: a small island with strong exchange and interlayer coupling, equal K and Ms
  in both layers and no demag turns coherently; in a field B along -z its barrier out of +z is
  K V (1 - h)^2 with h = Ms B / (2 K) (Stoner-Wohlfarth on the easy axis).
* Decoupled layers (A_int = 0): the soft and the hard layer reverse one after the other, so the
  path passes two saddles; E_B = max(K_s V_s (1 - h_s)^2, -2 Ms_s V_s B + K_h V_h (1 - h_h)^2).
* The redistribution puts images at equal arc length and leaves an evenly spaced chain alone;
  the parabola refinement is exact for a parabola.
* Table III: BER_tot is the sum of the three rates, and Eq. (3) inverts to a barrier in kT.
"""
import math

import numpy as np
import pytest

from oracle import barrier as OBar
from paper_1603_09493_amd import inputs as I

MU0 = 4e-7 * math.pi


@pytest.fixture(scope="module")
def small_island(oracle_mod):
    mesh = I.island_mesh(2e-9, 2e-9, 2e-9, 2e-9, 1.0e-9, seed=3)
    om = oracle_mod.OracleMesh(mesh)
    V = om.export()["V"]
    vol = {L: float(V[mesh.layer == L].sum()) for L in (0, 1)}
    return mesh, om, vol


def _mat(K, Ms, A_int, A=1e-10):
    return I.Material(Ms=(Ms, Ms), K=(K[0], K[1]), A=(A, A), A_int=A_int, alpha=1.0)


@pytest.mark.parametrize("h", [0.0, 0.25, 0.5])
def test_macrospin_barrier_closed_form(small_island, h):
    mesh, om, vol = small_island
    K, Ms = 0.5e6, 0.5e6
    B = h * 2 * K / Ms
    mat = _mat((K, K), Ms, A_int=1e-10)
    fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=B, dir=(0.0, 0.0, -1.0), t_rise=0.0)
    r = OBar.string_barrier(om, None, mat, fld, OBar.rotation_chain(mesh.n, 13), dtau=1e-12, iters=8)
    ref = K * (vol[0] + vol[1]) * (1 - h) ** 2
    assert abs(r["E_B"] / ref - 1) < 2e-3, (r["E_B"], ref)


def test_decoupled_layers_pass_two_saddles(small_island):
    mesh, om, vol = small_island
    Ks, Kh, Ms, B = 0.2e6, 0.8e6, 0.5e6, 0.3
    mat = _mat((Ks, Kh), Ms, A_int=0.0)
    fld = I.Field(kind=I.FIELD_UNIFORM, B_peak=B, dir=(0.0, 0.0, -1.0), t_rise=0.0)
    r = OBar.string_barrier(om, None, mat, fld, OBar.rotation_chain(mesh.n, 21), dtau=2e-12, iters=80)
    hs, hh = Ms * B / (2 * Ks), Ms * B / (2 * Kh)
    e1 = Ks * vol[0] * (1 - hs) ** 2
    e2 = -2 * Ms * vol[0] * B + Kh * vol[1] * (1 - hh) ** 2
    ref = max(e1, e2)
    # the coherent chain it started from is higher: the string really moved
    coherent = (Ks * vol[0] + Kh * vol[1]) * (1 - Ms * B * (vol[0] + vol[1]) / (2 * (Ks * vol[0] + Kh * vol[1]))) ** 2
    assert coherent > 1.2 * ref
    assert abs(r["E_B"] / ref - 1) < 0.02, (r["E_B"], ref, e1, e2)
    # the soft layer reverses first along the path: the middle image has soft down, hard up
    mid = r["images"][len(r["images"]) // 2]
    assert mid[2][mesh.layer == 0].mean() < -0.5 and mid[2][mesh.layer == 1].mean() > 0.5


def test_redistribution():
    n, P = 5, 9
    th = np.array([0.0, 0.05, 0.1, 0.2, 1.0, 1.5, 2.0, 3.0, math.pi])
    chain = np.zeros((P, 3, n))
    chain[:, 0, :] = np.sin(th)[:, None]
    chain[:, 2, :] = np.cos(th)[:, None]
    out, s = OBar.redistribute(chain)
    assert np.array_equal(out[0], chain[0]) and np.array_equal(out[-1], chain[-1])
    assert abs(s[-1] - sum(np.sqrt(n) * 2 * np.sin(np.diff(th) / 2))) < 1e-12
    # the new images sit at equal arc length along the old polyline: their angles follow from
    # inverting the piecewise-linear arc length of the chord polyline, checked here by brute force
    seg = np.sqrt(n) * 2 * np.sin(np.diff(th) / 2)
    cum = np.concatenate([[0], np.cumsum(seg)])
    for j in range(1, P - 1):
        t = cum[-1] * j / (P - 1)
        k = np.searchsorted(cum, t) - 1
        w = (t - cum[k]) / seg[k]
        p = (1 - w) * np.array([np.sin(th[k]), np.cos(th[k])]) + w * np.array([np.sin(th[k + 1]), np.cos(th[k + 1])])
        p /= np.linalg.norm(p)
        assert np.allclose(out[j][[0, 2], 0], p, atol=1e-14)
    # an evenly spaced chain stays
    even = OBar.rotation_chain(n, P)
    out2, _ = OBar.redistribute(even)
    assert np.abs(out2 - even).max() < 1e-12


def test_parabola_refinement_is_exact_on_a_parabola():
    s = np.array([0.0, 0.7, 1.1, 2.0, 2.6, 3.3])
    E = -3.0 * (s - 1.37) ** 2 + 5.0
    assert abs(OBar.barrier_of_profile(s, E) - (5.0 - E[0])) < 1e-12
    # monotone profile: the barrier is at the end image, no refinement
    assert OBar.barrier_of_profile(s, s) == pytest.approx(3.3)


def test_table_iii_rates():
    rows = [(1.3e-2, 5.9e-3, 3.8e-3, 3.4e-3), (2.9e-3, 2.8e-3, 3.2e-5, 3.6e-6),
            (2.1e-2, 2.1e-3, 1.9e-2, 5.3e-17), (1.8e-2, 8.9e-3, 8.9e-3, 2.8e-18),
            (8.4e-8, 4.2e-8, 4.2e-8, 3.2e-15), (1.5e-8, 9.9e-10, 9.9e-10, 1.3e-8)]
    for tot, a, b, c in rows:
        assert abs((a + b + c) / tot - 1) < 0.05    # the table rounds to two digits
    # Eq. (3) round trip: the barrier in the head field behind BER_adj = 3.4e-3 is 10.55 kT
    kT = OBar.KB * 300.0
    eb = kT * math.log(OBar.T_WRITE * OBar.F0 / 3.4e-3)
    assert abs(eb / kT - 10.5515) < 1e-3
    assert abs(OBar.ber_adj(eb) / 3.4e-3 - 1) < 1e-12
    # the zero-field barriers of Table III give rates far below any write error
    assert OBar.ber_adj(110 * kT) < 1e-45
