"""Host logic of the write-error driver (no GPU): the H_crit search of Sec. II.C, its early
abort, the H_ext direction and the sequencing of BER_targ / BER_prev, run against a stand-in
context whose islands switch exactly when the net field along the head direction exceeds a
threshold."""
import math

import numpy as np
import pytest

from oracle import ber as OB
from paper_1603_09493_amd import ber_driver as D
from paper_1603_09493_amd import inputs as I


class ThresholdCtx:
    """Switches an instance iff (head strength at its offset) + H_ext . hdir exceeds hsw,
    with the H_ext sign convention of the driver (target: against, previous: along)."""

    def __init__(self, strength):
        self.strength = strength          # offset tuple -> head strength (tesla)
        self.hsw = 1.0
        self.calls = []
        self.clear_instances()

    def clear_instances(self):
        self.inst = []

    def mesh_add(self, mesh, keep=3):
        self.meshes = getattr(self, "meshes", 0) + 1
        return self.meshes - 1

    def instance_add(self, mid, mat, fld, offset=None):
        self.inst.append((fld, tuple(offset)))
        return len(self.inst) - 1

    def run(self, **kw):
        self.calls.append(len(self.inst))

    def sync(self):
        pass

    def results(self, ids):
        out = []
        for i in ids:
            fld, off = self.inst[i]
            d = D.head_direction(fld, off, 1e-9)
            h = float(np.dot(np.asarray(fld.B_ext), d))
            out.append({"status": 0, "switched": int(self.strength[off] + h > self.hsw)})
        return out


MAT = I.media_material(K_hard=0.8e6)
SIG = D.sigma_T(MAT.K[1], MAT.Ms[1])
FLD = I.Field(kind=I.FIELD_UNIFORM, B_peak=1.0, dir=(0.6, 0.0, -0.8))


@pytest.mark.parametrize("margin_sig", [0.3, 2.26, 5.49, 9.7, 17.0])
def test_target_bracket_contains_threshold(margin_sig):
    # the target switches while H_ext < hc = strength - hsw
    ctx = ThresholdCtx({(0.0, 0.0, 0.0): 1.0 + margin_sig * SIG})
    r = D.critical_field(ctx, 0, MAT, FLD, t_end=1e-9)
    hc = margin_sig * SIG
    assert not r.aborted
    assert r.lo < hc <= r.hi + 1e-15
    # two refinements of a sigma/2 grid by 13 leave a bracket of sigma/2/169
    assert r.hi - r.lo <= 0.5 * SIG / 13 ** 2 * (1 + 1e-9)
    assert abs(r.ber - OB.ber_crit(r.h_crit, OB.sigma_T(MAT.K[1], 4e-7 * math.pi * MAT.Ms[1]))) < 1e-15
    assert all(n == 12 for n in ctx.calls)


def test_target_abort_when_head_cannot_write():
    ctx = ThresholdCtx({(0.0, 0.0, 0.0): 0.9})
    r = D.critical_field(ctx, 0, MAT, FLD)
    assert r.aborted and r.ber == 1.0 and len(ctx.calls) == 1


def test_previous_bracket_and_abort():
    # previous bit: switches (an error) once strength + H_ext > hsw, H_ext along the head field
    ctx = ThresholdCtx({(-1.0, 0.0, 0.0): 1.0 - 3.3 * SIG})
    r = D.critical_field(ctx, 0, MAT, FLD, previous=True, offset=(-1.0, 0.0, 0.0))
    assert not r.aborted and r.lo < 3.3 * SIG <= r.hi
    ctx = ThresholdCtx({(-1.0, 0.0, 0.0): 1.2})
    r = D.critical_field(ctx, 0, MAT, FLD, previous=True, offset=(-1.0, 0.0, 0.0))
    assert r.aborted and r.ber == 1.0


def test_write_errors_sequencing():
    lay = {"target": (0.0, 0.0, 0.0), "previous": (-1.0, 0.0, 0.0), "adjacent": (0.5, 1.0, 0.0)}
    mesh = I.media_mesh(n_target=300)
    adj_calls = []

    def adj():
        adj_calls.append(1)
        return 1e-9

    # target cannot be written: abort before the previous bit and BER_adj
    ctx = ThresholdCtx({(0.0, 0.0, 0.0): 0.5, (-1.0, 0.0, 0.0): 0.0})
    w = D.write_errors(ctx, mesh, 0, MAT, FLD, layout=lay, ber_adj=adj)
    assert (w.stage, w.ber_tot, w.prev) == ("targ", 1.0, None) and not adj_calls
    # previous bit always rewritten: abort before BER_adj
    ctx = ThresholdCtx({(0.0, 0.0, 0.0): 1.0 + 4 * SIG, (-1.0, 0.0, 0.0): 1.5})
    w = D.write_errors(ctx, mesh, 0, MAT, FLD, layout=lay, ber_adj=adj)
    assert (w.stage, w.ber_tot) == ("prev", 1.0) and not adj_calls
    # both pass: BER_tot = targ + prev + adj
    ctx = ThresholdCtx({(0.0, 0.0, 0.0): 1.0 + 4 * SIG, (-1.0, 0.0, 0.0): 1.0 - 6 * SIG})
    w = D.write_errors(ctx, mesh, 0, MAT, FLD, layout=lay, ber_adj=adj)
    assert w.stage == "done" and adj_calls == [1]
    assert w.ber_tot == pytest.approx(w.ber_targ + w.ber_prev + 1e-9, rel=1e-12)
    assert 1e-6 < w.ber_targ < 1e-3 and w.ber_prev < 1e-8


def test_head_direction_of_a_gridded_field():
    g, org, h = I.default_head_grid()
    fld = I.recording_field(g, org, h)
    d = D.head_direction(fld, (0.0, 0.0, 5e-9), I.BIT_PERIOD)
    psi = math.radians(25.0)
    assert np.allclose(d, [math.sin(psi), 0.0, -math.cos(psi)], atol=1e-6)
    # a grid with a field that turns in space: the direction follows the strongest sample
    g2 = np.zeros((3, 2, 2, 2), dtype=np.float32)
    g2[0, :, :, 0] = 1.0          # +x at the low-x face
    g2[2, :, :, 1] = -3.0         # -z at the high-x face
    f2 = I.Field(kind=I.FIELD_GRID, B_peak=1.0, t_rise=0.0, grid=g2, g_origin=(0, 0, 0), g_h=1e-9,
                 v=(1.0, 0.0, 0.0), x_off=(-1e-9, 0.0, 0.0))
    # the island at x = 0: s_x runs from 1 nm down to 0 over [0, 1 ns]
    assert np.allclose(D.head_direction(f2, (0.0, 0.5e-9, 0.5e-9), 1e-9), [0.0, 0.0, -1.0])
    with pytest.raises(ValueError):
        D.head_direction(f2, (0.0, 5e-9, 0.5e-9), 1e-9)


def test_recording_layout_is_pseudo_hexagonal():
    lay = I.recording_layout()
    t, p, a = (np.asarray(lay[k]) for k in ("target", "previous", "adjacent"))
    assert np.allclose(t - p, [13.5e-9, 0, 0]) and np.allclose(a - t, [6.75e-9, 11.7e-9, 0])
    # areal density of the 13.5 x 11.7 nm cell: 4.08 Tb/in^2 (Sec. II.B)
    dens = 0.0254 ** 2 / (13.5e-9 * 11.7e-9) / 1e12
    assert abs(dens - 4.08) < 0.01
    # filling factor of 12 nm dots: 71.6 %
    ff = math.pi * 6e-9 ** 2 / (13.5e-9 * 11.7e-9)
    assert abs(ff - 0.716) < 0.001
    assert abs(I.BIT_PERIOD - 1e-9) < 1e-21


def test_media_island_layers():
    """The media island of Fig. 3: a 12 nm cylinder, 6 nm soft phase on top of a 5 nm hard phase,
    the two coupled across the 1 nm interlayer (not meshed): layer extents, the interface plane
    with one partner per interface node, and layer volumes in the ratio 6 : 5."""
    mesh = I.media_mesh(n_target=300)
    z, lay = mesh.xyz[2], mesh.layer
    r = np.hypot(mesh.xyz[0], mesh.xyz[1])
    assert r.max() <= 6e-9 * (1 + 1e-12) and r.max() > 5.9e-9
    assert np.isclose(z[lay == 1].min(), 0.0) and np.isclose(z[lay == 1].max(), 5e-9)
    assert np.isclose(z[lay == 0].min(), 5e-9) and np.isclose(z[lay == 0].max(), 11e-9)
    s, h = mesh.iface[:, 0], mesh.iface[:, 1]
    assert np.all(lay[s] == 0) and np.all(lay[h] == 1)
    assert np.allclose(mesh.xyz[:, s], mesh.xyz[:, h]) and np.allclose(z[s], 5e-9)
    assert len(np.unique(s)) == len(s) == len(np.unique(h))
    assert abs(I.media_material().delta_int - 1e-9) < 1e-21
    p = mesh.xyz[:, mesh.tet]                                # [3][ntet][4]
    vol = np.abs(np.einsum("ij,ij->j", np.cross(p[:, :, 1] - p[:, :, 0], p[:, :, 2] - p[:, :, 0], axis=0),
                           p[:, :, 3] - p[:, :, 0])) / 6.0
    soft = lay[mesh.tet].max(axis=1) == 0
    assert np.all(lay[mesh.tet][~soft] == 1)               # no tetrahedron straddles the interface
    assert abs(vol[soft].sum() / vol[~soft].sum() - 6.0 / 5.0) < 1e-9


def test_lock_step_searches_match_the_single_design_driver():
    """write_errors_many over designs whose head strengths differ gives, design by design, the
    result of write_errors, in as many launches as the longest single search needs."""
    lay = {"target": (0.0, 0.0, 0.0), "previous": (-1.0, 0.0, 0.0), "adjacent": (0.5, 1.0, 0.0)}
    mesh = I.media_mesh(n_target=300)
    strengths = [(1.0 + m * SIG, 1.0 - p * SIG) for m, p in ((0.3, 4.0), (-0.5, 3.0), (2.26, 12.0),
                                                             (4.1, -0.5), (9.7, 7.7), (17.0, 2.0), (1.1, 30.0))]
    singles = []
    for st, sp in strengths:
        ctx = ThresholdCtx({(0.0, 0.0, 0.0): st, (-1.0, 0.0, 0.0): sp})
        singles.append(D.write_errors(ctx, mesh, 0, MAT, FLD, layout=lay))

    class Multi(ThresholdCtx):
        """each design's field carries its own head strength in B_peak (uniform field)"""
        def results(self, ids):
            out = []
            for i in ids:
                fld, off = self.inst[i]
                d = D.head_direction(fld, off, 1e-9)
                h = float(np.dot(np.asarray(fld.B_ext), d))
                out.append({"status": 0, "switched": int(fld.B_peak[off == (0.0, 0.0, 0.0)] + h > self.hsw)})
            return out

    import dataclasses
    designs = [(MAT, dataclasses.replace(FLD, B_peak=(sp, st))) for st, sp in strengths]
    ctx = Multi({})
    many = D.write_errors_many(ctx, mesh, designs, layout=lay)
    for a, b in zip(singles, many):
        assert a.stage == b.stage and a.ber_tot == b.ber_tot and a.ber_targ == b.ber_targ
        if a.prev is not None:
            assert a.prev.lo == b.prev.lo and a.prev.hi == b.prev.hi
    longest = max(len(w.targ.levels) for w in singles) + max(len(w.prev.levels) for w in singles if w.prev)
    assert len(ctx.calls) == longest
    assert max(ctx.calls) == 12 * len(designs)


def test_barrier_profile_refinement():
    """The library driver's barrier from a chain profile: the parabola vertex is exact on a
    parabola, an end maximum is taken as is, and the barrier is measured from the first image."""
    from paper_1603_09493_amd import barrier as B
    s = np.array([0.0, 0.5, 1.2, 1.9, 2.4, 3.1])
    E = -2.0 * (s - 1.55) ** 2 + 7.0
    assert abs(B.profile_barrier(s, E) - (7.0 - E[0])) < 1e-12
    assert B.profile_barrier(s, -s) == 0.0
    assert B.profile_barrier(s, s) == pytest.approx(3.1)
    # Eq. (3): 130 GHz attempts during 1 ns, suppressed by the Boltzmann factor
    assert B.ber_adj(0.0) == pytest.approx(130.0)
    assert B.ber_adj(40 * 1.380649e-23 * 300) == pytest.approx(130.0 * math.exp(-40))
