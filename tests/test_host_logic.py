"""Host-side logic of the learned screen (no GPU): the design prior and the network-input scaling."""
import numpy as np

from paper_1603_09493_amd import inputs as I
from paper_1603_09493_amd import surrogate as SG


def test_design_scaling_round_trip_and_bounds():
    x = SG.sample(2000, seed=3)
    assert np.all(x >= I.DESIGN_LO * (1 - 1e-12)) and np.all(x <= I.DESIGN_HI * (1 + 1e-12))
    X = SG.scale(x)
    assert np.all(np.abs(X) <= 1.0 + 1e-12)
    np.testing.assert_allclose(SG.unscale(X), x, rtol=1e-12, atol=0)
    # the corners map to -1 and +1
    np.testing.assert_allclose(SG.scale(I.DESIGN_LO[None]), -1.0, atol=1e-12)
    np.testing.assert_allclose(SG.scale(I.DESIGN_HI[None]), 1.0, atol=1e-12)


def test_prior_is_uniform_and_inputs_are_log_coordinates():
    """The surrogate's designs are uniform in the box (arithmetic midpoints are the medians);
    the network input of a parameter with a positive lower bound is its log coordinate (the
    geometric midpoint maps to 0), psi's is linear."""
    x = SG.sample(200_000, seed=5)
    med = np.median(x, axis=0)
    mid = 0.5 * (I.DESIGN_LO + I.DESIGN_HI)
    for f in range(12):
        assert abs(med[f] / mid[f] - 1) < 0.01, (I.DESIGN_NAMES[f], med[f], mid[f])
    geo = np.where(I.DESIGN_LOG, np.sqrt(np.abs(I.DESIGN_LO * I.DESIGN_HI)), mid)
    np.testing.assert_allclose(SG.scale(geo[None])[0], 0.0, atol=1e-12)
    assert not I.DESIGN_LOG[I.DESIGN_NAMES.index("psi")]


def test_linear_prior_unchanged_for_the_batched_workload():
    x = I.sample_designs(1000, seed=2)
    rng = np.random.default_rng(2)
    u = rng.random((1000, 12))
    ref = I.DESIGN_LO + (I.DESIGN_HI - I.DESIGN_LO) * u
    ref[:, 10] = 0.1
    ref[:, 11] = 0.1e-9
    np.testing.assert_array_equal(x, ref)


def _spread(mesh):
    out = np.zeros(mesh.n, int)
    for e in mesh.tet:
        out[e] = np.maximum(out[e], np.abs(e[:, None] - e[None, :]).max(axis=1))
    return out


def test_mesher_renumbering_is_a_relabelling_with_smaller_spread():
    """The reverse Cuthill-McKee renumbering is a relabelling of the level-major mesh (same node
    coordinates and layers, same tets and interface pairs up to the permutation, still positively
    oriented) and shrinks the index spread of every node's neighbours."""
    args = (9e-9, 2.25e-9, 3e-9, 7e-9, 1.0e-9)
    m0 = I.island_mesh(*args, seed=1, renumber=False)
    m1 = I.island_mesh(*args, seed=1)
    n = m0.n
    assert m1.n == n and m1.tet.shape == m0.tet.shape
    # the permutation: match nodes by (coordinates, layer) -- interface copies differ in layer
    def key(m):
        return [tuple(np.round(m.xyz[:, i] * 1e12).astype(np.int64)) + (int(m.layer[i]),) for i in range(m.n)]
    k0, k1 = key(m0), key(m1)
    pos1 = {k: i for i, k in enumerate(k1)}
    assert len(pos1) == n
    perm = np.array([pos1[k] for k in k0])          # old index -> new index
    assert np.array_equal(np.sort(perm), np.arange(n))
    np.testing.assert_array_equal(perm[m0.tet], m1.tet)
    np.testing.assert_array_equal(perm[m0.iface], m1.iface)
    P = m1.xyz.T
    t = m1.tet
    det = np.einsum("ij,ij->i", P[t[:, 1]] - P[t[:, 0]], np.cross(P[t[:, 2]] - P[t[:, 0]], P[t[:, 3]] - P[t[:, 0]]))
    assert np.all(det > 0)
    s0, s1 = _spread(m0), _spread(m1)
    assert s1.max() < 0.8 * s0.max() and s1.mean() < 0.8 * s0.mean(), (s0.max(), s1.max(), s0.mean(), s1.mean())


def test_erasure_label_and_count():
    import math
    from paper_1603_09493_amd import thermal
    assert abs(thermal.logit_label(0, 1024) - math.log(0.5 / 1024.5)) < 1e-12
    assert abs(thermal.logit_label(1024, 1024) + thermal.logit_label(0, 1024)) < 1e-12
    assert abs(thermal.logit_label(512, 1024)) < 1e-12
    res = [dict(status=0, mz_hard=-0.2), dict(status=0, mz_hard=0.9), dict(status=-5, mz_hard=-1.0)]
    assert thermal.count_erased(res) == (1, 2)
