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
