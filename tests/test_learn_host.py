"""Host-side logic of the learned warm start (CPU): parameter packing sizes,
initialization, the system map handed to the feature kernel, the race
length rule."""
import numpy as np

from oracle import learn as OL
from paper_1810_03358_amd import learn as L
from synth import chain_system


def test_parameter_vector_matches_the_oracle_packing():
    assert L.param_count() == OL.PARAM_COUNT == 35088
    theta = L.init_params(seed=3)
    assert theta.dtype == np.float32 and theta.size == OL.PARAM_COUNT
    p = OL.unpack(theta.astype(np.float64))
    assert np.all(p["b1"] == 0) and np.all(p["b2"] == 0) and np.all(p["b3"] == 0)
    # He-normal hidden layers, a small output layer
    assert 0.8 < p["W1"].std() / np.sqrt(2.0 / 128) < 1.2
    assert p["W3"].std() < 0.01
    np.testing.assert_array_equal(theta, L.init_params(seed=3))


def test_system_map_for_the_feature_kernel():
    systems = [chain_system(5, 1), chain_system(3, 2), chain_system(7, 3)]
    sa = L.SystemArrays(systems, device="cpu")
    assert sa.n == 15 and sa.n_sys == 3
    assert sa.sys_first.tolist() == [0, 5, 8, 15]
    assert sa.atom_sys.tolist() == [0] * 5 + [1] * 3 + [2] * 7
    np.testing.assert_array_equal(sa.q.numpy(), np.concatenate([s["q"] for s in systems]))


def test_race_length_grows_with_the_system():
    assert L.race_length(300) == 200
    assert L.race_length(2000) == 200
    assert L.race_length(5000) == 500
    assert L.race_length(10_000) == 1000
    assert L.race_length(50_000) == 1000
