"""Host-side pieces of the benchmark: the work count of the forward
projector must equal the oracle's sample count."""
import math

import pytest

import synth


@pytest.mark.parametrize("spec", [
    synth.config("cone3d_crop32").with_(n_proj=6),
    synth.config("cone3d_crop32").with_(vol_shape=(20, 26, 31), vol_spacing=(1.0, 0.7, 0.9), det_shape=(30, 40),
                                        n_proj=5, angular_range=200 * math.pi / 180, sid=200.0, sdd=350.0),
])
def test_sample_count_matches_oracle(ora, spec):
    import bench
    assert bench.count_samples(spec, "cpu") == ora.count_samples(spec)
