"""The 2048-point weighting and filter, where one wave takes a pair of
detector rows, against the oracle. The cases are the ones its row pairing
and range-checked row loads must get right:
* an odd number of rows, so the last pair has no second row;
* a single row;
* fewer row pairs than the waves of one workgroup;
* more pairs than the persistent grid has waves, so every wave takes several;
* rows 2048 bins wide under a learned response, where every element a lane
  holds is live;
* ragged widths;
* both weight tables present;
* a batch of two;
* half-precision storage;
* the equiangular (arc) detector with a learned response."""
import numpy as np
import pytest
import torch

import gpu_common as gc
import synth
from gpu_common import FP32_TOL, as_f32, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ph():
    gc.device()
    import paper_1904_13342_amd as ph
    return ph


def _cone(n_proj, nv, nu):
    return synth.config("cone3d_crop32").with_(det_shape=(nv, nu), n_proj=n_proj)


# name: (spec, learned response and weights, batch)
CASES_3D = {
    "one_row_ramlak": (_cone(1, 1, 1024), False, 1),
    "odd_rows_ragged_ramlak": (_cone(3, 5, 1023), False, 1),
    "odd_rows_batch2_learned": (_cone(3, 5, 700), True, 2),
    "full_width_learned": (_cone(3, 3, 2048), True, 1),
    "more_pairs_than_waves": (_cone(11, 373, 520), False, 1),
}


@pytest.mark.parametrize("name", list(CASES_3D))
def test_filter_2048_cone(ph, ora, name):
    spec, learned, batch = CASES_3D[name]
    n_proj, (nv, nu) = spec.n_proj, spec.det_shape
    say(f"[filter2048] {name}: batch {batch}, {n_proj} x {nv} rows of {nu}")
    g = ph.from_spec(spec)
    p = as_f32(synth.random_array((batch, n_proj, nv, nu), 11, dist="uniform"))
    K = W_red = W = None
    if learned:
        K = as_f32(np.abs(synth.random_array((2048,), 12)))
        W_red = as_f32(synth.random_array((n_proj, nu), 13, dist="uniform", low=0.5, high=1.5))
        W = as_f32(synth.random_array((nv, nu), 14, dist="uniform", low=0.5, high=1.5))
        out = ph.weight_filter_3d(g, to_dev(p), K=to_dev(K), W_red=to_dev(W_red), W=to_dev(W))
    else:
        out = ph.weight_filter_3d(g, to_dev(p))
    out = to_np(out)
    for b in range(batch):
        q = ora.weight(spec, p[b], W_red=W_red, W=W)
        ref = ora.filter_projections(spec, q, K=K).reshape(n_proj, nv, nu)
        err = rel_l2(out[b], ref)
        say(f"  batch {b}: rel-L2 {err:.2e}")
        assert err < FP32_TOL


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_filter_2048_half_storage(ph, ora, dtype):
    """Half-precision projections are widened on load: the result matches the
    oracle run on the stored (rounded) values to the FP32 tolerance."""
    spec = _cone(5, 7, 1000)
    say(f"[filter2048] {dtype} storage")
    g = ph.from_spec(spec)
    p = torch.from_numpy(as_f32(synth.random_array((spec.n_proj,) + tuple(spec.det_shape), 15))).to(dtype)
    stored = p.float().numpy()
    out = to_np(ph.weight_filter_3d(g, p.to(gc.device()).contiguous()))
    ref = ora.filter_projections(spec, ora.weight(spec, stored)).reshape(stored.shape)
    err = rel_l2(out, ref)
    say(f"  rel-L2 {err:.2e}")
    assert err < FP32_TOL


def test_filter_2048_arc_detector_learned(ph, ora):
    """Equiangular detector (cosine weight cos(gamma)) with a learned
    2048-point response and redundancy weights, 7 views of 1500 bins."""
    spec = synth.config("fan2d_512").with_(kind="fan2d_curved", det_shape=(1500,), n_proj=7)
    say("[filter2048] arc detector, learned K, 7 x 1500")
    g = ph.from_spec(spec)
    p = as_f32(synth.random_array((spec.n_proj, 1500), 16, dist="uniform"))
    K = as_f32(np.abs(synth.random_array((2048,), 17)))
    W_red = as_f32(synth.random_array((spec.n_proj, 1500), 18, dist="uniform", low=0.5, high=1.5))
    out = to_np(ph.weight_filter_2d(g, to_dev(p), True, K=to_dev(K), W_red=to_dev(W_red)))
    ref = ora.filter_projections(spec, ora.weight(spec, p, W_red=W_red), K=K).reshape(p.shape)
    err = rel_l2(out, ref)
    say(f"  rel-L2 {err:.2e}")
    assert err < FP32_TOL
