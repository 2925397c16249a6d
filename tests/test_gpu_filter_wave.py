"""The wave-level weighting and filter kernels against the oracle: M = 2048,
where one wave takes a pair of detector rows, and M = 1024, where each half
of a wave takes a pair and a wave four consecutive rows. The cases are the
ones their row grouping and range-checked loads and stores must get right:
* an odd number of rows, so the last pair has no second row;
* one, two or three rows, so a wave's group of rows is partial;
* a single detector row per view, so one group of rows spans views;
* fewer row pairs than the waves of one workgroup;
* more than the persistent grid has waves, so every wave takes several;
* rows as wide as the transform under a learned response, where every element
  a lane holds is live, and rows of a single bin;
* ragged widths;
* both weight tables present;
* a batch of two;
* half-precision storage;
* the equiangular (arc) detector with a learned response.
At M = 2048, rows of at most 1024 bins take the kernel variant that skips the
zero-padded half and prefetches the next pair; longer rows take the full one."""
import numpy as np
import pytest
import torch

import gpu_common as gc
import synth
from gpu_common import FP32_TOL, check, as_f32, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ph():
    gc.device()
    import paper_1904_13342_amd as ph
    return ph


def _cone(n_proj, nv, nu):
    return synth.config("cone3d_crop32").with_(det_shape=(nv, nu), n_proj=n_proj)


# name: (spec, transform length of a learned response (0: default Ram-Lak), batch)
CASES_3D = {
    "2048_one_row_ramlak": (_cone(1, 1, 1024), 0, 1),
    "2048_odd_rows_ragged_ramlak": (_cone(3, 5, 1023), 0, 1),
    "2048_odd_rows_batch2_learned": (_cone(3, 5, 700), 2048, 2),
    "2048_full_width_learned": (_cone(3, 3, 2048), 2048, 1),
    "2048_more_pairs_than_waves": (_cone(11, 373, 520), 0, 1),
    "1024_one_row_learned": (_cone(1, 1, 620), 1024, 1),
    "1024_two_rows_learned": (_cone(2, 1, 620), 1024, 1),
    "1024_one_row_per_view_learned": (_cone(7, 1, 620), 1024, 1),
    "1024_odd_rows_batch2_learned": (_cone(3, 5, 700), 1024, 2),
    "1024_full_width_learned": (_cone(3, 3, 1024), 1024, 1),
    "1024_ramlak": (_cone(5, 7, 500), 0, 1),
    "1024_more_groups_than_waves": (_cone(11, 751, 300), 1024, 1),
    "1024_single_bin_last_group_one_row": (_cone(1, 5, 1), 1024, 1),
    "2048_single_bin_odd_rows": (_cone(3, 1, 1), 2048, 1),
}


@pytest.mark.parametrize("name", list(CASES_3D))
def test_filter_wave_cone(ph, ora, name):
    spec, M, batch = CASES_3D[name]
    learned = M > 0
    n_proj, (nv, nu) = spec.n_proj, spec.det_shape
    say(f"[filter wave] {name}: batch {batch}, {n_proj} x {nv} rows of {nu}")
    g = ph.from_spec(spec)
    p = as_f32(synth.random_array((batch, n_proj, nv, nu), 11, dist="uniform"))
    K = W_red = W = None
    if learned:
        K = as_f32(np.abs(synth.random_array((M,), 12)))
        W_red = as_f32(synth.random_array((n_proj, nu), 13, dist="uniform", low=0.5, high=1.5))
        W = as_f32(synth.random_array((nv, nu), 14, dist="uniform", low=0.5, high=1.5))
        out = ph.weight_filter_3d(g, to_dev(p), K=to_dev(K), W_red=to_dev(W_red), W=to_dev(W))
    else:
        out = ph.weight_filter_3d(g, to_dev(p))
    out = to_np(out)
    for b in range(batch):
        q = ora.weight(spec, p[b], W_red=W_red, W=W)
        ref = ora.filter_projections(spec, q, K=K).reshape(n_proj, nv, nu)
        check(out[b], ref, f"batch {b}")


@pytest.mark.parametrize("M", [1024, 2048])
@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_filter_wave_half_storage(ph, ora, dtype, M):
    """Half-precision projections are widened on load: the result matches the
    oracle run on the stored (rounded) values to the FP32 tolerance."""
    spec = _cone(5, 7, 1000)
    say(f"[filter wave] {dtype} storage, M = {M}")
    g = ph.from_spec(spec)
    p = torch.from_numpy(as_f32(synth.random_array((spec.n_proj,) + tuple(spec.det_shape), 15))).to(dtype)
    stored = p.float().numpy()
    K = as_f32(np.abs(synth.random_array((M,), 19)))
    out = to_np(ph.weight_filter_3d(g, p.to(gc.device()).contiguous(), K=to_dev(K)))
    ref = ora.filter_projections(spec, ora.weight(spec, stored), K=K).reshape(stored.shape)
    check(out, ref, "")


@pytest.mark.parametrize("M,nu", [(1024, 1000), (2048, 1500), (2048, 1000)])
def test_filter_wave_arc_detector_learned(ph, ora, M, nu):
    """Equiangular detector (cosine weight cos(gamma)) with a learned
    response and redundancy weights, 7 views; at M = 2048 both with rows
    longer than half the transform and with rows of at most 1024 bins (whose
    zero-padded upper half the kernel skips)."""
    spec = synth.config("fan2d_512").with_(kind="fan2d_curved", det_shape=(nu,), n_proj=7)
    say(f"[filter wave] arc detector, learned K (M = {M}), 7 x {nu}")
    g = ph.from_spec(spec)
    p = as_f32(synth.random_array((spec.n_proj, nu), 16, dist="uniform"))
    K = as_f32(np.abs(synth.random_array((M,), 17)))
    W_red = as_f32(synth.random_array((spec.n_proj, nu), 18, dist="uniform", low=0.5, high=1.5))
    out = to_np(ph.weight_filter_2d(g, to_dev(p), True, K=to_dev(K), W_red=to_dev(W_red)))
    ref = ora.filter_projections(spec, ora.weight(spec, p, W_red=W_red), K=K).reshape(p.shape)
    check(out, ref, "")
