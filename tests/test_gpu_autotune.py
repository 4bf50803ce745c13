"""The autotuner: every candidate gives the same indices; the chosen one is a valid
candidate and round-trips through the cache."""
import numpy as np
import pytest

from paper_2305_14306_amd import synth

pytestmark = pytest.mark.gpu


def test_autotune_single_and_batch(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_14306_amd import autotune, hav
    x = torch.from_numpy(synth.scene_planes_blobs(80000, seed=41)).cuda()
    best, table = autotune.tune(x, 20000, reps=2)
    assert best in [c for c, _ in table] and len(table) == len(list(autotune.candidates()))
    clouds, Ms = synth.batch_lidar_clouds(n_clouds=6, n_min=5000, n_max=40000)
    offs = np.concatenate([[0], np.cumsum([c.shape[0] for c in clouds])])
    xb = torch.from_numpy(np.concatenate(clouds)).cuda()
    bbest, btable = autotune.tune_batch(xb, offs, Ms, reps=1,
                                        cands=list(autotune.candidates(depths=(1, 4), budgets=(16,))))
    assert bbest in [c for c, _ in btable]
    path = str(tmp_path / "tune.json")
    got = autotune.cached_or_tune(path, x, 20000)
    assert autotune.cached_or_tune(path, x, 20000) == got
    idx = hav.Sampler().sample(x, 20000, hav.params(**got)).cpu().numpy()
    ref = hav.Sampler().sample(x, 20000).cpu().numpy()
    assert np.array_equal(idx, ref)
