"""GPU parity of the batched call: every cloud of a batch must get exactly what the
oracle (and the single-cloud call) gives it alone, whatever the other clouds are.
"""
import sys

import numpy as np
import pytest

from paper_2305_14306_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_14306_amd import hav
    hav.lib()
    return hav


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_params(orc, p):
    fv = tuple(p.fixed_voxel) if p.flags & 1 else None
    return orc.params(layers=p.layers, layer_ratio=p.layer_ratio, t_max=p.t_max, sigma=p.sigma,
                      aspect=tuple(p.aspect), fixed_voxel=fv, select=p.select, seed=p.select_seed)


def _run_batch(gpu, clouds, Ms, p, sampler=None):
    import torch
    offs = np.concatenate([[0], np.cumsum([c.shape[0] for c in clouds])]).astype(np.int64)
    xyz = torch.from_numpy(np.ascontiguousarray(np.concatenate(clouds), dtype=np.float32)).cuda()
    s = sampler if sampler is not None else gpu.Sampler()
    parts, infos = s.sample_batch(xyz, offs, Ms, p, with_info=True)
    return [q.cpu().numpy() for q in parts], infos


def _check_batch(gpu, orc, clouds, Ms, p=None, label="", sampler=None):
    p = p if p is not None else gpu.params()
    _note(f"case batch {label} B={len(clouds)} N={[c.shape[0] for c in clouds][:8]}")
    got, infos = _run_batch(gpu, clouds, Ms, p, sampler)
    for i, (x, M) in enumerate(zip(clouds, Ms)):
        st, want, winfo = orc.sample(x, M, _oracle_params(orc, p))
        assert infos[i]["status"] == st, i
        if st != 0:
            continue
        assert infos[i] == winfo, (i, infos[i], winfo)
        assert np.array_equal(got[i], want), i
    return got, infos


def _mixed_small():
    kinds = ["uniform", "clustered", "quantised"]
    sizes = [1, 2, 17, 255, 1025, 4097, 9999, 3000, 20000, 12]
    clouds = [synth.random_cloud(n, 100 + n, scale=6.0, kind=kinds[i % 3]) for i, n in enumerate(sizes)]
    Ms = [1, 2, 5, 255, 300, 1000, 2500, 3000, 4000, 12]  # includes M == N clouds
    return clouds, Ms


def test_batch_small_uneven(gpu, orc):
    clouds, Ms = _mixed_small()
    _check_batch(gpu, orc, clouds, Ms, label="small")


@pytest.mark.parametrize("kw", [dict(layers=1), dict(layers=3, sigma=0.0), dict(t_max=3),
                                dict(fixed_voxel=0.5), dict(aspect=(1.0, 2.0, 0.5)),
                                dict(spec_depth=1), dict(spec_depth=3), dict(trim_window=-1.0),
                                dict(trim_window=0.02), dict(select=1, select_seed=7), dict(table_scale=1),
                                dict(bin_points=2048), dict(bin_points=8192, spec_depth=2)])
def test_batch_params(gpu, orc, kw):
    clouds, Ms = _mixed_small()
    _check_batch(gpu, orc, clouds, Ms, gpu.params(**kw), label=str(kw))


def test_batch_single_cloud_equals_single_call(gpu, orc):
    x = synth.scene_planes_blobs(150000, seed=5)
    got, _ = _check_batch(gpu, orc, [x], [150000 // 4], label="one cloud")
    import torch
    alone = gpu.Sampler().sample(torch.from_numpy(x).cuda(), 150000 // 4).cpu().numpy()
    assert np.array_equal(got[0], alone)


def test_batch_large_and_tiny(gpu, orc):
    # a 1M-point cloud beside tiny ones and a LiDAR sweep: the batched search serves
    # clouds of very different tile counts in one launch
    clouds = [synth.scene_planes_blobs(1 << 20, seed=41), synth.random_cloud(1, 3),
              synth.random_cloud(5, 4), synth.random_cloud(3000, 5, kind="clustered"),
              synth.lidar_points(200000, seed=42)]
    Ms = [max(1, c.shape[0] // 4) for c in clouds]
    _check_batch(gpu, orc, clouds, Ms, label="large and tiny")


def test_batch_lidar_64(gpu, orc):
    clouds, Ms = synth.batch_lidar_clouds()
    _check_batch(gpu, orc, clouds, Ms, label="lidar x64")


def test_batch_error_cloud_is_isolated(gpu, orc):
    clouds, Ms = _mixed_small()
    bad = clouds[6].copy()
    bad[17, 1] = np.nan
    clouds[6] = bad
    got, infos = _check_batch(gpu, orc, clouds, Ms, label="nan cloud")
    assert infos[6]["status"] == gpu.ERR_NONFINITE


def test_batch_workspace_reuse_and_order(gpu, orc):
    # the same sizes twice with other data, then the clouds reversed (new sizes order)
    s = gpu.Sampler()
    clouds, Ms = _mixed_small()
    _check_batch(gpu, orc, clouds, Ms, label="reuse 1", sampler=s)
    other = [synth.random_cloud(c.shape[0], 7 + c.shape[0], scale=3.0, kind="clustered") for c in clouds]
    _check_batch(gpu, orc, other, Ms, label="reuse 2", sampler=s)
    _check_batch(gpu, orc, clouds[::-1], Ms[::-1], label="reversed", sampler=s)
