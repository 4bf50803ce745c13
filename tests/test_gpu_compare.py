"""GPU parity of the latency-study comparators (Sec. 4.2, Fig. 7): farthest point
sampling and random point sampling, index for index against the oracle."""
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


def _fps(gpu, x, M, start=0, blocks=0):
    import torch
    f = gpu.FPS()
    out = f.sample(torch.from_numpy(np.ascontiguousarray(x)).cuda(), M, start, blocks).cpu().numpy()
    torch.cuda.synchronize()
    assert f.error_flag() == 0
    return out


@pytest.mark.parametrize("N,M,start,blocks", [
    (1, 1, 0, 0), (9, 9, 0, 0), (700, 300, 5, 0), (4096, 2048, 0, 0),     # one block
    (4097, 1000, 17, 0),                                                    # two blocks, ragged
    (12000, 3000, 0, 0), (12000, 3000, 11999, 7), (20000, 400, 3, 64),     # several / many
    (3000, 3000, 0, 3)])
def test_fps_matches_oracle(gpu, orc, N, M, start, blocks):
    x = synth.random_cloud(N, 40 + N, scale=5.0, kind="clustered")
    _note(f"case fps N={N} M={M} start={start} blocks={blocks}")
    assert np.array_equal(_fps(gpu, x, M, start, blocks), orc.fps(x, M, start))


def test_fps_duplicates_and_lattice(gpu, orc):
    x = synth.lattice(8)
    _note("case fps lattice")
    for blocks in (0, 2, 5):
        assert np.array_equal(_fps(gpu, x, 512, 0, blocks), orc.fps(x, 512, 0))
    d = np.repeat(synth.random_cloud(300, 3), 4, axis=0)  # every point four times
    _note("case fps duplicates")
    assert np.array_equal(_fps(gpu, d, 1200, 7, 2), orc.fps(d, 1200, 7))


def test_fps_scene_multiblock(gpu, orc):
    x = synth.scene_planes_blobs(50000, seed=8)
    _note("case fps scene 50k -> 2000")
    assert np.array_equal(_fps(gpu, x, 2000), orc.fps(x, 2000, 0))


@pytest.mark.parametrize("N,M,seed,window", [
    (1, 1, 0, 0.0), (10, 10, 1, 0.0), (100, 1, 2, 0.0), (100, 99, 2, 0.0), (2047, 1000, 3, 0.0),
    (2049, 1000, 3, 0.0), (65536, 32768, 4, 0.0), (262144, 131072, 5, 0.0), (300001, 7, 6, 0.0),
    (50000, 25000, 7, -1.0), (50000, 25000, 7, 0.05), (50000, 12345, 8, 64.0)])
def test_rps_matches_oracle(gpu, orc, N, M, seed, window):
    _note(f"case rps N={N} M={M} seed={seed} window={window}")
    got = gpu.RPS().sample(N, M, seed, window).cpu().numpy()
    assert np.array_equal(got, orc.rps(N, M, seed))


def test_rps_workspace_reuse(gpu, orc):
    r = gpu.RPS()
    _note("case rps reuse")
    for N, M, seed in [(100000, 50000, 1), (3000, 10, 2), (100000, 99999, 3), (77777, 1, 4)]:
        assert np.array_equal(r.sample(N, M, seed).cpu().numpy(), orc.rps(N, M, seed))
