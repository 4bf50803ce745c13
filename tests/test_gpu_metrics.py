"""GPU nearest-sample distances (coverage and spacing of a sample, Sec. 3.1, Fig. 3),
value for value against the oracle."""
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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _check(gpu, orc, s, q, label, nn=None):
    _note(f"case nn {label} M={s.shape[0]} Q={'self' if q is None else q.shape[0]}")
    nn = nn if nn is not None else gpu.NearestSample()
    d2, mx = nn.d2(_dev(s), None if q is None else _dev(q))
    got = d2.cpu().numpy()
    want = orc.nn_d2(s, s if q is None else q, q is None)
    assert np.array_equal(got, want)
    assert float(mx.cpu()[0]) == want.max()
    return got


@pytest.mark.parametrize("shape", ["box", "plane", "line", "dups", "one", "two"])
def test_nn_shapes(gpu, orc, shape):
    rng = np.random.default_rng(len(shape))
    n = 3000
    if shape == "box":
        s = rng.uniform(0, 5, (n, 3))
    elif shape == "plane":
        s = np.c_[rng.uniform(0, 50, (n, 2)), np.full(n, 1.5)]
    elif shape == "line":
        s = np.c_[rng.uniform(-30, 30, n), np.zeros((n, 2))]
    elif shape == "dups":
        s = np.repeat(rng.uniform(0, 2, (n // 4, 3)), 4, axis=0)
    elif shape == "one":
        s = rng.uniform(0, 1, (1, 3))
    else:
        s = rng.uniform(0, 1, (2, 3))
    s = s.astype(np.float32)
    q = rng.uniform(-10, 60, (5000, 3)).astype(np.float32)  # mostly outside the samples' box
    _check(gpu, orc, s, q, shape)
    if s.shape[0] > 1:
        _check(gpu, orc, s, None, shape + " spacing")


def test_nn_covering_of_sampler_output(gpu, orc):
    import torch
    x = synth.scene_planes_blobs(60000, seed=51)
    idx = gpu.Sampler().sample(_dev(x), 15000).cpu().numpy()
    s = x[idx]
    nn = gpu.NearestSample()
    d = _check(gpu, orc, s, x, "covering 60k/15k", nn)
    assert np.sqrt(d.max()) == pytest.approx(orc.covering_radius(x, idx), rel=0, abs=0)
    _check(gpu, orc, s, None, "spacing 15k", nn)
    _check(gpu, orc, s[:7000], x[:30000], "reuse smaller", nn)


def _check_ball(gpu, orc, x, c, radius, K, label, bq=None):
    _note(f"case ball {label} N={x.shape[0]} Q={c.shape[0]} r={radius} K={K}")
    bq = bq if bq is not None else gpu.BallQuery()
    idx, cnt = bq.query(_dev(x), _dev(c), radius, K)
    widx, wcnt = orc.ball_query(x, c, radius, K)
    assert np.array_equal(cnt.cpu().numpy(), wcnt)
    assert np.array_equal(idx.cpu().numpy(), widx)


def test_ball_query_lattice_and_edges(gpu, orc):
    x = synth.lattice(8)
    _check_ball(gpu, orc, x, x, 1.01, 4, "lattice r 1.01")
    _check_ball(gpu, orc, x, x, 1.0, 3, "lattice r 1 (strict)")
    _check_ball(gpu, orc, x, x[:50], 2.5, 64, "lattice K 64")
    far = np.array([[100.0, 0.0, 0.0], [-3.0, -3.0, -3.0]], dtype=np.float32)
    _check_ball(gpu, orc, x, far, 1.0, 8, "empty balls")
    _check_ball(gpu, orc, x[:1], x[:3], 1.5, 5, "one point")


@pytest.mark.parametrize("radius,K", [(0.2, 16), (0.8, 32), (3.0, 64)])
def test_ball_query_sampled_centres(gpu, orc, radius, K):
    # the set-abstraction pattern: sample centres with the sampler, group around them
    x = synth.scene_planes_blobs(40000, seed=61)
    idx = gpu.Sampler().sample(_dev(x), 2000).cpu().numpy()
    bq = gpu.BallQuery()
    _check_ball(gpu, orc, x, x[idx], radius, K, "scene", bq)
    d = np.repeat(synth.random_cloud(3000, 7, scale=2.0), 3, axis=0)  # duplicates
    _check_ball(gpu, orc, d, d[::7], radius, K, "duplicates", bq)
