"""GPU parity: libhav.so against the CPU oracle, bit for bit.

Sampling is index selection, so the bar is exact: the same M indices, and the same
per-layer search record (chosen scale, evaluations, voxel count, trim/pad), on the same
seeded inputs. Sizes span several scan tiles and hash-table blocks and end in ragged
tails; the full-size configurations run exactly as the bench launches them.
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


def _to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _oracle_params(orc, p):
    fv = tuple(p.fixed_voxel) if p.flags & 1 else None
    return orc.params(layers=p.layers, layer_ratio=p.layer_ratio, t_max=p.t_max, sigma=p.sigma,
                      aspect=tuple(p.aspect), fixed_voxel=fv, select=p.select, seed=p.select_seed)


def _check(gpu, orc, x, M, p=None, label=""):
    p = p if p is not None else gpu.params()
    _note(f"case {label} N={x.shape[0]} M={M}")
    st, want, winfo = orc.sample(x, M, _oracle_params(orc, p))
    assert st == 0
    idx, info = gpu.Sampler().sample(_to_dev(x), M, p, with_info=True)
    got = idx.cpu().numpy()
    assert info["status"] == 0
    assert info == winfo, (info, winfo)
    assert np.array_equal(got, want)
    return got, info


# ------------------------------------------------------------------ closed-form cases

@pytest.mark.parametrize("layers,M", [(1, 64), (1, 8), (1, 512), (2, 60), (2, 100), (3, 300),
                                      (2, 1), (2, 511)])
def test_lattice(gpu, orc, layers, M):
    _check(gpu, orc, synth.lattice(8), M, gpu.params(layers=layers), "lattice")


def test_ties_lowest_index(gpu, orc):
    pts = [(0.0, 0.0, 0.0)]
    for k in range(64):
        a, b = (2 * k + 0.5, 1.0, 1.0), (2 * k + 1.5, 1.0, 1.0)
        pts += [a, b] if k % 2 == 0 else [b, a]
    x = np.array(pts, dtype=np.float32)
    _check(gpu, orc, x, 64, gpu.params(layers=1, fixed_voxel=2.0), "ties")
    # subnormal squared distances must not be flushed to zero (they would tie):
    # voxel 2^-60, centre 2^-61; point 1 is 2^-70 + 2^-80 off centre (d2 just above
    # 2^-140, subnormal), point 2 is 2^-70 off (d2 = 2^-140): point 2 must win
    c, d = 2.0 ** -61, 2.0 ** -70
    y = np.array([[0, 0, 0], [c + d + 2.0 ** -80, c, c], [c + d, c, c]], dtype=np.float32)
    got, _ = _check(gpu, orc, y, 1, gpu.params(layers=1, fixed_voxel=2.0 ** -60), "subnormal")
    assert list(got) == [2]


# ------------------------------------------------------------------ small and ragged clouds

@pytest.mark.parametrize("kind", ["uniform", "clustered", "quantised"])
@pytest.mark.parametrize("n", [1, 2, 3, 17, 255, 1023, 1025, 4097, 9999])
def test_small_ragged(gpu, orc, kind, n):
    x = synth.random_cloud(n, n + 7, scale=8.0, kind=kind)
    for M in sorted({1, max(1, n // 3), max(1, n - 1), n}):
        _check(gpu, orc, x, M, label=kind)


def test_degenerate(gpu, orc):
    _check(gpu, orc, np.full((300, 3), 2.5, np.float32), 40, label="identical")
    y = np.repeat(synth.random_cloud(50, 3), 7, axis=0)
    _check(gpu, orc, y, 120, label="duplicates")
    line = np.zeros((2000, 3), np.float32)
    line[:, 0] = np.linspace(0, 1, 2000, dtype=np.float32)
    _check(gpu, orc, line, 700, label="line")
    _check(gpu, orc, -synth.random_cloud(3000, 4, scale=1e-3), 500, label="tiny extent")
    big = synth.random_cloud(3000, 5, scale=1.0) * np.float32(1e25)
    _check(gpu, orc, big, 500, label="huge extent")


def test_degenerate_at_scale(gpu, orc):
    # the pad paths across many scan blocks: one voxel at every size (every point
    # identical), heavy duplicates, and a cloud on a line
    _check(gpu, orc, np.full((200000, 3), -7.25, np.float32), 50000, label="identical 200k")
    y = np.repeat(synth.random_cloud(20000, 8, scale=5.0), 8, axis=0)
    _check(gpu, orc, y, 40000, label="duplicates 160k")
    line = np.zeros((300000, 3), np.float32)
    line[:, 1] = np.linspace(-3, 9, 300000, dtype=np.float32)
    _check(gpu, orc, line, 75000, label="line 300k")


# ------------------------------------------------------------------ parameters

@pytest.mark.parametrize("kw", [dict(), dict(layers=1), dict(layers=3), dict(layers=8, layer_ratio=2),
                                dict(sigma=0.0), dict(sigma=0.5), dict(t_max=1), dict(t_max=5),
                                dict(aspect=(1.0, 1.0, 0.5)), dict(aspect=(3.0, 0.75, 0.125)),
                                dict(fixed_voxel=0.34), dict(fixed_voxel=(0.34, 0.34, 0.30)),
                                dict(layers=1, fixed_voxel=2.0)])
def test_kitti_like_params(gpu, orc, kw):
    x = synth.uniform_box_with_ground()
    _check(gpu, orc, x, 4096, gpu.params(**kw), f"kitti-like 16384 {kw}")


@pytest.mark.parametrize("M", [1, 100, 1000, 4096, 8191, 16383, 16384])
def test_kitti_like_sizes(gpu, orc, M):
    _check(gpu, orc, synth.uniform_box_with_ground(), M, label="kitti-like 16384")


# ------------------------------------------------------------------ device-side errors

def test_device_errors(gpu, orc):
    x = synth.random_cloud(5000, 1)
    for bad, code in ((np.nan, gpu.ERR_NONFINITE), (np.inf, gpu.ERR_NONFINITE),
                      (-np.inf, gpu.ERR_NONFINITE), (np.float32(2.0 ** 101), gpu.ERR_UNSUPPORTED)):
        y = x.copy()
        y[4321, 2] = bad
        _note(f"case error {bad}")
        _, info = gpu.Sampler().sample(_to_dev(y), 100, gpu.params(), with_info=True)
        assert info["status"] == code
        assert orc.sample(y, 100)[0] == code
    _, info = gpu.Sampler().sample(_to_dev(x), 100, gpu.params(fixed_voxel=1e-6), with_info=True)
    assert info["status"] == gpu.ERR_UNSUPPORTED
    # the library keeps working after a device-side error
    _check(gpu, orc, x, 100, label="after error")


def test_scan_give_up_reports_and_recovers(gpu, orc):
    # the output scan's bounded waits give up after one poll (forced from the host): the
    # call reports HAV_ERR_HIP, every block still finishes, and the next calls on the same
    # workspace are exact again. Every point is identical, so layer 1 pads (in the marking
    # launch's last block) and the output scan pads the last layer; 1M points make 256
    # scan blocks.
    import torch
    x = np.full((1 << 20, 3), 2.5, np.float32)
    M = 1 << 18
    st, want, winfo = orc.sample(x, M, _oracle_params(orc, gpu.params()))
    assert st == 0
    xd = _to_dev(x)
    s = gpu.Sampler()
    seen = []
    torch.cuda.synchronize()
    gpu.debug_scan_spin_limit(1)
    try:
        for _ in range(3):
            _note("case scan give-up, spin limit 1, identical 1M")
            _, info = s.sample(xd, M, with_info=True)
            seen.append(info["status"])
    finally:
        torch.cuda.synchronize()
        gpu.debug_scan_spin_limit(0)
    assert set(seen) <= {0, gpu.ERR_HIP}, seen
    for _ in range(2):
        _note("case after scan give-up, identical 1M")
        idx, info = s.sample(xd, M, with_info=True)
        assert info["status"] == 0
        assert info == winfo, (info, winfo)
        assert np.array_equal(idx.cpu().numpy(), want)
    if gpu.ERR_HIP not in seen:
        pytest.skip("no scan wait gave up after one poll: the failure path was not reached")


def test_search_give_up_reports_and_sampler_recovers(gpu, orc):
    # a voxel search whose bounded waits give up after one poll (forced from the host):
    # the call reports HAV_ERR_HIP and leaves the workspace needing initialisation; the
    # Sampler sees the status, initialises it again, and the next calls are exact. The
    # one-shot hav.sample raises for such a call.
    import torch
    x = synth.scene_planes_blobs()
    M = x.shape[0] // 4
    st, want, winfo = orc.sample(x, M)
    assert st == 0
    xd = _to_dev(x)
    s = gpu.Sampler()
    torch.cuda.synchronize()
    gpu.debug_search_spin_limit(1)
    try:
        _note("case search give-up, spin limit 1, scene 1M")
        s.sample(xd, M)
        with pytest.raises(gpu.HavError) as e:
            s.check()
        assert e.value.status == gpu.ERR_HIP
        with pytest.raises(gpu.HavError):
            gpu.sample(xd, M)
    finally:
        torch.cuda.synchronize()
        gpu.debug_search_spin_limit(0)
    for _ in range(2):
        _note("case after search give-up, scene 1M")
        idx = s.sample(xd, M)
        info = s.check()[0]
        assert info == winfo, (info, winfo)
        assert np.array_equal(idx.cpu().numpy(), want)


def test_padding_in_layers_before_the_last(gpu, orc):
    # clouds with few distinct positions: every layer finds fewer voxels than its m and
    # pads with the lowest-index unsampled points, in layers before the last too (done
    # by the marking launch's last block); one cloud needs several 4,096-point tag tiles
    # of padding per layer; the points mode copies the padded points
    rng = np.random.default_rng(71)
    for n, ndist, M in ((20000, 37, 5000), (300000, 100, 100000)):
        base = rng.uniform(-5.0, 5.0, size=(ndist, 3)).astype(np.float32)
        x = base[rng.integers(0, ndist, n)]
        _, info = _check(gpu, orc, x, M, gpu.params(layers=3), f"{ndist} distinct, 3 layers")
        assert info["padded"][0] > 0 and info["padded"][1] > 0, info["padded"]
    x = np.repeat(rng.uniform(-5.0, 5.0, size=(40, 3)).astype(np.float32), 250, axis=0)
    _check_points(gpu, orc, x, 3000, gpu.params(select=3, layers=3), "40 distinct, mean, 3 layers")


def test_determinism_and_workspace_independence(gpu, orc):
    import torch
    x = synth.scene_planes_blobs(200000, seed=9)
    xd = _to_dev(x)
    s1, s2 = gpu.Sampler(), gpu.Sampler()
    a = s1.sample(xd, 50000).cpu().numpy()
    # a dirty, larger workspace must not change anything
    s2.ws = torch.full((gpu.workspace_size(200000, 50000) + 4096,), 0xAB, dtype=torch.uint8,
                       device="cuda")
    b = s2.sample(xd, 50000).cpu().numpy()
    for _ in range(3):
        assert np.array_equal(s1.sample(xd, 50000).cpu().numpy(), a)
    assert np.array_equal(a, b)
    assert np.array_equal(a, orc.sample(x, 50000)[1])


# ------------------------------------------------------------------ workloads at full size

def test_lidar_chain(gpu, orc):
    x = synth.lidar_scan()
    Ms = [16384, 4096, 1024, 256]
    _note(f"case lidar chain N={x.shape[0]}")
    st, want, winfo = orc.chain(x, Ms)
    assert st == 0
    parts, infos = gpu.Sampler().chain(_to_dev(x), Ms, with_info=True)
    for j in range(len(Ms)):
        assert infos[j] == winfo[j], j
        assert np.array_equal(parts[j].cpu().numpy(), want[j]), j


def test_scene_chain_1m(gpu, orc):
    x = synth.scene_planes_blobs()
    N = x.shape[0]
    Ms = [N // 4, N // 16, N // 64]
    _note(f"case scene chain N={N}")
    st, want, winfo = orc.chain(x, Ms)
    assert st == 0
    parts, infos = gpu.Sampler().chain(_to_dev(x), Ms, with_info=True)
    for j in range(len(Ms)):
        assert infos[j] == winfo[j], j
        assert np.array_equal(parts[j].cpu().numpy(), want[j]), j


def test_scene_single_stage_1m(gpu, orc):
    x = synth.scene_planes_blobs()
    _check(gpu, orc, x, x.shape[0] // 4, label="scene 1M->262144")


def test_scene_single_stage_8m_ragged(gpu, orc):
    # eight times the bench cloud and a ragged tail: the binning blocks take several
    # rounds of points each, every search block several tiles per pass
    x = synth.scene_planes_blobs((1 << 23) + 4321, seed=11)
    _check(gpu, orc, x, x.shape[0] // 4, label="scene 8M+4321 -> N/4")


# ------------------------------------------------------------------ workspace contract, tuning

def test_uninitialised_workspace_is_reported(gpu):
    import ctypes as C
    import torch
    x = _to_dev(synth.random_cloud(5000, 2))
    p = gpu.params()
    ws = torch.zeros(gpu.workspace_size(5000, 100, p), dtype=torch.uint8, device="cuda")
    idx = torch.empty(100, dtype=torch.int32, device="cuda")
    info = torch.zeros(C.sizeof(gpu.Info), dtype=torch.uint8, device="cuda")
    st = gpu.lib().hav_sample(C.c_void_p(x.data_ptr()), 5000, 100, C.byref(p),
                              C.c_void_p(idx.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                              C.c_void_p(info.data_ptr()), gpu._stream_ptr())
    assert st == gpu.OK
    assert gpu.read_info(info)[0]["status"] == gpu.ERR_WORKSPACE_NOT_INIT
    # initialised for another size: also refused
    big = gpu.workspace_size(8000, 100, p)
    ws2 = torch.zeros(big, dtype=torch.uint8, device="cuda")
    assert gpu.lib().hav_workspace_init(8000, C.byref(p), C.c_void_p(ws2.data_ptr()), big,
                                        gpu._stream_ptr()) == gpu.OK
    st = gpu.lib().hav_sample(C.c_void_p(x.data_ptr()), 5000, 100, C.byref(p),
                              C.c_void_p(idx.data_ptr()), C.c_void_p(ws2.data_ptr()), big,
                              C.c_void_p(info.data_ptr()), gpu._stream_ptr())
    assert st == gpu.OK
    assert gpu.read_info(info)[0]["status"] == gpu.ERR_WORKSPACE_NOT_INIT


def test_workspace_reuse_across_sizes(gpu, orc):
    # one sampler, alternating sizes and parameters: every call leaves the workspace
    # clean, and a size change re-initialises it
    s = gpu.Sampler()
    clouds = [synth.random_cloud(n, n, scale=20.0, kind="clustered") for n in (30000, 7000, 30000)]
    for rep in range(2):
        for x in clouds:
            for M, kw in ((x.shape[0] // 4, {}), (x.shape[0] // 10, dict(layers=3)),
                          (500, dict(fixed_voxel=0.7))):
                p = gpu.params(**kw)
                _note(f"case reuse rep={rep} N={x.shape[0]} M={M} {kw}")
                idx, info = s.sample(_to_dev(x), M, p, with_info=True)
                st, want, winfo = orc.sample(x, M, _oracle_params(orc, p))
                assert info == winfo
                assert np.array_equal(idx.cpu().numpy(), want)


@pytest.mark.parametrize("depth", [1, 2, 3, 4, 7])
def test_spec_depth_does_not_change_results(gpu, orc, depth):
    x = synth.scene_planes_blobs(100000, seed=21)
    for M in (25000, 6000):
        _check(gpu, orc, x, M, gpu.params(spec_depth=depth), f"depth {depth}")
    _check(gpu, orc, synth.lattice(8), 60, gpu.params(spec_depth=depth), f"lattice depth {depth}")


@pytest.mark.parametrize("n,depth", [(262144, 4), (262145, 4), (300000, 3), (300000, 7)])
def test_split_ticket_boundary(gpu, orc, n, depth):
    # a search pass of at most 512 tickets (tiles x depth) gives each tile's candidates
    # tickets of their own: both sides of that boundary, and depths on either side of it
    x = synth.scene_planes_blobs(n, seed=31)
    _check(gpu, orc, x, n // 4, gpu.params(spec_depth=depth), f"split boundary n={n} depth={depth}")


@pytest.mark.parametrize("kw", [dict(spec_budget=1), dict(spec_budget=1024), dict(search_blocks=1),
                                dict(search_blocks=7), dict(search_blocks=5000),
                                dict(spec_depth=3, spec_budget=1, search_blocks=64), dict(table_scale=2),
                                dict(table_scale=3, spec_depth=7), dict(bin_points=2048),
                                dict(bin_points=8192), dict(bin_points=2048, table_scale=1)])
def test_tuning_fields_do_not_change_results(gpu, orc, kw):
    x = synth.scene_planes_blobs(60000, seed=23)
    _check(gpu, orc, x, 15000, gpu.params(**kw), f"tuning {kw}")


@pytest.mark.parametrize("bp", [2048, 8192])
def test_binning_block_shape_at_scale(gpu, orc, bp):
    # the binning workgroup's share changes the binning blocks (and, past 512 blocks, is
    # capped): a 1M scene and a 2M+ ragged cloud, results unchanged
    x = synth.scene_planes_blobs()
    _check(gpu, orc, x, x.shape[0] // 4, gpu.params(bin_points=bp), f"bin points {bp} scene 1M")
    y = synth.scene_planes_blobs((1 << 21) + 77, seed=12)
    _check(gpu, orc, y, y.shape[0] // 16, gpu.params(bin_points=bp), f"bin points {bp} 2M ragged")


@pytest.mark.parametrize("tw", [-1.0, 0.02, 0.5, 64.0])
def test_trim_window_does_not_change_results(gpu, orc, tw):
    # a window too narrow to hold the threshold, or none at all, takes the every-voxel
    # bucket; a wide one a large bucket: the picks never change
    x = synth.scene_planes_blobs(60000, seed=29)
    _check(gpu, orc, x, 15000, gpu.params(trim_window=tw), f"trim window {tw}")
    _check(gpu, orc, x, 9000, gpu.params(trim_window=tw, sigma=0.6), f"trim window {tw} wide tolerance")
    _check(gpu, orc, x, 7000, gpu.params(trim_window=tw, t_max=4), f"trim window {tw} fallback")
    _check(gpu, orc, synth.lattice(8), 12, gpu.params(trim_window=tw, layers=1), f"lattice window {tw}")


@pytest.mark.parametrize("seed", [0, 99, 0xFFFFFFFF])
def test_random_member_selection(gpu, orc, seed):
    # the "RA" strategy of Table 6: a random member per voxel instead of the
    # centre-closest one; the search, trim and pad are unchanged
    x = synth.scene_planes_blobs(80000, seed=31)
    p = gpu.params(select=gpu.SELECT_RANDOM, select_seed=seed)
    got, _ = _check(gpu, orc, x, 20000, p, f"random member seed {seed}")
    cc, _ = _check(gpu, orc, x, 20000, gpu.params(), "centre-closest")
    assert not np.array_equal(got, cc)
    _check(gpu, orc, x, 5000, gpu.params(select=gpu.SELECT_RANDOM, select_seed=seed, fixed_voxel=0.7),
           "random member fixed voxel (RVS-like)")
    _check(gpu, orc, synth.lattice(8), 60, p, "random member lattice")


def _check_points(gpu, orc, x, M, p, label):
    _note(f"case points {label} N={x.shape[0]} M={M} select={p.select}")
    st, want_idx, want_pts, winfo = orc.sample_points(x, M, _oracle_params(orc, p))
    assert st == 0
    idx, pts, info = gpu.Sampler().sample_points(_to_dev(x), M, p, with_info=True)
    assert info == winfo, (info, winfo)
    assert np.array_equal(idx.cpu().numpy(), want_idx)
    got = pts.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want_pts.view(np.uint32))  # bit for bit
    return got


@pytest.mark.parametrize("sel", [2, 3])
def test_centre_and_mean_points(gpu, orc, sel):
    x = synth.scene_planes_blobs(70000, seed=41)
    _check_points(gpu, orc, x, 17500, gpu.params(select=sel), "scene")
    _check_points(gpu, orc, x, 3000, gpu.params(select=sel, layers=3), "scene 3 layers")
    _check_points(gpu, orc, x, 6000, gpu.params(select=sel, t_max=3), "fallback (trim or pad)")
    _check_points(gpu, orc, x, 2000, gpu.params(select=sel, fixed_voxel=0.6), "fixed voxel")
    lat = synth.lattice(8) + np.float32(10.25)
    got = _check_points(gpu, orc, lat, 64, gpu.params(select=sel, layers=1, fixed_voxel=2.0), "lattice")
    assert np.all(np.mod(got - (11.25 if sel == 2 else 10.75), 2.0) == 0.0)
    q = synth.random_cloud(20000, 5, kind="quantised")
    _check_points(gpu, orc, q, 9000, gpu.params(select=sel), "quantised (duplicates, pad)")
    _check_points(gpu, orc, q, 20000, gpu.params(select=sel), "identity")


def test_points_modes_rejected_elsewhere(gpu):
    import torch
    x = _to_dev(synth.random_cloud(1000, 1))
    with pytest.raises(gpu.HavError):
        gpu.Sampler().sample(x, 100, gpu.params(select=gpu.SELECT_MEAN))


@pytest.mark.parametrize("sel", [0, 1])
def test_points_of_point_selections(gpu, orc, sel):
    # centre-closest and random members stand for themselves
    x = synth.scene_planes_blobs(30000, seed=43)
    got = _check_points(gpu, orc, x, 7000, gpu.params(select=sel, select_seed=5), "self")
    st, idx, _ = orc.sample(x, 7000, orc.params(select=sel, seed=5))
    assert np.array_equal(got, x[idx])
