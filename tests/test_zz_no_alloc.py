"""hav_sample_static (the entry point that allocates nothing: its workspace is the
library's own device array) against hav_sample with a caller workspace, through the C
ABI: bit-identical indices and reports on two calls in a row, the second on a smaller
cloud, then a larger one again; sizes above the array's limit are refused."""
import ctypes as C
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


def _static(gpu, xd, M, p):
    import torch
    idx = torch.full((M,), -1, dtype=torch.int32, device="cuda")
    info = torch.zeros(C.sizeof(gpu.Info), dtype=torch.uint8, device="cuda")
    st = gpu.lib().hav_sample_static(C.c_void_p(xd.data_ptr()), xd.shape[0], M, C.byref(p),
                                     C.c_void_p(idx.data_ptr()), C.c_void_p(info.data_ptr()),
                                     gpu._stream_ptr())
    assert st == gpu.OK, st
    return idx.cpu().numpy(), gpu.read_info(info)[0]


def test_static_equals_workspace_call(gpu, orc):
    import torch
    cases = [(synth.uniform_box_with_ground(16384, seed=1), 4096, {}),
             (synth.random_cloud(5001, 7, scale=30.0, kind="clustered"), 1250, {}),
             (synth.lidar_points(32768, seed=5), 8192, {"spec_depth": 2}),
             (synth.random_cloud(3000, 8, kind="quantised"), 700, {"select": 1, "select_seed": 5})]
    for i, (x, M, kw) in enumerate(cases):
        _note(f"case static call {i} N={x.shape[0]} M={M} {kw}")
        p = gpu.params(**kw)
        xd = torch.from_numpy(x).cuda()
        got, info = _static(gpu, xd, M, p)
        want, winfo = gpu.Sampler().sample(xd, M, p, with_info=True)
        assert info["status"] == 0
        assert info == winfo, (info, winfo)
        assert np.array_equal(got, want.cpu().numpy()), i
        if i == 0:
            assert np.array_equal(got, orc.sample(x, M)[1])


def test_static_rejects_what_does_not_fit(gpu):
    import torch
    x = torch.from_numpy(synth.random_cloud(gpu.STATIC_MAX_POINTS + 1, 3)).cuda()
    idx = torch.empty(100, dtype=torch.int32, device="cuda")
    p = gpu.params()
    st = gpu.lib().hav_sample_static(C.c_void_p(x.data_ptr()), x.shape[0], 100, C.byref(p),
                                     C.c_void_p(idx.data_ptr()), None, gpu._stream_ptr())
    assert st == gpu.ERR_WORKSPACE_TOO_SMALL
    p = gpu.params(spec_depth=7)
    st = gpu.lib().hav_sample_static(C.c_void_p(x.data_ptr()), 1000, 100, C.byref(p),
                                     C.c_void_p(idx.data_ptr()), None, gpu._stream_ptr())
    assert st == gpu.ERR_WORKSPACE_TOO_SMALL
