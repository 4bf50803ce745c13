"""C-ABI checks that need no GPU: the library loads, exports every function the header
declares, its struct layouts match the Python binding, and host-checkable argument
errors are rejected before anything is enqueued."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"#.*", "", text)
        for m in re.finditer(r"\b(hav_\w+)\s*\(", text):
            names.append(m.group(1))
    return sorted(set(names))


@pytest.fixture(scope="module")
def hav():
    from paper_2305_14306_amd import hav as h
    h.lib()
    return h


def test_exports_every_declared_symbol(hav):
    names = _declared_functions()
    assert "hav_sample" in names and "hav_sample_chain" in names
    for n in names:
        assert hasattr(hav.lib(), n), n


def test_struct_layout_matches_header(hav, tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "hav.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(hav_params_t), offsetof(hav_params_t, sigma),
         offsetof(hav_params_t, flags), offsetof(hav_params_t, fixed_voxel), sizeof(hav_info_t));
  printf("%zu %zu %zu %zu %zu\n", offsetof(hav_info_t, m), offsetof(hav_info_t, count),
         offsetof(hav_info_t, padded), offsetof(hav_params_t, table_scale),
         offsetof(hav_params_t, bin_points));
  return 0;
}
''')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", HEADER_DIR, "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    P, I = hav.Params, hav.Info
    want = [C.sizeof(P), P.sigma.offset, P.flags.offset, P.fixed_voxel.offset, C.sizeof(I),
            I.m.offset, I.count.offset, I.padded.offset, P.table_scale.offset, P.bin_points.offset]
    assert [int(x) for x in out] == want


def test_params_default(hav):
    p = hav.lib().hav_params_default()
    assert p.abi_version == hav.ABI_VERSION
    assert (p.layers, p.layer_ratio, p.t_max, p.flags) == (2, 4, 20, 0)
    assert p.sigma == 0.05 and list(p.aspect) == [1.0, 1.0, 1.0]
    assert p.table_scale == 0


def test_status_strings(hav):
    for s in range(9):
        assert isinstance(hav.status_string(s), str) and hav.status_string(s)
    assert hav.status_string(99) == "unknown status"


def test_workspace_size(hav):
    p = hav.params()
    a = hav.workspace_size(16384, 4096, p)
    b = hav.workspace_size(1 << 20, 1 << 18, p)
    assert 0 < a < b
    # table_scale doubles the table slots per step (a tuning field: speed, never results)
    assert hav.workspace_size(1 << 20, 1 << 18, hav.params(table_scale=1)) > b
    assert hav.workspace_size(0, 1, p) == 0
    assert hav.workspace_size(10, 11, p) == 0
    assert hav.workspace_size(10, 0, p) == 0
    assert hav.workspace_size(1 << 31, 10, p) == 0
    bad = hav.params(layers=9)
    assert hav.workspace_size(100, 10, bad) == 0
    assert hav.chain_workspace_size(1000, [500, 100], p) > hav.workspace_size(1000, 500, p)
    assert hav.chain_workspace_size(1000, [100, 500], p) == 0  # stages must shrink


def _call(hav, xyz=0x10000, N=100, M=10, p=None, idx=0x20000, ws=0x30000, ws_bytes=1 << 30,
          info=None):
    p = p if p is not None else hav.params()
    return hav.lib().hav_sample(C.c_void_p(xyz), N, M, C.byref(p) if p is not False else None,
                                C.c_void_p(idx), C.c_void_p(ws), ws_bytes, info, None)


def test_host_rejects_bad_arguments(hav):
    # every case below must be rejected on the host: nothing is launched, so the
    # fake device addresses are never touched
    E = hav.ERR_INVALID_ARG
    assert _call(hav, xyz=0) == E
    assert _call(hav, idx=0) == E
    assert _call(hav, ws=0) == E
    assert _call(hav, M=0) == E
    assert _call(hav, M=101) == E
    assert _call(hav, N=0, M=0) == E
    assert _call(hav, N=1 << 31, M=5) == E
    assert _call(hav, ws=0x30010) == E  # misaligned workspace
    assert _call(hav, p=False) == E
    for kw in (dict(layers=0), dict(layers=9), dict(layer_ratio=1), dict(layer_ratio=17),
               dict(t_max=0), dict(t_max=21), dict(sigma=-1.0), dict(sigma=float("nan")),
               dict(aspect=(1.0, 0.0, 1.0)), dict(aspect=(1.0, float("inf"), 1.0)),
               dict(fixed_voxel=0.0), dict(fixed_voxel=float("nan")), dict(spec_depth=8),
               dict(spec_depth=-1), dict(spec_budget=-1), dict(spec_budget=1025),
               dict(search_blocks=-1), dict(search_blocks=65537), dict(table_scale=-1),
               dict(table_scale=4), dict(bin_points=1000), dict(bin_points=16384),
               dict(trim_window=64.5), dict(trim_window=float("nan")), dict(trim_window=float("inf")),
               dict(select=2), dict(select=-1)):
        assert _call(hav, p=hav.params(**kw)) == E, kw
    p = hav.params()
    p.abi_version = 2
    assert _call(hav, p=p) == E
    p = hav.params()
    p.flags = 2
    assert _call(hav, p=p) == E
    need = hav.workspace_size(100, 10)
    assert _call(hav, ws_bytes=need - 1) == hav.ERR_WORKSPACE_TOO_SMALL


def test_chain_host_rejects_bad_arguments(hav):
    p = hav.params()
    L = hav.lib()

    def call(Ms, ws_bytes=1 << 30, N=1000):
        arr = (C.c_int64 * len(Ms))(*Ms)
        return L.hav_sample_chain(C.c_void_p(0x10000), N, arr, len(Ms), C.byref(p),
                                  C.c_void_p(0x20000), C.c_void_p(0x30000), ws_bytes, None, None)

    assert call([2000]) == hav.ERR_INVALID_ARG
    assert call([500, 600]) == hav.ERR_INVALID_ARG
    assert call([500, 0]) == hav.ERR_INVALID_ARG
    assert call([500, 100], ws_bytes=10) == hav.ERR_WORKSPACE_TOO_SMALL


def test_binding_refuses_cpu_tensors(hav):
    import torch
    with pytest.raises(ValueError):
        hav.sample(torch.zeros(10, 3), 5)


def test_batch_workspace_size(hav):
    p = hav.params()
    one = hav.workspace_size(10000, 100, p)
    both = hav.batch_workspace_size([10000, 20000], [100, 200], p)
    assert both > one + hav.workspace_size(20000, 200, p)
    assert hav.batch_workspace_size([10000], None, p) > 0
    assert hav.batch_workspace_size([10000, 0], None, p) == 0
    assert hav.batch_workspace_size([10000, 5], [100, 6], p) == 0  # M > N
    assert hav.batch_workspace_size([], None, p) == 0
    assert hav.batch_workspace_size([1 << 30], None, p) == 0


def test_batch_host_rejects_bad_arguments(hav):
    p = hav.params()
    L = hav.lib()
    E = hav.ERR_INVALID_ARG

    def call(offs, Ms, ws_bytes=1 << 30, ws=0x30000):
        o = (C.c_int64 * len(offs))(*offs)
        m = (C.c_int64 * len(Ms))(*Ms)
        return L.hav_sample_batch(C.c_void_p(0x10000), o, m, len(Ms), C.byref(p), C.c_void_p(0x20000),
                                  C.c_void_p(ws), ws_bytes, None, None)

    assert call([1, 10, 20], [5, 5]) == E          # offsets must start at 0
    assert call([0, 10, 5], [5, 5]) == E           # a negative cloud size
    assert call([0, 10, 20], [5, 11]) == E         # M > N
    assert call([0, 10, 20], [0, 5]) == E          # M = 0
    assert call([0, 10, 20], [5, 5], ws=0x30010) == E
    assert call([0, 10, 20], [5, 5], ws_bytes=100) == hav.ERR_WORKSPACE_TOO_SMALL


def test_server_create_rejects_bad_arguments(hav):
    # rejected before any device call
    L = hav.lib()
    p = hav.params()
    assert not L.hav_server_create(1 << 30, 0, 2, C.byref(p))
    assert not L.hav_server_create(1 << 30, 2000, 2, C.byref(p))
    assert not L.hav_server_create(1 << 30, 16, 0, C.byref(p))
    assert not L.hav_server_create(1 << 30, 16, 9, C.byref(p))
    bad = hav.params(layers=0)
    assert not L.hav_server_create(1 << 30, 16, 2, C.byref(bad))
    t = C.c_uint64(0)
    assert L.hav_server_submit(None, C.c_void_p(0x1000), 10, 5, C.byref(t)) == hav.ERR_INVALID_ARG
    assert L.hav_server_poll(None, 1, None, None, None) == hav.ERR_INVALID_ARG


def test_comparators_reject_bad_arguments(hav):
    L = hav.lib()
    buf = C.create_string_buffer(1 << 16)
    ptr = C.addressof(buf)
    assert L.hav_fps_workspace_size(0) == 0
    assert L.hav_fps_workspace_size(hav.lib().hav_fps_workspace_size(1)) > 0
    ws = L.hav_fps_workspace_size(100)
    for args in [(0, 100, 10, 0, ptr, ptr, ws, 0),          # no xyz
                 (ptr, 100, 0, 0, ptr, ptr, ws, 0),         # M < 1
                 (ptr, 100, 101, 0, ptr, ptr, ws, 0),       # M > N
                 (ptr, 100, 10, 100, ptr, ptr, ws, 0),      # start out of range
                 (ptr, 100, 10, 0, ptr, ptr, ws, 257),      # too many blocks
                 (ptr, 1 << 21, 10, 0, ptr, ptr, ws, 0),    # above HAV_FPS_MAX_POINTS
                 (ptr, 20000, 10, 0, ptr, ptr, ws, 1)]:     # one block cannot hold it
        assert L.hav_fps(*args, None) == 1, args
    assert L.hav_fps(ptr, 100, 10, 0, ptr, ptr, 8, 0, None) == 2
    assert L.hav_rps_workspace_size(0) == 0
    rw = L.hav_rps_workspace_size(1000)
    assert rw > 0
    for args in [(1000, 0, 1, 0.0, ptr, ptr, rw), (1000, 1001, 1, 0.0, ptr, ptr, rw),
                 (1000, 10, 1, float("nan"), ptr, ptr, rw), (1000, 10, 1, 65.0, ptr, ptr, rw),
                 (1000, 10, 1, 0.0, 0, ptr, rw)]:
        assert L.hav_rps(*args, None) == 1, args
    assert L.hav_rps(1000, 10, 1, 0.0, ptr, ptr, 16, None) == 2


def test_nearest_sample_rejects_bad_arguments(hav):
    L = hav.lib()
    buf = C.create_string_buffer(1 << 16)
    ptr = C.addressof(buf)
    assert L.hav_nn_workspace_size(0) == 0
    ws = L.hav_nn_workspace_size(100)
    assert ws > 0
    for args in [(0, 100, ptr, 10, 0, ptr, ptr, ptr, ws),      # no samples
                 (ptr, 0, ptr, 10, 0, ptr, ptr, ptr, ws),      # M < 1
                 (ptr, 100, ptr, 0, 0, ptr, ptr, ptr, ws),     # Q < 1
                 (ptr, 100, ptr, 99, 1, ptr, ptr, ptr, ws),    # self needs Q == M
                 (ptr, 1, ptr, 1, 1, ptr, ptr, ptr, ws),       # self needs M >= 2
                 (ptr, 100, ptr, 10, 0, ptr, 0, ptr, ws)]:     # no max output
        assert L.hav_nn(*args, None) == 1, args
    assert L.hav_nn(ptr, 100, ptr, 10, 0, ptr, ptr, ptr, 64, None) == 2


def test_ball_query_rejects_bad_arguments(hav):
    L = hav.lib()
    buf = C.create_string_buffer(1 << 16)
    ptr = C.addressof(buf)
    ws = L.hav_ball_workspace_size(100)
    assert ws > 0 and L.hav_ball_workspace_size(0) == 0
    for args in [(0, 100, ptr, 10, 1.0, 8, ptr, ptr, ptr, ws),              # no points
                 (ptr, 100, ptr, 0, 1.0, 8, ptr, ptr, ptr, ws),             # Q < 1
                 (ptr, 100, ptr, 10, 0.0, 8, ptr, ptr, ptr, ws),            # radius 0
                 (ptr, 100, ptr, 10, float("nan"), 8, ptr, ptr, ptr, ws),   # radius NaN
                 (ptr, 100, ptr, 10, 1.0, 0, ptr, ptr, ptr, ws),            # K < 1
                 (ptr, 100, ptr, 10, 1.0, 65, ptr, ptr, ptr, ws)]:          # K > 64
        assert L.hav_ball_query(*args, None) == 1, args
    assert L.hav_ball_query(ptr, 100, ptr, 10, 1.0, 8, ptr, ptr, ptr, 64, None) == 2


def test_workspace_footprint(hav):
    # tables sized from N: a 16,384-point cloud needs at most 32 MiB, a 1M-point one at
    # most 320 MiB (27x its 12 MiB cloud)
    assert hav.workspace_size(16384, 4096) <= 32 << 20
    assert hav.workspace_size(1 << 20, 1 << 18) <= 320 << 20


def test_static_entry_rejects_on_the_host(hav):
    # argument errors and sizes the library's own workspace cannot hold are refused
    # before anything is enqueued (fake device addresses, never touched)
    lib = hav.lib()

    def call(N=100, M=10, p=None, xyz=0x10000, idx=0x20000):
        p = p if p is not None else hav.params()
        return lib.hav_sample_static(C.c_void_p(xyz), N, M, C.byref(p), C.c_void_p(idx), None, None)

    assert call(xyz=0) == hav.ERR_INVALID_ARG
    assert call(idx=0) == hav.ERR_INVALID_ARG
    assert call(M=101) == hav.ERR_INVALID_ARG
    assert call(p=hav.params(select=3)) == hav.ERR_INVALID_ARG
    assert call(N=hav.STATIC_MAX_POINTS + 1) == hav.ERR_WORKSPACE_TOO_SMALL
    assert call(p=hav.params(spec_depth=7)) == hav.ERR_WORKSPACE_TOO_SMALL
    assert call(p=hav.params(table_scale=1)) == hav.ERR_WORKSPACE_TOO_SMALL


def test_sampled_ball_query_rejects_on_the_host(hav):
    lib = hav.lib()
    p = hav.params()

    def call(N=100, M=10, r=0.5, K=8, ws_bytes=1 << 30, ws=0x30000, idx=0x20000):
        return lib.hav_ball_query_sampled(C.c_void_p(0x10000), N, C.c_void_p(idx), M, r, K,
                                          C.c_void_p(0x40000), None, C.c_void_p(ws), ws_bytes,
                                          C.byref(p), None)

    E = hav.ERR_INVALID_ARG
    assert call(idx=0) == E
    assert call(M=0) == E
    assert call(M=101) == E
    assert call(K=0) == E
    assert call(K=65) == E
    assert call(r=0.0) == E
    assert call(r=float("inf")) == E
    assert call(ws=0x30010) == E
    assert call(ws_bytes=hav.workspace_size(100, 10) - 1) == hav.ERR_WORKSPACE_TOO_SMALL
