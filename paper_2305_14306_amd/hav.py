"""ctypes binding of libhav.so (include/hav.h). Argument marshalling only.

PyTorch supplies device memory and the current stream; every step of the sampler runs
in the library's HIP kernels. If the library has not been built this module raises on
first use: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhav.so")

ABI_VERSION = 1
MAX_LAYERS = 8
FIXED_VOXEL = 1
SELECT_CENTRE_CLOSEST = 0
SELECT_RANDOM = 1
SELECT_CENTRE = 2
SELECT_MEAN = 3

OK, ERR_INVALID_ARG, ERR_WORKSPACE_TOO_SMALL, ERR_OUT_OF_MEMORY, ERR_UNSUPPORTED, \
    ERR_NONFINITE, ERR_HIP, ERR_WORKSPACE_NOT_INIT, NOT_READY = range(9)


class Params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32),
        ("layers", C.c_int32),
        ("layer_ratio", C.c_int32),
        ("t_max", C.c_int32),
        ("sigma", C.c_double),
        ("aspect", C.c_float * 3),
        ("flags", C.c_uint32),
        ("fixed_voxel", C.c_float * 3),
        ("spec_depth", C.c_int32),
        ("spec_budget", C.c_int32),
        ("search_blocks", C.c_int32),
        ("trim_window", C.c_float),
        ("select", C.c_int32),
        ("select_seed", C.c_uint32),
        ("table_scale", C.c_int32),
        ("bin_points", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("layers", C.c_int32),
        ("hi0", C.c_float),
        ("mn", C.c_float * 3),
        ("mx", C.c_float * 3),
        ("m", C.c_int32 * MAX_LAYERS),
        ("s", C.c_float * MAX_LAYERS),
        ("evals", C.c_int32 * MAX_LAYERS),
        ("count", C.c_int32 * MAX_LAYERS),
        ("accepted", C.c_int32 * MAX_LAYERS),
        ("trimmed", C.c_int32 * MAX_LAYERS),
        ("padded", C.c_int32 * MAX_LAYERS),
    ]

    def as_dict(self) -> dict:
        L = self.layers
        return {
            "status": self.status,
            "layers": L,
            "hi0": self.hi0,
            "mn": list(self.mn),
            "m": list(self.m)[:L],
            "s": list(self.s)[:L],
            "evals": list(self.evals)[:L],
            "count": list(self.count)[:L],
            "accepted": list(self.accepted)[:L],
            "trimmed": list(self.trimmed)[:L],
            "padded": list(self.padded)[:L],
        }


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "completed", "batches", "max_batch_seen", "slots",
                                         "slots_created", "evictions", "points_done")] + \
               [("hbm_used", C.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class HavError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})" if what else status_string(status))


_lib = None


def lib():
    """Load libhav.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2305_14306_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i64p, i32p = C.c_void_p, C.POINTER(C.c_int64), C.c_void_p
        L.hav_params_default.restype = Params
        L.hav_params_default.argtypes = []
        L.hav_status_string.restype = C.c_char_p
        L.hav_status_string.argtypes = [C.c_int]
        L.hav_workspace_size.restype = C.c_size_t
        L.hav_workspace_size.argtypes = [C.c_int64, C.c_int64, C.POINTER(Params)]
        L.hav_workspace_init.restype = C.c_int
        L.hav_workspace_init.argtypes = [C.c_int64, C.POINTER(Params), vp, C.c_size_t, vp]
        L.hav_sample.restype = C.c_int
        L.hav_sample.argtypes = [vp, C.c_int64, C.c_int64, C.POINTER(Params), i32p, vp, C.c_size_t,
                                 vp, vp]
        L.hav_sample_static.restype = C.c_int
        L.hav_sample_static.argtypes = [vp, C.c_int64, C.c_int64, C.POINTER(Params), i32p, vp, vp]
        L.hav_sample_points.restype = C.c_int
        L.hav_sample_points.argtypes = [vp, C.c_int64, C.c_int64, C.POINTER(Params), i32p, vp, vp,
                                        C.c_size_t, vp, vp]
        L.hav_chain_workspace_size.restype = C.c_size_t
        L.hav_chain_workspace_size.argtypes = [C.c_int64, i64p, C.c_int32, C.POINTER(Params)]
        L.hav_sample_chain.restype = C.c_int
        L.hav_sample_chain.argtypes = [vp, C.c_int64, i64p, C.c_int32, C.POINTER(Params), i32p, vp,
                                       C.c_size_t, vp, vp]
        L.hav_batch_workspace_size.restype = C.c_size_t
        L.hav_batch_workspace_size.argtypes = [C.c_int32, i64p, i64p, C.POINTER(Params)]
        L.hav_batch_workspace_init.restype = C.c_int
        L.hav_batch_workspace_init.argtypes = [C.c_int32, i64p, C.POINTER(Params), vp, C.c_size_t, vp]
        L.hav_sample_batch.restype = C.c_int
        L.hav_sample_batch.argtypes = [vp, i64p, i64p, C.c_int32, C.POINTER(Params), i32p, vp,
                                       C.c_size_t, vp, vp]
        L.hav_server_create.restype = C.c_void_p
        L.hav_server_create.argtypes = [C.c_size_t, C.c_int32, C.c_int32, C.POINTER(Params)]
        L.hav_server_submit.restype = C.c_int
        L.hav_server_submit.argtypes = [vp, vp, C.c_int64, C.c_int64, C.POINTER(C.c_uint64)]
        L.hav_server_poll.restype = C.c_int
        L.hav_server_poll.argtypes = [vp, C.c_uint64, vp, C.POINTER(Info), C.POINTER(C.c_double)]
        L.hav_server_stats.restype = C.c_int
        L.hav_server_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.hav_server_destroy.restype = None
        L.hav_server_destroy.argtypes = [vp]
        L.hav_graph_capture_begin.restype = C.c_int
        L.hav_graph_capture_begin.argtypes = [vp]
        L.hav_graph_capture_end.restype = C.c_int
        L.hav_graph_capture_end.argtypes = [vp, C.POINTER(C.c_void_p)]
        L.hav_graph_launch.restype = C.c_int
        L.hav_graph_launch.argtypes = [vp, vp]
        L.hav_graph_destroy.restype = None
        L.hav_graph_destroy.argtypes = [vp]
        L.hav_fps_workspace_size.restype = C.c_size_t
        L.hav_fps_workspace_size.argtypes = [C.c_int64]
        L.hav_fps.restype = C.c_int
        L.hav_fps.argtypes = [vp, C.c_int64, C.c_int64, C.c_int64, i32p, vp, C.c_size_t, C.c_int32, vp]
        L.hav_fps_error.restype = C.c_int
        L.hav_fps_error.argtypes = [vp, C.POINTER(C.c_uint32)]
        L.hav_rps_workspace_size.restype = C.c_size_t
        L.hav_rps_workspace_size.argtypes = [C.c_int64]
        L.hav_rps_workspace_init.restype = C.c_int
        L.hav_rps_workspace_init.argtypes = [vp, C.c_size_t, C.c_int64, vp]
        L.hav_rps.restype = C.c_int
        L.hav_rps.argtypes = [C.c_int64, C.c_int64, C.c_uint64, C.c_float, i32p, vp, C.c_size_t, vp]
        L.hav_nn_workspace_size.restype = C.c_size_t
        L.hav_nn_workspace_size.argtypes = [C.c_int64]
        L.hav_nn_workspace_init.restype = C.c_int
        L.hav_nn_workspace_init.argtypes = [vp, C.c_size_t, C.c_int64, vp]
        L.hav_nn.restype = C.c_int
        L.hav_nn.argtypes = [vp, C.c_int64, vp, C.c_int64, C.c_int32, vp, vp, vp, C.c_size_t, vp]
        L.hav_ball_workspace_size.restype = C.c_size_t
        L.hav_ball_workspace_size.argtypes = [C.c_int64]
        L.hav_ball_workspace_init.restype = C.c_int
        L.hav_ball_workspace_init.argtypes = [vp, C.c_size_t, C.c_int64, vp]
        L.hav_ball_query.restype = C.c_int
        L.hav_ball_query.argtypes = [vp, C.c_int64, vp, C.c_int64, C.c_float, C.c_int32, vp, vp, vp,
                                     C.c_size_t, vp]
        L.hav_ball_query_sampled.restype = C.c_int
        L.hav_ball_query_sampled.argtypes = [vp, C.c_int64, vp, C.c_int64, C.c_float, C.c_int32, vp, vp,
                                             vp, C.c_size_t, C.POINTER(Params), vp]
        L.hav_debug_scan_spin_limit.restype = C.c_int
        L.hav_debug_scan_spin_limit.argtypes = [C.c_uint32]
        L.hav_debug_search_spin_limit.restype = C.c_int
        L.hav_debug_search_spin_limit.argtypes = [C.c_uint32]
        L.hav_timing_enable.restype = C.c_int
        L.hav_timing_enable.argtypes = [C.c_int32]
        L.hav_timing_collect.restype = C.c_int
        L.hav_timing_collect.argtypes = [C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        _lib = L
    return _lib


def debug_scan_spin_limit(limit: int) -> None:
    """Test hook: polls before a tag scan's wait gives up on the current device (0 =
    default). Lets tests drive the scans' failure path from the host."""
    st = lib().hav_debug_scan_spin_limit(int(limit))
    if st != OK:
        raise HavError(st, "hav_debug_scan_spin_limit")


def debug_search_spin_limit(limit: int) -> None:
    """Test hook: polls before a voxel-search wait for a pass gives up on the current
    device (0 = default). Lets tests drive the search's failure path from the host."""
    st = lib().hav_debug_search_spin_limit(int(limit))
    if st != OK:
        raise HavError(st, "hav_debug_search_spin_limit")


def timing_enable(on: bool = True) -> None:
    """Bracket every library kernel launch with HIP events on its stream."""
    lib().hav_timing_enable(1 if on else 0)


def timing_collect(kernel: str):
    """(launches, total_ms) of the kept event pairs of one kernel; waits for them."""
    n, ms = C.c_int32(0), C.c_double(0.0)
    st = lib().hav_timing_collect(kernel.encode(), C.byref(n), C.byref(ms))
    if st != OK:
        raise HavError(st, "hav_timing_collect")
    return n.value, ms.value


def status_string(status: int) -> str:
    return lib().hav_status_string(int(status)).decode()


def params(layers=2, layer_ratio=4, t_max=20, sigma=0.05, aspect=(1.0, 1.0, 1.0),
           fixed_voxel=None, spec_depth=0, spec_budget=0, search_blocks=0,
           trim_window=0.0, select=0, select_seed=0, table_scale=0, bin_points=0) -> Params:
    p = lib().hav_params_default()
    p.layers, p.layer_ratio, p.t_max, p.sigma = layers, layer_ratio, t_max, sigma
    p.spec_depth, p.spec_budget, p.search_blocks = spec_depth, spec_budget, search_blocks
    p.trim_window = trim_window
    p.select, p.select_seed = select, select_seed
    p.table_scale = table_scale
    p.bin_points = bin_points
    for a in range(3):
        p.aspect[a] = aspect[a]
    if fixed_voxel is not None:
        p.flags |= FIXED_VOXEL
        fv = fixed_voxel if hasattr(fixed_voxel, "__len__") else (fixed_voxel,) * 3
        for a in range(3):
            p.fixed_voxel[a] = fv[a]
    return p


def workspace_size(N: int, M: int, p: Params | None = None) -> int:
    p = p if p is not None else params()
    return int(lib().hav_workspace_size(int(N), int(M), C.byref(p)))


def chain_workspace_size(N: int, Ms, p: Params | None = None) -> int:
    p = p if p is not None else params()
    arr = (C.c_int64 * len(Ms))(*[int(m) for m in Ms])
    return int(lib().hav_chain_workspace_size(int(N), arr, len(Ms), C.byref(p)))


def _i64(values):
    vals = [int(v) for v in values]
    return (C.c_int64 * len(vals))(*vals)


def batch_workspace_size(Ns, Ms=None, p: Params | None = None) -> int:
    p = p if p is not None else params()
    return int(lib().hav_batch_workspace_size(len(Ns), _i64(Ns), _i64(Ms) if Ms is not None else None,
                                              C.byref(p)))


def _torch():
    import torch
    return torch


def _check_xyz(xyz):
    torch = _torch()
    if not (isinstance(xyz, torch.Tensor) and xyz.is_cuda and xyz.dtype == torch.float32
            and xyz.dim() == 2 and xyz.shape[1] == 3 and xyz.is_contiguous()):
        raise ValueError("xyz must be a contiguous float32 CUDA tensor of shape [N, 3]")


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def read_info(info_dev, n: int = 1):
    """Copy device hav_info_t records to the host (synchronises with the stream)."""
    raw = info_dev.cpu().numpy().tobytes()
    size = C.sizeof(Info)
    return [Info.from_buffer_copy(raw[j * size:(j + 1) * size]).as_dict() for j in range(n)]


class Sampler:
    """Reusable caller-side state: a device workspace (grown on demand and initialised
    with hav_workspace_init whenever the problem size or speculation depth changes) and
    an info record, so repeated calls on one stream allocate and clear nothing."""

    def __init__(self, device="cuda"):
        self.device = device
        self.ws = None
        self.ws_key = None
        self.info = None
        self._n_info = 0

    def _workspace(self, nbytes: int, N, p: Params, stream=None):
        """N: a point count (single clouds and chains) or a tuple of counts (batches)."""
        torch = _torch()
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            self.ws_key = None
        pmode = int(p.select) if int(p.select) >= SELECT_CENTRE else 0  # layout differs
        key = (N if isinstance(N, tuple) else int(N), int(p.spec_depth), pmode, int(p.table_scale),
               int(p.bin_points))
        if self.ws_key != key:
            if isinstance(N, tuple):
                st = lib().hav_batch_workspace_init(len(N), _i64(N), C.byref(p),
                                                    C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                                    _stream_ptr(stream))
            else:
                st = lib().hav_workspace_init(int(N), C.byref(p), C.c_void_p(self.ws.data_ptr()),
                                              self.ws.numel(), _stream_ptr(stream))
            if st != OK:
                raise HavError(st, "workspace init")
            self.ws_key = key
        return self.ws

    def invalidate(self):
        """Forget the initialisation (call after writing into the workspace)."""
        self.ws_key = None

    def _info(self, n: int):
        torch = _torch()
        if self.info is None or self.info.numel() < n * C.sizeof(Info):
            self.info = torch.zeros(n * C.sizeof(Info), dtype=torch.uint8, device=self.device)
        return self.info

    def _read(self, n: int):
        """The reports of the last call (waits for it). A status that leaves the workspace
        needing initialisation (a search wait that gave up, a workspace set up for
        another size) makes the next call initialise it again."""
        out = read_info(self.info[:n * C.sizeof(Info)], n)
        if any(r["status"] in (ERR_HIP, ERR_WORKSPACE_NOT_INIT) for r in out):
            self.ws_key = None
        return out

    def check(self):
        """Wait for the last call on this Sampler and raise HavError if the device
        reported an error for it (non-finite input, an unsupported frame, a workspace
        that was not initialised, a wait that gave up). Returns its reports."""
        out = self._read(self._n_info)
        for r in out:
            if r["status"] != OK:
                raise HavError(r["status"], "device")
        return out

    def sample(self, xyz, M: int, p: Params | None = None, out=None, with_info: bool = False,
               stream=None):
        torch = _torch()
        _check_xyz(xyz)
        p = p if p is not None else params()
        N = xyz.shape[0]
        nbytes = workspace_size(N, M, p)
        if nbytes == 0:
            raise HavError(ERR_INVALID_ARG, "hav_workspace_size")
        ws = self._workspace(nbytes, N, p, stream)
        idx = out if out is not None else torch.empty(int(M), dtype=torch.int32, device=xyz.device)
        info = self._info(1)
        st = lib().hav_sample(C.c_void_p(xyz.data_ptr()), N, int(M), C.byref(p),
                              C.c_void_p(idx.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                              C.c_void_p(info.data_ptr()), _stream_ptr(stream))
        if st != OK:
            raise HavError(st, "hav_sample")
        self._n_info = 1
        if with_info:
            return idx, self._read(1)[0]
        return idx

    def sample_points(self, xyz, M: int, p: Params, with_info: bool = False, stream=None):
        """hav_sample_points: (idx [M] int32, pts [M, 3] float32), pts[j] standing for
        idx[j] (voxel centre / mean with select SELECT_CENTRE / SELECT_MEAN)."""
        torch = _torch()
        _check_xyz(xyz)
        N = xyz.shape[0]
        nbytes = workspace_size(N, M, p)
        if nbytes == 0:
            raise HavError(ERR_INVALID_ARG, "hav_workspace_size")
        ws = self._workspace(nbytes, N, p, stream)
        idx = torch.empty(int(M), dtype=torch.int32, device=xyz.device)
        pts = torch.empty((int(M), 3), dtype=torch.float32, device=xyz.device)
        info = self._info(1)
        st = lib().hav_sample_points(C.c_void_p(xyz.data_ptr()), N, int(M), C.byref(p),
                                     C.c_void_p(idx.data_ptr()), C.c_void_p(pts.data_ptr()),
                                     C.c_void_p(ws.data_ptr()), ws.numel(),
                                     C.c_void_p(info.data_ptr()), _stream_ptr(stream))
        if st != OK:
            raise HavError(st, "hav_sample_points")
        self._n_info = 1
        if with_info:
            return idx, pts, self._read(1)[0]
        return idx, pts

    def chain(self, xyz, Ms, p: Params | None = None, out=None, with_info: bool = False,
              stream=None):
        torch = _torch()
        _check_xyz(xyz)
        p = p if p is not None else params()
        N = xyz.shape[0]
        nbytes = chain_workspace_size(N, Ms, p)
        if nbytes == 0:
            raise HavError(ERR_INVALID_ARG, "hav_chain_workspace_size")
        ws = self._workspace(nbytes, N, p, stream)
        total = int(sum(int(m) for m in Ms))
        idx = out if out is not None else torch.empty(total, dtype=torch.int32, device=xyz.device)
        info = self._info(len(Ms))
        arr = (C.c_int64 * len(Ms))(*[int(m) for m in Ms])
        st = lib().hav_sample_chain(C.c_void_p(xyz.data_ptr()), N, arr, len(Ms), C.byref(p),
                                    C.c_void_p(idx.data_ptr()), C.c_void_p(ws.data_ptr()),
                                    ws.numel(), C.c_void_p(info.data_ptr()), _stream_ptr(stream))
        if st != OK:
            raise HavError(st, "hav_sample_chain")
        self._n_info = len(Ms)
        parts, off = [], 0
        for m in Ms:
            parts.append(idx[off:off + int(m)])
            off += int(m)
        if with_info:
            return parts, self._read(len(Ms))
        return parts


    def ball_query(self, xyz, idx, radius: float, K: int, p: Params | None = None, stream=None):
        """hav_ball_query_sampled: for each centre xyz[idx[j]] the K lowest-index points
        strictly inside the radius, found through this Sampler's workspace as the last
        sample() call on the same cloud left it (call it right after that sample(), with
        the same parameters). Returns (out [M, K] int32, count [M] int32)."""
        torch = _torch()
        _check_xyz(xyz)
        p = p if p is not None else params()
        if not (isinstance(idx, torch.Tensor) and idx.is_cuda and idx.dtype == torch.int32
                and idx.dim() == 1 and idx.is_contiguous()):
            raise ValueError("idx must be a contiguous int32 CUDA tensor of shape [M]")
        if self.ws is None:
            raise HavError(ERR_INVALID_ARG, "ball_query: sample() this cloud first")
        M = idx.shape[0]
        out = torch.empty((M, int(K)), dtype=torch.int32, device=xyz.device)
        cnt = torch.empty(M, dtype=torch.int32, device=xyz.device)
        st = lib().hav_ball_query_sampled(C.c_void_p(xyz.data_ptr()), xyz.shape[0],
                                          C.c_void_p(idx.data_ptr()), M, float(radius), int(K),
                                          C.c_void_p(out.data_ptr()), C.c_void_p(cnt.data_ptr()),
                                          C.c_void_p(self.ws.data_ptr()), self.ws.numel(), C.byref(p),
                                          _stream_ptr(stream))
        if st != OK:
            raise HavError(st, "hav_ball_query_sampled")
        return out, cnt

    def sample_batch(self, xyz_concat, offsets, Ms, p: Params | None = None, out=None,
                     with_info: bool = False, stream=None):
        """hav_sample_batch: cloud i is xyz_concat[offsets[i]:offsets[i+1]]; returns one
        tensor of local indices (ascending) per cloud."""
        torch = _torch()
        _check_xyz(xyz_concat)
        p = p if p is not None else params()
        offsets = [int(o) for o in offsets]
        Ms = [int(m) for m in Ms]
        B = len(Ms)
        if len(offsets) != B + 1 or offsets[-1] != xyz_concat.shape[0]:
            raise ValueError("offsets must have B+1 entries ending at the number of points")
        Ns = tuple(offsets[i + 1] - offsets[i] for i in range(B))
        nbytes = batch_workspace_size(Ns, Ms, p)
        if nbytes == 0:
            raise HavError(ERR_INVALID_ARG, "hav_batch_workspace_size")
        ws = self._workspace(nbytes, Ns, p, stream)
        total = sum(Ms)
        idx = out if out is not None else torch.empty(total, dtype=torch.int32, device=xyz_concat.device)
        info = self._info(B)
        st = lib().hav_sample_batch(C.c_void_p(xyz_concat.data_ptr()), _i64(offsets), _i64(Ms), B,
                                    C.byref(p), C.c_void_p(idx.data_ptr()), C.c_void_p(ws.data_ptr()),
                                    ws.numel(), C.c_void_p(info.data_ptr()), _stream_ptr(stream))
        if st != OK:
            raise HavError(st, "hav_sample_batch")
        self._n_info = B
        parts, off = [], 0
        for m in Ms:
            parts.append(idx[off:off + m])
            off += m
        if with_info:
            return parts, self._read(B)
        return parts


STATIC_MAX_POINTS = 32768


def sample_static(xyz, M: int, p: Params | None = None, out=None, info=None, stream=None):
    """hav_sample_static: hav_sample on the library's own per-device workspace (nothing
    is allocated by the call; N <= STATIC_MAX_POINTS). `out` [M] int32 and `info` (a
    device buffer of sizeof(Info) bytes) are optional; calls on one device must not
    overlap. Returns idx."""
    torch = _torch()
    _check_xyz(xyz)
    p = p if p is not None else params()
    idx = out if out is not None else torch.empty(int(M), dtype=torch.int32, device=xyz.device)
    st = lib().hav_sample_static(C.c_void_p(xyz.data_ptr()), xyz.shape[0], int(M), C.byref(p),
                                 C.c_void_p(idx.data_ptr()),
                                 C.c_void_p(info.data_ptr()) if info is not None else None,
                                 _stream_ptr(stream))
    if st != OK:
        raise HavError(st, "hav_sample_static")
    return idx


def sample(xyz, M: int, p: Params | None = None, with_info: bool = False):
    """One-shot hav_sample on the current stream: returns idx [M] int32 (ascending).
    Waits for the call and raises HavError if the device reported an error."""
    s = Sampler(xyz.device)
    idx = s.sample(xyz, M, p)
    info = s.check()[0]
    return (idx, info) if with_info else idx


def chain(xyz, Ms, p: Params | None = None, with_info: bool = False):
    """One-shot hav_sample_chain: returns one original-index tensor per stage. Waits for
    the call and raises HavError if the device reported an error for any stage."""
    s = Sampler(xyz.device)
    parts = s.chain(xyz, Ms, p)
    info = s.check()
    return (parts, info) if with_info else parts


class Server:
    """Serving loop of the library (hav_server_*): continuous batching of requests whose
    clouds sit in pinned host memory, within an HBM budget. The caller keeps each cloud's
    tensor alive until its request has been polled to completion."""

    def __init__(self, hbm_budget_bytes: int, max_batch: int = 64, streams: int = 2,
                 p: Params | None = None):
        self.p = p if p is not None else params()
        self.h = lib().hav_server_create(int(hbm_budget_bytes), int(max_batch), int(streams),
                                         C.byref(self.p))
        if not self.h:
            raise HavError(ERR_INVALID_ARG, "hav_server_create")
        self._m = {}

    def submit(self, xyz_pinned, M: int) -> int:
        torch = _torch()
        if not (isinstance(xyz_pinned, torch.Tensor) and not xyz_pinned.is_cuda
                and xyz_pinned.is_pinned() and xyz_pinned.dtype == torch.float32
                and xyz_pinned.dim() == 2 and xyz_pinned.shape[1] == 3 and xyz_pinned.is_contiguous()):
            raise ValueError("xyz must be a contiguous pinned float32 CPU tensor of shape [N, 3]")
        t = C.c_uint64(0)
        st = lib().hav_server_submit(C.c_void_p(self.h), C.c_void_p(xyz_pinned.data_ptr()),
                                     xyz_pinned.shape[0], int(M), C.byref(t))
        if st != OK:
            raise HavError(st, "hav_server_submit")
        self._m[t.value] = int(M)
        return t.value

    def poll(self, ticket: int):
        """None while running; else (status, idx int32 numpy array or None, info dict,
        latency in ms)."""
        import numpy as np
        M = self._m[ticket]
        out = np.empty(M, dtype=np.int32)
        info = Info()
        lat = C.c_double(0.0)
        st = lib().hav_server_poll(C.c_void_p(self.h), ticket, C.c_void_p(out.ctypes.data),
                                   C.byref(info), C.byref(lat))
        if st == NOT_READY:
            return None
        del self._m[ticket]
        return st, (out if st == OK else None), info.as_dict(), lat.value

    def wait(self, ticket: int, timeout_s: float = 60.0):
        import time
        t0 = time.perf_counter()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"request {ticket} not done after {timeout_s} s")
            time.sleep(50e-6)

    def stats(self) -> dict:
        s = ServerStats()
        lib().hav_server_stats(C.c_void_p(self.h), C.byref(s))
        return s.as_dict()

    def close(self):
        if self.h:
            lib().hav_server_destroy(C.c_void_p(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A recorded sequence of library calls (hav_graph_*), replayed with launch().

        g = Graph.capture(stream, lambda: sampler.chain(xyz, Ms, out=out, stream=stream))
        g.launch(stream)

    The stream must not be the null stream; workspaces must be initialised first (make
    the same calls once eagerly)."""

    def __init__(self, handle):
        self.h = handle

    @classmethod
    def capture(cls, stream, fn):
        sp = _stream_ptr(stream)
        st = lib().hav_graph_capture_begin(sp)
        if st != OK:
            raise HavError(st, "hav_graph_capture_begin")
        g = C.c_void_p(0)
        try:
            fn()
        finally:
            st = lib().hav_graph_capture_end(sp, C.byref(g))
        if st != OK:
            raise HavError(st, "hav_graph_capture_end")
        return cls(g.value)

    def launch(self, stream=None):
        st = lib().hav_graph_launch(C.c_void_p(self.h), _stream_ptr(stream))
        if st != OK:
            raise HavError(st, "hav_graph_launch")

    def close(self):
        if self.h:
            lib().hav_graph_destroy(C.c_void_p(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- comparators (Fig. 7)

class FPS:
    """Farthest point sampling on the GPU (hav_fps): the comparator of the latency
    study. Keeps its (small) workspace; calls run on the current stream."""

    def __init__(self, device=None):
        torch = _torch()
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self._ws = torch.empty(int(lib().hav_fps_workspace_size(1)), dtype=torch.uint8, device=self.device)

    def sample(self, xyz, M: int, start: int = 0, blocks: int = 0, out=None, stream=None):
        """idx [M] int32 in selection order."""
        torch = _torch()
        _check_xyz(xyz)
        N = xyz.shape[0]
        out = out if out is not None else torch.empty(int(M), dtype=torch.int32, device=xyz.device)
        st = lib().hav_fps(xyz.data_ptr(), N, int(M), int(start), out.data_ptr(), self._ws.data_ptr(),
                           self._ws.numel(), int(blocks), _stream_ptr(stream))
        if st != 0:
            raise HavError(st)
        return out

    def error_flag(self) -> int:
        f = C.c_uint32(0)
        st = lib().hav_fps_error(self._ws.data_ptr(), C.byref(f))
        if st != 0:
            raise HavError(st)
        return int(f.value)


class RPS:
    """Random point sampling on the GPU (hav_rps): the m points of smallest SplitMix64
    key, ascending. Keeps a workspace sized for the largest N seen."""

    def __init__(self, device=None):
        torch = _torch()
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self._ws = None
        self._n = 0

    def sample(self, N: int, M: int, seed: int = 0, window: float = 0.0, out=None, stream=None):
        torch = _torch()
        if N > self._n:
            nbytes = int(lib().hav_rps_workspace_size(int(N)))
            if nbytes == 0:
                raise HavError(1)
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            st = lib().hav_rps_workspace_init(self._ws.data_ptr(), nbytes, int(N), _stream_ptr(stream))
            if st != 0:
                raise HavError(st)
            self._n = int(N)
        out = out if out is not None else torch.empty(int(M), dtype=torch.int32, device=self.device)
        st = lib().hav_rps(int(N), int(M), int(seed) & ((1 << 64) - 1), float(window), out.data_ptr(),
                           self._ws.data_ptr(), self._ws.numel(), _stream_ptr(stream))
        if st != 0:
            raise HavError(st)
        return out


class NearestSample:
    """Nearest-sample distances on the GPU (hav_nn): coverage and spacing of a sample."""

    def __init__(self, device=None):
        torch = _torch()
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self._ws = None
        self._m = 0

    def d2(self, samples, queries=None, stream=None):
        """(d2 [Q] float64, max_d2 float64 tensor of one element). queries None: the
        samples' spacing (each skips itself)."""
        torch = _torch()
        _check_xyz(samples)
        M = samples.shape[0]
        if M > self._m:
            nbytes = int(lib().hav_nn_workspace_size(M))
            if nbytes == 0:
                raise HavError(ERR_INVALID_ARG, "hav_nn_workspace_size")
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            st = lib().hav_nn_workspace_init(self._ws.data_ptr(), nbytes, M, _stream_ptr(stream))
            if st != OK:
                raise HavError(st, "hav_nn_workspace_init")
            self._m = M
        self_q = queries is None
        q = samples if self_q else queries
        _check_xyz(q)
        out = torch.empty(q.shape[0], dtype=torch.float64, device=self.device)
        mx = torch.empty(1, dtype=torch.float64, device=self.device)
        st = lib().hav_nn(samples.data_ptr(), M, q.data_ptr(), q.shape[0], 1 if self_q else 0,
                          out.data_ptr(), mx.data_ptr(), self._ws.data_ptr(), self._ws.numel(),
                          _stream_ptr(stream))
        if st != OK:
            raise HavError(st, "hav_nn")
        return out, mx


class BallQuery:
    """Ball-query grouping on the GPU (hav_ball_query): for each centre the K lowest-index
    points strictly inside the radius."""

    def __init__(self, device=None):
        torch = _torch()
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self._ws = None
        self._n = 0

    def query(self, xyz, centres, radius: float, K: int, stream=None):
        """(idx [Q, K] int32, count [Q] int32)."""
        torch = _torch()
        _check_xyz(xyz)
        _check_xyz(centres)
        N = xyz.shape[0]
        if N > self._n:
            nbytes = int(lib().hav_ball_workspace_size(N))
            if nbytes == 0:
                raise HavError(ERR_INVALID_ARG, "hav_ball_workspace_size")
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            st = lib().hav_ball_workspace_init(self._ws.data_ptr(), nbytes, N, _stream_ptr(stream))
            if st != OK:
                raise HavError(st, "hav_ball_workspace_init")
            self._n = N
        Q = centres.shape[0]
        idx = torch.empty((Q, int(K)), dtype=torch.int32, device=self.device)
        cnt = torch.empty(Q, dtype=torch.int32, device=self.device)
        st = lib().hav_ball_query(xyz.data_ptr(), N, centres.data_ptr(), Q, float(radius), int(K),
                                  idx.data_ptr(), cnt.data_ptr(), self._ws.data_ptr(), self._ws.numel(),
                                  _stream_ptr(stream))
        if st != OK:
            raise HavError(st, "hav_ball_query")
        return idx, cnt
