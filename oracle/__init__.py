"""CPU oracle of HAVSampler (arXiv 2305.14306, Sec. 3) — test infrastructure.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package. The GPU library never does, and the two share no code: this
wrapper loads ``liboracle.so`` built from ``hav_oracle.cpp`` (plain single-threaded C++,
exact binary32, no FMA contraction) and marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "hav_oracle.cpp"), os.path.join(_HERE, "quality.cpp")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FIXED_VOXEL = 1
MAX_LAYERS = 8

# status codes (same meanings as the library's)
OK, INVALID_ARG, UNSUPPORTED, NONFINITE = 0, 1, 4, 5


class Params(C.Structure):
    _fields_ = [
        ("layers", C.c_int32),
        ("layer_ratio", C.c_int32),
        ("t_max", C.c_int32),
        ("flags", C.c_int32),
        ("sigma", C.c_double),
        ("aspect", C.c_float * 3),
        ("fixed_voxel", C.c_float * 3),
        ("select", C.c_int32),
        ("seed", C.c_uint32),
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


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (exact binary32: no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", _LIB_PATH + ".tmp"] + _SRC
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        f32p, i32p, i64p = C.POINTER(C.c_float), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        L.oracle_params_default.restype = Params
        L.oracle_sample.argtypes = [f32p, C.c_int64, C.c_int64, C.POINTER(Params), i32p, C.POINTER(Info)]
        L.oracle_sample.restype = C.c_int32
        L.oracle_sample_tags.argtypes = [f32p, C.c_int64, C.c_int64, C.POINTER(Params), i32p,
                                         C.POINTER(Info), C.POINTER(C.c_uint8)]
        L.oracle_sample_tags.restype = C.c_int32
        L.oracle_sample_points.argtypes = [f32p, C.c_int64, C.c_int64, C.POINTER(Params), i32p, f32p,
                                           C.POINTER(Info)]
        L.oracle_sample_points.restype = C.c_int32
        L.oracle_chain.argtypes = [f32p, C.c_int64, i64p, C.c_int32, C.POINTER(Params), i32p, C.POINTER(Info)]
        L.oracle_chain.restype = C.c_int32
        L.oracle_count.argtypes = [f32p, C.c_int64, f32p, f32p, C.POINTER(C.c_uint8)]
        L.oracle_count.restype = C.c_int64
        L.oracle_keys.argtypes = [f32p, C.c_int64, f32p, f32p, i32p, C.POINTER(C.c_uint64), f32p]
        L.oracle_keys.restype = None
        L.oracle_priority.argtypes = [C.c_uint64]
        L.oracle_take_visits.restype = C.c_int64
        L.oracle_take_visits.argtypes = []
        L.oracle_priority.restype = C.c_uint64
        L.oracle_pow2_ceil.argtypes = [C.c_float]
        L.oracle_pow2_ceil.restype = C.c_float
        L.oracle_layer_budgets.argtypes = [C.c_int64, C.c_int32, C.c_int32, i64p]
        L.oracle_layer_budgets.restype = None
        L.oracle_fps.argtypes = [f32p, C.c_int64, C.c_int64, C.c_int64, i32p]
        L.oracle_fps.restype = C.c_int32
        L.oracle_rps.argtypes = [C.c_int64, C.c_int64, C.c_uint64, i32p]
        L.oracle_rps.restype = C.c_int32
        L.oracle_nn_d2.argtypes = [f32p, C.c_int64, f32p, C.c_int64, C.c_int32, C.POINTER(C.c_double)]
        L.oracle_nn_d2.restype = C.c_int32
        L.oracle_ball_query.argtypes = [f32p, C.c_int64, f32p, C.c_int64, C.c_float, C.c_int32, i32p, i32p]
        L.oracle_ball_query.restype = C.c_int32
        L.oracle_covering_radius.argtypes = [f32p, C.c_int64, i32p, C.c_int64]
        L.oracle_covering_radius.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _xyz(xyz) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32))
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("xyz must be [N, 3]")
    return a


def params(layers=2, layer_ratio=4, t_max=20, sigma=0.05, aspect=(1.0, 1.0, 1.0),
           fixed_voxel=None, select=0, seed=0) -> Params:
    p = lib().oracle_params_default()
    p.layers, p.layer_ratio, p.t_max, p.sigma = layers, layer_ratio, t_max, sigma
    p.select, p.seed = select, seed
    for a in range(3):
        p.aspect[a] = aspect[a]
    if fixed_voxel is not None:
        p.flags |= FIXED_VOXEL
        fv = fixed_voxel if hasattr(fixed_voxel, "__len__") else (fixed_voxel,) * 3
        for a in range(3):
            p.fixed_voxel[a] = fv[a]
    return p


def sample(xyz, M: int, p: Params | None = None):
    """Returns (status, idx[M] int32 ascending, info dict)."""
    a = _xyz(xyz)
    p = p if p is not None else params()
    idx = np.zeros(max(int(M), 1), dtype=np.int32)
    info = Info()
    st = lib().oracle_sample(_ptr(a, C.c_float), a.shape[0], int(M), C.byref(p),
                             _ptr(idx, C.c_int32), C.byref(info))
    return st, idx[: int(M)] if M > 0 else idx[:0], info.as_dict()


def sample_tags(xyz, M: int, p: Params | None = None):
    """Returns (status, idx, info, tag[N] uint8) where tag[i] is the 1-based layer that
    picked point i (0 = not picked)."""
    a = _xyz(xyz)
    p = p if p is not None else params()
    idx = np.zeros(max(int(M), 1), dtype=np.int32)
    tag = np.zeros(a.shape[0], dtype=np.uint8)
    info = Info()
    st = lib().oracle_sample_tags(_ptr(a, C.c_float), a.shape[0], int(M), C.byref(p),
                                  _ptr(idx, C.c_int32), C.byref(info), _ptr(tag, C.c_uint8))
    return st, idx[: int(M)] if M > 0 else idx[:0], info.as_dict(), tag


def sample_points(xyz, M: int, p: Params | None = None):
    """Returns (status, idx[M], pts[M, 3] float32, info): pts[j] stands for idx[j] (the
    voxel centre / mean with select 2 / 3, else the point itself)."""
    a = _xyz(xyz)
    p = p if p is not None else params()
    idx = np.zeros(max(int(M), 1), dtype=np.int32)
    pts = np.zeros((max(int(M), 1), 3), dtype=np.float32)
    info = Info()
    st = lib().oracle_sample_points(_ptr(a, C.c_float), a.shape[0], int(M), C.byref(p),
                                    _ptr(idx, C.c_int32), _ptr(pts, C.c_float), C.byref(info))
    return st, idx[: int(M)], pts[: int(M)], info.as_dict()


def chain(xyz, Ms, p: Params | None = None):
    """Chained stages. Returns (status, list of per-stage original-index arrays, infos)."""
    a = _xyz(xyz)
    p = p if p is not None else params()
    Ms = np.ascontiguousarray(np.asarray(Ms, dtype=np.int64))
    out = np.zeros(int(Ms.sum()), dtype=np.int32)
    infos = (Info * len(Ms))()
    st = lib().oracle_chain(_ptr(a, C.c_float), a.shape[0], _ptr(Ms, C.c_int64), len(Ms),
                            C.byref(p), _ptr(out, C.c_int32), infos)
    parts, off = [], 0
    for m in Ms:
        parts.append(out[off: off + int(m)])
        off += int(m)
    return st, parts, [infos[j].as_dict() for j in range(len(Ms))]


def count(xyz, mn, v, mask=None) -> int:
    a = _xyz(xyz)
    mn = np.ascontiguousarray(np.asarray(mn, dtype=np.float32))
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float32))
    mk = None
    if mask is not None:
        mk = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
    return int(lib().oracle_count(_ptr(a, C.c_float), a.shape[0], _ptr(mn, C.c_float),
                                  _ptr(v, C.c_float), None if mk is None else _ptr(mk, C.c_uint8)))


def keys(xyz, mn, v):
    """Returns (g[N,3] int32, packed key[N] uint64, d2[N] float32)."""
    a = _xyz(xyz)
    n = a.shape[0]
    mn = np.ascontiguousarray(np.asarray(mn, dtype=np.float32))
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float32))
    g = np.zeros((n, 3), dtype=np.int32)
    k = np.zeros(n, dtype=np.uint64)
    d2 = np.zeros(n, dtype=np.float32)
    lib().oracle_keys(_ptr(a, C.c_float), n, _ptr(mn, C.c_float), _ptr(v, C.c_float),
                      _ptr(g, C.c_int32), _ptr(k, C.c_uint64), _ptr(d2, C.c_float))
    return g, k, d2


def take_visits() -> int:
    """Point visits (Cnt evaluations and selection passes, each point of R once) of the
    oracle calls made on this thread since the previous take_visits()."""
    return int(lib().oracle_take_visits())


def priority(key: int) -> int:
    return int(lib().oracle_priority(C.c_uint64(int(key))))


def pow2_ceil(E: float) -> float:
    return float(lib().oracle_pow2_ceil(C.c_float(E)))


def layer_budgets(M: int, k: int = 2, r: int = 4):
    m = np.zeros(k, dtype=np.int64)
    lib().oracle_layer_budgets(int(M), int(k), int(r), _ptr(m, C.c_int64))
    return [int(x) for x in m]


def fps(xyz, m: int, start: int = 0) -> np.ndarray:
    """Farthest point sampling (Sec. 3.1, Eq. 1), start index given, ties to lowest."""
    a = _xyz(xyz)
    out = np.zeros(int(m), dtype=np.int32)
    st = lib().oracle_fps(_ptr(a, C.c_float), a.shape[0], int(m), int(start), _ptr(out, C.c_int32))
    if st != 0:
        raise ValueError("fps: bad arguments")
    return out


def rps(N: int, m: int, seed: int) -> np.ndarray:
    """Random point sampling: the m points of smallest SplitMix64 key (output i+1 of
    the generator seeded with `seed` keys point i), ascending."""
    out = np.zeros(int(m), dtype=np.int32)
    st = lib().oracle_rps(int(N), int(m), C.c_uint64(int(seed) & ((1 << 64) - 1)), _ptr(out, C.c_int32))
    if st != 0:
        raise ValueError("rps: bad arguments")
    return out


def nn_d2(samples, queries, exclude_self: bool = False) -> np.ndarray:
    """Squared distance (double) from every query to its nearest sample; with
    exclude_self the queries are the samples and skip themselves (the spacing)."""
    s, q = _xyz(samples), _xyz(queries)
    out = np.zeros(q.shape[0], dtype=np.float64)
    st = lib().oracle_nn_d2(_ptr(s, C.c_float), s.shape[0], _ptr(q, C.c_float), q.shape[0],
                            1 if exclude_self else 0, _ptr(out, C.c_double))
    if st != 0:
        raise ValueError("nn_d2: bad arguments")
    return out


def ball_query(xyz, centres, radius: float, K: int):
    """(idx [Q, K] int32, count [Q] int32): the K lowest-index points strictly inside
    the radius of each centre."""
    a, c = _xyz(xyz), _xyz(centres)
    idx = np.zeros((c.shape[0], int(K)), dtype=np.int32)
    cnt = np.zeros(c.shape[0], dtype=np.int32)
    st = lib().oracle_ball_query(_ptr(a, C.c_float), a.shape[0], _ptr(c, C.c_float), c.shape[0],
                                 C.c_float(radius), int(K), _ptr(idx, C.c_int32), _ptr(cnt, C.c_int32))
    if st != 0:
        raise ValueError("ball_query: bad arguments")
    return idx, cnt


def covering_radius(xyz, idx) -> float:
    """Largest distance from any point of the cloud to its nearest sampled point."""
    a = _xyz(xyz)
    ii = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
    return float(lib().oracle_covering_radius(_ptr(a, C.c_float), a.shape[0],
                                              _ptr(ii, C.c_int32), ii.shape[0]))
