"""GPU tests of the serving loop: every request's result must be exactly what the
single-cloud call gives the same cloud alone (and what the oracle gives), whatever else
is in flight, under both a roomy and a tight HBM budget."""
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


def _requests(seed, count, n_lo=1000, n_hi=150000):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi))
        kind = ["uniform", "clustered", "quantised"][i % 3]
        x = synth.random_cloud(n, seed * 1000 + i, scale=float(rng.uniform(2.0, 60.0)), kind=kind)
        M = max(1, n // (4 if i % 2 == 0 else 16))
        reqs.append((x, M))
    return reqs


def _alone(gpu, x, M):
    import torch
    return gpu.Sampler().sample(torch.from_numpy(x).cuda(), M).cpu().numpy()


def _serve_all(gpu, server, reqs):
    import torch
    pinned = [torch.from_numpy(x).pin_memory() for x, _ in reqs]
    tickets = [server.submit(pinned[i], M) for i, (_, M) in enumerate(reqs)]
    out = []
    for t in tickets:
        st, idx, info, lat = server.wait(t)
        out.append((st, idx, info, lat))
    del pinned
    return out


def test_serve_mix_equals_alone(gpu, orc):
    reqs = _requests(3, 24)
    srv = gpu.Server(8 << 30, max_batch=16, streams=2)
    try:
        _note("case serve mix 24 requests")
        res = _serve_all(gpu, srv, reqs)
        stats = srv.stats()
    finally:
        srv.close()
    for i, ((x, M), (st, idx, info, lat)) in enumerate(zip(reqs, res)):
        assert st == 0, (i, st)
        assert lat > 0.0
        assert np.array_equal(idx, _alone(gpu, x, M)), i
        if x.shape[0] <= 40000:
            ost, want, winfo = orc.sample(x, M)
            assert np.array_equal(idx, want), i
            assert info == winfo, i
    assert stats["completed"] == stats["submitted"] == 24
    assert stats["max_batch_seen"] > 1  # requests were batched together


def test_serve_tight_budget(gpu, orc):
    # room for a few slots only: requests queue for slots and idle slots of other
    # classes are released; results are unchanged
    reqs = _requests(5, 12, n_lo=2000, n_hi=90000)
    budget = 200 << 20
    srv = gpu.Server(budget, max_batch=4, streams=2)
    try:
        _note("case serve tight budget")
        res = _serve_all(gpu, srv, reqs)
        stats = srv.stats()
    finally:
        srv.close()
    for i, ((x, M), (st, idx, info, lat)) in enumerate(zip(reqs, res)):
        assert st == 0, (i, st)
        assert np.array_equal(idx, _alone(gpu, x, M)), i
    assert stats["hbm_used"] <= budget
    assert stats["completed"] == 12


def test_serve_rejects_oversized(gpu):
    import torch
    srv = gpu.Server(64 << 20, max_batch=4, streams=1)
    try:
        x = torch.from_numpy(synth.random_cloud(300000, 1)).pin_memory()
        with pytest.raises(gpu.HavError):
            srv.submit(x, 1000)
    finally:
        srv.close()


def test_serve_errors_and_identity(gpu, orc):
    import torch
    good = synth.random_cloud(5000, 11)
    bad = good.copy()
    bad[3, 0] = np.inf
    reqs = [(good, 1000), (bad, 1000), (good, 5000), (synth.random_cloud(1, 2), 1)]
    srv = gpu.Server(2 << 30, max_batch=8, streams=2)
    try:
        res = _serve_all(gpu, srv, reqs)
    finally:
        srv.close()
    assert res[0][0] == 0 and np.array_equal(res[0][1], orc.sample(good, 1000)[1])
    assert res[1][0] == gpu.ERR_NONFINITE
    assert res[2][0] == 0 and np.array_equal(res[2][1], np.arange(5000, dtype=np.int32))
    assert res[3][0] == 0 and list(res[3][1]) == [0]


# ------------------------------------------------------------ the serving workload itself

@pytest.fixture(scope="module")
def trace_requests():
    """A slice of the serving workload: the first 48 requests of the Poisson trace
    (LiDAR sectors and scene windows, M = N/4 or N/16), plus the trace's first requests
    of the 2^20 and 2^21 slot classes, built exactly as the bench replays them."""
    tr = synth.serving_trace(10000)
    bases = synth.serving_bases()
    offs = synth.serving_windows(tr, bases[0].shape[0])
    n = tr["n"]
    pick = list(range(48))
    for lo, hi, extra in (((1 << 19), (1 << 20), 1), ((1 << 20), (1 << 21), 2)):
        cand = [int(i) for i in np.nonzero((n > lo) & (n <= hi))[0] if int(i) not in pick]
        pick += cand[:extra]
    reqs = []
    for i in pick:
        b = bases[int(tr["kind"][i])]
        o, k = int(offs[i]), int(n[i])
        reqs.append((np.ascontiguousarray(b[o:o + k]), int(tr["m"][i])))
    return reqs


def test_serve_trace_mix_equals_alone(gpu, orc, trace_requests):
    reqs = trace_requests
    classes = {int(np.ceil(np.log2(x.shape[0]))) for x, _ in reqs}
    assert {19, 20, 21} <= classes, classes  # the largest slot classes are exercised
    srv = gpu.Server(24 << 30, max_batch=16, streams=2)
    try:
        _note(f"case serve trace slice {len(reqs)} requests, classes {sorted(classes)}")
        res = _serve_all(gpu, srv, reqs)
        stats = srv.stats()
    finally:
        srv.close()
    assert stats["completed"] == stats["submitted"] == len(reqs)
    assert stats["max_batch_seen"] > 1
    for i, ((x, M), (st, idx, info, lat)) in enumerate(zip(reqs, res)):
        _note(f"  request {i} N={x.shape[0]} M={M}")
        assert st == 0, (i, st)
        assert np.array_equal(idx, _alone(gpu, x, M)), i
        ost, want, winfo = orc.sample(x, M)
        assert ost == 0
        assert np.array_equal(idx, want), i
        assert info == winfo, i


def test_serve_search_give_up_then_slot_recovers(gpu, orc, trace_requests):
    # a search whose bounded wait gives up (forced from the host) marks its workspace
    # for initialisation; the server must initialise the slot again, so the next request
    # on the same slot is exact
    x, M = max(trace_requests, key=lambda r: r[0].shape[0])
    import torch
    pinned = torch.from_numpy(x).pin_memory()
    srv = gpu.Server(4 << 30, max_batch=4, streams=1)
    try:
        _note(f"case serve search give-up N={x.shape[0]}")
        gpu.debug_search_spin_limit(1)
        try:
            st, _, info, _ = srv.wait(srv.submit(pinned, M))
        finally:
            gpu.debug_search_spin_limit(0)
        assert st == gpu.ERR_HIP, st
        st, idx, info, _ = srv.wait(srv.submit(pinned, M))
        stats = srv.stats()
    finally:
        srv.close()
    assert st == 0
    assert stats["slots_created"] == 1  # the same slot served both requests
    assert np.array_equal(idx, orc.sample(x, M)[1])
