"""Served form: continuous batching over resident graphs.  Every result must
equal the plain count exactly, whatever the mix it was served in."""
import sys
import time

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def drain(srv, n, timeout=120.0):
    out = []
    t0 = time.time()
    while len(out) < n:
        out += srv.poll()
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(out)} of {n} results after {timeout} s")
        time.sleep(0.001)
    return out


@pytest.fixture(scope="module")
def graphs(citron_gpu):
    gs = [gg.rmat(s, 16, seed=300 + s) for s in (10, 12, 13)] + [gg.erdos_renyi(4000, 30, seed=9),
                                                                 gg.complete(40)]
    hs = [citron_gpu.Graph.from_csr(g.row_ptr, g.col).order() for g in gs]
    plain = {(i, k): h.count(k) for i, h in enumerate(hs) for k in range(1, 9)}
    return hs, plain


def test_served_equals_plain_in_a_mix(citron_gpu, graphs):
    hs, plain = graphs
    srv = citron_gpu.Server(hbm_budget_bytes=1 << 30, max_slots=16)
    ids = [srv.add_graph(h) for h in hs]
    rng = np.random.default_rng(5)
    reqs = [(int(rng.integers(len(ids))), int(rng.integers(1, 9))) for _ in range(200)]
    for tag, (gi, k) in enumerate(reqs):
        srv.submit(ids[gi], k, tag)
        if tag % 17 == 0:
            time.sleep(0.002)          # arrivals while others run
    res = drain(srv, len(reqs))
    assert srv.pending() == 0
    for r in res:
        gi, k = reqs[r["tag"]]
        assert r["status"] == 0, r
        assert r["count"] == plain[(gi, k)], (gi, k)
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_done_ns"]
    srv.close()


def test_alone_equals_mix(citron_gpu, graphs):
    hs, plain = graphs
    srv = citron_gpu.Server(hbm_budget_bytes=1 << 30, max_slots=8)
    ids = [srv.add_graph(h) for h in hs]
    srv.submit(ids[2], 6, 0)
    alone = drain(srv, 1)[0]["count"]
    for t in range(1, 30):
        srv.submit(ids[t % len(ids)], 3 + t % 5, t)
    srv.submit(ids[2], 6, 99)
    res = drain(srv, 30)
    mixed = [r["count"] for r in res if r["tag"] == 99][0]
    assert alone == mixed == plain[(2, 6)]
    srv.close()


def test_small_budget_queues_instead_of_failing(citron_gpu, graphs):
    hs, plain = graphs
    # room for one request at a time (a request holds a few hundred bytes):
    # the rest wait in the queue
    srv = citron_gpu.Server(hbm_budget_bytes=300, max_slots=4)
    ids = [srv.add_graph(h) for h in hs]
    for t in range(12):
        srv.submit(ids[t % 3], 5, t)
    res = drain(srv, 12)
    for r in res:
        assert r["status"] == 0
        assert r["count"] == plain[(r["tag"] % 3, 5)]
    srv.close()


def test_refusals_and_bad_arguments(citron_gpu, graphs):
    hs, _ = graphs
    srv = citron_gpu.Server(hbm_budget_bytes=64, max_slots=2)   # below any footprint
    gid = srv.add_graph(hs[0])
    srv.submit(gid, 5, 1)
    srv.submit(gid, 0, 2)                                       # k out of range
    srv.submit(gid, 2, 3)                                       # trivial: m
    res = {r["tag"]: r for r in drain(srv, 3)}
    assert res[1]["status"] == 2                                # ENOMEM: can never fit
    assert res[2]["status"] == 1                                # EINVAL
    assert res[3]["status"] == 0 and res[3]["count"] == hs[0].m
    with pytest.raises(citron_gpu.CitronError):
        srv.submit(77, 4, 0)
    srv.close()
    with pytest.raises(citron_gpu.CitronError):
        citron_gpu.Server(hbm_budget_bytes=1 << 20, max_slots=0)
