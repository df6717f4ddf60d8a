"""k-clique listing on the GPU against the oracle's edge-rooted listing:
the same cliques, in the same order, grouped by arc with the same offsets;
every arc of small graphs and sampled arcs of R-MAT scale 20."""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _check(citron, g, ks, arcs=None, progress=None):
    h = citron.Graph.from_csr(g.row_ptr, g.col).order()
    dptr, dcol = h.dag()
    src = np.repeat(np.arange(g.n), np.diff(dptr)).astype(np.int32)
    idx = np.arange(g.m, dtype=np.int32) if arcs is None else np.asarray(arcs, dtype=np.int32)
    for k in ks:
        if progress:
            progress(f"  listing {g.name} k={k}, {idx.size} arcs")
        want, per_arc = oracle.list_arcs(g.n, dptr, dcol, k, src[idx], dcol[idx])
        got, offs = h.list_arcs(k, idx)
        offs = offs.cpu().numpy()
        assert offs[0] == 0 and np.array_equal(np.diff(offs), per_arc.astype(np.int64)), (g.name, k)
        assert got.shape == want.shape, (g.name, k)
        assert np.array_equal(got.cpu().numpy(), want), (g.name, k)
    h.free()


def test_listing_small_graphs_every_arc(citron_gpu):
    _check(citron_gpu, gg.fig1_example(), range(2, 6))
    _check(citron_gpu, gg.complete(12), range(2, 9))
    _check(citron_gpu, gg.complete(70), range(3, 5))           # two-word candidate masks
    _check(citron_gpu, gg.erdos_renyi(400, 0.5 * 399, seed=5), range(3, 5))
    _check(citron_gpu, gg.disjoint_cliques([3, 5, 9, 2]), range(2, 7))
    _check(citron_gpu, gg.empty(4), range(2, 4))
    rng = np.random.default_rng(9)
    for i in range(10):
        n = int(rng.integers(3, 120))
        iu, ju = np.triu_indices(n, 1)
        keep = rng.random(iu.size) < float(rng.uniform(0.05, 0.5))
        _check(citron_gpu, gg.csr_from_edges(n, iu[keep], ju[keep], perm_seed=i), range(2, 8))


def test_listing_rmat(citron_gpu, progress):
    _check(citron_gpu, gg.rmat(10, 16, seed=10), range(3, 8), progress=progress)
    _check(citron_gpu, gg.rmat(12, 16, seed=12), range(3, 6), progress=progress)
    # repeated and unordered arcs
    g = gg.rmat(9, 16, seed=9)
    rng = np.random.default_rng(4)
    _check(citron_gpu, g, (4, 5), arcs=rng.integers(0, g.m, 300))


def test_listing_rmat20_sampled_arcs(citron_gpu, progress):
    with open(os.path.join(GOLDEN, "rmat20.json")) as f:
        gold = json.load(f)
    g = gg.config_graph("rmat20")
    assert g.sha256() == gold["sha256"]
    # the stored sample: 192 uniform arcs and 64 with a heavy source (11.6 M
    # cliques at k = 5, 232 MB of output)
    idx = np.array(gold["arcs"]["index"], dtype=np.int32)
    _check(citron_gpu, g, (3, 4, 5), arcs=idx, progress=progress)


def test_listing_refuses_a_small_buffer(citron_gpu):
    import ctypes
    import torch
    g = gg.complete(10)
    h = citron_gpu.Graph.from_csr(g.row_ptr, g.col).order()
    lib = citron_gpu.load_library()
    arcs = torch.arange(g.m, dtype=torch.int32, device="cuda")
    offs = torch.zeros(g.m + 1, dtype=torch.int64, device="cuda")
    out = torch.zeros((5, 4), dtype=torch.int32, device="cuda")
    total = ctypes.c_int64(0)
    st = lib.citron_list_arcs(h._handle(), 4, arcs.data_ptr(), g.m, offs.data_ptr(), out.data_ptr(), 5,
                              ctypes.byref(total))
    assert st == 2 and total.value == 210                      # ENOMEM, C(10, 4) needed
    assert int(out.abs().sum()) == 0                           # nothing written
    st = lib.citron_list_arcs(h._handle(), 17, arcs.data_ptr(), g.m, offs.data_ptr(), out.data_ptr(), 5,
                              ctypes.byref(total))
    assert st == 1                                             # k outside 2..16
    bad = torch.tensor([0, g.m], dtype=torch.int32, device="cuda")
    st = lib.citron_list_arcs(h._handle(), 3, bad.data_ptr(), 2, offs.data_ptr(), out.data_ptr(), 5,
                              ctypes.byref(total))
    assert st == 1                                             # arc index out of range
