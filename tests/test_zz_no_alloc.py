"""The no-allocation ordering entry point (citron_order_noalloc) against the
allocating path (citron_load_csr + citron_order + citron_get_dag), through
the C ABI: two calls in a row, the second on a smaller graph, must both give
the DAG byte for byte; bad input is refused."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def _dev(citron, g):
    import torch
    rp = torch.from_numpy(g.row_ptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    return rp, col


def _noalloc(citron, g, fill=-7):
    import torch
    rp, col = _dev(citron, g)
    dptr = torch.full((g.n + 1,), fill, dtype=torch.int32, device="cuda")
    dcol = torch.full((max(g.m, 1),), fill, dtype=torch.int32, device="cuda")
    mx = citron.order_noalloc(rp, col, dptr, dcol[:g.m] if g.m else dcol[:0])
    torch.cuda.synchronize()
    return mx, dptr.cpu().numpy(), dcol[:g.m].cpu().numpy()


def _allocating(citron, g):
    h = citron.Graph.from_csr(g.row_ptr, g.col).order()
    dptr, dcol = h.dag()
    mx = h.info()["max_outdeg"]
    h.free()
    return mx, dptr, dcol


def test_noalloc_equals_the_allocating_path_twice(citron_gpu):
    big = gg.rmat(14, 16, seed=14)
    small = gg.rmat(9, 8, seed=3)          # second call: smaller, on the same static memory
    for g in (big, small):
        want = _allocating(citron_gpu, g)
        got = _noalloc(citron_gpu, g)
        assert got[0] == want[0]
        assert np.array_equal(got[1], want[1]) and np.array_equal(got[2], want[2]), g.name


def test_noalloc_after_a_larger_graph_and_edge_cases(citron_gpu):
    import torch
    # the Figure 1 graph, the empty graph and isolated vertices
    for g in (gg.fig1_example(), gg.empty(5), gg.complete(3)):
        want = _allocating(citron_gpu, g)
        got = _noalloc(citron_gpu, g)
        assert got[0] == want[0]
        assert np.array_equal(got[1], want[1]) and np.array_equal(got[2], want[2])
    # an asymmetric CSR is refused with EINVAL (validated on the device)
    rp = torch.tensor([0, 1, 2, 2], dtype=torch.int32, device="cuda")
    col = torch.tensor([1, 2], dtype=torch.int32, device="cuda")
    out_p = torch.zeros(4, dtype=torch.int32, device="cuda")
    out_c = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(citron_gpu.CitronError) as e:
        citron_gpu.order_noalloc(rp, col, out_p, out_c)
    assert e.value.status == 1
    # more vertices than the static memory holds
    n = (1 << 22) + 1
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    with pytest.raises(citron_gpu.CitronError) as e:
        citron_gpu.order_noalloc(rp, col, torch.zeros(n + 1, dtype=torch.int32, device="cuda"),
                                 torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert e.value.status == 1
    # and the path still works after the refusals
    g = gg.rmat(11, 16, seed=11)
    want = _allocating(citron_gpu, g)
    got = _noalloc(citron_gpu, g)
    assert got[0] == want[0] and np.array_equal(got[1], want[1]) and np.array_equal(got[2], want[2])
