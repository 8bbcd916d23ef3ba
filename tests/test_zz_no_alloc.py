"""The allocation-free batch entry point (ppsp_batch_query_noalloc) through
the C-ABI: on two calls in a row (the second with a smaller input) its
distances equal ppsp_batch_query's and the oracle's, bit for bit; batches
larger than the scratch run in several waves inside it; a second call
allocates no device memory; a graph on which one query cannot fit the
scratch is rejected with PPSP_E_OOM."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2506_16488_amd as P
    P.lib()
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return P


def _exp(g, pairs):
    return oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)


@pytest.mark.parametrize("algo,batch", [("bidastar", "plainstar"), ("bids", "plainstar"), ("astar", "plain"),
                                        ("et", "plainstar")])
def test_noalloc_equals_batch_query_two_calls(P, algo, batch):
    g = gen.lattice(180, 0.05, seed=41)
    G = P.Graph.from_host(g)
    big = gen.pairs_uniform(g.n, 120, seed=42)
    big[3, 1] = big[3, 0]                       # s = t
    small = gen.pairs_uniform(g.n, 17, seed=43)
    for pairs in (big, small):                  # two calls, the second smaller
        print("noalloc", algo, batch, pairs.shape[0], flush=True)
        got = G.batch_query_noalloc(pairs, algo=algo, batch=batch)
        ref = G.batch_query(pairs, algo=algo, batch=batch)
        assert np.array_equal(got, ref)
        assert np.array_equal(got, _exp(g, pairs))
    G.close()


def test_noalloc_waves_hubs_and_device_io(P):
    """A batch whose state exceeds the scratch runs in waves (60 queries of 2
    x 3.4 MB searches on a 600 x 600 lattice), an R-MAT graph exercises the
    hub list, and device-resident pairs and distances give the same result."""
    import torch
    g = gen.lattice(600, 0.05, seed=44)
    G = P.Graph.from_host(g)
    pairs = gen.pairs_uniform(g.n, 60, seed=45)
    print("noalloc waves", flush=True)
    got = G.batch_query_noalloc(pairs, algo="bidastar")
    assert G.stats()["waves"] >= 3
    assert np.array_equal(got, _exp(g, pairs))
    pd = torch.from_numpy(pairs[:25].astype(np.int32)).cuda()
    dd = torch.empty(25, dtype=torch.int64, device="cuda")
    G.batch_query_noalloc_device(pd, dd, algo="bids")
    torch.cuda.synchronize()
    assert np.array_equal(dd.cpu().numpy().view(np.uint64), got[:25])
    G.close()
    r = gen.rmat(14, seed=46)
    R = P.Graph.from_host(r)
    assert int(np.max(np.diff(r.row_ptr.astype(np.int64)))) > 512
    rp = gen.pairs_uniform(gen.lcc(r), 24, seed=47)
    print("noalloc rmat", flush=True)
    for k in (24, 9):
        assert np.array_equal(R.batch_query_noalloc(rp[:k], algo="bids"), _exp(r, rp[:k]))
    R.close()


def test_noalloc_second_call_allocates_nothing(P):
    """On a fresh graph the regular entry point grows the graph's workspace
    (free device memory drops); the allocation-free one leaves free memory
    exactly where it was on its second call."""
    import torch
    g = gen.lattice(256, 0.05, seed=48)
    G = P.Graph.from_host(g)
    a = gen.pairs_uniform(g.n, 50, seed=49)
    b = gen.pairs_uniform(g.n, 20, seed=50)
    G.batch_query_noalloc(a, algo="bidastar")          # first call on this device may load the scratch
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = G.batch_query_noalloc(b, algo="bidastar")
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert np.array_equal(got, _exp(g, b))
    G.batch_query(b, algo="bidastar")                 # the regular path allocates its workspace
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] < free0
    G.close()


def test_noalloc_rejects_graph_beyond_scratch(P):
    """One query on a 2,900 x 2,900 lattice needs 2 x 8.4 M x 8 bytes of
    state, more than the 128 MiB scratch: PPSP_E_OOM, saying why."""
    g = gen.lattice(2900, 0.0, seed=51)
    G = P.Graph.from_host(g)
    with pytest.raises(P.PPSPError) as e:
        G.batch_query_noalloc(np.array([[0, g.n - 1]], np.uint32), algo="bids")
    assert e.value.code == P.E_OOM
    assert "scratch" in str(e.value)
    G.close()


def test_noalloc_with_graph_options(P):
    """Options on the graph whose buffers live outside the scratch (dense
    frontiers, the hub list grouped by vertex) are off inside the call, a
    grouped state layout runs in the scratch, and the graph's own calls keep
    the options afterwards; two calls in a row, the second smaller."""
    g = gen.rmat(13, 16, seed=46)
    lcc = gen.lcc(g)
    pairs = gen.pairs_uniform(lcc, 40, seed=47)
    exp = _exp(g, pairs)
    G = P.Graph.from_host(g, reorder=True)
    G.set_option("dense_min", 64)
    G.set_option("plain_group", 8)
    for k in (40, 13):
        print("noalloc options", k, flush=True)
        assert np.array_equal(G.batch_query_noalloc(pairs[:k], algo="bids"), exp[:k])
        assert G.stats()["dense_searches"] == 0
    assert G.get_option("dense_min") == 64 and G.get_option("plain_group") == 8
    assert np.array_equal(G.batch_query(pairs, algo="bids"), exp)
    assert G.stats()["dense_searches"] > 0
    G.close()
