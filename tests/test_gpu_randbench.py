"""Measurement support. The scattered-access reference kernel that the
benchmark prices the round kernel against (libppsp_probe.so): both kinds run
and report a time, and a 16-byte scattered load is not slower per access
than a 64-bit atomic. The sampled timing of round-kernel launches."""
import pytest

pytestmark = pytest.mark.gpu


def test_randbench_runs():
    import torch
    from paper_2506_16488_amd import probe
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    ops = 1 << 24
    load_ms = probe.randbench(1 << 24, ops, 0)
    atom_ms = probe.randbench(1 << 24, ops, 1)
    assert 0 < load_ms < 1000 and 0 < atom_ms < 1000
    assert load_ms <= 1.5 * atom_ms


def test_sampled_round_kernel_timing():
    """"profile" K times every K-th round-kernel launch: relax_timed counts
    them, relax_kernel_ms sums their durations; results are unchanged."""
    import numpy as np
    import gen
    import oracle
    import paper_2506_16488_amd as P
    g = gen.lattice(120, 0.05, seed=77)
    pairs = gen.pairs_uniform(g.n, 40, seed=78)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs)
    G = P.Graph.from_host(g)
    for k in (0, 1, 4):
        G.set_option("profile", k)
        assert np.array_equal(G.batch_query(pairs, algo="bidastar"), exp)
        st = G.stats()
        if k == 0:
            assert st["relax_timed"] == 0 and st["relax_kernel_ms"] == 0
        else:
            assert st["relax_timed"] == (st["relax_launches"] + k - 1) // k
            assert st["relax_kernel_ms"] > 0
    G.close()
