"""The scattered-access reference kernel the benchmark prices the round
kernel against (ppsp_randbench): both kinds run and report a time, and a
16-byte scattered load is not slower per access than a 64-bit atomic."""
import pytest

pytestmark = pytest.mark.gpu


def test_randbench_runs():
    import torch
    import paper_2506_16488_amd as P
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    ops = 1 << 24
    load_ms = P.randbench(1 << 24, ops, 0)
    atom_ms = P.randbench(1 << 24, ops, 1)
    assert 0 < load_ms < 1000 and 0 < atom_ms < 1000
    assert load_ms <= 1.5 * atom_ms
