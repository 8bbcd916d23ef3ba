"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function include/ppsp.h declares, and
reject invalid arguments before touching the device. The heuristic of
Sections 3.3 and 3.5 is a host-callable function, pinned here against exact
integer arithmetic and against the consistency property the correctness
theorems assume.
"""
import math
import os
import re

import numpy as np
import pytest

import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ppsp():
    import paper_2506_16488_amd as P
    try:
        P.lib()
    except ImportError:
        from paper_2506_16488_amd import build
        build.build()
        P.lib()
    return P


def test_header_symbols_exported():
    P = _ppsp()
    text = open(os.path.join(ROOT, "include", "ppsp.h")).read()
    declared = set(re.findall(r"^\s*(?:int|uint64_t|const char \*)\s*(ppsp_\w+)\s*\(", text, re.M))
    assert {"ppsp_graph_create", "ppsp_query", "ppsp_batch_query"} <= declared
    for name in declared:
        assert hasattr(P.lib(), name), name
    assert set(P.EXPORTS) == declared


def test_status_strings_and_version():
    P = _ppsp()
    assert P.status_str(0) == "ok"
    for c in range(-11, 0):
        assert P.status_str(c) != "unknown status"
    assert re.match(r"\d+\.\d+\.\d+", P.version())


def _h_exact(x0, y0, x1, y1, ws, fb):
    return math.isqrt(ws * ws * ((x1 - x0) ** 2 + (y1 - y0) ** 2)) >> fb


def test_heuristic_exact_integer():
    P = _ppsp()
    rng = np.random.default_rng(0)
    cases = [(0, 0, 0, 0, 1000, 8), (0, 0, 256, 0, 1000, 8), (0, 0, 256, 256, 1000, 8),
             (5, 7, 5, 8, 1, 0), (-100, 3, 77, -9, 3, 2)]
    for _ in range(3000):
        a = rng.integers(-(1 << 20), 1 << 20, 4)
        cases.append((int(a[0]), int(a[1]), int(a[2]), int(a[3]), int(rng.choice([1, 7, 1000, 1024])),
                      int(rng.integers(0, 12))))
    for c in cases:
        assert P.heuristic_fx(*c) == _h_exact(*c), c
    # hand-worked values: 1 cell (256 units) at scale 1000 -> 1000; unit diagonal -> 1414
    assert P.heuristic_fx(0, 0, 256, 0, 1000, 8) == 1000
    assert P.heuristic_fx(0, 0, 256, 256, 1000, 8) == 1414
    assert P.heuristic_fx(0, 0, 3 * 256, 4 * 256, 1000, 8) == 5000


def test_heuristic_range_limit():
    P = _ppsp()
    big = (1 << 31) - 1
    assert P.heuristic_fx(-big, -big, big, big, 1000, 8) == (1 << 64) - 1


def test_heuristic_consistent_on_lattice():
    """h(u) <= w(u,v) + h(v) on sampled arcs and targets; h(t) = 0."""
    P = _ppsp()
    g = gen.lattice(64, 0.2, seed=8)
    rng = np.random.default_rng(2)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr.astype(np.int64)))
    xy = g.coords
    for t in rng.integers(0, g.n, 4).tolist():
        tx, ty = int(xy[t, 0]), int(xy[t, 1])
        assert P.heuristic_fx(tx, ty, tx, ty, 1000, 8) == 0
        for e in rng.integers(0, g.m, 1500).tolist():
            u, v, w = int(src[e]), int(g.col[e]), int(g.w[e])
            hu = P.heuristic_fx(int(xy[u, 0]), int(xy[u, 1]), tx, ty, 1000, 8)
            hv = P.heuristic_fx(int(xy[v, 0]), int(xy[v, 1]), tx, ty, 1000, 8)
            assert hu <= w + hv


def test_graph_create_rejects_bad_input_before_device():
    P = _ppsp()
    g = gen.grid(4, 4, 1, 9, seed=1)
    bad_rp = g.row_ptr.copy()
    bad_rp[3], bad_rp[4] = bad_rp[4], bad_rp[3] + 100    # decreasing / wrong total
    with pytest.raises(P.PPSPError) as e:
        P.graph_create(g.n, bad_rp, g.col, g.w)
    assert e.value.code == P.E_INVALID
    bad_col = g.col.copy()
    bad_col[5] = 99
    with pytest.raises(P.PPSPError) as e:
        P.graph_create(g.n, g.row_ptr, bad_col, g.w)
    assert e.value.code == P.E_RANGE
    big = np.array([[-(1 << 31), 0]] + [[(1 << 31) - 1, 0]] * 15, np.int32)
    with pytest.raises(P.PPSPError) as e:
        P.graph_create(g.n, g.row_ptr, g.col, g.w, coords=big, w_scale=1000)
    assert e.value.code == P.E_RANGE
    # exact in 64 bits, but the heuristic across the box, 2^16 * 2^23 * sqrt(2)
    # / 2^8 = 2^31.5, would not fit the kernels' signed 32-bit heuristic terms
    wide = np.zeros((g.n, 2), np.int32)
    wide[-1] = (1 << 23, 1 << 23)          # diagonal 2^23 * sqrt(2) units, 8 fractional bits
    with pytest.raises(P.PPSPError) as e:
        P.graph_create(g.n, g.row_ptr, g.col, g.w, coords=wide, w_scale=1 << 16, frac_bits=8)
    assert e.value.code == P.E_RANGE
    assert P.heuristic_fx(0, 0, 1 << 23, 1 << 23, 1 << 16, 8) >= 1 << 31


def test_no_cpu_fallback_in_binding():
    """The binding marshals arguments only: it never imports the oracle."""
    src = open(os.path.join(ROOT, "paper_2506_16488_amd", "__init__.py")).read()
    assert "oracle" not in src.replace("marshals", "")
    for f in os.listdir(os.path.join(ROOT, "paper_2506_16488_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_2506_16488_amd", "csrc", f)).read()


def test_randbench_probe_is_outside_the_search_library():
    """The scattered-access probe lives in its own library; it rejects bad
    arguments before touching a device."""
    P = _ppsp()
    from paper_2506_16488_amd import probe
    assert _not_exported(P.SO_PATH, "ppsp_randbench")
    for words, acc, kind in ((1, 10, 0), (1 << 20, 0, 0), (1 << 20, 10, 2), ((1 << 40) + 2, 10, 0)):
        with pytest.raises(ValueError):
            probe.randbench(words, acc, kind)


def _not_exported(so, name):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", so], capture_output=True, text=True).stdout
    return all(l.split()[-1] != name for l in out.splitlines() if l.strip())


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding passes through the C ABI has the size and
    field offsets the header gives it (a C program built against
    include/ppsp.h prints them)."""
    import ctypes
    import shutil
    import subprocess
    import paper_2506_16488_amd as P
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    pairs = [("ppsp_opts", P.Opts), ("ppsp_stats", P.Stats), ("ppsp_tune_result", P.TuneResult),
             ("ppsp_fit_report", P.FitReport), ("ppsp_trace_spec", P.TraceSpec),
             ("ppsp_server_counters", P.ServerCounters)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ppsp.h"', "int main(void) {"]
    for cname, cls in pairs:
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n") if l)
    for cname, cls in pairs:
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(cls, f).offset, (cname, f)
