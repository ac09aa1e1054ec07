"""The C-ABI library loads and exports every entry point its header declares;
host-only entry points (schedule, primality) match the input generator and
sympy.  No GPU needed."""
import os
import re

import numpy as np
import pytest
import sympy

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def _lib_or_skip():
    import paper_2505_24256_amd as zr
    if not os.path.exists(zr.LIB_PATH):
        pytest.skip("library not built")
    return zr


def declared_functions():
    text = "\n".join(open(os.path.join(INCLUDE, f)).read() for f in sorted(os.listdir(INCLUDE)) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"typedef\s+\w+\s*\(\s*\*\s*\w+\s*\)\s*\([^;]*\);", "", text)
    names = set()
    for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M):
        name = m.group(1)
        if name in ("typedef", "if", "return"):
            continue
        names.add(name)
    # function-pointer typedefs are not symbols
    names -= {"zr_blackbox_fn"}
    return sorted(names)


def test_header_lists_match_binding():
    zr = pytest.importorskip("paper_2505_24256_amd")
    assert set(declared_functions()) == set(zr.EXPORTS)


def test_library_exports_every_declared_symbol():
    zr = _lib_or_skip()
    L = zr.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_library_is_gfx950_code_object():
    zr = _lib_or_skip()
    data = open(zr.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_library_schedule_equals_input_generator():
    zr = _lib_or_skip()
    p = synth.make_prime()
    nn = [30, 7, 0, 41]
    ys, an, nodes, pr = zr.schedule(p, nn, seed=1234, nprobes=3)
    s = synth.make_schedule(p, 4, nn, 1234, 3)
    assert np.array_equal(ys, s.y)
    assert np.array_equal(an, s.anchor)
    assert np.array_equal(nodes, s.nodes_concat())
    assert np.array_equal(pr, s.probes)


def test_library_primality_matches_sympy():
    zr = _lib_or_skip()
    rng = np.random.default_rng(3)
    for x in list(rng.integers(1 << 61, 1 << 62, 400, dtype=np.int64) * 2 + 1) + [2047, 3215031751, (1 << 61) - 1,
                                                                                (1 << 63) - 25, 561]:
        assert zr.is_prime(int(x)) == sympy.isprime(int(x)), int(x)


def test_thiele_node_count():
    zr = _lib_or_skip()
    for a in range(0, 25):
        for b in range(0, 25):
            assert zr.thiele_nodes(a, b) == synth.thiele_nodes_needed(a, b)
