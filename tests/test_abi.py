"""The C ABI library on the host: it loads, exports every declared symbol, and
its host-side validation returns the documented status codes (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1209_6308_amd import _build, graphs, triad

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "triad.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(triad_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = triad.lib()
    syms = declared_symbols()
    assert "triad_census" in syms and "triad_census_device" in syms
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing
    assert L.triad_version() == 1


def test_binding_names_match_header():
    assert sorted(triad.EXPORTS) == declared_symbols()


def test_no_oracle_in_product_path():
    # the product library and its binding never import, load or name the oracle
    pkg = os.path.join(ROOT, "paper_1209_6308_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", src, re.M), fn
                if not fn.endswith(".py"):
                    assert "oracle" not in src.lower() or fn == "graphgen.cpp", fn


def _valid():
    g = graphs.rmat(8, 4, seed=1, recip_p=0.2)
    return g.n, g.offsets.copy(), g.nbrs.copy(), g.flags.copy()


def test_host_validation_ok():
    n, off, nb, fl = _valid()
    assert triad.triad_validate_host(n, off, nb, fl, 0) == 0
    assert triad.triad_validate_host(n, off, nb, fl, 1) == 0


def test_host_validation_errors():
    n, off, nb, fl = _valid()
    r = int(np.argmax(np.diff(off)))
    b = int(off[r])
    x = nb.copy(); x[b], x[b + 1] = x[b + 1], x[b]
    assert triad.triad_validate_host(n, off, x, fl, 0) == triad.EUNSORTED
    x = nb.copy(); x[b + 1] = x[b]
    assert triad.triad_validate_host(n, off, x, fl, 0) == triad.EUNSORTED  # duplicate entry
    x = nb.copy(); x[-1] = n
    assert triad.triad_validate_host(n, off, x, fl, 0) == triad.ERANGE
    x = nb.copy(); x[0] = -1
    assert triad.triad_validate_host(n, off, x, fl, 0) == triad.ERANGE
    f = fl.copy(); f[0] &= 0xFC
    assert triad.triad_validate_host(n, off, nb, f, 0) == triad.ERANGE
    o = off.copy(); o[5], o[6] = o[6], o[5] - 0
    if o[6] < o[5]:
        assert triad.triad_validate_host(n, o, nb, fl, 0) == triad.ERANGE
    o = off.copy(); o[0] = 1
    assert triad.triad_validate_host(n, o, nb, fl, 0) == triad.ERANGE
    # self-loop: put the row's own id into it (keeping it sorted)
    x = nb.copy(); seg = x[b:off[r + 1]].copy(); seg[0] = r; seg.sort(); x[b:off[r + 1]] = seg
    if len(set(seg.tolist())) == seg.size:
        assert triad.triad_validate_host(n, off, x, fl, 0) == triad.ESELFLOOP
    # asymmetric flags: only level 1 sees it
    f = fl.copy(); f0 = f[0] & 3; f[0] = (f[0] & 0xFC) | (3 if f0 != 3 else 1)
    assert triad.triad_validate_host(n, off, nb, f, 0) == 0
    assert triad.triad_validate_host(n, off, nb, f, 1) == triad.EASYM
    assert triad.triad_validate_host(-1, off, nb, fl, 0) == triad.EINVAL
    assert triad.triad_validate_host(1 << 30, off, nb, fl, 0) == triad.EINVAL


def test_census_errors_before_device_use():
    # an invalid input is rejected on the host, before any device call
    n, off, nb, fl = _valid()
    x = nb.copy(); x[-1] = n + 3
    with pytest.raises(triad.TriadError) as e:
        triad.triad_census(n, off, x, fl)
    assert e.value.status == triad.ERANGE
    assert "out of range" in triad.last_error()


def test_failure_controls_on_the_host():
    # the memory cap and the device-fault hook are host settings: bad values
    # are rejected, good ones accepted, with no device involved
    L = triad.lib()
    assert L.triad_set_memory_cap(-1) == triad.EINVAL
    assert "cap" in triad.last_error()
    assert L.triad_set_memory_cap(1 << 20) == 0 and L.triad_set_memory_cap(0) == 0
    assert L.triad_test_inject_device_error(-2) == triad.EINVAL
    assert L.triad_test_inject_device_error(5) == 0 and L.triad_test_inject_device_error(0) == 0
    # nothing is held before any device call; releasing nothing succeeds
    assert triad.held_memory() == 0 and L.triad_release_memory() == 0
    # a cap does not change host-side validation
    n, off, nb, fl = _valid()
    triad.set_memory_cap(1)
    try:
        assert triad.triad_validate_host(n, off, nb, fl, 1) == 0
    finally:
        triad.set_memory_cap(0)


def test_library_is_built_for_gfx950():
    path = _build.triad_lib_path()
    data = open(path, "rb").read()
    assert b"gfx950" in data
