"""The no-allocation census entry point (static device scratch) against the
allocating one, through the C ABI: identical counts on calls in a row, the
later ones smaller, and a clear error for graphs beyond the scratch size."""
import ctypes

import numpy as np
import pytest

from paper_1209_6308_amd import graphs, triad

from _helpers import random_digraph

pytestmark = pytest.mark.gpu

SCRATCH = 64 * 1024 * 1024


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no HIP device")
    return t


def _scratch_bound(n, nnz):
    """The library's scratch bound for a plain census, per buffer rounded up to
    256 bytes (the same buffers the allocating entry point takes)."""
    m = nnz // 2
    r = lambda b: (max(b, 1) + 255) // 256 * 256  # noqa: E731
    scan_b = 256 * 16
    b = r(4) + r(21 * 8)
    if n > 0:
        b += r(4 * n) + r(8 * n) + r(8 * (n + 1)) + r(4 * ((nnz >> 5) + 1)) + r(4 * (nnz + 1024))
        b += r(8 * ((n + scan_b - 1) // scan_b + 1))
    if m > 0:
        b += r(8 * m) + r(4 * m) + r(8 * m) + r(8 * m) + r(8 * (m + 1))
        b += r(8 * ((m + scan_b - 1) // scan_b + 1))
    return b


def _both(torch, g, **kw):
    d = triad.to_device(g, "cuda")
    want, st0, _ = triad.triad_census_device(g.n, g.nnz, *d, **kw)
    out = torch.full((17,), -1, dtype=torch.int64, device="cuda")
    got, st1 = triad.triad_census_device_noalloc(g.n, g.nnz, *d, d_out=out, **kw)
    dev = [int(x) & ((1 << 64) - 1) for x in out.cpu().tolist()]
    return want, got, st0, st1, dev


def test_noalloc_matches_allocating_entry(torch):
    # a large graph first, then smaller ones: the static scratch keeps the
    # previous call's contents, so each call must clear what it relies on
    big = graphs.rmat(16, 8, seed=3, recip_p=0.1)
    assert _scratch_bound(big.n, big.nnz) <= SCRATCH
    s, t = random_digraph(300, 0.05, 0.2, 11)
    cases = [(big, {}), (graphs.rmat(12, 8, seed=5, recip_p=0.15), {}),
             (graphs.rmat(12, 8, seed=5, recip_p=0.15), {"hub_threshold": 64, "chunk": 256}),
             (graphs.build_csr(300, s, t), {}), (graphs.from_arcs(3, [(0, 1), (1, 2)]), {}),
             (graphs.build_csr(5, np.zeros(0, np.int32), np.zeros(0, np.int32)), {})]
    for g, kw in cases:
        want, got, st0, st1, dev = _both(torch, g, **kw)
        assert got == want, (g.n, g.nnz, kw)
        assert st1 == st0
        assert dev[:16] == [x & ((1 << 64) - 1) for x in want]


def test_noalloc_near_the_limit(torch):
    # R-MAT scale 17, edge factor 12: 62.6 MiB of the 64 MiB scratch
    g = graphs.rmat(17, 12, seed=2)
    assert 0.97 * SCRATCH <= _scratch_bound(g.n, g.nnz) <= SCRATCH, _scratch_bound(g.n, g.nnz)
    want, got, _, _, _ = _both(torch, g)
    assert got == want


def test_noalloc_rejects_what_does_not_fit(torch):
    g = graphs.rmat(18, 16, seed=1)
    assert _scratch_bound(g.n, g.nnz) > SCRATCH
    d = triad.to_device(g, "cuda")
    out = torch.full((17,), 7, dtype=torch.int64, device="cuda")
    with pytest.raises(triad.TriadError) as e:
        triad.triad_census_device_noalloc(g.n, g.nnz, *d, d_out=out)
    assert e.value.status == triad.EINVAL and "too large" in str(e.value)
    small = graphs.rmat(10, 8, seed=1)
    ds = triad.to_device(small, "cuda")
    for kw in ({"schedule": "heuristic"}, {"timing": triad.Timing()}):
        with pytest.raises(triad.TriadError) as e:
            triad.triad_census_device_noalloc(small.n, small.nnz, *ds, d_out=out, **kw)
        assert e.value.status == triad.EINVAL
    assert torch.all(out == 7), "output written on error"
    # and the entry point still works after the rejections
    want, got, _, _, _ = _both(torch, small)
    assert got == want
