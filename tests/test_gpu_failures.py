"""Failure paths forced from the host: the memory cap (TRIAD_ENOMEM) and the
device-fault test hook (TRIAD_EDEVICE). A failing call must leave every output
as it was (sentinel-filled buffers stay intact); the same call without the
condition gives the oracle's census. Every kernel still runs to its normal end:
the cap stops a call before an allocation, the hook only sets the error flag."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1209_6308_amd import graphs, triad

pytestmark = pytest.mark.gpu

SENT = 0x5A5A5A5A5A5A5A5A


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no HIP device")
    return t


@pytest.fixture(autouse=True)
def _clear():
    yield
    triad.set_memory_cap(0)
    triad.inject_device_error(0)


def _raw(torch, fn, g, d, nout):
    """One call of a device census entry point with sentinel-filled outputs:
    (status, device output words, host output words)."""
    d_out = torch.full((nout,), SENT, dtype=torch.int64, device="cuda")
    h = np.full(nout, SENT, dtype=np.uint64)
    o = triad.make_opts()
    st = fn(g.n, g.nnz, triad._tp(d[0]), triad._tp(d[1]), triad._tp(d[2]), ctypes.byref(o), triad._stream(),
            triad._tp(d_out), triad._p(h))
    torch.cuda.synchronize()
    return st, d_out.cpu().numpy().view(np.uint64), h


def _counts(words):
    res = [int(x) for x in words[:16]]
    res[0] += int(words[16]) << 64
    return res


def _untouched(*arrays):
    return all(bool(np.all(np.asarray(a).view(np.uint64) == SENT)) for a in arrays)


def test_memory_cap_is_an_exact_bound(torch):
    """The smallest cap that lets the census through is found by bisection;
    one byte less gives TRIAD_ENOMEM with nothing written, and at that cap the
    counts equal the oracle's."""
    g = graphs.rmat(12, 8, seed=5, recip_p=0.15)
    d = triad.to_device(g)
    fn = triad.lib().triad_census_device
    want = oracle.census(g)
    lo, hi = 0, 1 << 26  # lo fails, hi passes
    triad.set_memory_cap(hi)
    st, dw, hw = _raw(torch, fn, g, d, 17)
    assert st == 0 and _counts(hw) == want and _counts(dw) == want
    while hi - lo > 1:
        mid = (lo + hi) // 2
        triad.set_memory_cap(mid)
        st, dw, hw = _raw(torch, fn, g, d, 17)
        if st == 0:
            hi = mid
        else:
            assert st == triad.ENOMEM, triad.last_error()
            assert _untouched(dw, hw)
            lo = mid
    # the bound exceeds the graph's own arrays' worth of task records
    assert hi > 8 * g.nnz // 2
    triad.set_memory_cap(hi - 1)
    st, dw, hw = _raw(torch, fn, g, d, 17)
    assert st == triad.ENOMEM and _untouched(dw, hw)
    assert "allocation" in triad.last_error()
    triad.set_memory_cap(hi)
    st, dw, hw = _raw(torch, fn, g, d, 17)
    assert st == 0 and _counts(hw) == want and _counts(dw) == want


def test_memory_cap_host_entry(torch):
    """triad_census_ex: the input copies count against the cap as well."""
    g = graphs.rmat(10, 8, seed=3, recip_p=0.2)
    L = triad.lib()

    def call():
        out = np.full(16, SENT, dtype=np.uint64)
        hi = np.full(1, SENT, dtype=np.uint64)
        st = L.triad_census_ex(g.n, triad._p(g.offsets), triad._p(g.nbrs), triad._p(g.flags), None,
                               triad._p(out), triad._p(hi))
        return st, out, hi

    in_bytes = 8 * (g.n + 1) + 4 * g.nnz + (g.nnz + 3) // 4 + 17 * 8
    triad.set_memory_cap(in_bytes - 1)
    st, out, hi = call()
    assert st == triad.ENOMEM and _untouched(out, hi)
    assert "input copy" in triad.last_error()
    triad.set_memory_cap(in_bytes + 256)  # the copies fit, the scratch does not
    st, out, hi = call()
    assert st == triad.ENOMEM and _untouched(out, hi)
    triad.set_memory_cap(0)
    st, out, hi = call()
    assert st == 0
    assert _counts(np.concatenate([out, hi])) == oracle.census(g)


def test_memory_cap_other_entry_points(torch):
    """CSR construction, the incremental census, the labelled census, the
    significance profile and batch plans all stop at the cap, writing nothing."""
    g = graphs.rmat(10, 8, seed=4, recip_p=0.1)
    d = triad.to_device(g)
    triad.set_memory_cap(1024)
    L = triad.lib()
    # CSR construction
    rng = np.random.default_rng(1)
    src = torch.from_numpy(rng.integers(0, 500, 4000).astype(np.int32)).cuda()
    dst = torch.from_numpy(rng.integers(0, 500, 4000).astype(np.int32)).cuda()
    off = torch.full((501,), SENT, dtype=torch.int64, device="cuda")
    nbr = torch.full((8000,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    flg = torch.full((2000,), 0x5A, dtype=torch.uint8, device="cuda")
    nnz = ctypes.c_int64(-7)
    st = L.triad_csr_from_arcs(500, 4000, triad._tp(src), triad._tp(dst), triad._stream(), triad._tp(off),
                               triad._tp(nbr), triad._tp(flg), ctypes.byref(nnz), None)
    torch.cuda.synchronize()
    assert st == triad.ENOMEM and nnz.value == -7
    assert _untouched(off.cpu().numpy()) and bool((nbr == 0x5A5A5A5A).all()) and bool((flg == 0x5A).all())
    # incremental census
    want = oracle.census(g)
    cin = np.zeros(17, dtype=np.uint64)
    cin[:16] = np.array([x & ((1 << 64) - 1) for x in want], dtype=np.uint64)
    cout = np.full(17, SENT, dtype=np.uint64)
    us = torch.tensor([1, 2, 3], dtype=torch.int32, device="cuda")
    ud = torch.tensor([4, 5, 6], dtype=torch.int32, device="cuda")
    ui = torch.tensor([1, 1, 0], dtype=torch.uint8, device="cuda")
    chg = ctypes.c_int64(-7)
    triad.set_memory_cap(64)
    st = L.triad_census_update(g.n, g.nnz, triad._tp(d[0]), triad._tp(d[1]), triad._tp(d[2]), 3, triad._tp(us),
                               triad._tp(ud), triad._tp(ui), triad._p(cin), triad._p(cout), None, None, None,
                               None, ctypes.byref(chg), triad._stream())
    assert st == triad.ENOMEM and _untouched(cout) and chg.value == -7
    # labelled census
    triad.set_memory_cap(1024)
    st, dw, hw = _raw(torch, L.triad_labelled_census_device, g, d, 65)
    assert st == triad.ENOMEM and _untouched(dw, hw)
    # significance profile (256 bytes of scratch)
    triad.set_memory_cap(255)
    ens = torch.zeros((4, 16), dtype=torch.int64, device="cuda")
    z = np.full(16, SENT, dtype=np.uint64)
    sp = np.full(16, SENT, dtype=np.uint64)
    real = np.zeros(16, dtype=np.uint64)
    st = L.triad_significance_profile(4, triad._tp(ens), triad._p(real), triad._p(z), triad._p(sp), triad._stream())
    assert st == triad.ENOMEM and _untouched(z, sp)
    # batch plan
    triad.set_memory_cap(1024)
    B = graphs.null_ensemble(G=4, seed=7, nmin=64, nmax=100, dmin=4, dmax=8)
    db = triad.batch_to_device(B)
    with pytest.raises(triad.TriadError) as e:
        triad.triad_census_batch(B.G, int(B.vbase[-1]), B.nnz, *db)
    assert e.value.status == triad.ENOMEM
    triad.set_memory_cap(0)
    got = triad.triad_census_batch(B.G, int(B.vbase[-1]), B.nnz, *db)
    assert got == [[x & ((1 << 64) - 1) for x in oracle.census(B.graph(i))] for i in range(B.G)]


def test_injected_device_error(torch):
    """Each injected fault fails exactly one census that got past validation,
    with TRIAD_EDEVICE and nothing written; a call that fails validation first
    leaves the fault pending."""
    g = graphs.rmat(11, 8, seed=6, recip_p=0.2)
    d = triad.to_device(g)
    L = triad.lib()
    want = oracle.census(g)
    triad.inject_device_error(2)
    for _ in range(2):
        st, dw, hw = _raw(torch, L.triad_census_device, g, d, 17)
        assert st == triad.EDEVICE and _untouched(dw, hw)
        assert "fault" in triad.last_error()
    st, dw, hw = _raw(torch, L.triad_census_device, g, d, 17)
    assert st == 0 and _counts(hw) == want and _counts(dw) == want
    # a call rejected before the census does not take the pending fault
    triad.inject_device_error(1)
    o = triad.make_opts()
    bad = torch.zeros(17, dtype=torch.int64, device="cuda")
    assert L.triad_census_device(-1, 0, triad._tp(d[0]), None, None, ctypes.byref(o), triad._stream(),
                                 triad._tp(bad), None) == triad.EINVAL
    st, dw, hw = _raw(torch, L.triad_census_device_noalloc, g, d, 17)
    assert st == triad.EDEVICE and _untouched(dw, hw)
    # the labelled census and the host-pointer entry take it the same way
    triad.inject_device_error(1)
    st, dw, hw = _raw(torch, L.triad_labelled_census_device, g, d, 65)
    assert st == triad.EDEVICE and _untouched(dw, hw)
    triad.inject_device_error(1)
    out = np.full(16, SENT, dtype=np.uint64)
    hi = np.full(1, SENT, dtype=np.uint64)
    st = L.triad_census_ex(g.n, triad._p(g.offsets), triad._p(g.nbrs), triad._p(g.flags), None, triad._p(out),
                           triad._p(hi))
    assert st == triad.EDEVICE and _untouched(out, hi)
    # count 0 cancels what is pending
    triad.inject_device_error(3)
    triad.inject_device_error(0)
    st, dw, hw = _raw(torch, L.triad_census_device, g, d, 17)
    assert st == 0 and _counts(hw) == want


def test_batch_error_writes_nothing(torch):
    """A member that fails the device-side checks: the batch reports it and
    leaves the caller's output as it was."""
    B = graphs.null_ensemble(G=4, seed=7, nmin=64, nmax=100, dmin=4, dmax=8)
    nb = B.nbrs.copy()
    nb[5] = 100000  # out of its graph's range
    d = list(triad.batch_to_device(B))
    d[2] = torch.from_numpy(nb).cuda()
    out = torch.full((B.G, 16), SENT, dtype=torch.int64, device="cuda")
    o = triad.make_opts()
    st = triad.lib().triad_census_batch(B.G, int(B.vbase[-1]), B.nnz, *(triad._tp(x) for x in d), ctypes.byref(o),
                                        triad._stream(), triad._tp(out))
    torch.cuda.synchronize()
    assert st == triad.ERANGE
    assert _untouched(out.cpu().numpy())


def test_held_memory_is_reused_and_released(torch):
    """Scratch blocks stay with the library between calls: a second call of the
    same shape takes them again (the held total is unchanged after it), the
    counts stay the oracle's, and releasing frees every held block."""
    g = graphs.rmat(12, 8, seed=9, recip_p=0.15)
    d = triad.to_device(g)
    want = oracle.census(g)
    triad.release_memory()
    assert triad.held_memory() == 0
    fn = triad.lib().triad_census_device
    st, dw, hw = _raw(torch, fn, g, d, 17)
    assert st == 0 and _counts(hw) == want
    held = triad.held_memory()
    assert held > 8 * g.nnz // 2  # at least the task list
    for _ in range(2):
        st, dw, hw = _raw(torch, fn, g, d, 17)
        assert st == 0 and _counts(hw) == want and _counts(dw) == want
        assert triad.held_memory() == held
    # a failing call (device fault flagged) gives its blocks back as well
    triad.inject_device_error(1)
    st, dw, hw = _raw(torch, fn, g, d, 17)
    assert st == triad.EDEVICE and _untouched(dw, hw)
    assert triad.held_memory() == held
    # the labelled census takes and gives back blocks as well
    st, dw, hw = _raw(torch, triad.lib().triad_labelled_census_device, g, d, 65)
    assert st == 0
    assert triad.release_memory() == 0 and triad.held_memory() == 0
    st, dw, hw = _raw(torch, fn, g, d, 17)
    assert st == 0 and _counts(hw) == want
    triad.release_memory()
