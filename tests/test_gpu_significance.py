"""Triad significance profile on the GPU (z-scores of a graph's census against
a batched census of its degree-preserving randomisations) against the
oracle's exact profile computed from oracle censuses."""
import numpy as np
import pytest

import oracle
from oracle.significance import profile
from paper_1209_6308_amd import graphs, triad

pytestmark = pytest.mark.gpu

# double-precision moments over G graphs: relative error of order G * 2^-52
TOL = dict(rel=1e-9, abs=1e-9)


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no HIP device")
    return t


def _ens_tensor(torch, rows):
    a = np.array([[int(x) & ((1 << 64) - 1) for x in r] for r in rows], dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).cuda()


@pytest.mark.parametrize("scale,K,seed", [(9, 16, 1), (12, 64, 2)])
def test_randomised_ensemble_profile(torch, scale, K, seed):
    g = graphs.rmat(scale, 8, seed=seed, recip_p=0.2)
    B = graphs.randomised_ensemble(g, K, seed=seed)
    d = triad.batch_to_device(B)
    out = torch.empty((B.G, 16), dtype=torch.int64, device="cuda")
    plan = triad.BatchPlan(B.G, int(B.vbase[-1]), B.nnz, *d, d_out=out)
    plan.launch()
    rows = plan.result()
    plan.close()
    want_rows = [oracle.census(B.graph(k)) for k in range(B.G)]
    assert rows == want_rows
    real = oracle.census(g)
    z, sp = triad.significance_profile(out, real)
    wz, wsp = profile(real, want_rows)
    assert z == pytest.approx(wz, **TOL)
    assert sp == pytest.approx(wsp, **TOL)


def test_hand_example_and_large_counts(torch):
    c = (1 << 62) + 99  # far above 2^53, small spread
    rows = [[0] * 16 for _ in range(3)]
    for k, x in enumerate((1, 2, 3)):
        rows[k][5] = x
        rows[k][9] = 10
        rows[k][7] = c + 2 * k
    real = [0] * 16
    real[5], real[9], real[7] = 5, 99, c + 7
    z, sp = triad.significance_profile(_ens_tensor(torch, rows), real)
    wz, wsp = profile(real, rows)
    assert z[5] == pytest.approx(3.0, rel=1e-15) and z[9] == 0.0
    assert z == pytest.approx(wz, **TOL)
    assert sp == pytest.approx(wsp, **TOL)


def test_constant_ensemble_and_errors(torch):
    g = graphs.rmat(8, 4, seed=1)
    c = oracle.census(g)
    z, sp = triad.significance_profile(_ens_tensor(torch, [c, c, c]), c)
    assert z == [0.0] * 16 and sp == [0.0] * 16
    with pytest.raises(triad.TriadError) as e:
        triad.significance_profile(_ens_tensor(torch, [c]), c)
    assert e.value.status == triad.EINVAL
