"""gwn_query_batch_noalloc (the batch query with its temporaries in the
library's fixed per-GPU scratch) against gwn_query_batch: the same kernels,
so the same bits, on two calls in a row -- a dense batch that takes the Morton
order (its sort runs in the scratch) and then a smaller one that takes the
per-point-workgroup path -- with and without caller crossing-count buffers,
in both precisions; the size limit is refused with an error."""
import numpy as np
import pytest

from paper_2605_01536_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torus(gwn):
    s = W.torus_soup(seed=2)
    m = gwn.Mesh(torch.from_numpy(s.V).cuda(), torch.from_numpy(s.F).cuda())
    return s, m


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_equals_batch_on_two_calls(gwn, torus, prec):
    s, m = torus
    rng = np.random.default_rng(77)
    lo, hi = s.bbox()
    big = torch.from_numpy(W.uniform_box(rng, 700_000, lo, hi)).cuda()      # >= 2^18: Morton-ordered
    small = torch.from_numpy(W.uniform_box(rng, 5_000, lo, hi)).cuda()      # <= 8,192: split boundary
    for Q in (big, small):
        w_ref, c_ref = gwn.query_batch(m, Q, prec=prec, want_chi=True)
        w_na, c_na = gwn.query_batch_noalloc(m, Q, prec=prec, want_chi=True)
        w_nc = gwn.query_batch_noalloc(m, Q, prec=prec)          # crossing counts in the scratch
        torch.cuda.synchronize()
        assert torch.equal(c_na, c_ref)
        assert torch.equal(w_na, w_ref)
        assert torch.equal(w_nc, w_ref)


def test_noalloc_limits(gwn, torus):
    s, m = torus
    Q = torch.zeros((gwn.NOALLOC_MAX_POINTS + 1, 3), device="cuda")
    with pytest.raises(gwn.GwnError, match="exceed the maximum"):
        gwn.query_batch_noalloc(m, Q)
    e = torch.empty((0, 3), device="cuda")
    assert gwn.query_batch_noalloc(m, e).numel() == 0
    # exactly the maximum is served
    lo, hi = s.bbox()
    Q = torch.from_numpy(W.uniform_box(np.random.default_rng(5), gwn.NOALLOC_MAX_POINTS, lo, hi)).cuda()
    assert torch.equal(gwn.query_batch_noalloc(m, Q), gwn.query_batch(m, Q))
