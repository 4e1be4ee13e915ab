"""Out-of-memory handling, driven from the host by the library's allocation
hook (include/gwn_test.h): the k-th device allocation of a call fails with
out-of-memory, for every k the call makes, without exhausting the device.
Every such call must return GWN_E_OOM with a message, create no handle,
leave the library usable, and the next call must give the same results as
before.  The allocation-free batch query must succeed with every allocation
failing."""
import ctypes

import numpy as np
import pytest

from paper_2605_01536_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture
def hook(gwn):
    L = gwn.load()
    L.gwn_test_fail_alloc_after.argtypes = [ctypes.c_int64]
    L.gwn_test_fail_alloc_after.restype = ctypes.c_int64
    L.gwn_test_fail_alloc_after(-1)
    yield L.gwn_test_fail_alloc_after
    L.gwn_test_fail_alloc_after(-1)


def _each_failure(gwn, hook, call):
    """Run call() once to count its allocations, then once per allocation with
    that allocation failing; returns the count."""
    hook(-1)
    call()
    torch.cuda.synchronize()
    n = hook(-1)
    assert n > 0
    for k in range(n):
        hook(k)
        with pytest.raises(gwn.GwnError) as e:
            call()
        hook(-1)
        assert e.value.status == 2, (k, e.value)
        assert "out of memory" in str(e.value), str(e.value)
    torch.cuda.synchronize()
    return n


def test_out_of_memory_in_build_and_queries(gwn, hook):
    s = W.torus_soup(seed=2)
    V, F = torch.from_numpy(s.V).cuda(), torch.from_numpy(s.F).cuda()
    free0 = torch.cuda.mem_get_info()[0]
    nb = _each_failure(gwn, hook, lambda: gwn.Mesh(V, F, weld=True))
    m = gwn.Mesh(V, F)
    lo, hi = s.bbox()
    # a dense batch takes the Morton order (its keys, permutation and sort scratch
    # are allocated), and without chi_out the crossing counts are too
    Q = torch.from_numpy(W.uniform_box(np.random.default_rng(3), 300_000, lo, hi)).cuda()
    ref = gwn.query_batch(m, Q)
    nq = _each_failure(gwn, hook, lambda: gwn.query_batch(m, Q))
    assert torch.equal(gwn.query_batch(m, Q), ref)
    # the allocation-free variant allocates nothing: it works with every allocation failing
    hook(0)
    w = gwn.query_batch_noalloc(m, Q)
    hook(-1)
    assert torch.equal(w, ref)
    # the library's sort
    keys = torch.randint(0, 2 ** 31 - 1, (100_000,), dtype=torch.int32, device="cuda")
    _each_failure(gwn, hook, lambda: gwn.radix_sort(keys, keys))
    # a multi-mesh plan and a network
    meshes = [m, gwn.Mesh(V, F)]
    offs = np.array([0, 1000, 2000], np.int64)
    _each_failure(gwn, hook, lambda: gwn.MultiPlan(meshes, Q[:2000], offs))
    _each_failure(gwn, hook, lambda: gwn.Surrogate(seed=1))
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"allocations: build {nb}, batch {nq}; free device memory {free0 / 2**30:.2f} -> {free1 / 2**30:.2f} GiB")
