"""The library's device radix sort and scans (include/gwn_prims.h) against
numpy's stable sort and cumulative sum / maximum, bit for bit: sizes around the
4,096-key tile and across several levels of the scan's recursion, full and
partial bit ranges, 64-bit keys, heavy duplicates (stability) and one-digit
inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = [1, 2, 255, 4095, 4096, 4097, 65537, 1 << 20, (1 << 22) + 13]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _ref(keys, begin, end, bits):
    k = keys.astype(np.uint64) if bits == 64 else keys.astype(np.uint64) & np.uint64(0xFFFFFFFF)
    width = end - begin
    mask = np.uint64((1 << width) - 1) if width < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    d = (k >> np.uint64(begin)) & mask
    return np.argsort(d, kind="stable")


@pytest.mark.parametrize("n", SIZES)
def test_sort_u32_pairs_full_range(gwn, n):
    rng = np.random.default_rng(n)
    keys = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(n, dtype=np.int32)
    ko, vo = gwn.radix_sort(_dev(keys.view(np.int32)), _dev(vals))
    order = _ref(keys, 0, 32, 32)
    assert np.array_equal(ko.cpu().numpy().view(np.uint32), keys[order])
    assert np.array_equal(vo.cpu().numpy(), vals[order])


@pytest.mark.parametrize("n", [4097, 300001, 1 << 21])
@pytest.mark.parametrize("rng_bits", [(0, 64), (32, 62), (0, 19), (5, 13), (60, 64)])
def test_sort_u64_pairs_bit_ranges(gwn, n, rng_bits):
    b0, b1 = rng_bits
    rng = np.random.default_rng(n + b0)
    # few distinct values in the sorted bits: long runs of equal keys test stability
    keys = rng.integers(0, 2 ** 63, n, dtype=np.int64).astype(np.uint64) * np.uint64(2) + rng.integers(0, 2, n).astype(np.uint64)
    keys[rng.random(n) < 0.5] = keys[0]
    vals = rng.permutation(n).astype(np.int32)
    ko, vo = gwn.radix_sort(_dev(keys.view(np.int64)), _dev(vals), b0, b1)
    order = _ref(keys, b0, b1, 64)
    assert np.array_equal(ko.cpu().numpy().view(np.uint64), keys[order])
    assert np.array_equal(vo.cpu().numpy(), vals[order])


def test_sort_keys_only_and_one_digit(gwn):
    n = 100000
    keys = np.full(n, 0x1234_5678_9ABC_DEF0, dtype=np.uint64)
    keys[::7] += np.uint64(1 << 40)
    ko, vo = gwn.radix_sort(_dev(keys.view(np.int64)), None, 32, 62)
    assert vo is None
    assert np.array_equal(ko.cpu().numpy().view(np.uint64), keys[_ref(keys, 32, 62, 64)])
    # an empty bit range copies the input
    ko, _ = gwn.radix_sort(_dev(keys.view(np.int64)), None, 8, 8)
    assert np.array_equal(ko.cpu().numpy().view(np.uint64), keys)
    with pytest.raises(gwn.GwnError):
        gwn.radix_sort(_dev(keys.view(np.int64)), None, 10, 65)


@pytest.mark.parametrize("n", SIZES + [(1 << 24) + 7])
def test_scans(gwn, n):
    rng = np.random.default_rng(n + 1)
    x = rng.integers(-1000, 1000, n).astype(np.int32)
    ex = gwn.scan(_dev(x), "exclusive_sum").cpu().numpy()
    ref = np.concatenate([[0], np.cumsum(x.astype(np.int64))[:-1]]).astype(np.int32)
    assert np.array_equal(ex, ref)
    mx = gwn.scan(_dev(x), "inclusive_max").cpu().numpy()
    assert np.array_equal(mx, np.maximum.accumulate(x))


def test_empty_inputs(gwn):
    e32 = torch.empty(0, dtype=torch.int32, device="cuda")
    k, v = gwn.radix_sort(e32, e32)
    assert k.numel() == 0 and v.numel() == 0
    assert gwn.scan(e32).numel() == 0
