"""The allocation-free sort entry point (hgs_sort_pairs_noalloc) through the
C ABI: two calls in a row, the second on a smaller input, each equal to the
allocating entry point (hgs_sort_pairs) on the same input bit for bit and to
a stable host sort of the low key bits; the largest size it accepts; and the
error for one pair more."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_15186_amd import hgs
    r = hgs.Renderer(0)
    yield r
    r.close()


def _pairs(n, key_bits, seed):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    # many equal digits, so that stability matters
    keys[: n // 3] &= np.uint32(0xFFFF00FF)
    vals = rng.permutation(n).astype(np.uint32)
    return keys, vals


def _dev(a):
    return torch.from_numpy(a.view(np.int32).copy()).cuda()


def _host_sorted(keys, vals, key_bits):
    low = keys & np.uint32((1 << key_bits) - 1 if key_bits < 32 else 0xFFFFFFFF)
    o = np.argsort(low, kind="stable")
    return keys[o], vals[o]


@pytest.mark.parametrize("digits", [8, 11])
def test_noalloc_sort_equals_the_allocating_sort(R, digits):
    from paper_2603_15186_amd import hgs
    R.set_option(hgs.HGS_OPT_SORT_DIGIT_BITS, digits)
    try:
        # two calls in a row, the second smaller: what the first left in the
        # shared scratch area must not leak into the second
        for n, bits, seed in ((3_000_001, 27, 1 + digits), (777_777, 13, 2 + digits), (1, 32, 3)):
            keys, vals = _pairs(n, bits, seed)
            k1, v1 = _dev(keys), _dev(vals)
            R.sort_pairs(k1, v1, bits)
            k2, v2 = _dev(keys), _dev(vals)
            R.sort_pairs_noalloc(k2, v2, bits)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(k2.cpu().numpy(), k1.cpu().numpy())
            np.testing.assert_array_equal(v2.cpu().numpy(), v1.cpu().numpy())
            wk, wv = _host_sorted(keys, vals, bits)
            np.testing.assert_array_equal(k2.cpu().numpy().view(np.uint32), wk)
            np.testing.assert_array_equal(v2.cpu().numpy().view(np.uint32), wv)
    finally:
        R.set_option(hgs.HGS_OPT_SORT_DIGIT_BITS, 8)


def test_noalloc_sort_limits(R):
    from paper_2603_15186_amd import hgs
    n = hgs.HGS_SORT_NOALLOC_MAX
    keys, vals = _pairs(n, 32, 9)
    k, v = _dev(keys), _dev(vals)
    R.sort_pairs_noalloc(k, v, 32)
    torch.cuda.synchronize()
    wk, wv = _host_sorted(keys, vals, 32)
    np.testing.assert_array_equal(k.cpu().numpy().view(np.uint32), wk)
    np.testing.assert_array_equal(v.cpu().numpy().view(np.uint32), wv)
    big = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(hgs.HgsError) as ei:
        R.sort_pairs_noalloc(big, big.clone(), 16)
    assert ei.value.status == hgs.HGS_E_INVALID
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    R.sort_pairs_noalloc(empty, empty, 16)
    # a captured graph of the call replays it on new contents of the buffers
    keys, vals = _pairs(200_000, 20, 10)
    k, v = _dev(keys), _dev(vals)
    src_k, src_v = k.clone(), v.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        g.capture_begin()
        R.sort_pairs_noalloc(k, v, 20, stream=s)
        g.capture_end()
    torch.cuda.synchronize()
    for rep in range(3):
        keys, vals = _pairs(200_000, 20, 11 + rep)
        k.copy_(_dev(keys))
        v.copy_(_dev(vals))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        wk, wv = _host_sorted(keys, vals, 20)
        np.testing.assert_array_equal(k.cpu().numpy().view(np.uint32), wk)
        np.testing.assert_array_equal(v.cpu().numpy().view(np.uint32), wv)
    del src_k, src_v
