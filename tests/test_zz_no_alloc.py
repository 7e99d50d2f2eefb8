"""svr_radix_sort_pairs_static (the sort with library-held scratch, for
callers that cannot allocate) against svr_radix_sort_pairs (caller scratch)
through the C ABI: identical sorted pairs on two calls in a row, the second
with a smaller input, and the size limit rejected before any launch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pairs(n, seed):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 2 ** 63, size=n, dtype=np.int64).view(np.uint64)
    keys[: n // 3] = keys[: n // 3] % np.uint64(97)  # many equal keys: stability matters
    vals = np.arange(n, dtype=np.uint32)
    return keys, vals


def _sort_with_caller_scratch(torch, keys, vals, bits):
    from paper_2412_04459_amd import _abi
    n = keys.size
    kt = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    vt = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    k2 = torch.empty_like(kt)
    v2 = torch.empty_like(vt)
    nb = _abi.svr_radix_sort_scratch_bytes(n, bits)
    sc = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    p = (sc.data_ptr() + 255) // 256 * 256
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = _abi.svr_radix_sort_pairs(ctypes.c_void_p(kt.data_ptr()), ctypes.c_void_p(vt.data_ptr()),
                                   ctypes.c_void_p(k2.data_ptr()), ctypes.c_void_p(v2.data_ptr()),
                                   n, bits, ctypes.c_void_p(p), nb, s)
    assert rc == _abi.SVR_OK, _abi.svr_last_error()
    torch.cuda.synchronize()
    return kt.cpu().numpy().view(np.uint64), vt.cpu().numpy().view(np.uint32)


def _sort_static(torch, keys, vals, bits):
    from paper_2412_04459_amd import _abi
    n = keys.size
    kt = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    vt = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = _abi.svr_radix_sort_pairs_static(ctypes.c_void_p(kt.data_ptr()),
                                          ctypes.c_void_p(vt.data_ptr()), n, bits, s)
    assert rc == _abi.SVR_OK, _abi.svr_last_error()
    torch.cuda.synchronize()
    return kt.cpu().numpy().view(np.uint64), vt.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n1,n2,bits", [(1 << 21, 300_001, 52), (1_000_003, 4097, 64),
                                        (70_000, 1, 17)])
def test_static_sort_matches_caller_scratch_sort(torch_dev, n1, n2, bits):
    torch = torch_dev
    print("static sort n=%d then n=%d, %d bits" % (n1, n2, bits), flush=True)
    for n, seed in ((n1, n1 + bits), (n2, n2 + bits)):
        keys, vals = _pairs(n, seed)
        ka, va = _sort_with_caller_scratch(torch, keys, vals, bits)
        kb, vb = _sort_static(torch, keys, vals, bits)
        assert np.array_equal(ka, kb) and np.array_equal(va, vb)
        mask = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
        order = np.argsort(keys & mask, kind="stable")
        assert np.array_equal(vb, vals[order])


def test_static_sort_rejects_sizes_beyond_its_array(torch_dev):
    from paper_2412_04459_amd import _abi
    rc = _abi.svr_radix_sort_pairs_static(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000),
                                          _abi.SVR_STATIC_SORT_MAX + 1, 32, None)
    assert rc == _abi.SVR_E_INVALID
    assert "scratch" in _abi.svr_last_error()
