"""The atomic throughput probe (svr_atomic_probe): every one of its 11-lane
atomic adds lands, on voxel rows inside the given arrays."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_atomic_probe_adds_every_update():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04459_amd import _abi
    n_rows, n_waves, iters = 1000, 4096, 7
    # guard rows on both sides must stay untouched
    corner = torch.zeros((n_rows + 2, 8), dtype=torch.float32, device="cuda")
    colour = torch.zeros((n_rows + 2, 3), dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = _abi.svr_atomic_probe(ctypes.c_void_p(corner[1:].data_ptr()),
                               ctypes.c_void_p(colour[1:].data_ptr()), n_rows, n_waves, iters, s)
    assert rc == _abi.SVR_OK, _abi.svr_last_error()
    torch.cuda.synchronize()
    c = corner.cpu().numpy()
    k = colour.cpu().numpy()
    assert not c[0].any() and not c[-1].any() and not k[0].any() and not k[-1].any()
    assert c.sum() == 8.0 * n_waves * iters and k.sum() == 3.0 * n_waves * iters
    # each instruction adds 1 to all 8 corner slots and all 3 colour slots of one row
    rows = c[1:-1]
    assert np.all(rows == rows[:, :1]) and np.all(k[1:-1] == rows[:, :3])
    assert (rows[:, 0] > 0).sum() > 0.9 * n_rows
