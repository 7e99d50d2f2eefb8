"""Entry-capacity overflow (the C ABI's error convention): a frame whose
duplicated list does not fit the workspace's capacity never writes past it;
with the count read back svr_preprocess returns SVR_E_CAPACITY and the
required count (the Python layer reallocates and retries once); without a
host synchronisation (and inside a captured hipGraph) the frame completes
and svr_check_overflow reports SVR_E_CAPACITY with the required count, after
which a frame sized to that count matches the reference."""
import ctypes

import numpy as np
import pytest

from paper_2412_04459_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(torch):
    from paper_2412_04459_amd.render import DeviceScene, Rasterizer
    scene = S.sphere_shell_scene(opaque=True)
    cams = [S.sphere_shell_camera(), S.look_at(77, 51, 60.0, [1.5, -1.2, 1.0], target=(0.3, 0.3, 0.3))]
    ds = DeviceScene(scene)
    ref = Rasterizer(ds, cams, K=2, tile=8)
    rgba = ref.forward()
    g = torch.from_numpy(S.upstream_grads(rgba.shape[0], 31)).cuda()
    gg, gs = ref.backward(g)
    torch.cuda.synchronize()
    assert ref.n_entries > 2000
    return ds, cams, ref, rgba, g, gg, gs


def _close(a, b):
    a = a.detach().cpu().double().numpy().reshape(-1)
    b = b.detach().cpu().double().numpy().reshape(-1)
    return bool(np.all(np.abs(a - b) <= 1e-4 * np.abs(b) + 1e-6 * np.abs(b).max()))


def test_sync_mode_reports_capacity_and_python_retries(torch_dev):
    torch = torch_dev
    from paper_2412_04459_amd import _abi
    from paper_2412_04459_amd.render import Rasterizer, _stream
    ds, cams, ref, rgba, g, gg, gs = _setup(torch)
    E = ref.n_entries
    small = Rasterizer(ds, cams, K=2, tile=8, capacity=1000, sync_count=True)
    # the C ABI itself: SVR_E_CAPACITY with the required count, nothing emitted
    n = ctypes.c_int64(-1)
    rc = _abi.svr_preprocess(ds.struct(), small.cam_arr, small.n_cams, small.opts,
                             small._ws_ptr(), small.ws_bytes, ctypes.byref(n), _stream())
    assert rc == _abi.SVR_E_CAPACITY
    assert n.value == E
    assert "capacity" in _abi.svr_last_error()
    # the Python layer reallocates and retries once
    out = small.forward()
    a, b = small.backward(g)
    torch.cuda.synchronize()
    assert small.capacity >= E and small.n_entries == E
    assert torch.equal(out, rgba)
    assert _close(a, gg) and _close(b, gs)


@pytest.mark.parametrize("graph", [False, True])
def test_no_sync_overflow_is_reported_after_the_frame(torch_dev, graph):
    torch = torch_dev
    from paper_2412_04459_amd import _abi
    from paper_2412_04459_amd.render import Rasterizer, _stream
    ds, cams, ref, rgba, g, gg, gs = _setup(torch)
    E = ref.n_entries
    cap = E // 3
    r = Rasterizer(ds, cams, K=2, tile=8, capacity=cap, sync_count=False)
    out = torch.empty_like(rgba)
    a = torch.empty_like(gg)
    b = torch.empty_like(gs)
    if graph:
        stream = torch.cuda.Stream()
        r.capture(out, g, a, b, stream)
        r.replay(stream)
        r.replay(stream)
    else:
        r.forward(out=out)
        r.backward(g, grad_grid=a, grad_sh=b)
    torch.cuda.synchronize()
    n = ctypes.c_int64(-1)
    rc = _abi.svr_check_overflow(ds.struct(), r.cam_arr, r.n_cams, r.opts, r._ws_ptr(),
                                 r.ws_bytes, ctypes.byref(n), _stream())
    assert rc == _abi.SVR_E_CAPACITY
    assert n.value == E
    assert r.check_overflow() == E
    r.release_graph()
    # sized to the reported count, the same frame matches the reference
    r2 = Rasterizer(ds, cams, K=2, tile=8, capacity=int(n.value), sync_count=False)
    out2 = torch.empty_like(rgba)
    a2 = torch.empty_like(gg)
    b2 = torch.empty_like(gs)
    if graph:
        r2.capture(out2, g, a2, b2, stream)
        r2.replay(stream)
    else:
        r2.forward(out=out2)
        r2.backward(g, grad_grid=a2, grad_sh=b2)
    torch.cuda.synchronize()
    assert r2.check_overflow() == E
    assert torch.equal(out2, rgba)
    assert _close(a2, gg) and _close(b2, gs)
    r2.release_graph()
