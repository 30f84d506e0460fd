"""lodgs_lod_select_noalloc (the HSPT cut with its workspace in the library's
static device array) against lodgs_lod_select (the frame's workspace), through
the C ABI: bit-exact index lists and counts on two calls in a row, the second
on a smaller scene, so stale workspace contents of the first would show."""
import numpy as np
import pytest

import scenegen
from scenegen import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _with_frame(scene, cam, tau, cull, conservative):
    from paper_2507_01110_amd.lodgs import Frame
    f = Frame(scene, scene.n_nodes, 1 << 16, cam.width, cam.height)
    idx, cnt = f.lod_select(cam, tau, cull=cull, conservative=conservative)
    n = int(cnt.item())
    st = f.stats()
    assert st["status"] == 0 and st["n_selected"] == n
    return idx[:n].cpu().numpy()


def _without_frame(torch, scene, cam, tau, cull, conservative, capacity=None):
    cap = scene.n_nodes if capacity is None else capacity
    idx = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    scene.lod_select_noalloc(cam, tau, idx, cnt, cull=cull, conservative=conservative)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), int(cnt.item())


def test_noalloc_select_matches_frame_select_two_calls(torch_cuda):
    from paper_2507_01110_amd.lodgs import Scene
    torch = torch_cuda
    big = scenegen.build_tree(configs.medium_spec(n=200_000, seed=3))
    small = scenegen.build_tree(configs.tiny_spec(n=4096, seed=5))
    cam_big = configs.medium_camera(seed=111)
    cam_small = configs.tiny_camera(256, 256)
    cases = [(Scene(big), cam_big, 1.0, True, False), (Scene(small), cam_small, 0.5, True, False)]
    for k, (S, cam, tau, cull, cons) in enumerate(cases):
        print(f"noalloc call {k}: {S.n_nodes} nodes, tau {tau}", flush=True)
        want = _with_frame(S, cam, tau, cull, cons)
        got, n = _without_frame(torch, S, cam, tau, cull, cons)
        assert n == len(want), (k, n, len(want))
        assert np.array_equal(got[:n], want), k
        assert np.all(got[n:] == -7), "wrote past the count"
    # the variants: no culling, the conservative cut, a cut-short list
    S, cam = cases[0][0], cam_big
    for cull, cons in ((False, False), (True, True)):
        want = _with_frame(S, cam, 2.0, cull, cons)
        got, n = _without_frame(torch, S, cam, 2.0, cull, cons)
        assert n == len(want) and np.array_equal(got[:n], want), (cull, cons)
    want = _with_frame(S, cam, 1.0, True, False)
    got, n = _without_frame(torch, S, cam, 1.0, True, False, capacity=len(want) // 2)
    assert n == len(want), "the full count is reported when the list is cut short"
    assert np.array_equal(got, want[: len(want) // 2])


def test_noalloc_select_rejects_other_cuts(torch_cuda):
    import ctypes
    from paper_2507_01110_amd import _lib
    from paper_2507_01110_amd.lodgs import Scene, camera_struct
    torch = torch_cuda
    S = Scene(scenegen.build_tree(configs.tiny_spec(n=1024, seed=2)))
    cam = configs.tiny_camera(64, 64)
    idx = torch.zeros(S.n_nodes, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    c = camera_struct(cam)
    rc = _lib.load().lodgs_lod_select_noalloc(S._h, ctypes.byref(c), 1.0, _lib.CUT_BFS, idx.data_ptr(),
                                              idx.numel(), cnt.data_ptr(), None)
    assert rc == _lib.E_INVALID
    with pytest.raises(_lib.LodgsError):
        S.lod_select_noalloc(cam, -1.0, idx, cnt)
