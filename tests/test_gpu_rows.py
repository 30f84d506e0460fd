"""Out-of-core parameters (lodgs_gather_rows, lodgs_render_rows through the C
ABI): the selected rows gathered from pinned host memory equal the scene's
rows bit for bit, and rendering and differentiating from them gives the
image, the instance order and the selection-indexed gradients of the
resident path bit for bit."""
import numpy as np
import pytest

import scenegen
from scenegen import configs

pytestmark = pytest.mark.gpu

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _compare(torch, tree, cam, tau, max_inst):
    from paper_2507_01110_amd.lodgs import Frame, HostParams, Scene, grads_like, rows_like
    S = Scene(tree)
    host = HostParams.from_scene(S)
    fa = Frame(S, S.n_nodes, max_inst, cam.width, cam.height)
    fb = Frame(S, S.n_nodes, max_inst, cam.width, cam.height)
    idx, cnt = fa.lod_select(cam, tau)
    n = int(cnt.item())
    img_a = fa.render(cam).clone()
    fb.lod_select(cam, tau)
    rows = rows_like(tree.sh_degree, S.n_nodes)
    fb.gather_rows(host, rows)
    sel_idx = idx[:n].long()
    for k in GROUPS:
        assert torch.equal(rows[k][:n], S.params[k][sel_idx]), k
    img_b = fb.render_rows(cam, rows)
    assert torch.equal(img_a, img_b)
    ta, pa = fa.instances()
    tb, pb = fb.instances()
    assert torch.equal(ta, tb) and torch.equal(pa, pb)
    dL = torch.from_numpy(scenegen.target_image(cam.height, cam.width, 5) - 0.5).cuda().float()
    ga, gb = grads_like(S, n), grads_like(S, n)
    fa.backward(dL, sel=ga)
    fb.backward(dL, sel=gb)
    for k in GROUPS:
        assert torch.equal(ga[k], gb[k]), k
    print("rows path equal:", n, "selected", flush=True)
    return S, fb, host, rows


def test_rows_path_equals_the_resident_path_tiny(torch_cuda):
    tree = scenegen.build_tree(configs.tiny_spec())
    _compare(torch_cuda, tree, configs.tiny_camera(), 1.0, 1 << 20)


def test_rows_path_equals_the_resident_path_medium_view(torch_cuda):
    tree = scenegen.build_tree(configs.medium_spec())
    _compare(torch_cuda, tree, configs.medium_camera(), 1.0, 1 << 24)


def test_rows_path_rejects_pageable_memory_and_node_gradients(torch_cuda):
    torch = torch_cuda
    from paper_2507_01110_amd import _lib
    from paper_2507_01110_amd.lodgs import HostParams, grads_like
    tree = scenegen.build_tree(configs.tiny_spec(n=2048))
    S, f, host, rows = _compare(torch, tree, configs.tiny_camera(128, 128), 1.0, 1 << 18)
    pageable = HostParams.__new__(HostParams)
    pageable.params = {k: v.clone() for k, v in host.params.items()}  # plain host memory
    assert not pageable.params["sh"].is_pinned()
    pageable.sh_degree, pageable.n_nodes = host.sh_degree, host.n_nodes
    with pytest.raises(_lib.LodgsError):
        f.gather_rows(pageable, rows)
    dL = torch.zeros((128, 128, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.LodgsError):
        f.backward(dL, nodes=grads_like(S))


def _against_oracle(torch, tree, cam, tau, max_inst):
    """The out-of-core form against the oracle: gathered rows rendered and
    differentiated (L1 against a seeded target) give the oracle's image within
    1e-4 max-abs and its gradients within 1e-3 relative L2 per group."""
    import oracle
    from paper_2507_01110_amd.lodgs import Frame, HostParams, Scene, grads_like, rows_like
    S = Scene(tree)
    host = HostParams.from_scene(S)
    f = Frame(S, S.n_nodes, max_inst, cam.width, cam.height)
    idx, cnt = f.lod_select(cam, tau)
    n = int(cnt.item())
    rows = rows_like(tree.sh_degree, n)
    f.gather_rows(host, rows)
    img = f.render_rows(cam, rows)
    assert f.stats()["status"] == 0
    O = oracle.OracleScene(tree)
    ids, _ = O.select(cam, tau)
    assert np.array_equal(idx[:n].cpu().numpy(), O.pos_of[ids])
    F = oracle.OracleFrame(tree, ids, cam)
    err = float(np.abs(img.cpu().numpy().astype(np.float64) - F.image).max())
    assert err <= 1e-4, err
    _, dL = oracle.l1_loss_grad(F.image, scenegen.target_image(cam.height, cam.width, 9))
    g = grads_like(S, n)
    f.backward(torch.from_numpy(dL.astype(np.float32)).cuda(), sel=g)
    _, g_o = F.backward(dL)
    got = np.concatenate([g[k].reshape(n, -1).cpu().numpy().astype(np.float64) for k in GROUPS], axis=1)
    off = 0
    for k in GROUPS:
        w = g[k].reshape(n, -1).shape[1]
        a, b = got[:, off:off + w], g_o[:, off:off + w]
        rel = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
        assert rel <= 1e-3, (k, rel)
        off += w
    print(f"rows path vs oracle: {n} selected, max|dimg| {err:.2e}", flush=True)


def test_rows_path_matches_the_oracle_tiny(torch_cuda):
    _against_oracle(torch_cuda, scenegen.build_tree(configs.tiny_spec()), configs.tiny_camera(), 1.0, 1 << 20)


def test_rows_path_matches_the_oracle_medium_view(torch_cuda):
    tree = scenegen.build_tree(configs.medium_spec(n=500_000, seed=12))
    _against_oracle(torch_cuda, tree, configs.medium_camera(seed=107), 1.0, 1 << 24)
