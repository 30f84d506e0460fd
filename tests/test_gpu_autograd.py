"""The torch.autograd.Function over the HIP path: gradients against the oracle's
FP64 backward and against FP64 central differences with frozen decisions."""
import sys

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import configs

pytestmark = pytest.mark.gpu

GROUPS = {"means": slice(0, 3), "log_scales": slice(3, 6), "quats": slice(6, 10), "opacity_logits": slice(10, 11),
          "sh": slice(11, None)}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(tree, cam):
    from paper_2507_01110_amd.lodgs import Frame, Scene
    S = Scene(tree)
    for t in S.params.values():
        t.requires_grad_(True)
    f = Frame(S, S.n_nodes, max(1 << 20, 16 * S.n_nodes), cam.width, cam.height)
    return S, f


def _flat(grads, rows):
    return np.concatenate([grads[k][rows].reshape(len(rows), -1).detach().cpu().numpy().astype(np.float64)
                           for k in ("means", "log_scales", "quats", "opacity_logits", "sh")], axis=1)


def test_autograd_matches_oracle_and_leaves_unselected_nodes_untouched(torch_cuda):
    import torch
    from paper_2507_01110_amd.autograd import render_lod
    tree = scenegen.build_tree(configs.tiny_spec(n=8192, seed=4))
    cam = configs.tiny_camera(200, 160)
    S, f = _setup(tree, cam)
    O = oracle.OracleScene(tree)
    ids, _ = O.select(cam, 2.0)
    F = oracle.OracleFrame(tree, ids, cam)
    W = np.random.default_rng(0).normal(size=F.image.shape)
    img = render_lod(f, cam, 2.0)
    assert np.abs(img.detach().cpu().numpy() - F.image).max() <= 1e-4
    (img * torch.from_numpy(W.astype(np.float32)).cuda()).sum().backward()
    _, g_o = F.backward(W)
    pos = O.pos_of[ids]
    got = _flat({k: S.params[k].grad for k in S.params}, pos)
    for name, sl in GROUPS.items():
        e = np.linalg.norm(got[:, sl] - g_o[:, sl]) / np.linalg.norm(g_o[:, sl])
        _say("autograd", name, e)
        assert e <= 1e-3, (name, e)
    untouched = np.ones(S.n_nodes, bool)
    untouched[pos] = False
    for k, t in S.params.items():
        assert torch.all(t.grad[torch.from_numpy(untouched).cuda()] == 0), k


def test_accumulate_mode_equals_dense_mode(torch_cuda):
    import torch
    from paper_2507_01110_amd.autograd import render_lod
    from paper_2507_01110_amd.lodgs import grads_like
    tree = scenegen.build_tree(configs.tiny_spec(n=4096, seed=5))
    cam = configs.tiny_camera(128, 128)
    S, f = _setup(tree, cam)
    W = torch.randn(128, 128, 3, device="cuda")
    (render_lod(f, cam, 1.5) * W).sum().backward()
    dense = {k: t.grad.clone() for k, t in S.params.items()}
    acc = grads_like(S)
    (render_lod(f, cam, 1.5, accumulate_into=acc) * W).sum().backward()
    for k in dense:
        scale = float(dense[k].abs().max())
        assert torch.allclose(acc[k], dense[k], rtol=1e-4, atol=1e-5 * scale), k


def test_batch_on_streams_with_a_scatter_stream_equals_one_stream(torch_cuda):
    # a batch of views on two streams, the node-array half of each backward on
    # one scatter stream (in the autograd engine's order), two steps in a row
    # with the frames reused: node gradients bit-identical to the same graph
    # run on one stream
    import torch
    from paper_2507_01110_amd.autograd import render_lod
    from paper_2507_01110_amd.lodgs import Frame, grads_like
    tree = scenegen.build_tree(configs.medium_spec(n=200_000, seed=8))
    rng = np.random.default_rng(12)
    cams = [configs.random_pose_camera(rng, 200.0, 320, 240) for _ in range(8)]
    S, _ = _setup(tree, cams[0])
    frames = [Frame(S, S.n_nodes, 1 << 22, 320, 240) for _ in range(4)]
    targets = [torch.rand(240, 320, 3, device="cuda") for _ in range(4)]

    def run(streams, scat):
        acc = grads_like(S)
        main = torch.cuda.current_stream()
        for step in range(2):
            losses = []
            for b in range(4):
                st = streams[b % len(streams)]
                st.wait_stream(main)
                with torch.cuda.stream(st):
                    img = render_lod(frames[b], cams[4 * step + b], 1.0, accumulate_into=acc, scatter_stream=scat)
                    losses.append((img - targets[b]).abs().mean())
            for st in streams:
                main.wait_stream(st)
            torch.stack(losses).sum().backward()
            if scat is not None:
                main.wait_stream(scat)
        torch.cuda.synchronize()
        for f in frames:
            assert f.stats()["status"] == 0
        return acc

    one = run([torch.cuda.current_stream()], None)
    many = run([torch.cuda.Stream(), torch.cuda.Stream()], torch.cuda.Stream())
    for k in one:
        assert float(one[k].abs().sum()) > 0.0, k
        assert torch.equal(one[k], many[k]), k


def test_autograd_vs_fp64_central_differences_medium_subset(torch_cuda):
    """Medium workload (2M leaves, 1080p): directional derivatives of 1,000 drawn
    nodes against FP64 central differences of the oracle with frozen decisions."""
    import torch
    from paper_2507_01110_amd.autograd import render_lod
    tree = scenegen.build_tree(configs.medium_spec())
    cam = configs.medium_camera()
    S, f = _setup(tree, cam)
    O = oracle.OracleScene(tree)
    ids, _ = O.select(cam, 1.0)
    F = oracle.OracleFrame(tree, ids, cam)
    target = scenegen.target_image(cam.height, cam.width, 201)
    _, dL = oracle.l1_loss_grad(F.image, target)
    img = render_lod(f, cam, 1.0)
    img.backward(torch.from_numpy(dL.astype(np.float32)).cuda())
    rng = np.random.default_rng(3)
    drawn = np.nonzero(F.splats()["tiles"] > 0)[0]
    pick = rng.choice(drawn, size=min(1000, len(drawn)), replace=False)
    pos = O.pos_of[ids[pick]]
    got = _flat({k: S.params[k].grad for k in S.params}, pos)
    P = F.params64()
    a, b = [], []
    for r, i in enumerate(pick):
        v = rng.normal(size=P.shape[1])
        h = 1e-6 * max(1.0, float(np.abs(P[i]).max()))
        b.append(F.fd_directional(dL, int(i), v, h))
        a.append(float(got[r] @ v))
    a, b = np.array(a), np.array(b)
    e = np.linalg.norm(a - b) / np.linalg.norm(b)
    _say("FD subset", len(pick), "rel L2", e, "nonzero", int(np.sum(b != 0)))
    assert np.sum(b != 0) > 100
    assert e <= 1e-3, e
