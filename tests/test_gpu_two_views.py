"""Several views in flight (the timed loop of the benchmark): four frames
take turns over three streams, view i's stream running its select, forward,
L1 and the frame-local half of its backward (lodgs_render_backward_phases,
PARTIALS), one more stream the scatter half into the node gradients (SCATTER)
in view order.  Also the two-frame form with the whole backward on one stream.
Images, dL/dimage and the accumulated node gradients equal those of one view
at a time bit for bit: frames share no mutable state, and the writes to the
node arrays stay in view order."""
import numpy as np
import pytest

import scenegen
from scenegen import configs

pytestmark = pytest.mark.gpu

W, H = 1280, 720


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_01110_amd.lodgs import Frame, Scene, grads_like
    S = Scene(scenegen.build_tree(configs.medium_spec(n=500_000, seed=21)))
    rng = np.random.default_rng(8)
    cams = [configs.random_pose_camera(rng, 200.0, W, H) for _ in range(8)]
    taus = [0.5, 1.0, 2.0, 1.0, 0.5, 2.0, 1.0, 0.5]
    targets = [torch.from_numpy(scenegen.target_image(H, W, 40 + k)).cuda() for k in range(len(cams))]
    f0 = Frame(S, 1 << 22, 1 << 24, W, H)
    g = grads_like(S)
    imgs, dls = [], []
    for k, cam in enumerate(cams):
        print(f"serial view {k}", flush=True)
        f0.lod_select(cam, taus[k])
        img = f0.render(cam)
        dL = f0.l1_loss(img, targets[k])
        f0.backward(dL, nodes=g)
        imgs.append(img.clone())
        dls.append(dL.clone())
    torch.cuda.synchronize()
    assert f0.stats()["status"] == 0
    return S, cams, taus, targets, g, imgs, dls


def _check(setup, g_pipe, got_imgs, got_dls, frames):
    import torch
    S, cams, taus, targets, g, imgs, dls = setup
    torch.cuda.synchronize()
    for f in frames:
        assert f.stats()["status"] == 0
    for k in range(len(cams)):
        assert torch.equal(got_imgs[k], imgs[k]), k
        assert torch.equal(got_dls[k], dls[k]), k
    for key in g:
        assert torch.equal(g_pipe[key], g[key]), key
    assert float(g_pipe["means"].abs().sum()) > 0.0


def test_views_in_flight_with_split_backward_equal_one_at_a_time(setup):
    import torch
    from paper_2507_01110_amd.lodgs import Frame, grads_like
    S, cams, taus, targets = setup[:4]
    n_fl, n_st = 4, 3  # four frames taking turns over three streams, as the benchmark's timed loop
    frames = [Frame(S, 1 << 22, 1 << 24, W, H) for _ in range(n_fl)]
    imgs = [torch.empty((H, W, 3), dtype=torch.float32, device="cuda") for _ in range(n_fl)]
    dls = [torch.empty_like(imgs[0]) for _ in range(n_fl)]
    g_pipe = grads_like(S)
    sF, sB = [torch.cuda.Stream() for _ in range(n_st)], torch.cuda.Stream()
    part_done = [torch.cuda.Event() for _ in range(n_fl)]
    scat_done = [torch.cuda.Event() for _ in range(n_fl)]
    got_imgs, got_dls = [None] * len(cams), [None] * len(cams)

    def frame_work(i):
        k = i % n_fl
        f, s = frames[k], sF[i % n_st]
        s.wait_event(scat_done[k])
        f.lod_select(cams[i], taus[i], stream=s)
        f.render(cams[i], out=imgs[k], stream=s)
        f.l1_loss(imgs[k], targets[i], grad=dls[k], stream=s)
        f.backward(dls[k], stream=s, phases="partials")
        with torch.cuda.stream(s):
            got_imgs[i] = imgs[k].clone()
            got_dls[i] = dls[k].clone()
        part_done[k].record(s)

    def scatter(i):
        k = i % n_fl
        sB.wait_event(part_done[k])
        frames[k].backward(None, nodes=g_pipe, stream=sB, phases="scatter")
        scat_done[k].record(sB)

    for t in range(len(cams) + n_fl - 1):
        print(f"in flight: step {t}", flush=True)
        if t < len(cams):
            frame_work(t)
        if t - (n_fl - 1) >= 0:
            scatter(t - (n_fl - 1))
    _check(setup, g_pipe, got_imgs, got_dls, frames)


def test_two_views_in_flight_whole_backward_equal_one_at_a_time(setup):
    import torch
    from paper_2507_01110_amd.lodgs import Frame, grads_like
    S, cams, taus, targets = setup[:4]
    frames = [Frame(S, 1 << 22, 1 << 24, W, H), Frame(S, 1 << 22, 1 << 24, W, H)]
    imgs = [torch.empty((H, W, 3), dtype=torch.float32, device="cuda") for _ in range(2)]
    dls = [torch.empty_like(imgs[0]) for _ in range(2)]
    g_pipe = grads_like(S)
    sF, sB = torch.cuda.Stream(), torch.cuda.Stream()
    fwd_done = [torch.cuda.Event(), torch.cuda.Event()]
    bwd_done = [torch.cuda.Event(), torch.cuda.Event()]
    got_imgs, got_dls = [], []

    def forward(i):
        f = frames[i % 2]
        sF.wait_event(bwd_done[i % 2])
        f.lod_select(cams[i], taus[i], stream=sF)
        f.render(cams[i], out=imgs[i % 2], stream=sF)
        fwd_done[i % 2].record(sF)

    def backward(i):
        f = frames[i % 2]
        sB.wait_event(fwd_done[i % 2])
        f.l1_loss(imgs[i % 2], targets[i], grad=dls[i % 2], stream=sB)
        f.backward(dls[i % 2], nodes=g_pipe, stream=sB)
        with torch.cuda.stream(sB):
            got_imgs.append(imgs[i % 2].clone())
            got_dls.append(dls[i % 2].clone())
        bwd_done[i % 2].record(sB)

    forward(0)
    for i in range(len(cams)):
        print(f"in flight: view {i}", flush=True)
        if i + 1 < len(cams):
            forward(i + 1)
        backward(i)
    _check(setup, g_pipe, got_imgs, got_dls, frames)


def test_scatter_half_needs_its_partials(setup):
    import torch
    from paper_2507_01110_amd import _lib
    from paper_2507_01110_amd.lodgs import Frame, grads_like
    S, cams, taus, targets = setup[:4]
    f = Frame(S, 1 << 22, 1 << 24, W, H)
    f.lod_select(cams[0], taus[0])
    img = f.render(cams[0])
    with pytest.raises(_lib.LodgsError):
        f.backward(None, nodes=grads_like(S), phases="scatter")  # no partials since the render
    dL = f.l1_loss(img, targets[0])
    f.backward(dL, phases="partials")
    g = grads_like(S)
    f.backward(None, nodes=g, phases="scatter")
    torch.cuda.synchronize()
    assert float(g["means"].abs().sum()) > 0.0
