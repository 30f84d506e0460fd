"""Graph-captured views and the continuous-batching server: every result must be
the same alone (plain launches) and in the mix (graph replays on slots)."""
import math
import sys

import numpy as np
import pytest

import scenegen
from scenegen import configs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def medium_scene():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_01110_amd.lodgs import Scene
    return Scene(scenegen.build_tree(configs.medium_spec(n=500_000, seed=11)))


def _cam(rng, w, h):
    return configs.random_pose_camera(rng, 200.0, w, h)


def test_graph_replays_equal_plain_renders(medium_scene):
    import torch
    from paper_2507_01110_amd.lodgs import Frame, ViewGraph
    S = medium_scene
    rng = np.random.default_rng(1)
    fg = Frame(S, 1 << 22, 1 << 24, 640, 360)
    fp = Frame(S, 1 << 22, 1 << 24, 640, 360)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        g = ViewGraph(fg, _cam(rng, 640, 360), 1.0, st)
    for k in range(6):
        cam, tau = _cam(rng, 640, 360), float([0.5, 1.0, 2.0][k % 3])
        _say("graph replay", k, tau)
        with torch.cuda.stream(st):
            out = g.launch(cam, tau, st)
            ref = fp.render(cam, idx=fp.lod_select(cam, tau, stream=st)[0], stream=st)
            a, b = out.clone(), ref.clone()
            ia, ib = fg.count.clone(), fp.count.clone()
        st.synchronize()
        torch.cuda.synchronize()
        assert int(ia) == int(ib)
        n = int(ia)
        assert torch.equal(fg.idx[:n], fp.idx[:n])
        assert torch.equal(a, b)
        assert fg.stats(stream=st)["status"] == 0
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays


def test_server_results_equal_alone_and_in_the_mix(medium_scene):
    import torch
    from paper_2507_01110_amd.lodgs import Frame
    from paper_2507_01110_amd.server import RenderServer, baseline_loop, poisson_requests, summarize
    S = medium_scene
    sizes = [(640, 360), (1280, 720)]
    rng = np.random.default_rng(2)
    make = lambda r: _cam(r, *sizes[r.integers(2)])
    reqs = poisson_requests(rng, 2000.0, 40, make)
    srv = RenderServer(S, sizes, 1 << 22, 1 << 24, max_slots=4, template_cam=lambda w, h: _cam(rng, w, h))
    _say("slots", len(srv.slots))
    assert len(srv.slots) >= 1
    out, span, imgs = srv.run(reqs, keep_images=True)
    assert all(r.status == 0 for r in out)
    base = [type(r)(r.rid, r.arrival, r.cam, r.tau) for r in reqs]
    f = Frame(S, 1 << 22, 1 << 24, 1280, 720)
    _, span_b, imgs_b = baseline_loop(f, base, keep_images=True)
    torch.cuda.synchronize()
    for r in reqs:
        assert torch.equal(imgs[r.rid], imgs_b[r.rid]), r.rid
    _say("server", summarize(out, span), "baseline", summarize(base, span_b))
