"""The training step captured in one HIP graph (lodgs_graph_capture_step):
every replay, with another camera, tau and target each time and the
program's own eager work and synchronisations between replays, gives the
image, dL/dimage and the accumulated node gradients of the same step run
with plain launches bit for bit, and its loss up to the rounding of an
atomic sum."""
import numpy as np
import pytest

import scenegen
from scenegen import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def medium_scene():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_01110_amd.lodgs import Scene
    return Scene(scenegen.build_tree(configs.medium_spec(n=500_000, seed=13)))


def test_step_graph_replays_equal_plain_steps(medium_scene):
    import torch
    from paper_2507_01110_amd.lodgs import Frame, StepGraph, grads_like
    S = medium_scene
    W, H = 1280, 720
    rng = np.random.default_rng(4)
    cams = [configs.random_pose_camera(rng, 200.0, W, H) for _ in range(6)]
    taus = [0.5, 1.0, 2.0, 1.0, 0.5, 2.0]
    targets = [torch.from_numpy(scenegen.target_image(H, W, 30 + k)).cuda() for k in range(6)]
    fp = Frame(S, 1 << 22, 1 << 24, W, H)
    fg = Frame(S, 1 << 22, 1 << 24, W, H)
    gp, gg = grads_like(S), grads_like(S)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        g = StepGraph(fg, cams[0], taus[0], targets[0], st, nodes=gg)
    st.synchronize()
    dL = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for k in range(6):
        print(f"step replay {k}: tau {taus[k]}", flush=True)
        with torch.cuda.stream(st):
            g.launch(cams[k], taus[k], targets[k], st)
            fp.lod_select(cams[k], taus[k], stream=st)
            img = fp.render(cams[k], stream=st)
            fp.l1_loss(img, targets[k], grad=dL, loss=loss, stream=st)
            fp.backward(dL, nodes=gp, stream=st)
        st.synchronize()
        torch.cuda.synchronize()
        assert fg.stats(stream=st)["status"] == 0 and fp.stats(stream=st)["status"] == 0
        n = int(fp.count.item())
        assert int(fg.count.item()) == n and torch.equal(fg.idx[:n], fp.idx[:n])
        assert torch.equal(g.out, img)
        assert torch.equal(g.dL, dL)
        # the loss is an FP32 sum of one atomic add per wave (16k of them, in
        # no fixed order): equal up to that sum's rounding
        assert abs(float(g.loss) - float(loss)) <= 1e-4 * abs(float(loss))
        for key in gp:
            assert torch.equal(gg[key], gp[key]), (k, key)
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
    assert float(gp["means"].abs().sum()) > 0.0
