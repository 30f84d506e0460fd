"""GPU parity of the cut-set Adam step (lodgs_adam_cut, called through the C
ABI by AdamCut) against the oracle's FP64 Adam.  Bars, from FP32 rounding of
a few operations per element: moments within 4 * 2^-23 of the magnitudes that
form them; parameters within 2^-22 |p| + 1e-5 |update|; rows outside the cut
bit-identical."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")
WIDTH = {"means": 3, "log_scales": 3, "quats": 4, "opacity_logits": 1, "sh": 48}
U = 2.0 ** -23


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _state(torch, rng, n):
    shape = lambda k: (n,) if k == "opacity_logits" else ((n, 16, 3) if k == "sh" else (n, WIDTH[k]))
    P = {k: torch.from_numpy(rng.normal(size=shape(k)).astype(np.float32)).cuda() for k in GROUPS}
    return P


def _check_step(torch, opt, before, grads, idx, n_sel):
    # the oracle takes the hyper-parameters as the library receives them (FP32)
    f32 = lambda x: float(np.float32(x))
    b1, b2, eps = f32(opt.betas[0]), f32(opt.betas[1]), f32(opt.eps)
    rows = idx[:n_sel].cpu().numpy()
    for k in GROUPS:
        w = WIDTH[k]
        p0, m0, v0 = (before[x][k].reshape(-1, w).astype(np.float64) for x in ("p", "m", "v"))
        g = grads[k].reshape(-1, w)[:n_sel].cpu().numpy().astype(np.float64)
        p_o, m_o, v_o = oracle.adam_cut(p0, m0, v0, g, rows, f32(opt.lr[k]), b1, b2, eps, opt.step_count)
        p = opt.params[k].reshape(-1, w).cpu().numpy().astype(np.float64)
        m = opt.exp_avg[k].reshape(-1, w).cpu().numpy().astype(np.float64)
        v = opt.exp_avg_sq[k].reshape(-1, w).cpu().numpy().astype(np.float64)
        rest = np.setdiff1d(np.arange(p.shape[0]), rows)
        for a, a0 in ((p, p0), (m, m0), (v, v0)):
            assert np.array_equal(a[rest], a0[rest]), k
        bm = 4 * U * (b1 * np.abs(m0[rows]) + (1 - b1) * np.abs(g))
        bv = 4 * U * (b2 * v0[rows] + (1 - b2) * g * g)
        assert np.all(np.abs(m[rows] - m_o[rows]) <= bm + 1e-38), k
        assert np.all(np.abs(v[rows] - v_o[rows]) <= bv + 1e-38), k
        upd = np.abs(p_o[rows] - p0[rows])
        err = np.abs(p[rows] - p_o[rows])
        assert np.all(err <= 2 * U * np.abs(p_o[rows]) + 1e-5 * upd + 1e-30), (k, float(err.max()))


def test_adam_cut_matches_the_oracle_over_steps(torch_cuda):
    torch = torch_cuda
    from paper_2507_01110_amd.lodgs import AdamCut
    rng = np.random.default_rng(81)
    n = 5000
    params = _state(torch, rng, n)
    opt = AdamCut(params, 3, lr={"means": 1e-3}, eps=1e-15)
    idx = torch.zeros(2048, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    for t, n_sel in enumerate((1500, 1999, 0, 2048)):
        sel = np.sort(rng.choice(n, n_sel, replace=False)).astype(np.int32)
        idx[:n_sel] = torch.from_numpy(sel).cuda()
        count.fill_(n_sel)
        grads = {k: torch.from_numpy((rng.normal(size=(2048,) + tuple(v.shape[1:])) *
                                      10.0 ** rng.uniform(-6, 1, (2048,) + (1,) * (v.dim() - 1)))
                                     .astype(np.float32)).cuda() for k, v in params.items()}
        before = {x: {k: d[k].cpu().numpy() for k in GROUPS}
                  for x, d in (("p", opt.params), ("m", opt.exp_avg), ("v", opt.exp_avg_sq))}
        opt.step(grads, idx, count)
        torch.cuda.synchronize()
        print("adam step", t + 1, "selected", n_sel, flush=True)
        _check_step(torch, opt, before, grads, idx, n_sel)


def test_adam_cut_clamps_the_count_and_skips_rows_outside_the_arrays(torch_cuda):
    torch = torch_cuda
    from paper_2507_01110_amd import _lib
    from paper_2507_01110_amd.lodgs import AdamCut
    rng = np.random.default_rng(82)
    n = 1000
    params = _state(torch, rng, n)
    opt = AdamCut(params, 3)
    idx = torch.tensor([5, 999, 1000, -3, 7, 8], dtype=torch.int32, device="cuda")
    count = torch.tensor([100], dtype=torch.int32, device="cuda")  # more than idx holds: clamped to 6
    grads = {k: torch.ones((6,) + tuple(v.shape[1:]), dtype=torch.float32, device="cuda") for k, v in params.items()}
    before = {k: v.clone() for k, v in params.items()}
    opt.step(grads, idx, count)
    torch.cuda.synchronize()
    for k, v in params.items():
        changed = (v != before[k]).reshape(n, -1).any(dim=1).nonzero().flatten().cpu().tolist()
        assert changed == [5, 7, 8, 999], (k, changed)
    with pytest.raises(_lib.LodgsError):
        opt.step({k: v for k, v in grads.items() if k != "sh"}, idx, count)


def test_training_iterations_lower_the_loss(torch_cuda):
    # the training loop of the per-view path: kNN view walk, LoD noise on tau,
    # cut, render, L1, backward into selection-indexed gradients, cut-set Adam
    torch = torch_cuda
    import scenegen
    from scenegen import configs
    from paper_2507_01110_amd.lodgs import AdamCut, Frame, Scene
    from paper_2507_01110_amd.training import ViewScheduler, lod_noise
    tree = scenegen.build_tree(configs.tiny_spec(n=4096))
    S = Scene(tree)
    cams = [scenegen.camera_look_at((30 * np.cos(a), 30 * np.sin(a), 8.0), (0, 0, 0), (0, 0, 1), 128, 96)
            for a in np.linspace(0, 2 * np.pi, 12, endpoint=False)]
    sched = ViewScheduler([c.pos for c in cams], k=3, explore_every=8, seed=4)
    f = Frame(S, S.n_nodes, 1 << 20, 128, 96)
    sel = {k: torch.zeros((S.n_nodes,) + tuple(v.shape[1:]), dtype=torch.float32, device="cuda")
           for k, v in S.params.items()}
    opt = AdamCut(S.params, tree.sh_degree, lr={"sh": 2e-2, "opacity_logits": 5e-2})
    target = torch.full((96, 128, 3), 0.5, dtype=torch.float32, device="cuda")
    bg = (0.5, 0.5, 0.5)  # uncovered pixels match the target: every pixel's loss is trainable
    rng = np.random.default_rng(6)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def mean_loss():
        out = []
        f.set_lod_noise(1.0)  # evaluation without the training noise
        for cam in cams:
            f.lod_select(cam, 1.0)
            f.l1_loss(f.render(cam, bg=bg), target, loss=loss)
            out.append(float(loss.item()))
        return float(np.mean(out))

    before = mean_loss()
    for it in range(100):
        cam = cams[sched.next()]
        f.set_lod_noise(lod_noise(rng))
        f.lod_select(cam, 1.0)
        img = f.render(cam, bg=bg)
        dL = f.l1_loss(img, target)
        f.backward(dL, sel=sel)
        opt.step(sel, f.idx, f.count)
    assert f.stats()["status"] == 0
    after = mean_loss()
    print("mean L1 over the views before / after 100 iterations", before, after, flush=True)
    assert after < 0.85 * before
