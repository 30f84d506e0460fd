"""GPU parity at the full city size: 50M leaves (100M nodes, 23.6 GB of
parameters), 1920x1080 views of the aerial-to-street path, in the frame
configuration the benchmark times (selection capacity 2^24, instance capacity
2^27, the default blend layouts, node-gradient accumulation).  The
CONSERVATIVE cut and the whole-hierarchy comparator cuts (BFS, Eq. 5) of the
same views are compared bit for bit too.  Whole views
are compared with the oracle: the selected index set and the instance order
bit-exact, pixels within 1e-4 max-abs, accumulated node gradients within 1e-3
relative L2 per parameter group, every node outside the selection untouched.
"""
import sys
import time

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import configs

pytestmark = pytest.mark.gpu

GROUPS = {"means": slice(0, 3), "log_scales": slice(3, 6), "quats": slice(6, 10), "opacity_logits": slice(10, 11),
          "sh": slice(11, None)}
# (path pose, tau): aerial, mid-path, street level at the finest tau
VIEWS = ((0, 2.0), (128, 1.0), (255, 0.5))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def city():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_01110_amd.lodgs import Scene
    t0 = time.time()
    tree = scenegen.build_tree(configs.city_spec())
    _say(f"city: {tree.n_nodes} nodes built in {time.time() - t0:.1f} s")
    S = Scene(tree)
    torch.cuda.synchronize()
    _say(f"city: uploaded {S.param_bytes() / 1e9:.1f} GB")
    # every device array holds the tree's rows in layout order (compared on
    # the host, in slices of 2^23 rows)
    perm = S.perm.astype(np.int64)
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        a = getattr(tree, k).reshape(S.n_nodes, -1)
        d = S.params[k].reshape(S.n_nodes, -1)
        for c in range(0, S.n_nodes, 1 << 23):
            e = min(S.n_nodes, c + (1 << 23))
            assert np.array_equal(d[c:e].cpu().numpy(), np.take(a, perm[c:e], axis=0)), (k, c)
    _say("city: device parameters checked")
    t0 = time.time()
    S.attach_hierarchy(tree)
    _say(f"city: hierarchy attached (height {S.hierarchy['height']}) in {time.time() - t0:.1f} s")
    t0 = time.time()
    O = oracle.OracleScene(tree)
    _say(f"city: oracle set up in {time.time() - t0:.1f} s")
    return tree, S, O


def test_city_views_select_render_backward(city):
    import torch
    from paper_2507_01110_amd.lodgs import Frame, grads_like
    tree, S, O = city
    cam0 = configs.city_path_camera(0)
    f = Frame(S, min(S.n_nodes, 1 << 24), 1 << 27, cam0.width, cam0.height)
    nodes = grads_like(S)
    for k, tau in VIEWS:
        cam = configs.city_path_camera(k)
        _say(f"city view: pose {k}, tau {tau}")
        idx, cnt = f.lod_select(cam, tau)
        img = f.render(cam)
        st = f.stats()
        assert st["status"] == 0, st
        n = int(cnt.item())
        t0 = time.time()
        ids, ost = O.select(cam, tau)
        got = idx[:n].cpu().numpy()
        assert np.array_equal(got, O.pos_of[ids]), (n, len(ids))
        assert st["n_spt_visible"] == ost["spt_visible"]
        F = oracle.OracleFrame(tree, ids, cam)
        info = F.info()
        assert st["n_drawn"] == info["n_visible"] and st["n_instances"] == info["n_inst"]
        t, p = f.instances()
        ot, op = F.instances()
        assert np.array_equal(t.cpu().numpy(), ot) and np.array_equal(p.cpu().numpy(), op)
        err = float(np.abs(img.cpu().numpy().astype(np.float64) - F.image).max())
        _say(f"  selected {n}, drawn {info['n_visible']}, instances {info['n_inst']}; max abs pixel err {err:.2e}"
             f" (oracle {time.time() - t0:.1f} s)")
        assert err <= 1e-4, err

        target = scenegen.target_image(cam.height, cam.width, 202 + k)
        _, dL = oracle.l1_loss_grad(F.image, target)
        for v in nodes.values():
            v.zero_()
        f.backward(torch.from_numpy(dL.astype(np.float32)).cuda(), nodes=nodes)
        _, g_o = F.backward(dL)
        rows = torch.from_numpy(O.pos_of[ids].astype(np.int64)).cuda()
        g = np.concatenate([nodes[key][rows].reshape(n, -1).cpu().numpy().astype(np.float64)
                            for key in ("means", "log_scales", "quats", "opacity_logits", "sh")], axis=1)
        errs = {name: float(np.linalg.norm(g[:, sl] - g_o[:, sl]) / max(np.linalg.norm(g_o[:, sl]), 1e-30))
                for name, sl in GROUPS.items()}
        _say("  grad rel L2 " + ", ".join(f"{name} {e:.2e}" for name, e in errs.items()))
        assert all(e <= 1e-3 for e in errs.values()), errs
        # nothing outside the selection was written
        for key, v in nodes.items():
            v[rows] = 0
            assert int(torch.count_nonzero(v)) == 0, key
        # the CONSERVATIVE cut of the same view
        idx, cnt = f.lod_select(cam, tau, conservative=True)
        nc = int(cnt.item())
        assert f.stats()["status"] == 0
        ids_c, _ = O.select(cam, tau, conservative=True)
        assert np.array_equal(idx[:nc].cpu().numpy(), O.pos_of[ids_c]), (nc, len(ids_c))
        _say(f"  conservative cut: {nc} selected (default {n})")
        # the whole-hierarchy comparator cuts of the same view
        for method in ("bfs", "parallel"):
            idx, cnt = f.lod_select(cam, tau, method=method)
            nm = int(cnt.item())
            assert f.stats()["status"] == 0
            want = O.pos_of[O.select_full(cam, tau, method)]
            assert np.array_equal(idx[:nm].cpu().numpy(), want), (method, nm, len(want))
            _say(f"  {method} cut: {nm} selected")


def test_city_cut_cache_along_the_path(city):
    # the SPT-cut cache over consecutive path poses, in lockstep with the
    # oracle's state machine (selection bit-exact, counters equal)
    from paper_2507_01110_amd.lodgs import CutCache, Frame
    tree, S, O = city
    cams = [configs.city_path_camera(k) for k in range(120, 126)]
    f = Frame(S, min(S.n_nodes, 1 << 24), 1 << 27, cams[0].width, cams[0].height)
    G = CutCache(S, 1_500_000, 0.8, 1.25, 4)
    C = oracle.OracleCutCache(O, 1_500_000, 0.8, 1.25, 4)
    for k, cam in enumerate(cams):
        idx, cnt = f.lod_select(cam, 1.0, cache=G)
        n = int(cnt.item())
        assert f.stats()["status"] == 0
        ids, _ = C.select(cam, 1.0)
        assert np.array_equal(idx[:n].cpu().numpy(), O.pos_of[ids]), (k, n, len(ids))
        g = G.stats()
        want = {"iterations": C.t, "hits": C.hits, "loads": C.loads, "evictions": C.evictions,
                "cached_spts": len(C.entries), "cached_nodes": sum(e[2] for e in C.entries.values())}
        assert g == want, (k, g, want)
        _say(f"  cached select, pose {120 + k}: {n} selected, {g}")
