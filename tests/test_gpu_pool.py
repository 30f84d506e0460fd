"""The device pool of cached SPT cuts' rows (lodgs_row_pool_*, Sec. 4.4
"Caching on the GPU", Alg. 3's load / insert / write-back) run beside the
oracle's SPT-cut cache state machine: after every view the assembled rows
equal the scene's rows of the selection bit for bit, the pooled nodes are
exactly the nodes of the cached entries' cuts, and the rows read from host
memory are exactly the selected nodes of the entries the view loaded that
their entry did not already hold.
Trained rows stored into the pool reach host memory when their entry
leaves."""
import sys

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import configs

pytestmark = pytest.mark.gpu

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _lockstep(torch, tree, cams, tau, max_nodes, d_min, d_max, flush, max_inst):
    from paper_2507_01110_amd.lodgs import CutCache, Frame, HostParams, RowPool, Scene, rows_like
    O = oracle.OracleScene(tree)
    S = Scene(tree)
    host = HostParams.from_scene(S)
    f = Frame(S, S.n_nodes, max_inst, cams[0].width, cams[0].height)
    G = CutCache(S, max_nodes, d_min, d_max, flush)
    P = RowPool(G, host, max_nodes)
    C = oracle.OracleCutCache(O, max_nodes, d_min, d_max, flush)
    rows = rows_like(tree.sh_degree, S.n_nodes)
    slot = torch.empty(S.n_nodes, dtype=torch.int32, device="cuda")
    spt_of = O.spt_of  # tree id -> its SPT's root tree id, -1 for upper nodes
    pooled = {}  # SPT root tree id -> layout positions of its cached cut
    totals = {"host": 0, "selected": 0}
    for it, cam in enumerate(cams):
        idx, cnt = f.lod_select(cam, tau, cache=G)
        P.gather(idx, cnt, rows)
        ids, _ = C.select(cam, tau)
        n = int(cnt.item())
        assert f.stats()["status"] == 0
        sel = idx[:n].long()
        assert np.array_equal(sel.cpu().numpy(), O.pos_of[ids]), it
        for k in GROUPS:
            assert torch.equal(rows[k][:n], S.params[k][sel]), (it, k)
        # the oracle's view of the pool: an entry cut afresh now holds this
        # view's nodes of its SPT and reads from host memory only those it did
        # not hold; entries that left hold nothing, and a loaded SPT that is
        # not cached reads all its nodes from host memory
        sp = spt_of[ids]
        fresh_rows = 0
        for r in C.last_loaded:
            old = pooled.pop(r, set())
            nodes = set(O.pos_of[ids[sp == r]].tolist())
            if r in C.entries:
                fresh_rows += len(nodes - old)
                pooled[r] = nodes
            else:
                fresh_rows += len(nodes)
        for r in list(pooled):
            if r not in C.entries:
                del pooled[r]
        st = P.stats(node_slot=slot)
        got = set(np.flatnonzero(slot.cpu().numpy() >= 0).tolist())
        want = set().union(*pooled.values()) if pooled else set()
        assert got == want, (it, len(got), len(want))
        assert st["host_rows"] == fresh_rows, (it, st, fresh_rows)
        assert st["pooled_rows"] == len(want) and st["insert_failures"] == 0
        totals["host"] += st["host_rows"]
        totals["selected"] += n
        _say(f"  view {it}: {n} selected, {st['host_rows']} rows from host, {st['pooled_rows']} pooled")
    return S, f, G, P, C, host, rows, totals


def test_pool_tiny_lockstep(torch_cuda):
    torch = torch_cuda
    tree = scenegen.build_tree(configs.tiny_spec())
    cams = [scenegen.camera_look_at((28 * np.cos(a), 28 * np.sin(a), 12.0), (0, 0, 0), (0, 0, 1), 256, 256)
            for a in np.linspace(0.0, 1.2, 8)]
    for prm in ((10 ** 6, 0.5, 1.5, 0), (6000, 0.6, 1.6, 5), (20000, 1.0, 1.0, 0)):
        _, _, _, _, _, _, _, tot = _lockstep(torch, tree, cams, 1.0, *prm, max_inst=1 << 20)
        _say("tiny", prm, tot)
        if prm[0] == 10 ** 6:
            assert tot["host"] < tot["selected"]  # hits read nothing over the host link


@pytest.mark.parametrize("sh_degree", [0, 1, 2])
def test_pool_lower_sh_degrees(torch_cuda, sh_degree):
    """Rows of 3, 12 and 27 SH floats (float and float4 moves) through the
    pool, stores and write-back included."""
    torch = torch_cuda
    tree = scenegen.build_tree(configs.tiny_spec(n=8192, seed=3, sh_degree=sh_degree))
    cams = [scenegen.camera_look_at((26 * np.cos(a), 26 * np.sin(a), 10.0), (0, 0, 0), (0, 0, 1), 192, 160)
            for a in np.linspace(0.0, 1.5, 6)]
    S, f, G, P, C, host, rows, tot = _lockstep(torch, tree, cams, 1.0, 5000, 0.6, 1.6, 4, max_inst=1 << 19)
    _say("sh degree", sh_degree, tot)
    idx, cnt = f.idx.clone(), f.count.clone()
    n = int(cnt.item())
    for k in GROUPS:
        rows[k][:n] = rows[k][:n] * 2.0 + 0.5
    P.store(idx, cnt, rows)
    rows_back = {k: torch.empty_like(v) for k, v in rows.items()}
    P.gather(idx, cnt, rows_back)  # the same selection again: nothing moves, rows read back
    for k in GROUPS:
        assert torch.equal(rows_back[k][:n], rows[k][:n]), k  # stored rows read back from upper, pool or host


def test_pool_medium_flyin_and_write_back(torch_cuda):
    torch = torch_cuda
    tree = scenegen.build_tree(configs.medium_spec(n=500_000, seed=14))
    cams = [scenegen.camera_yaw_pitch((4.0 * k, 1.2 * k, 40.0 - 3.0 * k), 0.3, np.radians(-45.0), 1280, 720)
            for k in range(6)]
    # flush every 8th select: the 8th below drops every entry
    S, f, G, P, C, host, rows, tot = _lockstep(torch, tree, cams, 1.0, 300000, 0.7, 1.4, 8, max_inst=1 << 23)
    _say("medium", tot)
    assert tot["host"] < tot["selected"]
    # trained rows: +1 on every row of the last view, stored; upper and
    # unpooled rows reach host memory at once, pooled ones when their entry
    # leaves (the flush of the 8th select)
    idx, cnt = f.idx.clone(), f.count.clone()
    n = int(cnt.item())
    for k in GROUPS:
        rows[k][:n] += 1.0
    P.store(idx, cnt, rows)
    torch.cuda.synchronize()
    before = {k: host.params[k].clone() for k in GROUPS}
    far = scenegen.camera_yaw_pitch((-200.0, -200.0, 60.0), 2.5, np.radians(-30.0), 1280, 720)
    for _ in range(2):  # selects 7 and 8
        i2, c2 = f.lod_select(far, 1.0, cache=G)
        P.gather(i2, c2, rows)
    torch.cuda.synchronize()
    st = P.stats()
    _say("after the flush", st)
    assert st["written_back"] > 0
    changed = (host.params["means"] != before["means"]).any(dim=1).nonzero().flatten()
    assert len(changed) == st["written_back"]
    diff = host.params["means"][changed] - S.params["means"][changed.cuda()].cpu()
    assert torch.allclose(diff, torch.ones_like(diff), atol=1e-4)  # the stored +1
    assert bool(torch.isin(changed, idx[:n].long().cpu()).all())


def test_pool_write_back_puts_every_stored_row_in_host_memory(torch_cuda):
    """After lodgs_row_pool_store, lodgs_row_pool_write_back makes host memory
    hold every stored row (pooled, upper or neither), the pool keeps its
    slots, and a second write-back writes nothing."""
    torch = torch_cuda
    tree = scenegen.build_tree(configs.tiny_spec(n=8192, seed=4))
    cams = [scenegen.camera_look_at((26 * np.cos(a), 26 * np.sin(a), 10.0), (0, 0, 0), (0, 0, 1), 192, 160)
            for a in np.linspace(0.0, 1.0, 4)]
    S, f, G, P, C, host, rows, tot = _lockstep(torch, tree, cams, 1.0, 10 ** 6, 0.5, 1.5, 0, max_inst=1 << 19)
    idx, cnt = f.idx.clone(), f.count.clone()
    n = int(cnt.item())
    for k in GROUPS:
        rows[k][:n] = rows[k][:n] * 3.0 - 0.25
    P.store(idx, cnt, rows)
    before = P.stats()
    P.write_back()
    torch.cuda.synchronize()
    after = P.stats()
    sel = idx[:n].long().cpu()
    for k in GROUPS:
        assert torch.equal(host.params[k][sel], rows[k][:n].cpu()), k
    assert after["pooled_rows"] == before["pooled_rows"]
    assert after["written_back"] > before["written_back"]
    P.write_back()
    torch.cuda.synchronize()
    assert P.stats()["written_back"] == after["written_back"]  # nothing changed since


def test_pool_views_in_flight_equal_one_at_a_time(torch_cuda):
    """The cached select and the pooled gather in view order on one stream, each
    view's render from its rows, L1 and backward on its frame's stream, three
    frames taking turns: images and selection-indexed gradients equal those of
    one view at a time bit for bit."""
    torch = torch_cuda
    from paper_2507_01110_amd.lodgs import CutCache, Frame, HostParams, RowPool, Scene, grads_like, rows_like
    tree = scenegen.build_tree(configs.medium_spec(n=500_000, seed=15))
    S = Scene(tree)
    host = HostParams.from_scene(S)
    W, H = 1280, 720
    cams = [scenegen.camera_yaw_pitch((3.0 * k, 1.0 * k, 40.0 - 2.0 * k), 0.3 + 0.05 * k, np.radians(-45.0), W, H)
            for k in range(8)]
    targets = [torch.from_numpy(scenegen.target_image(H, W, 70 + k)).cuda() for k in range(len(cams))]
    cap_sel, cap_inst = 1 << 21, 1 << 23

    def run(n_fl):
        G = CutCache(S, 300_000, 0.7, 1.4, 0)
        P = RowPool(G, host, 300_000)
        frames = [Frame(S, cap_sel, cap_inst, W, H) for _ in range(n_fl)]
        rows = [rows_like(tree.sh_degree, cap_sel) for _ in range(n_fl)]
        sels = [grads_like(S, cap_sel) for _ in range(n_fl)]
        imgs = [torch.empty((H, W, 3), dtype=torch.float32, device="cuda") for _ in range(n_fl)]
        dls = [torch.empty_like(imgs[0]) for _ in range(n_fl)]
        sS = torch.cuda.Stream()
        sF = [torch.cuda.Stream() for _ in range(n_fl)] if n_fl > 1 else [sS]
        gathered = [torch.cuda.Event() for _ in range(n_fl)]
        done = [torch.cuda.Event() for _ in range(n_fl)]
        out = []
        for i, cam in enumerate(cams):
            k = i % n_fl
            sS.wait_event(done[k])
            frames[k].lod_select(cam, 1.0, cache=G, stream=sS)
            P.gather(frames[k].idx, frames[k].count, rows[k], stream=sS)
            gathered[k].record(sS)
            s = sF[k]
            s.wait_event(gathered[k])
            frames[k].render_rows(cam, rows[k], out=imgs[k], stream=s)
            frames[k].l1_loss(imgs[k], targets[i], grad=dls[k], stream=s)
            frames[k].backward(dls[k], sel=sels[k], stream=s)
            with torch.cuda.stream(s):
                n = frames[k].count.clone()
                out.append((imgs[k].clone(), n, {g: t.clone() for g, t in sels[k].items()}))
            done[k].record(s)
        torch.cuda.synchronize()
        for f in frames:
            assert f.stats()["status"] == 0
        return out

    serial = run(1)
    flight = run(3)
    for i in range(len(cams)):
        (ia, na, ga), (ib, nb, gb) = serial[i], flight[i]
        assert torch.equal(ia, ib), i
        n = int(na.item())
        assert n == int(nb.item()) and n > 0, i
        for g in GROUPS:
            assert torch.equal(ga[g][:n], gb[g][:n]), (i, g)
        _say(f"  view {i}: {n} selected, equal")
