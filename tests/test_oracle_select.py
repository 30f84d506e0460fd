"""Pins of the oracle's LoD cut (Sec. 4.1 Eq. 4, Sec. 4.3, Alg. 1, Alg. 2)
against plain-Python references and the invariants the paper states."""
import math

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import configs

from _helpers import (ancestors, bfs_cut, culled64, g64, hspt_cut_reference, hspt_roles, leaves_under,
                      random_tree)


def _random_camera(rng, extent=10.0, w=64, h=48):
    pos = rng.uniform(-3 * extent, 3 * extent, 3)
    tgt = rng.uniform(-extent, extent, 3)
    up = np.array([0.0, 0.0, 1.0]) if rng.random() < 0.5 else np.array([0.0, 1.0, 0.0])
    if abs(np.dot((tgt - pos) / np.linalg.norm(tgt - pos), up)) > 0.99:
        up = np.array([1.0, 0.0, 0.0])
    return scenegen.camera_look_at(pos, tgt, up, w, h, hfov_deg=rng.uniform(30, 90))


def test_hspt_split_matches_bfs_definition():
    rng = np.random.default_rng(1)
    for _ in range(50):
        t = random_tree(rng, int(rng.integers(1, 65)))
        S = oracle.OracleScene(t)
        assert np.array_equal(S.role, hspt_roles(t))
        for v in range(t.n_nodes):
            if S.role[v] == 0:
                assert S.spt_of[v] == -1
            else:
                r = v
                while S.role[r] != 1:
                    r = t.parent[r]
                assert S.spt_of[v] == r


def test_intervals_are_prefix_minima_of_ancestor_sizes():
    rng = np.random.default_rng(2)
    for _ in range(50):
        t = random_tree(rng, int(rng.integers(1, 65)))
        S = oracle.OracleScene(t)
        g32 = g64(t).astype(np.float32)
        assert np.array_equal(S.g, g32)
        for v in range(t.n_nodes):
            if S.role[v] == 0:
                continue
            leaf = t.left[v] < 0
            assert S.r_min[v] == (0.0 if leaf else g32[v])
            m = np.float32(np.inf)
            p = v
            while S.role[p] != 1:
                p = t.parent[p]
                m = min(m, g32[p])
            assert S.r_max[v] == m


def test_layout_is_preorder_then_sorted_segments():
    rng = np.random.default_rng(3)
    for _ in range(30):
        t = random_tree(rng, int(rng.integers(1, 65)))
        S = oracle.OracleScene(t)
        n = t.n_nodes
        assert np.array_equal(np.sort(S.perm), np.arange(n))
        assert np.array_equal(S.pos_of[S.perm], np.arange(n))
        # upper prefix = left-first preorder of upper nodes
        pre, roots, st = [], [], [t.root]
        while st:
            u = st.pop()
            if S.role[u] == 0:
                pre.append(u)
                st += [t.right[u], t.left[u]]
            else:
                roots.append(u)
        assert list(S.perm[: S.n_upper]) == pre
        assert S.n_spt == len(roots)
        for j, r in enumerate(roots):
            seg = S.perm[S.spt_begin[j]: S.spt_begin[j + 1]]
            assert seg[0] == r
            assert set(seg.tolist()) == set(np.nonzero(S.spt_of == r)[0].tolist())
            keys = [(-S.r_max[v], -S.r_min[v], v) for v in seg]
            assert keys == sorted(keys)


@pytest.mark.parametrize("cull", [False, True])
def test_cut_matches_python_two_step_reference(cull):
    rng = np.random.default_rng(4 + cull)
    for _ in range(150):
        t = random_tree(rng, int(rng.integers(1, 65)))
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        tau = float(np.float32(10 ** rng.uniform(-1, 2)))
        ref = hspt_cut_reference(t, cam, tau, cull)
        for mode in (0, 1):
            ids, _ = S.select(cam, tau, cull=cull, mode=mode)
            assert sorted(ids.tolist()) == ref
            assert np.all(np.diff(S.pos_of[ids]) > 0)  # layout order


def test_all_upper_equals_alg1_bfs_with_own_distances():
    """With no SPTs below the leaves (threshold -inf) the HSPT cut is the plain
    BFS cut of Alg. 1 with the per-node size test of Eq. 3/6."""
    rng = np.random.default_rng(5)
    for _ in range(60):
        t = random_tree(rng, int(rng.integers(2, 65)), log_threshold=-math.inf)
        S = oracle.OracleScene(t)
        assert np.all(S.role[t.left >= 0] == 0)
        cam = _random_camera(rng)
        tau = float(np.float32(10 ** rng.uniform(-1, 2)))
        g = g64(t)
        k = tau / cam.fx
        pos = cam.pos.astype(np.float64)
        cond = lambda u: t.left[u] < 0 or g[u] <= np.linalg.norm(t.means[u].astype(np.float64) - pos) * k
        ids, _ = S.select(cam, tau, cull=False)
        assert sorted(ids.tolist()) == sorted(bfs_cut(t, cond))


def _check_proper_and_covering(t, ids):
    sel = set(int(i) for i in ids)
    for v in sel:  # proper: no ancestor of a selected node is selected
        assert not (set(ancestors(t, v)) & sel)
    covered = []
    for v in sel:
        covered += leaves_under(t, v)
    assert sorted(covered) == list(range(t.n_leaves))  # every root-leaf path exactly once


def test_cut_is_proper_and_covers_every_path_once_random():
    rng = np.random.default_rng(6)
    for _ in range(100):
        t = random_tree(rng, int(rng.integers(1, 65)))
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        ids, _ = S.select(cam, float(10 ** rng.uniform(-1, 2)), cull=False)
        _check_proper_and_covering(t, ids)


@pytest.mark.parametrize("tau", [0.5, 1.0, 8.0, 64.0])
def test_cut_is_proper_and_covers_every_path_once_tiny(tiny_tree, tiny_oracle, tau):
    ids, st = tiny_oracle.select(configs.tiny_camera(), tau, cull=False)
    sel = np.zeros(tiny_tree.n_nodes, bool)
    sel[ids] = True
    # coverage by counting selected ancestors-or-self of every leaf
    cnt = np.zeros(tiny_tree.n_leaves, int)
    for leaf in range(tiny_tree.n_leaves):
        cnt[leaf] = sel[leaf] + sum(sel[a] for a in ancestors(tiny_tree, leaf))
    assert np.all(cnt == 1)
    if tau >= 8:
        assert np.any(ids >= tiny_tree.n_leaves)  # interior nodes are chosen at coarse tau


def test_tau_limits():
    rng = np.random.default_rng(7)
    for _ in range(40):
        t = random_tree(rng, int(rng.integers(1, 65)))
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        ids, _ = S.select(cam, 1e30, cull=False)
        assert ids.tolist() == [t.root]
        ids, _ = S.select(cam, 0.0, cull=False)
        assert sorted(ids.tolist()) == list(range(t.n_leaves))


def test_cull_drops_exactly_the_culled_subtrees():
    rng = np.random.default_rng(8)
    for _ in range(100):
        t = random_tree(rng, int(rng.integers(1, 65)))
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        tau = float(10 ** rng.uniform(-1, 2))
        off = set(S.select(cam, tau, cull=False)[0].tolist())
        on = set(S.select(cam, tau, cull=True)[0].tolist())
        rho = 3.0 * np.exp(t.log_scales.astype(np.float64)).max(axis=1)

        def tested_path(v):  # nodes whose frustum test gates v: upper ancestors and the SPT root
            path = [v] + ancestors(t, v)
            return [u for u in path if S.role[u] in (0, 1)]
        expect = {v for v in off if not any(culled64(cam, t.means[u], rho[u]) for u in tested_path(v))}
        assert on == expect


def test_exact_ties_follow_eq4_inequalities():
    """X == g selects (>= in Eq. 4's distance form), X just below g does not."""
    # one interior node (a single SPT of 3 nodes) at distance exactly 5 from the camera
    means = np.array([[3.0, 4.0, 0.0], [3.0, 4.0, 0.1], [3.0, 4.0, -0.1]])
    ls = np.array([[0.0, 0.0, 0.0], [-2.0, -2.0, -2.0], [-2.0, -2.0, -2.0]])
    q = np.tile([1.0, 0.0, 0.0, 0.0], (3, 1))
    t = scenegen.tree_from_arrays(means, ls, q, np.zeros(3), np.zeros((3, 1, 3)), [1, -1, -1], [2, -1, -1],
                                  [-1, 0, 0], 0, 100.0, 0)
    S = oracle.OracleScene(t)
    assert S.role.tolist() == [1, 2, 2]
    cam = scenegen.Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), np.zeros(3, np.float32),
                          1.0, 1.0, 0.5, 0.5, 1, 1, 0.2)
    g = S.g[0]
    # find tau with float32(5 * float32(tau / 1)) == g exactly
    tau = np.float32(g / np.float32(5.0))
    for _ in range(8):
        if np.float32(np.float32(5.0) * tau) == g:
            break
        tau = np.nextafter(tau, np.float32(np.inf)) if np.float32(5.0) * tau < g else np.nextafter(tau, np.float32(0))
    assert np.float32(np.float32(5.0) * tau) == g
    ids, st = S.select(cam, float(tau), cull=False)
    assert ids.tolist() == [0] and st["ties_exact"] >= 1
    below = np.nextafter(tau, np.float32(0))
    while np.float32(np.float32(5.0) * below) == g:
        below = np.nextafter(below, np.float32(0))
    ids, _ = S.select(cam, float(below), cull=False)
    assert sorted(ids.tolist()) == [1, 2]


# ---------------------------------------------------------------------------
# CONSERVATIVE variant (Sec. 4.1, the conservative M_d): each SPT is cut at
# X = max(0, d_root - R) tau / fx with R the SPT's radius about its root.

def _own_x(t, v, cam, tau):
    return np.linalg.norm(t.means[v].astype(np.float64) - cam.pos.astype(np.float64)) * tau / cam.fx


def test_conservative_cut_is_never_coarser_than_each_nodes_own_distance():
    # the triangle inequality: no member is closer than d_root - R, so a
    # selected interior node passes the size test at its own distance
    rng = np.random.default_rng(31)
    checked = 0
    for _ in range(120):
        t = random_tree(rng, int(rng.integers(2, 65)))
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        tau = float(np.float32(10 ** rng.uniform(-1, 2)))
        ids, _ = S.select(cam, tau, cull=False, conservative=True)
        for v in ids.tolist():
            if t.left[v] < 0:
                continue
            assert S.g[v] <= _own_x(t, v, cam, tau) * (1 + 1e-5), (v, S.g[v], _own_x(t, v, cam, tau))
            checked += 1
    assert checked > 50


def test_conservative_cut_is_proper_covers_every_path_and_refines_the_default_cut():
    rng = np.random.default_rng(32)
    finer = 0
    for _ in range(100):
        t = random_tree(rng, int(rng.integers(1, 65)))
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        tau = float(np.float32(10 ** rng.uniform(-1, 2)))
        for mode in (0, 1):
            cons, _ = S.select(cam, tau, cull=False, mode=mode, conservative=True)
            _check_proper_and_covering(t, cons)
            base = set(S.select(cam, tau, cull=False, mode=mode)[0].tolist())
            for c in cons.tolist():  # every conservative node lies at or below a default node
                assert c in base or any(a in base for a in ancestors(t, c))
            finer += len(cons) > len(base)
    assert finer > 0


def test_conservative_cut_equals_the_default_cut_when_every_spt_has_zero_radius():
    rng = np.random.default_rng(33)
    for _ in range(40):
        t = random_tree(rng, int(rng.integers(1, 65)))
        t.means[:] = t.means[t.root]  # every SPT radius is 0
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        tau = float(np.float32(10 ** rng.uniform(-1, 2)))
        for cull in (False, True):
            a = S.select(cam, tau, cull=cull, conservative=True)[0]
            b = S.select(cam, tau, cull=cull)[0]
            assert np.array_equal(a, b)


def test_conservative_cut_takes_the_leaves_of_an_spt_whose_radius_holds_the_camera():
    # one SPT (the whole tree); the camera 0.1 R from the root's mean: X = 0,
    # so only the leaves (r_min = 0) are selected, while the default cut at
    # the same large tau stays coarse
    rng = np.random.default_rng(34)
    for _ in range(40):
        t = random_tree(rng, int(rng.integers(4, 65)), log_threshold=math.inf)
        S = oracle.OracleScene(t)
        assert S.n_upper == 0 and S.n_spt == 1
        m = t.means.astype(np.float64)
        R = np.linalg.norm(m - m[t.root], axis=1).max()
        d = rng.normal(size=3)
        pos = m[t.root] + 0.1 * R * d / np.linalg.norm(d)
        cam = scenegen.camera_look_at(pos, pos + [1.0, 0.3, 0.2], (0, 0, 1), 64, 48)
        ids = S.select(cam, 1e4, cull=False, conservative=True)[0]
        assert sorted(ids.tolist()) == list(range(t.n_leaves))
        assert len(S.select(cam, 1e4, cull=False)[0]) < t.n_leaves


# The whole-hierarchy comparator cuts the HSPT replaces (Sec. 4.3): the BFS
# cut and the parallel cut of Eq. 5, every node at its own distance.

def _depths(t):
    d = np.zeros(t.n_nodes, np.int64)
    st = [t.root]
    while st:
        u = st.pop()
        if t.left[u] >= 0:
            for c in (t.left[u], t.right[u]):
                d[c] = d[u] + 1
                st.append(c)
    return d


def _heap_tree(rng, n_leaves):
    """Every node at one point, and each child smaller than its parent along
    every axis: fineness at any camera passes from a parent to its children,
    and the cull spheres are nested."""
    t = random_tree(rng, n_leaves)
    t.means[:] = t.means[t.root]
    d = _depths(t)
    t.log_scales[:] = (0.5 - 0.3 * d[:, None] + rng.uniform(0.0, 0.1, (t.n_nodes, 3))).astype(np.float32)
    return t


@pytest.mark.parametrize("cull", [False, True])
def test_bfs_cut_equals_the_hspt_cut_when_every_interior_node_is_upper(cull):
    # with the SPTs reduced to single leaves the HSPT cut is Alg. 1 over the
    # whole hierarchy, culling included
    rng = np.random.default_rng(41)
    for _ in range(60):
        t = random_tree(rng, int(rng.integers(1, 65)), log_threshold=-math.inf)
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        tau = float(np.float32(10 ** rng.uniform(-1, 2)))
        assert np.array_equal(S.select_full(cam, tau, "bfs", cull=cull), S.select(cam, tau, cull=cull)[0])


def test_bfs_cut_matches_the_python_queue_reference_and_is_proper():
    rng = np.random.default_rng(42)
    for _ in range(80):
        t = random_tree(rng, int(rng.integers(1, 65)))
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        tau = float(np.float32(10 ** rng.uniform(-1, 2)))
        g = g64(t)
        k = tau / cam.fx
        pos = cam.pos.astype(np.float64)
        cond = lambda u: t.left[u] < 0 or g[u] <= np.linalg.norm(t.means[u].astype(np.float64) - pos) * k
        ids = S.select_full(cam, tau, "bfs", cull=False)
        assert sorted(ids.tolist()) == sorted(bfs_cut(t, cond))
        _check_proper_and_covering(t, ids)
        assert np.all(np.diff(S.pos_of[ids]) > 0)


@pytest.mark.parametrize("cull", [False, True])
def test_every_bfs_node_passes_eq5_so_the_parallel_cut_contains_the_bfs_cut(cull):
    # a BFS-selected node is fine and was reached through a parent that was not
    rng = np.random.default_rng(43)
    larger = 0
    for _ in range(80):
        t = random_tree(rng, int(rng.integers(1, 65)))
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        tau = float(np.float32(10 ** rng.uniform(-1, 2)))
        b = set(S.select_full(cam, tau, "bfs", cull=cull).tolist())
        p = S.select_full(cam, tau, "parallel", cull=cull)
        assert b <= set(p.tolist())
        assert np.all(np.diff(S.pos_of[p]) > 0)
        larger += len(p) > len(b)
    assert larger > 0  # random trees break the heap condition


@pytest.mark.parametrize("cull", [False, True])
def test_parallel_cut_equals_the_bfs_cut_under_the_heap_condition(cull):
    rng = np.random.default_rng(44)
    for _ in range(60):
        t = _heap_tree(rng, int(rng.integers(1, 65)))
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        tau = float(np.float32(10 ** rng.uniform(-1, 3)))
        p = S.select_full(cam, tau, "parallel", cull=cull)
        assert np.array_equal(p, S.select_full(cam, tau, "bfs", cull=cull))
        if not cull:
            _check_proper_and_covering(t, p)


def test_parallel_cut_selects_an_ancestor_and_its_descendants_when_a_child_outgrows_its_parent():
    # root R (g 1) with children A (g 3, above the threshold) and leaf B; A's
    # children are the leaves L1, L2; all at one point, X = 2: R is fine as the
    # root, A is not, so L1 and L2 pass Eq. 5 too: R and its grandchildren
    # are both selected, while the BFS stops at R
    import scenegen
    left = np.array([-1, -1, -1, 0, 3], np.int32)   # 0 L1, 1 L2, 2 B, 3 A, 4 R
    right = np.array([-1, -1, -1, 1, 2], np.int32)
    parent = np.array([3, 3, 4, 4, -1], np.int32)
    g_want = {3: 3.0, 4: 1.0}
    ls = np.full((5, 3), -3.0)
    for v, gv in g_want.items():  # isotropic: g = sqrt(3) s
        ls[v] = math.log(gv / math.sqrt(3.0))
    t = scenegen.tree_from_arrays(np.zeros((5, 3)), ls, np.tile([1.0, 0, 0, 0], (5, 1)), np.zeros(5),
                                  np.zeros((5, 4, 3)), left, right, parent, 4, -math.inf, 1)
    S = oracle.OracleScene(t)
    cam = scenegen.camera_look_at((0.0, 0.0, -10.0), (0.0, 0.0, 0.0), (0, 1, 0), 64, 48)
    tau = float(np.float32(2.0 / 10.0 * cam.fx))  # X = 2 at distance 10
    assert sorted(S.select_full(cam, tau, "parallel", cull=False).tolist()) == [0, 1, 4]
    assert S.select_full(cam, tau, "bfs", cull=False).tolist() == [4]


@pytest.mark.parametrize("cull", [False, True])
def test_lod_noise_scales_only_the_spt_root_distances(cull):
    """Varying level of detail (implementation appendix): the distances to the
    SPT centres are multiplied by the iteration's factor; the upper nodes keep
    their own distances.  Against the float64 two-step reference with the same
    rule; a factor on every distance (tau times the factor) gives a different
    cut on some of these trees."""
    rng = np.random.default_rng(71 + cull)
    differs = 0
    for _ in range(150):
        t = random_tree(rng, int(rng.integers(2, 65)))
        S = oracle.OracleScene(t)
        cam = _random_camera(rng)
        tau = float(np.float32(10 ** rng.uniform(-1, 2)))
        s = float(np.float32(1.0 + 5.0 * rng.uniform() ** 4))
        ref = hspt_cut_reference(t, cam, tau, cull, spt_scale=s)
        for mode in (0, 1):
            ids, _ = S.select(cam, tau, cull=cull, mode=mode, spt_scale=s)
            assert sorted(ids.tolist()) == ref
        differs += ref != hspt_cut_reference(t, cam, tau * s, cull)
    assert differs > 0
