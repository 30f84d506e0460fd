"""Densification on the hierarchy (host side): the spawn parameters against
their two defining conditions, and the tree edits (spawn, respawn and its
edge cases) against the structure they must keep: one binary tree over every
node, consistent parent links, and the HSPT builder and the cut accepting
the result."""
import math

import numpy as np

import oracle
import scenegen
from paper_2507_01110_amd.densify import densify, split_params

from _helpers import random_tree


def _check_tree(t):
    n = t.n_nodes
    seen = np.zeros(n, bool)
    st = [t.root]
    assert t.parent[t.root] == -1
    while st:
        u = st.pop()
        assert not seen[u]
        seen[u] = True
        if t.left[u] >= 0:
            assert t.right[u] >= 0
            for c in (t.left[u], t.right[u]):
                assert t.parent[c] == u
                st.append(c)
        else:
            assert t.right[u] < 0
    assert seen.all()


def test_split_keeps_the_centre_opacity_and_the_alpha_integral():
    for o in (0.01, 0.3, 0.7, 0.95):
        lo, ls = split_params(math.log(o / (1 - o)), np.zeros(3))
        oc = 1.0 / (1.0 + math.exp(-lo))
        assert abs((1 - (1 - oc) ** 2) - o) < 1e-12
        s = math.exp(ls[0])
        # integral over the plane of 1 - (1 - oc g)^2 with g of unit-free std s,
        # by quadrature, against the parent's o * 2 pi (std 1)
        r = np.linspace(0, 12 * max(s, 1.0), 200001)
        g = np.exp(-r * r / (2 * s * s))
        f = (1 - (1 - oc * g) ** 2) * 2 * np.pi * r
        integral = float(np.sum((f[1:] + f[:-1]) * 0.5 * np.diff(r)))
        assert abs(integral - o * 2 * np.pi) < 1e-6 * o * 2 * np.pi


def test_spawn_grows_two_children_under_the_chosen_leaves():
    rng = np.random.default_rng(51)
    t = random_tree(rng, 40)
    stat = rng.random(t.n_nodes)
    t.opacity_logits[:] = 2.0  # nothing dead
    t2, info = densify(t, stat, n_spawn=5)
    assert info == {"respawned": 0, "spawned": 5} and t2.n_nodes == t.n_nodes + 10
    _check_tree(t2)
    leaves = np.flatnonzero(t.left < 0)
    chosen = leaves[np.argsort(-stat[leaves], kind="stable")][:5]
    for u in chosen:
        a, b = t2.left[u], t2.right[u]
        assert a >= t.n_nodes and b >= t.n_nodes
        assert np.array_equal(t2.means[a], t.means[u]) and np.array_equal(t2.sh[b], t.sh[u])
    oracle.OracleScene(t2).select(scenegen.camera_look_at((0, 0, 30), (0, 0, 0), (0, 1, 0), 64, 48), 1.0)


def test_respawn_moves_the_sibling_up_and_the_pair_under_a_chosen_leaf():
    rng = np.random.default_rng(52)
    for it in range(30):
        t = random_tree(rng, int(rng.integers(3, 50)))
        t.opacity_logits[:] = 2.0
        leaves = np.flatnonzero(t.left < 0)
        d = int(rng.choice(leaves))
        t.opacity_logits[d] = -10.0  # dead
        stat = rng.random(t.n_nodes)
        p, g = int(t.parent[d]), int(t.parent[t.parent[d]]) if t.parent[d] >= 0 else -1
        s = int(t.right[p] if t.left[p] == d else t.left[p])
        t2, info = densify(t, stat, n_spawn=0)
        assert info["respawned"] == 1 and t2.n_nodes == t.n_nodes
        _check_tree(t2)
        assert t2.parent[s] == g and (g >= 0 or t2.root == s)  # the sibling, leaf or subtree, took the place
        tgt = int(t2.parent[d])
        assert t2.parent[p] == tgt and {int(t2.left[tgt]), int(t2.right[tgt])} == {d, p}
        assert t2.left[p] < 0 and t.left[tgt] < 0  # the chosen node was a leaf
        oracle.OracleScene(t2)


def test_two_dead_siblings_respawn_only_the_right_one():
    rng = np.random.default_rng(53)
    t = random_tree(rng, 30)
    t.opacity_logits[:] = 2.0
    pairs = [u for u in range(t.n_nodes) if t.left[u] >= 0 and t.left[t.left[u]] < 0 and t.left[t.right[u]] < 0]
    p = pairs[0]
    l, r = int(t.left[p]), int(t.right[p])
    t.opacity_logits[[l, r]] = -10.0
    t2, info = densify(t, rng.random(t.n_nodes), n_spawn=0)
    assert info["respawned"] == 1
    _check_tree(t2)
    assert t2.left[l] < 0 and t2.parent[l] == t.parent[p]  # the left one took the parent's place
    assert t2.parent[r] == t2.parent[p]  # the right one and the parent were respawned together


def _respawn_one_at_a_time(t, d, tgt):
    """Reference edit for one respawn (the definition): the sibling takes the
    parent's place, the dead leaf and its parent go under the chosen leaf."""
    left, right, parent = t["left"], t["right"], t["parent"]
    p = parent[d]
    s = right[p] if left[p] == d else left[p]
    g = parent[p]
    parent[s] = g
    if g >= 0:
        if left[g] == p:
            left[g] = s
        else:
            right[g] = s
    else:
        t["root"] = s
    left[tgt], right[tgt] = d, p
    parent[d] = parent[p] = tgt
    left[p] = right[p] = -1


def test_parallel_respawn_equals_the_edits_one_at_a_time():
    # many dead leaves in one step: the parallel edit gives the tree that the
    # planned respawns give applied one after another (they touch disjoint
    # links), and the plan obeys both rules
    from paper_2507_01110_amd.densify import respawn_plan
    rng = np.random.default_rng(54)
    for it in range(40):
        t = random_tree(rng, int(rng.integers(8, 120)))
        t.opacity_logits[:] = 2.0
        leaves = np.flatnonzero(t.left < 0)
        dead = rng.choice(leaves, size=max(1, len(leaves) // 4), replace=False)
        t.opacity_logits[dead] = -10.0
        stat = rng.random(t.n_nodes)
        plan = respawn_plan(t.left, t.right, t.parent, np.sort(dead))
        dead_set = set(dead.tolist())
        planned = set(plan.tolist())
        for d in plan:
            p = t.parent[d]
            s = t.right[p] if t.left[p] == d else t.left[p]
            assert not (t.left[p] == d and s in dead_set), "the left one of two dead siblings"
        sib = {int(t.right[t.parent[d]] if t.left[t.parent[d]] == d else t.left[t.parent[d]]) for d in plan}
        assert not any(int(t.parent[d]) in sib for d in plan), "a parent that is another's sibling"
        t2, info = densify(t, stat, n_spawn=0)
        _check_tree(t2)
        o = 1.0 / (1.0 + np.exp(-t.opacity_logits.astype(np.float64)))
        cand = np.flatnonzero((t.left < 0) & (o >= 0.005))
        targets = cand[np.lexsort((cand, -stat[cand]))][: len(plan)]
        ref = {"left": t.left.copy(), "right": t.right.copy(), "parent": t.parent.copy(), "root": int(t.root)}
        for d, tgt in zip(plan[: len(targets)], targets):
            _respawn_one_at_a_time(ref, int(d), int(tgt))
        assert info["respawned"] == min(len(plan), len(targets))
        assert np.array_equal(t2.left, ref["left"]) and np.array_equal(t2.right, ref["right"])
        assert np.array_equal(t2.parent, ref["parent"]) and int(t2.root) == ref["root"]
        assert planned <= dead_set


def test_chained_dead_leaves_wait_for_the_next_step():
    # d1's sibling is the parent of d2: only d1 is respawned now; the next
    # step respawns d2
    from paper_2507_01110_amd.densify import respawn_plan
    rng = np.random.default_rng(55)
    found = 0
    for it in range(200):
        t = random_tree(rng, 24)
        t.opacity_logits[:] = 2.0
        for p1 in range(t.n_nodes):
            l, r = int(t.left[p1]), int(t.right[p1])
            if l < 0 or t.left[l] >= 0 or t.left[r] < 0:
                continue
            d1, s1 = l, r  # a leaf whose sibling s1 is interior
            d2 = int(t.left[s1]) if t.left[t.left[s1]] < 0 else (int(t.right[s1]) if t.left[t.right[s1]] < 0 else -1)
            if d2 < 0:
                continue
            other = int(t.right[s1]) if d2 == int(t.left[s1]) else int(t.left[s1])
            if t.left[other] < 0:
                continue  # keep the sibling rule out of it
            t.opacity_logits[[d1, d2]] = -10.0
            assert respawn_plan(t.left, t.right, t.parent, np.array([min(d1, d2), max(d1, d2)])).tolist() == [d1]
            t2, info = densify(t, rng.random(t.n_nodes), n_spawn=0)
            assert info["respawned"] == 1
            _check_tree(t2)
            t3, info3 = densify(t2, rng.random(t2.n_nodes), n_spawn=0)
            assert info3["respawned"] >= 1
            _check_tree(t3)
            found += 1
            break
        if found >= 5:
            break
    assert found >= 5


def test_prune_zeroes_the_leaves_idle_for_twice_the_training_set():
    from paper_2507_01110_amd.densify import PRUNED_LOGIT, prune
    rng = np.random.default_rng(56)
    t = random_tree(rng, 50)
    t.opacity_logits[:] = 1.0
    last = rng.integers(0, 100, size=t.n_nodes)
    n = prune(t, last, iteration=100, train_views=20)
    leaf = t.left < 0
    idle = (100 - last >= 40) & leaf
    assert n == int(idle.sum()) > 0
    assert np.all(t.opacity_logits[idle] == PRUNED_LOGIT)
    assert np.all(t.opacity_logits[~idle] == 1.0)  # interior nodes and recent leaves untouched
    assert 1.0 / (1.0 + np.exp(-PRUNED_LOGIT)) < 1e-12
    assert prune(t, last, iteration=100, train_views=20) == 0  # already pruned
    # a pruned leaf is dead: the next densification step respawns it
    t2, info = densify(t, rng.random(t.n_nodes), n_spawn=0)
    assert info["respawned"] >= 1
    _check_tree(t2)
