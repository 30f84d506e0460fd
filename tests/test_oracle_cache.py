"""Pins of the oracle's SPT-cut cache (Sec. 4.4 "Caching on the GPU", Eq. 7,
Alg. 3): limits where it must equal the plain HSPT cut, the reuse of a cached
cut SPT by SPT, the flush, and the budget invariants."""
import numpy as np
import pytest

import oracle
import scenegen
from scenegen import configs


@pytest.fixture(scope="module")
def tiny():
    tree = scenegen.build_tree(configs.tiny_spec())
    return tree, oracle.OracleScene(tree)


def _cams():
    return [scenegen.camera_look_at((0.0, 0.0, z), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 256, 256) for z in (30.0, 24.0, 19.0)]


def _by_spt(O, ids):
    out = {}
    for v, r in zip(ids.tolist(), O.spt_of[ids].tolist()):
        out.setdefault(r, []).append(v)
    return out


def test_a_zero_budget_keeps_nothing_and_equals_the_plain_cut(tiny):
    tree, O = tiny
    C = oracle.OracleCutCache(O, 0, 0.0, 1e30)
    for cam in _cams() * 2:
        ids, _ = C.select(cam, 1.0)
        assert np.array_equal(ids, O.select(cam, 1.0)[0])
    assert C.hits == 0 and not C.entries


def test_the_same_view_twice_hits_every_visible_spt_and_cuts_the_same(tiny):
    tree, O = tiny
    C = oracle.OracleCutCache(O, 10 ** 9, 1.0, 1.0)
    cam = _cams()[0]
    a, st = C.select(cam, 1.0)
    assert C.hits == 0 and C.loads == st["spt_visible"]
    b, _ = C.select(cam, 1.0)
    assert C.hits == st["spt_visible"] and np.array_equal(a, b)
    assert sum(e[2] for e in C.entries.values()) == int(np.sum(O.spt_of[a] >= 0))


def test_hits_keep_the_cached_cut_and_loads_take_the_new_one(tiny):
    # moving closer by 0.8 (squared ratio 0.64) stays within [0.5, 1.5]: every
    # SPT seen before keeps the first view's cut, every new one gets its own
    tree, O = tiny
    cam1, cam2 = _cams()[0], _cams()[1]
    C = oracle.OracleCutCache(O, 10 ** 9, 0.5, 1.5)
    first, _ = C.select(cam1, 1.0)
    seen = set(C.entries)
    got, _ = C.select(cam2, 1.0)
    own = _by_spt(O, O.select(cam2, 1.0)[0])
    old = _by_spt(O, first)
    g = _by_spt(O, got)
    assert C.hits > 0
    changed = 0
    for r, nodes in g.items():
        if r < 0:
            assert nodes == own.get(r)  # the upper cut is never cached
        elif r in seen:
            assert nodes == old[r]
            changed += nodes != own.get(r)
        else:
            assert nodes == own[r]
    assert changed > 0  # the reuse is visible: some SPTs stay coarser than the new view's cut


def test_a_ratio_outside_the_window_reloads(tiny):
    tree, O = tiny
    # every root lies in [-10, 10]^3: from z = 30 to z = 10 each root's squared
    # distance ratio is at most (200 + 400) / (200 + 1600) = 0.33
    cam1 = _cams()[0]
    cam3 = scenegen.camera_look_at((0.0, 0.0, 10.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 256, 256)
    C = oracle.OracleCutCache(O, 10 ** 9, 0.5, 1.5)
    C.select(cam1, 1.0)
    ids, _ = C.select(cam3, 1.0)
    assert C.hits == 0 and np.array_equal(ids, O.select(cam3, 1.0)[0])


def test_flush_drops_every_entry(tiny):
    tree, O = tiny
    cam = _cams()[0]
    C = oracle.OracleCutCache(O, 10 ** 9, 0.5, 1.5, flush_every=2)
    C.select(cam, 1.0)
    C.select(cam, 1.0)  # iteration 2: flushed first, so all loads
    assert C.hits == 0
    C.select(cam, 1.0)
    assert C.hits > 0


def test_the_budget_holds_and_evicts_the_least_recently_used_first(tiny):
    tree, O = tiny
    rng = np.random.default_rng(3)
    C = oracle.OracleCutCache(O, 6000, 0.6, 1.6)
    for it in range(12):
        pos = np.array([rng.uniform(-12, 12), rng.uniform(-12, 12), rng.uniform(14, 34)])
        cam = scenegen.camera_look_at(pos, (pos[0] * 0.5, pos[1] * 0.5, 0.0), (0.0, 1.0, 0.0), 256, 256)
        before = {r: e[3] for r, e in C.entries.items()}
        C.select(cam, 1.0)
        assert sum(e[2] for e in C.entries.values()) <= 6000
        kept = [e[3] for e in C.entries.values()]
        dropped = [last for r, last in before.items() if r not in C.entries and last < C.t]
        if kept and dropped:  # nothing older survives a dropped entry
            assert max(dropped) <= min(kept)
    assert C.evictions > 0 and C.hits > 0


def test_dist32_is_within_its_rounding_bound_of_the_exact_distance():
    # five FP32 roundings (three products, two sums) and a correctly rounded
    # square root: within a few ulp of the exact distance of the FP32 inputs
    rng = np.random.default_rng(61)
    for _ in range(2000):
        mu = rng.uniform(-2000, 2000, 3).astype(np.float32)
        pos = (mu + rng.normal(0, 10.0 ** rng.uniform(-2, 3), 3)).astype(np.float32)
        d = oracle.dist32(mu, pos)
        exact = float(np.sqrt(np.sum((mu.astype(np.float64) - pos.astype(np.float64)) ** 2)))
        ulp = float(np.spacing(np.float32(exact)))
        assert abs(float(d) - exact) <= 4 * ulp + 1e-30, (d, exact)
