"""Host-side training adjuncts: the kNN view walk of Sec. 4.4 and the LoD
noise factor of the implementation appendix, checked against their
definitions by brute force and by sampling."""
import numpy as np

from paper_2507_01110_amd.training import ViewScheduler, lod_noise


def test_neighbours_are_the_k_nearest_other_views():
    rng = np.random.default_rng(91)
    pos = rng.uniform(-50, 50, (200, 3))
    S = ViewScheduler(pos, k=6, seed=1)
    d = np.linalg.norm(pos[:, None] - pos[None], axis=2)
    np.fill_diagonal(d, np.inf)
    for i in range(len(pos)):
        want = np.argsort(d[i])[:6]
        assert sorted(S.neighbours[i].tolist()) == sorted(want.tolist())
        np.testing.assert_allclose(np.sort(S.weights[i]), np.sort(d[i][want]), rtol=1e-12)


def test_duplicate_positions_never_list_the_view_itself():
    pos = np.repeat(np.arange(10.0)[:, None], 3, axis=1).repeat(2, axis=0)  # every position twice
    S = ViewScheduler(pos, k=3, W=1.0)
    for i in range(len(pos)):
        assert i not in S.neighbours[i].tolist()


def test_steps_follow_inverse_distance_weights():
    rng = np.random.default_rng(92)
    pos = rng.uniform(-10, 10, (40, 3))
    S = ViewScheduler(pos, k=5, W=2.0, explore_every=0, seed=3)
    i = 7
    counts = np.zeros(5)
    trials = 40000
    for _ in range(trials):
        S.current = i
        counts[S.neighbours[i].tolist().index(S.next())] += 1
    p = 1.0 / (S.weights[i] + 2.0)
    p /= p.sum()
    sd = np.sqrt(trials * p * (1 - p))
    assert np.all(np.abs(counts - trials * p) < 5 * sd), (counts, trials * p)


def test_every_explore_step_is_uniform_over_all_views():
    pos = np.stack([np.arange(64.0), np.zeros(64), np.zeros(64)], 1)  # a line: neighbours stay local
    S = ViewScheduler(pos, k=2, explore_every=4, seed=5)
    hits = np.zeros(64)
    for t in range(1, 4 * 16000 + 1):
        v = S.next()
        if t % 4 == 0:
            hits[v] += 1
    e = 16000 / 64
    assert np.all(np.abs(hits - e) < 5 * np.sqrt(e)), hits


def test_lod_noise_is_one_plus_five_r_to_the_fourth():
    rng = np.random.default_rng(93)
    f = np.array([lod_noise(rng) for _ in range(50000)])
    assert f.min() >= 1.0 and f.max() <= 6.0
    for t in (0.1, 0.5, 0.8, 0.95):  # P(f <= 1 + 5 t^4) = t
        frac = np.mean(f <= 1.0 + 5.0 * t ** 4)
        assert abs(frac - t) < 5 * np.sqrt(t * (1 - t) / len(f)), (t, frac)
