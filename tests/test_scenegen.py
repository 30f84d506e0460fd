"""The seeded input generator: Philox known answers, hierarchy shape and the
moment-matching merge of the hierarchy the paper takes as input (Sec. 3)."""
import ctypes

import numpy as np

import scenegen
from scenegen import configs


def test_philox_known_answers():
    L = scenegen.lib()
    out = (ctypes.c_uint32 * 4)()
    for ctr, key, expect in [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
                             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD))]:
        L.sg_philox((ctypes.c_uint32 * 4)(*ctr), (ctypes.c_uint32 * 2)(*key), out)
        assert tuple(out) == expect


def _quat_rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_hierarchy_is_binary_median_split_with_moment_matched_parents():
    t = scenegen.build_tree(configs.tiny_spec(n=1000, seed=5))
    n = t.n_leaves
    assert t.n_nodes == 2 * n - 1 and t.root == n and t.parent[t.root] == -1
    assert np.all(t.left[:n] < 0) and np.all(t.left[n:] >= 0)
    kids = np.concatenate([t.left[n:], t.right[n:]])
    assert np.array_equal(np.sort(kids), np.delete(np.arange(2 * n - 1), n))
    f64 = lambda a: a.astype(np.float64)
    for p in range(n, 2 * n - 1, 37):
        a, b = t.left[p], t.right[p]
        ws, mus, covs, ops = [], [], [], []
        for c in (a, b):
            s = np.exp(f64(t.log_scales[c]))
            R = _quat_rot(f64(t.quats[c]))
            o = 1 / (1 + np.exp(-f64(t.opacity_logits[c])))
            ws.append(o * s.prod())
            mus.append(f64(t.means[c]))
            covs.append(R @ np.diag(s * s) @ R.T)
            ops.append(o)
        W = sum(ws)
        mu = (ws[0] * mus[0] + ws[1] * mus[1]) / W
        cov = sum(w * (C + np.outer(m - mu, m - mu)) for w, C, m in zip(ws, covs, mus)) / W
        np.testing.assert_allclose(f64(t.means[p]), mu, rtol=1e-6, atol=1e-6)
        s = np.exp(f64(t.log_scales[p]))
        R = _quat_rot(f64(t.quats[p]))
        np.testing.assert_allclose(R @ np.diag(s * s) @ R.T, cov, rtol=1e-5, atol=1e-6 * np.abs(cov).max())
        assert s[0] >= s[1] >= s[2] and t.quats[p][0] >= 0
        o = 1 / (1 + np.exp(-f64(t.opacity_logits[p])))
        assert abs(o - (ws[0] * ops[0] + ws[1] * ops[1]) / W) < 1e-6
        np.testing.assert_allclose(f64(t.sh[p]), (ws[0] * f64(t.sh[a]) + ws[1] * f64(t.sh[b])) / W, atol=1e-6)


def test_median_split_halves():
    t = scenegen.build_tree(configs.tiny_spec(n=777, seed=6))

    def leaves(v):
        st, k = [v], 0
        while st:
            u = st.pop()
            if t.left[u] < 0:
                k += 1
            else:
                st += [t.left[u], t.right[u]]
        return k
    for p in range(t.n_leaves, t.n_nodes, 13):
        nl, nr = leaves(t.left[p]), leaves(t.right[p])
        assert nl == (nl + nr) // 2


def test_generation_is_deterministic_and_follows_the_city_recipe():
    spec = configs.medium_spec(n=20000, seed=9)
    a = scenegen.make_leaves(spec)
    b = scenegen.make_leaves(spec)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    means = a[0]
    plane = np.abs(means[:, 2]) < 0.3
    assert abs(plane[:12000].mean() - 1.0) < 1e-3 and means[12000:, 2].min() >= 0
    assert np.abs(means[:, :2]).max() < 260
    np.testing.assert_allclose(np.linalg.norm(a[2], axis=1), 1.0, atol=1e-6)
    assert abs(a[1].mean() + 3.0) < 0.02 and abs(a[1].std() - 0.5) < 0.02
