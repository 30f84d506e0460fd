"""Test helpers: small hand-made hierarchies and plain-Python reference cuts.

The reference cuts here are written from the paper's statements directly
(Alg. 1's queue-based BFS, Sec. 4.3's two-step HSPT cut) in float64, to pin
the oracle's traversal structure; they do not reproduce its FP32 mirror.
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np

import scenegen


def random_tree(rng: np.random.Generator, n_leaves: int, sh_degree: int = 1, extent: float = 10.0,
                log_threshold: float | None = None):
    """Random topology (repeated merges of two random roots) with independent
    random parameters per node, so the heap condition is often violated."""
    n = 2 * n_leaves - 1
    left = -np.ones(n, np.int32)
    right = -np.ones(n, np.int32)
    parent = -np.ones(n, np.int32)
    roots = list(range(n_leaves))
    nxt = n_leaves
    while len(roots) > 1:
        a, b = rng.choice(len(roots), 2, replace=False)
        ra, rb = roots[a], roots[b]
        for k in sorted((a, b), reverse=True):
            roots.pop(k)
        left[nxt], right[nxt] = ra, rb
        parent[ra] = parent[rb] = nxt
        roots.append(nxt)
        nxt += 1
    root = roots[0]
    means = rng.uniform(-extent, extent, (n, 3))
    ls = rng.normal(-1.0, 1.0, (n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = rng.normal(size=n)
    nb = (sh_degree + 1) ** 2
    sh = rng.normal(0, 0.2, (n, nb, 3))
    if log_threshold is None:
        lv = ls.astype(np.float32).astype(np.float64).sum(axis=1)
        log_threshold = float(np.quantile(lv, rng.uniform(0.0, 1.0)))
    return scenegen.tree_from_arrays(means, ls, q, op, sh, left, right, parent, root, log_threshold, sh_degree)


def caterpillar_tree(rng: np.random.Generator, n_leaves: int, sh_degree: int = 1, extent: float = 10.0):
    """Each internal node joins the previous root with a new leaf: depth
    n_leaves - 1.  With a very low volume threshold every internal node is in
    the upper hierarchy, which is then a chain of n_leaves - 1 nodes."""
    n = 2 * n_leaves - 1
    left = -np.ones(n, np.int32)
    right = -np.ones(n, np.int32)
    parent = -np.ones(n, np.int32)
    root = 0
    for k in range(1, n_leaves):
        nxt = n_leaves + k - 1
        left[nxt], right[nxt] = root, k
        parent[root] = parent[k] = nxt
        root = nxt
    means = rng.uniform(-extent, extent, (n, 3))
    ls = rng.normal(-1.0, 1.0, (n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = rng.normal(size=n)
    nb = (sh_degree + 1) ** 2
    sh = rng.normal(0, 0.2, (n, nb, 3))
    return scenegen.tree_from_arrays(means, ls, q, op, sh, left, right, parent, root, -1e30, sh_degree)


def g64(tree) -> np.ndarray:
    s = np.exp(tree.log_scales.astype(np.float64))
    return np.sqrt(s[:, 0] * s[:, 1] + s[:, 0] * s[:, 2] + s[:, 1] * s[:, 2])


def rho64(tree) -> np.ndarray:
    return 3.0 * np.exp(tree.log_scales.astype(np.float64)).max(axis=1)


def culled64(cam, mu, rho) -> bool:
    """Sphere entirely outside one of the four side planes or the near plane."""
    c = cam.R.astype(np.float64) @ np.asarray(mu, np.float64) + cam.t.astype(np.float64)
    if c[2] + rho < cam.z_near:
        return True
    hl, hr = cam.cx / cam.fx, (cam.width - cam.cx) / cam.fx
    ht, hb = cam.cy / cam.fy, (cam.height - cam.cy) / cam.fy
    return (c[0] - hr * c[2] > rho * math.sqrt(1 + hr * hr) or -c[0] - hl * c[2] > rho * math.sqrt(1 + hl * hl)
            or c[1] - hb * c[2] > rho * math.sqrt(1 + hb * hb) or -c[1] - ht * c[2] > rho * math.sqrt(1 + ht * ht))


def hspt_roles(tree):
    """BFS split on log-volume < threshold; returns role (0 upper, 1 SPT root, 2 member)."""
    lv = tree.log_scales.astype(np.float64).sum(axis=1)
    role = -np.ones(tree.n_nodes, np.int8)
    q = deque([tree.root])
    while q:
        u = q.popleft()
        if tree.left[u] < 0 or lv[u] < tree.log_volume_threshold:
            role[u] = 1
            st = [u]
            while st:
                v = st.pop()
                if v != u:
                    role[v] = 2
                if tree.left[v] >= 0:
                    st += [tree.left[v], tree.right[v]]
        else:
            role[u] = 0
            q += [tree.left[u], tree.right[u]]
    return role


def bfs_cut(tree, condition):
    """Alg. 1: a queue from the root; a node meeting the condition joins the cut
    and its children are skipped, otherwise both children are enqueued."""
    cut = []
    q = deque([tree.root])
    while q:
        u = q.popleft()
        if condition(u):
            cut.append(u)
        else:
            q.append(tree.left[u])
            q.append(tree.right[u])
    return cut


def hspt_cut_reference(tree, cam, tau: float, cull: bool, spt_scale: float = 1.0):
    """Sec. 4.3 two-step cut in float64: BFS on the upper hierarchy (cull, or
    fine enough at the node's own distance), then each reached SPT cut at the
    distance of its root (descend to the first node with g <= X; leaves always),
    that distance multiplied by spt_scale (the LoD noise of the implementation
    appendix, which scales the distances to the SPT centres only)."""
    role = hspt_roles(tree)
    g = g64(tree)
    rho = rho64(tree)
    pos = cam.pos.astype(np.float64)
    k = tau / cam.fx
    out = []
    q = deque([tree.root])
    while q:
        u = q.popleft()
        if cull and culled64(cam, tree.means[u], rho[u]):
            continue
        X = np.linalg.norm(tree.means[u].astype(np.float64) - pos) * k
        if role[u] != 0:
            X *= spt_scale
        if role[u] == 0:
            if g[u] <= X:
                out.append(u)
            else:
                q += [tree.left[u], tree.right[u]]
            continue
        st = [u]
        while st:
            v = st.pop()
            if tree.left[v] < 0 or g[v] <= X:
                out.append(v)
            else:
                st += [tree.left[v], tree.right[v]]
    return sorted(out)


def ancestors(tree, v):
    a = []
    p = tree.parent[v]
    while p >= 0:
        a.append(int(p))
        p = tree.parent[p]
    return a


def leaves_under(tree, v):
    st, out = [v], []
    while st:
        u = st.pop()
        if tree.left[u] < 0:
            out.append(u)
        else:
            st += [tree.left[u], tree.right[u]]
    return out


def single_splat_tree(params, sh_degree=0):
    """A Tree whose nodes are independent splats (no topology), for render pins.
    params: list of dicts with mean, log_scale, quat, logit, rgb (DC colour)."""
    n = len(params)
    nb = (sh_degree + 1) ** 2
    means = np.array([p["mean"] for p in params], np.float64)
    ls = np.array([p["log_scale"] for p in params], np.float64)
    q = np.array([p.get("quat", (1.0, 0.0, 0.0, 0.0)) for p in params], np.float64)
    op = np.array([p["logit"] for p in params], np.float64)
    sh = np.zeros((n, nb, 3))
    C0 = 0.28209479177387814
    for i, p in enumerate(params):
        sh[i, 0] = (np.asarray(p["rgb"], np.float64) - 0.5) / C0
        if "sh" in p:
            sh[i, 1:] = p["sh"]
    neg = -np.ones(n, np.int32)
    return scenegen.tree_from_arrays(means, ls, q, op, sh, neg, neg, neg, 0, 0.0, sh_degree)
