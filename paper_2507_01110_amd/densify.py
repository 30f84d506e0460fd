"""Densification on the hierarchy (Sec. 4.2 and the appendix on densification
details), host side, between training iterations.

* Selection: leaves are chosen by their largest screen-space mean gradient
  over views (the statistic that lodgs_frame_set_densify_stats accumulates).
* Spawn: a chosen leaf gets two new children that together look like it: both
  sit at its mean with its rotation and colour, with opacity
  o' = 1 - sqrt(1 - o) (two co-located copies composite to o at the centre)
  and standard deviations scaled by sqrt(o / (2 o' - o'^2 / 2)), which keeps
  the integral of the composited 2D alpha equal to the parent's.  READING: the
  paper takes its split from 3DGS-MCMC without the formula; this one is
  derived here from those two conditions.
* Respawn: a dead leaf (opacity below a threshold) leaves its place: its
  sibling, leaf or subtree, takes the parent's place; the dead leaf and its
  former parent become the two children of a chosen leaf, with the spawn
  parameters.  When both children of a node are dead leaves only the right
  one is respawned (the left one takes the parent's place and is respawned
  at the next step; so is any dead leaf moved up this way).  The node count is unchanged.
* The HSPT layout is rebuilt by constructing a new Scene from the result.
* Respawns run in parallel (vectorised over all dead leaves at once, every
  edit decided on the tree as it was): besides the rule for two dead
  siblings, a dead leaf whose parent is the sibling of another dead leaf
  respawned in the same step waits for the next step (READING: the paper
  names the sibling rule only; applied together, these two edits would both
  rewrite the same link, the removed parent's).
* Pruning: the opacity of a leaf that has not contributed to a pixel for 2 x
  the training-set size iterations is zeroed (logit -30), so the next step
  respawns it (READING: the paper says Gaussians; only leaves can be
  respawned, so interior nodes are left alone).  The last iteration each node
  contributed comes from lodgs_frame_set_contrib_stats.
"""
from __future__ import annotations

import math

import numpy as np

import scenegen


def split_params(opacity_logit: float, log_scales: np.ndarray):
    """(child opacity logit, child log-scales) of a spawn from the parent's."""
    o = 1.0 / (1.0 + math.exp(-float(opacity_logit)))
    oc = 1.0 - math.sqrt(max(0.0, 1.0 - o))
    oc = min(max(oc, 1e-7), 1.0 - 1e-7)
    f = math.sqrt(o / (2.0 * oc - 0.5 * oc * oc))
    return math.log(oc / (1.0 - oc)), np.asarray(log_scales, np.float64) + math.log(f)


def split_params_many(opacity_logits: np.ndarray, log_scales: np.ndarray):
    """split_params over arrays of parents (same formulas, elementwise)."""
    o = 1.0 / (1.0 + np.exp(-np.asarray(opacity_logits, np.float64)))
    oc = np.clip(1.0 - np.sqrt(np.maximum(0.0, 1.0 - o)), 1e-7, 1.0 - 1e-7)
    f = np.sqrt(o / (2.0 * oc - 0.5 * oc * oc))
    return np.log(oc / (1.0 - oc)), np.asarray(log_scales, np.float64) + np.log(f)[:, None]


def _arrays(tree):
    return {k: np.array(getattr(tree, k)) for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "left",
                                                    "right", "parent")}


def _finish(a, root, sh_degree):
    nn = a["means"].shape[0]
    ls = np.ascontiguousarray(a["log_scales"], np.float32)
    thr = scenegen.lib().sg_log_volume_kth_largest(nn, scenegen._p(ls), max(1, math.ceil(nn / 512)))
    return scenegen.tree_from_arrays(a["means"], ls, a["quats"], a["opacity_logits"], a["sh"], a["left"],
                                     a["right"], a["parent"], int(root), float(thr), sh_degree)


def _set_child_params(a, c, t):
    lo, ls = split_params(a["opacity_logits"][t], a["log_scales"][t])
    for k in ("means", "quats", "sh"):
        a[k][c] = a[k][t]
    a["log_scales"][c] = ls
    a["opacity_logits"][c] = lo


PRUNED_LOGIT = -30.0


def prune(tree, last_contrib: np.ndarray, iteration: int, train_views: int):
    """Zeroes the opacity (logit PRUNED_LOGIT) of every leaf with iteration -
    last_contrib[id] >= 2 * train_views (last_contrib by tree id: the last
    iteration the node contributed to a pixel).  Returns the number pruned;
    edits tree.opacity_logits in place."""
    last = np.asarray(last_contrib, np.int64)
    idle = (int(iteration) - last >= 2 * int(train_views)) & (np.asarray(tree.left) < 0)
    idle &= np.asarray(tree.opacity_logits) > PRUNED_LOGIT
    tree.opacity_logits[idle] = PRUNED_LOGIT
    return int(idle.sum())


def respawn_plan(left, right, parent, dead):
    """The dead leaves respawned this step (ascending id) under the parallel
    rules: not the root; of two dead sibling leaves only the right one; not a
    leaf whose parent is the sibling of another dead leaf of the step."""
    left, right, parent = np.asarray(left), np.asarray(right), np.asarray(parent)
    d = np.asarray(dead, np.int64)
    p = parent[d]
    d = d[p >= 0]
    p = parent[d]
    s = np.where(left[p] == d, right[p], left[p])
    is_dead = np.zeros(len(left), bool)
    is_dead[d] = True
    both = (left[p] == d) & is_dead[s] & (left[s] < 0)  # left one of two dead sibling leaves
    d, p, s = d[~both], p[~both], s[~both]
    chained = np.isin(p, s)  # its parent is the sibling of another one respawned now
    return np.sort(d[~chained])


def densify(tree, max_grad2d: np.ndarray, n_spawn: int, dead_opacity: float = 0.005):
    """One densification step.  max_grad2d: the statistic by tree id.  Dead
    leaves are respawned under the leaves with the largest statistic; then
    n_spawn more of those leaves (the next ones) get two new children.
    Returns (new tree, {"respawned": r, "spawned": s})."""
    a = _arrays(tree)
    left, right, parent = a["left"], a["right"], a["parent"]
    root = int(tree.root)
    o = 1.0 / (1.0 + np.exp(-a["opacity_logits"].astype(np.float64)))
    is_leaf = left < 0
    dead = np.flatnonzero(is_leaf & (o < dead_opacity))
    # chosen leaves, largest statistic first (ties by id), dead ones excluded
    cand = np.flatnonzero(is_leaf & (o >= dead_opacity))
    order = cand[np.lexsort((cand, -np.asarray(max_grad2d, np.float64)[cand]))]
    targets = order.tolist()
    # every respawn of the step decided on the tree as it is, then applied at once
    d = respawn_plan(left, right, parent, dead)[: len(targets)]
    t = np.asarray(targets[: len(d)], np.int64)
    p = parent[d]
    s = np.where(left[p] == d, right[p], left[p])
    g = parent[p]
    if np.any(np.isin(t, p)):
        raise AssertionError("a chosen leaf cannot be an interior node")
    # the sibling takes the parent's place
    parent[s] = g
    top = g < 0
    if top.any():
        root = int(s[top][0])
    gl = ~top & (left[np.maximum(g, 0)] == p)
    gr = ~top & ~gl
    left[g[gl]] = s[gl]
    right[g[gr]] = s[gr]
    # the dead leaf and its former parent become the chosen leaf's children
    left[t], right[t] = d, p
    parent[d] = t
    parent[p] = t
    left[p] = -1
    right[p] = -1
    lo, ls = split_params_many(a["opacity_logits"][t], a["log_scales"][t])
    for c in (d, p):
        for k in ("means", "quats", "sh"):
            a[k][c] = a[k][t]
        a["log_scales"][c] = ls
        a["opacity_logits"][c] = lo
    respawned = int(len(d))
    used = respawned
    spawn = targets[used:used + max(0, int(n_spawn))]
    if spawn:
        n0 = a["means"].shape[0]
        grow = 2 * len(spawn)
        for k in list(a):
            pad = np.zeros((grow,) + a[k].shape[1:], a[k].dtype)
            if k in ("left", "right", "parent"):
                pad[:] = -1
            a[k] = np.concatenate([a[k], pad])
        left, right, parent = a["left"], a["right"], a["parent"]
        for j, t in enumerate(spawn):
            c0, c1 = n0 + 2 * j, n0 + 2 * j + 1
            left[t], right[t] = c0, c1
            parent[c0] = parent[c1] = t
            _set_child_params(a, c0, t)
            _set_child_params(a, c1, t)
    return _finish(a, root, tree.sh_degree), {"respawned": respawned, "spawned": len(spawn)}
