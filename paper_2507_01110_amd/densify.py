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
Respawns are applied one after another in ascending node id, each on the tree
as the previous ones left it (READING: the paper runs them in parallel with
the edge-case rules above; this order reproduces those rules).
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
    dead_set = set(dead.tolist())
    # chosen leaves, largest statistic first (ties by id), dead ones excluded
    cand = np.flatnonzero(is_leaf & (o >= dead_opacity))
    order = cand[np.lexsort((cand, -np.asarray(max_grad2d, np.float64)[cand]))]
    targets = order.tolist()
    used = 0
    respawned = 0
    moved = set()  # nodes that took their parent's place in this step
    for d in dead.tolist():
        if used >= len(targets):
            break
        p = int(parent[d])
        if p < 0 or left[d] >= 0 or d in moved:
            continue  # the root, no longer a leaf, or moved up by its sibling's respawn (next step)
        s = int(right[p]) if int(left[p]) == d else int(left[p])
        if int(left[p]) == d and s in dead_set and left[s] < 0:
            continue  # both children dead: only the right one is respawned
        t = targets[used]
        used += 1
        g = int(parent[p])  # the sibling takes the parent's place
        moved.add(s)
        parent[s] = g
        if g < 0:
            root = s
        elif int(left[g]) == p:
            left[g] = s
        else:
            right[g] = s
        if t == p:
            raise AssertionError("a chosen leaf cannot be an interior node")
        left[t], right[t] = d, p  # the dead leaf and its parent under the chosen leaf
        parent[d] = parent[p] = t
        left[p] = right[p] = -1
        _set_child_params(a, d, t)
        _set_child_params(a, p, t)
        dead_set.discard(d)
        respawned += 1
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
