"""Training-loop adjuncts around the per-view path (host side).

* ViewScheduler: the view selection of Sec. 4.4 ("View Selection"): the next
  training view is drawn among the k nearest neighbours of the current one
  (by camera position) with probability proportional to 1 / (w_ij + W), w_ij
  the distance between the two views; every explore_every-th view is drawn
  uniformly from all views instead, against the bias of the local walk.
* lod_noise: the varying level of detail of the implementation appendix: the
  distances to the SPT centres of an iteration are multiplied by 1 + 5 r^4,
  r ~ U(0, 1), so most iterations train near the finest level and some train
  coarser ones.  The factor goes to Frame.set_lod_noise, which applies it to
  the SPT root distances only (the upper hierarchy keeps its own distances).
"""
from __future__ import annotations

import numpy as np


class ViewScheduler:
    def __init__(self, positions, k: int = 8, W: float | None = None, explore_every: int = 128, seed: int = 0):
        pos = np.asarray(positions, np.float64).reshape(-1, 3)
        n = len(pos)
        if n < 2:
            raise ValueError("ViewScheduler needs at least two views")
        self.n, self.k = n, min(int(k), n - 1)
        from scipy.spatial import cKDTree
        d, j = cKDTree(pos).query(pos, self.k + 1)
        d, j = np.atleast_2d(d), np.atleast_2d(j)
        nbr = np.empty((n, self.k), np.int64)
        w = np.empty((n, self.k), np.float64)
        for i in range(n):  # drop the view itself (it may not come first among duplicates)
            keep = np.flatnonzero(j[i] != i)[: self.k]
            nbr[i], w[i] = j[i][keep], d[i][keep]
        self.neighbours, self.weights = nbr, w
        # READING: W is not given; by default the mean neighbour distance, so
        # a neighbour at distance 0 is twice as likely as one at the mean
        self.W = float(w.mean()) if W is None else float(W)
        if not self.W > 0.0 and not np.all(w > 0.0):
            raise ValueError("W must be > 0 when views coincide")
        self.explore_every = int(explore_every)
        self.rng = np.random.default_rng(seed)
        self.current = int(self.rng.integers(n))
        self.iteration = 0

    def transition(self, i: int) -> np.ndarray:
        """P(j | i) over the k neighbours of view i (in self.neighbours[i] order)."""
        p = 1.0 / (self.weights[i] + self.W)
        return p / p.sum()

    def next(self) -> int:
        self.iteration += 1
        if self.explore_every > 0 and self.iteration % self.explore_every == 0:
            self.current = int(self.rng.integers(self.n))
        else:
            c = self.current
            self.current = int(self.neighbours[c][self.rng.choice(self.k, p=self.transition(c))])
        return self.current


def lod_noise(rng: np.random.Generator) -> float:
    """1 + 5 r^4 with r ~ U(0, 1): the factor on an iteration's cut distances."""
    r = rng.random()
    return 1.0 + 5.0 * r ** 4
