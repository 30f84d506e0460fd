"""Seeded synthetic inputs shared by the product path and the oracle.

Holds only input construction: leaf Gaussians, the binary hierarchy over them
(median split + moment-matching merge, the hierarchy the paper takes as given,
Sec. 3 "Gaussian Hierarchies"), the HSPT volume threshold (the per-scene
`size` of Sec. 4.3), cameras and target images.  None of the per-view
arithmetic (LoD test, projection, sort, blend) lives here.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libscenegen.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile libscenegen.so (host C++, OpenMP)."""
    import subprocess

    src = os.path.join(_HERE, "scenegen.cpp")
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           src, "-o", _LIB_PATH + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _LeafParams(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_coef", ctypes.c_int32),
                ("half_extent", ctypes.c_double), ("plane_frac", ctypes.c_double),
                ("plane_sigma", ctypes.c_double), ("n_boxes", ctypes.c_int64),
                ("side_lo", ctypes.c_double), ("side_hi", ctypes.c_double),
                ("height_lo", ctypes.c_double), ("height_hi", ctypes.c_double),
                ("ls_mean", ctypes.c_double), ("ls_sd", ctypes.c_double),
                ("sh_sd", ctypes.c_double), ("op_sd", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.sg_philox.argtypes = [P, P, P]
        L.sg_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32]
        L.sg_uniform.restype = ctypes.c_double
        L.sg_leaves.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(_LeafParams), P, P, P, P, P]
        L.sg_build_hierarchy.argtypes = [ctypes.c_int64, ctypes.c_int32] + [P] * 9
        L.sg_log_volume_kth_largest.argtypes = [ctypes.c_int64, P, ctypes.c_int64]
        L.sg_log_volume_kth_largest.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
@dataclass
class LeafSpec:
    """Leaf distribution (see sg_leaf_params in scenegen.cpp)."""
    n: int
    seed: int
    kind: int = 0               # 0 uniform cube, 1 city (plane + boxes)
    half_extent: float = 10.0
    plane_frac: float = 0.6
    plane_sigma: float = 0.05
    n_boxes: int = 0
    side_lo: float = 2.0
    side_hi: float = 20.0
    height_lo: float = -1.0     # < 0: cubes of one side
    height_hi: float = -1.0
    ls_mean: float = -3.0
    ls_sd: float = 0.5
    sh_sd: float = 0.2
    op_sd: float = 1.0
    sh_degree: int = 3


@dataclass
class Tree:
    """A binary Gaussian hierarchy, arrays indexed by tree node id.

    Leaves are ids [0, n_leaves); internal nodes [n_leaves, 2 n_leaves - 1)
    in preorder.  Parameters are the raw ones: mean, log-scale, quaternion
    (w, x, y, z), opacity logit, SH [coef][rgb].
    """
    n_leaves: int
    sh_degree: int
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    left: np.ndarray
    right: np.ndarray
    parent: np.ndarray
    root: int
    log_volume_threshold: float = 0.0

    @property
    def n_nodes(self) -> int:
        return int(self.means.shape[0])


def make_leaves(spec: LeafSpec, n_alloc: int | None = None):
    n = spec.n
    n_alloc = n if n_alloc is None else n_alloc
    n_coef = 3 * (spec.sh_degree + 1) ** 2
    means = np.empty((n_alloc, 3), np.float32)
    ls = np.empty((n_alloc, 3), np.float32)
    q = np.empty((n_alloc, 4), np.float32)
    op = np.empty((n_alloc,), np.float32)
    sh = np.empty((n_alloc, n_coef // 3, 3), np.float32)
    prm = _LeafParams(spec.kind, n_coef, spec.half_extent, spec.plane_frac, spec.plane_sigma,
                      spec.n_boxes, spec.side_lo, spec.side_hi, spec.height_lo, spec.height_hi,
                      spec.ls_mean, spec.ls_sd, spec.sh_sd, spec.op_sd)
    rc = lib().sg_leaves(n, spec.seed, ctypes.byref(prm), _p(means), _p(ls), _p(q), _p(op), _p(sh))
    if rc != 0:
        raise ValueError("sg_leaves failed")
    return means, ls, q, op, sh


def build_tree(spec: LeafSpec, spt_target: int = 512) -> Tree:
    """Leaves + hierarchy + HSPT volume threshold for about n_nodes/spt_target upper nodes."""
    n = spec.n
    nn = 2 * n - 1
    means, ls, q, op, sh = make_leaves(spec, nn)
    left = np.empty(nn, np.int32)
    right = np.empty(nn, np.int32)
    parent = np.empty(nn, np.int32)
    root = ctypes.c_int32(0)
    rc = lib().sg_build_hierarchy(n, sh.shape[1] * 3, _p(means), _p(ls), _p(q), _p(op), _p(sh),
                                  _p(left), _p(right), _p(parent), ctypes.byref(root))
    if rc != 0:
        raise ValueError("sg_build_hierarchy failed")
    k = max(1, math.ceil(nn / spt_target))
    thr = lib().sg_log_volume_kth_largest(nn, _p(ls), k)
    return Tree(n, spec.sh_degree, means, ls, q, op, sh, left, right, parent, int(root.value), float(thr))


def tree_from_arrays(means, log_scales, quats, opacity_logits, sh, left, right, parent, root,
                     log_volume_threshold, sh_degree) -> Tree:
    """Wrap hand-made arrays (small fixtures) as a Tree."""
    f = lambda a, dt: np.ascontiguousarray(a, dtype=dt)
    n_leaves = int(np.sum(np.asarray(left) < 0))
    return Tree(n_leaves, sh_degree, f(means, np.float32), f(log_scales, np.float32),
                f(quats, np.float32), f(opacity_logits, np.float32), f(sh, np.float32),
                f(left, np.int32), f(right, np.int32), f(parent, np.int32), int(root),
                float(log_volume_threshold))


# ---------------------------------------------------------------------------
@dataclass
class Camera:
    """Pinhole camera, world->camera x_c = R x_w + t, OpenCV axes
    (x right, y down, z forward); pos is the centre in world space."""
    R: np.ndarray
    t: np.ndarray
    pos: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.2


def _camera_from_axes(pos, right, down, fwd, width, height, hfov_deg, z_near) -> Camera:
    R = np.stack([right, down, fwd]).astype(np.float64)
    pos = np.asarray(pos, np.float64)
    t = -R @ pos
    f = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return Camera(R.astype(np.float32), t.astype(np.float32), pos.astype(np.float32),
                  float(np.float32(f)), float(np.float32(f)), float(np.float32(width / 2.0)),
                  float(np.float32(height / 2.0)), int(width), int(height), float(np.float32(z_near)))


def camera_look_at(pos, target, up, width, height, hfov_deg=60.0, z_near=0.2) -> Camera:
    pos = np.asarray(pos, np.float64)
    fwd = np.asarray(target, np.float64) - pos
    fwd /= np.linalg.norm(fwd)
    down = -np.asarray(up, np.float64)
    right = np.cross(down, fwd)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    return _camera_from_axes(pos, right, down, fwd, width, height, hfov_deg, z_near)


def camera_yaw_pitch(pos, yaw, pitch, width, height, hfov_deg=60.0, z_near=0.2) -> Camera:
    """World z is up; yaw about z from +x, pitch from the horizon (negative = down)."""
    cp, sp = math.cos(pitch), math.sin(pitch)
    fwd = np.array([cp * math.cos(yaw), cp * math.sin(yaw), sp])
    right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    down = np.cross(fwd, right)
    return _camera_from_axes(pos, right, down, fwd, width, height, hfov_deg, z_near)


def target_image(height: int, width: int, seed: int) -> np.ndarray:
    """Seeded U[0,1] RGB target, float32 [H][W][3]."""
    return np.random.default_rng(np.random.PCG64(seed)).random((height, width, 3), dtype=np.float32)
