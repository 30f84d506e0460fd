"""Workload recipes: leaf distributions, cameras and request streams.

Seeds: leaves k, cameras 100+k, targets 200+k, requests 300+k for workload k.
"""
from __future__ import annotations

import math

import numpy as np

from . import LeafSpec, camera_look_at, camera_yaw_pitch


def tiny_spec(n: int = 16384, seed: int = 0, sh_degree: int = 3) -> LeafSpec:
    """16,384 leaves, means U[-10,10]^3 (the tiny plain-forward workload)."""
    return LeafSpec(n=n, seed=seed, kind=0, half_extent=10.0, sh_degree=sh_degree)


def tiny_camera(width: int = 512, height: int = 512):
    return camera_look_at((0.0, 0.0, 30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), width, height)


def medium_spec(n: int = 2_000_000, seed: int = 1, sh_degree: int = 3) -> LeafSpec:
    """2M leaves over 500 x 500 m: 60% on z=0 (N(0,0.05) jitter), 40% in 200 cubes of side U(2,20)."""
    return LeafSpec(n=n, seed=seed, kind=1, half_extent=250.0, plane_frac=0.6, plane_sigma=0.05,
                    n_boxes=200, side_lo=2.0, side_hi=20.0, height_lo=-1.0, height_hi=-1.0,
                    sh_degree=sh_degree)


def medium_camera(seed: int = 101, width: int = 1920, height: int = 1080):
    """Altitude U(5,100), xy U[-125,125]^2, yaw U[0,2pi), pitch -45 deg."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    alt = rng.uniform(5.0, 100.0)
    xy = rng.uniform(-125.0, 125.0, size=2)
    yaw = rng.uniform(0.0, 2 * math.pi)
    return camera_yaw_pitch((xy[0], xy[1], alt), yaw, math.radians(-45.0), width, height)


def city_spec(n: int = 50_000_000, seed: int = 2, half_extent: float = 2000.0, n_boxes: int = 20000,
              sh_degree: int = 3) -> LeafSpec:
    """City scene: 60% plane, 40% in boxes with footprint U(2,20) per axis and height U(5,150)."""
    return LeafSpec(n=n, seed=seed, kind=1, half_extent=half_extent, plane_frac=0.6, plane_sigma=0.05,
                    n_boxes=n_boxes, side_lo=2.0, side_hi=20.0, height_lo=5.0, height_hi=150.0,
                    sh_degree=sh_degree)


def city_path_camera(k: int, n_poses: int = 256, width: int = 1920, height: int = 1080):
    """Pose k of the aerial-to-street path: altitude geometric 800 -> 1.8 m, pitch linear
    -60 -> 0 deg, yaw 45 deg, xy linear (-1000,-1000) -> (0,0)."""
    s = k / (n_poses - 1) if n_poses > 1 else 0.0
    alt = 800.0 * (1.8 / 800.0) ** s
    pitch = math.radians(-60.0 + 60.0 * s)
    xy = -1000.0 + 1000.0 * s
    return camera_yaw_pitch((xy, xy, alt), math.radians(45.0), pitch, width, height)


CITY_TAUS = (0.5, 1.0, 2.0)
SERVE_RESOLUTIONS = ((640, 360), (1280, 720), (1920, 1080), (3840, 2160))


def random_pose_camera(rng: np.random.Generator, half_extent: float, width: int, height: int):
    """Altitude log-uniform [1.8, 1000], xy uniform in the extent, yaw U[0,2pi), pitch U(-80,0) deg."""
    alt = math.exp(rng.uniform(math.log(1.8), math.log(1000.0)))
    xy = rng.uniform(-half_extent, half_extent, size=2)
    yaw = rng.uniform(0.0, 2 * math.pi)
    pitch = math.radians(rng.uniform(-80.0, 0.0))
    return camera_yaw_pitch((xy[0], xy[1], alt), yaw, pitch, width, height)
