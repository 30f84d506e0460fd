"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the C oracle (oracle.c).

Plain, slow CPU reference of the LoD-select + splat path (FP64 values, FP32
decision mirror).  Only tests/, the smoke check and the benchmark's CPU
baseline import this package; the product library never does, and the two
share no code.  Inputs come from `scenegen` only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CULL = 1
CONSERVATIVE = 2


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", src, "-o", _LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class OrcCamera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("pos", ctypes.c_float * 3),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("ppx", ctypes.c_float),
                ("ppy", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("z_near", ctypes.c_float)]


class SelectStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("upper_tested", "upper_selected", "spt_visible", "spt_culled",
                                              "spt_nodes_tested", "spt_selected", "ties_exact", "ties_1ulp")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class FrameInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_inst", ctypes.c_int64), ("n_visible", ctypes.c_int64),
                ("n_contrib", ctypes.c_int64), ("TX", ctypes.c_int32), ("TY", ctypes.c_int32),
                ("skip_1ulp", ctypes.c_int64), ("stop_1ulp", ctypes.c_int64), ("skip_flip64", ctypes.c_int64),
                ("stop_flip64", ctypes.c_int64), ("clamp_flip64", ctypes.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, f32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_float
        L.orc_pexp.argtypes = [f32]
        L.orc_pexp.restype = f32
        L.orc_metrics.argtypes = [i64, P, P, P, P]
        L.orc_hspt.argtypes = [i64, P, P, i32, P, ctypes.c_double, P, P, P, P, P]
        L.orc_hspt.restype = ctypes.c_int
        L.orc_layout.argtypes = [i64, P, P, i32, P, P, P, P, P, P, P, P, P]
        L.orc_layout.restype = ctypes.c_int
        L.orc_select.argtypes = [i64, P, P, i32, P, P, P, P, P, P, P, P, ctypes.POINTER(OrcCamera), f32, f32,
                                 ctypes.c_uint32, ctypes.c_int, P, i64, P, ctypes.POINTER(SelectStats), P, P]
        L.orc_select.restype = ctypes.c_int
        for name in ("orc_select_bfs", "orc_select_parallel"):
            fn = getattr(L, name)
            fn.argtypes = [i64, P, P, i32, P, P, P, P, ctypes.POINTER(OrcCamera), f32, ctypes.c_uint32, P, i64, P]
            fn.restype = ctypes.c_int
        L.orc_sh_basis.argtypes = [P, P, P]
        L.orc_render.argtypes = [i64, P, P, P, P, P, P, ctypes.c_int, ctypes.POINTER(OrcCamera), P, P]
        L.orc_render.restype = ctypes.c_void_p
        L.orc_frame_free.argtypes = [P]
        L.orc_eval_frozen.argtypes = [P, P, P]
        L.orc_backward.argtypes = [P, P, P, P]
        L.orc_backward.restype = ctypes.c_int
        L.orc_frame_get_info.argtypes = [P, ctypes.POINTER(FrameInfo)]
        L.orc_frame_get_splats.argtypes = [P, P, P, P, P]
        L.orc_frame_get_instances.argtypes = [P, P, P]
        L.orc_frame_get_pixel_counts.argtypes = [P, P]
        L.orc_frame_get_splat_contrib.argtypes = [P, P]
        L.orc_frame_get_values64.argtypes = [P, P]
        L.orc_project64_one.argtypes = [P, ctypes.c_int, ctypes.POINTER(OrcCamera), P]
        L.orc_fd_directional.argtypes = [P, P, i64, P, ctypes.c_double, P]
        L.orc_fd_directional.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert isinstance(a, np.ndarray) and a.flags["C_CONTIGUOUS"], "need a C-contiguous ndarray"
    return a.ctypes.data_as(ctypes.c_void_p)


def camera(cam) -> OrcCamera:
    c = OrcCamera()
    c.R[:] = [float(v) for v in np.asarray(cam.R, np.float32).reshape(9)]
    c.t[:] = [float(v) for v in np.asarray(cam.t, np.float32).reshape(3)]
    c.pos[:] = [float(v) for v in np.asarray(cam.pos, np.float32).reshape(3)]
    c.fx, c.fy, c.ppx, c.ppy = cam.fx, cam.fy, cam.cx, cam.cy
    c.width, c.height, c.z_near = cam.width, cam.height, cam.z_near
    return c


def pexp(x) -> np.ndarray:
    """FP32 portable exp (the decision path's exp), elementwise."""
    x = np.asarray(x, np.float32)
    f = lib().orc_pexp
    return np.array([f(float(v)) for v in x.reshape(-1)], np.float32).reshape(x.shape)


def sh_basis(d, with_grad: bool = False):
    d = np.ascontiguousarray(d, np.float64)
    Y = np.zeros(16)
    dY = np.zeros(48) if with_grad else None
    lib().orc_sh_basis(_p(d), _p(Y), _p(dY))
    return (Y, dY.reshape(16, 3)) if with_grad else Y


def project64_one(params: np.ndarray, n_coef: int, cam) -> np.ndarray:
    """[mx, my, A, B, C, conic a, b, c, opacity, r, g, b, depth] of one splat."""
    P = np.ascontiguousarray(params, np.float64)
    out = np.zeros(13)
    c = camera(cam)
    lib().orc_project64_one(_p(P), n_coef, ctypes.byref(c), _p(out))
    return out


class OracleScene:
    """Oracle view of a hierarchy: size metrics, HSPT split, SPT intervals and layout."""

    def __init__(self, tree):
        L = lib()
        self.tree = tree
        n = tree.n_nodes
        self.g = np.zeros(n, np.float32)
        self.rho = np.zeros(n, np.float32)
        self.lv = np.zeros(n, np.float64)
        L.orc_metrics(n, _p(tree.log_scales), _p(self.g), _p(self.rho), _p(self.lv))
        self.role = np.zeros(n, np.int8)
        self.spt_of = np.zeros(n, np.int32)
        self.r_min = np.zeros(n, np.float32)
        self.r_max = np.zeros(n, np.float32)
        rc = L.orc_hspt(n, _p(tree.left), _p(tree.right), tree.root, _p(self.lv), tree.log_volume_threshold,
                        _p(self.g), _p(self.role), _p(self.spt_of), _p(self.r_min), _p(self.r_max))
        if rc != 0:
            raise MemoryError("orc_hspt")
        self.pos_of = np.zeros(n, np.int32)
        self.perm = np.zeros(n, np.int32)
        self.spt_begin = np.zeros(n + 1, np.int32)
        nu, ns = ctypes.c_int32(0), ctypes.c_int32(0)
        rc = L.orc_layout(n, _p(tree.left), _p(tree.right), tree.root, _p(self.role), _p(self.spt_of),
                          _p(self.r_min), _p(self.r_max), _p(self.pos_of), _p(self.perm),
                          ctypes.byref(nu), ctypes.byref(ns), _p(self.spt_begin))
        if rc != 0:
            raise RuntimeError(f"orc_layout failed ({rc})")
        self.n_upper, self.n_spt = nu.value, ns.value
        self.spt_begin = self.spt_begin[: self.n_spt + 1].copy()

    def select(self, cam, tau: float, cull: bool = True, mode: int = 0, conservative: bool = False,
               spt_X: np.ndarray | None = None, spt_visible: np.ndarray | None = None, spt_scale: float = 1.0):
        """Tree ids of the cut, in layout order, and the decision statistics.
        spt_X (float32 [n_nodes], NaN = own): X of the SPT rooted at each tree id;
        spt_visible (uint8 [n_nodes]): receives 1 at the visible SPT roots;
        spt_scale: the LoD noise factor on the distances to the SPT roots."""
        t = self.tree
        n = t.n_nodes
        out = np.zeros(n, np.int32)
        cnt = ctypes.c_int64(0)
        st = SelectStats()
        c = camera(cam)
        rc = lib().orc_select(n, _p(t.left), _p(t.right), t.root, _p(t.means), _p(self.g), _p(self.rho),
                              _p(self.role), _p(self.spt_of), _p(self.r_min), _p(self.r_max), _p(self.pos_of),
                              ctypes.byref(c), float(np.float32(tau)), float(np.float32(spt_scale)),
                              (CULL if cull else 0) | (CONSERVATIVE if conservative else 0), mode, _p(out), n,
                              ctypes.byref(cnt), ctypes.byref(st),
                              None if spt_X is None else _p(spt_X), None if spt_visible is None else _p(spt_visible))
        if rc != 0:
            raise RuntimeError(f"orc_select failed ({rc})")
        return out[: cnt.value].copy(), st.as_dict()


    def select_full(self, cam, tau: float, method: str, cull: bool = True):
        """Tree ids of a whole-hierarchy comparator cut ("bfs" or "parallel"), in layout order."""
        fn = {"bfs": lib().orc_select_bfs, "parallel": lib().orc_select_parallel}[method]
        t = self.tree
        n = t.n_nodes
        out = np.zeros(n, np.int32)
        cnt = ctypes.c_int64(0)
        c = camera(cam)
        rc = fn(n, _p(t.left), _p(t.right), t.root, _p(t.means), _p(self.g), _p(self.rho), _p(self.pos_of),
                ctypes.byref(c), float(np.float32(tau)), CULL if cull else 0, _p(out), n, ctypes.byref(cnt))
        if rc != 0:
            raise RuntimeError(f"orc_select_{method} failed ({rc})")
        return out[: cnt.value].copy()


class OracleFrame:
    """One rendered view: FP32 decisions + FP64 image; backward and frozen re-evaluation."""

    def __init__(self, tree, ids: np.ndarray, cam, bg=(0.0, 0.0, 0.0)):
        self.tree = tree
        self.ids = np.ascontiguousarray(ids, np.int32)
        self.cam = cam
        self.n_coef = int(tree.sh.shape[1] * tree.sh.shape[2]) if tree.sh.ndim == 3 else int(tree.sh.shape[1])
        self.image = np.zeros((cam.height, cam.width, 3), np.float64)
        bgv = np.asarray(bg, np.float32)
        c = camera(cam)
        h = lib().orc_render(len(self.ids), _p(self.ids), _p(tree.means), _p(tree.log_scales), _p(tree.quats),
                             _p(tree.opacity_logits), _p(np.ascontiguousarray(tree.sh)), self.n_coef,
                             ctypes.byref(c), _p(bgv), _p(self.image))
        if not h:
            raise MemoryError("orc_render")
        self._h = ctypes.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_frame_free(h)
            self._h = None

    def info(self) -> dict:
        I = FrameInfo()
        lib().orc_frame_get_info(self._h, ctypes.byref(I))
        return {n: int(getattr(I, n)) for n, _ in I._fields_}

    def splats(self):
        n = len(self.ids)
        depth = np.zeros(n, np.uint32)
        tiles = np.zeros(n, np.int32)
        rect = np.zeros((n, 4), np.int32)
        f10 = np.zeros((n, 10), np.float32)
        lib().orc_frame_get_splats(self._h, _p(depth), _p(tiles), _p(rect), _p(f10))
        return {"depth_bits": depth, "tiles": tiles, "rect": rect, "f32": f10}

    def instances(self):
        ni = self.info()["n_inst"]
        tile = np.zeros(ni, np.int32)
        pos = np.zeros(ni, np.int32)
        lib().orc_frame_get_instances(self._h, _p(tile), _p(pos))
        return tile, pos

    def pixel_counts(self) -> np.ndarray:
        c = np.zeros((self.cam.height, self.cam.width), np.int32)
        lib().orc_frame_get_pixel_counts(self._h, _p(c))
        return c

    def splat_contrib(self) -> np.ndarray:
        """Pixels each selected splat is composited into (selection order)."""
        c = np.zeros(len(self.ids), np.int32)
        lib().orc_frame_get_splat_contrib(self._h, _p(c))
        return c

    def values64(self) -> np.ndarray:
        out = np.zeros((len(self.ids), 9))
        lib().orc_frame_get_values64(self._h, _p(out))
        return out

    def params64(self) -> np.ndarray:
        t = self.tree
        i = self.ids
        return np.ascontiguousarray(np.concatenate([
            t.means[i].astype(np.float64), t.log_scales[i].astype(np.float64), t.quats[i].astype(np.float64),
            t.opacity_logits[i, None].astype(np.float64), t.sh[i].reshape(len(i), -1).astype(np.float64)], axis=1))

    def eval_frozen(self, P: np.ndarray) -> np.ndarray:
        img = np.zeros_like(self.image)
        lib().orc_eval_frozen(self._h, _p(np.ascontiguousarray(P, np.float64)), _p(img))
        return img

    def fd_directional(self, W: np.ndarray, i: int, v: np.ndarray, h: float) -> float:
        """Central difference along v of sum(W * image) for the parameters of
        selected splat i (decisions frozen, FP64), recompositing only the
        pixels that splat contributes to."""
        out = ctypes.c_double(0.0)
        self._W = np.ascontiguousarray(W, np.float64)
        rc = lib().orc_fd_directional(self._h, _p(self._W), int(i), _p(np.ascontiguousarray(v, np.float64)),
                                      float(h), ctypes.byref(out))
        if rc != 0:
            raise RuntimeError(f"orc_fd_directional failed ({rc})")
        return out.value

    def backward(self, dL_dimg: np.ndarray):
        n = len(self.ids)
        g2 = np.zeros((n, 9))
        g = np.zeros((n, 11 + self.n_coef))
        rc = lib().orc_backward(self._h, _p(np.ascontiguousarray(dL_dimg, np.float64)), _p(g2), _p(g))
        if rc != 0:
            raise MemoryError("orc_backward")
        return g2, g


def l1_loss_grad(image: np.ndarray, target: np.ndarray):
    """L = mean |C - target| over H*W*3; dL/dC = sign(C - target) / (3 H W), sign(0) = 0."""
    d = image.astype(np.float64) - target.astype(np.float64)
    return float(np.abs(d).mean()), np.sign(d) / d.size


def adam_cut(p, m, v, grads, idx, lr, beta1, beta2, eps, step):
    """Adam (Kingma and Ba, Algorithm 1) applied to the rows idx of node-indexed
    arrays p, m, v: the cut-set update of the init/training appendix (only the
    nodes of the view's cut are touched).  grads[i] is the gradient of node
    idx[i]; step t >= 1 is the optimiser's step count, used for the bias
    corrections m / (1 - beta1^t) and v / (1 - beta2^t).  FP64; returns the
    new (p, m, v)."""
    p, m, v = (np.array(a, np.float64) for a in (p, m, v))
    g = np.asarray(grads, np.float64)
    for i, node in enumerate(np.asarray(idx).tolist()):
        m[node] = beta1 * m[node] + (1.0 - beta1) * g[i]
        v[node] = beta2 * v[node] + (1.0 - beta2) * g[i] * g[i]
        m_hat = m[node] / (1.0 - beta1 ** step)
        v_hat = v[node] / (1.0 - beta2 ** step)
        p[node] = p[node] - lr * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v


def dist32(mu, pos) -> np.float32:
    """|mu - pos| in FP32 with the cut's operation order (((dx dx + dy dy) + dz dz), then sqrt)."""
    mu, pos = np.asarray(mu, np.float32), np.asarray(pos, np.float32)
    dx, dy, dz = mu[0] - pos[0], mu[1] - pos[1], mu[2] - pos[2]
    s = dx * dx
    s = np.float32(s + dy * dy)
    s = np.float32(s + dz * dz)
    return np.float32(np.sqrt(s))


class OracleCutCache:
    """The GPU cache of SPT cuts (Sec. 4.4 "Caching on the GPU", Eq. 7, and the
    training loop of Alg. 3) as a plain state machine over the SPTs.

    Iteration t (1, 2, ...) of select: when flush_every > 0 and t is a multiple
    of it, every entry is dropped first.  A visible SPT j at root distance d
    (FP32, as the cut computes it) that has an entry (d_c, X_c) is a hit when
    d_min <= r * r <= d_max with r = d / d_c in FP32 (Alg. 3 compares squared
    ratios) and is cut at X_c; otherwise it is loaded: cut at its own
    X = d tau / fx, then entered with (d, X) and size = the number of its
    nodes the cut selected.  Every visible SPT's last use becomes t.  Then,
    oldest last use first (ties by SPT index), entries are dropped while the
    sizes of those left exceed max_nodes.  With LoD noise (spt_scale), d is
    the noisy root distance (the FP32 distance times the factor) throughout."""

    def __init__(self, scene: "OracleScene", max_nodes: int, d_min: float, d_max: float, flush_every: int = 0):
        self.S = scene
        self.max_nodes, self.flush_every = int(max_nodes), int(flush_every)
        self.d_min, self.d_max = np.float32(d_min), np.float32(d_max)
        self.entries = {}  # SPT root tree id -> [d_c, X_c, size, last_use]
        self.t = 0
        self.hits = self.loads = self.evictions = 0
        roots = scene.perm[scene.spt_begin[:-1]]
        self.spt_index = {int(r): j for j, r in enumerate(roots)}

    def select(self, cam, tau: float, cull: bool = True, spt_scale: float = 1.0):
        S = self.S
        tree = S.tree
        s = np.float32(spt_scale)
        self.t += 1
        if self.flush_every > 0 and self.t % self.flush_every == 0:
            self.entries.clear()
        n = tree.n_nodes
        vis = np.zeros(n, np.uint8)
        S.select(cam, tau, cull=cull, spt_visible=vis, spt_scale=s)
        k = np.float32(np.float32(tau) / np.float32(cam.fx))
        override = np.full(n, np.nan, np.float32)
        loaded = []
        for r in np.flatnonzero(vis).tolist():
            d = np.float32(dist32(tree.means[r], cam.pos) * s)  # the root distance the cut uses
            e = self.entries.get(r)
            hit = False
            if e is not None:
                with np.errstate(divide="ignore", invalid="ignore"):
                    q = np.float32(d / e[0])
                    q2 = np.float32(q * q)
                hit = bool(self.d_min <= q2) and bool(q2 <= self.d_max)
            if hit:
                override[r] = e[1]
                e[3] = self.t
                self.hits += 1
            else:
                loaded.append((r, d, np.float32(d * k)))
                self.loads += 1
        ids, st = S.select(cam, tau, cull=cull, spt_X=override, spt_scale=s)
        counts = {}
        for sp in S.spt_of[ids].tolist():
            if sp >= 0:
                counts[sp] = counts.get(sp, 0) + 1
        for r, d, X in loaded:
            self.entries[r] = [d, X, counts.get(r, 0), self.t]
        self.last_loaded = [r for r, _, _ in loaded]  # SPT roots cut afresh by this select
        remaining = sum(e[2] for e in self.entries.values())
        for r in sorted(self.entries, key=lambda r: (self.entries[r][3], self.spt_index[r])):
            if remaining <= self.max_nodes:
                break
            remaining -= self.entries[r][2]
            del self.entries[r]
            self.evictions += 1
        return ids, st
