"""Python front end of liblodgs: scene upload, frames and the three calls of
the path (lod_select, render, render_backward).  PyTorch provides device
memory and streams only."""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from ._lib import check


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def camera_struct(cam) -> _lib.Camera:
    if isinstance(cam, _lib.Camera):
        return cam
    c = _lib.Camera()
    c.R[:] = [float(v) for v in np.asarray(cam.R, np.float32).reshape(9)]
    c.t[:] = [float(v) for v in np.asarray(cam.t, np.float32).reshape(3)]
    c.pos[:] = [float(v) for v in np.asarray(cam.pos, np.float32).reshape(3)]
    c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
    c.width, c.height, c.z_near = cam.width, cam.height, cam.z_near
    return c


class HSPT:
    """Host-side HSPT layout of a hierarchy (lodgs_hspt_build)."""

    def __init__(self, n_nodes, left, right, root, log_scales, log_size):
        L = _lib.load()
        n = int(n_nodes)
        self.n_nodes = n
        self.perm = np.empty(n, np.int32)
        self.r_min = np.empty(n, np.float32)
        self.r_max = np.empty(n, np.float32)
        self.rho = np.empty(n, np.float32)
        self.upper_parent = np.empty(n, np.int32)
        self.spt_begin = np.empty(n + 1, np.int32)
        self.spt_parent = np.empty(n, np.int32)
        nu, ns = ctypes.c_int32(0), ctypes.c_int32(0)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        left = np.ascontiguousarray(left, np.int32)
        right = np.ascontiguousarray(right, np.int32)
        ls = np.ascontiguousarray(log_scales, np.float32)
        check(L.lodgs_hspt_build(n, p(left), p(right), int(root), p(ls), float(log_size), p(self.perm),
                                 p(self.r_min), p(self.r_max), p(self.rho), p(self.upper_parent), p(self.spt_begin),
                                 p(self.spt_parent), ctypes.byref(nu), ctypes.byref(ns)), "lodgs_hspt_build")
        self.n_upper, self.n_spt = nu.value, ns.value
        self.upper_parent = self.upper_parent[: self.n_upper]
        self.spt_begin = self.spt_begin[: self.n_spt + 1]
        self.spt_parent = self.spt_parent[: self.n_spt]


class Scene:
    """A hierarchy resident on the device in HSPT layout order.

    params: dict of torch tensors (layout order) means [n,3], log_scales [n,3],
    quats [n,4], opacity_logits [n], sh [n,K,3]; `perm` maps layout position to
    the input (tree) node id.
    """

    def __init__(self, tree, device="cuda", hspt: HSPT | None = None):
        self.device = torch.device(device)
        self.hspt = hspt or HSPT(tree.n_nodes, tree.left, tree.right, tree.root, tree.log_scales,
                                 tree.log_volume_threshold)
        h = self.hspt
        self.n_nodes, self.n_upper, self.n_spt = h.n_nodes, h.n_upper, h.n_spt
        self.sh_degree = int(tree.sh_degree)
        self.perm = h.perm

        def up(a):
            # Rows are put in layout order on the host, one array at a time.
            # torch's device index_select (2.10, ROCm) left the last 2^26 rows
            # of a 100M x 4 float32 gather unwritten, so it is not used here.
            return torch.from_numpy(np.take(np.ascontiguousarray(a), h.perm, axis=0)).to(self.device)

        self.params = {
            "means": up(tree.means), "log_scales": up(tree.log_scales), "quats": up(tree.quats),
            "opacity_logits": up(tree.opacity_logits), "sh": up(tree.sh.reshape(tree.n_nodes, -1, 3)),
        }
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.device)
        self.lod = {"r_min": dev(h.r_min), "r_max": dev(h.r_max), "rho": dev(h.rho),
                    "upper_parent": dev(h.upper_parent if h.n_upper else np.zeros(1, np.int32)),
                    "spt_begin": dev(h.spt_begin), "spt_parent": dev(h.spt_parent)}
        self._create()

    def _create(self):
        P, Lo = self.params, self.lod
        d = _lib.SceneDesc(self.n_nodes, self.n_upper, self.n_spt, self.sh_degree,
                           _ptr(P["means"]), _ptr(P["log_scales"]), _ptr(P["quats"]), _ptr(P["opacity_logits"]),
                           _ptr(P["sh"]), _ptr(Lo["r_min"]), _ptr(Lo["r_max"]), _ptr(Lo["rho"]),
                           _ptr(Lo["upper_parent"]), _ptr(Lo["spt_begin"]), _ptr(Lo["spt_parent"]))
        h = ctypes.c_void_p()
        check(_lib.load().lodgs_scene_create(ctypes.byref(d), ctypes.byref(h)), "lodgs_scene_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.lodgs_scene_destroy(h)
            self._h = None

    def lod_select_noalloc(self, cam, tau: float, idx, count, cull: bool = True, conservative: bool = False,
                           stream=None):
        """The HSPT cut into the caller's idx (int32 [capacity]) / count (int32
        [1]) device tensors through lodgs_lod_select_noalloc: no frame, no
        device allocation (the workspace is the library's static array)."""
        c = camera_struct(cam)
        flags = (_lib.CULL if cull else 0) | (_lib.CONSERVATIVE if conservative else 0)
        check(_lib.load().lodgs_lod_select_noalloc(self._h, ctypes.byref(c), float(tau), flags, _ptr(idx),
                                                   idx.numel(), _ptr(count), _stream(stream)),
              "lodgs_lod_select_noalloc")
        return idx, count

    def param_bytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in self.params.values())

    def attach_hierarchy(self, tree):
        """Uploads the whole hierarchy (parent and two children per layout
        position) for the comparator cuts, BFS and Eq. 5's parallel cut
        (lodgs_scene_set_hierarchy); frames created afterwards can run them."""
        n = self.n_nodes
        perm = self.perm.astype(np.int64)
        pos = np.empty(n, np.int32)
        pos[perm] = np.arange(n, dtype=np.int32)

        def at(a):  # tree ids -> layout positions, -1 kept, rows in layout order
            a = np.take(np.asarray(a), perm)
            return np.where(a >= 0, pos[np.maximum(a, 0)], -1).astype(np.int32)

        parent = at(tree.parent)
        parent[pos[tree.root]] = -1
        child = np.stack([at(tree.left), at(tree.right)], axis=1)
        height, front = 0, np.array([tree.root], np.int64)
        while front.size:
            height += 1
            front = front[tree.left[front] >= 0]
            front = np.concatenate([tree.left[front], tree.right[front]]).astype(np.int64)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.device)
        self.hierarchy = {"parent": dev(parent), "child": dev(child), "height": height}
        check(_lib.load().lodgs_scene_set_hierarchy(self._h, _ptr(self.hierarchy["parent"]),
                                                    _ptr(self.hierarchy["child"]), height),
              "lodgs_scene_set_hierarchy")


class HostParams:
    """Scene parameters in pinned host memory, rows in layout order: the
    out-of-core store that Frame.gather_rows reads over the host link."""

    def __init__(self, params: dict, sh_degree: int):
        self.params = {k: (v if v.is_pinned() else v.cpu().pin_memory()) for k, v in params.items()}
        self.sh_degree = int(sh_degree)
        self.n_nodes = int(self.params["means"].shape[0])

    @classmethod
    def from_scene(cls, scene: "Scene") -> "HostParams":
        return cls({k: v.detach().cpu() for k, v in scene.params.items()}, scene.sh_degree)


def rows_like(sh_degree: int, capacity: int, device="cuda") -> dict:
    """Device row arrays for capacity gathered nodes (the parameter layouts)."""
    nb = (int(sh_degree) + 1) ** 2
    shapes = {"means": (3,), "log_scales": (3,), "quats": (4,), "opacity_logits": (), "sh": (nb, 3)}
    return {k: torch.zeros((int(capacity),) + s, dtype=torch.float32, device=device) for k, s in shapes.items()}


class CutCache:
    """The GPU cache of SPT cuts (lodgs_cut_cache): a visible SPT whose squared
    root-distance ratio to its cached cut lies in [d_min, d_max] reuses that
    cut; entries beyond max_nodes are dropped least recently used first; every
    flush_every-th cached select starts from an empty cache."""

    def __init__(self, scene: Scene, max_nodes: int, d_min: float, d_max: float, flush_every: int = 0):
        self.scene = scene
        prm = _lib.CutCacheParams(int(max_nodes), float(d_min), float(d_max), int(flush_every))
        h = ctypes.c_void_p()
        check(_lib.load().lodgs_cut_cache_create(scene._h, ctypes.byref(prm), ctypes.byref(h)),
              "lodgs_cut_cache_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.lodgs_cut_cache_destroy(h)
            self._h = None

    def stats(self, stream=None) -> dict:
        s = _lib.CutCacheStats()
        check(_lib.load().lodgs_cut_cache_stats_read(self._h, ctypes.byref(s), _stream(stream)),
              "lodgs_cut_cache_stats_read")
        return s.as_dict()


GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


class RowPool:
    """Device pool of the rows of a CutCache's cached SPT cuts over a pinned
    host store (lodgs_row_pool_*): gather() after a cached lod_select fills
    the rows from the resident upper rows, the pool and, for what neither
    holds, host memory; store() writes trained rows back."""

    def __init__(self, cache: "CutCache", host: "HostParams", capacity: int):
        self.cache, self.host = cache, host
        g = _lib.Grads(*[_ptr(host.params[k]) for k in GROUPS])
        h = ctypes.c_void_p()
        check(_lib.load().lodgs_row_pool_create(cache._h, ctypes.byref(g), host.sh_degree, int(capacity),
                                                ctypes.byref(h)), "lodgs_row_pool_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.lodgs_row_pool_destroy(h)
            self._h = None

    def gather(self, idx, count, rows: dict, stream=None):
        g = _lib.Grads(*[_ptr(rows[k]) for k in GROUPS])
        check(_lib.load().lodgs_gather_rows_pooled(self._h, _ptr(idx), _ptr(count), ctypes.byref(g),
                                                   int(rows["means"].shape[0]), _stream(stream)),
              "lodgs_gather_rows_pooled")
        return rows

    def store(self, idx, count, rows: dict, stream=None):
        g = _lib.Grads(*[_ptr(rows[k]) for k in GROUPS])
        check(_lib.load().lodgs_row_pool_store(self._h, _ptr(idx), _ptr(count), ctypes.byref(g),
                                               int(rows["means"].shape[0]), _stream(stream)), "lodgs_row_pool_store")

    def write_back(self, stream=None):
        """Every changed pooled row to host memory now (lodgs_row_pool_write_back)."""
        check(_lib.load().lodgs_row_pool_write_back(self._h, _stream(stream)), "lodgs_row_pool_write_back")

    def stats(self, node_slot=None, stream=None) -> dict:
        s = _lib.RowPoolStats()
        check(_lib.load().lodgs_row_pool_stats_read(self._h, ctypes.byref(s), _ptr(node_slot), _stream(stream)),
              "lodgs_row_pool_stats_read")
        return s.as_dict()


class AdamCut:
    """Adam on the cut set (lodgs_adam_cut): node-indexed first and second
    moments beside each parameter group; step() updates the rows of the
    selected nodes from selection-indexed gradients (the sel output of
    Frame.backward).  lr: per-group learning rates (3DGS's defaults, one rate
    for all SH coefficients)."""

    DEFAULT_LR = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}

    def __init__(self, params: dict, sh_degree: int, lr: dict | None = None, betas=(0.9, 0.999), eps=1e-15):
        self.params = params
        self.sh_degree = int(sh_degree)
        self.lr = dict(self.DEFAULT_LR, **(lr or {}))
        self.betas, self.eps = betas, eps
        self.exp_avg = {k: torch.zeros_like(v) for k, v in params.items()}
        self.exp_avg_sq = {k: torch.zeros_like(v) for k, v in params.items()}
        self.step_count = 0

    def step(self, grads: dict, idx, count, stream=None):
        self.step_count += 1
        g = lambda d: _lib.Grads(*[_ptr(d.get(k)) if k in self.params else None for k in GROUPS])
        hp = _lib.Adam((ctypes.c_float * 5)(*[float(self.lr[k]) for k in GROUPS]), float(self.betas[0]),
                       float(self.betas[1]), float(self.eps), self.step_count, self.sh_degree)
        n_nodes = next(iter(self.params.values())).shape[0]
        check(_lib.load().lodgs_adam_cut(ctypes.byref(g(self.params)), ctypes.byref(g(grads)),
                                         ctypes.byref(g(self.exp_avg)), ctypes.byref(g(self.exp_avg_sq)),
                                         ctypes.byref(hp), _ptr(idx), _ptr(count), int(idx.numel()), int(n_nodes),
                                         _stream(stream)), "lodgs_adam_cut")


class Frame:
    """Device workspace of one view in flight (lodgs_frame)."""

    def __init__(self, scene: Scene, max_selected: int, max_instances: int, max_width: int, max_height: int):
        self.scene = scene
        caps = _lib.FrameCaps(int(max_selected), int(max_instances), int(max_width), int(max_height))
        self.caps = caps
        h = ctypes.c_void_p()
        check(_lib.load().lodgs_frame_create(scene._h, ctypes.byref(caps), ctypes.byref(h)), "lodgs_frame_create")
        self._h = h
        dev = scene.device
        self.idx = torch.zeros(int(max_selected), dtype=torch.int32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int32, device=dev)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.lodgs_frame_destroy(h)
            self._h = None

    def lod_select(self, cam, tau: float, cull: bool = True, conservative: bool = False, method: str = "hspt",
                   cache: CutCache | None = None, stream=None):
        """Runs the cut into self.idx / self.count (device); returns them.
        conservative: cut each SPT at max(0, d - R) tau / fx (LODGS_CONSERVATIVE).
        method: "hspt" (the HSPT cut), or the whole-hierarchy comparators "bfs"
        and "parallel" (Eq. 5), which need Scene.attach_hierarchy before the
        frame was created.  cache: select through an SPT-cut cache (HSPT cut,
        culling only)."""
        c = camera_struct(cam)
        if cache is not None:
            if conservative or method != "hspt":
                raise ValueError("the SPT-cut cache takes the default HSPT cut only")
            check(_lib.load().lodgs_lod_select_cached(self._h, cache._h, ctypes.byref(c), float(tau),
                                                      _lib.CULL if cull else 0, _ptr(self.idx), self.idx.numel(),
                                                      _ptr(self.count), _stream(stream)), "lodgs_lod_select_cached")
            return self.idx, self.count
        flags = (_lib.CULL if cull else 0) | (_lib.CONSERVATIVE if conservative else 0)
        flags |= {"hspt": 0, "bfs": _lib.CUT_BFS, "parallel": _lib.CUT_PARALLEL}[method]
        check(_lib.load().lodgs_lod_select(self._h, ctypes.byref(c), float(tau), flags,
                                           _ptr(self.idx), self.idx.numel(), _ptr(self.count), _stream(stream)),
              "lodgs_lod_select")
        return self.idx, self.count

    def render(self, cam, idx=None, count=None, bg=(0.0, 0.0, 0.0), out=None, stream=None):
        idx = self.idx if idx is None else idx
        count = self.count if count is None else count
        if out is None:
            out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device=self.scene.device)
        c = camera_struct(cam)
        b = (ctypes.c_float * 3)(*[float(x) for x in bg])
        check(_lib.load().lodgs_render(self._h, _ptr(idx), _ptr(count), ctypes.byref(c),
                                       ctypes.cast(b, ctypes.c_void_p), _ptr(out), _stream(stream)), "lodgs_render")
        self._last = (idx, count, out)
        return out

    def gather_rows(self, host: HostParams, rows: dict, idx=None, count=None, stream=None):
        """Copies the selected nodes' parameters from the host store into rows
        (row k = node idx[k]) with one kernel reading host memory."""
        idx = self.idx if idx is None else idx
        count = self.count if count is None else count
        g = lambda d: _lib.Grads(*[_ptr(d[k]) for k in GROUPS])
        check(_lib.load().lodgs_gather_rows(ctypes.byref(g(host.params)), ctypes.byref(g(rows)), host.sh_degree,
                                            _ptr(idx), _ptr(count), int(rows["means"].shape[0]), host.n_nodes,
                                            _stream(stream)), "lodgs_gather_rows")
        return rows

    def render_rows(self, cam, rows: dict, count=None, bg=(0.0, 0.0, 0.0), out=None, stream=None):
        """render() with the i-th rendered node's parameters at row i of rows."""
        count = self.count if count is None else count
        if out is None:
            out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device=self.scene.device)
        c = camera_struct(cam)
        b = (ctypes.c_float * 3)(*[float(x) for x in bg])
        g = _lib.Grads(*[_ptr(rows[k]) for k in GROUPS])
        check(_lib.load().lodgs_render_rows(self._h, ctypes.byref(g), _ptr(count), ctypes.byref(c),
                                            ctypes.cast(b, ctypes.c_void_p), _ptr(out), _stream(stream)),
              "lodgs_render_rows")
        self._last = (None, count, out)
        return out

    def backward(self, dL_drgb, sel: dict | None = None, nodes: dict | None = None, stream=None,
                 phases: str = "both"):
        """The backward of the last render.  phases: "both", or "partials"
        (blend backward and per-splat sums: frame-local) then "scatter"
        (colour and projection backward into sel / nodes), for several views
        in flight (lodgs_render_backward_phases)."""
        g = lambda d: _lib.Grads(*[_ptr(d.get(k)) if d else None for k in
                                   ("means", "log_scales", "quats", "opacity_logits", "sh")])
        gs, gn = g(sel), g(nodes)
        ph = {"both": _lib.BWD_PARTIALS | _lib.BWD_SCATTER, "partials": _lib.BWD_PARTIALS,
              "scatter": _lib.BWD_SCATTER}[phases]
        check(_lib.load().lodgs_render_backward_phases(self._h, _ptr(dL_drgb), ctypes.byref(gs) if sel else None,
                                                       ctypes.byref(gn) if nodes else None, ph, _stream(stream)),
              "lodgs_render_backward_phases")

    def stats(self, stream=None) -> dict:
        s = _lib.Stats()
        check(_lib.load().lodgs_frame_stats(self._h, ctypes.byref(s), _stream(stream)), "lodgs_frame_stats")
        return s.as_dict()

    def set_lod_noise(self, factor: float = 1.0):
        """The LoD noise of training: later selects on this frame multiply the
        distance to every SPT root by factor (1: none); see training.lod_noise."""
        check(_lib.load().lodgs_frame_set_lod_noise(self._h, float(factor)), "lodgs_frame_set_lod_noise")

    def set_densify_stats(self, max_grad2d=None):
        """Attach a node-indexed float32 array that every later backward raises
        to each drawn node's screen-space mean-gradient norm (None detaches)."""
        self._densify = max_grad2d
        check(_lib.load().lodgs_frame_set_densify_stats(self._h, _ptr(max_grad2d)), "lodgs_frame_set_densify_stats")

    def set_contrib_stats(self, last=None, count=None, iteration=None):
        """Attaches the pruning statistic: node-indexed int32 `last` receives
        the device int32 `iteration` for every node that contributes to a
        pixel in a later backward; `count` (optional) accumulates the
        contributing pixels.  last=None detaches."""
        check(_lib.load().lodgs_frame_set_contrib_stats(self._h, _ptr(last), _ptr(count) if last is not None else None,
                                                        _ptr(iteration) if last is not None else None),
              "lodgs_frame_set_contrib_stats")
        self._contrib = (last, count, iteration)

    def clear_status(self, stream=None):
        check(_lib.load().lodgs_frame_clear_status(self._h, _stream(stream)), "lodgs_frame_clear_status")

    def set_timing(self, enable: bool = True):
        check(_lib.load().lodgs_frame_set_timing(self._h, 1 if enable else 0), "lodgs_frame_set_timing")

    def timings(self) -> dict:
        """{stage: (total ms, calls)} since the last read (blocks)."""
        t = _lib.Timings()
        check(_lib.load().lodgs_frame_timings(self._h, ctypes.byref(t)), "lodgs_frame_timings")
        return t.as_dict()

    def blend_work(self, stream=None):
        """(evaluations, contributions) of the last render's forward blend."""
        e, c = ctypes.c_int64(0), ctypes.c_int64(0)
        check(_lib.load().lodgs_frame_blend_work(self._h, ctypes.byref(e), ctypes.byref(c), _stream(stream)),
              "lodgs_frame_blend_work")
        return e.value, c.value

    def l1_loss(self, img, target, grad=None, loss=None, stream=None):
        """dL/dimg of the mean absolute error (written to grad) and, optionally, L."""
        grad = torch.empty_like(img) if grad is None else grad
        check(_lib.load().lodgs_l1_loss(self._h, _ptr(img), _ptr(target), img.numel(), _ptr(grad), _ptr(loss),
                                        _stream(stream)), "lodgs_l1_loss")
        return grad

    def instances(self, stream=None):
        n_max = int(self.caps.max_instances)
        tiles = torch.empty(n_max, dtype=torch.int32, device=self.scene.device)
        pos = torch.empty(n_max, dtype=torch.int32, device=self.scene.device)
        n = ctypes.c_int64(0)
        check(_lib.load().lodgs_frame_read_instances(self._h, _ptr(tiles), _ptr(pos), n_max, ctypes.byref(n),
                                                     _stream(stream)), "lodgs_frame_read_instances")
        m = min(n.value, n_max)
        return tiles[:m], pos[:m]


class ViewGraph:
    """lod_select + render of one image size captured in a HIP graph
    (lodgs_graph_capture_view); replayed for any camera of that size and any tau.
    The image is written to ``self.out``; selection to the frame's idx/count."""

    def __init__(self, frame: Frame, cam, tau: float, stream, cull: bool = True, bg=(0.0, 0.0, 0.0)):
        self.frame = frame
        self.width, self.height = cam.width, cam.height
        self.stream = stream
        self.out = torch.zeros((cam.height, cam.width, 3), dtype=torch.float32, device=frame.scene.device)
        c = camera_struct(cam)
        b = (ctypes.c_float * 3)(*[float(x) for x in bg])
        h = ctypes.c_void_p()
        check(_lib.load().lodgs_graph_capture_view(frame._h, ctypes.byref(c), float(tau), _lib.CULL if cull else 0,
                                                   _ptr(frame.idx), frame.idx.numel(), _ptr(frame.count),
                                                   ctypes.cast(b, ctypes.c_void_p), _ptr(self.out),
                                                   stream.cuda_stream, ctypes.byref(h)), "lodgs_graph_capture_view")
        self._h = h

    def launch(self, cam, tau: float, stream=None):
        s = self.stream if stream is None else stream
        check(_lib.load().lodgs_graph_launch(self._h, ctypes.byref(camera_struct(cam)), float(tau), s.cuda_stream),
              "lodgs_graph_launch")
        return self.out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.lodgs_graph_destroy(h)
            self._h = None


class StepGraph:
    """A training step (lod_select, render, L1 loss against a target, backward
    into sel or nodes) captured in one HIP graph (lodgs_graph_capture_step);
    replayed for any camera of the captured size, any tau and any target.
    The image goes to ``self.out``, dL/dimage to ``self.dL``, the loss to
    ``self.loss``."""

    def __init__(self, frame: Frame, cam, tau: float, target, stream, sel: dict | None = None,
                 nodes: dict | None = None, cull: bool = True, bg=(0.0, 0.0, 0.0)):
        self.frame = frame
        self.width, self.height = cam.width, cam.height
        self.stream = stream
        dev = frame.scene.device
        self.out = torch.zeros((cam.height, cam.width, 3), dtype=torch.float32, device=dev)
        self.dL = torch.zeros_like(self.out)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self._keep = (target, sel, nodes)
        g = lambda d: _lib.Grads(*[_ptr(d.get(k)) for k in ("means", "log_scales", "quats", "opacity_logits", "sh")])
        gs = g(sel) if sel else None
        gn = g(nodes) if nodes else None
        c = camera_struct(cam)
        b = (ctypes.c_float * 3)(*[float(x) for x in bg])
        h = ctypes.c_void_p()
        check(_lib.load().lodgs_graph_capture_step(
            frame._h, ctypes.byref(c), float(tau), _lib.CULL if cull else 0, _ptr(frame.idx), frame.idx.numel(),
            _ptr(frame.count), ctypes.cast(b, ctypes.c_void_p), _ptr(self.out), _ptr(target), _ptr(self.dL),
            _ptr(self.loss), ctypes.byref(gs) if gs else None, ctypes.byref(gn) if gn else None,
            stream.cuda_stream, ctypes.byref(h)), "lodgs_graph_capture_step")
        self._h = h

    def launch(self, cam, tau: float, target, stream=None):
        s = self.stream if stream is None else stream
        check(_lib.load().lodgs_graph_launch_step(self._h, ctypes.byref(camera_struct(cam)), float(tau),
                                                  _ptr(target), s.cuda_stream), "lodgs_graph_launch_step")
        return self.out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.lodgs_graph_destroy(h)
            self._h = None


def grads_like(scene: Scene, n: int | None = None, zero: bool = True) -> dict:
    """Gradient arrays shaped like the scene parameters ([n, ...], default all nodes)."""
    out = {}
    for k, v in scene.params.items():
        shape = (v.shape[0] if n is None else n,) + tuple(v.shape[1:])
        out[k] = (torch.zeros if zero else torch.empty)(shape, dtype=v.dtype, device=v.device)
    return out
