"""ctypes declarations of liblodgs.so (include/lodgs.h).  Argument marshalling
only: every step of the path runs in the library's kernels.  Loading fails
loudly when the library has not been built; there is no fallback."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblodgs.so")

OK, E_INVALID, E_CAPACITY, E_HIP, E_OOM, E_STATE = 0, -1, -2, -3, -4, -5
CULL = 1
CONSERVATIVE = 2
BWD_PARTIALS = 1  # lodgs_render_backward_phases
BWD_SCATTER = 2
CUT_BFS = 4
CUT_PARALLEL = 8

c_p = ctypes.c_void_p
i32, i64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float


class Camera(ctypes.Structure):
    _fields_ = [("R", f32 * 9), ("t", f32 * 3), ("pos", f32 * 3), ("fx", f32), ("fy", f32), ("cx", f32),
                ("cy", f32), ("width", i32), ("height", i32), ("z_near", f32)]


class SceneDesc(ctypes.Structure):
    _fields_ = [("n_nodes", i64), ("n_upper", i32), ("n_spt", i32), ("sh_degree", i32),
                ("d_means", c_p), ("d_log_scales", c_p), ("d_quats", c_p), ("d_opacity_logits", c_p),
                ("d_sh", c_p), ("d_r_min", c_p), ("d_r_max", c_p), ("d_rho", c_p), ("d_upper_parent", c_p),
                ("d_spt_begin", c_p), ("d_spt_parent", c_p)]


class FrameCaps(ctypes.Structure):
    _fields_ = [("max_selected", i64), ("max_instances", i64), ("max_width", i32), ("max_height", i32)]


class Grads(ctypes.Structure):
    _fields_ = [("d_means", c_p), ("d_log_scales", c_p), ("d_quats", c_p), ("d_opacity_logits", c_p),
                ("d_sh", c_p)]


class Adam(ctypes.Structure):
    _fields_ = [("lr", f32 * 5), ("beta1", f32), ("beta2", f32), ("eps", f32), ("step", i32), ("sh_degree", i32)]


class CutCacheParams(ctypes.Structure):
    _fields_ = [("max_nodes", i64), ("d_min", f32), ("d_max", f32), ("flush_every", i32)]


class CutCacheStats(ctypes.Structure):
    _fields_ = [("iterations", i64), ("hits", i64), ("loads", i64), ("evictions", i64), ("cached_spts", i64),
                ("cached_nodes", i64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("status", i32), ("n_selected", i32), ("n_upper_selected", i32), ("n_spt_visible", i32),
                ("n_spt_candidates", i64), ("n_rendered", i32), ("n_drawn", i32), ("n_instances", i64)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


STAGES = ("select", "project", "depth_sort", "duplicate", "tile_sort", "ranges", "blend", "blend_bwd",
          "project_bwd", "loss")


class Timings(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 10), ("calls", i64 * 10)]

    def as_dict(self):
        return {name: (float(self.ms[k]), int(self.calls[k])) for k, name in enumerate(STAGES)}


class RowPoolStats(ctypes.Structure):
    _fields_ = [("capacity", i64), ("pooled_rows", i64), ("host_rows", i64), ("inserted", i64), ("released", i64),
                ("insert_failures", i64), ("written_back", i64)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


SERVER_MAX_SIZES = 8


class ServerCaps(ctypes.Structure):
    _fields_ = [("n_sizes", i32), ("sizes", (i32 * 2) * SERVER_MAX_SIZES), ("max_slots", i32),
                ("max_selected", i64), ("max_instances", i64), ("hbm_reserve", i64), ("flags", ctypes.c_uint32),
                ("bg", f32 * 3)]


class Request(ctypes.Structure):
    _fields_ = [("cam", Camera), ("tau", f32), ("d_rgb", c_p), ("user", ctypes.c_uint64)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("user", ctypes.c_uint64), ("status", i32), ("attempts", i32),
                ("n_selected", i32), ("n_drawn", i32), ("n_instances", i64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("slots", i32), ("busy", i32), ("queued", i32), ("unpolled", i32), ("slot_bytes", i64),
                ("base_slot_bytes", i64), ("retries", i64), ("rejected", i64), ("evicted", i64)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


EXPORTS = {
    "lodgs_hspt_build": ([i64, c_p, c_p, i32, c_p, ctypes.c_double, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p],
                         ctypes.c_int),
    "lodgs_scene_create": ([ctypes.POINTER(SceneDesc), ctypes.POINTER(c_p)], ctypes.c_int),
    "lodgs_scene_destroy": ([c_p], None),
    "lodgs_scene_set_hierarchy": ([c_p, c_p, c_p, ctypes.c_int32], ctypes.c_int),
    "lodgs_frame_create": ([c_p, ctypes.POINTER(FrameCaps), ctypes.POINTER(c_p)], ctypes.c_int),
    "lodgs_frame_destroy": ([c_p], None),
    "lodgs_lod_select": ([c_p, ctypes.POINTER(Camera), f32, ctypes.c_uint32, c_p, i64, c_p, c_p], ctypes.c_int),
    "lodgs_lod_select_noalloc": ([c_p, ctypes.POINTER(Camera), f32, ctypes.c_uint32, c_p, i64, c_p, c_p],
                                 ctypes.c_int),
    "lodgs_render": ([c_p, c_p, c_p, ctypes.POINTER(Camera), c_p, c_p, c_p], ctypes.c_int),
    "lodgs_render_backward": ([c_p, c_p, ctypes.POINTER(Grads), ctypes.POINTER(Grads), c_p], ctypes.c_int),
    "lodgs_render_backward_phases": ([c_p, c_p, ctypes.POINTER(Grads), ctypes.POINTER(Grads), ctypes.c_uint32, c_p],
                                     ctypes.c_int),
    "lodgs_frame_stats": ([c_p, ctypes.POINTER(Stats), c_p], ctypes.c_int),
    "lodgs_frame_read_instances": ([c_p, c_p, c_p, i64, ctypes.POINTER(i64), c_p], ctypes.c_int),
    "lodgs_frame_clear_status": ([c_p, c_p], ctypes.c_int),
    "lodgs_frame_set_timing": ([c_p, ctypes.c_int], ctypes.c_int),
    "lodgs_frame_timings": ([c_p, ctypes.POINTER(Timings)], ctypes.c_int),
    "lodgs_frame_blend_work": ([c_p, ctypes.POINTER(i64), ctypes.POINTER(i64), c_p], ctypes.c_int),
    "lodgs_l1_loss": ([c_p, c_p, c_p, i64, c_p, c_p, c_p], ctypes.c_int),
    "lodgs_selftest_arith": ([c_p, c_p, i64, c_p, c_p, c_p], ctypes.c_int),
    "lodgs_graph_capture_view": ([c_p, ctypes.POINTER(Camera), f32, ctypes.c_uint32, c_p, i64, c_p, c_p, c_p, c_p,
                                  ctypes.POINTER(c_p)], ctypes.c_int),
    "lodgs_graph_launch": ([c_p, ctypes.POINTER(Camera), f32, c_p], ctypes.c_int),
    "lodgs_graph_destroy": ([c_p], None),
    "lodgs_graph_capture_step": ([c_p, ctypes.POINTER(Camera), f32, ctypes.c_uint32, c_p, i64, c_p, c_p, c_p, c_p, c_p,
                                  c_p, ctypes.POINTER(Grads), ctypes.POINTER(Grads), c_p, ctypes.POINTER(c_p)],
                                 ctypes.c_int),
    "lodgs_graph_launch_step": ([c_p, ctypes.POINTER(Camera), f32, c_p, c_p], ctypes.c_int),
    "lodgs_adam_cut": ([ctypes.POINTER(Grads)] * 4 + [ctypes.POINTER(Adam), c_p, c_p, i64, i64, c_p], ctypes.c_int),
    "lodgs_cut_cache_create": ([c_p, ctypes.POINTER(CutCacheParams), ctypes.POINTER(c_p)], ctypes.c_int),
    "lodgs_cut_cache_destroy": ([c_p], None),
    "lodgs_lod_select_cached": ([c_p, c_p, ctypes.POINTER(Camera), f32, ctypes.c_uint32, c_p, i64, c_p, c_p],
                                ctypes.c_int),
    "lodgs_cut_cache_stats_read": ([c_p, ctypes.POINTER(CutCacheStats), c_p], ctypes.c_int),
    "lodgs_gather_rows": ([ctypes.POINTER(Grads), ctypes.POINTER(Grads), i32, c_p, c_p, i64, i64, c_p], ctypes.c_int),
    "lodgs_render_rows": ([c_p, ctypes.POINTER(Grads), c_p, ctypes.POINTER(Camera), c_p, c_p, c_p], ctypes.c_int),
    "lodgs_frame_set_lod_noise": ([c_p, ctypes.c_float], ctypes.c_int),
    "lodgs_frame_set_densify_stats": ([c_p, c_p], ctypes.c_int),
    "lodgs_row_pool_create": ([c_p, ctypes.POINTER(Grads), i32, i64, ctypes.POINTER(c_p)], ctypes.c_int),
    "lodgs_row_pool_destroy": ([c_p], None),
    "lodgs_gather_rows_pooled": ([c_p, c_p, c_p, ctypes.POINTER(Grads), i64, c_p], ctypes.c_int),
    "lodgs_row_pool_store": ([c_p, c_p, c_p, ctypes.POINTER(Grads), i64, c_p], ctypes.c_int),
    "lodgs_row_pool_write_back": ([c_p, c_p], ctypes.c_int),
    "lodgs_row_pool_stats_read": ([c_p, ctypes.POINTER(RowPoolStats), c_p, c_p], ctypes.c_int),
    "lodgs_frame_set_contrib_stats": ([c_p, c_p, c_p, c_p], ctypes.c_int),
    "lodgs_server_create": ([c_p, ctypes.POINTER(ServerCaps), ctypes.POINTER(c_p)], ctypes.c_int),
    "lodgs_server_destroy": ([c_p], None),
    "lodgs_server_submit": ([c_p, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "lodgs_server_poll": ([c_p, ctypes.POINTER(Completion), i32, ctypes.POINTER(i32)], ctypes.c_int),
    "lodgs_server_stats_read": ([c_p, ctypes.POINTER(ServerStats)], ctypes.c_int),
    "lodgs_last_error": ([], ctypes.c_char_p),
}

_lib = None


class LodgsError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def load():
    """Loads the in-tree liblodgs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2507_01110_amd.build` "
                              "(or __graft_entry__.build()); the path has no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in EXPORTS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(code: int, where: str):
    if code != OK:
        msg = load().lodgs_last_error()
        raise LodgsError(code, where, msg.decode() if msg else "")
