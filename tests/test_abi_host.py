"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host HSPT builder reproduces the oracle's layout bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import configs

from _helpers import random_tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2507_01110_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = L.load()
    hdr = open(os.path.join(ROOT, "include", "lodgs.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(lodgs_\w+)\s*\(", hdr))
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(L.EXPORTS), declared ^ set(L.EXPORTS)


def _check_layout(tree):
    from paper_2507_01110_amd.lodgs import HSPT
    O = oracle.OracleScene(tree)
    H = HSPT(tree.n_nodes, tree.left, tree.right, tree.root, tree.log_scales, tree.log_volume_threshold)
    assert (H.n_upper, H.n_spt) == (O.n_upper, O.n_spt)
    assert np.array_equal(H.perm, O.perm)
    assert np.array_equal(H.spt_begin, O.spt_begin)
    upper = O.perm[: O.n_upper]
    assert np.array_equal(H.r_min[: O.n_upper], O.g[upper])
    assert np.all(np.isinf(H.r_max[: O.n_upper]))
    spt = O.perm[O.n_upper:]
    assert np.array_equal(H.r_min[O.n_upper:], O.r_min[spt])
    assert np.array_equal(H.r_max[O.n_upper:], O.r_max[spt])
    assert np.array_equal(H.rho, O.rho[O.perm])
    par = tree.parent
    exp_up = np.array([O.pos_of[par[u]] if par[u] >= 0 else -1 for u in upper], np.int32)
    assert np.array_equal(H.upper_parent, exp_up)
    roots = O.perm[O.spt_begin[:-1]]
    exp_sp = np.array([O.pos_of[par[r]] if par[r] >= 0 else -1 for r in roots], np.int32)
    assert np.array_equal(H.spt_parent, exp_sp)


def test_hspt_builder_matches_oracle_layout_random_trees():
    rng = np.random.default_rng(11)
    for _ in range(40):
        _check_layout(random_tree(rng, int(rng.integers(1, 65))))


def test_hspt_builder_matches_oracle_layout_tiny(tiny_tree):
    _check_layout(tiny_tree)


@pytest.mark.slow
def test_hspt_builder_matches_oracle_layout_medium_subset():
    _check_layout(scenegen.build_tree(configs.medium_spec(n=200_000, seed=3)))


def test_hspt_builder_rejects_malformed_trees():
    from paper_2507_01110_amd.lodgs import HSPT
    from paper_2507_01110_amd._lib import LodgsError
    ls = np.zeros((3, 3), np.float32)
    with pytest.raises(LodgsError) as e:  # node with a single child
        HSPT(3, np.array([1, -1, -1]), np.array([-1, -1, -1]), 0, ls, 0.0)
    assert e.value.code == -1
    with pytest.raises(LodgsError):  # child out of range
        HSPT(3, np.array([1, -1, -1]), np.array([7, -1, -1]), 0, ls, 0.0)
    with pytest.raises(LodgsError):  # node 2 unreachable from the root
        HSPT(3, np.array([-1, -1, -1]), np.array([-1, -1, -1]), 0, ls, 0.0)
    with pytest.raises(LodgsError):  # cycle: 0 -> (1, 2), 1 -> (0, 2) is rejected (two parents)
        HSPT(3, np.array([1, 0, -1]), np.array([2, 2, -1]), 0, ls, 0.0)


def test_public_header_is_plain_c99(tmp_path):
    # callers of the C ABI need nothing but a C compiler and the header
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    src = tmp_path / "t.c"
    src.write_text('#include "lodgs.h"\nint main(void) { lodgs_adam a; lodgs_cut_cache_params p; (void)a; (void)p;'
                   ' return 0; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                        os.path.join(ROOT, "include"), "-c", str(src), "-o", str(tmp_path / "t.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_ctypes_structs_match_the_header_layout(tmp_path):
    # every struct the binding passes across the ABI has the C compiler's size
    # and field offsets
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    L = _lib()
    structs = {"lodgs_camera": L.Camera, "lodgs_scene_desc": L.SceneDesc, "lodgs_frame_caps": L.FrameCaps,
               "lodgs_grads": L.Grads, "lodgs_adam": L.Adam, "lodgs_cut_cache_params": L.CutCacheParams,
               "lodgs_cut_cache_stats": L.CutCacheStats, "lodgs_stats": L.Stats, "lodgs_timings": L.Timings,
               "lodgs_server_caps": L.ServerCaps, "lodgs_request": L.Request, "lodgs_completion": L.Completion,
               "lodgs_server_stats": L.ServerStats, "lodgs_row_pool_stats": L.RowPoolStats}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lodgs.h"', 'int main(void) {']
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        w = line.split()
        got[tuple(w[:-1])] = int(w[-1])
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])
