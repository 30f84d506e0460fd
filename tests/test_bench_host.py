"""bench.py's host logic: the one-GPU guard, the algorithmic byte model and the
keying of stored counter readings on the blend kernels' sources (no GPU)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_byte_model_sums_its_per_unit_terms():
    # one selected node, drawn, one instance, on a 16 x 16 image (one tile), SH degree 0
    c = {"n_upper": 1, "n_spt_visible": 1, "n_spt_candidates": 1, "n_selected": 1, "n_rendered": 1,
         "n_drawn": 1, "n_instances": 1}
    b = bench.stage_bytes(c, 16, 16, 3)
    par = 4 * (3 + 3 + 4 + 1 + 3)
    assert b["select"] == 24 + 32 + 8 + 4
    assert b["project"] == 48 + (4 + 12 + 64 + 4 + 8)
    assert b["depth_sort"] == 8 + 16 + 64
    assert b["tile_sort"] == 32
    assert b["blend"] == 76 + 256 * 12
    assert b["loss"] == 256 * 36
    assert b["blend_bwd"] == 114 + 256 * 24
    assert b["project_bwd"] == 16 + 3 * par + 40
    # every term is linear in the counts
    c2 = {k: 2 * v for k, v in c.items()}
    b2 = bench.stage_bytes(c2, 16, 16, 3)
    fixed = {"ranges": (256 // 256) * 20, "blend": 256 * 12, "loss": 256 * 36, "blend_bwd": 256 * 24}
    for k in b:
        assert b2[k] - fixed.get(k, 0) == 2 * (b[k] - fixed.get(k, 0)), k


def test_counter_readings_apply_only_to_the_current_blend_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16
    # the committed readings carry the hash of the sources they were taken from
    assert bench.stored_traffic("no_such_stage") is None
    found = bench.stored_traffic("blend_bwd")
    if found is not None:
        assert found > 0
        ex = bench.stored_executed("blend_bwd")
        assert ex is not None and 0.0 < ex["valu_issue_util"] <= 1.0
