#!/usr/bin/env python3
"""Benchmark of the per-view LoD-select + splat forward/backward path.

Workload (default "city"): 50M leaf Gaussians over a 4 x 4 km extent (60% on
the ground plane, 40% in 20,000 boxes of height U(5,150) m), about 100M
hierarchy nodes with SH degree 3, resident in HBM; views along the 256-pose
aerial-to-street path at tau in {0.5, 1, 2} (768 views), 1920 x 1080.  One
step = one view: LoD select, forward render, L1 loss against a seeded random
target, backward with the gradients accumulated into node-indexed arrays.

Prints one JSON line (metric, value = ms per view, roofline of the dominant
kernel, CPU baseline of the oracle on a bounded sample).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3
# FP32 operations of one (pixel, splat) evaluation of the blend that reaches
# the compositing step: offsets 2, power 7 (two fused), exp 21 (ten fused),
# alpha/skip/termination 6, weight and colour 7 (three fused); fused = 2.
FLOP_PER_EVAL = 43
# FP32 operations of one backward (pixel, splat) evaluation: the forward
# replay (43) plus the colour/alpha/conic/mean gradient terms (about 45).
FLOP_PER_EVAL_BWD = 88


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload(name, leaves):
    from scenegen import configs
    if name == "city":
        spec = configs.city_spec(n=leaves or 50_000_000)
        views = [(configs.city_path_camera(k), tau) for tau in configs.CITY_TAUS for k in range(256)]
        desc = {"workload": "city-50M-1080p-path", "leaves": spec.n, "extent_m": 4000, "boxes": spec.n_boxes,
                "resolution": [1920, 1080], "poses": 256, "taus": list(configs.CITY_TAUS), "sh_degree": 3}
    elif name == "medium":
        spec = configs.medium_spec(n=leaves or 2_000_000)
        import numpy as np
        views = []
        rng = np.random.default_rng(101)
        for k in range(32):
            views.append((configs.medium_camera(seed=101 + k), 1.0))
        desc = {"workload": "medium-2M-1080p", "leaves": spec.n, "resolution": [1920, 1080], "sh_degree": 3}
    else:
        spec = configs.tiny_spec(n=leaves or 16384)
        views = [(configs.tiny_camera(), 1.0)]
        desc = {"workload": "tiny-16k-512", "leaves": spec.n, "resolution": [512, 512], "sh_degree": 3}
    return spec, views, desc


def stage_bytes(c, H, W, n_coef):
    """Algorithmic HBM bytes of one view by stage (FP32 / int32 layouts)."""
    par = 4 * (3 + 3 + 4 + 1 + n_coef)  # bytes of one node's parameters
    b = {}
    b["select"] = c["n_upper"] * 24 + c["n_spt_visible"] * 32 + c["n_spt_candidates"] * 8 + c["n_selected"] * 4
    # every selected node: index, mean, scale, rotation (footprint), tile count
    b["project"] = c["n_rendered"] * (4 + 12 + 12 + 16 + 4) + c["n_drawn"] * (4 + 4 * n_coef + 64 + 4 + 8)
    # compaction of the drawn splats (two reads of the tile counts), then 4 radix passes
    b["depth_sort"] = c["n_rendered"] * 8 + c["n_drawn"] * 16 + 4 * c["n_drawn"] * 16
    # instances: tile key, emission index, owning splat, 16-bit block mask
    b["duplicate"] = c["n_drawn"] * 16 + c["n_instances"] * 14
    b["tile_sort"] = 2 * c["n_instances"] * 16
    # tile ranges (written, then read by the tile order), the tile order
    b["ranges"] = c["n_instances"] * 4 + (H * W // 256) * (8 + 8 + 4)
    # per instance: index, splat, 64-byte record, block mask, 16-bit events
    b["blend"] = c["n_instances"] * (8 + 64 + 2 + 2) + H * W * 12
    b["loss"] = H * W * 36
    # per instance: index, splat, record, events, 10-float partial
    b["blend_bwd"] = c["n_instances"] * (8 + 64 + 2 + 40) + H * W * 24
    b["project_bwd"] = c["n_drawn"] * (16 + 3 * par) + c["n_instances"] * 40
    return b


SERVE_RATES = (50.0, 200.0, 800.0, 1600.0)


def kernel_source_hash():
    """sha256 over what the measured kernels (the blend forward and backward)
    are compiled from: their two source files, every header they can include
    and the build flags.  A stored counter reading applies only to the kernels
    it was taken from; changes elsewhere in the library do not void it."""
    import glob
    import hashlib
    h = hashlib.sha256()
    pkg = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2507_01110_amd")
    csrc = os.path.join(pkg, "csrc")
    files = [os.path.join(csrc, "lodgs_render.hip"), os.path.join(csrc, "lodgs_backward.hip")]
    files += sorted(glob.glob(os.path.join(csrc, "*.h")))
    files += [os.path.join(os.path.dirname(pkg), "include", "lodgs.h"), os.path.join(pkg, "build.py")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(stage):
    """HBM bytes per launch of the stage's kernel from a committed rocprofv3
    summary (lines 'TRAFFIC <stage> <kernel> <bytes> <source hash>'), or None
    when none matches the current sources."""
    import glob
    here = os.path.dirname(os.path.abspath(__file__))
    want = kernel_source_hash()
    for f in sorted(glob.glob(os.path.join(here, "profiles", "*.txt"))):
        with open(f) as fh:
            for line in fh:
                w = line.split()
                if len(w) == 5 and w[0] == "TRAFFIC" and w[1] == stage and w[4] == want:
                    return int(w[3])
    return None


def stored_executed(stage):
    """The executed-work figures of the stage's kernel from a committed SQ
    counter summary (lines 'EXECUTED <stage> <kernel> <key=value> ... <source
    hash>'), or None when none matches the current sources."""
    import glob
    here = os.path.dirname(os.path.abspath(__file__))
    want = kernel_source_hash()
    for f in sorted(glob.glob(os.path.join(here, "profiles", "*.txt"))):
        with open(f) as fh:
            for line in fh:
                w = line.split()
                if len(w) >= 4 and w[0] == "EXECUTED" and w[1] == stage and w[-1] == want:
                    out = {"kernel": w[2], "source": os.path.basename(f)}
                    for kv in w[3:-1]:
                        k, _, v = kv.partition("=")
                        out[k] = float(v)
                    return out
    return None


def summarize_profiles(trace_csv, fetch_csv, write_csv, commands, dispatch_csv=None, stage_views=768):
    """Text summary of a rocprofv3 kernel-trace run and two --pmc runs
    (FETCH_SIZE, WRITE_SIZE): per-kernel average duration and HBM KiB per
    dispatch, the copy-kernel calibration (the 1 GiB device copies of
    --copy-calibration: 1 GiB read and 1 GiB written each) and one TRAFFIC line
    per blend stage."""
    import collections
    import csv
    import re
    short = lambda n: re.sub(r"\(.*", "", n.replace("(anonymous namespace)::", "")).replace("lodgs::", "").strip()
    out = ["rocprofv3 summary (kernel trace + FETCH_SIZE / WRITE_SIZE counters)", ""]
    out += ["commands:"] + ["  " + c for c in commands] + [""]
    rows = list(csv.DictReader(open(trace_csv)))
    out.append("%-52s %7s %12s %7s" % ("kernel", "calls", "avg_us", "pct"))
    for r in rows[:30]:
        out.append("%-52s %7s %12.2f %7.2f" % (short(r["Name"])[:52], r["Calls"], float(r["AverageNs"]) / 1e3,
                                                 float(r["Percentage"])))
    cnt = {}
    for path, name in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        d = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == name:
                d[short(r["Kernel_Name"])].append((int(r["Grid_Size"]), float(r["Counter_Value"])))
        cnt[name] = d
    gib_kib = float(1 << 20)
    copies = lambda name: [v for g, v in cnt[name].get("__amd_rocclr_copyBuffer", []) if v > 0.25 * gib_kib]
    cf, cw = copies("FETCH_SIZE"), copies("WRITE_SIZE")
    f_fetch = gib_kib / (sum(cf) / len(cf)) if cf else None
    f_write = gib_kib / (sum(cw) / len(cw)) if cw else None
    out += ["", "copy calibration (1 GiB device copy): FETCH_SIZE %s KiB, WRITE_SIZE %s KiB -> factors fetch %s, "
            "write %s" % ([round(x) for x in cf], [round(x) for x in cw],
                          None if f_fetch is None else round(f_fetch, 4), None if f_write is None else round(f_write, 4)),
            "", "%-52s %7s %14s %14s %14s" % ("kernel", "n", "FETCH_KiB", "WRITE_KiB", "HBM_MB_scaled")]
    hbm = {}
    for k in sorted(cnt["FETCH_SIZE"], key=lambda k: -sum(v for _, v in cnt["FETCH_SIZE"][k])):
        fv = [v for _, v in cnt["FETCH_SIZE"][k]]
        wv = [v for _, v in cnt["WRITE_SIZE"].get(k, [])] or [0.0]
        fa, wa = sum(fv) / len(fv), sum(wv) / len(wv)
        scaled = None
        if f_fetch and f_write:
            scaled = (fa * f_fetch + wa * f_write) * 1024.0
            hbm[k] = scaled
        out.append("%-52s %7d %14.0f %14.0f %14s" % (k[:52], len(fv), fa, wa,
                                                     "-" if scaled is None else "%.2f" % (scaled / 1e6)))
    out.append("")
    if dispatch_csv:
        # per dispatch, in time order: the stage pass (one view at a time, the
        # durations bench.py's roofline divides by) is the last stage_views
        # dispatches of a blend kernel, the timed loop the stage_views before
        d = collections.defaultdict(list)
        for r in csv.DictReader(open(dispatch_csv)):
            k = short(r["Kernel_Name"]).replace("void ", "").replace(" ", "")
            if k.startswith(("k_blend_bwd", "k_blend_q")):
                d[k].append((int(r["Start_Timestamp"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
        out.append("blend kernels per dispatch (us): stage pass = the last %d dispatches (one view at a time), "
                   "timed loop = the %d before them" % (stage_views, stage_views))
        for k in sorted(d):
            v = [x for _, x in sorted(d[k])]
            if len(v) >= 2 * stage_views:
                sp, tl = v[-stage_views:], v[-2 * stage_views:-stage_views]
                out.append("DISPATCH %s stage_pass_avg_us=%.2f timed_loop_avg_us=%.2f" %
                           (k, sum(sp) / len(sp), sum(tl) / len(tl)))
        out.append("")
    h = kernel_source_hash()
    for stage, pats in (("blend_bwd", ("k_blend_bwd",)), ("blend", ("k_blend_q", "k_blend<false"))):
        ks = [k for k in hbm if k.replace("void ", "").startswith(pats)]
        if ks:
            out.append("TRAFFIC %s %s %d %s" % (stage, ks[0].replace("void ", "").replace(" ", ""), round(hbm[ks[0]]), h))
    return "\n".join(out)


def summarize_counters(csvs, commands, trace_stats=None, kernels=("k_blend_q", "k_blend_bwd")):
    """Text summary of rocprofv3 --pmc runs (SQ counters): per kernel whose
    name starts with one of `kernels`, the sum of each counter over its
    dispatches, and the derived shares (active / wait / VALU / LDS per wave
    cycle, executed VALU instructions per busy cycle and SIMD, LDS bank
    conflicts per LDS-active cycle)."""
    import collections
    import csv
    import re
    short = lambda n: re.sub(r"\(.*", "", n.replace("(anonymous namespace)::", "")).replace("lodgs::", "").strip()
    sums = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    avg_us = {}
    if trace_stats:
        for r in csv.DictReader(open(trace_stats)):
            avg_us[short(r["Name"]).replace("void ", "")] = float(r["AverageNs"]) / 1e3
    for path in csvs:
        for r in csv.DictReader(open(path)):
            k = short(r["Kernel_Name"]).replace("void ", "")
            if not k.startswith(tuple(kernels)):
                continue
            sums[k][r["Counter_Name"]] += float(r["Counter_Value"])
            disp[k].add((path, r["Dispatch_Id"]))
    executed = []
    out = ["rocprofv3 SQ counter summary, kernel sources at hash %s" % kernel_source_hash(), "", "commands:"]
    out += ["  " + c for c in commands] + ["", "counter sums over the kernel's dispatches:", ""]
    for k in sorted(sums):
        c = sums[k]
        out.append("%s  (%d dispatches per counter pass)" % (k, len(disp[k]) // max(1, len(csvs))))
        for name in sorted(c):
            out.append("  %-24s %.4g" % (name, c[name]))
        g = lambda n: c.get(n, float("nan"))
        d = []
        wc = g("SQ_WAVE_CYCLES")
        for n, label in (("SQ_ACTIVE_INST_ANY", "active-any"), ("SQ_WAIT_ANY", "wait-any"),
                         ("SQ_WAIT_INST_ANY", "wait-inst-any"), ("SQ_ACTIVE_INST_VALU", "VALU active"),
                         ("SQ_ACTIVE_INST_LDS", "LDS active")):
            if n in c and wc == wc:
                d.append("%s / wave-cycles %.2f" % (label, c[n] / wc))
        if "SQ_LDS_BANK_CONFLICT" in c and "SQ_LDS_IDX_ACTIVE" in c:
            d.append("LDS bank-conflict / LDS-active cycles %.2f" % (c["SQ_LDS_BANK_CONFLICT"] / c["SQ_LDS_IDX_ACTIVE"]))
        nd = max(1, len(disp[k]) // max(1, len(csvs)))
        ex = {}
        if "SQ_INSTS_VALU" in c:
            per = c["SQ_INSTS_VALU"] / nd
            d.append("VALU wave-instructions per dispatch %.4g" % per)
            ex["valu_wave_instr_per_launch"] = per
            if k in avg_us:
                # 1024 SIMDs at 2.4 GHz issue at most one wave64 FP32 instruction per 4 cycles each
                # (the 78.6 TFLOP/s non-packed FMA peak)
                util = per / (avg_us[k] * 1e-6 * 1024 * 2.4e9 / 4.0)
                d.append("issue utilisation at the traced %.1f us per dispatch %.2f" % (avg_us[k], util))
                ex["traced_us"] = avg_us[k]
                ex["valu_issue_util"] = util
        for n, key in (("SQ_ACTIVE_INST_VALU", "valu_active_share"), ("SQ_WAIT_ANY", "wait_any_share")):
            if n in c and wc == wc:
                ex[key] = c[n] / wc
        if "SQ_LDS_BANK_CONFLICT" in c and "SQ_LDS_IDX_ACTIVE" in c:
            ex["lds_conflict_share"] = c["SQ_LDS_BANK_CONFLICT"] / c["SQ_LDS_IDX_ACTIVE"]
        out.append("  derived: " + "; ".join(d))
        out.append("")
        stage = "blend_bwd" if k.startswith("k_blend_bwd") else ("blend" if k.startswith("k_blend_q") else None)
        if stage and ex:
            executed.append("EXECUTED %s %s %s %s" % (stage, k.replace(" ", ""),
                                                      " ".join("%s=%.6g" % kv for kv in sorted(ex.items())),
                                                      kernel_source_hash()))
    return "\n".join(out + executed)


def configs_taus(workload):
    from scenegen import configs
    return configs.CITY_TAUS if workload == "city" else (1.0,)


def serve_bench(scene, n_per_rate, rates=SERVE_RATES, max_slots=8, warmup=100):
    """Serving on the resident scene: Poisson arrivals at each rate, image size
    uniform over 360p/720p/1080p/4K, random poses, tau in {0.5, 1, 2}, forward only;
    the library's slot server (graph replays on per-slot streams, admission by
    free HBM, overflowed requests re-served on grown slots) against the
    one-request-per-launch loop on the identical arrival trace.  The rates are
    the workload's 50/200/800 req/s plus 1600 req/s, beyond what the
    one-request-per-launch loop sustains."""
    import numpy as np
    from scenegen import configs
    from paper_2507_01110_amd.lodgs import Frame
    from paper_2507_01110_amd.server import RenderServer, baseline_loop, poisson_requests, summarize, Request
    sizes = list(configs.SERVE_RESOLUTIONS)
    ext = 2000.0
    cap_sel, cap_inst = 1 << 23, 24 << 20
    srv = RenderServer(scene, sizes, cap_sel, cap_inst, max_slots=max_slots, hbm_reserve=16 << 30)
    base_frame = Frame(scene, cap_sel, cap_inst, 3840, 2160)
    out = {"max_slots": max_slots, "base_slot_GB": round(srv.stats()["base_slot_bytes"] / 1e9, 2), "rates": {}}
    for k, lam in enumerate(rates):
        n = n_per_rate[k] if isinstance(n_per_rate, (list, tuple)) else n_per_rate
        rng = np.random.default_rng(300 + k)
        make = lambda r: configs.random_pose_camera(r, ext, *sizes[r.integers(len(sizes))])
        reqs = poisson_requests(rng, lam, n + warmup, make)
        base = [Request(r.rid, r.arrival, r.cam, r.tau) for r in reqs]
        got, span, _ = srv.run(reqs)
        bl, span_b, _, base_frame = baseline_loop(base_frame, base)
        out["rates"][str(int(lam))] = {"server": summarize(got, span, warmup),
                                       "baseline": summarize(bl, span_b, warmup)}
        log(f"serve lambda {lam}: server {out['rates'][str(int(lam))]['server']} "
            f"baseline {out['rates'][str(int(lam))]['baseline']}")
    out["server_stats"] = srv.stats()
    # the comparison at equal p99: the highest rate each sustains (throughput
    # within 5% of the arrival rate) with p99 at most the server's p99 at the
    # highest rate
    def sustained(kind, p99_cap):
        best = None
        for lam, r in out["rates"].items():
            x = r[kind]
            if x["throughput_rps"] and x["throughput_rps"] >= 0.95 * float(lam) and x["p99_ms"] <= p99_cap:
                best = max(best or 0.0, float(lam))
        return best
    hi = max(out["rates"], key=float)
    p99_server_hi = out["rates"][hi]["server"]["p99_ms"]
    out["equal_p99"] = {"p99_cap_ms": p99_server_hi,
                        "server_max_rate": sustained("server", p99_server_hi),
                        "baseline_max_rate": sustained("baseline", p99_server_hi)}
    return out


def cpu_baseline(tree, views, target, cut="hspt", conservative=False):
    """The oracle on a bounded sample of the same workload: for each (camera,
    tau) of views, select (the same cut), render, L1 and backward; mean
    wall-clock per view."""
    import oracle
    t0 = time.time()
    O = oracle.OracleScene(tree)
    setup = time.time() - t0
    per, nsel = [], []
    for cam, tau in views:
        t0 = time.time()
        if cut == "hspt":
            ids, _ = O.select(cam, tau, conservative=conservative)
        else:
            ids = O.select_full(cam, tau, cut)
        F = oracle.OracleFrame(tree, ids, cam)
        _, dL = oracle.l1_loss_grad(F.image, target)
        F.backward(dL)
        per.append(time.time() - t0)
        nsel.append(int(len(ids)))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    taus = ", ".join(str(t) for _, t in views)
    return {"value": round(1000.0 * sum(per) / len(per), 1), "unit": "ms per view", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{len(views)} views of the same scene (the middle path pose at tau {taus}): select + render + "
                      f"L1 + backward, mean per view; per-scene oracle setup ({setup:.1f} s) excluded",
            "per_view_ms": [round(1000.0 * x, 1) for x in per], "n_selected": nsel,
            "tiny_forward": tiny_forward_oracle(threads)}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def tiny_forward_oracle(threads, repeats=5):
    """The oracle on the tiny plain-forward workload (16,384 leaves, 512 x 512,
    tau 1: select + render), on 1 thread and on `threads`; mean ms per view."""
    import ctypes
    import oracle
    import scenegen
    from scenegen import configs
    tree = scenegen.build_tree(configs.tiny_spec())
    cam = configs.tiny_camera()
    O = oracle.OracleScene(tree)
    set_threads = oracle.lib().omp_set_num_threads
    set_threads.argtypes = [ctypes.c_int]
    out = {}
    for nt in (1, threads):
        set_threads(nt)
        t0 = time.time()
        for _ in range(repeats):
            ids, _ = O.select(cam, 1.0)
            oracle.OracleFrame(tree, ids, cam)
        out[f"ms_{nt}_thread" + ("s" if nt > 1 else "")] = round(1000.0 * (time.time() - t0) / repeats, 2)
    set_threads(threads)
    return out


def ultra_bench(args):
    """150M leaves over 8 x 8 km (60,000 boxes), ~300M nodes; each step renders a
    batch of 8 1080p views (c3-style random poses, tau 1) through the autograd
    Function, L1 against seeded targets, backward accumulating node gradients."""
    import numpy as np
    import torch
    import scenegen
    from scenegen import configs
    from paper_2507_01110_amd.autograd import render_lod
    from paper_2507_01110_amd.lodgs import Frame, Scene, grads_like

    spec = configs.city_spec(n=args.leaves or 150_000_000, seed=4, half_extent=4000.0, n_boxes=60000)
    t0 = time.time()
    tree = scenegen.build_tree(spec)
    log(f"ultra scene: {tree.n_nodes} nodes built in {time.time() - t0:.1f} s")
    scene = Scene(tree)
    n_nodes = tree.n_nodes
    del tree
    torch.cuda.synchronize()
    for t in scene.params.values():
        t.requires_grad_(True)
    grads = grads_like(scene)
    B = 8
    rng = np.random.default_rng(104)
    cams = [configs.random_pose_camera(rng, 4000.0, 1920, 1080) for _ in range(64)]
    frames = [Frame(scene, 1 << 24, 1 << 26, 1920, 1080) for _ in range(B)]
    targets = [torch.from_numpy(scenegen.target_image(1080, 1920, 204 + k)).cuda() for k in range(B)]

    # counting pass (untimed): per-view counts for the byte model of section S1-S11
    counts = []
    n_coef = 3 * (scene.sh_degree + 1) ** 2
    for c in cams:
        f = frames[0]
        f.lod_select(c, 1.0)
        f.render(c)
        st = f.stats()
        assert st["status"] == 0, st
        st["n_spt_candidates"] = int(st["n_spt_candidates"])
        st["n_upper"] = scene.n_upper
        counts.append(st)
    view_bytes = [sum(stage_bytes(c, 1080, 1920, n_coef).values()) for c in counts]

    # the batch's views on n_st streams (their forwards and the frame-local
    # halves of their backwards overlap), the additions into the node
    # gradients on one scatter stream in the autograd engine's order; with
    # --serial every view on the current stream
    main = torch.cuda.current_stream()
    n_st = 1 if args.serial else max(1, min(args.frame_streams, B))
    streams = [main] if args.serial else [torch.cuda.Stream() for _ in range(n_st)]
    scat = None if args.serial else torch.cuda.Stream()

    def step(s):
        losses = []
        for b in range(B):
            st = streams[b % n_st]
            st.wait_stream(main)
            with torch.cuda.stream(st):
                img = render_lod(frames[b], cams[(s * B + b) % len(cams)], 1.0, accumulate_into=grads,
                                 scatter_stream=scat)
                losses.append((img - targets[b]).abs().mean())
        for st in streams:
            main.wait_stream(st)
        torch.stack(losses).sum().backward()
        if scat is not None:
            main.wait_stream(scat)

    for s in range(args.warmup):
        step(s)
    torch.cuda.synchronize()
    for f in frames:
        assert f.stats()["status"] == 0
    torch.cuda.reset_peak_memory_stats()
    K = max(1, args.steps)
    t0 = time.perf_counter()
    for s in range(K):
        step(s)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    free, total = torch.cuda.mem_get_info()
    st = [f.stats() for f in frames]
    timed_bytes = sum(view_bytes[(s * B + b) % len(cams)] for s in range(K) for b in range(B))
    out = {"metric": "ms per 8-view 1080p training step @150M Gaussians (LoD+splat fwd/bwd, autograd)",
           "value": round(el * 1000.0 / K, 3), "unit": "ms per step", "n_gpus": 1, "steps": K, "warmup": args.warmup,
           "higher_is_better": False, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "ultra-150M-8x1080p", "leaves": spec.n, "nodes": n_nodes, "batch": B,
                      "streams": n_st, "scatter_stream": scat is not None},
           "views_per_s": round(B * K / el, 1), "param_GB": round(scene.param_bytes() / 1e9, 2),
           "peak_torch_allocated_GB": round(torch.cuda.max_memory_allocated() / 1e9, 2),
           "device_used_GB": round((total - free) / 1e9, 2),
           "algorithmic_GB_per_view": round(timed_bytes / (B * K) / 1e9, 4),
           "achieved_GB_s": round(timed_bytes / el / 1e9, 1),
           "hbm_fraction": round(timed_bytes / el / (HBM_PEAK_GBS * 1e9), 4),
           "last_batch": {k: int(np.mean([s[k] for s in st])) for k in ("n_selected", "n_drawn", "n_instances")}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=768)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--workload", choices=["city", "medium", "tiny", "ultra"], default="city")
    ap.add_argument("--conservative", action="store_true",
                    help="cut each SPT at max(0, d - R) tau / fx (the CONSERVATIVE variant) instead of d tau / fx")
    ap.add_argument("--cut", choices=["hspt", "bfs", "parallel"], default="hspt",
                    help="LoD cut: the HSPT cut, or a whole-hierarchy comparator (BFS, Eq. 5's parallel cut)")
    ap.add_argument("--adam", action="store_true",
                    help="training iteration: backward into selection-indexed gradients, then the cut-set Adam "
                         "step (instead of accumulating node gradients)")
    ap.add_argument("--cache", type=str, default="",
                    help="select through the SPT-cut cache: max_nodes,d_min,d_max,flush_every (e.g. 15000000,0.8,1.25,1000)")
    ap.add_argument("--rows", action="store_true",
                    help="out-of-core parameters: gather each cut's rows from pinned host memory, render from the "
                         "rows, backward into selection-indexed gradients")
    ap.add_argument("--pool", type=int, default=0,
                    help="with --rows and --cache: keep the cached cuts' rows in a device pool of this many rows "
                         "(at least the cache's max_nodes) and gather from it")
    ap.add_argument("--in-flight", type=int, default=4,
                    help="views in flight in the timed loop (frames taking turns, each on its own stream; the "
                         "scatter into the node gradients in view order on one more)")
    ap.add_argument("--frame-streams", type=int, default=3,
                    help="streams the frames' work is spread over (view i on stream i mod this; at most "
                         "--in-flight)")
    ap.add_argument("--serial", action="store_true",
                    help="one view at a time in the timed loop (the default keeps several views in flight, "
                         "see --in-flight)")
    ap.add_argument("--graph", action="store_true",
                    help="time the training step captured in one graph (lodgs_graph_capture_step) instead of plain "
                         "launches")
    ap.add_argument("--leaves", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--targets", type=int, default=8, help="distinct seeded targets resident in HBM")
    ap.add_argument("--diag", action="store_true", help="print per-tile load statistics of sampled views")
    ap.add_argument("--serve-requests", type=str, default="1000,2000,4000,4000",
                    help="measured requests per arrival rate 50,200,800,1600 req/s (0 disables serving)")
    ap.add_argument("--summarize-profiles", nargs=3, metavar=("TRACE_STATS_CSV", "FETCH_CSV", "WRITE_CSV"),
                    help="print a text summary of rocprofv3 outputs (no GPU work)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="COUNTER_CSV",
                    help="print a text summary of rocprofv3 --pmc SQ counter runs of the blend kernels (no GPU work)")
    ap.add_argument("--trace-stats", default=None,
                    help="with --summarize-counters: a rocprofv3 kernel-trace stats CSV for per-dispatch durations")
    ap.add_argument("--trace-csv", default=None,
                    help="with --summarize-profiles: the rocprofv3 kernel-trace CSV, for the blend kernels' "
                         "averages over the stage pass (the last --stage-views dispatches) and the timed loop")
    ap.add_argument("--stage-views", type=int, default=768,
                    help="with --trace-csv: views of the run's stage pass (its --steps)")
    ap.add_argument("--profile-command", action="append", default=[],
                    help="command line that produced the profiles (repeatable; recorded in the summary)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy (HBM byte-counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.summarize_profiles:
        print(summarize_profiles(*args.summarize_profiles, args.profile_command, args.trace_csv, args.stage_views))
        return
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters, args.profile_command, args.trace_stats))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): the path is a "
              "single-GPU pipeline here; views would shard across GPUs with a replicated scene.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import scenegen
    from paper_2507_01110_amd.lodgs import AdamCut, CutCache, Frame, HostParams, Scene, camera_struct, rows_like

    torch.cuda.set_device(0)
    if args.workload == "ultra":
        ultra_bench(args)
        return
    spec, views, desc = workload(args.workload, args.leaves)
    t0 = time.time()
    tree = scenegen.build_tree(spec)
    log(f"scene: {tree.n_nodes} nodes built in {time.time() - t0:.1f} s")
    t0 = time.time()
    scene = Scene(tree)
    torch.cuda.synchronize()
    log(f"HSPT {scene.n_upper} upper nodes, {scene.n_spt} SPTs; upload {scene.param_bytes() / 1e9:.1f} GB "
        f"in {time.time() - t0:.1f} s")
    if args.cut != "hspt":
        scene.attach_hierarchy(tree)
        log(f"whole hierarchy attached for the {args.cut} cut (height {scene.hierarchy['height']})")
    W, H = views[0][0].width, views[0][0].height
    n_coef = 3 * (tree.sh_degree + 1) ** 2
    K = max(1, args.steps)
    stride = max(1, len(views) // K) if K < len(views) else 1
    seq = [(i * stride) % len(views) for i in range(K)]

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x 1 GiB device-to-device copies")

    # Counting pass (untimed): per-view counts for the byte model and capacities.
    cap_sel, cap_inst = min(scene.n_nodes, 1 << 24), 1 << 27
    frame = Frame(scene, cap_sel, cap_inst, W, H)
    counts = []
    for v in seq:
        cam, tau = views[v]
        while True:
            frame.lod_select(cam, tau, conservative=args.conservative, method=args.cut)
            frame.render(cam)
            st = frame.stats()
            if st["status"] == 0:
                break
            grown = (cap_sel, cap_inst)
            cap_sel = max(cap_sel, int(st["n_selected"] * 1.25) + 1024)
            cap_inst = max(cap_inst, int(st["n_instances"] * 1.25) + 1024)
            if (cap_sel, cap_inst) == grown:  # a BFS frontier longer than the selection capacity
                cap_sel = min(2 * cap_sel, scene.n_nodes)
            log(f"capacity grown to {cap_sel} selected / {cap_inst} instances")
            del frame
            torch.cuda.empty_cache()
            frame = Frame(scene, cap_sel, cap_inst, W, H)
        ev, co = frame.blend_work()
        st["evaluations"], st["contributions"] = ev, co
        if args.diag and len(counts) % max(1, K // 12) == 0:
            tl, _ = frame.instances()
            per_tile = torch.bincount(tl.long(), minlength=(W // 16 + 1) * (H // 16 + 1)).cpu().numpy()
            log(f"view {v}: tau {tau} selected {st['n_selected']} drawn {st['n_drawn']} instances "
                f"{st['n_instances']} per-tile max {per_tile.max()} p99 {np.percentile(per_tile, 99):.0f} "
                f"mean {per_tile.mean():.1f} tiles>1000 {(per_tile > 1000).sum()} evals {ev} contrib {co}")
        counts.append(st)
    log(f"counting pass done: mean n_selected {np.mean([c['n_selected'] for c in counts]):.0f}, "
        f"mean instances {np.mean([c['n_instances'] for c in counts]):.0f}")

    targets = [torch.from_numpy(scenegen.target_image(H, W, 202 + k)).cuda() for k in range(args.targets)]
    if args.adam or args.rows:
        if args.adam:
            opt = AdamCut(scene.params, tree.sh_degree)
        sel = {k: torch.zeros((cap_sel,) + tuple(v.shape[1:]), dtype=torch.float32, device="cuda")
               for k, v in scene.params.items()}
        if args.rows:
            host = HostParams.from_scene(scene)
            rows = rows_like(tree.sh_degree, cap_sel)
            log(f"out-of-core store: {sum(v.numel() * 4 for v in host.params.values()) / 1e9:.1f} GB pinned host memory")
    else:
        grads = {k: torch.zeros_like(v) for k, v in scene.params.items()}
    img = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    dL = torch.empty_like(img)

    cstructs = [camera_struct(c) for c, _ in views]

    cache = None
    if args.cache:
        mx, dmin, dmax, fl = args.cache.split(",")
        cache = CutCache(scene, int(mx), float(dmin), float(dmax), int(fl))
    pool = None
    if args.pool:
        if not (args.rows and cache is not None):
            raise SystemExit("--pool needs --rows and --cache")
        from paper_2507_01110_amd.lodgs import RowPool
        pool = RowPool(cache, host, args.pool)
        log(f"row pool: {args.pool} rows in HBM")

    def step(i):
        cam, tau = cstructs[seq[i % K]], views[seq[i % K]][1]
        if cache is not None:
            frame.lod_select(cam, tau, cache=cache)
        else:
            frame.lod_select(cam, tau, conservative=args.conservative, method=args.cut)
        if args.rows:
            if pool is not None:
                pool.gather(frame.idx, frame.count, rows)
            else:
                frame.gather_rows(host, rows)
            frame.render_rows(cam, rows, out=img)
        else:
            frame.render(cam, out=img)
        frame.l1_loss(img, targets[seq[i % K] % len(targets)], grad=dL)
        if args.adam or args.rows:
            frame.backward(dL, sel=sel)
            if args.adam:
                opt.step(sel, frame.idx, frame.count)
        else:
            frame.backward(dL, nodes=grads)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    frame.timings()  # discard warmup records
    # The timed loop: plain launches (no stage events), or with --graph the
    # whole step captured in one graph and replayed per view.
    use_graph = args.graph and not (args.adam or args.rows or args.cache or args.cut != "hspt" or args.conservative)
    run_stream = torch.cuda.Stream() if use_graph else torch.cuda.current_stream()
    graph = None
    if use_graph:
        from paper_2507_01110_amd.lodgs import StepGraph
        v0 = seq[0]
        with torch.cuda.stream(run_stream):
            graph = StepGraph(frame, cstructs[v0], views[v0][1], targets[v0 % len(targets)], run_stream,
                              nodes=grads)

        def timed_step(i):
            v = seq[i % K]
            graph.launch(cstructs[v], views[v][1], targets[v % len(targets)], run_stream)

        for i in range(args.warmup):
            timed_step(i)
    else:
        timed_step = step
    # Several views in flight (node-gradient accumulation only: the parameters
    # do not change between views, so the forward of a later view may run
    # while an earlier view's backward does).  Frames take turns; view i's
    # select, forward, L1 and the frame-local half of its backward (blend
    # backward and per-splat sums) run on stream i mod n_st; one more stream
    # runs the other half (colour and projection backward into the node
    # gradients) in view order, so the gradients are those of one view at a
    # time bit for bit.  A frame takes its next view once the scatter of its
    # last is done.
    pipelined = not (args.serial or use_graph or args.adam or args.rows or cache is not None) and args.in_flight > 1
    n_fl = max(2, args.in_flight)
    n_st = max(1, min(args.frame_streams, n_fl))
    launch_desc = "one graph per step" if use_graph else (
        "plain launches, %d views in flight on %d frames (select, forward, L1 and blend backward of view i on "
        "stream i mod %d; the scatter into the node gradients in view order on one more stream)" % (n_fl, n_fl, n_st)
        if pipelined else "plain launches, one view at a time")
    if pipelined:
        frames = [frame] + [Frame(scene, cap_sel, cap_inst, W, H) for _ in range(n_fl - 1)]
        imgs = [img] + [torch.empty_like(img) for _ in range(n_fl - 1)]
        dLs = [dL] + [torch.empty_like(dL) for _ in range(n_fl - 1)]
        sFs, sB = [torch.cuda.Stream() for _ in range(n_st)], torch.cuda.current_stream()
        part_done = [torch.cuda.Event() for _ in range(n_fl)]
        scat_done = [torch.cuda.Event() for _ in range(n_fl)]

        def frame_work(i):  # on stream i mod n_st
            k, v = i % n_fl, seq[i % K]
            f, sF = frames[k], sFs[i % n_st]
            sF.wait_event(scat_done[k])  # the frame's previous view is done with it
            f.lod_select(cstructs[v], views[v][1], conservative=args.conservative, method=args.cut, stream=sF)
            f.render(cstructs[v], out=imgs[k], stream=sF)
            f.l1_loss(imgs[k], targets[v % len(targets)], grad=dLs[k], stream=sF)
            f.backward(dLs[k], stream=sF, phases="partials")
            part_done[k].record(sF)

        def scatter_on_B(i):  # in view order
            k = i % n_fl
            sB.wait_event(part_done[k])
            frames[k].backward(None, nodes=grads, stream=sB, phases="scatter")
            scat_done[k].record(sB)

        for i in range(max(args.warmup, n_fl)):  # every frame's warm-up
            frame_work(i)
            scatter_on_B(i)
    # The out-of-core path through the row pool, views in flight: the cached
    # select and the pool's gather change the cache's and the pool's state, so
    # they run in view order on one stream; view i's render from its rows, L1
    # and backward (into selection-indexed gradients) then run on stream
    # i mod n_st; a frame and its rows take the next view once that work is
    # done.
    pool_pipelined = not (args.serial or use_graph) and pool is not None and args.in_flight > 1
    if pool_pipelined:
        launch_desc = ("plain launches, %d views in flight on %d frames (cached select and pool gather in view "
                       "order on one stream; render, L1 and backward of view i on stream i mod %d)" % (n_fl, n_fl, n_st))
        frames = [frame] + [Frame(scene, cap_sel, cap_inst, W, H) for _ in range(n_fl - 1)]
        imgs = [img] + [torch.empty_like(img) for _ in range(n_fl - 1)]
        dLs = [dL] + [torch.empty_like(dL) for _ in range(n_fl - 1)]
        rowss = [rows] + [rows_like(tree.sh_degree, cap_sel) for _ in range(n_fl - 1)]
        sels = [sel] + [{k: torch.zeros_like(t) for k, t in sel.items()} for _ in range(n_fl - 1)]
        sS, sFs = torch.cuda.current_stream(), [torch.cuda.Stream() for _ in range(n_st)]
        gathered = [torch.cuda.Event() for _ in range(n_fl)]
        done = [torch.cuda.Event() for _ in range(n_fl)]

        def state_work(i):  # in view order
            k, v = i % n_fl, seq[i % K]
            sS.wait_event(done[k])  # the frame and its rows are free
            frames[k].lod_select(cstructs[v], views[v][1], cache=cache, stream=sS)
            pool.gather(frames[k].idx, frames[k].count, rowss[k], stream=sS)
            gathered[k].record(sS)

        def rows_work(i):  # on stream i mod n_st
            k, v = i % n_fl, seq[i % K]
            f, sF = frames[k], sFs[i % n_st]
            sF.wait_event(gathered[k])
            f.render_rows(cstructs[v], rowss[k], out=imgs[k], stream=sF)
            f.l1_loss(imgs[k], targets[v % len(targets)], grad=dLs[k], stream=sF)
            f.backward(dLs[k], sel=sels[k], stream=sF)
            done[k].record(sF)

        for i in range(max(args.warmup, n_fl)):  # every frame's warm-up
            state_work(i)
            rows_work(i)
    torch.cuda.synchronize()
    # events on the stream the library launches on: around every view, or,
    # with two views in flight, at every backward's end (per-view figures are
    # then the intervals between consecutive completions)
    ev = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(K)]
    t0 = time.perf_counter()
    if pool_pipelined:
        ev[0][0].record(sS)
        for i in range(K):
            state_work(i)
            rows_work(i)
            ev[i][1].record(sFs[i % n_st])
    elif pipelined:
        ev[0][0].record(sB)
        for t in range(K + n_fl - 1):
            if t < K:
                frame_work(t)
            i = t - (n_fl - 1)
            if i >= 0:
                scatter_on_B(i)
                ev[i][1].record(sB)
                if i + 1 < K:
                    ev[i + 1][0] = ev[i][1]
    else:
        for i in range(K):
            ev[i][0].record(run_stream)
            timed_step(i)
            ev[i][1].record(run_stream)
    t_enq = time.perf_counter() - t0  # the host's time to issue the loop's work
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if pool_pipelined:  # views may complete out of order: intervals between sorted completions
        done_ms = np.sort([ev[0][0].elapsed_time(e[1]) for e in ev])
        per_view = np.diff(np.concatenate([[0.0], done_ms]))
    else:
        per_view = np.array([a.elapsed_time(b) for a, b in ev])
    ms_per_view = elapsed * 1000.0 / K
    log(f"timed {K} views ({launch_desc}): {ms_per_view:.3f} ms per view "
        f"(the host issued the work in {t_enq * 1000.0 / K:.3f} ms per view)")
    if pipelined or pool_pipelined:
        for f in frames:
            st_p = f.stats()
            assert st_p["status"] == 0, st_p
        del frames[1:]
    st_fin = frame.stats()
    assert st_fin["status"] == 0, st_fin
    # Stage split: the same views again with plain launches and events around
    # every stage on the launch stream (the events add gaps between stages, so
    # these times sum to more than the timed loop's).
    frame.set_timing(True)
    for i in range(K):
        step(i)
    torch.cuda.synchronize()
    frame.set_timing(False)
    tm = frame.timings()
    del graph

    # Byte model and per-stage rates.
    tot_bytes = {}
    for c in counts:
        c["n_spt_candidates"] = int(c["n_spt_candidates"])
        c["n_upper"] = scene.n_upper
        for k, b in stage_bytes(c, H, W, n_coef).items():
            tot_bytes[k] = tot_bytes.get(k, 0) + b
    stages = {}
    for name, (ms, calls) in tm.items():
        if calls == 0:
            continue
        gb = tot_bytes.get(name, 0) / 1e9
        stages[name] = {"ms_per_view": round(ms / K, 4), "GB_per_view": round(gb / K, 4),
                        "GB_s": round(gb / (ms / 1000.0), 1) if ms > 0 else None}
    all_bytes = sum(tot_bytes.values())
    hbm_frac = all_bytes / (elapsed * HBM_PEAK_GBS * 1e9)
    evals = sum(c["evaluations"] for c in counts)
    dom = max(stages, key=lambda s: stages[s]["ms_per_view"])
    dom_ms_total = tm[dom][0]
    if dom in ("blend", "blend_bwd"):
        flop = evals * (FLOP_PER_EVAL if dom == "blend" else FLOP_PER_EVAL_BWD)
        ach = flop / (dom_ms_total / 1000.0) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": round(ach, 2), "peak": FP32_VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP32_VALU_PEAK_TFLOPS, 4), "traffic": stored_traffic(dom),
                "basis": "algorithmic: every (pixel, splat) evaluation the method defines x %d FLOP, including "
                         "those the block masks and events let the kernel skip" % (
                             FLOP_PER_EVAL if dom == "blend" else FLOP_PER_EVAL_BWD),
                "evaluations_per_view": int(evals / K), "algorithmic_bytes_per_launch": int(tot_bytes[dom] / K),
                # what the kernel executed (SQ counters of a committed run at these sources): the
                # nominal figure above credits evaluations that the block masks and events skip
                "executed": stored_executed(dom)}
    else:
        ach = tot_bytes[dom] / (dom_ms_total / 1000.0) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": stored_traffic(dom)}

    serving = None
    nreq = [int(x) for x in args.serve_requests.split(",") if x.strip()]
    if args.workload == "city" and nreq and all(x > 0 for x in nreq):
        del frame
        torch.cuda.empty_cache()
        serving = serve_bench(scene, nreq)
    cpu = None
    if not args.no_cpu_baseline:
        if args.workload == "city":  # the middle path pose (128) at each tau
            sample = [views[128 + 256 * t] for t in range(len(configs_taus(args.workload)))]
        else:
            sample = [views[0]]
        log(f"cpu baseline: oracle on {len(sample)} view(s) ...")
        cpu = cpu_baseline(tree, sample, scenegen.target_image(H, W, 202), args.cut, args.conservative)
        log(f"cpu baseline {cpu['value']} ms per view on {cpu['cores']} threads")

    mean = lambda k: float(np.mean([c[k] for c in counts]))
    out = {
        "metric": "ms per 1080p view (LoD+splat fwd/bwd) @50M Gaussians, %HBM peak; serve p50/p99",
        "value": round(ms_per_view, 4), "unit": "ms per view", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(ms_per_view, 4),
        "per_view_ms": {"median": round(float(np.median(per_view)), 4),
                        "p90": round(float(np.percentile(per_view, 90)), 4),
                        "max": round(float(per_view.max()), 4)}, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded scene, cameras and targets)",
        "config": dict(desc, nodes=int(scene.n_nodes), upper_nodes=int(scene.n_upper), spts=int(scene.n_spt),
                       views_timed=K, parallelism="none", cut="conservative" if args.conservative else ("default" if args.cut == "hspt" else args.cut),
                       update="cut-set Adam" if args.adam else ("selection-indexed gradients" if args.rows
                                                                else "node-gradient accumulation"),
                       params="pinned host memory, rows gathered per view" if args.rows else "resident in HBM"),
        "launch": launch_desc,
        "hbm_fraction_whole_path": round(hbm_frac, 4),
        "algorithmic_GB_per_view": round(all_bytes / K / 1e9, 4),
        "stages": stages,
        "mean_counts": {k: round(mean(k), 1) for k in ("n_selected", "n_spt_visible", "n_spt_candidates",
                                                       "n_drawn", "n_instances", "evaluations", "contributions")},
        "roofline": roof,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    if cache is not None:
        out["config"]["cut"] = "default through the SPT-cut cache " + args.cache
        out["cut_cache"] = cache.stats()
    if pool is not None:
        out["config"]["params"] = f"pinned host memory, rows through a device pool of {args.pool} rows"
        out["row_pool"] = pool.stats()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
