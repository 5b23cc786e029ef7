"""Benchmark of the ROI kernel density estimation hot path on one MI355X.

Default workload (the configuration the headline metric is quoted on): the
served request loop on a 1B-point clustered cloud (2,000 anisotropic Gaussian
clumps with power-law masses plus 20% uniform background, drawn on the
device, tree resident in HBM): 8 simulated VR streams with Poisson arrivals
at 90 Hz each (sides log-uniform in [1e-4, 1], panning centres, grids
32^3-128^3, Epanechnikov, h = 0.01 x side), admission by HBM budget (free
HBM after the tree and the grids, minus a reserve).

One step = one second of that offered trace (about 720 requests) served at
saturation: every request of the second is waiting when the step starts and
the continuous-batching loop drains them (4 batches in flight on 4 streams,
up to 64 ROIs per batch). value = useful kernel evaluations (node, particle
pairs inside the support, counted exactly by an untimed pass) of the timed
steps / their wall time. Outside the timed steps the line carries the same
seconds served at saturation one ROI per launch (FIFO), the whole trace
replayed in real time at 90 Hz for both arms (1 s warm-up, then p50 / p99
latency against the 11.1 ms frame budget), bitwise alone-vs-mix checks of
served grids, the oracle on sampled nodes (the CPU baseline), and the other
configurations as sub-records: the 10M-point per-point Gaussian step, the
batch of 256 uneven ROIs vs one launch per ROI and the nested zoom on 100M
points.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("kernel evals/s + ROI grid latency p50/p99 (ms), batched vs "
          "one-ROI-per-launch")
HBM_PEAK_GBS = 8000.0
# VALU issue ceiling of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane
# operations per second. Unpacked float32 and float64 add / mul / fma /
# compare each take one slot (the 78.6 TFLOP/s fp64 and unpacked fp32 vector
# peaks are this rate with an FMA counted as 2 flops); a transcendental
# (exp2) issues at quarter rate and takes 4 slots.
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
# Algorithmic VALU slots per useful evaluation (one (node, particle) term),
# the minimum any evaluation order pays: Epanechnikov with a uniform
# bandwidth 9 (3 differences, the squared distance as one multiply and two
# FMAs, the support compare, 1 - u2 as an FMA, a select, the accumulation);
# truncated Gaussian with a per-particle bandwidth 14 (10 VALU plus one exp2
# at quarter rate = 4 slots).
SLOTS_PER_EVAL = {"gauss_trunc3": 14, "epanechnikov": 9}
# counter summaries of the evaluation kernel (valid only for the kernel
# sources whose hash they record)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_eval_gauss_per_point_10m_128_traffic.md")
SERVED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "eval_served_1b_traffic.md")
KERNEL_SOURCES = ("paper_2601_20758_amd/csrc/eval.hip", "paper_2601_20758_amd/csrc/sfk_device.h",
                  "paper_2601_20758_amd/csrc/sfk_internal.h")


VALU_FILE = os.path.join(ROOT, "profiles", "k_knn_k_eval_per_point_10m_valu.md")


def profiled_valu_busy(kernel_prefix):
    """VALU busy fraction of a kernel from the committed counter summary
    (None if the summary or the kernel's row is missing)."""
    try:
        for line in open(VALU_FILE):
            if line.startswith("| `" + kernel_prefix):
                return float(line.split("|")[3].strip().rstrip("%")) / 100.0
    except (OSError, ValueError, IndexError):
        pass
    return None


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per launch of the evaluation kernel from a committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the reading of a
    reference kernel of known size), or None when the summary is missing or
    was taken on other kernel sources."""
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and line.startswith("- "):
                    k, v = line[2:].split(":", 1)
                    kv[k.strip()] = v.strip().strip("`")
        if kv.get("source_sha256") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10,
                   help="timed steps (seconds of the served trace at saturation)")
    p.add_argument("--warmup", type=int, default=1,
                   help="untimed warm-up steps (seconds of the trace)")
    p.add_argument("--workload", default="served_1b",
                   choices=["served_1b", "per_point_10m", "small"])
    p.add_argument("--serve-points", type=int, default=1_000_000_000,
                   help="cloud size of the served workload")
    p.add_argument("--serve-reserve-gb", type=float, default=16.0,
                   help="HBM kept out of the admission budget")
    p.add_argument("--no-realtime", action="store_true",
                   help="skip the real-time 90 Hz replays (latency arms)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-nodes", type=int, default=600)
    p.add_argument("--no-per-point", action="store_true",
                   help="skip the 10M-point per-point Gaussian step sub-record")
    p.add_argument("--per-point-steps", type=int, default=5)
    p.add_argument("--no-batch", action="store_true",
                   help="skip the batched vs one-ROI-per-launch comparison")
    p.add_argument("--n-batch", type=int, default=256)
    p.add_argument("--batch-points", type=int, default=100_000_000,
                   help="cloud size of the batched vs one-per-launch comparison")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run a 1 GiB fill and a 1 GiB elementwise scale first "
                        "(references for the hardware byte counters)")
    p.add_argument("--no-zoom", action="store_true",
                   help="skip the nested-zoom and MBE sections on the 100M cloud")
    p.add_argument("--view", action="store_true",
                   help="add the view-cache and adaptive-resolution sections on the 100M cloud")
    p.add_argument("--profile-served", action="store_true",
                   help="for counter runs: only the timed continuous-batching steps of the "
                        "served workload (the same trace windows; no warm-up, comparison "
                        "passes, checks or sub-records), so the evaluation kernels of the run "
                        "are exactly the timed launches")
    p.add_argument("--profile-section", choices=["zoom", "batch"],
                   help="for counter runs: only the nested-zoom series or only the 256-ROI "
                        "batch comparison on the 100M cloud (no served workload, no other "
                        "sub-record); prints that record")
    a = p.parse_args()
    if a.profile_served:
        a.no_realtime = a.no_cpu_baseline = a.no_per_point = a.no_batch = a.no_zoom = True
        a.view = False
    return a


def workload(name):
    import synth
    if name == "small":
        pts = synth.c1_cloud(1)
        roi = synth.c1_roi()
        return pts, roi, 0, {"workload": "20k points (half uniform, half in 8 clusters), unit box, "
                                         "32^3, Epanechnikov, fixed h=0.02",
                             "n_points": len(pts), "grid": [32, 32, 32]}
    pts = synth.clumpy_cloud(10_000_000, 2)
    roi = synth.c2_roi(128)
    return pts, roi, 32, {
        "workload": "10M clustered points (2,000 power-law clumps + 20% uniform), unit-box ROI, "
                    "128^3 grid, Gaussian truncated at 3h, per-point h from the 32nd nearest "
                    "neighbour; step = tree build + k-NN + range query + evaluation",
        "n_points": len(pts), "grid": [128, 128, 128], "kernel": "gauss_trunc3",
        "bandwidth": "per_point_knn32", "seed": 2, "particle_order": "hilbert"}


def cpu_baseline(pts, roi, h2, n_nodes, seed=7):
    """The FP64 oracle (brute force over every particle) timed on a random
    sample of grid nodes, reported as useful evaluations per second."""
    import oracle
    g = np.random.default_rng(seed)
    nodes = np.sort(g.choice(roi.n_nodes, size=min(n_nodes, roi.n_nodes), replace=False))
    t0 = time.perf_counter()
    oracle.density(pts, roi, nodes=nodes, h2=h2)
    dt = time.perf_counter() - t0
    useful = int(oracle.support_counts(pts, roi, nodes=nodes, h2=h2).sum())
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": useful / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": "%d random nodes of the grid, each brute-forced over all %d particles "
                      "(FP64 values, per-point h given); %.1f s, %d useful evals"
                      % (len(nodes), len(pts), dt, useful)}


def consumers(ctx, torch, roi, grid, xyz, reps=5):
    """The grid consumers on the step's grid and cloud: density at every
    particle, the selection at the median density and the Marching Cubes
    cells at that threshold (device time per call from events on the
    current stream). Algorithmic bytes of sampling: 12 B read + 4 B written
    per point plus one read of the grid."""
    n = xyz.shape[0]
    st = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            r = fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, r

    dens = torch.empty(n, dtype=torch.float32, device="cuda")
    t_s, _ = timed(lambda: ctx.sample_density(roi, grid, xyz, out=dens))
    iso = float(torch.median(dens[dens > 0]).item())
    t_sel, sel = timed(lambda: ctx.select_points(roi, grid, iso, xyz))
    t_iso, cells = timed(lambda: ctx.iso_cells(roi, grid, iso))
    sample_bytes = 16.0 * n + 4.0 * roi.n_nodes
    return {"workload": "%d particles on the %s grid of the step; threshold = median particle "
                        "density" % (n, "x".join(str(r) for r in roi.res)),
            "sample_ms": t_s, "sample_points_per_s": n / (t_s * 1e-3),
            "sample_gb_per_s": sample_bytes / (t_s * 1e-3) / 1e9,
            "sample_frac_of_hbm": sample_bytes / (t_s * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "select_ms": t_sel, "selected": int(sel.numel()),
            "iso_cells_ms": t_iso, "active_cells": int(cells[0].numel())}


def batch_vs_single(ctx, tree, torch, n_rois, label):
    """Many uneven ROIs in one persistent launch vs one launch per ROI, on
    the resident tree (same kernels, same results)."""
    import synth
    rois = synth.random_batch_rois(n_rois, seed=4)
    outs = [torch.empty(r.n_nodes, device="cuda") for r in rois]
    log("batch vs one launch per ROI:", n_rois, "ROIs")
    # warm both paths
    ctx.wait(ctx.submit(tree, rois, outs))
    for r, o in zip(rois, outs):
        ctx.eval_roi(tree, r, out=o)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # one launch per ROI: per-ROI completion events
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_rois + 1)]
    evs[0].record(stream)
    for i, (r, o) in enumerate(zip(rois, outs)):
        ctx.eval_roi(tree, r, out=o, stream=stream)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    single_ms = evs[0].elapsed_time(evs[-1])
    lat_single = np.array([evs[0].elapsed_time(e) for e in evs[1:]])
    ref = [o.clone() for o in outs]
    # batched: one submit
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = ctx.submit(tree, rois, outs)
    ctx.wait(t)
    batch_ms = (time.perf_counter() - t0) * 1e3
    same = all(torch.equal(a, b) for a, b in zip(ref, outs))
    useful = 0
    for r in rois:
        useful += ctx.debug_eval_count(tree, r)[0]
    return {
        "workload": "%d ROIs, sides log-uniform in [1e-3, 1], grids 16^3-128^3, Epanechnikov, "
                    "h = 0.01 x side, on the resident %s tree" % (n_rois, label),
        "nodes": int(sum(r.n_nodes for r in rois)), "useful_evals": int(useful),
        "batched_ms": batch_ms, "single_launch_ms": single_ms,
        "batched_evals_per_s": useful / (batch_ms * 1e-3),
        "batched_frac_of_valu_ceiling": useful / (batch_ms * 1e-3)
                                        * SLOTS_PER_EVAL["epanechnikov"] / VALU_SLOTS_PER_S,
        "single_launch_evals_per_s": useful / (single_ms * 1e-3),
        "speedup": single_ms / batch_ms,
        "single_launch_latency_p50_ms": float(np.percentile(lat_single, 50)),
        "single_launch_latency_p99_ms": float(np.percentile(lat_single, 99)),
        "batched_latency_ms": batch_ms,
        "bitwise_equal": bool(same),
    }


def serving(ctx, tree, torch, duration_s, label):
    """VR-like request loop on the resident tree: 8 streams of Poisson
    arrivals at 90 Hz each (sides log-uniform in [1e-4, 1], panning centres,
    grids 32^3-128^3, Epanechnikov, h = 0.01 x side). Continuous batching
    over 4 streams vs one ROI per launch in FIFO order."""
    import synth
    arr, _, rois = synth.serving_trace(seed=5, duration_s=duration_s)
    outs = [torch.empty(r.n_nodes, device="cuda") for r in rois]
    rec = {"workload": "%d requests over %.1f s from 8 streams at 90 Hz, sides log-uniform "
                       "in [1e-4, 1], grids 32^3-128^3, Epanechnikov, h = 0.01 x side, "
                       "on the resident %s tree" % (len(rois), duration_s, label),
           "frame_budget_ms": 1000.0 / 90.0}
    log("counting useful pairs of %d requests" % len(rois))
    useful = 0
    for r in rois:
        useful += ctx.debug_eval_count(tree, r)[0]
    rec["useful_evals"] = int(useful)
    for name, mode in (("continuous_batching", 0), ("one_roi_per_launch", 1)):
        log("serving:", name)
        res, s = ctx.serve(tree, arr, rois, outs, mode=mode, n_slots=4, max_batch=64,
                           budget_bytes=float(8 << 30))
        lat = np.array([res[i].latency_ms for i in range(len(rois))])
        rec[name] = {"p50_ms": s.p50_ms, "p99_ms": s.p99_ms, "max_ms": s.max_ms,
                     "deadline_miss_rate": float(np.mean(lat > 1000.0 / 90.0)),
                     "evals_per_s": useful / s.wall_s, "wall_s": s.wall_s,
                     "batches": s.n_batches, "mean_batch": s.mean_batch,
                     "mean_in_flight": s.mean_in_flight, "budget_waits": s.budget_waits}
    return rec


def view_cache(ctx, tree, torch, label, info, n_frames=180):
    """Recomputation policy (view cache) vs recomputing every frame: a smooth
    90 Hz camera path around a massive clump (pan plus a zoom breathing over
    three octaves). Every frame: Epanechnikov, h = 0.01 x the side of the
    wanted grid (64 nodes across the longest side). Recompute: one ROI per
    frame at 64^3. View cache: blocks of 16^3 on lattices reused within a
    spacing ratio of 1.5, a margin of 0.25 x side prefetched."""
    import synth
    boxes = synth.view_path(info, seed=7, n_frames=n_frames)
    res, h0 = 64, 0.01
    budget = 1000.0 / 90.0
    log("view path: %d frames, recompute every frame" % n_frames)
    out = torch.empty(res ** 3, device="cuda")
    lat_re, nodes_re = [], 0
    # warm-up frame (first-use growth of the workspace)
    ctx.eval_roi(tree, synth.Roi(boxes[0][0], boxes[0][1], (res,) * 3, kernel="epanechnikov",
                                 bw="roi_scaled", h=(h0,) * 3), out=out)
    torch.cuda.synchronize()
    for lo, hi in boxes:
        r = synth.Roi(lo, hi, (res,) * 3, kernel="epanechnikov", bw="roi_scaled", h=(h0,) * 3)
        t0 = time.perf_counter()
        ctx.eval_roi(tree, r, out=out)
        torch.cuda.synchronize()
        lat_re.append((time.perf_counter() - t0) * 1e3)
        nodes_re += r.n_nodes
    log("view path: view cache")
    view = ctx.view(tree, kernel="epanechnikov", bw="roi_scaled", h=(h0,), res=res, block=16,
                    scale_threshold=1.5, margin=0.25, max_blocks=16384)
    lat_v, blocks_ev, lattices, grid_nodes = [], 0, 0, 0
    gout = torch.empty(1 << 22, device="cuda")
    for lo, hi in boxes:
        t0 = time.perf_counter()
        g, inf = view.frame(lo, hi, out=gout)
        torch.cuda.synchronize()
        lat_v.append((time.perf_counter() - t0) * 1e3)
        blocks_ev += inf["blocks_evaluated"]
        lattices += 1 if inf["new_lattice"] else 0
        grid_nodes += g.numel()
    view.close()
    lat_re, lat_v = np.array(lat_re), np.array(lat_v)
    ev_nodes = blocks_ev * 16 ** 3
    return {
        "workload": "%d frames at 90 Hz around a massive clump of the resident %s tree: pan "
                    "radius 0.15, side 0.2 x 2^(+-1.5) over 2 s; Epanechnikov, h = 0.01 x "
                    "side at 64 nodes across" % (n_frames, label),
        "recompute_every_frame": {
            "p50_ms": float(np.percentile(lat_re, 50)), "p99_ms": float(np.percentile(lat_re, 99)),
            "deadline_miss_rate": float(np.mean(lat_re > budget)),
            "evaluated_nodes_per_frame": nodes_re / n_frames},
        "view_cache": {
            "p50_ms": float(np.percentile(lat_v, 50)), "p99_ms": float(np.percentile(lat_v, 99)),
            "deadline_miss_rate": float(np.mean(lat_v > budget)),
            "evaluated_nodes_per_frame": ev_nodes / n_frames,
            "returned_nodes_per_frame": grid_nodes / n_frames,
            "lattices_created": lattices, "block": 16, "scale_threshold": 1.5, "margin": 0.25},
        "evaluated_nodes_ratio": (ev_nodes / n_frames) / (nodes_re / n_frames),
    }


def nested_zoom(ctx, tree, torch, label, info):
    """Nested zoom: boxes of side 2^-i (i = 0..10) around one of the ten most
    massive clumps, each at 64^3, 128^3 and 256^3, Epanechnikov, h = 0.01 x
    side, one ROI per launch on the resident tree. Per ROI: the launch's time
    from HIP events on its stream and its useful evaluations (untimed count)."""
    import synth
    rois = synth.nested_zoom_rois(info, seed=3)
    stream = torch.cuda.current_stream()
    outs = [torch.empty(r.n_nodes, device="cuda") for r in rois]
    for r, o in zip(rois, outs):
        ctx.eval_roi(tree, r, out=o, stream=stream)
    torch.cuda.synchronize()
    ms = []
    for r, o in zip(rois, outs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = None
        for _ in range(3):
            e0.record(stream)
            ctx.eval_roi(tree, r, out=o, stream=stream)
            e1.record(stream)
            e1.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        ms.append(best)
    useful = [ctx.debug_eval_count(tree, r)[0] for r in rois]
    per_res = {}
    for res in (64, 128, 256):
        idx = [i for i, r in enumerate(rois) if r.res[0] == res]
        t = sum(ms[i] for i in idx)
        u = sum(useful[i] for i in idx)
        per_res["%d^3" % res] = {
            "rois": len(idx), "total_ms": t, "useful_evals": u,
            "evals_per_s": u / (t * 1e-3),
            "frac_of_valu_ceiling": u / (t * 1e-3) * SLOTS_PER_EVAL["epanechnikov"]
                                    / VALU_SLOTS_PER_S,
            "ms_by_side": [round(ms[i], 4) for i in idx]}
    return {"workload": "11 nested boxes (side 1 to 1/1024) around a top-10 clump of the "
                        "resident %s cloud, each at 64^3, 128^3, 256^3; Epanechnikov, "
                        "h = 0.01 x side; one ROI per launch" % label,
            "per_resolution": per_res}


def mbe_rois(ctx, tree, torch, label, info):
    """The paper's adaptive estimator (Eqs. 1-8, particles inside the box
    only) on boxes around the most massive clump of the resident cloud.
    Wall time per ROI (the path reads back Eq. 1's lengths, so it
    synchronises), the evaluation phases from the library's own events, and
    the useful evaluations of the pilot (the Eq. 1 ellipsoid over the
    particles in the box) and of the final grid, counted untimed."""
    import synth
    c = info.centres[int(np.argmax(info.masses))]
    recs = []
    for side in (0.02, 0.05, 0.1):
        lo, hi = synth.box_around(c, side)
        for res in (64, 128):
            roi = synth.Roi(lo, hi, (res, res, res), kernel="epanechnikov", bw="mbe",
                            set="in_roi")
            out = torch.empty(roi.n_nodes, device="cuda")
            ctx.eval_roi(tree, roi, out=out)
            torch.cuda.synchronize()
            ctx.profile_read(reset=True)
            walls = []
            for _ in range(3):
                t0 = time.perf_counter()
                ctx.eval_roi(tree, roi, out=out)
                torch.cuda.synchronize()
                walls.append((time.perf_counter() - t0) * 1e3)
            prof = ctx.profile_read(reset=True)
            d = ctx.debug_mbe(tree, roi, per_particle=False)
            ell0 = [float(v) for v in d["ell0"]]
            pilot_roi = synth.Roi(lo, hi, (res, res, res), kernel="epanechnikov", bw="fixed",
                                  set="in_roi", h=tuple(ell0))
            u_pilot = ctx.debug_eval_count(tree, pilot_roi)[0]
            u_final = ctx.debug_eval_count(tree, roi)[0]
            wall = float(np.median(walls))
            n_ev = max(1, prof["eval_launches"])
            recs.append({
                "side": side, "res": res, "n_b": int(d["n_b"]), "wall_ms": wall,
                "eval_kernels_ms": prof["eval_ms"] * 2 / n_ev,
                "range_query_ms": (prof["tile_count_ms"] + prof["plan_ms"]
                                   + prof["tile_fill_ms"]) * 2 / n_ev,
                "useful_evals_pilot": u_pilot, "useful_evals_final": u_final,
                "evals_per_s": (u_pilot + u_final) / (wall * 1e-3),
                "particles_in_box_per_s": d["n_b"] / (wall * 1e-3)})
    return {"workload": "MBE (Eqs. 1-8, set = particles in B) on boxes of side 0.02, 0.05, "
                        "0.1 around the most massive clump of the resident %s cloud, 64^3 "
                        "and 128^3" % label, "rois": recs}


def adaptive(ctx, tree, torch, label):
    """Adaptive resolution vs a uniform fine grid over the whole cloud: a 64^3
    base grid refined twice (bricks of 8 cells, threshold 0.2 of the peak)
    reaches the spacing of a uniform 253^3 grid inside the refined bricks.
    Epanechnikov, h = 0.01 (fixed, the ROI-scaled value of the unit box)."""
    import synth
    base_res, brick, levels, thr = 64, 8, 2, 0.2
    fine_res = (base_res - 1) * 2 ** levels + 1
    roi = synth.Roi((0, 0, 0), (1, 1, 1), (base_res,) * 3, kernel="epanechnikov", bw="fixed",
                    h=(0.01,) * 3)
    fine = roi.replace(res=(fine_res,) * 3)
    log("adaptive resolution: %d^3 base, %d levels vs uniform %d^3" % (base_res, levels, fine_res))
    fout = torch.empty(fine.n_nodes, device="cuda")
    ctx.eval_roi(tree, fine, out=fout)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.eval_roi(tree, fine, out=fout)
    torch.cuda.synchronize()
    fine_ms = (time.perf_counter() - t0) * 1e3
    ctx.eval_adaptive(tree, roi, brick=brick, max_level=levels, threshold=thr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    base, vals, bricks, info = ctx.eval_adaptive(tree, roi, brick=brick, max_level=levels,
                                                 threshold=thr)
    torch.cuda.synchronize()
    ad_ms = (time.perf_counter() - t0) * 1e3
    nodes = base.numel() + vals.numel()
    # which fine-grid nodes the deepest bricks cover (cell index ranges)
    cover = torch.zeros((fine_res - 1,) * 3, dtype=torch.bool, device="cuda")
    for i, b in enumerate(bricks):
        # the brick's first cell in the fine grid: walk up the parents
        c0 = list(b["cell0"])
        p, lev = b["parent"], b["level"]
        cells = [(r - 1) // 2 for r in b["res"]]
        f0 = [c * 2 ** (levels - lev + 1) for c in c0]
        while p >= 0:
            pb = bricks[p]
            f0 = [f0[k] + pb["cell0"][k] * 2 ** (levels - pb["level"] + 1) for k in range(3)]
            p = pb["parent"]
        if lev == levels:
            span = [cells[k] * 2 ** (levels - lev + 1) for k in range(3)]
            cover[f0[2]:f0[2] + span[2], f0[1]:f0[1] + span[1], f0[0]:f0[0] + span[0]] = True
    fg = fout.view(fine_res, fine_res, fine_res)[:-1, :-1, :-1]
    hot = fg >= 0.1 * float(fout.max())
    coverage = float((hot & cover).sum()) / max(1.0, float(hot.sum()))
    del fout, cover, fg, hot
    torch.cuda.empty_cache()
    per_level = [sum(1 for b in bricks if b["level"] == l) for l in range(1, levels + 1)]
    return {
        "workload": "unit box of the resident %s tree, Epanechnikov, h = 0.01; base %d^3, bricks "
                    "of %d cells, %d levels, threshold %.2f of the peak vs a uniform %d^3 grid"
                    % (label, base_res, brick, levels, thr, fine_res),
        "uniform_fine": {"nodes": fine.n_nodes, "ms": fine_ms},
        "adaptive": {"nodes": int(nodes), "ms": ad_ms, "bricks_per_level": per_level,
                     "complete": info["complete"]},
        "nodes_ratio": nodes / fine.n_nodes, "time_ratio": ad_ms / fine_ms,
        "hot_fine_nodes_in_deepest_bricks": coverage,
    }


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def served_cpu_baseline(pts_host, rois, outs, torch, ctx, tree, seed=11):
    """The FP64 oracle (brute force over every particle of the cloud) on
    sampled nodes of served requests: timed on all the host's threads and on
    one thread, reported as useful evaluations per second (support sizes of
    the sampled nodes from the evaluation kernel's counting pass, which the
    parity tests pin to the oracle's); the oracle values are also compared
    with the served grids."""
    import oracle
    g = np.random.default_rng(seed)
    heavy = int(np.argmax([r.n_nodes * (r.hi[0] - r.lo[0]) ** 3 for r in rois]))
    picks = [heavy] + [int(i) for i in g.choice(len(rois), size=2, replace=False)]
    model, avail = cpu_info()
    threads = int(os.environ.get("OMP_NUM_THREADS", avail))
    threads = max(1, min(threads, avail))
    rec = {"cpu_model": model, "host_threads_available": avail}
    worst = 0.0
    for label, nthr, per_req in (("all_threads", threads, 16), ("one_thread", 1, 2)):
        oracle.set_threads(nthr)
        t_tot, useful_tot, n_nodes = 0.0, 0, 0
        for i in picks:
            r = rois[i]
            got = outs[i].cpu().numpy()
            nodes = np.unique(np.concatenate([
                [int(np.argmax(got))],
                g.choice(r.n_nodes, size=per_req - 1, replace=False)])).astype(np.int64)
            t0 = time.perf_counter()
            ref = oracle.density(pts_host, r, nodes=nodes)
            t_tot += time.perf_counter() - t0
            cnt = ctx.debug_support_counts(tree, r)
            torch.cuda.synchronize()
            useful_tot += int(cnt[torch.from_numpy(nodes).cuda()].double().sum().item())
            n_nodes += len(nodes)
            peak = max(float(ref.max()), float(got.max()))
            big = ref >= 1e-3 * peak
            if big.any():
                worst = max(worst, float(np.max(np.abs(got[nodes][big] - ref[big]) / ref[big])))
        rec[label] = {"value": useful_tot / t_tot, "threads": nthr, "seconds": t_tot,
                      "nodes": n_nodes, "useful_evals": useful_tot}
    oracle.set_threads(threads)
    rec["max_rel_err_served_vs_oracle"] = worst
    a = rec["all_threads"]
    return {"value": a["value"], "unit": "evals/s", "cores": a["threads"], "kind": "oracle",
            "sample": "%d nodes (argmax + random) of 3 served requests (the heaviest + 2 random), "
                      "each brute-forced in FP64 over all %d particles: %.1f s on %d threads; "
                      "1 thread: %.3g evals/s over %d nodes; CPU %s"
                      % (a["nodes"], len(pts_host), a["seconds"], a["threads"],
                         rec["one_thread"]["value"], rec["one_thread"]["nodes"], model),
            "detail": rec}


def served_headline(ctx, torch, args):
    """The served workload: returns (headline fields, sub-record)."""
    import synth
    n = args.serve_points
    W, K = args.warmup, args.steps
    log("drawing %d clumpy points on the device" % n)
    xyz, info = synth.clumpy_cloud_device(n, 5)
    tree = ctx.build_tree(xyz)
    pts_host = None
    if not args.no_cpu_baseline:
        pts_host = xyz.cpu().numpy()
    del xyz
    torch.cuda.empty_cache()
    label = "%dB" % (n // 10**9) if n % 10**9 == 0 else "%dM" % (n // 10**6)
    arr, streams, rois = synth.serving_trace(seed=5, duration_s=float(W + K))
    arr = np.asarray(arr)
    log("trace: %d requests over %d s; counting useful pairs" % (len(rois), W + K))
    useful = np.array([ctx.debug_eval_count(tree, r)[0] for r in rois], dtype=np.int64)
    outs = [torch.empty(r.n_nodes, device="cuda") for r in rois]
    torch.cuda.synchronize()
    free, total = torch.cuda.mem_get_info()
    reserve = args.serve_reserve_gb * 2**30
    budget = max(float(free) - reserve, 1.0)
    win = np.floor(arr).astype(np.int64)
    idx_w = [np.nonzero(win == w)[0] for w in range(W + K)]

    def serve_window(w, mode):
        ids = idx_w[w]
        res, s = ctx.serve(tree, np.zeros(len(ids)), [rois[i] for i in ids],
                           [outs[i] for i in ids], mode=mode, n_slots=4, max_batch=64,
                           budget_bytes=budget)
        return s

    # warm-up steps, then the same seconds one ROI per launch in FIFO order
    # (an untimed comparison at saturation), then the timed region:
    # continuous batching at saturation
    for w in range(W):
        if args.profile_served:
            break  # counter runs: only the timed windows (the same seconds of the trace)
        serve_window(w, 0)
        log("warm-up step", w + 1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if not args.profile_served:
        for w in range(W, W + K):
            serve_window(w, 1)
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t1
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batches = 0
    for w in range(W, W + K):
        batches += serve_window(w, 0).n_batches
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    timed = np.concatenate(idx_w[W:W + K])
    e_timed = int(useful[timed].sum())
    log("timed %d steps (%d requests) in %.3f s" % (K, len(timed), dt))
    eval_ms = prof["eval_ms"]
    launches = max(1, prof["eval_launches"])
    slots = SLOTS_PER_EVAL["epanechnikov"] * e_timed
    achieved = slots / (eval_ms * 1e-3) / 1e12
    peak = VALU_SLOTS_PER_S / 1e12
    # the same seconds again on one stream (no batch overlaps another), so
    # each phase's event-timed duration is its own: an untimed breakdown
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    t2 = time.perf_counter()
    for w in range(W, W + K) if not args.profile_served else ():
        ids = idx_w[w]
        ctx.serve(tree, np.zeros(len(ids)), [rois[i] for i in ids], [outs[i] for i in ids],
                  mode=0, n_slots=1, max_batch=64, budget_bytes=budget)
    torch.cuda.synchronize()
    dt2 = time.perf_counter() - t2
    prof1 = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    sub = {
        "workload": "%d requests in %d s of a trace from 8 streams at 90 Hz on the resident "
                    "%s-point tree; sides log-uniform in [1e-4, 1], grids 32^3-128^3, "
                    "Epanechnikov, h = 0.01 x side" % (len(rois), W + K, label),
        "admission_budget_bytes": budget, "hbm_free_bytes": float(free),
        "saturated": {
            "continuous_batching": {"evals_per_s": e_timed / dt, "ms_per_second_of_trace":
                                    dt * 1e3 / K, "batches": batches,
                                    "requests": int(len(timed))},
            "one_roi_per_launch": None if args.profile_served else {
                "evals_per_s": e_timed / dt1, "ms_per_second_of_trace": dt1 * 1e3 / K},
            "throughput_ratio": None if args.profile_served else dt1 / dt},
        "phases_ms_per_step_4_streams": {k: prof[k] / K for k in (
            "tile_count_ms", "plan_ms", "tile_fill_ms", "eval_ms")},
        "one_stream": None if args.profile_served else {
            "evals_per_s": e_timed / dt2, "ms_per_second_of_trace": dt2 * 1e3 / K,
            "phases_ms_per_step": {k: prof1[k] / K for k in (
                "tile_count_ms", "plan_ms", "tile_fill_ms", "eval_ms")},
            "eval_frac_of_valu_ceiling": SLOTS_PER_EVAL["epanechnikov"] * e_timed
                                         / (prof1["eval_ms"] * 1e-3) / VALU_SLOTS_PER_S,
            "note": "batches one after another on one stream: each phase's HIP-event "
                    "duration is its own (on 4 streams a batch's events also span the "
                    "other streams' kernels that share the device)"},
        "eval_launches": int(prof["eval_launches"]),
    }
    if not args.no_realtime:
        budget_ms = 1000.0 / 90.0
        # continuous batching last, so the grids checked below are its results
        for name, mode in (("one_roi_per_launch", 1), ("continuous_batching", 0)):
            log("real-time replay at 90 Hz:", name)
            res, sm = ctx.serve(tree, arr, rois, outs, mode=mode, n_slots=4, max_batch=64,
                                budget_bytes=budget)
            lat = np.array([res[i].latency_ms for i in range(len(rois))])
            meas = arr >= W
            done = np.array([res[i].done_s for i in range(len(rois))])
            span = float(done[meas].max() - W)
            sub.setdefault("realtime_90hz", {})[name] = {
                "p50_ms": float(np.percentile(lat[meas], 50)),
                "p99_ms": float(np.percentile(lat[meas], 99)),
                "max_ms": float(lat[meas].max()),
                "deadline_miss_rate": float(np.mean(lat[meas] > budget_ms)),
                "evals_per_s": float(useful[meas].sum()) / span,
                "requests": int(meas.sum()), "batches": int(sm.n_batches),
                "mean_batch": sm.mean_batch, "mean_in_flight": sm.mean_in_flight,
                "budget_waits": int(sm.budget_waits)}
        sub["realtime_90hz"]["frame_budget_ms"] = budget_ms
        # the same stream statistics at three times the load (24 streams):
        # where requests queue, continuous batching's concurrency shows
        arr3, _, rois3 = synth.serving_trace(seed=6, duration_s=5.0, n_streams=24)
        arr3 = np.asarray(arr3)
        outs3 = [torch.empty(r.n_nodes, device="cuda") for r in rois3]
        rec3 = {"workload": "%d requests in 5 s from 24 streams at 90 Hz (3x the load; the first "
                            "second is warm-up), same request statistics" % len(rois3)}
        for name, mode in (("one_roi_per_launch", 1), ("continuous_batching", 0)):
            log("real-time replay at 3x load:", name)
            res, sm = ctx.serve(tree, arr3, rois3, outs3, mode=mode, n_slots=4, max_batch=64,
                                budget_bytes=budget)
            lat = np.array([res[i].latency_ms for i in range(len(rois3))])
            meas = arr3 >= 1.0
            rec3[name] = {"p50_ms": float(np.percentile(lat[meas], 50)),
                          "p99_ms": float(np.percentile(lat[meas], 99)),
                          "max_ms": float(lat[meas].max()),
                          "deadline_miss_rate": float(np.mean(lat[meas] > budget_ms)),
                          "requests": int(meas.sum()), "mean_batch": sm.mean_batch}
        sub["realtime_90hz_3x_load"] = rec3
        del outs3
        torch.cuda.empty_cache()
    # served grids (real-time continuous batching, else the saturated run)
    # against each request evaluated alone, bitwise
    g = np.random.default_rng(12)
    check = sorted(set(int(i) for i in g.choice(len(rois), size=48, replace=False))
                   | set(int(i) for i in np.argsort(-useful)[:8]))
    if args.profile_served:
        check = []
    alone = torch.empty(max(r.n_nodes for r in rois), device="cuda")
    same = True
    for i in check:
        o = ctx.eval_roi(tree, rois[i], out=alone[:rois[i].n_nodes])
        torch.cuda.synchronize()
        same &= bool(torch.equal(o, outs[i]))
    sub["bitwise_alone_vs_served"] = {"requests_checked": len(check), "equal": same}
    head = {
        "value": e_timed / dt, "ms_per_step": dt * 1e3 / K, "useful_evals": e_timed,
        "roofline": {"bound": "alu",
                     "kernel": "evaluation (k_eval tiles, k_splat bricks, k_sweep particle "
                               "sweep; Epanechnikov, "
                               "uniform bandwidth)",
                     "achieved": achieved, "peak": peak, "unit": "T VALU-slot/s",
                     "frac": achieved / peak, "traffic": measured_traffic(SERVED_TRAFFIC_FILE),
                     "slots_per_eval": SLOTS_PER_EVAL["epanechnikov"],
                     "evals_per_launch": e_timed / launches,
                     "avg_launch_ms": eval_ms / launches, "launches": int(launches),
                     "note": "achieved = 9 slots x useful evaluations of the timed steps / "
                             "summed evaluation-kernel durations (HIP events on each batch's "
                             "stream; batches on the 4 streams overlap, so a duration also "
                             "covers other streams' kernels: serving.one_stream gives the "
                             "same seconds without overlap); traffic from the committed "
                             "counter summary while the kernel sources match"},
    }
    if pts_host is not None:
        log("timing the oracle on sampled nodes of served requests")
        head["cpu_baseline"] = served_cpu_baseline(pts_host, rois, outs, torch, ctx, tree)
    tree.close()
    del outs, alone
    torch.cuda.empty_cache()
    return head, sub


def per_point_section(ctx, torch, args):
    """The 10M-point per-point Gaussian step: tree build + k-NN bandwidths +
    range query + evaluation of the unit-box 128^3 grid, from points resident
    in HBM (its own roofline: the per-ROI evaluation kernel)."""
    pts, roi, knn_k, config = workload("per_point_10m")
    xyz = torch.from_numpy(pts).cuda()
    out = torch.empty(roi.n_nodes, device="cuda")
    ctx.profile_enable(True)

    def step():
        tree = ctx.build_tree(xyz, knn_k=knn_k)
        ctx.eval_roi(tree, roi, out=out)
        return tree

    for _ in range(2):
        step().close()
        torch.cuda.synchronize()
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    steps = args.per_point_steps
    t0 = time.perf_counter()
    for i in range(steps):
        tree = step()
        if i + 1 < steps:
            tree.close()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    useful, tested = ctx.debug_eval_count(tree, roi)
    eval_ms = prof["eval_ms"] / max(1, prof["eval_launches"])
    slots = SLOTS_PER_EVAL[roi.kernel] * useful
    achieved = slots / (eval_ms * 1e-3) / 1e12
    peak = VALU_SLOTS_PER_S / 1e12
    rec = {
        "config": config, "steps": steps, "ms_per_step": dt * 1e3 / steps,
        "evals_per_s": useful * steps / dt,
        "roofline": {"bound": "alu", "kernel": "k_eval<4,4,4,gauss,per-point>",
                     "achieved": achieved, "peak": peak, "unit": "T VALU-slot/s",
                     "frac": achieved / peak, "traffic": measured_traffic(),
                     "slots_per_eval": SLOTS_PER_EVAL[roi.kernel], "evals_per_launch": useful,
                     "avg_launch_ms": eval_ms},
        "phases_ms": {k: prof[k] / steps for k in
                      ("build_ms", "knn_ms", "tile_count_ms", "plan_ms", "tile_fill_ms",
                       "eval_ms")},
        "dominant_kernel": {
            "kernel": "k_knn<32>", "ms_per_step": prof["knn_ms"] / steps,
            "share_of_step": prof["knn_ms"] / steps / (dt * 1e3 / steps),
            "bound": "alu (VALU instruction issue)",
            "valu_busy_profiled": profiled_valu_busy("k_knn<32>")},
        "eval_only_evals_per_s": useful / (eval_ms * 1e-3),
        "useful_evals": useful, "tested_pairs": tested,
        "candidate_leaves": prof["last_total_leaves"], "work_items": prof["last_items"],
        "consumers": consumers(ctx, torch, roi, out, xyz),
    }
    tree.close()
    del xyz, out
    torch.cuda.empty_cache()
    return rec


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2601_20758_amd as sfk

    if args.copy_calibration:
        # reference kernels of known traffic for the byte counters: a fill
        # writes 1 GiB; an elementwise scale reads 1 GiB and writes 1 GiB
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    ctx = sfk.Context(0)
    if args.profile_section:
        def only(t, lab, info):
            if args.profile_section == "batch":
                return {"batch_vs_single": batch_vs_single(ctx, t, torch, args.n_batch, lab)}
            return {"nested_zoom": nested_zoom(ctx, t, torch, lab, info)}
        rec = large_section(ctx, torch, args.batch_points, 3, only)
        ctx.close()
        print(json.dumps({"profile_section": args.profile_section, **rec}), flush=True)
        return
    result = {"metric": METRIC, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    if args.workload == "served_1b":
        head, sub = served_headline(ctx, torch, args)
        result.update({"value": head["value"], "ms_per_step": head["ms_per_step"],
                       "config": {"workload": "served request loop, 1B clustered points "
                                              "(tree resident), 8 VR streams x 90 Hz, sides "
                                              "log-uniform 1e-4..1, grids 32^3-128^3, "
                                              "Epanechnikov, h = 0.01 x side, HBM-budget "
                                              "admission; step = 1 s of the trace served at "
                                              "saturation by continuous batching",
                                  "n_points": args.serve_points,
                                  "trace_seconds": args.warmup + args.steps,
                                  "particle_order": "hilbert"},
                       "roofline": head["roofline"], "useful_evals": head["useful_evals"]})
        if "cpu_baseline" in head:
            result["cpu_baseline"] = head["cpu_baseline"]
        result["serving"] = sub
        if not args.no_per_point:
            log("sub-record: 10M per-point step")
            result["per_point_10m"] = per_point_section(ctx, torch, args)
    else:
        pts, roi, knn_k, config = workload(args.workload)
        xyz = torch.from_numpy(pts).cuda()
        out = torch.empty(roi.n_nodes, device="cuda")
        ctx.profile_enable(True)

        def step():
            tree = ctx.build_tree(xyz, knn_k=knn_k)
            ctx.eval_roi(tree, roi, out=out)
            return tree

        for i in range(args.warmup):
            step().close()
            torch.cuda.synchronize()
        ctx.profile_read(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            tree = step()
            if i + 1 < args.steps:
                tree.close()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = ctx.profile_read(reset=True)
        useful, tested = ctx.debug_eval_count(tree, roi)
        eval_ms = prof["eval_ms"] / max(1, prof["eval_launches"])
        achieved = SLOTS_PER_EVAL[roi.kernel] * useful / (eval_ms * 1e-3) / 1e12
        peak = VALU_SLOTS_PER_S / 1e12
        result.update({"value": useful * args.steps / dt, "ms_per_step": dt * 1e3 / args.steps,
                       "config": config,
                       "roofline": {"bound": "alu", "kernel": "k_eval", "achieved": achieved,
                                    "peak": peak, "unit": "T VALU-slot/s",
                                    "frac": achieved / peak,
                                    "traffic": measured_traffic() if knn_k else None,
                                    "slots_per_eval": SLOTS_PER_EVAL[roi.kernel],
                                    "evals_per_launch": useful, "avg_launch_ms": eval_ms},
                       "useful_evals": useful, "tested_pairs": tested})
        if not args.no_cpu_baseline:
            h2 = ctx.debug_point_h2(tree) if knn_k else None
            log("timing the oracle on a node sample")
            result["cpu_baseline"] = cpu_baseline(pts, roi, h2, args.cpu_sample_nodes)
        tree.close()
        del xyz, out
        torch.cuda.empty_cache()
    if args.workload != "small" and not (args.no_batch and args.no_zoom and not args.view):
        def on_100m(t, lab, info):
            rec = {}
            if not args.no_batch:
                rec["batch_vs_single"] = batch_vs_single(ctx, t, torch, args.n_batch, lab)
            if args.view:
                rec["view_cache"] = view_cache(ctx, t, torch, lab, info)
                rec["adaptive_resolution"] = adaptive(ctx, t, torch, lab)
            if not args.no_zoom:
                rec["nested_zoom"] = nested_zoom(ctx, t, torch, lab, info)
                ctx.profile_enable(True)
                rec["mbe"] = mbe_rois(ctx, t, torch, lab, info)
                ctx.profile_enable(False)
            return rec
        rec = large_section(ctx, torch, args.batch_points, 3, on_100m)
        if "error" in rec:
            result["batch_vs_single"] = rec
        else:
            result.update(rec)
    ctx.close()
    print(json.dumps(result), flush=True)


def large_section(ctx, torch, n, seed, fn):
    """Run fn(tree, label, clump_info) on a clumpy cloud of n points drawn on
    the device (tree built outside any timed region); errors are reported,
    not hidden."""
    import synth
    try:
        log("drawing %d clumpy points on the device" % n)
        xyz, info = synth.clumpy_cloud_device(n, seed)
        tree = ctx.build_tree(xyz)
        del xyz
        torch.cuda.empty_cache()
        label = "%s-point" % ("%dB" % (n // 10**9) if n % 10**9 == 0 else "%dM" % (n // 10**6))
        rec = fn(tree, label, info)
        tree.close()
        torch.cuda.empty_cache()
        return rec
    except Exception as e:  # report, never hide
        return {"error": repr(e)}


if __name__ == "__main__":
    main()
