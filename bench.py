#!/usr/bin/env python
"""Benchmark: ms per frame of the GN-PCG halfway-domain solve at 640x480.

One "step" is one whole solve of one frame (pyramid, 5 levels x 10
Gauss-Newton steps x 20 PCG iterations, step control, depth/3D-flow output)
with the four input images already resident in device memory.  Prints one
JSON line.  Besides the headline number it reports the roofline of the
dominant kernel (the PCG iteration's H p at the finest level: node blocks
by default, matrix-free with --apply-mode 0; timed live with HIP events on
the solver's stream) and, unless
--no-cpu-baseline, the FP64 CPU oracle timed on a bounded sample of the
same workload on the host.
"""
import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = ("ms/frame GN-PCG solve at 640x480 + HBM GB/s; learned-init vs "
          "plain at equal EPE")
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "vga": dict(desc="640x480 float32 quadruple, smooth Gaussian depth 1.5-4 m, "
                     "4-octave value-noise texture, smooth 3D motion up to 30 px, "
                     "noise sigma 0.01",
                width=640, height=480, seed=1,
                params=dict(levels=5, grid_stride=4, gn_iters=10, pcg_iters=20)),
    "tiny": dict(desc="64x48 translating textured plane",
                 width=64, height=48, seed=0,
                 params=dict(levels=3, grid_stride=8, gn_iters=5, pcg_iters=10)),
    "hd": dict(desc="1280x720 float32 quadruple, up to 80 px displacement, two "
                    "moving blobs",
               width=1280, height=720, seed=2,
               params=dict(levels=6, grid_stride=4, gn_iters=10, pcg_iters=20)),
    "learned": dict(desc="learned-init vs plain at equal EPE: 16 held-out 640x480 "
                         "generator frames (seeds 1000000..1000015, 30 px displacement); "
                         "target = mean EPE of the plain solver (zero initialisation) at "
                         "10 GN x 20 PCG per level; plain and learned (the stored "
                         "initialiser, trained on 256 frames, seeds 0..255, with the energy "
                         "fallback) each at the fewest GN steps per level reaching it; "
                         "stride 4, 5 levels",
                    width=640, height=480, n_eval=16, weights="init_640x480.npy",
                    params=dict(levels=5, grid_stride=4, gn_iters=10, pcg_iters=20)),
    "learned_hd": dict(desc="learned-init vs plain at equal EPE: 100 held-out 1280x720 "
                            "generator frames (seeds 1000000..1000099, 80 px displacement, "
                            "two moving blobs); target = mean EPE of the plain solver (zero "
                            "initialisation) at 10 GN x 20 PCG per level; plain and learned "
                            "(the stored 1280x720 initialiser, trained on 2000 frames, seeds "
                            "0..1999, with the energy fallback) each at the fewest GN steps "
                            "per level reaching it; stride 4, 6 levels",
                       width=1280, height=720, n_eval=100, weights="init_1280x720.npy",
                       max_disp=80.0, blobs=2,
                       params=dict(levels=6, grid_stride=4, gn_iters=10, pcg_iters=20)),
    "batch": dict(desc="batches of 64 frames, resolutions drawn by seed 3 from "
                       "320x240 / 640x480 / 960x540 / 1280x720 (4 / 5 / 5 / 6 "
                       "levels: 1 + floor(log2(W / 40))), displacement 30 px per "
                       "640 px of width, noise sigma 0.01, two generator scenes "
                       "per resolution reused across the batch; stride 4, "
                       "10 GN x 20 PCG, one HIP graph per batch",
                  n_frames=64, seed=3,
                  params=dict(levels=6, grid_stride=4, gn_iters=10, pcg_iters=20)),
    "batch_learned": dict(desc="learned-init + batched vs plain batched at equal EPE: the "
                               "batched workload's 64 frames (320x240 frames have 4 levels "
                               "and start from zero; the others run the network); target = "
                               "mean EPE of plain batches (zero initialisation) at 10 GN x "
                               "20 PCG per level; plain and learned batches each at the "
                               "fewest GN steps per level reaching it",
                          weights="init_640x480.npy"),
    "video": dict(desc="video mode vs plain at equal EPE: a 10-frame constant-velocity "
                       "640x480 generator sequence (seed 5, 30 px displacement per frame, "
                       "independent noise per frame); plain = every frame from zero, "
                       "10 GN x 20 PCG per level; video = each level's deltas from the "
                       "previous frame, fewest GN steps per level reaching the plain EPE "
                       "over frames 1..9 (frame 0 starts the sequence); stride 4, 5 levels",
                  width=640, height=480, seed=5, n_frames=10,
                  params=dict(levels=5, grid_stride=4, gn_iters=10, pcg_iters=20)),
    "illum": dict(desc="illumination correction on/off: 8 640x480 generator frames "
                       "(seeds 2000000..2000007, 30 px displacement) whose right camera "
                       "responds with gain 1.08, offset 0.06 and a horizontal ramp of 0.08; "
                       "EPE and ms/frame of the plain and the corrected solve; stride 4, "
                       "5 levels, 10 GN x 20 PCG",
                  width=640, height=480, n_eval=8, gain=1.08, bias=0.06, ramp=0.08,
                  params=dict(levels=5, grid_stride=4, gn_iters=10, pcg_iters=20)),
    "occlusion": dict(desc="occlusion maps on/off: 8 640x480 generator frames (seeds "
                           "3000000..3000007, 30 px displacement, two moving blobs); EPE "
                           "and ms/frame of the solve without and with the maps; stride 4, "
                           "5 levels, 10 GN x 20 PCG",
                      width=640, height=480, n_eval=8,
                      params=dict(levels=5, grid_stride=4, gn_iters=10, pcg_iters=20)),
}

# Bytes one PCG iteration kernel (H u plus the vector updates) must move per
# node at level 0, counting every value it loads or stores once.  Node
# vectors are packed 6-float records (24 B): it reads
# r, w, s, diag (for u and the halo) and u, x, p (the owned node), and writes
# s, r, w, p, x, u; plus the 16-float regulariser record.
VEC_BYTES = 6 * 4
APPLY_BYTES_PER_NODE = (7 + 6) * VEC_BYTES + 16 * 4          # 376 B
# matrix-free products: the 21 distinct floats of each pixel's
# Gauss-Newton block on top of the node traffic
APPLY_BYTES_PER_PIXEL = 21 * 4
# node-block products: the five stored 21-float blocks per node (self, E,
# S, SE, SW) on top of the node traffic: 420 + 376 = 796 B per node
APPLY_NB_BYTES_PER_NODE = 5 * 21 * 4 + APPLY_BYTES_PER_NODE
# the batched instantiation rebuilds u of the previous iteration as r / diag
# from the records it reads anyway and neither reads nor writes u: 48 B
# less per node (node blocks: 748 B)
APPLY_BATCH_SAVED_PER_NODE = 2 * VEC_BYTES


def apply_bytes(N0, G0, apply_mode, batched=False):
    node = APPLY_BYTES_PER_NODE - (APPLY_BATCH_SAVED_PER_NODE if batched else 0)
    if apply_mode >= 1:
        return (APPLY_NB_BYTES_PER_NODE - APPLY_BYTES_PER_NODE + node) * G0
    return APPLY_BYTES_PER_PIXEL * N0 + node * G0


def describe(desc, params):
    """Workload description with the schedule actually run."""
    gn = f"{params['gn_iters']} GN"
    if params.get("gn_fine"):
        gn = f"{params['gn_fine']} GN on the two finest levels and {params['gn_iters']} GN"
    return (f"{desc}; stride {params['grid_stride']}, {params['levels']} levels, "
            f"{gn} x {params['pcg_iters']} PCG")


def _gen_frame(args):
    from synth import make_frame, sized_config
    W, H, seed, truth = args
    imgs, calib, scene = make_frame(sized_config(W, H), seed)
    if truth:
        pos, ok = scene.halfway_truth()
        return imgs, calib, (pos.astype(np.float32), ok)
    return imgs, calib


def make_batch_workload(w, truth=False):
    """Frames of the batched workload: per-frame resolutions from the seed,
    images from two generator scenes per resolution (rendered in parallel
    on the host); with truth, each frame also carries the generator's
    halfway correspondences."""
    from concurrent.futures import ProcessPoolExecutor
    from synth import batch_resolutions
    res = batch_resolutions(w["n_frames"], w["seed"])
    jobs = sorted({(W, H, 100 + 10 * k + j) for k, (W, H) in enumerate(sorted(set(res)))
                   for j in range(2)})
    with ProcessPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        out = dict(zip(jobs, ex.map(_gen_frame, [j + (truth,) for j in jobs])))
    frames, count = [], {}
    for W, H in res:
        j = count.get((W, H), 0)
        count[(W, H)] = j + 1
        key = next(k for k in jobs if k[0] == W and k[1] == H and (k[2] % 10) == j % 2)
        frames.append(out[key])
    return res, frames


KERNEL_SOURCE = os.path.join(ROOT, "paper_1610_07159_amd", "csrc", "sf_kernels.hip")


def source_hash():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(workload, apply_mode, prefix):
    """(name, HBM bytes per launch) of the level-0 PCG iteration kernel the
    run timed, from the committed counter summary
    (profiles/pcg_apply_<workload>[_nb]_traffic.txt): of the kernels whose
    name starts with `prefix` (k_pcg<B, false, S, V, the last template
    argument, WD, follows from the launch's size), the one of the largest
    launch grid, which is level 0.  (None, None) if the summary is missing,
    lacks such a kernel or was taken on a different kernel source."""
    tag = "_nb" if apply_mode >= 1 else ""
    path = os.path.join(ROOT, "profiles", f"pcg_apply_{workload}{tag}_traffic.txt")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        return traffic_lookup(f.read().splitlines(), prefix, source_hash())


def traffic_lookup(lines, prefix, sha):
    """The (name, bytes per launch) entry of a counter summary (the lines
    `bench.py --traffic` prints) for the kernel starting with `prefix` of
    the largest launch grid; (None, None) unless the summary was taken on
    kernel source `sha` and holds such a kernel."""
    vals, grids = {}, {}
    for line in lines:
        m = re.match(r"# (k_pcg<[^>]*>), launch grid (\d+) threads", line)
        if m:
            grids[m.group(1)] = int(m.group(2))
        elif "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != sha:
        return None, None
    names = [k for k in grids if k.startswith(prefix + ",")
             and f"traffic_bytes_per_launch[{k}]" in vals]
    if not names:
        return None, None
    name = max(names, key=lambda k: grids[k])
    return name, int(vals[f"traffic_bytes_per_launch[{name}]"])


def pcg_kernel_prefix(batched, apply_mode, stride, variant):
    """The PCG iteration kernel k_pcg<B, FIRST, S, V, WD> as the traces and
    counter summaries print it, up to its last template argument."""
    S = 0 if apply_mode >= 1 else stride
    return f"k_pcg<{'true' if batched else 'false'}, false, {S}, {variant}"


def equal_epe_sweeps(run, full):
    """Equal-EPE comparison of the learned initialisation with the plain
    solver.  The target is the plain solver's mean EPE at the full schedule
    (`full` Gauss-Newton steps per level); for each method the number of
    steps per level is swept upward from 1 and the first (fastest) setting
    whose mean EPE reaches the target is reported.  run(init_mode, n)
    returns (mean EPE, result row)."""
    target, full_row = run(0, full)
    out = {"target_epe_px": round(target, 4), "plain_full_schedule": full_row}
    for name, mode in (("plain", 0), ("learned", 1)):
        sweep, reach = [], None
        for n in range(1, full + 1):
            if mode == 0 and n == full:
                e, row = target, full_row
            else:
                e, row = run(mode, n)
            sweep.append(row)
            if e <= target:
                reach = row
                break
        out[name + "_sweep"] = sweep
        out[name + "_at_target"] = reach
    p, l = out["plain_at_target"], out["learned_at_target"]
    out["speedup_at_equal_epe"] = (round(p["ms_per_frame"] / l["ms_per_frame"], 3)
                                   if p and l else None)
    return out


def single_frame_runner(frames, W, H, params, weights):
    """run(init_mode, n) of equal_epe_sweeps for single-frame solves of
    rendered frames (GPU time per frame, graph replay)."""
    from paper_1610_07159_amd import train_init as T

    def run(init_mode, n):
        fl, used, ms = T.solve_flows(frames, W, H, init_mode=init_mode,
                                     weights=weights if init_mode else None, timed=True,
                                     **dict(params, gn_iters=n))
        e = float(np.mean([T.epe(f, fr["truth"], W, H) for f, fr in zip(fl, frames)]))
        row = dict(gn_iters=n, epe_px=round(e, 4), ms_per_frame=round(ms, 3))
        if init_mode:
            row["prediction_kept"] = int(sum(used))
        return e, row
    return run


def learned_vs_plain(solver_params, frames):
    """Compact equal-EPE comparison for the headline line (see --workload
    learned); frames rendered beforehand."""
    weights = np.load(os.path.join(ROOT, "paper_1610_07159_amd", "weights", "init_640x480.npy"),
                      allow_pickle=False)
    r = equal_epe_sweeps(single_frame_runner(frames, 640, 480, solver_params, weights),
                         solver_params["gn_iters"])
    p, l = r["plain_at_target"], r["learned_at_target"]
    return dict(eval_frames=len(frames), target_epe_px=r["target_epe_px"],
                plain_gn_iters=p["gn_iters"], plain_epe_px=p["epe_px"],
                plain_ms_per_frame=p["ms_per_frame"],
                learned_gn_iters=l["gn_iters"] if l else None,
                learned_epe_px=l["epe_px"] if l else None,
                learned_ms_per_frame=l["ms_per_frame"] if l else None,
                prediction_kept=l["prediction_kept"] if l else None,
                speedup=r["speedup_at_equal_epe"])


def _render_video_frame(args):
    from synth import Scene, vga_config
    seed, k = args
    sc = Scene(vga_config(), seed)
    sc.noise_rng = np.random.default_rng((seed, k))
    imgs = sc.render(t0=k)
    pos, ok = sc.halfway_truth(t0=k)
    return imgs, (pos.astype(np.float32), ok)


def make_video_workload(w):
    """Frames and per-frame truth of the video workload (host processes,
    before anything touches the GPU)."""
    from concurrent.futures import ProcessPoolExecutor
    from synth import Scene, vga_config, calib_of
    with ProcessPoolExecutor(max_workers=8) as ex:
        out = list(ex.map(_render_video_frame, [(w["seed"], k) for k in range(w["n_frames"])]))
    return out, calib_of(Scene(vga_config(), w["seed"]))


def _render_illum_frame(args):
    from dataclasses import replace
    from synth import Scene, vga_config
    seed, gain, bias, ramp = args
    sc = Scene(replace(vga_config(), right_gain=gain, right_bias=bias, right_ramp=ramp), seed)
    pos, ok = sc.halfway_truth()
    from synth import calib_of
    return sc.render(), calib_of(sc), (pos.astype(np.float32), ok)


def make_illum_workload(w):
    from concurrent.futures import ProcessPoolExecutor
    jobs = [(2_000_000 + k, w["gain"], w["bias"], w["ramp"]) for k in range(w["n_eval"])]
    with ProcessPoolExecutor(max_workers=8) as ex:
        return list(ex.map(_render_illum_frame, jobs))


def _render_blob_frame(seed):
    from dataclasses import replace
    from synth import Scene, vga_config, calib_of
    sc = Scene(replace(vga_config(), n_blobs=2), seed)
    pos, ok = sc.halfway_truth()
    return sc.render(), calib_of(sc), (pos.astype(np.float32), ok)


def make_occlusion_workload(w):
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=8) as ex:
        return list(ex.map(_render_blob_frame, [3_000_000 + k for k in range(w["n_eval"])]))


def run_toggle(args, frames, name, flag, labels):
    """EPE and time of the solve with one option off and on (illumination
    correction on frames whose right camera has a different response;
    occlusion maps on frames with moving blobs)."""
    import torch
    from paper_1610_07159_amd import SceneFlowSolver
    from paper_1610_07159_amd import train_init as T
    w = WORKLOADS[name]
    W, H = w["width"], w["height"]
    params = dict(w["params"], apply_mode=args.apply_mode)
    dev = [torch.from_numpy(f).cuda().contiguous() for f, _, _ in frames]
    out_rows = {}
    for on in (0, 1):
        solver = SceneFlowSolver(W, H, exec_mode=args.exec_mode, tile_mode=args.tile_mode,
                                 **{flag: on}, **params)
        out = (torch.empty((H, W), device="cuda"), torch.empty((3, H, W), device="cuda"),
               torch.empty((6, H, W), device="cuda"))
        try:
            solver.solve(dev[0], frames[0][1], out=out)  # warm-up (graph, tiles)
            epes, times = [], []
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            for img, (_, calib, truth) in zip(dev, frames):
                e0.record(solver.stream)
                solver.solve(img, calib, out=out)
                e1.record(solver.stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
                epes.append(T.epe(out[2].cpu().numpy(), truth, W, H))
        finally:
            solver.close()
        out_rows[labels[on]] = dict(
            epe_px=round(float(np.mean(epes)), 4), ms_per_frame=round(float(np.mean(times)), 3))
    result = {
        "metric": METRIC,
        "value": out_rows[labels[1]]["ms_per_frame"],
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": len(dev),
        "warmup": 1,
        "ms_per_step": out_rows[labels[1]]["ms_per_frame"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["desc"], **params},
        **out_rows,
    }
    print(json.dumps(result), flush=True)


def run_video(args, workload):
    """Equal-EPE comparison of video mode with plain per-frame solves."""
    import torch
    from paper_1610_07159_amd import SceneFlowSolver
    from paper_1610_07159_amd import train_init as T
    w = WORKLOADS["video"]
    W, H = w["width"], w["height"]
    frames, calib = workload
    params = dict(w["params"], apply_mode=args.apply_mode)
    dev = [torch.from_numpy(f).cuda().contiguous() for f, _ in frames]

    def run(temporal, n_gn):
        solver = SceneFlowSolver(W, H, exec_mode=args.exec_mode, tile_mode=args.tile_mode,
                                 temporal=temporal, **dict(params, gn_iters=n_gn))
        out = (torch.empty((H, W), device="cuda"), torch.empty((3, H, W), device="cuda"),
               torch.empty((6, H, W), device="cuda"))
        try:
            solver.solve(dev[0], calib, out=out)  # warm-up (graph, tiles)
            if temporal:
                solver.reset_sequence()
            epes, times = [], []
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            for k, img in enumerate(dev):
                e0.record(solver.stream)
                solver.solve(img, calib, out=out)
                e1.record(solver.stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
                epes.append(T.epe(out[2].cpu().numpy(), frames[k][1], W, H))
        finally:
            solver.close()
        return epes, times

    plain_epe, plain_ms = run(0, params["gn_iters"])
    e_plain = float(np.mean(plain_epe[1:]))
    ms_plain = float(np.mean(plain_ms[1:]))
    sweep, reach = [], None
    for n in range(1, params["gn_iters"] + 1):
        epes, ms = run(1, n)
        e = float(np.mean(epes[1:]))
        sweep.append(dict(gn_iters=n, epe_px=round(e, 4), ms_per_frame=round(float(np.mean(ms[1:])), 3),
                          first_frame_epe_px=round(epes[0], 4)))
        if e <= e_plain:
            reach = sweep[-1]
            break
    result = {
        "metric": METRIC,
        "value": reach["ms_per_frame"] if reach else None,
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": len(dev) - 1,
        "warmup": 1,
        "ms_per_step": reach["ms_per_frame"] if reach else None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["desc"], **params},
        "plain": {"gn_iters": params["gn_iters"], "epe_px": round(e_plain, 4),
                  "ms_per_frame": round(ms_plain, 3)},
        "video_sweep": sweep,
        "equal_epe": (dict(gn_iters=reach["gn_iters"], ms_per_frame=reach["ms_per_frame"],
                           speedup=round(ms_plain / reach["ms_per_frame"], 3))
                      if reach else None),
    }
    print(json.dumps(result), flush=True)


def make_workload(name):
    from synth import make_frame, vga_config, hd_config, tiny_plane_config
    w = WORKLOADS[name]
    cfg = {"vga": vga_config, "hd": hd_config, "tiny": tiny_plane_config}[name]()
    imgs, calib, scene = make_frame(cfg, w["seed"])
    return w, imgs, calib, scene


def level_sizes(W, H, levels, s):
    out = []
    for l in range(levels):
        w, h = W >> l, H >> l
        gx, gy = -(-w // s), -(-h // s)
        out.append((w, h, w * h, gx * gy))
    return out


def epe(flows, scene, W, H):
    """Mean over valid halfway pixels of the mean endpoint error of the four
    correspondences against the generator's ground truth (px)."""
    pos, ok = scene.halfway_truth()
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    signs = np.array([[-1, -1, 1], [1, -1, -1], [-1, 1, -1], [1, 1, 1]], np.float64)
    err = np.zeros((H, W))
    inside = ok.copy()
    for c in range(4):
        px = xx + signs[c, 0] * flows[0] + signs[c, 1] * flows[2] + signs[c, 2] * flows[4]
        py = yy + signs[c, 0] * flows[1] + signs[c, 1] * flows[3] + signs[c, 2] * flows[5]
        err += np.hypot(px - pos[c, 0], py - pos[c, 1])
        inside &= (pos[c, 0] >= 0) & (pos[c, 0] <= W - 1) & (pos[c, 1] >= 0) & (pos[c, 1] <= H - 1)
    return float((err / 4.0)[inside].mean())


def cpu_model():
    """The host CPU's model name and logical CPU count (from /proc/cpuinfo)."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, os.cpu_count()


def _oracle_solve_seconds(imgs, calib, params, gn_iters, threads):
    from threadpoolctl import threadpool_limits
    import dataclasses
    import oracle.halfway as O
    names = {f.name for f in dataclasses.fields(O.Params)}
    p = O.Params(**{k: v for k, v in dict(params, gn_iters=gn_iters).items() if k in names})
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        O.solve(imgs.astype(np.float64), calib, p)
        return time.perf_counter() - t0


def cpu_baseline(imgs, calib, params, W, H):
    """The FP64 oracle on a bounded sample of the same frame: two whole
    solves (pyramid, every level's set-up, Gauss-Newton steps with PCG and
    step control, output) with 1 and with 2 Gauss-Newton steps per level,
    BLAS limited to one thread.  Their difference is the cost of one step on
    every level, so a frame of gn_iters steps costs t1 + (gn_iters - 1)
    (t2 - t1)."""
    t1 = _oracle_solve_seconds(imgs, calib, params, 1, 1)
    t2 = _oracle_solve_seconds(imgs, calib, params, 2, 1)
    n = params["gn_iters"]
    ms = (t1 + (n - 1) * (t2 - t1)) * 1e3
    model, ncpu = cpu_model()
    return dict(value=round(ms, 1), unit="ms/frame", cores=1, kind="oracle",
                cpu=model, host_cpus=ncpu,
                sample=(f"whole oracle solves of the same {W}x{H} frame with 1 and 2 "
                        f"Gauss-Newton steps per level ({t1:.1f} s, {t2:.1f} s; "
                        f"{params['levels']} levels, {params['pcg_iters']} PCG), extrapolated "
                        f"linearly to {n} steps per level; numpy/scipy float64, BLAS "
                        "limited to 1 thread"))


def cpu_full(imgs, calib, params, W, H):
    """Whole oracle solves at the full schedule, BLAS on every host CPU and
    on one thread (minutes each)."""
    model, ncpu = cpu_model()
    out = dict(cpu=model, host_cpus=ncpu, workload=f"{W}x{H}", **params)
    for threads in (ncpu, 1):
        out[f"seconds_threads_{threads}"] = round(
            _oracle_solve_seconds(imgs, calib, params, params["gn_iters"], threads), 2)
        print(json.dumps(out), file=sys.stderr, flush=True)
    return out


def _short_name(n):
    import re
    n = re.sub(r"\(anonymous namespace\)::", "", n)
    n = re.sub(r"std::conditional<(true|false), FrameMap, LevelArgs>::type", "", n)
    n = re.sub(r"\(.*\)$", "", n).replace("void ", "")
    return n


def trace_summary(path, focus=("k_",)):
    """Summary of a rocprofv3 CSV: per kernel (calls, total/avg/min/max us)
    for a kernel trace, or per kernel the mean counter values per dispatch
    for a counter-collection file; both also per launch grid for the
    kernels named in `focus`."""
    import collections
    import csv
    rows = list(csv.DictReader(open(path)))
    if not rows:
        print("empty file")
        return
    cols = rows[0].keys()
    grid = [c for c in ("Grid_Size_X", "Grid_Size") if c in cols][0]
    if "Counter_Name" in cols:
        acc = collections.OrderedDict()
        for r in rows:
            k = (_short_name(r["Kernel_Name"]), r[grid], r["Counter_Name"])
            a = acc.setdefault(k, [0, 0.0])
            a[0] += 1
            a[1] += float(r["Counter_Value"])
        print(f"{'kernel':44s} {'grid':>10s} {'counter':>12s} {'dispatches':>10s} {'mean':>14s}")
        for (k, g, c), (n, v) in sorted(acc.items(), key=lambda kv: -kv[1][1]):
            print(f"{k:44s} {g:>10s} {c:>12s} {n:10d} {v / n:14.1f}")
        return
    agg, grids = collections.OrderedDict(), collections.OrderedDict()
    tot = 0.0
    for r in rows:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        k = _short_name(r["Kernel_Name"])
        a = agg.setdefault(k, [0, 0.0, 1e30, 0.0])
        a[0] += 1
        a[1] += d
        a[2] = min(a[2], d)
        a[3] = max(a[3], d)
        tot += d
        if any(f in k for f in focus):
            g = grids.setdefault((k, int(r[grid])), [0, 0.0])
            g[0] += 1
            g[1] += d
    print(f"{'kernel':44s} {'calls':>7s} {'total_us':>11s} {'avg_us':>9s} {'min_us':>8s} "
          f"{'max_us':>9s} {'pct':>6s}")
    for k, (c, t, mn, mx) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        print(f"{k:44s} {c:7d} {t:11.1f} {t / c:9.2f} {mn:8.2f} {mx:9.2f} {100 * t / tot:6.2f}")
    print(f"total kernel time: {tot / 1e3:.3f} ms over {len(rows)} dispatches")
    print("\nby launch grid (total threads in x):")
    for (k, g), (c, t) in sorted(grids.items(), key=lambda kv: (kv[0][0], -kv[0][1])):
        print(f"  {k:44s} grid {g:9d}: calls {c:6d}, avg {t / c:8.2f} us")


def traffic_report(fetch_csv, write_csv, kernels, copy_mib):
    """HBM bytes per launch of each kernel in `kernels` (its largest launch
    grid found in both files; every k_pcg iteration kernel, FIRST = false,
    in the files if `kernels` is empty)
    from two rocprofv3 counter CSVs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch), each counter scaled by what it reads for the copy probe of
    copy_mib MiB (which reads and writes exactly that much).  Prints the
    summary that bench.py reads back as roofline.traffic."""
    import collections
    import csv

    def per_kernel(path, counter):
        acc = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                acc[(_short_name(r["Kernel_Name"]), int(r["Grid_Size"]))].append(
                    float(r["Counter_Value"]))
        return acc
    f = per_kernel(fetch_csv, "FETCH_SIZE")
    w = per_kernel(write_csv, "WRITE_SIZE")
    expect = copy_mib * 1024.0
    copy_w = min((v for (k, g), vs in w.items() if "copyBuffer" in k for v in vs),
                 key=lambda v: abs(v - expect))
    copy_f = max(v for (k, g), vs in f.items() if "copyBuffer" in k for v in vs)
    ff, fw = expect / copy_f, expect / copy_w
    # the counter runs autotune separately, so a kernel may run at a launch
    # grid in one run only: use the grids both runs saw
    if not kernels:
        kernels = sorted({k for k, g in f if re.match(r"k_pcg<(true|false), false, ", k)
                          and (k, g) in w})
    print(f"# copy probe {copy_mib} MiB: FETCH_SIZE reads {copy_f:.1f} KiB (factor {ff:.4f}), "
          f"WRITE_SIZE reads {copy_w:.1f} KiB (factor {fw:.4f})")
    print(f"source_sha256 = {source_hash()}")
    for kernel in kernels:
        common = [kg for kg in f if kg[0] == kernel and kg in w]
        if not common:
            continue
        key = max(common, key=lambda kg: kg[1])
        mf = float(np.mean(f[key]))
        mw = float(np.mean(w[key]))
        traffic = int(round((mf * ff + mw * fw) * 1024))
        print(f"# {kernel}, launch grid {key[1]} threads: FETCH_SIZE {mf:.1f} KiB, WRITE_SIZE "
              f"{mw:.1f} KiB per dispatch (means over {len(f[key])} / {len(w[key])} dispatches)")
        print(f"traffic_bytes_per_launch[{kernel}] = {traffic}")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="vga", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--weights", default=None,
                    help="initialiser file under paper_1610_07159_amd/weights/ for the "
                         "batch_learned workload (default: the workload's)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time whole oracle solves of the workload (all host CPUs and one "
                         "thread) and exit")
    ap.add_argument("--no-epe", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-init vs plain comparison")
    ap.add_argument("--exec-mode", type=int, default=0,
                    help="0 = captured HIP graph, 1 = direct launches")
    ap.add_argument("--apply-mode", type=int, default=2, choices=(0, 1, 2, 3),
                    help="0: matrix-free products from the pixel records, "
                         "1: per-node blocks, 2: per-node blocks and one-workgroup "
                         "PCG at levels of at most 336 nodes, 3: 2 plus the co-resident "
                         "tiled PCG at the larger levels (single frames)")
    ap.add_argument("--tile-mode", type=int, default=1,
                    help="PCG tile shapes: 0 = default, 1 = autotuned (timed on the "
                         "warm-up solve), 2 / 3 / 4 = the alternative shapes")
    ap.add_argument("--grid-stride", type=int, default=0,
                    help="warp-grid stride of the single-frame workloads (0: the workload's)")
    ap.add_argument("--pcg-iters", type=int, default=0,
                    help="PCG iterations per Gauss-Newton step of the single-frame "
                         "workloads (0: the workload's)")
    ap.add_argument("--gn-iters", type=int, default=0,
                    help="Gauss-Newton steps per level of the single-frame workloads "
                         "(0: the workload's)")
    ap.add_argument("--gn-fine", type=int, default=0,
                    help="Gauss-Newton steps on the two finest levels (the paper's split "
                         "schedule; 0: as every level)")
    ap.add_argument("--levels", type=int, default=0,
                    help="pyramid levels of the single-frame workloads (0: the workload's)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter "
                         "calibration under rocprofv3 --pmc)")
    ap.add_argument("--trace-summary", metavar="CSV",
                    help="summarise a rocprofv3 kernel-trace or counter CSV and exit")
    ap.add_argument("--traffic", nargs="+", metavar="CSV_OR_KERNEL",
                    help="FETCH_CSV WRITE_CSV [KERNEL ...]: HBM traffic per launch of each "
                         "KERNEL (default: every PCG iteration kernel in the files) from two "
                         "counter CSVs (calibrated by the copy probe) and exit")
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.traffic:
        if len(args.traffic) < 2:
            ap.error("--traffic needs FETCH_CSV WRITE_CSV [KERNEL ...]")
        traffic_report(args.traffic[0], args.traffic[1], args.traffic[2:],
                       copy_mib=args.copy_probe_mib or 512)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU "
              "path (frames would shard across GPUs with no exchange); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.cpu_full:
        w, imgs, calib, _ = make_workload(args.workload)
        params = dict(w["params"])
        if args.grid_stride:
            params["grid_stride"] = args.grid_stride
        print(json.dumps(cpu_full(imgs, calib, params, w["width"], w["height"])), flush=True)
        return

    # host process pools render before anything touches the GPU
    pre = {}
    if args.workload == "batch":
        pre["batch"] = make_batch_workload(WORKLOADS["batch"])
    if args.workload == "batch_learned":
        pre["batch"] = make_batch_workload(WORKLOADS["batch"], truth=True)
    if args.workload == "video":
        pre["video"] = make_video_workload(WORKLOADS["video"])
    if args.workload == "illum":
        pre["illum"] = make_illum_workload(WORKLOADS["illum"])
    if args.workload == "occlusion":
        pre["occlusion"] = make_occlusion_workload(WORKLOADS["occlusion"])
    if args.workload == "learned" or (args.workload == "vga" and not args.no_learned):
        from paper_1610_07159_amd.train_init import render_frames
        n_eval = WORKLOADS["learned"]["n_eval"]
        pre["eval"] = render_frames(640, 480, range(1_000_000, 1_000_000 + n_eval), True, 8,
                                    log=lambda m: None)
    if args.workload == "learned_hd":
        from paper_1610_07159_amd.train_init import render_frames
        w = WORKLOADS["learned_hd"]
        pre["eval"] = render_frames(w["width"], w["height"],
                                    range(1_000_000, 1_000_000 + w["n_eval"]), True, 16,
                                    log=lambda m: print(m, file=sys.stderr, flush=True),
                                    max_disp=w["max_disp"], blobs=w["blobs"])
    import torch
    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        # reference dispatch of known traffic: reads and writes exactly
        # copy_probe_mib MiB
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "batch":
        return run_batch(args, pre["batch"])
    if args.workload == "batch_learned":
        return run_batch_learned(args, pre["batch"])
    if args.workload in ("learned", "learned_hd"):
        return run_learned(args, pre["eval"], args.workload)
    if args.workload == "video":
        return run_video(args, pre["video"])
    if args.workload == "illum":
        return run_toggle(args, pre["illum"], "illum", "illum", ("plain", "corrected"))
    if args.workload == "occlusion":
        return run_toggle(args, pre["occlusion"], "occlusion", "occlusion",
                          ("plain", "occlusion_maps"))

    from paper_1610_07159_amd import SceneFlowSolver, sf

    w, imgs, calib, scene = make_workload(args.workload)
    W, H = w["width"], w["height"]
    params = dict(w["params"])
    if args.grid_stride:
        params["grid_stride"] = args.grid_stride
    if args.pcg_iters:
        params["pcg_iters"] = args.pcg_iters
    if args.gn_iters:
        params["gn_iters"] = args.gn_iters
    if args.gn_fine:
        params["gn_fine"] = args.gn_fine
    if args.levels:
        params["levels"] = args.levels
    img = torch.from_numpy(imgs).cuda().contiguous()
    params["apply_mode"] = args.apply_mode
    solver = SceneFlowSolver(W, H, exec_mode=args.exec_mode, tile_mode=args.tile_mode,
                             **params)
    stream = solver.stream
    out = (torch.empty((H, W), device="cuda"), torch.empty((3, H, W), device="cuda"),
           torch.empty((6, H, W), device="cuda"))
    for _ in range(args.warmup):
        solver.solve(img, calib, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        solver.solve(img, calib, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    log = solver.log()
    if not all(np.isfinite(r["energy"]) and np.isfinite(r["energy_after"]) for r in log):
        raise RuntimeError("non-finite energy in the solve log")
    flows = out[2].cpu().numpy()

    # dominant kernel: H p at level 0, timed live on the solver's stream
    reps = params["gn_iters"] * params["pcg_iters"]
    avg_ms = sf.sf_time_kernel(solver.ctx, sf.SF_KERNEL_APPLY, 0, reps)
    sizes = level_sizes(W, H, params["levels"], params["grid_stride"])
    N0, G0 = sizes[0][2], sizes[0][3]
    bytes_apply = apply_bytes(N0, G0, args.apply_mode)
    achieved = bytes_apply / (avg_ms * 1e-3) / 1e9
    per_level = [round(sf.sf_time_kernel(solver.ctx, sf.SF_KERNEL_APPLY, l, reps) * 1e3, 2)
                 for l in range(params["levels"])]
    prefix0 = pcg_kernel_prefix(False, args.apply_mode, params["grid_stride"],
                                sf.sf_tile_variant(solver.ctx, False, 0))
    kernel0, traffic0 = measured_traffic(args.workload, args.apply_mode, prefix0)
    if not (args.exec_mode == 0 and params == dict(w["params"], apply_mode=args.apply_mode)):
        kernel0, traffic0 = None, None  # the counters cover the default configuration only

    result = {
        "metric": METRIC,
        "value": round(ms, 4),
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": describe(w["desc"], params), "width": W, "height": H,
                   "exec": "hip graph" if args.exec_mode == 0 else "direct launches",
                   "tile_mode": args.tile_mode, **params},
        "frames_per_s": round(1e3 / ms, 2),
        "wall_ms_per_frame": round(wall * 1e3 / args.steps, 4),
        "roofline": {"bound": "hbm",
                     "kernel": (kernel0 or prefix0 + ", ...>") + (
                         " (node-block" if args.apply_mode >= 1 else " (matrix-free")
                     + " H p at level 0)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic0,
                     "bytes_per_launch": bytes_apply,
                     "avg_us_per_launch": round(bytes_apply / achieved / 1e3, 2),
                     "apply_us_per_level": per_level},
        "final_energy": log[-1]["energy_after"],
        "accepted_tau": {str(t): sum(1 for r in log if r["tau"] == t)
                         for t in sorted({r["tau"] for r in log}, reverse=True)},
    }
    if not args.no_epe:
        result["epe_px"] = round(epe(flows, scene, W, H), 4)
    if args.workload == "vga" and not args.no_learned:
        result["learned_vs_plain"] = learned_vs_plain(params, pre["eval"])
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(imgs, calib, params, W, H)
    solver.close()
    print(json.dumps(result), flush=True)


def run_learned(args, frames, name="learned"):
    """Equal-EPE comparison of the learned initialiser with the plain
    solver; value = ms/frame of the learned solve at the plain EPE."""
    w = WORKLOADS[name]
    W, H = w["width"], w["height"]
    params = dict(w["params"], apply_mode=args.apply_mode)
    weights = np.load(os.path.join(ROOT, "paper_1610_07159_amd", "weights", w["weights"]),
                      allow_pickle=False)
    r = equal_epe_sweeps(single_frame_runner(frames, W, H, params, weights),
                         params["gn_iters"])
    reach = r["learned_at_target"]
    result = {
        "metric": METRIC,
        "value": reach["ms_per_frame"] if reach else None,
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": 3 * w["n_eval"],
        "warmup": w["n_eval"],
        "ms_per_step": reach["ms_per_frame"] if reach else None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 solve, bf16 initialiser",
        "data": "synthetic",
        "config": {"workload": w["desc"], **params},
        **r,
    }
    print(json.dumps(result), flush=True)


def epe_device(flows, pos, ok):
    """The EPE of `epe` on the GPU (float64): flows (6, H, W), the
    generator's halfway correspondences pos (4, 2, H, W) and validity ok
    (H, W), all device tensors."""
    import torch
    H, W = flows.shape[1:]
    yy, xx = torch.meshgrid(torch.arange(H, device=flows.device, dtype=torch.float64),
                            torch.arange(W, device=flows.device, dtype=torch.float64),
                            indexing="ij")
    f = flows.double()
    pos = pos.double()
    signs = ((-1, -1, 1), (1, -1, -1), (-1, 1, -1), (1, 1, 1))
    err = torch.zeros((H, W), device=flows.device, dtype=torch.float64)
    inside = ok.clone()
    for c, (a, b, d) in enumerate(signs):
        px = xx + a * f[0] + b * f[2] + d * f[4]
        py = yy + a * f[1] + b * f[3] + d * f[5]
        err += torch.hypot(px - pos[c, 0], py - pos[c, 1])
        inside &= ((pos[c, 0] >= 0) & (pos[c, 0] <= W - 1) & (pos[c, 1] >= 0)
                   & (pos[c, 1] <= H - 1))
    return float((err / 4.0)[inside].mean())


def run_batch_learned(args, workload):
    """Equal-EPE comparison of batches started from the learned
    initialisation with plain batches (zero initialisation), on the batched
    workload; value = ms/frame of the learned batch at the plain EPE."""
    import torch
    from paper_1610_07159_amd import SceneFlowSolver, sf
    w = WORKLOADS["batch_learned"]
    params = dict(WORKLOADS["batch"]["params"], apply_mode=args.apply_mode)
    res, frames = workload
    n = len(frames)
    dev = [(torch.from_numpy(i).cuda().contiguous(), c) for i, c, _ in frames]
    truth = [(torch.from_numpy(t[0]).cuda(), torch.from_numpy(t[1]).cuda())
             for _, _, t in frames]
    weights = np.load(os.path.join(ROOT, "paper_1610_07159_amd", "weights",
                                   args.weights or w["weights"]), allow_pickle=False)
    W0, H0 = res[0]
    solver = SceneFlowSolver(W0, H0, exec_mode=args.exec_mode, tile_mode=args.tile_mode,
                             **params)
    sf.sf_set_initializer(solver.ctx, weights)
    reps = max(1, args.steps)

    def run(init_mode, n_gn):
        prm = sf.sf_params_default(exec_mode=args.exec_mode, tile_mode=args.tile_mode,
                                   **dict(params, gn_iters=n_gn, init_mode=init_mode))
        outs = solver.solve_batch(dev, params=prm)  # workspace, tiles, graph
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(solver.stream)
        for _ in range(reps):
            outs = solver.solve_batch(dev, outs=outs, params=prm)
        ev[1].record(solver.stream)
        torch.cuda.synchronize()
        batch_ms = ev[0].elapsed_time(ev[1]) / reps
        e = float(np.mean([epe_device(o[2], *t) for o, t in zip(outs, truth)]))
        row = dict(gn_iters=n_gn, epe_px=round(e, 4), ms_per_frame=round(batch_ms / n, 4),
                   batch_ms=round(batch_ms, 3))
        if init_mode:
            used = [solver.batch_init_result(f)[0] for f in range(n)]
            row["network_frames"] = sum(u >= 0 for u in used)
            row["prediction_kept"] = sum(u == 1 for u in used)
        return e, row

    r = equal_epe_sweeps(run, params["gn_iters"])
    solver.close()
    reach = r["learned_at_target"]
    sizes = {f"{W}x{H}": res.count((W, H)) for W, H in sorted(set(res))}
    result = {
        "metric": METRIC,
        "value": reach["ms_per_frame"] if reach else None,
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": reps,
        "warmup": 1,
        "ms_per_step": reach["batch_ms"] if reach else None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 solve, bf16 initialiser",
        "data": "synthetic",
        "config": {"workload": w["desc"], "frames_per_batch": n, "sizes": sizes,
                   "weights": args.weights or w["weights"],
                   "exec": "hip graph" if args.exec_mode == 0 else "direct launches",
                   "tile_mode": args.tile_mode, **params},
        **r,
    }
    print(json.dumps(result), flush=True)


def run_batch(args, workload):
    """Batches of frames of mixed sizes through sf_solve_batch.  One step is
    one batch; per-batch GPU time from HIP events on the solver's stream."""
    import torch
    from paper_1610_07159_amd import SceneFlowSolver, sf
    w = WORKLOADS["batch"]
    params = dict(w["params"], apply_mode=args.apply_mode)
    res, frames = workload
    dev = [(torch.from_numpy(i).cuda().contiguous(), c) for i, c in frames]
    W0, H0 = res[0]
    solver = SceneFlowSolver(W0, H0, exec_mode=args.exec_mode, tile_mode=args.tile_mode,
                             **params)
    stream = solver.stream
    prm = sf.sf_params_default(exec_mode=args.exec_mode, tile_mode=args.tile_mode, **params)
    outs = None
    for _ in range(args.warmup):
        outs = solver.solve_batch(dev, outs=outs, params=prm)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        outs = solver.solve_batch(dev, outs=outs, params=prm)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_batch = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    total_ms = float(per_batch.sum())
    n = len(frames)
    for f in range(n):
        log = solver.batch_log(f)
        if not all(np.isfinite(r["energy"]) and np.isfinite(r["energy_after"]) for r in log):
            raise RuntimeError(f"non-finite energy in the log of frame {f}")

    reps = params["gn_iters"] * params["pcg_iters"]
    avg_ms = sf.sf_time_batch_kernel(solver.ctx, sf.SF_KERNEL_APPLY, 0, reps)
    bytes_apply = 0
    for W, H in res:
        L = sf.sf_batch_levels(W, H, params["levels"])
        N0, G0 = level_sizes(W, H, L, params["grid_stride"])[0][2:]
        bytes_apply += apply_bytes(N0, G0, args.apply_mode, batched=True)
    achieved = bytes_apply / (avg_ms * 1e-3) / 1e9
    prefix0 = pcg_kernel_prefix(True, args.apply_mode, params["grid_stride"],
                                sf.sf_tile_variant(solver.ctx, True, 0))
    kernel0, traffic0 = measured_traffic("batch", args.apply_mode, prefix0)
    ms_frame = total_ms / (args.steps * n)
    sizes = {f"{W}x{H}": res.count((W, H)) for W, H in sorted(set(res))}
    result = {
        "metric": METRIC,
        "value": round(ms_frame, 4),
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["desc"], "frames_per_batch": n, "sizes": sizes,
                   "exec": "hip graph" if args.exec_mode == 0 else "direct launches",
                   "tile_mode": args.tile_mode, **params},
        "frames_per_s": round(1e3 / ms_frame, 1),
        "batch_ms_p50": round(float(np.percentile(per_batch, 50)), 3),
        "batch_ms_p99": round(float(np.percentile(per_batch, 99)), 3),
        "wall_ms_per_batch": round(wall * 1e3 / args.steps, 3),
        "roofline": {"bound": "hbm",
                     "kernel": (kernel0 or prefix0 + ", ...>") + (
                         " (node-block" if args.apply_mode >= 1 else " (matrix-free")
                     + " H p at level 0, all frames)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic0,
                     "bytes_per_launch": bytes_apply,
                     "avg_us_per_launch": round(avg_ms * 1e3, 2)},
    }
    solver.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
