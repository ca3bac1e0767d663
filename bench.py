#!/usr/bin/env python
"""Benchmark: ms per frame of the GN-PCG halfway-domain solve at 640x480.

One "step" is one whole solve of one frame (pyramid, 5 levels x 10
Gauss-Newton steps x 20 PCG iterations, step control, depth/3D-flow output)
with the four input images already resident in device memory.  Prints one
JSON line.  Besides the headline number it reports the roofline of the
dominant kernel (the matrix-free H p of the PCG at the finest level, timed
live with HIP events on the solver's stream) and, unless
--no-cpu-baseline, the FP64 CPU oracle timed on a bounded sample of the
same workload on the host.
"""
import argparse
import json
import os
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
                     "noise sigma 0.01; stride 4, 5 levels, 10 GN x 20 PCG",
                width=640, height=480, seed=1,
                params=dict(levels=5, grid_stride=4, gn_iters=10, pcg_iters=20)),
    "tiny": dict(desc="64x48 translating textured plane; stride 8, 3 levels, "
                      "5 GN x 10 PCG",
                 width=64, height=48, seed=0,
                 params=dict(levels=3, grid_stride=8, gn_iters=5, pcg_iters=10)),
    "hd": dict(desc="1280x720 float32 quadruple, up to 80 px displacement, two "
                    "moving blobs; stride 4, 6 levels, 10 GN x 20 PCG",
               width=1280, height=720, seed=2,
               params=dict(levels=6, grid_stride=4, gn_iters=10, pcg_iters=20)),
}

# Algorithmic bytes of one H p launch (matrix-free, per-pixel Gauss-Newton
# blocks): per pixel the 21 upper-triangular floats of its block; per node
# z, p_old, p (write), q (write), base, delta (6 floats each) and w_i.
APPLY_BYTES_PER_PIXEL = 21 * 4
APPLY_BYTES_PER_NODE = (6 * 6 + 1) * 4


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


def cpu_baseline(imgs, calib, params, W, H):
    """The FP64 oracle on a bounded sample of the same frame: the level-0
    set-up plus one Gauss-Newton step (linearise, assemble, PCG, step
    control) at level 0; scaled to a frame as (set-up + gn_iters steps) x
    (sum of level pixel counts / level-0 pixel count)."""
    from threadpoolctl import threadpool_limits
    import oracle.halfway as O
    p = O.Params(**params)
    with threadpool_limits(limits=1):
        pyr = O.pyramid(imgs.astype(np.float64), p.levels)
        grid = O.Grid(W, H, p.grid_stride)
        t0 = time.perf_counter()
        ls = O.setup_level(0, pyr, p, O.Calib.from_dict(calib), np.zeros((6, grid.G)))
        t1 = time.perf_counter()
        O.gn_step(ls, np.zeros((6, grid.G)), p)
        t2 = time.perf_counter()
    sizes = level_sizes(W, H, p.levels, p.grid_stride)
    scale = sum(s[2] for s in sizes) / sizes[0][2]
    ms = ((t1 - t0) + p.gn_iters * (t2 - t1)) * scale * 1e3
    return dict(value=round(ms, 1), unit="ms/frame", cores=1, kind="oracle",
                sample=(f"level-0 set-up ({t1 - t0:.2f} s) and one level-0 "
                        f"Gauss-Newton step ({t2 - t1:.2f} s, {W}x{H} px, "
                        f"{p.pcg_iters} PCG) of the same frame, scaled by "
                        f"{p.gn_iters} steps and sum(N_l)/N_0 = {scale:.3f}; "
                        "numpy/scipy float64, BLAS limited to 1 thread"))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="vga", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-epe", action="store_true")
    ap.add_argument("--exec-mode", type=int, default=0,
                    help="0 = captured HIP graph, 1 = direct launches")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter "
                         "calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU "
              "path (frames would shard across GPUs with no exchange); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1610_07159_amd import SceneFlowSolver, sf

    w, imgs, calib, scene = make_workload(args.workload)
    W, H = w["width"], w["height"]
    params = dict(w["params"])
    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    img = torch.from_numpy(imgs).cuda().contiguous()
    solver = SceneFlowSolver(W, H, exec_mode=args.exec_mode, **params)
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
    bytes_apply = APPLY_BYTES_PER_PIXEL * N0 + APPLY_BYTES_PER_NODE * G0
    achieved = bytes_apply / (avg_ms * 1e-3) / 1e9
    per_level = [round(sf.sf_time_kernel(solver.ctx, sf.SF_KERNEL_APPLY, l, reps) * 1e3, 2)
                 for l in range(params["levels"])]

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
        "config": {"workload": w["desc"], "width": W, "height": H,
                   "exec": "hip graph" if args.exec_mode == 0 else "direct launches",
                   **params},
        "frames_per_s": round(1e3 / ms, 2),
        "wall_ms_per_frame": round(wall * 1e3 / args.steps, 4),
        "roofline": {"bound": "hbm", "kernel": "k_apply (H p) at level 0",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "bytes_per_launch": bytes_apply,
                     "avg_us_per_launch": round(bytes_apply / achieved / 1e3, 2),
                     "apply_us_per_level": per_level},
        "final_energy": log[-1]["energy_after"],
    }
    if not args.no_epe:
        result["epe_px"] = round(epe(flows, scene, W, H), 4)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(imgs, calib, params, W, H)
    solver.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
