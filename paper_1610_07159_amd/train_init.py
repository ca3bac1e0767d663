"""Training and evaluation of the learned coarse-level initialiser.

    python -m paper_1610_07159_amd.train_init --frames 256 --eval 16 \\
        --out init_640x480.npy --report report.json

1. Renders seeded generator frames (training seeds 0.., evaluation seeds
   1,000,000..) in a process pool on the host.
2. Targets: the plain solver's (zero initialisation) level-0 flows of each
   training frame, restricted to level 4 (16 x 16 box average / 16).
3. Trains the network on the level-4 image quadruples with the GPU trainer
   (sf_trainer_*: bf16 matrix-core forward/backward, L1 loss, Adam with a
   cosine learning-rate decay), batches drawn by a seeded shuffle.
4. Evaluation on held-out frames: end-point error (EPE, mean over valid
   halfway pixels of the mean of the four correspondence errors) of the
   plain solver at the full schedule, and of the solver started from the
   network (with the energy fallback) for 1..gn_iters Gauss-Newton steps per
   level; reports the smallest step count that reaches the plain EPE and
   its time per frame.

Every solver, network and optimiser step runs in libsf.so; this script only
prepares data (rendering, box restriction on the host) and drives the loop.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SCHEDULE = dict(levels=5, grid_stride=4, gn_iters=10, pcg_iters=20)
LEVEL_IN = 4


def box_restrict(a, level=LEVEL_IN):
    """(C, H, W) -> (C, H >> l, W >> l): mean over 2^l x 2^l blocks (the
    pyramid's repeated 2 x 2 box with floor sizes)."""
    k = 1 << level
    C, H, W = a.shape
    h, w = H >> level, W >> level
    return a[:, :h * k, :w * k].reshape(C, h, k, w, k).mean(axis=(2, 4))


def _render(args):
    from synth import make_frame, sized_config
    W, H, seed, truth, max_disp, blobs = args
    imgs, calib, scene = make_frame(sized_config(W, H, max_disp=max_disp, n_blobs=blobs), seed)
    out = dict(imgs=imgs, calib=calib, seed=seed)
    if truth:
        pos, ok = scene.halfway_truth()
        out["truth"] = (pos.astype(np.float32), ok)
    return out


def render_frames(W, H, seeds, truth, workers, log=print, max_disp=None, blobs=0):
    """Generator frames of size W x H (displacement 30 px per 640 px of
    width unless max_disp is given; blobs independently moving blobs)."""
    from concurrent.futures import ProcessPoolExecutor
    jobs = [(W, H, s, truth, max_disp, blobs) for s in seeds]
    out = []
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for f in ex.map(_render, jobs, chunksize=1):
            out.append(f)
            if len(out) % 32 == 0:
                log(f"  rendered {len(out)}/{len(jobs)}")
    return out


def epe(flows, truth, W, H):
    pos, ok = truth
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


def solve_flows(frames, W, H, init_mode=0, weights=None, timed=False, **sched):
    """Runs the solver on every frame; returns per-frame level-0 flows and,
    if timed, the mean GPU time per frame (HIP events, graph replay)."""
    import torch
    from paper_1610_07159_amd import SceneFlowSolver, sf
    solver = SceneFlowSolver(W, H, init_mode=init_mode, **sched)
    try:
        if weights is not None:
            sf.sf_set_initializer(solver.ctx, weights)
        out = (torch.empty((H, W), device="cuda"), torch.empty((3, H, W), device="cuda"),
               torch.empty((6, H, W), device="cuda"))
        flows, used = [], []
        dev = [torch.from_numpy(f["imgs"]).cuda() for f in frames]
        for f, img in zip(frames, dev):
            solver.solve(img, f["calib"], out=out)
            flows.append(out[2].cpu().numpy())
            if init_mode == 1:
                used.append(sf.sf_get_init_result(solver.ctx)[0])
        ms = None
        if timed:
            reps = 3
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(solver.stream)
            for _ in range(reps):
                for f, img in zip(frames, dev):
                    solver.solve(img, f["calib"], out=out)
            e1.record(solver.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / (reps * len(frames))
    finally:
        solver.close()
    return flows, used, ms


def train_gpu(x, y, epochs, batch, lr, seed, init_seed=0, log=print):
    import torch
    from paper_1610_07159_amd import sf
    N, _, h, w = x.shape
    t = sf.sf_trainer_create(batch, h, w, torch.cuda.current_stream().cuda_stream)
    try:
        sf.sf_trainer_set_params(t, he_init(init_seed))
        xd = torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
        yd = torch.from_numpy(np.ascontiguousarray(y, np.float32)).cuda()
        rng = np.random.default_rng(seed)
        steps_per_epoch = N // batch
        total = epochs * steps_per_epoch
        curve, k = [], 0
        xb = torch.empty((batch, 4, h, w), device="cuda")
        yb = torch.empty((batch, 6, h, w), device="cuda")
        for ep in range(epochs):
            order = torch.from_numpy(rng.permutation(N)).cuda()
            ep_loss = []
            for s in range(steps_per_epoch):
                idx = order[s * batch:(s + 1) * batch]
                torch.index_select(xd, 0, idx, out=xb)
                torch.index_select(yd, 0, idx, out=yb)
                lr_k = lr * 0.5 * (1.0 + math.cos(math.pi * k / total))
                ep_loss.append(sf.sf_trainer_step(t, xb.data_ptr(), yb.data_ptr(), batch, lr_k))
                k += 1
            curve.append(float(np.mean(ep_loss)))
            log(f"epoch {ep + 1}/{epochs}: L1 {curve[-1]:.5f}")
        return sf.sf_trainer_get_params(t), curve
    finally:
        sf.sf_trainer_destroy(t)


def he_init(seed):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, last layer
    scaled by 0.1 (small initial predictions); flat layout of sf.h."""
    rng = np.random.default_rng(seed)
    chans = (4, 32, 32, 32, 32, 32, 6)
    parts = []
    for l, (ci, co) in enumerate(zip(chans[:-1], chans[1:])):
        std = math.sqrt(2.0 / (ci * 9)) * (0.1 if l == len(chans) - 2 else 1.0)
        parts += [rng.normal(0.0, std, co * ci * 9), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--frames", type=int, default=256)
    ap.add_argument("--eval", type=int, default=16)
    ap.add_argument("--width", type=int, default=640)
    ap.add_argument("--height", type=int, default=480)
    ap.add_argument("--levels", type=int, default=SCHEDULE["levels"])
    ap.add_argument("--max-disp", type=float, default=None,
                    help="largest image displacement in px (default 30 per 640 px of width)")
    ap.add_argument("--blobs", type=int, default=0, help="independently moving blobs")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default="init_weights.npy")
    ap.add_argument("--report", default="init_report.json")
    args = ap.parse_args()
    log = lambda m: print(m, flush=True)  # noqa: E731
    W, H = args.width, args.height
    sched_full = dict(SCHEDULE, levels=args.levels)
    scene = dict(max_disp=args.max_disp, blobs=args.blobs)
    t0 = time.time()
    train_frames = render_frames(W, H, range(args.frames), False, args.workers, log, **scene)
    log(f"rendered {len(train_frames)} training frames in {time.time() - t0:.0f} s")
    t1 = time.time()
    eval_frames = render_frames(W, H, range(1_000_000, 1_000_000 + args.eval), True,
                                args.workers, log, **scene)
    log(f"rendered {len(eval_frames)} evaluation frames with truth in {time.time() - t1:.0f} s")

    import torch
    torch.cuda.set_device(0)
    flows, _, _ = solve_flows(train_frames, W, H, **sched_full)
    x = np.stack([box_restrict(f["imgs"]) for f in train_frames]).astype(np.float32)
    y = np.stack([box_restrict(fl) / (1 << LEVEL_IN) for fl in flows]).astype(np.float32)
    log(f"targets from the plain solver: {y.shape}")
    t2 = time.time()
    params, curve = train_gpu(x, y, args.epochs, args.batch, args.lr, seed=1, log=log)
    log(f"trained in {time.time() - t2:.1f} s")
    np.save(args.out, params)

    plain, _, ms_plain = solve_flows(eval_frames, W, H, timed=True, **sched_full)
    epe_plain = float(np.mean([epe(fl, f["truth"], W, H) for fl, f in zip(plain, eval_frames)]))
    sweep = []
    for n in range(1, sched_full["gn_iters"] + 1):
        sched = dict(sched_full, gn_iters=n)
        fl, used, ms = solve_flows(eval_frames, W, H, init_mode=1, weights=params, timed=True,
                                   **sched)
        e = float(np.mean([epe(a, f["truth"], W, H) for a, f in zip(fl, eval_frames)]))
        sweep.append(dict(gn_iters=n, epe_px=round(e, 4), ms_per_frame=round(ms, 3),
                          init_used=int(sum(used))))
        log(f"learned init, {n} GN/level: EPE {e:.4f} px, {ms:.2f} ms/frame, "
            f"prediction kept on {sum(used)}/{len(used)} frames")
    zero_sweep = []
    for n in range(1, sched_full["gn_iters"] + 1):
        fl, _, ms = solve_flows(eval_frames, W, H, timed=True, **dict(sched_full, gn_iters=n))
        e = float(np.mean([epe(a, f["truth"], W, H) for a, f in zip(fl, eval_frames)]))
        zero_sweep.append(dict(gn_iters=n, epe_px=round(e, 4), ms_per_frame=round(ms, 3)))
    reach = next((s for s in sweep if s["epe_px"] <= epe_plain), None)
    report = dict(
        frames=args.frames, eval_frames=args.eval, size=f"{W}x{H}", schedule=sched_full,
        max_disp=args.max_disp, blobs=args.blobs,
        epochs=args.epochs, batch=args.batch, lr=args.lr, loss_curve=[round(c, 5) for c in curve],
        plain=dict(gn_iters=sched_full["gn_iters"], epe_px=round(epe_plain, 4),
                   ms_per_frame=round(ms_plain, 3)),
        learned_sweep=sweep, zero_init_sweep=zero_sweep,
        equal_epe=(dict(gn_iters=reach["gn_iters"], ms_per_frame=reach["ms_per_frame"],
                        speedup=round(ms_plain / reach["ms_per_frame"], 3))
                   if reach else None))
    with open(args.report, "w") as f:
        json.dump(report, f, indent=1)
    log(json.dumps(dict(plain=report["plain"], equal_epe=report["equal_epe"])))


if __name__ == "__main__":
    main()
