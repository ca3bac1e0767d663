"""Training and evaluation of the learned coarse-level initialiser.

    python -m paper_1610_07159_amd.train_init --frames 256 --eval 16 \\
        --out init_640x480.npy --report report.json

1. Renders seeded generator frames (training seeds 0.., evaluation seeds
   1,000,000..) in a pool of host processes started before anything
   touches the GPU; training frames stream through the GPU as they arrive,
   so only their level-4 data is kept.
2. Inputs: the level-4 intensities of the solver's own float32 pyramid (the
   images the network sees at inference).  Targets: the plain solver's
   (zero initialisation) level-0 flows of each training frame, restricted
   to level 4 (16 x 16 box average / 16).
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


def start_pool(workers):
    """A process pool whose workers are all running before the caller
    touches the GPU (they render on the host only)."""
    from concurrent.futures import ProcessPoolExecutor
    ex = ProcessPoolExecutor(max_workers=workers)
    list(ex.map(time.sleep, [0.2] * (2 * workers)))
    return ex


def level4_intensities(solver, H, W):
    """The four level-4 images of the solver's last frame from its own
    pyramid (float32 texels (I, G_x, G_y, 0)), shape (4, H >> 4, W >> 4)."""
    from paper_1610_07159_amd import sf
    tex = sf.sf_debug_read(solver.ctx, sf.SF_DBG_TEX, LEVEL_IN)
    return tex.reshape(4, H >> LEVEL_IN, W >> LEVEL_IN, 4)[..., 0].copy()


def stream_training_data(ex, W, H, seeds, sched, log=print, max_disp=None, blobs=0,
                         deadline=None):
    """Renders the training frames in the pool and solves each on the GPU
    as it arrives (plain solver, zero initialisation); returns the level-4
    inputs x (N, 4, h, w) and targets y (N, 6, h, w), float32, of the
    first N seeds (all of them, or those done when time.time() passes
    deadline)."""
    import torch
    from paper_1610_07159_amd import SceneFlowSolver
    jobs = [(W, H, s, False, max_disp, blobs) for s in seeds]
    solver = SceneFlowSolver(W, H, **sched)
    xs, ys = [], []
    try:
        out = (torch.empty((H, W), device="cuda"), torch.empty((3, H, W), device="cuda"),
               torch.empty((6, H, W), device="cuda"))
        for k, f in enumerate(ex.map(_render, jobs, chunksize=1)):
            img = torch.from_numpy(f["imgs"]).cuda()
            solver.solve(img, f["calib"], out=out)
            xs.append(level4_intensities(solver, H, W))
            # restriction to level 4 (16 x 16 box average, floor sizes) on
            # the device: only the small target crosses to the host
            c = 1 << LEVEL_IN
            fl = out[2][:, :(H // c) * c, :(W // c) * c]
            ys.append((torch.nn.functional.avg_pool2d(fl[None], c)[0] / c).cpu().numpy())
            if (k + 1) % 10 == 0:
                log(f"  rendered and solved {k + 1}/{len(jobs)}")
            if deadline is not None and time.time() > deadline:
                log(f"  time limit: stopping after {k + 1} frames")
                break
    finally:
        solver.close()
    return np.stack(xs), np.stack(ys)


def epe_gpu(flows, truth):
    """epe() on the GPU: flows (6, H, W) device tensor, truth (pos, ok) host
    arrays."""
    import torch
    pos, ok = truth
    dev = flows.device
    H, W = flows.shape[1:]
    yy, xx = torch.meshgrid(torch.arange(H, device=dev, dtype=torch.float64),
                            torch.arange(W, device=dev, dtype=torch.float64), indexing="ij")
    f = flows.double()
    p = torch.from_numpy(np.asarray(pos)).to(dev).double()
    inside = torch.from_numpy(np.asarray(ok)).to(dev).clone()
    err = torch.zeros((H, W), device=dev, dtype=torch.float64)
    for c, (a, b, d) in enumerate(((-1, -1, 1), (1, -1, -1), (-1, 1, -1), (1, 1, 1))):
        px = xx + a * f[0] + b * f[2] + d * f[4]
        py = yy + a * f[1] + b * f[3] + d * f[5]
        err += torch.hypot(px - p[c, 0], py - p[c, 1])
        inside &= (p[c, 0] >= 0) & (p[c, 0] <= W - 1) & (p[c, 1] >= 0) & (p[c, 1] <= H - 1)
    return float((err / 4.0)[inside].mean())


def eval_sweep(frames, W, H, sched, init_mode, weights, n):
    """Mean EPE (GPU) and GPU ms/frame of solves with n Gauss-Newton steps
    per level; prediction-kept count for init_mode 1."""
    import torch
    from paper_1610_07159_amd import SceneFlowSolver, sf
    solver = SceneFlowSolver(W, H, init_mode=init_mode, **dict(sched, gn_iters=n))
    try:
        if init_mode:
            sf.sf_set_initializer(solver.ctx, weights)
        out = (torch.empty((H, W), device="cuda"), torch.empty((3, H, W), device="cuda"),
               torch.empty((6, H, W), device="cuda"))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        epes, ms, used = [], [], 0
        for f in frames:
            img = torch.from_numpy(f["imgs"]).cuda()
            solver.solve(img, f["calib"], out=out)  # graph, tiles, caches
            e0.record(solver.stream)
            solver.solve(img, f["calib"], out=out)
            e1.record(solver.stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
            epes.append(epe_gpu(out[2], f["truth"]))
            if init_mode:
                used += int(sf.sf_get_init_result(solver.ctx)[0])
    finally:
        solver.close()
    row = dict(gn_iters=n, epe_px=round(float(np.mean(epes)), 4),
               ms_per_frame=round(float(np.mean(ms)), 3))
    if init_mode:
        row["prediction_kept"] = used
    return float(np.mean(epes)), row


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


def conv_flops(B, h, w):
    """Multiply-adds x 2 of one forward pass of the network on B inputs of
    h x w (3 x 3 convolutions 4 -> 32 -> 32 -> 32 -> 32 -> 32 -> 6)."""
    chans = (4, 32, 32, 32, 32, 32, 6)
    return 2 * 9 * B * h * w * sum(a * b for a, b in zip(chans[:-1], chans[1:]))


def profile_trainer(h, w, batch, steps, log=print):
    """Times `steps` trainer steps (forward, L1 loss, backward, Adam) on
    random inputs; reports the achieved rate counting forward + input
    gradient + weight gradient as 3 forward passes of flops."""
    import torch
    from paper_1610_07159_amd import sf
    t = sf.sf_trainer_create(batch, h, w, torch.cuda.current_stream().cuda_stream)
    try:
        sf.sf_trainer_set_params(t, he_init(0))
        g = torch.Generator(device="cuda").manual_seed(0)
        x = torch.rand((batch, 4, h, w), device="cuda", generator=g)
        y = torch.randn((batch, 6, h, w), device="cuda", generator=g)
        for _ in range(5):
            sf.sf_trainer_step(t, x.data_ptr(), y.data_ptr(), batch, 1e-4, want_loss=False)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            sf.sf_trainer_step(t, x.data_ptr(), y.data_ptr(), batch, 1e-4, want_loss=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
    finally:
        sf.sf_trainer_destroy(t)
    tflops = 3 * conv_flops(batch, h, w) / (ms * 1e-3) / 1e12
    log(json.dumps(dict(batch=batch, height=h, width=w, steps=steps, ms_per_step=round(ms, 4),
                        step_tflop=round(3 * conv_flops(batch, h, w) / 1e12, 5),
                        tflop_per_s=round(tflops, 2))))


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
    ap.add_argument("--seed0", type=int, default=0, help="first training seed")
    ap.add_argument("--save-data", default=None,
                    help="write this run's training inputs and targets (float16) to this file")
    ap.add_argument("--load-data", nargs="*", default=[],
                    help="training inputs and targets written by earlier --save-data runs, "
                         "used together with this run's frames")
    ap.add_argument("--no-train", action="store_true",
                    help="only render, solve and save the training data")
    ap.add_argument("--time-limit", type=float, default=None,
                    help="stop rendering training frames after this many seconds "
                         "(counted from the start) and keep those done")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only time this many trainer steps on random level-4 inputs of "
                         "the frame size (batch --batch) and exit")
    args = ap.parse_args()
    log = lambda m: print(m, flush=True)  # noqa: E731
    if args.profile_steps:
        return profile_trainer(args.height >> LEVEL_IN, args.width >> LEVEL_IN, args.batch,
                               args.profile_steps, log)
    t_start = time.time()
    W, H = args.width, args.height
    sched_full = dict(SCHEDULE, levels=args.levels)
    scene = dict(max_disp=args.max_disp, blobs=args.blobs)
    import torch  # (the first import on a fresh machine takes a while)
    log("torch imported")
    # host workers first: nothing has touched the GPU yet
    ex = start_pool(args.workers)
    t0 = time.time()
    eval_seeds = range(1_000_000, 1_000_000 + args.eval)
    eval_frames = []
    for k, f in enumerate(ex.map(_render, [(W, H, s, True, args.max_disp, args.blobs)
                                           for s in eval_seeds], chunksize=1)):
        eval_frames.append(f)
        if (k + 1) % 10 == 0:
            log(f"  rendered {k + 1}/{args.eval} evaluation frames")
    log(f"rendered {len(eval_frames)} evaluation frames with truth in {time.time() - t0:.0f} s")

    torch.cuda.set_device(0)
    t1 = time.time()
    x, y = stream_training_data(ex, W, H, range(args.seed0, args.seed0 + args.frames),
                                sched_full, log, **scene,
                                deadline=(t_start + args.time_limit if args.time_limit else None))
    ex.shutdown(cancel_futures=True)
    log(f"{len(x)} training frames rendered and solved in {time.time() - t1:.0f} s; "
        f"inputs {x.shape}, targets {y.shape}")
    if args.save_data:
        with open(args.save_data, "wb") as f:
            np.savez(f, x=x.astype(np.float16), y=y.astype(np.float16),
                     seeds=np.arange(args.seed0, args.seed0 + len(x)))
        log(f"saved {args.save_data}")
    n_loaded = 0
    for path in args.load_data:
        with open(path, "rb") as f:
            z = np.load(f, allow_pickle=False)
            x = np.concatenate([x, z["x"].astype(np.float32)])
            y = np.concatenate([y, z["y"].astype(np.float32)])
            n_loaded += len(z["x"])
    if n_loaded:
        log(f"training on {len(x)} frames ({n_loaded} from earlier runs)")
    if args.no_train:
        return
    t2 = time.time()
    params, curve = train_gpu(x, y, args.epochs, args.batch, args.lr, seed=1, log=log)
    log(f"trained in {time.time() - t2:.1f} s")
    np.save(args.out, params)

    # equal EPE: target = plain at the full schedule; fewest steps per level
    # reaching it for plain and learned
    full = sched_full["gn_iters"]
    target, full_row = eval_sweep(eval_frames, W, H, sched_full, 0, None, full)
    log(f"plain, {full} GN/level: EPE {target:.4f} px, {full_row['ms_per_frame']} ms/frame")
    sweeps, reach = {}, {}
    for name, mode in (("plain", 0), ("learned", 1)):
        sweeps[name], reach[name] = [], None
        for n in range(1, full + 1):
            e, row = (target, full_row) if (mode == 0 and n == full) else \
                eval_sweep(eval_frames, W, H, sched_full, mode, params, n)
            sweeps[name].append(row)
            log(f"{name}, {n} GN/level: {row}")
            if e <= target:
                reach[name] = row
                break
    speedup = (round(reach["plain"]["ms_per_frame"] / reach["learned"]["ms_per_frame"], 3)
               if reach["plain"] and reach["learned"] else None)
    report = dict(
        frames=len(x), eval_frames=args.eval, eval_seeds=[eval_seeds[0], eval_seeds[-1]],
        size=f"{W}x{H}", schedule=sched_full, max_disp=args.max_disp, blobs=args.blobs,
        epochs=args.epochs, batch=args.batch, lr=args.lr,
        loss_curve=[round(c, 5) for c in curve], target_epe_px=round(target, 4),
        plain_full_schedule=full_row, plain_sweep=sweeps["plain"],
        learned_sweep=sweeps["learned"], plain_at_target=reach["plain"],
        learned_at_target=reach["learned"], speedup_at_equal_epe=speedup,
        command="python -m paper_1610_07159_amd.train_init " + " ".join(sys.argv[1:]))
    with open(args.report, "w") as f:
        json.dump(report, f, indent=1)
    log(json.dumps(dict(target=report["target_epe_px"], plain=reach["plain"],
                        learned=reach["learned"], speedup=speedup)))


if __name__ == "__main__":
    main()
