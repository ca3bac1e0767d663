"""Writes the full-size solve goldens: the FP64 oracle's per-(level,
Gauss-Newton step) energies and its final level-0 node totals for the
benchmark workloads, so that GPU tests can compare whole solves at sizes the
oracle needs minutes for.

Calls only the oracle (oracle/halfway.py) and the seeded generator (synth/).
Each case is one solve of Algorithm 1 with the coarse-to-fine delta
hierarchy of Sec. 5.3 and the Gauss-Newton / PCG schedule of Sec. 5.1
(10 Gauss-Newton steps of 20 PCG iterations on every level).

Usage:  python tests/golden/make_fullsize.py [case ...]
        python tests/golden/make_fullsize.py --sensitivity [case ...]
Cases:  vga640x480_s4, hd1280x720_s4, hd1280x720_s8, hd1280x720_s2, and
        vga640x480_s4_learned: a frame outside the shipped network's
        training and evaluation seeds, solved with 2 Gauss-Newton steps
        per level from the learned initialisation (the network of
        paper_1610_07159_amd/weights/init_640x480.npy run by oracle/cnn.py in
        its bfloat16-emulating mode, with the energy fallback);
        vga640x480_s4_learned10: the same frame and network at the full
        schedule (10 Gauss-Newton steps per level)
Output: tests/golden/fullsize_<case>.npz with
  level, gn_iter (int32), energy, energy_after (float64), tau (float64)
      one entry per Gauss-Newton step, coarsest level first;
  terms (float64, n x 5): photo, grad, smooth, epi, mag before each step;
  total0 (float32, 6 x G_0): the final level-0 node totals, planes
      s_x, s_y, m_x, m_y, d_x, d_y (node-major within a plane);
  images_sha256: sha256 of the float32 input images (4, H, W), so a test
      can tell that the generator reproduced the same frame;
  meta: JSON string with the workload, seed, sizes and schedule (learned
      case: also whether the prediction was kept and both fallback
      energies).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle.cnn as C  # noqa: E402
import oracle.halfway as O  # noqa: E402
from synth import make_frame, vga_config, hd_config  # noqa: E402

# name -> (generator config, seed, width, height, levels, stride, gn_iters,
#          network weights file or None)
CASES = {
    "vga640x480_s4": ("vga", 1, 640, 480, 5, 4, 10, None),
    "hd1280x720_s4": ("hd", 2, 1280, 720, 6, 4, 10, None),
    "hd1280x720_s8": ("hd", 2, 1280, 720, 6, 8, 10, None),
    "hd1280x720_s2": ("hd", 2, 1280, 720, 6, 2, 10, None),
    "vga640x480_s4_learned": ("vga", 1_000_050, 640, 480, 5, 4, 2, "init_640x480.npy"),
    "vga640x480_s4_learned10": ("vga", 1_000_050, 640, 480, 5, 4, 10, "init_640x480.npy"),
}
PCG_ITERS = 20
WEIGHTS = os.path.join(ROOT, "paper_1610_07159_amd", "weights")


def frame(kind, seed):
    cfg = {"vga": vga_config, "hd": hd_config}[kind]()
    # the learned case's frame: the 640x480 generator as the stored
    # network was trained on
    imgs, calib, _ = make_frame(cfg, seed)
    return imgs, calib


def run(name):
    kind, seed, W, H, levels, stride, gn_iters, weights = CASES[name]
    imgs, calib = frame(kind, seed)
    assert imgs.shape == (4, H, W) and imgs.dtype == np.float32
    p = O.Params(levels=levels, grid_stride=stride, gn_iters=gn_iters,
                 pcg_iters=PCG_ITERS)
    rec = []
    extra = {}
    t0 = time.time()
    if weights is None:
        res = O.solve(imgs.astype(np.float64), calib, p, record=rec)
    else:
        flat = np.load(os.path.join(WEIGHTS, weights), allow_pickle=False).astype(np.float64)
        res, used, e_pred, e_zero = C.solve_learned(flat, imgs.astype(np.float64), calib, p,
                                                    record=rec, bf16=True)
        extra = dict(weights=weights, prediction_kept=bool(used), e_pred=float(e_pred),
                     e_zero=float(e_zero))
    dt = time.time() - t0
    levels_l, gn_l = [], []
    count = {}
    for r in rec:
        levels_l.append(r["level"])
        gn_l.append(count.get(r["level"], 0))
        count[r["level"]] = gn_l[-1] + 1
    terms = np.array([[r["terms"][k] for k in ("photo", "grad", "smooth", "epi", "mag")]
                      for r in rec])
    meta = dict(case=name, generator=kind, seed=seed, width=W, height=H,
                levels=levels, grid_stride=stride, gn_iters=gn_iters,
                pcg_iters=PCG_ITERS, oracle_seconds=round(dt, 1), **extra)
    out = os.path.join(HERE, f"fullsize_{name}.npz")
    np.savez_compressed(
        out,
        level=np.array(levels_l, np.int32), gn_iter=np.array(gn_l, np.int32),
        energy=np.array([r["energy"] for r in rec]),
        energy_after=np.array([r["energy_after"] for r in rec]),
        tau=np.array([r["tau"] for r in rec]), terms=terms,
        total0=np.asarray(res["total"], np.float32).reshape(6, -1),
        images_sha256=np.array(hashlib.sha256(imgs.tobytes()).hexdigest()),
        meta=np.array(json.dumps(meta)))
    print(f"{name}: {len(rec)} steps, {dt:.0f} s -> {out}", flush=True)


def sensitivity(name):
    """The oracle's own sensitivity at this case: the solve repeated with
    its input images perturbed by one float32 rounding (each value times
    1 +- 2^-24, seeded signs) or, for the learned cases, with the chosen
    start of the coarsest level perturbed by +-2e-4 px (seeded signs; the
    size of the bf16 rounding flips between two implementations of the
    network), against the stored solve.  Writes
    tests/golden/sensitivity_<case>.json with the node-wise max |change| of
    the final level-0 totals: max, 99.9th percentile, median."""
    kind, seed, W, H, levels, stride, gn_iters, weights = CASES[name]
    imgs, calib = frame(kind, seed)
    p = O.Params(levels=levels, grid_stride=stride, gn_iters=gn_iters,
                 pcg_iters=PCG_ITERS)
    rng = np.random.default_rng(12345)
    x = imgs.astype(np.float64)
    if weights is None:
        x = x * (1.0 + rng.choice([-1.0, 1.0], x.shape) * 2.0 ** -24)
        res = O.solve(x, calib, p)
        what = "input images times 1 +- 2^-24 (one float32 rounding), seeded signs"
    else:
        flat = np.load(os.path.join(WEIGHTS, weights), allow_pickle=False).astype(np.float64)
        cand, _ = C.predict_coarsest(flat, x, p, bf16=True)
        lc = p.levels - 1
        pyr = O.pyramid(x, p.levels)
        li = O.LevelImages.build(pyr[lc])
        grid = O.Grid(li.shape[1], li.shape[0], p.grid_stride)
        base, _, _, _ = C.choose_init(li, grid, O.level_calib_F(O.Calib.from_dict(calib).F, lc),
                                      p, cand)
        base = base + rng.choice([-1.0, 1.0], base.shape) * 2e-4
        res = O.solve(x, calib, p, init_coarsest=base)
        what = "coarsest-level start +- 2e-4 px, seeded signs"
    z = np.load(os.path.join(HERE, f"fullsize_{name}.npz"))
    d = np.abs(np.asarray(res["total"]) - z["total0"].astype(np.float64)).max(axis=0)
    out = dict(case=name, perturbation=what, max_px=float(d.max()),
               p999_px=float(np.quantile(d, 0.999)), median_px=float(np.median(d)))
    path = os.path.join(HERE, f"sensitivity_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args[:1] == ["--sensitivity"]:
        for n in args[1:] or list(CASES):
            sensitivity(n)
    else:
        for n in args or list(CASES):
            run(n)
