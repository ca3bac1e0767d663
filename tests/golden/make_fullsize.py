"""Writes the full-size solve goldens: the FP64 oracle's per-(level,
Gauss-Newton step) energies and its final level-0 node totals for the
benchmark workloads, so that GPU tests can compare whole solves at sizes the
oracle needs minutes for.

Calls only the oracle (oracle/halfway.py) and the seeded generator (synth/).
Each case is one solve of Algorithm 1 with the coarse-to-fine delta
hierarchy of Sec. 5.3 and the Gauss-Newton / PCG schedule of Sec. 5.1
(10 Gauss-Newton steps of 20 PCG iterations on every level).

Usage:  python tests/golden/make_fullsize.py [case ...]
Cases:  vga640x480_s4, hd1280x720_s4, hd1280x720_s8, hd1280x720_s2
Output: tests/golden/fullsize_<case>.npz with
  level, gn_iter (int32), energy, energy_after (float64), tau (float64)
      one entry per Gauss-Newton step, coarsest level first;
  terms (float64, n x 5): photo, grad, smooth, epi, mag before each step;
  total0 (float32, 6 x G_0): the final level-0 node totals, planes
      s_x, s_y, m_x, m_y, d_x, d_y (node-major within a plane);
  images_sha256: sha256 of the float32 input images (4, H, W), so a test
      can tell that the generator reproduced the same frame;
  meta: JSON string with the workload, seed, sizes and schedule.
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

import oracle.halfway as O  # noqa: E402
from synth import make_frame, vga_config, hd_config  # noqa: E402

# name -> (generator config, seed, width, height, levels, stride)
CASES = {
    "vga640x480_s4": ("vga", 1, 640, 480, 5, 4),
    "hd1280x720_s4": ("hd", 2, 1280, 720, 6, 4),
    "hd1280x720_s8": ("hd", 2, 1280, 720, 6, 8),
    "hd1280x720_s2": ("hd", 2, 1280, 720, 6, 2),
}
GN_ITERS = 10
PCG_ITERS = 20


def frame(kind, seed):
    cfg = {"vga": vga_config, "hd": hd_config}[kind]()
    imgs, calib, _ = make_frame(cfg, seed)
    return imgs, calib


def run(name):
    kind, seed, W, H, levels, stride = CASES[name]
    imgs, calib = frame(kind, seed)
    assert imgs.shape == (4, H, W) and imgs.dtype == np.float32
    p = O.Params(levels=levels, grid_stride=stride, gn_iters=GN_ITERS,
                 pcg_iters=PCG_ITERS)
    rec = []
    t0 = time.time()
    res = O.solve(imgs.astype(np.float64), calib, p, record=rec)
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
                levels=levels, grid_stride=stride, gn_iters=GN_ITERS,
                pcg_iters=PCG_ITERS, oracle_seconds=round(dt, 1))
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


if __name__ == "__main__":
    for n in sys.argv[1:] or list(CASES):
        run(n)
