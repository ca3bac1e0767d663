"""Occlusion maps (Sec. 5.3) against the oracle, through the C ABI.  The
map of one level is compared pixel by pixel on geometries with real
occlusions: a pixel may differ only where the oracle finds its decision
within float32 rounding of a threshold (occlusion_fragile: 1e-3 px,
5e-4 relative).  Solves with maps on: per-(level, GN step) energy within
1e-4 relative and final flows within 0.02 px, as for plain solves."""
import numpy as np
import pytest

import oracle.halfway as O
from synth import make_frame, sized_config

from gpu_util import GpuCase, oracle_params

pytestmark = pytest.mark.gpu


def _step_geometry(grid, seed, Df=10.0, Db=3.0):
    """Node values of a raised square (disparity Df) over a tilted
    background (Db): smooth flows with a depth discontinuity that occludes
    in all four views."""
    rng = np.random.default_rng(seed)
    nx, ny = grid.node_xy()
    u, v = nx / grid.W, ny / grid.H
    cx, cy = 0.5 + 0.1 * rng.random(), 0.5 + 0.1 * rng.random()
    fg = (np.abs(u - cx) < 0.25) & (np.abs(v - cy) < 0.25)
    D = np.where(fg, Df, Db) + 0.7 * u + 0.4 * v * v
    tot = np.zeros((6, grid.G))
    tot[4] = 0.17 * np.sin(3 * u + rng.random())
    tot[5] = 0.07 + 0.05 * u
    tot[0] = -D / 2 + tot[4]
    tot[1] = 0.13 + 0.1 * v
    tot[2] = 0.73 + 0.5 * u
    tot[3] = -0.41 + 0.2 * u * v
    return tot


@pytest.mark.parametrize("W,H,stride,levels,level", [
    (104, 78, 4, 2, 1), (161, 121, 3, 2, 1), (130, 98, 5, 3, 2),
    # full size: the 320 x 240 and 80 x 60 levels of the 640 x 480 pyramid
    (640, 480, 4, 5, 1), (640, 480, 4, 5, 3)])
def test_occlusion_stage_parity(W, H, stride, levels, level):
    cfg = sized_config(W, H, max_disp=0.05 * W)
    imgs, calib, _ = make_frame(cfg, 31)
    prm = dict(levels=levels, grid_stride=stride, gn_iters=2, pcg_iters=4, occlusion=1)
    g = GpuCase(imgs, calib, **prm)
    try:
        g.set_images()
        g.run(g.sf.SF_STAGE_LEVEL_INIT, level)
        Hl, Wl = H >> level, W >> level
        grid = O.Grid(Wl, Hl, stride)
        tot = _step_geometry(grid, level).astype(np.float32)
        g.write(g.sf.SF_DBG_BASE, level, np.zeros_like(tot))
        g.write(g.sf.SF_DBG_DELTA, level, tot)
        g.run(g.sf.SF_STAGE_OCC, level)
        got = g.read(g.sf.SF_DBG_OCC, level - 1).astype(bool)
    finally:
        g.close()
    Hf, Wf = H >> (level - 1), W >> (level - 1)
    t64 = tot.astype(np.float64)
    ref = O.box_upsample(O.occlusion_map(grid, t64), Wf, Hf).reshape(-1) > 0.5
    frag = O.box_upsample(O.occlusion_fragile(grid, t64).astype(np.float64), Wf, Hf)
    frag = frag.reshape(-1) > 0.5
    assert (~ref).sum() > 0.01 * ref.size   # the geometry does occlude
    assert frag.mean() < 0.02
    diff = got != ref
    assert not (diff & ~frag).any(), np.nonzero(diff & ~frag)[0][:10]


@pytest.mark.parametrize("W,H,stride,apply", [(100, 76, 4, 2), (96, 72, 3, 0),
                                              (160, 120, 4, 2)])
def test_occlusion_solve_parity(W, H, stride, apply):
    imgs, calib, _ = make_frame(sized_config(W, H, max_disp=0.05 * W, n_blobs=2), 21)
    prm = dict(levels=3, grid_stride=stride, gn_iters=4, pcg_iters=10, apply_mode=apply,
               occlusion=1)
    p = oracle_params(**prm)
    assert p.occlusion
    rec = []
    res = O.solve(imgs.astype(np.float64), calib, p, record=rec)
    g = GpuCase(imgs, calib, **prm)
    try:
        _, _, flows = g.solve()
        log, code = g.log()
    finally:
        g.close()
    assert code == 0 and len(log) == len(rec)
    for lg, ro in zip(log, rec):
        rel = abs(lg["energy"] - ro["energy"]) / abs(ro["energy"])
        assert rel <= 1e-4, (lg["level"], lg["gn_iter"], lg["energy"], ro["energy"])
    grid = res["grid"]
    ref = grid.to_pixels(res["total"]).reshape(6, grid.H, grid.W)
    assert np.abs(flows - ref).max() <= 0.02


def test_occlusion_batch_matches_single_frames_bitwise():
    import torch
    from paper_1610_07159_amd import sf, SceneFlowSolver
    prm = dict(levels=3, grid_stride=4, gn_iters=3, pcg_iters=8, occlusion=1)
    frames = [make_frame(sized_config(160, 120, n_blobs=2), 22)[:2],
              make_frame(sized_config(96, 72, n_blobs=2), 23)[:2]]
    solver = SceneFlowSolver(160, 120, exec_mode=0, **prm)
    try:
        dev = [(torch.from_numpy(i).cuda().contiguous(), c) for i, c in frames]
        outs = solver.solve_batch(dev, params=sf.sf_params_default(exec_mode=0, **prm))
        torch.cuda.synchronize()
        batched = [tuple(t.cpu().numpy() for t in o) for o in outs]
    finally:
        solver.close()
    for (imgs, calib), b in zip(frames, batched):
        L = sf.sf_batch_levels(imgs.shape[2], imgs.shape[1], prm["levels"])
        g = GpuCase(imgs, calib, **dict(prm, levels=L))
        try:
            single = g.solve()
        finally:
            g.close()
        for x, y in zip(single, b):
            np.testing.assert_array_equal(x, y)
