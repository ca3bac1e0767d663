"""Illumination correction (Sec. 5.3) against the oracle, through the C
ABI, on scenes whose right camera has a different gain and offset.
Tolerances as for single solves: per-(level, GN step) energy within 1e-4
relative, final flows within 0.02 px."""
from dataclasses import replace

import numpy as np
import pytest

import oracle.halfway as O
from synth import make_frame, sized_config

from gpu_util import GpuCase, oracle_params

pytestmark = pytest.mark.gpu


def _biased(W, H, seed, gain=1.08, bias=0.06, ramp=0.08):
    cfg = replace(sized_config(W, H, max_disp=0.05 * W), right_gain=gain, right_bias=bias,
                  right_ramp=ramp)
    imgs, calib, _ = make_frame(cfg, seed)
    return imgs, calib


@pytest.mark.parametrize("W,H,stride,apply", [(100, 76, 4, 0), (100, 76, 4, 2), (144, 104, 8, 2),
                                              (160, 120, 4, 2)])
def test_illum_solve_parity(W, H, stride, apply):
    imgs, calib = _biased(W, H, 21)
    prm = dict(levels=3, grid_stride=stride, gn_iters=4, pcg_iters=10, apply_mode=apply, illum=1)
    p = oracle_params(**prm)
    assert p.illum
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


def test_illum_batch_matches_single_frames_bitwise():
    import torch
    from paper_1610_07159_amd import sf, SceneFlowSolver
    prm = dict(levels=3, grid_stride=4, gn_iters=3, pcg_iters=8, illum=1)
    frames = [_biased(160, 120, 22), _biased(96, 72, 23)]
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
