"""Video mode (temporal initialisation of each level's deltas, Sec. 5.3)
against the oracle's frame-by-frame sequence solve, through the C ABI.
Tolerances as for single solves: per-(frame, level, GN step) energy within
1e-4 relative, final flows within 0.02 px."""
import numpy as np
import pytest

import oracle.halfway as O
from synth import make_sequence, sized_config

from gpu_util import GpuCase, oracle_params

pytestmark = pytest.mark.gpu


def _sequence(W=100, H=76, n=3, seed=11, disp=0.05):
    frames, calib, _ = make_sequence(sized_config(W, H, max_disp=disp * W), seed, n)
    return frames, calib


def _check_frame(log, rec, flows, res, e_tol=1e-4, f_tol=0.02):
    assert len(log) == len(rec)
    for lg, ro in zip(log, rec):
        assert lg["level"] == ro["level"]
        rel = abs(lg["energy"] - ro["energy"]) / abs(ro["energy"])
        assert rel <= e_tol, (lg["level"], lg["gn_iter"], lg["energy"], ro["energy"])
        assert lg["energy_after"] <= lg["energy"]
    grid = res["grid"]
    ref = grid.to_pixels(res["total"]).reshape(6, grid.H, grid.W)
    err = np.abs(flows - ref).max()
    assert err <= f_tol, err


@pytest.mark.parametrize("apply,stride,extra", [
    (0, 4, {}), (2, 4, {}), (2, 8, {}),
    # every map of Sec. 5.3 at once: illumination correction and occlusion
    # maps on top of the temporal initialisation
    (2, 4, dict(illum=1, occlusion=1))])
def test_sequence_parity(apply, stride, extra):
    frames, calib = _sequence()
    prm = dict(levels=3, grid_stride=stride, gn_iters=3, pcg_iters=8, apply_mode=apply,
               temporal=1, **extra)
    p = oracle_params(**prm)
    recs = []
    res = O.solve_sequence([f.astype(np.float64) for f in frames], calib, p, record=recs)
    g = GpuCase(frames[0], calib, **prm)
    try:
        for k, f in enumerate(frames):
            g.load(f)
            _, _, flows = g.solve()
            log, code = g.log()
            assert code == 0
            _check_frame(log, recs[k], flows, res[k])
    finally:
        g.close()


def test_first_frame_and_reset_equal_a_plain_solve():
    """The first solve of a video context, and the first after
    sf_reset_sequence, equal the solve of a context without video mode
    bitwise (the temporal state is not read); a second frame differs."""
    frames, calib = _sequence(seed=12)
    prm = dict(levels=3, grid_stride=4, gn_iters=3, pcg_iters=8)
    plain = GpuCase(frames[1], calib, **prm)
    try:
        ref = plain.solve()
    finally:
        plain.close()
    g = GpuCase(frames[0], calib, temporal=1, **prm)
    try:
        g.solve()
        g.load(frames[1])
        warm = g.solve()
        assert np.abs(warm[2] - ref[2]).max() > 0
        g.sf.sf_reset_sequence(g.ctx)
        fresh = g.solve()
        for a, b in zip(fresh, ref):
            np.testing.assert_array_equal(a, b)
    finally:
        g.close()


def test_batch_rejects_video_mode():
    import torch
    from paper_1610_07159_amd import sf, SceneFlowSolver
    frames, calib = _sequence(n=1)
    solver = SceneFlowSolver(100, 76, levels=3, grid_stride=4, gn_iters=2, pcg_iters=4)
    try:
        dev = [(torch.from_numpy(frames[0]).cuda().contiguous(), calib)]
        params = sf.sf_params_default(levels=3, grid_stride=4, gn_iters=2, pcg_iters=4,
                                      temporal=1)
        with pytest.raises(sf.SfError):
            solver.solve_batch(dev, params=params)
    finally:
        solver.close()
