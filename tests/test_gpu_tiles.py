"""sf_tile_variant names the PCG iteration kernel a solve ran: the shape
tile_mode forces (0: default, 2-4: the alternatives), one of the candidate
shapes under autotuning (tile_mode 1), for single frames and batches, and
SF_ERR_STATE before the first batch.  Measurements use it to report the
counters of the kernel they timed."""
import numpy as np
import pytest

from synth import make_frame, sized_config

pytestmark = pytest.mark.gpu

W, H = 200, 150
PRM = dict(levels=3, grid_stride=4, gn_iters=2, pcg_iters=4)


def _expected(tile_mode, apply):
    n_var = 4 if apply >= 1 else 3  # node-block shapes / matrix-free shapes at stride 4
    v = tile_mode - 1 if tile_mode >= 2 else 0
    return v if v < n_var else 0


@pytest.mark.parametrize("apply", [0, 2])
def test_tile_variant_reports_the_shape_that_ran(apply):
    import torch
    from paper_1610_07159_amd import sf, SceneFlowSolver
    imgs, calib, _ = make_frame(sized_config(W, H, max_disp=10.0), 7)
    x = torch.from_numpy(np.asarray(imgs, np.float32)).cuda().contiguous()
    for mode in (0, 1, 2, 3, 4):
        print(f"apply_mode {apply}, tile_mode {mode}", flush=True)
        s = SceneFlowSolver(W, H, tile_mode=mode, apply_mode=apply, **PRM)
        try:
            with pytest.raises(sf.SfError, match="SF_ERR_STATE"):
                sf.sf_tile_variant(s.ctx, True, 0)
            s.solve(x, calib)
            torch.cuda.synchronize()
            got = [sf.sf_tile_variant(s.ctx, False, l) for l in range(PRM["levels"])]
            with pytest.raises(sf.SfError, match="SF_ERR_INVALID_ARG"):
                sf.sf_tile_variant(s.ctx, False, PRM["levels"])
            s.solve_batch([(x, calib), (x, calib)])
            torch.cuda.synchronize()
            got_b = [sf.sf_tile_variant(s.ctx, True, l) for l in range(PRM["levels"])]
        finally:
            s.close()
        if mode == 1:
            n_var = 4 if apply >= 1 else 3
            assert all(0 <= v < n_var for v in got + got_b), (got, got_b)
        else:
            want = _expected(mode, apply)
            assert got == [want] * PRM["levels"], (mode, got)
            assert got_b == [want] * PRM["levels"], (mode, got_b)
