"""sf_solve_noalloc (workspace in the library's static device array, no
allocation) against sf_solve of a context with the same parameters: two
calls in a row, the second on a smaller frame, each bitwise equal to the
context's solve (direct launches, default tiles); a frame too large for the
array is rejected on the host."""
import numpy as np
import pytest

from synth import make_frame, sized_config

pytestmark = pytest.mark.gpu


def _frame(W, H, seed):
    imgs, calib, _ = make_frame(sized_config(W, H, max_disp=0.05 * W), seed)
    return imgs, calib


def _outputs(H, W):
    import torch
    return (torch.full((H, W), -1.0, device="cuda"), torch.full((3, H, W), -1.0, device="cuda"),
            torch.full((6, H, W), -1.0, device="cuda"))


def _solve_context(imgs, calib, prm):
    import torch
    from paper_1610_07159_amd import sf
    _, H, W = imgs.shape
    p = sf.sf_params_default(**dict(prm, exec_mode=1, tile_mode=0))
    stream = torch.cuda.current_stream()
    ctx = sf.sf_create(W, H, p, int(stream.cuda_stream))
    try:
        dev = torch.from_numpy(imgs).cuda().contiguous()
        out = _outputs(H, W)
        cal = sf.make_calib(calib["fx"], calib["fy"], calib["cx"], calib["cy"],
                            calib["baseline"], calib["F"])
        sf.sf_solve(ctx, *[dev[k].data_ptr() for k in range(4)], cal, None,
                    *[o.data_ptr() for o in out])
        torch.cuda.synchronize()
        return [o.cpu().numpy() for o in out]
    finally:
        sf.sf_destroy(ctx)


def _solve_noalloc(imgs, calib, prm):
    import torch
    from paper_1610_07159_amd import sf
    _, H, W = imgs.shape
    p = sf.sf_params_default(**prm)
    dev = torch.from_numpy(imgs).cuda().contiguous()
    out = _outputs(H, W)
    cal = sf.make_calib(calib["fx"], calib["fy"], calib["cx"], calib["cy"],
                        calib["baseline"], calib["F"])
    stream = torch.cuda.current_stream()
    sf.sf_solve_noalloc(W, H, [dev[k].data_ptr() for k in range(4)], cal, p,
                        *[o.data_ptr() for o in out], stream=int(stream.cuda_stream))
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


@pytest.mark.parametrize("apply", [0, 2])
def test_noalloc_matches_context_solve(apply):
    cases = [((320, 240), dict(levels=4, grid_stride=4, gn_iters=3, pcg_iters=10)),
             ((200, 150), dict(levels=3, grid_stride=4, gn_iters=3, pcg_iters=10))]
    for k, ((W, H), prm) in enumerate(cases):
        imgs, calib = _frame(W, H, 40 + k)
        prm = dict(prm, apply_mode=apply)
        got = _solve_noalloc(imgs, calib, prm)
        want = _solve_context(imgs, calib, prm)
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b)
        assert np.isfinite(got[2]).all() and np.abs(got[2]).max() > 0.1


def test_noalloc_rejects_a_frame_beyond_the_array():
    """1280 x 720 needs far more workspace than the array holds: rejected on
    the host before anything is enqueued."""
    import torch
    from paper_1610_07159_amd import sf
    _, calib = _frame(64, 48, 3)
    p = sf.sf_params_default(levels=5, grid_stride=2, gn_iters=1, pcg_iters=2)
    cal = sf.make_calib(calib["fx"], calib["fy"], calib["cx"], calib["cy"],
                        calib["baseline"], calib["F"])
    imgs = torch.zeros((4, 720, 1280), device="cuda")
    out = _outputs(720, 1280)
    with pytest.raises(sf.SfError) as e:
        sf.sf_solve_noalloc(1280, 720, [imgs[k].data_ptr() for k in range(4)], cal, p,
                            *[o.data_ptr() for o in out])
    assert e.value.code == -2
    assert "exceeds" in sf.lib.sf_last_error().decode()
    torch.cuda.synchronize()
    assert (out[0] == -1.0).all()
