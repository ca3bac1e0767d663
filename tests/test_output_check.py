"""The output checker of the GPU tests (depth and 3D flow, Sec. 3) must
accept the oracle's own output and reject plausible mistakes of an output
kernel: a sign error in the 3D flow, f_x and f_y swapped, the disparity of
the wrong time, a back-projection without c_y, a one-pixel shift.  Runs on the
CPU with the oracle's output standing in for a kernel's."""
import numpy as np
import pytest

import oracle.halfway as O
from gpu_util import check_output


def _case(seed=0, W=48, H=36):
    rng = np.random.default_rng(seed)
    calib = dict(fx=40.0, fy=46.0, cx=22.3, cy=18.1, baseline=0.1,
                 F=[0, 0, 0, 0, 0, -1, 0, 1, 0])
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    flows = np.stack([-1.5 + 0.02 * x, 0.05 * np.sin(y / 5), 0.3 + 0.01 * y,
                      -0.2 + 0.01 * x, 0.01 * np.cos(x / 7), 0.02 * y / H])
    flows += rng.normal(0, 1e-3, flows.shape)
    flows = flows.reshape(6, -1).astype(np.float32)
    depth, flow3d, _ = O.output_from_flows(flows, W, H, calib)
    return flows, depth.astype(np.float32), flow3d.astype(np.float32), calib, W, H


def test_accepts_oracle_output():
    flows, depth, flow3d, calib, W, H = _case()
    assert check_output(depth, flow3d, flows, W, H, calib) > 0.9 * W * H
    # end to end with a perturbed reference within the stated flow error
    ref = flows + np.float32(0.01) * np.sign(np.random.default_rng(1).normal(size=flows.shape))
    check_output(depth, flow3d, flows, W, H, calib, ref, 0.01)


def test_nan_where_disparity_not_positive():
    flows, depth, flow3d, calib, W, H = _case()
    flows = flows.copy()
    flows[0, : W * 6] = 1.0      # s_x > 0, d_x ~ 0: disparity 2(d_x - s_x) < 0
    depth, flow3d, _ = O.output_from_flows(flows, W, H, calib)
    assert np.isnan(depth.reshape(-1)[: W * 6]).all()
    check_output(depth, flow3d, flows, W, H, calib)
    bad = depth.copy().reshape(-1)
    bad[: W * 6] = 1.0
    with pytest.raises(AssertionError):
        check_output(bad, flow3d, flows, W, H, calib)


@pytest.mark.parametrize("mistake", ["flow_sign", "fx_fy", "time", "no_cy", "shift"])
def test_rejects_mistakes(mistake):
    flows, depth, flow3d, calib, W, H = _case()
    if mistake == "flow_sign":
        flow3d = -flow3d
    elif mistake == "fx_fy":
        swapped = dict(calib, fx=calib["fy"], fy=calib["fx"])
        depth, flow3d, _ = O.output_from_flows(flows, W, H, swapped)
    elif mistake == "time":
        f = flows.reshape(6, -1).copy()
        f[2:] = -f[2:]               # t and t+1 exchanged: m, d change sign
        depth, _, _ = O.output_from_flows(f, W, H, calib)
    elif mistake == "no_cy":
        # Y back-projected without the principal point's y offset
        d2, f2, _ = O.output_from_flows(flows, W, H, dict(calib, cy=0.0))
        flow3d = np.stack([flow3d[0], f2[1], flow3d[2]])
    elif mistake == "shift":
        depth = np.roll(depth, 1, axis=1)
    with pytest.raises(AssertionError):
        check_output(depth, flow3d, flows, W, H, calib)
