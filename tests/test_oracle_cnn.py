"""Pins of the learned-initialiser oracle (oracle/cnn.py) against
independent implementations: torch's float64 convolution and autograd,
torch.optim.Adam, torch's bfloat16 conversion, avg_pool2d, finite
differences, closed forms of the sampling, and the solver oracle's own
energy on a scene with known motion."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle.cnn as C
import oracle.halfway as O
from synth import make_frame, tiny_plane_config


def _torch_net(flat, x):
    params = C.unpack(flat)
    h = torch.tensor(x, dtype=torch.float64)
    ws = []
    for l, (W, b) in enumerate(params):
        Wt = torch.tensor(W, dtype=torch.float64, requires_grad=True)
        bt = torch.tensor(b, dtype=torch.float64, requires_grad=True)
        ws += [Wt, bt]
        h = F.conv2d(h, Wt, bt, padding=1)
        if l < len(params) - 1:
            h = torch.relu(h)
    return h, ws


def test_parameter_count_and_packing():
    assert C.N_PARAMS == 4 * 32 * 9 + 4 * 32 * 32 * 9 + 32 * 6 * 9 + 5 * 32 + 6 == 39910
    flat = np.arange(C.N_PARAMS, dtype=np.float64)
    np.testing.assert_array_equal(C.pack(C.unpack(flat)), flat)
    W0, b0 = C.unpack(flat)[0]
    assert W0.shape == (32, 4, 3, 3) and W0[1, 2, 0, 1] == 1 * 36 + 2 * 9 + 1
    assert b0[0] == 4 * 32 * 9


def test_forward_matches_torch_conv():
    rng = np.random.default_rng(0)
    flat = C.init_params(1) + rng.normal(0, 0.01, C.N_PARAMS)
    x = rng.normal(size=(2, 4, 9, 13))
    out, acts = C.forward(flat, x)
    ref, _ = _torch_net(flat, x)
    np.testing.assert_allclose(out, ref.detach().numpy(), rtol=0, atol=1e-12)
    assert len(acts) == 7 and acts[3].shape == (2, 32, 9, 13)


def test_backward_matches_torch_autograd():
    rng = np.random.default_rng(2)
    flat = C.init_params(3) + rng.normal(0, 0.05, C.N_PARAMS)
    x = rng.normal(size=(2, 4, 7, 10))
    tgt = rng.normal(size=(2, 6, 7, 10))
    out, acts = C.forward(flat, x)
    loss, dout = C.l1_loss(out, tgt)
    g = C.backward(flat, acts, dout)
    ref, ws = _torch_net(flat, x)
    tl = (ref - torch.tensor(tgt)).abs().mean()
    tl.backward()
    assert loss == pytest.approx(tl.item(), abs=1e-14)
    gref = np.concatenate([w.grad.numpy().ravel() for w in ws])
    np.testing.assert_allclose(g, gref, rtol=0, atol=1e-12)


def test_backward_finite_differences():
    rng = np.random.default_rng(4)
    flat = C.init_params(5)
    x = rng.normal(size=(1, 4, 6, 6))
    tgt = rng.normal(size=(1, 6, 6, 6))
    out, acts = C.forward(flat, x)
    g = C.backward(flat, acts, C.l1_loss(out, tgt)[1])
    h = 1e-6
    for k in rng.choice(C.N_PARAMS, 25, replace=False):
        e = np.zeros(C.N_PARAMS)
        e[k] = h
        lp = C.l1_loss(C.forward(flat + e, x)[0], tgt)[0]
        lm = C.l1_loss(C.forward(flat - e, x)[0], tgt)[0]
        # the L1 loss and ReLU have kinks; skip a parameter whose step
        # crosses one (the two one-sided slopes differ)
        l0 = C.l1_loss(out, tgt)[0]
        if abs((lp - l0) - (l0 - lm)) > 1e-9:
            continue
        assert g[k] == pytest.approx((lp - lm) / (2 * h), abs=1e-7)


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(4)]
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, 1):
        p, m, v = C.adam_step(p, g, m, v, t, 3e-3)
        opt.zero_grad()
        pt.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=0, atol=1e-13)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(7)
    a = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0]]).astype(np.float32)
    ref = torch.tensor(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(C.bf16_round(a), ref)


def test_restriction_is_box_average():
    rng = np.random.default_rng(8)
    f = rng.normal(size=(6, 96, 160))
    r = C.restrict_flows(f)
    ref = F.avg_pool2d(torch.tensor(f)[None], 16)[0].numpy() / 16
    np.testing.assert_allclose(r, ref, rtol=0, atol=1e-14)
    # odd sizes: the same as four 2x2 box steps of the oracle's pyramid
    g = rng.normal(size=(6, 75, 101))
    rep = g.copy()
    for _ in range(4):
        rep = O.downsample(rep)
    np.testing.assert_allclose(C.restrict_flows(g), rep / 16, rtol=0, atol=1e-14)


def test_sampling_at_nodes_closed_forms():
    # level 4 is the coarsest: nodes sample the prediction at their own
    # positions, which equals torch's bilinear sampling (pixel centres)
    rng = np.random.default_rng(9)
    pred = rng.normal(size=(6, 30, 40))
    grid = O.Grid(40, 30, 4)
    out = C.sample_at_nodes(pred, grid, 4)
    nx, ny = grid.node_xy()
    gx = (nx + 0.5) / 40 * 2 - 1
    gy = (ny + 0.5) / 30 * 2 - 1
    gridt = torch.tensor(np.stack([gx, gy], -1)[None, None])
    ref = F.grid_sample(torch.tensor(pred)[None], gridt, mode="bilinear",
                        padding_mode="border", align_corners=False)[0, :, 0].numpy()
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12)
    # coarsest level 5: a flow field affine in level-4 pixel coordinates is
    # reproduced exactly at interior nodes and halved in level-5 pixels
    yy, xx = np.mgrid[0:45, 0:80].astype(np.float64)
    aff = np.stack([0.3 * xx - 0.1 * yy + 2.0] * 6)
    g5 = O.Grid(40, 22, 4)
    s5 = C.sample_at_nodes(aff, g5, 5)
    nx5, ny5 = g5.node_xy()
    u, v = 2 * (nx5 + 0.5) - 0.5, 2 * (ny5 + 0.5) - 0.5
    inner = (u <= 79) & (v <= 44)
    np.testing.assert_allclose(s5[0][inner], ((0.3 * u - 0.1 * v + 2.0) / 2)[inner],
                               rtol=0, atol=1e-12)


def _plane_level():
    imgs, calib, scene = make_frame(tiny_plane_config(), 0, noise=False)
    p = O.Params(levels=1, grid_stride=8)
    pyr = O.pyramid(imgs.astype(np.float64), 1)
    li = O.LevelImages.build(pyr[0])
    grid = O.Grid(64, 48, 8)
    F_l = O.level_calib_F(O.Calib.from_dict(calib).F, 0)
    return li, grid, F_l, p, scene


def test_fallback_energies_against_solver_energy():
    li, grid, F_l, p, _ = _plane_level()
    zero = np.zeros((6, grid.G))
    rng = np.random.default_rng(10)
    cand = rng.normal(0, 0.3, (6, grid.G))
    ea, ez = C.fallback_energies(li, grid, F_l, p, cand, zero)
    # the same number from the solver oracle's energy: zero deltas, base =
    # candidate, cmask = the common visibility mask
    px, py = grid.pixel_xy()
    V = np.ones(grid.N, bool)
    for base in (cand, zero):
        P = O.positions(px, py, grid.to_pixels(base))
        V &= ((P[:, 0] >= 0) & (P[:, 0] <= 63) & (P[:, 1] >= 0) & (P[:, 1] <= 47)).all(0)
    for base, e in ((cand, ea), (zero, ez)):
        ls = O.LevelState(0, li, grid, base, V.astype(np.float64), np.ones(grid.G), F_l)
        assert e == pytest.approx(O.energy(ls, np.zeros((6, grid.G)), p)["total"], rel=1e-12)
    # identical candidates tie, and a tie keeps zero
    e1, e2 = C.fallback_energies(li, grid, F_l, p, zero, zero)
    assert e1 == e2
    base, used, _, _ = C.choose_init(li, grid, F_l, p, zero)
    assert not used and np.all(base == 0)


def test_fallback_prefers_the_true_motion_and_rejects_garbage():
    li, grid, F_l, p, scene = _plane_level()
    # closed-form node flows of the translating plane (generator truth)
    pos, ok = scene.halfway_truth()
    from synth import halfway_flows_from_positions
    s_, m_, d_ = halfway_flows_from_positions(pos)
    fl = np.concatenate([s_, m_, d_]).reshape(6, 48, 64)
    nx, ny = grid.node_xy()
    xi = np.clip(np.round(nx).astype(int), 0, 63)
    yi = np.clip(np.round(ny).astype(int), 0, 47)
    truth = fl[:, yi, xi]
    base, used, e_t, e_z = C.choose_init(li, grid, F_l, p, truth)
    assert used and e_t < e_z and np.array_equal(base, truth)
    garbage = np.random.default_rng(11).normal(0, 5.0, (6, grid.G))
    base, used, e_g, e_z2 = C.choose_init(li, grid, F_l, p, garbage)
    assert not used and e_g >= e_z2 and np.all(base == 0)


@pytest.mark.parametrize("name", ["init_640x480", "init_1280x720"])
def test_stored_networks_load_safely(name):
    """The shipped parameters are plain float32 arrays of the network's size
    (no pickled objects), with a report of their equal-EPE evaluation."""
    import json
    import os
    root = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1610_07159_amd", "weights")
    w = np.load(os.path.join(root, name + ".npy"), allow_pickle=False)
    assert w.dtype == np.float32 and w.shape == (C.N_PARAMS,)
    assert np.isfinite(w).all()
    with open(os.path.join(root, name + "_report.json")) as f:
        rep = json.load(f)
    if "learned_at_target" in rep:
        # each method at the fewest steps per level reaching the plain
        # solver's full-schedule EPE
        assert rep["learned_at_target"]["epe_px"] <= rep["target_epe_px"]
        assert rep["learned_at_target"]["gn_iters"] < rep["plain_at_target"]["gn_iters"]
    else:
        assert rep["equal_epe"]["gn_iters"] < rep["plain"]["gn_iters"]
