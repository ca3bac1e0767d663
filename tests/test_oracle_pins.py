"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics (closed forms, library routines, finite differences, invariants).
None of these re-type the oracle's own formulas."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import torch
import torch.nn.functional as F

import oracle.halfway as O
from synth import make_frame, tiny_plane_config, rectified_F
from synth.scene import Scene, halfway_flows_from_positions


def _rng(seed=0):
    return np.random.default_rng(seed)


def _smooth_images(rng, H, W, n=4, blur=2):
    img = rng.random((n, H + 4 * blur, W + 4 * blur))
    t = torch.from_numpy(img)[:, None]
    k = torch.ones(1, 1, 2 * blur + 1, 2 * blur + 1, dtype=torch.float64)
    k = k / k.sum()
    out = F.conv2d(t, k)[:, 0].numpy()
    return out[:, blur:blur + H, blur:blur + W].copy()


# --------------------------------------------------------------------------
# P1: pyramid and gradient images
# --------------------------------------------------------------------------

def test_pyramid_matches_avg_pool2d():
    imgs = _rng(1).random((4, 37, 53))
    pyr = O.pyramid(imgs, 4)
    assert [p.shape for p in pyr] == [(4, 37, 53), (4, 18, 26), (4, 9, 13),
                                      (4, 4, 6)]
    for l in range(1, 4):
        ref = F.avg_pool2d(torch.from_numpy(pyr[l - 1]), 2).numpy()
        np.testing.assert_allclose(pyr[l], ref, rtol=0, atol=1e-15)


def test_gradients_match_numpy_gradient():
    img = _rng(2).random((11, 17))
    gx, gy = O.image_gradients(img)
    ny, nx = np.gradient(img)
    np.testing.assert_allclose(gx, nx, atol=1e-15)
    np.testing.assert_allclose(gy, ny, atol=1e-15)


# --------------------------------------------------------------------------
# P2: bilinear sampling
# --------------------------------------------------------------------------

def test_sample_values_match_grid_sample():
    rng = _rng(3)
    H, W = 9, 13
    img = rng.random((H, W))
    px = rng.uniform(-3, W + 2, 500)
    py = rng.uniform(-3, H + 2, 500)
    px[:20] = np.arange(20) % W   # exact texel positions too
    py[:20] = np.arange(20) % H
    px[20:25] = W - 1.0
    py[25:30] = H - 1.0
    val, _, _ = O.sample(img, px, py)
    grid = torch.from_numpy(np.stack([2 * px / (W - 1) - 1,
                                      2 * py / (H - 1) - 1], -1))[None, None]
    ref = F.grid_sample(torch.from_numpy(img)[None, None], grid,
                        mode="bilinear", padding_mode="border",
                        align_corners=True)[0, 0, 0].numpy()
    np.testing.assert_allclose(val, ref, rtol=0, atol=1e-14)


def test_sample_derivatives_match_fd():
    rng = _rng(4)
    H, W = 9, 13
    img = rng.random((H, W))
    px = rng.uniform(0.01, W - 1.01, 400)
    py = rng.uniform(0.01, H - 1.01, 400)
    # keep away from the interpolant's kinks at integer coordinates
    ok = (np.abs(px - np.round(px)) > 1e-3) & (np.abs(py - np.round(py)) > 1e-3)
    px, py = px[ok], py[ok]
    h = 1e-6
    _, dx, dy = O.sample(img, px, py)
    fdx = (O.sample(img, px + h, py)[0] - O.sample(img, px - h, py)[0]) / (2 * h)
    fdy = (O.sample(img, px, py + h)[0] - O.sample(img, px, py - h)[0]) / (2 * h)
    np.testing.assert_allclose(dx, fdx, rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(dy, fdy, rtol=1e-6, atol=1e-8)
    # clamped coordinates have zero derivative in the clamped direction
    _, dx, _ = O.sample(img, np.array([-1.5, W + 0.5]), np.array([3.3, 3.3]))
    assert np.all(dx == 0)


# --------------------------------------------------------------------------
# P3: warp grid interpolation (Eq. (7)) and prolongation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("W,H,s", [(64, 48, 8), (37, 29, 4), (20, 14, 2),
                                   (33, 17, 8), (16, 12, 8), (40, 30, 4)])
def test_warp_interp_matches_interpolate(W, H, s):
    grid = O.Grid(W, H, s)
    assert grid.Gx == math.ceil(W / s) and grid.Gy == math.ceil(H / s)
    nodes = _rng(5).normal(size=(6, grid.Gy, grid.Gx))
    ref = F.interpolate(torch.from_numpy(nodes)[None],
                        size=(grid.Gy * s, grid.Gx * s), mode="bilinear",
                        align_corners=False)[0, :, :H, :W].numpy()
    got = grid.to_pixels(nodes.reshape(6, -1)).reshape(6, H, W)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)
    # partition of unity (Sec. 3.3)
    np.testing.assert_allclose(grid.alpha.sum(0), 1.0, atol=1e-15)
    assert np.all(grid.alpha >= 0)


@pytest.mark.parametrize("Wf,Hf,s", [(64, 48, 4), (81, 37, 4), (40, 30, 8),
                                     (30, 22, 2)])
def test_prolong_matches_grid_sample(Wf, Hf, s):
    gf = O.Grid(Wf, Hf, s)
    gc = O.Grid(Wf // 2, Hf // 2, s)
    tc = _rng(6).normal(size=(6, gc.Gy, gc.Gx))
    got = O.prolong(tc.reshape(6, -1), gc, gf).reshape(6, gf.Gy, gf.Gx)
    # fine node i has coarse-node coordinate i/2 - 1/4 (border clamped)
    ux = np.arange(gf.Gx) / 2.0 - 0.25
    uy = np.arange(gf.Gy) / 2.0 - 0.25
    UX, UY = np.meshgrid(ux, uy)
    gxn = 2 * UX / max(gc.Gx - 1, 1) - 1 if gc.Gx > 1 else np.zeros_like(UX)
    gyn = 2 * UY / max(gc.Gy - 1, 1) - 1 if gc.Gy > 1 else np.zeros_like(UY)
    ref = F.grid_sample(torch.from_numpy(tc)[None],
                        torch.from_numpy(np.stack([gxn, gyn], -1))[None],
                        mode="bilinear", padding_mode="border",
                        align_corners=True)[0].numpy()
    np.testing.assert_allclose(got, 2.0 * ref, rtol=0, atol=1e-13)
    if gf.Gx == 2 * gc.Gx and gf.Gy == 2 * gc.Gy:
        ref2 = F.interpolate(torch.from_numpy(tc)[None], scale_factor=2,
                             mode="bilinear", align_corners=False)[0].numpy()
        np.testing.assert_allclose(got, 2.0 * ref2, rtol=0, atol=1e-13)


# --------------------------------------------------------------------------
# helpers to build a level problem
# --------------------------------------------------------------------------

def _level(imgs, s, base=None, cmask=None, wnode=None, F_l=None, level=0):
    li = O.LevelImages.build(imgs)
    H, W = li.shape
    grid = O.Grid(W, H, s)
    if base is None:
        base = np.zeros((6, grid.G))
    if cmask is None:
        cmask = np.ones(grid.N)
    if wnode is None:
        wnode = np.ones(grid.G)
    if F_l is None:
        F_l = rectified_F()
    return O.LevelState(level, li, grid, base, cmask, wnode, F_l)


# --------------------------------------------------------------------------
# P4: identity invariant and constant images
# --------------------------------------------------------------------------

def test_identity_invariant():
    p = O.Params()
    img = _smooth_images(_rng(7), 24, 32, n=1)[0]
    imgs = np.stack([img] * 4)
    li = O.LevelImages.build(imgs)
    grid = O.Grid(32, 24, 4)
    zero = np.zeros((6, grid.G))
    V, Wm = O.masks(li, grid, zero, p)
    assert V.all() and Wm.all()
    ls = _level(imgs, 4, cmask=(V & Wm).astype(float))
    t = O.pixel_terms(li, grid, grid.to_pixels(zero))
    assert np.all(t.d == 0) and np.all(t.g == 0)
    e = O.energy(ls, zero, p)
    closed = grid.N * 6 * p.eps * (p.w_photo + p.w_grad)
    assert e["total"] == pytest.approx(closed, rel=1e-14)
    assert e["smooth"] == 0 and e["epi"] == 0 and e["mag"] == 0
    grad, H = O.linearize(ls, zero, p)
    assert np.abs(grad).max() == 0.0
    assert np.all(O.pcg(H, -grad, 10) == 0.0)
    # the whole hierarchy leaves the flows exactly zero
    calib = dict(fx=30.0, fy=30.0, cx=15.5, cy=11.5, baseline=0.1,
                 F=rectified_F())
    res = O.solve(imgs, calib, O.Params(levels=2, grid_stride=4, gn_iters=2,
                                        pcg_iters=5))
    assert np.all(res["total"] == 0.0)


def test_constant_images_zero_alignment_gradient():
    p = O.Params()
    imgs = np.full((4, 12, 16), 0.37)
    ls = _level(imgs, 4)
    delta = _rng(8).normal(scale=0.7, size=(6, ls.grid.G))
    J, r, w = O.robust_rows(ls, delta, p)
    assert np.abs(J).max() == 0.0 and np.abs(r).max() <= 1e-15


# --------------------------------------------------------------------------
# P5: residual count M = 2N + 14G (Sec. 5.1)
# --------------------------------------------------------------------------

def test_residual_count():
    p = O.Params()
    ls = _level(_rng(9).random((4, 20, 28)), 4)
    g = ls.grid
    delta = np.zeros((6, g.G))
    rs, _ = O.smooth_residuals(g, delta, ls.wnode, p)
    re, _ = O.epi_residuals(g, delta, ls.F_l)
    rm, _ = O.mag_residuals(g, delta, p)
    t = O.pixel_terms(ls.li, g, g.to_pixels(delta))
    # one photometric and one gradient group per pixel; per node 6 smoothness
    # groups (one per component, over its neighbours), 2 epipolar, 6 magnitude
    n_smooth_groups = 6 * len(np.unique(O._neighbour_pairs(g)[0]))
    groups = (t.d.shape[1] + t.g.shape[2] + n_smooth_groups + re.size
              + rm.size)
    assert groups == O.residual_count(g) == 2 * g.N + 14 * g.G


# --------------------------------------------------------------------------
# P6: analytic Jacobians vs central finite differences
# --------------------------------------------------------------------------

def _random_problem(seed, W=16, H=12, s=4, general_F=False):
    rng = _rng(seed)
    imgs = _smooth_images(rng, H, W, blur=1)
    grid = O.Grid(W, H, s)
    base = rng.normal(scale=0.8, size=(6, grid.G))
    cmask = (rng.random(grid.N) < 0.8).astype(float)
    wnode = rng.uniform(1.0, 5.0, grid.G)
    F_l = rng.normal(size=(3, 3)) * 0.1 if general_F else rectified_F()
    ls = _level(imgs, s, base, cmask, wnode, F_l)
    delta = rng.normal(scale=0.3, size=(6, grid.G))
    return ls, delta


def _kink_margin(ls, delta):
    flows = ls.grid.to_pixels(ls.base + delta)
    px, py = ls.grid.pixel_xy()
    P = O.positions(px, py, flows)
    return min(np.abs(P - np.round(P)).min(), 1.0)


@pytest.mark.parametrize("seed,general_F", [(10, False), (11, True), (12, False)])
def test_energy_gradient_matches_fd(seed, general_F):
    p = O.Params()
    ls, delta = _random_problem(seed, general_F=general_F)
    h = 1e-6
    assert _kink_margin(ls, delta) > 10 * h * 4
    grad, _ = O.linearize(ls, delta, p)
    fd = np.zeros(delta.size)
    for k in range(delta.size):
        e = np.zeros(delta.size)
        e[k] = h
        ep = O.energy(ls, delta + e.reshape(6, -1), p)["total"]
        em = O.energy(ls, delta - e.reshape(6, -1), p)["total"]
        fd[k] = (ep - em) / (2 * h)
    np.testing.assert_allclose(grad, fd, rtol=1e-6,
                               atol=1e-6 * np.abs(fd).max())


def test_pixel_jacobians_match_fd():
    ls, delta = _random_problem(13)
    flows = ls.grid.to_pixels(ls.base + delta)
    t = O.pixel_terms(ls.li, ls.grid, flows)
    h = 1e-6
    for q in range(6):
        e = np.zeros((6, 1))
        e[q] = h
        tp = O.pixel_terms(ls.li, ls.grid, flows + e)
        tm = O.pixel_terms(ls.li, ls.grid, flows - e)
        np.testing.assert_allclose(t.Jd[:, q], (tp.d - tm.d) / (2 * h),
                                   rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(t.Jg[:, :, q], (tp.g - tm.g) / (2 * h),
                                   rtol=1e-6, atol=1e-7)


def test_epi_jacobian_matches_fd():
    rng = _rng(14)
    grid = O.Grid(24, 16, 4)
    total = rng.normal(size=(6, grid.G))
    Fm = rng.normal(size=(3, 3))
    r, J = O.epi_residuals(grid, total, Fm)
    h = 1e-6
    Jd = J.toarray()
    for k in range(total.size):
        e = np.zeros(total.size)
        e[k] = h
        rp, _ = O.epi_residuals(grid, total + e.reshape(6, -1), Fm)
        rm, _ = O.epi_residuals(grid, total - e.reshape(6, -1), Fm)
        # the residual is quadratic, so central differences carry only
        # rounding error (~1e-16 |r| / h)
        np.testing.assert_allclose(Jd[:, k], (rp - rm) / (2 * h), rtol=1e-6,
                                   atol=1e-9 * np.abs(r).max())


def test_gauss_newton_matrix_quadratic_form():
    """P7: v^T H v = sum omega (J_r v)^2 + 2 ||J_reg v||^2, with the
    directional derivatives J v of every residual taken by central FD."""
    p = O.Params()
    ls, delta = _random_problem(15, general_F=True)
    _, H = O.linearize(ls, delta, p)
    rng = _rng(16)
    h = 1e-6
    for _ in range(3):
        v = rng.normal(size=delta.shape)
        _, _, w = O.robust_rows(ls, delta, p)
        _, rp, _ = O.robust_rows(ls, delta + h * v, p)
        _, rm, _ = O.robust_rows(ls, delta - h * v, p)
        Jv = (rp - rm) / (2 * h)
        tot = ls.base + delta
        rrp, _, _ = O.reg_terms(ls.grid, delta + h * v, tot + h * v, ls.wnode,
                                ls.F_l, p)
        rrm, _, _ = O.reg_terms(ls.grid, delta - h * v, tot - h * v, ls.wnode,
                                ls.F_l, p)
        Jrv = (rrp - rrm) / (2 * h)
        expect = float((w * Jv * Jv).sum() + 2.0 * Jrv @ Jrv)
        vf = v.reshape(-1)
        assert float(vf @ (H @ vf)) == pytest.approx(expect, rel=1e-6)


# --------------------------------------------------------------------------
# P7: the linear solve
# --------------------------------------------------------------------------

def test_pcg_converged_matches_cholesky():
    p = O.Params()
    ls, delta = _random_problem(17, W=24, H=16, s=8)
    grad, H = O.linearize(ls, delta, p)
    Hd = H.toarray()
    assert np.abs(Hd - Hd.T).max() <= 1e-12 * np.abs(Hd).max()
    c = scipy.linalg.cho_factor(Hd)   # SPD since m_f > 0
    ref = scipy.linalg.cho_solve(c, -grad)
    x = O.pcg(H, -grad, 400)
    np.testing.assert_allclose(x, ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())


def test_pcg_iterate_is_krylov_minimiser():
    """After k steps, preconditioned CG returns the minimiser of
    1/2 x^T H x - b^T x over x in span{M^-1 b, (M^-1 H) M^-1 b, ...} (k
    vectors), computed here with dense linear algebra."""
    p = O.Params()
    ls, delta = _random_problem(18, W=24, H=16, s=8)
    grad, H = O.linearize(ls, delta, p)
    Hd = H.toarray()
    b = -grad
    Minv = 1.0 / np.diag(Hd)
    for k in (1, 3, 6, 10):
        K = [Minv * b]
        for _ in range(k - 1):
            K.append(Minv * (Hd @ K[-1]))
        Q, _ = np.linalg.qr(np.stack(K, 1))
        y = np.linalg.solve(Q.T @ Hd @ Q, Q.T @ b)
        ref = Q @ y
        x = O.pcg(H, b, k)
        np.testing.assert_allclose(x, ref, rtol=1e-6,
                                   atol=1e-7 * np.abs(ref).max())


# --------------------------------------------------------------------------
# P9: rectified epipolar closed form
# --------------------------------------------------------------------------

def test_rectified_epipolar_closed_form():
    grid = O.Grid(40, 24, 4)
    total = _rng(19).normal(size=(6, grid.G))
    r, _ = O.epi_residuals(grid, total, rectified_F())
    closed = 8.0 * (total[1] ** 2 + total[5] ** 2).sum()
    assert float(r @ r) == pytest.approx(closed, rel=1e-12)
    # and per level the residual stays in level pixels
    for l in range(4):
        Fl = O.level_calib_F(rectified_F(), l)
        r2, _ = O.epi_residuals(grid, total, Fl)
        np.testing.assert_allclose(r2, r, atol=1e-12)


# --------------------------------------------------------------------------
# P8, P10: tiny plane
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def tiny_solve():
    imgs, calib, scene = make_frame(tiny_plane_config(), 0)
    p = O.Params(levels=3, grid_stride=8, gn_iters=5, pcg_iters=10)
    rec = []
    res = O.solve(imgs, calib, p, record=rec)
    return imgs, calib, scene, p, rec, res


def test_tiny_energy_monotone(tiny_solve):
    _, _, _, p, rec, _ = tiny_solve
    assert len(rec) == p.levels * p.gn_iters
    for r in rec:
        assert r["energy_after"] <= r["energy"]
    acc = np.mean([r["tau"] == 1.0 for r in rec])
    assert acc >= 0.8


def test_split_schedule_counts_and_prefix():
    """gn_fine (the split schedule of Sec. 6.2): the two finest levels take
    gn_fine steps and the others gn_iters, and the coarse levels' steps are
    exactly those of the uniform schedule (the split changes nothing
    before level 1)."""
    imgs, calib, _ = make_frame(tiny_plane_config(), 0)
    p = O.Params(levels=3, grid_stride=8, gn_iters=3, gn_fine=1, pcg_iters=6)
    rec, rec_u = [], []
    O.solve(imgs, calib, p, record=rec)
    O.solve(imgs, calib, O.Params(levels=3, grid_stride=8, gn_iters=3, pcg_iters=6),
            record=rec_u)
    assert [r["level"] for r in rec] == [2, 2, 2, 1, 0]
    assert [p.gn_at(l) for l in range(3)] == [1, 1, 3]
    for a, b in zip(rec[:4], rec_u[:4]):
        assert a["energy"] == b["energy"] and a["tau"] == b["tau"]


def _plane_closed_form(grid, f=60.0, B=0.1, Z0=2.0, T=(0.01, 0.0, 0.02),
                       cx=31.5, cy=23.5):
    """Halfway flows of the translating fronto-parallel plane, derived from
    the position relations of Eqs. (1)-(6) / (16)-(17): with a = f/Z0,
    b = f/Z1, s_x = -(a+b)B/4, d_x = (a-b)B/4, s_y = d_y = 0, and m affine
    in the halfway pixel."""
    a = f / Z0
    Z1 = Z0 + T[2]
    b = f / Z1
    xy = grid.node_xy()
    # the point seen at halfway pixel x: solve mean of four projections = x
    # for a plane point (X, Y) at t; projections are affine in (X, Y)
    # x_L0 = a X + cx, x_R0 = a (X - B) + cx, x_L1 = b (X + Tx) + cx,
    # x_R1 = b (X + Tx - B) + cx; y likewise without B.
    out = np.zeros((6, grid.G))
    X = (xy[0] - cx - (-a * B / 2 + b * T[0] - b * B / 2) / 2) / ((a + b) / 2)
    Y = (xy[1] - cy - (b * T[1]) / 2) / ((a + b) / 2)
    P = np.array([[a * X + cx, a * Y + cy],
                  [a * (X - B) + cx, a * Y + cy],
                  [b * (X + T[0]) + cx, b * (Y + T[1]) + cy],
                  [b * (X + T[0] - B) + cx, b * (Y + T[1]) + cy]])
    s, m, d = halfway_flows_from_positions(P)
    out[0:2], out[2:4], out[4:6] = s, m, d
    assert np.allclose(out[0], -(a + b) * B / 4)
    assert np.allclose(out[4], (a - b) * B / 4)
    return out


def test_generator_plane_truth_matches_closed_form():
    """P15: the generator's ground-truth halfway correspondences on the plane
    equal the closed form."""
    sc = Scene(tiny_plane_config(), 0)
    pos, ok = sc.halfway_truth()
    assert ok.all()
    s, m, d = halfway_flows_from_positions(pos)
    grid = O.Grid(64, 48, 1)
    cf = _plane_closed_form(grid)
    got = np.concatenate([s.reshape(2, -1), m.reshape(2, -1), d.reshape(2, -1)])
    np.testing.assert_allclose(got, cf, atol=1e-8)
    # by hand: D_t = f B / Z_t = 60 * 0.1 / Z_t with Z_0 = 2 m and Z_1 = 2.02 m;
    # D_0 = -2 s_x + 2 d_x and D_1 = -2 s_x - 2 d_x (Eqs. (1)-(6)), so
    # s_x = -(D_0 + D_1) / 4 and d_x = (D_0 - D_1) / 4
    assert cf[0, 0] == pytest.approx(-1.492574, abs=1e-6)
    assert cf[4, 0] == pytest.approx(0.0074257, abs=1e-7)


def test_tiny_plane_recovery(tiny_solve):
    _, calib, _, p, _, res = tiny_solve
    grid = res["grid"]
    cf = _plane_closed_form(grid)
    tot = res["total"]
    # nodes whose bilinear support lies inside the image at every camera
    xy = grid.node_xy()
    inner = ((xy[0] >= 8) & (xy[0] <= 64 - 9) & (xy[1] >= 8) & (xy[1] <= 48 - 9))
    err = np.abs(tot - cf)[:, inner]
    assert err.mean() <= 0.05
    assert err.max() <= 0.15
    depth, flow3d, _ = O.output(grid, tot, O.Calib.from_dict(calib))
    inner_px = np.zeros((48, 64), bool)
    inner_px[12:-12, 12:-12] = True
    assert np.nanmedian(np.abs(depth[inner_px] - 2.0)) < 0.01
    # 3D flow amplifies flow errors (0.05 px of m or d is several mm at
    # 2 m with f = 60 px); exactness of the conversion is pinned separately
    med = np.nanmedian(flow3d[:, inner_px], axis=1)
    np.testing.assert_allclose(med, [0.01, 0.0, 0.02], atol=1e-2)


def test_output_closed_form():
    """Depth and 3D flow of the exact plane flows reproduce the plane."""
    grid = O.Grid(64, 48, 1)
    cf = _plane_closed_form(grid)
    calib = O.Calib(60.0, 60.0, 31.5, 23.5, 0.1)
    depth, flow3d, _ = O.output(grid, cf, calib)
    np.testing.assert_allclose(depth, 2.0, atol=1e-12)
    np.testing.assert_allclose(
        flow3d.reshape(3, -1).T,
        np.broadcast_to([0.01, 0.0, 0.02], (flow3d[0].size, 3)), atol=1e-12)


# --------------------------------------------------------------------------
# P11, P12: equivariances
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_scene():
    from synth import sized_config
    cfg = sized_config(48, 36, max_disp=3.0, noise_sigma=0.0)
    cfg.focal = 40.0
    imgs, calib, _ = make_frame(cfg, 3)
    p = O.Params(levels=2, grid_stride=4, gn_iters=3, pcg_iters=8)
    res = O.solve(imgs, calib, p)
    return imgs, calib, p, res


def test_time_reversal_equivariance(small_scene):
    imgs, calib, p, res = small_scene
    swapped = imgs[[2, 3, 0, 1]]
    r2 = O.solve(swapped, calib, p)
    a = res["total"]
    b = r2["total"]
    np.testing.assert_allclose(b[0:2], a[0:2], atol=1e-9)
    np.testing.assert_allclose(b[2:6], -a[2:6], atol=1e-9)


def test_camera_swap_equivariance(small_scene):
    imgs, calib, p, res = small_scene
    swapped = imgs[[1, 0, 3, 2]]
    c2 = dict(calib)
    c2["F"] = np.asarray(calib["F"]).T
    r2 = O.solve(swapped, c2, p)
    a = res["total"]
    b = r2["total"]
    np.testing.assert_allclose(b[0:2], -a[0:2], atol=1e-9)
    np.testing.assert_allclose(b[2:4], a[2:4], atol=1e-9)
    np.testing.assert_allclose(b[4:6], -a[4:6], atol=1e-9)


# --------------------------------------------------------------------------
# P13: pure integer disparity
# --------------------------------------------------------------------------

def test_pure_disparity():
    rng = _rng(20)
    k = 2
    H, W = 40, 56
    big = _smooth_images(rng, H, W + k, n=1, blur=1)[0]
    left = big[:, :W]
    right = big[:, k:]       # right(x) = left(x + k): disparity x_L - x_R = k
    imgs = np.stack([left, right, left, right])
    calib = dict(fx=40.0, fy=40.0, cx=(W - 1) / 2, cy=(H - 1) / 2,
                 baseline=0.1, F=rectified_F())
    p = O.Params(levels=2, grid_stride=4, gn_iters=6, pcg_iters=30)
    res = O.solve(imgs, calib, p)
    g = res["grid"]
    tot = res["total"].reshape(6, g.Gy, g.Gx)
    inner = tot[:, 2:-2, 2:-3]
    np.testing.assert_allclose(inner[0], -k / 2.0, atol=0.03)
    assert np.abs(inner[1]).max() < 0.02
    assert np.abs(inner[2:]).max() < 0.03


# --------------------------------------------------------------------------
# P14: brute force on a tiny problem
# --------------------------------------------------------------------------

def test_gn_fixed_point_matches_lbfgs():
    rng = _rng(21)
    imgs = _smooth_images(rng, 12, 16, blur=2)
    # a small coherent shift of the right images
    imgs[1] = np.roll(imgs[0], -1, axis=1) * 0.9 + imgs[1] * 0.1
    imgs[3] = np.roll(imgs[2], -1, axis=1) * 0.9 + imgs[3] * 0.1
    p = O.Params(eps=0.05, pcg_iters=200)
    ls = _level(imgs, 8, wnode=np.full(4, 2.0))
    delta = np.zeros((6, ls.grid.G))
    g0, _ = O.linearize(ls, delta, p)
    for _ in range(150):
        delta = O.gn_step(ls, delta, p)
    grad, _ = O.linearize(ls, delta, p)
    # reweighted Gauss-Newton converges linearly: a stationary point to
    # 1e-9 of the starting gradient
    assert np.abs(grad).max() <= 1e-9 * np.abs(g0).max()

    def f(x):
        e = O.energy(ls, x.reshape(6, -1), p)["total"]
        g, _ = O.linearize(ls, x.reshape(6, -1), p)
        return e, g

    # E is non-convex (and only piecewise smooth through the bilinear
    # warps), so an independent optimiser may end in another basin from the
    # zero start; restricted to a box around the Gauss-Newton fixed point and
    # started off it, it must return to it: the fixed point is a minimiser
    xs = delta.reshape(-1)
    x0 = xs + _rng(22).uniform(-2e-3, 2e-3, size=delta.size)
    box = [(v - 5e-3, v + 5e-3) for v in xs]
    opt = scipy.optimize.minimize(f, x0, jac=True, method="L-BFGS-B",
                                  bounds=box,
                                  options=dict(ftol=1e-15, gtol=1e-11,
                                               maxiter=5000))
    np.testing.assert_allclose(opt.x, xs, atol=1e-5)
    assert opt.fun >= O.energy(ls, delta, p)["total"] - 1e-9


# --------------------------------------------------------------------------
# masks and per-level calibration
# --------------------------------------------------------------------------

def test_visibility_mask_uniform_stereo_flow():
    """A uniform stereo flow s_x = 1.5 moves P_L0 and P_L1 by -1.5 and P_R0,
    P_R1 by +1.5 px: exactly the pixels with 1.5 <= x <= W - 2.5 stay in."""
    p = O.Params()
    H, W = 12, 20
    li = O.LevelImages.build(_rng(23).random((4, H, W)))
    grid = O.Grid(W, H, 4)
    tot = np.zeros((6, grid.G))
    tot[0] = 1.5
    V, _ = O.masks(li, grid, tot, p)
    x = np.tile(np.arange(W), H)
    np.testing.assert_array_equal(V, (x >= 1.5) & (x <= W - 2.5))


def test_pruning_mask_threshold():
    p = O.Params()
    base = _smooth_images(_rng(24), 10, 14, n=1)[0]
    grid = O.Grid(14, 10, 4)
    zero = np.zeros((6, grid.G))
    for off, expect in ((0.1, True), (0.3, False)):
        imgs = np.stack([base, base + off, base, base + off])
        _, Wm = O.masks(O.LevelImages.build(imgs), grid, zero, p)
        assert np.all(Wm == expect)


@pytest.mark.parametrize("level", [1, 2, 3])
def test_level_fundamental_matrix(level):
    """Mapping level-l pixels to level 0 by p0 = 2^l p_l + (2^l - 1)/2, the
    level-l epipolar residual is the level-0 residual divided by 2^l."""
    rng = _rng(25)
    Fm = rng.normal(size=(3, 3))
    Fl = O.level_calib_F(Fm, level)
    k = 2.0 ** level
    for _ in range(5):
        l = rng.uniform(0, 50, 2)
        r = rng.uniform(0, 50, 2)
        l0 = np.append(k * l + (k - 1) / 2, 1.0)
        r0 = np.append(k * r + (k - 1) / 2, 1.0)
        lh = np.append(l, 1.0)
        rh = np.append(r, 1.0)
        assert lh @ Fl @ rh == pytest.approx((l0 @ Fm @ r0) / k, rel=1e-12)


def test_sampled_rows_and_node_rows_equal_full_assembly():
    """The sampled evaluators used by the full-size GPU checks give the
    same numbers as the full robust_rows / linearize."""
    imgs, calib, _ = make_frame(tiny_plane_config(), 0)
    p = O.Params(levels=1, grid_stride=8)
    pyr = O.pyramid(imgs.astype(np.float64), 1)
    grid = O.Grid(64, 48, 8)
    rng = np.random.default_rng(3)
    base = rng.normal(0, 0.3, (6, grid.G))
    ls = O.setup_level(0, pyr, p, O.Calib.from_dict(calib), base)
    delta = rng.normal(0, 0.2, (6, grid.G))
    J, r, w = O.robust_rows(ls, delta, p)
    pix = rng.choice(grid.N, 40, replace=False)
    Js, rs, ws = O.rows_at(ls, delta, p, pix)
    np.testing.assert_allclose(Js, J[pix], rtol=0, atol=1e-13)
    np.testing.assert_allclose(rs, r[pix], rtol=0, atol=1e-13)
    np.testing.assert_allclose(ws, w[pix], rtol=0, atol=1e-13)
    grad, H = O.linearize(ls, delta, p)
    u = rng.normal(size=6 * grid.G)
    nodes = rng.choice(grid.G, 12, replace=False)
    g, dg, Hu = O.node_rows(ls, delta, p, nodes, u)
    idx = (np.arange(6)[:, None] * grid.G + nodes[None]).reshape(6, -1)
    np.testing.assert_allclose(g, grad[idx], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dg, H.diagonal()[idx], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Hu, (H @ u)[idx], rtol=1e-12, atol=1e-11)


# ---- temporal initialisation (Sec. 5.3) --------------------------------------

def test_sample_nodes_is_clamped_bilinear_on_the_node_grid():
    """sample_nodes against scipy's linear interpolation with nearest-edge
    extension in node coordinates u = (x + 1/2) / s - 1/2 (positions inside,
    outside and on the nodes)."""
    import scipy.ndimage as ndi
    rng = np.random.default_rng(5)
    for W, H, s in ((40, 30, 4), (33, 17, 8), (9, 9, 8)):
        grid = O.Grid(W, H, s)
        f = rng.normal(size=(2, grid.G))
        x = rng.uniform(-20, W + 20, 200)
        y = rng.uniform(-20, H + 20, 200)
        x[:5] = (np.arange(5) % grid.Gx + 0.5) * s - 0.5  # exactly on nodes
        got = O.sample_nodes(grid, f, x, y)
        u = np.clip((x + 0.5) / s - 0.5, 0, grid.Gx - 1)
        v = np.clip((y + 0.5) / s - 0.5, 0, grid.Gy - 1)
        for c in range(2):
            ref = ndi.map_coordinates(f[c].reshape(grid.Gy, grid.Gx), [v, u], order=1,
                                      mode="nearest")
            np.testing.assert_allclose(got[c], ref, rtol=0, atol=1e-12)


def test_temporal_init_identity_and_one_node_shift():
    """No motion transfers every delta unchanged; a motion of half a stride
    (2 m = one node spacing) shifts the deltas by exactly one node, the
    first column repeating (clamped)."""
    rng = np.random.default_rng(6)
    grids = {0: O.Grid(48, 32, 4), 1: O.Grid(24, 16, 4)}
    deltas = {l: rng.normal(size=(6, g.G)) for l, g in grids.items()}
    zero = {l: np.zeros((6, g.G)) for l, g in grids.items()}
    out = O.temporal_init(zero, deltas, grids)
    for l in grids:
        np.testing.assert_array_equal(out[l], deltas[l])
    totals = {}
    for l, g in grids.items():
        t = rng.normal(size=(6, g.G))
        t[2] = g.s / 2.0
        t[3] = 0.0
        totals[l] = t
    out = O.temporal_init(totals, deltas, grids)
    for l, g in grids.items():
        d = deltas[l].reshape(6, g.Gy, g.Gx)
        o = out[l].reshape(6, g.Gy, g.Gx)
        np.testing.assert_allclose(o[:, :, 1:], d[:, :, :-1], rtol=0, atol=1e-12)
        np.testing.assert_allclose(o[:, :, 0], d[:, :, 0], rtol=0, atol=1e-12)


def test_sequence_of_the_translating_plane_starts_closer():
    """A constant-velocity sequence of the translating plane: the generator
    renders frame k at times k and k + 1 (frame 0 equals the single-frame
    render), and the second frame started from the temporal initialisation
    has a lower energy at its start than from zero and ends closer to the
    true flows after one Gauss-Newton step per level."""
    from synth import make_sequence
    cfg = tiny_plane_config()
    frames, calib, sc = make_sequence(cfg, 0, 2)
    single, _, _ = make_frame(cfg, 0)
    np.testing.assert_array_equal(frames[0], single)
    p = O.Params(levels=2, grid_stride=8, gn_iters=1, pcg_iters=20)
    seq_rec, zero_rec = [], []
    res = O.solve_sequence([f.astype(np.float64) for f in frames], calib, p, record=seq_rec)
    zero = O.solve(frames[1].astype(np.float64), calib, p, record=zero_rec)
    # energies at the start of the first (coarsest) step of frame 2
    assert seq_rec[1][0]["energy"] < zero_rec[0]["energy"]
    pos, ok = sc.halfway_truth(t0=1)
    truth = np.concatenate(halfway_flows_from_positions(pos))
    grid = res[1]["grid"]
    err_seq = np.abs(grid.to_pixels(res[1]["total"]).reshape(6, grid.H, grid.W) - truth)[:, ok]
    err_zero = np.abs(grid.to_pixels(zero["total"]).reshape(6, grid.H, grid.W) - truth)[:, ok]
    assert err_seq.mean() < err_zero.mean()


# ---- illumination correction (Sec. 5.3) ---------------------------------------

def test_gaussian_blur_and_box_upsample():
    """The separable blur equals scipy's Gaussian filter with the same
    radius (ceil(3 sigma) = 10 taps a side) and nearest-edge borders; the
    box upsample equals repeating each pixel 2 x 2 (odd sizes clamp)."""
    import scipy.ndimage as ndi
    rng = np.random.default_rng(8)
    img = rng.normal(size=(23, 37))
    ref = ndi.gaussian_filter(img, O.ILLUM_SIGMA, mode="nearest",
                              truncate=math.ceil(3 * O.ILLUM_SIGMA) / O.ILLUM_SIGMA)
    np.testing.assert_allclose(O.gaussian_blur(img), ref, rtol=0, atol=1e-12)
    up = O.box_upsample(img, 74, 46)
    np.testing.assert_array_equal(up, np.repeat(np.repeat(img, 2, 0), 2, 1))
    up = O.box_upsample(img, 75, 47)
    assert up.shape == (47, 75)
    np.testing.assert_array_equal(up[-1, -1], img[-1, -1])


def test_illumination_residual_recovers_a_right_camera_offset():
    """Right images = left images + b and zero flow: the stereo residual is
    b at every pixel, the blurred map is b, and with the correction applied
    the stereo differences vanish."""
    rng = np.random.default_rng(9)
    left = rng.uniform(0.2, 0.8, (2, 20, 30))
    imgs = np.stack([left[0], left[0] + 0.07, left[1], left[1] + 0.07])
    li = O.LevelImages.build(imgs)
    grid = O.Grid(30, 20, 4)
    e = O.illumination_residual(li, grid, np.zeros((6, grid.G)))
    np.testing.assert_allclose(e, 0.07, rtol=0, atol=1e-12)
    m = O.illumination_map(li, grid, np.zeros((6, grid.G)), 30, 20)
    np.testing.assert_allclose(m, 0.07, rtol=0, atol=1e-12)
    li2 = O.LevelImages.build(imgs, np.full(grid.N, 0.07))
    t = O.pixel_terms(li2, grid, np.zeros((6, grid.N)))
    np.testing.assert_allclose(t.d[[0, 1]], 0.0, atol=1e-12)  # stereo pairs


def test_illumination_correction_helps_a_biased_right_camera():
    """The translating plane with a right camera of different gain and
    offset: the corrected solve ends closer to the true flows."""
    from dataclasses import replace
    cfg = replace(tiny_plane_config(), right_gain=1.1, right_bias=0.08, right_ramp=0.05)
    sc = Scene(cfg, 0)
    imgs = sc.render(noise=False).astype(np.float64)
    from synth.scene import calib_of
    calib = calib_of(sc)
    truth = np.concatenate(halfway_flows_from_positions(sc.halfway_truth()[0]))
    errs = []
    for on in (False, True):
        p = O.Params(levels=3, grid_stride=8, gn_iters=5, pcg_iters=10, illum=on)
        res = O.solve(imgs, calib, p)
        g = res["grid"]
        errs.append(np.abs(g.to_pixels(res["total"]).reshape(6, g.H, g.W) - truth).mean())
    assert errs[1] < errs[0]


# ---- occlusion maps (Sec. 5.3) -------------------------------------------------

def _strip_flows(grid, a, b, Df, Db):
    """Per-pixel flows (stride 1) of a fronto-parallel strip of disparity Df
    over columns [a, b) in front of a background of disparity Db, no motion:
    s.x = -D / 2 so that P_L.x = x + D / 2 and P_R.x = x - D / 2."""
    px, _ = grid.pixel_xy()
    D = np.where((px >= a) & (px < b), Df, Db)
    tot = np.zeros((6, grid.G))
    tot[0] = -D / 2
    return tot


@pytest.mark.parametrize("a,b", [(15, 25), (9, 30), (12, 14), (20, 23)])
def test_occlusion_strip_closed_form(a, b):
    """A strip of disparity 10 (columns [a, b), b - a >= 2) in front of a
    background of disparity 2.  In the left views strip column x lands on
    x + 5 and background column x on x + 1, so the strip covers the pixel
    centres a + 5 .. b + 4 and hides the background columns right of it
    whose x + 1 falls there: max(b, a + 4) .. b + 3.  In the right views
    (x - 5 and x - 1) it hides a - 4 .. min(a - 1, b - 5).  Nothing else is
    occluded: the triangles that join strip and background are longer than
    2 px and are not drawn."""
    W, H = 44, 9
    g = O.Grid(W, H, 1)
    vis = O.occlusion_map(g, _strip_flows(g, a, b, 10.0, 2.0))
    hidden = set(range(a - 4, min(a - 1, b - 5) + 1)) | set(range(max(b, a + 4), b + 4))
    expect = np.array([0.0 if x in hidden else 1.0 for x in range(W)])
    np.testing.assert_array_equal(vis, np.tile(expect, (H, 1)))


def test_occlusion_of_a_plane_is_empty():
    """Constant flows (a fronto-parallel plane seen with uniform motion):
    every pixel is visible in every view."""
    g = O.Grid(30, 20, 5)
    tot = np.zeros((6, g.G))
    tot[:, :] = np.array([-2.3, 0.1, 0.7, -0.4, 0.2, 0.05])[:, None]
    assert np.all(O.occlusion_map(g, tot) == 1.0)
    assert not O.occlusion_fragile(g, tot).any()


def _brute_visibility(P, D, W, H, tol, max_edge):
    """Independent z-buffer: every pixel centre against every triangle of the
    halfway grid, barycentric coordinates from a 2x2 linear solve."""
    vis = np.ones(H * W, bool)
    for cam in range(4):
        X, Y, Dc = P[cam, 0], P[cam, 1], D[cam]
        zb = np.zeros(H * W)
        tris = []
        for y in range(H - 1):
            for x in range(W - 1):
                i00, i10, i01, i11 = y * W + x, y * W + x + 1, (y + 1) * W + x, (y + 1) * W + x + 1
                tris += [(i00, i10, i01), (i10, i11, i01)]
        for t in tris:
            v = np.array([[X[k], Y[k]] for k in t])
            if max(np.linalg.norm(v[i] - v[(i + 1) % 3]) for i in range(3)) > max_edge:
                continue
            if min(Dc[k] for k in t) <= 0:
                continue
            M = np.array([v[1] - v[0], v[2] - v[0]]).T
            if abs(np.linalg.det(M)) < 1e-12:
                continue
            for qy in range(H):
                for qx in range(W):
                    lb, lc = np.linalg.solve(M, np.array([qx, qy]) - v[0])
                    lam = (1 - lb - lc, lb, lc)
                    if min(lam) >= 0:
                        z = sum(l * Dc[k] for l, k in zip(lam, t))
                        zb[qy * W + qx] = max(zb[qy * W + qx], z)
        for i in range(H * W):
            nx, ny = math.floor(X[i] + 0.5), math.floor(Y[i] + 0.5)
            if 0 <= nx < W and 0 <= ny < H and Dc[i] > 0 and Dc[i] < (1 - tol) * zb[ny * W + nx]:
                vis[i] = False
    return vis


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_occlusion_matches_brute_force(seed):
    rng = _rng(seed)
    W, H = 9, 7
    g = O.Grid(W, H, 1)
    px, py = g.pixel_xy()
    fg = (px >= 3) & (px < 6) & (py >= 2)
    D = np.where(fg, 4.5, 1.5) + 0.3 * rng.standard_normal(g.N)
    D[rng.integers(0, g.N, 2)] = -0.5
    tot = np.zeros((6, g.G))
    tot[4] = 0.2 * rng.standard_normal(g.N)
    tot[5] = 0.2 * rng.standard_normal(g.N)
    tot[0] = -D / 2 + tot[4]
    tot[1] = 0.2 * rng.standard_normal(g.N)
    tot[2] = 0.3 * rng.standard_normal(g.N)
    tot[3] = 0.3 * rng.standard_normal(g.N)
    P = O.positions(px, py, tot)
    Ds = [P[0, 0] - P[1, 0], P[0, 0] - P[1, 0], P[2, 0] - P[3, 0], P[2, 0] - P[3, 0]]
    ref = _brute_visibility(P, Ds, W, H, O.OCC_TOL, O.OCC_EDGE)
    got = O.occlusion_map(g, tot).reshape(-1) > 0.5
    assert (~ref).sum() > 0
    np.testing.assert_array_equal(got, ref)


def test_occlusion_solve_of_the_translating_plane_is_unchanged():
    """The fold-free plane scene has nothing occluded at any level, so the
    solve with occlusion maps equals the one without."""
    sc = Scene(tiny_plane_config(), 0)
    imgs = sc.render(noise=False).astype(np.float64)
    from synth.scene import calib_of
    calib = calib_of(sc)
    out = []
    for on in (False, True):
        p = O.Params(levels=3, grid_stride=8, gn_iters=2, pcg_iters=6, occlusion=on)
        out.append(O.solve(imgs, calib, p)["total"])
    np.testing.assert_array_equal(out[0], out[1])


# --------------------------------------------------------------------------
# Smoothness weights w_i (Sec. 4.3): structure tensor of the mean warped
# image over a 3x3 window at the node, smaller eigenvalue, w = 1 + gamma
# exp(-lambda_min / tau_l).  The map from lambda_min to w is the library's
# reading; every ingredient is pinned here: the warp, the gradient
# convention, the window and its centre, the eigenvalue, tau_l.
# --------------------------------------------------------------------------

def _quadratic(a, b, ox=0.0, oy=0.0, H=40, W=56):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    return a * (x - ox) ** 2 + b * (y - oy) ** 2


def test_node_weights_constant_and_ramp_are_featureless():
    """A constant image and a linear ramp have a rank-deficient structure
    tensor (lambda_min = 0), so every node gets 1 + gamma."""
    p = O.Params(st_gamma=4.0, st_tau=1e-3)
    grid = O.Grid(56, 40, 4)
    y, x = np.mgrid[0:40, 0:56].astype(np.float64)
    for img in (np.full((40, 56), 0.42), 0.01 * x - 0.02 * y + 0.3):
        li = O.LevelImages.build(np.stack([img] * 4))
        w = O.node_weights(li, grid, np.zeros((6, grid.G)), 0, p)
        np.testing.assert_allclose(w, 1.0 + p.st_gamma, rtol=0, atol=1e-9)


def test_node_weights_quadratic_closed_form():
    """I = a x^2 + b y^2: inside the image the central differences are
    exactly 2 a x and 2 b y, so the 3x3 window at pixel (cx, cy) sums to
    A = 4 [[a^2 (9 cx^2 + 6), 9 a b cx cy], [9 a b cx cy, b^2 (9 cy^2 + 6)]]
    (sum over dx in {-1, 0, 1} of (cx + dx)^2 = 3 cx^2 + 2).  Nodes sit at
    (i + 1/2) s - 1/2 and the window is centred on the rounded position.
    Camera c sees the quadratic Q_c = a_c x^2 + b_c y^2 shifted by the
    integer offset that the flows (s, m, d) put on it (Eqs. (1)-(6)), so the
    mean warped image is the quadratic with the mean coefficients a, b
    wherever no sample is clamped (unwarped, the mean would carry a linear
    term, since the a_c differ)."""
    ac = 1e-3 * np.array([1.0, 1.3, 0.7, 1.0])
    bc = -7e-4 * np.array([1.0, 0.8, 1.2, 1.0])
    a, b = ac.mean(), bc.mean()
    flows = np.array([1.0, 0.0, 0.0, 1.0, 1.0, -1.0])   # s, m, d (x, y)
    signs = np.array([[-1, -1, 1], [1, -1, -1], [-1, 1, -1], [1, 1, 1]], float)
    imgs = []
    for c in range(4):
        off = signs[c, 0] * flows[0:2] + signs[c, 1] * flows[2:4] + signs[c, 2] * flows[4:6]
        imgs.append(_quadratic(ac[c], bc[c], off[0], off[1]))   # I_c(x + off) = Q_c(x)
    li = O.LevelImages.build(np.stack(imgs))
    for s in (4, 5):
        grid = O.Grid(56, 40, s)
        total = np.repeat(flows[:, None], grid.G, 1)
        nx, ny = grid.node_xy()
        cx = np.floor(nx + 0.5)
        cy = np.floor(ny + 0.5)
        A = 4.0 * np.array([[a * a * (9 * cx ** 2 + 6), 9 * a * b * cx * cy],
                            [9 * a * b * cx * cy, b * b * (9 * cy ** 2 + 6)]])
        lmin = np.array([np.linalg.eigvalsh(A[:, :, k])[0] for k in range(grid.G)])
        # the window and its central differences stay 3 px inside the image
        # (the warps move samples by up to 3 px)
        inner = (cx >= 5) & (cx <= 56 - 6) & (cy >= 5) & (cy <= 40 - 6)
        assert inner.sum() >= 20
        for tau in (1e-5, 2e-5):
            p = O.Params(st_gamma=4.0, st_tau=tau)
            w = O.node_weights(li, grid, total, 0, p)
            want = 1.0 + 4.0 * np.exp(-lmin / tau)
            np.testing.assert_allclose(w[inner], want[inner], rtol=1e-12)
            # the weights are not saturated: they distinguish lambda_min
            # from lambda_max and from an off-centre window
            assert np.ptp(want[inner]) > 0.3


def test_node_weights_match_eigvalsh_on_random_images():
    """Random smooth images at zero flow: the mean warped image is the mean
    of the four images (exact samples), its gradients are numpy.gradient's,
    and the window tensor's smaller eigenvalue comes from
    numpy.linalg.eigvalsh.  A node whose rounded position falls outside the
    image (the last node row or column when the stride does not divide the
    size) is centred on the nearest border pixel, and window rows or
    columns beyond the border repeat the border."""
    rng = _rng(40)
    imgs = _smooth_images(rng, 30, 44) * 0.05
    li = O.LevelImages.build(imgs)
    p = O.Params(st_gamma=4.0, st_tau=2e-5)
    for s in (3, 4, 8):
        grid = O.Grid(44, 30, s)
        w = O.node_weights(li, grid, np.zeros((6, grid.G)), 0, p)
        gy, gx = np.gradient(imgs.mean(0))
        nx, ny = grid.node_xy()
        want = np.empty(grid.G)
        for k in range(grid.G):
            cx = min(int(np.floor(nx[k] + 0.5)), 43)
            cy = min(int(np.floor(ny[k] + 0.5)), 29)
            A = np.zeros((2, 2))
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    yy = min(max(cy + dy, 0), 29)
                    xx = min(max(cx + dx, 0), 43)
                    g = np.array([gx[yy, xx], gy[yy, xx]])
                    A += np.outer(g, g)
            want[k] = 1.0 + 4.0 * math.exp(-max(np.linalg.eigvalsh(A)[0], 0.0) / 2e-5)
        np.testing.assert_allclose(w, want, rtol=1e-10)
        assert np.ptp(w) > 0.3


def test_node_weights_tau_scales_four_per_level():
    """Gradients double per coarser level at equal structure (squared: x4),
    so tau_l = tau 4^l makes level l on an image scaled by 2^l give the
    level-0 weights of the unscaled image."""
    imgs = _smooth_images(_rng(41), 30, 44) * 0.05
    grid = O.Grid(44, 30, 4)
    p = O.Params(st_gamma=4.0, st_tau=2e-5)
    w0 = O.node_weights(O.LevelImages.build(imgs), grid, np.zeros((6, grid.G)), 0, p)
    assert np.ptp(w0) > 0.3
    for l in (1, 2, 3):
        wl = O.node_weights(O.LevelImages.build(imgs * 2.0 ** l), grid,
                            np.zeros((6, grid.G)), l, p)
        np.testing.assert_allclose(wl, w0, rtol=1e-10)


# --------------------------------------------------------------------------
# E_smooth (Eq. (14)) and E_mag (Eq. (18)): values in closed form
# --------------------------------------------------------------------------

def test_smooth_energy_of_a_delta_ramp():
    """Delta_f = c_f i + e_f j on node (i, j): every horizontal neighbour
    pair differs by c_f and every vertical one by e_f.  Summing over ordered
    pairs as Eq. (14) is written, node n contributes
    w_n (h_n sum_f w_f c_f^2 + v_n sum_f w_f e_f^2), with h_n / v_n its
    number of horizontal / vertical neighbours (2 inside, 1 on the border
    rows or columns).  Over ordered pairs w_i and w_j weightings give the
    same sum, so only the pair count and the per-component weights are
    at stake.  Evaluated through energy() on a non-zero, rough base: the
    term acts on the deltas, not the totals."""
    p = O.Params()
    imgs = _smooth_images(_rng(42), 28, 40)
    for (W, H, s) in ((40, 28, 4), (40, 28, 8), (40, 28, 13)):
        grid = O.Grid(W, H, s)
        rng = _rng(43 + s)
        base = rng.normal(scale=2.0, size=(6, grid.G))
        wnode = rng.uniform(1.0, 5.0, grid.G)
        c = rng.normal(size=6)
        e = rng.normal(size=6)
        j, i = np.mgrid[0:grid.Gy, 0:grid.Gx]
        delta = c[:, None] * i.reshape(-1)[None] + e[:, None] * j.reshape(-1)[None]
        hn = (np.minimum(i, 1) + np.minimum(grid.Gx - 1 - i, 1)).reshape(-1)
        vn = (np.minimum(j, 1) + np.minimum(grid.Gy - 1 - j, 1)).reshape(-1)
        wf = np.array([p.w_s, p.w_s, p.w_m, p.w_m, p.w_d, p.w_d])
        want = float((wnode * (hn * (wf * c * c).sum() + vn * (wf * e * e).sum())).sum())
        ls = _level(imgs, s, base=base, wnode=wnode)
        got = O.energy(ls, delta, p)["smooth"]
        assert got == pytest.approx(want, rel=1e-12)
        # a constant delta is not penalised at all, whatever the base
        assert O.energy(ls, np.repeat(c[:, None], grid.G, 1), p)["smooth"] == \
            pytest.approx(0.0, abs=1e-20)


def test_magnitude_energy_of_a_constant_delta():
    """Delta_f = c_f on every node gives E_mag = G sum_f m_f c_f^2, the same
    on any base (the term acts on the deltas: Sec. 5.1 asks only the deltas
    to stay small), and zero for a zero delta on a large base."""
    p = O.Params()
    imgs = _smooth_images(_rng(44), 24, 32)
    grid = O.Grid(32, 24, 4)
    c = _rng(45).normal(size=6)
    mf = np.array([p.m_s, p.m_s, p.m_m, p.m_m, p.m_d, p.m_d])
    want = grid.G * float((mf * c * c).sum())
    delta = np.repeat(c[:, None], grid.G, 1)
    for scale in (0.0, 1.0, 5.0):
        base = _rng(46).normal(scale=scale, size=(6, grid.G))
        ls = _level(imgs, 4, base=base)
        assert O.energy(ls, delta, p)["mag"] == pytest.approx(want, rel=1e-12)
        assert O.energy(ls, np.zeros((6, grid.G)), p)["mag"] == 0.0


def test_output_recovers_random_points_with_distinct_focal_lengths():
    """Dense geometry and motion (Sec. 3): for every halfway pixel x pick a
    depth Z_0 and a 3D motion M, place the point (X, Y, Z_0) whose four
    projections into the rectified pair at t and t + 1 (focal lengths
    f_x != f_y, principal point off-centre, baseline B along x) average to
    x, derive the halfway flows from the four positions, and require the
    output to return Z_0 and M exactly."""
    rng = _rng(47)
    H, W = 12, 16
    fx, fy, cx, cy, B = 70.0, 83.0, 7.3, 4.1, 0.12
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    Z0 = rng.uniform(1.5, 4.0, (H, W))
    M = rng.normal(scale=0.05, size=(3, H, W))
    Z1 = Z0 + M[2]
    # mean of the four x projections: fx/4 [ (2X - B)/Z0 + (2 (X + Mx) - B)/Z1 ] + cx
    a, b = 1.0 / Z0, 1.0 / Z1
    X = ((x - cx) * 4.0 / fx + B * a - (2.0 * M[0] - B) * b) / (2.0 * (a + b))
    Y = ((y - cy) * 2.0 / fy - M[1] * b) / (a + b)
    P = np.array([[fx * X / Z0 + cx, fy * Y / Z0 + cy],
                  [fx * (X - B) / Z0 + cx, fy * Y / Z0 + cy],
                  [fx * (X + M[0]) / Z1 + cx, fy * (Y + M[1]) / Z1 + cy],
                  [fx * (X + M[0] - B) / Z1 + cx, fy * (Y + M[1]) / Z1 + cy]])
    np.testing.assert_allclose(P[:, 0].mean(0), x, atol=1e-12)
    np.testing.assert_allclose(P[:, 1].mean(0), y, atol=1e-12)
    s, m, d = halfway_flows_from_positions(P)
    flows = np.concatenate([s, m, d]).reshape(6, -1)
    depth, flow3d, _ = O.output_from_flows(flows, W, H, O.Calib(fx, fy, cx, cy, B))
    np.testing.assert_allclose(depth, Z0, rtol=1e-12)
    np.testing.assert_allclose(flow3d, M, atol=1e-12)
