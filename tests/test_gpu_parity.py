"""GPU path vs the FP64 oracle, stage by stage and end to end, through the
C ABI.  Tolerances: per-(level, step) energy within 1e-4 relative and final
flows within 0.02 px (float32 path vs float64 oracle); per-stage quantities
as stated at each check."""
import numpy as np
import pytest

import oracle.halfway as O
from synth import make_frame, tiny_plane_config, sized_config

from gpu_util import check_output, GpuCase, oracle_params, mask_flip_ok, rel_err

pytestmark = pytest.mark.gpu

MED = dict(levels=3, grid_stride=4, gn_iters=3, pcg_iters=8)


def _frame(W, H, seed=5, disp=None):
    cfg = sized_config(W, H, max_disp=disp if disp is not None else 0.05 * W)
    imgs, calib, _ = make_frame(cfg, seed)
    return imgs, calib


def _stage_case(W=100, H=76, **kw):
    prm = dict(MED)
    prm.update(kw)
    imgs, calib = _frame(W, H)
    g = GpuCase(imgs, calib, **prm)
    g.set_images()
    return g, imgs, calib, oracle_params(**prm)


def _oracle_level(imgs, calib, p, level):
    pyr = O.pyramid(imgs.astype(np.float64), p.levels)
    H, W = pyr[level].shape[1:]
    grid = O.Grid(W, H, p.grid_stride)
    return O.setup_level(level, pyr, p, O.Calib.from_dict(calib),
                         np.zeros((6, grid.G))), pyr


def _kink_pixels(ls, delta, margin=1e-4):
    """Pixels with a sample position within `margin` px of an integer
    coordinate, where the bilinear interpolant has a kink: there float32
    and float64 may pick different cells, and both one-sided derivatives
    are valid.  Also returns the nodes such pixels touch."""
    flows = ls.grid.to_pixels(ls.base + delta)
    px, py = ls.grid.pixel_xy()
    P = O.positions(px, py, flows)
    kink = (np.abs(P - np.round(P)) < margin).any(axis=(0, 1))
    touched = np.zeros(ls.grid.G, bool)
    for k in range(4):
        touched[ls.grid.nodes[k][kink]] = True
    return kink, touched


# ----------------------------------------------------------------------------

@pytest.mark.parametrize("W,H,levels", [(64, 48, 3), (100, 76, 3), (81, 53, 2),
                                        (640, 480, 5)])
def test_pyramid_parity(W, H, levels):
    imgs = np.random.default_rng(1).random((4, H, W)).astype(np.float32)
    calib = dict(fx=50.0, fy=50.0, cx=(W - 1) / 2, cy=(H - 1) / 2,
                 baseline=0.1, F=np.array([[0, 0, 0], [0, 0, -1], [0, 1, 0.]]))
    g = GpuCase(imgs, calib, levels=levels, grid_stride=4)
    try:
        g.set_images()
        pyr = O.pyramid(imgs.astype(np.float64), levels)
        for l in range(levels):
            tex = g.read(g.sf.SF_DBG_TEX, l).reshape(4, pyr[l].shape[1], pyr[l].shape[2], 4)
            # box filter in float32 vs float64: within a few float32 ulps
            np.testing.assert_allclose(tex[..., 0], pyr[l], rtol=0, atol=2e-7 * (l + 1))
            for c in range(4):
                gx, gy = O.image_gradients(pyr[l][c])
                np.testing.assert_allclose(tex[c, ..., 1], gx, rtol=0, atol=4e-7 * (l + 1))
                np.testing.assert_allclose(tex[c, ..., 2], gy, rtol=0, atol=4e-7 * (l + 1))
            assert np.all(tex[..., 3] == 0)
    finally:
        g.close()


@pytest.mark.parametrize("level", [0, 2])
def test_level_init_parity(level):
    g, imgs, calib, p = _stage_case()
    try:
        g.run(g.sf.SF_STAGE_LEVEL_INIT, level)
        ls, _ = _oracle_level(imgs, calib, p, level)
        cm = g.read(g.sf.SF_DBG_CMASK, level)
        _, flips = mask_flip_ok(ls.li, ls.grid, ls.base, p, cm)
        assert flips == 0
        np.testing.assert_array_equal(cm.astype(bool), ls.cmask.astype(bool))
        w = g.read(g.sf.SF_DBG_WNODE, level)
        np.testing.assert_allclose(w, ls.wnode, rtol=1e-4, atol=1e-5)
        assert np.all(g.read(g.sf.SF_DBG_BASE, level) == 0)
        assert np.all(g.read(g.sf.SF_DBG_DELTA, level) == 0)
    finally:
        g.close()


def _gram_upper(Gx):
    iu = np.triu_indices(6)
    return Gx[:, iu[0], iu[1]].T  # (21, N)


@pytest.mark.parametrize("level,stride,apply", [
    (0, 4, 0), (2, 4, 0), (0, 8, 0), (1, 2, 0), (0, 3, 0),
    # node-block products: every assembly tile shape (strides 1..8)
    (0, 4, 1), (2, 4, 1), (0, 8, 1), (1, 2, 1), (0, 3, 1), (0, 5, 1), (0, 6, 1),
    (0, 7, 1), (2, 1, 1),
    # whole-PCG single-workgroup kernel (levels of at most 336 nodes; 21 x 16
    # = 336 at stride 5 fills it exactly)
    (2, 4, 2), (0, 8, 2), (1, 4, 2), (0, 6, 2), (0, 5, 2)])
def test_linearize_apply_pcg_parity(level, stride, apply):
    g, imgs, calib, p = _stage_case(W=104, H=78, grid_stride=stride, apply_mode=apply)
    try:
        g.run(g.sf.SF_STAGE_LEVEL_INIT, level)
        ls, _ = _oracle_level(imgs, calib, p, level)
        assert np.array_equal(g.read(g.sf.SF_DBG_CMASK, level).astype(bool),
                              ls.cmask.astype(bool))
        delta = np.random.default_rng(10 + level).normal(scale=0.4, size=(6, ls.grid.G))
        g.write(g.sf.SF_DBG_DELTA, level, delta.astype(np.float32))
        delta = g.read(g.sf.SF_DBG_DELTA, level).reshape(6, -1).astype(np.float64)
        g.run(g.sf.SF_STAGE_LINEARIZE, level)
        kink, kink_nodes = _kink_pixels(ls, delta)
        smooth_px = ~kink
        nodes6 = np.tile(~kink_nodes, 6)
        assert smooth_px.mean() > 0.98

        # per-pixel records: reweighted gradient (6) and Gauss-Newton block (21)
        J, r, w = O.robust_rows(ls, delta, p)
        gpx = np.einsum("nri,nr->in", J, w * r)
        gram = _gram_upper(np.einsum("nri,nr,nrj->nij", J, w, J))
        rec = g.read(g.sf.SF_DBG_REC, level).reshape(27, -1)
        for k in range(6):
            assert rel_err(rec[k][smooth_px], gpx[k][smooth_px]) < 2e-4, ("grad", k)
        for k in range(21):
            assert rel_err(rec[6 + k][smooth_px], gram[k][smooth_px]) < 2e-4, ("gram", k)

        # energy terms at the linearisation point
        e = O.energy(ls, delta, p)
        eg = g.read(g.sf.SF_DBG_ENERGY, level)
        for k, name in enumerate(("photo", "grad", "smooth", "epi", "mag", "total")):
            assert eg[k] == pytest.approx(e[name], rel=2e-5, abs=1e-6), name

        # right-hand side (r = -grad E) and diag(H)
        grad, Hm = O.linearize(ls, delta, p)
        R = g.read(g.sf.SF_DBG_R, level)
        assert rel_err(R[nodes6], -grad[nodes6]) < 2e-4
        D = g.read(g.sf.SF_DBG_DIAG, level)
        np.testing.assert_allclose(D[nodes6], Hm.diagonal()[nodes6], rtol=2e-4)

        # q = H p for a random p
        pv = np.random.default_rng(3).normal(size=6 * ls.grid.G).astype(np.float32)
        g.write(g.sf.SF_DBG_Z, level, pv)
        g.run(g.sf.SF_STAGE_APPLY, level)
        Q = g.read(g.sf.SF_DBG_Q, level)
        assert rel_err(Q[nodes6], (Hm @ pv.astype(np.float64))[nodes6]) < 2e-4
        np.testing.assert_array_equal(g.read(g.sf.SF_DBG_P, level), pv)

        # PCG from x = 0 on the same system
        g.run(g.sf.SF_STAGE_LINEARIZE, level)
        g.run(g.sf.SF_STAGE_PCG, level)
        dx = g.read(g.sf.SF_DBG_DX, level)
        ref = O.pcg(Hm, -grad, p.pcg_iters)
        assert rel_err(dx, ref) < 5e-3
    finally:
        g.close()


@pytest.mark.parametrize("apply", [0, 2])
def test_step_control_parity(apply):
    """Step control alone (SF_STAGE_STEP) against the oracle's rule: delta
    moves by tau dx for the first tau in 1, 1/2, ..., 1/16 whose energy does
    not exceed E(delta), or stays.  dx is the oracle's Gauss-Newton step
    scaled so that tau = 1, a shorter step and no step are each chosen;
    cases whose trial energies lie within 1e-4 of E(delta) (where float32
    and float64 may decide differently) are not counted."""
    g, imgs, calib, p = _stage_case(W=104, H=78, grid_stride=4, apply_mode=apply,
                                    max_backtracks=4)
    level = 1
    try:
        g.run(g.sf.SF_STAGE_LEVEL_INIT, level)
        ls, _ = _oracle_level(imgs, calib, p, level)
        delta = np.random.default_rng(4).normal(scale=0.3, size=(6, ls.grid.G))
        g.write(g.sf.SF_DBG_DELTA, level, delta.astype(np.float32))
        delta = g.read(g.sf.SF_DBG_DELTA, level).reshape(6, -1).astype(np.float64)
        grad, Hm = O.linearize(ls, delta, p)
        step = O.pcg(Hm, -grad, 40).reshape(6, -1)
        e0 = O.energy(ls, delta, p)["total"]
        taus = [2.0 ** -k for k in range(5)]
        seen = set()
        for scale in (1.0, 12.0, 40.0, -1.0):
            dx = (scale * step).astype(np.float32)
            g.write(g.sf.SF_DBG_DELTA, level, delta.astype(np.float32))
            g.run(g.sf.SF_STAGE_LINEARIZE, level)
            g.write(g.sf.SF_DBG_DX, level, dx)
            g.run(g.sf.SF_STAGE_STEP, level)
            got = g.read(g.sf.SF_DBG_DELTA, level).reshape(6, -1).astype(np.float64)
            et = [O.energy(ls, delta + t * dx.astype(np.float64), p)["total"] for t in taus]
            if min(abs(e - e0) for e in et) < 1e-4 * abs(e0):
                continue
            tau = next((t for t, e in zip(taus, et) if e <= e0), 0.0)
            want = delta + tau * dx.astype(np.float64)
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-5 * (1 + np.abs(want).max()))
            seen.add("full" if tau == 1.0 else ("none" if tau == 0.0 else "short"))
        assert seen == {"full", "short", "none"}, seen
    finally:
        g.close()


@pytest.mark.parametrize("level,apply", [(1, 1), (1, 2), (0, 2), (0, 3)])
def test_speculative_step_parity(level, apply):
    """The solve's speculative step control (SF_STAGE_SPEC_STEP: the
    linearisation at delta + dx, the shorter trials, then the next step's
    right-hand side and PCG) against the oracle's rule: delta moves by
    tau dx for the first acceptable tau (1, a shorter step, or none), and
    the energy, diag(H) and PCG solution that follow are the oracle's at
    the new delta.  A shorter step or none is the path where the
    right-hand-side kernel forms the pixel records itself and the PCG's
    first kernel moves delta.  Level 1 of 104 x 78 at stride 4 takes the
    one-workgroup PCG in apply_mode 2, level 0 the multi-kernel (2) or the
    co-resident (3) one."""
    g, imgs, calib, p = _stage_case(W=104, H=78, grid_stride=4, apply_mode=apply,
                                    max_backtracks=4)
    sf = g.sf
    try:
        g.run(sf.SF_STAGE_LEVEL_INIT, level)
        ls, _ = _oracle_level(imgs, calib, p, level)
        delta = np.random.default_rng(4).normal(scale=0.3, size=(6, ls.grid.G))
        g.write(sf.SF_DBG_DELTA, level, delta.astype(np.float32))
        delta = g.read(sf.SF_DBG_DELTA, level).reshape(6, -1).astype(np.float64)
        grad, Hm = O.linearize(ls, delta, p)
        step = O.pcg(Hm, -grad, 40).reshape(6, -1)
        e0 = O.energy(ls, delta, p)["total"]
        taus = [2.0 ** -k for k in range(5)]
        seen = set()
        for scale in (1.0, 12.0, 40.0, -1.0):
            dx = (scale * step).astype(np.float32)
            g.write(sf.SF_DBG_DELTA, level, delta.astype(np.float32))
            g.run(sf.SF_STAGE_LINEARIZE, level)
            g.write(sf.SF_DBG_DX, level, dx)
            g.run(sf.SF_STAGE_SPEC_STEP, level)
            got = g.read(sf.SF_DBG_DELTA, level).reshape(6, -1).astype(np.float64)
            et = [O.energy(ls, delta + t * dx.astype(np.float64), p)["total"] for t in taus]
            if min(abs(e - e0) for e in et) < 1e-4 * abs(e0):
                continue
            tau = next((t for t, e in zip(taus, et) if e <= e0), 0.0)
            want = delta + tau * dx.astype(np.float64)
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-5 * (1 + np.abs(want).max()))
            # the next step, at the new delta as the GPU holds it
            e = O.energy(ls, got, p)
            eg = g.read(sf.SF_DBG_ENERGY, level)
            for k, name in enumerate(("photo", "grad", "smooth", "epi", "mag", "total")):
                assert eg[k] == pytest.approx(e[name], rel=2e-5, abs=1e-6), (scale, name)
            grad2, H2 = O.linearize(ls, got, p)
            _, kink_nodes = _kink_pixels(ls, got)
            nodes6 = np.tile(~kink_nodes, 6)
            D = g.read(sf.SF_DBG_DIAG, level)
            np.testing.assert_allclose(D[nodes6], H2.diagonal()[nodes6], rtol=2e-4)
            dxn = g.read(sf.SF_DBG_DX, level)
            assert rel_err(dxn, O.pcg(H2, -grad2, p.pcg_iters)) < 5e-3, scale
            seen.add("full" if tau == 1.0 else ("none" if tau == 0.0 else "short"))
        assert seen == {"full", "short", "none"}, seen
    finally:
        g.close()


def _solve_parity(imgs, calib, prm, e_tol=1e-4, f_tol=0.02):
    p = oracle_params(**prm)
    rec = []
    res = O.solve(imgs.astype(np.float64), calib, p, record=rec)
    g = GpuCase(imgs, calib, **prm)
    try:
        depth, flow3d, flows = g.solve()
        log, code = g.log()
    finally:
        g.close()
    assert code == 0
    assert len(log) == len(rec)
    worst = 0.0
    for lg, ro in zip(log, rec):
        assert lg["level"] == ro["level"]
        rel = abs(lg["energy"] - ro["energy"]) / abs(ro["energy"])
        worst = max(worst, rel)
        assert rel <= e_tol, (lg["level"], lg["gn_iter"], lg["energy"], ro["energy"],
                              [l["tau"] for l in log], [r["tau"] for r in rec])
        assert lg["energy_after"] <= lg["energy"]
    grid = res["grid"]
    ref_flows = grid.to_pixels(res["total"]).reshape(6, grid.H, grid.W)
    err = np.abs(flows - ref_flows).max()
    assert err <= f_tol, err
    check_output(depth, flow3d, flows, grid.W, grid.H, calib, ref_flows, err)
    return worst, err, log, rec


def test_solve_tiny_parity():
    imgs, calib, _ = make_frame(tiny_plane_config(), 0)
    prm = dict(levels=3, grid_stride=8, gn_iters=5, pcg_iters=10)
    _solve_parity(imgs, calib, prm)


@pytest.mark.parametrize("W,H,stride,apply", [(100, 76, 4, 0), (160, 120, 4, 0), (96, 72, 2, 0),
                                              (144, 104, 8, 0), (100, 76, 4, 1),
                                              (160, 120, 4, 1), (96, 72, 2, 1),
                                              (144, 104, 8, 1), (90, 70, 3, 1),
                                              (100, 76, 4, 2), (160, 120, 4, 2),
                                              (96, 72, 2, 2), (144, 104, 8, 2),
                                              (160, 120, 4, 3), (96, 72, 2, 3),
                                              (144, 104, 4, 3), (200, 150, 2, 3)])
def test_solve_medium_parity(W, H, stride, apply):
    imgs, calib = _frame(W, H, seed=7)
    prm = dict(levels=3, grid_stride=stride, gn_iters=4, pcg_iters=10, apply_mode=apply)
    _solve_parity(imgs, calib, prm)


@pytest.mark.parametrize("apply", [1, 2])
def test_solve_tiny_parity_node_blocks(apply):
    imgs, calib, _ = make_frame(tiny_plane_config(), 0)
    prm = dict(levels=3, grid_stride=8, gn_iters=5, pcg_iters=10, apply_mode=apply)
    _solve_parity(imgs, calib, prm)


@pytest.mark.parametrize("apply", [0, 1, 2, 3])
def test_graph_replay_matches_eager_and_repeats(apply):
    imgs, calib = _frame(128, 96, seed=9)
    prm = dict(levels=3, grid_stride=4, gn_iters=3, pcg_iters=8, apply_mode=apply)
    outs = []
    for mode in (1, 0, 0):
        g = GpuCase(imgs, calib, exec_mode=mode, **prm)
        try:
            first = g.solve()
            second = g.solve() if mode == 0 else first
            outs.append((first, second, g.log()[0]))
        finally:
            g.close()
    eager = outs[0][0]
    for first, second, log in outs[1:]:
        for a, b in zip(eager, first):
            np.testing.assert_array_equal(a, b)
        for a, b in zip(first, second):
            np.testing.assert_array_equal(a, b)
        assert [l["energy"] for l in log] == [l["energy"] for l in outs[0][2]]


@pytest.mark.parametrize("apply", [0, 2])
@pytest.mark.parametrize("W,H,stride,mode", [(100, 76, 4, 2), (100, 76, 4, 3), (96, 72, 2, 2),
                                             (96, 72, 2, 3), (144, 104, 8, 2),
                                             (144, 104, 8, 3), (100, 76, 4, 4)])
def test_solve_pcg_tile_variants(W, H, stride, mode, apply):
    """The alternative PCG tile shapes (matrix-free per stride, node-block
    16 x 8, 8 x 4 and 4 x 4 nodes) give the oracle's solve too."""
    imgs, calib = _frame(W, H, seed=7)
    prm = dict(levels=3, grid_stride=stride, gn_iters=4, pcg_iters=10, tile_mode=mode,
               apply_mode=apply)
    _solve_parity(imgs, calib, prm)


@pytest.mark.parametrize("apply", [0, 2])
def test_autotuned_tiles_parity_and_cache(tmp_path, monkeypatch, apply):
    """tile_mode 1: every level's shape is timed on the first solve and
    cached (process and SF_TUNE_CACHE file); a second context reuses the
    cache and gives the same result bitwise."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SF_TUNE_CACHE", str(cache))
    imgs, calib = _frame(160, 120, seed=7)
    prm = dict(levels=3, grid_stride=4, gn_iters=4, pcg_iters=10, tile_mode=1, apply_mode=apply)
    _solve_parity(imgs, calib, prm)
    g = GpuCase(imgs, calib, **prm)
    try:
        first = g.solve()
    finally:
        g.close()
    g = GpuCase(imgs, calib, **prm)
    try:
        second = g.solve()
    finally:
        g.close()
    for a, b in zip(first, second):
        np.testing.assert_array_equal(a, b)
    lines = cache.read_text().split("\n") if cache.exists() else []
    # entries of this process may have been cached before the variable was
    # set (a shape tuned earlier in the session); at least the file parses
    for ln in filter(None, lines):
        key, v = ln.split()
        assert "/s4/" in key and v in ("0", "1", "2", "3")


@pytest.mark.parametrize("apply", [0, 2])
def test_solve_split_schedule_parity(apply):
    """gn_fine: the paper's split schedule (fewer Gauss-Newton steps on the
    two finest levels, Sec. 6.2)."""
    imgs, calib = _frame(160, 120, seed=7)
    prm = dict(levels=4, grid_stride=4, gn_iters=4, gn_fine=2, pcg_iters=5, apply_mode=apply)
    _, _, log, _ = _solve_parity(imgs, calib, prm)
    assert [r["level"] for r in log] == [3] * 4 + [2] * 4 + [1] * 2 + [0] * 2


@pytest.mark.parametrize("apply", [0, 2])
def test_identity_images_give_zero_flow(apply):
    """Degenerate case: four identical images and the zero start.  Every
    photometric and gradient residual is exactly zero (every position is the
    pixel itself), the rectified epipolar residual r_y - l_y is zero, so the
    right-hand side vanishes, the PCG takes its breakdown exit (r.z = 0) and
    the flows stay exactly zero; E = 6 sum_x V W eps (w_photo + w_grad) at
    every step, with V = W = 1 (Eqs. (8)-(12); Sec. 5.1).  Depth is NaN
    everywhere (zero disparity)."""
    imgs, calib = _frame(96, 72, seed=3)
    same = np.repeat(imgs[:1], 4, axis=0)
    prm = dict(levels=3, grid_stride=4, gn_iters=3, pcg_iters=8, apply_mode=apply)
    g = GpuCase(same, calib, **prm)
    try:
        depth, flow3d, flows = g.solve()
        log, code = g.log()
    finally:
        g.close()
    assert code == 0 and len(log) == 9
    p = oracle_params(**prm)
    for lg in log:
        H, W = 72 >> lg["level"], 96 >> lg["level"]
        e = 6 * H * W * p.eps * (p.w_photo + p.w_grad)
        assert abs(lg["energy"] - e) <= 2e-6 * e, (lg, e)
        assert lg["energy_after"] == lg["energy"]
        assert lg["n_valid"] == H * W
        assert all(r == 0.0 for r in lg["pcg_res"]), lg["pcg_res"]
    assert not flows.any()
    assert np.isnan(depth).all() and np.isnan(flow3d).all()


@pytest.mark.parametrize("apply", [0, 2])
def test_stereo_only_call(apply):
    """Stereo-only reconstruction is the same call with the pair at t
    passed again as the pair at t+1 (Sec. 6.4).  The energy is then
    symmetric under exchanging the two times, which maps (s, m, d) to
    (s, -m, -d) (Eqs. (1)-(6)), so from the zero start the motion and the
    temporal disparity change stay zero up to rounding; the solve matches
    the oracle's, and depth and 3D flow match its output (the 3D flow is
    zero up to rounding)."""
    imgs, calib = _frame(128, 96, seed=4, disp=6.0)
    stereo = np.stack([imgs[0], imgs[1], imgs[0], imgs[1]])
    prm = dict(levels=3, grid_stride=4, gn_iters=4, pcg_iters=10, apply_mode=apply)
    _, err, log, _ = _solve_parity(stereo, calib, prm)
    g = GpuCase(stereo, calib, **prm)
    try:
        depth, flow3d, flows = g.solve()
    finally:
        g.close()
    assert np.abs(flows[2:]).max() <= 1e-4, np.abs(flows[2:]).max()
    assert np.abs(flows[0]).max() > 0.5           # the stereo disparity was found
    fin = np.isfinite(flow3d).all(0)
    assert fin.mean() > 0.9
    assert np.abs(flow3d[:, fin]).max() <= 1e-3 * np.nanmax(depth)


def test_tiled_pcg_gives_up_without_hanging(monkeypatch):
    """apply_mode 3 with the co-resident tiled PCG's waits forced to give up
    at once (a spin limit of zero set from the host): every workgroup still
    exits, sf_get_log reports SF_ERR_STATE for that solve, and the next
    solve of the context runs the per-iteration kernels and matches the
    oracle."""
    from paper_1610_07159_amd import sf
    imgs, calib = _frame(160, 120, seed=7)
    prm = dict(levels=3, grid_stride=4, gn_iters=4, pcg_iters=10, apply_mode=3)
    monkeypatch.setenv("SF_MID_SPIN_LIMIT", "0")
    g = GpuCase(imgs, calib, exec_mode=0, **prm)
    try:
        g.solve()
        with pytest.raises(sf.SfError) as e:
            g.log()
        assert e.value.code == -6
        assert "gave up" in sf.lib.sf_last_error().decode()
        monkeypatch.delenv("SF_MID_SPIN_LIMIT")
        depth, flow3d, flows = g.solve()
        log, code = g.log()
    finally:
        g.close()
    assert code == 0
    p = oracle_params(**prm)
    rec = []
    res = O.solve(imgs.astype(np.float64), calib, p, record=rec)
    for lg, ro in zip(log, rec):
        assert abs(lg["energy"] - ro["energy"]) <= 1e-4 * abs(ro["energy"])
    grid = res["grid"]
    ref = grid.to_pixels(res["total"]).reshape(6, grid.H, grid.W)
    assert np.abs(flows - ref).max() <= 0.02
