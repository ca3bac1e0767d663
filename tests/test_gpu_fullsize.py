"""Parity at the benchmark workloads' full sizes (640x480 and 1280x720 at
strides 2, 4, 8), in the launch configuration bench.py times (captured
graph, autotuned PCG tiles), on outputs the oracle computes one by one:
masks and smoothness weights, the total energy, the linearisation records
of sampled pixels and the gradient, diag(H) and H u of sampled nodes, at a
level-0 state the test sets; plus properties of the full solve (energy never
increases, finite outputs).

Tolerances: those of test_gpu_parity.py (2e-4 relative for records, node
rows and products) scaled by the float32 spacing of the largest sample
coordinate relative to 640 px: a position near x carries a rounding error
of up to half an ulp of x, which enters the bilinear fractions and through
them the interpolant derivatives, so the attainable agreement halves
beyond 1024 px (spacing 2^-13 px instead of 2^-14).  Pixels whose sample
positions lie within two such spacings (and at least 1e-4 px) of a
bilinear kink, and pixels whose mask flips at a threshold, are left out of
the sampled comparisons (both choices there are valid), and so are pixels
where one of their residuals d_k or |g_k| lies within 10 eps of zero: there
the reweighting c / Phi has curvature ~ 1 / eps and amplifies the float32
rounding of the sample positions a thousandfold.  Those pixels still enter
the total energy and the node sums compared above and below."""
import functools

import numpy as np
import pytest

import oracle.halfway as O
from synth import make_frame, vga_config, hd_config

from gpu_util import GpuCase, oracle_params, mask_flip_ok, rel_err

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=2)
def _frame(name):
    cfg, seed = {"vga": (vga_config(), 1), "hd": (hd_config(), 2)}[name]
    imgs, calib, _ = make_frame(cfg, seed)
    return imgs, calib


def _smooth_field(grid, amp, seed):
    """Node flows varying smoothly over the image (bilinear of a 4x4 random
    lattice), amplitude amp px."""
    rng = np.random.default_rng(seed)
    lat = rng.normal(0, amp, (6, 4, 4))
    nx, ny = grid.node_xy()
    u = np.clip(nx / (grid.W - 1), 0, 1) * 3
    v = np.clip(ny / (grid.H - 1), 0, 1) * 3
    i0 = np.minimum(np.floor(u).astype(int), 2)
    j0 = np.minimum(np.floor(v).astype(int), 2)
    fu, fv = u - i0, v - j0
    return ((1 - fv) * ((1 - fu) * lat[:, j0, i0] + fu * lat[:, j0, i0 + 1])
            + fv * ((1 - fu) * lat[:, j0 + 1, i0] + fu * lat[:, j0 + 1, i0 + 1]))


@pytest.mark.parametrize("name,W,H,stride,levels", [("vga", 640, 480, 4, 5),
                                                    ("hd", 1280, 720, 2, 6),
                                                    ("hd", 1280, 720, 4, 6),
                                                    ("hd", 1280, 720, 8, 6)])
def test_fullsize_parity(name, W, H, stride, levels):
    imgs, calib = _frame(name)
    prm = dict(levels=levels, grid_stride=stride, gn_iters=10, pcg_iters=20, tile_mode=1)
    p = oracle_params(**prm)
    g = GpuCase(imgs, calib, exec_mode=0, **prm)
    try:
        # the full solve as benchmarked (also tunes the tiles)
        depth, flow3d, flows = g.solve()
        log, code = g.log()
        assert code == 0 and len(log) == levels * 10
        assert all(r["energy_after"] <= r["energy"] for r in log)
        assert np.isfinite(flows).all() and np.isfinite(flow3d[:, np.isfinite(depth)]).all()
        assert np.isfinite(depth).mean() > 0.95

        # a level-0 state chosen here
        sf = g.sf
        grid = O.Grid(W, H, stride)
        base = _smooth_field(grid, 1.5, 11)
        delta = np.random.default_rng(12).normal(0, 0.3, (6, grid.G))
        g.write(sf.SF_DBG_BASE, 0, base.astype(np.float32))
        g.write(sf.SF_DBG_DELTA, 0, np.zeros((6, grid.G), np.float32))  # level start
        g.run(sf.SF_STAGE_MASKS, 0)
        g.write(sf.SF_DBG_DELTA, 0, delta.astype(np.float32))
        g.run(sf.SF_STAGE_LINEARIZE, 0)
        base = base.astype(np.float32).astype(np.float64)
        delta = delta.astype(np.float32).astype(np.float64)
        np.testing.assert_array_equal(g.read(sf.SF_DBG_BASE, 0).reshape(6, -1), base)
        np.testing.assert_array_equal(g.read(sf.SF_DBG_DELTA, 0).reshape(6, -1), delta)

        pyr = O.pyramid(imgs.astype(np.float64), 1)
        li = O.LevelImages.build(pyr[0])
        F0 = O.level_calib_F(O.Calib.from_dict(calib).F, 0)
        cm_gpu = g.read(sf.SF_DBG_CMASK, 0).astype(bool)
        cm_ref, flips = mask_flip_ok(li, grid, base, p, cm_gpu)
        assert flips <= 1e-4 * grid.N
        w_ref = O.node_weights(li, grid, base, 0, p)
        np.testing.assert_allclose(g.read(sf.SF_DBG_WNODE, 0), w_ref, rtol=1e-4, atol=1e-5)
        ls = O.LevelState(0, li, grid, base, cm_ref, w_ref, F0)

        # total energy: float32 sums, plus the energy of any flipped pixel
        e_ref = O.energy(ls, delta, p)
        flip_pix = np.nonzero(cm_ref.astype(bool) != cm_gpu)[0]
        e_flip = 0.0
        if flip_pix.size:
            J, r, w = O.rows_at(ls, delta, p, flip_pix)
            t = O.pixel_terms_xy(li, (flip_pix % W).astype(float), (flip_pix // W).astype(float),
                                 O.flows_at(grid, base + delta, flip_pix))
            ep, eg = O.pixel_energy(t, np.ones(flip_pix.size), p)
            e_flip = float(p.w_photo * ep.sum() + p.w_grad * eg.sum())
        eg_gpu = g.read(sf.SF_DBG_ENERGY, 0)
        assert abs(eg_gpu[5] - e_ref["total"]) <= 2e-5 * abs(e_ref["total"]) + e_flip

        # sampled pixels away from kinks and mask flips
        ulp = float(np.spacing(np.float32(max(W, H))))
        tol = 2e-4 * ulp / float(np.spacing(np.float32(640)))
        P = O.positions(*grid.pixel_xy(), grid.to_pixels(base + delta))
        kink = (np.abs(P - np.round(P)) < max(1e-4, 2 * ulp)).any(axis=(0, 1))
        ok_pix = ~kink & (cm_ref.astype(bool) == cm_gpu)
        rng = np.random.default_rng(13)
        cand = rng.choice(np.nonzero(ok_pix)[0], 30000, replace=False)
        _, rc, _ = O.rows_at(ls, delta, p, cand)
        gnorm = np.hypot(rc[:, 6:18:2], rc[:, 7:18:2])
        well = (np.abs(rc[:, :6]).min(1) > 10 * p.eps) & (gnorm.min(1) > 10 * p.eps)
        pix = cand[well][:300]
        assert pix.size == 300
        J, r, w = O.rows_at(ls, delta, p, pix)
        gpx = np.einsum("nri,nr->in", J, w * r)
        iu = np.triu_indices(6)
        gram = np.einsum("nri,nr,nrj->nij", J, w, J)[:, iu[0], iu[1]].T
        rec = g.read(sf.SF_DBG_REC, 0).reshape(27, -1)[:, pix]
        assert rel_err(rec[:6], gpx) < tol
        assert rel_err(rec[6:], gram) < tol

        # sampled nodes whose support has no kink or flipped pixel
        bad = np.zeros(grid.G, bool)
        for k in range(4):
            bad[grid.nodes[k][~ok_pix]] = True
        nodes = rng.choice(np.nonzero(~bad)[0], 24, replace=False)
        u = rng.normal(size=(6, grid.G))
        grad, diag, _ = O.node_rows(ls, delta, p, nodes, u)
        R = g.read(sf.SF_DBG_R, 0).reshape(6, -1)[:, nodes]
        D = g.read(sf.SF_DBG_DIAG, 0).reshape(6, -1)[:, nodes]
        assert rel_err(R, -grad) < tol
        assert rel_err(D, diag) < tol
        u32 = u.astype(np.float32)
        g.write(sf.SF_DBG_Z, 0, u32.reshape(-1))
        g.run(sf.SF_STAGE_APPLY, 0)
        np.testing.assert_array_equal(g.read(sf.SF_DBG_P, 0), u32.reshape(-1))
        Q = g.read(sf.SF_DBG_Q, 0).reshape(6, -1)[:, nodes]
        _, _, Hu32 = O.node_rows(ls, delta, p, nodes, u32.astype(np.float64))
        assert rel_err(Q, Hu32) < tol
    finally:
        g.close()
