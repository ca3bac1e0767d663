"""Batched solves through sf_solve_batch: every frame of a batch of mixed
sizes (and level counts) must give bitwise the result of a single-frame
solve with the same parameters and level count, the batch graph must replay
identically, and a frame of the batch is checked against the FP64 oracle
directly (per-step energy 1e-4 relative, flows 0.02 px)."""
import numpy as np
import pytest

import oracle.halfway as O
from synth import make_frame, sized_config

from gpu_util import GpuCase, oracle_params

pytestmark = pytest.mark.gpu

PRM = dict(levels=3, grid_stride=4, gn_iters=3, pcg_iters=8)


def _frames(sizes, seed0=20):
    out = []
    for k, (W, H) in enumerate(sizes):
        imgs, calib, _ = make_frame(sized_config(W, H, max_disp=0.05 * W), seed0 + k)
        out.append((imgs, calib))
    return out


def _batch(frames, exec_mode=0, repeat=1, **prm):
    import torch
    from paper_1610_07159_amd import sf, SceneFlowSolver
    W0, H0 = frames[0][0].shape[2], frames[0][0].shape[1]
    solver = SceneFlowSolver(W0, H0, exec_mode=exec_mode, **prm)
    try:
        dev = [(torch.from_numpy(np.asarray(i, np.float32)).cuda().contiguous(), c)
               for i, c in frames]
        params = sf.sf_params_default(exec_mode=exec_mode, **prm)
        results = []
        for _ in range(repeat):
            outs = solver.solve_batch(dev, params=params)
            torch.cuda.synchronize()
            results.append([tuple(t.cpu().numpy() for t in o) for o in outs])
        logs = [solver.batch_log(f) for f in range(len(frames))]
    finally:
        solver.close()
    return results, logs


@pytest.mark.parametrize("stride,apply", [(4, 0), (8, 0), (4, 1), (8, 1), (4, 2), (8, 2)])
def test_batch_matches_single_frames_bitwise(stride, apply):
    from paper_1610_07159_amd import sf
    sizes = [(160, 120), (96, 72), (128, 96), (100, 76), (200, 150)]
    frames = _frames(sizes)
    prm = dict(PRM, grid_stride=stride, apply_mode=apply)
    (res, res2), logs = _batch(frames, exec_mode=0, repeat=2, **prm)
    for f, ((imgs, calib), (W, H)) in enumerate(zip(frames, sizes)):
        L = sf.sf_batch_levels(W, H, prm["levels"])
        assert L == (3 if W >= 160 else 2)
        g = GpuCase(imgs, calib, exec_mode=1, **dict(prm, levels=L))
        try:
            single = g.solve()
            slog, code = g.log()
        finally:
            g.close()
        assert code == 0
        es, eb = [r["energy"] for r in slog], [r["energy"] for r in logs[f]]
        first = next((k for k, (x, y) in enumerate(zip(es, eb)) if x != y), None)
        assert first is None, (f, first, es[first], eb[first])
        assert [r["tau"] for r in slog] == [r["tau"] for r in logs[f]]
        for a, b, c in zip(single, res[f], res2[f]):
            np.testing.assert_array_equal(a, b)
            np.testing.assert_array_equal(b, c)
        assert [r["level"] for r in logs[f]] == [l for l in range(L - 1, -1, -1)
                                                for _ in range(prm["gn_iters"])]


def test_batch_rejected_speculative_step_matches_single_frame():
    """A frame whose solve rejects tau = 1 in a speculative step (level 2,
    Gauss-Newton step 8 of 10, tau = 1/2: the right-hand-side kernel forms
    the pixel records at delta + tau dx itself, over eight tiles that share
    region pixels, and writes the gradients it recomputes over the
    per-pixel records) solves bitwise alike alone and inside a batch of
    other frames, in every log entry and output."""
    from paper_1610_07159_amd import sf
    W, H = 160, 120
    imgs, calib, _ = make_frame(sized_config(W, H, max_disp=0.12 * W), 134)
    prm = dict(levels=4, grid_stride=4, gn_iters=10, pcg_iters=20)
    L = sf.sf_batch_levels(W, H, prm["levels"])
    frames = [(imgs, calib)] + _frames([(200, 150), (160, 120), (128, 96)], seed0=60)
    (res, res2), logs = _batch(frames, exec_mode=0, repeat=2, **prm)
    g = GpuCase(imgs, calib, exec_mode=1, **dict(prm, levels=L))
    try:
        single = g.solve()
        slog, code = g.log()
    finally:
        g.close()
    assert code == 0
    rejected = [(r["level"], r["gn_iter"], r["tau"]) for r in slog
                if r["tau"] < 1.0 and r["gn_iter"] < prm["gn_iters"] - 1]
    assert rejected, "the frame no longer rejects a speculative step"
    assert [r["energy"] for r in slog] == [r["energy"] for r in logs[0]]
    assert [r["energy_after"] for r in slog] == [r["energy_after"] for r in logs[0]]
    assert [r["tau"] for r in slog] == [r["tau"] for r in logs[0]]
    for a, b, c in zip(single, res[0], res2[0]):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(b, c)


def test_batch_direct_launches_match_graph_and_reshape():
    frames = _frames([(128, 96), (160, 120), (112, 80)], seed0=40)
    g_res, g_logs = _batch(frames, exec_mode=0, **PRM)
    d_res, d_logs = _batch(frames, exec_mode=1, **PRM)
    for a, b in zip(g_res[0], d_res[0]):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
    # a different batch shape on the same context rebuilds the workspace
    import torch
    from paper_1610_07159_amd import sf, SceneFlowSolver
    solver = SceneFlowSolver(128, 96, exec_mode=0, **PRM)
    try:
        params = sf.sf_params_default(exec_mode=0, **PRM)
        dev = [(torch.from_numpy(i).cuda().contiguous(), c) for i, c in frames]
        first = solver.solve_batch(dev, params=params)
        second = solver.solve_batch(dev[1:], params=params)
        again = solver.solve_batch(dev, params=params)
        torch.cuda.synchronize()
        for a, b in zip(first, again):
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
        for a, b in zip(first[1:], second):
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    finally:
        solver.close()


def test_batch_frame_oracle_parity():
    frames = _frames([(160, 120), (96, 72)], seed0=60)
    res, logs = _batch(frames, exec_mode=0, **PRM)
    for f, (imgs, calib) in enumerate(frames):
        W = imgs.shape[2]
        L = 3 if W >= 160 else 2
        p = oracle_params(**dict(PRM, levels=L))
        rec = []
        ref = O.solve(imgs.astype(np.float64), calib, p, record=rec)
        assert len(rec) == len(logs[f])
        for lg, ro in zip(logs[f], rec):
            assert abs(lg["energy"] - ro["energy"]) <= 1e-4 * abs(ro["energy"])
        grid = ref["grid"]
        flows = grid.to_pixels(ref["total"]).reshape(6, grid.H, grid.W)
        assert np.abs(res[0][f][2] - flows).max() <= 0.02


def test_batch_learned_init_matches_single_frames_and_oracle():
    """init_mode 1 in a batch: the frames with a level 4 (640x480 and
    960x540 at 5 levels) run the shipped network, grouped by level-4 size,
    each with its own fallback decision; the 320x240 frame (4 levels by the
    batch's rule) starts from zero.  Every frame equals its single-frame
    solve bitwise (learned or zero-initialised), and the 640x480 frame
    matches the oracle's learned solve stored in tests/golden/."""
    import hashlib
    import json
    import os
    import torch
    from paper_1610_07159_amd import sf, SceneFlowSolver
    from synth import vga_config
    from gpu_util import check_output
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    z = np.load(os.path.join(root, "tests", "golden", "fullsize_vga640x480_s4_learned.npz"))
    meta = json.loads(str(z["meta"]))
    weights = np.load(os.path.join(root, "paper_1610_07159_amd", "weights", meta["weights"]),
                      allow_pickle=False)
    gold_imgs, gold_calib, _ = make_frame(vga_config(), meta["seed"])
    assert hashlib.sha256(gold_imgs.tobytes()).hexdigest() == str(z["images_sha256"])
    frames = [(gold_imgs, gold_calib)] + _frames([(320, 240), (960, 540), (640, 480)], seed0=70)
    prm = dict(levels=5, grid_stride=4, gn_iters=meta["gn_iters"], pcg_iters=meta["pcg_iters"],
               init_mode=1)
    solver = SceneFlowSolver(640, 480, exec_mode=0, **prm)
    try:
        sf.sf_set_initializer(solver.ctx, weights)
        dev = [(torch.from_numpy(i).cuda().contiguous(), c) for i, c in frames]
        outs = solver.solve_batch(dev, params=sf.sf_params_default(exec_mode=0, **prm))
        torch.cuda.synchronize()
        res = [tuple(t.cpu().numpy() for t in o) for o in outs]
        logs = [solver.batch_log(f) for f in range(len(frames))]
        init = [solver.batch_init_result(f) for f in range(len(frames))]
    finally:
        solver.close()
    for f, (imgs, calib) in enumerate(frames):
        H, W = imgs.shape[1:]
        L = sf.sf_batch_levels(W, H, 5)
        learned = L >= 5
        assert (init[f][0] >= 0) == learned
        g = GpuCase(imgs, calib, exec_mode=1, **dict(prm, levels=L, init_mode=int(learned)))
        try:
            if learned:
                sf.sf_set_initializer(g.ctx, weights)
            single = g.solve()
            slog, code = g.log()
            if learned:
                used, ep, ez = sf.sf_get_init_result(g.ctx)
                assert (bool(init[f][0]), init[f][1], init[f][2]) == (used, ep, ez)
        finally:
            g.close()
        assert code == 0
        for a, b in zip(res[f], single):
            np.testing.assert_array_equal(a, b)
        assert [r["energy"] for r in logs[f]] == [r["energy"] for r in slog]
    # the golden frame against the oracle's learned solve
    from test_gpu_fullsize import learned_energy_tol, network_difference, _sensitivity
    assert bool(init[0][0]) == meta["prediction_kept"]
    assert init[0][2] == pytest.approx(meta["e_zero"], rel=1e-5)
    e_tol = learned_energy_tol(init[0][1], meta["e_pred"])
    for k, lg in enumerate(logs[0]):
        assert abs(lg["energy"] - z["energy"][k]) <= e_tol * abs(z["energy"][k])
    grid = O.Grid(640, 480, 4)
    ref = grid.to_pixels(z["total0"].astype(np.float64)).reshape(6, 480, 640)
    # the network's bf16 flips move the start; the final flows are held to
    # the learned bar of test_gpu_fullsize
    assert network_difference(weights, gold_imgs) <= 2e-4
    sens = _sensitivity("vga640x480_s4_learned")
    diff = np.abs(res[0][2] - ref).max(axis=0)
    err = float(diff.max())
    assert (diff <= 0.02 + 2 * sens["p999_px"]).mean() >= 0.999
    assert err <= 0.02 + 2 * sens["max_px"]
    check_output(res[0][0], res[0][1], res[0][2], 640, 480, gold_calib, ref, err)


def test_batch_learned_init_needs_weights():
    import torch
    from paper_1610_07159_amd import sf, SceneFlowSolver
    frames = _frames([(640, 480)], seed0=80)
    prm = dict(levels=5, grid_stride=4, gn_iters=1, pcg_iters=4, init_mode=1)
    solver = SceneFlowSolver(640, 480, exec_mode=0, **dict(prm, init_mode=0))
    try:
        dev = [(torch.from_numpy(i).cuda().contiguous(), c) for i, c in frames]
        with pytest.raises(sf.SfError) as e:
            solver.solve_batch(dev, params=sf.sf_params_default(exec_mode=0, **prm))
        assert e.value.code == -6
    finally:
        solver.close()
