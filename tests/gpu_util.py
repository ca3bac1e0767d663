"""Shared helpers of the GPU parity tests: build a solver context through the
C ABI, mirror its parameters into the oracle, and compare with flip-aware
mask checks.  Inputs come from the seeded generator only."""
import numpy as np

import oracle.halfway as O

PARAM_FIELDS = ("levels", "grid_stride", "gn_iters", "pcg_iters",
                "max_backtracks", "w_reg", "w_photo", "w_grad", "w_epi",
                "w_smooth", "w_mag", "w_s", "w_m", "w_d", "m_s", "m_m", "m_d",
                "eps", "eps_p", "st_gamma", "st_tau", "illum", "occlusion")


def oracle_params(**kw):
    out = {k: v for k, v in kw.items() if k in PARAM_FIELDS}
    for k in ("illum", "occlusion"):
        if k in out:
            out[k] = bool(out[k])
    return O.Params(**out)


class GpuCase:
    """A context plus its device images; everything through the C ABI."""

    def __init__(self, images, calib, exec_mode=1, **params):
        import torch
        from paper_1610_07159_amd import sf
        self.sf = sf
        self.torch = torch
        self.images_np = np.asarray(images, np.float32)
        self.calib = calib
        _, H, W = self.images_np.shape
        self.W, self.H = W, H
        self.kw = dict(params)
        self.p = sf.sf_params_default(exec_mode=exec_mode, **params)
        self.stream = torch.cuda.current_stream()
        self.ctx = sf.sf_create(W, H, self.p, int(self.stream.cuda_stream))
        self.img = torch.from_numpy(self.images_np).cuda().contiguous()
        self.cal = sf.make_calib(calib["fx"], calib["fy"], calib["cx"],
                                 calib["cy"], calib["baseline"], calib["F"])

    def ptrs(self):
        return [self.img[k].data_ptr() for k in range(4)]

    def load(self, images):
        """Replaces the device images (the next frame of a sequence)."""
        self.images_np = np.asarray(images, np.float32)
        self.img.copy_(self.torch.from_numpy(self.images_np))

    def set_images(self):
        self.sf.sf_debug_set_images(self.ctx, *self.ptrs(), self.cal)

    def run(self, stage, level):
        self.sf.sf_debug_run(self.ctx, stage, level)

    def read(self, what, level):
        return self.sf.sf_debug_read(self.ctx, what, level)

    def write(self, what, level, arr):
        self.sf.sf_debug_write(self.ctx, what, level, arr)

    def solve(self):
        torch = self.torch
        H, W = self.H, self.W
        depth = torch.empty((H, W), device="cuda")
        flow3d = torch.empty((3, H, W), device="cuda")
        flows = torch.empty((6, H, W), device="cuda")
        self.sf.sf_solve(self.ctx, *self.ptrs(), self.cal, None,
                         depth.data_ptr(), flow3d.data_ptr(), flows.data_ptr())
        torch.cuda.synchronize()
        return depth.cpu().numpy(), flow3d.cpu().numpy(), flows.cpu().numpy()

    def log(self):
        return self.sf.sf_get_log(self.ctx)

    def close(self):
        if self.ctx is not None:
            self.sf.sf_destroy(self.ctx)
            self.ctx = None


def mask_flip_ok(li, grid, total, p, gpu_mask):
    """Compares V W with the oracle's; a differing pixel is accepted only if
    the oracle's deciding quantity is within float32 rounding of its
    threshold (max_k |d_k| vs eps_p, or a position vs an image border).
    Returns (oracle mask, number of flips)."""
    V, Wm = O.masks(li, grid, total, p)
    ref = (V & Wm)
    diff = np.nonzero(ref != gpu_mask.astype(bool))[0]
    if diff.size:
        flows = grid.to_pixels(total)
        px, py = grid.pixel_xy()
        P = O.positions(px, py, flows)
        t = O.pixel_terms(li, grid, flows)
        H, W = li.shape
        dmax = np.abs(t.d).max(0)
        for i in diff:
            near_p = abs(dmax[i] - p.eps_p) < 1e-5
            b = np.concatenate([P[:, 0, i], W - 1 - P[:, 0, i], P[:, 1, i],
                                H - 1 - P[:, 1, i]])
            near_v = np.abs(b).min() < 1e-4
            assert near_p or near_v, (
                f"mask differs at pixel {i} away from any threshold "
                f"(dmax {dmax[i]}, border distance {np.abs(b).min()})")
    return ref.astype(np.float64), int(diff.size)


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
