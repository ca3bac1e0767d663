"""Torch-facing convenience wrapper over the C ABI: allocates the output
tensors with torch and passes device addresses and the current HIP stream
to libsf.so.  No computation happens here."""
from __future__ import annotations

import numpy as np

from . import sf


def calib_from_dict(d) -> sf.sf_calib:
    return sf.make_calib(d["fx"], d["fy"], d["cx"], d["cy"], d["baseline"],
                         d["F"])


class SceneFlowSolver:
    """One solver context for frames of a fixed size on the current device
    and stream."""

    def __init__(self, width: int, height: int, stream=None, **params):
        import torch
        self.width, self.height = int(width), int(height)
        self.params = sf.sf_params_default(**params)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.ctx = sf.sf_create(self.width, self.height, self.params,
                                int(stream.cuda_stream))

    def solve(self, images, calib, out=None, with_flows=True):
        """images: (4, H, W) float32 CUDA tensor ordered left t, right t,
        left t+1, right t+1.  Returns (depth, flow3d, flows)."""
        import torch
        assert images.is_cuda and images.dtype == torch.float32
        assert tuple(images.shape) == (4, self.height, self.width)
        images = images.contiguous()
        H, W = self.height, self.width
        if out is None:
            dev = images.device
            out = (torch.empty((H, W), device=dev, dtype=torch.float32),
                   torch.empty((3, H, W), device=dev, dtype=torch.float32),
                   torch.empty((6, H, W), device=dev, dtype=torch.float32)
                   if with_flows else None)
        depth, flow3d, flows = out
        cal = calib if isinstance(calib, sf.sf_calib) else calib_from_dict(calib)
        sf.sf_solve(self.ctx, images[0].data_ptr(), images[1].data_ptr(),
                    images[2].data_ptr(), images[3].data_ptr(), cal, None,
                    depth.data_ptr(), flow3d.data_ptr(),
                    flows.data_ptr() if flows is not None else 0)
        return depth, flow3d, flows

    def solve_batch(self, frames, outs=None, params=None, with_flows=True):
        """frames: list of (images (4, H_i, W_i) float32 CUDA tensor, calib)
        of any sizes (up to 64).  Solves them together in one batch of the
        context (see sf_solve_batch); returns a list of (depth, flow3d,
        flows) tensors."""
        import torch
        if outs is None:
            outs = []
            for img, _ in frames:
                _, H, W = img.shape
                dev = img.device
                outs.append((torch.empty((H, W), device=dev),
                             torch.empty((3, H, W), device=dev),
                             torch.empty((6, H, W), device=dev) if with_flows else None))
        recs = []
        for (img, cal), (depth, flow3d, flows) in zip(frames, outs):
            assert img.is_cuda and img.dtype == torch.float32 and img.is_contiguous()
            _, H, W = img.shape
            c = cal if isinstance(cal, sf.sf_calib) else calib_from_dict(cal)
            recs.append(sf.make_frame([img[k].data_ptr() for k in range(4)], W, H, c,
                                      depth.data_ptr(), flow3d.data_ptr(),
                                      flows.data_ptr() if flows is not None else 0))
        sf.sf_solve_batch(self.ctx, recs, params)
        self._batch_frames = recs  # keep the records alive with the call
        return outs

    def batch_log(self, frame):
        return sf.sf_get_batch_log(self.ctx, frame)[0]

    def batch_init_result(self, frame):
        """(used, e_pred, e_zero) of a batch frame solved with init_mode 1
        (used = -1: too few levels for the network, started from zero)."""
        return sf.sf_get_batch_init_result(self.ctx, frame)

    def log(self):
        return sf.sf_get_log(self.ctx)[0]

    def reset_sequence(self):
        """Video mode: the next solve starts a new sequence (from zero)."""
        sf.sf_reset_sequence(self.ctx)

    def close(self):
        if self.ctx is not None:
            sf.sf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
