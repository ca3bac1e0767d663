"""FP64 oracle of the learned coarse-level initialiser.

TEST INFRASTRUCTURE ONLY.  Like the rest of `oracle/`, this module exists to
check the GPU path: only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import it.  It shares no code with the HIP
library.

The paper (Sec. 7) names a smarter initialisation of the coarse level as
future work; the initialiser here is a small fully convolutional network
that predicts the coarsest-level flows from the 1/16-resolution images, and
a fallback that keeps the zero initialisation whenever the prediction does
not lower the coarsest-level energy of Eq. (8).  What it computes:

* network: six 3x3 convolutions, zero padding, 4 -> 32 -> 32 -> 32 -> 32 ->
  32 -> 6 channels, ReLU after the first five; input = the four level-4
  images (left t, right t, left t+1, right t+1) minus 0.5; output = per
  pixel (s_x, s_y, m_x, m_y, d_x, d_y) in level-4 pixels;
* training: L1 loss against the solver's level-0 flows restricted to level 4
  (box average over 16 x 16 pixels, divided by 16), backpropagation, and
  Adam (Kingma and Ba, 2015, Algorithm 1);
* use: the prediction is sampled bilinearly (clamp-to-edge) at the warp
  nodes of the coarsest level and converted to that level's pixels; the
  fallback compares E at the predicted and at the zero initialisation with
  a common visibility mask (all four positions inside the image under both
  candidates), no colour pruning, and zero deltas, and keeps the lower
  (ties keep zero).
"""
from __future__ import annotations

import numpy as np

from . import halfway as HW

CHANNELS = (4, 32, 32, 32, 32, 32, 6)
INPUT_LEVEL = 4


def param_shapes():
    """(weight, bias) shapes per layer; weights are (c_out, c_in, 3, 3)."""
    return [((co, ci, 3, 3), (co,)) for ci, co in zip(CHANNELS[:-1], CHANNELS[1:])]


N_PARAMS = sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes())


def unpack(flat):
    """Flat parameter vector -> [(W, b), ...]; layer by layer, each weight
    tensor row-major (c_out, c_in, ky, kx) followed by its bias."""
    flat = np.asarray(flat, np.float64)
    assert flat.size == N_PARAMS
    out, k = [], 0
    for ws, bs in param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((flat[k:k + nw].reshape(ws), flat[k + nw:k + nw + nb].copy()))
        k += nw + nb
    return out


def pack(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def init_params(seed):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; the last layer
    scaled by 0.1 so an untrained network predicts small flows."""
    rng = np.random.default_rng(seed)
    params = []
    n = len(CHANNELS) - 1
    for l, (ws, bs) in enumerate(param_shapes()):
        std = np.sqrt(2.0 / (ws[1] * 9))
        if l == n - 1:
            std *= 0.1
        params.append((rng.normal(0.0, std, ws), np.zeros(bs)))
    return pack(params)


def conv3x3(x, W, b):
    """Cross-correlation with zero padding 1: x (B, Ci, H, W) -> (B, Co, H, W)."""
    B, Ci, H, Wd = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.broadcast_to(b[None, :, None, None], (B, W.shape[0], H, Wd)).copy()
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("bchw,oc->bohw", xp[:, :, ky:ky + H, kx:kx + Wd], W[:, :, ky, kx])
    return out


def conv3x3_backward(x, W, d):
    """Gradients of a 3x3 convolution (zero padding 1) w.r.t. its weights,
    bias and input, given its input x and the gradient d w.r.t. its
    output."""
    B, Ci, H, Wd = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for ky in range(3):
        for kx in range(3):
            dW[:, :, ky, kx] = np.einsum("bohw,bchw->oc", d, xp[:, :, ky:ky + H, kx:kx + Wd])
            dxp[:, :, ky:ky + H, kx:kx + Wd] += np.einsum("bohw,oc->bchw", d, W[:, :, ky, kx])
    return dW, d.sum(axis=(0, 2, 3)), dxp[:, :, 1:-1, 1:-1]


def forward(flat, x, bf16=False):
    """Network output (B, 6, H, W) and the per-layer inputs needed by the
    backward pass.  bf16=True gives the arithmetic the network is meant to
    run in on the matrix cores: weights, input and hidden activations
    rounded to bfloat16, biases rounded to float32, exact sums (the
    accumulation precision is the only remaining difference)."""
    params = unpack(flat)
    h = np.asarray(x, np.float64)
    if bf16:
        params = [(bf16_round(W), np.asarray(b, np.float32).astype(np.float64))
                  for W, b in params]
        h = bf16_round(h)
    acts = [h]
    for l, (W, b) in enumerate(params):
        h = conv3x3(h, W, b)
        if l < len(params) - 1:
            h = np.maximum(h, 0.0)
            if bf16:
                h = bf16_round(h)
        acts.append(h)
    return h, acts


def backward(flat, acts, dout, bf16=False):
    """Gradient of a loss w.r.t. the flat parameters given dLoss/dout.
    bf16=True: bfloat16 weights and gradients w.r.t. the hidden
    pre-activations rounded to bfloat16 (dout is taken as given)."""
    params = unpack(flat)
    if bf16:
        params = [(bf16_round(W), b) for W, b in params]
    grads = [None] * len(params)
    d = np.asarray(dout, np.float64)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        dW, db, dx = conv3x3_backward(acts[l], W, d)
        grads[l] = (dW, db)
        if l > 0:
            d = dx * (acts[l] > 0.0)          # through the ReLU of layer l - 1
            if bf16:
                d = bf16_round(d)
    return pack(grads)


def hidden_gradients(flat, acts, dout, bf16=False):
    """Gradients w.r.t. the pre-activations of the hidden layers 0..4, in
    the order of the backward pass's use (for checking its stages)."""
    params = unpack(flat)
    if bf16:
        params = [(bf16_round(W), b) for W, b in params]
    out = [None] * (len(params) - 1)
    d = np.asarray(dout, np.float64)
    for l in range(len(params) - 1, 0, -1):
        _, _, dx = conv3x3_backward(acts[l], params[l][0], d)
        d = dx * (acts[l] > 0.0)
        if bf16:
            d = bf16_round(d)
        out[l - 1] = d
    return out


def l1_loss(out, target, bf16=False):
    """Mean absolute error and its gradient (sign(out - target) / count,
    zero where they are equal); bf16=True rounds the gradient to bfloat16
    with 1 / count taken in float32."""
    r = np.asarray(out, np.float64) - np.asarray(target, np.float64)
    if bf16:
        inv = bf16_round(np.float32(1.0) / np.float32(r.size))
        return float(np.abs(r).mean()), np.sign(r) * inv
    return float(np.abs(r).mean()), np.sign(r) / r.size


def adam_step(flat, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1), t counted from 1.
    Returns new (flat, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    Operates on the float32 value of `a`."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def network_input(level_images):
    """(4, H, W) level-4 intensities -> network input (1, 4, H, W)."""
    return (np.asarray(level_images, np.float64) - 0.5)[None]


def restrict_flows(flows0, level=INPUT_LEVEL):
    """Level-0 per-pixel flows (6, H, W) -> level `level` flows in that
    level's pixels: average over each 2^l x 2^l block (the pyramid's
    repeated 2 x 2 box, floor sizes) divided by 2^l."""
    f = np.asarray(flows0, np.float64)
    k = 1 << level
    H, W = f.shape[1] >> level, f.shape[2] >> level
    blocks = f[:, :H * k, :W * k].reshape(6, H, k, W, k)
    return blocks.mean(axis=(2, 4)) / k


def sample_at_nodes(pred, grid, level_c, level_in=INPUT_LEVEL):
    """Network prediction (6, H_in, W_in) in level-`level_in` pixels ->
    node flows (6, G) of the coarsest level `level_c` in its pixels: node
    position p (level-l_c pixels) maps to 2^(l_c - l_in) (p + 1/2) - 1/2
    (pixel-centre convention), clamp-to-edge bilinear sampling, and the
    flows scale by 2^(l_in - l_c)."""
    pred = np.asarray(pred, np.float64)
    Hi, Wi = pred.shape[1:]
    r = 2.0 ** (level_c - level_in)
    nx, ny = grid.node_xy()
    u = np.clip(r * (nx + 0.5) - 0.5, 0.0, Wi - 1.0)
    v = np.clip(r * (ny + 0.5) - 0.5, 0.0, Hi - 1.0)
    x0 = np.minimum(np.floor(u), max(Wi - 2, 0)).astype(np.int64)
    y0 = np.minimum(np.floor(v), max(Hi - 2, 0)).astype(np.int64)
    x1 = np.minimum(x0 + 1, Wi - 1)
    y1 = np.minimum(y0 + 1, Hi - 1)
    fx, fy = u - x0, v - y0
    out = ((1 - fy) * ((1 - fx) * pred[:, y0, x0] + fx * pred[:, y0, x1])
           + fy * ((1 - fx) * pred[:, y1, x0] + fx * pred[:, y1, x1]))
    return out / r


def fallback_energies(li, grid, F_l, p, base_a, base_b):
    """E of Eq. (8) at zero deltas for two candidate initialisations of the
    coarsest level, with the same visibility mask for both (all four
    positions inside the image under both candidates) and no colour
    pruning; the smoothness and magnitude terms vanish at zero deltas."""
    H, W = li.shape
    px, py = grid.pixel_xy()
    V = np.ones(grid.N, bool)
    for base in (base_a, base_b):
        P = HW.positions(px, py, grid.to_pixels(base))
        for c in range(4):
            V &= (P[c, 0] >= 0) & (P[c, 0] <= W - 1) & (P[c, 1] >= 0) & (P[c, 1] <= H - 1)
    out = []
    for base in (base_a, base_b):
        t = HW.pixel_terms(li, grid, grid.to_pixels(base))
        e_photo, e_grad = HW.pixel_energy(t, V.astype(np.float64), p)
        r_epi, _ = HW.epi_residuals(grid, np.asarray(base, np.float64).reshape(6, -1), F_l)
        out.append(p.w_photo * float(e_photo.sum()) + p.w_grad * float(e_grad.sum())
                   + p.w_reg * p.w_epi * float(np.sum(r_epi ** 2)))
    return out[0], out[1]


def choose_init(li, grid, F_l, p, base_cnn):
    """The fallback: the predicted initialisation if its energy is strictly
    lower than the zero initialisation's, else zero.  Returns (base,
    used_prediction, E_pred, E_zero)."""
    zero = np.zeros_like(np.asarray(base_cnn, np.float64))
    e_cnn, e_zero = fallback_energies(li, grid, F_l, p, base_cnn, zero)
    use = e_cnn < e_zero
    return (np.asarray(base_cnn, np.float64) if use else zero), bool(use), e_cnn, e_zero


def predict_coarsest(flat, images, p, bf16=False):
    """Whole inference path on a frame (4, H, W): pyramid, network on level
    4, sampling at the coarsest level's nodes.  Needs p.levels >= 5."""
    assert p.levels > INPUT_LEVEL
    pyr = HW.pyramid(np.asarray(images, np.float64), p.levels)
    out, _ = forward(flat, network_input(pyr[INPUT_LEVEL]), bf16=bf16)
    lc = p.levels - 1
    H, W = pyr[lc].shape[1:]
    grid = HW.Grid(W, H, p.grid_stride)
    return sample_at_nodes(out[0], grid, lc), out[0]


def solve_learned(flat, images, calib, p, record=None, bf16=False):
    """The solve of Algorithm 1 started from the learned initialisation with
    the fallback: predict, choose against zero at the coarsest level, then
    the usual hierarchy.  Returns (oracle solve result, used_prediction,
    E_pred, E_zero)."""
    if isinstance(calib, dict):
        calib = HW.Calib.from_dict(calib)
    cand, _ = predict_coarsest(flat, images, p, bf16=bf16)
    lc = p.levels - 1
    pyr = HW.pyramid(np.asarray(images, np.float64), p.levels)
    li = HW.LevelImages.build(pyr[lc])
    H, W = li.shape
    grid = HW.Grid(W, H, p.grid_stride)
    base, used, e_cnn, e_zero = choose_init(li, grid, HW.level_calib_F(calib.F, lc), p, cand)
    res = HW.solve(images, calib, p, init_coarsest=base, record=record)
    return res, used, e_cnn, e_zero
