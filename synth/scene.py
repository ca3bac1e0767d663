"""Seeded synthetic stereo-quadruple generator.

Renders the four grayscale images of a rectified binocular rig at two time
steps (left/right camera at t and t+1), the input the halfway-domain method
consumes (two synchronized, pre-calibrated monochrome stereo pairs, Sec. 3
and Sec. 3.1 of the paper).  The paper evaluates on webcam footage and on
public datasets that are not available here; these scenes stand in for them
with the image sizes and displacement magnitudes of the workloads measured.

This module holds scene geometry and rendering only: no part of the
scene-flow energy or its solver.  Both the CPU oracle and the GPU path take
their inputs from here.

Camera model: left camera at the origin, right camera at (B, 0, 0), shared
pinhole intrinsics (f, cx, cy), so a point X projects to
    x_c = f (X_x - c B) / X_z + cx,   y_c = f X_y / X_z + cy,   c in {0, 1}.
The surface is parameterised by (u, v), the left-camera pixel of the point at
time t.  Motion carries the surface point X_0(u, v) to X_1 = X_0 + M(u, v).
Rendering is inverse mapping: for every pixel of camera c at time t solve
pi_c(X_t(u, v)) = p for (u, v) by Newton's method and look up the texture at
(u, v).  All arithmetic is float64; images are returned as float32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# image order used everywhere: (left t, right t, left t+1, right t+1)
IMAGE_NAMES = ("L0", "R0", "L1", "R1")
_CAM = (0, 1, 0, 1)
_TIME = (0, 0, 1, 1)


@dataclass
class SceneConfig:
    width: int
    height: int
    kind: str = "gauss"          # "plane" or "gauss"
    focal: float | None = None   # default 0.8 * width
    baseline: float = 0.1
    # plane scene
    plane_depth: float = 2.0
    plane_motion: tuple = (0.01, 0.0, 0.02)
    # gaussian scene
    depth_range: tuple = (1.5, 4.0)
    n_depth_gauss: int = 8
    max_disp: float = 30.0       # max left-camera image displacement (px)
    n_blobs: int = 0             # independently moving non-rigid blobs
    noise_sigma: float = 0.0
    noise_octaves: int = 4
    noise_period: float = 64.0
    # right-camera response: I_R = gain I + bias + ramp (x / W - 1/2)
    right_gain: float = 1.0
    right_bias: float = 0.0
    right_ramp: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def f(self) -> float:
        return float(self.focal) if self.focal is not None else 0.8 * self.width

    @property
    def cx(self) -> float:
        return (self.width - 1) / 2.0

    @property
    def cy(self) -> float:
        return (self.height - 1) / 2.0


def tiny_plane_config() -> SceneConfig:
    """64x48 fronto-parallel textured plane at 2 m translating (0.01, 0, 0.02) m,
    focal 60 px, baseline 0.1 m, uniform per-texel texture, no noise."""
    return SceneConfig(width=64, height=48, kind="plane", focal=60.0,
                       baseline=0.1, plane_depth=2.0,
                       plane_motion=(0.01, 0.0, 0.02), noise_sigma=0.0)


def vga_config() -> SceneConfig:
    """640x480 smooth Gaussian depth in [1.5, 4] m, 4-octave value noise,
    smooth 3D motion of up to 30 px image displacement, noise sigma 0.01."""
    return SceneConfig(width=640, height=480, kind="gauss", max_disp=30.0,
                       noise_sigma=0.01)


def hd_config() -> SceneConfig:
    """1280x720, same generator with up to 80 px displacement and two
    independently moving non-rigid blobs."""
    return SceneConfig(width=1280, height=720, kind="gauss", max_disp=80.0,
                       n_blobs=2, noise_sigma=0.01)


def sized_config(width: int, height: int, max_disp: float | None = None,
                 noise_sigma: float = 0.01, n_blobs: int = 0) -> SceneConfig:
    """The Gaussian-depth generator at another resolution; displacement
    scales with width (30 px at 640) unless given."""
    if max_disp is None:
        max_disp = 30.0 * width / 640.0
    return SceneConfig(width=width, height=height, kind="gauss",
                       max_disp=max_disp, noise_sigma=noise_sigma,
                       n_blobs=n_blobs)


# --------------------------------------------------------------------------
# smooth fields
# --------------------------------------------------------------------------

class _Gaussians:
    """Sum of isotropic 2D Gaussians with analytic gradient.  `amp` is (K,)
    for a scalar field or (K, D) for a D-vector field (leading axis D)."""

    def __init__(self, mu, sigma, amp):
        self.mu = np.asarray(mu, np.float64)        # (K, 2)
        self.sigma = np.asarray(sigma, np.float64)  # (K,)
        self.amp = np.asarray(amp, np.float64)      # (K,) or (K, D)

    def __call__(self, u, v):
        u = np.asarray(u, np.float64)
        v = np.asarray(v, np.float64)
        shape = np.broadcast(u, v).shape
        lead = () if self.amp.ndim == 1 else (self.amp.shape[1],)
        val = np.zeros(lead + shape)
        du = np.zeros(lead + shape)
        dv = np.zeros(lead + shape)
        for k in range(len(self.sigma)):
            ex = u - self.mu[k, 0]
            ey = v - self.mu[k, 1]
            s2 = self.sigma[k] ** 2
            g = np.exp(-(ex * ex + ey * ey) / (2.0 * s2))
            a = self.amp[k].reshape(lead + (1,) * len(shape)) \
                if lead else self.amp[k]
            val += a * g
            du += a * (g * (-ex / s2))
            dv += a * (g * (-ey / s2))
        return val, du, dv


class _ValueNoise:
    """Multi-octave value noise on an integer lattice with smoothstep
    interpolation; lattice values uniform in [0, 1].  Output in [0, 1]."""

    def __init__(self, rng, lo, hi, period, octaves, persistence=0.5):
        self.levels = []
        amp = 1.0
        total = 0.0
        for o in range(octaves):
            p = period / (2 ** o)
            nx = int(math.ceil((hi[0] - lo[0]) / p)) + 3
            ny = int(math.ceil((hi[1] - lo[1]) / p)) + 3
            lat = rng.random((ny, nx))
            self.levels.append((p, amp, lat))
            total += amp
            amp *= persistence
        self.lo = (float(lo[0]) - 0.0, float(lo[1]) - 0.0)
        self.total = total

    def __call__(self, u, v):
        out = np.zeros(np.broadcast(u, v).shape)
        for p, amp, lat in self.levels:
            gx = (u - self.lo[0]) / p + 1.0
            gy = (v - self.lo[1]) / p + 1.0
            ix = np.floor(gx).astype(np.int64)
            iy = np.floor(gy).astype(np.int64)
            ix = np.clip(ix, 0, lat.shape[1] - 2)
            iy = np.clip(iy, 0, lat.shape[0] - 2)
            tx = np.clip(gx - ix, 0.0, 1.0)
            ty = np.clip(gy - iy, 0.0, 1.0)
            sx = tx * tx * (3 - 2 * tx)
            sy = ty * ty * (3 - 2 * ty)
            a = lat[iy, ix] * (1 - sx) + lat[iy, ix + 1] * sx
            b = lat[iy + 1, ix] * (1 - sx) + lat[iy + 1, ix + 1] * sx
            out += amp * (a * (1 - sy) + b * sy)
        return out / self.total


class _TexelTexture:
    """Per-texel uniform [0, 1] texture on the integer (u, v) lattice with
    bilinear lookup (texel pitch = one left-camera pixel at time t)."""

    def __init__(self, rng, lo, hi):
        self.x0 = int(math.floor(lo[0])) - 2
        self.y0 = int(math.floor(lo[1])) - 2
        nx = int(math.ceil(hi[0])) - self.x0 + 4
        ny = int(math.ceil(hi[1])) - self.y0 + 4
        self.lat = rng.random((ny, nx))

    def __call__(self, u, v):
        gx = u - self.x0
        gy = v - self.y0
        ix = np.clip(np.floor(gx).astype(np.int64), 0, self.lat.shape[1] - 2)
        iy = np.clip(np.floor(gy).astype(np.int64), 0, self.lat.shape[0] - 2)
        tx = gx - ix
        ty = gy - iy
        L = self.lat
        a = L[iy, ix] * (1 - tx) + L[iy, ix + 1] * tx
        b = L[iy + 1, ix] * (1 - tx) + L[iy + 1, ix + 1] * tx
        return a * (1 - ty) + b * ty


# --------------------------------------------------------------------------
# scene
# --------------------------------------------------------------------------

class Scene:
    """A seeded scene: depth Z0(u, v), motion M(u, v), texture T(u, v)."""

    def __init__(self, cfg: SceneConfig, seed: int):
        self.cfg = cfg
        self.seed = int(seed)
        rng = np.random.default_rng(self.seed)
        W, H = cfg.width, cfg.height
        f, cx, cy = cfg.f, cfg.cx, cfg.cy
        self.f, self.cx, self.cy, self.B = f, cx, cy, cfg.baseline
        margin = 0.25 * max(W, H) + 4.0 * cfg.max_disp + 16
        lo = (-margin, -margin)
        hi = (W + margin, H + margin)
        if cfg.kind == "plane":
            self._plane = True
            self.texture = _TexelTexture(rng, lo, hi)
            self.T = np.asarray(cfg.plane_motion, np.float64)
            self.Z0 = float(cfg.plane_depth)
        elif cfg.kind == "gauss":
            self._plane = False
            K = cfg.n_depth_gauss
            mu = np.stack([rng.uniform(0, W, K), rng.uniform(0, H, K)], 1)
            sig = rng.uniform(W / 8.0, W / 4.0, K)
            amp = rng.uniform(-1.0, 1.0, K)
            self.depth_g = _Gaussians(mu, sig, amp)
            # rescale the sum to [zmin, zmax] over the image domain
            uu, vv = np.meshgrid(np.linspace(0, W - 1, 97),
                                 np.linspace(0, H - 1, 73))
            s, _, _ = self.depth_g(uu, vv)
            self.dlo, self.dhi = float(s.min()), float(s.max())
            self.zmin, self.zmax = cfg.depth_range
            self.texture = _ValueNoise(rng, lo, hi, cfg.noise_period,
                                       cfg.noise_octaves)
            # motion: global translation + 4 RBFs (+ blobs), 3D amplitudes
            Km = 4
            mmu = np.stack([rng.uniform(0, W, Km), rng.uniform(0, H, Km)], 1)
            msig = rng.uniform(W / 5.0, W / 2.5, Km)
            mamp = rng.normal(0.0, 1.0, (Km, 3)) * np.array([1.0, 1.0, 2.0])
            glob = rng.normal(0.0, 1.0, 3) * np.array([1.0, 1.0, 2.0])
            mus = [mmu]
            sigs = [msig]
            amps = [mamp]
            for b in range(cfg.n_blobs):
                bmu = np.array([[rng.uniform(0.2 * W, 0.8 * W),
                                 rng.uniform(0.2 * H, 0.8 * H)]])
                bsig = np.array([rng.uniform(W / 8.0, W / 5.0)])
                bamp = rng.normal(0.0, 1.0, (1, 3)) * np.array([2.0, 2.0, 3.0])
                mus.append(bmu)
                sigs.append(bsig)
                amps.append(bamp)
            self.motion_g = _Gaussians(np.concatenate(mus), np.concatenate(sigs),
                                       np.concatenate(amps))
            self.motion_glob = glob
            self.motion_scale = 1.0
            self._calibrate_motion()
        else:
            raise ValueError(cfg.kind)
        self.noise_rng = np.random.default_rng(self.seed + 7919)

    # ---- surface ---------------------------------------------------------
    def depth(self, u, v):
        """Z0(u, v) and its (u, v) derivatives."""
        if self._plane:
            z = np.full(np.broadcast(u, v).shape, self.Z0)
            return z, np.zeros_like(z), np.zeros_like(z)
        s, du, dv = self.depth_g(u, v)
        k = (self.zmax - self.zmin) / (self.dhi - self.dlo)
        return self.zmin + (s - self.dlo) * k, du * k, dv * k

    def motion(self, u, v):
        """M(u, v) (3, ...) and derivatives."""
        shape = np.broadcast(u, v).shape
        if self._plane:
            m = np.broadcast_to(self.T.reshape((3,) + (1,) * len(shape)),
                                (3,) + shape).copy()
            return m, np.zeros_like(m), np.zeros_like(m)
        val, du, dv = self.motion_g(u, v)
        sc = self.motion_scale
        g = self.motion_glob.reshape((3,) + (1,) * len(shape))
        return (val + g) * sc * 0.05, du * sc * 0.05, dv * sc * 0.05

    def point(self, u, v, t):
        """Surface point X_t(u, v) (3, ...) and its (u, v) derivatives."""
        f, cx, cy = self.f, self.cx, self.cy
        z, zu, zv = self.depth(u, v)
        X = np.stack([(u - cx) * z / f, (v - cy) * z / f, z])
        Xu = np.stack([(z + (u - cx) * zu) / f, (v - cy) * zu / f, zu])
        Xv = np.stack([(u - cx) * zv / f, (z + (v - cy) * zv) / f, zv])
        if t:
            # constant velocity: X_t = X_0 + t M
            m, mu, mv = self.motion(u, v)
            X = X + t * m
            Xu = Xu + t * mu
            Xv = Xv + t * mv
        return X, Xu, Xv

    def project(self, X, cam):
        f, cx, cy, B = self.f, self.cx, self.cy, self.B
        x = f * (X[0] - cam * B) / X[2] + cx
        y = f * X[1] / X[2] + cy
        return x, y

    def _proj_jac(self, X, Xu, Xv, cam):
        f, B = self.f, self.B
        Xx = X[0] - cam * B
        iz = 1.0 / X[2]
        # d(x)/d(u) = f (Xu_x z - Xx Xu_z) / z^2
        xu = f * (Xu[0] * X[2] - Xx * Xu[2]) * iz * iz
        xv = f * (Xv[0] * X[2] - Xx * Xv[2]) * iz * iz
        yu = f * (Xu[1] * X[2] - X[1] * Xu[2]) * iz * iz
        yv = f * (Xv[1] * X[2] - X[1] * Xv[2]) * iz * iz
        return xu, xv, yu, yv

    def _calibrate_motion(self):
        W, H = self.cfg.width, self.cfg.height
        uu, vv = np.meshgrid(np.linspace(0, W - 1, 81), np.linspace(0, H - 1, 61))
        for _ in range(4):
            X0, _, _ = self.point(uu, vv, 0)
            X1, _, _ = self.point(uu, vv, 1)
            x0, y0 = self.project(X0, 0)
            x1, y1 = self.project(X1, 0)
            dmax = float(np.sqrt((x1 - x0) ** 2 + (y1 - y0) ** 2).max())
            self.motion_scale *= self.cfg.max_disp / max(dmax, 1e-9)

    # ---- inverse mapping -------------------------------------------------
    def surface_coords(self, cam, t, px, py, iters=30):
        """(u, v) with pi_cam(X_t(u, v)) = (px, py), by Newton's method."""
        if self._plane:
            f, cx, cy, B = self.f, self.cx, self.cy, self.B
            zt = self.Z0 + t * self.T[2]
            X = (px - cx) * zt / f + cam * B
            Y = (py - cy) * zt / f
            if t:
                X = X - t * self.T[0]
                Y = Y - t * self.T[1]
            return f * X / self.Z0 + cx, f * Y / self.Z0 + cy
        u = np.array(px, np.float64, copy=True)
        v = np.array(py, np.float64, copy=True)
        if cam == 1:  # start from the mean disparity
            u = u + self.f * self.B / (0.5 * (self.zmin + self.zmax))
        for _ in range(iters):
            X, Xu, Xv = self.point(u, v, t)
            x, y = self.project(X, cam)
            xu, xv, yu, yv = self._proj_jac(X, Xu, Xv, cam)
            rx = x - px
            ry = y - py
            det = xu * yv - xv * yu
            du = (yv * rx - xv * ry) / det
            dv = (-yu * rx + xu * ry) / det
            # damp very large steps
            step = np.sqrt(du * du + dv * dv)
            sc = np.minimum(1.0, 20.0 / np.maximum(step, 1e-300))
            u = u - du * sc
            v = v - dv * sc
            if float(np.max(np.abs(rx)) + np.max(np.abs(ry))) < 1e-10:
                break
        return u, v

    def render(self, noise=True, t0=0):
        """(4, H, W) float32 images in the order L0, R0, L1, R1, taken at
        times t0 and t0 + 1 of the constant-velocity motion."""
        W, H = self.cfg.width, self.cfg.height
        py, px = np.mgrid[0:H, 0:W].astype(np.float64)
        out = np.empty((4, H, W), np.float32)
        for k in range(4):
            u, v = self.surface_coords(_CAM[k], _TIME[k] + t0, px, py)
            img = self.texture(u, v)
            if _CAM[k] == 1:
                c = self.cfg
                img = c.right_gain * img + c.right_bias + c.right_ramp * (px / W - 0.5)
            if noise and self.cfg.noise_sigma > 0:
                img = img + self.noise_rng.normal(0.0, self.cfg.noise_sigma,
                                                  img.shape)
            out[k] = img.astype(np.float32)
        return out

    # ---- ground truth ----------------------------------------------------
    def projections(self, u, v, t0=0):
        """The four image positions (x, y) of surface point (u, v):
        order L0, R0, L1, R1 (times t0, t0, t0 + 1, t0 + 1)."""
        out = []
        for k in range(4):
            X, _, _ = self.point(u, v, _TIME[k] + t0)
            out.append(self.project(X, _CAM[k]))
        return out

    def halfway_truth(self, width=None, height=None, scale=1.0, iters=40, t0=0):
        """Ground-truth correspondences of every halfway-domain pixel x: the
        surface point whose four projections average to x.  Returns
        (P, ok) with P of shape (4, 2, H, W) (positions in L0, R0, L1, R1,
        in pixels of a grid `scale` times finer than the input) and ok the
        mask of pixels where the Newton solve converged."""
        W = width or self.cfg.width
        H = height or self.cfg.height
        py, px = np.mgrid[0:H, 0:W].astype(np.float64)
        # target in full-resolution pixels (pixel-centre convention)
        tx = (px + 0.5) / scale - 0.5
        ty = (py + 0.5) / scale - 0.5
        u = tx.copy()
        v = ty.copy()
        h = 1e-4
        for _ in range(iters):
            P = self.projections(u, v, t0)
            mx = sum(p[0] for p in P) / 4.0 - tx
            my = sum(p[1] for p in P) / 4.0 - ty
            Pu = self.projections(u + h, v, t0)
            Pv = self.projections(u, v + h, t0)
            a = (sum(p[0] for p in Pu) / 4.0 - tx - mx) / h
            b = (sum(p[0] for p in Pv) / 4.0 - tx - mx) / h
            c = (sum(p[1] for p in Pu) / 4.0 - ty - my) / h
            d = (sum(p[1] for p in Pv) / 4.0 - ty - my) / h
            det = a * d - b * c
            u = u - (d * mx - b * my) / det
            v = v - (-c * mx + a * my) / det
            if float(np.max(np.abs(mx)) + np.max(np.abs(my))) < 1e-9:
                break
        P = self.projections(u, v, t0)
        res = np.abs(sum(p[0] for p in P) / 4.0 - tx) + \
            np.abs(sum(p[1] for p in P) / 4.0 - ty)
        pos = np.empty((4, 2, H, W))
        for k in range(4):
            pos[k, 0] = (P[k][0] + 0.5) * scale - 0.5
            pos[k, 1] = (P[k][1] + 0.5) * scale - 0.5
        return pos, res < 1e-6


def halfway_flows_from_positions(pos):
    """Inverts the four-position relations of the halfway domain for a set of
    correspondences: given positions P_L0, P_R0, P_L1, P_R1 (shape (4, 2, ...))
    return s, m, d (each (2, ...)).  Used only to state ground truth."""
    L0, R0, L1, R1 = pos
    s = ((R0 + R1) - (L0 + L1)) / 4.0
    m = ((L1 + R1) - (L0 + R0)) / 4.0
    d = ((L0 + R1) - (R0 + L1)) / 4.0
    return s, m, d


def rectified_F():
    """Fundamental matrix of the rectified rig with x_L^T F x_R = 0,
    normalised so that the epipolar residual is r_y - l_y in pixels."""
    return np.array([[0.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]])


def calib_of(scene: Scene) -> dict:
    return dict(fx=scene.f, fy=scene.f, cx=scene.cx, cy=scene.cy,
                baseline=scene.B, F=rectified_F())


def make_frame(cfg: SceneConfig, seed: int, noise=True):
    """Render one quadruple: returns (images (4, H, W) float32, calib dict,
    scene)."""
    sc = Scene(cfg, seed)
    return sc.render(noise=noise), calib_of(sc), sc


def make_sequence(cfg: SceneConfig, seed: int, n_frames: int, noise=True):
    """A constant-velocity video of one scene: n_frames quadruples, frame
    k taken at times k and k + 1.  Returns (list of images, calib, scene)."""
    sc = Scene(cfg, seed)
    return [sc.render(noise=noise, t0=k) for k in range(n_frames)], calib_of(sc), sc


def batch_resolutions(n: int, seed: int):
    """Per-frame resolutions drawn uniformly from the four batched sizes."""
    choices = [(320, 240), (640, 480), (960, 540), (1280, 720)]
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, 4, n)
    return [choices[i] for i in idx]
