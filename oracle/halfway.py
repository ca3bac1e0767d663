"""FP64 CPU oracle of the halfway-domain scene-flow solve.

TEST INFRASTRUCTURE ONLY.  This module exists to check the GPU path: only the
test suite, the smoke entry point and the benchmark's CPU-baseline leg may
import it.  It shares no code with the HIP library and imports nothing from
it.

What it computes (paper: "Real-time Halfway Domain Reconstruction of Motion
and Geometry", Thies et al., 3DV 2016):

* Sec. 3.1/3.2, Eqs. (1)-(6): a halfway-domain pixel x maps into the four
  images through stereo flow s, motion flow m and difference flow d; six
  brightness-consistency differences d_0..d_5 compare the four images.
* Sec. 3.3, Eq. (7): per-pixel flows are bilinear blends of warp-grid nodes.
* Sec. 4, Eqs. (8)-(18): E = w_photo E_photo + w_grad E_grad
  + w_reg (w_smooth E_smooth + w_epi E_epi + w_mag E_mag), with the
  pseudo-Huber penalty of Eq. (12), visibility V and colour pruning W.
* Sec. 5.1, Eqs. (19)-(24): Gauss-Newton on the least-squares form, with the
  normal equations solved by Jacobi-preconditioned conjugate gradients.
* Sec. 5.3: coarse-to-fine hierarchy in which each level solves only for a
  delta on top of the bilinearly upsampled coarser result.

Everything is float64, vectorised over pixels with numpy; the Gauss-Newton
system matrix is assembled explicitly as a scipy CSR matrix (the GPU path is
matrix-free).  Readings of points the paper leaves open are marked
"reading:" where they are applied.

Parity pins: every function here is pinned by a test in tests/test_oracle_*.py
against closed forms, library routines, finite differences or invariants.
The structure-tensor smoothness weight w_i (`node_weights`) is the one
reading of a formula the paper does not print (it names only the
ingredients: eigenvalues of a 3x3-window autocorrelation matrix, high for
featureless regions); its ingredients are pinned (the warp, the gradient
convention, the window and its centre, the smaller eigenvalue against
numpy.linalg.eigvalsh and a hand-derived quadratic-image tensor, the 4^l
scaling of tau_l), while the choice of the map w = 1 + gamma exp(-l / tau)
itself has no external truth.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np
import scipy.sparse as sp

# ---------------------------------------------------------------------------
# constants of the halfway-domain geometry (Sec. 3.1, Eqs. (1)-(6), (16)-(17))
# ---------------------------------------------------------------------------

#: camera order L0 (left, t), R0 (right, t), L1 (left, t+1), R1 (right, t+1)
CAMERAS = ("L0", "R0", "L1", "R1")

#: sign of (s, m, d) in the position of each camera's sample:
#: P_L0 = x - s - m + d, P_R0 = x + s - m - d,
#: P_L1 = x - s + m - d, P_R1 = x + s + m + d   (Eqs. (1)-(6), (16)-(17))
SIGNS = np.array([[-1.0, -1.0, +1.0],
                  [+1.0, -1.0, -1.0],
                  [-1.0, +1.0, -1.0],
                  [+1.0, +1.0, +1.0]])

#: d_k = I_a(P_a) - I_b(P_b) for the six consistency checks, Eqs. (1)-(6):
#: stereo (R0,L0), (R1,L1); motion (L1,L0), (R1,R0); cross (R1,L0), (L1,R0)
PAIRS = ((1, 0), (3, 2), (2, 0), (3, 1), (3, 0), (2, 1))

#: flow components in unknown order (the 6 planes of one node)
COMPONENTS = ("s_x", "s_y", "m_x", "m_y", "d_x", "d_y")


@dataclass
class Params:
    """Energy weights and solver schedule.  Defaults are the paper's
    parameter table (Appendix A, column "Figures 5, 6, 8"), with
    w_smooth = w_mag = 1 (constant in all experiments), eps = 0.001
    (Sec. 4.1, after Eq. (12)) and eps_p = 0.2 (Sec. 4.1)."""
    levels: int = 3
    grid_stride: int = 8
    gn_iters: int = 5
    gn_fine: int = 0  # if > 0: steps on the two finest levels (Sec. 6.2 schedule)
    pcg_iters: int = 10
    max_backtracks: int = 4
    w_reg: float = 0.5
    w_photo: float = 0.5
    w_grad: float = 5.0
    w_epi: float = 0.5
    w_smooth: float = 1.0
    w_mag: float = 1.0
    w_s: float = 0.75
    w_m: float = 0.5
    w_d: float = 0.01
    m_s: float = 0.5
    m_m: float = 10.0
    m_d: float = 100.0
    eps: float = 0.001
    eps_p: float = 0.2
    st_gamma: float = 4.0
    st_tau: float = 1e-3
    illum: bool = False  # illumination correction (Sec. 5.3)
    occlusion: bool = False  # occlusion maps from a z-buffer (Sec. 5.3)

    def gn_at(self, level):
        """Gauss-Newton steps at a level.  The paper's real-time runs use
        2 steps on the two finest levels and 5 on the others (Sec. 6.2);
        gn_fine > 0 selects such a split, else every level takes gn_iters."""
        return self.gn_fine if (self.gn_fine > 0 and level < 2) else self.gn_iters

    def flow_weights(self):
        """w_f per unknown component (s_x, s_y, m_x, m_y, d_x, d_y)."""
        return np.array([self.w_s, self.w_s, self.w_m, self.w_m,
                         self.w_d, self.w_d])

    def mag_weights(self):
        """m_f per unknown component."""
        return np.array([self.m_s, self.m_s, self.m_m, self.m_m,
                         self.m_d, self.m_d])


@dataclass
class Calib:
    """Rectified pinhole pair: focal lengths and principal point in pixels,
    baseline in metres, fundamental matrix F with x_L^T F x_R = 0."""
    fx: float
    fy: float
    cx: float
    cy: float
    baseline: float
    F: np.ndarray = field(default_factory=lambda: np.array(
        [[0.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]]))

    @staticmethod
    def from_dict(d):
        return Calib(float(d["fx"]), float(d["fy"]), float(d["cx"]),
                     float(d["cy"]), float(d["baseline"]),
                     np.asarray(d["F"], np.float64).reshape(3, 3))


# ---------------------------------------------------------------------------
# image pyramid (Sec. 5.3 "downsampling factor of 2"; Sec. 7 "mip-map")
# ---------------------------------------------------------------------------

def downsample(img):
    """One mip-map step: 2x2 box average, odd last row/column dropped
    (reading: floor sizes)."""
    H, W = img.shape[-2] // 2, img.shape[-1] // 2
    a = img[..., 0:2 * H:2, 0:2 * W:2]
    b = img[..., 0:2 * H:2, 1:2 * W:2]
    c = img[..., 1:2 * H:2, 0:2 * W:2]
    d = img[..., 1:2 * H:2, 1:2 * W:2]
    return 0.25 * (a + b + c + d)


def pyramid(images, levels):
    """List of `levels` arrays (4, H_l, W_l); level 0 is the input."""
    out = [np.asarray(images, np.float64)]
    for _ in range(1, levels):
        out.append(downsample(out[-1]))
    return out


def image_gradients(img):
    """Gradient images (d/dx, d/dy) of one image: central differences inside,
    one-sided at the borders (reading: the numpy.gradient convention).
    Written out rather than calling numpy.gradient, which pins it."""
    gx = np.empty_like(img)
    gy = np.empty_like(img)
    gx[:, 1:-1] = 0.5 * (img[:, 2:] - img[:, :-2])
    gx[:, 0] = img[:, 1] - img[:, 0]
    gx[:, -1] = img[:, -1] - img[:, -2]
    gy[1:-1, :] = 0.5 * (img[2:, :] - img[:-2, :])
    gy[0, :] = img[1, :] - img[0, :]
    gy[-1, :] = img[-1, :] - img[-2, :]
    return gx, gy


@dataclass
class LevelImages:
    """The four images of one level with their gradient images, and the
    illumination correction of the level (per halfway-domain pixel,
    subtracted from both right-camera samples; None = no correction)."""
    I: np.ndarray   # (4, H, W)
    Gx: np.ndarray  # (4, H, W)
    Gy: np.ndarray  # (4, H, W)
    illum: np.ndarray | None = None  # (H * W,)

    @staticmethod
    def build(imgs4, illum=None):
        imgs4 = np.asarray(imgs4, np.float64)
        gx = np.empty_like(imgs4)
        gy = np.empty_like(imgs4)
        for c in range(4):
            gx[c], gy[c] = image_gradients(imgs4[c])
        return LevelImages(imgs4, gx, gy,
                           None if illum is None else np.asarray(illum, np.float64).reshape(-1))

    @property
    def shape(self):
        return self.I.shape[1:]


# ---------------------------------------------------------------------------
# bilinear sampling (the warps of Eqs. (1)-(6))
# ---------------------------------------------------------------------------

def sample(img, px, py):
    """Bilinear sample of `img` at (px, py) with clamp-to-edge coordinates.
    Returns the value and the exact derivatives of the bilinear interpolant
    with respect to px and py (zero where the coordinate was clamped).
    Pixel (i, j) is at integer coordinates (x = j, y = i)."""
    H, W = img.shape
    inx = (px >= 0.0) & (px <= W - 1.0)
    iny = (py >= 0.0) & (py <= H - 1.0)
    cx = np.clip(px, 0.0, W - 1.0)
    cy = np.clip(py, 0.0, H - 1.0)
    x0 = np.minimum(np.floor(cx), W - 2).astype(np.int64)
    y0 = np.minimum(np.floor(cy), H - 2).astype(np.int64)
    fx = cx - x0
    fy = cy - y0
    v00 = img[y0, x0]
    v01 = img[y0, x0 + 1]
    v10 = img[y0 + 1, x0]
    v11 = img[y0 + 1, x0 + 1]
    val = (1 - fy) * ((1 - fx) * v00 + fx * v01) + fy * ((1 - fx) * v10 + fx * v11)
    ddx = ((1 - fy) * (v01 - v00) + fy * (v11 - v10)) * inx
    ddy = ((1 - fx) * (v10 - v00) + fx * (v11 - v01)) * iny
    return val, ddx, ddy


# ---------------------------------------------------------------------------
# warp grid (Sec. 3.3, Eq. (7))
# ---------------------------------------------------------------------------

def _interp_1d(n_px, n_nodes, s):
    """Per pixel: the two bracketing nodes and their linear weights.
    reading: nodes sit at cell centres (i + 1/2) s - 1/2, so pixel x has
    node coordinate u = (x + 1/2)/s - 1/2, clamped to the node range."""
    x = np.arange(n_px, dtype=np.float64)
    u = np.clip((x + 0.5) / s - 0.5, 0.0, n_nodes - 1.0)
    if n_nodes == 1:
        i0 = np.zeros(n_px, np.int64)
        return i0, i0.copy(), np.ones(n_px), np.zeros(n_px)
    i0 = np.minimum(np.floor(u), n_nodes - 2).astype(np.int64)
    f = u - i0
    return i0, i0 + 1, 1.0 - f, f


@dataclass
class Grid:
    """Warp grid of one level: W x H pixels, stride s, Gx x Gy nodes.
    reading: Gx = ceil(W/s), Gy = ceil(H/s), node (i, j) at pixel
    ((i + 1/2) s - 1/2, (j + 1/2) s - 1/2), clamp-to-edge weights."""
    W: int
    H: int
    s: int

    def __post_init__(self):
        self.Gx = -(-self.W // self.s)
        self.Gy = -(-self.H // self.s)
        self.G = self.Gx * self.Gy
        ix0, ix1, wx0, wx1 = _interp_1d(self.W, self.Gx, self.s)
        iy0, iy1, wy0, wy1 = _interp_1d(self.H, self.Gy, self.s)
        # the four nodes of every pixel (row-major pixels) and weights alpha
        IX0, IY0 = np.meshgrid(ix0, iy0)
        IX1, IY1 = np.meshgrid(ix1, iy1)
        WX0, WY0 = np.meshgrid(wx0, wy0)
        WX1, WY1 = np.meshgrid(wx1, wy1)
        self.nodes = np.stack([IY0 * self.Gx + IX0, IY0 * self.Gx + IX1,
                               IY1 * self.Gx + IX0, IY1 * self.Gx + IX1]
                              ).reshape(4, -1)
        self.alpha = np.stack([WY0 * WX0, WY0 * WX1, WY1 * WX0, WY1 * WX1]
                              ).reshape(4, -1)
        self.N = self.W * self.H

    def node_xy(self):
        """Reference pixel position g^x of every node, (2, G)."""
        j, i = np.mgrid[0:self.Gy, 0:self.Gx].astype(np.float64)
        return np.stack([(i + 0.5) * self.s - 0.5,
                         (j + 0.5) * self.s - 0.5]).reshape(2, -1)

    def pixel_xy(self):
        y, x = np.mgrid[0:self.H, 0:self.W].astype(np.float64)
        return x.reshape(-1), y.reshape(-1)

    def to_pixels(self, nodes6):
        """Eq. (7): per-pixel flows (6, N) from node values (6, G)."""
        nodes6 = np.asarray(nodes6, np.float64).reshape(6, self.G)
        out = np.zeros((6, self.N))
        for k in range(4):
            out += self.alpha[k] * nodes6[:, self.nodes[k]]
        return out

    def interp_matrix(self):
        """Sparse N x G matrix of the weights alpha_{x,k} (Eq. (7))."""
        rows = np.tile(np.arange(self.N), 4)
        return sp.csr_matrix((self.alpha.reshape(-1),
                              (rows, self.nodes.reshape(-1))),
                             shape=(self.N, self.G))


def level_calib_F(F, level):
    """Fundamental matrix in level-l pixel coordinates.
    reading: level-l pixel p_l maps to level-0 pixel 2^l p_l + (2^l - 1)/2
    (pixel-centre convention); F_l = A^T F A / 2^l keeps the residual in
    level-l pixel units."""
    k = 2.0 ** level
    A = np.array([[k, 0.0, (k - 1.0) / 2.0], [0.0, k, (k - 1.0) / 2.0],
                  [0.0, 0.0, 1.0]])
    return A.T @ np.asarray(F, np.float64) @ A / k


# ---------------------------------------------------------------------------
# per-pixel residuals (Eqs. (1)-(6), (11)-(13))
# ---------------------------------------------------------------------------

def phi(x, eps):
    """Pseudo-Huber penalty, Eq. (12)."""
    return np.sqrt(x * x + eps * eps)


def positions(px, py, flows):
    """The four sample positions of each pixel, (4, 2, N): P_c = x +
    SIGNS[c] . (s, m, d), Eqs. (1)-(6)."""
    s = flows[0:2]
    m = flows[2:4]
    d = flows[4:6]
    out = np.empty((4, 2, px.shape[0]))
    base = np.stack([px, py])
    for c in range(4):
        out[c] = base + SIGNS[c, 0] * s + SIGNS[c, 1] * m + SIGNS[c, 2] * d
    return out


@dataclass
class PixelTerms:
    d: np.ndarray        # (6, N)   brightness differences d_k
    g: np.ndarray        # (6, 2, N) gradient differences g_k
    Jd: np.ndarray       # (6, 6, N) d d_k / d flow_q
    Jg: np.ndarray       # (6, 2, 6, N) d g_k[r] / d flow_q
    P: np.ndarray        # (4, 2, N) positions


def pixel_terms(li: LevelImages, grid: Grid, flows):
    """Residuals of Eqs. (1)-(6) and of the gradient-constancy term with
    their derivatives with respect to the six per-pixel flow components.
    reading: the gradient residual of pair k is
    g_k = grad I_a(P_a) - grad I_b(P_b), with grad I the gradient images
    sampled bilinearly (gradient constancy)."""
    px, py = grid.pixel_xy()
    return pixel_terms_xy(li, px, py, flows)


def pixel_terms_xy(li: LevelImages, px, py, flows):
    """pixel_terms for the pixels at integer coordinates (px, py) with
    their flows (6, n)."""
    P = positions(px, py, flows)
    val = np.empty((4, px.shape[0]))
    dI = np.empty((4, 2, px.shape[0]))     # d I_c / d P
    gv = np.empty((4, 2, px.shape[0]))     # (Gx, Gy)(P_c)
    dG = np.empty((4, 2, 2, px.shape[0]))  # d G_r / d P_j
    for c in range(4):
        val[c], dI[c, 0], dI[c, 1] = sample(li.I[c], P[c, 0], P[c, 1])
        gv[c, 0], dG[c, 0, 0], dG[c, 0, 1] = sample(li.Gx[c], P[c, 0], P[c, 1])
        gv[c, 1], dG[c, 1, 0], dG[c, 1, 1] = sample(li.Gy[c], P[c, 0], P[c, 1])
    if li.illum is not None:
        # normalised right-camera intensities (the correction does not
        # depend on the flows; gradients are unaffected by an offset)
        corr = li.illum[(np.asarray(py, np.int64) * li.shape[1] + np.asarray(px, np.int64))]
        val[1] -= corr
        val[3] -= corr
    N = px.shape[0]
    d = np.empty((6, N))
    g = np.empty((6, 2, N))
    Jd = np.zeros((6, 6, N))
    Jg = np.zeros((6, 2, 6, N))
    for k, (a, b) in enumerate(PAIRS):
        d[k] = val[a] - val[b]
        g[k] = gv[a] - gv[b]
        for f in range(3):          # s, m, d
            for j in range(2):      # x, y
                q = 2 * f + j
                Jd[k, q] = SIGNS[a, f] * dI[a, j] - SIGNS[b, f] * dI[b, j]
                for r in range(2):
                    Jg[k, r, q] = SIGNS[a, f] * dG[a, r, j] - SIGNS[b, f] * dG[b, r, j]
    return PixelTerms(d, g, Jd, Jg, P)


def pixel_energy(terms: PixelTerms, cmask, p: Params):
    """Per-pixel photometric and gradient energies, Eqs. (11) and (13).
    reading: the gradient penalty is Phi(||g_k||) = sqrt(||g_k||^2 + eps^2),
    robust like the photometric one.  cmask = V(x) W(x)."""
    e_photo = cmask * phi(terms.d, p.eps).sum(0)
    gn = np.sqrt((terms.g ** 2).sum(1))
    e_grad = cmask * phi(gn, p.eps).sum(0)
    return e_photo, e_grad


# ---------------------------------------------------------------------------
# regulariser residuals (Eqs. (14), (15)-(17), (18)), on node values
# ---------------------------------------------------------------------------

def _neighbour_pairs(grid: Grid):
    """Ordered pairs (i, j) with j in the 4-neighbourhood of i (reading:
    N_i = 4-neighbourhood; each undirected edge appears twice as written)."""
    idx = np.arange(grid.G).reshape(grid.Gy, grid.Gx)
    pairs = [
        (idx[:, :-1], idx[:, 1:]),   # right neighbour
        (idx[:, 1:], idx[:, :-1]),   # left neighbour
        (idx[:-1, :], idx[1:, :]),   # lower neighbour
        (idx[1:, :], idx[:-1, :]),   # upper neighbour
    ]
    return np.concatenate([np.stack([a.reshape(-1), b.reshape(-1)])
                           for a, b in pairs], 1)


def smooth_residuals(grid: Grid, delta, wnode, p: Params):
    """E_smooth, Eq. (14), as squared residuals on the delta unknowns:
    r = sqrt(w_i w_f) (g_i^f - g_j^f) per ordered neighbour pair and component.
    Returns (r, J) with J sparse over the 6G unknowns (component-major)."""
    pr = _neighbour_pairs(grid)
    i, j = pr
    wf = p.flow_weights()
    G = grid.G
    rs = []
    rows = []
    cols = []
    vals = []
    n = i.shape[0]
    for q in range(6):
        sw = np.sqrt(wnode[i] * wf[q])
        rs.append(sw * (delta[q, i] - delta[q, j]))
        base = q * n
        rows += [base + np.arange(n), base + np.arange(n)]
        cols += [q * G + i, q * G + j]
        vals += [sw, -sw]
    J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows),
                       np.concatenate(cols))), shape=(6 * n, 6 * G))
    return np.concatenate(rs), J


def epi_residuals(grid: Grid, total, F_l):
    """E_epi, Eqs. (15)-(17), on the total node flows: for t = 0, 1,
    r_t = l_t^T F r_t with homogeneous node positions
    l^0 = g - s - m + d, r^0 = g + s - m - d, l^1 = g - s + m - d,
    r^1 = g + s + m + d.  Returns (r (2G,), J sparse (2G, 6G))."""
    G = grid.G
    gx = grid.node_xy()
    s, m, d = total[0:2], total[2:4], total[4:6]
    rs = []
    rows = []
    cols = []
    vals = []
    for t, (cl, cr) in enumerate(((0, 1), (2, 3))):
        L = gx + SIGNS[cl, 0] * s + SIGNS[cl, 1] * m + SIGNS[cl, 2] * d
        R = gx + SIGNS[cr, 0] * s + SIGNS[cr, 1] * m + SIGNS[cr, 2] * d
        Lh = np.vstack([L, np.ones(G)])
        Rh = np.vstack([R, np.ones(G)])
        FR = F_l @ Rh          # d r / d L (first two rows)
        FtL = F_l.T @ Lh       # d r / d R
        rs.append((Lh * FR).sum(0))
        for f in range(3):
            for j in range(2):
                q = 2 * f + j
                rows.append(t * G + np.arange(G))
                cols.append(q * G + np.arange(G))
                vals.append(SIGNS[cl, f] * FR[j] + SIGNS[cr, f] * FtL[j])
    J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows),
                       np.concatenate(cols))), shape=(2 * G, 6 * G))
    return np.concatenate(rs), J


def mag_residuals(grid: Grid, delta, p: Params):
    """E_mag, Eq. (18), on the delta unknowns: r = sqrt(m_f) g_i^f."""
    G = grid.G
    mf = np.repeat(np.sqrt(p.mag_weights()), G)
    r = mf * delta.reshape(-1)
    J = sp.diags(mf).tocsr()
    return r, J


def reg_terms(grid: Grid, delta, total, wnode, F_l, p: Params):
    """Stacked regulariser residuals with weights folded in so that
    w_reg (w_smooth E_smooth + w_epi E_epi + w_mag E_mag) = ||r||^2.
    reading: smoothness and magnitude act on the per-level delta unknowns,
    the epipolar term on the total flows (it measures geometry)."""
    rs, Js = smooth_residuals(grid, delta, wnode, p)
    re, Je = epi_residuals(grid, total, F_l)
    rm, Jm = mag_residuals(grid, delta, p)
    a = math.sqrt(p.w_reg * p.w_smooth)
    b = math.sqrt(p.w_reg * p.w_epi)
    c = math.sqrt(p.w_reg * p.w_mag)
    r = np.concatenate([a * rs, b * re, c * rm])
    J = sp.vstack([a * Js, b * Je, c * Jm]).tocsr()
    parts = dict(smooth=float(rs @ rs), epi=float(re @ re), mag=float(rm @ rm))
    return r, J, parts


# ---------------------------------------------------------------------------
# the level problem
# ---------------------------------------------------------------------------

@dataclass
class LevelState:
    """Everything frozen while one level is solved."""
    level: int
    li: LevelImages
    grid: Grid
    base: np.ndarray      # (6, G) prolongated total of the coarser level
    cmask: np.ndarray     # (N,)  V(x) W(x), frozen for the level
    wnode: np.ndarray     # (G,)  smoothness weights w_i
    F_l: np.ndarray       # (3, 3)


def energy(ls: LevelState, delta, p: Params):
    """E of Eq. (8) at delta (total = base + delta) and its five raw terms
    (E_photo, E_grad, E_smooth, E_epi, E_mag, unweighted)."""
    total = ls.base + delta
    flows = ls.grid.to_pixels(total)
    terms = pixel_terms(ls.li, ls.grid, flows)
    ep, eg = pixel_energy(terms, ls.cmask, p)
    _, _, parts = reg_terms(ls.grid, delta, total, ls.wnode, ls.F_l, p)
    out = dict(photo=float(ep.sum()), grad=float(eg.sum()), **parts)
    out["total"] = (p.w_photo * out["photo"] + p.w_grad * out["grad"]
                    + p.w_reg * (p.w_smooth * out["smooth"]
                                 + p.w_epi * out["epi"]
                                 + p.w_mag * out["mag"]))
    return out


def robust_rows(ls: LevelState, delta, p: Params):
    """The alignment part in least-squares form (Sec. 5, Eq. (19)).
    reading: the robust terms enter as iteratively reweighted least squares:
    each residual r of a penalty c Phi(.) gets weight omega = c / Phi at the
    linearisation point, so that E has gradient sum omega r dr and the
    Gauss-Newton matrix sum omega dr dr^T.  Returns per pixel the 18 rows
    (6 photometric, 6x2 gradient) as J (N, 18, 6) in flow space, residuals
    r (N, 18) and weights omega (N, 18)."""
    total = ls.base + delta
    flows = ls.grid.to_pixels(total)
    t = pixel_terms(ls.li, ls.grid, flows)
    N = flows.shape[1]
    ph = phi(t.d, p.eps)                                  # (6, N)
    gph = phi(np.sqrt((t.g ** 2).sum(1)), p.eps)          # (6, N)
    J = np.empty((N, 18, 6))
    r = np.empty((N, 18))
    w = np.empty((N, 18))
    J[:, 0:6, :] = np.transpose(t.Jd, (2, 0, 1))
    r[:, 0:6] = t.d.T
    w[:, 0:6] = (ls.cmask * p.w_photo / ph).T
    for k in range(6):
        for rr in range(2):
            row = 6 + 2 * k + rr
            J[:, row, :] = t.Jg[k, rr].T
            r[:, row] = t.g[k, rr]
            w[:, row] = ls.cmask * p.w_grad / gph[k]
    return J, r, w


# ---------------------------------------------------------------------------
# the same quantities on a sample of pixels or nodes (full-size checks)
# ---------------------------------------------------------------------------

def flows_at(grid: Grid, nodes6, pix):
    """Eq. (7) flows (6, n) of the pixels with flat indices pix."""
    nodes6 = np.asarray(nodes6, np.float64).reshape(6, grid.G)
    out = np.zeros((6, len(pix)))
    for k in range(4):
        out += grid.alpha[k][pix] * nodes6[:, grid.nodes[k][pix]]
    return out


def rows_at(ls: LevelState, delta, p: Params, pix):
    """robust_rows evaluated for the pixels pix only: J (n, 18, 6), r, w."""
    grid = ls.grid
    pix = np.asarray(pix, np.int64)
    fl = flows_at(grid, ls.base + delta, pix)
    px = (pix % grid.W).astype(np.float64)
    py = (pix // grid.W).astype(np.float64)
    t = pixel_terms_xy(ls.li, px, py, fl)
    n = len(pix)
    cm = ls.cmask[pix]
    ph = phi(t.d, p.eps)
    gph = phi(np.sqrt((t.g ** 2).sum(1)), p.eps)
    J = np.empty((n, 18, 6))
    r = np.empty((n, 18))
    w = np.empty((n, 18))
    J[:, 0:6, :] = np.transpose(t.Jd, (2, 0, 1))
    r[:, 0:6] = t.d.T
    w[:, 0:6] = (cm * p.w_photo / ph).T
    for k in range(6):
        for rr in range(2):
            row = 6 + 2 * k + rr
            J[:, row, :] = t.Jg[k, rr].T
            r[:, row] = t.g[k, rr]
            w[:, row] = cm * p.w_grad / gph[k]
    return J, r, w


def node_rows(ls: LevelState, delta, p: Params, nodes, u):
    """For the nodes listed: the gradient of E (6, n), diag(H) (6, n) and
    (H u) (6, n) for a vector u (6, G), from the pixels in each node's
    support and the regularisers (the rows of linearize's grad and H)."""
    grid = ls.grid
    nodes = np.asarray(nodes, np.int64)
    u = np.asarray(u, np.float64).reshape(6, grid.G)
    total = ls.base + delta
    rr, Jr, _ = reg_terms(grid, delta, total, ls.wnode, ls.F_l, p)
    g_reg = (2.0 * (Jr.T @ rr)).reshape(6, grid.G)
    JtJ = (Jr.T @ Jr).tocsr()
    Hu_reg = (2.0 * (JtJ @ u.reshape(-1))).reshape(6, grid.G)
    d_reg = (2.0 * JtJ.diagonal()).reshape(6, grid.G)
    grad = np.zeros((6, len(nodes)))
    diag = np.zeros((6, len(nodes)))
    Hu = np.zeros((6, len(nodes)))
    for t_, n in enumerate(nodes):
        sup = np.nonzero((grid.nodes == n).any(0) & (
            np.where(grid.nodes == n, grid.alpha, 0.0).sum(0) != 0.0))[0]
        a_n = np.where(grid.nodes[:, sup] == n, grid.alpha[:, sup], 0.0).sum(0)
        J, r, w = rows_at(ls, delta, p, sup)
        gpx = np.einsum("nri,nr->ni", J, w * r)
        Gx = np.einsum("nri,nr,nrj->nij", J, w, J)
        v = flows_at(grid, u, sup)                         # interpolated u
        grad[:, t_] = (a_n[:, None] * gpx).sum(0) + g_reg[:, n]
        diag[:, t_] = (a_n[:, None] ** 2 * np.einsum("nii->ni", Gx)).sum(0) + d_reg[:, n]
        Hu[:, t_] = (a_n[:, None] * np.einsum("nij,jn->ni", Gx, v)).sum(0) + Hu_reg[:, n]
    return grad, diag, Hu


def linearize(ls: LevelState, delta, p: Params):
    """Gradient of E and the Gauss-Newton matrix H at delta (Eqs. (21)-(24)):
    H = sum_x A_x^T (J_x^T Omega_x J_x) A_x + 2 J_reg^T J_reg and
    grad = sum_x A_x^T J_x^T Omega_x r_x + 2 J_reg^T r_reg, where A_x holds
    the bilinear weights of Eq. (7) (chain rule: node unknowns enter the
    pixel flows linearly).  H is assembled explicitly in CSR over the 6G
    unknowns (component-major: unknown q*G + node)."""
    grid = ls.grid
    G = grid.G
    J, r, w = robust_rows(ls, delta, p)
    gpx = np.einsum("nri,nr->ni", J, w * r)               # (N, 6)
    Gx = np.einsum("nri,nr,nrj->nij", J, w, J)            # (N, 6, 6)
    grad = np.zeros((6, G))
    for k in range(4):
        for q in range(6):
            grad[q] += np.bincount(grid.nodes[k], grid.alpha[k] * gpx[:, q],
                                   minlength=G)
    H = sp.csr_matrix((6 * G, 6 * G))
    qi, qj = np.meshgrid(np.arange(6), np.arange(6), indexing="ij")
    for a in range(4):
        for b in range(4):
            wab = grid.alpha[a] * grid.alpha[b]
            vals = (wab[:, None, None] * Gx).reshape(-1)
            rows = (qi[None] * G + grid.nodes[a][:, None, None]).reshape(-1)
            cols = (qj[None] * G + grid.nodes[b][:, None, None]).reshape(-1)
            H = H + sp.csr_matrix((vals, (rows, cols)), shape=(6 * G, 6 * G))
    total = ls.base + delta
    rr, Jr, _ = reg_terms(grid, delta, total, ls.wnode, ls.F_l, p)
    grad = grad.reshape(-1) + 2.0 * (Jr.T @ rr)
    H = (H + 2.0 * (Jr.T @ Jr)).tocsr()
    return grad, H


def pcg(H, b, iters, log=None):
    """Jacobi-preconditioned conjugate gradients on H x = b, x0 = 0, exactly
    `iters` iterations (Sec. 5.1, after Eq. (24): the normal equations are
    solved by PCG).  reading: preconditioner M = diag(H); once p.q <= 1e-30
    ||p||^2 or r.z <= 1e-30 the remaining iterations change nothing
    (alpha = 0).  Appends ||r|| after every iteration to `log` if given."""
    M = H.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    z = r / M
    pvec = z.copy()
    rz = float(r @ z)
    active = rz > 1e-30
    for _ in range(iters):
        if active:
            q = H @ pvec
            pq = float(pvec @ q)
            pp = float(pvec @ pvec)
            active = pq > 1e-30 * pp
        if active:
            alpha = rz / pq
            x = x + alpha * pvec
            r = r - alpha * q
            z = r / M
            rz_new = float(r @ z)
            if rz_new > 1e-30:
                beta = rz_new / rz
                pvec = z + beta * pvec
                rz = rz_new
            else:
                active = False
        if log is not None:
            log.append(float(np.sqrt(r @ r)))
    return x


TAUS = (1.0, 0.5, 0.25, 0.125, 0.0625)


def gn_step(ls: LevelState, delta, p: Params, record=None):
    """One Gauss-Newton step with step control.
    reading (the paper has no step control): try delta + tau dx for
    tau = 1, 1/2, 1/4, 1/8, 1/16 (max_backtracks + 1 values) and accept the
    first with E_trial <= E; otherwise keep delta (tau = 0)."""
    e0 = energy(ls, delta, p)
    grad, H = linearize(ls, delta, p)
    res = []
    dx = pcg(H, -grad, p.pcg_iters, res).reshape(6, -1)
    tau = 0.0
    e_new = e0
    for t in TAUS[:p.max_backtracks + 1]:
        et = energy(ls, delta + t * dx, p)
        if et["total"] <= e0["total"]:
            tau = t
            e_new = et
            break
    if record is not None:
        record.append(dict(level=ls.level, energy=e0["total"], terms=e0,
                           tau=tau, energy_after=e_new["total"],
                           pcg_res=res))
    return delta + tau * dx


# ---------------------------------------------------------------------------
# level set-up: visibility, pruning and smoothness weights
# ---------------------------------------------------------------------------

def masks(li: LevelImages, grid: Grid, total, p: Params, occ=None):
    """V(x) and W(x) of Eq. (11) at the level-start flow.
    reading: V(x) = 1 iff all four positions lie inside the level image
    (occlusion maps are not built); W(x) = 1 iff max_k |d_k(x)| < eps_p.
    Both are frozen for the whole level."""
    flows = grid.to_pixels(total)
    px, py = grid.pixel_xy()
    P = positions(px, py, flows)
    H, W = li.shape
    V = np.ones(grid.N, bool)
    for c in range(4):
        V &= (P[c, 0] >= 0) & (P[c, 0] <= W - 1) & (P[c, 1] >= 0) & (P[c, 1] <= H - 1)
    if occ is not None:
        V &= np.asarray(occ, bool).reshape(-1)
    t = pixel_terms(li, grid, flows)
    Wm = np.abs(t.d).max(0) < p.eps_p
    return V, Wm


def node_weights(li: LevelImages, grid: Grid, total, level, p: Params):
    """Smoothness weight w_i of Eq. (14) (Sec. 4.3): structure-tensor
    analysis of a 3x3 pixel window at each node.
    reading (the paper does not print the formula; see the module notes
    for what pins it):
    I_bar = mean of the four images warped to the halfway domain by the
    level-start flow; A_i = sum over the 3x3 window around the node's
    rounded position of grad I_bar grad I_bar^T, with the gradient-image
    convention of `image_gradients`; the rounded position is clamped into
    the image (the last node row or column can lie beyond it) and window
    rows or columns beyond the border repeat the border; lambda_min = the
    smaller eigenvalue; w_i = 1 + gamma exp(-lambda_min / tau_l) with
    tau_l = st_tau 4^l (squared gradients grow fourfold per coarser level
    at equal structure).  High for featureless regions as required."""
    flows = grid.to_pixels(total)
    px, py = grid.pixel_xy()
    P = positions(px, py, flows)
    ibar = np.zeros(grid.N)
    for c in range(4):
        ibar += sample(li.I[c], P[c, 0], P[c, 1])[0]
    ibar = (0.25 * ibar).reshape(grid.H, grid.W)
    gx, gy = image_gradients(ibar)
    nxy = grid.node_xy()
    cxi = np.clip(np.floor(nxy[0] + 0.5).astype(np.int64), 0, grid.W - 1)
    cyi = np.clip(np.floor(nxy[1] + 0.5).astype(np.int64), 0, grid.H - 1)
    a = np.zeros(grid.G)
    b = np.zeros(grid.G)
    c = np.zeros(grid.G)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            yy = np.clip(cyi + dy, 0, grid.H - 1)
            xx = np.clip(cxi + dx, 0, grid.W - 1)
            u = gx[yy, xx]
            v = gy[yy, xx]
            a += u * u
            b += u * v
            c += v * v
    lmin = 0.5 * (a + c) - np.sqrt((0.5 * (a - c)) ** 2 + b * b)
    tau = p.st_tau * 4.0 ** level
    return 1.0 + p.st_gamma * np.exp(-np.maximum(lmin, 0.0) / tau)


# ---------------------------------------------------------------------------
# hierarchy (Algorithm 1, Sec. 5.3)
# ---------------------------------------------------------------------------

def prolong(total_c, grid_c: Grid, grid_f: Grid):
    """Prolongation to the next finer level (Sec. 5.3, "upsampling ... based
    on bilinear interpolation"): fine node i sits at coarse node coordinate
    i/2 - 1/4 (from the node placement and the pixel-centre convention),
    clamp-to-edge bilinear, and flows double because pixels halve."""
    def coords(n_f, n_c):
        u = np.clip(np.arange(n_f) / 2.0 - 0.25, 0.0, n_c - 1.0)
        if n_c == 1:
            z = np.zeros(n_f, np.int64)
            return z, z, np.ones(n_f), np.zeros(n_f)
        i0 = np.minimum(np.floor(u), n_c - 2).astype(np.int64)
        f = u - i0
        return i0, i0 + 1, 1 - f, f
    ix0, ix1, wx0, wx1 = coords(grid_f.Gx, grid_c.Gx)
    iy0, iy1, wy0, wy1 = coords(grid_f.Gy, grid_c.Gy)
    tc = np.asarray(total_c).reshape(6, grid_c.Gy, grid_c.Gx)
    out = (wy0[:, None] * (wx0[None] * tc[:, iy0][:, :, ix0]
                           + wx1[None] * tc[:, iy0][:, :, ix1])
           + wy1[:, None] * (wx0[None] * tc[:, iy1][:, :, ix0]
                             + wx1[None] * tc[:, iy1][:, :, ix1]))
    return 2.0 * out.reshape(6, -1)


def setup_level(level, pyr, p: Params, calib: Calib, base, delta0=None, illum=None,
                occ=None):
    """Level set-up at the level-start flow base + delta0 (delta0 = 0
    unless the level starts from a temporal initialisation), with the
    level's illumination correction and occlusion map (None = none)."""
    li = LevelImages.build(pyr[level], illum)
    H, W = li.shape
    grid = Grid(W, H, p.grid_stride)
    start = base if delta0 is None else np.asarray(base, np.float64) + delta0
    V, Wm = masks(li, grid, start, p, occ)
    wnode = node_weights(li, grid, start, level, p)
    return LevelState(level, li, grid, np.asarray(base, np.float64),
                      (V & Wm).astype(np.float64), wnode,
                      level_calib_F(calib.F, level))


def solve(images, calib, p: Params, init_coarsest=None, record=None, init_deltas=None):
    """Algorithm 1 without the occlusion/illumination map updates: for each
    level from coarsest to finest, prolongate the coarser total, start the
    delta at zero (or at init_deltas[level], the temporal initialisation),
    freeze masks and weights, run gn_at(level) Gauss-Newton steps.  Returns a
    dict with the finest-level grid, total node flows (6, G) and the
    per-level totals, deltas and grids."""
    if isinstance(calib, dict):
        calib = Calib.from_dict(calib)
    pyr = pyramid(images, p.levels)
    totals, deltas, grids = {}, {}, {}
    total = None
    grid_prev = None
    for level in range(p.levels - 1, -1, -1):
        H, W = pyr[level].shape[1:]
        grid = Grid(W, H, p.grid_stride)
        if total is None:
            base = (np.zeros((6, grid.G)) if init_coarsest is None
                    else np.asarray(init_coarsest, np.float64).reshape(6, -1))
        else:
            base = prolong(total, grid_prev, grid)
        delta = (np.zeros((6, grid.G)) if init_deltas is None
                 else np.asarray(init_deltas[level], np.float64).reshape(6, grid.G))
        illum = None
        if p.illum:
            illum = np.zeros(grid.N) if total is None else illum_next
        occ = occ_next if (p.occlusion and total is not None) else None
        ls = setup_level(level, pyr, p, calib, base,
                         None if init_deltas is None else delta, illum, occ)
        for _ in range(p.gn_at(level)):
            delta = gn_step(ls, delta, p, record)
        total = ls.base + delta
        totals[level] = total
        deltas[level] = delta
        grids[level] = grid
        if p.illum and level > 0:
            Hf, Wf = pyr[level - 1].shape[1:]
            illum_next = illumination_map(ls.li, grid, total, Wf, Hf)
        if p.occlusion and level > 0:
            Hf, Wf = pyr[level - 1].shape[1:]
            occ_next = box_upsample(occlusion_map(grid, total), Wf, Hf) > 0.5
        grid_prev = grid
    return dict(grid=grid_prev, total=total, totals=totals, deltas=deltas, grids=grids)


# ---------------------------------------------------------------------------
# illumination correction (Sec. 5.3)
# ---------------------------------------------------------------------------

#: Gaussian of the illumination extraction, in level pixels (Sec. 5.3)
ILLUM_SIGMA = 3.2


def illumination_residual(li: LevelImages, grid: Grid, total):
    """Intensity residual between the two stereo pairs in the halfway
    domain at the level's final flow.
    reading: e(x) = ((I_R0(P_R0) - I_L0(P_L0)) + (I_R1(P_R1) - I_L1(P_L1))) / 2
    on the raw images (the absolute left/right difference, re-estimated on
    every level), 0 where a position lies outside its image (V = 0)."""
    flows = grid.to_pixels(total)
    px, py = grid.pixel_xy()
    P = positions(px, py, flows)
    H, W = li.shape
    V = np.ones(grid.N, bool)
    val = np.empty((4, grid.N))
    for c in range(4):
        V &= (P[c, 0] >= 0) & (P[c, 0] <= W - 1) & (P[c, 1] >= 0) & (P[c, 1] <= H - 1)
        val[c] = sample(li.I[c], P[c, 0], P[c, 1])[0]
    e = 0.5 * ((val[1] - val[0]) + (val[3] - val[2]))
    return np.where(V, e, 0.0).reshape(H, W)


def gaussian_blur(img, sigma=ILLUM_SIGMA):
    """Separable Gaussian, taps k = -R..R with R = ceil(3 sigma), weights
    exp(-k^2 / (2 sigma^2)) normalised to 1, clamp-to-edge borders (rows,
    then columns)."""
    R = int(math.ceil(3.0 * sigma))
    k = np.arange(-R, R + 1)
    w = np.exp(-(k ** 2) / (2.0 * sigma * sigma))
    w /= w.sum()
    img = np.asarray(img, np.float64)
    H, W = img.shape
    xi = np.clip(np.arange(W)[:, None] + k[None, :], 0, W - 1)
    tmp = (img[:, xi] * w).sum(-1)
    yi = np.clip(np.arange(H)[:, None] + k[None, :], 0, H - 1)
    return np.einsum("ykx,k->yx", tmp[yi], w)


def box_upsample(img, Wf, Hf):
    """Box filter to the next finer level: fine pixel (x, y) takes coarse
    pixel (x // 2, y // 2), clamped to the coarse image."""
    img = np.asarray(img, np.float64)
    H, W = img.shape
    yi = np.minimum(np.arange(Hf) // 2, H - 1)
    xi = np.minimum(np.arange(Wf) // 2, W - 1)
    return img[yi][:, xi]


def illumination_map(li: LevelImages, grid: Grid, total, Wf, Hf):
    """The next finer level's correction (Sec. 5.3): the low-frequency part
    of the stereo residual (Gaussian, sigma = 3.2 px), box-upsampled; flat
    (Hf * Wf,).  The coarsest level has none (zero)."""
    return box_upsample(gaussian_blur(illumination_residual(li, grid, total)), Wf, Hf).reshape(-1)


# ---------------------------------------------------------------------------
# occlusion maps (Sec. 5.3)
# ---------------------------------------------------------------------------

#: relative disparity tolerance of the z-buffer test
OCC_TOL = 0.02
#: longest triangle edge (px, in the camera) that is rendered
OCC_EDGE = 2.0


def _halfway_triangles(H, W):
    """Triangulation of the halfway pixel grid: every quad (x, y), (x+1, y),
    (x, y+1), (x+1, y+1) split along its (x+1, y)-(x, y+1) diagonal; (n, 3)
    flat pixel indices."""
    idx = np.arange(H * W).reshape(H, W)
    a = idx[:-1, :-1].ravel()
    b = idx[:-1, 1:].ravel()
    c = idx[1:, :-1].ravel()
    d = idx[1:, 1:].ravel()
    return np.concatenate([np.stack([a, b, c], 1), np.stack([b, d, c], 1)])


def _edge(ax, ay, bx, by, qx, qy):
    """Twice the signed area of (a, b, q): > 0 if q is left of a -> b."""
    return (bx - ax) * (qy - ay) - (by - ay) * (qx - ax)


def _occlusion(grid: Grid, total, margin=0.0, margin_rel=0.0):
    """Visibility from a z-buffer of the triangulated geometry (Sec. 5.3).
    reading: each halfway pixel is a vertex of the mesh that triangulates
    the halfway grid; in camera c a vertex sits at P_c and carries the
    stereo disparity of its time t, D_t = P_Lt.x - P_Rt.x (larger = nearer;
    depth f B / D_t).  A triangle is rendered in camera c unless an edge is
    longer than OCC_EDGE px there (it spans a depth discontinuity), a vertex
    has D_t <= 0, or it has zero area; it covers the integer pixel centres q
    on or inside it and writes its barycentric interpolation of D_t there;
    the z-buffer keeps the largest value per pixel (0 where nothing is
    drawn).  A halfway pixel is visible in c unless its nearest pixel
    centre floor(P_c + 1/2) is in the image, D_t > 0 and D_t < (1 -
    OCC_TOL) times the z-buffer there; visible overall if visible in all
    four views.
    margin > 0 (px; margin_rel relative, for the disparity test) also finds
    the pixels whose result could change if positions moved by less than
    margin: every decision is taken both ways where its deciding quantity is
    within the margin of its threshold (z-buffers of the certain and of the
    possible writes).  Returns (visibility (N,) bool, fragile (N,) bool)."""
    flows = grid.to_pixels(total)
    px, py = grid.pixel_xy()
    P = positions(px, py, flows)
    H, W = grid.H, grid.W
    N = grid.N
    D0 = P[0, 0] - P[1, 0]
    D1 = P[2, 0] - P[3, 0]
    disp = (D0, D0, D1, D1)
    tri = _halfway_triangles(H, W)
    vis = np.ones(N, bool)
    frag = np.zeros(N, bool)
    for cam in range(4):
        X, Y, D = P[cam, 0], P[cam, 1], disp[cam]
        ax, ay, ad = X[tri[:, 0]], Y[tri[:, 0]], D[tri[:, 0]]
        bx, by, bd = X[tri[:, 1]], Y[tri[:, 1]], D[tri[:, 1]]
        cx, cy, cd = X[tri[:, 2]], Y[tri[:, 2]], D[tri[:, 2]]
        lab = np.hypot(bx - ax, by - ay)
        lbc = np.hypot(cx - bx, cy - by)
        lca = np.hypot(ax - cx, ay - cy)
        lmax = np.maximum(np.maximum(lab, lbc), lca)
        dmin = np.minimum(np.minimum(ad, bd), cd)
        area = _edge(ax, ay, bx, by, cx, cy)
        scale = lab + lbc + lca
        keep_lo = (lmax <= OCC_EDGE - margin) & (dmin > margin) & (np.abs(area) > margin * scale)
        keep_hi = (lmax <= OCC_EDGE + margin) & (dmin > -margin) & (np.abs(area) > -margin * scale)
        if margin == 0.0:
            keep_hi = keep_lo
        sg = np.where(area < 0, -1.0, 1.0)
        safe = np.where(area == 0, 1.0, area)
        x0 = np.ceil(np.minimum(np.minimum(ax, bx), cx) - margin).astype(np.int64)
        y0 = np.ceil(np.minimum(np.minimum(ay, by), cy) - margin).astype(np.int64)
        x1 = np.floor(np.maximum(np.maximum(ax, bx), cx) + margin).astype(np.int64)
        y1 = np.floor(np.maximum(np.maximum(ay, by), cy) + margin).astype(np.int64)
        zlo = np.zeros(N)
        zhi = np.zeros(N)
        span = int(np.ceil(OCC_EDGE + 2 * margin)) + 1
        for oy in range(span):
            for ox in range(span):
                qx = x0 + ox
                qy = y0 + oy
                inb = (qx <= x1) & (qy <= y1) & (qx >= 0) & (qx < W) & (qy >= 0) & (qy < H)
                E_bc = _edge(bx, by, cx, cy, qx, qy)
                E_ca = _edge(cx, cy, ax, ay, qx, qy)
                E_ab = _edge(ax, ay, bx, by, qx, qy)
                e_bc, e_ca, e_ab = sg * E_bc, sg * E_ca, sg * E_ab
                ins_lo = (e_bc >= margin * lbc) & (e_ca >= margin * lca) & (e_ab >= margin * lab)
                ins_hi = (e_bc >= -margin * lbc) & (e_ca >= -margin * lca) & (e_ab >= -margin * lab)
                # barycentric interpolation: the weight of a vertex is the
                # area opposite it over the whole area
                z = (E_bc * ad + E_ca * bd + E_ab * cd) / safe
                q = np.where(inb, qy * W + qx, 0)
                w_lo = inb & keep_lo & ins_lo
                w_hi = inb & keep_hi & ins_hi
                np.maximum.at(zlo, q[w_lo], z[w_lo])
                np.maximum.at(zhi, q[w_hi], z[w_hi])
        # the test at the nearest pixel centre, both ways where it is fragile
        fx = X - np.floor(X)
        fy = Y - np.floor(Y)
        res = []
        for rx in (0.0, 1.0):
            for ry in (0.0, 1.0):
                for zb in (zlo, zhi):
                    for dr in (-margin_rel, margin_rel):
                        nx = np.floor(X + 0.5)
                        ny = np.floor(Y + 0.5)
                        if margin > 0:
                            nx = np.where(np.abs(fx - 0.5) < margin, np.floor(X) + rx, nx)
                            ny = np.where(np.abs(fy - 0.5) < margin, np.floor(Y) + ry, ny)
                        qx = nx.astype(np.int64)
                        qy = ny.astype(np.int64)
                        inb = (qx >= 0) & (qx < W) & (qy >= 0) & (qy < H)
                        dd = D + dr * np.abs(D) + (margin if dr > 0 else -margin) * (margin > 0)
                        q = np.where(inb, qy * W + qx, 0)
                        occl = inb & (dd > 0) & (dd < (1.0 - OCC_TOL) * zb[q])
                        res.append(~occl)
        nominal = res[0] if margin == 0.0 else None
        if margin == 0.0:
            vc = nominal
            fc = np.zeros(N, bool)
        else:
            stack = np.stack(res)
            vc = stack.all(0)
            fc = stack.any(0) & ~stack.all(0)
        vis &= vc
        frag |= fc
    return vis, frag


def occlusion_map(grid: Grid, total):
    """Visibility of every halfway pixel in all four views, (H, W) float
    0/1, from a z-buffer of the current geometry (Sec. 5.3; the reading is
    stated in _occlusion)."""
    return _occlusion(grid, total)[0].reshape(grid.H, grid.W).astype(np.float64)


def occlusion_fragile(grid: Grid, total, margin=1e-3, margin_rel=5e-4):
    """Pixels whose visibility could flip if the positions moved by less
    than margin px (or disparities by margin_rel relative): where a float32
    evaluation of the same geometry may legitimately differ; (H, W) bool."""
    return _occlusion(grid, total, margin, margin_rel)[1].reshape(grid.H, grid.W)


# ---------------------------------------------------------------------------
# temporal initialisation (Sec. 5.3)
# ---------------------------------------------------------------------------

def sample_nodes(grid: Grid, field6, x, y):
    """Bilinear sample of a node field (c, G) at level-pixel positions
    (x, y): node (i, j) sits at ((i + 1/2) s - 1/2, (j + 1/2) s - 1/2); the
    node coordinate is clamped to the grid."""
    f = np.asarray(field6, np.float64).reshape(-1, grid.Gy, grid.Gx)

    def axis(pos, G):
        u = np.clip((np.asarray(pos, np.float64) + 0.5) / grid.s - 0.5, 0.0, G - 1.0)
        i0 = np.minimum(np.floor(u), max(G - 2, 0)).astype(np.int64)
        return i0, np.minimum(i0 + 1, G - 1), u - i0

    i0, i1, fx = axis(x, grid.Gx)
    j0, j1, fy = axis(y, grid.Gy)
    return ((1 - fy) * ((1 - fx) * f[:, j0, i0] + fx * f[:, j0, i1]) +
            fy * ((1 - fx) * f[:, j1, i0] + fx * f[:, j1, i1]))


def temporal_init(prev_totals, prev_deltas, grids):
    """Per-level initial deltas of the next frame from the previous one
    (Sec. 5.3: constant velocity, the motion flow propagates the flows, each
    level's delta transferred separately).
    reading: the halfway domain moves by 2 m per frame (the stereo average
    of the positions is x - m at t and x + m at t + 1), so node y of the next
    frame takes the previous delta at y - 2 m(y), with m the motion
    components of the previous frame's level total at node y:
    delta_init(y) = delta_prev(y - 2 m_prev(y)), sampled by sample_nodes."""
    out = {}
    for level, grid in grids.items():
        gx, gy = grid.node_xy()
        m = np.asarray(prev_totals[level], np.float64).reshape(6, -1)[2:4]
        out[level] = sample_nodes(grid, prev_deltas[level], gx - 2.0 * m[0], gy - 2.0 * m[1])
    return out


def solve_sequence(frames, calib, p: Params, record=None):
    """Solves a video frame by frame: the first frame from zero, every
    later one from temporal_init of the previous result.  Returns the list
    of solve results (record, if given, collects one list per frame)."""
    out, prev = [], None
    for images in frames:
        rec = [] if record is not None else None
        init = None if prev is None else temporal_init(prev["totals"], prev["deltas"],
                                                        prev["grids"])
        res = solve(images, calib, p, record=rec, init_deltas=init)
        if record is not None:
            record.append(rec)
        out.append(res)
        prev = res
    return out


# ---------------------------------------------------------------------------
# output: depth and 3D flow (dense geometry and its motion)
# ---------------------------------------------------------------------------

def output(grid: Grid, total, calib: Calib):
    """Per halfway pixel at level 0: disparities disp_t = P_Lt.x - P_Rt.x,
    depth Z_t = f_x B / disp_t (NaN where disp_t <= 0), back-projection
    X_t = ((P_Lt.x - c_x) Z_t / f_x, (P_Lt.y - c_y) Z_t / f_y, Z_t) in the
    left camera; depth = Z_0 and flow3d = X_1 - X_0 (reading of "dense 3D
    geometry and its motion").  Returns depth (H, W), flow3d (3, H, W) and
    the per-pixel flows (6, H, W)."""
    flows = grid.to_pixels(total)
    return output_from_flows(flows, grid.W, grid.H, calib)


def output_from_flows(flows, W, H, calib):
    """`output` for per-pixel flows (6, H*W) (s_x, s_y, m_x, m_y, d_x, d_y
    planes of a W x H level-0 image) instead of node totals."""
    if isinstance(calib, dict):
        calib = Calib.from_dict(calib)
    flows = np.asarray(flows, np.float64).reshape(6, -1)
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    px, py = x.reshape(-1), y.reshape(-1)
    P = positions(px, py, flows)
    Xs = []
    for cl, cr in ((0, 1), (2, 3)):
        disp = P[cl, 0] - P[cr, 0]
        with np.errstate(divide="ignore", invalid="ignore"):
            Z = np.where(disp > 0, calib.fx * calib.baseline / disp, np.nan)
        X = np.stack([(P[cl, 0] - calib.cx) * Z / calib.fx,
                      (P[cl, 1] - calib.cy) * Z / calib.fy, Z])
        Xs.append(X)
    depth = Xs[0][2].reshape(H, W)
    flow3d = (Xs[1] - Xs[0]).reshape(3, H, W)
    return depth, flow3d, flows.reshape(6, H, W)


def residual_count(grid: Grid):
    """M = 2N + 14G residual groups (Sec. 5.1): N photometric, N gradient,
    6G smoothness, 2G epipolar, 6G magnitude."""
    return 2 * grid.N + 14 * grid.G
