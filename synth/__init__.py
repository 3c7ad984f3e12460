"""Seeded synthetic inputs for the MFA evaluator and renderer.

This module produces *inputs only*: knot vectors, control points of
tensor-product B-spline models, point sets, parameter grids, cameras and
the transfer-function table.  It holds none of the evaluation arithmetic
(span location, basis functions, contraction, shading, compositing), so it
can feed both the FP64 oracle and the GPU library without coupling them.

The paper's own workloads (Marschner-Lobb volumes, Fuel, Nucleon, Aneurysm,
Bonsai and the Richtmyer-Meshkov timestep of Sec. V-A) are not available
here; seeded Gaussian-sum fields of the same structure stand in for them.

Recipes (all draws use ``np.random.default_rng(seed)``):

* ``model_c1``: 8 Gaussians, centres U[0.1,0.9]^3, sigma U[0.08,0.25],
  amplitude U[0.5,1]; 16^3 control points, degree 3, clamped uniform knots;
  control points = field at the Greville abscissae plus uniform noise of
  +-1 % of the field's range.
* ``model_c2``: 64 Gaussians, sigma U[0.03,0.15]; 128^3 control points, no
  noise.
* ``model_c3_fit48``: the c1 field sampled on a 128^3 grid (with 1 % noise),
  fitted by fixed-knot tensor least squares with 48^3 control points.
* ``model_c4``: 8x8x8 blocks over [0,1]^3, per-block control-point counts
  U{24..72} per axis, 512 Gaussians with log-uniform sigma in [0.004,0.1]
  and amplitude +-(sigma/0.1)^(1/3), truncated at 5 sigma.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "BlockSpec", "ModelSpec", "GaussianField", "clamped_uniform_knots",
    "greville", "gaussian_field", "model_c1", "model_c2", "model_c3_fit48",
    "model_c4", "single_block_model", "random_points", "grid_axis",
    "tf_table_A", "tf_table_constant", "ortho_camera", "perspective_camera",
    "render_params", "linear_precision_ctrl",
]


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclasses.dataclass
class BlockSpec:
    """One tensor-product B-spline block (inputs only)."""
    degree: List[int]               # per axis
    knots: List[np.ndarray]         # per axis, float64, n+p+1, clamped
    ctrl: np.ndarray                # float64 [n0][n1][n2], axis 2 fastest

    @property
    def n_ctrl(self) -> List[int]:
        return [int(s) for s in self.ctrl.shape]


@dataclasses.dataclass
class ModelSpec:
    """A model: world box split into grid[0]*grid[1]*grid[2] blocks."""
    grid: List[int]
    lo: np.ndarray                  # float64 (3,)
    hi: np.ndarray                  # float64 (3,)
    edges: List[np.ndarray]         # per axis float64, grid[a]+1 entries
    blocks: List[BlockSpec]         # C order over the block grid
    voxel: float                    # reference voxel size (world units)

    def n_ctrl_total(self) -> int:
        return int(sum(b.ctrl.size for b in self.blocks))

    def ctrl_min_max(self):
        lo = min(float(b.ctrl.min()) for b in self.blocks)
        hi = max(float(b.ctrl.max()) for b in self.blocks)
        return lo, hi


# --------------------------------------------------------------------------
# knots and abscissae (input data)
# --------------------------------------------------------------------------
def clamped_uniform_knots(n: int, p: int) -> np.ndarray:
    """Clamped (open) uniform knot vector on [0,1] with n control points.

    T[0..p] = 0, T[n..n+p] = 1 and T[p+j] = j/(n-p), each interior knot one
    IEEE double division.
    """
    if n < p + 1:
        raise ValueError("need n >= p+1")
    T = np.zeros(n + p + 1, dtype=np.float64)
    nsp = np.float64(n - p)
    for j in range(1, n - p):
        T[p + j] = np.float64(j) / nsp
    T[n:] = 1.0
    return T


def greville(T: np.ndarray, p: int, n: int) -> np.ndarray:
    """Greville abscissae xi_i = mean(T[i+1..i+p]); used to place samples."""
    if p == 0:
        return 0.5 * (T[:n] + T[1:n + 1])
    return np.array([T[i + 1:i + p + 1].sum() / p for i in range(n)])


# --------------------------------------------------------------------------
# Gaussian-sum fields
# --------------------------------------------------------------------------
@dataclasses.dataclass
class GaussianField:
    centres: np.ndarray   # (G,3)
    sigmas: np.ndarray    # (G,)
    amps: np.ndarray      # (G,)
    trunc: Optional[float] = None   # truncate each Gaussian at trunc*sigma

    def value_grad(self, x: np.ndarray, chunk: int = 1 << 16):
        """Analytic value and gradient at world points x (m,3)."""
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        f = np.zeros(len(x))
        g = np.zeros((len(x), 3))
        for c0 in range(0, len(x), chunk):
            xs = x[c0:c0 + chunk]
            for c, s, a in zip(self.centres, self.sigmas, self.amps):
                d = xs - c
                r2 = (d * d).sum(axis=1)
                e = a * np.exp(-r2 / (2.0 * s * s))
                if self.trunc is not None:
                    e = np.where(r2 <= (self.trunc * s) ** 2, e, 0.0)
                f[c0:c0 + chunk] += e
                g[c0:c0 + chunk] += (-e / (s * s))[:, None] * d
        return f, g

    def value(self, x):
        return self.value_grad(x)[0]

    def value_separable(self, xs, ys, zs):
        """Field on the tensor grid xs x ys x zs (each 1-D), float64."""
        out = np.zeros((len(xs), len(ys), len(zs)))
        for c, s, a in zip(self.centres, self.sigmas, self.amps):
            ex = np.exp(-(xs - c[0]) ** 2 / (2 * s * s))
            ey = np.exp(-(ys - c[1]) ** 2 / (2 * s * s))
            ez = np.exp(-(zs - c[2]) ** 2 / (2 * s * s))
            if self.trunc is None:
                out += a * ex[:, None, None] * ey[None, :, None] * ez[None, None, :]
            else:
                r = self.trunc * s
                ix = np.nonzero(np.abs(xs - c[0]) <= r)[0]
                iy = np.nonzero(np.abs(ys - c[1]) <= r)[0]
                iz = np.nonzero(np.abs(zs - c[2]) <= r)[0]
                if len(ix) == 0 or len(iy) == 0 or len(iz) == 0:
                    continue
                sub = (a * ex[ix][:, None, None] * ey[iy][None, :, None]
                       * ez[iz][None, None, :])
                dx = (xs[ix] - c[0])[:, None, None]
                dy = (ys[iy] - c[1])[None, :, None]
                dz = (zs[iz] - c[2])[None, None, :]
                sub = np.where(dx * dx + dy * dy + dz * dz <= r * r, sub, 0.0)
                out[ix[0]:ix[-1] + 1, iy[0]:iy[-1] + 1, iz[0]:iz[-1] + 1] += sub
        return out


def gaussian_field(G: int, seed: int, sigma_range=(0.08, 0.25),
                   amp_range=(0.5, 1.0), centre_range=(0.1, 0.9)) -> GaussianField:
    rng = np.random.default_rng(seed)
    c = rng.uniform(centre_range[0], centre_range[1], size=(G, 3))
    s = rng.uniform(sigma_range[0], sigma_range[1], size=G)
    a = rng.uniform(amp_range[0], amp_range[1], size=G)
    return GaussianField(c, s, a)


def turbulence_field(G: int, seed: int) -> GaussianField:
    """512-Gaussian 'turbulence-like' field: log-uniform scales, signed amps."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, size=(G, 3))
    s = np.exp(rng.uniform(math.log(0.004), math.log(0.1), size=G))
    sign = np.where(rng.random(G) < 0.5, -1.0, 1.0)
    a = sign * (s / 0.1) ** (1.0 / 3.0)
    return GaussianField(c, s, a, trunc=5.0)


# --------------------------------------------------------------------------
# models
# --------------------------------------------------------------------------
def _ctrl_from_field(field: GaussianField, knots, degree, lo, hi, noise: float,
                     rng: Optional[np.random.Generator]) -> np.ndarray:
    xs = [lo[a] + greville(knots[a], degree[a], len(knots[a]) - degree[a] - 1)
          * (hi[a] - lo[a]) for a in range(3)]
    F = field.value_separable(*xs)
    if noise > 0.0:
        span = float(F.max() - F.min())
        F = F + rng.uniform(-noise, noise, size=F.shape) * span
    return F


def single_block_model(ctrl: np.ndarray, degree: Sequence[int],
                       knots: Optional[Sequence[np.ndarray]] = None,
                       lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                       voxel: Optional[float] = None) -> ModelSpec:
    ctrl = np.ascontiguousarray(ctrl, dtype=np.float64)
    deg = [int(d) for d in degree]
    if knots is None:
        knots = [clamped_uniform_knots(ctrl.shape[a], deg[a]) for a in range(3)]
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    if voxel is None:
        voxel = float(np.min(hi - lo)) / 63.0
    blk = BlockSpec(deg, [np.asarray(k, dtype=np.float64) for k in knots], ctrl)
    return ModelSpec([1, 1, 1], lo, hi, [np.array([lo[a], hi[a]]) for a in range(3)],
                     [blk], float(voxel))


def model_c1(p: int = 3, n: int = 16, seed: int = 1) -> ModelSpec:
    """Single block, 16^3 control points, 8 Gaussians + 1 % noise."""
    field = gaussian_field(8, seed)
    deg = [p, p, p]
    knots = [clamped_uniform_knots(n, p) for _ in range(3)]
    rng = np.random.default_rng(seed + 1000)
    ctrl = _ctrl_from_field(field, knots, deg, np.zeros(3), np.ones(3), 0.01, rng)
    return single_block_model(ctrl, deg, knots, voxel=1.0 / 63.0)


def field_c1(seed: int = 1) -> GaussianField:
    return gaussian_field(8, seed)


def field_c2(seed: int = 2) -> GaussianField:
    return gaussian_field(64, seed, sigma_range=(0.03, 0.15))


def model_c2(n: int = 128, p: int = 3, seed: int = 2) -> ModelSpec:
    """Single block, 128^3 control points, 64 Gaussians, no noise."""
    field = field_c2(seed)
    deg = [p, p, p]
    knots = [clamped_uniform_knots(n, p) for _ in range(3)]
    ctrl = _ctrl_from_field(field, knots, deg, np.zeros(3), np.ones(3), 0.0, None)
    return single_block_model(ctrl, deg, knots, voxel=1.0 / 511.0)


def marschner_lobb_samples(N: int, lo=(0.0, 0.0, 0.0), hi=(7.0, 7.0, 7.0), fm: float = 6.0,
                           alpha: float = 0.25) -> np.ndarray:
    """FP32 samples (N, N, N) of the Marschner-Lobb test function (the
    paper's Sec. V-A1 definition, f_M = 6, alpha = 0.25, on its printed
    domain [0, 7]^3) at x_i = lo + i (hi - lo) / (N - 1), axis 2 fastest."""
    ax = [lo[a] + np.arange(N, dtype=np.float64) * ((hi[a] - lo[a]) / (N - 1)) for a in range(3)]
    r = np.sqrt(ax[0][:, None] ** 2 + ax[1][None, :] ** 2)                  # (N, N)
    rho = np.cos(2.0 * np.pi * fm * np.cos(0.5 * np.pi * r))
    zpart = 1.0 - np.sin(0.5 * np.pi * ax[2])                               # (N,)
    F = (zpart[None, None, :] + alpha * (1.0 + rho)[:, :, None]) / (2.0 * (1.0 + alpha))
    return F.astype(np.float32)


def graded_knot_vector(n: int, p: int, amp: float = 0.75, waves: int = 3) -> np.ndarray:
    """Clamped knots T[p+j] = phi(j / (n-p)) with the monotone map
    phi(t) = t - amp sin(2 pi waves t) / (2 pi waves): span widths vary by
    (1 + amp) / (1 - amp) (7x at amp = 0.75), the shape of knot vectors
    refined where a field varies most."""
    t = np.arange(1, n - p, dtype=np.float64) / (n - p)
    inner = t - amp * np.sin(2 * np.pi * waves * t) / (2 * np.pi * waves)
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def model_c2_graded(n: int = 128, p: int = 3, seed: int = 2) -> ModelSpec:
    """The 128^3 model of the 64-Gaussian field on graded (non-uniform)
    knots, a different phase per axis; control points at the Greville
    abscissae."""
    field = field_c2(seed)
    deg = [p, p, p]
    knots = [graded_knot_vector(n, p, waves=3 + a) for a in range(3)]
    ctrl = _ctrl_from_field(field, knots, deg, np.zeros(3), np.ones(3), 0.0, None)
    return single_block_model(ctrl, deg, knots, voxel=1.0 / 511.0)


def model_c3_fit48(n_ctrl: int = 48, n_in: int = 128, p: int = 3,
                   seed: int = 1) -> ModelSpec:
    """Compressed model: c1 field sampled on n_in^3 (+1 % noise), fixed-knot
    tensor least-squares fit with n_ctrl^3 control points (scipy design
    matrices + numpy least squares, one axis at a time)."""
    from scipy.interpolate import BSpline
    field = field_c1(seed)
    xs = np.arange(n_in, dtype=np.float64) / (n_in - 1)
    F = field.value_separable(xs, xs, xs)
    rng = np.random.default_rng(seed + 3)
    F = F + rng.uniform(-0.01, 0.01, size=F.shape) * float(F.max() - F.min())
    T = clamped_uniform_knots(n_ctrl, p)
    B = BSpline.design_matrix(xs, T, p).toarray()          # (n_in, n_ctrl)
    pinv = np.linalg.pinv(B)                                # (n_ctrl, n_in)
    C = np.einsum("ia,abc->ibc", pinv, F)
    C = np.einsum("jb,ibc->ijc", pinv, C)
    C = np.einsum("kc,ijc->ijk", pinv, C)
    return single_block_model(C, [p, p, p], [T, T, T], voxel=1.0 / (n_in - 1))


def model_c4(seed: int = 4, grid: int = 8, nmin: int = 24, nmax: int = 72,
             p: int = 3, G: int = 512) -> ModelSpec:
    """8x8x8 blocks over [0,1]^3 with uneven per-block control-point counts."""
    rng = np.random.default_rng(seed)
    field = turbulence_field(G, seed + 100)
    edges = [np.arange(grid + 1, dtype=np.float64) / grid for _ in range(3)]
    blocks = []
    for b0 in range(grid):
        for b1 in range(grid):
            for b2 in range(grid):
                n = [int(v) for v in rng.integers(nmin, nmax + 1, size=3)]
                knots = [clamped_uniform_knots(n[a], p) for a in range(3)]
                lo = np.array([edges[0][b0], edges[1][b1], edges[2][b2]])
                hi = np.array([edges[0][b0 + 1], edges[1][b1 + 1], edges[2][b2 + 1]])
                ctrl = _ctrl_from_field(field, knots, [p, p, p], lo, hi, 0.0, None)
                blocks.append(BlockSpec([p, p, p], knots, ctrl))
    return ModelSpec([grid] * 3, np.zeros(3), np.ones(3), edges, blocks,
                     voxel=1.0 / 383.0)


def linear_precision_ctrl(knots, degree, coeffs) -> np.ndarray:
    """Control points c0 + c1*xi0 + c2*xi1 + c3*xi2 at the Greville abscissae
    (a spline that is exactly this affine function of the parameters)."""
    xi = [greville(knots[a], degree[a], len(knots[a]) - degree[a] - 1) for a in range(3)]
    return (coeffs[0] + coeffs[1] * xi[0][:, None, None]
            + coeffs[2] * xi[1][None, :, None] + coeffs[3] * xi[2][None, None, :])


# --------------------------------------------------------------------------
# query inputs
# --------------------------------------------------------------------------
def random_points(n: int, seed: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> np.ndarray:
    """World points as FP32 structure-of-arrays (3, n), uniform in the box."""
    rng = np.random.default_rng(seed)
    u = rng.random((3, n), dtype=np.float32)
    lo = np.asarray(lo, dtype=np.float32)[:, None]
    hi = np.asarray(hi, dtype=np.float32)[:, None]
    return np.ascontiguousarray(lo + u * (hi - lo), dtype=np.float32)


def grid_axis(N: int) -> np.ndarray:
    """Parameter table u_i = i/(N-1), float64, endpoints included."""
    if N == 1:
        return np.zeros(1)
    return np.arange(N, dtype=np.float64) / np.float64(N - 1)


# --------------------------------------------------------------------------
# transfer functions
# --------------------------------------------------------------------------
def tf_table_A() -> np.ndarray:
    """256-entry RGBA table (FP32, not premultiplied): blue->white->red ramp,
    transparent below s=0.25 and quadratic opacity up to 0.35."""
    s = np.arange(256, dtype=np.float64) / 255.0
    r = np.where(s <= 0.5, 2 * s, 1.0)
    g = np.where(s <= 0.5, 2 * s, 2 - 2 * s)
    b = np.where(s <= 0.5, 1.0, 2 - 2 * s)
    a = np.where(s < 0.25, 0.0, 0.35 * ((s - 0.25) / 0.75) ** 2)
    return np.ascontiguousarray(np.stack([r, g, b, a], axis=1), dtype=np.float32)


def tf_table_constant(rgba) -> np.ndarray:
    return np.ascontiguousarray(np.tile(np.asarray(rgba, dtype=np.float32), (256, 1)))


# --------------------------------------------------------------------------
# cameras: orthonormal right-handed (right, up, forward) basis, pixel scales
# --------------------------------------------------------------------------
def _orbit_basis(az_deg, el_deg, dist, centre):
    az, el = math.radians(az_deg), math.radians(el_deg)
    c = np.asarray(centre, dtype=np.float64)
    view = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    eye = c + dist * view
    fwd = -view / np.linalg.norm(view)
    world_up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, world_up)
    if np.linalg.norm(right) < 1e-12:
        right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right = right / np.linalg.norm(right)
    up = np.cross(right, fwd)
    up = up / np.linalg.norm(up)
    return eye, fwd, right, up


ORTHO, PERSPECTIVE = 0, 1


def ortho_camera(W: int, H: int, az_deg=30.0, el_deg=20.0, half_extent=0.9,
                 dist=2.0, centre=(0.5, 0.5, 0.5)) -> dict:
    eye, fwd, right, up = _orbit_basis(az_deg, el_deg, dist, centre)
    sy = half_extent / H
    sx = half_extent / H
    return dict(kind=ORTHO, eye=eye, forward=fwd, right=right, up=up, sx=sx, sy=sy)


def perspective_camera(W: int, H: int, az_deg=30.0, el_deg=20.0, fov_y_deg=45.0,
                       dist=2.0, centre=(0.5, 0.5, 0.5)) -> dict:
    eye, fwd, right, up = _orbit_basis(az_deg, el_deg, dist, centre)
    sy = math.tan(math.radians(fov_y_deg) / 2.0) / H
    return dict(kind=PERSPECTIVE, eye=eye, forward=fwd, right=right, up=up, sx=sy, sy=sy)


def axis_camera(W: int, H: int, axis: int = 0, half_extent=0.5,
                centre=(0.5, 0.5, 0.5), dist=2.0) -> dict:
    """Orthographic camera looking along +axis (exact basis vectors)."""
    fwd = np.zeros(3); fwd[axis] = 1.0
    a1, a2 = (axis + 1) % 3, (axis + 2) % 3
    right = np.zeros(3); right[a1] = 1.0
    up = np.cross(right, fwd)
    eye = np.asarray(centre, dtype=np.float64) - dist * fwd
    return dict(kind=ORTHO, eye=eye, forward=fwd, right=right, up=up,
                sx=half_extent / W, sy=half_extent / H)


def render_params(model: ModelSpec, tf=None, step=None, max_samples=1024,
                  ert_alpha=0.99, ka=0.3, kd=0.6, ks=0.3, shininess=16,
                  vmin=None, vmax=None) -> dict:
    """Render parameters with the defaults of the workloads (vmin/vmax from
    the FP64 control points, rounded to FP32; g0 = 1 % of the value range
    times the smallest inverse block extent)."""
    cmin, cmax = model.ctrl_min_max()
    vmin = np.float32(cmin if vmin is None else vmin)
    vmax = np.float32(cmax if vmax is None else vmax)
    inv_ext_min = min(1.0 / (model.edges[a][i + 1] - model.edges[a][i])
                      for a in range(3) for i in range(model.grid[a]))
    g0 = np.float32(0.01 * (float(vmax) - float(vmin)) * inv_ext_min)
    return dict(tf=tf_table_A() if tf is None else tf,
                vmin=vmin, vmax=vmax,
                step=float(0.5 * model.voxel if step is None else step),
                max_samples=int(max_samples), ert_alpha=np.float32(ert_alpha),
                ka=np.float32(ka), kd=np.float32(kd), ks=np.float32(ks),
                g0=g0, shininess=int(shininess))
