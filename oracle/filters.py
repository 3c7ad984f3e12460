"""FP64 reference of the local-filter baselines and of the Marschner-Lobb
test function (test infrastructure only).

The paper compares MFA queries with local reconstruction filters applied
to the raw samples -- nearest neighbour and trilinear (low order),
tricubic and Catmull-Rom (high order), Sec. I and Sec. V -- and measures
rendering quality against the analytic Marschner-Lobb function (Sec. V-A1,
Table II).  It defines the function but none of the filters.  Readings:

* samples v[i0, i1, i2] sit at x_a = lo_a + i_a h_a, h_a = (hi_a - lo_a) /
  (N_a - 1); a point maps to the grid coordinate g_a = (x_a - lo_a) / h_a,
  clamped to [0, N_a - 1];
* trilinear: cell c = min(floor(g), N - 2), t = g - c, weights (1 - t, t);
* Catmull-Rom: the cubic interpolating spline with tangents
  (v[c+1] - v[c-1]) / 2, on samples c-1 .. c+2 with c = min(floor(g), N - 2);
* tricubic: the uniform cubic B-spline filter applied to the samples
  themselves (approximating, no prefilter), same stencil;
* stencil indices outside [0, N-1] repeat the edge sample;
* gradients: the analytic derivative of the filter's piecewise polynomial
  (one weight per axis replaced by its derivative, times 1 / h_a).

Marschner-Lobb as the paper prints it: F = (1 - sin(pi z / 2) + alpha (1 +
rho(sqrt(x^2 + y^2)))) / (2 (1 + alpha)), rho(r) = cos(2 pi f_M cos(pi r /
2)), f_M = 6, alpha = 0.25, on the printed domain [0, 7]^3.
"""
from __future__ import annotations

import numpy as np

TRILINEAR, CATMULL_ROM, BSPLINE3 = 0, 1, 2
ML_FM, ML_ALPHA = 6.0, 0.25
ML_LO, ML_HI = (0.0, 0.0, 0.0), (7.0, 7.0, 7.0)


def ml_value_grad(x: np.ndarray, fm: float = ML_FM, alpha: float = ML_ALPHA):
    """Marschner-Lobb value and analytic gradient at points x (m, 3)."""
    x = np.asarray(x, dtype=np.float64)
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    r = np.sqrt(X * X + Y * Y)
    inner = 2.0 * np.pi * fm * np.cos(0.5 * np.pi * r)
    rho = np.cos(inner)
    den = 2.0 * (1.0 + alpha)
    f = (1.0 - np.sin(0.5 * np.pi * Z) + alpha * (1.0 + rho)) / den
    # d rho / d r = sin(inner) * 2 pi fm * sin(pi r / 2) * pi / 2
    drho = np.sin(inner) * 2.0 * np.pi * fm * np.sin(0.5 * np.pi * r) * 0.5 * np.pi
    with np.errstate(invalid="ignore", divide="ignore"):
        rx = np.where(r > 0.0, X / r, 0.0)
        ry = np.where(r > 0.0, Y / r, 0.0)
    g = np.stack([alpha * drho * rx / den, alpha * drho * ry / den,
                  -0.5 * np.pi * np.cos(0.5 * np.pi * Z) / den], axis=1)
    return f, g


def ml_samples(N: int, lo=ML_LO, hi=ML_HI) -> np.ndarray:
    """F_ML at the N^3 grid points x_i = lo + i (hi - lo) / (N - 1)."""
    ax = [lo[a] + np.arange(N, dtype=np.float64) * ((hi[a] - lo[a]) / (N - 1)) for a in range(3)]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    f, _ = ml_value_grad(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))
    return f.reshape(N, N, N)


def weights(kind: int, t: np.ndarray):
    """Per-axis stencil weights and their derivatives d/dt: (m, K) each,
    K = 2 (trilinear, samples c, c+1) or 4 (cubic, samples c-1 .. c+2)."""
    t = np.asarray(t, dtype=np.float64)
    if kind == TRILINEAR:
        w = np.stack([1.0 - t, t], axis=1)
        dw = np.stack([-np.ones_like(t), np.ones_like(t)], axis=1)
        return w, dw
    t2, t3 = t * t, t * t * t
    if kind == CATMULL_ROM:
        w = np.stack([(-t3 + 2 * t2 - t) / 2, (3 * t3 - 5 * t2 + 2) / 2,
                      (-3 * t3 + 4 * t2 + t) / 2, (t3 - t2) / 2], axis=1)
        dw = np.stack([(-3 * t2 + 4 * t - 1) / 2, (9 * t2 - 10 * t) / 2,
                       (-9 * t2 + 8 * t + 1) / 2, (3 * t2 - 2 * t) / 2], axis=1)
        return w, dw
    if kind == BSPLINE3:
        s = 1.0 - t
        w = np.stack([s * s * s / 6, (3 * t3 - 6 * t2 + 4) / 6,
                      (-3 * t3 + 3 * t2 + 3 * t + 1) / 6, t3 / 6], axis=1)
        dw = np.stack([-s * s / 2, (9 * t2 - 12 * t) / 6, (-9 * t2 + 6 * t + 3) / 6, t2 / 2],
                      axis=1)
        return w, dw
    raise ValueError(f"unknown filter {kind}")


def grid_field(volume: np.ndarray, lo, hi, kind: int):
    """Field callable x (m,3) -> (value (m,), world gradient (m,3)) of the
    local filter 'kind' over the samples 'volume' (N0, N1, N2) on the box."""
    V = np.asarray(volume, dtype=np.float64)
    N = V.shape
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    h = (hi - lo) / (np.asarray(N, dtype=np.float64) - 1.0)
    K = 2 if kind == TRILINEAR else 4
    off = 0 if kind == TRILINEAR else -1

    def fn(x):
        x = np.asarray(x, dtype=np.float64)
        m = x.shape[0]
        idx, w, dw = [], [], []
        for a in range(3):
            g = np.clip((x[:, a] - lo[a]) / h[a], 0.0, N[a] - 1.0)
            c = np.minimum(np.floor(g), N[a] - 2).astype(np.int64)
            wa, dwa = weights(kind, g - c)
            ia = np.clip(c[:, None] + off + np.arange(K)[None, :], 0, N[a] - 1)
            idx.append(ia)
            w.append(wa)
            dw.append(dwa / h[a])
        f = np.zeros(m)
        gr = np.zeros((m, 3))
        for i in range(K):
            for j in range(K):
                for k in range(K):
                    v = V[idx[0][:, i], idx[1][:, j], idx[2][:, k]]
                    f += w[0][:, i] * w[1][:, j] * w[2][:, k] * v
                    gr[:, 0] += dw[0][:, i] * w[1][:, j] * w[2][:, k] * v
                    gr[:, 1] += w[0][:, i] * dw[1][:, j] * w[2][:, k] * v
                    gr[:, 2] += w[0][:, i] * w[1][:, j] * dw[2][:, k] * v
        return f, gr
    return fn
