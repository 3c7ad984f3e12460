"""FP64 reference of fixed-knot MFA encoding (test infrastructure only).

Encoding (paper, Sec. III-A and Fig. 1; Sec. IV-A2 "MFA Encoding"): a block
of samples is represented by the control points of a tensor-product B-spline
of given degrees and control-point counts; MFA approximates the samples
rather than interpolating them (Sec. III-B: one global optimisation over the
domain).  The paper prints no fitting formula.  Reading taken (the fixed-knot
step of Fig. 1: parameterisation and an initial knot distribution, before
any knot insertion): the control points are the least-squares solution

    P = argmin_P  sum_{i0,i1,i2} ( f(u0[i0], u1[i1], u2[i2]; P) - F[i0,i1,i2] )^2,

with f the spline of the model (oracle.bspline definitions) and the samples
F on a tensor grid of parameters u_a.  On a tensor grid the design matrix is
the Kronecker product B0 (x) B1 (x) B2 of the per-axis collocation matrices
B_a[i, j] = N_{j,p_a}(u_a[i]), and the pseudo-inverse of a Kronecker product
is the Kronecker product of the pseudo-inverses, so the minimiser (unique
when every B_a has full column rank) is the three mode products

    P = F x_0 B0^+ x_1 B1^+ x_2 B2^+.

This module writes that out: collocation matrices from the oracle's span
rule and Cox-de Boor basis, pseudo-inverses by numpy's SVD-based
``pinv`` (a library step), mode products by ``tensordot``.  The CPU tests pin
it against the dense Kronecker least-squares problem solved directly on tiny
grids, exact reproduction of splines of the same space, reproduction of
polynomials of degree <= p, and the normal equations of the residual.
"""
from __future__ import annotations

import numpy as np

from .bspline import basis_and_derivs, find_span


def collocation(T: np.ndarray, p: int, n: int, u: np.ndarray) -> np.ndarray:
    """B[i, j] = N_{j,p}(u[i]) (N x n, FP64) for clamped knots T (n + p + 1)."""
    u = np.asarray(u, dtype=np.float64)
    s = find_span(T, p, n, u)
    N, _ = basis_and_derivs(T, p, s, u)
    B = np.zeros((u.shape[0], n))
    rows = np.arange(u.shape[0])
    for r in range(p + 1):
        B[rows, s - p + r] = N[:, r]
    return B


def mode_product(X: np.ndarray, M: np.ndarray, axis: int) -> np.ndarray:
    """(X x_axis M)[.., j, ..] = sum_i M[j, i] X[.., i, ..]."""
    Y = np.tensordot(M, X, axes=([1], [axis]))      # new axis first
    return np.moveaxis(Y, 0, axis)


def fit_grid(F: np.ndarray, axis_u, degree, knots, n_ctrl) -> np.ndarray:
    """Least-squares control points (n0, n1, n2) of samples F (N0, N1, N2)
    at the tensor grid of parameters axis_u (FP64, each in [0, 1])."""
    P = np.asarray(F, dtype=np.float64)
    for a in range(3):
        B = collocation(np.asarray(knots[a], np.float64), int(degree[a]), int(n_ctrl[a]), axis_u[a])
        P = mode_product(P, np.linalg.pinv(B), a)
    return P


def reconstruct_grid(P: np.ndarray, axis_u, degree, knots) -> np.ndarray:
    """Values of the spline with control points P on the tensor grid of
    parameters axis_u: P x_0 B0 x_1 B1 x_2 B2."""
    R = np.asarray(P, dtype=np.float64)
    for a in range(3):
        B = collocation(np.asarray(knots[a], np.float64), int(degree[a]), R.shape[a], axis_u[a])
        R = mode_product(R, B, a)
    return R


def span_errors(err: np.ndarray, axis_u, degree, knots):
    """Per axis, the largest error over the samples whose parameter lies in
    each knot span (span rule D2): a list of three arrays (n_a - p_a,)."""
    out = []
    for a in range(3):
        T = np.asarray(knots[a], np.float64)
        p, n = int(degree[a]), len(knots[a]) - int(degree[a]) - 1
        s = find_span(T, p, n, axis_u[a]) - p
        axes = tuple(b for b in range(3) if b != a)
        marg = err.max(axis=axes)                    # max over the other two axes
        e = np.zeros(n - p)
        np.maximum.at(e, s, marg)
        out.append(e)
    return out


def fit_adaptive(F: np.ndarray, axis_u, degree, n_init, e_max: float, max_iter: int = 10,
                 max_ctrl=None):
    """Fixed-knot fits with knot insertion (paper Fig. 1): starting from
    clamped uniform knots with n_init control points per axis, fit, measure
    the error of every sample relative to the data range, and halve every
    knot span (per axis) whose largest error exceeds e_max and whose two
    halves would each hold a sample parameter; refit; stop when no span is
    halved or after max_iter fits.  Returns (knots, P, history), history
    holding per fit the control-point counts and the largest error.

    max_ctrl (a per-axis cap on the control-point count; the paper sets
    none, a storage budget is an implementation's choice): when more spans
    qualify than the cap leaves room for, the spans of largest error are
    halved, ties going to the lower span."""
    F = np.asarray(F, dtype=np.float64)
    rng = float(F.max() - F.min()) or 1.0
    knots = []
    for a in range(3):
        p, n = int(degree[a]), int(n_init[a])
        inner = np.arange(1, n - p) / (n - p)
        knots.append(np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)]))
    history = []
    for _ in range(max_iter):
        n_ctrl = [len(knots[a]) - degree[a] - 1 for a in range(3)]
        fitted = [k.copy() for k in knots]
        P = fit_grid(F, axis_u, degree, knots, n_ctrl)
        err = np.abs(reconstruct_grid(P, axis_u, degree, knots) - F) / rng
        history.append((list(n_ctrl), float(err.max())))
        E = span_errors(err, axis_u, degree, knots)
        grown = False
        for a in range(3):
            p = int(degree[a])
            T = knots[a]
            u = np.asarray(axis_u[a], np.float64)
            new = []
            for j, e in enumerate(E[a]):
                t0, t1 = T[p + j], T[p + j + 1]
                mid = 0.5 * (t0 + t1)
                if e > e_max and np.any((u >= t0) & (u < mid)) and np.any((u >= mid) & (u <= t1)):
                    new.append((e, mid))
            if max_ctrl is not None:
                room = int(max_ctrl[a]) - n_ctrl[a]
                if len(new) > room:
                    new = sorted(new, key=lambda c: -c[0])[:room]      # stable: ties keep span order
            new = [m for _, m in new]
            if new:
                knots[a] = np.sort(np.concatenate([T, new]))
                grown = True
        if not grown:
            break
    return fitted, P, history
