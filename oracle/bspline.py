"""FP64 reference evaluation of an MFA model (test infrastructure only).

The model (paper, Sec. III-A; Sec. IV-A2) is a tensor product of B-spline
functions: per block and per axis a degree p_a, n_a control-point indices and
a knot vector T_a; control points P[i][j][k] are the coefficients.  Blocks
come from partitioning the volume (Sec. IV-A1); each block is an
independent model over its own box, and a world point is evaluated by the
block that owns it.  The paper prints no B-spline formulas, so the
definitions below are the textbook ones of de Boor's "A Practical Guide to
Splines", which the paper cites for spline bases (Sec. I):

* degree-0 basis: N_{i,0}(u) = 1 on [T_i, T_{i+1}), else 0, with the last
  non-empty span closed at u = T_n;
* recursion: N_{i,q} = w_{i,q} N_{i,q-1} + (1 - w_{i+1,q}) N_{i+1,q-1},
  w_{i,q}(u) = (u - T_i) / (T_{i+q} - T_i), any term with a zero
  denominator taken as 0;
* first derivative: N'_{i,p} = p/(T_{i+p}-T_i) N_{i,p-1}
  - p/(T_{i+p+1}-T_{i+1}) N_{i+1,p-1} (zero-denominator terms dropped);
* value f(u) = sum_{ijk} N_{i,p0}(u0) N_{j,p1}(u1) N_{k,p2}(u2) P_ijk and
  the gradient with one factor replaced by its derivative (Sec. III-B: the
  model gives analytic derivatives).

Only the p+1 basis functions that are non-zero on the span holding u are
formed (the others vanish by the support property of the recursion); the
sum over the (p+1)^3 active control points is the plain triple sum, in
FP64, with no factorisation.

Decisions (span, block) are exact FP64 comparisons on data:
* D1 map:   xc = clamp(x, E[0], E[G]);  u = clamp((xc - lo_b) * inv_ext_b, 0, 1)
            with inv_ext_b = 1.0 / (hi_b - lo_b) (one IEEE division);
* D2 span:  s = max{ i in [p, n-1] : T[i] <= u };
* D3 block: b = max{ i in [0, G-1] : E[i] <= xc }.
"""
from __future__ import annotations

import numpy as np

CHUNK = 1 << 14


def find_span(T: np.ndarray, p: int, n: int, u: np.ndarray) -> np.ndarray:
    """D2: index of the knot span holding u (right-continuous, last closed)."""
    u = np.asarray(u, dtype=np.float64)
    s = np.searchsorted(T[p:n], u, side="right") - 1 + p
    return np.clip(s, p, n - 1).astype(np.int64)


def _term(num, den):
    """num/den with the 0/0 := 0 convention of the recursion (any zero
    denominator makes the whole term vanish)."""
    num = np.asarray(num, dtype=np.float64)
    den = np.asarray(den, dtype=np.float64)
    out = np.zeros(np.broadcast(num, den).shape)
    nz = np.broadcast_to(den != 0.0, out.shape)
    numb = np.broadcast_to(num, out.shape)
    denb = np.broadcast_to(den, out.shape)
    out[nz] = numb[nz] / denb[nz]
    return out


def basis_and_derivs(T: np.ndarray, p: int, s: np.ndarray, u: np.ndarray):
    """Values N_{s-p+r,p}(u) and derivatives N'_{s-p+r,p}(u), r = 0..p.

    Built level by level from the degree-0 indicator of span s by the
    recursion above (only the functions active on span s are kept).
    Returns (N, D), each (m, p+1) float64.
    """
    u = np.asarray(u, dtype=np.float64)
    s = np.asarray(s, dtype=np.int64)
    m = u.shape[0]
    N = np.ones((m, 1))            # level 0: N_{s,0} = 1 on its span
    prev = np.zeros((m, 0))
    for q in range(1, p + 1):
        nxt = np.zeros((m, q + 1))
        for r in range(q + 1):
            i = s - q + r                  # global index of N_{i,q}
            if r >= 1:                     # w_{i,q} N_{i,q-1}
                w = _term(u - T[i], T[i + q] - T[i])
                nxt[:, r] += w * N[:, r - 1]
            if r <= q - 1:                 # (1 - w_{i+1,q}) N_{i+1,q-1}
                v = _term(T[i + q + 1] - u, T[i + q + 1] - T[i + 1])
                nxt[:, r] += v * N[:, r]
        prev = N
        N = nxt
    D = np.zeros((m, p + 1))
    if p >= 1:
        for r in range(p + 1):
            i = s - p + r
            if r >= 1:
                D[:, r] += _term(float(p), T[i + p] - T[i]) * prev[:, r - 1]
            if r <= p - 1:
                D[:, r] -= _term(float(p), T[i + p + 1] - T[i + 1]) * prev[:, r]
    return N, D


def block_eval_param(block, u: np.ndarray):
    """Value and parameter-space gradient of one block at u (m,3) in [0,1].

    Returns f (m,), dfdu (m,3), spans (m,3).
    """
    u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
    P = block.ctrl
    deg = [int(d) for d in block.degree]
    nn = P.shape
    m = u.shape[0]
    f = np.zeros(m)
    g = np.zeros((m, 3))
    spans = np.zeros((m, 3), dtype=np.int64)
    for c0 in range(0, m, CHUNK):
        uc = u[c0:c0 + CHUNK]
        NN, DD, idx = [], [], []
        for a in range(3):
            s = find_span(block.knots[a], deg[a], nn[a], uc[:, a])
            spans[c0:c0 + CHUNK, a] = s
            Na, Da = basis_and_derivs(block.knots[a], deg[a], s, uc[:, a])
            NN.append(Na)
            DD.append(Da)
            idx.append(s[:, None] - deg[a] + np.arange(deg[a] + 1)[None, :])
        Pg = P[idx[0][:, :, None, None], idx[1][:, None, :, None], idx[2][:, None, None, :]]
        X = (NN[0][:, :, None, None], NN[1][:, None, :, None], NN[2][:, None, None, :])
        Xd = (DD[0][:, :, None, None], DD[1][:, None, :, None], DD[2][:, None, None, :])
        f[c0:c0 + CHUNK] = (X[0] * X[1] * X[2] * Pg).sum(axis=(1, 2, 3))
        g[c0:c0 + CHUNK, 0] = (Xd[0] * X[1] * X[2] * Pg).sum(axis=(1, 2, 3))
        g[c0:c0 + CHUNK, 1] = (X[0] * Xd[1] * X[2] * Pg).sum(axis=(1, 2, 3))
        g[c0:c0 + CHUNK, 2] = (X[0] * X[1] * Xd[2] * Pg).sum(axis=(1, 2, 3))
    return f, g, spans


def block_owner(E: np.ndarray, G: int, x: np.ndarray):
    """D3: owning block index along one axis and the clamped coordinate."""
    x = np.asarray(x, dtype=np.float64)
    xc = np.minimum(np.maximum(x, E[0]), E[G])
    b = np.searchsorted(E[:G], xc, side="right") - 1
    return np.clip(b, 0, G - 1).astype(np.int64), xc


def world_to_param(model, xyz: np.ndarray):
    """D1 + D3 for world points (m,3): block ids (m,3), u (m,3), inv_ext (m,3)."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    bids = np.zeros(xyz.shape, dtype=np.int64)
    u = np.zeros(xyz.shape)
    inv_ext = np.zeros(xyz.shape)
    for a in range(3):
        E = np.asarray(model.edges[a], dtype=np.float64)
        G = int(model.grid[a])
        b, xc = block_owner(E, G, xyz[:, a])
        lo = E[b]
        hi = E[b + 1]
        ie = 1.0 / (hi - lo)
        ua = (xc - lo) * ie
        u[:, a] = np.minimum(np.maximum(ua, 0.0), 1.0)
        bids[:, a] = b
        inv_ext[:, a] = ie
    return bids, u, inv_ext


def evaluate(model, xyz: np.ndarray):
    """Value and world-space gradient at world points (m,3).

    Returns dict(f (m,), grad (m,3), spans (m,3), blocks (m,3)).  The world
    gradient is the parameter gradient times inv_ext of the owning block
    (chain rule of the affine map D1).
    """
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    bids, u, inv_ext = world_to_param(model, xyz)
    g0, g1, g2 = model.grid
    flat = (bids[:, 0] * g1 + bids[:, 1]) * g2 + bids[:, 2]
    f = np.zeros(len(xyz))
    grad = np.zeros((len(xyz), 3))
    spans = np.zeros((len(xyz), 3), dtype=np.int64)
    for b in np.unique(flat):
        sel = np.nonzero(flat == b)[0]
        fb, gb, sb = block_eval_param(model.blocks[int(b)], u[sel])
        f[sel] = fb
        grad[sel] = gb * inv_ext[sel]
        spans[sel] = sb
    return dict(f=f, grad=grad, spans=spans, blocks=bids)


def decode_grid(model, axis_u, out_index=None):
    """Value and world gradient on the tensor grid axis_u[0] x axis_u[1] x
    axis_u[2] of parameters of a single-block model (parameters clamped to
    [0,1]).  Returns (res0,res1,res2,4) float64: (f, df/dx, df/dy, df/dz).

    If out_index (k,3) of grid indices is given, only those outputs are
    computed and (k,4) is returned.
    """
    if list(model.grid) != [1, 1, 1]:
        raise ValueError("grid decode is defined for single-block models")
    U = [np.minimum(np.maximum(np.asarray(a, dtype=np.float64), 0.0), 1.0) for a in axis_u]
    inv_ext = np.array([1.0 / (model.hi[a] - model.lo[a]) for a in range(3)])
    blk = model.blocks[0]
    if out_index is None:
        g = np.stack(np.meshgrid(U[0], U[1], U[2], indexing="ij"), axis=-1).reshape(-1, 3)
    else:
        idx = np.asarray(out_index, dtype=np.int64).reshape(-1, 3)
        g = np.stack([U[0][idx[:, 0]], U[1][idx[:, 1]], U[2][idx[:, 2]]], axis=1)
    f, du, spans = block_eval_param(blk, g)
    out = np.concatenate([f[:, None], du * inv_ext[None, :]], axis=1)
    if out_index is None:
        return out.reshape(len(U[0]), len(U[1]), len(U[2]), 4)
    return out


def grid_spans(model, axis_u):
    """Per-axis spans of the grid tables (D2), for integer parity."""
    blk = model.blocks[0]
    out = []
    for a in range(3):
        u = np.minimum(np.maximum(np.asarray(axis_u[a], dtype=np.float64), 0.0), 1.0)
        out.append(find_span(blk.knots[a], int(blk.degree[a]), blk.ctrl.shape[a], u))
    return out
