"""FP64 reference ray caster (test infrastructure only).

The paper's MFA-VV step (Sec. IV-A4) casts rays through the volume, queries
the model for value and gradient at each sample, and accumulates samples
with the "over" operator; its cost is linear in the number of queries.
Transfer function and shading parameters are user inputs (Sec. IV-B).  The
paper fixes none of the formulas, so the readings below are used:

* camera (pixel centres, row 0 at the top):
  px = (2i + 1 - W) sx,  py = (H - 2j - 1) sy;
  orthographic:  o = (eye + px right) + py up,  d = forward;
  perspective:   o = eye,  d = (forward + px right) + py up  (unnormalised,
  so t measures depth along the unit forward vector);
* slab test per axis with inv_d = 1/d_a; an axis with d_a = 0 misses unless
  lo_a <= o_a <= hi_a; t_near = max(0, max_a min(t1,t2)),
  t_far = min_a max(t1,t2); the ray misses if t_near >= t_far;
* schedule K = min(floor((t_far - t_near) / dt), max_samples) samples at
  t_k = t_near + (k + 1/2) dt,  x_k = o + t_k d;
* transfer function: s = clamp((f - vmin)/(vmax - vmin), 0, 1) * 255,
  i0 = min(floor(s), 254), linear interpolation between entries i0 and
  i0+1 of a 256-entry RGBA table (not premultiplied); no opacity
  correction for the step;
* Phong with a headlight: L = -d/|d|, n = g / max(|g|, g0),
  diff = |n . L| (two-sided), spec = diff^m,
  c' = rgb (ka + kd diff) + ks spec;
* front-to-back "over" on premultiplied colour: C += (1-A) alpha c',
  A += (1-A) alpha (the operator whose associativity the paper's
  compositing relies on, Sec. IV-A5);
* early termination after the first sample with A >= ert_alpha (that
  sample included).
"""
from __future__ import annotations

import numpy as np

ORTHO, PERSPECTIVE = 0, 1


def pixel_rays(cam: dict, W: int, H: int, pixels=None):
    """Origins and directions (float64) of the rays of the listed pixels.

    pixels: None for all pixels in row-major order, else (k,2) (row, col).
    """
    if pixels is None:
        jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        jj = jj.reshape(-1)
        ii = ii.reshape(-1)
    else:
        pix = np.asarray(pixels, dtype=np.int64).reshape(-1, 2)
        jj, ii = pix[:, 0], pix[:, 1]
    px = (2 * ii + 1 - W).astype(np.float64) * float(cam["sx"])
    py = (H - 2 * jj - 1).astype(np.float64) * float(cam["sy"])
    eye = np.asarray(cam["eye"], dtype=np.float64)
    fwd = np.asarray(cam["forward"], dtype=np.float64)
    right = np.asarray(cam["right"], dtype=np.float64)
    up = np.asarray(cam["up"], dtype=np.float64)
    m = len(ii)
    o = np.zeros((m, 3))
    d = np.zeros((m, 3))
    for a in range(3):
        if int(cam["kind"]) == ORTHO:
            o[:, a] = (eye[a] + px * right[a]) + py * up[a]
            d[:, a] = fwd[a]
        else:
            o[:, a] = eye[a]
            d[:, a] = (fwd[a] + px * right[a]) + py * up[a]
    return o, d


def slab(o: np.ndarray, d: np.ndarray, lo, hi):
    """Entry/exit parameters of rays against the box [lo, hi]; miss flags."""
    m = o.shape[0]
    t_near = np.zeros(m)
    t_far = np.full(m, np.inf)
    miss = np.zeros(m, dtype=bool)
    for a in range(3):
        da = d[:, a]
        oa = o[:, a]
        zero = da == 0.0
        miss |= zero & ((oa < lo[a]) | (oa > hi[a]))
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / np.where(zero, 1.0, da)
            t1 = (lo[a] - oa) * inv
            t2 = (hi[a] - oa) * inv
        t_near = np.where(zero, t_near, np.maximum(t_near, np.minimum(t1, t2)))
        t_far = np.where(zero, t_far, np.minimum(t_far, np.maximum(t1, t2)))
    miss |= t_near >= t_far
    return t_near, t_far, miss


def sample_counts(t_near, t_far, miss, dt: float, max_samples: int):
    """K per ray: min(floor((t_far - t_near)/dt), max_samples), 0 on a miss."""
    with np.errstate(invalid="ignore"):
        q = np.floor((t_far - t_near) / dt)
    q = np.where(miss, 0.0, np.minimum(q, float(max_samples)))
    return q.astype(np.int64)


def transfer(f: np.ndarray, tf: np.ndarray, vmin: float, vmax: float):
    """Piecewise-linear lookup in a 256-entry RGBA table."""
    tf = np.asarray(tf, dtype=np.float64)
    s = (f - float(vmin)) / (float(vmax) - float(vmin))
    s = np.minimum(np.maximum(s, 0.0), 1.0) * 255.0
    i0 = np.minimum(np.floor(s), 254.0).astype(np.int64)
    w = s - i0
    return (1.0 - w)[:, None] * tf[i0] + w[:, None] * tf[i0 + 1]


def phong(rgb: np.ndarray, g: np.ndarray, L: np.ndarray, ka, kd, ks, g0, m: int):
    """Headlight Phong on the non-premultiplied colour (two-sided)."""
    gn = np.sqrt((g * g).sum(axis=1))
    n = g / np.maximum(gn, float(g0))[:, None]
    diff = np.abs((n * L).sum(axis=1))
    spec = np.ones_like(diff)
    for _ in range(int(m)):
        spec = spec * diff
    return rgb * (float(ka) + float(kd) * diff)[:, None] + float(ks) * spec[:, None]


def render(field, box_lo, box_hi, cam: dict, params: dict, W: int, H: int,
           pixels=None, record_alpha: bool = False, k_range=None, region=None):
    """Ray-cast the field (callable x(m,3) -> (f (m,), grad (m,3))).

    Returns dict(rgba (m,4) premultiplied colour + opacity, K (m,) scheduled
    samples, used (m,) samples composited, alpha (m, Kmax) if recorded) for
    the m listed pixels (all pixels in row-major order by default).
    k_range=(k0,k1) composites only samples k0 <= k < k1 (for segment
    compositing; termination then disabled).

    region=(owner, blo, bhi, rlo, rhi): a partial render of the paper's
    object-space split (Sec. IV-A4: each node renders its own blocks to a
    partial image, composited afterwards by "over", Sec. IV-A5).  Reading:
    the model's sample schedule is kept and only samples whose owning block
    (owner(x) -> (m,3) block indices, D3) lies in the block box [blo, bhi)
    are composited; termination applies to the partial's own opacity.  The
    result also holds key (m,): the entry parameter of the ray into the
    region's world box [rlo, rhi] (slab test as above), +inf when the ray
    misses that box or the model box; partial images are composited in the
    order of their keys (regions are disjoint boxes, so along a ray the
    samples of each form one run, in key order).
    """
    lo = np.asarray(box_lo, dtype=np.float64)
    hi = np.asarray(box_hi, dtype=np.float64)
    o, d = pixel_rays(cam, W, H, pixels)
    m = o.shape[0]
    t_near, t_far, miss = slab(o, d, lo, hi)
    key = None
    if region is not None:
        owner, blo, bhi, rlo, rhi = region
        r_near, _, r_miss = slab(o, d, np.asarray(rlo, np.float64), np.asarray(rhi, np.float64))
    dt = float(params["step"])
    K = sample_counts(t_near, t_far, miss, dt, int(params["max_samples"]))
    L = -d / np.sqrt((d * d).sum(axis=1))[:, None]
    C = np.zeros((m, 3))
    A = np.zeros(m)
    used = np.zeros(m, dtype=np.int64)
    active = K > 0
    kmax = int(K.max()) if m else 0
    alpha_rec = np.zeros((m, max(kmax, 1)), dtype=np.float64) if record_alpha else None
    ert = float(params["ert_alpha"])
    k0, k1 = (0, kmax) if k_range is None else k_range
    use_ert = k_range is None
    if region is not None:
        key = np.where(r_miss | (K == 0), np.inf, r_near)
    for k in range(kmax):
        sel = np.nonzero(active & (k < K))[0]
        if len(sel) == 0:
            break
        if not (k0 <= k < k1):
            continue
        tk = t_near[sel] + (k + 0.5) * dt
        x = o[sel] + tk[:, None] * d[sel]
        if region is not None:
            b = owner(x)
            inr = np.all((b >= np.asarray(blo)) & (b < np.asarray(bhi)), axis=1)
            sel, x = sel[inr], x[inr]
            if len(sel) == 0:
                continue
        f, g = field(x)
        rgba = transfer(f, params["tf"], params["vmin"], params["vmax"])
        a = rgba[:, 3]
        c = phong(rgba[:, :3], g, L[sel], params["ka"], params["kd"], params["ks"],
                  params["g0"], params["shininess"])
        om = 1.0 - A[sel]
        C[sel] = C[sel] + (om * a)[:, None] * c
        A[sel] = A[sel] + om * a
        used[sel] = k + 1
        if record_alpha:
            alpha_rec[sel, k] = a
        if use_ert:
            stop = sel[A[sel] >= ert]
            active[stop] = False
    rgba_out = np.concatenate([C, A[:, None]], axis=1)
    out = dict(rgba=rgba_out, K=K, used=used, t_near=t_near, t_far=t_far, miss=miss)
    if key is not None:
        out["key"] = key
    if record_alpha:
        out["alpha"] = alpha_rec
    return out


def render_iso(field, box_lo, box_hi, cam: dict, params: dict, W: int, H: int, iso: float,
               rgb, pixels=None):
    """First-hit isosurface ray casting from the same value and gradient
    queries (the paper names isosurface rendering as another product of the
    MFA-VV step, Sec. IV-A4, without a method).  Reading taken: the volume
    renderer's ray schedule (same rays, slab, K, t_k); the side of a sample
    is f_k >= iso; the surface is hit between the first two consecutive
    samples k-1, k whose sides differ (k >= 1, either direction); the hit
    parameter is the linear interpolation of f between them,
        w = (iso - f_{k-1}) / (f_k - f_{k-1}),  t* = t_near + (k - 1/2 + w) dt,
    x* = o + t* d; the pixel is the Phong colour (the volume renderer's
    headlight shading, params ka, kd, ks, g0, shininess) of the surface
    colour rgb with the gradient at x*, opacity 1; no hit: (0, 0, 0, 0).

    Returns dict(rgba (m,4), depth (m,) t* (+inf without a hit), hit (m,)
    index k of the hit (-1 without), K (m,), fa, fb (m,) the values at the
    bracketing samples, margin (m,) the smallest |f_j - iso| over the
    samples j examined (those up to the hit, else all K), for the m listed
    pixels."""
    lo = np.asarray(box_lo, dtype=np.float64)
    hi = np.asarray(box_hi, dtype=np.float64)
    o, d = pixel_rays(cam, W, H, pixels)
    m = o.shape[0]
    t_near, t_far, miss = slab(o, d, lo, hi)
    dt = float(params["step"])
    K = sample_counts(t_near, t_far, miss, dt, int(params["max_samples"]))
    iso = float(iso)
    hit = np.full(m, -1, dtype=np.int64)
    fa = np.full(m, np.nan)
    fb = np.full(m, np.nan)
    margin = np.full(m, np.inf)
    prev_f = np.full(m, np.nan)
    active = K > 0
    kmax = int(K.max()) if m else 0
    for k in range(kmax):
        sel = np.nonzero(active & (k < K))[0]
        if len(sel) == 0:
            break
        tk = t_near[sel] + (k + 0.5) * dt
        f, _ = field(o[sel] + tk[:, None] * d[sel])
        margin[sel] = np.minimum(margin[sel], np.abs(f - iso))
        if k > 0:
            cross = (f >= iso) != (prev_f[sel] >= iso)
            c = sel[cross]
            hit[c] = k
            fa[c] = prev_f[c]
            fb[c] = f[cross]
            active[c] = False
        prev_f[sel] = f
    rgba = np.zeros((m, 4))
    depth = np.full(m, np.inf)
    h = np.nonzero(hit >= 0)[0]
    if len(h):
        w = (iso - fa[h]) / (fb[h] - fa[h])
        t = t_near[h] + ((hit[h] - 1) + 0.5 + w) * dt
        _, g = field(o[h] + t[:, None] * d[h])
        L = -d[h] / np.sqrt((d[h] * d[h]).sum(axis=1))[:, None]
        c = phong(np.tile(np.asarray(rgb, np.float64), (len(h), 1)), g, L, params["ka"],
                  params["kd"], params["ks"], params["g0"], params["shininess"])
        rgba[h, :3] = c
        rgba[h, 3] = 1.0
        depth[h] = t
    return dict(rgba=rgba, depth=depth, hit=hit, K=K, fa=fa, fb=fb, margin=margin)


def model_field(model):
    """Field callable for an MFA model (value + world gradient)."""
    from .bspline import evaluate

    def fn(x):
        r = evaluate(model, x)
        return r["f"], r["grad"]
    return fn


def over(front: np.ndarray, back: np.ndarray) -> np.ndarray:
    """Composite premultiplied RGBA 'front' over 'back' (Sec. IV-A5)."""
    af = front[..., 3:4]
    return front + (1.0 - af) * back


def composite(images, keys) -> np.ndarray:
    """Depth-ordered compositing of partial images (Sec. IV-A5): per pixel
    the partials in increasing key order (ties in list order), folded front
    to back with "over".  images: (G, m, 4), keys: (G, m)."""
    images = np.asarray(images, dtype=np.float64)
    keys = np.asarray(keys, dtype=np.float64)
    order = np.argsort(keys, axis=0, kind="stable")          # (G, m)
    m = images.shape[1]
    out = np.zeros((m, 4))
    cols = np.arange(m)
    for g in range(images.shape[0]):
        out = over(out, images[order[g], cols])
    return out


def block_owner_fn(model):
    """owner(x) -> (m,3) owning block per axis (D3) for region renders."""
    from .bspline import world_to_param

    def fn(x):
        bids, _, _ = world_to_param(model, x)
        return bids
    return fn


def ert_replay_f32(alpha: np.ndarray, K: np.ndarray, ert_alpha) -> np.ndarray:
    """Samples used per ray when A is accumulated in FP32 as
    om = 1 - A; t = om * alpha; A = A + t (each op rounded to FP32) and the
    ray stops after the first sample with A >= ert_alpha (FP32 compare).

    alpha: (m, Kmax) per-sample opacities as FP32; K: (m,) scheduled counts.
    """
    alpha = np.asarray(alpha, dtype=np.float32)
    K = np.asarray(K, dtype=np.int64)
    m = alpha.shape[0]
    A = np.zeros(m, dtype=np.float32)
    used = K.copy()
    active = K > 0
    one = np.float32(1.0)
    thr = np.float32(ert_alpha)
    for k in range(alpha.shape[1]):
        sel = active & (k < K)
        if not sel.any():
            break
        om = one - A[sel]
        t = om * alpha[sel, k]
        A[sel] = A[sel] + t
        hit = np.zeros(m, dtype=bool)
        hit[sel] = A[sel] >= thr
        used[hit] = k + 1
        active &= ~hit
    return used
