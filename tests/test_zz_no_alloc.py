"""The allocation-free sorted decode (mfa_decode_points_noalloc) against the
sorted decode with model-held scratch (mfa_decode_points with
MFA_DECODE_SORTED), through the C ABI: two calls in a row, the second with
a smaller input (the static scratch keeps the first call's contents), value
and gradient and value-only, single-block and multi-block models; results
bit for bit equal, and the oracle's within the FP32 tolerance.  Sizes above
the static scratch are rejected before any device work."""
import numpy as np
import pytest

import synth
from oracle import bspline as ob
from paper_2312_15073_amd import _lib as L
from tests.gpu_common import announce, assert_values_close

pytestmark = pytest.mark.gpu


def _multiblock():
    rng = np.random.default_rng(80)
    field = synth.field_c1(80)
    edges = [np.array([0.0, 0.4, 1.0]), np.array([0.0, 0.7, 1.0]), np.array([0.0, 0.5, 1.0])]
    blocks = []
    for b0 in range(2):
        for b1 in range(2):
            for b2 in range(2):
                n = [int(v) for v in rng.integers(5, 30, size=3)]
                knots = [synth.clamped_uniform_knots(n[a], 3) for a in range(3)]
                lo = np.array([edges[0][b0], edges[1][b1], edges[2][b2]])
                hi = np.array([edges[0][b0 + 1], edges[1][b1 + 1], edges[2][b2 + 1]])
                xs = [lo[a] + synth.greville(knots[a], 3, n[a]) * (hi[a] - lo[a]) for a in range(3)]
                blocks.append(synth.BlockSpec([3] * 3, knots, field.value_separable(*xs)))
    return synth.ModelSpec([2, 2, 2], np.zeros(3), np.ones(3), edges, blocks, voxel=1.0 / 63)


@pytest.mark.parametrize("which", ["c1", "c2", "multiblock", "c4"])
def test_noalloc_sorted_decode_equals_sorted_decode(dev, which):
    """c4 (the 8x8x8-block model, more than 1024 buckets) takes the
    two-level sort, 36 bytes of scratch per point."""
    import torch
    import paper_2312_15073_amd as mfa
    spec = {"c1": synth.model_c1, "c2": synth.model_c2, "multiblock": _multiblock,
            "c4": synth.model_c4}[which]()
    pmax = max(np.abs(b.ctrl).max() for b in spec.blocks)
    with mfa.Model(spec, "f32") as M:
        for k, n in enumerate((1_500_000, 40_001)):        # second call smaller
            pts = synth.random_points(n, seed=90 + k, lo=(-0.05,) * 3, hi=(1.05,) * 3)
            x = torch.as_tensor(pts, device=dev)
            announce(f"noalloc {which} call {k} n={n}")
            for value_only in (False, True):
                want = mfa.decode_points(M, x, sorted_order=True, value_only=value_only)
                got = torch.full_like(want, -7.0)
                flags = L.MFA_DECODE_SORTED | (L.MFA_DECODE_VALUE if value_only else 0)
                st = L.lib().mfa_decode_points_noalloc(M.handle, x.data_ptr(), n, flags,
                                                       got.data_ptr(), None,
                                                       torch.cuda.current_stream().cuda_stream)
                assert st == L.MFA_OK, L.lib().mfa_last_error().decode()
                torch.cuda.synchronize()
                g, w = got.cpu().numpy(), want.cpu().numpy()
                np.testing.assert_array_equal(g.view(np.uint32), w.view(np.uint32))
            sel = np.arange(0, n, 97)
            ref = ob.evaluate(spec, pts[:, sel].T.astype(np.float64))
            full = mfa.decode_points(M, x, noalloc=True).cpu().numpy()[sel]
            assert_values_close(full, ref["f"], ref["grad"], pmax)


def test_noalloc_rejects_sizes_beyond_the_static_scratch(dev):
    import torch
    import paper_2312_15073_amd as mfa
    with mfa.Model(synth.model_c2(), "f32") as M:
        n = 5_000_000                      # 16 bytes per point (512 buckets, one level): > 64 MiB
        x = torch.zeros((3, n), dtype=torch.float32, device=dev)
        out = torch.zeros((n, 4), dtype=torch.float32, device=dev)
        st = L.lib().mfa_decode_points_noalloc(M.handle, x.data_ptr(), n, L.MFA_DECODE_SORTED,
                                               out.data_ptr(), None, None)
        assert st == L.MFA_E_ARG
        assert "at most" in L.lib().mfa_last_error().decode()
        assert float(out.abs().max()) == 0.0     # nothing was enqueued
