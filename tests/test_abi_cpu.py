"""CPU checks of the C ABI: the library loads, exports every function the
header declares, its host-only helpers agree bit for bit with the oracle's
independent definitions, and argument validation rejects bad calls before
any device work (no compute call is made here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import quant
from paper_2312_15073_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfa.h")

pytestmark = pytest.mark.skipif(not os.path.exists(L.LIB_PATH),
                                reason="libmfa.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfa_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert "mfa_render_frame" in names and "mfa_decode_points" in names
    lib = C.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in mfa.h but not exported"
    assert set(names) == set(L.SIGNATURES), "binding signatures out of sync with the header"


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_library_storage_rounding_matches_oracle_bits(dtype):
    import paper_2312_15073_amd as mfa
    rng = np.random.default_rng(21)
    x = np.concatenate([
        rng.standard_normal(50000) * 10.0 ** rng.integers(-9, 5, size=50000),
        np.array([0.0, -0.0, 1.0, 65504.0, 65519.0, 65520.0, 1e-8, 5.9604644775390625e-08,
                  2.98e-8, 1 + 2 ** -9, 1 + 3 * 2 ** -9, 1 + 2 ** -12, 1 + 3 * 2 ** -12,
                  3.0e38, -6.1e-5]),
        synth.model_c1().blocks[0].ctrl.reshape(-1),
    ])
    got = mfa.quantize(x, dtype)
    want = quant.stored_bits(x, dtype)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n,p", [(4, 3), (16, 3), (128, 3), (9, 2), (40, 5), (2, 1)])
def test_library_default_knots_equal_input_knots(n, p):
    import paper_2312_15073_amd as mfa
    np.testing.assert_array_equal(mfa.default_knots(n, p), synth.clamped_uniform_knots(n, p))


def _domain(grid=(1, 1, 1)):
    d = L.DomainDesc()
    for a in range(3):
        d.grid[a] = grid[a]
        d.lo[a] = 0.0
        d.hi[a] = 1.0
    d.voxel = 1.0 / 63
    return d


def _block(n=(8, 8, 8), p=3, ctrl=None):
    b = L.BlockDesc()
    for a in range(3):
        b.degree[a] = p
        b.n_ctrl[a] = n[a]
    if ctrl is None:
        ctrl = np.zeros(n)
    b.ctrl = ctrl.ctypes.data
    b.ctrl_dtype = L.MFA_F64
    return b, ctrl


def _create(dom, blocks, nb, storage=L.MFA_F32):
    h = C.c_void_p()
    arr = (L.BlockDesc * len(blocks))(*blocks)
    st = L.lib().mfa_model_create(C.byref(dom), arr, nb, storage, C.byref(h))
    return st, L.lib().mfa_last_error().decode()


def test_model_create_rejects_bad_arguments_before_device_work():
    lib = L.lib()
    b, keep = _block()
    st, msg = _create(_domain(), [b], 2)
    assert st == L.MFA_E_ARG and "nblocks" in msg
    d = _domain()
    d.hi[1] = 0.0
    assert _create(d, [b], 1)[0] == L.MFA_E_ARG
    d = _domain()
    d.voxel = 0.0
    assert _create(d, [b], 1)[0] == L.MFA_E_ARG
    assert _create(_domain(), [b], 1, storage=L.MFA_F64)[0] == L.MFA_E_ARG
    b2, k2 = _block(p=6)
    assert _create(_domain(), [b2], 1)[0] == L.MFA_E_UNSUPPORTED
    b3, k3 = _block(n=(3, 8, 8))
    st, msg = _create(_domain(), [b3], 1)
    assert st == L.MFA_E_ARG and "n_ctrl" in msg
    b4, k4 = _block()
    b4.degree[1] = 2
    assert _create(_domain(), [b4], 1)[0] == L.MFA_E_UNSUPPORTED
    b5, k5 = _block()
    b5.ctrl = None
    assert _create(_domain(), [b5], 1)[0] == L.MFA_E_ARG
    assert lib.mfa_model_create(None, None, 1, L.MFA_F32, None) == L.MFA_E_ARG


def test_null_model_calls_are_rejected():
    lib = L.lib()
    assert lib.mfa_decode_points(None, None, 10, 0, None, None, None) == L.MFA_E_ARG
    assert lib.mfa_decode_points_noalloc(None, None, 10, 0, None, None, None) == L.MFA_E_ARG
    assert lib.mfa_decode_grid(None, None, None, 0, None, None, None) == L.MFA_E_ARG
    assert lib.mfa_render_frame(None, None, None, 4, 4, None, None, None) == L.MFA_E_ARG
    assert lib.mfa_model_info(None, None) == L.MFA_E_ARG
    assert lib.mfa_model_destroy(None) == L.MFA_OK
    assert lib.mfa_quantize(None, 5, L.MFA_F32, None) == L.MFA_E_ARG
    assert lib.mfa_default_knots(2, 3, None) == L.MFA_E_ARG
    assert "mfa-gfx950" in lib.mfa_version().decode()


def _i3(*v):
    return (C.c_int32 * 3)(*v)


def test_encode_workspace_size_and_rejections():
    lib = L.lib()
    nb = C.c_int64()
    assert lib.mfa_encode_workspace(_i3(10, 12, 14), _i3(5, 6, 7), C.byref(nb)) == L.MFA_OK
    al = lambda v: (v + 255) // 256 * 256
    # few fibers (12 x 14): three GEMMs, tables B_a+ (FP64) and the two
    # intermediates
    want = sum(al(8 * n * r) for n, r in ((5, 10), (6, 12), (7, 14))) \
        + al(8 * 5 * 12 * 14) + al(8 * 5 * 6 * 14)
    assert nb.value == want
    # 2^17 fibers (512 x 256) and 90 control points from 300 samples along
    # axis 0: the banded route, its tables (sample order and supports, int32;
    # basis values, 8 per sample; factor rows, 8 per control point;
    # reciprocal diagonal; degree) instead of B0+
    assert lib.mfa_encode_workspace(_i3(300, 512, 256), _i3(90, 6, 7), C.byref(nb)) == L.MFA_OK
    want = al(4 * 300) + al(4 * 300) + al(8 * 300 * 8) + al(8 * 90 * 8) + al(8 * 90) + 256 \
        + sum(al(8 * n * r) for n, r in ((6, 512), (7, 256))) \
        + al(8 * 90 * 512 * 256) + al(8 * 90 * 6 * 256)
    assert nb.value == want
    # the same fibers with 20 control points along axis 0: the dense product
    assert lib.mfa_encode_workspace(_i3(300, 512, 256), _i3(20, 6, 7), C.byref(nb)) == L.MFA_OK
    want = sum(al(8 * n * r) for n, r in ((20, 300), (6, 512), (7, 256))) \
        + al(8 * 20 * 512 * 256) + al(8 * 20 * 6 * 256)
    assert nb.value == want
    assert lib.mfa_encode_workspace(_i3(4, 12, 14), _i3(5, 6, 7), C.byref(nb)) == L.MFA_E_ARG
    assert lib.mfa_encode_workspace(_i3(10, 12, 14), _i3(5, 6, 7), None) == L.MFA_E_ARG


def test_encode_rejects_bad_arguments_before_device_work():
    """Every call here fails validation on the host, so the fake device
    pointers are never used."""
    lib = L.lib()
    res, nc = (10, 9, 8), (5, 5, 6)
    tabs = [np.linspace(0.0, 1.0, r) for r in res]
    fake = C.c_void_p(0x1000)

    def call(tabs=tabs, degree=(3, 3, 3), nc=nc, res=res, knots=None, work_bytes=1 << 30):
        ptrs = (C.c_void_p * 3)(*[t.ctypes.data for t in tabs])
        kn = None if knots is None else (C.c_void_p * 3)(*[k.ctypes.data for k in knots])
        st = lib.mfa_encode_grid(_i3(*res), ptrs, fake, _i3(*degree), _i3(*nc), kn, fake, fake,
                                 work_bytes, None)
        return st, lib.mfa_last_error().decode()

    assert call(degree=(0, 3, 3))[0] == L.MFA_E_ARG
    assert call(nc=(11, 5, 6))[0] == L.MFA_E_ARG                        # res < n_ctrl
    assert call(work_bytes=16)[0] == L.MFA_E_ARG
    bad = [t.copy() for t in tabs]
    bad[1][3] = 1.5
    st, msg = call(tabs=bad)
    assert st == L.MFA_E_ARG and "outside [0, 1]" in msg
    bad = [t.copy() for t in tabs]
    bad[2][:] = 0.5                                                     # every sample in one span
    st, msg = call(tabs=bad)
    assert st == L.MFA_E_ARG and "dependent columns" in msg
    k = [synth.clamped_uniform_knots(n, 3) for n in nc]
    k[0] = k[0][::-1].copy()                                            # decreasing knots
    assert call(knots=k)[0] == L.MFA_E_ARG
    assert lib.mfa_encode_grid(None, None, None, None, None, None, None, None, 0, None) == L.MFA_E_ARG


def test_encode_adaptive_workspace_size_and_rejections():
    lib = L.lib()
    nb = C.c_int64()
    (N0, N1, N2), (m0, m1, m2) = (10, 12, 700), (5, 6, 7)
    assert lib.mfa_encode_adaptive_workspace(_i3(N0, N1, N2), _i3(m0, m1, m2),
                                             C.byref(nb)) == L.MFA_OK
    al = lambda v: (v + 255) // 256 * 256
    want = 2 * sum(al(8 * n * r) for n, r in ((m0, N0), (m1, N1), (m2, N2)))
    M, up = N0 * N1, (lambda v, d: (v + d - 1) // d)
    tm, tn = up(M, 32), up(N2, 32)                           # 32 x 32 tiles of the error GEMM
    red = max(up(tm, 64) * N2, up(tn, 64) * M if tn > 64 else 0, up(N0, 64) * N1)
    want += al(8 * m0 * N1 * N2) + al(8 * N2 * m0 * m1) + al(8 * N0 * m1 * m2) + al(8 * m2 * M) \
        + al(8 * tn * M) + al(8 * tm * N2) + al(8 * M) + 2 * al(8 * red) \
        + al(8 * (N0 + N1 + N2)) + al(8 * 2048) + al(8 * min(1 << 21, 8 * m0 * m1 * N2)) \
        + al(8 * (N0 + N1 + N2)) + al(8 * (m0 + m1 + m2 + 3 * 8 + 8 * (m0 + m1 + m2))) \
        + al(8 * (m0 * m0 + m1 * m1 + m2 * m2)) + al(8)
    assert nb.value == want
    assert lib.mfa_encode_adaptive_workspace(_i3(4, 12, 14), _i3(5, 6, 7), C.byref(nb)) == L.MFA_E_ARG

    res, tabs = (10, 9, 8), [np.linspace(0.0, 1.0, r) for r in (10, 9, 8)]
    fake = C.c_void_p(0x1000)
    kout = [np.zeros(20) for _ in range(3)]

    def call(degree=(3, 3, 3), n_init=(4, 4, 5), max_ctrl=(8, 8, 8), e_max=1e-3, max_fits=5,
             cap=512, work_bytes=1 << 30, tabs=tabs):
        st = lib.mfa_encode_adaptive(
            _i3(*res), (C.c_void_p * 3)(*[t.ctypes.data for t in tabs]), fake, _i3(*degree),
            _i3(*n_init), _i3(*max_ctrl), e_max, max_fits,
            (C.c_void_p * 3)(*[k.ctypes.data for k in kout]), (C.c_int32 * 3)(), fake, cap, None,
            C.byref(C.c_int32()), fake, work_bytes, None)
        return st, lib.mfa_last_error().decode()

    assert call(n_init=(3, 4, 5))[0] == L.MFA_E_ARG                     # n_init < p + 1
    assert call(max_ctrl=(8, 8, 9))[0] == L.MFA_E_ARG                   # max_ctrl > res
    assert call(n_init=(4, 9, 5), max_ctrl=(8, 8, 8))[0] == L.MFA_E_ARG  # n_init > max_ctrl
    assert call(e_max=0.0)[0] == L.MFA_E_ARG
    assert call(e_max=float("nan"))[0] == L.MFA_E_ARG
    assert call(max_fits=0)[0] == L.MFA_E_ARG
    assert call(cap=511)[0] == L.MFA_E_ARG
    assert call(work_bytes=16)[0] == L.MFA_E_ARG
    bad = [t.copy() for t in tabs]
    bad[0][2] = -0.25
    st, msg = call(tabs=bad)
    assert st == L.MFA_E_ARG and "outside [0, 1]" in msg


def test_render_volume_rejects_bad_arguments_before_device_work():
    lib = L.lib()
    cam = L.Camera()
    cam.kind = 1
    for a in range(3):
        cam.eye[a], cam.forward[a], cam.right[a], cam.up[a] = 0.5, float(a == 2), float(a == 0), float(a == 1)
    cam.sx = cam.sy = 0.01
    rp = L.RenderParams()
    rp.tf_rgba = 0x1000
    rp.vmin, rp.vmax, rp.step, rp.max_samples, rp.ert_alpha = 0.0, 1.0, 0.01, 64, 0.99
    rp.ka, rp.kd, rp.ks, rp.g0, rp.shininess = 0.3, 0.6, 0.3, 0.01, 16

    def call(kind=0, dims=(8, 8, 8), lo=(0, 0, 0), hi=(1, 1, 1), samples=0x1000, w=8):
        d = L.VolumeDesc()
        d.samples, d.kind = samples, kind
        for a in range(3):
            d.dims[a], d.lo[a], d.hi[a] = dims[a], lo[a], hi[a]
        return lib.mfa_render_volume(C.byref(d), C.byref(cam), C.byref(rp), w, 8, C.c_void_p(0x1000),
                                     None, None)

    assert call(kind=4) == L.MFA_E_ARG
    assert call(kind=-1) == L.MFA_E_ARG
    assert call(dims=(8, 1, 8)) == L.MFA_E_ARG
    assert call(lo=(0, 1, 0)) == L.MFA_E_ARG                       # lo >= hi on axis 1
    assert call(hi=(1, float("inf"), 1)) == L.MFA_E_ARG
    assert call(samples=None) == L.MFA_E_ARG                       # a filter needs samples
    assert call(w=0) == L.MFA_E_ARG
    assert lib.mfa_render_volume(None, C.byref(cam), C.byref(rp), 8, 8, C.c_void_p(0x1000), None,
                                 None) == L.MFA_E_ARG
