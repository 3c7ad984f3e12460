"""FP64 CPU oracle for the MFA evaluator and ray-caster.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
reference of what the GPU library computes.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import it; the GPU library never
calls it, and it shares no code with the GPU library.

Contents
--------
bspline  model evaluation: parameter map, knot span, Cox-de Boor basis and
         first derivatives, direct (p+1)^3 tensor sum, world gradient.
render   ray generation, slab test, sample schedule, transfer function,
         Phong shading, front-to-back "over" and early ray termination.
quant    storage rounding FP64 -> FP32 -> BF16 / FP16 (bit level).
metrics  MSE, RMSE, 8-bit PSNR, compression ratio.
encode   fixed-knot least-squares encoding of samples on a tensor grid
         (collocation matrices, per-axis pseudo-inverses, mode products).

Every function cites the passage of the paper it follows.  The paper gives
the model as a tensor product of B-spline functions with control points and
knots (Sec. III-A) and the renderer as ray casting with the "over" operator
(Sec. IV-A4, IV-A5); where it is silent the reading taken is stated at the
function (spline definitions follow de Boor's text, which the paper cites).

Parity status: every function here is pinned by the CPU tests (partition of
unity, polynomial reproduction, scipy agreement, finite differences, closed
forms, brute force on tiny inputs, library conversions, the paper's printed
PSNR and compression-ratio values) except the early-termination decision for
rays whose accumulated opacity lies within 1e-5 of the threshold, which is
"parity unpinned" (an FP64 reference cannot decide it for an FP32 kernel; the
FP32 replay in ``render.ert_replay_f32`` covers it instead).
"""
from . import bspline, render, quant, metrics, encode  # noqa: F401
