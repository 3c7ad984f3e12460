"""Shared helpers of the GPU parity tests: tolerances and comparisons.

Tolerance (values and gradients, FP32 arithmetic against the FP64 oracle):
normwise, |df| <= 1e-5 * max|P| and |d grad| <= 1e-5 * G with G the largest
|component| of the reference gradient over the evaluated set.  Integer
outputs (spans, blocks, sample counts) must be equal.
"""
import sys

import numpy as np

REL = 1e-5


def announce(msg: str) -> None:
    """Names the case on the real stderr before a GPU step (survives a
    crash of the process, unlike pytest's captured output)."""
    sys.__stderr__.write(f"[gpu] {msg}\n")
    sys.__stderr__.flush()


def assert_values_close(got: np.ndarray, f_ref: np.ndarray, g_ref: np.ndarray, pmax: float,
                        rel: float = REL, extra_f: float = 0.0, extra_g: float = 0.0):
    """got (m,4) float32 vs reference value (m,) and gradient (m,3)."""
    got = np.asarray(got, dtype=np.float64)
    G = float(np.max(np.abs(g_ref))) if g_ref.size else 0.0
    df = np.max(np.abs(got[:, 0] - f_ref)) if len(f_ref) else 0.0
    dg = np.max(np.abs(got[:, 1:] - g_ref)) if len(f_ref) else 0.0
    tf = rel * pmax + extra_f
    tg = rel * G + extra_g
    assert df <= tf, f"value error {df:.3e} > {tf:.3e} (max|P| {pmax:.3e})"
    assert dg <= tg, f"gradient error {dg:.3e} > {tg:.3e} (G {G:.3e})"
    return df / max(pmax, 1e-300), dg / max(G, 1e-300)


def composite_band(alpha64: np.ndarray, used: np.ndarray, ert: float, delta: float = 1e-5):
    """Rays whose FP64 opacity passes within delta of the threshold at any
    sample up to the decision (their FP32 decision may legitimately differ)."""
    m, kmax = alpha64.shape
    A = np.zeros(m)
    band = np.zeros(m, dtype=bool)
    for k in range(kmax):
        live = k < used
        if not live.any():
            break
        A = np.where(live, A + (1.0 - A) * alpha64[:, k], A)
        band |= live & (np.abs(A - ert) <= delta)
    return band
