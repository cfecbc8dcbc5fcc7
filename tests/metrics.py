"""Error metrics shared by the parity tests and the benchmark (no method arithmetic).

The headline metric is peak-normalised per transition:
    err_s = max_q | |f_s|^2_test - |f_s|^2_ref | / max_q |f_s|^2_ref,
because the per-point relative error of |f|^2 is unbounded near the zeros of
f.  The complex error max|f_test - f_ref| / max|f_ref| and the per-point
relative error where |f_ref|^2 >= 1e-3 peak are reported beside it.
"""
import numpy as np

TOL_F2 = {"fp32": 1e-6, "bf16x3": 1e-4}
# FFT method against the oracle's FFT method on the same grid (FP32 density
# and FP32 radix-2 transforms)
TOL_FFT = 1e-6
# split-BF16 density contraction: three products of 8-bit halves (about
# 2^-16 relative each, over sums of a few hundred terms)
TOL_FFT_BF16 = 1e-4

# Error lines recorded by the GPU tests, printed in the terminal summary of
# the run (so the error of every transition is visible without -s).
REPORT = []


def report(line: str):
    REPORT.append(line)
    print(line, flush=True)


def errors(f_test, f_ref):
    """f_*: complex [n_states, ...].  Returns dict of per-state arrays."""
    ns = f_ref.shape[0]
    ft = f_test.reshape(ns, -1).astype(np.complex128)
    fr = f_ref.reshape(ns, -1).astype(np.complex128)
    a2t, a2r = np.abs(ft) ** 2, np.abs(fr) ** 2
    peak2 = a2r.max(axis=1)
    peak = np.abs(fr).max(axis=1)
    e_f2 = np.abs(a2t - a2r).max(axis=1) / peak2
    e_c = np.abs(ft - fr).max(axis=1) / peak
    big = a2r >= 1e-3 * peak2[:, None]
    rel = np.where(big, np.abs(a2t - a2r) / np.maximum(a2r, 1e-300), 0.0).max(axis=1)
    return {"f2_peak_norm": e_f2, "complex": e_c, "f2_rel_big": rel}
