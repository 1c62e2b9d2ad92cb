"""The FP32 running sum of the Taylor terms, emulated on the CPU.

The FP32 sweeps add the Taylor terms of a sub-step into the running sum two
at a time, acc <- (acc + y_{j-1}) + y_j, with plain FP32 additions and no
compensation term.  This file backs that choice with an emulation in NumPy
float32 of the same recurrence (section 2.2: y_1 = h (A x + b),
y_j = (h/j) A y_{j-1}, x <- x + sum_j y_j) at the widest scaled step the FP32
plan allows, theta = h ||A||_1 = ln 64, where the Taylor terms reach
theta^4/4! ~ 12.5 times the input while the result of a rough input is about
1/64 of it (10 bits of cancellation):

* on the roughest vector a uniform grid carries (the top no-flux eigenmode)
  and on uniform noise, the FP32 error stays about 1e-6 of the input;
* a Kahan-compensated running sum leaves the error where it was (within a few
  per cent): it is the rounding of the terms themselves, which compensation
  cannot reach, so a compensation field (8 more bytes per voxel and flush
  sweep) would buy nothing.

Smooth data, as in the workloads, loses far less (the GPU's FP32 run of the
128^3 head ends 1.1e-7 from the FP64 oracle after 100 steps).
"""

import math

import numpy as np


def lap32(u, d):
    """7-point no-flux Laplacian times d, in float32 arithmetic."""
    out = np.zeros_like(u)
    for ax in range(3):
        df = np.diff(u, axis=ax)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        out[tuple(lo)] += df
        out[tuple(hi)] -= df
    return (d * out).astype(np.float32)


def substep(x, b, h, m, d, dtype, compensated=False):
    """One sub-step of the augmented Taylor recurrence in `dtype` with the
    sweeps' running sum: acc = x + y_1 from the first term; a term either
    waits (skip) or adds the waiting term and itself, (acc + y_{j-1}) + y_j,
    left to right; the last term always adds.  Optionally Kahan-compensated."""
    hh = dtype(h)
    A = (lambda v: lap32(v, np.float32(d))) if dtype == np.float32 else (lambda v: d * lap64(v))
    comp = np.zeros_like(x)

    def add(acc, t):
        nonlocal comp
        if not compensated:
            return (acc + t).astype(dtype)
        yk = (t - comp).astype(dtype)
        tk = (acc + yk).astype(dtype)
        comp = ((tk - acc) - yk).astype(dtype)
        return tk

    y = (hh * (A(x) + b)).astype(dtype)
    acc = add(x.copy(), y)
    pend = None
    for j in range(2, m + 1):
        y = ((hh / dtype(j)) * A(y)).astype(dtype)
        if pend is None and j != m:
            pend = y
            continue
        if pend is not None:
            acc = add(acc, pend)
        acc = add(acc, y)
        pend = None
    return acc


def lap64(u):
    out = np.zeros_like(u)
    for ax in range(3):
        df = np.diff(u, axis=ax)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        out[tuple(lo)] += df
        out[tuple(hi)] -= df
    return out


def truncation_ok(theta, m, tol):
    return theta ** (m + 1) / math.factorial(m + 1) <= tol


def _widest_fp32_substep(v, d=0.13):
    theta = math.log(64.0)
    h = theta / (12.0 * d)  # ||A||_1 = 12 d at h = 1: twice the largest diagonal
    m = next(k for k in range(1, 61) if truncation_ok(theta, k, 1e-6))
    z = np.zeros_like(v)
    x64 = substep(v.copy(), z, h, m, d, np.float64)
    v32, z32 = v.astype(np.float32), z.astype(np.float32)
    x32 = substep(v32, z32, h, m, d, np.float32)
    x32k = substep(v32, z32, h, m, d, np.float32, compensated=True)
    scale = np.linalg.norm(v)
    return x64, np.linalg.norm(x32 - x64) / scale, np.linalg.norm(x32k - x64) / scale


def test_rough_inputs_at_widest_fp32_step():
    n = 24
    i = np.arange(n)
    mode = np.cos(np.pi * (n - 1) * (i + 0.5) / n)  # top no-flux DCT-II mode
    top = mode[:, None, None] * mode[None, :, None] * mode[None, None, :]
    noise = np.random.default_rng(0).uniform(-1.0, 1.0, (n, n, n))
    for v, shrink in ((top, 1.0 / 50), (noise, 0.5)):
        x64, e, ek = _widest_fp32_substep(v)
        assert np.linalg.norm(x64) / np.linalg.norm(v) < shrink  # strongly damped: heavy cancellation
        assert e < 2e-6
        assert ek > 0.9 * e  # compensation does not reduce it


def test_smooth_field_several_substeps():
    # a blob, s = 3 sub-steps of theta = ln 64 each, source b = 0: the error
    # of the uncompensated FP32 sum stays near the FP32 unit roundoff
    n, d = 24, 0.13
    c = (n - 1) / 2
    g = np.exp(-((np.arange(n) - c) ** 2) / 18.0)
    v = g[:, None, None] * g[None, :, None] * g[None, None, :]
    theta = math.log(64.0)
    h = theta / (12.0 * d)
    m = next(k for k in range(1, 61) if truncation_ok(theta, k, 1e-6))
    x64, x32 = v.copy(), v.astype(np.float32)
    z64, z32 = np.zeros_like(v), np.zeros_like(x32)
    for _ in range(3):
        x64 = substep(x64, z64, h, m, d, np.float64)
        x32 = substep(x32, z32, h, m, d, np.float32)
    assert np.linalg.norm(x32 - x64) / np.linalg.norm(x64) < 1e-6
