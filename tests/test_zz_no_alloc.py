"""The allocation-free tumour size (expint_tumour_size_static) against the
context entry point expint_tumour_size, through the C ABI: two calls in a
row on one device, the second on a smaller grid, in both dtypes."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2402_02273_amd import _native as N
from workloads import c2_head, make_head

DEV = "cuda:0"


def static_size(u, threshold):
    L = N.lib()
    d2 = ctypes.c_int64()
    pair = (ctypes.c_int64 * 2)()
    dt = N.F64 if u.dtype == torch.float64 else N.F32
    nx, ny, nz = u.shape
    rc = L.expint_tumour_size_static(ctypes.c_void_p(u.data_ptr()), dt, nx, ny, nz, float(threshold),
                                     ctypes.byref(d2), pair, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == N.OK, N.last_error()
    return int(d2.value), (int(pair[0]), int(pair[1]))


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_static_tumour_size_matches_context_entry(native, dtype):
    from paper_2402_02273_amd.expint import ExpInt

    cases = []
    big = c2_head()  # 128^3, then a 48^3 head: the second call is smaller
    small = make_head(48, seed=5)
    for labels, class_D, u0, steps in ((big.labels, big.class_D, big.u0, 6), (small.labels, (0.0, 0.13, 0.013),
                                                                             small.u0, 3)):
        print(f"[case] static tumour size {labels.shape} {dtype}", flush=True)
        ctx = ExpInt(labels.shape, labels=labels, class_D=class_D, rho=0.025, tau=7.3, dtype=dtype, device=DEV)
        u = torch.as_tensor(u0, dtype=dtype, device=DEV).contiguous()
        ctx.advance(u, steps)
        torch.cuda.synchronize()
        for thr in (1e-3, 0.3):
            want = ctx.tumour_size(u, thr)
            got = static_size(u, thr)
            cases.append((labels.shape, thr, want, got))
            assert got == want, (labels.shape, thr, got, want)
        ctx.close()
    # an empty set and a single point on the smaller grid, after the big call
    z = torch.zeros((7, 9, 11), dtype=dtype, device=DEV)
    assert static_size(z, 0.5) == (-1, (-1, -1))
    z[3, 4, 5] = 1.0
    assert static_size(z, 0.5) == (0, (3 * 99 + 4 * 11 + 5,) * 2)
    print(f"[result] {cases}", flush=True)


def test_static_tumour_size_rejects_oversize_grids():
    # 363^3 needs more than the static workspace: refused before any HIP call
    L = N.lib()
    d2 = ctypes.c_int64()
    rc = L.expint_tumour_size_static(ctypes.c_void_p(1), N.F32, 363, 363, 363, 0.5, ctypes.byref(d2), None, None)
    assert rc == N.EINVAL
    assert "static workspace" in N.last_error()
    rc = L.expint_tumour_size_static(ctypes.c_void_p(1), N.F32, 362, 362, 362, float("nan"), ctypes.byref(d2), None,
                                     None)
    assert rc == N.EINVAL and "NaN" in N.last_error()
