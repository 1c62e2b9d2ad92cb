"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, and rejects invalid arguments before touching HIP."""

import ctypes

import pytest

from paper_2402_02273_amd import _native as N


def test_library_exports_every_declared_function():
    L = N.lib()
    declared = N.header_functions()
    assert len(declared) >= 20
    missing = [f for f in declared if not hasattr(L, f)]
    assert not missing, missing
    # and the binding knows a signature for each of them
    assert sorted(N.SIGNATURES) == declared


def test_opts_default_and_null():
    L = N.lib()
    o = N.Opts()
    assert L.expint_opts_default(ctypes.byref(o)) == N.OK
    assert o.dtype == N.F32 and o.tau == pytest.approx(7.3) and o.s == 0 and o.m == 0
    assert L.expint_opts_default(None) == N.EINVAL
    assert "NULL" in N.last_error()


def _create(grid, df, rho=0.025, bc=N.NOFLUX, **kw):
    L = N.lib()
    o = N.Opts()
    L.expint_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    ctx = ctypes.c_void_p()
    rc = L.expint_create(ctypes.byref(grid) if grid is not None else None, ctypes.byref(df) if df is not None else None,
                         rho, bc, ctypes.byref(o), ctypes.byref(ctx))
    return rc, ctx


def _labels_df():
    cd = (ctypes.c_double * 3)(0.0, 0.13, 0.013)
    df = N.DField()
    df.labels = 1234  # never dereferenced: validation fails first
    df.n_classes = 3
    df.class_D = ctypes.cast(cd, ctypes.POINTER(ctypes.c_double))
    return df, cd


@pytest.mark.parametrize(
    "change,needle",
    [
        (lambda g, d, o: g.__setattr__("nx", 0), "dims"),
        (lambda g, d, o: g.__setattr__("h", -1.0), "h must"),
        (lambda g, d, o: o.__setitem__("tau", 0.0), "tau"),
        (lambda g, d, o: o.__setitem__("tau", float("nan")), "tau"),
        (lambda g, d, o: o.__setitem__("s", 3), "s and m"),
        (lambda g, d, o: o.__setitem__("m", 61) or o.__setitem__("s", 1), "m must"),
        (lambda g, d, o: d.__setattr__("n_classes", 9), "n_classes"),
        (lambda g, d, o: d.__setattr__("n_classes", 0), "n_classes"),
        (lambda g, d, o: d.__setattr__("D", 99), "exactly one"),
        (lambda g, d, o: o.__setitem__("dtype", 7), "dtype"),
        (lambda g, d, o: o.__setitem__("sweeps", 3), "sweeps"),
        (lambda g, d, o: o.__setitem__("scheme", 3), "scheme"),
    ],
)
def test_create_rejects_invalid_arguments(change, needle):
    grid = N.Grid(4, 4, 4, 1.0)
    df, cd = _labels_df()
    opts = {}
    change(grid, df, opts)
    rc, ctx = _create(grid, df, **opts)
    assert rc == N.EINVAL
    assert ctx.value is None
    assert needle in N.last_error()


def test_create_rejects_bad_class_D_and_rho():
    grid = N.Grid(4, 4, 4, 1.0)
    df, cd = _labels_df()
    cd[1] = -0.1
    assert _create(grid, df)[0] == N.EINVAL and "class_D[1]" in N.last_error()
    cd[1] = float("inf")
    assert _create(grid, df)[0] == N.EINVAL
    cd[1] = 0.13
    assert _create(grid, df, rho=-1.0)[0] == N.EINVAL and "rho" in N.last_error()
    assert _create(None, df)[0] == N.EINVAL


def test_unsupported_modal_requests_rejected_before_hip():
    df, cd = _labels_df()
    rc, _ = _create(N.Grid(32, 32, 32, 1.0), df, algo=N.ALGO_MODAL, mp=N.MP_BF16_SPLIT, dtype=N.F64)
    assert rc == N.EUNSUPPORTED and "FP32" in N.last_error()
    rc, _ = _create(N.Grid(32, 32, 40, 1.0), df, algo=N.ALGO_MODAL)
    assert rc == N.EUNSUPPORTED and "multiple of 32" in N.last_error()
    rc, _ = _create(N.Grid(32, 32, 32, 1.0), df, mp=N.MP_FP16_SPLIT)
    assert rc == N.EUNSUPPORTED and "modal" in N.last_error()


def test_pair_sweeps_need_label_form():
    df = N.DField()
    df.D = 1234  # never dereferenced: rejected first
    rc, _ = _create(N.Grid(8, 8, 8, 1.0), df, sweeps=N.SWEEPS_PAIRS)
    assert rc == N.EUNSUPPORTED and "label form" in N.last_error()


def test_scheme_limits_rejected_before_hip():
    df, cd = _labels_df()
    lin = N.SCHEME_LINEARISED
    rc, _ = _create(N.Grid(32, 32, 32, 1.0), df, algo=N.ALGO_MODAL, scheme=lin)
    assert rc == N.EUNSUPPORTED and "separable" in N.last_error()
    rc, _ = _create(N.Grid(8, 8, 8, 1.0), df, sweeps=N.SWEEPS_PAIRS, scheme=lin)
    assert rc == N.EUNSUPPORTED and "single-term" in N.last_error()
    rc, _ = _create(N.Grid(32, 32, 32, 1.0), df, algo=N.ALGO_MODAL, scheme=N.SCHEME_EXPRK2)
    assert rc == N.EUNSUPPORTED and "stencil-Taylor" in N.last_error()
    rc, _ = _create(N.Grid(8, 8, 8, 1.0), df, sweeps=N.SWEEPS_PAIRS, scheme=N.SCHEME_EXPRK2)
    assert rc == N.EUNSUPPORTED and "single-term" in N.last_error()
    L = N.lib()
    o = N.Opts()
    L.expint_opts_default(ctypes.byref(o))
    assert o.scheme == N.SCHEME_EXP_EULER
    grids = (N.Grid * 1)(N.Grid(8, 8, 8, 1.0))
    dfs = (N.DField * 1)(df)
    rho = (ctypes.c_double * 1)(0.025)
    b = ctypes.c_void_p()
    o.scheme = N.SCHEME_EXPRK2
    assert L.expint_batch_create(1, grids, dfs, rho, N.NOFLUX, ctypes.byref(o), ctypes.byref(b)) == N.EUNSUPPORTED
    assert "LINEARISED" in N.last_error()


def test_null_context_calls():
    L = N.lib()
    assert L.expint_phi1_lin(None, None, None, None) == N.EINVAL
    assert L.expint_phi12(None, None, None, None) == N.EINVAL
    assert L.expint_step(None, None) == N.EINVAL
    assert L.expint_advance(None, None, 1) == N.EINVAL
    assert L.expint_get_plan(None, None, None, None) == N.EINVAL
    assert L.expint_get_launch(None, None) == N.EINVAL
    L.expint_destroy(None)  # NULL-safe
    L.expint_batch_destroy(None)


def test_probes_reject_bad_arguments():
    L = N.lib()
    ms = ctypes.c_double()
    assert L.expint_probe_copy(None, None, 1024, 1, 0, None, ctypes.byref(ms)) == N.EINVAL
    assert L.expint_probe_copy(16, 4096, 1000, 1, 0, None, ctypes.byref(ms)) == N.EINVAL  # not a multiple of 16
    assert L.expint_probe_copy(17, 4096, 1024, 1, 1, None, ctypes.byref(ms)) == N.EINVAL  # misaligned
    assert L.expint_probe_copy(16, 512, 1024, 1, 0, None, ctypes.byref(ms)) == N.EINVAL  # overlapping
    assert L.expint_probe_copy(16, 1 << 40, 1 << 45, 1, 1, None, ctypes.byref(ms)) == N.EINVAL  # beyond one launch
    assert L.expint_probe_mfma(0, 0, 1, 16, None, ctypes.byref(ms)) == N.EINVAL


@pytest.mark.parametrize("scheme,fields", [(0, 5), (2, 7)])
def test_workspace_cap_gives_enomem_before_hip(monkeypatch, scheme, fields):
    # EXPINT_MAX_BYTES below the field buffers a context needs: EXPINT_ENOMEM
    # and a NULL context, decided before any HIP call (so it holds here too)
    n = 16
    need = fields * n**3 * 4 + n**3  # FP32 fields plus the uint8 labels
    grid = N.Grid(n, n, n, 1.0)
    df, cd = _labels_df()
    monkeypatch.setenv("EXPINT_MAX_BYTES", str(need - 1))
    rc, ctx = _create(grid, df, scheme=scheme)
    assert rc == N.ENOMEM
    assert ctx.value is None
    assert "EXPINT_MAX_BYTES" in N.last_error() and str(need) in N.last_error()
