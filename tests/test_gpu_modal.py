"""GPU parity of the modal path (uniform D: per-axis mode products on the
closed-form cosine / sine bases) against the oracle's DCT/DST references."""

import numpy as np
import pytest
import torch

from oracle import integrator as oit
from oracle import operator as oop
from oracle import plan as oplan
from oracle import reference as oref
from workloads import c5_separable, gaussian_blob
from workloads.configs import random_field

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
MPS = ["none", "bf16_split", "fp16_split"]
# rel-L2 bars for one phi1 application (six mode products).  A hi + lo split
# keeps ~16 significant bits for bfloat16 (8 + 8) and ~22 for float16
# (11 + 11), so each product errs by about 2^-17 (7.6e-6) resp. 2^-23
# (1.2e-7) relative; FP32 storage bounds everything below by ~1e-7.
PHI1_TOL = {"none": 2e-6, "bf16_split": 3e-5, "fp16_split": 1e-6}


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def modal_ctx(shape, dtype, mp="none", bc="noflux", D=0.1, rho=0.025, tau=7.3):
    from paper_2402_02273_amd.expint import ExpInt

    print(f"[case] modal {shape} {dtype} {mp} {bc}", flush=True)
    labels = np.ones(shape, dtype=np.uint8)
    return ExpInt(shape, labels=labels, class_D=(0.0, D), rho=rho, tau=tau, dtype=dtype, algo="modal", mp=mp,
                  bc=bc, device=DEV)


@pytest.mark.parametrize("shape", [(32, 32, 32), (32, 64, 96), (96, 32, 64)])
@pytest.mark.parametrize("bc", ["noflux", "dirichlet0"])
def test_modal_phi1_f64(native, shape, bc):
    # zero flux: the power-of-two axes run as fast cosine transforms; the
    # sine basis of zero ghost values keeps the dense products
    b = random_field(shape, seed=3, lo=-1, hi=1)
    ctx = modal_ctx(shape, torch.float64, bc=bc)
    want = sum(1 << ax for ax, n in enumerate(shape) if n in (32, 64, 128, 256)) if bc == "noflux" else 0
    assert ctx.launch_info()["modal_dct"] == want
    got = ctx.phi1(dev(b, torch.float64)).cpu().numpy()
    ref = oref.modal_phi1(b, 0.1, 1.0, 7.3, bc)
    assert rel(got, ref) < 1e-13


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-13), (torch.float32, 1e-6)])
# every transform length (32, 64, 128, 256) on each axis, and axes of other
# lengths (96, 160) that keep the dense products in the same chain
@pytest.mark.parametrize("shape", [(32, 64, 128), (256, 32, 64), (64, 256, 32), (128, 96, 256), (160, 128, 32)])
def test_modal_fast_transforms_vs_oracle(native, monkeypatch, dtype, tol, shape):
    # zero-flux products along power-of-two axes run as fast cosine
    # transforms (the x pass fused with the multiplier); the same phi1 and
    # the same step through the dense products (EXPINT_MODAL_DCT=0) and the
    # FP64 oracle agree
    b = random_field(shape, seed=13, lo=-1, hi=1)
    u0 = random_field(shape, seed=14)
    ref = oref.modal_phi1(b, 0.1, 1.0, 7.3, "noflux")
    out = {}
    for mode in ("fast", "dense"):
        if mode == "dense":
            monkeypatch.setenv("EXPINT_MODAL_DCT", "0")
        else:
            monkeypatch.delenv("EXPINT_MODAL_DCT", raising=False)
        ctx = modal_ctx(shape, dtype)
        want = sum(1 << ax for ax, n in enumerate(shape) if n in (32, 64, 128, 256)) if mode == "fast" else 0
        assert ctx.launch_info()["modal_dct"] == want
        assert ctx.profile("mode_x", reps=2) > 0 and ctx.profile("mode_z", reps=2) > 0
        got = ctx.phi1(dev(b, dtype)).cpu().numpy()
        u = dev(u0, dtype)
        ctx.advance(u, 2)
        out[mode] = (got, u.cpu().numpy())
        err = rel(got, ref)
        print(f"[result] modal phi1 {shape} {dtype} {mode}: rel-L2 vs FP64 oracle {err:.2e}", flush=True)
        assert err < tol, mode
        del ctx
    assert rel(out["fast"][1], out["dense"][1]) < tol
    uref = oref.modal_advance(u0, 0.1, 1.0, 0.025, 7.3, 2)
    assert rel(out["fast"][1], uref) < tol


@pytest.mark.parametrize("mp", MPS)
# 224 and 160: 128-wide tiles with a partial last tile; 288: all-mode tiles
# of 256 with a partial one
@pytest.mark.parametrize("shape", [(32, 32, 32), (64, 32, 96), (224, 32, 160), (288, 64, 32)])
def test_modal_phi1_f32_precisions(native, mp, shape):
    c = tuple((n - 1) / 2 for n in shape)
    b = gaussian_blob(shape, c, amplitude=0.5, sigma=4.0) + 0.01 * random_field(shape, seed=5)
    ctx = modal_ctx(shape, torch.float32, mp=mp)
    got = ctx.phi1(dev(b, torch.float32)).cpu().numpy()
    err = rel(got, oref.modal_phi1(b, 0.1, 1.0, 7.3))
    print(f"[result] modal phi1 {shape} {mp}: rel-L2 vs FP64 oracle {err:.2e}", flush=True)
    assert err < PHI1_TOL[mp]


@pytest.mark.parametrize("dtype,mp,tol", [(torch.float64, "none", 1e-13), (torch.float32, "none", 1e-6),
                                          (torch.float32, "bf16_split", 1e-5), (torch.float32, "fp16_split", 1e-6)])
def test_modal_advance_vs_oracle(native, dtype, mp, tol):
    w = c5_separable(n=32, nsteps=10)
    ctx = modal_ctx(w.shape, dtype, mp=mp, rho=w.rho, tau=w.tau)
    u = dev(w.u0, dtype)
    ctx.advance(u, w.nsteps)
    ref = oref.modal_advance(w.u0, 0.1, 1.0, w.rho, w.tau, w.nsteps)
    err = rel(u.cpu().numpy(), ref)
    print(f"[result] modal 32^3 x10 {dtype} {mp}: rel-L2 vs FP64 oracle {err:.2e}", flush=True)
    assert err < tol


def test_modal_equals_stencil_taylor(native):
    from paper_2402_02273_amd.expint import ExpInt

    w = c5_separable(n=64, nsteps=5)
    cm = modal_ctx(w.shape, torch.float64, rho=w.rho, tau=w.tau)
    cs = ExpInt(w.shape, labels=np.ones(w.shape, np.uint8), class_D=(0.0, 0.1), rho=w.rho, tau=w.tau,
                dtype=torch.float64, device=DEV)
    um, us = dev(w.u0, torch.float64), dev(w.u0, torch.float64)
    cm.advance(um, w.nsteps)
    cs.advance(us, w.nsteps)
    a, b = um.cpu().numpy(), us.cpu().numpy()
    vox = np.abs(a - b).max() / np.abs(b).max()
    print(f"[result] modal vs stencil-Taylor FP64 64^3 x5: rel-L2 {rel(a, b):.2e}, max voxel {vox:.2e}", flush=True)
    assert rel(a, b) < 1e-12
    # every voxel, not only the norm: a wrong face at a tile edge would show here
    assert vox < 1e-12


def test_modal_rejections(native):
    from paper_2402_02273_amd import ExpIntError
    from paper_2402_02273_amd.expint import ExpInt

    lab = np.ones((32, 32, 32), np.uint8)
    lab[3, 4, 5] = 2
    with pytest.raises(ExpIntError, match="EUNSUPPORTED"):
        ExpInt(lab.shape, labels=lab, class_D=(0.0, 0.1, 0.01), algo="modal", device=DEV)
    # a class with a different D that is absent from the grid is fine
    ExpInt(lab.shape, labels=np.ones_like(lab), class_D=(0.0, 0.1, 0.01), algo="modal", device=DEV).close()
    with pytest.raises(ExpIntError, match="EUNSUPPORTED"):
        ExpInt((32, 32, 40), labels=np.ones((32, 32, 40), np.uint8), class_D=(0.0, 0.1), algo="modal", device=DEV)
    with pytest.raises(ExpIntError, match="EUNSUPPORTED"):
        ExpInt(lab.shape, labels=np.ones_like(lab), class_D=(0.0, 0.1), algo="modal", mp="bf16_split",
               dtype=torch.float64, device=DEV)
    with pytest.raises(ExpIntError, match="EUNSUPPORTED"):
        ExpInt(lab.shape, labels=np.ones_like(lab), class_D=(0.0, 0.1), mp="bf16_split", device=DEV)


@pytest.mark.parametrize("dtype,mp,tol", [(torch.float64, "none", 1e-13), (torch.float32, "none", 1e-6),
                                          (torch.float32, "bf16_split", 2e-5), (torch.float32, "fp16_split", 1e-6)])
def test_c5_full_size_pure_diffusion_exact(native, dtype, mp, tol):
    # rho = 0: each exponential Euler step is exactly exp(tau A), so 100 steps
    # equal exp(100 tau A) u0, one DCT pair in the oracle.
    w = c5_separable()
    ctx = modal_ctx(w.shape, dtype, mp=mp, rho=0.0, tau=w.tau)
    u = dev(w.u0, dtype)
    ctx.advance(u, w.nsteps)
    ref = oref.modal_expm(w.u0, 0.1, 1.0, w.tau * w.nsteps)
    err = rel(u.cpu().numpy(), ref)
    print(f"[result] c5 256^3 x100 rho=0 {dtype} {mp}: rel-L2 vs exact exponential {err:.2e}", flush=True)
    assert err < tol


def test_c5_full_size_one_step_elementwise(native):
    w = c5_separable()
    ref = oref.modal_step(w.u0, 0.1, 1.0, w.rho, w.tau)
    for dtype, mp, tol in ((torch.float64, "none", 1e-13), (torch.float32, "none", 1e-6),
                           (torch.float32, "bf16_split", 1e-5), (torch.float32, "fp16_split", 1e-6)):
        ctx = modal_ctx(w.shape, dtype, mp=mp, rho=w.rho, tau=w.tau)
        u = dev(w.u0, dtype)
        ctx.step(u)
        got = u.cpu().numpy()
        err = rel(got, ref)
        emax = float(np.abs(got - ref).max() / np.abs(ref).max())
        print(f"[result] c5 256^3 one step {dtype} {mp}: rel-L2 {err:.2e}, max-abs/max {emax:.2e}", flush=True)
        assert err < tol
        assert emax < tol  # voxel by voxel, relative to the field's largest value
        ctx.close()


def test_modal_gradient_rejected(native):
    # the reverse pass is the adjoint of the Taylor map, not of the mode
    # products, so modal contexts give no gradients
    from paper_2402_02273_amd import ExpIntError

    ctx = modal_ctx((32, 32, 32), torch.float64)
    u0 = dev(random_field((32, 32, 32), seed=5), torch.float64)
    with pytest.raises(ExpIntError, match="EUNSUPPORTED"):
        ctx.grad(u0, 2, u0, ckpt_every=1)
    with pytest.raises(ExpIntError, match="EUNSUPPORTED"):
        ctx.vjp(u0, 2, u0, ckpt_every=1)


@pytest.mark.parametrize("dense", [False, True])
def test_modal_set_params_keeps_one_diffusivity(native, monkeypatch, dense):
    # two classes present with one D: set_params may change it (and rho) if
    # the classes stay equal, and the step (its right-hand side formed inside
    # the first transform pass, or by the stencil sweep with dense products)
    # then follows the new values; unequal values are refused and change
    # nothing
    from paper_2402_02273_amd import _native as N
    from paper_2402_02273_amd.expint import ExpInt

    if dense:
        monkeypatch.setenv("EXPINT_MODAL_DCT", "0")
    shape = (32, 64, 32)
    labels = np.ones(shape, dtype=np.uint8)
    labels[:16] = 2
    u0 = random_field(shape, seed=21)
    ctx = ExpInt(shape, labels=labels, class_D=(0.0, 0.1, 0.1), rho=0.025, tau=7.3, dtype=torch.float64,
                 algo="modal", device=DEV)
    assert ctx.launch_info()["modal_dct"] == (0 if dense else 7)
    ctx.set_params(rho=0.02, class_D=(0.5, 0.2, 0.2))  # class 0 is absent: its D does not count
    with pytest.raises(N.ExpIntError) as err:
        ctx.set_params(rho=0.03, class_D=(0.0, 0.2, 0.3))
    assert err.value.code == N.EUNSUPPORTED
    u = dev(u0, torch.float64)
    ctx.advance(u, 3)
    ref = oref.modal_advance(u0, 0.2, 1.0, 0.02, 7.3, 3)
    assert rel(u.cpu().numpy(), ref) < 1e-13


@pytest.mark.parametrize("dense", [False, True])
def test_modal_step_with_grid_spacing(native, monkeypatch, dense):
    # h = 0.5: the eigenvalues scale by 1/h^2, and so does the Laplacian of
    # the right-hand side formed inside the first transform pass
    from paper_2402_02273_amd.expint import ExpInt

    if dense:
        monkeypatch.setenv("EXPINT_MODAL_DCT", "0")
    shape, h, D, rho, tau, K = (32, 64, 32), 0.5, 0.05, 0.025, 3.0, 3
    labels = np.ones(shape, dtype=np.uint8)
    u0 = random_field(shape, seed=31)
    ctx = ExpInt(shape, h, labels=labels, class_D=(0.0, D), rho=rho, tau=tau, dtype=torch.float64, algo="modal",
                 device=DEV)
    assert ctx.launch_info()["modal_dct"] == (0 if dense else 7)
    u = dev(u0, torch.float64)
    ctx.advance(u, K)
    ref = oref.modal_advance(u0, D, h, rho, tau, K)
    assert rel(u.cpu().numpy(), ref) < 1e-13
