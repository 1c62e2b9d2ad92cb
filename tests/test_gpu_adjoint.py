"""GPU parity of the discrete adjoint (gradients of 0.5 ||u_T - u_target||^2
with respect to u0, rho and the class diffusivities) against the FP64 oracle
adjoint, and against central differences of the GPU forward map."""

import os

import numpy as np
import pytest
import torch

from oracle import adjoint as oadj
from oracle import operator as oop
from oracle import plan as oplan
from workloads import c4_adjoint, make_head
from workloads.configs import c4_synthetic_target, random_field, random_labels

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def case_small(n=12, seed=3):
    head = make_head(n, seed)
    rng = np.random.default_rng(seed + 7)
    u0 = head.u0 + 0.05 * rng.random(head.labels.shape) * (head.labels != 0)
    target = np.clip(u0 + 0.1 * rng.random(head.labels.shape), 0, 1) * (head.labels != 0)
    return head.labels, u0, target


def oracle_grad(labels, cd, rho, tau, u0, target, nsteps, ckpt, bc="noflux", s=None, m=None):
    op = oop.Operator(1.0, bc=bc, labels=labels, class_D=cd)
    if s is None:
        s, m = oplan.for_dtype(tau * op.norm1(), "f64")
    return oadj.loss_and_grad(op, u0, rho, tau, s, m, nsteps, target, ckpt, classes=list(range(len(cd))))


def make_ctx(labels, cd, dtype, **kw):
    from paper_2402_02273_amd.expint import ExpInt

    print(f"[case] adjoint ctx {labels.shape} {dtype} {kw}", flush=True)
    return ExpInt(labels.shape, labels=labels, class_D=cd, dtype=dtype, device=DEV, **kw)


def check_scalars(got_rho, got_D, ref_rho, ref_D, tol):
    assert got_rho == pytest.approx(ref_rho, rel=tol)
    scale = max(abs(v) for v in ref_D.values())
    for c, v in ref_D.items():
        assert abs(got_D[c] - v) <= tol * scale, (c, got_D[c], v)


@pytest.mark.parametrize("ckpt", [1, 3, 10])
def test_grad_f64_matches_oracle(native, ckpt):
    labels, u0, target = case_small()
    cd, rho, tau, K = (0.0, 0.10, 0.010), 0.02, 7.3, 4
    L, gu, grho, gD = oracle_grad(labels, cd, rho, tau, u0, target, K, ckpt)
    ctx = make_ctx(labels, cd, torch.float64, rho=rho, tau=tau)
    loss, gu_g, grho_g, gD_g = ctx.grad(dev(u0, torch.float64), K, dev(target, torch.float64), ckpt_every=ckpt)
    assert loss == pytest.approx(L, rel=1e-12)
    assert rel(gu_g.cpu().numpy(), gu) < 1e-10
    check_scalars(grho_g, gD_g, grho, gD, 1e-10)


def test_grad_dirichlet_ragged(native):
    shape = (7, 9, 11)
    labels = random_labels(shape, 3, seed=5)
    u0 = random_field(shape, seed=6) * (labels != 0)
    target = random_field(shape, seed=7)
    cd, rho, tau, K = (0.02, 0.13, 0.013), 0.03, 7.3, 3
    L, gu, grho, gD = oracle_grad(labels, cd, rho, tau, u0, target, K, 2, bc="dirichlet0")
    ctx = make_ctx(labels, cd, torch.float64, rho=rho, tau=tau, bc="dirichlet0")
    loss, gu_g, grho_g, gD_g = ctx.grad(dev(u0, torch.float64), K, dev(target, torch.float64), ckpt_every=2)
    assert loss == pytest.approx(L, rel=1e-12)
    assert rel(gu_g.cpu().numpy(), gu) < 1e-10
    check_scalars(grho_g, gD_g, grho, gD, 1e-10)


@pytest.mark.parametrize("sm", [(1, 1), (2, 1), (1, 3), (3, 5)])
def test_vjp_f64_fixed_plans(native, sm):
    labels, u0, _ = case_small(n=10, seed=9)
    cd, rho, tau, K = (0.0, 0.10, 0.010), 0.02, 3.0, 2
    gout = random_field(labels.shape, seed=10, lo=-1, hi=1)
    op = oop.Operator(1.0, labels=labels, class_D=cd)
    gu, grho, gD = oadj.vjp(op, u0, rho, tau, sm[0], sm[1], K, gout, 1, classes=[0, 1, 2])
    ctx = make_ctx(labels, cd, torch.float64, rho=rho, tau=tau, s=sm[0], m=sm[1])
    gu_g, grho_g, gD_g = ctx.vjp(dev(u0, torch.float64), K, dev(gout, torch.float64), ckpt_every=1)
    assert rel(gu_g.cpu().numpy(), gu) < 1e-10
    check_scalars(grho_g, gD_g, grho, gD, 1e-10)


def test_grad_f32_vs_f64_oracle(native):
    labels, u0, target = case_small(n=16, seed=4)
    cd, rho, tau, K = (0.0, 0.10, 0.010), 0.02, 7.3, 5
    L, gu, grho, gD = oracle_grad(labels, cd, rho, tau, u0, target, K, 2)
    ctx = make_ctx(labels, cd, torch.float32, rho=rho, tau=tau)
    loss, gu_g, grho_g, gD_g = ctx.grad(dev(u0, torch.float32), K, dev(target, torch.float32), ckpt_every=2)
    err_u = rel(gu_g.cpu().numpy(), gu)
    print(f"[result] f32 adjoint: loss {abs(loss - L) / L:.2e}, grad_u0 {err_u:.2e}, rho {abs(grho_g - grho) / abs(grho):.2e}")
    assert loss == pytest.approx(L, rel=1e-5)
    assert err_u < 1e-4
    check_scalars(grho_g, gD_g, grho, gD, 1e-4)


def test_gpu_gradient_vs_central_differences(native):
    # Richardson-extrapolated central differences of the GPU FP64 loss, plan frozen.
    labels, u0, target = case_small(n=14, seed=8)
    cd, rho, tau, K = (0.0, 0.10, 0.010), 0.02, 7.3, 4
    ctx = make_ctx(labels, cd, torch.float64, rho=rho, tau=tau)
    u0d, td = dev(u0, torch.float64), dev(target, torch.float64)
    _, gu, grho, gD = ctx.grad(u0d, K, td, ckpt_every=2)

    def loss(r, c):
        ctx.set_params(rho=r, class_D=c, replan=False)
        u = u0d.clone()
        ctx.advance(u, K)
        return 0.5 * float(((u - td) ** 2).sum())

    def fd(f, eps):
        return (f(eps) - f(-eps)) / (2 * eps)

    def rich(f, eps=1e-4):
        a, b = fd(f, eps), fd(f, eps / 2)
        return (4 * b - a) / 3

    assert grho == pytest.approx(rich(lambda e: loss(rho + e, cd)), rel=1e-7)
    for c in (1, 2):
        def fc(e, c=c):
            cc = list(cd)
            cc[c] += e
            return loss(rho, tuple(cc))

        assert gD[c] == pytest.approx(rich(fc), rel=1e-7)
    ctx.set_params(rho=rho, class_D=cd, replan=False)
    v = dev(np.random.default_rng(3).standard_normal(u0.shape), torch.float64)

    def fu(e):
        u = u0d + e * v
        ctx.advance(u, K)
        return 0.5 * float(((u - td) ** 2).sum())

    assert float((gu * v).sum()) == pytest.approx(rich(fu), rel=1e-7)


def _golden_c4(target):
    name = {"model": "c4m_adjoint_96_k50_f64.npz", "blob": "c4_adjoint_96_k50_f64.npz"}[target]
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"stored oracle gradient missing ({name}, tests/golden/make_golden.py)")
    return np.load(path)


@pytest.mark.parametrize("target_kind", ["model", "blob"])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 1e-4)])
def test_c4_full_size_vs_stored_oracle(native, dtype, tol, target_kind):
    # model: the configured target, the forward model at the hidden
    # parameters plus noise (stored with the oracle gradients); blob: a
    # model-free target of the same size
    g = _golden_c4(target_kind)
    w, _ = c4_adjoint()
    if target_kind == "model":
        import hashlib

        assert hashlib.sha256(w.labels.tobytes()).hexdigest() == str(g["labels_sha256"])
        assert hashlib.sha256(w.u0.tobytes()).hexdigest() == str(g["u0_sha256"])
        target = g["target"].astype(np.float64)
    else:
        target = c4_synthetic_target()
    print(f"[case] c4 96^3 x50 {dtype} target={target_kind}", flush=True)
    ctx = make_ctx(w.labels, w.class_D, dtype, rho=w.rho, tau=w.tau)
    if dtype == torch.float64:
        assert (ctx.plan.s, ctx.plan.m) == (int(g["s"]), int(g["m"]))
    loss, gu, grho, gD = ctx.grad(dev(w.u0, dtype), w.nsteps, dev(target, dtype), ckpt_every=10)
    err_u = rel(gu.cpu().numpy(), g["grad_u0"])
    ref_D = {c: float(v) for c, v in enumerate(g["grad_D"])}
    print(
        f"[result] c4 96^3 x50 {dtype} {target_kind}: loss {abs(loss - float(g['loss'])) / float(g['loss']):.2e} "
        f"grad_u0 {err_u:.2e} rho {abs(grho - float(g['grad_rho'])) / abs(float(g['grad_rho'])):.2e} "
        f"D {[abs(gD[c] - ref_D[c]) / max(abs(v) for v in ref_D.values()) for c in range(3)]}",
        flush=True,
    )
    assert loss == pytest.approx(float(g["loss"]), rel=tol)
    assert err_u < tol
    check_scalars(grho, gD, float(g["grad_rho"]), ref_D, tol)


def test_autograd_function_matches_oracle(native):
    from paper_2402_02273_amd.autograd import advance

    labels, u0, target = case_small(n=10, seed=12)
    cd, rho, tau, K = (0.0, 0.10, 0.010), 0.02, 7.3, 3
    L, gu, grho, gD = oracle_grad(labels, cd, rho, tau, u0, target, K, 2)
    ctx = make_ctx(labels, cd, torch.float64, rho=rho, tau=tau)
    u0t = dev(u0, torch.float64).requires_grad_(True)
    rt = torch.tensor(rho, dtype=torch.float64, requires_grad=True)
    ct = torch.tensor(cd, dtype=torch.float64, requires_grad=True)
    uT = advance(ctx, u0t, rt, ct, K, ckpt_every=2)
    loss = 0.5 * ((uT - dev(target, torch.float64)) ** 2).sum()
    loss.backward()
    assert float(loss.detach()) == pytest.approx(L, rel=1e-12)
    assert rel(u0t.grad.cpu().numpy(), gu) < 1e-10
    check_scalars(float(rt.grad), [float(v) for v in ct.grad], grho, gD, 1e-10)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-4)])
def test_repeated_gradients(native, dtype, tol):
    # Repeated calls on one context (three streams, workspace reused) give the
    # same bits with new u0 / target buffers each time; a new target, a
    # general cotangent and new parameters give the oracle's new gradients.
    labels, u0, target = case_small(n=14, seed=5)
    cd, rho, tau, K, ck = (0.0, 0.10, 0.010), 0.02, 7.3, 5, 2
    L, gu, grho, gD = oracle_grad(labels, cd, rho, tau, u0, target, K, ck)
    ctx = make_ctx(labels, cd, dtype, rho=rho, tau=tau)
    outs = [ctx.grad(dev(u0, dtype), K, dev(target, dtype), ckpt_every=ck) for _ in range(4)]
    for o in outs[1:]:
        assert o[0] == outs[0][0] and o[2] == outs[0][2] and o[3] == outs[0][3]
        assert torch.equal(o[1], outs[0][1])
    assert outs[0][0] == pytest.approx(L, rel=tol)
    assert rel(outs[0][1].cpu().numpy(), gu) < tol
    check_scalars(outs[0][2], outs[0][3], grho, gD, tol)
    # another target
    target2 = np.clip(target * 0.7 + 0.05, 0, 1) * (labels != 0)
    L2, gu2, grho2, gD2 = oracle_grad(labels, cd, rho, tau, u0, target2, K, ck)
    loss2, g2, r2, d2 = ctx.grad(dev(u0, dtype), K, dev(target2, dtype), ckpt_every=ck)
    assert loss2 == pytest.approx(L2, rel=tol)
    assert rel(g2.cpu().numpy(), gu2) < tol
    check_scalars(r2, d2, grho2, gD2, tol)
    # a general cotangent (vjp)
    cot = 0.25 * (labels != 0).astype(np.float64)
    op = oop.Operator(1.0, labels=labels, class_D=cd)
    s, m = oplan.for_dtype(tau * op.norm1(), "f64")
    gv, rv, dv = oadj.vjp(op, u0, rho, tau, s, m, K, cot, ck, classes=[0, 1, 2])
    for _ in range(3):
        g3, r3, d3 = ctx.vjp(dev(u0, dtype), K, dev(cot, dtype), ckpt_every=ck)
        assert rel(g3.cpu().numpy(), gv) < tol
        check_scalars(r3, d3, rv, {c: dv[c] for c in range(3)}, tol)
    # new rho (plan kept)
    ctx.set_params(rho=0.03, replan=False)
    L4, gu4, grho4, gD4 = oracle_grad(labels, cd, 0.03, tau, u0, target, K, ck, s=s, m=m)
    for _ in range(3):
        loss4, g4, r4, d4 = ctx.grad(dev(u0, dtype), K, dev(target, dtype), ckpt_every=ck)
        assert loss4 == pytest.approx(L4, rel=tol)
        assert rel(g4.cpu().numpy(), gu4) < tol
        check_scalars(r4, d4, grho4, gD4, tol)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_profile_of_the_reverse_sweep_leaves_the_gradient_alone(native, dtype):
    # expint_profile id 6 times the gradient's fused reverse sweep on the
    # gradient's own workspace: refused before a gradient has set that up;
    # afterwards it times, and the next gradient has the same bits
    from paper_2402_02273_amd import _native as N

    shape = (12, 10, 32)
    labels = random_labels(shape, 3, seed=61)
    u0 = random_field(shape, seed=62) * (labels != 0)
    target = random_field(shape, seed=63)
    cd, rho, tau, K = (0.0, 0.10, 0.010), 0.02, 7.3, 3
    ctx = make_ctx(labels, cd, dtype, rho=rho, tau=tau)
    with pytest.raises(N.ExpIntError) as err:
        ctx.profile("face", reps=2)
    assert err.value.code == N.EUNSUPPORTED
    first = ctx.grad(dev(u0, dtype), K, dev(target, dtype), ckpt_every=2)
    if ctx.launch_info()["vec"]:
        assert ctx.profile("face", reps=5) > 0
    second = ctx.grad(dev(u0, dtype), K, dev(target, dtype), ckpt_every=2)
    assert first[0] == second[0] and first[2] == second[2] and list(first[3]) == list(second[3])
    assert torch.equal(first[1], second[1])
