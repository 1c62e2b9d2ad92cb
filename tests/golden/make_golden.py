"""Writes the stored oracle results the GPU parity tests compare against.

Calls only ``oracle/`` (FP64, CPU) on inputs from ``workloads``.  Run from
the repository root:

    python tests/golden/make_golden.py c2      # 128^3 head, states after 20 and 100 steps (~12 min)
    python tests/golden/make_golden.py c2l     # the same with the linearised step (~13 min)
    python tests/golden/make_golden.py c2e     # 20 second-order exponential Runge-Kutta steps (~6 min)
    python tests/golden/make_golden.py c3      # one batch instance per grid size above 48^3, 50 steps (~10 min)
    python tests/golden/make_golden.py c4      # 96^3 gradients, 50 steps, model-free target (~15 min)
    python tests/golden/make_golden.py c4m     # 96^3 gradients against the forward-model target (~17 min)
    python tests/golden/make_golden.py c5      # 256^3 separable run, 100 steps, DCT modal (~10 min)
    python tests/golden/make_golden.py c5d     # the same without reaction: exp(100 tau A) u0 (~1 min)

Each file records the plan, the input hashes and the oracle result.  Results
compared only with FP32 GPU runs (c3) are rounded to FP32 on storage, a
relative change of at most 6e-8 against their 1e-5 bar.
"""

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint, exprk2, integrator, operator, plan, reference, rosenbrock  # noqa: E402
from workloads import c2_head, c3_batch, c4_adjoint, c5_separable  # noqa: E402
from workloads.configs import c4_synthetic_target  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
from store import pack_cube  # noqa: E402

# batch instances stored per grid size (the first of each size in the
# workload's order); the 48^3 ones are cheap enough to run in the test
C3_STORED = {64: 1, 96: 5, 128: 0}


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def make_c2(n=128, nsteps=100, keep=(20,)):
    """The headline run; besides the final state it keeps the states after
    the step counts in ``keep`` (u_step20: the length of a short timed run)."""
    w = c2_head(n=n, nsteps=nsteps)
    op = operator.Operator(w.h, labels=w.labels, class_D=w.class_D)
    nu = w.tau * op.norm1()
    s, m = plan.for_dtype(nu, "f64")
    t0 = time.time()
    kept = {}

    def progress(k, u):
        if k in keep:
            kept[f"u_step{k}"] = u.copy()
        if k % 10 == 0:
            print(f"step {k}/{nsteps}  {time.time() - t0:.0f}s", flush=True)

    u = integrator.advance(op, w.u0, w.rho, w.tau, s, m, nsteps, callback=progress)
    out = os.path.join(HERE, f"c2_head_{n}_u{nsteps}_f64.npz")
    np.savez_compressed(
        out,
        u=u,
        **kept,
        s=s,
        m=m,
        norm1=op.norm1(),
        labels_sha256=digest(w.labels),
        u0_sha256=digest(w.u0),
        rho=w.rho,
        tau=w.tau,
        class_D=np.asarray(w.class_D),
    )
    print("wrote", out, "plan", (s, m), "seconds", round(time.time() - t0, 1))


def make_c2l(n=128, nsteps=100):
    """The headline head run with the linearised step (section 2.1's
    splitting), plan chosen for tau (||A||_1 + rho)."""
    w = c2_head(n=n, nsteps=nsteps)
    op = operator.Operator(w.h, labels=w.labels, class_D=w.class_D)
    s, m = plan.for_dtype(w.tau * rosenbrock.norm1_bound(op.norm1(), w.rho), "f64")
    t0 = time.time()

    def progress(k, u):
        if k % 10 == 0:
            print(f"step {k}/{nsteps}  {time.time() - t0:.0f}s", flush=True)

    u = rosenbrock.advance(op, w.u0, w.rho, w.tau, s, m, nsteps, callback=progress)
    out = os.path.join(HERE, f"c2l_head_{n}_u{nsteps}_f64.npz")
    np.savez_compressed(
        out,
        u=u,
        s=s,
        m=m,
        norm1=op.norm1(),
        labels_sha256=digest(w.labels),
        u0_sha256=digest(w.u0),
        rho=w.rho,
        tau=w.tau,
        class_D=np.asarray(w.class_D),
    )
    print("wrote", out, "plan", (s, m), "seconds", round(time.time() - t0, 1))


def make_c2e(n=128, nsteps=20):
    """The headline head with the second-order exponential Runge-Kutta step
    (phi2 from the augmented matrix), plan with the degree floor m >= 2."""
    w = c2_head(n=n, nsteps=nsteps)
    op = operator.Operator(w.h, labels=w.labels, class_D=w.class_D)
    s, m = plan.for_dtype(w.tau * op.norm1(), "f64", m_min=exprk2.M_MIN)
    t0 = time.time()

    def progress(k, u):
        print(f"step {k}/{nsteps}  {time.time() - t0:.0f}s", flush=True)

    u = exprk2.advance(op, w.u0, w.rho, w.tau, s, m, nsteps, callback=progress)
    out = os.path.join(HERE, f"c2e_head_{n}_u{nsteps}_f64.npz")
    np.savez_compressed(
        out,
        u=u,
        s=s,
        m=m,
        norm1=op.norm1(),
        labels_sha256=digest(w.labels),
        u0_sha256=digest(w.u0),
        rho=w.rho,
        tau=w.tau,
        class_D=np.asarray(w.class_D),
    )
    print("wrote", out, "plan", (s, m), "seconds", round(time.time() - t0, 1))


def make_c4(n=96, nsteps=50, ckpt=10):
    """Oracle loss and gradients at the evaluation parameters of the
    calibration workload, against the synthetic (model-free) target."""
    w, _ = c4_adjoint(n=n, nsteps=nsteps)
    target = c4_synthetic_target(n=n)
    op = operator.Operator(w.h, labels=w.labels, class_D=w.class_D)
    s, m = plan.for_dtype(w.tau * op.norm1(), "f64")
    t0 = time.time()
    loss, gu0, grho, gD = adjoint.loss_and_grad(op, w.u0, w.rho, w.tau, s, m, nsteps, target, ckpt, classes=[0, 1, 2])
    out = os.path.join(HERE, f"c4_adjoint_{n}_k{nsteps}_f64.npz")
    np.savez_compressed(
        out,
        loss=loss,
        grad_u0=gu0,
        grad_rho=grho,
        grad_D=np.array([gD[0], gD[1], gD[2]]),
        s=s,
        m=m,
        labels_sha256=digest(w.labels),
        target_sha256=digest(target),
    )
    print("wrote", out, "plan", (s, m), "loss", loss, "grad_rho", grho, "grad_D", gD, "seconds", round(time.time() - t0, 1))


def make_c3(nsteps=50):
    """One instance of each grid size of the batched workload (FP64 oracle at
    the instance's FP64 plan), rounded to FP32 on storage."""
    insts, _ = c3_batch(nsteps=nsteps)
    t0 = time.time()
    arrays = {}
    for n, i in sorted(C3_STORED.items()):
        inst = insts[i]
        assert inst.n == n, (i, inst.n)
        op = operator.Operator(1.0, labels=inst.labels, class_D=inst.class_D)
        s, m = plan.for_dtype(7.3 * op.norm1(), "f64")
        u = integrator.advance(op, inst.u0, inst.rho, 7.3, s, m, nsteps)
        arrays[f"u_inst{i}"] = u.astype(np.float32)
        arrays[f"plan_inst{i}"] = np.array([s, m])
        arrays[f"labels_sha256_inst{i}"] = digest(inst.labels)
        print(f"instance {i} ({n}^3) plan {(s, m)}  {time.time() - t0:.0f}s", flush=True)
    out = os.path.join(HERE, f"c3_instances_u{nsteps}_f32.npz")
    np.savez_compressed(out, instances=np.array(sorted(C3_STORED.values())), tau=7.3, **arrays)
    print("wrote", out, "seconds", round(time.time() - t0, 1))


def make_c4m(n=96, nsteps=50, ckpt=10):
    """The calibration workload as configured: the target is the oracle
    forward run at the hidden parameters (0.025, 0.13, 0.013) after 50 steps
    plus N(0, 0.01^2) noise (seed 2405) on the tissue voxels (outside the head
    the density is known to be zero), rounded to FP32 so that the GPU runs and
    the oracle see the same target.  Loss and gradients are the oracle's at the
    evaluation parameters (0.02, 0.10, 0.010)."""
    w, noise = c4_adjoint(n=n, nsteps=nsteps)
    rho_h, dw_h, dg_h = w.extra["hidden"]
    hidden = operator.Operator(w.h, labels=w.labels, class_D=(0.0, dw_h, dg_h))
    sh, mh = plan.for_dtype(w.tau * hidden.norm1(), "f64")
    t0 = time.time()
    u_hidden = integrator.advance(hidden, w.u0, rho_h, w.tau, sh, mh, nsteps)
    target = ((u_hidden + noise) * (w.labels != 0)).astype(np.float32)
    print(f"target from the hidden parameters, plan {(sh, mh)}  {time.time() - t0:.0f}s", flush=True)
    op = operator.Operator(w.h, labels=w.labels, class_D=w.class_D)
    s, m = plan.for_dtype(w.tau * op.norm1(), "f64")
    loss, gu0, grho, gD = adjoint.loss_and_grad(op, w.u0, w.rho, w.tau, s, m, nsteps, target.astype(np.float64), ckpt,
                                                classes=[0, 1, 2])
    out = os.path.join(HERE, f"c4m_adjoint_{n}_k{nsteps}_f64.npz")
    np.savez_compressed(
        out,
        target=target,
        loss=loss,
        grad_u0=gu0,
        grad_rho=grho,
        grad_D=np.array([gD[0], gD[1], gD[2]]),
        s=s,
        m=m,
        hidden=np.array([rho_h, dw_h, dg_h]),
        hidden_plan=np.array([sh, mh]),
        labels_sha256=digest(w.labels),
        u0_sha256=digest(w.u0),
    )
    print("wrote", out, "plan", (s, m), "loss", loss, "grad_rho", grho, "grad_D", gD, "seconds",
          round(time.time() - t0, 1))


def make_c5(n=256, nsteps=100):
    """The separable run: exponential Euler with the exact phi1 of the DCT
    modal reference, FP64, stored on the fundamental domain of the cube's
    symmetries (the run is symmetric under them; the largest asymmetry of the
    computed field, rounding only, is stored as ``sym_defect``)."""
    w = c5_separable(n=n, nsteps=nsteps)
    D = w.class_D[1]
    t0 = time.time()
    u = np.array(w.u0, dtype=np.float64, copy=True)
    for k in range(nsteps):
        u = reference.modal_step(u, D, w.h, w.rho, w.tau)
        if (k + 1) % 10 == 0:
            print(f"step {k + 1}/{nsteps}  {time.time() - t0:.0f}s", flush=True)
    defect = max(float(np.abs(u - np.flip(u, axis=0)).max()), float(np.abs(u - u.transpose(1, 0, 2)).max()),
                 float(np.abs(u - u.transpose(2, 1, 0)).max()))
    out = os.path.join(HERE, f"c5_modal_{n}_u{nsteps}_f64.npz")
    np.savez_compressed(
        out,
        u_domain=pack_cube(u),
        n=n,
        nsteps=nsteps,
        D=D,
        rho=w.rho,
        tau=w.tau,
        norm2=float(np.linalg.norm(u)),
        sym_defect=defect,
        u0_sha256=digest(w.u0),
    )
    print("wrote", out, "sym_defect", defect, "seconds", round(time.time() - t0, 1))


def make_c5d(n=256, nsteps=100):
    """The separable run without reaction: each step is exp(tau A) exactly,
    so the result is exp(100 tau A) u0, one DCT pair of the modal reference."""
    w = c5_separable(n=n, nsteps=nsteps)
    D = w.class_D[1]
    t0 = time.time()
    u = reference.modal_expm(w.u0, D, w.h, w.tau * nsteps)
    out = os.path.join(HERE, f"c5_modal_{n}_rho0_u{nsteps}_f64.npz")
    np.savez_compressed(out, u_domain=pack_cube(u), n=n, nsteps=nsteps, D=D, rho=0.0, tau=w.tau,
                        norm2=float(np.linalg.norm(u)), u0_sha256=digest(w.u0))
    print("wrote", out, "seconds", round(time.time() - t0, 1))


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c2"
    if which == "c2":
        make_c2()
    elif which == "c2l":
        make_c2l()
    elif which == "c2e":
        make_c2e()
    elif which == "c3":
        make_c3()
    elif which == "c4":
        make_c4()
    elif which == "c4m":
        make_c4m()
    elif which == "c5":
        make_c5()
    elif which == "c5d":
        make_c5d()
    else:
        raise SystemExit(f"unknown golden {which}")
