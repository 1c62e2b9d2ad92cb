"""Writes the stored oracle results the GPU parity tests compare against.

Calls only ``oracle/`` (FP64, CPU) on inputs from ``workloads``.  Run from
the repository root:

    python tests/golden/make_golden.py c2      # 128^3 head, 100 steps (~12 min)
    python tests/golden/make_golden.py c2l     # the same with the linearised step (~13 min)
    python tests/golden/make_golden.py c2e     # 20 second-order exponential Runge-Kutta steps (~6 min)
    python tests/golden/make_golden.py c4      # 96^3 gradients, 50 steps (~15 min)

Each file records the plan, the input hashes and the oracle result.
"""

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint, exprk2, integrator, operator, plan, rosenbrock  # noqa: E402
from workloads import c2_head, c4_adjoint  # noqa: E402
from workloads.configs import c4_synthetic_target  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def make_c2(n=128, nsteps=100):
    w = c2_head(n=n, nsteps=nsteps)
    op = operator.Operator(w.h, labels=w.labels, class_D=w.class_D)
    nu = w.tau * op.norm1()
    s, m = plan.for_dtype(nu, "f64")
    t0 = time.time()

    def progress(k, u):
        if k % 10 == 0:
            print(f"step {k}/{nsteps}  {time.time() - t0:.0f}s", flush=True)

    u = integrator.advance(op, w.u0, w.rho, w.tau, s, m, nsteps, callback=progress)
    out = os.path.join(HERE, f"c2_head_{n}_u{nsteps}_f64.npz")
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


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c2"
    if which == "c2":
        make_c2()
    elif which == "c2l":
        make_c2l()
    elif which == "c2e":
        make_c2e()
    elif which == "c4":
        make_c4()
    else:
        raise SystemExit(f"unknown golden {which}")
