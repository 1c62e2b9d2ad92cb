"""Writes the stored oracle results the GPU parity tests compare against.

Calls only ``oracle/`` (FP64, CPU) on inputs from ``workloads``.  Run from
the repository root:

    python tests/golden/make_golden.py c2      # 128^3 head, 100 steps (~6 min)

Each file records the plan, the input hashes and the oracle result.
"""

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import integrator, operator, plan  # noqa: E402
from workloads import c2_head  # noqa: E402

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


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c2"
    if which == "c2":
        make_c2()
    else:
        raise SystemExit(f"unknown golden {which}")
