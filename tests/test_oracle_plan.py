"""Pins of the (s, m) rule: optimality by exhaustive search, and the actual
truncation error of the chosen plan measured against dense expm."""

import math

import numpy as np
import pytest

from oracle import integrator as it
from oracle import operator as op
from oracle import plan
from oracle import reference as ref
from workloads.configs import random_field, random_labels


def _bound(s, m, theta):
    return s * theta ** (m + 1) / math.factorial(m + 1)


@pytest.mark.parametrize("nu", [1e-3, 0.29, 4.38, 8.76, 11.39, 17.52, 21.07, 60.0])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_plan_is_exhaustive_optimum(nu, dtype):
    tol, thmax = plan.DEFAULTS[dtype]
    s, m = plan.for_dtype(nu, dtype)
    assert nu / s <= thmax and m <= plan.M_MAX
    assert _bound(s, m, nu / s) <= tol
    best = None
    for ss in range(1, 400):
        th = nu / ss
        if th > thmax:
            continue
        for mm in range(1, plan.M_MAX + 1):
            if _bound(ss, mm, th) <= tol:
                if best is None or ss * mm < best[0] or (ss * mm == best[0] and ss < best[1]):
                    best = (ss * mm, ss, mm)
                break
    assert (s, m) == (best[1], best[2])


@pytest.mark.parametrize("nu,dtype", [(0.3, "f64"), (0.05, "f32"), (4.38, "f32"), (11.39, "f64")])
def test_plan_with_degree_floor_is_exhaustive_optimum(nu, dtype):
    # the rule restricted to m >= 2 (schemes that need phi2)
    tol, thmax = plan.DEFAULTS[dtype]
    s, m = plan.for_dtype(nu, dtype, m_min=2)
    best = None
    for ss in range(1, 400):
        th = nu / ss
        if th > thmax:
            continue
        for mm in range(2, plan.M_MAX + 1):
            if _bound(ss, mm, th) <= tol:
                if best is None or ss * mm < best[0] or (ss * mm == best[0] and ss < best[1]):
                    best = (ss * mm, ss, mm)
                break
    assert (s, m) == (best[1], best[2]) and m >= 2


def test_plan_zero_operator():
    assert plan.choose(0.0, 1e-13, 1.0) == (1, 1)
    assert plan.choose(0.0, 1e-13, 1.0, m_min=2) == (1, 2)
    with pytest.raises(ValueError):
        plan.choose(1.0, 1e-13, 1.0, m_min=0)


def test_plan_rejects_bad_nu():
    with pytest.raises(ValueError):
        plan.choose(float("nan"), 1e-6, 1.0)
    with pytest.raises(ValueError):
        plan.choose(-1.0, 1e-6, 1.0)


@pytest.mark.parametrize("dtype,nu_target", [("f64", 11.39), ("f32", 11.39), ("f64", 21.07), ("f32", 4.38)])
def test_chosen_plan_meets_bound_vs_expm(dtype, nu_target):
    # Scale an 8^3 heterogeneous operator so that tau ||A||_1 = nu_target and
    # measure the Taylor scheme against expm.  Per sub-step the exp part errs by
    # at most theta^(m+1)/(m+1)! ||x|| and the phi1 part by h theta^m/(m+1)! ||b||,
    # with ||x|| <= tau ||b||, so the total is within (1 + 1/theta) tol tau ||b||.
    shape = (8, 8, 8)
    labels = random_labels(shape, 3, seed=5)
    A_op = op.Operator(1.0, labels=labels, class_D=(0.0, 0.13, 0.013))
    tau = nu_target / A_op.norm1()
    b = random_field(shape, seed=6, lo=-1, hi=1)
    s, m = plan.for_dtype(tau * A_op.norm1(), dtype)
    tol, _ = plan.DEFAULTS[dtype]
    x = it.phi1_action(A_op, b, tau, s, m).ravel()
    xe, _ = ref.dense_phi1_augmented(A_op.dense(), b, tau)
    theta = tau * A_op.norm1() / s
    err = np.linalg.norm(x - xe)
    assert err <= (1 + 1 / theta) * tol * tau * np.linalg.norm(b) + 1e-13
