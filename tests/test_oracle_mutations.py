"""Planted mistakes in the oracle, each of which the pins must catch.

Every case replaces one oracle function by a copy with a plausible error (a
dropped term, a flipped sign, a wrong index, coefficient or mean) and runs the
pin tests that cover it; the case passes only if at least one pin fails.  This
checks the pins, not the library: a mistake that no pin catches would let a
wrong oracle certify a wrong kernel.  CPU only; the mutants live in this file
and never reach the oracle package.
"""

import numpy as np
import pytest

import test_oracle_adjoint as T_adj
import test_oracle_exprk2 as T_ek
import test_oracle_integrator as T_int
import test_oracle_operator as T_op
import test_oracle_plan as T_plan
import test_oracle_rosenbrock as T_rb
from oracle import adjoint as oadj
from oracle import exprk2 as oek
from oracle import integrator as oit
from oracle import operator as oop
from oracle import plan as oplan
from oracle import rosenbrock as orb


def caught(*checks):
    """True if at least one pin check fails its assertions."""
    for check in checks:
        try:
            check()
        except AssertionError:
            return True
    return False


def operator_pins():
    return (
        lambda: T_op.test_apply_matches_bruteforce((3, 2, 4), "noflux"),
        lambda: T_op.test_apply_matches_bruteforce((4, 3, 3), "dirichlet0"),
        T_op.test_two_voxel_hand_values,
        T_op.test_zero_diffusivity_blocks_flux,
        lambda: T_op.test_eigenpairs_uniform("noflux"),
        lambda: T_op.test_eigenpairs_uniform("dirichlet0"),
    )


def integrator_pins():
    return (
        lambda: T_int.test_phi1_action_vs_dense_expm(7.3),
        lambda: T_int.test_eigenmode_decay("noflux"),
        T_int.test_logistic_special_case_is_forward_euler,
        T_int.test_logistic_first_order_convergence,
        T_int.test_uniform_state_stays_uniform,
    )


# ---- mutants of the operator (section 2.1 reading) ----

def _apply_A_variant(mistake):
    """apply_A with one planted mistake."""
    def apply_A(u, D, h, bc="noflux", kind="harmonic"):
        u = np.asarray(u, dtype=np.float64)
        D = np.asarray(D, dtype=np.float64)
        out = np.zeros_like(u)
        axes = list(enumerate(oop.face_coefficients(D, kind)))
        if mistake == "drop_z":
            axes = axes[:2]
        for ax, K in axes:
            lo = oop._sl(ax, slice(0, -1))
            hi = oop._sl(ax, slice(1, None))
            flux = K * (u[hi] - u[lo])
            if mistake == "sign":
                flux = -flux
            out[lo] += flux
            if mistake != "one_sided":
                out[hi] -= flux
            if bc == "dirichlet0" and mistake != "no_wall":
                first = oop._sl(ax, slice(0, 1))
                last = oop._sl(ax, slice(-1, None))
                out[first] -= D[first] * u[first]
                out[last] -= D[last] * u[last]
        return out / (h * h)
    return apply_A


@pytest.mark.parametrize("mistake", ["drop_z", "sign", "one_sided", "no_wall"])
def test_operator_mutants_caught(monkeypatch, mistake):
    monkeypatch.setattr(oop, "apply_A", _apply_A_variant(mistake))
    assert caught(*operator_pins()), mistake


def test_arithmetic_face_mean_caught(monkeypatch):
    orig = oop.face_mean
    monkeypatch.setattr(oop, "face_mean", lambda a, b, kind="harmonic": orig(a, b, "arithmetic"))
    assert caught(*operator_pins())


def test_shifted_neighbour_caught(monkeypatch):
    # a coupling to the voxel two steps away along z (a wrong neighbour index)
    orig = oop.apply_A

    def apply_A(u, D, h, bc="noflux", kind="harmonic"):
        u = np.asarray(u, dtype=np.float64)
        D = np.asarray(D, dtype=np.float64)
        extra = np.zeros_like(u)
        extra[:, :, :-2] = D[:, :, :-2] * (u[:, :, 2:] - u[:, :, :-2])
        return orig(u, D, h, bc, kind) + extra / (h * h)

    monkeypatch.setattr(oop, "apply_A", apply_A)
    assert caught(*operator_pins())


def test_class_derivative_mutant_caught(monkeypatch):
    # derivative of the arithmetic mean (1/2 per side) instead of the harmonic one
    def dK(la, lb, class_D, c):
        return 0.5 * ((la == c).astype(float) + (lb == c).astype(float))
    monkeypatch.setattr(oop, "_dK_dDc", dK)
    assert caught(T_op.test_class_derivative_by_difference, lambda: T_adj.test_gradients_vs_central_fd(2, "exp_euler"))


# ---- mutants of the integrator (section 2.2) ----

def _phi1_variant(mistake):
    def phi1_action(apply_A, b, tau, s, m):
        b = np.asarray(b, dtype=np.float64)
        h = tau / s
        x = np.zeros_like(b)
        for _ in range(s):
            y = h * apply_A(x) if mistake == "drop_b" else h * (apply_A(x) + b)
            acc = x + y
            for j in range(2, m + 1):
                c = h / (j + 1) if mistake == "coef" else h / j
                y = c * apply_A(y)
                acc = acc + y
            x = y if mistake == "no_carry" else acc
        return x
    return phi1_action


@pytest.mark.parametrize("mistake", ["drop_b", "coef", "no_carry"])
def test_phi1_mutants_caught(monkeypatch, mistake):
    monkeypatch.setattr(oit, "phi1_action", _phi1_variant(mistake))
    assert caught(*integrator_pins()), mistake


def test_reaction_sign_caught(monkeypatch):
    monkeypatch.setattr(oit, "reaction", lambda u, rho: rho * u * (1.0 + u))
    assert caught(*integrator_pins())


def test_dropped_reaction_caught(monkeypatch):
    monkeypatch.setattr(oit, "rhs", lambda apply_A, u, rho: apply_A(u))
    assert caught(*integrator_pins())


def test_step_without_u_caught(monkeypatch):
    monkeypatch.setattr(oit, "step", lambda apply_A, u, rho, tau, s, m: oit.phi1_action(apply_A, oit.rhs(apply_A, u, rho),
                                                                                        tau, s, m))
    assert caught(*integrator_pins())


# ---- mutants of the plan rule ----

def _bound_with_power(shift):
    """s theta^(m + shift) / (m + shift)! in place of the (m + 1) remainder."""
    def bound(s, m, theta):
        t = float(s)
        for k in range(1, m + shift + 1):
            t = t * (theta / k)
        return t
    return bound


@pytest.mark.parametrize("shift", [0, 2])
def test_remainder_bound_off_by_one_degree_caught(monkeypatch, shift):
    # theta^m / m! (a degree too many) or theta^(m+2) / (m+2)! (one too few):
    # the true truncation error lies far below the bound, so the outputs stay
    # accurate and only the exhaustive search over the rule's definition sees it
    monkeypatch.setattr(oplan, "remainder_bound", _bound_with_power(shift))
    assert caught(lambda: T_plan.test_plan_is_exhaustive_optimum(11.39, "f64"),
                  lambda: T_plan.test_plan_is_exhaustive_optimum(4.38, "f32"))


def test_remainder_bound_far_too_loose_caught_by_expm(monkeypatch):
    # theta^(m+6) / (m+6)!: plans too short to meet the tolerance, which the
    # comparison of their results with scipy's expm detects
    monkeypatch.setattr(oplan, "remainder_bound", _bound_with_power(6))
    assert caught(lambda: T_plan.test_chosen_plan_meets_bound_vs_expm("f32", 4.38))


def test_theta_cap_ignored_caught(monkeypatch):
    orig = oplan.choose
    monkeypatch.setattr(oplan, "choose",
                        lambda nu, tol, theta_max, m_max=oplan.M_MAX, m_min=1: orig(nu, tol, 1e9, m_max, m_min))
    assert caught(lambda: T_plan.test_plan_is_exhaustive_optimum(11.39, "f32"))


# ---- mutants of the adjoint ----

def test_adjoint_reaction_derivative_sign_caught(monkeypatch):
    monkeypatch.setattr(oadj, "reaction_prime", lambda u, rho: rho * (1.0 + 2.0 * u))
    assert caught(lambda: T_adj.test_gradients_vs_central_fd(2, "exp_euler"), lambda: T_adj.test_taylor_remainder_second_order("exp_euler"))


def test_adjoint_forward_mutant_caught(monkeypatch):
    # a wrong Taylor coefficient in the adjoint's own forward pass: consistent
    # with its reverse pass, so only a pin against the integrator catches it
    def taylor_terms(apply_A, x, b, h, m):
        ys = []
        y = h * (apply_A(x) + b)
        ys.append(y)
        for j in range(2, m + 1):
            y = (h / (j + 1)) * apply_A(y)
            ys.append(y)
        return ys
    monkeypatch.setattr(oadj, "taylor_terms", taylor_terms)
    assert caught(T_adj.test_forward_matches_integrator)


# ---- mutants of the linearised step (section 2.1's splitting, section 2.2) ----

def rosenbrock_pins():
    return (
        lambda: T_rb.test_pure_reaction_closed_form(7.3),
        lambda: T_rb.test_step_vs_dense_expm("noflux"),
        T_rb.test_phi1_action_vs_dense,
        T_rb.test_logistic_second_order_convergence,
        T_rb.test_rhs_equals_plain_rhs,
        T_rb.test_uniform_state_takes_scalar_map,
    )


_DIAGONAL_MUTANTS = {
    "sign": lambda u, rho: rho * (2.0 * np.asarray(u, dtype=np.float64) - 1.0),
    "factor": lambda u, rho: rho * (1.0 - np.asarray(u, dtype=np.float64)),
    "none": lambda u, rho: np.zeros_like(np.asarray(u, dtype=np.float64)),
}


@pytest.mark.parametrize("mistake", sorted(_DIAGONAL_MUTANTS))
def test_rosenbrock_diagonal_mutants_caught(monkeypatch, mistake):
    monkeypatch.setattr(orb, "jacobian_diagonal", _DIAGONAL_MUTANTS[mistake])
    assert caught(*rosenbrock_pins()), mistake


def test_rosenbrock_source_dropped_caught(monkeypatch):
    monkeypatch.setattr(orb, "source", lambda u, rho: np.zeros_like(np.asarray(u, dtype=np.float64)))
    assert caught(*rosenbrock_pins())


def test_rosenbrock_whole_reaction_as_source_caught(monkeypatch):
    # the full reaction kept as the source on top of the linear part moved
    # into the matrix: the linear part is counted twice
    monkeypatch.setattr(orb, "source", lambda u, rho: rho * np.asarray(u) * (1.0 - np.asarray(u)))
    assert caught(*rosenbrock_pins())


def test_rosenbrock_phi1_of_A_caught(monkeypatch):
    # phi1 of A instead of J_n: the plain step, first order
    monkeypatch.setattr(orb, "phi1_action",
                        lambda apply_A, u, b, rho, tau, s, m: oit.phi1_action(apply_A, b, tau, s, m))
    assert caught(*rosenbrock_pins())


def test_rosenbrock_jacobian_at_wrong_field_caught(monkeypatch):
    # J taken at the vector phi1 acts on instead of at the state u_n
    monkeypatch.setattr(orb, "phi1_action",
                        lambda apply_A, u, b, rho, tau, s, m: oit.phi1_action(orb.linearised(apply_A, b, rho), b,
                                                                             tau, s, m))
    assert caught(*rosenbrock_pins())


# ---- mutants of the phi1 + phi2 action and the second-order step ----

def exprk2_pins():
    return (
        lambda: T_ek.test_phi12_vs_dense_expm_and_eigh("noflux", 7.3),
        T_ek.test_each_vector_alone,
        lambda: T_ek.test_low_degree_truncations_are_the_taylor_polynomial((3, 3)),
        T_ek.test_pure_reaction_is_heun,
        T_ek.test_logistic_second_order_convergence,
    )


def _phi12_variant(mistake):
    def phi12_action(apply_A, b, d, tau, s, m):
        ref = b if b is not None else d
        zero = np.zeros(np.shape(ref))
        w2 = zero if b is None else np.asarray(b, dtype=np.float64)
        w1 = zero if d is None else np.asarray(d, dtype=np.float64) / (1.0 if mistake == "no_scale" else tau)
        if mistake == "swap":
            w1, w2 = w2 / tau, w1 * tau
        h = tau / s
        x = np.zeros(np.shape(ref))
        eta = np.array([0.0, 1.0])
        J = np.array([[0.0, 1.0], [0.0, 0.0]])
        for _ in range(s):
            acc, acc_eta = x.copy(), eta.copy()
            y, ye = x, eta
            for j in range(1, m + 1):
                by = apply_A(y) + ye[0] * w1 + ye[1] * w2
                be = J @ ye
                y, ye = (h / j) * by, (h / j) * be
                acc, acc_eta = acc + y, acc_eta + ye
            x = acc
            if mistake != "frozen_eta":
                eta = acc_eta
        return x
    return phi12_action


@pytest.mark.parametrize("mistake", ["no_scale", "swap", "frozen_eta"])
def test_phi12_mutants_caught(monkeypatch, mistake):
    monkeypatch.setattr(oek, "phi12_action", _phi12_variant(mistake))
    assert caught(*exprk2_pins()), mistake


def test_exprk2_correction_sign_caught(monkeypatch):
    def step(apply_A, u, rho, tau, s, m):
        u = np.asarray(u, dtype=np.float64)
        U = u + oek.phi12_action(apply_A, oit.rhs(apply_A, u, rho), None, tau, s, m)
        d = oit.reaction(u, rho) - oit.reaction(U, rho)
        return U + oek.phi12_action(apply_A, None, d, tau, s, m)
    monkeypatch.setattr(oek, "step", step)
    assert caught(*exprk2_pins())


def test_exprk2_correction_through_phi1_caught(monkeypatch):
    # the correction weighted by phi1 instead of phi2
    def step(apply_A, u, rho, tau, s, m):
        u = np.asarray(u, dtype=np.float64)
        U = u + oek.phi12_action(apply_A, oit.rhs(apply_A, u, rho), None, tau, s, m)
        d = oit.reaction(U, rho) - oit.reaction(u, rho)
        return U + oek.phi12_action(apply_A, d, None, tau, s, m)
    monkeypatch.setattr(oek, "step", step)
    assert caught(*exprk2_pins())
