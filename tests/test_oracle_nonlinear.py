"""Pins for the oracle's exact nonlinear substep (Sec. 3.2, eq. solution2): a high
accuracy ODE integration of the nonlinear subproblem written from its definition,
the invariants of the flow (rho, F, |A00|), the closed-form A00(t), the group law,
and the degenerate limits |F| -> 0, S -> 0 and c1 = c2 = 0."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from tests.spin2 import densities, nl_rhs


def ode_solution(psi, params, V, d):
    def f(t, y):
        r = nl_rhs(y[:5] + 1j * y[5:], params, V)
        return np.concatenate([r.real, r.imag])
    s = solve_ivp(f, (0.0, d), np.concatenate([psi.real, psi.imag]), method="DOP853", rtol=1e-13, atol=1e-15)
    return s.y[:5, -1] + 1j * s.y[5:, -1]


def random_case(rng):
    params = (rng.uniform(0, 500), rng.uniform(-12, 12), rng.uniform(-15, 15), 0, 0, 1, 1, 1)
    psi = (rng.standard_normal(5) + 1j * rng.standard_normal(5)) * rng.uniform(0.05, 0.6)
    return params, psi, rng.uniform(0, 20), rng.uniform(-0.02, 0.02)


def test_matches_ode_integration():
    rng = np.random.default_rng(21)
    worst = 0.0
    for _ in range(25):
        params, psi, V, d = random_case(rng)
        got = oracle.nl_point(params, V, d, psi)
        ref = ode_solution(psi, params, V, d)
        worst = max(worst, np.abs(got - ref).max() / np.abs(ref).max())
    assert worst < 1e-11


def test_invariants_and_A00_phase():
    rng = np.random.default_rng(22)
    for _ in range(200):
        params, psi, V, d = random_case(rng)
        rho0, F0, A0 = densities(psi)
        out = oracle.nl_point(params, V, d, psi)
        rho1, F1, A1 = densities(out)
        assert abs(rho1 - rho0) <= 1e-14 * rho0
        assert np.abs(F1 - F0).max() <= 1e-13 * rho0
        # A00(t) = exp(-2 i t [V + (c0 + c2/5) rho]) A00(0)
        ref = np.exp(-2j * d * (V + (params[0] + params[2] / 5) * rho0)) * A0
        assert abs(A1 - ref) <= 1e-13 * rho0


def test_group_law_and_reversibility():
    rng = np.random.default_rng(23)
    for _ in range(100):
        params, psi, V, d = random_case(rng)
        a = oracle.nl_point(params, V, 0.3 * d, oracle.nl_point(params, V, 0.7 * d, psi))
        b = oracle.nl_point(params, V, d, psi)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(psi).max()
        back = oracle.nl_point(params, V, -d, b)
        assert np.abs(back - psi).max() <= 1e-13 * np.abs(psi).max()


def test_degenerate_limits():
    rng = np.random.default_rng(24)
    params = (120.0, 3.0, -4.0, 0, 0, 1, 1, 1)
    # |F| = 0: a single psi_0 component (F_z = 0, F_+ = 0) -- spin rotation is the identity
    psi = np.array([0, 0, 0.4 + 0.1j, 0, 0], complex)
    got = oracle.nl_point(params, 2.0, 0.01, psi)
    np.testing.assert_allclose(got, ode_solution(psi, params, 2.0, 0.01), atol=1e-13)
    # S = 0: |A00|^2 = rho^2/5, reached by psi = (1, 0, 0, 0, 1)/sqrt2 up to a phase
    psi = np.array([1, 0, 0, 0, 1], complex) * (0.3 / np.sqrt(2)) * np.exp(0.4j)
    rho, F, A00 = densities(psi)
    assert abs((rho / 5) ** 2 - abs(A00) ** 2 / 5) < 1e-16
    got = oracle.nl_point(params, 1.0, 0.02, psi)
    np.testing.assert_allclose(got, ode_solution(psi, params, 1.0, 0.02), atol=1e-13)
    # zero state stays zero
    assert np.all(oracle.nl_point(params, 1.0, 0.02, np.zeros(5, complex)) == 0)
    # c1 = c2 = 0: pure phase exp(-i d (V + c0 rho))
    psi = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    rho = np.vdot(psi, psi).real
    got = oracle.nl_point((50.0, 0.0, 0.0, 0, 0, 1, 1, 1), 3.0, 0.01, psi)
    np.testing.assert_allclose(got, np.exp(-0.01j * (3.0 + 50.0 * rho)) * psi, atol=1e-14)


def test_tiny_spin_density_is_smooth():
    # |F| -> 0 continuously: the result must approach the |F| = 0 value, no 0/0.
    params = (100.0, -5.0, 10.0, 0, 0, 1, 1, 1)
    base = np.array([0, 0, 0.5, 0, 0], complex)
    pert = np.array([1e-9, 0, 0, 0, 0], complex)
    a = oracle.nl_point(params, 0.5, 0.01, base + pert)
    b = ode_solution(base + pert, params, 0.5, 0.01)
    assert np.abs(a - b).max() < 1e-13
