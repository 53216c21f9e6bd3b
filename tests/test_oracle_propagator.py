"""Pins for the oracle's closed-form exp(i tau Q) (Sec. 3.1): an independent matrix
exponential of i tau Q built from the definition of Q, unitarity, the group law,
P(tau)^H = P(-tau), the gamma = 0 diagonal limit (eq. NonSOCMat) and lam = 0."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from tests.spin2 import Qmat


def draws(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        yield (rng.uniform(-2, 2), rng.uniform(0, 3), rng.uniform(-60, 60), rng.uniform(-60, 60),
               rng.choice([rng.uniform(-1e-3, 1e-3), rng.uniform(-0.1, 0.1), rng.uniform(-2, 2)]))


def test_closed_form_matches_expm():
    worst = 0.0
    for Om, ga, p, q, d in draws(300, 1):
        E = oracle.propagator(Om, ga, p, q, d)
        R = sl.expm(1j * d * Qmat(Om, ga, p, q))
        worst = max(worst, np.abs(E - R).max())
    assert worst < 1e-13


def test_closed_form_matches_eigendecomposition():
    # Second independent route: Q is Hermitian, exp(i d Q) = V diag(exp(i d w)) V^H.
    worst = 0.0
    for Om, ga, p, q, d in draws(100, 2):
        w, V = np.linalg.eigh(Qmat(Om, ga, p, q))
        R = (V * np.exp(1j * d * w)) @ V.conj().T
        worst = max(worst, np.abs(oracle.propagator(Om, ga, p, q, d) - R).max())
    assert worst < 1e-13


def test_unitary_group_law_and_adjoint():
    for Om, ga, p, q, d in draws(100, 3):
        E = oracle.propagator(Om, ga, p, q, d)
        assert np.abs(E.conj().T @ E - np.eye(5)).max() < 1e-13
        E2 = oracle.propagator(Om, ga, p, q, 0.37 * d)
        E3 = oracle.propagator(Om, ga, p, q, 1.37 * d)
        assert np.abs(E @ E2 - E3).max() < 1e-13
        assert np.abs(E.conj().T - oracle.propagator(Om, ga, p, q, -d)).max() < 1e-13


@pytest.mark.parametrize("Om", [0.2, -0.9, 1.5])
def test_gamma_zero_limit(Om):
    d = 0.013
    E = oracle.propagator(Om, 0.0, 3.0, -7.0, d)
    ref = np.diag(np.exp(-1j * d * Om * np.array([2, 1, 0, -1, -2])))
    assert np.abs(E - ref).max() < 1e-15


def test_lambda_zero_is_identity():
    assert np.abs(oracle.propagator(0.0, 0.7, 0.0, 0.0, 0.3) - np.eye(5)).max() == 0.0
    # Omega = 0 with a nonzero wavevector is the pure SOC exponential
    E = oracle.propagator(0.0, 0.7, 1.0, 2.0, 0.3)
    assert np.abs(E - sl.expm(0.3j * Qmat(0.0, 0.7, 1.0, 2.0))).max() < 1e-14
