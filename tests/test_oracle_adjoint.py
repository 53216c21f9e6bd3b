"""Pins for the oracle's discrete adjoint: central finite differences of the FP64
forward evolution (state directions and the five parameters), independence of the
checkpoint interval, and the loss of the differentiation workload."""
import numpy as np
import pytest

import oracle
from paper_2603_25282_amd import inputs as I
from tests.adjoint_loss import loss_and_grad
from tests.test_oracle_scheme import smooth_state

PNAMES = ["gamma", "Omega", "c0", "c1", "c2"]
PIDX = {"gamma": 4, "Omega": 3, "c0": 0, "c1": 1, "c2": 2}


def setup(shape=(32, 32), L=6.0, aniso=1.2):
    params = (60.0, -2.0, 3.0, 0.7, 0.9, 1.0, aniso, 1.0)
    psi = smooth_state(shape, L, 21, lz=0.3)
    return params, psi, L


def forward_J(psi, params, L, w, order, tau, n):
    u = oracle.evolve(psi, L, params, order, tau, n)
    return np.real(np.vdot(w, u))


@pytest.mark.parametrize("order", [2, 4])
def test_linear_functional_matches_finite_differences(order):
    params, psi, L = setup()
    rng = np.random.default_rng(5)
    w = rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape)
    tau, n = 4e-3, 6
    g0, dpar = oracle.adjoint(psi, w, L, params, order, tau, n, K=4)
    eps = 1e-6
    for _ in range(3):
        v = rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape)
        fd = (forward_J(psi + eps * v, params, L, w, order, tau, n) -
              forward_J(psi - eps * v, params, L, w, order, tau, n)) / (2 * eps)
        assert abs(fd - np.real(np.vdot(g0, v))) <= 1e-6 * max(1.0, abs(fd))
    for k, name in enumerate(PNAMES):
        pp = list(params); pm = list(params)
        i = PIDX[name]
        pp[i] += eps; pm[i] -= eps
        fd = (forward_J(psi, pp, L, w, order, tau, n) - forward_J(psi, pm, L, w, order, tau, n)) / (2 * eps)
        assert abs(fd - dpar[k]) <= 1e-6 * max(1.0, abs(fd)), (name, fd, dpar[k])


def test_checkpoint_interval_does_not_change_the_gradient():
    params, psi, L = setup()
    w = np.random.default_rng(6).standard_normal(psi.shape) + 0j
    a = oracle.adjoint(psi, w, L, params, 4, 3e-3, 7, K=1)
    b = oracle.adjoint(psi, w, L, params, 4, 3e-3, 7, K=7)
    c = oracle.adjoint(psi, w, L, params, 4, 3e-3, 7, K=3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[0], c[0])
    assert np.allclose(a[1], b[1], rtol=1e-14, atol=1e-14) and np.allclose(a[1], c[1], rtol=1e-14, atol=1e-14)


def test_workload_loss_gradient_matches_finite_differences():
    # The loss of the differentiation workload on a reduced grid and horizon.
    cfg = I.with_(I.C5, shape=(32, 32), L=6.0)
    psi = I.initial_state(I.with_(cfg, init="gauss_phase"))
    psi = smooth_state(cfg.shape, cfg.L, 31, lz=0.4)
    target = smooth_state(cfg.shape, cfg.L, 32, lz=0.1)
    tau, n = 2e-3, 8

    def J_of(p0, params):
        u = oracle.evolve(p0, cfg.L, params, 4, tau, n)
        return loss_and_grad(u, target, cfg.L)[0]

    u = oracle.evolve(psi, cfg.L, cfg.params, 4, tau, n)
    J, gT = loss_and_grad(u, target, cfg.L)
    g0, dpar = oracle.adjoint(psi, gT, cfg.L, cfg.params, 4, tau, n, K=3)
    rng = np.random.default_rng(7)
    eps = 1e-6
    for _ in range(2):
        v = rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape)
        fd = (J_of(psi + eps * v, cfg.params) - J_of(psi - eps * v, cfg.params)) / (2 * eps)
        assert abs(fd - np.real(np.vdot(g0, v))) <= 1e-6 * max(1.0, abs(fd))
    for k, name in enumerate(PNAMES):
        pp = list(cfg.params); pm = list(cfg.params)
        pp[PIDX[name]] += eps; pm[PIDX[name]] -= eps
        fd = (J_of(psi, pp) - J_of(psi, pm)) / (2 * eps)
        assert abs(fd - dpar[k]) <= 1e-6 * max(1.0, abs(fd)), (name, fd, dpar[k])
