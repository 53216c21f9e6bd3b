"""GPU adjoint (C ABI sgp_step_store / sgp_adjoint_segment and the autograd
Function) against the FP64 oracle's discrete adjoint and against finite differences
of the GPU forward.  Gradient convention: 2 dJ/d conj(psi)."""
import numpy as np
import pytest

import oracle
from paper_2603_25282_amd import inputs as I
from tests.adjoint_loss import loss_and_grad
from tests.gpu_util import rel_l2
from tests.test_oracle_scheme import smooth_state

pytestmark = pytest.mark.gpu

PIDX = [4, 3, 0, 1, 2]  # (gamma, Omega, c0, c1, c2) in the params tuple


def gpu_adjoint(psi0, gT, L, params, order, tau, n, K, dtype):
    import torch
    from paper_2603_25282_amd.autograd import evolve
    from paper_2603_25282_amd.sgp import Solver
    dev = torch.device("cuda:0")
    tdt = torch.complex64 if dtype == "complex64" else torch.complex128
    p0 = torch.from_numpy(Solver.to_device_layout(psi0)).to(tdt).to(dev).requires_grad_(True)
    par = torch.tensor([params[i] for i in PIDX], dtype=torch.float64, requires_grad=True)
    out = evolve(p0, par, psi0.shape[1:], L, params[5:8], tau, n, order=order, K=K)
    g = torch.from_numpy(Solver.to_device_layout(gT)).to(tdt).to(dev)
    # J = Re sum conj(gT) phi_T  ->  dJ = Re <gT, dphi>, so the incoming gradient is gT
    J = torch.sum((torch.conj(g) * out).real)
    J.backward()
    g0 = Solver.from_device_layout(p0.grad.cpu().numpy().astype(np.complex128))
    return g0, par.grad.numpy(), Solver.from_device_layout(out.detach().cpu().numpy().astype(np.complex128))


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("order", [2, 4, 6])
def test_adjoint_matches_oracle_adjoint(dtype, order):
    params = (60.0, -2.0, 3.0, 0.7, 0.9, 1.0, 1.2, 1.0)
    L, shape = 6.0, (32, 32)
    psi = smooth_state(shape, L, 21, lz=0.3)
    w = np.random.default_rng(5).standard_normal(psi.shape) + 1j * np.random.default_rng(6).standard_normal(psi.shape)
    tau, n = 4e-3, 7
    print(f"case adjoint 32^2 {dtype} TS{order}", flush=True)
    g_ref, d_ref = oracle.adjoint(psi, w, L, params, order, tau, n, K=3)
    g, d, _ = gpu_adjoint(psi, w, L, params, order, tau, n, K=3, dtype=dtype)
    eg = rel_l2(g, g_ref)
    ed = np.abs(d - d_ref) / np.maximum(1.0, np.abs(d_ref))
    print("state grad rel l2", eg, "param grads", d, "oracle", d_ref, "rel", ed)
    tol = 1e-11 if dtype == "complex128" else 5e-5
    assert eg <= tol
    assert np.all(ed <= (1e-10 if dtype == "complex128" else 2e-4))


def test_workload_loss_gradients_fd_and_oracle():
    # The differentiation workload's loss on 64^2 with checkpoints: GPU FP64 adjoint vs
    # oracle adjoint, and the GPU FP32 adjoint vs central finite differences of the
    # GPU FP64 forward (relative 1e-4).
    import torch
    from paper_2603_25282_amd.autograd import evolve
    from paper_2603_25282_amd.sgp import Solver
    cfg = I.with_(I.C5, shape=(64, 64), L=8.0)
    psi0 = I.initial_state(I.with_(cfg, init="gauss_phase"))
    psi0 = smooth_state(cfg.shape, cfg.L, 41, lz=0.4)
    target = smooth_state(cfg.shape, cfg.L, 42, lz=0.1)
    tau, n, K = 1e-3, 12, 5
    u = oracle.evolve(psi0, cfg.L, cfg.params, 4, tau, n)
    J0, gT = loss_and_grad(u, target, cfg.L)
    g_ref, d_ref = oracle.adjoint(psi0, gT, cfg.L, cfg.params, 4, tau, n, K=K)
    g64, d64, out64 = gpu_adjoint(psi0, gT, cfg.L, cfg.params, 4, tau, n, K, "complex128")
    assert rel_l2(out64, u) < 1e-11
    assert rel_l2(g64, g_ref) < 1e-10
    assert np.all(np.abs(d64 - d_ref) <= 1e-9 * np.maximum(1.0, np.abs(d_ref)))

    def J_gpu(p0, params):
        s = Solver(cfg.shape, cfg.L, params, dtype="complex128")
        s.build_propagator(tau, 4)
        t = torch.from_numpy(Solver.to_device_layout(p0)).cuda()
        s.step(t, n)
        phi = Solver.from_device_layout(t.cpu().numpy())
        return loss_and_grad(phi, target, cfg.L)[0]

    g32, d32, _ = gpu_adjoint(psi0, gT, cfg.L, cfg.params, 4, tau, n, K, "complex64")
    eps = 1e-6
    rng = np.random.default_rng(9)
    for _ in range(2):
        v = rng.standard_normal(psi0.shape) + 1j * rng.standard_normal(psi0.shape)
        fd = (J_gpu(psi0 + eps * v, cfg.params) - J_gpu(psi0 - eps * v, cfg.params)) / (2 * eps)
        an = np.real(np.vdot(g32, v))
        print("state direction fd", fd, "adjoint fp32", an)
        assert abs(fd - an) <= 1e-4 * max(1e-3, abs(fd))
    for k, i in enumerate(PIDX):
        pp, pm = list(cfg.params), list(cfg.params)
        pp[i] += eps
        pm[i] -= eps
        fd = (J_gpu(psi0, pp) - J_gpu(psi0, pm)) / (2 * eps)
        print("param", k, "fd", fd, "adjoint fp32", d32[k], "fp64", d64[k])
        assert abs(fd - d32[k]) <= 1e-4 * max(1e-3, abs(fd))


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_differentiation_workload_full(dtype):
    # Full differentiation workload: 256^2 on [-12, 12]^2, TS4, tau = 1e-3, 500 steps,
    # checkpoints every 50 steps; loss of tests/adjoint_loss.py.  Against the oracle's
    # stored J, dJ/d(gamma, Omega, c0, c1, c2) and whole state gradient
    # (tests/golden/make_c5_reference.py calls only the oracle).
    import os
    import torch
    from paper_2603_25282_amd.autograd import evolve
    from paper_2603_25282_amd.sgp import Solver
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "c5_reference.npz"))
    cfg = I.C5
    psi0 = I.initial_state(cfg)
    target = I.initial_state(I.with_(cfg, seed=cfg.extra["target_seed"]))
    tdt = torch.complex64 if dtype == "complex64" else torch.complex128
    dev = torch.device("cuda:0")
    prm = cfg.params
    print(f"case differentiation workload {cfg.shape} {dtype} steps={cfg.steps} K={cfg.extra['K']}", flush=True)
    p0 = torch.from_numpy(Solver.to_device_layout(psi0)).to(tdt).to(dev).requires_grad_(True)
    par = torch.tensor([prm[i] for i in PIDX], dtype=torch.float64, requires_grad=True)
    out = evolve(p0, par, cfg.shape, cfg.L, prm[5:8], cfg.tau, cfg.steps, order=cfg.order, K=cfg.extra["K"])
    phi = Solver.from_device_layout(out.detach().cpu().numpy().astype(np.complex128))
    J, gT = loss_and_grad(phi, target, cfg.L)
    out.backward(torch.from_numpy(Solver.to_device_layout(gT)).to(tdt).to(dev))
    g0 = Solver.from_device_layout(p0.grad.cpu().numpy().astype(np.complex128))
    d = par.grad.numpy()
    eg = rel_l2(g0, ref["g0"])
    eJ = abs(J - float(ref["J"])) / abs(float(ref["J"]))
    ed = np.abs(d - ref["dpar"]) / np.abs(ref["dpar"])
    print(f"J {J} (oracle {float(ref['J'])}, rel {eJ:.2e}); full state gradient rel l2 {eg:.2e}; "
          f"dpar {d} (oracle {ref['dpar']}, rel {ed})", flush=True)
    if dtype == "complex128":
        assert eJ <= 1e-10 and eg <= 1e-10 and np.all(ed <= 1e-8)
    else:
        assert eJ <= 1e-4 and eg <= 1e-4 and np.all(ed <= 1e-3)


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("order", [2, 4])
def test_3d_adjoint_matches_oracle_adjoint(dtype, order):
    # 3D adjoint passes (X adjoint; y forward, z adjoint with the propagator partials,
    # y inverse) on an anisotropic rotating trap, with checkpoints
    params = (40.0, -1.5, 2.0, 0.6, 0.8, 1.0, 1.3, 2.0)
    L, shape = 5.0, (16, 16, 32)
    from paper_2603_25282_amd import inputs as II
    cfg = II.with_(II.C3, shape=shape, L=L, params=params, name="adj3d")
    psi = II.initial_state(cfg)
    w = np.random.default_rng(9).standard_normal(psi.shape) + 1j * np.random.default_rng(10).standard_normal(psi.shape)
    tau, n = 3e-3, 5
    print(f"case 3D adjoint {shape} {dtype} TS{order}", flush=True)
    g_ref, d_ref = oracle.adjoint(psi, w, L, params, order, tau, n, K=2)
    g, d, _ = gpu_adjoint(psi, w, L, params, order, tau, n, K=2, dtype=dtype)
    eg = rel_l2(g, g_ref)
    ed = np.abs(d - d_ref) / np.maximum(1.0, np.abs(d_ref))
    print("state grad rel l2", eg, "param grads", d, "oracle", d_ref, "rel", ed)
    tol = 1e-11 if dtype == "complex128" else 5e-5
    assert eg <= tol
    assert np.all(ed <= (1e-10 if dtype == "complex128" else 2e-4))


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_evolve_keeps_last_segment_and_second_backward(dtype):
    # evolve runs the last checkpoint segment with stores and the first backward uses
    # them without recomputing it: the output equals plain steps in the same chunks
    # bitwise, a second backward (recomputing every segment) gives bitwise the same
    # gradients, and both match the oracle's discrete adjoint
    import torch
    from paper_2603_25282_amd.autograd import evolve
    from paper_2603_25282_amd.sgp import Solver
    cfg = I.with_(I.C5, shape=(64, 64), L=8.0)
    psi0 = I.initial_state(I.with_(cfg, init="gauss_phase"))
    prm = cfg.params
    tau, n, K = 1e-3, 7, 3
    tdt = torch.complex64 if dtype == "complex64" else torch.complex128
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(21)
    w = rng.standard_normal(psi0.shape) + 1j * rng.standard_normal(psi0.shape)
    print(f"case evolve last-segment store {dtype}", flush=True)
    p0 = torch.from_numpy(Solver.to_device_layout(psi0)).to(tdt).to(dev).requires_grad_(True)
    par = torch.tensor([prm[i] for i in PIDX], dtype=torch.float64, requires_grad=True)
    out = evolve(p0, par, cfg.shape, cfg.L, prm[5:8], tau, n, order=4, K=K)
    s = Solver(cfg.shape, cfg.L, prm, dtype=dtype)
    s.build_propagator(tau, 4)
    q = p0.detach().clone()
    for ns in (3, 3, 1):
        s.step(q, ns)
    torch.cuda.synchronize()
    assert torch.equal(out.detach(), q)
    g = torch.from_numpy(Solver.to_device_layout(w)).to(tdt).to(dev)
    J = torch.sum((torch.conj(g) * out).real)
    J.backward(retain_graph=True)
    g1, d1 = p0.grad.clone(), par.grad.clone()
    p0.grad, par.grad = None, None
    J.backward()
    assert torch.equal(p0.grad, g1) and torch.equal(par.grad, d1)
    g_ref, d_ref = oracle.adjoint(psi0, w, cfg.L, prm, 4, tau, n, K=K)
    eg = rel_l2(Solver.from_device_layout(g1.cpu().numpy().astype(np.complex128)), g_ref)
    ed = np.abs(d1.numpy() - d_ref) / np.maximum(1.0, np.abs(d_ref))
    print(f"  state grad {eg:.3e}, params {ed}", flush=True)
    assert eg <= (1e-11 if dtype == "complex128" else 5e-5)
    assert np.all(ed <= (1e-10 if dtype == "complex128" else 2e-4))


@pytest.mark.parametrize("shape", [(32, 64), (16, 16, 16)])
@pytest.mark.parametrize("order", [2, 4])
def test_dot_product_of_the_linear_step(shape, order):
    # With c0 = c1 = c2 = 0 the split step is linear in the state (the nonlinear flow
    # reduces to the trap phase), so the adjoint must satisfy Re<w, S v> = Re<S^H w, v>
    # to rounding, for any v and w: a check of the adjoint that needs no oracle.
    L = 6.0
    params = (0.0, 0.0, 0.0, 0.7, 0.9, 1.0, 1.2, 1.5)
    rng = np.random.default_rng(31)
    v = rng.standard_normal((5,) + shape) + 1j * rng.standard_normal((5,) + shape)
    w = rng.standard_normal((5,) + shape) + 1j * rng.standard_normal((5,) + shape)
    print(f"case dot product {shape} TS{order}", flush=True)
    g0, _, Sv = gpu_adjoint(v, w, L, params, order, 4e-3, 9, K=4, dtype="complex128")
    lhs = np.sum(np.conj(w) * Sv).real
    rhs = np.sum(np.conj(g0) * v).real
    scale = np.linalg.norm(w) * np.linalg.norm(Sv)
    print("  Re<w, Sv>", lhs, "Re<S^H w, v>", rhs, "rel", abs(lhs - rhs) / scale, flush=True)
    assert abs(lhs - rhs) <= 1e-12 * scale
