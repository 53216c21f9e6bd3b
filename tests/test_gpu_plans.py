"""Every register plan (elements per thread E of the FFT line kernels, set per axis)
against the FP64 oracle, through the C ABI; the autotuner's choice and its JSON
plan cache.  All plans compute the same transforms, so each must meet the same
tolerances as the default plan."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2603_25282_amd import inputs as I
from tests.gpu_util import rel_l2, to_gpu

pytestmark = pytest.mark.gpu

TOL = {"complex128": 1e-11, "complex64": 5e-5}


def run_plan(cfg, dtype, widths, steps, order=4, tau=1e-3):
    import torch
    from paper_2603_25282_amd.sgp import Solver
    psi0 = I.initial_state(cfg)
    s = Solver(cfg.shape, cfg.L, cfg.params, dtype=dtype)
    s.set_plan(widths)
    assert s.get_plan() == list(widths)
    s.build_propagator(tau, order)
    psi = to_gpu(s, psi0)
    s.step(psi, steps)
    torch.cuda.synchronize()
    got = Solver.from_device_layout(psi.cpu().numpy().astype(np.complex128))
    return got, psi0, s


def plans_2d(nx, ny, dtype="complex64"):
    from paper_2603_25282_amd.sgp import plan_widths
    return [(ex, ey) for ex in plan_widths(nx, dtype) for ey in plan_widths(ny, dtype)]


@pytest.mark.parametrize("n", [16, 64, 128, 256])
@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_every_plan_2d(n, dtype):
    cfg = I.with_(I.C2, shape=(n, n), L=8.0, name=f"plans-{n}")
    ref = None
    for widths in plans_2d(n, n, dtype):
        print(f"case plans 2D {n}^2 {dtype} widths={widths}", flush=True)
        got, psi0, _ = run_plan(cfg, dtype, widths, steps=6)
        if ref is None:
            ref = oracle.evolve(psi0, cfg.L, cfg.params, 4, 1e-3, 6)
        err = rel_l2(got, ref)
        print("  rel l2", err)
        assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_every_plan_512_and_384(dtype):
    # the full 512 lines with each plan (x and y set independently), and 384 lines
    # (E = 12 / 24) in a rectangular grid
    cfg = I.C2
    psi0 = I.initial_state(cfg)
    ref = oracle.evolve(psi0, cfg.L, cfg.params, cfg.order, cfg.tau, 2)
    for widths in plans_2d(512, 512, dtype):
        print(f"case plans 512^2 {dtype} widths={widths}", flush=True)
        got, _, _ = run_plan(cfg, dtype, widths, steps=2, tau=cfg.tau)
        err = rel_l2(got, ref)
        print("  rel l2", err)
        assert err <= TOL[dtype]
    rc = I.with_(I.C2, shape=(64, 384), L=12.0, name="rect-384")
    psi0 = I.initial_state(rc)
    ref = oracle.evolve(psi0, rc.L, rc.params, 4, 1e-3, 4)
    for widths in plans_2d(384, 64, dtype):
        print(f"case plans 64x384 {dtype} widths={widths}", flush=True)
        got, _, _ = run_plan(rc, dtype, widths, steps=4)
        err = rel_l2(got, ref)
        print("  rel l2", err)
        assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_every_plan_192_and_768(dtype):
    # the other 3 * 2^k lengths (radix 3 with radix 4, or radix 8), x = 768 and
    # y = 192 in one rectangular grid, every plan pair
    cfg = I.with_(I.C2, shape=(192, 768), L=24.0, name="rect-192-768")
    psi0 = I.initial_state(cfg)
    ref = oracle.evolve(psi0, cfg.L, cfg.params, 4, 1e-3, 3)
    for widths in plans_2d(768, 192, dtype):
        print(f"case plans 192x768 {dtype} widths={widths}", flush=True)
        got, _, _ = run_plan(cfg, dtype, widths, steps=3)
        err = rel_l2(got, ref)
        print("  rel l2", err)
        assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_plans_3d(dtype):
    base = I.with_(I.C3, shape=(16, 32, 64), name="c3-plans")
    p = list(base.params)
    p[6] = 1.3
    cfg = I.with_(base, params=tuple(p))
    psi0 = I.initial_state(cfg)
    ref = oracle.evolve(psi0, cfg.L, cfg.params, 4, 1e-3, 4)
    # the fourth entry: the linear substep's split (0: whole propagator in the
    # z-pass; 1: its spin part in the forward y-pass)
    for widths in [(4, 4, 4, 0), (16, 8, 4, 1), (4, 8, 8, 0), (4, 8, 8, 1), (16, 4, 8, 1), (8, 4, 8, 0)]:
        print(f"case plans 3D {cfg.shape} {dtype} widths={widths}", flush=True)
        got, _, _ = run_plan(cfg, dtype, widths, steps=4)
        err = rel_l2(got, ref)
        print("  rel l2", err)
        assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_observables_with_plans(dtype):
    from paper_2603_25282_amd.sgp import Solver
    cfg = I.with_(I.C2, shape=(128, 128))
    psi0 = I.initial_state(cfg)
    ref = oracle.observables(psi0, cfg.L, cfg.params, theta=cfg.params[3] * 0.25)
    tol = 1e-12 if dtype == "complex128" else 2e-6
    scale = np.array([1.0, abs(ref[1]) + 1.0, 1.0, 1.0])
    for widths in [(4, 16), (16, 4)]:
        s = Solver(cfg.shape, cfg.L, cfg.params, dtype=dtype)
        s.set_plan(widths)
        s.time = 0.25
        got = s.observables(to_gpu(s, psi0))
        print(f"case observables plans {widths} {dtype}: gpu {got} oracle {ref}", flush=True)
        assert np.all(np.abs(got - ref) <= tol * scale)


def test_adjoint_with_plans_matches_default_plan():
    # the adjoint passes follow the plan too: FP64 gradients of every plan agree
    import torch
    from paper_2603_25282_amd.autograd import evolve
    from paper_2603_25282_amd.sgp import Solver
    cfg = I.with_(I.C5, shape=(64, 64), L=8.0)
    psi0 = I.initial_state(I.with_(cfg, init="gauss_phase"))
    w = np.random.default_rng(11).standard_normal(psi0.shape) + 1j * np.random.default_rng(12).standard_normal(
        psi0.shape)
    prm = cfg.params
    res = []
    for plan in (None, (4, 16), (16, 4)):
        print(f"case adjoint plan {plan}", flush=True)
        p0 = torch.from_numpy(Solver.to_device_layout(psi0)).cuda().requires_grad_(True)
        par = torch.tensor([prm[4], prm[3], prm[0], prm[1], prm[2]], dtype=torch.float64, requires_grad=True)
        out = evolve(p0, par, cfg.shape, cfg.L, prm[5:8], 1e-3, 9, order=4, K=4, plan=plan)
        g = torch.from_numpy(Solver.to_device_layout(w)).cuda()
        torch.sum((torch.conj(g) * out).real).backward()
        res.append((p0.grad.cpu().numpy(), par.grad.numpy()))
    for g0, dp in res[1:]:
        assert rel_l2(g0, res[0][0]) <= 1e-12
        assert np.all(np.abs(dp - res[0][1]) <= 1e-10 * np.maximum(1.0, np.abs(res[0][1])))


def test_autotune_choice_cache_and_parity(tmp_path, monkeypatch):
    import torch
    from paper_2603_25282_amd.sgp import Solver, plan_widths
    monkeypatch.setenv("SGP_PLAN_CACHE", str(tmp_path / "plans.json"))
    cfg = I.with_(I.C2, shape=(128, 256), L=8.0, name="tune")
    psi0 = I.initial_state(cfg)
    s = Solver(cfg.shape, cfg.L, cfg.params, dtype="complex64")
    s.build_propagator(1e-3, 4)
    s.time = 0.05
    psi = to_gpu(s, psi0)
    widths, ms = s.autotune(psi, 4, steps=4)
    print("autotuned", widths, ms, flush=True)
    assert widths[0] in plan_widths(256) and widths[1] in plan_widths(128)
    assert ms is not None and ms > 0
    assert s.get_plan() == widths
    assert abs(s.time - 0.05) < 1e-15  # context time restored
    # the caller's state is untouched (the tuner ran on a scratch copy)
    assert np.array_equal(Solver.from_device_layout(psi.cpu().numpy()).astype(np.complex128),
                          psi0.astype(np.complex64).astype(np.complex128))
    # the chosen plan is correct
    s.step(psi, 5)
    torch.cuda.synchronize()
    got = Solver.from_device_layout(psi.cpu().numpy().astype(np.complex128))
    ref = oracle.evolve(psi0, cfg.L, cfg.params, 4, 1e-3, 5, t0=0.05)
    assert rel_l2(got, ref) <= 5e-5
    # the cache: a second solver takes the stored choice without timing
    table = json.load(open(os.environ["SGP_PLAN_CACHE"]))
    assert table[s.plan_key(4)]["widths"] == widths
    s2 = Solver(cfg.shape, cfg.L, cfg.params, dtype="complex64")
    s2.build_propagator(1e-3, 4)
    w2, ms2 = s2.autotune(to_gpu(s2, psi0), 4)
    assert w2 == widths and ms2 is None


def test_autotune_3d_picks_widths_and_split(tmp_path, monkeypatch):
    # in 3D the tuner also chooses the linear substep's split; its choice is a
    # four-entry plan that round-trips through the cache and is correct
    import torch
    from paper_2603_25282_amd.sgp import Solver, plan_widths
    monkeypatch.setenv("SGP_PLAN_CACHE", str(tmp_path / "plans.json"))
    cfg = I.with_(I.C3, shape=(16, 32, 32), name="tune3d")
    psi0 = I.initial_state(cfg)
    s = Solver(cfg.shape, cfg.L, cfg.params, dtype="complex64")
    s.build_propagator(1e-3, 4)
    psi = to_gpu(s, psi0)
    widths, ms = s.autotune(psi, 4, steps=2)
    print("autotuned 3D", widths, ms, flush=True)
    assert len(widths) == 4 and widths[3] in (0, 1)
    assert widths[0] in plan_widths(32) and widths[1] in plan_widths(32) and widths[2] in plan_widths(16)
    assert s.get_plan() == widths
    s.step(psi, 3)
    torch.cuda.synchronize()
    got = Solver.from_device_layout(psi.cpu().numpy().astype(np.complex128))
    assert rel_l2(got, oracle.evolve(psi0, cfg.L, cfg.params, 4, 1e-3, 3)) <= 5e-5
    s2 = Solver(cfg.shape, cfg.L, cfg.params, dtype="complex64")
    s2.build_propagator(1e-3, 4)
    w2, ms2 = s2.autotune(to_gpu(s2, psi0), 4)
    assert w2 == widths and ms2 is None
