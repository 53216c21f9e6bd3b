"""Lab frame on the GPU: the rotation mapping (three spectral shears, eqs.
RSDA1/RSDA2) and Algorithm 1 run literally (mapping before and after every linear
substep, nonlinear substeps with the trap at x), against the FP64 oracle's
rotation_map and its lab-frame evolution mode."""
import numpy as np
import pytest

import oracle
from paper_2603_25282_amd import inputs as I
from tests.gpu_util import rel_l2, to_gpu

pytestmark = pytest.mark.gpu

TOL = {"complex128": 1e-11, "complex64": 5e-5}


def gpu_map(cfg, psi0, t, direction, dtype):
    import torch
    from paper_2603_25282_amd.sgp import Solver
    s = Solver(cfg.shape, cfg.L, cfg.params, dtype=dtype)
    psi = to_gpu(s, psi0)
    s.rotation_map(psi, t, direction)
    torch.cuda.synchronize()
    return Solver.from_device_layout(psi.cpu().numpy().astype(np.complex128))


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("shape", [(32, 64), (16, 32, 32)])
def test_rotation_map_matches_oracle(dtype, shape):
    base = I.C2 if len(shape) == 2 else I.C3
    cfg = I.with_(base, shape=shape, L=8.0 if len(shape) == 2 else 6.0, name="rsda")
    psi0 = I.initial_state(cfg)
    for t, direction in ((0.7, 1), (0.7, -1), (-1.9, 1), (2.6, -1)):
        print(f"case rotation map {shape} {dtype} t={t} dir={direction}", flush=True)
        ref = oracle.rotation_map(psi0, cfg.L, cfg.params, t, forward=direction > 0)
        got = gpu_map(cfg, psi0, t, direction, dtype)
        err = rel_l2(got, ref)
        print("  rel l2", err)
        assert err <= TOL[dtype]


def test_rotation_map_round_trip_and_degenerate_angle():
    from paper_2603_25282_amd.sgp import SgpError, Solver
    cfg = I.with_(I.C2, shape=(64, 64), L=8.0, name="rsda-rt")
    psi0 = I.initial_state(cfg)
    fwd = gpu_map(cfg, psi0, 0.9, 1, "complex128")
    back = gpu_map(cfg, fwd, 0.9, -1, "complex128")
    ref = oracle.rotation_map(oracle.rotation_map(psi0, cfg.L, cfg.params, 0.9, True), cfg.L, cfg.params, 0.9,
                              False)
    assert rel_l2(back, ref) <= 1e-11
    s = Solver(cfg.shape, cfg.L, cfg.params, dtype="complex128")
    t_pi = np.pi / cfg.params[3]  # Omega t = pi: tan(Omega t / 2) is infinite
    with pytest.raises(SgpError):
        s.rotation_map(to_gpu(s, psi0), t_pi, 1)


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("order", [2, 4])
def test_lab_frame_algorithm1_matches_oracle(dtype, order):
    import torch
    from paper_2603_25282_amd.sgp import SgpError, Solver
    cfg = I.with_(I.C2, shape=(64, 64), L=8.0, name="lab")
    psi0 = I.initial_state(cfg)
    tau, n, t0 = 2e-3, 6, 0.15
    print(f"case lab frame 64^2 {dtype} TS{order}", flush=True)
    ref = oracle.evolve(psi0, cfg.L, cfg.params, order, tau, n, t0=t0, frame="lab")
    s = Solver(cfg.shape, cfg.L, cfg.params, dtype=dtype)
    s.set_frame("lab")
    s.build_propagator(tau, order)
    s.time = t0
    psi = to_gpu(s, psi0)
    s.step(psi, n)
    torch.cuda.synchronize()
    got = Solver.from_device_layout(psi.cpu().numpy().astype(np.complex128))
    err = rel_l2(got, ref)
    print("  rel l2", err)
    assert err <= TOL[dtype]
    assert abs(s.time - (t0 + n * tau)) < 1e-15
    # the adjoint is rotating-frame only
    store = torch.empty(s.store_size(1), dtype=torch.uint8, device=psi.device)
    with pytest.raises(SgpError):
        s.step_store(psi, 1, store)


def test_lab_frame_3d_matches_oracle():
    import torch
    from paper_2603_25282_amd.sgp import Solver
    base = I.with_(I.C3, shape=(16, 32, 32), L=6.0, name="lab3d")
    p = list(base.params)
    p[6] = 1.3
    cfg = I.with_(base, params=tuple(p))
    psi0 = I.initial_state(cfg)
    ref = oracle.evolve(psi0, cfg.L, cfg.params, 4, 2e-3, 4, frame="lab")
    s = Solver(cfg.shape, cfg.L, cfg.params, dtype="complex128")
    s.set_frame("lab")
    s.build_propagator(2e-3, 4)
    psi = to_gpu(s, psi0)
    s.step(psi, 4)
    torch.cuda.synchronize()
    err = rel_l2(Solver.from_device_layout(psi.cpu().numpy()), ref)
    print("3D lab frame rel l2", err)
    assert err <= 1e-11
