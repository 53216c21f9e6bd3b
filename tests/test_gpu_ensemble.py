"""Batched ensemble of uneven 2D grids: one launch per pass type over all instances.
Each instance must match (bitwise) its own unbatched evolution and the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2603_25282_amd import inputs as I
from tests.gpu_util import rel_l2, run_gpu

pytestmark = pytest.mark.gpu


def make(insts, dtype):
    import torch
    from paper_2603_25282_amd.sgp import Ensemble, Solver
    ens = Ensemble([c.shape for c in insts], [c.L for c in insts], [c.params for c in insts], dtype=dtype)
    psis = [torch.from_numpy(Solver.to_device_layout(I.initial_state(c))).to(ens.torch_dtype).cuda().contiguous()
            for c in insts]
    return ens, psis


def test_384_single_grid_radix3():
    cfg = I.with_(I.C1, shape=(384, 384), L=12.0, name="c1-384")
    psi0 = I.initial_state(cfg)
    for dtype, tol in (("complex128", 1e-11), ("complex64", 5e-5)):
        print(f"case 384^2 {dtype}", flush=True)
        ref = oracle.evolve(psi0, cfg.L, cfg.params, 2, cfg.tau, 5)
        got, _ = run_gpu(cfg.shape, cfg.L, cfg.params, psi0, 2, cfg.tau, 5, dtype=dtype)
        err = rel_l2(got, ref)
        print("rel l2", err)
        assert err <= tol


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("order", [2, 4])
def test_small_ensemble_batched_equals_unbatched_and_oracle(dtype, order):
    import torch
    from paper_2603_25282_amd.sgp import SGP_OPT_BATCHED, Solver
    insts = I.ensemble_instances(seed=4, n128=2, n256=1, n384=2, L=12.0, order=order, tau=1e-3, steps=0)
    insts = [I.with_(insts[0], shape=(64, 64), L=8.0, name="e64")] + insts
    nsteps = 20  # > 16: one graph replay plus remainder
    print(f"case ensemble {len(insts)} instances {dtype} TS{order}", flush=True)
    ens, psis = make(insts, dtype)
    ens.build_propagator(1e-3, order)
    ens.step(psis, nsteps)
    ens2, psis2 = make(insts, dtype)
    ens2.build_propagator(1e-3, order)
    ens2.set_option(SGP_OPT_BATCHED, 0)
    ens2.step(psis2, nsteps)
    torch.cuda.synchronize()
    for k, c in enumerate(insts):
        a = psis[k].cpu().numpy()
        b = psis2[k].cpu().numpy()
        assert np.array_equal(a, b), f"instance {k} ({c.shape}) batched != unbatched"
    tol = 1e-11 if dtype == "complex128" else 5e-5
    for k in (0, 1, 4):
        c = insts[k]
        ref = oracle.evolve(I.initial_state(c), c.L, c.params, order, 1e-3, nsteps)
        got = Solver.from_device_layout(psis[k].cpu().numpy().astype(np.complex128))
        err = rel_l2(got, ref)
        print(f"instance {k} {c.shape} rel l2 {err:.3e}")
        assert err <= tol


def test_full_ensemble_workload_consistency():
    # The 96-instance workload (32 x 128^2, 48 x 256^2, 16 x 384^2), 40 TS2 steps:
    # batched == unbatched bitwise for every instance, finite, and one instance of
    # each size against the oracle.
    import torch
    from paper_2603_25282_amd.sgp import SGP_OPT_BATCHED, Solver
    insts = I.ensemble_instances(steps=40)
    ens, psis = make(insts, "complex64")
    ens.build_propagator(1e-3, 2)
    ens.step(psis, 40)
    ens2, psis2 = make(insts, "complex64")
    ens2.build_propagator(1e-3, 2)
    ens2.set_option(SGP_OPT_BATCHED, 0)
    ens2.step(psis2, 40)
    torch.cuda.synchronize()
    for k in range(len(insts)):
        assert torch.equal(psis[k], psis2[k]), f"instance {k}"
    for k in (0, 40, 90):
        c = insts[k]
        ref = oracle.evolve(I.initial_state(c), c.L, c.params, 2, 1e-3, 40)
        got = Solver.from_device_layout(psis[k].cpu().numpy().astype(np.complex128))
        err = rel_l2(got, ref)
        print(f"instance {k} {c.shape} rel l2 {err:.3e}")
        assert err <= 5e-5
