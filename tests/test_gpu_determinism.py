"""Determinism of the GPU path: the same inputs give bitwise the same outputs on
every run (no atomics in any reduction: block partials are summed in a fixed
order), for single-grid steps (graph replay included), observables and
diagnostics, the adjoint's state and parameter gradients, and batched ensembles."""
import numpy as np
import pytest

from paper_2603_25282_amd import inputs as I
from paper_2603_25282_amd.sgp import Ensemble, Solver
from tests.gpu_util import to_gpu

pytestmark = pytest.mark.gpu

PARAMS = (120.0, -2.0, 4.0, 0.7, 0.8, 1.0, 1.1, 1.5)


def _state(shape, L, seed):
    rng = np.random.default_rng(seed)
    co = I.mesh(shape, L)
    g = np.exp(-sum(c * c for c in co) / 2.0)
    return I.normalise(g[None] * np.exp(1j * rng.uniform(0, 2 * np.pi, (5,) + shape)), shape, L)


def _run(shape, dtype, psi0, n):
    s = Solver(shape, 8.0, PARAMS, dtype=dtype)
    s.build_propagator(1e-3, 4)
    psi = to_gpu(s, psi0)
    s.step(psi, n)
    return psi, s.observables(psi), np.array(list(s.diagnostics(psi).values()))


@pytest.mark.parametrize("shape,dtype", [((128, 256), "complex64"), ((256, 128), "complex128"),
                                         ((32, 64, 32), "complex64")])
def test_steps_and_reductions_repeat_bitwise(shape, dtype):
    import torch
    print(f"case determinism {shape} {dtype}", flush=True)
    psi0 = _state(shape, 8.0, 41)
    a, oa, da = _run(shape, dtype, psi0, 40)  # 40 steps: graph replay for 32 of them
    b, ob, db = _run(shape, dtype, psi0, 40)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert np.array_equal(oa, ob) and np.array_equal(da, db)


@pytest.mark.parametrize("shape,dtype,slabs", [((32, 64, 32), "complex64", 4), ((32, 32, 64), "complex128", 2),
                                               ((32, 16, 16), "complex64", 32)])
def test_z_slab_body_is_bitwise_the_plain_body(shape, dtype, slabs):
    # the pipelined graph body runs the same kernels on the same lines, in z-slabs on
    # two streams: bitwise the same state (40 steps: graph replays of 1..32 steps)
    import torch
    print(f"case z-slabs {shape} {dtype} {slabs}", flush=True)
    psi0 = _state(shape, 8.0, 43)
    outs = []
    for S in (0, slabs):
        s = Solver(shape, 8.0, PARAMS, dtype=dtype)
        s.build_propagator(1e-3, 4)
        s.set_slabs(S)
        psi = to_gpu(s, psi0)
        s.step(psi, 40)
        s.step(psi, 3)
        torch.cuda.synchronize()
        outs.append(psi)
    assert torch.equal(outs[0], outs[1])


def test_z_slabs_rejected_where_they_do_not_fit():
    from paper_2603_25282_amd.sgp import SgpError
    s2 = Solver((32, 32), 8.0, PARAMS, dtype="complex64")
    with pytest.raises(SgpError):
        s2.set_slabs(2)
    s3 = Solver((32, 32, 32), 8.0, PARAMS, dtype="complex64")
    for bad in (3, 64, -2):
        with pytest.raises(SgpError):
            s3.set_slabs(bad)
    s3.set_slabs(8)
    s3.set_slabs(0)


def test_adjoint_repeats_bitwise():
    import torch
    from paper_2603_25282_amd.autograd import evolve
    shape = (64, 128)
    psi0 = _state(shape, 8.0, 42)
    w = torch.randn(shape + (5,), dtype=torch.complex64, generator=torch.Generator().manual_seed(3)).cuda()
    outs = []
    for _ in range(2):
        p0 = torch.from_numpy(Solver.to_device_layout(psi0)).to(torch.complex64).cuda().requires_grad_(True)
        par = torch.tensor([PARAMS[i] for i in (4, 3, 0, 1, 2)], dtype=torch.float64, requires_grad=True)
        out = evolve(p0, par, shape, 8.0, PARAMS[5:8], 1e-3, 12, order=4, K=5)
        torch.sum((torch.conj(w) * out).real).backward()
        outs.append((p0.grad.clone(), par.grad.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_ensemble_repeats_bitwise():
    import torch
    insts = I.ensemble_instances(n128=3, n256=2, n384=1)
    res = []
    for _ in range(2):
        ens = Ensemble([c.shape for c in insts], [c.L for c in insts], [c.params for c in insts], dtype="complex64")
        ens.build_propagator(insts[0].tau, insts[0].order)
        psis = [torch.from_numpy(Solver.to_device_layout(I.initial_state(c))).to(torch.complex64).cuda().contiguous()
                for c in insts]
        ens.step(psis, 20)  # 20 steps: graph replay for 16 of them
        torch.cuda.synchronize()
        res.append(psis)
    assert all(torch.equal(x, y) for x, y in zip(res[0], res[1]))


@pytest.mark.parametrize("shape,dtype", [((128, 64), "complex64"), ((32, 32, 32), "complex128")])
def test_poisoned_workspace_changes_nothing(shape, dtype):
    # A workspace filled with NaN bytes before the library takes it: every value the
    # kernels read from it (tables, twiddles, clock, partial sums) must have been
    # written first, so the results are bitwise those of a workspace as allocated.
    import torch
    print(f"case poison {shape} {dtype}", flush=True)
    psi0 = _state(shape, 8.0, 43)
    out = []
    for poison in (False, True):
        s = Solver(shape, 8.0, PARAMS, dtype=dtype, poison=poison)
        s.build_propagator(1e-3, 4)
        psi = to_gpu(s, psi0)
        s.step(psi, 40)
        out.append((psi, s.observables(psi), np.array(list(s.diagnostics(psi).values()))))
    torch.cuda.synchronize()
    assert torch.equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])


def test_poisoned_ensemble_workspace_changes_nothing():
    import torch
    insts = I.ensemble_instances(n128=2, n256=1, n384=1)
    res = []
    for poison in (False, True):
        ens = Ensemble([c.shape for c in insts], [c.L for c in insts], [c.params for c in insts], dtype="complex64",
                       poison=poison)
        ens.build_propagator(insts[0].tau, insts[0].order)
        psis = [torch.from_numpy(Solver.to_device_layout(I.initial_state(c))).to(torch.complex64).cuda().contiguous()
                for c in insts]
        ens.step(psis, 20)
        torch.cuda.synchronize()
        res.append(psis)
    assert all(torch.equal(x, y) for x, y in zip(res[0], res[1]))
