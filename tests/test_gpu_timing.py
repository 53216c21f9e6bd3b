"""The measurement entry point sgp_time_pass through the C ABI: the SGP_TIME_STEPS
mode runs whole steps of the step schedule (launched without the graph) and times
every launch of one pass with start/end events stamped by its dispatch.  Those
steps must be the steps sgp_step takes (bitwise, graph replay or not), the context
time must come back unchanged, and the arguments are checked."""
import numpy as np
import pytest

from paper_2603_25282_amd import inputs as I
from paper_2603_25282_amd.sgp import SgpError, Solver
from tests.gpu_util import to_gpu

pytestmark = pytest.mark.gpu


def _state(shape, L, seed):
    rng = np.random.default_rng(seed)
    co = I.mesh(shape, L)
    g = np.exp(-sum(c * c for c in co) / 2.0)
    psi = g[None] * np.exp(1j * rng.uniform(0, 2 * np.pi, (5,) + shape))
    return I.normalise(psi, shape, L)


@pytest.mark.parametrize("shape,passes,nsteps", [((64, 128), (0, 1), 40), ((32, 32, 32), (0, 1, 2, 3), 6)])
def test_steps_timing_runs_the_step_schedule(shape, passes, nsteps):
    import torch
    L = 8.0
    params = (100.0, -1.0, 5.0, 0.6, 0.7, 1.0, 1.1, 2.0)
    s = Solver(shape, L, params, dtype="complex64")
    s.build_propagator(1e-3, 4)
    psi0 = _state(shape, L, 11)
    for k in passes:
        print(f"case {shape} pass {k} steps {nsteps}", flush=True)
        s.time = 0.25
        a = to_gpu(s, psi0)
        ms = s.time_pass(a, k, nsteps, in_steps=True)
        assert ms > 0.0 and np.isfinite(ms)
        assert s.time == 0.25  # restored
        b = to_gpu(s, psi0)
        s.step(b, nsteps)  # 40 steps replay the captured graph for 32 of them
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_steps_timing_rejects_bad_arguments():
    s = Solver((64, 64), 8.0, (100.0, -1.0, 5.0, 0.6, 0.7, 1.0, 1.0, 1.0), dtype="complex64")
    s.build_propagator(1e-3, 2)
    a = to_gpu(s, _state((64, 64), 8.0, 12))
    with pytest.raises(SgpError):
        s.time_pass(a, 0, 1, in_steps=True)  # fewer than 2 steps
    with pytest.raises(SgpError):
        s.time_pass(a, 0, 4, in_step=True, in_steps=True)  # both modes
    with pytest.raises(SgpError):
        s.time_pass(a, 2, 4, in_steps=True)  # no z-pass in 2D
