"""Failure handling through the C ABI: a NaN or an infinity in the state is
reported as SGP_ERR_NONFINITE by the observables (the kernels' memory accesses do
not depend on the data, so such a state is read like any other), and a run cut
after k steps resumes from its checkpoint (the state and the time) in a fresh
context bitwise as if it had not been cut."""
import os

import numpy as np
import pytest

from paper_2603_25282_amd import inputs as I
from paper_2603_25282_amd.sgp import SgpError, Solver
from tests.gpu_util import to_gpu

pytestmark = pytest.mark.gpu

PARAMS = (100.0, -1.0, 5.0, 0.6, 0.7, 1.0, 1.1, 1.0)


def _state(shape, L, seed):
    rng = np.random.default_rng(seed)
    co = I.mesh(shape, L)
    g = np.exp(-sum(c * c for c in co) / 2.0)
    return I.normalise(g[None] * np.exp(1j * rng.uniform(0, 2 * np.pi, (5,) + shape)), shape, L)


@pytest.mark.parametrize("dtype", ["complex64", "complex128"])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_nonfinite_state_is_reported(dtype, bad):
    shape, L = (64, 64), 8.0
    print(f"case nonfinite {dtype} {bad}", flush=True)
    s = Solver(shape, L, PARAMS, dtype=dtype)
    s.build_propagator(1e-3, 4)
    psi = to_gpu(s, _state(shape, L, 21))
    m = s.observables(psi)
    assert np.all(np.isfinite(m))
    psi[17, 40, 3] = complex(bad, 0.0)  # one value of one component at one point
    with pytest.raises(SgpError, match="error -4"):
        s.observables(psi)
    with pytest.raises(SgpError, match="error -4"):
        s.diagnostics(psi)


@pytest.mark.parametrize("shape,dtype", [((128, 64), "complex64"), ((32, 32, 32), "complex128")])
def test_resume_from_checkpoint_is_bitwise(shape, dtype):
    import torch
    L, n1, n2 = 8.0, 17, 23
    print(f"case resume {shape} {dtype}", flush=True)
    psi0 = _state(shape, L, 22)
    # the uninterrupted run: the same two calls in one context (a call ends with its
    # last nonlinear substep unmerged, so the cut sits at the same place)
    ref = Solver(shape, L, PARAMS, dtype=dtype)
    ref.build_propagator(1e-3, 4)
    a = to_gpu(ref, psi0)
    ref.step(a, n1)
    ref.step(a, n2)
    s1 = Solver(shape, L, PARAMS, dtype=dtype)
    s1.build_propagator(1e-3, 4)
    b = to_gpu(s1, psi0)
    s1.step(b, n1)
    checkpoint, t = b.clone(), s1.time
    del s1, b
    s2 = Solver(shape, L, PARAMS, dtype=dtype)  # a fresh context
    s2.build_propagator(1e-3, 4)
    s2.time = t
    c = checkpoint.clone()
    s2.step(c, n2)
    torch.cuda.synchronize()
    assert s2.time == ref.time
    assert torch.equal(a, c)


def test_checkpoint_file_roundtrip(tmp_path):
    # kill after k steps, write the checkpoint file, resume from it in a fresh
    # context: bitwise the run that went on in place (plans and clock restored)
    import torch
    from paper_2603_25282_amd import checkpoint
    shape, L, n1, n2 = (64, 128), 8.0, 17, 23
    print(f"case checkpoint file {shape}", flush=True)
    s = Solver(shape, L, PARAMS, dtype="complex64")
    s.set_plan([4, 4])  # not the default plans, so that they must come back from the file
    s.build_propagator(1e-3, 4)
    psi = to_gpu(s, _state(shape, L, 23))
    s.step(psi, n1)
    path = str(tmp_path / "run.npz")
    checkpoint.save(path, s, psi)
    s.step(psi, n2)  # the run that is not cut
    torch.cuda.synchronize()
    s2, psi2 = checkpoint.load(path)
    assert s2.get_plan() == [4, 4] and s2.shape == shape and s2.params == s.params
    s2.step(psi2, n2)
    torch.cuda.synchronize()
    assert s2.time == s.time
    assert torch.equal(psi, psi2)
    with np.load(path, allow_pickle=False) as f:  # plain arrays only
        assert set(f.files) >= {"state", "time", "shape", "L", "params", "tau", "scheme", "plan", "dtype",
                                "frame"}


def test_checkpoint_3d_plan_with_split(tmp_path):
    # a 3D run whose plan includes the linear substep's split (the non-default one):
    # the file carries all four plan entries and the resumed run is bitwise the same
    import torch
    from paper_2603_25282_amd import checkpoint
    shape, L, n1, n2 = (16, 32, 32), 6.0, 5, 4
    print(f"case checkpoint 3D split plan {shape}", flush=True)
    s = Solver(shape, L, PARAMS, dtype="complex64")
    s.set_plan([4, 8, 4, 1])
    s.build_propagator(1e-3, 4)
    psi = to_gpu(s, _state(shape, L, 29))
    s.step(psi, n1)
    path = str(tmp_path / "run3d.npz")
    checkpoint.save(path, s, psi)
    s.step(psi, n2)
    torch.cuda.synchronize()
    s2, psi2 = checkpoint.load(path)
    assert s2.get_plan() == [4, 8, 4, 1]
    s2.step(psi2, n2)
    torch.cuda.synchronize()
    assert torch.equal(psi, psi2)


def test_checkpoint_lab_frame_side_stream(tmp_path):
    # a lab-frame run (Algorithm 1 literally) on a side stream: the file written right
    # after the steps were queued holds the finished state and the frame, so the
    # resumed run continues in the lab frame bitwise; the path has no .npz suffix
    import torch
    from paper_2603_25282_amd import checkpoint
    shape, L, n1, n2 = (64, 64), 8.0, 9, 7
    print(f"case checkpoint lab frame side stream {shape}", flush=True)
    side = torch.cuda.Stream()
    s = Solver(shape, L, PARAMS, dtype="complex128", stream=side)
    s.set_frame("lab")
    s.build_propagator(1e-3, 2)
    psi = to_gpu(s, _state(shape, L, 25))
    torch.cuda.synchronize()
    s.step(psi, n1)  # queued on the side stream; save() must wait for it
    path = str(tmp_path / "lab_run")
    checkpoint.save(path, s, psi)
    assert os.path.exists(path) and not os.path.exists(path + ".npz")
    s.step(psi, n2)
    side.synchronize()
    s2, psi2 = checkpoint.load(path)
    assert s2.frame == "lab"
    s2.step(psi2, n2)
    torch.cuda.synchronize()
    assert s2.time == s.time
    assert torch.equal(psi, psi2)
    # the same data resumed in the rotating frame would differ
    s3, psi3 = checkpoint.load(path)
    s3.set_frame("rotating")
    s3.step(psi3, n2)
    torch.cuda.synchronize()
    assert not torch.equal(psi, psi3)


def test_watchdog_runs_and_stops(tmp_path):
    import torch
    from paper_2603_25282_amd import checkpoint
    shape, L = (64, 64), 8.0
    print("case watchdog", flush=True)
    s = Solver(shape, L, PARAMS, dtype="complex128")
    s.build_propagator(1e-3, 4)
    psi = to_gpu(s, _state(shape, L, 24))
    path = str(tmp_path / "w.npz")
    checkpoint.run_checked(s, psi, 25, every=10, path=path, mass_tol=1e-10)
    assert abs(s.time - 0.025) < 1e-15
    s2, psi2 = checkpoint.load(path)  # the last checkpoint is the final state
    assert torch.equal(psi, psi2) and s2.time == s.time
    # a mass tolerance below the rounding of the steps stops the run after the first call
    with pytest.raises(checkpoint.WatchdogError, match="step 10: relative mass change"):
        checkpoint.run_checked(s, psi.clone(), 20, every=10, mass_tol=1e-30)
    psi[5, 7, 1] = complex(float("nan"), 0.0)  # a corrupted state stops the run at once
    with pytest.raises(checkpoint.WatchdogError, match="step 0: sgp error -4"):
        checkpoint.run_checked(s, psi, 20, every=10)
