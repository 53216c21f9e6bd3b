"""Checkpoint files of a run: the state together with everything that determines
its continuation -- the clock t of the rotating frame (the trap angle Omega t and
the first nonlinear substep of the next call depend on it), grid, half-widths,
physics parameters, element type, time step, composition, register plans and the
frame option (rotating-frame Phi, or the lab-frame state of Algorithm 1).

A call of sgp_step ends with its last nonlinear substep unmerged, so a run
resumed from a checkpoint written between two calls continues bitwise as the
same calls in one context would.  Files are numpy .npz archives of plain arrays
(no pickled objects); load() reads them with allow_pickle=False."""
import os

import numpy as np

from .sgp import Solver

# 2: the frame option (rotating-frame Phi or the literal lab-frame Algorithm 1) is stored
FORMAT = 2


def save(path, solver, psi):
    """Write psi (the solver's state tensor, library layout) and the solver's
    configuration to `path` exactly (no suffix is added).  The propagator must have
    been built.  The state is copied only after the solver's stream has finished
    every queued step, and the file is written to a temporary name and then renamed,
    so that a process killed while writing leaves the previous checkpoint whole."""
    import torch
    if solver.tau is None:
        raise ValueError("build the propagator before saving a checkpoint")
    with torch.cuda.device(solver.device):
        if solver.stream is not None:
            solver.stream.synchronize()
        torch.cuda.current_stream().synchronize()
    state = psi.detach().cpu().numpy()
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "wb") as f:
        np.savez(f, format=np.int64(FORMAT), state=state, time=np.float64(solver.time),
                 shape=np.asarray(solver.shape, dtype=np.int64), L=np.asarray(solver.L, dtype=np.float64),
                 params=np.asarray(solver.params, dtype=np.float64), tau=np.float64(solver.tau),
                 scheme=np.int64(solver.scheme), plan=np.asarray(solver.get_plan(), dtype=np.int64),
                 frame=np.bytes_(solver.frame),
                 dtype=np.bytes_(str(solver.torch_dtype).replace("torch.", "")))
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, path)


def load(path, device="cuda:0", stream=None):
    """Read a checkpoint; returns (solver, psi) with the propagator built, the plans,
    the frame and the clock restored, and psi on `device` in the library layout."""
    import torch
    with open(path, "rb") as fh, np.load(fh, allow_pickle=False) as f:
        if int(f["format"]) != FORMAT:
            raise ValueError(f"unknown checkpoint format {int(f['format'])}")
        dtype = f["dtype"].item().decode()
        s = Solver(tuple(int(x) for x in f["shape"]), tuple(float(x) for x in f["L"]),
                   tuple(float(x) for x in f["params"]), dtype=dtype, device=device, stream=stream)
        s.set_plan([int(x) for x in f["plan"]])
        s.set_frame(f["frame"].item().decode())
        s.build_propagator(float(f["tau"]), int(f["scheme"]))
        s.time = float(f["time"])
        psi = torch.from_numpy(np.array(f["state"])).to(s.device).contiguous()
    if psi.dtype != s.torch_dtype or tuple(psi.shape) != s.shape + (5,):
        raise ValueError("checkpoint state does not match its configuration")
    return s, psi


class WatchdogError(RuntimeError):
    pass


def run_checked(solver, psi, nsteps, every, path=None, mass_tol=None):
    """Advance psi by nsteps in calls of `every` steps; after each call check the
    state (sgp_observables reports a NaN or an infinity anywhere in it as
    SGP_ERR_NONFINITE) and, with mass_tol, the relative change of the mass since
    the start; with path, write a checkpoint file after each call.  Raises
    WatchdogError naming the step where a check failed (the last checkpoint
    written, if any, is the state `every` steps earlier).  Each call ends with
    its last nonlinear substep unmerged, so the result depends on `every` at the
    level of rounding."""
    from .sgp import SgpError
    if every < 1:
        raise ValueError("every must be >= 1")
    try:
        m0 = float(solver.observables(psi)[0])
    except SgpError as e:
        raise WatchdogError(f"step 0: {e}") from e
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        solver.step(psi, k)
        done += k
        try:
            m = float(solver.observables(psi)[0])
        except SgpError as e:
            raise WatchdogError(f"step {done}: {e}") from e
        if mass_tol is not None and abs(m / m0 - 1.0) > mass_tol:
            raise WatchdogError(f"step {done}: relative mass change {m / m0 - 1.0:.3e} exceeds {mass_tol:.3e}")
        if path is not None:
            save(path, solver, psi)
    return psi
