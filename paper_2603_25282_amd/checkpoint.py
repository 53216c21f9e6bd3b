"""Checkpoint files of a run: the state together with everything that determines
its continuation -- the clock t of the rotating frame (the trap angle Omega t and
the first nonlinear substep of the next call depend on it), grid, half-widths,
physics parameters, element type, time step, composition and register plans.

A call of sgp_step ends with its last nonlinear substep unmerged, so a run
resumed from a checkpoint written between two calls continues bitwise as the
same calls in one context would.  Files are numpy .npz archives of plain arrays
(no pickled objects); load() reads them with allow_pickle=False."""
import numpy as np

from .sgp import Solver

FORMAT = 1


def save(path, solver, psi):
    """Write psi (the solver's state tensor, library layout) and the solver's
    configuration to `path` (.npz).  The propagator must have been built."""
    if solver.tau is None:
        raise ValueError("build the propagator before saving a checkpoint")
    state = psi.detach().cpu().numpy()
    np.savez(path, format=np.int64(FORMAT), state=state, time=np.float64(solver.time),
             shape=np.asarray(solver.shape, dtype=np.int64), L=np.asarray(solver.L, dtype=np.float64),
             params=np.asarray(solver.params, dtype=np.float64), tau=np.float64(solver.tau),
             scheme=np.int64(solver.scheme), plan=np.asarray(solver.get_plan(), dtype=np.int64),
             dtype=np.bytes_(str(solver.torch_dtype).replace("torch.", "")))


def load(path, device="cuda:0", stream=None):
    """Read a checkpoint; returns (solver, psi) with the propagator built, the plans
    and the clock restored, and psi on `device` in the library layout."""
    import torch
    with np.load(path, allow_pickle=False) as f:
        if int(f["format"]) != FORMAT:
            raise ValueError(f"unknown checkpoint format {int(f['format'])}")
        dtype = f["dtype"].item().decode()
        s = Solver(tuple(int(x) for x in f["shape"]), tuple(float(x) for x in f["L"]),
                   tuple(float(x) for x in f["params"]), dtype=dtype, device=device, stream=stream)
        s.set_plan([int(x) for x in f["plan"]])
        s.build_propagator(float(f["tau"]), int(f["scheme"]))
        s.time = float(f["time"])
        psi = torch.from_numpy(np.array(f["state"])).to(s.device).contiguous()
    if psi.dtype != s.torch_dtype or tuple(psi.shape) != s.shape + (5,):
        raise ValueError("checkpoint state does not match its configuration")
    return s, psi
