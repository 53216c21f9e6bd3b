"""Helpers shared by the GPU parity tests."""
import numpy as np


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run_gpu(cfg_or_shape, L, params, psi0, order, tau, nsteps, dtype="complex128", t0=0.0, chunks=None):
    """Evolve psi0 (numpy complex128) on the GPU through the C ABI; returns numpy."""
    import torch
    from paper_2603_25282_amd.sgp import Solver
    shape = psi0.shape[1:]
    s = Solver(shape, L, params, dtype=dtype)
    s.build_propagator(tau, order)
    s.time = t0
    psi = torch.from_numpy(Solver.to_device_layout(psi0)).to(s.torch_dtype).to(s.device).contiguous()
    for n in (chunks if chunks is not None else [nsteps]):
        s.step(psi, n)
    torch.cuda.synchronize()
    out = Solver.from_device_layout(psi.cpu().numpy().astype(np.complex128))
    return out, s


def to_gpu(s, psi0):
    """numpy (5, ...) complex128 -> device tensor in the library layout."""
    import torch
    from paper_2603_25282_amd.sgp import Solver
    return torch.from_numpy(Solver.to_device_layout(psi0)).to(s.torch_dtype).to(s.device).contiguous()
