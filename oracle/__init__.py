"""FP64 CPU oracle for the compact splitting Fourier spectral method (rotating
spin-orbit-coupled spin-2 GPE, arXiv 2603.25282).

TEST INFRASTRUCTURE ONLY: plain, slow and written to be read against the paper.
Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use it.
It shares no code with the HIP library in paper_2603_25282_amd/.

State arrays are complex128 of shape (5, [nz,] ny, nx), component i <-> spin
projection l = 2, 1, 0, -1, -2.  Parameters are (c0, c1, c2, Omega, gamma, gx, gy, gz).
"""
import ctypes
import os

import numpy as np

from .build import LIB, build_oracle

_lib = None


def lib():
    global _lib
    if _lib is None:
        build_oracle(force=False)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_fft.argtypes = [ctypes.c_int, ip, dp, ctypes.c_int]
        L.orc_propagator.argtypes = [ctypes.c_double] * 5 + [dp]
        L.orc_nl_point.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_linear_step.argtypes = [ctypes.c_int, ip, dp, dp, ctypes.c_double, dp]
        L.orc_nl_step.argtypes = [ctypes.c_int, ip, dp, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_rotation_map.argtypes = [ctypes.c_int, ip, dp, dp, ctypes.c_double, ctypes.c_int, dp]
        L.orc_evolve.argtypes = [ctypes.c_int, ip, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_long,
                                 ctypes.c_double, ctypes.c_int, dp]
        L.orc_observables.argtypes = [ctypes.c_int, ip, dp, dp, ctypes.c_double, dp, dp]
        L.orc_adjoint.argtypes = [ctypes.c_int, ip, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_long,
                                  ctypes.c_double, dp, dp, dp, dp, ctypes.c_long]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        if "OMP_NUM_THREADS" not in os.environ:
            # One core is left to the caller: a full-width OpenMP team on a fully
            # subscribed host spends most of its time in barrier waits.
            L.orc_set_threads(max(1, (os.cpu_count() or 2) - 1))
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _grid(shape, L):
    """shape is the spatial shape (ny, nx) or (nz, ny, nx); returns (dim, n[x,y,z], L[x,y,z])."""
    dim = len(shape)
    n = np.array(list(shape[::-1]) + [1] * (3 - dim), dtype=np.int32)
    Ls = np.broadcast_to(np.asarray(L, dtype=np.float64), (dim,))
    Larr = np.array(list(Ls) + [1.0] * (3 - dim), dtype=np.float64)
    return dim, n, Larr


def _params(p):
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
    assert p.shape == (8,)
    return p


def num_threads():
    return lib().orc_num_threads()


def set_threads(n):
    lib().orc_set_threads(int(n))


def fft(x, sign=-1):
    """d-dim transform (own FFT); sign -1 forward with 1/N^d, +1 inverse unscaled."""
    a = np.ascontiguousarray(np.array(x, dtype=np.complex128))
    dim, n, _ = _grid(a.shape, 1.0)
    lib().orc_fft(dim, _i(n), _d(a.view(np.float64)), int(sign))
    return a


def propagator(Omega, gamma, nu_p, nu_q, delta):
    """exp(i delta Q) for one wavevector from the paper's closed form (5x5 complex)."""
    out = np.zeros((5, 5), dtype=np.complex128)
    lib().orc_propagator(Omega, gamma, nu_p, nu_q, delta, _d(out.view(np.float64)))
    return out


def nl_point(params, V, delta, psi5):
    """Exact nonlinear flow at one point for time delta (eq. solution2)."""
    a = np.ascontiguousarray(np.array(psi5, dtype=np.complex128))
    lib().orc_nl_point(_d(_params(params)), float(V), float(delta), _d(a.view(np.float64)))
    return a


def linear_step(psi, L, params, delta):
    a = np.ascontiguousarray(np.array(psi, dtype=np.complex128))
    dim, n, Ls = _grid(a.shape[1:], L)
    lib().orc_linear_step(dim, _i(n), _d(Ls), _d(_params(params)), float(delta), _d(a.view(np.float64)))
    return a


def nl_step(psi, L, params, delta, theta=0.0):
    a = np.ascontiguousarray(np.array(psi, dtype=np.complex128))
    dim, n, Ls = _grid(a.shape[1:], L)
    lib().orc_nl_step(dim, _i(n), _d(Ls), _d(_params(params)), float(delta), float(theta),
                      _d(a.view(np.float64)))
    return a


def rotation_map(psi, L, params, t, forward=True):
    """RSDA mapping: forward Phi = M_t Psi; backward Psi = M_t^{-1} Phi."""
    a = np.ascontiguousarray(np.array(psi, dtype=np.complex128))
    dim, n, Ls = _grid(a.shape[1:], L)
    lib().orc_rotation_map(dim, _i(n), _d(Ls), _d(_params(params)), float(t), int(bool(forward)),
                           _d(a.view(np.float64)))
    return a


def evolve(psi, L, params, order, tau, nsteps, t0=0.0, frame="rotating"):
    """nsteps of TS2 (order=2) or TS4 (order=4) from clock t0.  frame='rotating'
    evolves Phi with the trap rotated by Omega*s; frame='lab' is the literal
    Algorithm 1 with the RSDA mapping around every linear substep."""
    a = np.ascontiguousarray(np.array(psi, dtype=np.complex128))
    dim, n, Ls = _grid(a.shape[1:], L)
    mode = {"rotating": 0, "lab": 1}[frame]
    lib().orc_evolve(dim, _i(n), _d(Ls), _d(_params(params)), int(order), float(tau), int(nsteps),
                     float(t0), mode, _d(a.view(np.float64)))
    return a


def observables(psi, L, params, theta=0.0):
    """(mass, energy, magnetization, <Lz>) with the trap rotated by theta."""
    a = np.ascontiguousarray(np.array(psi, dtype=np.complex128))
    dim, n, Ls = _grid(a.shape[1:], L)
    out = np.zeros(4)
    lib().orc_observables(dim, _i(n), _d(Ls), _d(_params(params)), float(theta), _d(a.view(np.float64)),
                          _d(out))
    return out


def adjoint(psi0, gT, L, params, order, tau, nsteps, t0=0.0, K=50):
    """Discrete adjoint of evolve(): given gT = 2 dJ/d conj(Phi(T)) returns
    (g0 = 2 dJ/d conj(Psi0), dJ/d(gamma, Omega, c0, c1, c2)) for the rotating-frame
    evolution, with checkpoints every K steps."""
    a = np.ascontiguousarray(np.array(psi0, dtype=np.complex128))
    gt = np.ascontiguousarray(np.array(gT, dtype=np.complex128))
    dim, n, Ls = _grid(a.shape[1:], L)
    g0 = np.zeros_like(a)
    dpar = np.zeros(5)
    lib().orc_adjoint(dim, _i(n), _d(Ls), _d(_params(params)), int(order), float(tau), int(nsteps), float(t0),
                      _d(a.view(np.float64)), _d(gt.view(np.float64)), _d(g0.view(np.float64)), _d(dpar), int(K))
    return g0, dpar
