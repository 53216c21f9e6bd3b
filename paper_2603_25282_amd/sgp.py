"""Thin Python binding of the C ABI in include/sgp.h (argument marshalling only).

Every numerical step runs in the HIP library libsgp.so; this module only loads it,
converts torch tensors to device pointers and turns error codes into exceptions.
PyTorch provides device memory (state and workspace tensors) and the stream.

State tensors: torch.complex64 or torch.complex128, shape (ny, nx, 5) or
(nz, ny, nx, 5) (the 5 components of a grid point adjacent), contiguous, on a
ROCm device; component i <-> l = 2, 1, 0, -1, -2.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgp.so")

SGP_OK = 0
SGP_C64, SGP_C128 = 0, 1
SGP_TS2, SGP_TS4, SGP_TS6 = 2, 4, 6
SGP_PASS_X, SGP_PASS_Y, SGP_PASS_Z, SGP_PASS_YINV = 0, 1, 2, 3
SGP_OPT_GRAPH, SGP_OPT_BATCHED = 1, 2
SGP_TIME_IN_STEP = 256
SGP_TIME_STEPS = 512
SGP_OPT_FRAME = 3
SGP_OPT_SLABS = 4
SGP_FRAME_ROTATING, SGP_FRAME_LAB = 0, 1
SGP_PLAN_LINEAR = 3


class SgpError(RuntimeError):
    pass


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("L", ctypes.c_double * 3)]


class _Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("c0", "c1", "c2", "Omega", "gamma", "gx", "gy", "gz")]


_lib = None


def lib():
    """Load libsgp.so (built in-tree by paper_2603_25282_amd/build.py).  Raises if
    it is missing: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SgpError(f"{LIB_PATH} not built; run python -m paper_2603_25282_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, cp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)
    L.sgp_create.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Params), ctypes.c_int, vp, cp]
    L.sgp_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.sgp_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
    L.sgp_build_propagator.argtypes = [vp, ctypes.c_double, ctypes.c_int]
    L.sgp_step.argtypes = [vp, vp, ctypes.c_long]
    L.sgp_observables.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    L.sgp_get_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.sgp_set_time.argtypes = [vp, ctypes.c_double]
    L.sgp_time_pass.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.sgp_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_long]
    L.sgp_store_size.argtypes = [vp, ctypes.c_long, ctypes.POINTER(ctypes.c_size_t)]
    L.sgp_step_store.argtypes = [vp, vp, ctypes.c_long, vp, ctypes.c_size_t]
    L.sgp_adjoint_segment.argtypes = [vp, vp, ctypes.c_long, vp, ctypes.c_size_t]
    L.sgp_adjoint_gradients.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    ip = ctypes.POINTER(ctypes.c_int)
    L.sgp_plan_widths.argtypes = [ctypes.c_int, ctypes.c_int, ip, ctypes.c_int]
    L.sgp_rotation_map.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int]
    L.sgp_diagnostics.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    L.sgp_jz_inner.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_double)]
    L.sgp_set_plan.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.sgp_get_plan.argtypes = [vp, ctypes.c_int, ip]
    L.sgp_autotune.argtypes = [vp, vp, ctypes.c_int, ip, ctypes.POINTER(ctypes.c_double)]
    L.sgp_destroy.argtypes = [vp]
    L.sgp_destroy.restype = None
    L.sgp_last_error.argtypes = [vp]
    L.sgp_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def exported_symbols():
    """Names of the C-ABI entry points this binding expects (all declared in sgp.h)."""
    return ["sgp_create", "sgp_workspace_size", "sgp_set_workspace", "sgp_build_propagator", "sgp_step",
            "sgp_observables", "sgp_get_time", "sgp_set_time", "sgp_time_pass", "sgp_set_option", "sgp_destroy",
            "sgp_last_error", "sgp_store_size", "sgp_step_store", "sgp_adjoint_segment", "sgp_adjoint_gradients",
            "sgp_plan_widths", "sgp_set_plan", "sgp_get_plan", "sgp_autotune", "sgp_rotation_map",
            "sgp_diagnostics", "sgp_jz_inner", "sgp_observables_device",
            "sgp_ensemble_create", "sgp_ensemble_workspace_size", "sgp_ensemble_set_workspace",
            "sgp_ensemble_build_propagator", "sgp_ensemble_step", "sgp_ensemble_set_option", "sgp_ensemble_destroy",
            "sgp_ensemble_set_plan", "sgp_ensemble_get_plan", "sgp_ensemble_autotune",
            "sgp_ensemble_store_size", "sgp_ensemble_step_store", "sgp_ensemble_adjoint_segment",
            "sgp_ensemble_adjoint_gradients", "sgp_ensemble_get_time", "sgp_ensemble_set_time",
            "sgp_ensemble_last_error"]


def plan_widths(n, dtype="complex64"):
    """Register plan widths E compiled for line length n and element type (the
    default first)."""
    out = (ctypes.c_int * 8)()
    code = SGP_C64 if str(dtype).replace("torch.", "") == "complex64" else SGP_C128
    k = lib().sgp_plan_widths(int(n), code, out, 8)
    if k < 0:
        raise SgpError(f"unsupported line length {n}")
    return list(out[:k])


def plan_cache_path():
    """JSON file of autotuned plans: $SGP_PLAN_CACHE, else ~/.cache/sgp/plans.json."""
    return os.environ.get("SGP_PLAN_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "sgp", "plans.json")


def _check(rc, ctx=None):
    if rc != SGP_OK:
        msg = lib().sgp_last_error(ctx)
        raise SgpError(f"sgp error {rc}: {msg.decode() if msg else ''}")


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """One context: grid, physics, element type, stream and workspace.

    shape: spatial shape (ny, nx) or (nz, ny, nx); L: half-width (scalar or per
    axis in x, y, z order); params: (c0, c1, c2, Omega, gamma, gx, gy, gz).
    """

    @staticmethod
    def to_device_layout(psi_cfirst):
        """(5, ..., nx) component-first array -> (..., nx, 5) layout of the library."""
        import numpy as np
        return np.ascontiguousarray(np.moveaxis(np.asarray(psi_cfirst), 0, -1))

    @staticmethod
    def from_device_layout(psi_clast):
        """(..., nx, 5) -> (5, ..., nx)."""
        import numpy as np
        return np.ascontiguousarray(np.moveaxis(np.asarray(psi_clast), -1, 0))

    def __init__(self, shape, L, params, dtype="complex64", device="cuda:0", stream=None, poison=False):
        """poison: fill the workspace with NaN bytes (0xFF) before the library takes
        it, so that a read of workspace memory the library has not written shows up
        in the results (a checking mode)."""
        import torch
        self.shape = tuple(int(s) for s in shape)
        dim = len(self.shape)
        Ls = np.broadcast_to(np.asarray(L, dtype=np.float64), (dim,))
        g = _Grid()
        g.dim = dim
        for i in range(3):
            g.n[i] = self.shape[::-1][i] if i < dim else 1
            g.L[i] = float(Ls[i]) if i < dim else 0.0
        p = _Params(*[float(x) for x in params])
        self.L = tuple(float(x) for x in Ls)
        self.params = tuple(float(x) for x in params)
        self.tau, self.scheme = None, None
        self.frame = "rotating"
        self.torch_dtype = {"complex64": torch.complex64, "complex128": torch.complex128}[str(dtype).replace(
            "torch.", "")]
        code = SGP_C64 if self.torch_dtype == torch.complex64 else SGP_C128
        self.device = torch.device(device)
        self.stream = stream
        with torch.cuda.device(self.device):
            sp = _stream_ptr(stream)
        ctx = ctypes.c_void_p()
        _check(lib().sgp_create(ctypes.byref(g), ctypes.byref(p), code, sp, ctypes.byref(ctx)), None)
        self._ctx = ctx
        nb = ctypes.c_size_t()
        _check(lib().sgp_workspace_size(ctx, ctypes.byref(nb)), ctx)
        # uint8 buffer; torch's caching allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        if poison:
            with torch.cuda.device(self.device):
                self.workspace.fill_(0xFF)
                torch.cuda.current_stream().synchronize()
        _check(lib().sgp_set_workspace(ctx, ctypes.c_void_p(self.workspace.data_ptr()), nb.value), ctx)

    def _psi_ptr(self, psi):
        if psi.dtype != self.torch_dtype or tuple(psi.shape) != self.shape + (5,):
            raise SgpError(f"state must be {self.torch_dtype} of shape {self.shape + (5,)}, got {psi.dtype} "
                           f"{tuple(psi.shape)}")
        if not psi.is_contiguous() or psi.device != self.device:
            raise SgpError("state must be contiguous on the solver's device")
        return ctypes.c_void_p(psi.data_ptr())

    def build_propagator(self, tau, scheme):
        _check(lib().sgp_build_propagator(self._ctx, float(tau), int(scheme)), self._ctx)
        self.tau, self.scheme = float(tau), int(scheme)

    def step(self, psi, nsteps):
        _check(lib().sgp_step(self._ctx, self._psi_ptr(psi), int(nsteps)), self._ctx)

    def observables(self, psi):
        out = (ctypes.c_double * 4)()
        _check(lib().sgp_observables(self._ctx, self._psi_ptr(psi), out), self._ctx)
        return np.array(out[:])

    def observables_device(self, psi, out):
        """sgp_observables_device: mass, energy, magnetization and <Lz> written to
        out[0:4] (a float64 device tensor), asynchronously on the solver's stream, with
        no allocation and no host synchronisation."""
        import torch
        L = lib()
        L.sgp_observables_device.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        if out.dtype != torch.float64 or out.numel() < 4 or not out.is_contiguous() or out.device != self.device:
            raise SgpError("out must be a contiguous float64 tensor of at least 4 values on the solver's device")
        _check(L.sgp_observables_device(self._ctx, self._psi_ptr(psi), ctypes.c_void_p(out.data_ptr())),
               self._ctx)

    def jz_inner(self, u, v):
        """<u, J_z v>_h (sgp_jz_inner) as a Python complex."""
        out = (ctypes.c_double * 2)()
        _check(lib().sgp_jz_inner(self._ctx, self._psi_ptr(u), self._psi_ptr(v), out), self._ctx)
        return complex(out[0], out[1])

    def diagnostics(self, psi):
        """sgp_diagnostics as a dict: mass, energy, magnetization, lz, delta_x,
        delta_y, delta_z, xy_rho, width_rate (= d delta_r/dt when gamma = 0),
        dM_dt and dLz_dt (the magnetization and angular-momentum laws, spin-orbit
        terms included) and soc_width_term (G of Lemma 2's width law)."""
        out = (ctypes.c_double * 12)()
        _check(lib().sgp_diagnostics(self._ctx, self._psi_ptr(psi), out), self._ctx)
        keys = ("mass", "energy", "magnetization", "lz", "delta_x", "delta_y", "delta_z", "xy_rho", "width_rate",
                "dM_dt", "dLz_dt", "soc_width_term")
        return dict(zip(keys, out[:]))

    def time_pass(self, psi, pass_kind, reps, in_step=False, in_steps=False):
        """Average milliseconds of one pass (0 X, 1 Y, 2 Z, 3 inverse Y), timed with
        HIP events on the library's stream: reps launches back to back; (in_step)
        reps rounds of one substep's passes in step order; or (in_steps) every launch
        of the pass inside reps whole steps of the step schedule, each launch timed
        by start/end events its dispatch stamps (psi advances reps steps)."""
        pass_kind = int(pass_kind) | (SGP_TIME_IN_STEP if in_step else 0) | (SGP_TIME_STEPS if in_steps else 0)
        ms = ctypes.c_double()
        _check(lib().sgp_time_pass(self._ctx, self._psi_ptr(psi), int(pass_kind), int(reps), ctypes.byref(ms)),
               self._ctx)
        return ms.value

    def store_size(self, nsteps):
        nb = ctypes.c_size_t()
        _check(lib().sgp_store_size(self._ctx, int(nsteps), ctypes.byref(nb)), self._ctx)
        return int(nb.value)

    def step_store(self, psi, nsteps, store):
        """sgp_step_store: forward nsteps, keeping every pass's pointwise-stage input in
        `store` (a uint8 device tensor of at least store_size(nsteps) bytes)."""
        _check(lib().sgp_step_store(self._ctx, self._psi_ptr(psi), int(nsteps), ctypes.c_void_p(store.data_ptr()),
                                    store.numel() * store.element_size()), self._ctx)

    def adjoint_segment(self, lam, nsteps, store):
        """sgp_adjoint_segment: reverse sweep of the step_store call that started at the
        current clock; lam is overwritten with the gradient at the segment start."""
        _check(lib().sgp_adjoint_segment(self._ctx, self._psi_ptr(lam), int(nsteps),
                                         ctypes.c_void_p(store.data_ptr()), store.numel() * store.element_size()),
               self._ctx)

    def adjoint_gradients(self, reset=True):
        """dJ/d(gamma, Omega, c0, c1, c2) accumulated by adjoint_segment calls."""
        out = (ctypes.c_double * 5)()
        _check(lib().sgp_adjoint_gradients(self._ctx, out, int(bool(reset))), self._ctx)
        return np.array(out[:])

    def get_plan(self):
        """Plan width E of the passes along x, y (, z); in 3D a fourth entry, the
        linear substep's split (SGP_PLAN_LINEAR: 0 = the whole propagator in the
        z-pass, 1 = its spin part in the forward y-pass)."""
        e = ctypes.c_int()
        out = []
        for ax in range(len(self.shape)) if len(self.shape) == 2 else (0, 1, 2, SGP_PLAN_LINEAR):
            _check(lib().sgp_get_plan(self._ctx, ax, ctypes.byref(e)), self._ctx)
            out.append(e.value)
        return out

    def set_plan(self, widths):
        """Plan widths per axis (x, y (, z)); 0 = default; in 3D an optional fourth
        entry sets the linear substep's split (see get_plan)."""
        if len(widths) > len(self.shape) + (1 if len(self.shape) == 3 else 0):
            raise SgpError(f"plan {list(widths)} has too many entries for a {len(self.shape)}D grid")
        for ax, e in enumerate(widths):
            _check(lib().sgp_set_plan(self._ctx, ax, int(e)), self._ctx)

    def plan_key(self, scheme):
        import torch
        prop = torch.cuda.get_device_properties(self.device)
        arch = getattr(prop, "gcnArchName", "") or prop.name
        return f"{arch}|{'x'.join(map(str, self.shape))}|{str(self.torch_dtype).replace('torch.', '')}|TS{scheme}"

    def autotune(self, psi, scheme, steps=20, cache=True):
        """Pick the plan width of every axis (sgp_autotune on a scratch copy of psi)
        and keep the choice in the JSON plan cache (plan_cache_path()); with cache,
        a stored choice for this device, shape, dtype and scheme is applied without
        timing.  Returns (widths, ms_per_step or None)."""
        import json
        key = self.plan_key(scheme)
        path = plan_cache_path()
        table = {}
        if cache and os.path.exists(path):
            try:
                with open(path) as f:
                    table = json.load(f)
            except (OSError, ValueError):
                table = {}
            if key in table:
                self.set_plan(table[key]["widths"])
                return self.get_plan(), None
        scratch = psi.clone()
        out = (ctypes.c_int * 3)()
        ms = ctypes.c_double()
        _check(lib().sgp_autotune(self._ctx, self._psi_ptr(scratch), int(steps), out, ctypes.byref(ms)), self._ctx)
        del scratch
        widths = self.get_plan()
        if cache:
            table[key] = {"widths": widths, "ms_per_step": ms.value}
            try:
                os.makedirs(os.path.dirname(path), exist_ok=True)
                tmp = path + f".{os.getpid()}.tmp"
                with open(tmp, "w") as f:
                    json.dump(table, f, indent=1, sort_keys=True)
                os.replace(tmp, path)
            except OSError:
                pass
        return widths, ms.value

    def rotation_map(self, psi, t, direction):
        """In place: direction +1 lab -> rotating frame (Phi = M_t Psi), -1 back."""
        _check(lib().sgp_rotation_map(self._ctx, self._psi_ptr(psi), float(t), int(direction)), self._ctx)

    def set_frame(self, frame):
        """'rotating' (default) or 'lab' (Algorithm 1 literally on the lab-frame state)."""
        v = {"rotating": SGP_FRAME_ROTATING, "lab": SGP_FRAME_LAB}[frame]
        _check(lib().sgp_set_option(self._ctx, SGP_OPT_FRAME, v), self._ctx)
        self.frame = frame

    def set_graph(self, on):
        _check(lib().sgp_set_option(self._ctx, 1, int(bool(on))), self._ctx)

    def set_slabs(self, n):
        """3D: run the z-local passes of the replayed step body in n z-slabs on two
        streams (0 or 1: off; n must divide nz)."""
        _check(lib().sgp_set_option(self._ctx, SGP_OPT_SLABS, int(n)), self._ctx)

    @property
    def time(self):
        t = ctypes.c_double()
        _check(lib().sgp_get_time(self._ctx, ctypes.byref(t)), self._ctx)
        return t.value

    @time.setter
    def time(self, t):
        _check(lib().sgp_set_time(self._ctx, float(t)), self._ctx)

    def close(self):
        if getattr(self, "_ctx", None):
            lib().sgp_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """Many 2D grids advanced together (C ABI sgp_ensemble_*): each pass type of a
    step is one batched launch over every instance's tiles.

    shapes: list of (N, N); Ls: list of half-widths; params_list: list of
    (c0, c1, c2, Omega, gamma, gx, gy, gz)."""

    def __init__(self, shapes, Ls, params_list, dtype="complex64", device="cuda:0", stream=None, poison=False):
        import torch
        L = lib()
        vp = ctypes.c_void_p
        L.sgp_ensemble_create.argtypes = [ctypes.c_int, ctypes.POINTER(_Grid), ctypes.POINTER(_Params), ctypes.c_int,
                                          vp, ctypes.POINTER(vp)]
        L.sgp_ensemble_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.sgp_ensemble_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
        L.sgp_ensemble_build_propagator.argtypes = [vp, ctypes.c_double, ctypes.c_int]
        L.sgp_ensemble_step.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_long]
        L.sgp_ensemble_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_long]
        L.sgp_ensemble_set_plan.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.sgp_ensemble_get_plan.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.sgp_ensemble_autotune.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.sgp_ensemble_store_size.argtypes = [vp, ctypes.c_long, ctypes.POINTER(ctypes.c_size_t)]
        L.sgp_ensemble_step_store.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_long, vp, ctypes.c_size_t]
        L.sgp_ensemble_adjoint_segment.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_long, vp, ctypes.c_size_t]
        L.sgp_ensemble_adjoint_gradients.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        L.sgp_ensemble_get_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.sgp_ensemble_set_time.argtypes = [vp, ctypes.c_double]
        L.sgp_ensemble_destroy.argtypes = [vp]
        L.sgp_ensemble_destroy.restype = None
        L.sgp_ensemble_last_error.argtypes = [vp]
        L.sgp_ensemble_last_error.restype = ctypes.c_char_p
        n = len(shapes)
        grids = (_Grid * n)()
        pars = (_Params * n)()
        for i, (sh, Li, pr) in enumerate(zip(shapes, Ls, params_list)):
            grids[i].dim = 2
            grids[i].n[0], grids[i].n[1], grids[i].n[2] = sh[1], sh[0], 1
            grids[i].L[0] = grids[i].L[1] = float(Li)
            pars[i] = _Params(*[float(x) for x in pr])
        self.shapes = [tuple(sh) for sh in shapes]
        self.torch_dtype = {"complex64": torch.complex64, "complex128": torch.complex128}[dtype]
        code = SGP_C64 if dtype == "complex64" else SGP_C128
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            sp = _stream_ptr(stream)
        h = vp()
        rc = L.sgp_ensemble_create(n, grids, pars, code, sp, ctypes.byref(h))
        if rc != SGP_OK:
            raise SgpError(f"sgp_ensemble_create {rc}: {L.sgp_ensemble_last_error(None).decode()}")
        self._h = h
        nb = ctypes.c_size_t()
        self._chk(L.sgp_ensemble_workspace_size(h, ctypes.byref(nb)))
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        if poison:  # NaN bytes, as for Solver(poison=True)
            with torch.cuda.device(self.device):
                self.workspace.fill_(0xFF)
                torch.cuda.current_stream().synchronize()
        self._chk(L.sgp_ensemble_set_workspace(h, vp(self.workspace.data_ptr()), nb.value))

    def _chk(self, rc):
        if rc != SGP_OK:
            raise SgpError(f"sgp ensemble error {rc}: {lib().sgp_ensemble_last_error(self._h).decode()}")

    def build_propagator(self, tau, scheme):
        self._chk(lib().sgp_ensemble_build_propagator(self._h, float(tau), int(scheme)))

    def step(self, psis, nsteps):
        self._chk(lib().sgp_ensemble_step(self._h, self._ptrs(psis), int(nsteps)))

    def set_option(self, option, value):
        self._chk(lib().sgp_ensemble_set_option(self._h, int(option), int(value)))

    @property
    def time(self):
        t = ctypes.c_double()
        self._chk(lib().sgp_ensemble_get_time(self._h, ctypes.byref(t)))
        return t.value

    @time.setter
    def time(self, t):
        self._chk(lib().sgp_ensemble_set_time(self._h, float(t)))

    def _ptrs(self, psis):
        """Pointer array for the C ABI, which reads one pointer per instance: refuse a
        list of the wrong length before any library call."""
        psis = list(psis)
        if len(psis) != len(self.shapes):
            raise SgpError(f"ensemble of {len(self.shapes)} instances given {len(psis)} states")
        for p, sh in zip(psis, self.shapes):
            if p.dtype != self.torch_dtype or tuple(p.shape) != sh + (5,) or not p.is_contiguous():
                raise SgpError("ensemble states must be contiguous (N, N, 5) tensors of the ensemble dtype")
            if p.device != self.device:
                raise SgpError("ensemble states must be on the ensemble's device")
        return (ctypes.c_void_p * len(psis))(*[p.data_ptr() for p in psis])

    def store_size(self, nsteps):
        nb = ctypes.c_size_t()
        self._chk(lib().sgp_ensemble_store_size(self._h, int(nsteps), ctypes.byref(nb)))
        return int(nb.value)

    def step_store(self, psis, nsteps, store):
        self._chk(lib().sgp_ensemble_step_store(self._h, self._ptrs(psis), int(nsteps),
                                                ctypes.c_void_p(store.data_ptr()), store.numel()))

    def adjoint_segment(self, lams, nsteps, store):
        self._chk(lib().sgp_ensemble_adjoint_segment(self._h, self._ptrs(lams), int(nsteps),
                                                     ctypes.c_void_p(store.data_ptr()), store.numel()))

    def adjoint_gradients(self, reset=True):
        """(n_inst, 5) array: dJ/d(gamma, Omega, c0, c1, c2) per instance."""
        out = (ctypes.c_double * (5 * len(self.shapes)))()
        self._chk(lib().sgp_ensemble_adjoint_gradients(self._h, out, int(bool(reset))))
        return np.array(out[:]).reshape(len(self.shapes), 5)

    def set_plan(self, n, axis, elems):
        """Plan width along axis (0 x, 1 y) of every instance of size n x n (0 = default)."""
        self._chk(lib().sgp_ensemble_set_plan(self._h, int(n), int(axis), int(elems)))

    def get_plan(self, n, axis):
        e = ctypes.c_int()
        self._chk(lib().sgp_ensemble_get_plan(self._h, int(n), int(axis), ctypes.byref(e)))
        return e.value

    def plans(self):
        """{n: (x width, y width)} over the instance sizes."""
        return {n: (self.get_plan(n, 0), self.get_plan(n, 1)) for n in sorted({sh[0] for sh in self.shapes})}

    def plan_key(self, scheme):
        """JSON plan-cache key: device architecture, the instance sizes with their
        counts, element type and scheme."""
        import torch
        from collections import Counter
        prop = torch.cuda.get_device_properties(self.device)
        arch = getattr(prop, "gcnArchName", "") or prop.name
        sizes = "+".join(f"{k}x{n}^2" for n, k in sorted(Counter(sh[0] for sh in self.shapes).items()))
        return f"{arch}|ensemble:{sizes}|{str(self.torch_dtype).replace('torch.', '')}|TS{scheme}"

    def autotune(self, psis, steps=10, scheme=None, cache=False):
        """sgp_ensemble_autotune on scratch copies of psis; returns (plans(), ms per
        step).  With cache (and the ensemble's scheme), a choice stored in the JSON plan
        cache (plan_cache_path(), shared with Solver.autotune) for this device, set of
        instance sizes, element type and scheme is applied without timing (ms None),
        and a new choice is stored there."""
        import json
        self._ptrs(psis)
        key = self.plan_key(scheme) if cache and scheme is not None else None
        path = plan_cache_path()
        table = {}
        if key is not None and os.path.exists(path):
            try:
                with open(path) as f:
                    table = json.load(f)
            except (OSError, ValueError):
                table = {}
            if key in table:
                for n, (ex, ey) in table[key]["plans"].items():
                    self.set_plan(int(n), 0, int(ex))
                    self.set_plan(int(n), 1, int(ey))
                return self.plans(), None
        scratch = [p.clone() for p in psis]
        arr = self._ptrs(scratch)
        ms = ctypes.c_double()
        self._chk(lib().sgp_ensemble_autotune(self._h, arr, int(steps), ctypes.byref(ms)))
        del scratch
        plans = self.plans()
        if key is not None:
            table[key] = {"plans": {str(n): list(v) for n, v in plans.items()}, "ms_per_step": ms.value}
            try:
                os.makedirs(os.path.dirname(path), exist_ok=True)
                tmp = path + f".{os.getpid()}.tmp"
                with open(tmp, "w") as f:
                    json.dump(table, f, indent=1, sort_keys=True)
                os.replace(tmp, path)
            except OSError:
                pass
        return plans, ms.value

    def close(self):
        if getattr(self, "_h", None):
            lib().sgp_ensemble_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
