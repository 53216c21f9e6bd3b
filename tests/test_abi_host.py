"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function include/sgp.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2603_25282_amd import sgp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sgp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(sgp_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", sgp.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(line.split()[-1] for line in out.stdout.splitlines() if line.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = sgp.lib()
    for n in names:
        assert hasattr(L, n)
    assert set(sgp.exported_symbols()) <= set(names)


def _create(dim=2, n=(64, 64, 1), L=(8.0, 8.0, 1.0), params=(1, 1, 1, 0.5, 0.5, 1, 1, 1), dtype=0):
    g = sgp._Grid()
    g.dim = dim
    for i in range(3):
        g.n[i] = n[i]
        g.L[i] = L[i]
    p = sgp._Params(*[float(x) for x in params])
    ctx = ctypes.c_void_p()
    rc = sgp.lib().sgp_create(ctypes.byref(g), ctypes.byref(p), dtype, None, ctypes.byref(ctx))
    return rc, ctx


def test_create_validates_arguments():
    L = sgp.lib()
    for kw in (dict(n=(48, 64, 1)), dict(n=(64, 1024, 1)), dict(L=(0.0, 8.0, 1.0)), dict(dim=4),
               dict(params=(1, 1, float("nan"), 0, 0, 1, 1, 1)), dict(dtype=7),
               # 5 x 768^3 state elements do not fit the kernels' 32-bit offsets
               dict(dim=3, n=(768, 768, 768), L=(8.0, 8.0, 8.0))):
        rc, ctx = _create(**kw)
        assert rc == -1, kw
        assert L.sgp_last_error(None)
    assert b"too large" in L.sgp_last_error(None)
    # the largest grids that fit are accepted
    for n in ((768, 768, 512), (512, 512, 512)):
        rc, ctx = _create(dim=3, n=n, L=(8.0, 8.0, 8.0))
        assert rc == 0, n
        L.sgp_destroy(ctx)
    rc, ctx = _create()
    assert rc == 0
    nb = ctypes.c_size_t()
    assert L.sgp_workspace_size(ctx, ctypes.byref(nb)) == 0 and nb.value > 64 * 64 * 8
    # calls out of order fail cleanly without a device
    assert L.sgp_build_propagator(ctx, 1e-3, 2) == -2
    assert L.sgp_step(ctx, ctypes.c_void_p(1), 1) == -2
    assert b"workspace" in L.sgp_last_error(ctx)
    assert L.sgp_set_workspace(ctx, ctypes.c_void_p(256), 1) == -5
    assert L.sgp_set_option(ctx, 99, 0) == -1
    # pass timing: both timing modes at once, an unknown flag, or a z-pass in 2D are
    # argument errors, checked before any device work
    ms = ctypes.c_double()
    for pk in (256 | 512, 1024, 2 | 512, -1):
        assert L.sgp_time_pass(ctx, ctypes.c_void_p(1), pk, 4, ctypes.byref(ms)) == -1, pk
    assert L.sgp_time_pass(ctx, ctypes.c_void_p(1), 512, 5000, ctypes.byref(ms)) == -1  # too many timed steps
    t = ctypes.c_double(-1.0)
    assert L.sgp_set_time(ctx, 0.25) == 0 and L.sgp_get_time(ctx, ctypes.byref(t)) == 0 and t.value == 0.25
    L.sgp_destroy(ctx)


def test_workspace_size_scales_with_grid_and_dtype():
    L = sgp.lib()
    sizes = {}
    for n, dt in ((64, 0), (64, 1), (256, 0)):
        rc, ctx = _create(n=(n, n, 1), dtype=dt)
        nb = ctypes.c_size_t()
        L.sgp_workspace_size(ctx, ctypes.byref(nb))
        sizes[(n, dt)] = nb.value
        L.sgp_destroy(ctx)
    assert sizes[(64, 1)] > sizes[(64, 0)] and sizes[(256, 0)] > 10 * sizes[(64, 0)]


def test_plan_widths_and_plan_setters_without_device():
    L = sgp.lib()
    for n, want in ((16, [8, 4]), (32, [8, 4]), (64, [8, 4, 16]), (128, [8, 4, 16]), (256, [8, 4, 16]),
                    (512, [8, 4, 16]), (192, [12, 24]), (384, [12, 24]), (768, [12, 24])):
        assert sgp.plan_widths(n) == want
        assert sgp.plan_widths(n, "complex128") == [e for e in want if e != 24]
    out = (ctypes.c_int * 1)()
    assert L.sgp_plan_widths(512, 0, out, 1) == 3 and out[0] == 8  # count even when truncated
    assert L.sgp_plan_widths(48, 0, out, 1) == -1
    assert L.sgp_plan_widths(64, 5, out, 1) == -1
    rc, ctx = _create(n=(512, 64, 1))
    assert rc == 0
    e = ctypes.c_int()
    assert L.sgp_get_plan(ctx, 0, ctypes.byref(e)) == 0 and e.value == 8
    assert L.sgp_set_plan(ctx, 0, 4) == 0
    assert L.sgp_get_plan(ctx, 0, ctypes.byref(e)) == 0 and e.value == 4
    assert L.sgp_set_plan(ctx, 1, 16) == 0
    assert L.sgp_set_plan(ctx, 1, 12) == -1 and b"not available" in L.sgp_last_error(ctx)
    assert L.sgp_set_plan(ctx, 2, 8) == -1  # 2D: no z axis
    assert L.sgp_set_plan(ctx, 0, 0) == 0
    assert L.sgp_get_plan(ctx, 0, ctypes.byref(e)) == 0 and e.value == 8
    outw = (ctypes.c_int * 3)()
    assert L.sgp_autotune(ctx, ctypes.c_void_p(1), 5, outw, None) == -2  # no workspace yet
    assert L.sgp_autotune(ctx, ctypes.c_void_p(1), 0, outw, None) == -1
    # the linear-substep split (pseudo-axis 3) exists for 3D contexts only
    assert L.sgp_set_plan(ctx, 3, 1) == -1 and L.sgp_get_plan(ctx, 3, ctypes.byref(e)) == -1
    L.sgp_destroy(ctx)
    rc, ctx = _create(dim=3, n=(32, 32, 16), L=(8.0, 8.0, 8.0))
    assert rc == 0
    assert L.sgp_get_plan(ctx, 3, ctypes.byref(e)) == 0 and e.value == 0
    assert L.sgp_set_plan(ctx, 3, 1) == 0
    assert L.sgp_get_plan(ctx, 3, ctypes.byref(e)) == 0 and e.value == 1
    assert L.sgp_set_plan(ctx, 3, 2) == -1 and b"split" in L.sgp_last_error(ctx)
    assert L.sgp_set_plan(ctx, 4, 0) == -1
    # z-slabs of the pipelined step body (option 4): a divisor of nz (16 here), 0/1 = off
    for S in (0, 1, 2, 4, 8, 16):
        assert L.sgp_set_option(ctx, sgp.SGP_OPT_SLABS, S) == 0
    for S in (3, 32, -2):
        assert L.sgp_set_option(ctx, sgp.SGP_OPT_SLABS, S) == -1 and b"z-slabs" in L.sgp_last_error(ctx)
    L.sgp_destroy(ctx)
    rc, ctx = _create(n=(64, 64, 1))
    assert rc == 0
    assert L.sgp_set_option(ctx, sgp.SGP_OPT_SLABS, 2) == -1 and b"3D" in L.sgp_last_error(ctx)
    assert L.sgp_set_option(ctx, sgp.SGP_OPT_SLABS, 0) == 0
    L.sgp_destroy(ctx)


def test_ensemble_plan_setters_without_device():
    L = sgp.lib()
    grids = (sgp._Grid * 3)()
    pars = (sgp._Params * 3)()
    for i, n in enumerate((128, 512, 128)):
        grids[i].dim = 2
        grids[i].n[0] = grids[i].n[1] = n
        grids[i].n[2] = 1
        grids[i].L[0] = grids[i].L[1] = 8.0
        pars[i] = sgp._Params(1, 1, 1, 0.5, 0.5, 1, 1, 1)
    L.sgp_ensemble_create.argtypes = [ctypes.c_int, ctypes.POINTER(sgp._Grid), ctypes.POINTER(sgp._Params),
                                      ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    L.sgp_ensemble_set_plan.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.sgp_ensemble_get_plan.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.sgp_ensemble_autotune.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double)]
    L.sgp_ensemble_destroy.argtypes = [ctypes.c_void_p]
    L.sgp_ensemble_destroy.restype = None
    h = ctypes.c_void_p()
    assert L.sgp_ensemble_create(3, grids, pars, 0, None, ctypes.byref(h)) == 0
    e = ctypes.c_int()
    assert L.sgp_ensemble_get_plan(h, 128, 0, ctypes.byref(e)) == 0 and e.value == 8
    assert L.sgp_ensemble_set_plan(h, 128, 1, 16) == 0
    assert L.sgp_ensemble_get_plan(h, 128, 1, ctypes.byref(e)) == 0 and e.value == 16
    assert L.sgp_ensemble_set_plan(h, 512, 0, 4) == -1  # 640-thread geometry: not batched
    assert L.sgp_ensemble_set_plan(h, 256, 0, 8) == -1  # no instance of that size
    assert L.sgp_ensemble_set_plan(h, 128, 2, 8) == -1
    ptrs = (ctypes.c_void_p * 3)(1, 2, 3)
    assert L.sgp_ensemble_autotune(h, ptrs, 4, None) == -2  # no workspace
    L.sgp_ensemble_destroy(h)


def test_ensemble_adjoint_entry_points_validate_without_device():
    L = sgp.lib()
    grids = (sgp._Grid * 1)()
    pars = (sgp._Params * 1)()
    grids[0].dim = 2
    grids[0].n[0] = grids[0].n[1] = 64
    grids[0].n[2] = 1
    grids[0].L[0] = grids[0].L[1] = 8.0
    pars[0] = sgp._Params(1, 1, 1, 0.5, 0.5, 1, 1, 1)
    vp = ctypes.c_void_p
    L.sgp_ensemble_create.argtypes = [ctypes.c_int, ctypes.POINTER(sgp._Grid), ctypes.POINTER(sgp._Params),
                                      ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.sgp_ensemble_store_size.argtypes = [vp, ctypes.c_long, ctypes.POINTER(ctypes.c_size_t)]
    L.sgp_ensemble_step_store.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_long, vp, ctypes.c_size_t]
    L.sgp_ensemble_set_time.argtypes = [vp, ctypes.c_double]
    L.sgp_ensemble_get_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.sgp_ensemble_destroy.argtypes = [vp]
    L.sgp_ensemble_destroy.restype = None
    h = vp()
    assert L.sgp_ensemble_create(1, grids, pars, 1, None, ctypes.byref(h)) == 0
    nb = ctypes.c_size_t()
    assert L.sgp_ensemble_store_size(h, 4, ctypes.byref(nb)) == -2  # no scheme yet
    ptrs = (vp * 1)(256)
    assert L.sgp_ensemble_step_store(h, ptrs, 4, vp(256), 1 << 20) == -2  # no workspace
    assert L.sgp_ensemble_set_time(h, 0.25) == 0
    t = ctypes.c_double()
    assert L.sgp_ensemble_get_time(h, ctypes.byref(t)) == 0 and t.value == 0.25
    L.sgp_ensemble_destroy(h)


def test_ensemble_binding_refuses_a_state_list_of_the_wrong_length():
    # the C ABI reads one state pointer per instance: the binding must refuse a list
    # of another length before any library call (here there is no library handle at
    # all, so reaching the library would fail differently)
    import torch
    e = object.__new__(sgp.Ensemble)
    e.shapes = [(64, 64), (128, 128)]
    e.torch_dtype = torch.complex64
    e.device = torch.device("cpu")
    e._h = None
    one = [torch.zeros((64, 64, 5), dtype=torch.complex64)]
    three = one + [torch.zeros((128, 128, 5), dtype=torch.complex64), torch.zeros((8, 8, 5), dtype=torch.complex64)]
    for psis in (one, three):
        for call in (lambda p: e.step(p, 1), lambda p: e.step_store(p, 1, torch.zeros(8, dtype=torch.uint8)),
                     lambda p: e.adjoint_segment(p, 1, torch.zeros(8, dtype=torch.uint8)),
                     lambda p: e.autotune(p)):
            with pytest.raises(sgp.SgpError, match="instances given"):
                call(psis)
