"""Dynamical-law quantities on the GPU (sgp_diagnostics: widths, the x y rho moment,
the width rate) against their definitions (Sec. 2, eq. ConWid) written out in numpy
on the same state, and the paper's dynamical laws (Lemmas 1 and 2) checked on the
Example "dynamical laws" workload evolved on the GPU in FP64."""
import numpy as np
import pytest

import oracle
from paper_2603_25282_amd import inputs as I
from tests.gpu_util import to_gpu
from tests.spin2 import soc_width_term
from tests.test_oracle_scheme import smooth_state, spectral_grad

pytestmark = pytest.mark.gpu


def reference(psi, L, theta):
    ny, nx = psi.shape[1:]
    X, Y = I.mesh((ny, nx), L)
    h2 = (2 * L / nx) * (2 * L / ny)
    rho = np.sum(np.abs(psi) ** 2, axis=0)
    Xr, Yr = np.cos(theta) * X + np.sin(theta) * Y, -np.sin(theta) * X + np.cos(theta) * Y
    W = 0.0
    for c in range(5):
        gx, gy = spectral_grad(psi[c], L)
        W += 2 * h2 * np.sum(np.imag(np.conj(psi[c]) * (X * gx + Y * gy)))
    return (h2 * np.sum(Xr ** 2 * rho), h2 * np.sum(Yr ** 2 * rho), h2 * np.sum(Xr * Yr * rho), W)


def soc_rates(psi, L, params, xy):
    """dM/dt and d<Lz>/dt by the laws of Sec. 2 written out in numpy (L_+- = i d_y +- d_x,
    spectral derivatives), for checking the device sums against their definition."""
    ny, nx = psi.shape[1:]
    h2 = (2 * L / nx) * (2 * L / ny)
    g = [spectral_grad(psi[c], L) for c in range(5)]  # (d_x, d_y) per component; index 0..4 = l 2..-2
    lp = lambda c: 1j * g[c][1] + g[c][0]
    lm = lambda c: 1j * g[c][1] - g[c][0]
    ip = lambda a, b: h2 * np.sum(np.conj(psi[a]) * b)
    q1, q2, q3 = ip(0, lm(1)), ip(3, lm(4)), ip(1, lm(2))
    q4, q5 = ip(3, lp(2)), ip(1, lp(0))
    r6h = np.sqrt(6.0) / 2
    gam, gx, gy = params[4], params[5], params[6]
    dM = -2 * gam * np.imag(q1 + q2 + r6h * (q3 - q4))
    dLz = (gx ** 2 - gy ** 2) * xy + 2 * gam * np.imag(q2 - q5 + r6h * (q3 - q4))
    return dM, dLz


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_diagnostics_match_definitions(dtype):
    from paper_2603_25282_amd.sgp import Solver
    shape, L = (64, 128), 8.0
    params = (50.0, -1.0, 2.0, 0.7, 0.4, 1.0, 1.2, 1.0)
    psi = smooth_state(shape, L, 31, lz=0.4)
    s = Solver(shape, L, params, dtype=dtype)
    t = 0.83
    s.time = t
    d = s.diagnostics(to_gpu(s, psi))
    dx, dy, xy, W = reference(psi, L, params[3] * t)
    dM, dLz = soc_rates(psi, L, params, xy)
    # Lemma 2's spin-orbit term on the lab-frame state (psi is the rotating-frame state
    # at clock t; the oracle's mapping takes it to the lab frame)
    G = soc_width_term(oracle.rotation_map(psi, L, params, t, forward=False), L, params)
    got = np.array([d["delta_x"], d["delta_y"], d["xy_rho"], d["width_rate"], d["dM_dt"], d["dLz_dt"],
                    d["soc_width_term"]])
    ref = np.array([dx, dy, xy, W, dM, dLz, G])
    print("gpu", got, "ref", ref, flush=True)
    tol = 1e-12 if dtype == "complex128" else 3e-6
    assert np.all(np.abs(got - ref) <= tol * np.maximum(1.0, np.abs(ref)))
    assert d["delta_z"] == 0.0


def run_ex3(cfg, T, every, extra_times=()):
    """Evolve on the GPU (FP64) and return {t: diagnostics} at multiples of `every`
    and at extra_times."""
    from paper_2603_25282_amd.sgp import Solver
    s = Solver(cfg.shape, cfg.L, cfg.params, dtype="complex128")
    s.build_propagator(cfg.tau, cfg.order)
    psi = to_gpu(s, I.initial_state(cfg))
    marks = sorted(set([round(k * every / cfg.tau) for k in range(int(round(T / every)) + 1)] +
                       [round(x / cfg.tau) for x in extra_times]))
    out, done = {}, 0
    for m in marks:
        if m > done:
            s.step(psi, m - done)
            done = m
        out[m] = s.diagnostics(psi)
    return out


def test_example_dynamical_laws_case_i():
    # gamma = 0, isotropic trap: mass, magnetization and <Lz> conserved; delta_r by
    # the closed form of Lemma 2 (real, radially symmetric data: delta_r'(0) = 0, and
    # delta_x = delta_y = delta_r / 2); energy conserved up to the time discretisation.
    # To the example's horizon t = 12 (12000 TS4 steps of tau = 1e-3 on its 768^2
    # grid of [-24, 24]^2).
    cfg = I.EX3
    T = 12.0
    print(f"case Example dynamical laws i, 768^2 FP64, T={T}", flush=True)
    out = run_ex3(cfg, T, 0.5)
    d0 = out[0]
    E0, lz0 = d0["energy"], d0["lz"]
    dr0 = d0["delta_x"] + d0["delta_y"]
    assert abs(d0["width_rate"]) < 1e-14
    Om = cfg.params[3]
    for m, d in out.items():
        t = m * cfg.tau
        dr = d["delta_x"] + d["delta_y"]
        closed = (E0 + Om * lz0) * (1 - np.cos(2 * t)) + dr0 * np.cos(2 * t)
        print(f"t={t:.2f} mass {d['mass']:.15f} M {d['magnetization']:.3e} Lz {d['lz']:.3e} "
              f"E {d['energy']:.12f} delta_r {dr:.10f} closed {closed:.10f}", flush=True)
        assert abs(d["mass"] - 1.0) < 1e-11  # FP64 rounding over thousands of passes
        assert abs(d["magnetization"] - d0["magnetization"]) < 1e-11
        assert abs(d["lz"] - lz0) < 1e-10
        assert abs(dr - closed) < 1e-8 * closed
        assert abs(d["delta_x"] - d["delta_y"]) < 1e-10 * dr
        assert abs(d["energy"] - E0) < 1e-8 * abs(E0)
    assert max(abs(d["delta_x"] + d["delta_y"] - dr0) for d in out.values()) > 0.1 * dr0  # it breathes


def test_example_dynamical_laws_cases_ii_iii():
    # ii: SOC on (gamma = 0.9): mass and energy conserved, to the example's horizon t = 12.
    # iii: anisotropic trap (gx = 1.3), gamma = 0: mass and magnetization conserved,
    # and d<Lz>/dt = (gx^2 - gy^2) int x y rho (Lemma 1), checked by central differences
    # at t = 1 and t = 11.
    p = list(I.EX3.params)
    p[4] = 0.9
    cii = I.with_(I.EX3, params=tuple(p), name="ex3-ii")
    print("case Example dynamical laws ii, T = 12", flush=True)
    out = run_ex3(cii, 12.0, 1.0)
    E0 = out[0]["energy"]
    for d in out.values():
        assert abs(d["mass"] - 1.0) < 1e-11  # FP64 rounding over thousands of passes
        assert abs(d["energy"] - E0) < 1e-7 * abs(E0)
    p = list(I.EX3.params)
    p[5] = 1.3
    ciii = I.with_(I.EX3, params=tuple(p), name="ex3-iii")
    print("case Example dynamical laws iii", flush=True)
    dt = 0.02
    out = run_ex3(ciii, 11.0, 1.0, extra_times=(1.0 - dt, 1.0 + dt, 11.0 - dt, 11.0 + dt))
    for d in out.values():
        assert abs(d["mass"] - 1.0) < 1e-11  # FP64 rounding over thousands of passes
        assert abs(d["magnetization"] - out[0]["magnetization"]) < 1e-11
    for tc in (1.0, 11.0):
        m0, mm, mp = round(tc / ciii.tau), round((tc - dt) / ciii.tau), round((tc + dt) / ciii.tau)
        dlz = (out[mp]["lz"] - out[mm]["lz"]) / (2 * dt)
        law = (1.3 ** 2 - 1.0) * out[m0]["xy_rho"]
        print(f"t = {tc}: d<Lz>/dt by differences {dlz:.10e}, law {law:.10e}", flush=True)
        if tc == 1.0:
            assert abs(law) > 1e-4
        assert abs(dlz - law) < 1e-3 * max(abs(law), 1e-3)


def test_spin_orbit_laws_by_differences():
    # gamma = 0.9 and an anisotropic trap (gx = 1.3) on the dynamical-laws example:
    # the device's dM/dt (magnetization law, spin-orbit term) and d<Lz>/dt (Lemma 1
    # with its spin-orbit term) against central differences of M(t) and <Lz>(t) of the
    # same GPU trajectory (FP64, TS4, tau = 1e-3)
    p = list(I.EX3.params)
    p[4], p[5] = 0.9, 1.3
    cfg = I.with_(I.EX3, params=tuple(p), name="ex3-soc-aniso")
    # central differences at dt and dt/2, Richardson-extrapolated (error O(dt^4));
    # the trajectory's own error is O(tau^4)
    t0, dt = 0.5, 0.02
    print("case spin-orbit laws by differences, 768^2 FP64", flush=True)
    out = run_ex3(cfg, t0, t0, extra_times=(t0 - dt, t0 + dt, t0 - dt / 2, t0 + dt / 2))
    m = lambda t: round(t / cfg.tau)
    for key, rate in (("magnetization", "dM_dt"), ("lz", "dLz_dt")):
        f1 = (out[m(t0 + dt)][key] - out[m(t0 - dt)][key]) / (2 * dt)
        f2 = (out[m(t0 + dt / 2)][key] - out[m(t0 - dt / 2)][key]) / dt
        fd = (4 * f2 - f1) / 3
        law = out[m(t0)][rate]
        print(f"  d{key}/dt by differences {f1:.10e} (dt), {f2:.10e} (dt/2), extrapolated {fd:.10e}; "
              f"law {law:.10e}", flush=True)
        assert abs(law) > 1e-3
        assert abs(fd - law) <= 1e-5 * abs(law)


def test_width_law_with_spin_orbit_term():
    # Lemma 2 with gamma = 0.9 on the dynamical-laws example's grid and a radial trap:
    # the device's delta_x + delta_y, energy, <Lz> and spin-orbit term G(gamma, Psi)
    # (sgp_diagnostics) satisfy d^2 delta_r/dt^2 = -4 delta_r + 4 E(0) + 4 Omega <Lz> + G,
    # the second derivative by central differences of the same GPU trajectory (FP64,
    # TS4, tau = 1e-3) at dt and dt/2, Richardson-extrapolated
    p = list(I.EX3.params)
    p[4], p[5], p[6] = 0.9, 1.0, 1.0
    cfg = I.with_(I.EX3, params=tuple(p), name="ex3-soc-radial")
    t0, dt = 0.5, 0.02
    print("case width law with the spin-orbit term, 768^2 FP64", flush=True)
    out = run_ex3(cfg, t0, t0, extra_times=(t0 - dt, t0 + dt, t0 - dt / 2, t0 + dt / 2))
    m = lambda t: round(t / cfg.tau)
    dr = lambda t: out[m(t)]["delta_x"] + out[m(t)]["delta_y"]
    d2a = (dr(t0 + dt) - 2 * dr(t0) + dr(t0 - dt)) / dt ** 2
    d2b = (dr(t0 + dt / 2) - 2 * dr(t0) + dr(t0 - dt / 2)) / (dt / 2) ** 2
    d2 = (4 * d2b - d2a) / 3
    o = out[m(t0)]
    law = -4 * dr(t0) + 4 * out[0]["energy"] + 4 * cfg.params[3] * o["lz"] + o["soc_width_term"]
    print(f"  d2 delta_r {d2a:.10e} (dt), {d2b:.10e} (dt/2), extrapolated {d2:.10e}; law {law:.10e} "
          f"(G {o['soc_width_term']:.6e})", flush=True)
    assert abs(o["soc_width_term"]) > 1e-2 * abs(law)
    assert abs(d2 - law) <= 1e-6 * abs(law)


def jz_reference(u, v, Ls):
    """<u, J_z v>_h written out in numpy: J_z = -i (x d_y - y d_x) + F_z, spectral
    derivatives along x and y (any number of dimensions; arrays (5, [nz,] ny, nx))."""
    shape = v.shape[1:]
    dim = len(shape)
    nx, ny = shape[-1], shape[-2]
    x = -Ls[0] + (2 * Ls[0] / nx) * np.arange(nx)
    y = -Ls[1] + (2 * Ls[1] / ny) * np.arange(ny)
    kx = np.pi * np.fft.fftfreq(nx, d=1.0 / nx) / Ls[0]
    ky = np.pi * np.fft.fftfreq(ny, d=1.0 / ny) / Ls[1]
    bx = (1,) * (dim - 1) + (nx,)
    by = (1,) * (dim - 2) + (ny, 1)
    dvx = np.fft.ifft(1j * kx.reshape(bx)[None] * np.fft.fft(v, axis=-1), axis=-1)
    dvy = np.fft.ifft(1j * ky.reshape(by)[None] * np.fft.fft(v, axis=-2), axis=-2)
    X, Y = x.reshape(bx)[None], y.reshape(by)[None]
    m = np.array([2.0, 1.0, 0.0, -1.0, -2.0]).reshape((5,) + (1,) * dim)
    jv = -1j * (X * dvy - Y * dvx) + m * v
    hd = np.prod([2 * Ls[i] / shape[::-1][i] for i in range(dim)])
    return hd * np.vdot(u, jv)


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
@pytest.mark.parametrize("dim", [2, 3])
def test_jz_inner_matches_definition(dtype, dim):
    # sgp_jz_inner against its definition on two unrelated smooth states, on a
    # rectangular grid with different half-widths per axis (a swapped axis or a sign
    # shows); <u, J_z u> is real and equals <Lz> + M of the observables
    from paper_2603_25282_amd.sgp import Solver
    rng = np.random.default_rng(40 + dim)
    if dim == 2:
        shape, Ls = (64, 128), (8.0, 6.0)
    else:
        shape, Ls = (16, 32, 64), (7.0, 6.0, 5.0)
    co = np.meshgrid(*[-Ls[i] + (2 * Ls[i] / shape[::-1][i]) * np.arange(shape[::-1][i]) for i in range(dim)][::-1],
                     indexing="ij")[::-1]
    r2 = sum(c * c for c in co)

    def state():
        a = rng.standard_normal((5, 3)) + 1j * rng.standard_normal((5, 3))
        return np.stack([(a[c, 0] + a[c, 1] * (co[0] + 1j * co[1]) + a[c, 2] * co[0] * co[1]) * np.exp(-r2 / 2)
                         for c in range(5)])
    u, v = state(), state()
    print(f"case jz_inner {shape} {dtype}", flush=True)
    s = Solver(shape, Ls, (0, 0, 0, 0.5, 0.3, 1, 1, 1), dtype=dtype)
    got = s.jz_inner(to_gpu(s, u), to_gpu(s, v))
    ref = jz_reference(u, v, Ls)
    tol = 1e-12 if dtype == "complex128" else 2e-6
    print("gpu", got, "numpy", ref, flush=True)
    assert abs(got - ref) <= tol * abs(ref)
    self_ip = s.jz_inner(to_gpu(s, v), to_gpu(s, v))
    m, E, M, lz = s.observables(to_gpu(s, v))
    assert abs(self_ip.imag) <= tol * abs(self_ip) and abs(self_ip.real - (lz + M)) <= tol * abs(self_ip)
    # the device sum is deterministic
    assert s.jz_inner(to_gpu(s, u), to_gpu(s, v)) == got
