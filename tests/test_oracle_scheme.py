"""Scheme-level pins for the oracle (Secs. 2, 3.3, 3.4): exact plane-wave evolution
with the nonlinearity off, discrete mass and magnetization conservation, <Lz>
conservation, the condensate-width closed form of Lemma 2 and its law with the
spin-orbit term, approximate energy
conservation, time reversibility, and equivalence of the rotating-frame evolution
with the paper's literal lab-frame Algorithm 1 (RSDA mapping every step)."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from paper_2603_25282_amd import inputs as I
from tests.spin2 import Qmat, Smat, soc_width_term


def spectral_grad(f, L):
    n = f.shape
    ky = np.pi * np.fft.fftfreq(n[0], d=1.0 / n[0]) / L
    kx = np.pi * np.fft.fftfreq(n[1], d=1.0 / n[1]) / L
    F = np.fft.fft2(f)
    return np.fft.ifft2(1j * kx[None, :] * F), np.fft.ifft2(1j * ky[:, None] * F)


def smooth_state(shape, L, seed, lz=0.3):
    """Smooth, decaying 5-component data with nonzero angular momentum."""
    rng = np.random.default_rng(seed)
    X, Y = I.mesh(shape, L)
    comps = []
    for _ in range(5):
        c = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        w = rng.uniform(0.8, 1.2)
        comps.append((c[0] + lz * c[1] * (X + 1j * Y) + 0.1 * c[2] * X * Y) * np.exp(-w * (X ** 2 + Y ** 2) / 2))
    return I.normalise(np.stack(comps), shape, L)


def test_plane_wave_exact_linear_evolution():
    # V = 0 and c = 0: the nonlinear substep is the identity and a single Fourier mode
    # evolves as exp(-i n tau |nu|^2/2) exp(i n tau Q) v (eq. sl1).
    L, N = 4.0, 16
    params = (0.0, 0.0, 0.0, 0.7, 0.9, 0.0, 0.0, 0.0)
    X, Y = I.mesh((N, N), L)
    p, q = 3, -2
    nup, nuq = np.pi * p / L, np.pi * q / L
    v = np.array([0.3, -0.2j, 0.5, 0.1 + 0.1j, -0.4])
    mode = np.exp(1j * (nup * (X + L) + nuq * (Y + L)))
    psi = v[:, None, None] * mode[None]
    tau, n = 0.013, 7
    for order in (2, 4):
        out = oracle.evolve(psi, L, params, order, tau, n)
        w = np.exp(-0.5j * n * tau * (nup ** 2 + nuq ** 2)) * (sl.expm(1j * n * tau * Qmat(0.7, 0.9, nup, nuq)) @ v)
        assert np.abs(out - w[:, None, None] * mode[None]).max() < 1e-13


def test_observables_on_known_states():
    L, N = 10.0, 96
    X, Y = I.mesh((N, N), L)
    h2 = (2 * L / N) ** 2
    # Harmonic ground state, no interactions: E = d/2 = 1, <Lz> = 0.
    g = np.exp(-(X ** 2 + Y ** 2) / 2) / np.sqrt(np.pi)
    psi = np.zeros((5, N, N), complex)
    psi[2] = g
    m, E, M, lz = oracle.observables(psi, L, (0, 0, 0, 0.4, 0, 1, 1, 1))
    assert abs(m - 1) < 1e-12 and abs(E - 1) < 1e-12 and abs(lz) < 1e-12 and abs(M) < 1e-14
    # (x + i y) exp(-r^2/2) is an Lz eigenstate with eigenvalue +1; put it in l = -1.
    psi = np.zeros((5, N, N), complex)
    psi[3] = (X + 1j * Y) * np.exp(-(X ** 2 + Y ** 2) / 2)
    psi = I.normalise(psi, (N, N), L)
    m, E, M, lz = oracle.observables(psi, L, (0, 0, 0, 0.4, 0, 1, 1, 1))
    assert abs(lz - 1) < 1e-12 and abs(M + 1) < 1e-12
    # E = 2 (trap level) - Omega <Lz>
    assert abs(E - (2.0 - 0.4)) < 1e-11
    # Plane wave, Omega = 0, c = 0, V = 0: E = |nu|^2/2 |v|^2 - gamma v^H S(nu) v.
    p, q = 2, -3
    nup, nuq = np.pi * p / L, np.pi * q / L
    v = np.array([0.2, 0.3j, -0.5, 0.1, 0.4 - 0.2j])
    psi = v[:, None, None] * np.exp(1j * (nup * X + nuq * Y))[None] / np.sqrt(4 * L * L)
    ga = 0.8
    m, E, M, lz = oracle.observables(psi, L, (0, 0, 0, 0, ga, 0, 0, 0))
    ref = 0.5 * (nup ** 2 + nuq ** 2) * np.vdot(v, v).real - ga * np.vdot(v, Smat(nup, nuq) @ v).real
    assert abs(m - np.vdot(v, v).real) < 1e-12 and abs(E - ref) < 1e-11
    # Interaction energy of a constant state: c0 rho^2/2 + c1 |F|^2/2 + c2 |A00|^2/2 per area.
    psi = np.ones((5, N, N), complex) * np.array([0.1, 0.2j, 0.3, -0.1, 0.05])[:, None, None]
    from tests.spin2 import densities
    rho, F, A00 = densities(psi[:, 0, 0])
    m, E, M, lz = oracle.observables(psi, L, (7.0, -3.0, 5.0, 0, 0, 0, 0, 0))
    ref = 4 * L * L * (3.5 * rho ** 2 - 1.5 * np.dot(F, F) + 2.5 * abs(A00) ** 2)
    assert abs(E - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("order", [2, 4])
def test_mass_conserved_any_gamma_omega(order):
    cfg = I.with_(I.C1, shape=(32, 32))
    psi = I.initial_state(cfg)
    out = oracle.evolve(psi, cfg.L, cfg.params, order, 2e-3, 60)
    m0 = oracle.observables(psi, cfg.L, cfg.params)[0]
    m1 = oracle.observables(out, cfg.L, cfg.params)[0]
    assert abs(m1 - m0) < 1e-13


def test_magnetization_and_lz_conserved_without_soc():
    # gamma = 0: discrete magnetization is conserved exactly (Sec. 3.4); with an
    # isotropic trap <Lz> is conserved as well (Lemma 1), up to the spatial
    # discretisation error (spectrally small on a resolved grid).
    shape, L = (96, 96), 8.0
    params = (80.0, 2.0, -3.0, 0.6, 0.0, 1.0, 1.0, 1.0)
    psi = smooth_state(shape, L, 7)
    out = oracle.evolve(psi, L, params, 4, 5e-3, 60)
    o0 = oracle.observables(psi, L, params)
    o1 = oracle.observables(out, L, params, theta=params[3] * 0.3)
    assert abs(o1[2] - o0[2]) < 1e-12
    assert abs(o1[3] - o0[3]) < 1e-10
    assert abs(o0[3]) > 0.05
    # with SOC on, magnetization is not conserved
    params2 = params[:4] + (0.8,) + params[5:]
    out2 = oracle.evolve(psi, L, params2, 4, 5e-3, 60)
    assert abs(oracle.observables(out2, L, params2)[2] - o0[2]) > 1e-4


def test_energy_drift_shrinks_with_order():
    shape, L = (64, 64), 8.0
    params = (60.0, -1.0, 2.0, 0.5, 0.6, 1.0, 1.2, 1.0)
    psi = smooth_state(shape, L, 8)
    tau, n = 1e-2, 30
    e0 = oracle.observables(psi, L, params)[1]
    drift = {}
    for order in (2, 4):
        out = oracle.evolve(psi, L, params, order, tau, n)
        e1 = oracle.observables(out, L, params, theta=params[3] * tau * n)[1]
        drift[order] = abs(e1 - e0) / abs(e0)
    assert drift[2] < 1e-3 and drift[4] < drift[2] / 10


def test_width_closed_form_without_soc():
    # Lemma 2: gamma = 0, isotropic trap gamma_r = 1:
    # delta_r(t) = (E(0) + Omega <Lz>(0)) (1 - cos 2t) + delta_r(0) cos 2t + delta_r'(0)/2 sin 2t.
    shape, L = (96, 96), 12.0
    params = (20.0, 1.0, 1.0, 0.3, 0.0, 1.0, 1.0, 1.0)
    psi = smooth_state(shape, L, 9, lz=0.5)
    X, Y = I.mesh(shape, L)
    h2 = (2 * L / shape[0]) ** 2
    r2 = X ** 2 + Y ** 2
    d0 = h2 * np.sum(r2 * np.abs(psi) ** 2)
    d1 = 0.0
    for c in range(5):
        gx, gy = spectral_grad(psi[c], L)
        d1 += 2 * h2 * np.sum(np.imag(np.conj(psi[c]) * (X * gx + Y * gy)))
    m, E, M, lz = oracle.observables(psi, L, params)
    tau, n = 5e-3, 60
    out = oracle.evolve(psi, L, params, 4, tau, n)
    t = tau * n
    dr = h2 * np.sum(r2 * np.abs(out) ** 2)
    ref = (E + params[3] * lz) * (1 - np.cos(2 * t)) + d0 * np.cos(2 * t) + d1 / 2 * np.sin(2 * t)
    assert abs(dr - ref) < 1e-8 * abs(ref)
    assert abs(dr - d0) > 1e-2  # the width really moves


def test_width_law_with_spin_orbit_term():
    # Lemma 2 with gamma != 0 (radial trap gr = 1): d^2 delta_r/dt^2 = -4 delta_r + 4 E(0)
    # + 4 Omega <Lz>(t) + G(gamma, Psi), G written out from its definition
    # (tests.spin2.soc_width_term) on the lab-frame state; the second derivative of the
    # oracle's delta_r(t) by central differences at dt and dt/2, Richardson-extrapolated.
    # G's three parts (the Omega F_+ term, the weighted density, the F_z L_z term) are
    # -5 %, 105 % and 0.2 % of it here, so dropping or mis-signing any one fails.
    shape, L = (128, 128), 8.0
    params = (10.0, 1.0, 1.0, 0.3, 0.5, 1.0, 1.0, 1.0)
    X, Y = I.mesh(shape, L)
    g = np.exp(-((X - 0.3) ** 2 + (Y + 0.2) ** 2) / 2.0)
    psi0 = I.normalise(np.stack([g * (0.3 + 0.1j * X), g * (0.5 + 0.2 * Y), g * (1.0 + 0.1j * X * Y),
                                 g * (0.4 - 0.1j * Y), g * 0.2 * (1 + 1j * X)]), shape, L)
    h2 = (2 * L / shape[0]) ** 2
    tau, n0, k = 1e-3, 100, 10
    E0 = oracle.observables(psi0, L, params)[1]
    states = {}
    phi = oracle.evolve(psi0, L, params, 4, tau, n0 - 2 * k)
    for j in range(-2, 3):
        if j > -2:
            phi = oracle.evolve(phi, L, params, 4, tau, k, t0=(n0 + (j - 1) * k) * tau)
        states[j] = phi
    t0 = n0 * tau
    lab = {j: oracle.rotation_map(p, L, params, (n0 + j * k) * tau, forward=False) for j, p in states.items()}
    dr = {j: h2 * np.sum((X ** 2 + Y ** 2) * np.abs(p) ** 2) for j, p in lab.items()}
    dt = k * tau
    d2a = (dr[2] - 2 * dr[0] + dr[-2]) / (2 * dt) ** 2
    d2b = (dr[1] - 2 * dr[0] + dr[-1]) / dt ** 2
    d2 = (4 * d2b - d2a) / 3
    lz = oracle.observables(states[0], L, params, theta=params[3] * t0)[3]
    G = soc_width_term(lab[0], L, params)
    law = -4 * dr[0] + 4 * E0 + 4 * params[3] * lz + G
    print(f"d2 delta_r: {d2a:.8f} (2 dt), {d2b:.8f} (dt), extrapolated {d2:.8f}; law {law:.8f} (G {G:.8f})")
    assert abs(G) > 1.0
    assert abs(d2 - law) <= 1e-7 * abs(law)


@pytest.mark.parametrize("order", [2, 4])
def test_time_reversibility(order):
    cfg = I.with_(I.C1, shape=(32, 32))
    psi = I.initial_state(cfg)
    n, tau = 25, 2e-3
    fwd = oracle.evolve(psi, cfg.L, cfg.params, order, tau, n)
    back = oracle.evolve(fwd, cfg.L, cfg.params, order, -tau, n, t0=n * tau)
    assert np.abs(back - psi).max() < 1e-12 * np.abs(psi).max()


@pytest.mark.parametrize("order", [2, 4])
def test_rotating_frame_equals_lab_frame_algorithm(order):
    # The rotating-frame evolution with the trap at R(Omega s) x (s the linear-substep
    # clock), mapped back with RSDA, equals Algorithm 1 with the mapping every step,
    # up to spectral interpolation error (which shrinks with h).
    shape, L = (96, 96), 8.0
    params = (40.0, -1.0, 2.0, 0.8, 0.5, 1.0, 1.3, 1.0)
    psi = smooth_state(shape, L, 10, lz=0.2)
    tau, n = 1e-2, 15
    rot = oracle.evolve(psi, L, params, order, tau, n, frame="rotating")
    lab = oracle.evolve(psi, L, params, order, tau, n, frame="lab")
    lab_in_rot = oracle.rotation_map(lab, L, params, tau * n, forward=True)
    rel = np.linalg.norm(rot - lab_in_rot) / np.linalg.norm(rot)
    assert rel < 1e-8
    # and the rotation mapping is not the identity here
    assert np.linalg.norm(lab - lab_in_rot) / np.linalg.norm(rot) > 1e-2


def test_rotation_map_round_trip_and_pure_rotation():
    shape, L = (64, 64), 10.0
    params = (0, 0, 0, 0.9, 0, 1, 1, 1)
    psi = smooth_state(shape, L, 11)
    t = 0.7
    fwd = oracle.rotation_map(psi, L, params, t, forward=True)
    back = oracle.rotation_map(fwd, L, params, t, forward=False)
    assert np.abs(back - psi).max() < 1e-12
    # phi_l(x) = exp(-i l Omega t) psi_l(R(t) x): check on an analytic function
    X, Y = I.mesh(shape, L)
    th = 0.9 * t
    f = lambda x, y: (x + 0.5 * y) * np.exp(-((x - 1) ** 2 + 2 * y ** 2) / 2)
    psi = np.stack([f(X, Y)] * 5).astype(complex)
    fwd = oracle.rotation_map(psi, L, params, t, forward=True)
    Xr, Yr = np.cos(th) * X + np.sin(th) * Y, -np.sin(th) * X + np.cos(th) * Y
    for c, l in enumerate([2, 1, 0, -1, -2]):
        assert np.abs(fwd[c] - np.exp(-1j * l * th) * f(Xr, Yr)).max() < 1e-10


def test_observed_temporal_orders_rotating_anisotropic():
    # Observed orders 2 (TS2) and 4 (TS4) with rotation, SOC and an anisotropic trap,
    # against a TS4 reference at tau/16.
    shape, L = (64, 64), 8.0
    params = (100.0, -2.0, 4.0, 0.9, 1.0, 1.0, 1.1, 1.0)
    psi = smooth_state(shape, L, 12, lz=0.2)
    T = 0.05
    ref = oracle.evolve(psi, L, params, 4, T / 160, 160)
    for order, want in ((2, 2.0), (4, 4.0)):
        e = []
        for n in (5, 10):
            u = oracle.evolve(psi, L, params, order, T / n, n)
            e.append(np.linalg.norm(u - ref))
        rate = np.log2(e[0] / e[1])
        assert abs(rate - want) < 0.15, (order, rate)


def test_sixth_order_composition_observed_order():
    # The triple jump S4(z1) S4(z0) S4(z1) (Yoshida's construction, which Sec. 3.3
    # cites for higher orders) converges at order 6; its coefficients sum to 1 on
    # both flows.
    cfg = I.with_(I.C2, shape=(64, 64), name="order6")
    psi0 = I.initial_state(cfg)
    T = 0.05
    ref = oracle.evolve(psi0, cfg.L, cfg.params, 6, T / 320, 320)
    errs = []
    for k in (5, 10, 20, 40):
        got = oracle.evolve(psi0, cfg.L, cfg.params, 6, T / k, k)
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    print("TS6 errors", errs, "orders", rates)
    assert all(5.5 < r < 6.3 for r in rates) and rates[-1] > 5.85
