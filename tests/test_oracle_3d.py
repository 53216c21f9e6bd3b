"""Pins of the oracle's 3D branches against closed forms (Sec. 3.1's remark on the
3D extension: rotation and spin-orbit coupling act in the x-y plane only, so the
spin part of the Fourier-space propagator depends on (nu_p, nu_q) alone while the
Laplace phase carries nu_r too; the harmonic trap, eq. harmonic, gains
gamma_z^2 z^2 / 2).  Each term the 3D path adds has a check here that a dropped
term, a wrong axis or a wrong sign fails:

* the nu_r term of the kinetic phase: exact evolution of one 3D Fourier mode
  with the nonlinearity and the trap off (anisotropic grid and domain, so that a
  swapped axis shows);
* the gamma_z^2 z^2 term of the trap: the nonlinear substep with c = 0 is the
  exact phase exp(-i d V(R(theta) x)) at every point, and the harmonic ground state
  of an anisotropic trap has the closed-form energy (gx + gy + gz)/2;
* the z derivative of the energy: kinetic energy of a 3D plane wave, and the
  energy of an L_z eigenstate (the energy minus Omega <Lz>, Sec. 2);
* the 3D rotation mapping: phi_l(x) = exp(-i l Omega t) psi_l(R(t) x) with z fixed;
* the whole 3D scheme: mass conservation, magnetization and <Lz> conservation
  without spin-orbit coupling (Sec. 3.4, Lemma 1), the ground state evolving by the
  phase exp(-i E t).
Table Acc2 itself is reproduced in tests/test_oracle_paper_table_3d.py."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
from paper_2603_25282_amd import inputs as I
from tests.spin2 import Qmat, Smat

# an anisotropic grid: (nz, ny, nx) = (8, 12, 16) on half-widths (Lx, Ly, Lz) = (5, 3, 4)
SHAPE = (8, 12, 16)
LS = (5.0, 3.0, 4.0)


def mesh3(shape, Ls):
    nz, ny, nx = shape
    x = -Ls[0] + (2 * Ls[0] / nx) * np.arange(nx)
    y = -Ls[1] + (2 * Ls[1] / ny) * np.arange(ny)
    z = -Ls[2] + (2 * Ls[2] / nz) * np.arange(nz)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def test_plane_wave_3d_exact_linear_evolution():
    # V = 0 and c = 0: the nonlinear substep is the identity and the mode
    # exp(i (nu_p x + nu_q y + nu_r z)) v evolves as
    # exp(-i n tau (nu_p^2 + nu_q^2 + nu_r^2)/2) exp(i n tau Q(nu_p, nu_q)) v.
    params = (0.0, 0.0, 0.0, 0.7, 0.9, 0.0, 0.0, 0.0)
    X, Y, Z = mesh3(SHAPE, LS)
    p, q, r = 3, -2, 3
    nup, nuq, nur = np.pi * p / LS[0], np.pi * q / LS[1], np.pi * r / LS[2]
    v = np.array([0.3, -0.2j, 0.5, 0.1 + 0.1j, -0.4])
    mode = np.exp(1j * (nup * X + nuq * Y + nur * Z))
    psi = v[:, None, None, None] * mode[None]
    tau, n = 0.013, 7
    for order in (2, 4):
        out = oracle.evolve(psi, LS, params, order, tau, n)
        w = np.exp(-0.5j * n * tau * (nup ** 2 + nuq ** 2 + nur ** 2)) * (
            sl.expm(1j * n * tau * Qmat(0.7, 0.9, nup, nuq)) @ v)
        assert np.abs(out - w[:, None, None, None] * mode[None]).max() < 1e-13
        # without the nu_r term the phase would be off by n tau nu_r^2 / 2 = 0.05
        wrong = w * np.exp(0.5j * n * tau * nur ** 2)
        assert np.abs(out - wrong[:, None, None, None] * mode[None]).max() > 1e-2


@pytest.mark.parametrize("theta", [0.0, 0.6])
def test_nonlinear_substep_3d_trap_phase(theta):
    # c = 0: the nonlinear flow is exp(-i d V) psi with V at the rotated point,
    # V = (gx^2 X^2 + gy^2 Y^2 + gz^2 z^2)/2, (X, Y) = R(theta)(x, y)
    params = (0.0, 0.0, 0.0, 0.4, 0.3, 1.0, 1.3, 2.5)
    X, Y, Z = mesh3(SHAPE, LS)
    rng = np.random.default_rng(31)
    psi = rng.standard_normal((5,) + SHAPE) + 1j * rng.standard_normal((5,) + SHAPE)
    d = 0.021
    out = oracle.nl_step(psi, LS, params, d, theta=theta)
    Xr = np.cos(theta) * X + np.sin(theta) * Y
    Yr = -np.sin(theta) * X + np.cos(theta) * Y
    V = 0.5 * (1.0 * Xr ** 2 + 1.3 ** 2 * Yr ** 2 + 2.5 ** 2 * Z ** 2)
    assert np.abs(out - np.exp(-1j * d * V)[None] * psi).max() < 1e-13 * np.abs(psi).max()


def test_observables_3d_known_states():
    N, L = 64, 8.0
    shape = (N, N, N)
    X, Y, Z = mesh3(shape, (L, L, L))
    gx, gy, gz = 1.0, 1.3, 2.0
    # anisotropic harmonic ground state, no interactions: E = (gx + gy + gz)/2, <Lz> = 0
    g = (gx * gy * gz / np.pi ** 3) ** 0.25 * np.exp(-(gx * X ** 2 + gy * Y ** 2 + gz * Z ** 2) / 2)
    psi = np.zeros((5,) + shape, complex)
    psi[2] = g
    m, E, M, lz = oracle.observables(psi, L, (0, 0, 0, 0.4, 0, gx, gy, gz))
    assert abs(m - 1) < 1e-12 and abs(E - (gx + gy + gz) / 2) < 1e-12 and abs(lz) < 1e-12 and abs(M) < 1e-14
    # (x + i y) exp(-(x^2 + y^2)/2) exp(-gz z^2/2) in l = -1: <Lz> = 1 and the energy
    # 2 (first excited level in the plane) + gz/2 (z ground level) - Omega <Lz>
    psi = np.zeros((5,) + shape, complex)
    psi[3] = (X + 1j * Y) * np.exp(-(X ** 2 + Y ** 2) / 2 - gz * Z ** 2 / 2)
    psi = I.normalise(psi, shape, L)
    m, E, M, lz = oracle.observables(psi, L, (0, 0, 0, 0.4, 0, 1.0, 1.0, gz))
    assert abs(lz - 1) < 1e-12 and abs(M + 1) < 1e-12
    assert abs(E - (2.0 + gz / 2 - 0.4)) < 1e-11
    # 3D plane wave, Omega = 0, c = 0, V = 0 on the anisotropic grid:
    # E = |nu|^2/2 |v|^2 - gamma v^H S(nu_p, nu_q) v (nu_r in the kinetic term only)
    X, Y, Z = mesh3(SHAPE, LS)
    p, q, r = 2, -3, 2
    nup, nuq, nur = np.pi * p / LS[0], np.pi * q / LS[1], np.pi * r / LS[2]
    v = np.array([0.2, 0.3j, -0.5, 0.1, 0.4 - 0.2j])
    vol = 8 * LS[0] * LS[1] * LS[2]
    psi = v[:, None, None, None] * np.exp(1j * (nup * X + nuq * Y + nur * Z))[None] / np.sqrt(vol)
    ga = 0.8
    m, E, M, lz = oracle.observables(psi, LS, (0, 0, 0, 0, ga, 0, 0, 0))
    vv = np.vdot(v, v).real
    ref = 0.5 * (nup ** 2 + nuq ** 2 + nur ** 2) * vv - ga * np.vdot(v, Smat(nup, nuq) @ v).real
    assert abs(m - vv) < 1e-12 and abs(E - ref) < 1e-11
    assert abs(0.5 * nur ** 2 * vv) > 0.1  # the z part is not negligible here


def test_rotation_map_3d_pure_rotation():
    # phi_l(x, y, z) = exp(-i l Omega t) psi_l(R(t)(x, y), z) on an analytic function
    shape, L = (16, 64, 64), 10.0
    params = (0, 0, 0, 0.9, 0, 1, 1, 1)
    X, Y, Z = mesh3(shape, (L, L, L))
    t = 0.7
    th = 0.9 * t
    f = lambda x, y, z: (x + 0.5 * y + 0.3 * z) * np.exp(-((x - 1) ** 2 + 2 * y ** 2 + z ** 2) / 2)
    psi = np.stack([f(X, Y, Z)] * 5).astype(complex)
    fwd = oracle.rotation_map(psi, L, params, t, forward=True)
    Xr, Yr = np.cos(th) * X + np.sin(th) * Y, -np.sin(th) * X + np.cos(th) * Y
    for c, l in enumerate([2, 1, 0, -1, -2]):
        assert np.abs(fwd[c] - np.exp(-1j * l * th) * f(Xr, Yr, Z)).max() < 1e-10
    back = oracle.rotation_map(fwd, L, params, t, forward=False)
    assert np.abs(back - psi).max() < 1e-12


def smooth_state_3d(shape, L, seed, lz=0.3):
    rng = np.random.default_rng(seed)
    X, Y, Z = mesh3(shape, (L, L, L))
    comps = []
    for _ in range(5):
        c = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        w = rng.uniform(0.8, 1.2)
        comps.append((c[0] + lz * c[1] * (X + 1j * Y) + 0.1 * c[2] * Z) * np.exp(-w * (X ** 2 + Y ** 2 + 2 * Z ** 2) / 2))
    return I.normalise(np.stack(comps), shape, L)


def test_conservation_3d():
    # mass for any gamma and Omega (Sec. 3.4); without spin-orbit coupling the
    # magnetization exactly and, with gx = gy, <Lz> (Lemma 1) to spectral accuracy
    shape, L = (24, 36, 36), 6.0
    psi = smooth_state_3d(shape, L, 41)
    params = (60.0, 2.0, -3.0, 0.6, 0.0, 1.0, 1.0, 1.7)
    tau, n = 5e-3, 12
    out = oracle.evolve(psi, L, params, 4, tau, n)
    o0 = oracle.observables(psi, L, params)
    o1 = oracle.observables(out, L, params, theta=params[3] * tau * n)
    assert abs(o1[0] - o0[0]) < 1e-13
    assert abs(o1[2] - o0[2]) < 1e-12
    assert abs(o1[3] - o0[3]) < 1e-9 and abs(o0[3]) > 0.05
    # with spin-orbit coupling and an anisotropic trap: mass only
    params2 = (60.0, 2.0, -3.0, 0.6, 0.8, 1.0, 1.2, 1.7)
    out2 = oracle.evolve(psi, L, params2, 4, tau, n)
    o2 = oracle.observables(out2, L, params2, theta=params2[3] * tau * n)
    assert abs(o2[0] - o0[0]) < 1e-13 and abs(o2[2] - o0[2]) > 1e-5


def test_ground_state_3d_evolves_by_its_energy_phase():
    # c = 0, gamma = 0, isotropic in the plane: the anisotropic ground state is an
    # eigenstate, psi(t) = exp(-i E t) psi(0), E = (gx + gy + gz)/2; the splitting
    # only adds its O(tau^4) error.  A missing gz^2 z^2 / 2 or nu_r^2 / 2 term moves
    # the state off the eigenstate.
    N, L = 32, 6.0
    shape = (N, N, N)
    X, Y, Z = mesh3(shape, (L, L, L))
    gz = 1.8
    g = (gz / np.pi ** 3) ** 0.25 * np.exp(-(X ** 2 + Y ** 2 + gz * Z ** 2) / 2)
    psi = np.zeros((5,) + shape, complex)
    psi[1] = g
    params = (0.0, 0.0, 0.0, 0.5, 0.0, 1.0, 1.0, gz)
    tau, n = 0.01, 20
    out = oracle.evolve(psi, L, params, 4, tau, n)
    E = (2.0 + gz) / 2
    # in the rotating frame component l also turns by exp(-i l Omega t) (the Omega f_z
    # term of the mapped linear operator, eq. linearEQ2); here l = 1
    want = np.exp(-1j * (E + 0.5) * tau * n) * psi
    rel = np.linalg.norm(out - want) / np.linalg.norm(psi)
    assert rel < 1e-7, rel
