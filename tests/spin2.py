"""Spin-2 matrices and operators written out from the paper's definitions (Sec. 1),
used by the tests to build independent checks (matrix exponentials, ODE right-hand
sides).  Component order l = 2, 1, 0, -1, -2."""
import numpy as np

H6 = np.sqrt(6.0) / 2.0

FX = np.zeros((5, 5), complex)
FY = np.zeros((5, 5), complex)
for _i, _w in enumerate([1.0, H6, H6, 1.0]):
    FX[_i, _i + 1] = FX[_i + 1, _i] = _w
    FY[_i, _i + 1] = -1j * _w
    FY[_i + 1, _i] = 1j * _w
FZ = np.diag([2.0, 1.0, 0.0, -1.0, -2.0]).astype(complex)
# A_ij = (-1)^(i-1) delta_{i+j,6} / sqrt5 (1-based)
AS = np.zeros((5, 5))
for _i in range(5):
    AS[_i, 4 - _i] = (-1.0) ** _i / np.sqrt(5.0)


def Qmat(Omega, gamma, nu_p, nu_q):
    """Q of the Fourier-space linear system: diagonal -Omega(2,1,0,-1,-2),
    super-diagonal gamma a (1, sqrt6/2, sqrt6/2, 1), a = -nu_q - i nu_p."""
    a = -nu_q - 1j * nu_p
    M = np.diag([-2 * Omega, -Omega, 0.0, Omega, 2 * Omega]).astype(complex)
    for i, w in enumerate([1.0, H6, H6, 1.0]):
        M[i, i + 1] = gamma * a * w
        M[i + 1, i] = gamma * np.conj(a) * w
    return M


def Smat(nu_p, nu_q):
    """Symbol of the SOC operator matrix S: L+- = i d_y +- d_x -> -nu_q +- i nu_p."""
    Lp = -nu_q + 1j * nu_p
    Lm = -nu_q - 1j * nu_p
    S = np.zeros((5, 5), complex)
    for i, w in enumerate([1.0, H6, H6, 1.0]):
        S[i, i + 1] = w * Lm
        S[i + 1, i] = w * Lp
    return S


def densities(psi):
    rho = np.vdot(psi, psi).real
    F = np.array([np.vdot(psi, f @ psi).real for f in (FX, FY, FZ)])
    A00 = psi @ AS @ psi
    return rho, F, A00


def nl_rhs(psi, params, V):
    """Right-hand side of the nonlinear subproblem:
    -i{[(V + c0 rho) + c1 F.f] psi + c2 A00 A conj(psi)}."""
    c0, c1, c2 = params[:3]
    rho, F, A00 = densities(psi)
    Ff = F[0] * FX + F[1] * FY + F[2] * FZ
    return -1j * ((V + c0 * rho) * psi + c1 * Ff @ psi + c2 * A00 * (AS @ np.conj(psi)))


def soc_width_term(psi, L, params):
    """G(gamma, Psi), the spin-orbit term of Lemma 2's width law (Sec. 2), written out
    from its definition on a lab-frame 2D state (5, ny, nx) on [-L, L]^2:
    2 gamma Re h^2 sum [Omega (i y - x) F_+ + gamma (2 rho + 3|psi_1|^2 + 4|psi_0|^2 +
    3|psi_-1|^2 + sum_m m conj(psi_m) L_z psi_m)], F_+ = 2 (conj(psi_2) psi_1 +
    conj(psi_-1) psi_-2) + sqrt6 (conj(psi_1) psi_0 + conj(psi_0) psi_-1),
    L_z = -i (x d_y - y d_x) with spectral derivatives."""
    ny, nx = psi.shape[1:]
    h = 2.0 * L / nx
    x = -L + h * np.arange(nx)
    y = -L + (2.0 * L / ny) * np.arange(ny)
    X, Y = np.meshgrid(x, y)
    kx = np.pi * np.fft.fftfreq(nx, d=1.0 / nx) / L
    ky = np.pi * np.fft.fftfreq(ny, d=1.0 / ny) / L
    dx = np.fft.ifft(1j * kx[None, None, :] * np.fft.fft(psi, axis=-1), axis=-1)
    dy = np.fft.ifft(1j * ky[None, :, None] * np.fft.fft(psi, axis=-2), axis=-2)
    lz = -1j * (X[None] * dy - Y[None] * dx)
    p = psi
    fp = 2 * (np.conj(p[0]) * p[1] + np.conj(p[3]) * p[4]) + np.sqrt(6.0) * (np.conj(p[1]) * p[2] + np.conj(p[2]) * p[3])
    n = np.abs(p) ** 2
    rho = n.sum(axis=0)
    m = np.array([2.0, 1.0, 0.0, -1.0, -2.0])[:, None, None]
    Om, gam = params[3], params[4]
    dens = Om * (1j * Y - X) * fp + gam * (2 * rho + 3 * n[1] + 4 * n[2] + 3 * n[3] +
                                          np.sum(m * np.conj(p) * lz, axis=0))
    return 2.0 * gam * np.real(h * (2.0 * L / ny) * np.sum(dens))
