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
