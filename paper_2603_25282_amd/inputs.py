"""Seeded synthetic inputs: grids, parameters and initial wave functions.

This module holds no arithmetic of the method itself; it only builds the
configurations (grid, physics, scheme) and the initial states that both the HIP
path and the test oracle consume.  Every random draw uses numpy's PCG64
(`numpy.random.default_rng(seed)`), so a state is reproducible on any machine.

Conventions: a state is complex128 of shape (5, [nz,] ny, nx); component i holds
spin projection l = 2, 1, 0, -1, -2.  Parameters are the tuple
(c0, c1, c2, Omega, gamma, gamma_x, gamma_y, gamma_z).
"""
from dataclasses import dataclass, field
from typing import Tuple

import numpy as np


@dataclass(frozen=True)
class Config:
    name: str
    shape: Tuple[int, ...]          # spatial shape, (ny, nx) or (nz, ny, nx)
    L: float                        # domain [-L, L]^d
    params: Tuple[float, ...]       # (c0, c1, c2, Omega, gamma, gx, gy, gz)
    order: int                      # 2 (TS2) or 4 (TS4)
    tau: float
    steps: int
    seed: int
    init: str = "gauss_phase"       # initial-state recipe, see initial_state()
    extra: dict = field(default_factory=dict)

    @property
    def dim(self):
        return len(self.shape)

    @property
    def points(self):
        return int(np.prod(self.shape))

    def h(self):
        return tuple(2.0 * self.L / n for n in self.shape[::-1])


def axes(shape, L):
    """Grid coordinates x_j = -L + j h per axis, returned in (x, y[, z]) order."""
    return [(-L + (2.0 * L / n) * np.arange(n)) for n in shape[::-1]]


def mesh(shape, L):
    """Broadcastable coordinate arrays X, Y[, Z] with the state's spatial shape."""
    ax = axes(shape, L)
    if len(shape) == 2:
        Y, X = np.meshgrid(ax[1], ax[0], indexing="ij")
        return X, Y
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


def normalise(psi, shape, L):
    hd = np.prod([2.0 * L / n for n in shape])
    m = hd * np.sum(np.abs(psi) ** 2)
    return psi / np.sqrt(m)


def initial_state(cfg: Config):
    """Initial data for a configuration (complex128, shape (5, *cfg.shape))."""
    shape, L = cfg.shape, cfg.L
    rng = np.random.default_rng(cfg.seed)
    co = mesh(shape, L)
    if cfg.init == "gauss_phase":
        # Gaussian times an independent uniform random phase per point and component.
        r2 = sum(c * c for c in co[:2])
        if len(shape) == 3:
            r2 = r2 + co[2] ** 2
        g = np.exp(-r2 / 2.0)
        th = rng.uniform(0.0, 2.0 * np.pi, size=(5,) + shape)
        psi = g[None] * np.exp(1j * th)
    elif cfg.init == "gauss_noise":
        # Gaussian times (1 + eps*eta), eta complex white noise low-passed by
        # exp(-|nu|^2/8) in Fourier space and rescaled to unit RMS.
        eps = cfg.extra.get("eps", 1e-2)
        r2 = sum(c * c for c in co)
        g = np.exp(-r2 / 2.0)
        eta = rng.standard_normal((5,) + shape) + 1j * rng.standard_normal((5,) + shape)
        nus = [np.pi * np.fft.fftfreq(n, d=1.0 / n) / L for n in shape]
        k2 = sum(np.meshgrid(*[nu ** 2 for nu in nus], indexing="ij"))
        eta = np.fft.ifftn(np.fft.fftn(eta, axes=tuple(range(1, len(shape) + 1))) * np.exp(-k2 / 8.0)[None],
                           axes=tuple(range(1, len(shape) + 1)))
        eta = eta / np.sqrt(np.mean(np.abs(eta) ** 2, axis=tuple(range(1, len(shape) + 1)), keepdims=True))
        psi = g[None] * (1.0 + eps * eta)
    elif cfg.init == "gauss_phase_noise":
        # Anisotropic Gaussian exp(-(x^2 + y^2 + 4 z^2)/2) times exp(i sigma zeta),
        # zeta iid N(0, 1) per point and component.
        sigma = cfg.extra.get("sigma", 0.5)
        X, Y, Z = co
        g = np.exp(-(X ** 2 + Y ** 2 + 4.0 * Z ** 2) / 2.0)
        zeta = rng.standard_normal((5,) + shape)
        psi = g[None] * np.exp(1j * sigma * zeta)
    elif cfg.init == "ini1":
        # Example "Accuracy" initial data: psi_{+-2} = psi_{+-1} = phi, psi_0 = 2 phi,
        # phi = exp(-|x|^2/2) / (sqrt(8) pi^(d/4)); already of unit mass.
        r2 = sum(c * c for c in co)
        d = len(shape)
        phi = np.exp(-r2 / 2.0) / (np.sqrt(8.0) * np.pi ** (d / 4.0))
        psi = np.stack([phi, phi, 2.0 * phi, phi, phi]).astype(np.complex128)
        return psi
    elif cfg.init == "ex3":
        # Example "dynamical laws" initial data: psi_{+-2} = psi_{+-1} = phi,
        # psi_0 = 6 sqrt7 phi, phi = exp(-|x|^2/8) / (32 sqrt(pi)) (2D); unit mass.
        r2 = sum(c * c for c in co)
        phi = np.exp(-r2 / 8.0) / (32.0 * np.sqrt(np.pi))
        psi = np.stack([phi, phi, 6.0 * np.sqrt(7.0) * phi, phi, phi]).astype(np.complex128)
        return psi
    elif cfg.init in ("soc_i", "soc_ii"):
        # Example "SOC effects" initial data, phi = exp(-|x|^2/2) / (16 sqrt(pi)) (2D):
        # case i: psi_{+-2} = psi_{+-1} = phi, psi_0 = 6 sqrt7 phi;
        # case ii: psi_{+-2} = phi (x + i y), psi_{+-1} = phi, psi_0 = 6 sqrt7 phi (x + i y);
        # both of unit mass (the integral of r^2 exp(-r^2) is that of exp(-r^2), pi).
        X, Y = co[:2]
        phi = np.exp(-(X * X + Y * Y) / 2.0) / (16.0 * np.sqrt(np.pi))
        w = np.ones_like(X, dtype=np.complex128) if cfg.init == "soc_i" else (X + 1j * Y)
        psi = np.stack([phi * w, phi, 6.0 * np.sqrt(7.0) * phi * w, phi, phi * w]).astype(np.complex128)
        return psi
    else:
        raise ValueError(cfg.init)
    return normalise(psi.astype(np.complex128), shape, L)


# ---------------------------------------------------------------------------
# Named workloads.  Trap frequencies (gx, gy, gz); 2D configurations carry gz = 1.
# ---------------------------------------------------------------------------
C1 = Config("2d-64-ts2", (64, 64), 8.0, (100.0, -1.0, 5.0, 0.5, 0.5, 1.0, 1.0, 1.0),
            order=2, tau=1e-3, steps=100, seed=1, init="gauss_phase")
C2 = Config("2d-512-ts4", (512, 512), 16.0, (500.0, -5.0, 10.0, 0.9, 1.0, 1.0, 1.1, 1.0),
            order=4, tau=5e-4, steps=1000, seed=2, init="gauss_noise", extra={"eps": 1e-2})
C3 = Config("3d-128-ts4", (128, 128, 128), 8.0, (200.0, -2.0, 4.0, 0.7, 0.8, 1.0, 1.0, 4.0),
            order=4, tau=1e-3, steps=200, seed=3, init="gauss_phase_noise", extra={"sigma": 0.5})
C5 = Config("2d-256-ts4-adjoint", (256, 256), 12.0, (300.0, -3.0, 6.0, 0.8, 1.0, 1.0, 1.0, 1.0),
            order=4, tau=1e-3, steps=500, seed=5, init="gauss_phase", extra={"target_seed": 6, "K": 50})

# Example "Accuracy" (2D case) of the paper: [-12, 12]^2, t = 0.5.
ACC2D = Config("paper-acc-2d", (192, 192), 12.0, (100.0, -1.0, 1.0, 0.2, 0.3, 1.0, 1.0, 1.0),
               order=2, tau=1.0 / 80.0, steps=40, seed=0, init="ini1")
# Example "dynamical laws" (2D), case i: c = (120, 1, 1), Omega = 0.2, isotropic trap,
# no SOC, tau = 1e-3, on the paper's domain [-24, 24]^2 at h = 1/16 (768^2).  Cases
# ii (gamma = 0.9) and iii (gx = 1.3) via with_().
EX3 = Config("paper-ex3-case1", (768, 768), 24.0, (120.0, 1.0, 1.0, 0.2, 0.0, 1.0, 1.0, 1.0),
             order=4, tau=1e-3, steps=12000, seed=0, init="ex3")
# Example "Accuracy" (3D case): [-8, 8]^3, t = 0.3.
ACC3D = Config("paper-acc-3d", (64, 64, 64), 8.0, (10.0, -1.0, 1.0, 0.2, 0.1, 1.0, 1.0, 1.0),
               order=2, tau=1.0 / 40.0, steps=12, seed=0, init="ini1")

# Example "SOC effects" (2D): c = (243, 12.1, -13), Omega = 0.2, [-24, 24]^2 at
# h = 1/16 (768^2), TS2, tau = 1e-3 to t = 1; gamma varies (case i: 0, 0.7, 2; case
# ii: 0, 0.3, 1.2).  The example states no trap: the harmonic trap with
# gx = gy = 1 is taken.
SOC_I = Config("paper-soc-case1", (768, 768), 24.0, (243.0, 12.1, -13.0, 0.2, 0.7, 1.0, 1.0, 1.0),
               order=2, tau=1e-3, steps=1000, seed=0, init="soc_i")
SOC_II = Config("paper-soc-case2", (768, 768), 24.0, (243.0, 12.1, -13.0, 0.2, 0.3, 1.0, 1.0, 1.0),
                order=2, tau=1e-3, steps=1000, seed=0, init="soc_ii")

CONFIGS = {c.name: c for c in (C1, C2, C3, C5, ACC2D, ACC3D)}


def _c3_256():
    # the 3D workload above at 256^3 on the same domain (h = 1/16): a 640 MiB
    # complex64 state, larger than the 256 MB Infinity Cache, so every pass streams
    # from and to HBM
    return Config("3d-256-ts4-hbm", (256, 256, 256), C3.L, C3.params, order=C3.order, tau=C3.tau,
                  steps=C3.steps, seed=C3.seed, init=C3.init, extra=dict(C3.extra))


C3_256 = _c3_256()


def with_(cfg: Config, **kw):
    d = dict(cfg.__dict__)
    d.update(kw)
    return Config(**d)


def ensemble_instances(seed=4, n128=32, n256=48, n384=16, L=12.0, c0=100.0, order=2, tau=1e-3, steps=500):
    """Uneven-grid parameter ensemble: n128 x 128^2, n256 x 256^2, n384 x 384^2 on
    [-L, L]^2, isotropic trap; per instance Omega ~ U[0.3, 0.95], gamma ~ U[0, 2],
    c1 ~ U[-5, 5], c2 ~ U[0, 10] drawn in instance order; initial data of the
    Gaussian-random-phase form with seed 1000 + i."""
    rng = np.random.default_rng(seed)
    sizes = [128] * n128 + [256] * n256 + [384] * n384
    out = []
    for i, n in enumerate(sizes):
        Om = rng.uniform(0.3, 0.95)
        ga = rng.uniform(0.0, 2.0)
        c1 = rng.uniform(-5.0, 5.0)
        c2 = rng.uniform(0.0, 10.0)
        out.append(Config(f"ens-{i}-{n}", (n, n), L, (c0, c1, c2, Om, ga, 1.0, 1.0, 1.0), order=order,
                          tau=tau, steps=steps, seed=1000 + i, init="gauss_phase"))
    return out
