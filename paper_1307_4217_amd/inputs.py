"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module holds the problem *inputs* only: grids, quadrature nodes and the
seeded random atmosphere.  It contains none of the method's arithmetic (no
interpolation, no formal solution, no radiation-field tensors, no statistical
equilibrium), so both the HIP path and the CPU oracle can be fed from it.

Shapes follow the benchmark model of the paper (Appendix A: horizontally
periodic box of L_x = L_y = 2000 km, Gaussian inclinations times trapezoidal
azimuths, ~100 frequencies per line).  The physical model atmosphere of that
appendix (FAL-C, five-level Ca II) is not available, so a synthetic two-level
atmosphere with the same geometry stands in for it:

* line-centre opacity  kappa = kappa0 * exp(-z/H) * f(x, y), H = 150 km,
  kappa0 * H = 1e3, f = exp(0.3 g - 0.045) with g ~ N(0,1) per column
  (lognormal lateral noise of unit mean on the line-centre optical depth);
* dichroism / anomalous dispersion eta_Q,U,V and rho_Q,U,V = kappa * U(-0.05, 0.05);
* emissivity multipoles eps^K_Q = kappa * S^K_Q with S^0_0 ~ U(0.5, 1.5) and
  the K=2 components (S^2_0 real; Re/Im of S^2_1, S^2_2) ~ U(-0.05, 0.05);
* magnetic field |B| ~ U(0, 100) G, direction uniform on the sphere; the Hanle
  parameter H_u = 8.794e6 g_u |B| / A_ul with g_u = 1, A_ul = 1e8 s^-1.

All arrays are stored x-fastest: index p = (k * ny + j) * nx + i.
"""
from __future__ import annotations

import dataclasses

import numpy as np

KM_HORIZONTAL = 2000.0      # L_x = L_y (km), Appendix A of the paper
Z_TOP = 2000.0              # vertical extent of the synthetic box (km)
SCALE_HEIGHT = 150.0        # opacity scale height H (km)
TAU_BASE = 1.0e3            # kappa0 * H: line-centre vertical optical depth scale
HANLE_PER_GAUSS = 8.794e6 / 1.0e8   # H_u per gauss for g_u = 1, A_ul = 1e8 s^-1
EPS_COLL = 1.0e-2           # collisional destruction probability
PLANCK = 1.0                # isothermal Planck function (bottom boundary too)


@dataclasses.dataclass(frozen=True)
class Config:
    """One problem size.  `nmu` is the number of inclinations per hemisphere."""
    name: str
    nx: int
    ny: int
    nz: int
    nmu: int
    nchi: int
    nfreq: int
    magnetic: bool

    @property
    def npoints(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nrays(self) -> int:
        return 2 * self.nmu * self.nchi

    @property
    def updates(self) -> int:
        """Point x ray x frequency updates of one formal solution."""
        return self.npoints * self.nrays * self.nfreq


CONFIGS = {
    # small FP64 instance the oracle finishes in seconds
    "C1": Config("C1", 16, 16, 32, 5, 8, 21, False),
    # FP64 Jacobi-iteration instance with Hanle rotation
    "C2": Config("C2", 128, 128, 96, 5, 16, 41, True),
    # precision / throughput instance (FP32 sweep, FP64 J and SEE)
    "C3": Config("C3", 256, 256, 128, 5, 16, 101, True),
    # differentiation instance
    "C4": Config("C4", 64, 64, 64, 5, 8, 41, False),
    # large combined instance (40.6 M points)
    "C5": Config("C5", 504, 504, 160, 5, 16, 101, True),
}


@dataclasses.dataclass
class Quadrature:
    mu: np.ndarray      # (nmu,) inclination cosines of one hemisphere, in (0, 1]
    wmu: np.ndarray     # (nmu,) weights, sum 1
    nchi: int           # azimuths per full circle (trapezoid, nodes at (m+1/2) 2 pi / nchi)
    x: np.ndarray       # (nfreq,) reduced frequency (Doppler units)
    phi: np.ndarray     # (nfreq,) profile relative to line centre, exp(-x^2)
    wfreq: np.ndarray   # (nfreq,) trapezoid weights in x


def gauss_legendre_hemisphere(nmu: int):
    """Gauss-Legendre nodes on (0, 1) with weights summing to one."""
    t, w = np.polynomial.legendre.leggauss(nmu)
    return 0.5 * (t + 1.0), 0.5 * w


def frequency_grid(nfreq: int, xmax: float = 4.0):
    """Uniform reduced frequencies on [-xmax, xmax] with trapezoid weights."""
    if nfreq == 1:
        x = np.zeros(1)
        w = np.ones(1)
    else:
        x = np.linspace(-xmax, xmax, nfreq)
        dx = x[1] - x[0]
        w = np.full(nfreq, dx)
        w[0] = w[-1] = 0.5 * dx
    return x, np.exp(-x * x), w


def make_quadrature(cfg: Config) -> Quadrature:
    mu, wmu = gauss_legendre_hemisphere(cfg.nmu)
    x, phi, w = frequency_grid(cfg.nfreq)
    return Quadrature(mu=mu, wmu=wmu, nchi=cfg.nchi, x=x, phi=phi, wfreq=w)


@dataclasses.dataclass
class Atmosphere:
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    z: np.ndarray          # (nz,)
    kappa: np.ndarray      # (N,)     line-centre eta_I
    propmat: np.ndarray    # (6, N)   eta_Q, eta_U, eta_V, rho_Q, rho_U, rho_V
    emis: np.ndarray       # (6, N)   eps00, eps20, Re eps21, Im eps21, Re eps22, Im eps22
    source: np.ndarray     # (6, N)   S^K_Q in the same component order
    hanle: np.ndarray | None   # (N,)   H_u, or None for no field
    bhat: np.ndarray | None    # (3, N) unit field direction, or None
    i_bottom: float = PLANCK
    eps_c: float = EPS_COLL
    delta2: float = 0.0
    w2: float = 1.0
    planck: float = PLANCK

    @property
    def npoints(self) -> int:
        return self.nx * self.ny * self.nz


def make_atmosphere(cfg: Config, seed: int = 0, dtype=np.float64,
                    magnetic: bool | None = None) -> Atmosphere:
    """Seeded synthetic two-level atmosphere with the geometry of `cfg`."""
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    n = nx * ny * nz
    z = np.linspace(0.0, Z_TOP, nz)
    kappa0 = TAU_BASE / SCALE_HEIGHT
    g = np.random.default_rng(1 + 100 * seed).standard_normal((ny, nx))
    lateral = np.exp(0.3 * g - 0.045)
    kappa = (kappa0 * np.exp(-z / SCALE_HEIGHT))[:, None, None] * lateral[None, :, :]
    kappa = kappa.reshape(n)
    rng2 = np.random.default_rng(2 + 100 * seed)
    propmat = kappa[None, :] * rng2.uniform(-0.05, 0.05, size=(6, n))
    rng3 = np.random.default_rng(3 + 100 * seed)
    source = np.empty((6, n))
    source[0] = rng3.uniform(0.5, 1.5, size=n)
    source[1:] = rng3.uniform(-0.05, 0.05, size=(5, n))
    emis = kappa[None, :] * source
    hanle = bhat = None
    if cfg.magnetic if magnetic is None else magnetic:
        rng4 = np.random.default_rng(4 + 100 * seed)
        bmag = rng4.uniform(0.0, 100.0, size=n)
        v = rng4.standard_normal((3, n))
        bhat = v / np.linalg.norm(v, axis=0, keepdims=True)
        hanle = HANLE_PER_GAUSS * bmag
    return Atmosphere(nx=nx, ny=ny, nz=nz, lx=KM_HORIZONTAL, ly=KM_HORIZONTAL, z=z,
                      kappa=kappa.astype(dtype), propmat=propmat.astype(dtype),
                      emis=emis.astype(dtype), source=source,
                      hanle=hanle, bhat=bhat)


def perturbed_target_atmosphere(atm: Atmosphere, seed: int = 5) -> Atmosphere:
    """Seeded perturbation kappa*exp(0.1 n), eps*(1 + 0.05 n) used to make a loss target."""
    rng = np.random.default_rng(seed)
    n = atm.npoints
    k = atm.kappa.astype(np.float64) * np.exp(0.1 * rng.standard_normal(n))
    e = atm.emis.astype(np.float64) * (1.0 + 0.05 * rng.standard_normal((6, n)))
    return dataclasses.replace(atm, kappa=k.astype(atm.kappa.dtype),
                               emis=e.astype(atm.emis.dtype))


def ray_count(q: Quadrature) -> int:
    return 2 * len(q.mu) * q.nchi


def sample_indices(total: int, count: int, seed: int) -> np.ndarray:
    """Distinct sorted random indices in [0, total)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(total, size=min(count, total), replace=False))


def describe(cfg: Config) -> str:
    return (f"{cfg.nx}x{cfg.ny}x{cfg.nz} grid, {cfg.nrays} rays "
            f"({cfg.nmu} GL x {cfg.nchi} azimuths per hemisphere), {cfg.nfreq} freqs")


__all__ = ["Config", "CONFIGS", "Quadrature", "Atmosphere", "make_quadrature",
           "make_atmosphere", "perturbed_target_atmosphere", "gauss_legendre_hemisphere",
           "frequency_grid", "sample_indices", "describe", "ray_count"]
