"""Seeded synthetic inputs for the LTNE lattice Boltzmann step.

This module holds parameter sets and seeded random fields only: none of the
method's arithmetic.  Both the GPU path (binding, benchmark) and the FP64
oracle (tests) take their inputs from here, so the two see identical inputs.

A parameter set is a plain dict.  Its keys are the physical inputs of the
problem statement of the paper (Sec. 2 groups, Sec. 4 setup) plus the lattice
bookkeeping the C structures need; ``complete`` fills every key so neither
side relies on a default of its own.

Workloads (the paper uses no public dataset; every workload is synthetic):

* ``cavity_small``   -- 64 x 64 side-heated porous cavity, FP64.
* ``cavity_large``   -- 1024 x 1024 side-heated porous cavity, FP32.
* ``channel``        -- 1024 x 256 Brinkman-Forchheimer channel, FP32.
* ``throughput``     -- 8192 x 8192 periodic-x / walled-y layer heated from
                        below, seeded porosity and temperature noise.
* ``batch``          -- 256 cavities of uneven size and parameters.
* ``adjoint_cavity`` -- 512 x 512 cavity with seeded porosity and interphase
                        coefficient fields.
* ``paper_cavity``   -- the cavity of the paper's own runs (Sec. 4), h_v from
                        the correlation of Eq. 52.
"""
from __future__ import annotations

import math

import numpy as np

FP64, FP32, FP16S, FP32SR = 0, 1, 2, 3
DIRICHLET, ADIABATIC = 0, 1

# Free relaxation rates and the D2Q5 weight parameter of the paper's cavity
# runs (Sec. 4).
PAPER_RATES = dict(varpi=0.4, s_e=1.1, s_eps=1.1, s_q=1.2,
                   zeta_e=1.1, zeta_nu=1.1, eta_e=1.1, eta_nu=1.1)

_BASE = dict(
    nx=64, ny=64, precision=FP64, periodic_x=0, periodic_y=0,
    wall_thermal=(DIRICHLET, DIRICHLET, ADIABATIC, ADIABATIC), nu_wall=-1,
    T_wall=(1.0, 0.0, 0.0, 0.0), T0=0.0, T_init_f=0.0, T_init_s=0.0,
    L=0.0, dT=0.0,
    phi=0.6, Da=1e-2, F_phi=-1.0,
    Ra=1e4, Pr=1.0, Je=1.0,
    gamma_sf=1.0, sigma=1.0, Hv=10.0,
    Qf=0.0, Qs=0.0,
    Ma=0.1, nu_f=0.0,
    body_force=(0.0, 0.0),
    rho0=1.0,
    T_ref=float("nan"), fp16_scale_f=0.0, fp16_scale_g=0.0,
    thermal_correction=0, pore_size=0.0, diag_every=0,
    **PAPER_RATES,
)


def complete(**kw) -> dict:
    """A full parameter dict: the paper's cavity setup overridden by ``kw``."""
    unknown = set(kw) - set(_BASE)
    if unknown:
        raise KeyError("unknown parameters: %s" % ", ".join(sorted(unknown)))
    p = dict(_BASE)
    p.update(kw)
    p["wall_thermal"] = tuple(int(v) for v in p["wall_thermal"])
    p["T_wall"] = tuple(float(v) for v in p["T_wall"])
    p["body_force"] = tuple(float(v) for v in p["body_force"])
    return p


def smoothed_noise(seed: int, ny: int, nx: int, sigma: float = 16.0) -> np.ndarray:
    """Standard-normal noise smoothed by a Gaussian of ``sigma`` cells on the
    torus (FFT), then standardised to zero mean and unit variance."""
    z = np.random.default_rng(seed).standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.rfftfreq(nx)[None, :]
    kern = np.exp(-2.0 * (math.pi * sigma) ** 2 * (kx * kx + ky * ky))
    s = np.fft.irfft2(np.fft.rfft2(z) * kern, s=(ny, nx))
    s -= s.mean()
    sd = s.std()
    return s / sd if sd > 0 else s


def cavity_small(**kw) -> dict:
    """64 x 64 nodes, FP64: phi = 0.6, Da = 1e-2, Ra = 1e4, H_v = 10, left wall
    T = 1, right wall T = 0, adiabatic top and bottom, fluid at rest."""
    base = dict(nx=64, ny=64, precision=FP64, phi=0.6, Da=1e-2, Ra=1e4, Pr=1.0,
                gamma_sf=1.0, sigma=1.0, Hv=10.0, T_wall=(1.0, 0.0, 0.0, 0.0),
                T0=0.0, T_init_f=0.0, T_init_s=0.0)
    base.update(kw)
    return complete(**base)


def cavity_large(**kw) -> dict:
    """1024 x 1024 nodes, FP32 with shifted populations: Ra = 1e6, Da = 1e-4,
    phi = 0.4, conductivity ratio 10, H_v = 100."""
    base = dict(nx=1024, ny=1024, precision=FP32, phi=0.4, Da=1e-4, Ra=1e6, Pr=1.0,
                gamma_sf=10.0, sigma=1.0, Hv=100.0, T_wall=(1.0, 0.0, 0.0, 0.0),
                T0=0.0, T_init_f=0.0, T_init_s=0.0)
    base.update(kw)
    return complete(**base)


def channel(nx=1024, ny=256, Da=1e-4, Re=10.0, axis="x", **kw) -> dict:
    """Brinkman-Forchheimer channel: periodic x, no-slip walls at y = 0 and
    y = ny - 1, no buoyancy, nu_f = 0.1, driven by a body acceleration G_b
    along x.  G_b is set from the Brinkman (Forchheimer-free) centre-line
    velocity u_max = (G_b K / nu_f)(1 - 1/cosh(r L / 2)),
    r = sqrt(phi nu_f / (nu_e K)), so that Re = u_max L / nu_f is close to
    ``Re`` (the Forchheimer drag lowers it slightly).  ``axis="y"`` gives
    the same channel turned by a quarter: flow along y between walls at
    x = 0 and x = nx - 1 (nx, ny then name the wall-normal and the periodic
    extent the other way round)."""
    phi, nu_f, Je = kw.pop("phi", 0.4), kw.pop("nu_f", 0.1), kw.pop("Je", 1.0)
    L = (ny if axis == "x" else nx) - 1
    K = Da * L * L
    r = math.sqrt(phi * nu_f / (Je * nu_f * K))
    u_max = Re * nu_f / L
    Gb = u_max * nu_f / K / (1.0 - 1.0 / math.cosh(0.5 * r * L))
    base = dict(nx=nx, ny=ny, precision=FP32, periodic_x=1, periodic_y=0,
                wall_thermal=(DIRICHLET, DIRICHLET, DIRICHLET, DIRICHLET),
                T_wall=(0.0, 0.0, 0.0, 0.0), T0=0.0, T_init_f=0.0, T_init_s=0.0,
                phi=phi, Da=Da, Ra=0.0, nu_f=nu_f, Ma=0.0, Je=Je, Pr=1.0,
                gamma_sf=10.0, Hv=100.0, body_force=(Gb, 0.0), nu_wall=2)
    if axis == "y":
        base.update(periodic_x=0, periodic_y=1, body_force=(0.0, Gb), nu_wall=0)
    base.update(kw)
    return complete(**base)


def throughput(n: int = 8192, precision: int = FP32, **kw):
    """Periodic-x / walled-y layer of n x n nodes heated from below (bottom
    T = 1, top T = 0), Ra = 1e5, Da = 1e-3, H_v = 10.  Porosity is smoothed
    Gaussian noise (sigma = 16 cells, seed 3) mapped to 0.65 + 0.1 z and
    clipped to [0.4, 0.9]; initial T_f and T_s are 0.5 plus independent
    uniform noise in [-0.05, 0.05] (seeds 4 and 5).

    Returns (params, phi, Tf0, Ts0)."""
    ny = kw.pop("ny", n)
    base = dict(nx=n, ny=ny, precision=precision, periodic_x=1, periodic_y=0,
                wall_thermal=(ADIABATIC, ADIABATIC, DIRICHLET, DIRICHLET),
                T_wall=(0.0, 0.0, 1.0, 0.0), T0=0.5, T_init_f=0.5, T_init_s=0.5,
                phi=0.65, Da=1e-3, Ra=1e5, Pr=1.0, gamma_sf=1.0, sigma=1.0, Hv=10.0,
                nu_wall=2)
    base.update(kw)
    p = complete(**base)
    phi = np.clip(0.65 + 0.1 * smoothed_noise(3, ny, n), 0.4, 0.9)
    Tf0 = 0.5 + np.random.default_rng(4).uniform(-0.05, 0.05, (ny, n))
    Ts0 = 0.5 + np.random.default_rng(5).uniform(-0.05, 0.05, (ny, n))
    return p, phi, Tf0, Ts0


BATCH_SIDES = tuple(range(64, 513, 32))


def batch(count: int = 256, seed: int = 42, precision: int = FP32):
    """``count`` independent cavities (physics as ``cavity_small``), drawn
    with ``default_rng(seed)`` in this order, ``count`` values each: side in
    {64, 96, ..., 512}; log10 Ra ~ U[3, 6]; log10 Da ~ U[-4, -2];
    phi ~ U[0.4, 0.9]; log10 gamma_sf ~ U[-1, 2]; log10 H_v ~ U[0, 3]."""
    rng = np.random.default_rng(seed)
    sides = rng.choice(np.array(BATCH_SIDES), size=count)
    lra = rng.uniform(3.0, 6.0, count)
    lda = rng.uniform(-4.0, -2.0, count)
    phis = rng.uniform(0.4, 0.9, count)
    lgs = rng.uniform(-1.0, 2.0, count)
    lhv = rng.uniform(0.0, 3.0, count)
    out = []
    for k in range(count):
        n = int(sides[k])
        out.append(cavity_small(nx=n, ny=n, precision=precision, Ra=float(10 ** lra[k]),
                                Da=float(10 ** lda[k]), phi=float(phis[k]),
                                gamma_sf=float(10 ** lgs[k]), Hv=float(10 ** lhv[k])))
    return out


def adjoint_cavity(n: int = 512, precision: int = FP32, **kw):
    """n x n cavity (walls as ``cavity_small``), Ra = 1e5, Da = 1e-3, porosity
    clip(0.65 + 0.1 z_a, 0.4, 0.9) (seed 6) and interphase coefficient
    10 (1 + 0.5 clip(z_b, -1, 1)) (seed 7), z smoothed noise with sigma = 16.

    Returns (params, phi, Hv)."""
    base = dict(nx=n, ny=n, precision=precision, Ra=1e5, Da=1e-3, phi=0.65, Hv=10.0)
    base.update(kw)
    p = cavity_small(**base)
    phi = np.clip(0.65 + 0.1 * smoothed_noise(6, n, n), 0.4, 0.9)
    Hv = 10.0 * (1.0 + 0.5 * np.clip(smoothed_noise(7, n, n), -1.0, 1.0))
    return p, phi, Hv


def paper_cavity(n: int = 128, Ra: float = 1e6, pore_size: float = 0.0135, **kw) -> dict:
    """The cavity of the paper's own runs (Sec. 4): n x n nodes, hot left wall
    T_h = 11, cold right wall T_c = T_0 = 1 (dT = 10), adiabatic top and
    bottom, fluid and solid initially at T_0; phi = 0.8, Da = 1e-4,
    F_phi = 0.068, Pr = 1, J_e = 1, sigma = 1, gamma_sf = 1000, and h_v from
    the correlation of Eq. 52 with D_p = 0.0135 L (pore_size = 0: no
    interphase exchange, the H_p = 0 case).  FP64 unless overridden."""
    base = dict(nx=n, ny=n, precision=FP64, T_wall=(11.0, 1.0, 0.0, 0.0), T0=1.0, T_init_f=1.0,
                T_init_s=1.0, wall_thermal=(DIRICHLET, DIRICHLET, ADIABATIC, ADIABATIC), phi=0.8,
                Da=1e-4, F_phi=0.068, Ra=Ra, Pr=1.0, Je=1.0, gamma_sf=1000.0, sigma=1.0, Hv=0.0,
                pore_size=pore_size)
    base.update(kw)
    return complete(**base)


def fd_cells(n: int = 512, count: int = 32, seed: int = 8):
    """Interior cells (y, x) for the finite-difference gradient check."""
    rng = np.random.default_rng(seed)
    ys = rng.integers(1, n - 1, count)
    xs = rng.integers(1, n - 1, count)
    return list(zip(ys.tolist(), xs.tolist()))
