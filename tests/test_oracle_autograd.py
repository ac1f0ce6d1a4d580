"""The differentiable transcription of the oracle (torch, binary64, CPU), pinned
to the C oracle: identical forward states, and reverse-mode gradients of the
mean hot-wall Nusselt number equal to central finite differences of the C
oracle's own forward map (a different program: the C oracle shares no code
with the torch transcription).  These gradients are what the GPU adjoint is
compared with."""
import numpy as np
import pytest

import oracle as O
from oracle import autograd as AG
from paper_1608_04118_amd import inputs as I


def _case(kind, seed=1):
    nx, ny = 12, 10
    r = np.random.default_rng(seed)
    base = dict(nx=nx, ny=ny, Ma=0.0, nu_f=0.05, Ra=3e4, dT=1.0, L=12.0, T0=0.4, body_force=(2e-5, -1e-5),
                Hv=80.0, gamma_sf=4.0, sigma=1.7, phi=0.55, Qf=1e-5, Qs=-2e-5)
    phi = np.clip(0.55 + 0.05 * r.standard_normal((ny, nx)), 0.4, 0.7)
    Hv = 80.0 * (1 + 0.3 * r.uniform(-1, 1, (ny, nx)))
    Tf0 = Ts0 = None
    if kind == "cavity":      # Dirichlet left/right, adiabatic bottom/top, Ergun F_phi
        p = I.complete(**base, wall_thermal=(0, 0, 1, 1), T_wall=(1.0, 0, 0, 0), F_phi=-1.0)
    elif kind == "periodic":  # periodic x, heated from below, fixed F_phi
        p = I.complete(**base, periodic_x=1, wall_thermal=(1, 1, 0, 0), T_wall=(0, 0, 1.0, 0), F_phi=0.1)
    elif kind == "init":      # initial temperature fields, loss on the cold wall
        p = I.complete(**base, wall_thermal=(0, 0, 1, 1), T_wall=(1.0, 0, 0, 0), F_phi=-1.0, nu_wall=1)
        Tf0 = 0.4 + 0.3 * r.uniform(size=(ny, nx))
        Ts0 = 0.4 + 0.3 * r.uniform(size=(ny, nx))
    elif kind == "correction":  # correction term of Sec. 3.2, adiabatic walls included
        p = I.complete(**base, wall_thermal=(1, 0, 0, 1), T_wall=(0, 0, 1.0, 0), F_phi=-1.0,
                       thermal_correction=1)
    else:                     # adiabatic left wall next to the Dirichlet loss wall
        p = I.complete(**base, wall_thermal=(1, 0, 0, 1), T_wall=(0, 0, 1.0, 0), F_phi=-1.0)
    return p, phi, Hv, Tf0, Ts0


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("kind", ["cavity", "periodic", "init", "adiabatic", "correction"])
def test_forward_equals_c_oracle(kind):
    p, phi, Hv, Tf0, Ts0 = _case(kind)
    for steps in (0, 1, 30):
        o = O.Oracle(p, phi=phi, Hv=Hv, Tf0=Tf0, Ts0=Ts0).step(steps)
        t = AG.DiffLattice(p, phi, Hv, Tf0, Ts0).step(steps)
        a = {k: v.detach().numpy() for k, v in t.macros.items()}
        b = o.macros()
        du = np.hypot(a["ux"] - b["ux"], a["uy"] - b["uy"]).max() / max(np.hypot(b["ux"], b["uy"]).max(), 1e-300)
        assert du <= 1e-12, (steps, du)
        for k in ("rho", "Tf", "Ts"):
            assert _rel(a[k], b[k]) <= 1e-13, (steps, k)
        assert abs(float(t.nusselt().detach()) - o.nusselt()[0]) <= 1e-13 * abs(o.nusselt()[0])


def _fd(p, field, phi, Hv, cell, h, Tf0=None, Ts0=None, t0=0, pops=None, steps=25):
    vals = []
    for s in (1, -1):
        a = {"phi": phi.copy(), "Hv": Hv.copy()}
        a[field][cell] += s * h
        o = O.Oracle(p, phi=a["phi"], Hv=a["Hv"], Tf0=Tf0, Ts0=Ts0)
        if pops is not None:
            o.set_populations(*pops)
        vals.append(o.step(steps).nusselt()[0])
    return (vals[0] - vals[1]) / (2 * h)


CELLS = [(5, 6), (1, 1), (0, 0), (0, 5), (5, 0), (9, 11), (2, 2), (8, 3), (1, 10), (9, 4)]


@pytest.mark.parametrize("kind", ["cavity", "periodic", "init", "adiabatic", "correction"])
def test_gradients_equal_central_differences(kind):
    """Central differences with a relative step of 3e-4 have a truncation
    error near 1e-8 of the gradient scale and a rounding error below that."""
    p, phi, Hv, Tf0, Ts0 = _case(kind)
    loss, gp, gh = AG.gradients(p, 25, phi, Hv, Tf0, Ts0)
    assert abs(loss - O.Oracle(p, phi=phi, Hv=Hv, Tf0=Tf0, Ts0=Ts0).step(25).nusselt()[0]) <= 1e-13 * abs(loss)
    assert np.abs(gp).max() > 0 and np.abs(gh).max() > 0
    for cell in CELLS:
        for field, g, scale in (("phi", gp, phi), ("Hv", gh, Hv)):
            fd = _fd(p, field, phi, Hv, cell, 3e-4 * scale[cell], Tf0, Ts0)
            assert abs(g[cell] - fd) <= 1e-6 * np.abs(g).max(), (field, cell, g[cell], fd)


def test_gradients_from_a_given_state():
    """With t0 > 0 the state reached at t0 is an input: the gradient covers
    only the steps after it (checked by restarting the C oracle from that
    state with the perturbed coefficients)."""
    p, phi, Hv, _, _ = _case("cavity")
    t0, n = 15, 20
    loss, gp, gh = AG.gradients(p, n, phi, Hv, t0=t0)
    pops = O.Oracle(p, phi=phi, Hv=Hv).step(t0).populations()
    for cell in [(5, 6), (1, 1), (0, 5), (9, 11)]:
        for field, g, scale in (("phi", gp, phi), ("Hv", gh, Hv)):
            fd = _fd(p, field, phi, Hv, cell, 3e-4 * scale[cell], pops=pops, steps=n)
            assert abs(g[cell] - fd) <= 1e-6 * np.abs(g).max(), (field, cell, g[cell], fd)
