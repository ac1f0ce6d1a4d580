"""Pins of the oracle's steady-state residual (CPU).

The paper gives no residual; the reading used by both sides is
r = max over u, T_f, T_s of sum_x |a(x) - a_prev(x)| / sum_x |a(x)|, where
a_prev are the macros at the end of the previous step call (velocity as
|u_x| + |u_y| per node).  The pins fix it on states whose fields are known
without the oracle:

- a uniform periodic lattice with no buoyancy, a body acceleration G and a
  gap T_s - T_f: the velocity follows the linear recurrence of Eqs. 19-22
  with F_phi = 0 (j grows by rho F per step, F = phi G - phi nu_f u / K,
  u = (j / rho + phi G / 2) / (1 + phi nu_f / (2 K))), the gap decays by
  (1 - d0 - d1) / (1 + d0 + d1) per step (Crank-Nicolson form of the
  interphase source, Eqs. 41-46) and phi T_f + (1 - phi) sigma T_s stays
  constant -- closed forms for every field after any number of steps, over
  three successive step calls;
- a state set by hand: temperature populations w~_i P(x) and flow
  populations at rest, so after one step the macros are the D2Q5 weighted
  average of P over each node's pull stencil (Eqs. 34, 35 and the zeroth
  moment), a non-uniform field against the given initial one.

A copy of the oracle source with a planted mistake (normalisation by the
previous field, a previous buffer never refreshed, maxima instead of sums,
the solid term fed by the fluid field, the y velocity left out) must fail
at least one pin."""
import os

import numpy as np
import pytest

from paper_1608_04118_amd import inputs as I

TOL = 1e-11


def _uniform_case(G=(3e-5, -2e-5), Tf0=1.0, Ts0=0.2):
    return I.complete(nx=7, ny=5, periodic_x=1, periodic_y=1, Ra=0.0, Ma=0.0, nu_f=0.1, L=100.0,
                      dT=1.0, Da=0.05, F_phi=0.0, phi=0.6, sigma=1.7, gamma_sf=2.0, Hv=1000.0,
                      T_init_f=Tf0, T_init_s=Ts0, T0=0.0, body_force=G)


def _closed_form(p, k):
    """(u_x, u_y, T_f, T_s) of the uniform case after k steps."""
    L, phi, sig, nu = p["L"], p["phi"], p["sigma"], p["nu_f"]
    K = p["Da"] * L * L
    alpha_f = nu / p["Pr"]
    hv = p["Hv"] * alpha_f / (L * L)
    d0, d1 = 0.5 * hv / phi, 0.5 * hv / ((1.0 - phi) * sig)
    r = (1.0 - d0 - d1) / (1.0 + d0 + d1)
    c = phi + (1.0 - phi) * sig
    E = phi * p["T_init_f"] + (1.0 - phi) * sig * p["T_init_s"]
    D = (p["T_init_s"] - p["T_init_f"]) * r ** k
    Tf = (E - (1.0 - phi) * sig * D) / c
    a = (phi * nu / K) / (1.0 + phi * nu / (2.0 * K))
    us = []
    for g in p["body_force"]:
        b = phi * g * (1.0 - 0.5 * a)
        w = b / a * (1.0 - (1.0 - a) ** k)   # j / rho, from rest
        us.append((w + 0.5 * phi * g) / (1.0 + phi * nu / (2.0 * K)))
    return us[0], us[1], Tf, Tf + D


def _expected_residual(p, k_prev, k):
    a, b = _closed_form(p, k), _closed_form(p, k_prev)
    den_u = abs(a[0]) + abs(a[1])
    q_u = (abs(a[0] - b[0]) + abs(a[1] - b[1])) / den_u if den_u > 0 else abs(a[0] - b[0]) + abs(a[1] - b[1])
    return max(q_u, abs(a[2] - b[2]) / abs(a[2]), abs(a[3] - b[3]) / abs(a[3]))


def _pins(oracle, lib=None):
    """Runs every pin against the oracle built into lib; returns the largest
    relative deviation from the closed forms."""
    worst = 0.0
    cases = [_uniform_case(), _uniform_case(G=(0.0, 0.0), Tf0=1.0, Ts0=0.05),
             _uniform_case(G=(0.0, 4e-5), Tf0=0.3, Ts0=0.31)]
    for p in cases:
        o = oracle.Oracle(p, lib=lib)
        m = o.macros()
        ux0, uy0, tf0, ts0 = _closed_form(p, 0)
        assert abs(m["Tf"][0, 0] - tf0) <= 1e-14 and abs(m["ux"][0, 0] - ux0) <= 1e-14 * max(abs(ux0), 1e-30)
        done = 0
        for n in (3, 4, 13):
            o.step(n)
            got = o.diagnostics()[2]
            exp = _expected_residual(p, done, done + n)
            worst = max(worst, abs(got - exp) / exp)
            done += n
        o.step(0)  # a call that advances nothing keeps the reference
        got = o.diagnostics()[2]
        worst = max(worst, abs(got - exp) / exp)
    # non-uniform: populations set by hand, one step of pure pull averaging
    nx, ny = 11, 9
    p = I.complete(nx=nx, ny=ny, periodic_x=1, periodic_y=1, Ra=0.0, Ma=0.0, nu_f=0.1, L=50.0, dT=1.0,
                   Da=0.05, F_phi=0.0, phi=0.6, Hv=30.0, T0=0.0)
    rng = np.random.default_rng(11)
    Q = 0.5 + 0.3 * rng.standard_normal((ny, nx))
    P = 0.4 + 0.3 * rng.standard_normal((ny, nx))
    o = oracle.Oracle(p, Tf0=Q, Ts0=Q, lib=lib)
    vp = p["varpi"]
    w5 = np.array([1.0 - vp, vp / 4, vp / 4, vp / 4, vp / 4])
    w9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    g = (P.reshape(-1, 1) * w5[None, :])
    f = np.broadcast_to(w9[None, :] * p["rho0"], (nx * ny, 9))
    o.set_populations(f=f, gf=g, gs=g)
    o.step(1)
    # node x pulls population i from x - e_i: rest, +x, +y, -x, -y
    S = ((1.0 - vp) * P + 0.25 * vp * (np.roll(P, 1, axis=1) + np.roll(P, 1, axis=0) +
                                       np.roll(P, -1, axis=1) + np.roll(P, -1, axis=0)))
    m = o.macros()
    assert np.abs(m["Tf"] - S).max() <= 1e-14 and np.abs(m["Ts"] - S).max() <= 1e-14
    assert np.abs(m["ux"]).max() <= 1e-16 and np.abs(m["uy"]).max() <= 1e-16
    exp = np.abs(S - Q).sum() / np.abs(S).sum()
    got = o.diagnostics()[2]
    worst = max(worst, abs(got - exp) / exp)
    return worst


def test_residual_closed_forms(oracle):
    worst = _pins(oracle)
    assert worst <= TOL, worst


MUTATIONS = {
    "normalised by the previous field": [
        ("nu += fabs(o->ux[c]) + fabs(o->uy[c]);", "nu += fabs(o->pux[c]) + fabs(o->puy[c]);"),
        ("ntf += fabs(o->Tf[c]);", "ntf += fabs(o->pTf[c]);"),
        ("nts += fabs(o->Ts[c]);", "nts += fabs(o->pTs[c]);")],
    "previous buffer never refreshed": [
        ("  memcpy(o->pux, o->ux, n * sizeof(double));\n  memcpy(o->puy, o->uy, n * sizeof(double));\n"
         "  memcpy(o->pTf, o->Tf, n * sizeof(double));\n  memcpy(o->pTs, o->Ts, n * sizeof(double));\n"
         "  for (int64_t s", "  for (int64_t s")],
    "maxima instead of sums": [
        ("dtf += fabs(o->Tf[c] - o->pTf[c]);", "dtf = fmax(dtf, fabs(o->Tf[c] - o->pTf[c]));"),
        ("ntf += fabs(o->Tf[c]);", "ntf = fmax(ntf, fabs(o->Tf[c]));"),
        ("dts += fabs(o->Ts[c] - o->pTs[c]);", "dts = fmax(dts, fabs(o->Ts[c] - o->pTs[c]));"),
        ("nts += fabs(o->Ts[c]);", "nts = fmax(nts, fabs(o->Ts[c]));")],
    "solid term from the fluid field": [
        ("dts += fabs(o->Ts[c] - o->pTs[c]);", "dts += fabs(o->Tf[c] - o->pTf[c]);")],
    "y velocity left out": [
        ("du += fabs(o->ux[c] - o->pux[c]) + fabs(o->uy[c] - o->puy[c]);",
         "du += fabs(o->ux[c] - o->pux[c]);"),
        ("nu += fabs(o->ux[c]) + fabs(o->uy[c]);", "nu += fabs(o->ux[c]);")],
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_residual_pins_catch_planted_mistakes(oracle, tmp_path, name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "ltne_oracle.c")).read()
    for old, new in MUTATIONS[name]:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    lib = oracle.load_library(oracle.compile_source(src, str(tmp_path / "libmutant.so")))
    assert _pins(oracle, lib=lib) > 1e-6, name


# A cavity whose parameters are outside the scheme's stability range (Mach
# number 1, relaxation time 0.5017): its fields overflow to non-finite
# values within a few hundred steps.  Both sides must report that as a
# non-finite mass and energy (the GPU side through diag_every).
def unstable_cavity(precision=I.FP64, **kw):
    base = dict(nx=32, ny=32, Ma=1.0, Ra=1e9, Da=1e4, phi=0.9, precision=precision)
    base.update(kw)
    return I.cavity_small(**base)


def test_unstable_cavity_diverges_in_the_oracle(oracle):
    o = oracle.Oracle(unstable_cavity())
    o.step(2000)
    mass, energy, _ = o.diagnostics()
    assert not np.isfinite(mass) and not np.isfinite(energy)
    s = oracle.Oracle(unstable_cavity(Ma=0.1)).step(2000)  # the same cavity at Mach 0.1 stays finite
    assert all(np.isfinite(s.diagnostics()[:2]))
