"""Error measures shared by the GPU parity tests.

Tolerance semantics: max-relative per field, max|gpu - oracle| / max|oracle|,
velocity as a vector.  For binary64 the gate is max(tol, 10 x the oracle's
own change when one input field is perturbed by about one ulp): a field whose
magnitude is small against the populations it is computed from (a flow that
has barely started) cannot be resolved to 1e-12 of itself by any binary64
implementation, the oracle included."""
import numpy as np


def rel(a, b):
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def rel_u(g, o):
    du = np.hypot(g["ux"] - o["ux"], g["uy"] - o["uy"]).max()
    um = np.hypot(o["ux"], o["uy"]).max()
    return du / (um if um > 0 else 1.0)


def errors(g, o, fields=("u", "Tf", "Ts")):
    return {k: (rel_u(g, o) if k == "u" else rel(g[k], o[k])) for k in fields}


def oracle_floor(oracle, p, steps, phi=None, Hv=None, Tf0=None, Ts0=None, fields=("u", "Tf", "Ts")):
    """The oracle's own relative change under a one-ulp perturbation of the
    initial fluid temperature (or of the porosity field when given)."""
    ny, nx = int(p["ny"]), int(p["nx"])
    r = np.random.default_rng(123)
    base = oracle.Oracle(p, phi=phi, Hv=Hv, Tf0=Tf0, Ts0=Ts0).step(steps).macros()
    if phi is not None:
        phi2 = np.asarray(phi) * (1 + 1.1e-16 * r.standard_normal((ny, nx)))
        pert = oracle.Oracle(p, phi=phi2, Hv=Hv, Tf0=Tf0, Ts0=Ts0).step(steps).macros()
    else:
        tf = np.broadcast_to(p["T_init_f"] if Tf0 is None else Tf0, (ny, nx)).astype(float)
        tf2 = tf + 2.2e-16 * np.maximum(np.abs(tf), 1.0) * r.standard_normal((ny, nx))
        pert = oracle.Oracle(p, phi=phi, Hv=Hv, Tf0=tf2, Ts0=Ts0).step(steps).macros()
    return errors(pert, base, fields)
