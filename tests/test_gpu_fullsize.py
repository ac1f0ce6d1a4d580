"""Full-size runs of the workloads (GPU only), checked through properties that
hold at any size where the oracle cannot follow the whole run:

- the 1024 x 256 Brinkman-Forchheimer channel (FP32) at steady state against
  the 1-D boundary-value problem its profile must solve (closed form up to a
  converged quadrature), at Da = 1e-2 and 1e-4;
- the 1024 x 1024 cavity (Ra = 1e6) over its full 50000 steps: the binary32
  storage forms against the FP64 form, which equals the oracle to 1e-12 on
  every case the oracle can run (tests/test_gpu_parity.py);
- the 8192 x 8192 layer over 1000 steps in each form: FP32, FP32 storage with
  FP64 arithmetic, and FP16 storage against FP64.
"""
import math
import sys

import numpy as np
import pytest

from paper_1608_04118_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-full]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1608_04118_amd import binding
    binding.lib()
    return binding


def _rel(a, b, keys=("u", "Tf", "Ts")):
    out = {}
    if "u" in keys:
        out["u"] = np.hypot(a["ux"] - b["ux"], a["uy"] - b["uy"]).max() / np.hypot(b["ux"], b["uy"]).max()
    for k in keys:
        if k != "u":
            out[k] = np.abs(a[k] - b[k]).max() / np.abs(b[k]).max()
    return out


@pytest.mark.parametrize("Da,gate", [(1e-2, 1e-3), (1e-4, 1e-2)])
def test_channel_steady_profile(B, Da, gate):
    """Steady streamwise velocity across the channel against
    nu_e u'' - phi nu_f u / K - phi F_phi u^2 / sqrt(K) + phi G_b = 0 with
    u = 0 on the wall nodes, solved to round-off on a 64x finer grid; L2
    relative error gates 1e-3 (Da = 1e-2) and 1e-2 (Da = 1e-4, a Brinkman
    layer of about four cells)."""
    from test_oracle_physics import _bvp_forchheimer
    p = I.channel(Da=Da)
    lat = B.Lattice(p)
    d = lat.derived()
    K, nu, phi, L = d["K"], d["nu_f"], p["phi"], d["L"]
    relax = K / (phi * nu)  # Darcy relaxation time of the flow, in steps
    steps = int(min(2e5, max(2e4, 15 * relax)))
    say("channel Da %.0e: %d steps (Darcy time %.0f)" % (Da, steps, relax))
    lat.step(steps - 1000)
    m0 = lat.macros()
    lat.step(1000)
    m = lat.macros()
    u = m["ux"].mean(axis=1)  # periodic along x: average the columns
    drift = np.abs(m["ux"] - m0["ux"]).max() / np.abs(m["ux"]).max()
    spread = np.abs(m["ux"] - u[:, None]).max() / np.abs(u).max()
    Fphi = p["F_phi"] if p["F_phi"] >= 0 else 1.75 / math.sqrt(150 * phi ** 3)
    y, ub = _bvp_forchheimer(d["nu_e"], phi * nu / K, phi * Fphi / math.sqrt(K), phi * p["body_force"][0], L,
                             n=(p["ny"] - 1) * 64 + 1)
    ex = ub[::64]
    err = math.sqrt(((u - ex) ** 2).sum() / (ex ** 2).sum())
    Re = ex.max() * L / nu
    say("channel Da %.0e: L2 error %.2e, drift over the last 1000 steps %.1e, x-spread %.1e, Re %.2f"
        % (Da, err, drift, spread, Re))
    assert drift < 1e-6 and spread < 1e-6
    assert err <= gate


def test_cavity_large_full_length(B):
    """1024^2 cavity, Ra = 1e6, 50000 steps: the FP32 form (binary32 storage,
    binary32 flow arithmetic, binary64 temperature arithmetic with
    stochastically rounded stores) and FP32SR (binary64 arithmetic throughout)
    both stay within 1e-5 of FP64 on u, T_f and T_s after every 10000 steps,
    and their hot-wall Nusselt numbers within 1e-6.  The thermal diffusion
    time of this cavity is about 2e7 steps, so a rounding error that repeats
    at every step would add up over the whole run."""
    p32 = I.cavity_large()
    b = B.Lattice(dict(p32, precision=I.FP64))
    forms = {"fp32": B.Lattice(p32), "fp32sr": B.Lattice(dict(p32, precision=I.FP32SR))}
    worst = {name: 0.0 for name in forms}
    for chunk in range(5):
        b.step(10000)
        mb = b.macros()
        for name, a in forms.items():
            a.step(10000)
            e = _rel(a.macros(), mb)
            worst[name] = max(worst[name], max(e.values()))
            say("cavity 1024^2 after %d steps: %s vs fp64" % (10000 * (chunk + 1), name),
                {k: "%.2e" % v for k, v in e.items()})
    nb = b.nusselt()
    for name, a in forms.items():
        na = a.nusselt()
        say("Nu %s" % name, na, "fp64", nb)
        assert worst[name] <= 1e-5, (name, worst[name])
        assert abs(na[0] - nb[0]) <= 1e-6 * abs(nb[0]), (name, na, nb)


def test_layer_full_size_forms(B):
    """8192^2 layer, 1000 steps in each form, whole field: FP32 against FP64
    within 1e-5, FP32 storage with FP64 arithmetic within 1e-6; the
    FP16-storage error is reported."""
    p, phi, Tf0, Ts0 = I.throughput(n=8192, precision=I.FP64)
    ref = B.Lattice(p, phi=phi, Tf0=Tf0, Ts0=Ts0).step(1000)
    mr = ref.macros()
    ref.close()
    out = {}
    for prec, name in ((I.FP32, "fp32"), (I.FP32SR, "fp32sr"), (I.FP16S, "fp16s")):
        lat = B.Lattice(dict(p, precision=prec), phi=phi, Tf0=Tf0, Ts0=Ts0).step(1000)
        out[name] = _rel(lat.macros(), mr)
        lat.close()
        say("layer 8192^2 1000 steps: %s vs fp64" % name, {k: "%.2e" % v for k, v in out[name].items()})
    for k, v in out["fp32"].items():
        assert v <= 1e-5, (k, v)
    for k, v in out["fp32sr"].items():
        assert v <= 1e-6, (k, v)
    for k, v in out["fp16s"].items():
        assert np.isfinite(v) and v < 0.5, (k, v)
