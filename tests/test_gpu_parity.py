"""Parity of the HIP step with the FP64 oracle, element by element on the same
seeded inputs (GPU only).

Tolerances (max-relative per field, max|gpu - oracle| / max|oracle|): 1e-12
for the binary64 form, 1e-5 for the binary32 form on u, T_f, T_s.  The
binary16-storage form has no gate; its error is printed and only bounded
loosely to catch gross faults.

The full-size 8192 x 8192 layer is compared on strips: a periodic strip of
the same seeded inputs, wide enough to contain the dependence cone of its
middle columns, is run by the oracle (the strip identity is pinned in the
oracle's own tests)."""
import sys

import numpy as np
import pytest

from paper_1608_04118_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "Tf", "Ts")
GATED = ("rho", "u", "Tf", "Ts")


def say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1608_04118_amd import binding
    binding.lib()
    return binding


def rel(a, b):
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def rel_u(g, o):
    """Velocity error relative to the largest speed (vector norm)."""
    du = np.hypot(g["ux"] - o["ux"], g["uy"] - o["uy"]).max()
    um = np.hypot(o["ux"], o["uy"]).max()
    return du / (um if um > 0 else 1.0)


def compare(gm, om, tol, fields=("u", "Tf", "Ts"), label=""):
    errs = {k: (rel_u(gm, om) if k == "u" else rel(gm[k], om[k])) for k in fields}
    say(label, {k: "%.2e" % v for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= tol, (label, k, v)
    return errs


def pair(B, oracle, p, steps, **fields):
    kw = {k: fields.get(k) for k in ("phi", "Hv", "Tf0", "Ts0")}
    g = B.Lattice(p, **kw)
    o = oracle.Oracle(p, **kw)
    if steps:
        g.step(steps)
        o.step(steps)
    return g, o


def test_initial_state(B, oracle):
    say("initial state 64x64 fp64")
    p = I.cavity_small()
    g, o = pair(B, oracle, p, 0)
    compare(g.macros(), o.macros(), 1e-15, GATED, "t=0")


def test_cavity_small_fp64_full_length(B, oracle):
    """64 x 64 cavity, FP64, 2000 steps: fields, Nusselt numbers, sums."""
    say("cavity 64x64 fp64 2000 steps")
    p = I.cavity_small()
    g, o = pair(B, oracle, p, 2000)
    gm, om = g.macros(), o.macros()
    compare(gm, om, 1e-12, GATED, "cavity_small fp64")
    gn, on = g.nusselt(), o.nusselt()
    say("Nu gpu", gn, "oracle", on)
    for a, b in zip(gn, on):
        assert abs(a - b) <= 1e-12 * abs(b)
    gd, od = g.diagnostics(), o.diagnostics()
    say("diag gpu", gd, "oracle", od)
    assert abs(gd[0] - od[0]) <= 1e-12 * abs(od[0])
    assert abs(gd[1] - od[1]) <= 1e-12 * abs(od[1])
    # the residual of a second call compares two evolved states (the first
    # call's compares with the fluid at rest, where it is 1 on both sides)
    g.step(150)
    o.step(150)
    gd, od = g.diagnostics(), o.diagnostics()
    say("diag after a second call: gpu", gd, "oracle", od)
    assert 0.0 < od[2] < 0.5
    for a, b in zip(gd, od):
        assert abs(a - b) <= 1e-12 * abs(b), (a, b)


def test_residual_closed_form(B):
    """The residual on the uniform periodic lattice whose velocity and
    temperatures have closed forms (body acceleration, decaying T_s - T_f
    gap; see the oracle's residual pins), over three successive calls, FP64
    against the closed form."""
    from test_oracle_residual import _uniform_case, _expected_residual
    for p in (_uniform_case(), _uniform_case(G=(0.0, 4e-5), Tf0=0.3, Ts0=0.31)):
        g = B.Lattice(p)
        done = 0
        for n in (3, 4, 13):
            g.step(n)
            got = g.diagnostics()[2]
            exp = _expected_residual(p, done, done + n)
            say("residual after %d + %d steps: gpu %.15e closed form %.15e" % (done, n, got, exp))
            assert abs(got - exp) <= 1e-11 * exp
            done += n
        g.step(0)
        assert g.diagnostics()[2] == got


GEOMS = [
    # nx, ny, periodic_x, periodic_y, wall_thermal, T_wall, body force
    (4, 4, 0, 0, (0, 0, 1, 1), (1.0, 0.0, 0.0, 0.0), (1.6e-3, -1.2e-3)),
    (3, 3, 1, 1, (0, 0, 0, 0), (0.0, 0.0, 0.0, 0.0), (2e-5, -1e-5)),
    (67, 45, 0, 0, (0, 1, 0, 1), (1.0, 0.0, 0.7, 0.0), (2e-5, -1e-5)),  # ragged, mixed walls, corners
    (130, 9, 1, 0, (1, 1, 0, 0), (0.0, 0.0, 1.0, 0.0), (1e-4, 0.0)),    # periodic x, two tile widths
    (9, 130, 0, 1, (0, 0, 1, 1), (1.0, 0.2, 0.0, 0.0), (0.0, 1e-4)),    # periodic y
    (300, 17, 1, 1, (0, 0, 0, 0), (0.0, 0.0, 0.0, 0.0), (2e-5, -1e-5)),  # fully periodic, ragged tiles
    (257, 6, 0, 0, (1, 0, 0, 1), (0.0, 1.0, 0.5, 0.0), (2e-4, 0.0)),
]


@pytest.mark.parametrize("geom", GEOMS, ids=["%dx%d_p%d%d" % g[:4] for g in GEOMS])
@pytest.mark.parametrize("fields", [False, True], ids=["uniform", "fields"])
def test_fp64_geometries(B, oracle, geom, fields):
    nx, ny, px, py, wt, tw, bf = geom
    say("geometry", geom, "fields" if fields else "uniform")
    p = I.complete(nx=nx, ny=ny, periodic_x=px, periodic_y=py, wall_thermal=wt, T_wall=tw,
                   Ma=0.0, nu_f=0.05, Ra=3e4, dT=1.0, L=64.0, T0=0.4,
                   body_force=bf, Hv=80.0, gamma_sf=4.0, sigma=1.7, phi=0.55,
                   F_phi=-1.0, Qf=1e-5, Qs=-2e-5)
    r = np.random.default_rng(nx * 1000 + ny)
    kw = {}
    if fields:
        kw = dict(phi=np.clip(0.55 + 0.15 * r.standard_normal((ny, nx)), 0.3, 0.9),
                  Hv=80.0 * (1 + 0.5 * r.uniform(-1, 1, (ny, nx))),
                  Tf0=0.4 + 0.2 * r.standard_normal((ny, nx)),
                  Ts0=0.4 + 0.2 * r.standard_normal((ny, nx)))
    g, o = pair(B, oracle, p, 300, **kw)
    compare(g.macros(), o.macros(), 1e-12, GATED, "geom %s" % (geom,))


@pytest.mark.parametrize("precision,tol", [(I.FP32, 1e-5), (I.FP32SR, 1e-6)], ids=["fp32", "fp32sr"])
def test_cavity_small_fp32_full_length(B, oracle, precision, tol):
    """binary32 storage, 2000 steps: binary32 arithmetic within 1e-5; binary64
    arithmetic with stochastic rounding on store within 1e-6."""
    say("cavity 64x64 precision", precision, "2000 steps")
    p = I.cavity_small(precision=precision)
    g, o = pair(B, oracle, p, 2000)
    compare(g.macros(), o.macros(), tol, label="cavity_small precision %d" % precision)


def test_cavity_large_fp32(B, oracle):
    """1024 x 1024 cavity in the FP32 form, 300 steps, whole field."""
    say("cavity 1024x1024 fp32 300 steps")
    p = I.cavity_large()
    g, o = pair(B, oracle, p, 300)
    compare(g.macros(), o.macros(), 1e-5, label="cavity_large fp32")
    gn, on = g.nusselt(), o.nusselt()
    say("Nu gpu", gn, "oracle", on)
    assert abs(gn[0] - on[0]) <= 1e-4 * abs(on[0])


def test_channel_fp32(B, oracle):
    say("channel 1024x256 fp32 500 steps")
    p = I.channel()
    g, o = pair(B, oracle, p, 500)
    compare(g.macros(), o.macros(), 1e-5, fields=("u",), label="channel fp32")


def _strip_check(B, oracle, precision, steps, tol, windows=((0, 16), (4000, 16), (8176, 16)),
                 noise_floor=False, **extra):
    """GPU run of the full 8192 x 8192 layer; oracle runs of periodic strips
    around the windows.  Errors are relative to the field's magnitude over the
    whole lattice (velocity as a vector).  With noise_floor, the gate is
    max(tol, 10 x the oracle's own sensitivity to a one-ulp perturbation of
    its inputs), for fields so small after few steps that tol lies below what
    binary64 populations of size 0.1 resolve."""
    n = 8192
    p, phi, Tf0, Ts0 = I.throughput(n=n, precision=precision, **extra)
    say("throughput 8192x8192 precision", precision, "steps", steps, extra)
    g = B.Lattice(p, phi=phi, Tf0=Tf0, Ts0=Ts0).step(steps)
    gm = g.macros()
    g.close()
    umax = np.hypot(gm["ux"], gm["uy"]).max()
    scale = {"u": umax, "Tf": np.abs(gm["Tf"]).max(), "Ts": np.abs(gm["Ts"]).max()}
    margin = steps + 2
    worst, floor = {}, {}
    rng = np.random.default_rng(17)
    for x0, w in windows:
        cols = np.arange(x0 - margin, x0 + w + margin) % n
        ps = dict(p, nx=len(cols), L=n - 1.0)
        sl = (phi[:, cols], Tf0[:, cols], Ts0[:, cols])
        om = oracle.Oracle(ps, phi=sl[0], Tf0=sl[1], Ts0=sl[2]).step(steps).macros()
        inner = cols[margin:margin + w]
        sub = {k: gm[k][:, inner] for k in FIELDS}
        ref = {k: om[k][:, margin:margin + w] for k in FIELDS}
        err = {"u": np.hypot(sub["ux"] - ref["ux"], sub["uy"] - ref["uy"]).max(),
               "Tf": np.abs(sub["Tf"] - ref["Tf"]).max(), "Ts": np.abs(sub["Ts"] - ref["Ts"]).max()}
        for k in err:
            worst[k] = max(worst.get(k, 0.0), err[k] / scale[k])
        if noise_floor:
            pert = sl[1] * (1 + 2.2e-16 * rng.standard_normal(sl[1].shape))
            om2 = oracle.Oracle(ps, phi=sl[0], Tf0=pert, Ts0=sl[2]).step(steps).macros()
            fl = {"u": np.hypot(om2["ux"] - om["ux"], om2["uy"] - om["uy"]).max(),
                  "Tf": np.abs(om2["Tf"] - om["Tf"]).max(), "Ts": np.abs(om2["Ts"] - om["Ts"]).max()}
            for k in fl:
                floor[k] = max(floor.get(k, 0.0), fl[k] / scale[k])
    say("strips precision", precision, {k: "%.2e" % v for k, v in worst.items()},
        "oracle floor", {k: "%.2e" % v for k, v in floor.items()})
    for k, v in worst.items():
        gate = max(tol, 10.0 * floor.get(k, 0.0))
        assert v <= gate, (k, v, gate)
    return worst


def test_throughput_fp32_strips(B, oracle):
    _strip_check(B, oracle, I.FP32, 50, 1e-5)


def test_throughput_fp32sr_strips(B, oracle):
    _strip_check(B, oracle, I.FP32SR, 50, 1e-6)


def test_throughput_fp64_strips(B, oracle):
    _strip_check(B, oracle, I.FP64, 50, 1e-12, noise_floor=True)


def test_throughput_fp16_error(B, oracle):
    worst = _strip_check(B, oracle, I.FP16S, 50, 1e-2)
    say("fp16 storage error after 50 steps:", worst)


def test_fp16_cavity_error(B, oracle):
    """binary16 storage with stochastic rounding, 2000 steps: the error is
    reported; the bound only catches a broken form (round-to-nearest storage
    gave 5e-2 here, stochastic rounding about 2e-3)."""
    p = I.cavity_small(precision=I.FP16S)
    g, o = pair(B, oracle, p, 2000)
    compare(g.macros(), o.macros(), 1e-2, label="cavity_small fp16 storage (reported)")


def test_save_load_bitwise(B):
    say("save/load")
    p = I.cavity_small(nx=40, ny=33, precision=I.FP32)
    g = B.Lattice(p).step(50)
    buf = g.save()
    g.step(70)
    a = g.macros()
    g.load(buf)
    assert g.steps == 50
    g.step(70)
    b = g.macros()
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), k


def test_deterministic_and_diag(B):
    p, phi, Tf0, Ts0 = I.throughput(n=256, ny=128)
    runs = []
    for _ in range(2):
        g = B.Lattice(p, phi=phi, Tf0=Tf0, Ts0=Ts0).step(100)
        runs.append((g.macros(), g.nusselt(), g.diagnostics()))
    for k in FIELDS:
        assert np.array_equal(runs[0][0][k], runs[1][0][k])
    assert runs[0][1] == runs[1][1] and runs[0][2] == runs[1][2]


def test_step_zero_and_errors(B):
    g = B.Lattice(I.cavity_small(nx=16, ny=16))
    g.step(0)
    assert g.steps == 0
    with pytest.raises(B.LtneError):
        B.lbm_ltne_step(g.h, -1)


# Lattices large enough for two-step launches (at least 1024 wavefronts of
# 61 or 62 columns x 8 rows), with the strip and chunk edges falling on the
# awkward places: a wall column at the start of a strip (1038 = 17 x 61 + 1),
# a ragged last chunk, periodic wraps on either axis.
TWO_STEP_CASES = [
    ("layer 1100x1027, phi field", lambda: I.throughput(n=1100, ny=1027)),
    ("cavity 1038x1030", lambda: (I.cavity_small(nx=1038, ny=1030, precision=I.FP32, Ra=1e5), None, None, None)),
    ("torus 1030x1030", lambda: (I.complete(nx=1030, ny=1030, periodic_x=1, periodic_y=1, precision=I.FP32,
                                            Ra=1e4, body_force=(1e-4, -2e-5)), None, None, None)),
    ("channel along y 1030x1040", lambda: (I.channel(nx=1030, ny=1040, axis="y"), None, None, None)),
    ("cavity 1024x1024, both extensions", lambda: (I.cavity_small(nx=1024, ny=1024, precision=I.FP32, Ra=1e5,
                                                                  thermal_correction=1, pore_size=0.0135),
                                                   None, None, None)),
    # lattices that take taller chunks (FP32: the tallest of 32, 24, 16, 12 rows
    # giving 16384 wavefronts): 12 rows with x walls (66 strips x 251
    # chunks), 24 rows periodic (97 x 209) and the 8192^2 layer, 32 rows
    # (133 x 256), ragged last chunks in the first two
    ("cavity 4000x3004, tall chunks", lambda: (I.cavity_small(nx=4000, ny=3004, precision=I.FP32, Ra=1e6),
                                                None, None, None)),
    ("layer 6000x5000, tall chunks", lambda: I.throughput(n=6000, ny=5000)),
    ("layer 8192x8192, tall chunks", lambda: I.throughput(n=8192)),
    # the FP64 form (pairs from 2560 wavefronts of 8 rows on): 27 strips x
    # 191 chunks with a ragged last chunk, x walls at a strip start
    # (1648 = 27 x 61 + 1), periodic wraps on both axes
    ("fp64 layer 1650x1527, phi field", lambda: I.throughput(n=1650, ny=1527, precision=I.FP64)),
    ("fp64 cavity 1648x1630", lambda: (I.cavity_small(nx=1648, ny=1630, Ra=1e5), None, None, None)),
    ("fp64 torus 1600x1600", lambda: (I.complete(nx=1600, ny=1600, periodic_x=1, periodic_y=1, precision=I.FP64,
                                                 Ra=1e4, body_force=(1e-4, -2e-5)), None, None, None)),
    ("fp64 cavity 1600x1600, both extensions", lambda: (I.cavity_small(nx=1600, ny=1600, Ra=1e5,
                                                                       thermal_correction=1, pore_size=0.0135),
                                                        None, None, None)),
    # 64-row chunks (the binary64 kernel's tallest, taken from 8192
    # wavefronts on): the full layer (133 strips x 128 chunks) and a walled
    # cavity with a ragged last chunk of 4 rows (135 x 65)
    ("fp64 layer 8192x8192, tall chunks", lambda: I.throughput(n=8192, precision=I.FP64)),
    ("fp64 cavity 8200x4100, tall chunks", lambda: (I.cavity_small(nx=8200, ny=4100, Ra=1e6), None, None, None)),
]


@pytest.mark.parametrize("nsteps", [41, 40], ids=["odd", "even"])
@pytest.mark.parametrize("case", TWO_STEP_CASES, ids=[c[0] for c in TWO_STEP_CASES])
def test_two_step_launch_equals_single_steps(B, case, nsteps):
    """The FP32 and FP64 forms advance pairs of steps in one launch on
    lattices this size (an odd call ends with one single step, which writes
    the macros; in an even call the last pair writes them); the result equals
    single steps bit for bit: nsteps steps in one call against nsteps calls of
    one step."""
    name, make = case
    p, phi, Tf0, Ts0 = make()
    a = B.Lattice(p, phi=phi, Tf0=Tf0, Ts0=Ts0).step(nsteps)
    b = B.Lattice(p, phi=phi, Tf0=Tf0, Ts0=Ts0)
    for _ in range(nsteps):
        b.step(1)
    ma, mb = a.macros(), b.macros()
    for k in FIELDS:
        assert np.array_equal(ma[k], mb[k]), (name, k, np.abs(ma[k] - mb[k]).max())
    # mass and energy of the final macros (the residual compares with the
    # previous call's macros, which differ between the two runs)
    assert a.diagnostics()[:2] == b.diagnostics()[:2]
    say("two-step launches equal single steps bit for bit:", name, nsteps, "steps")


def test_fp64_pairs_match_oracle(B, oracle):
    """The FP64 form's two-step launches against the oracle directly (the
    bit-for-bit cases above tie them to single steps): a walled 1648 x 1630
    cavity (28 strips x 204 chunks of 8 rows) with smoothed porosity and H_v
    fields, initial temperature fields and a body acceleration (velocities
    of 1e-3, which binary64 resolves to 1e-12: a cavity heated only from a
    wall moves at 1e-4 after 200 steps, below that resolution, see the
    strips), 200 steps in pairs, the last pair writing the macros; whole
    field at 1e-12, and the mass and energy sums."""
    say("fp64 pairs 1648x1630 cavity with fields, 200 steps, against the oracle")
    nx, ny = 1648, 1630
    z1 = I.smoothed_noise(21, ny, nx, sigma=8.0)
    z2 = I.smoothed_noise(22, ny, nx, sigma=8.0)
    p = I.complete(nx=nx, ny=ny, Ra=1e5, body_force=(2e-5, -1e-5), T_wall=(1.0, 0.0, 0.0, 0.0))
    phi = np.clip(0.6 + 0.1 * z1, 0.35, 0.9)
    Hv = 10.0 * (1 + 0.3 * np.clip(z2, -1, 1))
    g, o = pair(B, oracle, p, 200, phi=phi, Hv=Hv, Tf0=0.5 + 0.1 * z2, Ts0=0.5 - 0.1 * z1)
    compare(g.macros(), o.macros(), 1e-12, GATED, "fp64 pairs cavity 1648x1630")
    gd, od = g.diagnostics(), o.diagnostics()
    for a, b in zip(gd[:2], od[:2]):
        assert abs(a - b) <= 1e-12 * abs(b), (a, b)


RECORDED_CASES = [
    ("fp64 64x64", lambda: (I.cavity_small(), None, None)),
    ("fp32 96x80 phi field", lambda: (I.cavity_small(nx=96, ny=80, precision=I.FP32, Ra=3e4),
                                      np.clip(0.6 + 0.1 * np.random.default_rng(2).standard_normal((80, 96)),
                                              0.3, 0.9), None)),
    ("fp16 storage 70x64 Hv field", lambda: (I.cavity_small(nx=70, ny=64, precision=I.FP16S), None,
                                             10.0 * (1 + 0.5 * np.random.default_rng(3).uniform(-1, 1, (64, 70))))),
    ("fp32sr 130x9 periodic x", lambda: (I.throughput(n=130, ny=9, precision=I.FP32SR)[0], None, None)),
]


@pytest.mark.parametrize("case", RECORDED_CASES, ids=[c[0] for c in RECORDED_CASES])
def test_recorded_runs_equal_single_steps(B, case):
    """Small lattices take runs of 32 steps as one recorded sequence of
    launches (a HIP graph replayed whole, the step number read from device
    memory); the result equals single-step calls bit for bit, from either
    population buffer, and parity with the oracle is unchanged (the 64^2
    cavity tests above run through it)."""
    name, make = case
    p, phi, Hv = make()
    a = B.Lattice(p, phi=phi, Hv=Hv).step(1).step(70).step(33)
    b = B.Lattice(p, phi=phi, Hv=Hv)
    for _ in range(104):
        b.step(1)
    ma, mb = a.macros(), b.macros()
    for k in FIELDS:
        assert np.array_equal(ma[k], mb[k]), (name, k, np.abs(ma[k] - mb[k]).max())
    assert a.steps == b.steps == 104
    say("recorded runs equal single steps bit for bit:", name)
