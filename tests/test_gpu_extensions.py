"""Parity of the two model extensions with the FP64 oracle (GPU only): the
interphase coefficient from the correlation of Eq. 52 (pore_size > 0) and the
correction term of Sec. 3.2 (thermal_correction = 1), each alone and both
together, with the gates of the base model (1e-12 for binary64, 1e-5 for
binary32, 1e-6 for binary32 storage with binary64 arithmetic)."""
import sys

import numpy as np
import pytest

from paper_1608_04118_amd import inputs as I
from test_gpu_parity import GATED, compare, pair, _strip_check

pytestmark = pytest.mark.gpu

VARIANTS = [(1, 0.0), (0, 0.0135), (1, 0.0135)]
IDS = ["correction", "correlation", "both"]


def say(*a):
    print("[gpu-ext]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1608_04118_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("tc,pore", VARIANTS, ids=IDS)
def test_cavity_fp64(B, oracle, tc, pore):
    """64 x 64 cavity, FP64, 2000 steps: fields and Nusselt numbers; the
    extension must change the oracle's result well beyond the gate."""
    say("cavity 64x64 fp64 2000 steps, correction %d, pore size %g" % (tc, pore))
    p = I.cavity_small(thermal_correction=tc, pore_size=pore)
    g, o = pair(B, oracle, p, 2000)
    om = o.macros()
    compare(g.macros(), om, 1e-12, GATED, "ext fp64 tc=%d pore=%g" % (tc, pore))
    for a, b in zip(g.nusselt(), o.nusselt()):
        assert abs(a - b) <= 1e-12 * abs(b)
    base = oracle.Oracle(I.cavity_small()).step(2000).macros()
    effect = max(np.abs(om[k] - base[k]).max() / np.abs(base[k]).max() for k in ("Tf", "Ts", "ux"))
    say("effect of the extension on the oracle's fields: %.2e" % effect)
    assert effect > 1e-6


GEOMS = [
    (67, 45, 0, 0, (0, 1, 0, 1), (1.0, 0.0, 0.7, 0.0), (2e-5, -1e-5)),
    (130, 9, 1, 0, (1, 1, 0, 0), (0.0, 0.0, 1.0, 0.0), (1e-4, 0.0)),
    (9, 130, 0, 1, (0, 0, 1, 1), (1.0, 0.2, 0.0, 0.0), (0.0, 1e-4)),
    (300, 17, 1, 1, (0, 0, 0, 0), (0.0, 0.0, 0.0, 0.0), (2e-5, -1e-5)),
]


@pytest.mark.parametrize("geom", GEOMS, ids=["%dx%d_p%d%d" % g[:4] for g in GEOMS])
def test_geometries_fp64_both(B, oracle, geom):
    """Ragged and periodic lattices, mixed walls, per-node porosity and
    initial temperatures, both extensions, 300 steps."""
    nx, ny, px, py, wt, tw, bf = geom
    say("geometry", geom)
    p = I.complete(nx=nx, ny=ny, periodic_x=px, periodic_y=py, wall_thermal=wt, T_wall=tw,
                   Ma=0.0, nu_f=0.05, Ra=3e4, dT=1.0, L=64.0, T0=0.4, body_force=bf,
                   gamma_sf=4.0, sigma=1.7, phi=0.55, F_phi=-1.0, Qf=1e-5, Qs=-2e-5,
                   thermal_correction=1, pore_size=0.05)
    r = np.random.default_rng(nx * 1000 + ny + 7)
    kw = dict(phi=np.clip(0.55 + 0.15 * r.standard_normal((ny, nx)), 0.3, 0.9),
              Tf0=0.4 + 0.2 * r.standard_normal((ny, nx)),
              Ts0=0.4 + 0.2 * r.standard_normal((ny, nx)))
    g, o = pair(B, oracle, p, 300, **kw)
    compare(g.macros(), o.macros(), 1e-12, GATED, "ext geom %s" % (geom,))


@pytest.mark.parametrize("precision,tol", [(I.FP32, 1e-5), (I.FP32SR, 1e-6)], ids=["fp32", "fp32sr"])
def test_cavity_binary32_both(B, oracle, precision, tol):
    say("cavity 64x64 precision", precision, "2000 steps, both extensions")
    p = I.cavity_small(precision=precision, thermal_correction=1, pore_size=0.0135)
    g, o = pair(B, oracle, p, 2000)
    compare(g.macros(), o.macros(), tol, label="ext cavity precision %d" % precision)


def test_layer_strips_fp32_both(B, oracle):
    """The full 8192 x 8192 layer with both extensions, on strips (50 steps)."""
    _strip_check(B, oracle, I.FP32, 50, 1e-5, thermal_correction=1, pore_size=0.0135)


def test_fp16_cavity_both_bounded(B, oracle):
    p = I.cavity_small(precision=I.FP16S, thermal_correction=1, pore_size=0.0135)
    g, o = pair(B, oracle, p, 2000)
    errs = compare(g.macros(), o.macros(), 1e-2, label="ext cavity fp16 storage (bounded)")
    assert all(np.isfinite(v) for v in errs.values())


def test_batch_equals_single_with_extensions(B):
    """A batch whose lattices mix the extensions evolves each lattice exactly
    as when it runs alone."""
    ps = [I.cavity_small(nx=64, ny=64, precision=I.FP32, thermal_correction=1),
          I.cavity_small(nx=96, ny=96, precision=I.FP32, pore_size=0.0135, Ra=3e4),
          I.cavity_small(nx=130, ny=70, precision=I.FP32, thermal_correction=1, pore_size=0.02),
          I.cavity_small(nx=77, ny=77, precision=I.FP32)]
    bt = B.Batch(ps)
    bt.step(120)
    for i, p in enumerate(ps):
        a = bt.macros(i)
        b = B.Lattice(p).step(120).macros()
        for k in ("rho", "ux", "uy", "Tf", "Ts"):
            assert np.array_equal(a[k], b[k]), (i, k)
    say("batch with extensions bitwise equal to single runs")


def test_adjoint_refuses_the_correlation(B):
    """The correlation's derivative is unbounded at rest; the adjoint refuses
    it (the correction term is covered, tests/test_gpu_adjoint.py)."""
    lat = B.Lattice(I.cavity_small(nx=24, ny=20, pore_size=0.0135))
    with pytest.raises(B.LtneError) as e:
        lat.adjoint(10, 5)
    assert e.value.code == B.LBM_EUNSUPPORTED
    lat.step(3)  # the lattice is still usable
