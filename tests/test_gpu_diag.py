"""Divergence checks during stepping (GPU only): with diag_every > 0 the
library sums the mass and energy of every diag_every-th step in binary64 on
the device, and the next synchronizing call reports a non-finite sum as
LBM_EDIVERGED.  The unstable cavity (Mach 1, relaxation time 0.5017) is the
one whose oracle run turns non-finite (tests/test_oracle_residual.py).
Checked steps run one step per launch; the results stay those of plain
stepping bit for bit."""
import sys

import numpy as np
import pytest

from paper_1608_04118_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "Tf", "Ts")


def say(*a):
    print("[gpu-diag]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1608_04118_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("precision", [I.FP64, I.FP32], ids=["fp64", "fp32"])
def test_divergence_is_reported(B, precision):
    from test_oracle_residual import unstable_cavity
    p = unstable_cavity(precision=precision, diag_every=50)
    say("unstable cavity, precision", precision)
    g = B.Lattice(p)
    g.step(10)
    saved = g.save()
    g.step(1990)  # asynchronous: no error yet
    for call in (g.macros, g.nusselt, g.diagnostics):
        with pytest.raises(B.LtneError) as e:
            call()
        assert e.value.code == B.LBM_EDIVERGED, call
    say("reported:", B.lbm_ltne_last_error())
    g.load(saved)  # a loaded state clears the record
    m = g.macros()
    assert np.isfinite(m["rho"]).all()
    # without the check the same run returns no error until diagnostics
    q = B.Lattice(dict(p, diag_every=0)).step(2000)
    q.macros()
    with pytest.raises(B.LtneError) as e:
        q.diagnostics()
    assert e.value.code == B.LBM_EDIVERGED


@pytest.mark.parametrize("make", [lambda: I.cavity_small(nx=1038, ny=1030, precision=I.FP32, Ra=1e5),
                                  lambda: I.cavity_small(nx=70, ny=50, precision=I.FP64)],
                         ids=["fp32_two_step_1038x1030", "fp64_70x50"])
def test_checked_steps_change_nothing(B, make):
    p = make()
    a = B.Lattice(dict(p, diag_every=7)).step(41).step(16)
    b = B.Lattice(p).step(41).step(16)
    ma, mb = a.macros(), b.macros()
    for k in FIELDS:
        assert np.array_equal(ma[k], mb[k]), k
    assert a.diagnostics() == b.diagnostics()
