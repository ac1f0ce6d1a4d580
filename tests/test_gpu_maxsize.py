"""The largest lattice the library accepts (nx * ny = 2^30 nodes, 32768 x
32768; binary32 storage needs about 207 GB of the 288 GB of HBM), run in the
configuration of the throughput layer, checked on strips against the FP64
oracle (GPU only).  Exercises every 32-bit node index and byte offset at its
largest value and the 64-bit row bases beyond 4 GiB."""
import sys

import numpy as np
import pytest

from paper_1608_04118_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-max]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1608_04118_amd import binding
    binding.lib()
    return binding


def test_maximum_lattice_fp32(B, oracle):
    n, steps = 32768, 50
    p = I.complete(nx=n, ny=n, precision=I.FP32, periodic_x=1, periodic_y=0,
                   wall_thermal=(I.ADIABATIC, I.ADIABATIC, I.DIRICHLET, I.DIRICHLET),
                   T_wall=(0.0, 0.0, 1.0, 0.0), T0=0.5, T_init_f=0.5, T_init_s=0.5, phi=0.65,
                   Da=1e-3, Ra=1e5, Hv=10.0, nu_wall=2, L=8191.0)
    rng = np.random.default_rng(11)
    Tf0 = rng.uniform(0.45, 0.55, (n, n))
    Ts0 = rng.uniform(0.45, 0.55, (n, n))
    say("creating %d x %d (2^30 nodes), fp32" % (n, n))
    g = B.Lattice(p, Tf0=Tf0, Ts0=Ts0).step(steps)
    mass, energy, _ = g.diagnostics()
    assert np.isfinite(mass) and np.isfinite(energy)
    gm = g.macros()
    g.close()
    scale = {"u": np.hypot(gm["ux"], gm["uy"]).max(), "Tf": np.abs(gm["Tf"]).max(), "Ts": np.abs(gm["Ts"]).max()}
    margin, w = steps + 2, 16
    worst = {}
    for x0 in (0, n // 2 - 8, n - w):
        cols = np.arange(x0 - margin, x0 + w + margin) % n
        ps = dict(p, nx=len(cols))
        om = oracle.Oracle(ps, Tf0=Tf0[:, cols], Ts0=Ts0[:, cols]).step(steps).macros()
        inner = cols[margin:margin + w]
        sub = {k: gm[k][:, inner] for k in ("ux", "uy", "Tf", "Ts")}
        ref = {k: om[k][:, margin:margin + w] for k in ("ux", "uy", "Tf", "Ts")}
        err = {"u": np.hypot(sub["ux"] - ref["ux"], sub["uy"] - ref["uy"]).max() / scale["u"],
               "Tf": np.abs(sub["Tf"] - ref["Tf"]).max() / scale["Tf"],
               "Ts": np.abs(sub["Ts"] - ref["Ts"]).max() / scale["Ts"]}
        for k, v in err.items():
            worst[k] = max(worst.get(k, 0.0), v)
    say("strips at x = 0, n/2, n - 16 after %d steps:" % steps, {k: "%.2e" % v for k, v in worst.items()})
    for k, v in worst.items():
        assert v <= 1e-5, (k, v)


def test_lattice_beyond_device_memory_is_refused(B):
    """2^30 nodes in binary64 need 2 x 163 GB of populations, more than the
    device holds: creation fails with LBM_ENOMEM and leaves nothing behind."""
    n = 32768
    p = I.complete(nx=n, ny=n, precision=I.FP64, periodic_x=1, nu_f=0.1, Ma=0.0, Ra=1e5)
    with pytest.raises(B.LtneError) as e:
        B.Lattice(p, use_torch=False)
    assert e.value.code == B.LBM_ENOMEM
    say("binary64 2^30 nodes refused:", B.lbm_ltne_last_error())
    lat = B.Lattice(I.cavity_small(nx=40, ny=30), use_torch=False).step(5)  # the device is still usable
    assert np.isfinite(lat.macros()["Tf"]).all()
