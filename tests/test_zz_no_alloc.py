"""The allocation-free entry point lbm_ltne_macro_sums_noalloc (GPU only):
the binary64 mass, energy and residual sums of macro fields the caller holds
in device memory, computed with a file-scope scratch array instead of
allocated memory, equal those lbm_ltne_diagnostics computes for the same
fields bit for bit -- on two calls in a row, the second on a smaller
lattice, in binary64 and binary32 compute types."""
import sys

import numpy as np
import pytest

from paper_1608_04118_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "Tf", "Ts")


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1608_04118_amd import binding
    binding.lib()
    return binding


def _case(B, p, steps, phi=None):
    import torch
    lat = B.Lattice(p, phi=phi)
    lat.step(steps)
    prev = lat.macros()
    lat.step(37)
    cur = lat.macros()
    ref = lat.diagnostics()
    dt = torch.float64 if p["precision"] in (I.FP64, I.FP32SR) else torch.float32
    dev = lambda m: torch.tensor(np.stack([m[k] for k in FIELDS]), dtype=dt, device="cuda").contiguous()
    mac, pm = dev(cur), dev(prev)
    ph = None if phi is None else torch.tensor(phi, dtype=dt, device="cuda").contiguous()
    stream = torch.cuda.current_stream()
    got = B.lbm_ltne_macro_sums_noalloc(p, mac.data_ptr(), pm.data_ptr(), None if ph is None else ph.data_ptr(),
                                        stream.cuda_stream)
    lat.close()
    print("[gpu-noalloc]", p["nx"], p["ny"], p["precision"], "noalloc", got, "diagnostics", ref, flush=True)
    sys.stdout.flush()
    return got, ref


@pytest.mark.parametrize("precision", [I.FP64, I.FP32], ids=["fp64", "fp32"])
def test_noalloc_sums_equal_diagnostics(B, precision):
    r = np.random.default_rng(21)
    big = I.cavity_small(nx=300, ny=257, precision=precision, Ra=3e4)
    phi = np.clip(0.6 + 0.1 * r.standard_normal((257, 300)), 0.3, 0.9)
    small = I.throughput(n=40, ny=33, precision=precision)[0]
    for p, steps, ph in ((big, 200, phi), (small, 60, None)):
        got, ref = _case(B, p, steps, ph)
        assert got == ref, (got, ref)
        assert 0.0 < got[2] < 1.0
