"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the header declares, the parameter struct layout matches,
validation rejects what it must, and the parameter mapping agrees with the
oracle's independent mapping."""
import math
import os
import re

import numpy as np
import pytest

from paper_1608_04118_amd import binding as B
from paper_1608_04118_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm_ltne.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_1608_04118_amd import build
        build.build()
    return B.lib()


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_ltne_\w+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert B.lbm_ltne_abi_version() == 3


def test_struct_layout_roundtrip(lib):
    p = B.lbm_ltne_default_params()
    # the setup of Sec. 4, read back field by field through the mirror
    assert (p.nx, p.ny, p.precision) == (64, 64, B.LBM_FP64)
    assert tuple(p.wall_thermal) == (0, 0, 1, 1) and p.nu_wall == -1
    assert tuple(p.T_wall)[:2] == (11.0, 1.0) and p.T0 == 1.0
    assert (p.phi, p.Da, p.F_phi, p.gamma_sf, p.sigma) == (0.8, 1e-4, 0.068, 1000.0, 1.0)
    assert (p.varpi, p.s_e, p.s_eps, p.s_q) == (0.4, 1.1, 1.1, 1.2)
    assert (p.zeta_e, p.zeta_nu, p.eta_e, p.eta_nu, p.rho0) == (1.1, 1.1, 1.1, 1.1, 1.0)
    assert math.isnan(p.T_ref) and p.fp16_scale_f == 0.0 and p.fp16_scale_g == 0.0
    assert p.pore_size == 0.0 and p.diag_every == 0
    q = B.params_from_dict(I.cavity_small(diag_every=7, pore_size=0.25))
    assert (q.diag_every, q.pore_size) == (7, 0.25)


@pytest.mark.parametrize("mk", [I.cavity_small, I.cavity_large, lambda: I.channel(),
                                lambda: I.throughput(n=512)[0], lambda: I.adjoint_cavity(n=64)[0]])
def test_mapping_matches_oracle(lib, oracle, mk):
    p = mk()
    d = B.lbm_ltne_derive(p)
    o = oracle.derive(p)
    for k in ("L", "dT", "gbeta", "u_c", "nu_f", "nu_e", "s_nu", "alpha_f", "alpha_s",
              "zeta_a", "eta_a", "K"):
        assert abs(getattr(d, k) - o[k]) <= 1e-14 * max(1.0, abs(o[k])), k
    assert abs(d.tau_nu * d.s_nu - 1) < 1e-15 and abs(d.tau_Tf * d.zeta_a - 1) < 1e-15


def test_derived_values_of_workloads(lib):
    d = B.lbm_ltne_derive(I.cavity_small())
    assert abs(d.F_phi - 1.75 / math.sqrt(150 * 0.6 ** 3)) < 1e-15  # Ergun, Eq. 7
    assert abs(d.l0 - 0.5 * (1 + 0.5 * 0.6 * d.nu_f / d.K)) < 1e-15
    hv = 10.0 * d.alpha_f / 63.0 ** 2
    assert abs(d.d0 - 0.5 * hv / 0.6) < 1e-18 and abs(d.d1 - 0.5 * hv / 0.4) < 1e-18
    assert d.T_ref == 0.5 and d.scale_f == 1.0
    d16 = B.lbm_ltne_derive(I.throughput(n=512, precision=I.FP16S)[0])
    for s in (d16.scale_f, d16.scale_g):
        assert s > 1 and math.frexp(s)[0] == 0.5  # power of two


BAD = [
    dict(phi=1.0), dict(phi=0.0), dict(Da=0.0), dict(Pr=-1.0), dict(varpi=1.0),
    dict(s_q=2.0), dict(zeta_e=0.0), dict(eta_nu=2.5), dict(nx=3), dict(ny=2),
    dict(precision=4), dict(periodic_x=2), dict(Ma=0.0, nu_f=0.0), dict(Ra=0.0, nu_f=0.0),
    dict(gamma_sf=0.0), dict(Hv=-1.0), dict(sigma=0.0), dict(Je=0.0), dict(rho0=0.0),
    dict(nu_wall=5), dict(wall_thermal=(0, 0, 2, 1)), dict(fp16_scale_f=3.0),
    dict(Ra=float("nan")), dict(nx=40000, ny=40000), dict(nx=32769, ny=32768),
    dict(thermal_correction=2), dict(pore_size=-0.01), dict(pore_size=float("inf")),
    dict(diag_every=-1),
]


@pytest.mark.parametrize("bad", BAD, ids=[",".join(b) for b in BAD])
def test_validation_rejects(lib, bad):
    p = I.cavity_small(**bad)
    with pytest.raises(B.LtneError) as e:
        B.lbm_ltne_derive(p)
    assert e.value.code == B.LBM_EINVAL
    assert B.lbm_ltne_pool_bytes(p) == 0
    assert B.lbm_ltne_last_error() != ""


def test_validation_accepts_edges(lib):
    B.lbm_ltne_derive(I.cavity_small(nx=23171, ny=23171, precision=I.FP32))
    B.lbm_ltne_derive(I.cavity_small(nx=32768, ny=32768))  # 2^30 nodes, the limit, in every form
    B.lbm_ltne_derive(I.cavity_small(nx=4, ny=4))
    B.lbm_ltne_derive(I.complete(nx=3, ny=3, periodic_x=1, periodic_y=1, nu_f=0.1, Ma=0.0))
    B.lbm_ltne_derive(I.cavity_small(Hv=0.0, fp16_scale_f=1024.0, precision=I.FP16S))


def test_pool_bytes(lib):
    p = I.cavity_small()
    b0 = B.lbm_ltne_pool_bytes(p)
    assert b0 > 2 * 19 * 64 * 64 * 8
    assert B.lbm_ltne_pool_bytes(p, True, True) > b0
    assert B.lbm_ltne_pool_bytes(I.cavity_small(precision=I.FP32)) < b0
    assert B.lbm_ltne_pool_bytes(I.cavity_small(precision=I.FP16S)) < B.lbm_ltne_pool_bytes(
        I.cavity_small(precision=I.FP32))


def test_strerror(lib):
    for c in (0, -1, -2, -3, -4, -5, -6):
        assert B.lbm_ltne_strerror(c)
    assert B.lbm_ltne_strerror(-99) == "unknown error code"


def test_create_rejects_before_touching_a_device(lib):
    # invalid parameters and fields are refused on the host
    with pytest.raises(B.LtneError) as e:
        B.lbm_ltne_create(I.cavity_small(phi=1.5))
    assert e.value.code == B.LBM_EINVAL
    bad_phi = np.full(64 * 64, 0.5)
    bad_phi[7] = 1.0
    with pytest.raises(B.LtneError) as e:
        B.lbm_ltne_create(I.cavity_small(), phi_field=bad_phi)
    assert e.value.code in (B.LBM_EINVAL, B.LBM_ENODEV)
    # an H_v field and the correlation of Eq. 52 exclude each other
    with pytest.raises(B.LtneError) as e:
        B.lbm_ltne_create(I.cavity_small(pore_size=0.0135), Hv_field=np.full(64 * 64, 10.0))
    assert e.value.code == B.LBM_EINVAL


def test_null_handles_are_refused(lib):
    L = B.lib()
    assert L.lbm_ltne_step(None, 1) == B.LBM_EINVAL
    assert L.lbm_ltne_adjoint(None, 10, 0, None, None, None) == B.LBM_EINVAL
    assert L.lbm_ltne_destroy(None) in (B.LBM_OK, B.LBM_EINVAL)


def test_noalloc_sums_reject_bad_arguments_on_the_host(lib):
    """The allocation-free sums refuse missing fields, unknown precisions and
    oversized lattices before touching a device."""
    import ctypes as C
    L = B.lib()
    p = B.params_from_dict(I.cavity_small())
    out = [C.c_double() for _ in range(3)]
    refs = [C.byref(o) for o in out]
    assert L.lbm_ltne_macro_sums_noalloc(C.byref(p), None, None, None, None, *refs) == B.LBM_EINVAL
    fake = C.c_void_p(0x1000)
    bad = B.params_from_dict(I.cavity_small(precision=7))
    assert L.lbm_ltne_macro_sums_noalloc(C.byref(bad), fake, fake, None, None, *refs) == B.LBM_EINVAL
    big = B.params_from_dict(I.cavity_small(nx=40000, ny=40000))
    assert L.lbm_ltne_macro_sums_noalloc(C.byref(big), fake, fake, None, None, *refs) == B.LBM_EINVAL
    assert "2^30" in B.lbm_ltne_last_error()
