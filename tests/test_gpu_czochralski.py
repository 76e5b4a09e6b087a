"""Wheeler's Czochralski problem (Section 3.6) on the GPU against the
oracle: a lid split into the turning crystal (r < R_x) and a flat free
surface beyond it with a linear wall temperature, the crucible (side wall
and bottom) turning the other way, and buoyancy.  Every layout after 1000
steps at the parity bars, the derivative time levels, the stream function
of the fields, and the rejection of rules a split face cannot take."""
import numpy as np
import pytest

from conftest import say
from paper_1806_10241_amd import inputs as I
from test_gpu_parity import TOL, TOL_DRHO, assert_parity, field_errors, max_errors

pytestmark = pytest.mark.gpu

STEPS = 1000


def case():
    return I.czochralski_melt(N=40, Re_x=100.0, Re_c=-25.0, Gr=1e3)


@pytest.fixture(scope="module")
def oracle_runs(orc):
    cache = {}

    def get(mode):
        if mode not in cache:
            c = case()
            L = orc.Lattice(c, deriv_mode=mode, fields=c["fields"]())
            L.step(STEPS)
            cache[mode] = (L.fields(), L.stream_function())
        return cache[mode]
    return get


@pytest.mark.parametrize("layout,storage,deriv", [
    ("aa", "f32", "lagged"), ("ab", "f32", "lagged"), ("ab2", "f32", "lagged"),
    ("ab", "f32", "current"), ("aa", "f16", "lagged"), ("aa", "bf16", "lagged"),
    ("ab2", "bf16", "lagged")])
def test_czochralski_parity(gpu, orc, oracle_runs, layout, storage, deriv):
    say("czochralski parity", layout, storage, deriv)
    from paper_1806_10241_amd import axlb
    ref, (psi_ref, lo_ref, hi_ref) = oracle_runs(orc.DERIV_CURRENT if deriv == "current"
                                                 else orc.DERIV_PREVIOUS)
    lat = axlb.Lattice(case(), storage=storage, layout=layout, deriv=deriv)
    lat.step(STEPS)
    F = lat.fields()
    psi, lo, hi = lat.stream_function()
    say("  errors", {k: "%.2e" % v[0] for k, v in field_errors(F, ref).items()},
        "max", {k: "%.2e" % v for k, v in max_errors(F, ref).items()},
        "psi range %.6g %.6g (oracle %.6g %.6g)" % (lo, hi, lo_ref, hi_ref))
    assert_parity(F, ref, TOL[storage], (layout, storage, deriv), TOL_DRHO[storage])
    scale = max(-lo_ref, hi_ref)
    assert np.linalg.norm(psi - psi_ref) <= TOL[storage] * np.linalg.norm(psi_ref)
    assert abs(lo - lo_ref) <= TOL[storage] * scale and abs(hi - hi_ref) <= TOL[storage] * scale


def test_stream_function_of_the_fields(gpu):
    """axlb_stream_function integrates the fields axlb_get_moments returns:
    psi = -cumsum(r u_z) along r, to FP64 round-off."""
    from paper_1806_10241_amd import axlb
    c = case()
    lat = axlb.Lattice(c)
    lat.step(300)
    F = lat.fields()
    psi, lo, hi = lat.stream_function()
    r = np.arange(c["Nr"]) + 0.5
    want = -np.cumsum(r[None, :] * F["uz"], axis=1)
    np.testing.assert_allclose(psi, want, rtol=0, atol=1e-13 * np.abs(want).max())
    assert lo == pytest.approx(min(want.min(), 0.0), rel=1e-14)
    assert hi == pytest.approx(max(want.max(), 0.0), rel=1e-14)
    assert lo < 0.0 < hi                          # two cells


def test_split_face_rules_are_validated(gpu):
    from paper_1806_10241_amd import axlb
    lib = axlb.load()
    c = case()
    lat = axlb.Lattice(c)
    h = lat.handle
    E = axlb.EINVAL
    # radial faces have no outer part; the split must lie inside the face
    assert lib.axlb_set_bc_outer(h, axlb.R_OUT, 5, axlb.FLOW, axlb.SLIP, 0.0, 0.0) == E
    assert lib.axlb_set_bc_outer(h, axlb.Z_LO, 0, axlb.FLOW, axlb.SLIP, 0.0, 0.0) == E
    assert lib.axlb_set_bc_outer(h, axlb.Z_LO, c["Nr"], axlb.FLOW, axlb.SLIP, 0.0, 0.0) == E
    # one split per face; SLIP only for f; a slope only with DIRICHLET
    assert lib.axlb_set_bc_outer(h, axlb.Z_HI, 7, axlb.FLOW, axlb.SLIP, 0.0, 0.0) == E
    assert lib.axlb_set_bc_outer(h, axlb.Z_HI, 16, axlb.THERMAL, axlb.SLIP, 0.0, 0.0) == E
    assert lib.axlb_set_bc_outer(h, axlb.Z_HI, 16, axlb.SWIRL, axlb.OMEGA_R, 0.0, 1.0) == E
    assert lib.axlb_set_bc(h, axlb.R_OUT, axlb.FLOW, axlb.SLIP, 0.0) == E
    # a split lid has no Nusselt number
    with pytest.raises(axlb.AxlbError):
        lat.nusselt()
    with pytest.raises(axlb.AxlbError):
        lat.nusselt_noalloc()
    # a split face cannot be periodic
    lat2 = axlb.Lattice(I.rayleigh_benard_cylinder(Nr=12, Nz=8))
    h2 = lat2.handle
    for face in (axlb.Z_LO, axlb.Z_HI):
        for fld in (axlb.FLOW, axlb.SWIRL, axlb.THERMAL):
            assert lib.axlb_set_bc(h2, face, fld, axlb.PERIODIC, 0.0) == axlb.OK
    assert lib.axlb_set_bc_outer(h2, axlb.Z_HI, 4, axlb.FLOW, axlb.SLIP, 0.0, 0.0) == axlb.OK
    assert lib.axlb_step(h2, 1) == E
