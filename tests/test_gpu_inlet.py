"""Walls the fluid crosses (imposed normal velocity: inlets and outlets) on
the GPU against the oracle, and against the closed forms of radial
throughflow between porous cylinders.

* porous annulus (radial inflow through the inner wall, outflow through the
  outer one, swirl and heat carried across): every layout and FP32 against
  the oracle after 1000 steps, binary16 at the 16-bit bar, and the steady
  state against u_theta = A r^(1+Q/nu) + B/r, T = C + D r^(Q/alpha) and the
  axial profile;
* a pipe with plug inflow through the bottom face and outflow through the top
  face (the rule on axial faces, and its corners with the axis and the side
  wall) against the oracle after 1000 steps.
"""
import numpy as np
import pytest

from conftest import say
from paper_1806_10241_amd import inputs as I
from test_gpu_parity import TOL, TOL_DRHO, assert_parity, field_errors, max_errors
from test_oracle_pins import porous_closed_forms, rel_l2

pytestmark = pytest.mark.gpu

STEPS = 1000


def porous_case():
    return I.porous_annulus(Nr=60, Nz=20, r_inner=20.0, Q=0.1, u_inner=0.02, u_outer=0.004,
                            g=2e-6)


def pipe_case():
    return I.pipe_throughflow(Nr=40, Nz=90, U=0.02, u_wall=0.01)


CASES = {"porous": porous_case, "pipe": pipe_case}


@pytest.fixture(scope="module")
def oracle_runs(orc):
    cache = {}

    def get(name):
        if name not in cache:
            c = CASES[name]()
            L = orc.Lattice(c, deriv_mode=orc.DERIV_PREVIOUS, fields=c["fields"]())
            L.step(STEPS)
            cache[name] = L.fields()
        return cache[name]
    return get


@pytest.mark.parametrize("name", ["porous", "pipe"])
@pytest.mark.parametrize("layout,storage", [("aa", "f32"), ("ab", "f32"), ("ab2", "f32"),
                                            ("aa", "f16")])
def test_inlet_parity(gpu, oracle_runs, name, layout, storage):
    say("inlet parity", name, layout, storage)
    from paper_1806_10241_amd import axlb
    ref = oracle_runs(name)
    lat = axlb.Lattice(CASES[name](), storage=storage, layout=layout)
    lat.step(STEPS)
    F = lat.fields()
    say("  errors", {k: "%.2e" % v[0] for k, v in field_errors(F, ref).items()},
        "max", {k: "%.2e" % v for k, v in max_errors(F, ref).items()})
    assert_parity(F, ref, TOL[storage], (name, layout, storage), TOL_DRHO[storage])


def test_porous_annulus_steady_state_on_gpu(gpu):
    """FP32 on the GPU, run to a steady state, against the closed forms at 30
    rows (the oracle reaches 1.4e-3 at this size)."""
    say("porous annulus steady state")
    from paper_1806_10241_amd import axlb
    c = I.porous_annulus(Nr=30, Nz=4, r_inner=10.0, Q=0.1, u_inner=1e-3, u_outer=2e-4)
    lat = axlb.Lattice(c)
    lat.step(30000)
    F = lat.fields()
    cf = porous_closed_forms(c)
    errs = {k: rel_l2(F[k][0], cf[k]) for k in cf}
    say("  closed-form errors", {k: "%.2e" % v for k, v in errs.items()})
    for k, e in errs.items():
        assert e < 3e-3, (k, e)
    # every row equal along the periodic axis
    assert np.abs(F["ur"] - F["ur"][0]).max() < 1e-9


def test_velocity_rule_is_validated(gpu):
    say("velocity rule validation")
    from paper_1806_10241_amd import axlb
    lib = axlb.load()
    lat = axlb.Lattice(I.annulus_convection(Nr=20, Nz=10))
    h = lat.handle
    # VELOCITY is a rule for f only
    assert lib.axlb_set_bc(h, axlb.R_IN, axlb.THERMAL, axlb.VELOCITY, 0.01) == axlb.EINVAL
    assert lib.axlb_set_bc(h, axlb.R_IN, axlb.FLOW, axlb.VELOCITY, float("nan")) == axlb.EINVAL
    # the lids are adiabatic: a VELOCITY lid is refused at the first step
    assert lib.axlb_set_bc(h, axlb.Z_LO, axlb.FLOW, axlb.VELOCITY, 0.01) == axlb.OK
    assert lib.axlb_step(h, 1) == axlb.EINVAL
    assert b"VELOCITY" in lib.axlb_last_error(h)
