"""Current-step derivatives (the central differences of the geometric
sources take this step's output fields; two population buffers): parity
with the oracle's current-field mode after 1000 steps on the cases of
test_gpu_parity, FP32 and binary16 storage; identical results for every
tile shape (the LDS ring, periodic images in partial tiles); graph bundles
equal single launches; the same steady state as the lagged form."""
import numpy as np
import pytest

from conftest import say
from test_gpu_parity import CASES, STEPS, TOL, TOL_DRHO, assert_parity, field_errors
from paper_1806_10241_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oracle_current(orc):
    cache = {}

    def get(name):
        if name not in cache:
            c = CASES[name]()
            L = orc.Lattice(c, deriv_mode=orc.DERIV_CURRENT, fields=c["fields"]())
            L.step(STEPS)
            cache[name] = (L.fields(), L.nusselt() if name != "c1" else None)
        return cache[name]
    return get


@pytest.mark.parametrize("name,storage", [("c1", "f32"), ("c2", "f32"), ("c3", "f32"),
                                          ("c2", "f16"), ("c3", "f16")])
def test_current_derivatives_parity(gpu, oracle_current, name, storage):
    """Binary16 runs on the two buoyancy-driven cases, as the lagged form's
    16-bit parity test does."""
    say("current-step derivatives", name, storage)
    from paper_1806_10241_amd import axlb
    ref, nu_ref = oracle_current(name)
    lat = axlb.Lattice(CASES[name](), storage=storage, layout="ab", deriv="current")
    lat.step(STEPS)
    F = lat.fields()
    say("  errors", {k: "%.2e" % v[0] for k, v in field_errors(F, ref).items()})
    assert_parity(F, ref, TOL[storage], (name, storage), TOL_DRHO[storage])
    if nu_ref is not None:
        for x, y in zip(lat.nusselt(), nu_ref):
            assert abs(x - y) <= 5e-3 * abs(y)


@pytest.mark.parametrize("name", ["c1", "c3"])
def test_current_derivatives_every_tile_identical(gpu, name):
    say("current-step derivatives, tiles", name)
    from paper_1806_10241_amd import axlb
    c = CASES[name]()
    ref = None
    for t in range(axlb.NTILES):
        lat = axlb.Lattice(c, layout="ab", deriv="current")
        lat.set_tile(t)
        lat.step(137)
        img = lat.save()
        if ref is None:
            ref = img
        assert img == ref, axlb.tile_shape(t)


def test_current_derivatives_graphs_equal_single_launches(gpu):
    say("current-step derivatives, graphs")
    from paper_1806_10241_amd import axlb
    c = CASES["c2"]()
    a = axlb.Lattice(c, layout="ab", deriv="current")
    a.step(230)
    b = axlb.Lattice(c, layout="ab", deriv="current")
    for _ in range(230):
        b.step(1)
    assert a.save() == b.save()


def test_current_and_lagged_share_the_steady_state(gpu):
    """Conduction with Couette and Poiseuille flow between cylinders: the
    two derivative inputs differ by the half-step source (F/(2 rho) in the
    velocity), so their steady states agree to that order (the oracle's
    bar for the same comparison)."""
    say("current vs lagged steady state")
    from paper_1806_10241_amd import axlb
    c = I.couette_poiseuille_conduction(Nr=30, Nz=8)
    a = axlb.Lattice(c, layout="ab", deriv="current")
    b = axlb.Lattice(c)
    a.step(30000)
    b.step(30000)
    fa, fb = a.fields(), b.fields()
    for k in ("uz", "uth", "T"):
        assert np.linalg.norm(fa[k] - fb[k]) <= 5e-4 * np.linalg.norm(fb[k]), k


def test_current_derivatives_need_two_buffers(gpu):
    from paper_1806_10241_amd import axlb
    with pytest.raises(axlb.AxlbError):
        axlb.Lattice(CASES["c1"](), layout="aa", deriv="current")
