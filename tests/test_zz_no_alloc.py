"""The Nusselt entry point that allocates no device memory
(axlb_nusselt_noalloc) against axlb_nusselt, through the C interface: two
calls in a row on the same device, the second on a smaller lattice (fewer
partial sums than the first left in the shared scratch array), for every
storage, layout and derivative time level, at both AA phases."""
import pytest

from conftest import say
from paper_1806_10241_amd import inputs as I

pytestmark = pytest.mark.gpu


def _pair(axlb, case, steps, **kw):
    lat = axlb.Lattice(case, **kw)
    lat.step(steps)
    ref = lat.nusselt()
    got = lat.nusselt_noalloc()
    lat.close()
    return ref, got


def _close(ref, got):
    for a, b in zip(ref, got):
        assert b == pytest.approx(a, rel=1e-12, abs=1e-13), (ref, got)


CASES = [
    # (case factory of (Nr, Nz), larger size, smaller size, steps)
    ("annulus", lambda nr, nz: I.annulus_convection(Nr=nr, Nz=nz, Ra=1e4), (96, 700), (40, 90)),
    ("cylinder", lambda nr, nz: I.rotating_lid_cylinder(Nr=nr, Nz=nz, Re=300.0, Ri=0.5),
     (600, 64), (70, 33)),
]
KW = [dict(storage="f32", layout="aa"), dict(storage="f16", layout="aa"),
      dict(storage="bf16", layout="ab"), dict(storage="f32", layout="ab2"),
      dict(storage="f32", layout="ab", deriv="current")]


@pytest.mark.parametrize("kw", KW, ids=lambda k: "-".join(k.values()))
@pytest.mark.parametrize("name,make,big,small", CASES, ids=[c[0] for c in CASES])
def test_noalloc_nusselt_matches(gpu, name, make, big, small, kw):
    from paper_1806_10241_amd import axlb
    for steps in (201, 200):
        say("noalloc nusselt: %s %s %s then %s, %d steps" % (name, kw, big, small, steps))
        _close(*_pair(axlb, make(*big), steps, **kw))
        _close(*_pair(axlb, make(*small), steps, **kw))


def test_noalloc_nusselt_rejects_lattices_without_heated_walls(gpu):
    from paper_1806_10241_amd import axlb
    c = I.rayleigh_benard_cylinder(Nr=20, Nz=20)
    c["bc"][(I.Z_HI, I.THERMAL)] = (I.ADIABATIC, 0.0)
    lat = axlb.Lattice(c)
    with pytest.raises(axlb.AxlbError) as e:
        lat.nusselt_noalloc()
    assert e.value.code == axlb.ESTATE
    lat.close()
