"""The seeded workload generator: splitmix64 known answers and the
dimensionless groups of the recipes."""
import math

import numpy as np

from paper_1806_10241_amd import inputs as I


def test_splitmix64_known_answers():
    # first outputs of the published splitmix64 generator seeded with 0
    assert [int(x) for x in I.splitmix64(0, 3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = I.uniform(7, 100000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 5e-3


def test_annulus_convection_groups():
    c = I.annulus_convection(Nr=256, Nz=256, Pr=0.71, Ra=1e5)
    L = c["Nr"]
    gbeta = c["Ra"] * c["nu"] * c["alpha"] / L ** 3
    assert math.isclose(c["nu"] / c["alpha"], 0.71, rel_tol=1e-12)
    assert math.isclose(gbeta, 0.05 ** 2 / L, rel_tol=1e-12)   # U^2 / L with U = 0.05
    assert math.isclose(c["Ra"], 1e5, rel_tol=1e-12)
    assert math.isclose(c["r_inner"] + L, 2 * c["r_inner"])    # R_o / R_i = 2
    T = c["fields"]()["T"]
    assert T.shape == (256, 256) and np.abs(T - 0.5).max() <= 1e-4


def test_floor_on_transport_coefficients():
    nu, alpha, Ra_eff = I.convection_velocity_scale_params(48, 0.02, 1e6)
    assert min(nu, alpha) >= 0.01 - 1e-15 and Ra_eff < 1e6


def test_rotating_lid_groups():
    c = I.rotating_lid_cylinder(Nr=1024, Nz=2048, Re=1000.0, Ri=0.5)
    R = 1024.0
    assert math.isclose(c["Omega"] * R * R / c["nu"], 1000.0, rel_tol=1e-12)
    gbeta = c["Ra"] * c["nu"] * c["alpha"] / R ** 3
    assert math.isclose(gbeta * R / (c["Omega"] * R) ** 2, 0.5, rel_tol=1e-12)
    assert c["bc"][(I.Z_LO, I.SWIRL)] == (I.OMEGA_R, c["Omega"])


def test_batched_and_served_recipes():
    cases = I.batched_annuli(256, seed=4)
    Nr = np.array([c["Nr"] for c in cases])
    Nz = np.array([c["Nz"] for c in cases])
    assert Nr.min() >= 48 and Nr.max() <= 256 and Nz.min() >= 48 and Nz.max() <= 512
    assert 1.0e7 < (Nr * Nz).sum() < 1.2e7
    trace = I.serving_trace(2000, rate=200.0, seed=5)
    t = np.array([a for a, _, _ in trace])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 200.0) < 0.1 / 200.0
    for _, c, st in trace[:200]:
        assert c["Nr"] % 16 == 0 and c["Nz"] % 16 == 0 and 64 <= c["Nr"] <= 1024
        assert st in ("f32", "f16")


def test_rotating_lid_velocity_noise():
    """u_noise seeds u_r, u_z, u_theta from streams of their own (disjoint
    from the temperature's), within the amplitude; the default is a rest
    state with temperature noise only."""
    quiet = I.rotating_lid_cylinder(Nr=64, Nz=32)["fields"]()
    assert sorted(quiet) == ["T"]
    f = I.rotating_lid_cylinder(Nr=64, Nz=32, u_noise=1e-4)["fields"]()
    assert sorted(f) == ["T", "ur", "uth", "uz"]
    assert np.array_equal(f["T"], quiet["T"])
    for k in ("ur", "uz", "uth"):
        assert f[k].shape == (32, 64) and np.abs(f[k]).max() <= 1e-4 and np.abs(f[k]).min() > 0
    # independent draws: no two fields share a value pattern
    assert not np.allclose(f["ur"], f["uz"]) and not np.allclose(f["uz"], f["uth"])
    assert abs(np.corrcoef(f["ur"].ravel(), (f["T"] - 0.5).ravel())[0, 1]) < 0.1
