"""Pins of oracle parts that the closed-form flows leave open (no GPU):

* the per-node loops give the same bits on any number of threads;
* the pre-collision half step (eq. 21, 38, 48) returns a state at which the
  split relations hold with the geometric sources of eq. (4), (5), (7), (9)
  evaluated at that same state; the sources are written out here from the
  paper, not taken from the oracle;
* the convergence residual on snapshots whose differences are known;
* the r-weighted lid Nusselt number of a closed cylinder (Section 3.3
  geometry): pure conduction between the lids gives exactly 1 at both lids,
  a result that a wrong radial weight, normalisation or sign cannot give.
"""
import math

import numpy as np
import pytest

from paper_1806_10241_amd import inputs as I


def test_thread_count_does_not_change_results(orc):
    c = I.rotating_lid_cylinder(Nr=40, Nz=60, Re=400.0, Ri=0.5, u_noise=1e-3)
    states = []
    t0 = orc.threads()
    for t in (1, 3, 8):
        orc.set_threads(t)
        L = orc.Lattice(c, fields=c["fields"]())
        L.step(30)
        states.append(L.get_state())
    orc.set_threads(t0)
    for s in states[1:]:
        assert np.array_equal(s, states[0])


# ---------------------------------------------------------------- half step
def paper_sources(case, y, rho, jx, jy, psi, phi, d):
    """Eq. (4a)-(4c), (5), (7) and (9) at the state (rho, rho u_x = jx,
    rho u_y = jy, psi, phi) of a node at radius y; d = (d_x u_y, d_y u_x,
    d_y u_y, d_y u_theta, d_y phi).  Body force F^b_x = g + g beta (phi - T0)
    (Boussinesq, rho_0 = 1), F^b_y = 0."""
    nu, alpha = case["nu"], case["alpha"]
    gbeta = case["Ra"] * nu * alpha / case["Nr"] ** 3
    ux, uy, mu = jx / rho, jy / rho, rho * nu
    MA = -rho * uy / y
    FAx = -rho * ux * uy / y + mu * (d[0] + d[1]) / y
    FAy = psi ** 2 / (rho * y) - rho * uy ** 2 / y + 2 * mu * d[2] / y - 2 * mu * uy / y ** 2
    Fx = FAx + case["g_axial"] + gbeta * (phi - case["T0"])
    Fy = FAy
    Spsi = -2 * uy * psi / y + mu * d[3] / y - nu * psi / y ** 2
    Sphi = -uy * phi / y + alpha * d[4] / y
    return MA, Fx, Fy, Spsi, Sphi


@pytest.mark.parametrize("seed", range(6))
def test_half_step_satisfies_split_relations(orc, seed):
    """rho = rho^o + M^A/2, rho u = j^o + F/2, psi = psi^o + S_psi/2,
    phi = phi^o + S_phi/2, with every source evaluated at the returned
    (rho, u, psi, phi) itself; random states with strong swirl and radial
    flow, from the axis region (y = 0.5) outwards."""
    u = I.uniform(100 + seed, 20)
    case = I.rotating_lid_cylinder(Nr=64, Nz=64, Re=50.0 + 400 * u[0], Ri=2.0 * u[1])
    case["g_axial"] = 1e-5 * (u[2] - 0.5)
    y = [0.5, 1.5, 3.5, 17.5, 63.5, 1000.5][seed]
    mom = [1.0 + 0.02 * (u[3] - 0.5), 0.1 * (u[4] - 0.5), 0.1 * (u[5] - 0.5),
           0.1 * (u[6] - 0.5), u[7]]
    d = [0.02 * (x - 0.5) for x in u[8:13]]
    h = orc.half_step(case, y, mom, d)
    src = paper_sources(case, y, h["rho"], h["rho"] * h["ux"], h["rho"] * h["uy"], h["psi"],
                        h["phi"], d)
    for name, v in zip(("MA", "Fx", "Fy", "Spsi", "Sphi"), src):
        assert h[name] == pytest.approx(v, rel=1e-13, abs=1e-16), name
    assert h["rho"] == pytest.approx(mom[0] + 0.5 * src[0], rel=1e-15)
    assert h["rho"] * h["ux"] == pytest.approx(mom[1] + 0.5 * src[1], rel=1e-13, abs=1e-17)
    assert h["rho"] * h["uy"] == pytest.approx(mom[2] + 0.5 * src[2], rel=1e-13, abs=1e-17)
    assert h["psi"] == pytest.approx(mom[3] + 0.5 * src[3], rel=1e-13, abs=1e-17)
    assert h["phi"] == pytest.approx(mom[4] + 0.5 * src[4], rel=1e-13, abs=1e-17)


def test_half_step_without_sources_is_identity(orc):
    """Far from the axis with no motion, no gradient and no force every
    source vanishes and the half step leaves the output moments alone."""
    case = I.couette_poiseuille_conduction()
    case["g_axial"] = 0.0
    h = orc.half_step(case, 1e9, [1.3, 0.0, 0.0, 0.0, 0.7], [0.0] * 5)
    assert h["rho"] == pytest.approx(1.3, rel=1e-15)
    assert h["phi"] == pytest.approx(0.7, rel=1e-15)
    assert h["ux"] == h["uy"] == h["psi"] == 0.0


# ---------------------------------------------------------------- residual
def test_residual_definition(orc):
    n = 257
    u = I.uniform(11, 4 * n).reshape(4, n)
    now = {"ur": u[0] - 0.5, "uz": u[1] - 0.5, "uth": u[2] - 0.5, "T": u[3]}
    speed = math.sqrt(sum(float(np.sum(now[k] ** 2)) for k in ("ur", "uz", "uth")))
    # only u_z changed, by a known field
    dz = 1e-6 * np.cos(np.arange(n))
    then = dict(now, uz=now["uz"] - dz)
    K = 100
    assert orc.residual(now, then, K) == pytest.approx(np.linalg.norm(dz) / (K * speed),
                                                       rel=1e-12)
    # a uniform relative change of T by eps gives eps / K when it dominates
    eps = 3e-5
    then = dict(now, T=now["T"] * (1 - eps))
    assert orc.residual(now, then, 7) == pytest.approx(eps / 7, rel=1e-9)
    # identical snapshots give 0; K <= 0 gives +inf
    assert orc.residual(now, now, 5) == 0.0
    assert math.isinf(orc.residual(now, then, 0))
    # a field with zero norm is skipped, not divided by
    zero = {k: np.zeros(n) for k in now}
    assert orc.residual(zero, zero, 3) == 0.0


# ---------------------------------------------------------------- lid Nusselt
def conduction_cylinder(Nr, Nz, T_bottom=1.0, T_top=0.0, alpha=0.25):
    """Closed cylinder at rest, no buoyancy: lids at fixed temperatures,
    adiabatic side wall, axis by the mirror rule."""
    c = I.rayleigh_benard_cylinder(Nr=Nr, Nz=Nz, Ra=5e3)
    c.update(nu=alpha, alpha=alpha, Pr=1.0, Ra=0.0)
    c["bc"][(I.Z_LO, I.THERMAL)] = (I.DIRICHLET, T_bottom)
    c["bc"][(I.Z_HI, I.THERMAL)] = (I.DIRICHLET, T_top)
    c["fields"] = lambda: {"T": np.full((Nz, Nr), 0.5 * (T_bottom + T_top))}
    return c


@pytest.mark.parametrize("Nr,Nz", [(5, 12), (11, 8)])
def test_lid_nusselt_of_conduction_is_one(orc, Nr, Nz):
    """T relaxes to the linear profile between the lids, which the
    anti-bounce-back rule and the one-sided wall gradient reproduce exactly;
    the area weight 2/R^2 sum y_j then gives Nu = 1 at both lids.  A weight
    of (j + 1) instead of y_j = j + 1/2, a missing factor 2 or a flipped
    gradient sign would give 1 + 1/R, 1/2 or -1."""
    c = conduction_cylinder(Nr, Nz)
    L = orc.Lattice(c, fields=c["fields"]())
    L.step(int(30 * Nz * Nz / c["alpha"]))
    a, b, m = L.nusselt()
    assert a == pytest.approx(1.0, abs=1e-10)
    assert b == pytest.approx(1.0, abs=1e-10)
    T = L.fields()["T"]
    x = np.arange(Nz) + 0.5
    assert np.abs(T - (1.0 - x / Nz)[:, None]).max() < 1e-10
    # reversing the temperature difference keeps Nu positive (Nu is scaled by
    # the lid difference); swapping which lid is hot flips the flux direction
    c2 = conduction_cylinder(Nr, Nz, T_bottom=0.25, T_top=2.25)
    L2 = orc.Lattice(c2, fields=c2["fields"]())
    L2.step(int(30 * Nz * Nz / c2["alpha"]))
    a2, b2, _ = L2.nusselt()
    assert a2 == pytest.approx(1.0, abs=1e-10) and b2 == pytest.approx(1.0, abs=1e-10)


# ---------------------------------------------------------------- radial throughflow
def porous_closed_forms(c):
    """Steady radial throughflow between porous cylinders (u_r = Q/r, which
    satisfies the axisymmetric continuity equation with the geometric mass
    source of eq. 4a exactly).  With it, eq. (1d) for u_theta, (1e) for T
    and (1c) for u_z become ordinary differential equations in r whose
    solutions are powers of r:
      (Q/r)(u' + u/r) = nu (u'' + u'/r - u/r^2)  ->  u_theta = A r^(1+Q/nu) + B/r,
      (Q/r) T' = alpha (T'' + T'/r)             ->  T = C + D r^(Q/alpha),
      (Q/r) w' = nu (w'' + w'/r) + g            ->  u_z = g r^2/(2Q - 4 nu) + E + F r^(Q/nu),
    with the constants from the wall values."""
    Q, nu, al, g = c["Q"], c["nu"], c["alpha"], c["g_axial"]
    Ri, Ro = c["r_inner"], c["r_inner"] + c["Nr"]
    r = Ri + np.arange(c["Nr"]) + 0.5
    ui = c["bc"][(I.R_IN, I.SWIRL)][1]
    uo = c["bc"][(I.R_OUT, I.SWIRL)][1]
    m, k = Q / nu, Q / al
    A, B = np.linalg.solve([[Ri ** (1 + m), 1 / Ri], [Ro ** (1 + m), 1 / Ro]], [ui, uo])
    C, D = np.linalg.solve([[1.0, Ri ** k], [1.0, Ro ** k]], [1.0, 0.0])
    cz = g / (2 * Q - 4 * nu)
    E, F = np.linalg.solve([[1.0, Ri ** m], [1.0, Ro ** m]], [-cz * Ri ** 2, -cz * Ro ** 2])
    return {"ur": Q / r, "uth": A * r ** (1 + m) + B / r, "T": C + D * r ** k,
            "uz": cz * r ** 2 + E + F * r ** m}


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def porous_runs(orc):
    """Q/nu = 1 and 2.5, at 30 and 60 rows (R_i, R_o doubled, g quartered),
    each run for several diffusion times."""
    out = {}
    for Q in (0.1, 0.25):
        for s in (1, 2):
            c = I.porous_annulus(Nr=30 * s, r_inner=10.0 * s, Q=Q, g=1e-6 / s ** 2,
                                 u_inner=1e-3, u_outer=2e-4)
            L = orc.Lattice(c, fields=c["fields"]())
            L.step(25000 * s * s)
            rho_a = L.fields()["rho"].mean()
            L.step(500)
            out[(Q, s)] = (c, L.fields(), rho_a)
    return out


@pytest.mark.parametrize("Q", [0.1, 0.25])
def test_porous_annulus_closed_forms(porous_runs, Q):
    """The imposed-velocity walls carry the throughflow, and the r-dependent
    terms of the sources with u_r != 0 (M^A of eq. 4a, -rho u_x u_y / y of
    eq. 4b, -2 u_y psi / y and the viscous terms of eq. 7, -u_y phi / y of
    eq. 9) shape the profiles: rel-L2 below 3e-3 at 30 rows and observed
    order above 1.8 from 30 to 60 rows, for every field."""
    errs = []
    for s in (1, 2):
        c, F, rho_a = porous_runs[(Q, s)]
        cf = porous_closed_forms(c)
        e = {k: rel_l2(F[k][0], cf[k]) for k in cf}
        errs.append(e)
        # steady, uniform along the periodic axis, and no drift of the mass
        assert np.abs(F["ur"] - F["ur"][0]).max() < 1e-12
        assert abs(F["rho"].mean() - rho_a) < 1e-10
    for k in errs[0]:
        assert errs[0][k] < 3e-3, (k, errs[0][k])
        assert math.log2(errs[0][k] / errs[1][k]) > 1.8, (k, errs)


# ------------------------------------------------- derivative time levels
def test_current_and_lagged_derivatives_transient_gap(orc):
    """The two readings of the time level of the central differences (this
    step's output fields, or the previous step's half-step fields) differ
    by a one-step lag inside the geometric sources only, so their fields
    stay close through a transient: in convection between coaxial
    cylinders (Ra = 1e4, 32 x 32) from rest the velocity gap is 1.7e-4 of
    the speed norm after 10 steps and falls to 1.1e-5 as the flow settles
    (T: 8e-5 to 5e-6), while the fields themselves change by O(1); the
    same holds for the rotating lid (2e-5 to 8e-5)."""
    c = I.annulus_convection(Nr=32, Nz=32, Ra=1e4)
    F0 = c["fields"]()
    A = orc.Lattice(c, deriv_mode=orc.DERIV_CURRENT, fields=F0)
    B = orc.Lattice(c, deriv_mode=orc.DERIV_PREVIOUS, fields=F0)
    for n, bar_u, bar_T in ((10, 5e-4, 2e-4), (100, 5e-4, 2e-4), (1000, 1e-4, 1e-4),
                            (10000, 3e-5, 2e-5)):
        A.step(n - A.steps)
        B.step(n - B.steps)
        a, b = A.fields(), B.fields()
        speed = np.linalg.norm(np.sqrt(b["ur"] ** 2 + b["uz"] ** 2 + b["uth"] ** 2))
        gap_u = max(np.linalg.norm(a[k] - b[k]) for k in ("ur", "uz", "uth")) / speed
        gap_T = np.linalg.norm(a["T"] - b["T"]) / np.linalg.norm(b["T"] - 0.5)
        assert 0.0 < gap_u < bar_u and gap_T < bar_T, (n, gap_u, gap_T)
