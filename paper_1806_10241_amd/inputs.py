"""Seeded synthetic workloads for the axisymmetric cascaded LB time step.

This module only builds inputs: case geometry, boundary settings, transport
coefficients chosen from the dimensionless groups of the paper's Section 3
problems, and seeded initial fields.  It holds none of the method's
arithmetic, and it is the one module that both the HIP library's callers and
the oracle's callers use.

Random numbers come from splitmix64 (Steele, Lea & Flood, 2014), a
counter-based generator: value k of a stream with seed s is the 64-bit mix
of s + (k + 1) * 0x9E3779B97F4A7C15, mapped to a double in [0, 1) by its top
53 bits.

A case is a plain dict:
  Nr, Nz            fluid nodes along r (y) and z (x)
  cylinder          1 = solid cylinder with the axis at y = 0, 0 = annulus
  r_inner           annulus inner-wall radius (lattice units)
  nu, alpha         kinematic viscosity and thermal diffusivity
  Pr, Ra            Prandtl and Rayleigh numbers (Ra uses L = Nr, dT = 1)
  g_axial, T0       uniform axial body force, Boussinesq reference T
  omega3            bulk-viscosity rate (the higher-order rates default to 1)
  bc                {(face, field): (kind, value)}
  T_ref             reference temperature about which h is stored on the GPU
  fields            callable () -> dict of initial host fields [iz][ir]
"""
from __future__ import annotations

import math

import numpy as np

# Faces, distributions and boundary kinds (numbering of the C interface).
R_IN, R_OUT, Z_LO, Z_HI = 0, 1, 2, 3
FLOW, SWIRL, THERMAL = 0, 1, 2
NOSLIP, PERIODIC, MIRROR, DIRICHLET, OMEGA_R, ADIABATIC, VELOCITY, SLIP = 0, 1, 2, 3, 4, 5, 7, 8

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n raw 64-bit outputs of the splitmix64 stream `seed`, from `offset`."""
    k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n doubles in [0, 1) from the top 53 bits of splitmix64."""
    return (splitmix64(seed, n, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ------------------------------------------------------------------ helpers
def _walls(bc, face, inner_swirl=(NOSLIP, 0.0), thermal=(ADIABATIC, 0.0)):
    bc[(face, FLOW)] = (NOSLIP, 0.0)
    bc[(face, SWIRL)] = inner_swirl
    bc[(face, THERMAL)] = thermal


def _periodic_z(bc):
    for face in (Z_LO, Z_HI):
        for fld in (FLOW, SWIRL, THERMAL):
            bc[(face, fld)] = (PERIODIC, 0.0)


def _axis(bc):
    for fld in (FLOW, SWIRL, THERMAL):
        bc[(R_IN, fld)] = (MIRROR, 0.0)


def convection_velocity_scale_params(L: float, Pr: float, Ra: float, U: float = 0.05,
                                     floor: float = 0.01):
    """nu, alpha for a buoyancy velocity scale sqrt(g beta dT L) = U (kept
    small, Section 3.2): nu = U L sqrt(Pr/Ra), alpha = nu/Pr.  Coefficients
    are floored at `floor` (relaxation time 0.53: below it the cell Reynolds
    number U/nu of the under-resolved corners exceeds 5 and runs blow up);
    the effective Ra is then recomputed from g beta = U^2/L and returned."""
    nu = U * L * math.sqrt(Pr / Ra)
    alpha = nu / Pr
    if nu < floor or alpha < floor:
        scale = max(floor / nu, floor / alpha)
        nu, alpha = nu * scale, alpha * scale
    gbeta = U * U / L
    Ra_eff = gbeta * L ** 3 / (nu * alpha)
    return nu, alpha, Ra_eff


def _perturbed_T(seed: int, Nz: int, Nr: int, base: float = 0.5, amp: float = 1e-4,
                 u_amp: float = 0.0):
    """T = base + seeded uniform noise of amplitude amp; with u_amp > 0 also
    u_r, u_z, u_theta = seeded uniform noise of amplitude u_amp (streams
    offset from the temperature's, so every field draws its own numbers)."""
    def make():
        N = Nz * Nr
        T = base + amp * (2.0 * uniform(seed, N) - 1.0)
        out = {"T": T.reshape(Nz, Nr)}
        if u_amp > 0.0:
            for k, name in enumerate(("ur", "uz", "uth")):
                u = u_amp * (2.0 * uniform(seed, N, offset=(k + 1) * N) - 1.0)
                out[name] = u.reshape(Nz, Nr)
        return out
    return make


# ------------------------------------------------------------------ cases
def couette_poiseuille_conduction(Nr: int = 30, Nz: int = 8, r_inner: float = 10.0,
                                  u_wall: float = 1e-3, g: float = 1e-6,
                                  nu: float = 0.1, alpha: float = 0.1) -> dict:
    """Annulus between coaxial cylinders, periodic along z: an axial body
    force drives annular Poiseuille flow, the inner wall turns (circular
    Couette flow in u_theta) and is hot (T = 1) against a cold outer wall
    (T = 0), no buoyancy (Section 3.1 geometry).  Nr counts fluid rows; the
    half-way walls sit at r_inner and r_inner + Nr."""
    bc = {}
    _walls(bc, R_IN, (DIRICHLET, u_wall), (DIRICHLET, 1.0))
    _walls(bc, R_OUT, (DIRICHLET, 0.0), (DIRICHLET, 0.0))
    _periodic_z(bc)
    return dict(name="couette_poiseuille_conduction", Nr=Nr, Nz=Nz, cylinder=0,
                r_inner=float(r_inner), nu=nu, alpha=alpha, Pr=nu / alpha, Ra=0.0,
                g_axial=g, T0=0.5, omega3=1.0, bc=bc, T_ref=0.5,
                fields=lambda: {"T": np.full((Nz, Nr), 0.5)})


def porous_annulus(Nr: int = 30, Nz: int = 4, r_inner: float = 10.0, Q: float = 0.1,
                   u_inner: float = 1e-3, u_outer: float = 0.0, g: float = 1e-6,
                   nu: float = 0.1, alpha: float = 0.1) -> dict:
    """Radial throughflow between porous coaxial cylinders, periodic along z:
    fluid enters through the inner wall with u_r = Q/R_i and leaves through
    the outer wall with u_r = Q/R_o (imposed-velocity walls), the inner wall
    turns (u_theta = u_inner) and is hot (T = 1), the outer wall turns with
    u_outer and is cold (T = 0), and an axial body force g drives axial flow.
    No buoyancy.  Nr counts fluid rows; the walls sit at r_inner and
    r_inner + Nr."""
    Ri, Ro = float(r_inner), float(r_inner) + Nr
    bc = {}
    bc[(R_IN, FLOW)] = (VELOCITY, Q / Ri)
    bc[(R_IN, SWIRL)] = (DIRICHLET, u_inner)
    bc[(R_IN, THERMAL)] = (DIRICHLET, 1.0)
    bc[(R_OUT, FLOW)] = (VELOCITY, Q / Ro)
    bc[(R_OUT, SWIRL)] = (DIRICHLET, u_outer)
    bc[(R_OUT, THERMAL)] = (DIRICHLET, 0.0)
    _periodic_z(bc)
    return dict(name="porous_annulus", Nr=Nr, Nz=Nz, cylinder=0, r_inner=Ri, nu=nu,
                alpha=alpha, Pr=nu / alpha, Ra=0.0, g_axial=g, T0=0.5, omega3=1.0, bc=bc,
                T_ref=0.5, Q=Q, fields=lambda: {"T": np.full((Nz, Nr), 0.5)})


def pipe_throughflow(Nr: int = 24, Nz: int = 48, U: float = 0.01, nu: float = 0.05,
                     alpha: float = 0.05, u_wall: float = 0.0, seed: int = 8) -> dict:
    """Flow through a circular pipe (cylinder, axis by the mirror rule): a
    uniform axial velocity U enters through the bottom face and leaves
    through the top face (imposed-velocity faces), the side wall is at rest
    (or turns with u_theta = u_wall) and held at T = 0 while the inflow
    carries T = 1 and the outflow face is held at T = 0.  Starts at rest at
    T = 0 plus seeded noise of amplitude 1e-4."""
    bc = {}
    _axis(bc)
    _walls(bc, R_OUT, (DIRICHLET, u_wall), (DIRICHLET, 0.0))
    bc[(Z_LO, FLOW)] = (VELOCITY, U)
    bc[(Z_LO, SWIRL)] = (NOSLIP, 0.0)
    bc[(Z_LO, THERMAL)] = (DIRICHLET, 1.0)
    bc[(Z_HI, FLOW)] = (VELOCITY, U)
    bc[(Z_HI, SWIRL)] = (NOSLIP, 0.0)
    bc[(Z_HI, THERMAL)] = (DIRICHLET, 0.0)
    return dict(name="pipe_throughflow", Nr=Nr, Nz=Nz, cylinder=1, r_inner=0.0, nu=nu,
                alpha=alpha, Pr=nu / alpha, Ra=0.0, g_axial=0.0, T0=0.5, omega3=1.0, bc=bc,
                T_ref=0.5, U=U, seed=seed, fields=_perturbed_T(seed, Nz, Nr, base=0.0))


def annulus_convection(Nr: int = 256, Nz: int = 256, radius_ratio: float = 2.0,
                       Pr: float = 0.71, Ra: float = 1e5, seed: int = 1,
                       U: float = 0.05) -> dict:
    """Buoyant natural convection in a vertical annulus (Section 3.2): hot
    inner wall T = 1, cold outer wall T = 0, adiabatic no-slip lids, gravity
    along -z.  L = R_o - R_i = Nr, R_o/R_i = radius_ratio.  Initial state at
    rest with T = 0.5 + seeded uniform noise of amplitude 1e-4."""
    r_inner = Nr / (radius_ratio - 1.0)
    nu, alpha, Ra_eff = convection_velocity_scale_params(Nr, Pr, Ra, U)
    bc = {}
    _walls(bc, R_IN, (NOSLIP, 0.0), (DIRICHLET, 1.0))
    _walls(bc, R_OUT, (NOSLIP, 0.0), (DIRICHLET, 0.0))
    _walls(bc, Z_LO)
    _walls(bc, Z_HI)
    return dict(name="annulus_convection", Nr=Nr, Nz=Nz, cylinder=0, r_inner=r_inner,
                nu=nu, alpha=alpha, Pr=nu / alpha, Ra=Ra_eff, g_axial=0.0, T0=0.5,
                omega3=1.0, bc=bc, T_ref=0.5, seed=seed,
                fields=_perturbed_T(seed, Nz, Nr))


def rotating_lid_cylinder(Nr: int = 1024, Nz: int = 2048, Re: float = 1000.0,
                          Ri: float = 0.5, Pr: float = 1.0, u_lid: float = 0.05,
                          seed: int = 3, u_noise: float = 0.0) -> dict:
    """Closed cylinder H = Nz, R = Nr with a rotating bottom lid (u_theta =
    Omega r, Omega R = u_lid), Re = Omega R^2 / nu, axial temperature
    difference (top T = 1, bottom T = 0, adiabatic side wall) with
    Richardson number Ri = g beta dT R / (Omega R)^2, Pr = nu / alpha
    (Section 3.4 geometry with the buoyancy of Section 3.3).  The axis uses
    the mirror condition.  u_noise > 0 adds seeded velocity noise of that
    amplitude to the initial rest state (every population then differs from
    its rest value from the first step on)."""
    R = float(Nr)
    Omega = u_lid / R
    nu = u_lid * R / Re
    alpha = nu / Pr
    gbeta = Ri * u_lid * u_lid / R
    Ra = gbeta * R ** 3 / (nu * alpha)
    bc = {}
    _axis(bc)
    _walls(bc, R_OUT, (NOSLIP, 0.0), (ADIABATIC, 0.0))
    _walls(bc, Z_LO, (OMEGA_R, Omega), (DIRICHLET, 0.0))
    _walls(bc, Z_HI, (NOSLIP, 0.0), (DIRICHLET, 1.0))
    return dict(name="rotating_lid_cylinder", Nr=Nr, Nz=Nz, cylinder=1, r_inner=0.0,
                nu=nu, alpha=alpha, Pr=Pr, Ra=Ra, Re=Re, Ri=Ri, Omega=Omega,
                g_axial=0.0, T0=0.5, omega3=1.0, bc=bc, T_ref=0.5, seed=seed,
                fields=_perturbed_T(seed, Nz, Nr, u_amp=u_noise))


def rayleigh_benard_cylinder(Nr: int = 100, Nz: int = 100, Pr: float = 0.7, Ra: float = 5e3,
                             T_init: float = 0.0, T0: float = 0.0, seed: int = 6,
                             U: float = 0.05) -> dict:
    """Rayleigh-Benard convection in a closed vertical cylinder (Section 3.3):
    hot bottom lid T = 1, cold top lid T = 0, adiabatic no-slip side wall,
    axis by the mirror rule, gravity along -z.  R = Nr, H = Nz, Ra uses
    L = H and the free-fall velocity sqrt(g beta dT H) = U.  The fluid starts
    at rest at T_init (0: the cold start, 1: the hot start) plus seeded
    noise of amplitude 1e-4.  T0 is the reference temperature of the
    Boussinesq force g beta (T - T0), which Section 3.3 leaves unstated:
    T0 = T_L = 0 (the default) gives the cold start no initial buoyancy
    force; T0 = 1/2, the mean temperature of Section 3.2, starts it under a
    uniform downward force g beta dT / 2."""
    nu, alpha, Ra_eff = convection_velocity_scale_params(Nz, Pr, Ra, U)
    bc = {}
    _axis(bc)
    _walls(bc, R_OUT)
    _walls(bc, Z_LO, thermal=(DIRICHLET, 1.0))
    _walls(bc, Z_HI, thermal=(DIRICHLET, 0.0))
    # Ra is defined with H here: g beta = U^2 / H, expressed in the
    # library's convention Ra_lib = g beta Nr^3 / (nu alpha)
    gbeta = U * U / Nz
    return dict(name="rayleigh_benard_cylinder", Nr=Nr, Nz=Nz, cylinder=1, r_inner=0.0,
                nu=nu, alpha=alpha, Pr=nu / alpha, Ra=gbeta * Nr ** 3 / (nu * alpha),
                Ra_H=Ra_eff, U_ff=U, g_axial=0.0, T0=T0, omega3=1.0, bc=bc, T_ref=0.5,
                seed=seed, fields=_perturbed_T(seed, Nz, Nr, base=T_init))


def mixed_convection_annulus(Nr: int = 40, slenderness: float = 10.0, Re: float = 100.0,
                             sigma: float = 0.0, Pr: float = 0.7, u_wall: float = 0.05,
                             seed: int = 7) -> dict:
    """Mixed convection in a slender annulus with a rotating inner cylinder
    (Section 3.5): D = R_o - R_i = Nr, R_o/R_i = 2, H = slenderness * D,
    inner wall u_theta = Omega_i R_i = u_wall and T = 1, outer wall at rest
    and T = 0, adiabatic no-slip lids, gravity along -z.  Re = u_wall D/nu,
    Gr = g beta dT D^3/nu^2 = sigma Re^2, Pr = nu/alpha.  Starts at rest at
    T = 0.5 plus seeded noise of amplitude 1e-4."""
    D = float(Nr)
    Nz = int(round(slenderness * Nr))
    nu = u_wall * D / Re
    alpha = nu / Pr
    gbeta = sigma * u_wall * u_wall / D
    bc = {}
    _walls(bc, R_IN, (DIRICHLET, u_wall), (DIRICHLET, 1.0))
    _walls(bc, R_OUT, (NOSLIP, 0.0), (DIRICHLET, 0.0))
    _walls(bc, Z_LO)
    _walls(bc, Z_HI)
    return dict(name="mixed_convection_annulus", Nr=Nr, Nz=Nz, cylinder=0, r_inner=D,
                nu=nu, alpha=alpha, Pr=Pr, Ra=gbeta * D ** 3 / (nu * alpha), Re=Re,
                sigma=sigma, g_axial=0.0, T0=0.5, omega3=1.0, bc=bc, T_ref=0.5, seed=seed,
                fields=_perturbed_T(seed, Nz, Nr))


def czochralski_melt(N: int = 40, Re_x: float = 100.0, Re_c: float = -25.0, Pr: float = 0.05,
                     beta: float = 0.4, aspect: float = 1.0, Gr: float = 0.0, u_max: float = 0.05,
                     seed: int = 24) -> dict:
    """Melt in a turning crucible under a turning crystal (Wheeler's
    Czochralski problem, Section 3.6).

    Crucible radius R_c = N, melt depth H = aspect * R_c, crystal radius
    R_x = beta * R_c (a whole number of nodes).  The crucible (side wall and
    bottom) turns at Omega_c = Re_c nu / R_c^2 and the crystal at Omega_x =
    Re_x nu / R_c^2 (opposite senses for Re_c < 0): both Reynolds numbers on
    the crucible radius, the length scale of the problem's other groups;
    nu is set so that the faster of the two rims moves at u_max.  Side wall
    T = 1, crystal T = 0, the free surface between them (R_x < r < R_c,
    flat, no shear) T linear in r from 0 to 1, adiabatic bottom.  Pr =
    nu / alpha, Gr = g beta (T_H - T_L) R_c^3 / nu^2 (Section 3.6 gives none:
    0 by default, where T is carried by the flow but does not drive it).
    The fluid starts at rest at T = 1/2 plus seeded noise of amplitude
    1e-4."""
    Nz = int(round(aspect * N))
    s = int(round(beta * N))
    Rx, Rc = float(s), float(N)
    # rim speeds Omega R = Re nu R / R_c^2; the faster one is u_max
    nu = u_max * Rc ** 2 / max(abs(Re_x) * Rx, abs(Re_c) * Rc)
    alpha = nu / Pr
    Om_x, Om_c = Re_x * nu / Rc ** 2, Re_c * nu / Rc ** 2
    bc = {}
    _axis(bc)
    bc[(R_OUT, FLOW)] = (NOSLIP, 0.0)
    bc[(R_OUT, SWIRL)] = (OMEGA_R, Om_c)
    bc[(R_OUT, THERMAL)] = (DIRICHLET, 1.0)
    bc[(Z_LO, FLOW)] = (NOSLIP, 0.0)
    bc[(Z_LO, SWIRL)] = (OMEGA_R, Om_c)
    bc[(Z_LO, THERMAL)] = (ADIABATIC, 0.0)
    # the top: the crystal for r < R_x, the free surface beyond
    bc[(Z_HI, FLOW)] = (NOSLIP, 0.0)
    bc[(Z_HI, SWIRL)] = (OMEGA_R, Om_x)
    bc[(Z_HI, THERMAL)] = (DIRICHLET, 0.0)
    b = Rx / Rc
    outer = {(Z_HI, FLOW): (SLIP, 0.0), (Z_HI, SWIRL): (ADIABATIC, 0.0),
             # T = (r / R_c - beta) / (1 - beta) = value + slope * r
             (Z_HI, THERMAL): (DIRICHLET, -b / (1.0 - b), 1.0 / ((1.0 - b) * Rc))}
    return dict(name="czochralski_melt", Nr=N, Nz=Nz, cylinder=1, r_inner=0.0, nu=nu,
                alpha=alpha, Pr=Pr, Ra=Gr * Pr, Gr=Gr, Re_x=Re_x, Re_c=Re_c, Omega_x=Om_x,
                Omega_c=Om_c,
                R_x=Rx, R_c=Rc, g_axial=0.0, T0=0.5, omega3=1.0, bc=bc, split={Z_HI: s},
                outer=outer, T_ref=0.5, seed=seed, fields=_perturbed_T(seed, Nz, N))


def batched_annuli(n: int = 256, seed: int = 4, nr=(48, 256), nz=(48, 512)):
    """Uneven annulus convection instances: Nr ~ U{48..256}, Nz ~ U{48..512}
    (or the given ranges), Ra log-uniform in [1e3, 1e6], Pr log-uniform in
    [0.02, 7], radius ratio uniform in [1.5, 4]; instance k uses
    seed*1000 + k for its noise."""
    u = uniform(seed, 5 * n).reshape(n, 5)
    cases = []
    for k in range(n):
        Nr = nr[0] + int(u[k, 0] * (nr[1] - nr[0] + 1))
        Nz = nz[0] + int(u[k, 1] * (nz[1] - nz[0] + 1))
        Ra = 10.0 ** (3.0 + 3.0 * u[k, 2])
        Pr = 10.0 ** (math.log10(0.02) + (math.log10(7.0) - math.log10(0.02)) * u[k, 3])
        ratio = 1.5 + 2.5 * u[k, 4]
        c = annulus_convection(Nr=Nr, Nz=Nz, radius_ratio=ratio, Pr=Pr, Ra=Ra,
                               seed=seed * 1000 + k)
        c["name"] = "batched_annulus_%d" % k
        cases.append(c)
    return cases


def serving_trace(n: int = 2000, rate: float = 200.0, seed: int = 5,
                  max_nr_log2: float = 10.0, max_nz_log2: float = 11.0):
    """Poisson arrivals at `rate` per second of solve requests mixing the
    three problem types, grids N_r = 2^U(6, max_nr_log2), N_z = 2^U(6,
    max_nz_log2) rounded to multiples of 16, storage FP32 or 16-bit with
    probability 1/2 each.  Rotating-lid requests draw Re log-uniform in
    [500, 2000], capped at 8 N_r so that nu = 0.05 N_r / Re stays at or above
    0.00625 on small grids.  Returns a list of (arrival_s, case, storage)."""
    u = uniform(seed, 6 * n).reshape(n, 6)
    t = 0.0
    out = []
    for k in range(n):
        t += -math.log(1.0 - u[k, 0]) / rate
        kind = min(int(u[k, 1] * 3), 2)
        Nr = int(round(2.0 ** (6 + (max_nr_log2 - 6) * u[k, 2]) / 16.0)) * 16
        Nz = int(round(2.0 ** (6 + (max_nz_log2 - 6) * u[k, 3]) / 16.0)) * 16
        Nr, Nz = max(Nr, 16), max(Nz, 16)
        storage = "f32" if u[k, 4] < 0.5 else "f16"
        if kind == 0:
            c = couette_poiseuille_conduction(Nr=Nr, Nz=Nz, r_inner=Nr / 3.0)
        elif kind == 1:
            c = annulus_convection(Nr=Nr, Nz=Nz, Ra=10.0 ** (3 + 2 * u[k, 5]),
                                   seed=seed * 100000 + k)
        else:
            Re = min(500.0 * 4.0 ** u[k, 5], 8.0 * Nr)
            c = rotating_lid_cylinder(Nr=Nr, Nz=Nz, Re=Re, seed=seed * 100000 + k)
        c["name"] = "request_%d" % k
        out.append((t, c, storage))
    return out
