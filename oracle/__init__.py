"""Python access to the FP64 reference oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The HIP library never imports,
links or calls anything here.

The oracle implements the time step of Section 2 of arXiv 1806.10241
(cascaded central-moment LB for axisymmetric thermal flows with swirl); see
``oracle.c`` for the equation-by-equation correspondence.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

R_IN, R_OUT, Z_LO, Z_HI = 0, 1, 2, 3
FLOW, SWIRL, THERMAL = 0, 1, 2
NOSLIP, PERIODIC, MIRROR, DIRICHLET, OMEGA_R, ADIABATIC, VELOCITY, SLIP = 0, 1, 2, 3, 4, 5, 7, 8
DERIV_CURRENT, DERIV_PREVIOUS = 1, 2


# Plain C11 in FP64; every operation rounded on its own (no contraction into
# fused multiply-adds); OpenMP over the per-node loops.  The instruction set
# is the portable x86-64-v3 level, since the library built here also runs on
# other hosts; build_native() makes a copy for the host it runs on.
CFLAGS = ["-std=c11", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC",
          "-shared", "-Wall"]


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + CFLAGS + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_native(path: str) -> str:
    """Compile a copy of the oracle tuned for this host's CPU (-march=native)
    at ``path``; the arithmetic is the same as build()'s."""
    flags = [f if not f.startswith("-march=") else "-march=native" for f in CFLAGS]
    subprocess.check_call(["gcc"] + flags + ["-o", path, _SRC, "-lm"])
    return path


class _BC(C.Structure):
    _fields_ = [("kind", C.c_int), ("value", C.c_double), ("slope", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("Nr", C.c_int), ("Nz", C.c_int), ("cylinder", C.c_int),
                ("r_inner", C.c_double), ("nu", C.c_double), ("alpha", C.c_double),
                ("omega3", C.c_double), ("omega6", C.c_double), ("omega7", C.c_double),
                ("omega8", C.c_double), ("omega_psi3", C.c_double),
                ("omega_psi4", C.c_double), ("omega_phi3", C.c_double),
                ("omega_phi4", C.c_double), ("g_axial", C.c_double), ("gbeta", C.c_double),
                ("T0", C.c_double), ("deriv_mode", C.c_int), ("bc", (_BC * 3) * 4),
                ("split", C.c_int * 2), ("outer", (_BC * 3) * 2)]


_lib = None
_dp = C.POINTER(C.c_double)


def _load(path: str | None = None):
    """The oracle library (``path``: another build of the same source, such
    as build_native()'s, loaded instead of the in-tree one)."""
    global _lib
    if _lib is None or path is not None:
        if path is None and not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(path or _LIB)
        lib.orc_create.restype = C.c_void_p
        lib.orc_create.argtypes = [C.POINTER(_Params)] + [_dp] * 5
        lib.orc_destroy.argtypes = [C.c_void_p]
        lib.orc_step.argtypes = [C.c_void_p, C.c_long]
        lib.orc_steps_done.argtypes = [C.c_void_p]
        lib.orc_steps_done.restype = C.c_long
        lib.orc_fields.argtypes = [C.c_void_p] + [_dp] * 5
        lib.orc_nusselt.argtypes = [C.c_void_p] + [_dp] * 3
        lib.orc_all_finite.argtypes = [C.c_void_p]
        lib.orc_state_len.argtypes = [C.c_void_p]
        lib.orc_state_len.restype = C.c_long
        lib.orc_get_state.argtypes = [C.c_void_p, _dp]
        lib.orc_set_state.argtypes = [C.c_void_p, _dp, C.c_long]
        lib.orc_get_populations.argtypes = [C.c_void_p, _dp, _dp, _dp]
        lib.orc_equilibrium_f.argtypes = [C.c_double] * 3 + [_dp]
        lib.orc_equilibrium_adv.argtypes = [C.c_double] * 3 + [_dp]
        lib.orc_collide_f.argtypes = [_dp] + [C.c_double] * 6 + [_dp, _dp]
        lib.orc_collide_adv.argtypes = [_dp] + [C.c_double] * 4 + [_dp, _dp]
        lib.orc_half_step.argtypes = [C.POINTER(_Params), C.c_double, _dp, _dp, _dp]
        lib.orc_residual.argtypes = [C.c_long] + [_dp] * 8 + [C.c_long]
        lib.orc_residual.restype = C.c_double
        lib.orc_stream_function.argtypes = [C.c_void_p, _dp, _dp, _dp]
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_threads.restype = C.c_int
        if path is not None:
            return lib
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's per-node loops (results do not depend on it)."""
    _load().orc_set_threads(int(n))


def threads() -> int:
    return int(_load().orc_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64).ravel()
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


# ---------------------------------------------------------------- node level
def equilibrium_f(rho, ux, uy):
    out = np.zeros(9)
    _load().orc_equilibrium_f(rho, ux, uy, _ptr(out))
    return out


def equilibrium_adv(s, ux, uy):
    out = np.zeros(5)
    _load().orc_equilibrium_adv(s, ux, uy, _ptr(out))
    return out


def collide_f(f, rho, ux, uy, MA, Fx, Fy, om):
    f = _f64(f, 9)
    om = _f64(om, 9)
    out = np.zeros(9)
    _load().orc_collide_f(_ptr(f), rho, ux, uy, MA, Fx, Fy, _ptr(om), _ptr(out))
    return out


def collide_adv(g, s, ux, uy, S, om):
    g = _f64(g, 5)
    om = _f64(om, 5)
    out = np.zeros(5)
    _load().orc_collide_adv(_ptr(g), s, ux, uy, S, _ptr(om), _ptr(out))
    return out


def params(case: dict, deriv_mode: int = DERIV_PREVIOUS) -> _Params:
    """The oracle's parameter block for a case dict as produced by
    ``paper_1806_10241_amd.inputs``."""
    p = _Params()
    p.Nr, p.Nz = case["Nr"], case["Nz"]
    p.cylinder = int(case.get("cylinder", 0))
    p.r_inner = float(case.get("r_inner", 0.0))
    p.nu, p.alpha = float(case["nu"]), float(case["alpha"])
    p.omega3 = float(case.get("omega3", 1.0))
    for k in ("omega6", "omega7", "omega8", "omega_psi3", "omega_psi4",
              "omega_phi3", "omega_phi4"):
        setattr(p, k, float(case.get(k, 1.0)))
    p.g_axial = float(case.get("g_axial", 0.0))
    # Rayleigh number with L = Nr (gap or cylinder radius) and dT = 1
    # (Section 3.2): g beta = Ra nu alpha / L^3.
    p.gbeta = float(case.get("Ra", 0.0)) * p.nu * p.alpha / float(p.Nr) ** 3
    p.T0 = float(case.get("T0", 0.0))
    p.deriv_mode = int(deriv_mode)
    def put(bc, rule):
        bc.kind, bc.value = int(rule[0]), float(rule[1])
        bc.slope = float(rule[2]) if len(rule) > 2 else 0.0

    for (face, fld), rule in case["bc"].items():
        put(p.bc[face][fld], rule)
    # axial faces in two parts: case["split"][face] = first radial node of
    # the outer part, case["outer"][(face, fld)] = its rule
    for face, first in case.get("split", {}).items():
        p.split[face - Z_LO] = int(first)
    for (face, fld), rule in case.get("outer", {}).items():
        put(p.outer[face - Z_LO][fld], rule)
    return p


def half_step(case: dict, y: float, mom, d) -> dict:
    """The oracle's pre-collision half step of one node at radius y with
    output moments mom = (rho, j_x, j_y, psi, phi) and central differences
    d = (d_x u_y, d_y u_x, d_y u_y, d_y u_theta, d_y phi)."""
    p = params(case)
    mom = _f64(mom, 5)
    d = _f64(d, 5)
    out = np.zeros(10)
    _load().orc_half_step(C.byref(p), float(y), _ptr(mom), _ptr(d), _ptr(out))
    keys = ("MA", "Fx", "Fy", "Spsi", "Sphi", "rho", "ux", "uy", "psi", "phi")
    return dict(zip(keys, out.tolist()))


def residual(now: dict, then: dict, K: int) -> float:
    """The oracle's convergence residual between field snapshots ``now`` and
    ``then`` (dicts with ur, uz, uth, T) taken K steps apart."""
    a = [_f64(now[k]) for k in ("ur", "uz", "uth", "T")]
    b = [_f64(then[k], a[0].size) for k in ("ur", "uz", "uth", "T")]
    return float(_load().orc_residual(a[0].size, *[_ptr(x) for x in a + b], int(K)))


# ---------------------------------------------------------------- lattice
class Lattice:
    """One oracle lattice.  ``case`` is a dict as produced by
    ``paper_1806_10241_amd.inputs`` (keys Nr, Nz, cylinder, r_inner, nu,
    alpha, omega3, ..., g_axial, gbeta, T0, bc); ``deriv_mode`` selects the
    time level of the fields inside the central differences."""

    def __init__(self, case: dict, deriv_mode: int = DERIV_PREVIOUS, fields: dict | None = None,
                 lib=None):
        lib = lib or _load()
        p = params(case, deriv_mode)
        self.Nr, self.Nz = p.Nr, p.Nz
        self.N = p.Nr * p.Nz
        fields = fields or {}
        arrs = [_f64(fields.get(k), self.N) for k in ("rho", "ur", "uz", "uth", "T")]
        self._keep = arrs
        h = lib.orc_create(C.byref(p), *[_ptr(a) for a in arrs])
        if not h:
            raise ValueError("oracle rejected the case parameters")
        self._h = C.c_void_p(h)
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.orc_destroy(h)
            self._h = None

    def step(self, n: int = 1):
        self._lib.orc_step(self._h, int(n))

    @property
    def steps(self) -> int:
        return int(self._lib.orc_steps_done(self._h))

    def fields(self) -> dict:
        out = {k: np.zeros(self.N) for k in ("rho", "ur", "uz", "uth", "T")}
        self._lib.orc_fields(self._h, *[_ptr(out[k]) for k in ("rho", "ur", "uz", "uth", "T")])
        return {k: v.reshape(self.Nz, self.Nr) for k, v in out.items()}

    def nusselt(self):
        a, b, m = C.c_double(), C.c_double(), C.c_double()
        self._lib.orc_nusselt(self._h, C.byref(a), C.byref(b), C.byref(m))
        return a.value, b.value, m.value

    def stream_function(self):
        """(psi [Nz, Nr] at the outer edge of each node's cell, min psi,
        max psi)."""
        psi = np.zeros(self.N)
        lo, hi = C.c_double(), C.c_double()
        self._lib.orc_stream_function(self._h, _ptr(psi), C.byref(lo), C.byref(hi))
        return psi.reshape(self.Nz, self.Nr), lo.value, hi.value

    def all_finite(self) -> bool:
        return bool(self._lib.orc_all_finite(self._h))

    def get_state(self) -> np.ndarray:
        out = np.zeros(int(self._lib.orc_state_len(self._h)))
        self._lib.orc_get_state(self._h, _ptr(out))
        return out

    def set_state(self, st: np.ndarray, steps_done: int):
        st = _f64(st, int(self._lib.orc_state_len(self._h)))
        self._lib.orc_set_state(self._h, _ptr(st), int(steps_done))

    def populations(self):
        f = np.zeros(9 * self.N)
        g = np.zeros(5 * self.N)
        h = np.zeros(5 * self.N)
        self._lib.orc_get_populations(self._h, _ptr(f), _ptr(g), _ptr(h))
        return (f.reshape(9, self.Nz, self.Nr), g.reshape(5, self.Nz, self.Nr),
                h.reshape(5, self.Nz, self.Nr))
