"""ctypes binding of ``libaxlb.so`` (the C interface in ``include/axlb.h``).

Argument marshalling only: every step of the lattice Boltzmann path runs in
the HIP kernels of the library.  PyTorch is used for device memory (the
lattice state lives in a ``torch.uint8`` CUDA tensor lent to the library) and
for streams.  There is no fallback: if the library is not built, or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaxlb.so")

OK, EINVAL, ENOMEM, EUNSTABLE, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5
F32, F16, BF16 = 0, 1, 2
LAYOUT_AA, LAYOUT_AB = 0, 1
ANNULUS, CYLINDER = 0, 1
R_IN, R_OUT, Z_LO, Z_HI = 0, 1, 2, 3
FLOW, SWIRL, THERMAL = 0, 1, 2
NOSLIP, PERIODIC, MIRROR, DIRICHLET, OMEGA_R, ADIABATIC = 0, 1, 2, 3, 4, 5

STORAGE = {"f32": F32, "f16": F16, "bf16": BF16}
LAYOUT = {"aa": LAYOUT_AA, "ab": LAYOUT_AB}

# Every symbol include/axlb.h declares.
EXPORTS = [
    "axlb_state_bytes", "axlb_lattice_create", "axlb_set_bc", "axlb_set_body_force",
    "axlb_set_fields", "axlb_step", "axlb_steps_done", "axlb_sync", "axlb_get_moments",
    "axlb_nusselt", "axlb_residual", "axlb_state_size", "axlb_save", "axlb_load",
    "axlb_destroy", "axlb_last_error",
]


class AxlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("axlb error %d: %s" % (code, msg))
        self.code = code


class Geometry(C.Structure):
    _fields_ = [("kind", C.c_int), ("r_inner", C.c_double)]


class Relax(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("omega3", "omega6", "omega7", "omega8", "omega_psi3",
                                          "omega_psi4", "omega_phi3", "omega_phi4")]


class Options(C.Structure):
    _fields_ = [("storage", C.c_int), ("layout", C.c_int), ("T_ref", C.c_double),
                ("stream", C.c_void_p), ("device", C.c_int), ("device_buf", C.c_void_p),
                ("device_bytes", C.c_size_t)]


_lib = None
_dp = C.POINTER(C.c_double)
_vp = C.c_void_p


def load():
    """Loads the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libaxlb.so is not built (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    sig = {
        "axlb_state_bytes": ([C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)], C.c_int),
        "axlb_lattice_create": ([C.c_int, C.c_int, C.POINTER(Geometry), C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.POINTER(Relax),
                                 C.POINTER(Options), C.POINTER(_vp)], C.c_int),
        "axlb_set_bc": ([_vp, C.c_int, C.c_int, C.c_int, C.c_double], C.c_int),
        "axlb_set_body_force": ([_vp, C.c_double, C.c_double], C.c_int),
        "axlb_set_fields": ([_vp] + [_dp] * 5, C.c_int),
        "axlb_step": ([_vp, C.c_long], C.c_int),
        "axlb_steps_done": ([_vp], C.c_long),
        "axlb_sync": ([_vp], C.c_int),
        "axlb_get_moments": ([_vp] + [_dp] * 5, C.c_int),
        "axlb_nusselt": ([_vp] + [_dp] * 3, C.c_int),
        "axlb_residual": ([_vp, _dp], C.c_int),
        "axlb_state_size": ([_vp, C.POINTER(C.c_size_t)], C.c_int),
        "axlb_save": ([_vp, _vp, C.c_size_t], C.c_int),
        "axlb_load": ([_vp, _vp, C.c_size_t], C.c_int),
        "axlb_destroy": ([_vp], None),
        "axlb_last_error": ([_vp], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def state_bytes(Nr, Nz, storage="f32", layout="aa") -> int:
    lib = load()
    n = C.c_size_t()
    rc = lib.axlb_state_bytes(Nr, Nz, STORAGE[storage], LAYOUT[layout], C.byref(n))
    if rc:
        raise AxlbError(rc, lib.axlb_last_error(None).decode())
    return n.value


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


class Lattice:
    """One lattice of the HIP library, set up from a case dict of
    ``paper_1806_10241_amd.inputs``.

    storage: "f32" | "f16" | "bf16"; layout: "aa" (one buffer) | "ab".
    stream: a ``torch.cuda.Stream`` to run on (None: the library's own).
    torch_memory: lend the state as a torch CUDA tensor (else hipMalloc).
    """

    def __init__(self, case: dict, storage: str = "f32", layout: str = "aa", stream=None,
                 device: int = 0, torch_memory: bool = True, init_fields: bool = True):
        lib = load()
        self._lib = lib
        self._h = _vp()
        self.Nr, self.Nz = int(case["Nr"]), int(case["Nz"])
        self.N = self.Nr * self.Nz
        self.storage, self.layout = storage, layout
        geo = Geometry(CYLINDER if case.get("cylinder") else ANNULUS, float(case.get("r_inner", 0.0)))
        rel = Relax(*[float(case.get(k, 1.0)) for k, _ in Relax._fields_])
        opt = Options()
        opt.storage = STORAGE[storage]
        opt.layout = LAYOUT[layout]
        opt.T_ref = float(case.get("T_ref", 0.5))
        opt.device = int(device)
        self._stream = stream
        opt.stream = stream.cuda_stream if stream is not None else None
        self._buf = None
        if torch_memory:
            import torch
            nbytes = state_bytes(self.Nr, self.Nz, storage, layout)
            self._buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda:%d" % device)
            opt.device_buf = self._buf.data_ptr()
            opt.device_bytes = nbytes
        Omega = float(case.get("Omega", float("nan")))
        rc = lib.axlb_lattice_create(self.Nr, self.Nz, C.byref(geo), float(case["nu"]),
                                     float(case["alpha"]), float(case.get("Pr", 0.0)),
                                     float(case.get("Ra", 0.0)), Omega, C.byref(rel),
                                     C.byref(opt), C.byref(self._h))
        if rc:
            raise AxlbError(rc, lib.axlb_last_error(None).decode())
        for (face, fld), (kind, value) in sorted(case["bc"].items()):
            if kind == MIRROR:
                continue  # the axis of a cylinder is set by the library
            self._check(lib.axlb_set_bc(self._h, face, fld, kind, float(value)))
        self._check(lib.axlb_set_body_force(self._h, float(case.get("g_axial", 0.0)),
                                            float(case.get("T0", 0.5))))
        if init_fields and case.get("fields") is not None:
            self.set_fields(**case["fields"]())

    def _check(self, rc):
        if rc:
            raise AxlbError(rc, self._lib.axlb_last_error(self._h).decode())

    def close(self):
        if self._h:
            self._lib.axlb_destroy(self._h)
            self._h = _vp()
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fields(self, rho=None, ur=None, uz=None, uth=None, T=None):
        arrs = []
        for a in (rho, ur, uz, uth, T):
            arrs.append(None if a is None else np.ascontiguousarray(a, dtype=np.float64).ravel())
        for a in arrs:
            if a is not None and a.size != self.N:
                raise ValueError("field size %d != %d" % (a.size, self.N))
        self._check(self._lib.axlb_set_fields(self._h, *[_ptr(a) for a in arrs]))

    def step(self, n: int = 1):
        self._check(self._lib.axlb_step(self._h, int(n)))

    def sync(self):
        self._check(self._lib.axlb_sync(self._h))

    @property
    def steps(self) -> int:
        return int(self._lib.axlb_steps_done(self._h))

    def fields(self) -> dict:
        out = {k: np.empty(self.N) for k in ("rho", "ur", "uz", "uth", "T")}
        self._check(self._lib.axlb_get_moments(self._h, *[_ptr(out[k]) for k in
                                                          ("rho", "ur", "uz", "uth", "T")]))
        return {k: v.reshape(self.Nz, self.Nr) for k, v in out.items()}

    def nusselt(self):
        a, b, m = C.c_double(), C.c_double(), C.c_double()
        self._check(self._lib.axlb_nusselt(self._h, C.byref(a), C.byref(b), C.byref(m)))
        return a.value, b.value, m.value

    def residual(self) -> float:
        r = C.c_double()
        self._check(self._lib.axlb_residual(self._h, C.byref(r)))
        return r.value

    def save(self) -> bytes:
        n = C.c_size_t()
        self._check(self._lib.axlb_state_size(self._h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self._lib.axlb_save(self._h, buf, n.value))
        return buf.raw

    def load(self, image: bytes):
        buf = C.create_string_buffer(image, len(image))
        self._check(self._lib.axlb_load(self._h, buf, len(image)))

    @property
    def handle(self):
        return self._h
