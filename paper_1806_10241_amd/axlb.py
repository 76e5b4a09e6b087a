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
LAYOUT_AA, LAYOUT_AB, LAYOUT_AB2 = 0, 1, 2
ANNULUS, CYLINDER = 0, 1
R_IN, R_OUT, Z_LO, Z_HI = 0, 1, 2, 3
FLOW, SWIRL, THERMAL = 0, 1, 2
NOSLIP, PERIODIC, MIRROR, DIRICHLET, OMEGA_R, ADIABATIC, HALO, VELOCITY, SLIP = 0, 1, 2, 3, 4, 5, 6, 7, 8

STORAGE = {"f32": F32, "f16": F16, "bf16": BF16}
LAYOUT = {"aa": LAYOUT_AA, "ab": LAYOUT_AB, "ab2": LAYOUT_AB2}
DERIV = {"lagged": 0, "current": 1}

# Every symbol include/axlb.h declares.
EXPORTS = [
    "axlb_state_bytes", "axlb_lattice_create", "axlb_set_bc", "axlb_set_body_force",
    "axlb_set_fields", "axlb_step", "axlb_steps_done", "axlb_sync", "axlb_get_moments",
    "axlb_nusselt", "axlb_residual", "axlb_state_size", "axlb_save", "axlb_load",
    "axlb_destroy", "axlb_last_error", "axlb_tile_shape", "axlb_set_tile", "axlb_get_tile",
    "axlb_autotune", "axlb_batch_create", "axlb_batch_size", "axlb_batch_step",
    "axlb_batch_sync", "axlb_batch_set_schedule", "axlb_batch_get_schedule",
    "axlb_batch_set_whole", "axlb_batch_get_whole",
    "axlb_batch_autotune", "axlb_batch_destroy", "axlb_batch_last_error", "axlb_step_each",
    "axlb_halo_bytes", "axlb_halo_export", "axlb_halo_import",
    "axlb_pool_create", "axlb_pool_set_policy", "axlb_pool_submit", "axlb_pool_tick",
    "axlb_pool_status",
    "axlb_pool_result", "axlb_pool_usage", "axlb_pool_destroy", "axlb_pool_last_error",
    "axlb_nusselt_noalloc", "axlb_prepare_steps", "axlb_set_graphs", "axlb_set_bc_outer",
    "axlb_stream_function",
]
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3
POOL_ORDER = {"fifo": 0, "smallest": 1}
NTILES = 8
NSCHEDULES = 4
WHOLE_MAX_NODES = 65536


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
                ("device_bytes", C.c_size_t), ("deriv", C.c_int), ("row0", C.c_int)]


class Request(C.Structure):
    _fields_ = [("Nr", C.c_int), ("Nz", C.c_int), ("geo", Geometry), ("nu", C.c_double),
                ("alpha", C.c_double), ("Pr", C.c_double), ("Ra", C.c_double),
                ("Omega", C.c_double), ("g_axial", C.c_double), ("T0", C.c_double),
                ("bc_kind", (C.c_int * 3) * 4), ("bc_value", (C.c_double * 3) * 4),
                ("storage", C.c_int), ("T_ref", C.c_double),
                ("init", C.POINTER(C.c_double) * 5), ("tol", C.c_double),
                ("max_steps", C.c_long)]


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
    # torch ships its own HIP runtime under the same soname as the system's:
    # loading torch first makes the library bind to that one, so that one
    # runtime owns the device, its memory and its streams in this process.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    sig = {
        "axlb_state_bytes": ([C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)], C.c_int),
        "axlb_lattice_create": ([C.c_int, C.c_int, C.POINTER(Geometry), C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.POINTER(Relax),
                                 C.POINTER(Options), C.POINTER(_vp)], C.c_int),
        "axlb_set_bc": ([_vp, C.c_int, C.c_int, C.c_int, C.c_double], C.c_int),
        "axlb_set_bc_outer": ([_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double],
                              C.c_int),
        "axlb_stream_function": ([_vp, _dp, _dp, _dp], C.c_int),
        "axlb_set_body_force": ([_vp, C.c_double, C.c_double], C.c_int),
        "axlb_set_fields": ([_vp] + [_dp] * 5, C.c_int),
        "axlb_step": ([_vp, C.c_long], C.c_int),
        "axlb_prepare_steps": ([_vp, C.c_long], C.c_int),
        "axlb_set_graphs": ([_vp, C.c_int], C.c_int),
        "axlb_steps_done": ([_vp], C.c_long),
        "axlb_sync": ([_vp], C.c_int),
        "axlb_get_moments": ([_vp] + [_dp] * 5, C.c_int),
        "axlb_nusselt": ([_vp] + [_dp] * 3, C.c_int),
        "axlb_residual": ([_vp, _dp], C.c_int),
        "axlb_state_size": ([_vp, C.POINTER(C.c_size_t)], C.c_int),
        "axlb_save": ([_vp, _vp, C.c_size_t], C.c_int),
        "axlb_load": ([_vp, _vp, C.c_size_t], C.c_int),
        "axlb_destroy": ([_vp], C.c_int),
        "axlb_nusselt_noalloc": ([_vp] + [_dp] * 3, C.c_int),
        "axlb_tile_shape": ([C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
        "axlb_set_tile": ([_vp, C.c_int], C.c_int),
        "axlb_get_tile": ([_vp] + [C.POINTER(C.c_int)] * 3, C.c_int),
        "axlb_autotune": ([_vp, C.c_int, _dp, C.POINTER(C.c_int)], C.c_int),
        "axlb_last_error": ([_vp], C.c_char_p),
        "axlb_batch_create": ([C.POINTER(_vp), C.c_int, C.POINTER(_vp)], C.c_int),
        "axlb_batch_size": ([_vp, C.POINTER(C.c_int), C.POINTER(C.c_longlong)], C.c_int),
        "axlb_batch_step": ([_vp, C.c_long], C.c_int),
        "axlb_batch_sync": ([_vp], C.c_int),
        "axlb_batch_set_schedule": ([_vp, C.c_int, C.c_int], C.c_int),
        "axlb_batch_get_schedule": ([_vp, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
        "axlb_batch_set_whole": ([_vp, C.c_longlong], C.c_int),
        "axlb_batch_get_whole": ([_vp, C.POINTER(C.c_longlong), C.POINTER(C.c_int)], C.c_int),
        "axlb_batch_autotune": ([_vp, C.c_int, _dp, C.POINTER(C.c_int), C.POINTER(C.c_int)],
                                C.c_int),
        "axlb_batch_destroy": ([_vp], None),
        "axlb_batch_last_error": ([_vp], C.c_char_p),
        "axlb_step_each": ([C.POINTER(_vp), C.c_int, C.c_long], C.c_int),
        "axlb_halo_bytes": ([_vp, C.POINTER(C.c_size_t)], C.c_int),
        "axlb_halo_export": ([_vp, C.c_int, _vp], C.c_int),
        "axlb_halo_import": ([_vp, C.c_int, _vp], C.c_int),
        "axlb_pool_create": ([C.c_size_t, C.c_int, C.c_int, C.POINTER(_vp)], C.c_int),
        "axlb_pool_set_policy": ([_vp, C.c_int, C.c_longlong], C.c_int),
        "axlb_pool_submit": ([_vp, C.POINTER(Request), C.POINTER(C.c_long)], C.c_int),
        "axlb_pool_tick": ([_vp, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
        "axlb_pool_status": ([_vp, C.c_long, C.POINTER(C.c_int), C.POINTER(C.c_long), _dp],
                             C.c_int),
        "axlb_pool_result": ([_vp, C.c_long] + [_dp] * 6, C.c_int),
        "axlb_pool_usage": ([_vp, C.POINTER(C.c_size_t), C.POINTER(C.c_longlong)], C.c_int),
        "axlb_pool_destroy": ([_vp], None),
        "axlb_pool_last_error": ([_vp], C.c_char_p),
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


def tile_shape(tile: int):
    lib = load()
    r, z = C.c_int(), C.c_int()
    rc = lib.axlb_tile_shape(int(tile), C.byref(r), C.byref(z))
    if rc:
        raise AxlbError(rc, lib.axlb_last_error(None).decode())
    return r.value, z.value


class Lattice:
    """One lattice of the HIP library, set up from a case dict of
    ``paper_1806_10241_amd.inputs``.

    storage: "f32" | "f16" | "bf16"; layout: "aa" (one buffer) | "ab" (two
    buffers) | "ab2" (two buffers, two steps per launch).
    deriv: "lagged" (previous-step fields) | "current" (this step's output
    fields; needs layout "ab").
    stream: a ``torch.cuda.Stream`` to run on (None: the library's own).
    torch_memory: lend the state as a torch CUDA tensor (else hipMalloc).
    row0: global index of row 0 for a slab of a taller lattice (the
    rounding keys of 16-bit storage).
    """

    def __init__(self, case: dict, storage: str = "f32", layout: str = "aa", stream=None,
                 device: int = 0, torch_memory: bool = True, init_fields: bool = True,
                 deriv: str = "lagged", row0: int = 0):
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
        opt.deriv = DERIV[deriv]
        opt.row0 = int(row0)
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
        for (face, fld), rule in sorted(case["bc"].items()):
            kind, value = rule[0], rule[1]
            if len(rule) > 2 and rule[2] != 0.0:
                raise ValueError("a sloped value is only for the outer part of a z face")
            if kind == MIRROR:
                continue  # the axis of a cylinder is set by the library
            self._check(lib.axlb_set_bc(self._h, face, fld, kind, float(value)))
        # z faces in two parts: case["split"][face] = first radial node of the
        # outer part, case["outer"][(face, fld)] = (kind, value[, slope])
        for (face, fld), rule in sorted(case.get("outer", {}).items()):
            slope = float(rule[2]) if len(rule) > 2 else 0.0
            self._check(lib.axlb_set_bc_outer(self._h, face, int(case["split"][face]), fld,
                                              rule[0], float(rule[1]), slope))
        self._check(lib.axlb_set_body_force(self._h, float(case.get("g_axial", 0.0)),
                                            float(case.get("T0", 0.5))))
        if init_fields and case.get("fields") is not None:
            self.set_fields(**case["fields"]())

    def _check(self, rc):
        if rc:
            raise AxlbError(rc, self._lib.axlb_last_error(self._h).decode())

    def close(self):
        """Releases the lattice.  Raises AxlbError (and keeps the lattice and
        its memory) while it is a member of a live batch."""
        if self._h:
            self._check(self._lib.axlb_destroy(self._h))
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

    def set_graphs(self, enable: bool):
        """Graph replay on or off (off: one plain launch per step or pair)."""
        self._check(self._lib.axlb_set_graphs(self._h, int(bool(enable))))

    def prepare_steps(self, n: int):
        """Captures the graphs that step(n) would replay from here."""
        self._check(self._lib.axlb_prepare_steps(self._h, int(n)))

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

    def stream_function(self):
        """(psi [Nz, Nr] at the outer edge of each node's cell, min psi,
        max psi) of the meridian flow (axlb_stream_function)."""
        psi = np.empty(self.N)
        lo, hi = C.c_double(), C.c_double()
        self._check(self._lib.axlb_stream_function(self._h, _ptr(psi), C.byref(lo),
                                                   C.byref(hi)))
        return psi.reshape(self.Nz, self.Nr), lo.value, hi.value

    def nusselt_noalloc(self):
        """The wall Nusselt numbers through the entry point that allocates
        no device memory (axlb_nusselt_noalloc)."""
        a, b, m = C.c_double(), C.c_double(), C.c_double()
        self._check(self._lib.axlb_nusselt_noalloc(self._h, C.byref(a), C.byref(b), C.byref(m)))
        return a.value, b.value, m.value

    def residual(self) -> float:
        r = C.c_double()
        self._check(self._lib.axlb_residual(self._h, C.byref(r)))
        return r.value

    def halo_bytes(self) -> int:
        n = C.c_size_t()
        self._check(self._lib.axlb_halo_bytes(self._h, C.byref(n)))
        return n.value

    def halo_export(self, face: int, device_ptr: int):
        """Packs the boundary row next to z face `face` into device memory."""
        self._check(self._lib.axlb_halo_export(self._h, int(face), _vp(device_ptr)))

    def halo_import(self, face: int, device_ptr: int):
        """Copies a packed neighbour row into the halo of z face `face`."""
        self._check(self._lib.axlb_halo_import(self._h, int(face), _vp(device_ptr)))

    def save(self) -> bytes:
        n = C.c_size_t()
        self._check(self._lib.axlb_state_size(self._h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self._lib.axlb_save(self._h, buf, n.value))
        return buf.raw

    def load(self, image: bytes):
        buf = C.create_string_buffer(image, len(image))
        self._check(self._lib.axlb_load(self._h, buf, len(image)))

    def set_tile(self, tile: int):
        self._check(self._lib.axlb_set_tile(self._h, int(tile)))

    def tile(self):
        t, r, z = C.c_int(), C.c_int(), C.c_int()
        self._check(self._lib.axlb_get_tile(self._h, C.byref(t), C.byref(r), C.byref(z)))
        return t.value, (r.value, z.value)

    def autotune(self, steps_per_trial: int = 50):
        """Times every tile shape on this lattice (state restored), keeps the
        fastest; returns (best, [ms per step per tile])."""
        ms = np.zeros(NTILES)
        best = C.c_int()
        self._check(self._lib.axlb_autotune(self._h, int(steps_per_trial), _ptr(ms), C.byref(best)))
        return best.value, list(ms)

    @property
    def handle(self):
        return self._h


def _handles(lattices):
    arr = (_vp * len(lattices))()
    for k, lat in enumerate(lattices):
        arr[k] = lat.handle
    return arr


def step_each(lattices, steps: int):
    """The unbatched form: one launch per lattice per step."""
    lib = load()
    rc = lib.axlb_step_each(_handles(lattices), len(lattices), int(steps))
    if rc:
        raise AxlbError(rc, lib.axlb_batch_last_error(None).decode())


class Batch:
    """Fused stepping of several lattices (``axlb_batch_*``).  Keeps the
    member objects alive; close the batch before the members."""

    def __init__(self, lattices):
        lib = load()
        self._lib = lib
        self.members = list(lattices)
        self._h = _vp()
        rc = lib.axlb_batch_create(_handles(self.members), len(self.members), C.byref(self._h))
        if rc:
            raise AxlbError(rc, lib.axlb_batch_last_error(None).decode())

    def _check(self, rc):
        if rc:
            raise AxlbError(rc, self._lib.axlb_batch_last_error(self._h).decode())

    def close(self):
        if self._h:
            self._lib.axlb_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        self._check(self._lib.axlb_batch_step(self._h, int(n)))

    def sync(self):
        self._check(self._lib.axlb_batch_sync(self._h))

    def size(self):
        m, nodes = C.c_int(), C.c_longlong()
        self._check(self._lib.axlb_batch_size(self._h, C.byref(m), C.byref(nodes)))
        return m.value, nodes.value

    def set_schedule(self, tile: int, blocks: int = 0):
        self._check(self._lib.axlb_batch_set_schedule(self._h, int(tile), int(blocks)))

    def schedule(self):
        t, b = C.c_int(), C.c_int()
        self._check(self._lib.axlb_batch_get_schedule(self._h, C.byref(t), C.byref(b)))
        return t.value, b.value

    def autotune(self, steps_per_trial: int = 10):
        """Times every (tile shape, schedule), then the best one with and
        without whole members; keeps the fastest (``whole()`` tells whether
        members run whole).  Returns (tile, blocks, ms[tile][schedule])."""
        ms = np.zeros(NTILES * NSCHEDULES)
        t, b = C.c_int(), C.c_int()
        self._check(self._lib.axlb_batch_autotune(self._h, int(steps_per_trial), _ptr(ms),
                                                  C.byref(t), C.byref(b)))
        return t.value, b.value, ms.reshape(NTILES, NSCHEDULES)

    def set_whole(self, max_nodes: int):
        """Members of at most max_nodes nodes (<= WHOLE_MAX_NODES) run one
        per workgroup, a bundle per launch; 0 turns the mode off."""
        self._check(self._lib.axlb_batch_set_whole(self._h, int(max_nodes)))

    def whole(self):
        """(max_nodes, members that run whole)."""
        m, k = C.c_longlong(), C.c_int()
        self._check(self._lib.axlb_batch_get_whole(self._h, C.byref(m), C.byref(k)))
        return m.value, k.value


def make_request(case: dict, storage: str = "f32", tol: float = 1e-7,
                 max_steps: int = 100000, keep=None) -> Request:
    """C request for a case dict of ``inputs``; `keep` collects the host
    arrays that must stay alive until submission."""
    r = Request()
    r.Nr, r.Nz = int(case["Nr"]), int(case["Nz"])
    r.geo = Geometry(CYLINDER if case.get("cylinder") else ANNULUS, float(case.get("r_inner", 0.0)))
    r.nu, r.alpha = float(case["nu"]), float(case["alpha"])
    r.Pr, r.Ra = float(case.get("Pr", 0.0)), float(case.get("Ra", 0.0))
    r.Omega = float(case.get("Omega", float("nan")))
    r.g_axial, r.T0 = float(case.get("g_axial", 0.0)), float(case.get("T0", 0.5))
    for face in range(4):
        for fld in range(3):
            kind, value = case["bc"].get((face, fld), (NOSLIP if fld < 2 else ADIABATIC, 0.0))
            r.bc_kind[face][fld] = int(kind)
            r.bc_value[face][fld] = float(value)
    r.storage = STORAGE[storage]
    r.T_ref = float(case.get("T_ref", 0.5))
    fields = case["fields"]() if case.get("fields") is not None else {}
    keep = keep if keep is not None else []
    for c, k in enumerate(("rho", "ur", "uz", "uth", "T")):
        a = fields.get(k)
        if a is not None:
            a = np.ascontiguousarray(a, dtype=np.float64).ravel()
            keep.append(a)
            r.init[c] = _ptr(a)
    r.tol, r.max_steps = float(tol), int(max_steps)
    return r


class Pool:
    """Continuous-batching request pool (``axlb_pool_*``)."""

    def __init__(self, budget_bytes: int, device: int = 0, max_members: int = 4096,
                 order: str = "fifo", node_window: int = 0):
        lib = load()
        self._lib = lib
        self._h = _vp()
        rc = lib.axlb_pool_create(int(budget_bytes), int(device), int(max_members),
                                  C.byref(self._h))
        if rc:
            raise AxlbError(rc, lib.axlb_pool_last_error(None).decode())
        self.shapes = {}
        self.set_policy(order, node_window)

    def set_policy(self, order: str = "fifo", node_window: int = 0):
        """order: "fifo" | "smallest" (least Nr*Nz*max_steps first);
        node_window: cap on resident fluid nodes (0: none)."""
        self._check(self._lib.axlb_pool_set_policy(self._h, POOL_ORDER[order], int(node_window)))

    def _check(self, rc):
        if rc:
            raise AxlbError(rc, self._lib.axlb_pool_last_error(self._h).decode())

    def close(self):
        if self._h:
            self._lib.axlb_pool_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, case: dict, storage: str = "f32", tol: float = 1e-7,
               max_steps: int = 100000) -> int:
        keep = []
        r = make_request(case, storage, tol, max_steps, keep)
        rid = C.c_long()
        self._check(self._lib.axlb_pool_submit(self._h, C.byref(r), C.byref(rid)))
        self.shapes[rid.value] = (int(case["Nz"]), int(case["Nr"]))
        return rid.value

    def tick(self):
        run, q = C.c_int(), C.c_int()
        self._check(self._lib.axlb_pool_tick(self._h, C.byref(run), C.byref(q)))
        return run.value, q.value

    def status(self, rid: int):
        st, steps, res = C.c_int(), C.c_long(), C.c_double()
        self._check(self._lib.axlb_pool_status(self._h, int(rid), C.byref(st), C.byref(steps),
                                               C.byref(res)))
        return st.value, steps.value, res.value

    def result(self, rid: int):
        Nz, Nr = self.shapes.pop(rid)
        out = {k: np.empty(Nz * Nr) for k in ("rho", "ur", "uz", "uth", "T")}
        nu = np.empty(3)
        self._check(self._lib.axlb_pool_result(self._h, int(rid),
                                               *[_ptr(out[k]) for k in ("rho", "ur", "uz", "uth", "T")],
                                               _ptr(nu)))
        return {k: v.reshape(Nz, Nr) for k, v in out.items()}, tuple(nu)

    def usage(self):
        used, nodes = C.c_size_t(), C.c_longlong()
        self._check(self._lib.axlb_pool_usage(self._h, C.byref(used), C.byref(nodes)))
        return used.value, nodes.value
