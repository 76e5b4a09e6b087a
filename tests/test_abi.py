"""The C-ABI library loads on a host without a GPU and exports every
function that include/axlb.h declares; argument validation that needs no
device works (no compute calls here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "axlb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(axlb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_bound_functions():
    from paper_1806_10241_amd import axlb
    assert header_functions() == sorted(axlb.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_1806_10241_amd import axlb
    lib = axlb.load()
    for name in header_functions():
        assert hasattr(lib, name), name


def test_state_bytes_and_argument_checks():
    from paper_1806_10241_amd import axlb
    n32 = axlb.state_bytes(1024, 2048, "f32", "aa")
    n16 = axlb.state_bytes(1024, 2048, "f16", "aa")
    nab = axlb.state_bytes(1024, 2048, "f32", "ab")
    pop32 = 19 * 1024 * 2048 * 4
    halo32 = 2 * 19 * 1024 * 4  # the halo rows of the two z faces
    # lagged fields: 16 B per node with FP32 populations, 10 B with 16-bit
    # ones; two time levels, plus the halo rows of the two z faces
    lag_extra = 2 * 6 * 1024 * 2048 + 2 * 6 * 1024
    assert n32 - n16 == (pop32 + halo32) // 2 + lag_extra
    assert nab - n32 == pop32
    with pytest.raises(axlb.AxlbError):
        axlb.state_bytes(1, 10)
    lib = axlb.load()
    import ctypes as C
    out = C.c_void_p()
    geo = axlb.Geometry(axlb.ANNULUS, 10.0)
    # nu <= 0 (relaxation time <= 1/2) is rejected before any device call
    rc = lib.axlb_lattice_create(32, 8, C.byref(geo), 0.0, 0.1, 0.0, 0.0, 0.0, None, None,
                                 C.byref(out))
    assert rc == axlb.EINVAL and not out.value
    assert b"nu" in lib.axlb_last_error(None)
    rc = lib.axlb_lattice_create(32, 8, C.byref(geo), 0.1, 0.1, 0.7, 0.0, 0.0, None, None,
                                 C.byref(out))
    assert rc == axlb.EINVAL  # Pr != nu/alpha
    # a plane of more than 2^30 nodes (rows padded to 64) exceeds the 32-bit
    # byte offsets of the step kernel; exactly 2^30 is accepted by the check
    rc = lib.axlb_lattice_create(1000, (1 << 20) + 1, C.byref(geo), 0.1, 0.1, 0.0, 0.0, 0.0,
                                 None, None, C.byref(out))
    assert rc == axlb.EINVAL and b"2^30" in lib.axlb_last_error(None)


def test_current_derivatives_rejected_with_one_buffer():
    """Option validation happens before any device call: current-step
    derivatives with the single-buffer layout, and an unknown time level,
    are refused with AXLB_EINVAL."""
    import ctypes as C
    from paper_1806_10241_amd import axlb
    lib = axlb.load()
    geo = axlb.Geometry(axlb.ANNULUS, 10.0)
    for layout, deriv in ((axlb.LAYOUT_AA, 1), (axlb.LAYOUT_AB, 2)):
        opt = axlb.Options()
        opt.layout, opt.deriv, opt.T_ref, opt.device = layout, deriv, 0.5, 0
        h = C.c_void_p()
        rc = lib.axlb_lattice_create(30, 8, C.byref(geo), 0.1, 0.1, 0.0, 0.0, float("nan"), None,
                                     C.byref(opt), C.byref(h))
        assert rc == axlb.EINVAL and not h.value


def test_slab_row_and_whole_member_arguments_are_checked():
    """A negative global row 0 is refused before any device call, and the
    whole-member batch calls refuse a NULL batch."""
    import ctypes as C
    from paper_1806_10241_amd import axlb
    lib = axlb.load()
    geo = axlb.Geometry(axlb.ANNULUS, 10.0)
    opt = axlb.Options()
    opt.layout, opt.T_ref, opt.device, opt.row0 = axlb.LAYOUT_AB, 0.5, 0, -1
    h = C.c_void_p()
    rc = lib.axlb_lattice_create(30, 8, C.byref(geo), 0.1, 0.1, 0.0, 0.0, float("nan"), None,
                                 C.byref(opt), C.byref(h))
    assert rc == axlb.EINVAL and not h.value and b"row0" in lib.axlb_last_error(None)
    # bfloat16 with current-step derivatives is refused before any device call
    opt = axlb.Options()
    opt.layout, opt.deriv, opt.storage, opt.T_ref, opt.device = axlb.LAYOUT_AB, 1, 2, 0.5, 0
    rc = lib.axlb_lattice_create(30, 8, C.byref(geo), 0.1, 0.1, 0.0, 0.0, float("nan"), None,
                                 C.byref(opt), C.byref(h))
    assert rc == axlb.EINVAL and not h.value and b"bfloat16" in lib.axlb_last_error(None)
    assert lib.axlb_batch_set_whole(None, 100) == axlb.EINVAL
    m, k = C.c_longlong(), C.c_int()
    assert lib.axlb_batch_get_whole(None, C.byref(m), C.byref(k)) == axlb.EINVAL
