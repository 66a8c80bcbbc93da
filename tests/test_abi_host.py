"""Host-side checks of the C ABI that need no GPU: the shared library loads,
exports every function include/pcorr.h declares, and rejects bad arguments
before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcorr.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|int64_t)\s+(pc_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for want in ("pc_wls_build", "pc_div_to_grid", "pc_poisson_fft_solve", "pc_grad_to_nodes",
                 "pc_project", "pc_ib_update", "pc_pressure_correct"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2304_14690_amd import pcorr
    lib = ctypes.CDLL(pcorr.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(pcorr.EXPORTS) == declared()


def test_host_side_validation():
    from paper_2304_14690_amd import pcorr
    lib = pcorr.lib()
    assert lib.pc_version() == 115
    out = ctypes.c_void_p()
    n = (ctypes.c_int32 * 3)(64, 64, 1)
    h = (ctypes.c_double * 3)(1 / 64, 1 / 64, 1.0)
    assert lib.pc_plan_create(4, n, h, None, ctypes.byref(out)) == pcorr.PC_ERR_UNSUPPORTED_SIZE
    assert "d must be" in pcorr.last_error()
    bad = (ctypes.c_int32 * 3)(49, 64, 1)
    assert lib.pc_plan_create(2, bad, h, None, ctypes.byref(out)) == pcorr.PC_ERR_UNSUPPORTED_SIZE
    assert lib.pc_plan_create(2, None, h, None, ctypes.byref(out)) == pcorr.PC_ERR_INVALID_ARG
    negh = (ctypes.c_double * 3)(-1.0, 1.0, 1.0)
    assert lib.pc_plan_create(2, n, negh, None, ctypes.byref(out)) == pcorr.PC_ERR_INVALID_ARG
    assert lib.pc_poisson_fft_solve(None, 1, None, None, 0, None, None, None) == \
        pcorr.PC_ERR_INVALID_ARG
    assert lib.pc_wls_build(None, None, None, 0, None, None, ctypes.byref(out)) == \
        pcorr.PC_ERR_INVALID_ARG
    assert lib.pc_plan_destroy(None) == pcorr.PC_OK
    # flat grid indices are int32: more than 2^31 - 2 points is refused
    huge = (ctypes.c_int32 * 3)(2048, 2048, 1024)
    hh = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    assert lib.pc_plan_create(3, huge, hh, None, ctypes.byref(out)) == \
        pcorr.PC_ERR_UNSUPPORTED_SIZE
    assert "2^31" in pcorr.last_error()
    # the allocation-free IB update validates before touching a device
    assert lib.pc_ib_update_noalloc(None, 1, None, None, None, 1e-3, None, None, None) == \
        pcorr.PC_ERR_INVALID_ARG
    # the caller's allocator: both functions or neither
    assert lib.pc_set_allocator(pcorr.ALLOC_FN(lambda u, n, p: 1), pcorr.FREE_FN(), None) == \
        pcorr.PC_ERR_INVALID_ARG
    assert lib.pc_set_allocator(pcorr.ALLOC_FN(), pcorr.FREE_FN(), None) == pcorr.PC_OK
    # per-axis conditions: unknown codes, and an odd periodic axis
    bc = (ctypes.c_int32 * 3)(pcorr.PC_BC_PERIODIC, 7, 0)
    assert lib.pc_plan_create_ex(2, n, h, bc, 0, 0, None, ctypes.byref(out)) == \
        pcorr.PC_ERR_INVALID_ARG
    assert lib.pc_plan_create_ex(2, n, h, None, 5, 0, None, ctypes.byref(out)) == \
        pcorr.PC_ERR_INVALID_ARG
    assert "eig" in pcorr.last_error()
    odd = (ctypes.c_int32 * 3)(401, 64, 1)
    bc = (ctypes.c_int32 * 3)(pcorr.PC_BC_PERIODIC, pcorr.PC_BC_NEUMANN, 0)
    assert lib.pc_plan_create_ex(2, odd, h, bc, 0, 0, None, ctypes.byref(out)) == \
        pcorr.PC_ERR_UNSUPPORTED_SIZE
    assert "even" in pcorr.last_error()
    # grid placement: unknown codes, vertex grids with a periodic axis or too short
    assert lib.pc_plan_create_ex(2, n, h, None, 0, 7, None, ctypes.byref(out)) == \
        pcorr.PC_ERR_INVALID_ARG
    vb = (ctypes.c_int32 * 3)(pcorr.PC_BC_PERIODIC, pcorr.PC_BC_NEUMANN, 0)
    vn = (ctypes.c_int32 * 3)(65, 65, 1)
    assert lib.pc_plan_create_ex(2, vn, h, vb, 0, 1, None, ctypes.byref(out)) == \
        pcorr.PC_ERR_INVALID_ARG
    v8 = (ctypes.c_int32 * 3)(8, 65, 1)
    assert lib.pc_plan_create_ex(2, v8, h, None, 0, 1, None, ctypes.byref(out)) == \
        pcorr.PC_ERR_UNSUPPORTED_SIZE


def test_no_device_is_an_error_not_a_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is visible")
    from paper_2304_14690_amd import pcorr
    with pytest.raises(pcorr.PcError) as e:
        pcorr.Plan(2, (64, 64), (1 / 64, 1 / 64))
    assert e.value.code in (pcorr.PC_ERR_NO_DEVICE, pcorr.PC_ERR_HIP)
