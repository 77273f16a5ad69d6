"""C ABI: the library loads, exports every function include/msrs.h declares,
and validates arguments on the host (no device work)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msrs.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(msrs_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    from paper_1807_08848_amd import msrs
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(msrs.lib, n), n


def test_version_and_device_count():
    from paper_1807_08848_amd import msrs
    assert msrs.version() >= 100
    assert msrs.device_count() >= 0


@pytest.mark.parametrize("args,msg", [
    ((0, 128, 3, [8] * 9, 10, 6), "M must divide"),
    ((0, 128, 4, [8] * 16, 10, 11), "rank"),
    ((0, 128, 4, [8] * 16, 65, 6), "n_samples"),
    ((0, 1024, 4, [128] * 16, 10, 6), "too large"),
    ((0, 128, 4, [-1] * 16, 10, 6), "negative overlap"),
    ((1, 4096, 32, [64] * 32, 48, 10), "n_vel"),
    ((7, 128, 4, [8] * 16, 10, 6), "unknown kind"),
])
def test_create_validates_arguments(args, msg):
    from paper_1807_08848_amd import msrs
    with pytest.raises(msrs.MsrsError) as e:
        msrs.Problem(msrs.make_desc(*args))
    assert e.value.status == msrs.ERR_ARG and msg in str(e.value)


def test_rank_tol_below_the_range_finders_resolution_is_refused():
    """The range finder resolves sigma_j / sigma_1 down to about u (its second
    pass): a tolerance below 1e-12 would choose directions inside the
    snapshots' own rounding."""
    from paper_1807_08848_amd import msrs
    with pytest.raises(msrs.MsrsError) as e:
        msrs.Problem(msrs.make_desc(0, 128, 4, [8] * 16, 32, 6, rank_tol=1e-13))
    assert e.value.status == msrs.ERR_ARG and "resolution" in str(e.value)
    with pytest.raises(msrs.MsrsError) as e:
        msrs.Problem(msrs.make_desc(0, 128, 4, [8] * 16, 32, 6, ir_stop=-1.0))
    assert e.value.status == msrs.ERR_ARG and "ir_stop" in str(e.value)


def test_full_basis_boundary_needs_small_patches():
    from paper_1807_08848_amd import msrs
    with pytest.raises(msrs.MsrsError) as e:
        msrs.Problem(msrs.make_desc(0, 128, 4, [8] * 16, 10, 6, flags=msrs.FLAG_FULL_BASIS_BOUNDARY))
    assert e.value.status == msrs.ERR_ARG and "4 N/M <= 64" in str(e.value)
    with pytest.raises(msrs.MsrsError) as e:
        msrs.Problem(msrs.make_desc(0, 128, 4, [8] * 16, 10, 6, flags=msrs.FLAG_FULL_BASIS))
    assert e.value.status == msrs.ERR_ARG and "4 N/M <= 64" in str(e.value)


def test_least_squares_solver_flags_are_validated():
    """MSRS_FLAG_LS_NORMAL and MSRS_FLAG_LS_CORRECTED exclude each other, and
    the corrected semi-normal step does not apply to the constrained variant."""
    from paper_1807_08848_amd import msrs
    with pytest.raises(msrs.MsrsError) as e:
        msrs.Problem(msrs.make_desc(0, 128, 4, [8] * 16, 10, 6, flags=msrs.FLAG_LS_NORMAL | msrs.FLAG_LS_CORRECTED))
    assert e.value.status == msrs.ERR_ARG and "exclude each other" in str(e.value)
    with pytest.raises(msrs.MsrsError) as e:
        msrs.Problem(msrs.make_desc(0, 64, 4, [8] * 16, 10, 6,
                                    flags=msrs.FLAG_LS_CORRECTED | msrs.FLAG_CONSTRAINED_BC | msrs.FLAG_FULL_BASIS_BOUNDARY))
    assert e.value.status == msrs.ERR_ARG and "constrained" in str(e.value)


def test_null_handle_calls_fail_cleanly():
    from paper_1807_08848_amd import msrs
    L = msrs.lib
    assert L.msrs_assemble_patch(None, None) == msrs.ERR_ARG
    assert L.msrs_sample_local_solutions(None, None, None) == msrs.ERR_ARG
    assert L.msrs_range_finder(None, None, None) == msrs.ERR_ARG
    assert L.msrs_assemble_coarse(None) == msrs.ERR_ARG
    assert L.msrs_solve_global(None, 1, None, None, None) == msrs.ERR_ARG
    assert L.msrs_coarse_corrected(None, None) == msrs.ERR_ARG
    L.msrs_destroy(None)


def test_no_device_is_reported_without_a_gpu():
    from paper_1807_08848_amd import msrs
    if msrs.device_count() > 0:
        pytest.skip("a device is visible")
    with pytest.raises(msrs.MsrsError) as e:
        msrs.Problem(msrs.make_desc(0, 128, 4, [8] * 16, 10, 6))
    assert e.value.status == msrs.ERR_NO_DEVICE


def test_null_server_calls_fail_cleanly():
    import ctypes as C
    from paper_1807_08848_amd import msrs
    L = msrs.lib
    t = C.c_int64()
    f = (C.c_double * 4)()
    assert L.msrs_server_create(None, None, 0, None) == msrs.ERR_ARG
    out = C.c_void_p()
    assert L.msrs_server_create(C.byref(out), None, 0, None) == msrs.ERR_ARG
    hs = (C.c_void_p * 1)(None)
    assert L.msrs_server_create(C.byref(out), hs, 1, None) == msrs.ERR_ARG
    assert "NULL" in L.msrs_server_last_error().decode()
    assert L.msrs_server_submit(None, 0, f, 0.0, C.byref(t)) == msrs.ERR_ARG
    assert L.msrs_server_wait(None, 1, 0.0) == msrs.ERR_ARG
    assert L.msrs_server_fetch(None, 1, None, None) == msrs.ERR_ARG
    assert L.msrs_solve_global_banded(None, 1, None, None, None) == msrs.ERR_ARG
    L.msrs_server_destroy(None)
    assert L.msrs_server_clock() > 0
